"""Autotuner host logic (no GPU): graph classes, table validation, lookup."""
import pytest

from paper_1903_01665_amd import gg

V, E, S, A = gg.VERTEX, gg.EDGE, gg.SYNC, gg.ASYNC


@pytest.fixture(autouse=True)
def _restore_table():
    saved = gg.tune_get()
    yield
    gg.tune_set(saved)


def test_class_of_workloads():
    # rmat22: m = 2^26, hub degree 159873 vs average 16 -> skew class 2
    assert gg.class_of(1 << 26, 1 << 22, 159873, 8) == (13, 2, 0)
    # grid4096: m ~ 67.8M, max degree 8 vs average ~4 -> skew 0, thousands of levels
    assert gg.class_of(67763404, 1 << 24, 8, 2622) == (13, 0, 2)
    # er23: max 26 vs average 8 -> skew 0; 13 levels -> depth 0; unknown depth
    assert gg.class_of(1 << 26, 1 << 23, 26, 13) == (13, 0, 0)
    assert gg.class_of(1 << 26, 1 << 23, 26, -1)[2] == -1
    assert gg.class_of(0, 5, 0, -1) == (0, 0, -1)
    with pytest.raises(gg.GGError):
        gg.class_of(10, 0, 1)


def test_builtin_rules_without_table():
    gg.tune_set([])
    assert gg.tune_lookup(gg.ALGO_SSSP, 13, 2, 0) == (V, A, gg.MAP_BALANCED)
    assert gg.tune_lookup(gg.ALGO_BFS, 13, 0, 0) == (V, S, gg.MAP_BALANCED)
    assert gg.tune_lookup(gg.ALGO_BFS, 13, 0, 2) == (V, A, gg.MAP_BALANCED)
    assert gg.tune_lookup(gg.ALGO_CC, 13, 0, 2)[:2] == (E, S)


def test_lookup_takes_the_nearest_entry_of_the_algorithm():
    mk = lambda algo, sc, kc, dc, mode, sched, mp: dict(algo=algo, size_class=sc, skew_class=kc,
                                                       depth_class=dc, mode=mode, sched=sched,
                                                       mapping=mp)
    gg.tune_set([mk(0, 6, 2, 0, E, S, 0), mk(0, 12, 2, 0, V, A, 3), mk(0, 12, 0, 2, V, S, 1),
                 mk(1, 10, 0, -1, E, A, 0)])
    assert gg.tune_lookup(0, 13, 2, 0) == (V, A, 3)      # nearest size, same skew/depth
    assert gg.tune_lookup(0, 7, 2, 0) == (E, S, 3)       # mapping AUTO -> balanced
    assert gg.tune_lookup(0, 13, 0, 2) == (V, S, 1)      # skew and depth decide
    assert gg.tune_lookup(1, 3, 2, 1) == (E, A, 3)       # only entry of the algorithm
    assert gg.tune_lookup(2, 13, 0, 0)[:2] == (E, S)     # no CC entry: built-in
    assert len(gg.tune_get()) == 4


def test_table_validation():
    bad = dict(algo=3, size_class=1, skew_class=0, depth_class=0, mode=0, sched=0, mapping=0)
    with pytest.raises(gg.GGError):
        gg.tune_set([bad])
    bad.update(algo=0, mode=2)
    with pytest.raises(gg.GGError):
        gg.tune_set([bad])
    bad.update(mode=0, depth_class=-2)
    with pytest.raises(gg.GGError):
        gg.tune_set([bad])
    assert gg.lib().gg_tune_set(None, 2) == -1


def test_table_takes_only_runnable_schedules():
    """Near-far is an SSSP vertex schedule; the per-round dense/sparse choice
    is a BFS and SSSP vertex schedule and a CC schedule in either mode."""
    saved = gg.tune_get()
    try:
        def entry(algo, mode, sched):
            return dict(algo=algo, size_class=5, skew_class=0, depth_class=0, mode=mode,
                        sched=sched, mapping=3)
        for ok in (entry(0, 0, gg.NEARFAR), entry(1, 0, gg.DIROPT), entry(2, 1, gg.DIROPT),
                   entry(0, 0, gg.DIROPT), entry(2, 0, gg.DIROPT)):
            gg.tune_set([ok])
        for bad in (entry(1, 0, gg.NEARFAR), entry(0, 1, gg.DIROPT), entry(1, 1, gg.DIROPT),
                    entry(0, 1, gg.NEARFAR)):
            with pytest.raises(gg.GGError):
                gg.tune_set([bad])
    finally:
        gg.tune_set(saved)


def test_schedule_knobs_in_the_table():
    base = dict(algo=0, size_class=13, skew_class=0, depth_class=2, mode=V, sched=gg.NEARFAR,
                mapping=3, delta_eighths=32)
    gg.tune_set([dict(base, hops=32, far_degree=64),
                 dict(base, algo=1, sched=A, mapping=0, delta_eighths=0, hops=8)])
    assert gg.tune_lookup(0, 13, 0, 2, full=True) == dict(mode=V, sched=gg.NEARFAR, mapping=3,
                                                          delta_eighths=32, hops=32, far_degree=64)
    assert gg.tune_lookup(1, 13, 0, 2, full=True) == dict(mode=V, sched=A, mapping=3, delta_eighths=0,
                                                          hops=8, far_degree=0)
    # entries without the fields, and the built-in rules, set none of them
    gg.tune_set([base])
    e = gg.tune_lookup(0, 13, 0, 2, full=True)
    assert (e["delta_eighths"], e["hops"], e["far_degree"]) == (32, 0, 0)
    gg.tune_set([])
    e = gg.tune_lookup(0, 13, 0, 2, full=True)
    assert (e["delta_eighths"], e["hops"], e["far_degree"]) == (0, 0, 0)
    # out of range, or on a variant the knob does not apply to
    for bad in (dict(base, hops=-1), dict(base, hops=65), dict(base, sched=S, hops=2),
                dict(base, mode=E, sched=A, hops=2), dict(base, sched=A, mapping=1, hops=2),
                dict(base, far_degree=-1), dict(base, sched=A, far_degree=64),
                dict(base, delta_eighths=-1), dict(base, delta_eighths=(1 << 23) + 1)):
        with pytest.raises(gg.GGError):
            gg.tune_set([bad])


def test_calibration_ties_go_to_fewer_knobs():
    from paper_1903_01665_amd import tune
    plain = (V, A, 3, 0, 0, 0)
    nf = (V, gg.NEARFAR, 3, 3, 4, 64)
    cls = (13, 2, 0)

    def pick(t_plain, t_nf):
        entries, _ = tune.choose([("sssp", cls, {plain: t_plain, nf: t_nf})])
        e = entries[0]
        return (e["mode"], e["sched"], e["mapping"], e["delta_eighths"], e["hops"], e["far_degree"])

    assert pick(1.00, 0.98) == plain   # within 3 %: the plain worklist
    assert pick(1.00, 0.90) == nf      # a clear win keeps the knobs
    assert pick(0.90, 1.00) == plain
    # the score is the geometric mean over the graphs of the class
    entries, _ = tune.choose([("bfs", cls, {plain: 1.0, nf: 0.5}),
                              ("bfs", cls, {plain: 1.0, nf: 3.0})])
    assert (entries[0]["sched"], entries[0]["hops"]) == (A, 0)


def test_table_rederived_from_recorded_measurements(tmp_path):
    """tune.py --from-measurements rebuilds the entries from a table's
    recorded timings (no GPU): the best variant per class, ties to fewer
    knobs, every field of the chosen variant carried into the entry."""
    import json
    from paper_1903_01665_amd import tune
    ms = {"0/1/3/0/0/0": 2.00, "0/3/3/2/4/96": 1.50, "0/3/3/3/4/32": 1.52,
          "1/0/0/0/0/0": 4.0, "0/0/1/0/0/0": None}
    raw = {"measurements": [{"algo": "sssp", "class": [13, 2, 0], "ms": ms},
                            {"algo": "bfs", "class": [8, 0, 1],
                             "ms": {"0/1/3/0/0/0": 1.0, "0/1/3/0/8/0": 0.99}}]}
    src = tmp_path / "recorded.json"
    src.write_text(json.dumps(raw))
    out = tmp_path / "table.json"
    tune.main(["--from-measurements", str(src), "--out", str(out)])
    t = json.loads(out.read_text())
    by = {(e["algo"], e["size_class"]): e for e in t["entries"]}
    sssp = by[(0, 13)]
    # 1.50 beats 1.52 by less than the tie margin, and both have 3 knobs: the score decides
    assert (sssp["sched"], sssp["delta_eighths"], sssp["hops"], sssp["far_degree"]) == (3, 2, 4, 96)
    # a 1% win of local expansion is a tie: the plain worklist stays
    assert (by[(1, 8)]["sched"], by[(1, 8)]["hops"]) == (A, 0)
    # the measurements are kept (a failed run as null)
    assert t["measurements"][0]["ms"]["0/0/1/0/0/0"] is None
