"""Batched traversals: each instance's slice equals the oracle (bit-exact),
on the eager first run and on HIP-graph replays."""
import sys

import numpy as np
import pytest

import oracle
from paper_1903_01665_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_instances(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = rng.integers(0, 3)
        if kind == 0:
            s = int(rng.integers(6, 12))
            hg = gen.rmat(s, int(rng.integers(8, 33)) << s, stream=5000 + i, name=f"rmat{s}")
        elif kind == 1:
            n = int(rng.integers(1, 3000))
            hg = gen.uniform(n, int(rng.integers(0, 8 * n + 1)) if n > 1 else 0, 1, 100,
                             stream=6000 + i, name=f"er{n}")
        else:
            side = int(rng.integers(2, 40))
            hg = gen.grid(side, side, 0, 8, 1, 1000, stream=7000 + i, name=f"grid{side}")
        algo = int(rng.integers(0, 2))
        src = int(gen.pick_sources(hg, 1, stream=8000 + i)[0]) if hg.m > 0 else 0
        out.append((algo, hg, src))
    return out


def expected(instances):
    want = []
    for algo, hg, s in instances:
        if algo == 0:
            want.append(oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s))
        else:
            want.append(oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
    return want


def check(batch, instances, want, out):
    got = out.cpu().numpy()
    off = batch.offsets()
    for i, (algo, hg, s) in enumerate(instances):
        sl = got[off[i]: off[i] + hg.n]
        bad = np.flatnonzero(sl != want[i])
        assert bad.size == 0, (i, hg.name, algo, bad.size)


@pytest.fixture(scope="module")
def gg():
    import torch
    assert torch.cuda.is_available()
    from paper_1903_01665_amd import gg as _gg
    return _gg


@pytest.mark.parametrize("flags", [0, 1, 2])
def test_batch_matches_oracle_eager_and_replayed(gg, flags):
    import torch
    inst = make_instances(60, 11 + flags)
    want = expected(inst)
    b = gg.Batch(inst, flags=flags)
    try:
        info = b.info()
        assert info["total_n"] == sum(hg.n for _, hg, _ in inst)
        out = torch.full((info["total_n"],), -7, dtype=torch.int32, device="cuda")
        for rep in range(3):
            say(f"[gpu] batch flags={flags} rep={rep} groups={info['groups']}")
            out.fill_(-7)
            b.run(out)
            torch.cuda.synchronize()
            check(b, inst, want, out)
        groups = [b.group(i) for i in range(info["groups"])]
        assert sum(g["instances"] for g in groups) == 60
        if flags & 1 == 0:
            assert all(g["captured_rounds"] > 0 for g in groups)
        # a different output buffer forces an eager run and a new capture
        out2 = torch.zeros(info["total_n"], dtype=torch.int32, device="cuda")
        b.run(out2)
        b.run(out2)
        torch.cuda.synchronize()
        check(b, inst, want, out2)
    finally:
        b.free()


def test_batch_rejects_bad_instances(gg):
    hg = gen.uniform(10, 30, stream=3)
    with pytest.raises(gg.GGError):
        gg.Batch([(0, hg, 10)])       # source out of range
    with pytest.raises(gg.GGError):
        gg.Batch([(2, hg, 0)])        # CC is not a batch algorithm
    uw = gen.HostGraph(hg.n, hg.row_ptr, hg.col, None)
    with pytest.raises(gg.GGError):
        gg.Batch([(0, uw, 0)])        # SSSP without weights


@pytest.mark.parametrize("flags", [0, 1])
def test_batch_with_local_expansion(gg, flags):
    """Groups whose tuned variant expands locally (worklist SSSP and BFS
    with hops > 0) still give every instance's exact result, in the
    multi-source traversal of the group, eagerly and replayed; a near-far
    pick runs as the plain worklist."""
    import torch
    saved = gg.tune_get()
    entries = []
    for sc in range(0, 16):
        for kc in range(3):
            entries.append(dict(algo=0, size_class=sc, skew_class=kc, depth_class=-1, mode=0,
                                sched=gg.ASYNC if sc % 2 else gg.NEARFAR, mapping=3,
                                delta_eighths=16 if sc % 2 == 0 else 0, hops=8,
                                far_degree=4 if sc % 2 == 0 else 0))
            entries.append(dict(algo=1, size_class=sc, skew_class=kc, depth_class=-1, mode=0,
                                sched=gg.ASYNC, mapping=3, delta_eighths=0, hops=3))
    gg.tune_set(entries)
    try:
        inst = make_instances(40, 77 + flags)
        want = expected(inst)
        b = gg.Batch(inst, flags=flags)
    finally:
        gg.tune_set(saved)
    try:
        info = b.info()
        out = torch.full((info["total_n"],), -7, dtype=torch.int32, device="cuda")
        for rep in range(3):
            say(f"[gpu] batch local flags={flags} rep={rep} groups={info['groups']}")
            out.fill_(-7)
            b.run(out)
            torch.cuda.synchronize()
            check(b, inst, want, out)
    finally:
        b.free()


@pytest.mark.slow
def test_batch_at_full_scale_matches_the_oracle(gg):
    """The batched workload at its real size -- 512 R-MAT instances of scale
    10..18 and edge factor 8..32 (about 5.6e8 edges), half SSSP, half BFS --
    run as one batch (eager, then replayed from its HIP graphs): every
    instance's slice equals the oracle's result for it.  The oracle runs on
    a pool of host threads (each call releases the interpreter lock)."""
    import os
    import time
    from concurrent.futures import ThreadPoolExecutor

    import torch
    t = time.time()
    inst = gen.batch_instances(512)
    say(f"[gpu] batch full scale: {len(inst)} instances, "
        f"{sum(hg.m for _, hg, _ in inst)} edges generated in {time.time() - t:.1f}s")
    b = gg.Batch(inst)
    try:
        out = torch.full((b.total_n,), -7, dtype=torch.int32, device="cuda")
        b.run(out)
        torch.cuda.synchronize()
        first = out.cpu().numpy()
        out.fill_(-7)
        b.run(out)  # replayed from the captured graphs
        torch.cuda.synchronize()
        second = out.cpu().numpy()
        off = b.offsets()
    finally:
        b.free()
    t = time.time()
    workers = min(16, os.cpu_count() or 1)

    def one(k):
        algo, hg, s = inst[k]
        want = (oracle.sssp(hg.n, hg.row_ptr, hg.col, hg.w, s) if algo == 0
                else oracle.bfs(hg.n, hg.row_ptr, hg.col, s))
        a, z = off[k], off[k] + hg.n
        return (k, int(np.count_nonzero(first[a:z] != want)),
                int(np.count_nonzero(second[a:z] != want)))

    with ThreadPoolExecutor(max_workers=workers) as pool:
        res = list(pool.map(one, range(len(inst))))
    say(f"[gpu] batch full scale: oracle on {workers} threads in {time.time() - t:.1f}s")
    bad = [r for r in res if r[1] or r[2]]
    assert not bad, bad[:5]
