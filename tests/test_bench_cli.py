"""bench.py's command line on the CPU: the one-GPU build refuses --gpus N > 1
with a message, before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_model():
    """The per-unit byte figures of the roofline (documented beside the
    kernels): a vertex-async SSSP round over E edges, V vertices, P pushes."""
    sys.path.insert(0, ROOT)
    import bench
    prof = {"edges_processed": 1000, "vertices_processed": 100, "updates": 0, "pushes": 50,
            "swept_edges": 0}
    n = 6400
    # tile flags per launch + 16 B per vertex + 12 B per edge + 2 B per push
    assert bench.algorithmic_bytes("sssp", 0, 1, "round", n, prof, 2) == \
        2 * (n // 64) + 16 * 100 + 12 * 1000 + 2 * 50
    assert bench.algorithmic_bytes("sssp", 0, 1, "heavy", n, prof, 2) == 12 * 1000 + 2 * 50
    # edge sweep: 20 B per SSSP edge, 16 B per BFS/CC edge, 4 B per update
    prof["updates"] = 7
    assert bench.algorithmic_bytes("cc", 1, 0, "round", n, prof, 3) == 16 * 1000 + 4 * 7
    # CC per-round schedule: swept edges at 16 B, the rest at 8 B
    prof["swept_edges"] = 600
    assert bench.algorithmic_bytes("cc", 1, 4, "round", n, prof, 3) == \
        16 * 600 + 8 * 400 + 16 * 100 + 3 * (n // 64) + 4 * 7 + 10 * 50


def test_traffic_summary_is_keyed_to_the_kernel_code():
    """The committed HBM traffic summary stays valid across comment edits of
    the kernel source and is dropped when the code changes."""
    import bench
    src = "__global__ void k(int* p) {\n    p[0] = 1;  // store\n}\n"
    h = bench.kernel_code_hash(src)
    assert bench.kernel_code_hash("// header\n" + src + "\n/* block\n comment */\n") == h
    assert bench.kernel_code_hash(src.replace("// store", "// a different note")) == h
    assert bench.kernel_code_hash(src.replace("p[0] = 1", "p[0] = 2")) != h
    csrc = bench.os.path.join(bench.ROOT, "paper_1903_01665_amd", "csrc")
    both = "".join(open(bench.os.path.join(csrc, f)).read() + "\n"
                   for f in ("gg_internal.h", "gg_kernels.hip"))
    assert bench.kernel_code_hash() == bench.kernel_code_hash(both)


def test_tuned_rmat22_kernels_are_in_the_traffic_summary():
    """The kernels the tuned variants of rmat22's class launch carry the
    symbols under which the committed HBM traffic summary lists them, so the
    bench's roofline finds its traffic figure."""
    import json
    import bench
    from paper_1903_01665_amd import gg
    summary = json.load(open(bench.os.path.join(bench.ROOT, "profiles",
                                                "hbm_traffic_rmat22.json")))
    keys = set(summary["bytes_per_dispatch"])
    for ai, algo in enumerate(bench.ALGOS):
        # rmat22: m = 2^26, hub degree 159873, 7 levels
        e = gg.tune_lookup(ai, *gg.class_of(1 << 26, 1 << 22, 159873, 7), full=True)
        for kind in ("round", "heavy"):
            sym = bench.kernel_symbol(algo, kind, e["mode"], e["sched"], e["mapping"], e["hops"])
            if sym is None:  # no kernel of this kind (union-find CC has no chunk kernel)
                assert e["sched"] == 5 and kind == "heavy", (algo, kind, e)
                continue
            assert sym in keys, (algo, kind, e, sym)
