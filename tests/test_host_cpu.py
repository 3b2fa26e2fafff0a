"""Host-side logic that needs no GPU: generators, workload recipes, tuner keys, serving stats."""
import os
import subprocess
import sys

import numpy as np

import graphgen as gg
import graphgen.workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_generators_are_deterministic_across_thread_counts():
    code = ("import sys; sys.path.insert(0, %r); import graphgen as gg, hashlib;"
            "g = gg.rmat(14, 16, seed=3); e = gg.erdos_renyi(5000, 40000, seed=2);"
            "print(hashlib.sha1(g.src.tobytes() + g.dst.tobytes() + e.src.tobytes() + e.dst.tobytes()).hexdigest())"
            % ROOT)
    outs = set()
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.add(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert len(outs) == 1


def test_rmat_shape_and_skew():
    g = gg.rmat(12, 16, seed=1)
    assert g.n == 4096 and g.m_in == 16 * 4096
    assert int(g.src.max()) < g.n and int(g.dst.max()) < g.n
    # quadrant a (both bits 0) is the most likely: low ids dominate
    assert (g.src < 2048).mean() > 0.7


def test_ba_edge_count_and_distinct_targets():
    for n, k in [(10, 4), (500, 3), (2000, 16)]:
        g = gg.barabasi_albert(n, k, seed=5)
        assert g.m_in == (k + 1) * k // 2 + (n - k - 1) * k
        pairs = set(zip(g.src.tolist(), g.dst.tolist()))
        assert len(pairs) == g.m_in  # no repeated pair, no self-loop
        assert all(a != b for a, b in pairs)


def test_batch_spec_recipe():
    sp = W.batch_spec(4096, seed=1)
    assert sp == W.batch_spec(4096, seed=1)
    kinds = [s[0] for s in sp]
    assert kinds[::2] == ["er"] * 2048 and kinds[1::2] == ["ba"] * 2048
    ns = np.array([s[1] for s in sp])
    ks = np.array([s[2] for s in sp])
    assert ns.min() >= 100 and ns.max() <= 50000 and 4 <= ks.min() and ks.max() <= 16
    # log-uniform: median near the geometric mean of the range
    assert 1500 < np.median(ns) < 3000


def test_serving_pool_and_arrivals():
    sp = W.serving_pool(40, seed=7)
    assert [s[0] for s in sp[:4]] == ["rmat", "ba", "rmat", "ba"]
    assert all(10 <= s[1] <= 20 for s in sp if s[0] == "rmat")
    t = W.poisson_arrivals(2000.0, 2.0, seed=11)
    assert np.all(np.diff(t) >= 0) and t[-1] < 2.0
    assert abs(len(t) - 4000) < 5 * np.sqrt(4000)


def test_tuner_feature_key():
    from paper_2103_08053_amd.autotune import feature_key
    from paper_2103_08053_amd.tc import GraphInfo
    a = GraphInfo(n=4194304, m=64153814, wedges_plus=28919811070, max_dplus=1053, n_hub=0, n_wg=1, n_wave=1,
                  wave_cap=1, wg_cap=1)
    assert feature_key(a, True) == "n22_m26_d10_w9_pv1_k0"
    assert feature_key(a, False, 4096) == "n22_m26_d10_w9_pv0_k12"


def test_serving_summary():
    from paper_2103_08053_amd.serve import Request, summarize

    class T:
        def __init__(self, n):
            self.n = n

        def numel(self):
            return self.n

    reqs = [Request(i, 10, T(100), T(100), arrival=0.1 * i, done=0.1 * i + 0.01 * (i + 1)) for i in range(10)]
    st = summarize(reqs, 2.0, 3)
    assert st["requests"] == 10 and abs(st["throughput_rps"] - 5.0) < 1e-9
    assert abs(st["p50_ms"] - 55.0) < 1e-6 and st["p99_ms"] > 99.0


def test_algorithmic_bytes_formula():
    sys.path.insert(0, ROOT)
    import bench
    # 32-bit offsets: 4n (u bounds) + 4m (u lists) + 8m (out-neighbour bounds) + 4 W+ + 8 (+ 8n counts)
    assert bench.algorithmic_bytes(10, 20, 300, False) == 40 + 80 + 160 + 1200 + 8
    assert bench.algorithmic_bytes(10, 20, 300, True) == 40 + 80 + 160 + 1200 + 8 + 80


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_tuner_flag_knobs_compose():
    """The vertex-order and intra-vertex knobs live in the flags: setting one keeps the other bits,
    and every combination the space can produce is accepted by the library's parameter check."""
    from paper_2103_08053_amd import Params, autotune
    from paper_2103_08053_amd.tc import _Params, load_library
    p = Params(flags=0x1)  # keep rank order
    q = autotune._with(autotune._with(p, "order", 0x80), "intra", 0x200)
    assert q.flags == 0x1 | 0x80 | 0x200
    assert autotune._get(q, "order") == 0x80 and autotune._get(q, "intra") == 0x200
    q = autotune._with(q, "order", 0x40)
    assert q.flags == 0x1 | 0x40 | 0x200
    assert autotune._get(q, "slots_per_bucket") == q.slots_per_bucket
    lib = load_library()
    import ctypes
    for order in autotune.SPACE["order"]:
        for intra in autotune.SPACE["intra"]:
            cp = _Params()
            lib.tc_default_params(ctypes.byref(cp))
            cp.flags = order | intra
            h = ctypes.c_void_p()
            # parameters are checked before any device is touched
            st = lib.tc_create(0, ctypes.byref(cp), ctypes.byref(h))
            assert st != 1, (order, intra)  # TC_E_INVALID would mean the check rejects them
            if st == 0:
                lib.tc_destroy(h)


def test_measured_traffic_needs_matching_source_workload_and_mode(tmp_path, monkeypatch):
    import bench
    for w in ("rmat22", "er25", "rmat26"):
        t = bench.measured_traffic(True, w)
        if t is not None:  # committed profile taken on the current kernel source
            assert t > 0
    assert bench.measured_traffic(True, "rmat16") is None  # no profile for it
    f = tmp_path / "summary.md"
    sha = bench.kernel_source_sha1()

    def summary(src, mode, workload):
        f.write_text(f"- kernel_source_sha1: `{src}`\n- per_vertex: {mode}\n- workload: {workload}\n"
                     "- traffic_bytes_per_launch: 123\n")

    monkeypatch.setattr(bench, "pmc_summary", lambda w: str(f))
    summary(sha, True, "er25")
    assert bench.measured_traffic(True, "er25") == 123
    assert bench.measured_traffic(False, "er25") is None
    assert bench.measured_traffic(True, "rmat22") is None
    summary("0" * 40, True, "er25")
    assert bench.measured_traffic(True, "er25") is None
