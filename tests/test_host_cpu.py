"""CPU checks of the host-side logic: input generators, the autotuner's
search space, the bench's traffic bookkeeping, and the tuning structure
the binding passes across the C ABI."""
import ctypes
import importlib.util
import os
import re

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batch_suite_is_deterministic_and_worker_independent():
    a = gg.batch_suite(count=6, seed0=4000, scale_max=10)
    b = gg.batch_suite(count=6, seed0=4000, scale_max=10, workers=2)
    assert [g.sha256() for g in a] == [g.sha256() for g in b]
    assert len({g.name[:2] for g in a}) == 2          # R-MAT and Erdos-Renyi mixed


def test_serve_suite_shape():
    big = gg.rmat(9, 8, seed=1)
    gs = gg.serve_suite(count=5, seed0=5000, scale_min=8, scale_max=9, big=big)
    assert len(gs) == 5 and gs[-1] is big
    assert all(g.n in (256, 512) for g in gs[:-1])


def test_chung_lu_sampling_keeps_the_degree_law():
    g = gg.chung_lu(n=1 << 14, mean_degree=20.0, w_max=600.0, planted=0, seed=3)
    d = g.degrees()
    assert 15.0 < d.mean() < 21.0                     # duplicates merged: at most the mean
    assert d.max() > 10 * d.mean()                    # heavy tail


def test_autotune_candidates_cover_the_space():
    from paper_2112_10913_amd.autotune import candidates, signature, MAX_WAVES_PER_CU
    c = candidates({"wg_waves": [2, 8], "blocks_per_cu": [1, 4], "flush_rows": [128],
                    "arc_lds_max": [128, 256], "split_pct": [50, 100]})
    assert all(t.wg_waves * t.blocks_per_cu <= MAX_WAVES_PER_CU for t in c)
    assert len(c) == 3 * 2 * 2                        # 8 x 4 waves per CU is dropped
    assert {t.split_pct for t in c} == {50, 100} and {t.arc_lds_max for t in c} == {128, 256}

    class G:
        def __init__(self, n, m):
            self.n, self.m = n, m
    assert signature([G(3, 4)], [5]) != signature([G(3, 4)], [6])


def test_tuning_struct_matches_the_header():
    from paper_2112_10913_amd._lib import _Tuning, Tuning
    text = open(os.path.join(ROOT, "include", "citron.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} citron_tuning;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert [f for f, _ in _Tuning._fields_] == fields
    assert ctypes.sizeof(_Tuning) == 4 * len(fields)
    assert set(Tuning().__dict__) == set(fields) - {"size"}


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_digest_ignores_comments(tmp_path):
    b = _bench()
    p1, p2, p3 = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    p1.write_text("int f() {  // one\n  return 1;\n}\n")
    p2.write_text("// header\nint f() {\n\n  return 1;   // two\n}\n")
    p3.write_text("int f() {\n  return 2;\n}\n")
    assert b.kernel_digest(str(p1)) == b.kernel_digest(str(p2)) != b.kernel_digest(str(p3))


def test_traffic_summary_bookkeeping():
    b = _bench()
    text = open(os.path.join(ROOT, "profiles", "count_kernel_rmat20_hbm.md")).read()
    rec = re.search(r"kernel code sha256: `([0-9a-f]+)`", text).group(1)
    digest = b.kernel_digest(os.path.join(ROOT, "paper_2112_10913_amd", "csrc", "kernels_count.hip"))
    assert b.traffic_per_launch([5, 6]) is None        # other k sets have no figure
    if rec != digest:
        pytest.skip("the HBM counter summary was taken on other kernel code: traffic is reported as null")
    v = b.traffic_per_launch([5, 6, 7])
    assert v is not None and v > 0


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: the refusal comes before anything touches a device
    import subprocess
    import sys
    root = ROOT
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv], capture_output=True,
                           text=True, timeout=120, env={**os.environ, **env})
        assert r.returncode == 2, r.stderr
        assert "one GPU only" in r.stderr
        assert r.stdout == ""


def test_served_latency_breakdown():
    b = _bench()
    req = [(0, 3), (1, 5), (0, 3), (1, 5), (0, 4)]
    ms = [1.0, 10.0, 3.0, 30.0, 7.0]
    res = [{"tag": i, "t_submit_ns": 1000, "t_done_ns": 1000 + int(x * 1e6)} for i, x in enumerate(ms)]
    out = b.latency_breakdown(req, res[::-1], ["rmat12", "rmat16"])
    assert [(e["graph"], e["k"], e["n"]) for e in out] == [("rmat12", 3, 2), ("rmat12", 4, 1), ("rmat16", 5, 2)]
    assert out[0]["p50_ms"] == 2.0 and out[1]["p99_ms"] == 7.0
    assert abs(out[2]["p99_ms"] - (10.0 + 0.99 * 20.0)) < 1e-9


@pytest.mark.parametrize("name", ["rmat14", "rmat20", "chunglu22"])
def test_config_graphs_match_their_golden_files(name):
    # the stored oracle values hold for exactly the graph the generator
    # gives today (numpy PCG64 streams and the cleaning steps)
    import json
    with open(os.path.join(ROOT, "tests", "golden", f"{name}.json")) as f:
        gold = json.load(f)
    g = gg.config_graph(name)
    assert (g.n, g.m) == (gold["n"], gold["m"])
    assert g.sha256() == gold["sha256"]


class _StubGraph:
    """Stands in for a device graph: only the tuning the autotuner sets."""

    def __init__(self, n, m):
        from paper_2112_10913_amd import Tuning
        self.n, self.m = n, m
        self.t = Tuning(split_pct=100)

    def get_tuning(self):
        from dataclasses import replace
        return replace(self.t)

    def set_tuning(self, t):
        self.t = t


def test_autotune_picks_the_fastest_caches_it_and_rejects_changed_counts(tmp_path, monkeypatch):
    import paper_2112_10913_amd.autotune as at
    from paper_2112_10913_amd import CitronError, Tuning
    calls = []

    def fake_batch(graphs, ks, tuning=None):
        calls.append(tuning)
        if tuning.wg_waves == 8:
            raise CitronError(1, "refused")
        if tuning.wg_waves == 1 and tuning.blocks_per_cu == 2:
            at.time.sleep(0)                                 # the fast one
        else:
            at.time.sleep(0.01 * tuning.wg_waves)
        return [7] * len(ks)

    monkeypatch.setattr(at, "count_batch", fake_batch)
    monkeypatch.setattr(at, "device_info", lambda: {"arch": "gfx950", "cus": 256, "lds_bytes": 163840})
    gs = [_StubGraph(10, 20), _StubGraph(30, 40)]
    trials = [Tuning(wg_waves=w, blocks_per_cu=b, split_pct=s)
              for w, b, s in ((4, 2, 100), (1, 2, 50), (8, 1, 100), (2, 2, 200))]
    cache = str(tmp_path / "tune.json")
    best, rep = at.autotune(gs, [5, 6], reps=3, cache_path=cache, tunings=trials)
    assert (best.wg_waves, best.blocks_per_cu, best.split_pct) == (1, 2, 50)
    assert all(g.t.split_pct == 50 for g in gs)               # the schedule is set on the graphs
    assert [t["seconds"] is None for t in rep["trials"]] == [False, False, True, False]
    n_calls = len(calls)
    again, rep2 = at.autotune(gs, [5, 6], cache_path=cache, tunings=trials)
    assert rep2["cached"] and again == best and len(calls) == n_calls

    def changing(graphs, ks, tuning=None):
        return [tuning.wg_waves] * len(ks)
    monkeypatch.setattr(at, "count_batch", changing)
    with pytest.raises(RuntimeError, match="changed a count"):
        at.autotune(gs, [5, 6], reps=1, use_cache=False, tunings=trials[:2])


def test_cpu_baseline_line():
    b = _bench()
    g = gg.rmat(12, 16, seed=5)
    cb = b.cpu_baseline(g, 4, budget_s=0.5, workers=3)
    assert set(cb) >= {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["cores"] == 3 and cb["unit"] == "edges/s"
    assert cb["value"] > 0 and "mod" in cb["sample"] and cb["stride"] >= 3
    assert abs(cb["value"] * cb["est_full_graph_s"] - g.m) < 1e-6 * g.m


def test_alg_bytes_model():
    b = _bench()
    gold = {"work_model": {"5": {"kept_sum_duv": 10, "kept_sum_dw": 20, "kept_sum_s": 3, "arcs_kept": 2}}}
    assert b.alg_bytes(gold, 5) == 4 * 10 + 4 * 20 + 8 * (3 + 2)
    assert b.alg_bytes(gold, 6) is None and b.alg_bytes(None, 5) is None
    # the stored R-MAT 20 model: 2.95e11 bytes at k = 5
    assert abs(b.alg_bytes(b.load_golden("rmat20"), 5) - 2.953e11) < 1e9
