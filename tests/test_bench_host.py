"""Host-side logic of bench.py and the profile readers (no GPU)."""
import argparse
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_summary_is_tied_to_the_kernel_source():
    from paper_0911_4114_amd.profiling import file_sha256, read_traffic
    bench = load_bench()
    args = argparse.Namespace(n=1 << 20, kappa=177.0, eps=1e-4)
    rel, kernel = bench.TRAFFIC_FILES["p2p"]
    t = read_traffic(os.path.join(ROOT, rel))
    assert t["kernel"] == kernel
    assert float(t["fetch_scale"]) == pytest.approx(2.0, rel=1e-3)
    assert float(t["write_scale"]) == pytest.approx(1.0, rel=1e-3)
    hbm = 1024.0 * (float(t["fetch_kib_per_dispatch"]) * float(t["fetch_scale"])
                    + float(t["write_kib_per_dispatch"]) * float(t["write_scale"]))
    assert float(t["hbm_bytes_per_dispatch"]) == pytest.approx(hbm, rel=1e-4)   # scales printed to 4 digits
    got = bench.measured_traffic("p2p", args)
    same = t["source_sha256"] == file_sha256(os.path.join(ROOT, t["source"]))
    assert (got == pytest.approx(float(t["hbm_bytes_per_dispatch"]))) if same else got is None
    # other workloads and stages carry no measured traffic
    assert bench.measured_traffic("p2p", argparse.Namespace(n=4096, kappa=177.0, eps=1e-4)) is None
    assert bench.measured_traffic("m2m", args) is None


def test_bench_refuses_more_than_one_gpu(monkeypatch, capsys):
    bench = load_bench()
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_stage_roofline_takes_the_largest_bound():
    """Each stage's roofline time is the largest of FLOPs / peak, transcendentals / rate and
    bytes / HBM bandwidth, and its fraction is that time over the measured one."""
    bench = load_bench()
    info = {"depth": 3, "n_points": 1000, "precision": 1, "K": [0, 0, 400, 100],
            "n_boxes": [1, 8, 64, 512], "n_ilist": [0, 0, 200, 5000], "n_near_pairs": 10 ** 6}
    for st in ("p2m", "l2p", "p2p", "m2l", "m2m", "l2l", "gather", "scatter"):
        w = bench.stage_work(info, st)
        r = bench.stage_roofline(info, st, 1.0)
        t = {"alu": w["flops"] / (w["peak"] * 1e12), "trans": w["trans"] / (bench.TRANS_PEAK_TPS * 1e12),
             "hbm": w["bytes"] / (bench.HBM_PEAK_GBS * 1e9)}
        assert r["bound"] == max(t, key=t.get)
        assert r["roofline_ms"] == pytest.approx(round(1e3 * max(t.values()), 4), abs=1e-4)
        assert r["frac"] == pytest.approx(max(t.values()) / 1e-3)
    # M2L: 8 flops per interaction-list entry and direction over every level
    assert bench.stage_work(info, "m2l")["flops"] == 8.0 * (200 * 400 + 5000 * 100)
    assert bench.stage_work(info, "leaf_m2l")["flops"] == 8.0 * 5000 * 100
