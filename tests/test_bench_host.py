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
