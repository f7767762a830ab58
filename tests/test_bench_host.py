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


def _counter_csv(path, rows):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for d, name, counter, value in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": 256, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_total_sums_a_kernel_group_per_call(tmp_path):
    """traffic-total: the scaled FETCH_SIZE + WRITE_SIZE of every dispatch of the group (name
    prefixes, instances of one dispatch summed), over the number of calls of the reference kernel;
    other kernels are left out."""
    from argparse import Namespace
    from paper_0911_4114_amd.profiling import traffic_total
    k1 = "void ffmm::(anonymous namespace)::rs1_mfma<float, false, 16>(long)"
    k2 = "void ffmm::(anonymous namespace)::rs5q_mfma<float, true, 32>(long)"
    other = "void ffmm::(anonymous namespace)::l2p_kernel<float>(int)"
    ref = "void ffmm::(anonymous namespace)::p2p_kernel<float, HIP_vector_type<float, 2u>, false, false, 1>(double)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = [(1, ref, "FETCH_SIZE", 1.0), (2, k1, "FETCH_SIZE", 10.0), (2, k1, "FETCH_SIZE", 6.0),
             (3, k2, "FETCH_SIZE", 20.0), (4, other, "FETCH_SIZE", 1000.0), (5, ref, "FETCH_SIZE", 1.0),
             (6, k1, "FETCH_SIZE", 8.0)]
    write = [(1, ref, "WRITE_SIZE", 1.0), (2, k1, "WRITE_SIZE", 4.0), (3, k2, "WRITE_SIZE", 2.0),
             (4, other, "WRITE_SIZE", 500.0), (5, ref, "WRITE_SIZE", 1.0), (6, k1, "WRITE_SIZE", 2.0)]
    _counter_csv(tmp_path / "f.csv", fetch)
    _counter_csv(tmp_path / "w.csv", write)
    # copy probe: 2048 bytes moved, FETCH reads half (1 KiB), WRITE all (2 KiB): scales 2 and 1
    _counter_csv(tmp_path / "cf.csv", [(1, copy, "FETCH_SIZE", 1.0)])
    _counter_csv(tmp_path / "cw.csv", [(1, copy, "WRITE_SIZE", 2.0)])
    a = Namespace(prefix=["rs1_mfma", "rs5q_mfma"], per="p2p_kernel<float, float2, false, false, 1>",
                  fetch=str(tmp_path / "f.csv"), write=str(tmp_path / "w.csv"),
                  copy_fetch=str(tmp_path / "cf.csv"), copy_write=str(tmp_path / "cw.csv"), copy_bytes=2048,
                  copy_kernel=copy)
    out = dict(line.split(": ") for line in traffic_total(a).splitlines())
    assert int(out["calls"]) == 2
    # fetch (10 + 6 + 20 + 8) KiB x 2 + write (4 + 2 + 2) KiB x 1, over 2 calls
    assert float(out["hbm_bytes_per_call"]) == pytest.approx(1024.0 * (2 * 44 + 8) / 2)
