"""Host-side pieces of bench.py that feed the roofline fields: the
algorithmic bytes per node of each storage form and the calibration of the
rocprofv3 HBM counters against a copy of known size."""
import csv
import json

import pytest

import bench


def test_algorithmic_bytes_per_node():
    # 27 populations read and written once per node and step
    assert bench.alg_bytes_per_node("fp64") == 432
    assert bench.alg_bytes_per_node("fp32") == 216
    assert bench.alg_bytes_per_node("fp16dev") == 108
    # 26 FP16 deviations and the rest population in FP32
    assert bench.alg_bytes_per_node("fp16dev_f0fp32") == 2 * (26 * 2 + 4)


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, value in rows:
            w.writerow({"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})
        # a row of another counter must be ignored
        w.writerow({"Kernel_Name": "k_collide<0>", "Counter_Name": "SQ_WAVES", "Counter_Value": 1e9})


def test_counter_calibration(tmp_path):
    gib_kib = (1 << 30) / 1024.0
    copy = "__amd_rocclr_copyBuffer"
    # the counters read half the copy's bytes on fetch and all on write; a
    # smaller copy dispatch of the same run must not set the factor
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(copy, gib_kib / 2), (copy, 10.0), ("k_collide<0>", 1000.0), ("k_collide<0>", 1200.0),
                  ("k_moments<0>", 300.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(copy, gib_kib), (copy, 10.0), ("k_collide<0>", 500.0), ("k_collide<0>", 500.0),
                  ("k_moments<0>", 40.0)])
    out = tmp_path / "c.json"
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "fp64", "moving", str(out))
    c = json.load(open(out))
    assert c["copy_fetch_factor"] == pytest.approx(2.0)
    assert c["copy_write_factor"] == pytest.approx(1.0)
    assert c["fetch_kib_per_launch"] == pytest.approx(1100.0)
    assert c["bytes_per_launch"] == pytest.approx((1100.0 * 2.0 + 500.0) * 1024.0)
    assert c["kernels"]["fetch_kib"]["k_moments<0>"] == pytest.approx(300.0)
    # one step: the step-path kernels launched as often as the dominant one
    # (k_moments ran once here, as the initial refresh of the fused path does)
    assert c["kernels"]["launches"]["k_collide<0>"] == 2
    assert bench.step_kernels(c) == {"k_collide<0>"}
    assert c["source_hash"] == bench.kernel_source_hash()
    assert (c["form"], c["workload"]) == ("fp64", "moving")


def test_counter_calibration_needs_the_copy(tmp_path):
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [("k_collide<0>", 1000.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [("k_collide<0>", 500.0)])
    with pytest.raises(SystemExit):
        bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "fp64", "moving",
                                 str(tmp_path / "c.json"))


def test_adjoint_counter_summary(tmp_path):
    """Bytes per adjoint step: every adjoint-step dispatch, calibrated by the
    1 GiB copy, over the number of collision-adjoint dispatches; the seed and
    the forward kernels of the run are left out."""
    gib_kib = (1 << 30) / 1024.0
    copy = "__amd_rocclr_copyBuffer"
    k_c, k_p, k_r = "k_adj_collide<1, true, false>", "k_adj_phimu<1, false>", "k_adj_wall_gather"
    fetch = [(copy, gib_kib / 2), (k_c, 100.0), (k_c, 120.0), (k_p, 40.0), (k_p, 40.0),
             (k_r, 1.0), (k_r, 1.0), (k_r, 1.0), (k_r, 1.0), ("k_adj_seed<1>", 1e6), ("k_collide<1>", 1e6)]
    write = [(copy, gib_kib), (k_c, 50.0), (k_c, 50.0), (k_p, 10.0), (k_p, 10.0),
             (k_r, 2.0), (k_r, 2.0), (k_r, 2.0), (k_r, 2.0), ("k_adj_seed<1>", 1e6)]
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    out = tmp_path / "a.json"
    bench.summarize_adjoint_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out))
    c = json.load(open(out))
    assert c["adjoint_steps"] == 2
    per_step_kib = ((100 + 120 + 40 + 40 + 4 * 1.0) * 2.0 + (50 + 50 + 10 + 10 + 4 * 2.0)) / 2
    assert c["bytes_per_adjoint_step"] == pytest.approx(per_step_kib * 1024.0)
    assert c["kernels_bytes_per_step"]["k_adj_wall_gather"]["WRITE_SIZE"] == pytest.approx(4 * 2.0 * 1024.0 / 2)
    assert c["source_hash"] == bench.kernel_source_hash()
    adj = {"ms_per_adjoint_step": 0.5}
    bench.ADJ_COUNTERS, saved = str(out), bench.ADJ_COUNTERS
    try:
        bench.adjoint_achieved(adj)
    finally:
        bench.ADJ_COUNTERS = saved
    assert adj["achieved_frac"] == pytest.approx(per_step_kib * 1024.0 / 0.5e-3 / 1e9 / bench.HBM_PEAK_GBS)


def test_step_kernels_of_the_two_pass_path():
    """On the two-pass path every step launches the moments, chain,
    wall-density and collide-stream kernels once; the initialiser's kernels
    ran once in the whole run and are not part of a step."""
    n = 5
    launches = {"k_moments<1>": n, "k_chain<1, true>": n, "k_wall_rho": n, "k_collide<1>": n,
                "k_init<1>": 1, "k_mu": 1, "__amd_rocclr_copyBuffer": 7}
    c = {"dominant_kernel": "k_collide<1>", "kernels": {"launches": launches}}
    assert bench.step_kernels(c) == {"k_moments<1>", "k_chain<1, true>", "k_wall_rho", "k_collide<1>"}


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
