"""The benchmark script's host-side contract, without a GPU: the one-GPU
refusal, the per-particle work figures behind its roofline, and the traffic
record it builds from two hardware-counter runs."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def separable_fma(I, gradient):
    """FMAs per particle of the separable tensor-product sum (Sec. 2.2) for
    three components, counted stage by stage: the x1 contraction of every
    (x3, x2) row, the x2 contraction of every plane, the x3 contraction, and
    Horner's rule for each weight polynomial (I coefficients, I - 1 FMAs).
    With the gradient the x1 stage also contracts with the derivative
    weights, the x2 stage forms three combinations and the x3 stage four."""
    rows, planes = I * I, I
    if not gradient:
        return 3 * (rows * I + planes * I + I) + 3 * I * (I - 1)
    return 3 * (2 * rows * I + 3 * planes * I + 4 * I) + 3 * 2 * I * (I - 1)


def test_roofline_work_figures(bench):
    assert bench.FLOP_VALUE_I8 == 2 * separable_fma(8, False) == 3840
    assert bench.FLOP_GRAD_I8 == 2 * separable_fma(8, True) == 8160
    # 1024^3 FP32 nodes of 3 components read once, 24-byte positions read,
    # 12 bytes of velocity (and 36 of gradient) written per particle
    assert bench.algorithmic_bytes(1024, 10 ** 8, 12, 12) == 1024 ** 3 * 12 + 10 ** 8 * 36
    assert bench.algorithmic_bytes(1024, 10 ** 8, 12, 48) == 20_084_901_888
    # learned form: forward 195-128-128, backward dh1, dW2 and dW1 products
    assert bench.TRAIN_MFMA_FLOP_PER_PAIR == 2 * 128 * (195 + 128) + 2 * 128 * 128 * 2 + 2 * 195 * 128


def _counter_run(d, counter, values):
    os.makedirs(d)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, vals in values.items():
            for v in vals:
                w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_record(bench, tmp_path, monkeypatch, capsys):
    record = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(record))
    copy = "void at::native::bitwise_not_kernel(int*)"
    grad = "void ptk::k_interp<1, 8, true, false>(ptk::InterpArgs)"
    val = "void ptk::k_interp<1, 8, false, false>(ptk::InterpArgs)"
    # FETCH_SIZE counts half of the copy's 1 GiB, WRITE_SIZE all of it (KiB)
    _counter_run(str(tmp_path / "fetch"), "FETCH_SIZE", {copy: [524288.0], grad: [1000.0, 3000.0], val: [500.0]})
    _counter_run(str(tmp_path / "write"), "WRITE_SIZE", {copy: [1048576.0], grad: [400.0], val: [100.0]})
    bench.summarize_pmc(str(tmp_path / "fetch"), str(tmp_path / "write"))
    capsys.readouterr()
    rec = json.loads(record.read_text())
    assert rec["copy_fetch_factor"] == pytest.approx(0.5)
    assert rec["copy_write_factor"] == pytest.approx(1.0)
    # mean KiB per dispatch, scaled by the copy's factor, in bytes
    assert rec["interp_grad_fetch"] == pytest.approx(2000.0 * 1024 / 0.5)
    assert rec["interp_grad"] == pytest.approx(2000.0 * 1024 / 0.5 + 400.0 * 1024)
    assert rec["interp"] == pytest.approx(500.0 * 1024 / 0.5 + 100.0 * 1024)
    # the record is reported only for the kernel source it was taken on
    assert bench.traffic_for("interp_grad") == pytest.approx(rec["interp_grad"])
    rec["kernel_sha"] = "0" * 16
    record.write_text(json.dumps(rec))
    assert bench.traffic_for("interp_grad") is None
