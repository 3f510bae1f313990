"""Host logic of bench.py: the one-GPU guard and the roofline accounting
(algorithmic bytes and FLOPs per launch, the dominant kernel, its fraction of
the peak), on synthetic work counts; no GPU needed."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counts(block_fp64=0, block_mixed=0):
    # 10 real elements (4 general), 3 fields each on average, 30 face slots
    return dict(real_elements=10, general_elements=4, fields=30, slots=30, ndof=1000,
                face_coef_doubles=5000, block_bytes_fp64=block_fp64, block_bytes_mixed=block_mixed)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_update_bytes_count_vectors_and_stored_blocks():
    b = _bench()
    W = 2
    plain = b.kernel_work(_counts(), W)
    blocks = b.kernel_work(_counts(123456, 61728), W, fp32=False, block_precond=True)
    blocks32 = b.kernel_work(_counts(123456, 61728), W, fp32=True, block_precond=True)
    # r in and z out, FP64, per unknown
    assert plain["update"] == (0.0, 16.0 * 1000)
    assert blocks["update"][1] == 16.0 * 1000 + 123456
    assert blocks32["update"][1] == 16.0 * 1000 + 61728
    # the operator kernels do not depend on the preconditioner
    for k in ("volume", "face", "gather"):
        assert blocks[k] == plain[k]


def test_volume_flops_formula():
    b = _bench()
    W = 3
    n, m = W + 1, 2 * W + 1
    c = _counts()
    Ed, Eg, nf = 6, 4, 30
    want = 4 * (Ed * (2 * m * n ** 3 + 3 * m * m * n * n) + Eg * (3 * m * n ** 3 + 6 * m * m * n * n)
                + nf * m ** 3 * n) + 3 * nf * m ** 3
    assert b.kernel_work(c, W)["volume"][0] == pytest.approx(want)
    # float halves the operator bytes but not the FP64 vector bytes
    v64 = b.kernel_work(c, W)["volume"][1]
    v32 = b.kernel_work(c, W, fp32=True)["volume"][1]
    assert v32 < v64 and v64 - v32 == pytest.approx(4 * (nf * m ** 3 + c["slots"] * 4 * n * n))


def test_roofline_entry_of_the_dominant_kernel():
    b = _bench()
    W = 2
    c = _counts(8_000_000, 4_000_000)
    ms = [0.5, 0.2, 0.05, 1.0]                     # the update kernel dominates
    r = b.roofline(c, W, ms, fp32=True, block_precond=True)
    by = 16.0 * 1000 + 4_000_000
    assert r["kernel"] == "k_update_mfma"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(by / 1e-3 / 1e9)
    assert r["peak"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["avg_ms"] == 1.0 and r["algorithmic_bytes"] == by
    # with the separable preconditioner the same kernel is k_update
    r2 = b.roofline(_counts(), W, ms, fp32=False, block_precond=False)
    assert r2["kernel"] == "k_update"
    assert set(r2["all_kernels"]) == {"volume", "face", "gather", "update"}
