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
    # 10 real elements (4 general), 3 fields each on average, 30 face slots, 12 face terms
    return dict(real_elements=10, general_elements=4, fields=30, slots=30, faces=12, ndof=1000,
                face_coef_doubles=5000, block_bytes_fp64=block_fp64, block_bytes_mixed=block_mixed)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_update_work_is_the_methods_preconditioner():
    """The preconditioner step counts 12 n^4 + n^3 FLOPs per element and the
    r / z vectors, whatever block data a preconditioner stores."""
    b = _bench()
    W = 2
    n = W + 1
    plain = b.kernel_work(_counts(), W)
    blocks = b.kernel_work(_counts(123456, 61728), W, fp32=True)
    assert plain["update"] == (10.0 * (12 * n ** 4 + n ** 3), 16.0 * 1000)
    assert blocks["update"] == plain["update"]
    for k in ("volume", "face", "gather"):
        assert blocks[k][0] == plain[k][0]


def test_face_flops_formula():
    b = _bench()
    W = 3
    n, m = W + 1, 2 * W + 1
    want = 12 * (32 * (m * n * n + m * m * n) + 16 * m ** 3 + 12 * m * m)
    assert b.kernel_work(_counts(), W)["face"][0] == pytest.approx(want)


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
    n = W + 1
    c = _counts(8_000_000, 4_000_000)
    ms = [0.5, 0.2, 0.05, 1.0]                     # the update kernel dominates
    r = b.roofline(c, W, ms, fp32=True, block_precond=True, ms_per_step=2.0)
    by = 16.0 * 1000
    fl = 10.0 * (12 * n ** 4 + n ** 3)
    assert r["kernel"] == "k_update_mfma"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(by / 1e-3 / 1e9)
    assert r["peak"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["avg_ms"] == 1.0 and r["algorithmic_bytes"] == by and r["algorithmic_flops"] == fl
    # the stored block stream is reported beside it, not as algorithmic work
    assert r["block_stream"]["stream_gbps"] == pytest.approx(4_000_000 / 1e-3 / 1e9)
    # the whole iteration against the time per step
    ifl, iby = b.iteration_work(c, W, fp32=True)
    assert r["iteration"]["achieved"] == pytest.approx(iby / 2e-3 / 1e9)
    assert iby == pytest.approx(sum(v[1] for v in b.kernel_work(c, W, True).values()) + 7 * 8 * 1000)
    # with the separable preconditioner the same kernel is k_update, no block stream
    r2 = b.roofline(_counts(), W, ms, fp32=False, block_precond=False, ms_per_step=2.0)
    assert r2["kernel"] == "k_update" and "block_stream" not in r2
    assert set(r2["all_kernels"]) == {"volume", "face", "gather", "update"}
