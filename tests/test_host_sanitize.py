"""The library's host setup (sem_setup.cpp: mesh checks, chart geometry,
coefficient fields, face terms, separable bases, degree projectors) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, and under
ThreadSanitizer (the per-element and per-face loops run on several host
threads), and run on a box mesh with a Neumann face and on the Fichera mesh
(every chart, face kind and corner element): no sanitizer report, the
expected sizes."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")


SANITIZERS = {
    "address_undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "thread": ["-fsanitize=thread"],
}


@pytest.fixture(scope="module", params=sorted(SANITIZERS))
def driver(request, tmp_path_factory):
    d = tmp_path_factory.mktemp("san_" + request.param)
    exe = str(d / "host_setup_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread"] + SANITIZERS[request.param] + [
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "host_setup_driver.cpp"),
           os.path.join(ROOT, "paper_1110_2316_amd", "csrc", "sem_setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _write_mesh(mesh, path):
    a = mesh.as_arrays()
    with open(path, "wb") as fh:
        fh.write(np.array([mesh.W, mesh.E, mesh.n_corner_dof], np.int32).tobytes())
        for k in ("region", "kind", "chart", "frame", "mframe", "origin", "box", "patch",
                  "nbr", "nbr_face", "orient", "bc", "cdof", "cdir"):
            fh.write(np.ascontiguousarray(a[k]).tobytes())


@pytest.mark.parametrize("name", ["box_neumann_w3", "fichera_n2w3"])
def test_host_setup_is_clean_under_sanitizers(driver, tmp_path, name):
    if name.startswith("box"):
        mesh = M.box_mesh(3, (2, 2, 1), neumann=((2, 1),))
    else:
        mesh = fichera_mesh(N=2, W=3)
    f = str(tmp_path / "mesh.bin")
    _write_mesh(mesh, f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([driver, f], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    for report in ("ERROR: AddressSanitizer", "runtime error", "WARNING: ThreadSanitizer"):
        assert report not in r.stderr, r.stderr[-3000:]
    sizes = [x for x in r.stdout.splitlines() if x.startswith("ndof")][0]
    ndof = int(sizes.split()[1])
    assert ndof == mesh.ndof()


@pytest.fixture(scope="module")
def plain_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("plain")
    exe = str(d / "host_setup_driver")
    cmd = ["g++", "-std=c++17", "-O2", "-pthread", "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "host_setup_driver.cpp"),
           os.path.join(ROOT, "paper_1110_2316_amd", "csrc", "sem_setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


@pytest.mark.parametrize("name", ["box_neumann_w3", "fichera_n2w3"])
def test_host_setup_does_not_depend_on_the_thread_count(plain_driver, tmp_path, name):
    """The per-element and per-face loops hand out one item at a time and
    record face terms in mesh order: one thread and eight give the same bits
    in every array of the setup."""
    if name.startswith("box"):
        mesh = M.box_mesh(3, (2, 2, 1), neumann=((2, 1),))
    else:
        mesh = fichera_mesh(N=2, W=3)
    f = str(tmp_path / "mesh.bin")
    _write_mesh(mesh, f)
    sums = []
    for threads in ("1", "8"):
        r = subprocess.run([plain_driver, f], capture_output=True, text=True, timeout=600,
                           env=dict(os.environ, SEM_HOST_THREADS=threads))
        assert r.returncode == 0, r.stderr[-3000:]
        line = [x for x in r.stdout.splitlines() if x.startswith("setup-checksum")]
        assert len(line) == 1, r.stdout
        sums.append(line[0])
    assert sums[0] == sums[1], sums
