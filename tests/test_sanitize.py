"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* ``sanitize_driver.c`` drives the FP64 oracle (real and complex builds) and the input
  mesh builder through every routine on a small jittered mesh, with invariant checks;
* ``sanitize_host_mesh.cpp`` runs the host half of the library's mesh upload (tessellation
  checks, half-face index, staging sizes, workgroup orders) on valid, invalid and random
  face lists, against brute force.

Both are built with gcc / g++ ``-fsanitize=address,undefined -fno-sanitize-recover=all``
(plain host compilers: no GPU code is involved) and must exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, f"{' '.join(cmd)} failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc / g++ not found")
    return str(tmp_path_factory.mktemp("sanitize"))


def test_oracle_and_mesh_builder_under_sanitizers(workdir):
    oracle = os.path.join(ROOT, "oracle", "rt_oracle.c")
    objs = []
    for name, src, extra in (("or_real.o", oracle, []), ("or_cs.o", oracle, ["-DOR_COMPLEX"]),
                             ("vor.o", os.path.join(ROOT, "paper_2002_08377_amd", "inputs", "voronoi.c"), []),
                             ("drv.o", os.path.join(ROOT, "tests", "sanitize_driver.c"), [])):
        _run(["gcc", "-std=c11", *SAN, *extra, "-c", src, "-o", name], workdir)
        objs.append(name)
    _run(["gcc", *SAN, "-o", "oracle_driver", *objs, "-lm"], workdir)
    out = _run([os.path.join(workdir, "oracle_driver")], workdir)
    assert "sanitize driver OK" in out


def test_host_mesh_build_under_sanitizers(workdir):
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2002_08377_amd", "csrc"),
          os.path.join(ROOT, "tests", "sanitize_host_mesh.cpp"), "-o", "host_mesh_driver"], workdir)
    out = _run([os.path.join(workdir, "host_mesh_driver")], workdir)
    assert "host mesh driver OK" in out
