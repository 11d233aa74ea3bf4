"""A plain C program drives the library on the GPU: no Python binding, no torch.

tests/c_caller/rt_demo.c (built by build() with gcc against include/rtmm.h, librtmm.so
and HIP's runtime library) uploads a periodic cubic lattice whose generators drift,
verifies an antipodal angle set on the device, and runs both precision forms through the
ABI alone: radiative equilibrium survives 5 fused steps (section 2.3: the quartic's root is
T^n); fused steps away from equilibrium keep the energy and momentum totals that
rt_diagnostics reports (section 2.3.1); first-order and PLM-VL2 transport conserve every
angle's total (first order keeps I >= 0, PLM keeps a uniform field uniform; section 2.2);
rt_moments gives E_r = 4 pi B, F_r = 0, P_r = E_r/3 for an isotropic field (section 2.1);
and at zero opacity rt_step_adjoint is the transpose of the step.  The program prints one
line per check and "ok" last."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_caller", "rt_demo")


def test_c_program_runs_the_step_on_the_gpu():
    assert os.path.exists(EXE), "tests/c_caller/rt_demo is not built: run __graft_entry__.build()"
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[-1] == "ok"
    assert sum(line.startswith("pass ") for line in lines) == 29, r.stdout
