"""A plain C program drives the library on the GPU: no Python binding, no torch.

tests/c_caller/rt_demo.c (built by build() with gcc against include/rtmm.h, librtmm.so
and HIP's runtime library) uploads a periodic cubic lattice whose generators drift,
verifies an antipodal angle set on the device, and runs both precision forms through the
ABI alone: radiative equilibrium survives 5 fused steps (section 2.3: the quartic's root is
T^n); fused steps away from equilibrium keep the energy and momentum totals that
rt_diagnostics reports (section 2.3.1); first-order and PLM-VL2 transport conserve every
angle's total (first order keeps I >= 0, PLM keeps a uniform field uniform; section 2.2);
rt_moments gives E_r = 4 pi B, F_r = 0, P_r = E_r/3 for an isotropic field (section 2.1);
at zero opacity rt_step_adjoint is the transpose of the step; the multigroup and kappa(T)
steps keep equilibrium; rt_flux_loss_noalloc reproduces rt_flux_loss bit for bit and an
isotropic field's loss vanishes; rt_gradient is exact for a linear field away from the
periodic wrap.  The program prints one line per check and "ok" last."""
import importlib.util
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_caller", "rt_demo")


def _build():
    """build() makes the program; where it has not run, compile it here (gcc, under a second)."""
    spec = importlib.util.spec_from_file_location("rt_demo_build", os.path.join(HERE, "c_caller", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.build_demo()


def test_c_program_runs_the_step_on_the_gpu():
    if not os.path.exists(EXE):
        print("building", _build(), flush=True)
    print("running", EXE, flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[-1] == "ok"
    assert sum(line.startswith("pass ") for line in lines) == 73, r.stdout
