"""Build the plain C caller of librtmm (rt_demo.c) next to its source: gcc, C99, linked
against the in-tree librtmm.so (found through an rpath relative to the executable) and
HIP's runtime library.  `python tests/c_caller/build.py` rebuilds it."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "rt_demo.c")
EXE = os.path.join(HERE, "rt_demo")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_demo() -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", EXE,
           "-L", os.path.join(ROOT, "paper_2002_08377_amd"), "-lrtmm", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-lm", "-Wl,-rpath,$ORIGIN/../../paper_2002_08377_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building {SRC} failed:\n{r.stdout}\n{r.stderr}")
    return EXE


if __name__ == "__main__":
    print(build_demo())
    sys.exit(0)
