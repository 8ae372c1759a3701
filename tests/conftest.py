import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU statistics run")


def build_c_client(out_dir):
    """Compile tests/c_client.c, a C11 program that links liblbfluct and the HIP runtime
    and nothing else, with warnings as errors (the HIP headers are treated as system
    headers).  Returns the executable's path."""
    import subprocess
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    pkg = os.path.join(ROOT, "paper_1009_0254_amd")
    exe = os.path.join(str(out_dir), "c_client")
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_client.c"), "-o", exe,
           "-L", pkg, "-llbfluct", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath," + pkg, "-Wl,-rpath," + os.path.join(rocm, "lib")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe
