"""Host builds of the CPU model programs under tests/model (test helper).

They compile the library's own layout and planning code (paper_2506_07164_amd/csrc) for
the host with g++, so the tests check the arithmetic the kernels and the C ABI use."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]


def build(name, sources, extra=(), libs=()):
    """Compile tests/model/<sources> into a temporary executable; returns its path."""
    out = os.path.join(tempfile.mkdtemp(prefix="ofmodel"), name)
    cmd = ["g++", *FLAGS, *extra, *[os.path.join(HERE, "model", s) for s in sources], "-o", out,
           *libs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("host build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    return out


def run(exe, *args, timeout=600):
    return subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=timeout)
