"""The C-ABI from plain C: include/ss.h compiles as C99 with warnings as
errors, a C client links against libss.so, and (on a GPU) solves."""
import os
import subprocess

import pytest

import paper_2108_13162_amd as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "poisson_c_abi.c")


def _build(tmp_path):
    exe = str(tmp_path / "poisson_c_abi")
    libdir = os.path.dirname(ss.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-O2", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include", SRC, "-o", exe,
           f"-L{libdir}", "-lss", f"-Wl,-rpath,{libdir}", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_header_compiles_as_c_and_client_links(tmp_path):
    assert os.path.exists(ss.LIB_PATH)
    _build(tmp_path)


@pytest.mark.gpu
def test_c_client_solves(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe, "48"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "iterations=" in r.stdout
    # the product, the allocation-free solve and a batch solved as one graph
    # launch, from C
    assert "noalloc: iterations=" in r.stdout and "identical=1" in r.stdout
    assert "batch: graphs=1 chunks=0 kernels=0" in r.stdout
    # a caller's allocator returning blocks off a 256-byte boundary is refused
    # cleanly, every block handed back
    assert "misaligned allocator: out of memory, blocks left 0" in r.stdout
