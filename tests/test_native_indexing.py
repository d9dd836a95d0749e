"""Host-only bounds check of the tile kernels' indexing (tests/native/index_bounds.hip):
the kernels' own __host__ __device__ index functions are run for every thread of
1D and 2D launches over ragged, tiny, periodic and non-periodic meshes."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "index_bounds.hip")
OUT = os.path.join(os.path.dirname(HERE), "paper_2309_12019_amd", "_build", "index_bounds")


def test_kernel_indices_stay_in_bounds():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.run([hipcc, "--offload-host-only", "-O1", "-std=c++17", "-fconstexpr-steps=100000000",
                    SRC, "-o", OUT], check=True, capture_output=True)
    r = subprocess.run([OUT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
