"""Host-only bounds check of the tile kernels' indexing (tests/native/index_bounds.hip):
the kernels' own __host__ __device__ index functions are run for every thread of
1D and 2D launches over ragged, tiny, periodic and non-periodic meshes; and the
batched runs' plan (classes, arena offsets, tile lists, persistent grids, from
the library's own dg_batch_plan.hpp) is checked for the benchmark's 512-problem
mix and two other seeds, every tile shape, tile order and grid size."""
import os
import subprocess

import pytest

from paper_2309_12019_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "index_bounds.hip")
OUT = os.path.join(os.path.dirname(HERE), "paper_2309_12019_amd", "_build", "index_bounds")


@pytest.fixture(scope="module")
def harness():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.run([hipcc, "--offload-host-only", "-O1", "-std=c++17", "-fconstexpr-steps=100000000",
                    SRC, "-o", OUT], check=True, capture_output=True)
    return OUT


def test_kernel_indices_stay_in_bounds(harness):
    r = subprocess.run([harness], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_batch_plan_stays_in_bounds(harness, tmp_path, seed):
    """The benchmark's batch (512 problems: 1D advection and Burgers, 64-4096
    cells; 2D rotation, 32^2-512^2; p = 1..4) for seed 0, and two more mixes."""
    ws = inputs.batch_mix(seed, 512, 100)
    path = tmp_path / "problems.txt"
    with open(path, "w") as f:
        for w in ws:
            f.write(f"{w.dim} {w.nx} {w.ny if w.dim == 2 else 1} {w.p} {w.flux} {w.mode} "
                    f"{int(w.periodic_x)} {int(w.periodic_y)}\n")
    r = subprocess.run([harness, str(path)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "512 problems" in r.stdout
