"""Device utilities outside the method: the streaming copy that measures the
bandwidth ceiling, and the device-side count of non-finite entries."""
import sys

import pytest
import torch

from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,off", [(0, 0), (1, 0), (2, 0), (7, 0), (300001, 0), (300001, 1), (4096, 1)])
def test_stream_copy_exact_and_in_bounds(n, off):
    """Exact copy for even and odd lengths, 16-byte aligned (off 0) and
    8-byte aligned (off 1) views; guard entries around the destination stay."""
    from paper_2309_12019_amd import dgweno
    _note(f"[stream copy] n={n} off={off}")
    src_all = torch.arange(n + off + 3, dtype=torch.float64, device="cuda") * 1.5 + 0.25
    dst_all = torch.full((n + off + 3,), -7.0, dtype=torch.float64, device="cuda")
    src, dst = src_all[off:off + n], dst_all[off:off + n]
    dgweno.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert bool((dst_all[:off] == -7.0).all()) and bool((dst_all[off + n:] == -7.0).all())


def test_stream_copy_rejects_overlap_and_size_mismatch():
    from paper_2309_12019_amd import dgweno
    a = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(dgweno.DGError):
        dgweno.stream_copy(a[:60], a[40:])
    with pytest.raises(ValueError):
        dgweno.stream_copy(a[:10], a[20:31])


def test_count_nonfinite_on_device_large_state():
    """More entries than one grid-stride pass of the counting grid covers."""
    from paper_2309_12019_amd import dgweno
    w = inputs.burgers2d(512, 2, steps=1)
    g = dgweno.DG.from_workload(w)
    U = torch.zeros(w.ncells, w.nloc, dtype=torch.float64, device="cuda")
    assert g.count_nonfinite(U) == 0
    flat = U.view(-1)
    idx = [0, 1, 12345, 2359295, 1048576, 777777]
    for k, i in enumerate(idx):
        flat[i] = float("nan") if k % 2 else float("-inf")
    torch.cuda.synchronize()
    assert g.count_nonfinite(U) == len(idx)
