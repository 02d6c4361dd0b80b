"""lattice_norm2_noalloc (C ABI) against lattice_norm2.

The allocation-free variant uses the same kernels in the same order with its
partial sums in a static device buffer, so its norms must equal lattice_norm2's
bit for bit, on two calls in a row (the second with a smaller input, over the
buffer's leftover contents), in both precisions; a request larger than the
static buffer must be refused with an error.
"""
import numpy as np
import pytest
import torch

from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, TAU, G

pytestmark = pytest.mark.gpu


def _norms_noalloc(L, x):
    out = torch.full((x.shape[0],), float("nan"), dtype=torch.float64, device=x.device)
    L.norm2_noalloc(x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_norm2_matches_lattice_norm2(dtype):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau = 8, 40
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma_field(nx, ntau, 990)))
    big = to_dev(gaussian_rhs(nx, ntau, range(991, 997)) * 3.0, dtype)  # 6 rhs
    small = to_dev(gaussian_rhs(nx, ntau, [997, 998]), dtype)            # 2 rhs
    for x in (big, small):
        got = _norms_noalloc(L, x)
        ref = np.array(L.norm2(x))
        assert np.array_equal(got, ref), (got, ref)
        xh = x.cpu().numpy().astype(np.complex128)
        direct = np.array([np.vdot(v, v).real for v in xh])
        assert np.max(np.abs(got - direct) / direct) < 1e-13
    # a smaller lattice after the larger one, same process and buffer
    L2 = Lattice(4, 6, TAU, G, dtype)
    x2 = to_dev(gaussian_rhs(4, 6, [999]), dtype)
    assert np.array_equal(_norms_noalloc(L2, x2), np.array(L2.norm2(x2)))


def test_noalloc_norm2_rejects_oversized_requests():
    require_gpu()
    from paper_1008_3647_amd import Lattice, UfgError
    L = Lattice(8, 40, TAU, G, torch.complex128)
    x = torch.zeros((32, 40, 8, 8, 8), dtype=torch.complex128, device="cuda")
    L.tune(vec_blocks=4096)  # 32 * 4096 * 32 bytes of partials > 2 MiB
    out = torch.empty(32, dtype=torch.float64, device="cuda")
    with pytest.raises(UfgError, match="scratch"):
        L.norm2_noalloc(x, out)
    L.tune(vec_blocks=0)
    assert np.array_equal(_norms_noalloc(L, x), np.zeros(32))
