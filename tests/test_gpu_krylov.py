"""Fused Krylov reductions on the device: FP64 partial sums per workgroup and a
fixed-order finalize (the BLAS-1 layer under every solver, Eqs. 1-2 of the
paper use these inner products). Checked against numpy in FP64 on the same
(already rounded) inputs, for several vector-kernel launch shapes, and for
bitwise repeatability."""
import numpy as np
import pytest
import torch

from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, to_host, say, TAU, G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("nx,ntau,nrhs,vec_blocks", [(4, 7, 1, 0), (6, 13, 3, 0), (8, 40, 2, 1),
                                                     (16, 25, 2, 0), (12, 30, 5, 4096)])
def test_norm2_matches_fp64(nx, ntau, nrhs, vec_blocks, dtype):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    say(f"norm2 nx={nx} ntau={ntau} nrhs={nrhs} vec_blocks={vec_blocks} {dtype}")
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma_field(nx, ntau, 501)))
    L.tune(0, vec_blocks)
    b = gaussian_rhs(nx, ntau, list(range(502, 502 + nrhs)))
    # a spread of magnitudes across the rhs and the slices
    b = b * (10.0 ** np.arange(nrhs))[:, None, None, None, None]
    b[:, ::3] *= 1e-3
    xd = to_dev(b, dtype)
    xh = to_host(xd).astype(np.complex128)  # the values the device holds, exactly
    got = L.norm2(xd)
    ref = [float(np.vdot(xi.ravel(), xi.ravel()).real) for xi in xh]
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-13 * r
    # fixed-order sums: a second call gives the same bits
    assert L.norm2(xd) == got
