"""apply_M, apply_Mdag and lattice_norm2_noalloc recorded into a HIP graph
(torch.cuda.graph on the lattice's own stream) and replayed: the calls are
asynchronous kernel launches with no host synchronisation, device memset or
allocation, so they capture as they are. Four replays, each after eager work
on the same buffers and a device synchronisation, give the eager results bit
for bit; the eager results match the oracle (Sec. 1, Eq. MatrixM). Covers the
streaming kernel (Nx = 16), the general slice kernel (Nx = 6) and the
lower-dimensional kernel (a 2D lattice)."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-13, torch.complex64: 5e-6}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("dim,nx,ntau", [(3, 16, 24), (3, 6, 10), (2, 16, 9)])
def test_operator_and_norm_replay_from_a_captured_graph(dim, nx, ntau, dtype):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    say(f"graph capture dim={dim} nx={nx} ntau={ntau} {dtype}")
    sigma = sigma_field(nx, ntau, 1010, dim)
    L = Lattice(nx, ntau, TAU, G, dtype, dim=dim)
    L.set_aux_field(to_dev(sigma))
    xh = gaussian_rhs(nx, ntau, [1011, 1012, 1013], dim)
    x = to_dev(xh, dtype)
    y, z = torch.empty_like(x), torch.empty_like(x)
    nrm = torch.empty(3, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    L.set_stream(s)
    try:
        def work():
            L.apply_M(x, out=y)
            L.apply_Mdag(y, out=z)
            L.norm2_noalloc(z, nrm)

        with torch.cuda.stream(s):  # eager reference (and first-call set-up)
            work()
        s.synchronize()
        ref_y, ref_z, ref_n = y.clone(), z.clone(), nrm.clone()
        xr = to_host(x)
        for k in range(3):
            yo = oracle.apply_M(xr[k], sigma, TAU, G)
            assert rel_err(to_host(ref_y)[k], yo) < TOL[dtype]
            assert rel_err(to_host(ref_z)[k], oracle.apply_Mdag(to_host(ref_y)[k], sigma, TAU,
                                                                 G)) < TOL[dtype]
        zz = to_host(ref_z).astype(np.complex128)
        assert np.allclose(to_host(ref_n), [np.vdot(v, v).real for v in zz], rtol=1e-12)

        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            work()
        for rep in range(4):
            # eager work on the same buffers between replays
            with torch.cuda.stream(s):
                L.apply_Mdag(x, out=y)
                L.apply_M(y, out=z)
                L.norm2_noalloc(y, nrm)
            torch.cuda.synchronize()
            assert not torch.equal(z, ref_z)
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(y, ref_y), rep
            assert torch.equal(z, ref_z), rep
            assert torch.equal(nrm, ref_n), rep
    finally:
        L.set_stream(None)
