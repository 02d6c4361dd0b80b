"""The library driven from plain C (paper_1008_3647_amd/examples/solve_from_c,
built with gcc against include/ufg.h and libufg.so by build()), in a process
of its own: no Python binding and no torch between the caller and the C ABI.
Its y = M b is compared with the oracle's apply_M element by element
(Sec. 1, Eq. MatrixM; 1e-13 of the largest entry), its BiCGStab solution of
M x = b (tol 1e-12) with dense LU on a tiny lattice and with the oracle's
residual on a larger one."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import operator as op
from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1008_3647_amd", "examples", "solve_from_c")


def _run(tmp_path, nx, ntau, seeds):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: build() compiles it")
    sigma = sigma_field(nx, ntau, seeds[0])
    b = gaussian_rhs(nx, ntau, seeds[1:])
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([nx, ntau, len(b)], np.int32).tobytes())
        f.write(np.array([TAU, G], np.float64).tobytes())
        f.write(np.ascontiguousarray(sigma, np.float64).tobytes())
        f.write(np.ascontiguousarray(b, np.complex128).tobytes())
    say(f"solve_from_c {nx}^3 x {ntau}, {len(b)} rhs")
    r = subprocess.run([EXE, str(src), str(dst)], capture_output=True, text=True, timeout=120)
    say(r.stdout.strip() + r.stderr.strip())
    assert r.returncode == 0, r.stderr
    data = open(dst, "rb").read()
    nv = b.size * 16
    assert len(data) == 2 * nv + 16
    y = np.frombuffer(data[:nv], np.complex128).reshape(b.shape)
    x = np.frombuffer(data[nv:2 * nv], np.complex128).reshape(b.shape)
    status, iters = np.frombuffer(data[2 * nv:2 * nv + 8], np.int32)
    relres = float(np.frombuffer(data[2 * nv + 8:], np.float64)[0])
    return sigma, b, y, x, int(status), int(iters), relres


def test_c_program_tiny_lattice_against_dense_lu(tmp_path):
    require_gpu()
    sigma, b, y, x, status, iters, relres = _run(tmp_path, 4, 10, [960, 961, 962])
    assert status == 0 and iters > 0 and relres <= 1e-12
    Md = op.dense_M(sigma, TAU, G)
    for k in range(len(b)):
        assert rel_err(y[k], oracle.apply_M(b[k], sigma, TAU, G)) < 1e-13
        ref = np.linalg.solve(Md, b[k].ravel())
        assert rel_err(x[k].ravel(), ref) < 1e-9


def test_c_program_against_oracle_residual(tmp_path):
    require_gpu()
    sigma, b, y, x, status, iters, relres = _run(tmp_path, 8, 40, [970, 971, 972, 973, 974])
    assert status == 0 and relres <= 1e-12
    for k in range(len(b)):
        assert rel_err(y[k], oracle.apply_M(b[k], sigma, TAU, G)) < 1e-13
        r = b[k] - oracle.apply_M(x[k], sigma, TAU, G)
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) < 1e-11
