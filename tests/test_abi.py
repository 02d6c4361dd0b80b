"""The C-ABI library loads, exports every declared symbol, and its host-side
helpers agree with the oracle (no device work: runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import operator as op
from oracle import precond as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ufg.h")
LIB = os.path.join(ROOT, "paper_1008_3647_amd", "libufg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("create_lattice", "set_aux_field", "apply_M", "apply_Mdag", "apply_precond",
              "solve_cg_normal", "solve_bicgstab", "solve_batched", "force_dS_dsigma",
              "destroy_lattice", "ufg_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_host_chebyshev_roots_match_oracle():
    from paper_1008_3647_amd.lattice import cheb_roots
    for deg in (8, 16, 32):
        for eps in (1e-2, 1e-3):
            roots, cf = cheb_roots(deg, eps)
            ref = pc.cheb_roots(deg, eps)[pc.bit_reversal_order(deg)]
            assert np.allclose(roots, ref, atol=1e-15)
            assert cf ** deg == pytest.approx(pc.cheb_constant(deg, eps), rel=1e-12)


def test_host_rejects_bad_chebyshev_degree():
    from paper_1008_3647_amd.lattice import cheb_roots
    from paper_1008_3647_amd._lib import UfgError
    with pytest.raises(UfgError):
        cheb_roots(12, 1e-2)
    with pytest.raises(UfgError):
        cheb_roots(8, 1.5)


def test_host_euler_weights_match_oracle_recursion():
    from paper_1008_3647_amd.lattice import euler_weights
    for d in range(0, 9):
        for p in (0.5, 0.3):
            assert np.allclose(euler_weights(d, p), pc.euler_weights(d, p), atol=1e-15)
            rng = np.random.default_rng(d)
            terms = rng.standard_normal(d + 1)
            est = pc.euler_estimate(list(np.cumsum(terms)), p)
            assert np.dot(euler_weights(d, p), terms) == pytest.approx(est, rel=1e-12)


def test_host_transfer_matrix_matches_oracle():
    from paper_1008_3647_amd.lattice import transfer_matrix
    for nx in (2, 4, 6, 8, 10, 12, 14, 16):
        assert np.allclose(transfer_matrix(nx, 0.05), op.transfer_matrix_1d(nx, 0.05), atol=1e-15)


def test_create_lattice_dim_rejects_bad_arguments_on_the_host():
    """create_lattice_dim validates dim (1, 2, 3) and the sizes before any
    device call, so the rejections need no GPU."""
    from paper_1008_3647_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    for nx, ntau, dim in ((4, 4, 0), (4, 4, 4), (3, 4, 2), (4, 1, 1), (18, 4, 1)):
        code = lib.create_lattice_dim(nx, ntau, dim, 0.05, 5.0, _lib.UFG_C128, _lib.UFG_DISP_FREE,
                                      None, ctypes.byref(h))
        assert code == _lib.UFG_EINVAL, (nx, ntau, dim, code)
    msg = lib.ufg_last_error().decode()
    assert "nx" in msg


def test_header_is_plain_c_and_the_c_example_links(tmp_path):
    """include/ufg.h compiles as C11 with every warning an error, the example
    program that uses it links against libufg.so, and it rejects malformed
    input files before touching the device."""
    import subprocess
    from paper_1008_3647_amd import build as b
    src = os.path.join(b.EXAMPLES, "solve_from_c.c")
    out = str(tmp_path / "solve_from_c")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include", src, "-o", out,
           f"-L{os.path.dirname(LIB)}", "-lufg", "-L/opt/rocm/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert os.path.exists(out)
    # its input checks run before any device call: bad files end with exit
    # status 1 and a message, and no output
    env = dict(os.environ, LD_LIBRARY_PATH=os.pathsep.join(
        [os.path.dirname(LIB), "/opt/rocm/lib", os.environ.get("LD_LIBRARY_PATH", "")]))
    head = np.array([4, 6, 1], np.int32).tobytes() + np.array([0.05, 5.0]).tobytes()
    cases = {b"": "short header",
             np.array([20, 6, 1], np.int32).tobytes() + np.array([0.05, 5.0]).tobytes():
                 "sizes out of range",
             np.array([4, 6, 0], np.int32).tobytes() + np.array([0.05, 5.0]).tobytes():
                 "sizes out of range",
             head + np.zeros(4 * 4 * 4 * 6).tobytes(): "short body"}
    for i, (data, msg) in enumerate(cases.items()):
        src, dst = tmp_path / f"in{i}.bin", tmp_path / f"out{i}.bin"
        src.write_bytes(data)
        r = subprocess.run([out, str(src), str(dst)], capture_output=True, text=True, env=env,
                           timeout=60)
        assert r.returncode == 1 and msg in r.stderr, (i, r.returncode, r.stderr)
    r = subprocess.run([out], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
