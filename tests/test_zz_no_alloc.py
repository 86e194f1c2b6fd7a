"""rsf_solve_noalloc (the solve for callers that cannot allocate device memory)
against rsf_solve, through the C ABI: the same F^-1 b to the solve parity bar
(kappa(F) u growth, 1e-8 of the largest entry), on two calls in a row with the
second one smaller, and the rejection of a call too large for the fixed work
space with the output left untouched."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1603_08057_amd as R
from paper_1603_08057_amd import _lib
import workloads as W

pytestmark = pytest.mark.gpu

SOLVE_RTOL = 1e-8
NOALLOC_BYTES = 64 << 20


def _colmajor(B, ld):
    """Device column-major n x nrhs buffer with leading dimension ld."""
    n, nrhs = B.shape
    buf = torch.full((nrhs, ld), 7.0, dtype=torch.float64, device="cuda")
    buf[:, :n] = torch.tensor(B.T, dtype=torch.float64, device="cuda")
    return buf


def _solve(fn, F, B, ld):
    n, nrhs = B.shape
    b = _colmajor(B, ld)
    x = torch.full_like(b, -3.0)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(F._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, ld, s)
    torch.cuda.synchronize()
    return rc, x.cpu().numpy()


def _check(F, B, ld):
    lib = _lib.load()
    n = B.shape[0]
    rc0, X0 = _solve(lib.rsf_solve, F, B, ld)
    rc1, X1 = _solve(lib.rsf_solve_noalloc, F, B, ld)
    assert rc0 == 0 and rc1 == 0, lib.rsf_last_error()
    ref = X0[:, :n]
    np.testing.assert_allclose(X1[:, :n], ref, rtol=0, atol=SOLVE_RTOL * np.abs(ref).max())
    # rows beyond n of each column are the caller's and stay untouched
    assert np.all(X1[:, n:] == -3.0)


def test_noalloc_solve_matches_solve_on_two_calls_the_second_smaller():
    lib = _lib.load()
    theta = (0.08, 1.0, 1e-3)
    P1 = W.uniform_points(3001, 61)
    print("case n=3001 nrhs=5 ld=3009, then nrhs=2", flush=True)
    F1 = R.Factor(torch.tensor(P1, device="cuda"), theta, kernel=R.MATERN32, eps=1e-9, leaf=32, n_prox=128,
                  prox_rings=2)
    assert F1.tree_info()["depth"] >= 3
    _check(F1, W.gaussian((3001, 5), 62), 3009)
    _check(F1, W.gaussian((3001, 2), 63), 3001)
    # a second handle with fewer sites, after the first one's calls
    P2 = W.uniform_points(700, 64)
    print("case n=700 nrhs=1", flush=True)
    F2 = R.Factor(torch.tensor(P2, device="cuda"), theta, kernel=R.MATERN32, eps=1e-9, leaf=32, n_prox=128,
                  prox_rings=2)
    _check(F2, W.gaussian((700, 1), 65), 700)
    # the binding's method goes through the same entry point
    b = W.gaussian(700, 66)
    x = F2.solve_noalloc(torch.tensor(b, device="cuda")).cpu().numpy()
    xr = F2.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(x, xr, rtol=0, atol=SOLVE_RTOL * np.abs(xr).max())
    # a call beyond the fixed work space is refused before any device work
    nrhs = NOALLOC_BYTES // (8 * 3001) + 1
    print("case n=3001 nrhs=%d (refused)" % nrhs, flush=True)
    big = np.ones((3001, nrhs))
    rc, X = _solve(lib.rsf_solve_noalloc, F1, big, 3001)
    assert rc == -1
    assert b"work space" in lib.rsf_last_error()
    assert np.all(X == -3.0)
    F1.close()
    F2.close()
