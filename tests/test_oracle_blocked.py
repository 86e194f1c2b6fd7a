"""Pins for the blocked dense oracle (the large-n route that writes the dense
references at n = 65536): the in-place block Cholesky, the block triangular
solves, the in-place triangular inverse and Sigma^-1 = L^-T L^-1, and the
blocked score terms.

Each is tied to a different algorithm on the same matrix: LAPACK's unblocked
factorization and solves (dense.loglik, dense.sample), numpy's general solve,
the eigendecomposition of Sigma, and the closed form of a diagonal covariance.
Block sizes are chosen so that the last block is ragged and several blocks
take part in every update.
"""
import numpy as np
import pytest

from oracle import dense
from oracle import kernels as K
import workloads as W

N = 700
THETA = (0.12, 1.3, 1e-3)


def _eig_inverse(P, theta, kernel, alpha=1.0):
    S = dense.cov_matrix(P, theta, kernel, alpha)
    lam, V = np.linalg.eigh(S)
    assert lam.min() > 0
    return (V / lam) @ V.T, float(np.sum(np.log(lam)))


@pytest.mark.parametrize("bs", [64, 128, 256, 1024])
def test_blocked_cholesky_matches_lapack(bs):
    P = W.uniform_points(N, 5)
    S, blk, logdet = dense._blocked_cholesky(P, THETA, K.MATERN32, 1.0, bs)
    assert blk[-1][1] == N and (N % bs != 0 or bs >= N)
    L = np.linalg.cholesky(dense.cov_matrix(P, THETA, K.MATERN32))
    Lb = np.zeros((N, N))
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            Lb[k0:k1, j0:j1] = S[k0:k1, j0:j1]
    assert np.array_equal(np.triu(Lb, 1), np.zeros((N, N)))
    np.testing.assert_allclose(Lb, L, rtol=0, atol=1e-12 * np.abs(L).max())
    ref = np.linalg.slogdet(dense.cov_matrix(P, THETA, K.MATERN32))[1]
    assert logdet == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("kernel", [K.MATERN32, K.RQ, K.MATERN32_ANISO])
def test_loglik_large_matches_dense(kernel):
    theta = (0.2, 0.15, 1e-3) if K.is_aniso(kernel) else THETA
    P = W.uniform_points(N, 6)
    z = W.gaussian(N, 7)
    ell, logdet, a = dense.loglik_large(P, z, theta, kernel, 0.8, bs=96)
    ell0, logdet0, a0 = dense.loglik(P, z, theta, kernel, 0.8)
    assert ell == pytest.approx(ell0, rel=1e-12)
    assert logdet == pytest.approx(logdet0, rel=1e-12)
    # an independent solver: Sigma a = z by numpy's LU
    a1 = np.linalg.solve(dense.cov_matrix(P, theta, kernel, 0.8), z)
    np.testing.assert_allclose(a, a1, rtol=0, atol=1e-9 * np.abs(a1).max())
    np.testing.assert_allclose(a, a0, rtol=0, atol=1e-9 * np.abs(a0).max())


def test_sample_loglik_large_model_draw():
    P = W.uniform_points(N, 8)
    w = W.gaussian(N, 9)
    z, ell, logdet, a = dense.sample_loglik_large(P, w, THETA, K.MATERN32, bs=160)
    z0 = dense.sample(P, w, THETA, K.MATERN32)
    np.testing.assert_allclose(z, z0, rtol=0, atol=1e-12 * np.abs(z0).max())
    S = dense.cov_matrix(P, THETA, K.MATERN32)
    # Sigma^-1 z by numpy's LU, and z^T Sigma^-1 z = w^T w
    a1 = np.linalg.solve(S, z)
    np.testing.assert_allclose(a, a1, rtol=0, atol=1e-9 * np.abs(a1).max())
    assert float(z @ a1) == pytest.approx(float(w @ w), rel=1e-9)
    ell0, logdet0, _ = dense.loglik(P, z, THETA, K.MATERN32)
    assert ell == pytest.approx(ell0, rel=1e-10)
    assert logdet == pytest.approx(logdet0, rel=1e-12)


@pytest.mark.parametrize("bs", [64, 300])
def test_blocked_triangular_inverse_and_inverse(bs):
    P = W.uniform_points(N, 10)
    S, blk, _ = dense._blocked_cholesky(P, THETA, K.MATERN32, 1.0, bs)
    L = np.zeros((N, N))
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            L[k0:k1, j0:j1] = S[k0:k1, j0:j1]
    dense._blocked_tri_inverse(S, blk)
    X = np.zeros((N, N))
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            X[k0:k1, j0:j1] = S[k0:k1, j0:j1]
    assert np.array_equal(np.triu(X, 1), np.zeros((N, N)))
    # X L = I and L X = I
    np.testing.assert_allclose(X @ L, np.eye(N), rtol=0, atol=1e-10)
    np.testing.assert_allclose(L @ X, np.eye(N), rtol=0, atol=1e-10)
    dense._blocked_inverse_from_tri_inverse(S, blk)
    Si, _ = _eig_inverse(P, THETA, K.MATERN32)
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            np.testing.assert_allclose(S[k0:k1, j0:j1], Si[k0:k1, j0:j1], rtol=0,
                                       atol=1e-9 * np.abs(Si).max())
    # diagonal blocks are full and symmetric
    for (k0, k1) in blk:
        D = S[k0:k1, k0:k1]
        np.testing.assert_allclose(D, D.T, rtol=0, atol=1e-10 * np.abs(D).max())


@pytest.mark.parametrize("kernel", [K.MATERN32, K.MATERN52, K.RQ, K.MATERN32_ANISO, K.RQ_ANISO])
def test_score_large_matches_dense_and_eigendecomposition(kernel):
    theta = (0.2, 0.15, 1e-3) if K.is_aniso(kernel) else THETA
    alpha = 0.5 if kernel == K.RQ_ANISO else 0.8
    P = W.uniform_points(N, 11)
    z = W.gaussian(N, 12)
    o = dense.score_large(P, theta, kernel, alpha, bs=128, z=z)
    d = dense.loglik_and_grad(P, z, theta, kernel, alpha, want_terms=True)
    assert o["ell"] == pytest.approx(d["ell"], rel=1e-12)
    np.testing.assert_allclose(o["q"], d["q"], rtol=1e-10)
    np.testing.assert_allclose(o["t"], d["t"], rtol=1e-10)
    # an independent route: Sigma^-1 from the eigendecomposition, the
    # derivative matrices formed in full, q from numpy's LU solve
    Si, _ = _eig_inverse(P, theta, kernel, alpha)
    a1 = np.linalg.solve(dense.cov_matrix(P, theta, kernel, alpha), z)
    for i in range(3):
        Di = dense.dcov_matrix(P, i, theta, kernel, alpha)
        assert o["t"][i] == pytest.approx(float(np.sum(Si * Di)), rel=1e-9)
        assert o["q"][i] == pytest.approx(0.5 * float(a1 @ Di @ a1), rel=1e-9)
    np.testing.assert_allclose(o["g"], o["q"] - 0.5 * o["t"], rtol=0, atol=0)


def test_score_large_model_draw_and_single_block():
    P = W.uniform_points(N, 13)
    w = W.gaussian(N, 14)
    o = dense.score_large(P, THETA, K.MATERN32, bs=200, w=w)
    z0 = dense.sample(P, w, THETA, K.MATERN32)
    np.testing.assert_allclose(o["z"], z0, rtol=0, atol=1e-12 * np.abs(z0).max())
    d = dense.loglik_and_grad(P, o["z"], THETA, K.MATERN32, want_terms=True)
    assert o["ell"] == pytest.approx(d["ell"], rel=1e-10)
    np.testing.assert_allclose(o["q"], d["q"], rtol=1e-9)
    np.testing.assert_allclose(o["t"], d["t"], rtol=1e-10)
    # one block: the same numbers as several blocks
    o1 = dense.score_large(P, THETA, K.MATERN32, bs=N, w=w)
    np.testing.assert_allclose(o1["t"], o["t"], rtol=1e-11)
    np.testing.assert_allclose(o1["q"], o["q"], rtol=1e-9)


def test_score_large_diagonal_closed_form():
    # sites on a lattice of spacing 1 with rho = 0.001: every off-diagonal
    # entry underflows to 0, Sigma = (sigma2 + nugget) I
    side = 23
    P = W.grid_points(side, float(side))
    n = side * side
    theta = (0.001, 0.7, 0.2)
    z = W.gaussian(n, 15)
    o = dense.score_large(P, theta, K.MATERN32, bs=100, z=z)
    v = theta[1] + theta[2]
    zz = float(z @ z)
    assert o["ell"] == pytest.approx(-0.5 * zz / v - 0.5 * n * np.log(v) - 0.5 * n * np.log(2 * np.pi), rel=1e-13)
    assert o["t"][0] == 0.0 and o["q"][0] == 0.0
    assert o["t"][1] == pytest.approx(n / v, rel=1e-13)
    assert o["t"][2] == pytest.approx(n / v, rel=1e-13)
    assert o["g"][2] == pytest.approx(0.5 * zz / v ** 2 - 0.5 * n / v, rel=1e-12)
