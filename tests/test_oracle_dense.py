"""Pins for the dense oracle (kernels, log-likelihood, score equations).

Each check ties the oracle to something other than itself: the general Matern
formula through the Bessel function, finite differences, exact rational
arithmetic, an independent LAPACK route (eigendecomposition), closed forms for
n = 1, 2 and for a diagonal covariance, and invariants of the model.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import special

from oracle import dense
from oracle import kernels as K
import workloads as W

KERNELS = [K.MATERN12, K.MATERN32, K.MATERN52, K.RQ]


@pytest.mark.parametrize("nu,kernel", [(0.5, K.MATERN12), (1.5, K.MATERN32), (2.5, K.MATERN52)])
def test_matern_closed_forms_match_bessel_definition(nu, kernel):
    # eq. matern: (Gamma(nu) 2^(nu-1))^-1 (sqrt(2 nu) s)^nu K_nu(sqrt(2 nu) s)
    s = np.linspace(1e-3, 8.0, 400)
    t = np.sqrt(2.0 * nu) * s
    bessel = t ** nu * special.kv(nu, t) / (special.gamma(nu) * 2.0 ** (nu - 1.0))
    np.testing.assert_allclose(K.corr(s, kernel), bessel, rtol=1e-12, atol=1e-300)
    assert K.corr(0.0, kernel) == 1.0


def test_rq_limits():
    s = np.linspace(0.0, 3.0, 50)
    # alpha = 1: 1 / (1 + s^2 / 2)
    np.testing.assert_allclose(K.corr(s, K.RQ, 1.0), 1.0 / (1.0 + s * s / 2.0), rtol=1e-15)
    # alpha -> infinity: the squared exponential (the limit named after eq. rationalquadratic)
    np.testing.assert_allclose(K.corr(s, K.RQ, 1e7), np.exp(-s * s / 2.0), rtol=5e-6)


@pytest.mark.parametrize("kernel", KERNELS)
def test_rho_derivative_matches_central_difference(kernel):
    r = np.linspace(1e-3, 0.4, 200)
    rho, h = 0.07, 1e-6
    fd = (K.corr(r / (rho + h), kernel, 0.8) - K.corr(r / (rho - h), kernel, 0.8)) / (2 * h)
    np.testing.assert_allclose(K.dcorr_drho(r, rho, kernel, 0.8), fd, rtol=1e-7, atol=1e-9)


def _rational_chol_terms(S, z):
    """Exact log|S| (as det) and z^T S^-1 z by Gaussian elimination in Fractions."""
    n = S.shape[0]
    A = [[Fraction(float(S[i, j])) for j in range(n)] for i in range(n)]
    b = [Fraction(float(v)) for v in z]
    det = Fraction(1)
    for c in range(n):
        piv = A[c][c]
        det *= piv
        for r in range(c + 1, n):
            f = A[r][c] / piv
            if f:
                for j in range(c, n):
                    A[r][j] -= f * A[c][j]
                b[r] -= f * b[c]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        s = b[r] - sum(A[r][j] * x[j] for j in range(r + 1, n))
        x[r] = s / A[r][r]
    quad = sum(Fraction(float(z[i])) * x[i] for i in range(n))
    return det, quad


@pytest.mark.parametrize("kernel", KERNELS)
def test_loglik_exact_rational_small(kernel):
    P = W.uniform_points(9, 3)
    z = W.gaussian(9, 4)
    theta = (0.3, 1.2, 0.05)
    S = dense.cov_matrix(P, theta, kernel, 0.9)
    det, quad = _rational_chol_terms(S, z)
    ell, logdet, _ = dense.loglik(P, z, theta, kernel, 0.9)
    assert logdet == pytest.approx(math.log(det), rel=1e-13, abs=1e-13)
    exact = -0.5 * float(quad) - 0.5 * math.log(det) - 4.5 * math.log(2 * math.pi)
    assert ell == pytest.approx(exact, rel=1e-13)


@pytest.mark.parametrize("kernel", KERNELS)
def test_loglik_matches_eigendecomposition_route(kernel):
    P = W.uniform_points(60, 5)
    z = W.gaussian(60, 6)
    theta = (0.15, 0.8, 1e-3)
    S = dense.cov_matrix(P, theta, kernel, 1.0)
    lam, V = np.linalg.eigh(S)
    assert lam.min() > 0
    ell, logdet, a = dense.loglik(P, z, theta, kernel)
    a_eig = V @ ((V.T @ z) / lam)
    assert logdet == pytest.approx(float(np.sum(np.log(lam))), rel=1e-10)
    np.testing.assert_allclose(a, a_eig, rtol=1e-8, atol=1e-8 * np.abs(a_eig).max())


def test_n1_and_n2_closed_forms():
    theta = (0.2, 1.5, 0.1)
    s = theta[1] + theta[2]
    P1 = np.array([[0.3, 0.4]])
    ell, logdet, a = dense.loglik(P1, np.array([0.7]), theta, K.MATERN32)
    assert logdet == pytest.approx(math.log(s), rel=1e-15)
    assert ell == pytest.approx(-0.5 * 0.49 / s - 0.5 * math.log(s) - 0.5 * math.log(2 * math.pi), rel=1e-15)
    P2 = np.array([[0.0, 0.0], [0.3, 0.4]])  # r = 0.5
    kv = theta[1] * (1 + math.sqrt(3) * 0.5 / 0.2) * math.exp(-math.sqrt(3) * 0.5 / 0.2)
    z = np.array([0.3, -1.1])
    det = s * s - kv * kv
    quad = (s * z[0] ** 2 - 2 * kv * z[0] * z[1] + s * z[1] ** 2) / det
    ell, logdet, _ = dense.loglik(P2, z, theta, K.MATERN32)
    assert logdet == pytest.approx(math.log(det), rel=1e-14)
    assert ell == pytest.approx(-0.5 * quad - 0.5 * math.log(det) - math.log(2 * math.pi), rel=1e-14)


def test_diagonal_covariance_closed_form():
    # lattice spacing 1 and rho = 1e-3: off-diagonal Matern entries underflow to 0
    g = np.arange(8.0)
    P = np.stack(np.meshgrid(g, g), axis=-1).reshape(-1, 2)
    n = P.shape[0]
    z = W.gaussian(n, 9)
    theta = (1e-3, 1.3, 0.2)
    s = theta[1] + theta[2]
    o = dense.loglik_and_grad(P, z, theta, K.MATERN32, want_terms=True)
    zz = float(z @ z)
    assert o["ell"] == pytest.approx(-0.5 * zz / s - 0.5 * n * math.log(s) - 0.5 * n * math.log(2 * math.pi), rel=1e-14)
    gs = 0.5 * zz / s ** 2 - n / (2 * s)
    np.testing.assert_allclose(o["g"], [0.0, gs, gs], rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("kernel", KERNELS)
def test_gradient_matches_central_difference_of_loglik(kernel):
    P = W.uniform_points(80, 7)
    theta = np.array([0.12, 0.9, 0.02])
    z = dense.sample(P, W.gaussian(80, 8), theta, kernel, 0.7)
    o = dense.loglik_and_grad(P, z, theta, kernel, 0.7, block=32)
    for i in range(3):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (dense.loglik(P, z, tp, kernel, 0.7)[0] - dense.loglik(P, z, tm, kernel, 0.7)[0]) / (2 * h)
        assert o["g"][i] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_euler_identity_and_sigma2_trace():
    # Sigma is homogeneous of degree one in (sigma2, nugget):
    #   sigma2 g_sigma2 + nugget g_nugget = 1/2 z^T Sigma^-1 z - n/2
    # and Tr(Sigma^-1 Sigma_sigma2) = (n - nugget Tr Sigma^-1) / sigma2.
    P = W.uniform_points(150, 10)
    theta = (0.09, 1.7, 3e-3)
    z = W.gaussian(150, 11)
    o = dense.loglik_and_grad(P, z, theta, K.MATERN52, block=64, want_terms=True)
    lhs = theta[1] * o["g"][1] + theta[2] * o["g"][2]
    rhs = 0.5 * float(z @ o["alpha"]) - 75.0
    assert lhs == pytest.approx(rhs, rel=1e-10)
    tinv = dense.trace_inverse(P, theta, K.MATERN52)
    assert o["t"][2] == pytest.approx(tinv, rel=1e-10)
    assert o["t"][1] == pytest.approx((150 - theta[2] * tinv) / theta[1], rel=1e-9)


def test_symmetry_and_spd():
    P = W.uniform_points(400, 12)
    for kernel in KERNELS:
        S = dense.cov_matrix(P, (0.1, 1.0, 1e-4), kernel)
        assert np.array_equal(S, S.T)
        assert np.linalg.eigvalsh(S).min() > 0


def test_not_spd_is_reported():
    P = W.uniform_points(50, 13)
    with pytest.raises(dense.NotSPD):
        dense.loglik(P, W.gaussian(50, 1), (0.3, 1.0, -0.5), K.MATERN32)


ANISO = [(K.MATERN32_ANISO, K.MATERN32), (K.RQ_ANISO, K.RQ)]


@pytest.mark.parametrize("kernel,iso", ANISO)
def test_aniso_isotropic_limit(kernel, iso):
    """theta_1 = theta_2 = rho gives the isotropic kernel with sigma2 = 1, and
    the two derivatives add up to d/drho of it (dx^2 + dy^2 = r^2)."""
    P = W.uniform_points(60, 21)
    rho = 0.17
    A = K.cross_cov(P, P[:40], (rho, rho, 0.0), kernel, 0.7)
    np.testing.assert_allclose(A, K.cross_cov(P, P[:40], (rho, 1.0, 0.0), iso, 0.7), rtol=1e-14, atol=1e-300)
    D = K.cross_dcov(P, P[:40], 0, (rho, rho, 0.0), kernel, 0.7) + K.cross_dcov(P, P[:40], 1, (rho, rho, 0.0), kernel, 0.7)
    np.testing.assert_allclose(D, K.cross_dcov_drho(P, P[:40], (rho, 1.0, 0.0), iso, 0.7), rtol=1e-12, atol=1e-14)
    S = dense.cov_matrix(P, (rho, rho, 0.03), kernel, 0.7)
    np.testing.assert_allclose(S, dense.cov_matrix(P, (rho, 1.0, 0.03), iso, 0.7), rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("kernel,iso", ANISO)
def test_aniso_axis_stretch(kernel, iso):
    """Scaling the y coordinates by theta_1 / theta_2 turns the anisotropic
    kernel into the isotropic one of range theta_1; a separation along one
    axis sees only that axis' range."""
    P = W.uniform_points(50, 22)
    th = (0.2, 0.05, 0.0)
    Q = P.copy()
    Q[:, 1] *= th[0] / th[1]
    np.testing.assert_allclose(K.cross_cov(P, P, th, kernel, 0.7), K.cross_cov(Q, Q, (th[0], 1.0, 0.0), iso, 0.7),
                               rtol=1e-12, atol=1e-300)
    x = np.array([[0.3, 0.3]])
    y = np.array([[0.3, 0.34]])
    assert K.cross_cov(x, y, th, kernel, 0.7)[0, 0] == pytest.approx(float(K.corr(np.array([0.04 / th[1]]), iso, 0.7)[0]), rel=1e-13)
    assert K.cross_dcov(x, y, 0, th, kernel, 0.7)[0, 0] == 0.0


@pytest.mark.parametrize("kernel,iso", ANISO)
def test_aniso_derivatives_match_central_difference(kernel, iso):
    P = W.uniform_points(40, 23)
    th = np.array([0.13, 0.07, 0.0])
    for which in (0, 1):
        h = 1e-6 * th[which]
        tp, tm = th.copy(), th.copy()
        tp[which] += h
        tm[which] -= h
        fd = (K.cross_cov(P, P, tp, kernel, 0.7) - K.cross_cov(P, P, tm, kernel, 0.7)) / (2 * h)
        np.testing.assert_allclose(K.cross_dcov(P, P, which, th, kernel, 0.7), fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("kernel,iso", ANISO)
def test_aniso_gradient_matches_central_difference_of_loglik(kernel, iso):
    P = W.uniform_points(80, 24)
    theta = np.array([0.15, 0.06, 0.02])
    z = dense.sample(P, W.gaussian(80, 25), theta, kernel, 0.7)
    o = dense.loglik_and_grad(P, z, theta, kernel, 0.7, block=32)
    for i in range(3):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (dense.loglik(P, z, tp, kernel, 0.7)[0] - dense.loglik(P, z, tm, kernel, 0.7)[0]) / (2 * h)
        assert o["g"][i] == pytest.approx(fd, rel=1e-6, abs=1e-6)
