"""Plain dense FP64 evaluation of the Gaussian-process log-likelihood and its
score equations (oracle; TEST INFRASTRUCTURE ONLY).

Follows the paper's problem statement directly:

  eq. normaldist      z ~ N(0, Sigma(theta)), Sigma_ij = K(x_i, x_j; theta)
  eq. loglikelihood   l = -1/2 z^T Sigma^-1 z - 1/2 log|Sigma| - (n/2) log 2 pi
  eq. gradient        g_i = 1/2 z^T Sigma^-1 Sigma_i Sigma^-1 z
                            - 1/2 Tr(Sigma^-1 Sigma_i)

through a dense Cholesky factorisation Sigma = L L^T (LAPACK dpotrf), which is
the O(n^3) route the introduction describes.  log|Sigma| = 2 sum log L_jj,
alpha = Sigma^-1 z = L^-T L^-1 z, Sigma^-1 from dpotri, and
Tr(Sigma^-1 Sigma_i) = sum_jk (Sigma^-1)_jk (Sigma_i)_jk (Sigma_i symmetric).

Large n is handled blockwise (the derivative matrices are never stored), with
the factor and the inverse held in one n x n buffer.
"""
import math

import numpy as np
from scipy.linalg import lapack

from . import kernels as K

LOG2PI = math.log(2.0 * math.pi)


class NotSPD(RuntimeError):
    """Cholesky breakdown: the covariance matrix is not numerically SPD."""


def cov_matrix(P, theta, kernel, alpha=1.0, out=None, block=2048):
    """Dense Sigma(theta) for points P (n x 2), assembled by row blocks."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    n = P.shape[0]
    S = np.empty((n, n)) if out is None else out
    idx = np.arange(n)
    for b in range(0, n, block):
        e = min(n, b + block)
        S[b:e, :] = K.cov_block(P, idx[b:e], idx, theta, kernel, alpha)
    return S


def dcov_matrix(P, which, theta, kernel, alpha=1.0):
    """Dense Sigma_i = dSigma/dtheta_i (small n only)."""
    idx = np.arange(P.shape[0])
    return K.dcov_block(P, idx, idx, which, theta, kernel, alpha)


def _potrf_inplace(S):
    # S is symmetric and C-contiguous, so S.T is the same matrix in Fortran
    # order: the factorisation then works in place in S's buffer.
    L, info = lapack.dpotrf(S.T, lower=1, overwrite_a=1, clean=1)
    if info > 0:
        raise NotSPD("dpotrf failed at column %d" % info)
    if info < 0:
        raise ValueError("dpotrf argument error %d" % info)
    return L  # Fortran-ordered lower factor sharing S's memory


def loglik(P, z, theta, kernel, alpha=1.0):
    """(l, log|Sigma|, alpha_vec = Sigma^-1 z) by dense Cholesky."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    S = cov_matrix(P, theta, kernel, alpha)
    L = _potrf_inplace(S)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    a, info = lapack.dpotrs(L, z, lower=1)
    if info != 0:
        raise ValueError("dpotrs info %d" % info)
    ell = -0.5 * float(z @ a) - 0.5 * logdet - 0.5 * n * LOG2PI
    return ell, logdet, a


def loglik_and_grad(P, z, theta, kernel, alpha=1.0, block=2048, want_terms=False):
    """Dense l and g = (g_rho, g_sigma2, g_nugget).

    Returns a dict with ell, logdet, alpha (Sigma^-1 z), g (3,), and the two
    halves of each score component: q_i = 1/2 alpha^T Sigma_i alpha and
    t_i = Tr(Sigma^-1 Sigma_i), so g_i = q_i - t_i / 2."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    S = cov_matrix(P, theta, kernel, alpha, block=block)
    L = _potrf_inplace(S)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    a, info = lapack.dpotrs(L, z, lower=1)
    if info != 0:
        raise ValueError("dpotrs info %d" % info)
    ell = -0.5 * float(z @ a) - 0.5 * logdet - 0.5 * n * LOG2PI
    Linv, info = lapack.dpotri(L, lower=1, overwrite_c=1)
    if info != 0:
        raise NotSPD("dpotri info %d" % info)
    if not np.shares_memory(Linv, S):
        raise RuntimeError("dpotri did not work in place")
    # Linv is Fortran-ordered with its lower triangle valid, i.e. in the
    # C-ordered buffer S the entries S[j, k] with k >= j hold (Sigma^-1)_jk.
    # Sigma^-1 and Sigma_i are symmetric, so
    #   Tr(Sigma^-1 Sigma_i) = sum_j (.)_jj + 2 sum_{j<k} (.)_jk.
    idx = np.arange(n)
    q = np.zeros(3)
    t = np.zeros(3)
    for b in range(0, n, block):
        e = min(n, b + block)
        diag_w = np.triu(np.full((e - b, e - b), 2.0), 1) + np.eye(e - b)
        for which in range(3):
            D = K.dcov_block(P, idx[b:e], idx, which, theta, kernel, alpha)
            q[which] += 0.5 * float(a[b:e] @ (D @ a))
            t[which] += float(np.sum(S[b:e, b:e] * D[:, b:e] * diag_w))
            if e < n:
                t[which] += 2.0 * float(np.sum(S[b:e, e:] * D[:, e:]))
    g = q - 0.5 * t
    out = {"ell": ell, "logdet": logdet, "alpha": a, "g": g}
    if want_terms:
        out["q"] = q
        out["t"] = t
    return out


def profile_loglik(P, z, theta, kernel, alpha=1.0, want_grad=False):
    """The log profile likelihood of eq. prof and its gradient, dense:
      l~ = -1/2 log|Sigma| - n/2 log(z^T (Sigma + 1 1^T)^-1 z) + n/2 (log n - 1 - log 2 pi),
      g~_i = -1/2 Tr(Sigma^-1 Sigma_i) + n/2 (beta^T Sigma_i beta) / (z^T beta),
    beta = (Sigma + 1 1^T)^-1 z, for theta = (rho, sigma2, nugget).
    Returns l~ or (l~, g~)."""
    P = np.asarray(P, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = P.shape[0]
    S = cov_matrix(P, theta, kernel, alpha)
    one = np.ones(n)
    A = S + np.outer(one, one)
    beta = np.linalg.solve(A, z)
    zb = float(z @ beta)
    ld = np.linalg.slogdet(S)[1]
    ell = -0.5 * ld - 0.5 * n * np.log(zb) + 0.5 * n * (np.log(n) - 1.0 - np.log(2.0 * np.pi))
    if not want_grad:
        return ell
    Si = np.linalg.inv(S)
    g = np.zeros(3)
    for i in range(3):
        Di = dcov_matrix(P, i, theta, kernel, alpha)
        g[i] = -0.5 * np.sum(Si * Di.T) + 0.5 * n * float(beta @ (Di @ beta)) / zb
    return ell, g


def trace_inverse(P, theta, kernel, alpha=1.0):
    """Tr(Sigma^-1) (small n)."""
    S = cov_matrix(P, theta, kernel, alpha)
    return float(np.trace(np.linalg.inv(S)))


def sample(P, w, theta, kernel, alpha=1.0):
    """z = L w with Sigma = L L^T: a draw from N(0, Sigma) given w ~ N(0, I)."""
    S = cov_matrix(P, theta, kernel, alpha)
    L = _potrf_inplace(S)
    return np.asarray(L @ np.asarray(w, dtype=np.float64)) if L.shape[0] < 4096 else _trmv(L, w)


def _trmv(L, w):
    from scipy.linalg import blas
    return blas.dtrmv(L, np.asarray(w, dtype=np.float64), lower=1)


def _blocked_cholesky(P, theta, kernel, alpha, bs):
    """Lower Cholesky factor of Sigma in one n x n buffer (lower triangle),
    right-looking over bs x bs blocks; returns (S, blocks, log|Sigma|)."""
    import scipy.linalg as sla
    n = P.shape[0]
    S = np.empty((n, n))
    idx = np.arange(n)
    nb = (n + bs - 1) // bs
    blk = [(k * bs, min(n, (k + 1) * bs)) for k in range(nb)]
    for (b0, b1) in blk:
        S[b0:b1, :b1] = K.cov_block(P, idx[b0:b1], idx[:b1], theta, kernel, alpha)
    logdet = 0.0
    for k, (k0, k1) in enumerate(blk):
        Lkk = sla.cholesky(S[k0:k1, k0:k1], lower=True, check_finite=False)
        S[k0:k1, k0:k1] = Lkk
        logdet += 2.0 * float(np.sum(np.log(np.diag(Lkk))))
        for (i0, i1) in blk[k + 1:]:
            S[i0:i1, k0:k1] = sla.solve_triangular(Lkk, S[i0:i1, k0:k1].T, lower=True, check_finite=False).T
        for i, (i0, i1) in enumerate(blk[k + 1:], start=k + 1):
            Lik = S[i0:i1, k0:k1]
            for (j0, j1) in blk[k + 1:i + 1]:
                S[i0:i1, j0:j1] -= Lik @ S[j0:j1, k0:k1].T
    return S, blk, logdet


def sample_loglik_large(P, w, theta, kernel, alpha=1.0, bs=8192):
    """For large n: z = L w (a draw from N(0, Sigma) given w ~ N(0, I)) with the
    blocked Cholesky factor L, and for that z the exact l, log|Sigma| and
    Sigma^-1 z = L^-T w (so z^T Sigma^-1 z = w^T w)."""
    import scipy.linalg as sla
    P = np.ascontiguousarray(P, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = P.shape[0]
    S, blk, logdet = _blocked_cholesky(P, theta, kernel, alpha, bs)
    z = np.zeros(n)
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            Lkj = np.tril(S[k0:k1, j0:j1]) if j0 == k0 else S[k0:k1, j0:j1]
            z[k0:k1] += Lkj @ w[j0:j1]
    x = w.copy()
    for k in range(len(blk) - 1, -1, -1):
        k0, k1 = blk[k]
        for (j0, j1) in blk[k + 1:]:
            x[k0:k1] -= S[j0:j1, k0:k1].T @ x[j0:j1]
        x[k0:k1] = sla.solve_triangular(S[k0:k1, k0:k1], x[k0:k1], lower=True, trans="T", check_finite=False)
    ell = -0.5 * float(w @ w) - 0.5 * logdet - 0.5 * n * LOG2PI
    return z, ell, logdet, x


def loglik_large(P, z, theta, kernel, alpha=1.0, bs=8192):
    """(l, log|Sigma|, Sigma^-1 z) for large n by a blocked, in-place, right-
    looking Cholesky over bs x bs blocks of one n x n buffer: diagonal blocks
    by LAPACK dpotrf, panels by triangular solves, trailing blocks by matrix
    products (so no single LAPACK call sees more than bs x n entries)."""
    import scipy.linalg as sla
    P = np.ascontiguousarray(P, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = P.shape[0]
    S = np.empty((n, n))
    idx = np.arange(n)
    nb = (n + bs - 1) // bs
    blk = [(k * bs, min(n, (k + 1) * bs)) for k in range(nb)]
    # lower triangle only, block rows
    for (b0, b1) in blk:
        S[b0:b1, :b1] = K.cov_block(P, idx[b0:b1], idx[:b1], theta, kernel, alpha)
    logdet = 0.0
    for k, (k0, k1) in enumerate(blk):
        Lkk = sla.cholesky(S[k0:k1, k0:k1], lower=True, check_finite=False)
        S[k0:k1, k0:k1] = Lkk
        logdet += 2.0 * float(np.sum(np.log(np.diag(Lkk))))
        for (i0, i1) in blk[k + 1:]:
            # L_ik = A_ik L_kk^-T
            S[i0:i1, k0:k1] = sla.solve_triangular(Lkk, S[i0:i1, k0:k1].T, lower=True, check_finite=False).T
        for i, (i0, i1) in enumerate(blk[k + 1:], start=k + 1):
            Lik = S[i0:i1, k0:k1]
            for (j0, j1) in blk[k + 1:i + 1]:
                S[i0:i1, j0:j1] -= Lik @ S[j0:j1, k0:k1].T
    # forward and back substitution with the block factor
    y = z.copy()
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k]:
            y[k0:k1] -= S[k0:k1, j0:j1] @ y[j0:j1]
        y[k0:k1] = sla.solve_triangular(S[k0:k1, k0:k1], y[k0:k1], lower=True, check_finite=False)
    x = y
    for k in range(nb - 1, -1, -1):
        k0, k1 = blk[k]
        for (j0, j1) in blk[k + 1:]:
            x[k0:k1] -= S[j0:j1, k0:k1].T @ x[j0:j1]
        x[k0:k1] = sla.solve_triangular(S[k0:k1, k0:k1], x[k0:k1], lower=True, trans="T", check_finite=False)
    ell = -0.5 * float(z @ x) - 0.5 * logdet - 0.5 * n * LOG2PI
    return ell, logdet, x
