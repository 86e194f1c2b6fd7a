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


def _blocks(n, bs):
    """Row/column ranges [b0, b1) of the bs x bs blocks of an n x n matrix
    (the last one ragged when bs does not divide n)."""
    return [(b, min(n, b + bs)) for b in range(0, n, bs)]


def _blocked_cholesky(P, theta, kernel, alpha, bs):
    """Lower Cholesky factor of Sigma in one n x n buffer, right-looking over
    bs x bs blocks: diagonal blocks by LAPACK, panels by triangular solves,
    trailing blocks by matrix products (no single LAPACK call sees more than
    bs x n entries).  Only the block lower triangle of the buffer is defined
    (diagonal blocks hold L_kk with zeros above the diagonal); the blocks above
    it are never written or read.  Returns (S, blocks, log|Sigma|)."""
    import scipy.linalg as sla
    n = P.shape[0]
    S = np.empty((n, n))
    idx = np.arange(n)
    blk = _blocks(n, bs)
    for (b0, b1) in blk:
        S[b0:b1, :b1] = K.cov_block(P, idx[b0:b1], idx[:b1], theta, kernel, alpha)
    logdet = 0.0
    for k, (k0, k1) in enumerate(blk):
        try:
            Lkk = sla.cholesky(S[k0:k1, k0:k1], lower=True, check_finite=False)
        except np.linalg.LinAlgError as e:
            raise NotSPD("block Cholesky failed in block %d: %s" % (k, e))
        S[k0:k1, k0:k1] = Lkk
        logdet += 2.0 * float(np.sum(np.log(np.diag(Lkk))))
        for (i0, i1) in blk[k + 1:]:
            # L_ik = A_ik L_kk^-T
            S[i0:i1, k0:k1] = sla.solve_triangular(Lkk, S[i0:i1, k0:k1].T, lower=True, check_finite=False).T
        for i, (i0, i1) in enumerate(blk[k + 1:], start=k + 1):
            Lik = S[i0:i1, k0:k1]
            for (j0, j1) in blk[k + 1:i + 1]:
                S[i0:i1, j0:j1] -= Lik @ S[j0:j1, k0:k1].T
    return S, blk, logdet


def _blocked_lower_matvec(S, blk, w):
    """L w for the block lower-triangular factor held in S."""
    z = np.zeros(S.shape[0])
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k + 1]:
            z[k0:k1] += S[k0:k1, j0:j1] @ w[j0:j1]
    return z


def _blocked_forward(S, blk, b):
    """L^-1 b for the block lower-triangular factor held in S."""
    import scipy.linalg as sla
    y = np.array(b, dtype=np.float64)
    for k, (k0, k1) in enumerate(blk):
        for (j0, j1) in blk[:k]:
            y[k0:k1] -= S[k0:k1, j0:j1] @ y[j0:j1]
        y[k0:k1] = sla.solve_triangular(S[k0:k1, k0:k1], y[k0:k1], lower=True, check_finite=False)
    return y


def _blocked_backward(S, blk, y):
    """L^-T y for the block lower-triangular factor held in S."""
    import scipy.linalg as sla
    x = np.array(y, dtype=np.float64)
    for k in range(len(blk) - 1, -1, -1):
        k0, k1 = blk[k]
        for (j0, j1) in blk[k + 1:]:
            x[k0:k1] -= S[j0:j1, k0:k1].T @ x[j0:j1]
        x[k0:k1] = sla.solve_triangular(S[k0:k1, k0:k1], x[k0:k1], lower=True, trans="T", check_finite=False)
    return x


def _blocked_tri_inverse(S, blk):
    """Overwrites the block lower-triangular L held in S with X = L^-1.

    From X L = I, block (i, k) with i > k satisfies
      X_ik L_kk = - sum_{j = k+1 .. i} X_ij L_jk,
    which needs the inverse's blocks of columns k+1 .. (already final when the
    block columns are taken from the last to the first) and the factor's
    blocks L_jk, j = k+1 .. i, of column k.  Taking the rows of column k from
    the bottom up, writing X_ik destroys only L_ik, which no block above row i
    needs.  The diagonal block is X_kk = L_kk^-1."""
    import scipy.linalg as sla
    for k in range(len(blk) - 1, -1, -1):
        k0, k1 = blk[k]
        Xkk = np.tril(sla.solve_triangular(S[k0:k1, k0:k1], np.eye(k1 - k0), lower=True, check_finite=False))
        for i in range(len(blk) - 1, k, -1):
            i0, i1 = blk[i]
            T = np.zeros((i1 - i0, k1 - k0))
            for j in range(k + 1, i + 1):
                j0, j1 = blk[j]
                T += S[i0:i1, j0:j1] @ S[j0:j1, k0:k1]
            S[i0:i1, k0:k1] = -(T @ Xkk)
        S[k0:k1, k0:k1] = Xkk


def _blocked_inverse_from_tri_inverse(S, blk):
    """Overwrites X = L^-1 (block lower triangle of S) with the block lower
    triangle of Sigma^-1 = X^T X:
      (Sigma^-1)_ik = sum_{j >= i} X_ji^T X_jk,   i >= k.
    Block (i, k) reads the inverse's column blocks i and k at rows >= i.
    Taking the columns from the first to the last and the rows of a column
    from the top down, every block it reads is still X when it is formed, and
    the X_ik it overwrites is read by no later block.  Diagonal blocks receive
    the full symmetric block of Sigma^-1."""
    nb = len(blk)
    for k in range(nb):
        k0, k1 = blk[k]
        for i in range(k, nb):
            i0, i1 = blk[i]
            acc = np.zeros((i1 - i0, k1 - k0))
            for j in range(i, nb):
                j0, j1 = blk[j]
                acc += S[j0:j1, i0:i1].T @ S[j0:j1, k0:k1]
            S[i0:i1, k0:k1] = acc


def _blocked_score_terms(S, blk, P, a, theta, kernel, alpha, row_block=1024):
    """q_i = 1/2 a^T Sigma_i a and t_i = Tr(Sigma^-1 Sigma_i) = sum_jk
    (Sigma^-1)_jk (Sigma_i)_jk (eq. gradient) for the three parameters, with
    Sigma^-1 in the block lower triangle of S (full symmetric diagonal blocks)
    and Sigma_i generated row block by row block over the lower triangle only
    (both matrices symmetric: the strictly lower part counts twice)."""
    n = P.shape[0]
    idx = np.arange(n)
    q = np.zeros(3)
    t = np.zeros(3)
    for (k0, k1) in blk:
        for r0 in range(k0, k1, row_block):
            r1 = min(k1, r0 + row_block)
            for which in range(3):
                if which == 2:
                    # Sigma_nugget = I: only the diagonal
                    q[2] += 0.5 * float(a[r0:r1] @ a[r0:r1])
                    t[2] += float(np.sum(np.diag(S[r0:r1, r0:r1])))
                    continue
                # rows r0..r1 against columns 0 .. k1 (to the end of the diagonal block)
                D = K.dcov_block(P, idx[r0:r1], idx[:k1], which, theta, kernel, alpha)
                # columns before the diagonal block: strictly lower, twice
                q[which] += float(a[r0:r1] @ (D[:, :k0] @ a[:k0]))
                t[which] += 2.0 * float(np.sum(S[r0:r1, :k0] * D[:, :k0]))
                # the diagonal block (full and symmetric in both matrices):
                # its rows r0..r1 contribute once each
                q[which] += 0.5 * float(a[r0:r1] @ (D[:, k0:k1] @ a[k0:k1]))
                t[which] += float(np.sum(S[r0:r1, k0:k1] * D[:, k0:k1]))
    # 1/2 a^T D a: a strictly lower entry stands for the pair (j, k), (k, j),
    # so it carries 1/2 * 2 = 1; the diagonal blocks carry 1/2
    return q, t


def loglik_large(P, z, theta, kernel, alpha=1.0, bs=8192):
    """(l, log|Sigma|, Sigma^-1 z) for large n by the blocked in-place
    Cholesky factorization of one n x n buffer (eq. loglikelihood)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = P.shape[0]
    S, blk, logdet = _blocked_cholesky(P, theta, kernel, alpha, bs)
    x = _blocked_backward(S, blk, _blocked_forward(S, blk, z))
    ell = -0.5 * float(z @ x) - 0.5 * logdet - 0.5 * n * LOG2PI
    return ell, logdet, x


def sample_loglik_large(P, w, theta, kernel, alpha=1.0, bs=8192):
    """For large n: z = L w (a draw from N(0, Sigma) given w ~ N(0, I)) with the
    blocked Cholesky factor L, and for that z the exact l, log|Sigma| and
    Sigma^-1 z = L^-T w (so z^T Sigma^-1 z = w^T w)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = P.shape[0]
    S, blk, logdet = _blocked_cholesky(P, theta, kernel, alpha, bs)
    z = _blocked_lower_matvec(S, blk, w)
    x = _blocked_backward(S, blk, w)
    ell = -0.5 * float(w @ w) - 0.5 * logdet - 0.5 * n * LOG2PI
    return z, ell, logdet, x


def score_large(P, theta, kernel, alpha=1.0, bs=8192, z=None, w=None, log=None):
    """l, log|Sigma|, Sigma^-1 z and the score g = q - t/2 (eq. gradient) for
    large n in one n x n buffer: blocked Cholesky Sigma = L L^T, then
    L^-1 in place, then the lower triangle of Sigma^-1 = L^-T L^-1 in place,
    and the traces Tr(Sigma^-1 Sigma_i) against Sigma_i generated blockwise.
    Give either z, or w for the model draw z = L w (then z^T Sigma^-1 z =
    w^T w and Sigma^-1 z = L^-T w).  Returns a dict with ell, logdet, alpha,
    q, t, g and, for a model draw, z."""
    import time
    P = np.ascontiguousarray(P, dtype=np.float64)
    n = P.shape[0]
    say = log or (lambda *_: None)
    t0 = time.time()
    S, blk, logdet = _blocked_cholesky(P, theta, kernel, alpha, bs)
    say("cholesky %.1f s" % (time.time() - t0))
    out = {"logdet": logdet}
    if w is not None:
        w = np.asarray(w, dtype=np.float64)
        z = _blocked_lower_matvec(S, blk, w)
        a = _blocked_backward(S, blk, w)
        quad = float(w @ w)
        out["z"] = z
    else:
        z = np.asarray(z, dtype=np.float64)
        a = _blocked_backward(S, blk, _blocked_forward(S, blk, z))
        quad = float(z @ a)
    out["ell"] = -0.5 * quad - 0.5 * logdet - 0.5 * n * LOG2PI
    out["alpha"] = a
    _blocked_tri_inverse(S, blk)
    say("triangular inverse %.1f s" % (time.time() - t0))
    _blocked_inverse_from_tri_inverse(S, blk)
    say("inverse %.1f s" % (time.time() - t0))
    q, t = _blocked_score_terms(S, blk, P, a, theta, kernel, alpha)
    say("score terms %.1f s" % (time.time() - t0))
    out["q"], out["t"], out["g"] = q, t, q - 0.5 * t
    return out
