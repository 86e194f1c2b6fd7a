"""Covariance kernels and their parameter derivatives (oracle, FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parameterisation (a reading of the paper, which leaves the variance implicit):
theta = (rho, sigma2, nugget).  For two *distinct* observations i != j at
distance r,

    Sigma_ij = sigma2 * k(r / rho),        Sigma_ii = sigma2 * k(0) + nugget,

with the scaled correlation k(s) from the closed forms of the Matern family
(eq. diffkernels, nu = 1/2, 3/2, 5/2) or the rational quadratic kernel with a
length scale (eq. rationalquadratic and the rho form that follows it):

    Matern 1/2   k(s) = exp(-s)
    Matern 3/2   k(s) = (1 + sqrt3 s) exp(-sqrt3 s)
    Matern 5/2   k(s) = (1 + sqrt5 s + 5 s^2 / 3) exp(-sqrt5 s)
    RQ(alpha)    k(s) = (1 + s^2 / (2 alpha))^(-alpha)

k(0) = 1 for all four.  The nugget term is the Kronecker delta on observation
indices (the additive white-noise model of the remark after eq. specmatern).

Derivatives with respect to rho (Sigma_i = dSigma/dtheta_i in eq. gradient):

    Matern 1/2   sigma2 * (r / rho^2) exp(-r/rho)
    Matern 3/2   sigma2 * 3 r^2 / rho^3 * exp(-sqrt3 r / rho)
    Matern 5/2   sigma2 * 5 r^2 / (3 rho^3) * (1 + sqrt5 r / rho) exp(-sqrt5 r / rho)
    RQ(alpha)    sigma2 * r^2 / rho^3 * (1 + r^2 / (2 alpha rho^2))^(-alpha-1)

and they vanish on the diagonal.  d/dsigma2 gives k(r/rho) (1 on the diagonal),
d/dnugget gives the identity.

Anisotropic kernels of the runtime experiments (eq. specmatern, eq. specrq),
theta = (theta_1, theta_2, nugget), no variance factor:

    Sigma_ij = k(s),  s^2 = dx^2 / theta_1^2 + dy^2 / theta_2^2,   Sigma_ii = 1 + nugget,

with k the Matern 3/2 or RQ(alpha) form above.  Writing h = -dk/d(s^2)
(Matern 3/2: 3/2 exp(-sqrt3 s); RQ: 1/2 (1 + s^2/(2 alpha))^(-alpha-1)),
dSigma_ij/dtheta_1 = h 2 dx^2 / theta_1^3 and dSigma_ij/dtheta_2 = h 2 dy^2 / theta_2^3
(zero on the diagonal), and d/dnugget gives the identity.
"""
import numpy as np

MATERN12, MATERN32, MATERN52, RQ, MATERN32_ANISO, RQ_ANISO = 0, 1, 2, 3, 4, 5
KERNEL_NAMES = {MATERN12: "matern12", MATERN32: "matern32", MATERN52: "matern52", RQ: "rq",
                MATERN32_ANISO: "matern32_aniso", RQ_ANISO: "rq_aniso"}


def is_aniso(kernel):
    return kernel in (MATERN32_ANISO, RQ_ANISO)
SQRT3 = np.sqrt(3.0)
SQRT5 = np.sqrt(5.0)


def corr(s, kernel, alpha=1.0):
    """Scaled correlation k(s), s = r / rho >= 0 (elementwise)."""
    s = np.asarray(s, dtype=np.float64)
    if kernel == MATERN12:
        return np.exp(-s)
    if kernel == MATERN32:
        return (1.0 + SQRT3 * s) * np.exp(-SQRT3 * s)
    if kernel == MATERN52:
        return (1.0 + SQRT5 * s + (5.0 / 3.0) * s * s) * np.exp(-SQRT5 * s)
    if kernel == RQ:
        return (1.0 + s * s / (2.0 * alpha)) ** (-alpha)
    raise ValueError("unknown kernel %r" % (kernel,))


def dcorr_drho(r, rho, kernel, alpha=1.0):
    """d/drho of k(r / rho) at fixed r (elementwise); zero at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    s = r / rho
    if kernel == MATERN12:
        return (r / (rho * rho)) * np.exp(-s)
    if kernel == MATERN32:
        return 3.0 * r * r / (rho ** 3) * np.exp(-SQRT3 * s)
    if kernel == MATERN52:
        return (5.0 * r * r / (3.0 * rho ** 3)) * (1.0 + SQRT5 * s) * np.exp(-SQRT5 * s)
    if kernel == RQ:
        return (r * r / rho ** 3) * (1.0 + s * s / (2.0 * alpha)) ** (-alpha - 1.0)
    raise ValueError("unknown kernel %r" % (kernel,))


def distances(X, Y):
    """Euclidean distances between rows of X (m x 2) and rows of Y (n x 2).

    Written with explicit coordinate differences so that D(X, Y) = D(Y, X)^T
    holds bitwise (|a - b| and |b - a| round identically)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    dx = X[:, 0][:, None] - Y[:, 0][None, :]
    dy = X[:, 1][:, None] - Y[:, 1][None, :]
    return np.sqrt(dx * dx + dy * dy)


def _aniso_parts(X, Y, theta):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    dx = X[:, 0][:, None] - Y[:, 0][None, :]
    dy = X[:, 1][:, None] - Y[:, 1][None, :]
    ux, uy = dx / float(theta[0]), dy / float(theta[1])
    return dx, dy, ux * ux + uy * uy


def cross_cov(X, Y, theta, kernel, alpha=1.0):
    """Kernel entries for every pair (no nugget: distinct observations):
    sigma2 k(|x - y| / rho), or k(s) of the scaled distance for the
    anisotropic kernels."""
    if is_aniso(kernel):
        _, _, s2 = _aniso_parts(X, Y, theta)
        return corr(np.sqrt(s2), MATERN32 if kernel == MATERN32_ANISO else RQ, alpha)
    rho, sigma2 = float(theta[0]), float(theta[1])
    return sigma2 * corr(distances(X, Y) / rho, kernel, alpha)


def cross_dcov(X, Y, which, theta, kernel, alpha=1.0):
    """d/dtheta_which of the kernel entries for every pair (which = 0: rho or
    theta_1; 1: theta_2 of the anisotropic kernels)."""
    if is_aniso(kernel):
        dx, dy, s2 = _aniso_parts(X, Y, theta)
        if kernel == MATERN32_ANISO:
            h = 1.5 * np.exp(-SQRT3 * np.sqrt(s2))
        else:
            h = 0.5 * (1.0 + s2 / (2.0 * alpha)) ** (-alpha - 1.0)
        d, th = (dx, float(theta[0])) if which == 0 else (dy, float(theta[1]))
        return h * 2.0 * d * d / th ** 3
    assert which == 0
    rho, sigma2 = float(theta[0]), float(theta[1])
    return sigma2 * dcorr_drho(distances(X, Y), rho, kernel, alpha)


def cross_dcov_drho(X, Y, theta, kernel, alpha=1.0):
    """d/drho (d/dtheta_1) of the kernel entries for every pair."""
    return cross_dcov(X, Y, 0, theta, kernel, alpha)


def cov_block(P, rows, cols, theta, kernel, alpha=1.0):
    """Sigma(rows, cols) for observation index arrays rows, cols into P.

    The nugget is added where the observation index of the row equals that of
    the column (Kronecker delta on indices)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    B = cross_cov(P[rows], P[cols], theta, kernel, alpha)
    same = rows[:, None] == cols[None, :]
    if np.any(same):
        # k(0) = 1 exactly; rebuild the diagonal entries without rounding noise.
        B[same] = (1.0 if is_aniso(kernel) else float(theta[1])) + float(theta[2])
    return B


def dcov_block(P, rows, cols, which, theta, kernel, alpha=1.0):
    """Sigma_i(rows, cols) for parameter index which (0 = rho, 1 = sigma2, 2 = nugget)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    same = rows[:, None] == cols[None, :]
    if which == 0 or (which == 1 and is_aniso(kernel)):
        B = cross_dcov(P[rows], P[cols], which, theta, kernel, alpha)
        B[same] = 0.0
        return B
    if which == 1:
        rho = float(theta[0])
        B = corr(distances(P[rows], P[cols]) / rho, kernel, alpha)
        B[same] = 1.0
        return B
    if which == 2:
        return same.astype(np.float64)
    raise ValueError("parameter index must be 0, 1 or 2")
