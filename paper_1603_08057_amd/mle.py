"""Maximum likelihood estimation driver (the outer loop around Algorithm 1).

Each objective call factors Sigma(theta) (with the derivative factorizations
beside it) and returns -l(theta) and -g(theta) from the HIP library: the
log-likelihood of eq. loglikelihood and the score of eq. gradient with the
traces peeled.  A first-order quasi-Newton method (as in the paper's
Section 5 MLE example) takes the steps; here scipy's L-BFGS-B over
log theta, so that every parameter stays positive, with any subset of the
parameters held fixed (the paper fits theta_1, theta_2 of the anisotropic
kernel with the noise variance fixed).

Only the optimizer's own bookkeeping runs on the host: every likelihood and
score value comes from the library.
"""
import numpy as np

from ._lib import Factor


class FitResult:
    def __init__(self, theta, ell, grad, nfev, nit, success, message, history):
        self.theta = theta
        self.ell = ell
        self.grad = grad
        self.nfev = nfev
        self.nit = nit
        self.success = success
        self.message = message
        self.history = history

    def __repr__(self):
        return "FitResult(theta=%s, ell=%.10g, nit=%d, nfev=%d, success=%s)" % (
            list(self.theta), self.ell, self.nit, self.nfev, self.success)


def fit(points, z, theta0, kernel, eps=1e-9, eps_peel=1e-6, leaf=64, seed=0, fixed=(False, False, True),
        maxiter=50, gtol=1e-5, ftol=1e-12, log=None, **opts):
    """Maximise l(theta) from theta0 (a 3-vector in the kernel's order).

    points: (n, 2) float64 device tensor; z: (n,) float64 device tensor.
    fixed: which entries of theta stay at theta0 (default: the nugget).
    log: a writable text stream that gets one line per objective call, or None.
    Returns a FitResult with theta, l(theta), the score g(theta), and the
    (theta, l, g) history of every objective call."""
    from scipy.optimize import minimize

    theta0 = np.asarray(theta0, dtype=np.float64)
    assert theta0.shape == (3,) and np.all(theta0 > 0), "theta0 must hold three positive values"
    free = np.array([not f for f in fixed])
    assert free.any(), "nothing to fit"
    history = []

    def theta_of(x):
        th = theta0.copy()
        th[free] = np.exp(x)
        return th

    def objective(x):
        th = theta_of(x)
        F = Factor(points, tuple(float(v) for v in th), kernel=kernel, eps=eps, leaf=leaf, with_score=True,
                   **opts)
        try:
            ell = F.loglik(z)
            g, _ = F.grad(z, eps_peel, seed)
        finally:
            F.close()
        g = np.asarray(g, dtype=np.float64)
        history.append((th.copy(), ell, g.copy()))
        if log is not None:
            log.write("fit call %d: theta %s l %.10e g %s\n" % (len(history), th.tolist(), ell, g.tolist()))
            log.flush()
        # d(-l)/d(log theta_i) = -g_i theta_i
        return -ell, -(g * th)[free]

    r = minimize(objective, np.log(theta0[free]), jac=True, method="L-BFGS-B",
                 options=dict(maxiter=maxiter, gtol=gtol, ftol=ftol))
    th = theta_of(r.x)
    last = [h for h in history if np.array_equal(h[0], th)]
    if not last:
        objective(r.x)
        last = history[-1:]
    _, ell, g = last[-1]
    return FitResult(th, ell, g, r.nfev, r.nit, bool(r.success), str(r.message), history)
