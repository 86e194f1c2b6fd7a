"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers (points, Gaussian vectors) and names the
parameters of each workload; it holds none of the method's arithmetic.  Both the
HIP path's tests/benchmark and the oracle consume what it returns.

All draws use numpy's PCG64 ``default_rng(seed)``.
"""
import numpy as np

MATERN12, MATERN32, MATERN52, RQ, MATERN32_ANISO, RQ_ANISO = 0, 1, 2, 3, 4, 5


def uniform_points(n, seed):
    """n points iid uniform in [0, 1]^2 (the scattered-data stand-in)."""
    return np.random.default_rng(seed).random((n, 2))


def grid_points(side, extent=100.0):
    """side x side regular grid discretising [0, extent]^2 (Section 5.1 setup)."""
    g = (np.arange(side) + 0.5) * (extent / side)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def mixed_points(n, n_blobs, blob_sigma, seed_points, seed_centres):
    """Half uniform in [0,1]^2, half in n_blobs Gaussian blobs (non-uniform density)."""
    rng = np.random.default_rng(seed_points)
    n_uni = n // 2
    per = (n - n_uni) // n_blobs
    cen = np.random.default_rng(seed_centres).random((n_blobs, 2))
    parts = [rng.random((n_uni, 2))]
    for b in range(n_blobs):
        m = per if b < n_blobs - 1 else (n - n_uni) - per * (n_blobs - 1)
        parts.append(cen[b] + blob_sigma * rng.standard_normal((m, 2)))
    return np.concatenate(parts, axis=0)


def gaussian(shape, seed):
    """iid N(0, 1) draws (right-hand sides; w in z = Sigma^(1/2) w)."""
    return np.random.default_rng(seed).standard_normal(shape)


# The named workloads.  theta = (length scale rho, variance sigma2, nugget), or
# (theta_1, theta_2, nugget) for the anisotropic kernels.
WORKLOADS = {
    # small case: Matern 3/2, single 64-point proxy ring, tight tolerance
    "c1_matern32_n1024": dict(n=1024, points=("uniform", 11), w_seed=12, kernel=MATERN32,
                              theta=(0.1, 1.0, 1e-4), alpha=1.0, eps=1e-9, leaf=64,
                              n_prox=64, prox_rings=1, nrhs=1),
    # rational quadratic, 8 right-hand sides
    "c2_rq_n16384": dict(n=16384, points=("uniform", 21), w_seed=22, kernel=RQ,
                         theta=(0.05, 1.0, 1e-3), alpha=1.0, eps=1e-6, leaf=64,
                         n_prox=256, prox_rings=4, nrhs=8),
    # the log-likelihood + score workload
    "c3_matern32_n65536": dict(n=65536, points=("uniform", 31), w_seed=32, peel_seed=33,
                               kernel=MATERN32, theta=(0.05, 1.0, 1e-4), alpha=1.0, eps=1e-6,
                               leaf=64, n_prox=256, prox_rings=4, nrhs=1),
    # non-uniform density, Matern 5/2, larger leaves
    "c5_matern52_n262144": dict(n=262144, points=("mixed", 51, 52), w_seed=53, peel_seed=54,
                                kernel=MATERN52, theta=(0.03, 1.0, 1e-4), alpha=1.0, eps=1e-6,
                                leaf=128, n_prox=256, prox_rings=4, nrhs=1),
    # the paper's MLE profiling setup (Section 5): a 256 x 256 grid on
    # [0, 100]^2, anisotropic Matern 3/2 with theta = (10, 7), noise 1e-4,
    # eps_peel 1e-6 and eps_fact = eps_peel / 1000
    "g1_matern32aniso_grid256": dict(n=65536, points=("grid", 100.0), w_seed=62, peel_seed=63,
                                     kernel=MATERN32_ANISO, theta=(10.0, 7.0, 1e-4), alpha=1.0,
                                     eps=1e-9, eps_peel=1e-6, leaf=64, n_prox=256, prox_rings=4, nrhs=1),
    # the paper's MLE example (Section 5): 2^16 scattered sites (here uniform
    # in [0, 100]^2), anisotropic Matern 3/2, theta* = (10, 7), noise 1e-4 held
    # fixed, eps_fact 1e-9, eps_peel 1e-6, the fit starting from (3, 30)
    "m1_matern32aniso_scattered65536": dict(n=65536, points=("uniform", 71, 100.0), w_seed=72, peel_seed=73,
                                            kernel=MATERN32_ANISO, theta=(10.0, 7.0, 1e-4),
                                            theta0=(3.0, 30.0, 1e-4), alpha=1.0, eps=1e-9, eps_peel=1e-6,
                                            leaf=64, n_prox=256, prox_rings=4, nrhs=1),
    # the same grid with the rational quadratic kernel of eq. specrq (alpha = 1/2)
    "g2_rqaniso_grid256": dict(n=65536, points=("grid", 100.0), w_seed=64, peel_seed=65,
                               kernel=RQ_ANISO, theta=(10.0, 7.0, 1e-4), alpha=0.5,
                               eps=1e-9, eps_peel=1e-6, leaf=64, n_prox=256, prox_rings=4, nrhs=1),
}


def batch_instances(count, master_seed, n_lo=2048, n_hi=32768, rho_lo=0.02, rho_hi=0.2, sigma2=1.0,
                    nugget=1e-4):
    """Independent instances: n_i log-uniform in [n_lo, n_hi]; points uniform
    in a rectangle of unit area and aspect A_i ~ U[1, 4] (sqrt(A_i) x
    1/sqrt(A_i), the two sides swapped with probability 1/2); length scale
    rho_i ~ U[rho_lo, rho_hi].  The master seed draws the sizes, shapes and
    length scales; instance i draws its points with seed 100 * master_seed + i.
    Returns a list of (points, theta)."""
    rng = np.random.default_rng(master_seed)
    n = np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))).astype(int)
    aspect = rng.uniform(1.0, 4.0, count)
    swap = rng.random(count) < 0.5
    rho = rng.uniform(rho_lo, rho_hi, count)
    out = []
    for i in range(count):
        w, h = np.sqrt(aspect[i]), 1.0 / np.sqrt(aspect[i])
        if swap[i]:
            w, h = h, w
        P = np.random.default_rng(100 * master_seed + i).random((int(n[i]), 2)) * np.array([w, h])
        out.append((P, (float(rho[i]), sigma2, nugget)))
    return out


# batches of independent instances (Matern 3/2)
BATCHES = {
    "c4_batch64_matern32": dict(count=64, master_seed=41, w_seed=42, peel_seed=43, kernel=MATERN32,
                                alpha=1.0, eps=1e-6, leaf=64, n_prox=256, prox_rings=4),
}


def workload_points(name, n=None):
    """Points of a named workload (optionally with a different n, same recipe)."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    kind = w["points"]
    if kind[0] == "uniform":
        return uniform_points(n, kind[1]) * (kind[2] if len(kind) > 2 else 1.0)
    if kind[0] == "mixed":
        return mixed_points(n, 16, 0.02, kind[1], kind[2])
    if kind[0] == "grid":
        side = int(round(np.sqrt(n)))
        assert side * side == n, "grid workloads take square n"
        return grid_points(side, kind[1])
    raise ValueError(kind)
