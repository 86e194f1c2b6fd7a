"""Anisotropic kernels (eq. specmatern, eq. specrq) on the HIP path against the
oracle and the dense definitions: skeletons, log|F|, solves, l, the score
(three factorizations: Sigma, Sigma_theta1, Sigma_theta2; B B^T, B F_theta1 B^T
and B F_theta2 B^T peeled from one set of probes), Hutchinson traces, batches,
and the MLE driver against a dense MLE.
"""
import math

import numpy as np
import pytest
import torch

import paper_1603_08057_amd as R
from oracle import dense, rsf
from oracle import kernels as K
import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _entrywise(got, ref, rtol, what):
    """Every entry within rtol of the reference's largest entry (a few wrong
    rows cannot hide under the norm of the whole block)."""
    err = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(ref)))
    print("  %s: max entry error %.2e of max |ref| (bar %.0e)" % (what, err, rtol), flush=True)
    np.testing.assert_allclose(got, ref, rtol=0, atol=rtol * float(np.max(np.abs(ref))))


@pytest.mark.parametrize("kernel,pts,theta,eps,leaf", [
    (K.MATERN32_ANISO, ("grid", 48), (10.0, 7.0, 1e-4), 1e-9, 64),
    (K.RQ_ANISO, ("uniform", 3001), (0.12, 0.05, 1e-3), 1e-7, 50),
])
def test_aniso_factor_matches_oracle(kernel, pts, theta, eps, leaf):
    print("aniso factor kernel=%d %s" % (kernel, pts), flush=True)
    P = W.grid_points(pts[1]) if pts[0] == "grid" else W.uniform_points(pts[1], 41)
    n = P.shape[0]
    F = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=leaf)
    O = rsf.Factor(P, theta, kernel, eps, leaf)
    info = F.tree_info(want_perm=True)
    assert np.array_equal(np.array(info["perm"]), O.tree.perm)
    for lev in range(1, info["depth"] + 1):
        offs, idx = F.skeletons(lev)
        for i, b in enumerate(O.tree.levels[lev]):
            assert np.array_equal(np.array(idx[offs[i]:offs[i + 1]], dtype=np.int64), O.tree.perm[O.S[int(b)]])
    assert F.logdet == pytest.approx(O.logdet, rel=1e-11)
    B = W.gaussian((n, 2), 5)
    X = F.solve(_t(B)).cpu().numpy()
    Xo = O.from_tree(O.solve(O.to_tree(B)))
    _entrywise(X, Xo, 1e-9, "F^-1 B")
    Y = F.apply(_t(B)).cpu().numpy()
    Yo = O.from_tree(O.apply(O.to_tree(B)))
    _entrywise(Y, Yo, 1e-12, "F B")
    z = B[:, 0]
    ello = -0.5 * float(z @ Xo[:, 0]) - 0.5 * O.logdet - 0.5 * n * math.log(2 * math.pi)
    assert F.loglik(_t(z)) == pytest.approx(ello, rel=1e-9)
    # the approximation: log|F| near the dense log|Sigma|
    _, logdet_d, _ = dense.loglik(P, z, theta, kernel)
    assert abs(F.logdet - logdet_d) <= 1e3 * eps * abs(logdet_d)


@pytest.mark.parametrize("kernel,pts,theta,eps,n_prox,rings", [
    (K.MATERN32_ANISO, ("grid", 32), (10.0, 7.0, 1e-4), 1e-9, 64, 1),
    (K.RQ_ANISO, ("uniform", 2500), (0.12, 0.05, 1e-3), 1e-7, 256, 4),
])
def test_aniso_grad_matches_oracle_and_dense(kernel, pts, theta, eps, n_prox, rings, monkeypatch):
    print("aniso grad kernel=%d %s" % (kernel, pts), flush=True)
    P = W.grid_points(pts[1]) if pts[0] == "grid" else W.uniform_points(pts[1], 42)
    n = P.shape[0]
    z = dense.sample(P, W.gaussian(n, 12), theta, kernel)
    eps_peel = 1e-6
    F = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=64, n_prox=n_prox, prox_rings=rings)
    g, info = F.grad(_t(z), eps_peel, 33)
    o = rsf.loglik_grad(P, z, theta, kernel, eps, 64, eps_peel=eps_peel, seed=33, n_prox=n_prox,
                        prox_rings=rings)
    same = all(info.peel_cols[lev] == c for lev, c in o["peel_cols"].items())
    print("  own probe schedule %s the oracle's" % ("equals" if same else "differs from"), flush=True)
    for lev, c in o["peel_cols"].items():
        assert abs(info.peel_rank[lev] - o["peel_ranks"][lev]) <= 2
    np.testing.assert_allclose(list(info.q), o["q"], rtol=1e-9)
    # rounding-level parity on the oracle's probe schedule (no tolerance fallback)
    monkeypatch.setenv("RSFGP_TEST_PEEL_COLS", ",".join(str(o["peel_cols"][lev]) for lev in sorted(o["peel_cols"])))
    gs, infs = F.grad(_t(z), eps_peel, 33)
    monkeypatch.delenv("RSFGP_TEST_PEEL_COLS")
    for lev, c in o["peel_cols"].items():
        assert infs.peel_cols[lev] == c
    np.testing.assert_allclose(list(infs.t), o["t"], rtol=1e-8)
    oscale = np.abs(o["q"]) + 0.5 * np.abs(o["t"])
    assert np.all(np.abs(np.array(gs) - o["g"]) <= 1e-8 * oscale)
    d = dense.loglik_and_grad(P, z, theta, kernel, want_terms=True)
    np.testing.assert_allclose(list(info.t), d["t"], rtol=20 * eps_peel)
    scale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
    assert np.all(np.abs(np.array(g) - d["g"]) <= 1e3 * eps * scale + 50 * eps_peel * scale)
    # a handle built with the score factorizations beside Sigma gives the same answer
    F2 = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=64, n_prox=n_prox, prox_rings=rings,
                  with_score=True)
    g2, _ = F2.grad(_t(z), eps_peel, 33)
    np.testing.assert_array_equal(np.array(g2), np.array(g))


def test_aniso_hutchinson_matches_oracle():
    print("aniso hutchinson", flush=True)
    theta = (0.12, 0.05, 1e-3)
    P = W.uniform_points(2500, 43)
    z = dense.sample(P, W.gaussian(2500, 12), theta, K.MATERN32_ANISO)
    F = R.Factor(_t(P), theta, kernel=K.MATERN32_ANISO, eps=1e-7, leaf=64)
    g, info = F.grad_hutch(_t(z), 8, 5)
    o = rsf.loglik_grad(P, z, theta, K.MATERN32_ANISO, 1e-7, 64, seed=5, hutch_probes=8)
    np.testing.assert_allclose(list(info.t), o["t"], rtol=1e-9)
    np.testing.assert_allclose(list(info.q), o["q"], rtol=1e-9)


def test_aniso_refusals():
    P = _t(W.uniform_points(256, 1))
    with pytest.raises(R.RsfError):
        R.Factor(P, (0.1, 0.1, 1e-3), kernel=K.MATERN32_ANISO, eps=1e-6, leaf=64, precision="mixed")
    F = R.Factor(P, (0.1, 0.1, 1e-3), kernel=K.MATERN32_ANISO, eps=1e-6, leaf=64)
    with pytest.raises(R.RsfError):
        F.profile_loglik(_t(W.gaussian(256, 2)))


def test_mle_matches_dense_mle():
    """The MLE driver (L-BFGS-B over log theta_1, log theta_2, nugget fixed,
    as in the paper's Section 5 example: theta* = (10, 7), start (3, 30),
    scattered points in [0, 100]^2) lands where a dense-likelihood MLE with
    the same optimizer lands."""
    from scipy.optimize import minimize
    print("mle n=1024", flush=True)
    n = 1024
    P = 100.0 * W.uniform_points(n, 71)
    kernel = K.MATERN32_ANISO
    z = dense.sample(P, W.gaussian(n, 72), (10.0, 7.0, 1e-4), kernel)
    r = R.fit(_t(P), _t(z), (3.0, 30.0, 1e-4), kernel, eps=1e-9, eps_peel=1e-6, seed=3)
    print(r, flush=True)

    def negl(x):
        th = np.array([math.exp(x[0]), math.exp(x[1]), 1e-4])
        d = dense.loglik_and_grad(P, z, th, kernel)
        return -d["ell"], -(d["g"] * th)[:2]

    rd = minimize(negl, np.log([3.0, 30.0]), jac=True, method="L-BFGS-B",
                  options=dict(maxiter=50, gtol=1e-5, ftol=1e-12))
    thd = np.exp(rd.x)
    print("dense MLE", thd, -rd.fun, flush=True)
    np.testing.assert_allclose(r.theta[:2], thd, rtol=2e-3)
    assert r.ell == pytest.approx(-rd.fun, abs=1e-3)
    assert r.theta[2] == 1e-4
    # the score at the estimate is small against its value at the start
    g0 = r.history[0][2]
    assert np.max(np.abs(r.grad[:2] * r.theta[:2])) <= 1e-2 * np.max(np.abs(g0[:2] * r.history[0][0][:2]))


def test_aniso_batched_scores_against_dense():
    """A batch of anisotropic instances (own theta_1, theta_2 each): every
    instance's score within the dense bound, and its log-det equal to a
    single-instance handle's."""
    print("aniso batch", flush=True)
    inst = [(W.uniform_points(700, 81), (0.15, 0.06, 1e-3)), (W.uniform_points(1500, 82), (0.05, 0.12, 1e-3)),
            (W.uniform_points(1100, 83), (0.1, 0.1, 1e-3))]
    B = R.BatchedFactor([_t(p) for p, _ in inst], [th for _, th in inst], kernel=K.MATERN32_ANISO, eps=1e-8,
                        leaf=64)
    zs = [dense.sample(p, W.gaussian(len(p), 90 + i), th, K.MATERN32_ANISO) for i, (p, th) in enumerate(inst)]
    eps_peel = 1e-6
    gs, _ = B.grad([_t(z) for z in zs], eps_peel, 19)
    for i, ((P, th), z) in enumerate(zip(inst, zs)):
        F = R.Factor(_t(P), th, kernel=K.MATERN32_ANISO, eps=1e-8, leaf=64)
        assert B.logdets[i] == pytest.approx(F.logdet, rel=1e-12)
        d = dense.loglik_and_grad(P, z, th, K.MATERN32_ANISO, want_terms=True)
        scale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
        err = np.abs(np.array(gs[i]) - d["g"]) / scale
        print("instance %d: g %s dense %s err/scale %s" % (i, np.array(gs[i]), d["g"], err), flush=True)
        assert np.all(err <= 1e3 * 1e-8 + 50 * eps_peel)
