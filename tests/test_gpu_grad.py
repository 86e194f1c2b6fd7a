"""Parity of the HIP score equations (peeled traces) with the oracle.

The oracle's peeling (oracle/peel.py) draws the same Philox probes and follows
the same adaptive rule, so the per-level probe counts must match exactly and
the traces / quadratic terms agree to rounding (relative 1e-8: the peeled
low-rank blocks are formed from the same samples through different but
equivalent range finders, so the difference is rounding amplified by the
conditioning of the core matrices).  Against the dense definitions the traces
must be within a few eps_peel.
"""
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


def _schedule(o):
    """The oracle run's probe columns per level as the test-only override."""
    return ",".join(str(o["peel_cols"][lev]) for lev in sorted(o["peel_cols"]))


@pytest.mark.parametrize("n,eps,n_prox,rings,kernel,theta", [
    (1024, 1e-9, 64, 1, K.MATERN32, (0.1, 1.0, 1e-4)),
    (2500, 1e-7, 256, 4, K.MATERN52, (0.06, 1.2, 1e-3)),
    (4096, 1e-6, 256, 4, K.MATERN32, (0.05, 1.0, 1e-4)),
])
def test_grad_matches_oracle_and_dense(n, eps, n_prox, rings, kernel, theta, monkeypatch):
    print("grad case n=%d eps=%g" % (n, eps), flush=True)
    P = W.uniform_points(n, 11)
    z = dense.sample(P, W.gaussian(n, 12), theta, kernel)
    eps_peel = 1e-6
    F = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=64, n_prox=n_prox, prox_rings=rings)
    g, info = F.grad(_t(z), eps_peel, 33)
    o = rsf.loglik_grad(P, z, theta, kernel, eps, 64, eps_peel=eps_peel, seed=33, n_prox=n_prox,
                        prox_rings=rings)
    # the rank of a sample block is a threshold decision on a decaying
    # spectrum taken by different (equivalent) factorizations on each side
    # (pivoted Cholesky of the Gram matrix here, pivoted QR in the oracle): a
    # difference of 1 or 2 at the threshold is rounding, and it can move the
    # next level's probe count
    same = all(info.peel_cols[lev] == c for lev, c in o["peel_cols"].items())
    print("  own probe schedule %s, oracle's %s (%s)" % ([info.peel_cols[lev] for lev in sorted(o["peel_cols"])],
          [o["peel_cols"][lev] for lev in sorted(o["peel_cols"])], "same" if same else "different"), flush=True)
    for lev, c in o["peel_cols"].items():
        assert abs(info.peel_rank[lev] - o["peel_ranks"][lev]) <= 2
    np.testing.assert_allclose(list(info.q), o["q"], rtol=1e-9)
    # parity at rounding level: the same probes, run with the oracle's probe
    # schedule (no tolerance fallback)
    monkeypatch.setenv("RSFGP_TEST_PEEL_COLS", _schedule(o))
    gs, infs = F.grad(_t(z), eps_peel, 33)
    monkeypatch.delenv("RSFGP_TEST_PEEL_COLS")
    for lev, c in o["peel_cols"].items():
        assert infs.peel_cols[lev] == c
    terr = np.abs(np.array(list(infs.t)) - o["t"]) / np.abs(o["t"])
    print("  traces vs oracle on its schedule: %s" % ["%.1e" % v for v in terr], flush=True)
    np.testing.assert_allclose(list(infs.t), o["t"], rtol=1e-8)
    np.testing.assert_allclose(list(infs.q), o["q"], rtol=1e-9)
    # g = q - t/2 cancels to O(sqrt n) at the generating theta: compare on the
    # scale of its halves
    oscale = np.abs(o["q"]) + 0.5 * np.abs(o["t"])
    assert np.all(np.abs(np.array(gs) - o["g"]) <= 1e-8 * oscale)
    d = dense.loglik_and_grad(P, z, theta, kernel, want_terms=True)
    np.testing.assert_allclose(list(info.t), d["t"], rtol=20 * eps_peel)
    # the score itself: relative to the scale of its two halves (they cancel)
    scale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
    gerr = np.abs(np.array(g) - d["g"]) / scale
    print("  vs dense: traces %s, score over |q| + |t|/2 %s, |g - g_dense| / |g_dense| %.1e"
          % (["%.1e" % v for v in np.abs(np.array(list(info.t)) - d["t"]) / np.abs(d["t"])],
             ["%.1e" % v for v in gerr], np.linalg.norm(np.array(g) - d["g"]) / np.linalg.norm(d["g"])), flush=True)
    # q_nugget = a^T a / 2 carries the forward error of a = F^-1 z, about
    # kappa(Sigma) times the factorization's backward error: 100 eps_fact
    # beside the traces' 10 eps_peel
    assert np.all(gerr <= 100 * eps + 10 * eps_peel)
    # repeatable: same seed, same answer
    g2, _ = F.grad(_t(z), eps_peel, 33)
    assert g2 == g


def test_grad_diagonal_covariance_exact():
    g0 = np.arange(16.0)
    P = np.stack(np.meshgrid(g0, g0), axis=-1).reshape(-1, 2)
    n = P.shape[0]
    theta = (1e-3, 1.3, 0.2)
    z = W.gaussian(n, 3)
    F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-9, leaf=16)
    g, info = F.grad(_t(z), 1e-8, 1)
    s = 1.5
    gs = 0.5 * float(z @ z) / s ** 2 - n / (2 * s)
    np.testing.assert_allclose(g, [0.0, gs, gs], rtol=1e-12, atol=1e-9)


def test_autograd_function_backward():
    P = W.uniform_points(1200, 13)
    theta = (0.08, 1.0, 1e-3)
    z = dense.sample(P, W.gaussian(1200, 14), theta, K.MATERN32)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    ell = R.loglik_fn(th, _t(P), _t(z), kernel=K.MATERN32, eps=1e-8, leaf=64, eps_peel=1e-7, seed=5)
    ell.backward()
    d = dense.loglik_and_grad(P, z, theta, K.MATERN32, want_terms=True)
    lscale = 0.5 * abs(float(z @ d["alpha"])) + 0.5 * abs(d["logdet"]) + 600 * np.log(2 * np.pi)
    assert abs(float(ell.detach()) - d["ell"]) <= 10 * 1e-8 * lscale
    gscale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
    assert np.all(np.abs(th.grad.numpy() - d["g"]) <= 1e-4 * gscale)


def test_autograd_recomputed_factor_gives_the_same_score():
    # backward with the forward factorization released and made again (the
    # memory-short path) against backward on the kept factorization
    P = W.uniform_points(1500, 17)
    theta = (0.07, 1.2, 1e-3)
    z = dense.sample(P, W.gaussian(1500, 18), theta, K.MATERN32)
    grads, ells = [], []
    # the first call also settles the level-step autotuner's choices
    for keep in (True, True, False, "auto"):
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        ell = R.loglik_fn(th, _t(P), _t(z), kernel=K.MATERN32, eps=1e-8, leaf=64, eps_peel=1e-7, seed=3,
                          keep_factor=keep)
        ell.backward()
        ells.append(float(ell.detach()))
        grads.append(th.grad.numpy().copy())
    for e, g in zip(ells[2:], grads[2:]):
        assert e == pytest.approx(ells[1], rel=1e-13)
        np.testing.assert_allclose(g, grads[1], rtol=1e-12, atol=0)


def test_tile_choice_changes_no_result(monkeypatch):
    # the batched products run on 128 x 128 or 64 x 64 tiles (the tile-shape
    # autotuner's choice); both accumulate every entry in the same order with
    # the same instruction, and split-K does not depend on the choice, so l,
    # log|Sigma| and the score agree bit for bit under either form and the tuned one
    P = W.uniform_points(4000, 21)
    theta = (0.06, 1.0, 1e-3)
    z = W.gaussian(4000, 22)
    out = []
    for tiles in ("128", "64", None):
        if tiles:
            monkeypatch.setenv("RSFGP_TEST_TILES", tiles)
        else:
            monkeypatch.delenv("RSFGP_TEST_TILES", raising=False)
        F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-8, leaf=64)
        ell = F.loglik(_t(z))
        ld = F.logdet
        g, _ = F.grad(_t(z), 1e-7, 4)
        F.close()
        out.append((ell, ld, np.array(g)))
    for ell, ld, g in out[1:]:
        assert ell == out[0][0] and ld == out[0][1]
        np.testing.assert_array_equal(g, out[0][2])


def test_grad_matches_central_difference_of_frozen_loglik():
    # the score of the approximate log-likelihood, with every ID tolerance tight,
    # against a central difference of the dense log-likelihood (relative step 1e-5)
    P = W.uniform_points(900, 15)
    theta = np.array([0.09, 1.0, 1e-3])
    z = dense.sample(P, W.gaussian(900, 16), theta, K.MATERN32)
    F = R.Factor(_t(P), tuple(theta), kernel=K.MATERN32, eps=1e-10, leaf=64)
    g, _ = F.grad(_t(z), 1e-9, 2)
    for i in range(3):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (dense.loglik(P, z, tp, K.MATERN32)[0] - dense.loglik(P, z, tm, K.MATERN32)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-4, abs=1e-3)


def test_with_score_builds_sigma_rho_alongside():
    """with_score: Sigma_rho factored on the side stream during the create
    call gives the same score, bitwise, as factoring it inside the grad call;
    the batched handle too."""
    print("with_score n=4096", flush=True)
    n, theta = 4096, (0.05, 1.0, 1e-4)
    P = W.uniform_points(n, 11)
    z = _t(W.gaussian(n, 12))
    kw = dict(kernel=K.MATERN32, eps=1e-6, leaf=64)
    F = R.Factor(_t(P), theta, **kw)
    g0, i0 = F.grad(z, 1e-6, 33)
    l0 = F.loglik(z)
    F.close()
    G = R.Factor(_t(P), theta, with_score=True, **kw)
    g1, i1 = G.grad(z, 1e-6, 33)
    l1 = G.loglik(z)
    G.close()
    assert l1 == l0
    assert list(g1) == list(g0)
    assert list(i1.peel_cols) == list(i0.peel_cols)
    pts = [_t(W.uniform_points(m, 20 + m)) for m in (700, 1500)]
    zs = [_t(W.gaussian(m, 30 + m)) for m in (700, 1500)]
    th = [theta, (0.08, 1.5, 1e-3)]
    B0 = R.BatchedFactor(pts, th, **kw)
    B1 = R.BatchedFactor(pts, th, with_score=True, **kw)
    a0, _ = B0.grad(zs, 1e-6, 7)
    a1, _ = B1.grad(zs, 1e-6, 7)
    assert np.array_equal(np.asarray(a0), np.asarray(a1))


@pytest.mark.parametrize("n,q", [(2500, 16), (4096, 8)])
def test_hutchinson_matches_oracle(n, q):
    """Hutchinson traces (eq. hutch) from the same Rademacher probes through
    B^T and F_rho: equal to the oracle's to rounding."""
    print("hutchinson n=%d q=%d" % (n, q), flush=True)
    theta = (0.06, 1.2, 1e-3)
    P = W.uniform_points(n, 11)
    z = dense.sample(P, W.gaussian(n, 12), theta, K.MATERN52)
    F = R.Factor(_t(P), theta, kernel=K.MATERN52, eps=1e-7, leaf=64)
    g, info = F.grad_hutch(_t(z), q, 5)
    o = rsf.loglik_grad(P, z, theta, K.MATERN52, 1e-7, 64, seed=5, hutch_probes=q)
    np.testing.assert_allclose(list(info.t), o["t"], rtol=1e-9)
    np.testing.assert_allclose(list(info.q), o["q"], rtol=1e-9)
    scale = np.abs(o["q"]) + 0.5 * np.abs(o["t"])
    assert np.all(np.abs(np.array(g) - o["g"]) <= 1e-9 * scale)
    # unbiased estimate of the peeled trace: within a generous statistical band
    gp, ip = F.grad(_t(z), 1e-6, 33)
    assert abs(info.t[2] - ip.t[2]) < 0.2 * abs(ip.t[2])


def test_hutchinson_exact_on_diagonal_and_batched():
    """A diagonal covariance makes every Rademacher probe exact; a batch draws
    the probes each instance draws alone."""
    P = W.uniform_points(700, 4) * 1e3
    theta = (1e-3, 2.0, 0.5)
    F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-9, leaf=32)
    z = _t(W.gaussian(700, 3))
    g, info = F.grad_hutch(z, 3, 9)
    assert info.t[2] == pytest.approx(700 / 2.5, rel=1e-12)
    pts = [W.uniform_points(m, 40 + m) for m in (900, 1700)]
    zs = [W.gaussian(m, 50 + m) for m in (900, 1700)]
    th = [(0.05, 1.0, 1e-4), (0.08, 1.5, 1e-3)]
    B = R.BatchedFactor([_t(p) for p in pts], th, kernel=K.MATERN32, eps=1e-6, leaf=64)
    gb, _ = B.grad_hutch([_t(x) for x in zs], 12, 4)
    for i in range(2):
        Fi = R.Factor(_t(pts[i]), th[i], kernel=K.MATERN32, eps=1e-6, leaf=64)
        gi, _ = Fi.grad_hutch(_t(zs[i]), 12, 4)
        np.testing.assert_allclose(gb[i], gi, rtol=1e-9, atol=1e-9 * np.max(np.abs(gi)))


def test_profile_likelihood_matches_oracle_and_dense():
    """eq. prof on the GPU: l~ and its gradient against the oracle's RSF
    version (same peeling, rounding level) and the dense definition."""
    print("profile likelihood n=1024 and 4096", flush=True)
    theta = (0.12, 1.0, 2e-3)
    P = W.uniform_points(1024, 17)
    z = dense.sample(P, W.gaussian(1024, 18), theta, K.MATERN32) + 0.3
    F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-10, leaf=64, n_prox=64, prox_rings=1)
    ell, g, info = F.profile_loglik(_t(z), 1e-9, 3)
    assert F.profile_loglik(_t(z), grad=False) == ell
    ld, gd = dense.profile_loglik(P, z, theta, K.MATERN32, want_grad=True)
    assert ell == pytest.approx(ld, rel=1e-8)
    assert np.linalg.norm(np.array(g) - gd) <= 1e-6 * np.linalg.norm(gd)
    P = W.uniform_points(4096, 19)
    theta = (0.05, 1.0, 1e-4)
    z = W.gaussian(4096, 20) + 1.0
    F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-6, leaf=64)
    ell, g, info = F.profile_loglik(_t(z), 1e-6, 33)
    o = rsf.profile_loglik_grad(P, z, theta, K.MATERN32, 1e-6, 64, eps_peel=1e-6, seed=33)
    assert ell == pytest.approx(o["ell"], rel=1e-10)
    np.testing.assert_allclose(list(info.t), o["t"], rtol=1e-8)
    np.testing.assert_allclose(list(info.q), o["quad"], rtol=1e-8)
    scale = 0.5 * np.abs(o["t"]) + 0.5 * 4096 * np.abs(o["quad"]) / o["zbeta"]
    assert np.all(np.abs(np.array(g) - o["g"]) <= 1e-8 * scale)
