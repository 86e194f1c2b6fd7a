"""Pins for the oracle's recursive skeletonization factorization and peeling.

The RSF is an approximation, so it is pinned by: brute-force checks of the
quadtree rules, the ID against LAPACK's pivoted QR (dgeqp3) and against its
own defining inequality, the exact cases (one box = dense Cholesky; a diagonal
covariance = every ID has rank 0), exact algebraic identities of the sweeps,
agreement with the dense matrix to the ID tolerance, power-of-two scale
invariance, and peeling on operators whose trace is known.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, peel, rsf
from oracle import kernels as K
from oracle import philox
import workloads as W

GOLD = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(GOLD + "/philox4x32_10_kat.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_box_muller_moments():
    d = np.arange(200000, dtype=np.uint64)
    x = philox.normal(d, 3, 2, 0, 12345)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1.0) < 0.01


def _brute_tree_check(P, tree, leaf):
    n = P.shape[0]
    assert sorted(tree.perm.tolist()) == list(range(n))
    for b in range(tree.nbox):
        idx = tree.perm[tree.begin[b]:tree.begin[b] + tree.count[b]]
        # points lie in the box (closed on the south/west, by the >= split rule)
        assert np.all(np.abs(P[idx, 0] - tree.cx[b]) <= tree.half[b] + 1e-14 * (1.0 + np.abs(P).max()))
        assert np.all(np.abs(P[idx, 1] - tree.cy[b]) <= tree.half[b] + 1e-14 * (1.0 + np.abs(P).max()))
        kids = tree.kids(b)
        if tree.is_leaf[b]:
            assert tree.count[b] <= leaf
            # stable partition: a leaf keeps the relative input order
            assert np.all(np.diff(idx) > 0)
        else:
            assert tree.count[b] > leaf
            assert sum(tree.count[c] for c in kids) == tree.count[b]
            for c in kids:
                q = tree.quad[c]
                sub = tree.perm[tree.begin[c]:tree.begin[c] + tree.count[c]]
                east = P[sub, 0] >= tree.cx[b]
                north = P[sub, 1] >= tree.cy[b]
                assert np.all(east == (q in (1, 3))) and np.all(north == (q in (0, 1)))
            # children are laid out NW, NE, SW, SE one after the other
            assert [tree.quad[c] for c in kids] == sorted(tree.quad[c] for c in kids)


@pytest.mark.parametrize("n,leaf,seed", [(1, 4, 1), (7, 8, 2), (300, 16, 3), (1000, 64, 4)])
def test_tree_rules_brute_force(n, leaf, seed):
    P = W.uniform_points(n, seed)
    tree = rsf.Tree(P, leaf)
    _brute_tree_check(P, tree, leaf)


def test_tree_adaptive_clustered():
    P = W.mixed_points(2000, 4, 0.01, 5, 6)
    tree = rsf.Tree(P, 32)
    _brute_tree_check(P, tree, 32)
    leaf_depths = {int(tree.depth[b]) for b in range(tree.nbox) if tree.is_leaf[b]}
    assert len(leaf_depths) > 1  # adaptive: leaves at several depths


def test_id_matches_lapack_pivoted_qr_and_definition():
    rng = np.random.default_rng(0)
    m, a, r = 120, 40, 12
    sv = np.logspace(0, -14, a)
    U, _ = np.linalg.qr(rng.standard_normal((m, a)))
    V, _ = np.linalg.qr(rng.standard_normal((a, a)))
    A = (U * sv) @ V.T
    eps = 1e-7
    k, piv, T = rsf.cpqr_id(A, eps)
    _, R, P = sla.qr(A, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    k_lapack = int(np.sum(d > eps * d[0]))
    assert k == k_lapack
    assert list(piv[:k]) == list(P[:k])
    err = np.linalg.norm(A[:, piv[k:]] - A[:, piv[:k]] @ T, 2)
    assert err <= 10 * eps * np.linalg.norm(A, 2)
    # exactly rank-deficient: rank r, exact reconstruction up to rounding
    B = rng.standard_normal((m, r)) @ rng.standard_normal((r, a))
    k, piv, T = rsf.cpqr_id(B, 1e-12)
    assert k == r
    assert np.linalg.norm(B[:, piv[k:]] - B[:, piv[:k]] @ T) <= 1e-10 * np.linalg.norm(B)
    # zero matrix: rank 0
    k, piv, T = rsf.cpqr_id(np.zeros((5, 3)), 1e-6)
    assert k == 0


def test_single_box_is_dense_cholesky():
    P = W.uniform_points(50, 3)
    theta = (0.2, 1.0, 1e-3)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-6, 64)
    assert F.tree.max_depth == 0
    z = W.gaussian(50, 4)
    ell, logdet, a = dense.loglik(P, z, theta, K.MATERN32)
    assert F.logdet == pytest.approx(logdet, rel=1e-13)
    np.testing.assert_allclose(F.from_tree(F.solve(F.to_tree(z))), a, rtol=1e-10)


def test_diagonal_covariance_is_exact():
    g = np.arange(16.0)
    P = np.stack(np.meshgrid(g, g), axis=-1).reshape(-1, 2)
    theta = (1e-3, 1.3, 0.2)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-9, 16, n_prox=64, prox_rings=1)
    assert F.tree.max_depth >= 2
    assert all(v == 0 for v in F.rank.values())
    n = P.shape[0]
    assert F.logdet == pytest.approx(n * math.log(1.5), rel=1e-14)
    z = W.gaussian(n, 2)
    np.testing.assert_allclose(F.from_tree(F.solve(F.to_tree(z))), z / 1.5, rtol=1e-15)


@pytest.fixture(scope="module")
def f1024():
    P = W.uniform_points(1024, 11)
    theta = (0.1, 1.0, 1e-4)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-9, 64, n_prox=256, prox_rings=4)
    Fr = rsf.Factor(P, theta, K.MATERN32, 1e-9, 64, n_prox=256, prox_rings=4, mode="mult", tree=F.tree)
    return P, theta, F, Fr


def test_sweep_identities(f1024):
    P, theta, F, Fr = f1024
    v = W.gaussian((1024, 3), 5)
    np.testing.assert_allclose(F.apply(F.solve(v)), v, rtol=0, atol=1e-10 * np.abs(v).max())
    np.testing.assert_allclose(F.sqrt(F.sqrt_t(v)), F.apply(v), rtol=1e-14, atol=1e-14)
    # multi-column sweeps equal column-by-column sweeps
    x1 = F.solve(v[:, 1])
    np.testing.assert_allclose(F.solve(v)[:, 1], x1, rtol=0, atol=1e-11 * np.abs(x1).max())
    # F and F_rho are symmetric: u^T F v = v^T F u
    u = W.gaussian(1024, 6)
    w = W.gaussian(1024, 7)
    assert u @ F.apply(w) == pytest.approx(w @ F.apply(u), rel=1e-12)
    assert u @ Fr.apply(w) == pytest.approx(w @ Fr.apply(u), rel=1e-10)
    # the solve's halves: B is the inverse of the separately written F^(1/2),
    # B^T is its transpose, and B^T B is the solve
    np.testing.assert_allclose(F.half_up(F.sqrt(v)), v, rtol=0, atol=1e-11 * np.abs(v).max())
    assert u @ F.half_up(w) == pytest.approx(F.half_down(u) @ w, rel=1e-12)
    x = F.solve(v)
    np.testing.assert_allclose(F.half_down(F.half_up(v)), x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_factor_approximates_sigma(f1024):
    P, theta, F, Fr = f1024
    S = dense.cov_matrix(P, theta, K.MATERN32)
    Sr = dense.dcov_matrix(P, 0, theta, K.MATERN32)
    V = W.gaussian((1024, 4), 8)
    Vt = F.to_tree(V)
    err = np.linalg.norm(F.from_tree(F.apply(Vt)) - S @ V) / np.linalg.norm(S @ V)
    assert err < 1e-8
    err_r = np.linalg.norm(Fr.from_tree(Fr.apply(Vt)) - Sr @ V) / np.linalg.norm(Sr @ V)
    assert err_r < 1e-8
    # B Sigma B^T = I to the factorization accuracy (F^-1 = B^T B)
    SVt = F.to_tree(S @ F.from_tree(F.half_down(Vt)))
    assert np.linalg.norm(F.half_up(SVt) - Vt) <= 1e-6 * np.linalg.norm(Vt)
    ld = dense.loglik(P, V[:, 0], theta, K.MATERN32)[1]
    assert abs(F.logdet - ld) <= 10 * 1e-9 * abs(ld)


def test_accuracy_improves_with_eps():
    P = W.uniform_points(1024, 11)
    theta = (0.1, 1.0, 1e-4)
    S = dense.cov_matrix(P, theta, K.MATERN32)
    V = W.gaussian((1024, 2), 9)
    errs = []
    for eps in (1e-4, 1e-6, 1e-8):
        F = rsf.Factor(P, theta, K.MATERN32, eps, 64)
        errs.append(np.linalg.norm(F.from_tree(F.apply(F.to_tree(V))) - S @ V) / np.linalg.norm(S @ V))
    assert errs[0] > 10 * errs[1] > 100 * errs[2] * 0.1
    assert all(e < 10 * eps for e, eps in zip(errs, (1e-4, 1e-6, 1e-8)))


def test_power_of_two_scale_invariance():
    P = W.uniform_points(600, 3)
    theta = (0.1, 1.0, 1e-4)
    F1 = rsf.Factor(P, theta, K.MATERN32, 1e-7, 32)
    F2 = rsf.Factor(P * 8.0, (0.8, 1.0, 1e-4), K.MATERN32, 1e-7, 32)
    assert np.array_equal(F1.tree.perm, F2.tree.perm)
    for b in F1.S:
        assert np.array_equal(F1.S[b], F2.S[b])
    assert F1.logdet == F2.logdet


def test_peel_exact_on_block_diagonal_and_hodlr():
    P = W.uniform_points(700, 21)
    tree = rsf.Tree(P, 40)
    n = 700
    rng = np.random.default_rng(3)
    # block-diagonal over the leaves: every sibling block is 0, trace exact
    G = np.zeros((n, n))
    for b in range(tree.nbox):
        if tree.is_leaf[b]:
            s = slice(tree.begin[b], tree.begin[b] + tree.count[b])
            B = rng.standard_normal((tree.count[b], tree.count[b]))
            G[s, s] = B + B.T
    tr = peel.peel_traces(lambda X: [G @ X], tree, 1, 1e-10, 5)[0]
    assert tr == pytest.approx(np.trace(G), rel=1e-12, abs=1e-9)
    # explicit HODLR matrix: rank-3 sibling blocks at every level plus diagonal leaf blocks
    H = G.copy()
    for lev in range(1, tree.max_depth + 1):
        for p in tree.levels[lev - 1]:
            ks = tree.kids(int(p))
            for a in range(len(ks)):
                for c in range(a + 1, len(ks)):
                    i, j = ks[a], ks[c]
                    si = slice(tree.begin[i], tree.begin[i] + tree.count[i])
                    sj = slice(tree.begin[j], tree.begin[j] + tree.count[j])
                    B = rng.standard_normal((tree.count[i], 3)) @ rng.standard_normal((3, tree.count[j]))
                    H[si, sj] += B
                    H[sj, si] += B.T
    pl = peel.Peeler(tree, lambda X: [H @ X], 1, 1e-10, 6)
    tr = pl.run()[0]
    assert tr == pytest.approx(np.trace(H), rel=1e-10, abs=1e-8)
    assert all(r <= 3 for r in pl.ranks.values())


def test_peeled_traces_of_factor(f1024):
    P, theta, F, Fr = f1024
    n = 1024
    # Tr F = n (sigma2 + nugget) exactly for the true Sigma; F matches Sigma to ~eps
    trF = peel.peel_traces(lambda X: [F.apply(X)], F.tree, 1, 1e-9, 3)[0]
    assert trF == pytest.approx(n * (theta[1] + theta[2]), rel=1e-8)
    trinv = peel.peel_traces(lambda X: [F.solve(X)], F.tree, 1, 1e-9, 4)[0]
    assert trinv == pytest.approx(dense.trace_inverse(P, theta, K.MATERN32), rel=1e-6)


def test_method_gradient_close_to_dense():
    P = W.uniform_points(1024, 11)
    theta = (0.1, 1.0, 1e-4)
    z = dense.sample(P, W.gaussian(1024, 12), theta, K.MATERN32)
    o = rsf.loglik_grad(P, z, theta, K.MATERN32, 1e-9, 64, seed=33, n_prox=64, prox_rings=1)
    d = dense.loglik_and_grad(P, z, theta, K.MATERN32, want_terms=True)
    assert o["ell"] == pytest.approx(d["ell"], rel=1e-7)
    assert o["logdet"] == pytest.approx(d["logdet"], rel=1e-10)
    np.testing.assert_allclose(o["t"], d["t"], rtol=1e-8)
    assert np.linalg.norm(o["g"] - d["g"]) <= 1e-5 * np.linalg.norm(d["g"])


def test_rademacher_draws():
    """+1/-1 from the lowest bit of Philox word 0 (counter (d, j, 0, 1)):
    balanced and uncorrelated across DOFs and columns."""
    d = np.arange(4096)[:, None]
    j = np.arange(64)[None, :]
    U = philox.rademacher(d, j, 77)
    assert set(np.unique(U)) == {-1.0, 1.0}
    assert abs(U.mean()) < 4.0 / np.sqrt(U.size)
    C = U.T @ U / U.shape[0]
    off = C[~np.eye(64, dtype=bool)]
    assert np.abs(off).max() < 5.0 / np.sqrt(U.shape[0])
    # the draw is the published generator's word, not a reseeded stream
    x0 = philox.philox4x32_10(d[:5, 0], 3, 0, 1, 77, 0)[0]
    assert np.array_equal(philox.rademacher(d[:5, 0], 3, 77), np.where(x0 % 2 == 0, 1.0, -1.0))


def test_hutchinson_exact_on_diagonal_and_unbiased():
    """Hutchinson (eq. hutch) on a diagonal covariance is exact for every
    probe; on a correlated one its mean over many probes lies within the
    Rademacher standard error sqrt(2 sum_{i != j} G_ij^2 / q) of the dense
    traces of B B^T and B F_rho B^T."""
    # far-apart sites: Sigma = (sigma2 + nugget) I to rounding
    P = W.uniform_points(300, 4) * 1e3
    theta = (1e-3, 2.0, 0.5)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-9, 32, n_prox=64, prox_rings=1)
    Fr = rsf.Factor(P, theta, K.MATERN32, 1e-9, 32, n_prox=64, prox_rings=1, mode="mult", tree=F.tree)
    ti, tr = rsf.hutchinson_traces(F, Fr, 3, 5)
    assert ti == pytest.approx(300 / 2.5, rel=1e-12)
    assert abs(tr) < 1e-12
    # correlated: exact traces of the two symmetric operators from dense matrices
    n = 512
    P = W.uniform_points(n, 21)
    theta = (0.1, 1.0, 1e-2)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-10, 64, n_prox=64, prox_rings=1)
    Fr = rsf.Factor(P, theta, K.MATERN32, 1e-10, 64, n_prox=64, prox_rings=1, mode="mult", tree=F.tree)
    Bt = F.half_down(np.eye(n))          # B^T
    G0 = Bt.T @ Bt                        # B B^T
    G1 = Bt.T @ Fr.apply(Bt)              # B F_rho B^T
    q = 4000
    ti, tr = rsf.hutchinson_traces(F, Fr, q, 9)
    for est, G in ((ti, G0), (tr, 0.5 * (G1 + G1.T))):
        se = np.sqrt(2.0 * (np.sum(G * G) - np.sum(np.diag(G) ** 2)) / q)
        assert abs(est - np.trace(G)) < 4.0 * se
    # and the traces are those of Sigma^-1 and Sigma^-1 Sigma_rho
    S = dense.cov_matrix(P, theta, K.MATERN32)
    Si = np.linalg.inv(S)
    Sr = dense.dcov_matrix(P, 0, theta, K.MATERN32)
    assert np.trace(G0) == pytest.approx(np.trace(Si), rel=1e-8)
    assert np.trace(G1) == pytest.approx(np.sum(Si * Sr.T), rel=1e-7)


def test_conditional_mean_and_covariance():
    """The remark after Algorithm 1: with F on [x'; x] and F22 on x, the
    conditional mean matches Sigma_12 Sigma_22^-1 z and the square root S of
    the deviation satisfies S S^T = Sigma_11 - Sigma_12 Sigma_22^-1 Sigma_21,
    both from the dense covariance, to the factorization accuracy."""
    n1, n2 = 60, 700
    Pall = W.uniform_points(n1 + n2, 31)
    theta = (0.1, 1.0, 1e-3)
    F = rsf.Factor(Pall, theta, K.MATERN32, 1e-10, 32, n_prox=64, prox_rings=1)
    F22 = rsf.Factor(Pall[n1:], theta, K.MATERN32, 1e-10, 32, n_prox=64, prox_rings=1)
    S = dense.cov_matrix(Pall, theta, K.MATERN32)
    S11, S12, S22 = S[:n1, :n1], S[:n1, n1:], S[n1:, n1:]
    z = W.gaussian((n2, 2), 33)
    mu = rsf.conditional_mean(F, F22, z)
    mu_d = S12 @ np.linalg.solve(S22, z)
    assert np.linalg.norm(mu - mu_d) <= 1e-6 * np.linalg.norm(mu_d)
    Sq = rsf.conditional_deviation(F, F22, np.eye(n1 + n2))  # the n1 x n operator S
    C = Sq @ Sq.T
    C_d = S11 - S12 @ np.linalg.solve(S22, S12.T)
    assert np.linalg.norm(C - C_d) <= 1e-6 * np.linalg.norm(C_d)


def test_profile_likelihood_gradient_and_rsf():
    """eq. prof: the dense gradient formula agrees with central differences of
    the dense profile likelihood, and the RSF version (Sherman-Morrison, peeled
    traces) agrees with the dense one to the factorization / peeling accuracy."""
    P = W.uniform_points(400, 17)
    theta = np.array([0.12, 1.0, 2e-3])
    z = dense.sample(P, W.gaussian(400, 18), tuple(theta), K.MATERN32) + 0.3
    ell, g = dense.profile_loglik(P, z, tuple(theta), K.MATERN32, want_grad=True)
    for i in range(3):
        h = 1e-5 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (dense.profile_loglik(P, z, tuple(tp), K.MATERN32) - dense.profile_loglik(P, z, tuple(tm), K.MATERN32)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-6 * np.abs(g).max())
    o = rsf.profile_loglik_grad(P, z, tuple(theta), K.MATERN32, 1e-10, 64, eps_peel=1e-9, seed=3, n_prox=64,
                                prox_rings=1)
    assert o["ell"] == pytest.approx(ell, rel=1e-9)
    assert np.linalg.norm(o["g"] - g) <= 1e-6 * np.linalg.norm(g)


@pytest.mark.parametrize("kernel", [K.MATERN32_ANISO, K.RQ_ANISO])
def test_aniso_method_gradient_close_to_dense(kernel):
    """Anisotropic kernels: the factorization's l and log|F| and the peeled
    traces Tr F^-1 F_theta1, Tr F^-1 F_theta2, Tr F^-1 against the dense
    definitions."""
    P = W.uniform_points(1024, 13)
    theta = (0.12, 0.05, 1e-4)
    z = dense.sample(P, W.gaussian(1024, 14), theta, kernel)
    o = rsf.loglik_grad(P, z, theta, kernel, 1e-9, 64, seed=35, n_prox=64, prox_rings=1)
    d = dense.loglik_and_grad(P, z, theta, kernel, want_terms=True)
    # l is a small difference of terms of size n (z^T Sigma^-1 z ~ n): compare on that scale
    assert o["ell"] == pytest.approx(d["ell"], rel=1e-7, abs=1e-8 * 1024)
    assert o["logdet"] == pytest.approx(d["logdet"], rel=1e-9)
    np.testing.assert_allclose(o["q"], d["q"], rtol=1e-6)
    np.testing.assert_allclose(o["t"], d["t"], rtol=1e-7)
    assert np.linalg.norm(o["g"] - d["g"]) <= 1e-5 * np.linalg.norm(d["g"])
