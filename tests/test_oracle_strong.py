"""Pins of the strong-admissibility peeling oracle (oracle/peel_strong.py):
the block structure (every pair of separated leaves compressed at exactly one
level, touching leaves never), the probe colourings (each sampled row block
sees one source per colour), exact recovery of an explicit strongly
admissible hierarchical matrix and of a block-diagonal one, and the traces of
an RSF's operators against their dense traces."""
import numpy as np
import pytest

from oracle import kernels as K
from oracle import peel, rsf
from oracle import peel_strong as ps
import workloads as W


def _grid(m):
    g = (np.arange(m) + 0.5) / m
    return np.stack(np.meshgrid(g, g), axis=-1).reshape(-1, 2)


def _trees():
    return {"complete": rsf.Tree(_grid(32), 16),
            "adaptive": rsf.Tree(W.mixed_points(900, 3, 0.03, 5, 6), 20)}


def _inside(t, a, i):
    """Leaf a lies inside node i."""
    return t.begin[i] <= t.begin[a] < t.begin[i] + t.count[i]


@pytest.mark.parametrize("kind", ["complete", "adaptive"])
def test_every_separated_leaf_pair_is_compressed_exactly_once(kind):
    t = _trees()[kind]
    X, Y = ps.cell_coords(t)
    leaves = [b for b in range(t.nbox) if t.is_leaf[b]]
    pairs = [(lev, i, j) for lev in range(1, t.max_depth + 1) for (i, j) in ps.admissible_pairs(t, X, Y, lev)]
    # the integer touch test against the geometry of the squares
    for a in leaves[:40]:
        for b in leaves[:40]:
            gx = abs(t.cx[a] - t.cx[b]) <= t.half[a] + t.half[b] + 1e-12
            gy = abs(t.cy[a] - t.cy[b]) <= t.half[a] + t.half[b] + 1e-12
            assert ps.touch(t, X, Y, a, b) == (gx and gy)
    for ia, a in enumerate(leaves):
        for b in leaves[ia + 1:]:
            cover = [(lev, i, j) for (lev, i, j) in pairs
                     if (_inside(t, a, i) and _inside(t, b, j)) or (_inside(t, a, j) and _inside(t, b, i))]
            if ps.touch(t, X, Y, a, b):
                assert cover == []
            else:
                assert len(cover) == 1
    for lev, i, j in pairs:
        assert not ps.touch(t, X, Y, i, j)


@pytest.mark.parametrize("kind", ["complete", "adaptive"])
def test_colourings_separate_every_sampled_window(kind):
    t = _trees()[kind]
    X, Y = ps.cell_coords(t)
    for lev in range(1, t.max_depth + 1):
        nodes = ps.level_nodes(t, lev)
        col = ps.probe_colors(t, X, Y, lev)
        par = {b: ps.parent_node(t, b, lev) for b in nodes}
        for i in nodes:
            seen = {}
            for j in nodes:
                if ps.touch(t, X, Y, par[i], par[j]):
                    assert col[j] not in seen, (lev, i, j, seen.get(col[j]))
                    seen[col[j]] = j
        if kind == "complete" and lev >= 3:
            assert 1 + max(col.values()) == 36
        if kind == "complete" and lev == 2:
            assert 1 + max(col.values()) == 16
    lcol, leaves = ps.leaf_colors(t, X, Y)
    for a in leaves:
        for b in leaves:
            if a != b and ps.touch(t, X, Y, a, b):
                assert lcol[a] != lcol[b]


def _explicit_strong_matrix(t, rank, seed):
    """A symmetric matrix in the strongly admissible format of tree t (tree
    order): a random rank-`rank` block for every admissible pair and random
    dense blocks between touching leaves."""
    X, Y = ps.cell_coords(t)
    rng = np.random.default_rng(seed)
    n = t.n
    G = np.zeros((n, n))
    sl = lambda b: slice(int(t.begin[b]), int(t.begin[b] + t.count[b]))  # noqa: E731
    for lev in range(1, t.max_depth + 1):
        for (i, j) in ps.admissible_pairs(t, X, Y, lev):
            U = rng.standard_normal((t.count[i], rank))
            V = rng.standard_normal((t.count[j], rank))
            Bl = U @ rng.standard_normal((rank, rank)) @ V.T
            G[sl(i), sl(j)] = Bl
            G[sl(j), sl(i)] = Bl.T
    leaves = [b for b in range(t.nbox) if t.is_leaf[b]]
    for ia, a in enumerate(leaves):
        for b in leaves[ia:]:
            if a == b:
                D = rng.standard_normal((t.count[a], t.count[a]))
                G[sl(a), sl(a)] = D + D.T
            elif ps.touch(t, X, Y, a, b):
                D = rng.standard_normal((t.count[a], t.count[b]))
                G[sl(a), sl(b)] = D
                G[sl(b), sl(a)] = D.T
    return G


@pytest.mark.parametrize("kind", ["complete", "adaptive"])
def test_exact_on_explicit_strongly_admissible_matrix(kind):
    t = _trees()[kind]
    G = _explicit_strong_matrix(t, 3, 7)
    sp = ps.StrongPeeler(t, lambda Wm: [G @ Wm], 1, 1e-10, 9)
    tr = sp.run()[0]
    assert tr == pytest.approx(np.trace(G), rel=1e-10)
    # every recovered block equals the planted one
    X, Y = ps.cell_coords(t)
    for lev in range(1, t.max_depth + 1):
        for (i, j), (U1, M, U2) in sp.blocks[0][lev - 1].items():
            Gij = G[t.begin[i]:t.begin[i] + t.count[i], t.begin[j]:t.begin[j] + t.count[j]]
            r = min(3, int(t.count[i]), int(t.count[j]))
            assert U1.shape[1] == r and U2.shape[1] == r
            np.testing.assert_allclose(U1 @ M @ U2.T, Gij, rtol=0, atol=1e-9 * np.abs(Gij).max())


def test_exact_on_block_diagonal():
    t = _trees()["adaptive"]
    rng = np.random.default_rng(4)
    G = np.zeros((t.n, t.n))
    for b in range(t.nbox):
        if t.is_leaf[b]:
            D = rng.standard_normal((t.count[b], t.count[b]))
            s = slice(int(t.begin[b]), int(t.begin[b] + t.count[b]))
            G[s, s] = D @ D.T
    tr = ps.peel_traces_strong(lambda Wm: [G @ Wm], t, 1, 1e-8, 3)[0]
    assert tr == pytest.approx(np.trace(G), rel=1e-13)


def test_traces_of_factor_against_dense_and_weak():
    """B B^T and B F_rho B^T of the oracle RSF (F^-1 = B^T B): the strongly
    admissible peel within 20 eps_peel of the dense traces, and next to the
    weakly admissible peel."""
    P = W.uniform_points(700, 11)
    theta = (0.08, 1.0, 1e-3)
    F = rsf.Factor(P, theta, K.MATERN32, 1e-9, 24)
    Fr = rsf.Factor(P, theta, K.MATERN32, 1e-9, 24, mode="mult", tree=F.tree)

    def applies(Wm):
        H = F.half_down(Wm)
        return [F.half_up(H), F.half_up(Fr.apply(H))]

    eps_peel = 1e-6
    sp = ps.StrongPeeler(F.tree, applies, 2, eps_peel, 5)
    tr = sp.run()
    Bt = F.half_down(np.eye(700))
    dense = [np.trace(F.half_up(Bt.copy())), np.trace(F.half_up(Fr.apply(Bt.copy())))]
    np.testing.assert_allclose(tr, dense, rtol=20 * eps_peel)
    tw = peel.peel_traces(applies, F.tree, 2, eps_peel, 5)
    np.testing.assert_allclose(tr, tw, rtol=40 * eps_peel)
    assert max(sp.colors.values()) <= 36
