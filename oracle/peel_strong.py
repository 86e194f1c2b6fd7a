"""Matrix peeling of a symmetric operator in the strongly admissible
hierarchical format, and the trace from the leaves' diagonal blocks (oracle;
TEST INFRASTRUCTURE ONLY).

Section 3 of the paper peels the weakly admissible format (every sibling
block compressed) and points to the strongly admissible form of the peeling
algorithm for kernels whose adjacent blocks are not of low rank (the remark
after Theorem 2; the "strong" columns of the peeling tables).  The paper
leaves that form's details to its reference, so this module states the reading
it follows, on the same quadtree as the factorization:

* Level-l nodes: the boxes of depth l and the leaves of depth below l (a leaf
  stays itself on every finer level).  The parent node of a depth-l box is its
  parent; a leaf carried down from a coarser level is its own parent node.
  Two nodes touch when their closed squares intersect (computed exactly on
  integer cell coordinates).
* Admissible blocks of level l: pairs (i, j) of level-l nodes that do not
  touch while their parent nodes touch (or coincide).  Every pair of distinct
  leaves that do not touch is admissible at exactly one level; touching
  leaves form the near field, which is never compressed.
* After the blocks of the coarser levels are subtracted, G_l = G - sum_{m<l}
  G^(m) is zero between level-l nodes whose parent nodes do not touch.  So a
  probe block that gives every node j of one colour a Gaussian block Omega_j
  samples, in the rows of a node i, exactly G_l(I_i, I_j) Omega_j for the one
  node j of that colour whose parent touches i's parent, provided no two nodes
  of a colour share such an i.  The colouring: greedy, in node order, over
  the conflict graph "j and j' both have a parent touching the parent of some
  node".  On a complete quadtree this needs 36 colours (6 x 6 cells around
  each parent's neighbourhood).
* Per admissible pair, the randomized low-rank approximation of eq.
  lowrankapprox, with the same orth (column-pivoted QR, |R_jj| > eps_peel
  |R_11|), oversampling, adaptive probe counts and stored form
  (U_ij, M_ij, U_ji) as the weak form (oracle.peel).
* Extraction: leaves coloured so that no two touching leaves share a colour;
  E gives every leaf of one colour an identity block in that colour's columns,
  H = (G - sum_m G^(m)) E, and Tr G ~= sum over leaves of Tr H(I_b, block of
  b's colour) (only the leaf's own diagonal block reaches those entries).

Probes: Philox4x32-10 normals with counter (DOF, column, level, 2) keyed by the
seed (the weak form uses stream 0 and the Hutchinson estimator stream 1).
"""
import numpy as np

from . import philox
from .peel import orth, round8, OVERSAMPLE, MIN_COLS

STRONG_STREAM = 2
FIRST_COLS = 64


def cell_coords(tree):
    """Integer cell coordinates (X, Y) of every box at its own depth: the
    root is (0, 0); a child at quadrant q (NW, NE, SW, SE) of (X, Y) is
    (2X + [q east], 2Y + [q north])."""
    X = np.zeros(tree.nbox, dtype=np.int64)
    Y = np.zeros(tree.nbox, dtype=np.int64)
    for b in range(1, tree.nbox):
        p, q = int(tree.parent[b]), int(tree.quad[b])
        X[b] = 2 * X[p] + (1 if q in (1, 3) else 0)
        Y[b] = 2 * Y[p] + (1 if q in (0, 1) else 0)
    return X, Y


def touch(tree, X, Y, a, b):
    """Closed squares of boxes a and b intersect (exact integer test)."""
    da, db = int(tree.depth[a]), int(tree.depth[b])
    D = max(da, db)
    sa, sb = 1 << (D - da), 1 << (D - db)
    ax0, ax1 = X[a] * sa, (X[a] + 1) * sa
    bx0, bx1 = X[b] * sb, (X[b] + 1) * sb
    ay0, ay1 = Y[a] * sa, (Y[a] + 1) * sa
    by0, by1 = Y[b] * sb, (Y[b] + 1) * sb
    return ax0 <= bx1 and bx0 <= ax1 and ay0 <= by1 and by0 <= ay1


def level_nodes(tree, lev):
    """Level-lev nodes: the boxes of depth lev and the leaves of depth < lev,
    in box-id order."""
    return [b for b in range(tree.nbox)
            if tree.depth[b] == lev or (tree.is_leaf[b] and tree.depth[b] < lev)]


def parent_node(tree, b, lev):
    return int(tree.parent[b]) if tree.depth[b] == lev else b


def admissible_pairs(tree, X, Y, lev):
    """Pairs (i, j), i < j in node order, of level-lev nodes that do not touch
    while their parent nodes touch."""
    nodes = level_nodes(tree, lev)
    out = []
    for a in range(len(nodes)):
        for c in range(a + 1, len(nodes)):
            i, j = nodes[a], nodes[c]
            if touch(tree, X, Y, i, j):
                continue
            if touch(tree, X, Y, parent_node(tree, i, lev), parent_node(tree, j, lev)):
                out.append((i, j))
    return out


def greedy_colors(nodes, conflicts):
    """Smallest colour not used by an already coloured conflicting node, in
    the given node order.  conflicts: dict node -> set of nodes."""
    color = {}
    for b in nodes:
        used = {color[c] for c in conflicts[b] if c in color}
        k = 0
        while k in used:
            k += 1
        color[b] = k
    return color


def probe_colors(tree, X, Y, lev):
    """Colours of the level-lev nodes for the sampling at that level: nodes
    whose parents both touch the parent of some node get different colours."""
    nodes = level_nodes(tree, lev)
    par = {b: parent_node(tree, b, lev) for b in nodes}
    conflicts = {b: set() for b in nodes}
    parents = sorted(set(par.values()))
    for p in parents:
        window = [b for b in nodes if touch(tree, X, Y, p, par[b])]
        for b in window:
            conflicts[b].update(c for c in window if c != b)
    return greedy_colors(nodes, conflicts)


def leaf_colors(tree, X, Y):
    """Colours of the leaves with no two touching leaves alike."""
    leaves = [b for b in range(tree.nbox) if tree.is_leaf[b]]
    conflicts = {b: {c for c in leaves if c != b and touch(tree, X, Y, b, c)} for b in leaves}
    return greedy_colors(leaves, conflicts), leaves


def next_cols(prev_rank):
    """Probe count per colour at the next level: the largest admissible-block
    rank of the level above plus the oversampling (the ranks of separated
    blocks change little from level to level), at least MIN_COLS."""
    return round8(max(MIN_COLS, prev_rank + OVERSAMPLE))


def grow_cols(total, maxrank):
    return round8(max((3 * total + 1) // 2, maxrank + 2 * OVERSAMPLE))


class StrongPeeler:
    """Joint strong-admissibility peeling of nop symmetric operators given as
    one apply W -> [G_op W]."""

    def __init__(self, tree, applies, nop, eps_peel, seed):
        self.t = tree
        self.applies = applies
        self.nop = nop
        self.eps = eps_peel
        self.seed = int(seed)
        self.X, self.Y = cell_coords(tree)
        self.blocks = [[] for _ in range(nop)]  # per op, per level: {(i, j): (U_ij, M_ij, U_ji)}
        self.cols = {}
        self.ranks = {}
        self.colors = {}

    def rows(self, b):
        t = self.t
        return slice(int(t.begin[b]), int(t.begin[b]) + int(t.count[b]))

    def probes(self, lev, box, j0, c):
        t = self.t
        d = np.arange(t.begin[box], t.begin[box] + t.count[box], dtype=np.uint64)
        j = np.arange(j0, j0 + c, dtype=np.uint64)
        D, J = np.meshgrid(d, j, indexing="ij")
        return philox.normal(D, J, lev, STRONG_STREAM, self.seed)

    def lowrank_apply(self, op, Xm, upto):
        """sum_{m < upto} G^(m) Xm for operator op."""
        out = np.zeros_like(Xm)
        for m in range(1, upto):
            for (i, j), (U1, M, U2) in self.blocks[op][m - 1].items():
                Ii, Ij = self.rows(i), self.rows(j)
                out[Ii] += U1 @ (M @ (U2.T @ Xm[Ij]))
                out[Ij] += U2 @ (M.T @ (U1.T @ Xm[Ii]))
        return out

    def run(self):
        t = self.t
        n = t.n
        prev = None
        for lev in range(1, t.max_depth + 1):
            pairs = admissible_pairs(t, self.X, self.Y, lev)
            if not pairs:
                for op in range(self.nop):
                    self.blocks[op].append({})
                continue
            color = probe_colors(t, self.X, self.Y, lev)
            ncol = 1 + max(color.values())
            self.colors[lev] = ncol
            nodes = sorted(color)
            c = FIRST_COLS if prev is None else next_cols(prev)
            total = 0
            Om = {b: np.zeros((int(t.count[b]), 0)) for b in nodes}
            # Yc[op][b][k]: rows of node b in the column block of colour k
            Yc = [{b: [np.zeros((int(t.count[b]), 0)) for _ in range(ncol)] for b in nodes}
                  for _ in range(self.nop)]
            while True:
                newc = c - total
                Wm = np.zeros((n, ncol * newc))
                for b in nodes:
                    k = color[b]
                    blk = self.probes(lev, b, total, newc)
                    Om[b] = np.concatenate([Om[b], blk], axis=1)
                    Wm[self.rows(b), k * newc:(k + 1) * newc] = blk
                outs = self.applies(Wm)
                for op in range(self.nop):
                    B = outs[op] - self.lowrank_apply(op, Wm, lev)
                    for b in nodes:
                        rb = B[self.rows(b)]
                        for k in range(ncol):
                            Yc[op][b][k] = np.concatenate([Yc[op][b][k], rb[:, k * newc:(k + 1) * newc]], axis=1)
                total = c
                need = False
                maxrank = 0
                for op in range(self.nop):
                    for (i, j) in pairs:
                        for (a, bb) in ((i, j), (j, i)):
                            kk = orth(Yc[op][a][color[bb]], self.eps).shape[1]
                            maxrank = max(maxrank, kk)
                            if kk + OVERSAMPLE > total and total < t.count[bb]:
                                need = True
                if not need:
                    break
                c = grow_cols(total, maxrank)
            prev = maxrank
            self.cols[lev] = total
            self.ranks[lev] = maxrank
            for op in range(self.nop):
                blk = {}
                for (i, j) in pairs:
                    Yij = Yc[op][i][color[j]]
                    Yji = Yc[op][j][color[i]]
                    U1 = orth(Yij, self.eps)
                    U2 = orth(Yji, self.eps)
                    A1 = Om[i].T @ U1
                    C = Om[i].T @ Yij
                    A2 = U2.T @ Om[j]
                    M = np.linalg.pinv(A1) @ C @ np.linalg.pinv(A2)
                    blk[(i, j)] = (U1, M, U2)
                self.blocks[op].append(blk)
        # extraction of the leaves' diagonal blocks
        lcol, leaves = leaf_colors(t, self.X, self.Y)
        ncl = 1 + max(lcol.values())
        nL = int(max(t.count[b] for b in leaves))
        E = np.zeros((n, ncl * nL))
        for b in leaves:
            k = lcol[b]
            E[t.begin[b] + np.arange(t.count[b]), k * nL + np.arange(t.count[b])] = 1.0
        outs = self.applies(E)
        traces = []
        for op in range(self.nop):
            H = outs[op] - self.lowrank_apply(op, E, t.max_depth + 1)
            tr = 0.0
            for b in leaves:
                k = lcol[b]
                tr += float(np.sum(H[t.begin[b] + np.arange(t.count[b]), k * nL + np.arange(t.count[b])]))
            traces.append(tr)
        self.leaf_colors = ncl
        self.n_leaf_cols = nL
        return traces


def peel_traces_strong(applies, tree, nop, eps_peel, seed):
    """Traces of nop symmetric operators, peeled in the strongly admissible format."""
    return StrongPeeler(tree, applies, nop, eps_peel, seed).run()
