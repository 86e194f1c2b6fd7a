"""Matrix peeling for weakly admissible symmetric operators and the trace
extraction at the leaves (oracle; TEST INFRASTRUCTURE ONLY).

Section 3.2 of the paper, written out plainly over the same quadtree as the
factorization (boxes are contiguous ranges of tree order):

* level l = 1 .. L, top down.  For every box j of depth l draw a Gaussian probe
  block Omega_j (|I_j| x c) and place it in the column block of W_k with k the
  quadrant of j inside its parent (Section 3.2.2; for an adaptive tree "j = k
  mod 4" is read as "quadrant index k").  Apply B = (G - sum_{m<l} G^(m)) W.
  For siblings i != j the rows I_i of the column block of j's quadrant sample
  G_ij Omega_j; by symmetry the rows I_j of i's block sample G_ij^T Omega_i.
* randomized low-rank approximation (eq. lowrankapprox):
      U_1 = orth(G_ij Omega_j), U_2 = orth(G_ji Omega_i),
      M   = (Omega_i^T U_1)^+ (Omega_i^T G_ij Omega_j) (U_2^T Omega_j)^+,
      G_ij ~= U_1 M U_2^T,    G_ji ~= U_2 M^T U_1^T,
  with orth by column-pivoted QR truncated where |R_jj| <= eps_peel |R_11|.
* ranks are found adaptively (the paper says "an adaptive procedure is used"):
  c columns per quadrant block are drawn; if some sibling block needs rank
  k > c - oversample (and c is still below the block's column count), the
  count grows by half (at least to the rank found plus twice the
  oversampling) and only the new columns are applied.
* extraction (Section 3.2.4): E has one identity block per leaf in n_L columns,
  H = (G - sum_m G^(m)) E, and Tr G ~= sum over leaves of Tr H(I_i, 1:n_i).

Several operators can be peeled together from the same probes (``applies``
returns one product per operator), which is how B B^T and B F_rho B^T
(F^-1 = B^T B) share the product B^T W.
"""
import numpy as np
import scipy.linalg as sla

from . import philox

OVERSAMPLE = 10
FIRST_COLS = 64
MIN_COLS = 24


def orth(Y, eps):
    """Orthonormal basis of the numerical range of Y (pivoted QR, relative
    threshold eps on |R_jj|)."""
    if Y.shape[1] == 0 or Y.shape[0] == 0:
        return np.zeros((Y.shape[0], 0))
    Q, R, _ = sla.qr(Y, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    if d.shape[0] == 0 or d[0] == 0.0:
        return np.zeros((Y.shape[0], 0))
    k = int(np.sum(d > eps * d[0]))
    return Q[:, :k]


def round8(c):
    return (c + 7) // 8 * 8


def first_cols(n):
    """Probe count at the first peeled level: the top-level sibling blocks have
    ranks that grow like sqrt(n) (Section 3.3), so 9/4 sqrt(n) (integer
    arithmetic), at least FIRST_COLS, rounded up to a multiple of 8."""
    import math
    return round8(max(FIRST_COLS, 9 * math.isqrt(n) // 4))


def next_cols(prev_rank, peeled):
    """Initial probe count per quadrant block at the next level from the
    largest rank found at the level above (peeled = levels peeled so far):
    1.5x after the first peeled level (the second level's sibling blocks of
    B F_rho B^T and B B^T have the larger ranks), 0.7x after the second,
    0.6x below that (the ranks shrink by at most half per level there), plus
    the oversampling, at least MIN_COLS, rounded up to a multiple of 8."""
    if peeled == 1:
        c = (3 * prev_rank + 1) // 2
    elif peeled == 2:
        c = (7 * prev_rank + 9) // 10
    else:
        c = (3 * prev_rank + 4) // 5
    return round8(max(MIN_COLS, c + OVERSAMPLE))


def grow_cols(total, maxrank):
    """Probe count after a level whose ranks were not resolved: 1.5x, at least
    the largest rank found plus twice the oversampling."""
    return round8(max((3 * total + 1) // 2, maxrank + 2 * OVERSAMPLE))


class Peeler:
    """Joint weak-admissibility peeling of nop symmetric operators."""

    def __init__(self, tree, applies, nop, eps_peel, seed):
        self.t = tree
        self.applies = applies
        self.nop = nop
        self.eps = eps_peel
        self.seed = int(seed)
        # per operator: list over levels of dict {(i, j): (U_i_seg, M_ij, U_j_seg)} for i < j
        self.blocks = [[] for _ in range(nop)]
        self.cols = {}
        self.ranks = {}

    def probes(self, level, box, j0, c):
        t = self.t
        d = np.arange(t.begin[box], t.begin[box] + t.count[box], dtype=np.uint64)
        j = np.arange(j0, j0 + c, dtype=np.uint64)
        D, J = np.meshgrid(d, j, indexing="ij")
        return philox.normal(D, J, level, 0, self.seed)

    def lowrank_apply(self, op, X, upto):
        """sum_{m < upto} G^(m) X for operator op (X in tree order, n x c)."""
        t = self.t
        out = np.zeros_like(X)
        for m in range(1, upto):
            for (i, j), (U1, M, U2) in self.blocks[op][m - 1].items():
                Ii = slice(t.begin[i], t.begin[i] + t.count[i])
                Ij = slice(t.begin[j], t.begin[j] + t.count[j])
                out[Ii] += U1 @ (M @ (U2.T @ X[Ij]))
                out[Ij] += U2 @ (M.T @ (U1.T @ X[Ii]))
        return out

    def run(self):
        t = self.t
        n = t.n
        prev = None
        peeled = 0
        for lev in range(1, t.max_depth + 1):
            boxes = [int(b) for b in t.levels[lev]]
            pairs = []
            for p in t.levels[lev - 1]:
                ks = t.kids(int(p))
                for a in range(len(ks)):
                    for b in range(a + 1, len(ks)):
                        pairs.append((ks[a], ks[b]))
            if not pairs:
                for op in range(self.nop):
                    self.blocks[op].append({})
                continue
            c = first_cols(n) if prev is None else next_cols(prev, peeled)
            total = 0
            Om = {b: np.zeros((t.count[b], 0)) for b in boxes}
            Y = [{b: np.zeros((t.count[b], 0)) for b in boxes} for _ in range(self.nop)]
            # Y[op][b] holds, for box b, its rows of the column blocks of every
            # quadrant: dict quadrant -> samples, kept as a (count x 4*total) array
            Yq = [{b: [np.zeros((t.count[b], 0)) for _ in range(4)] for b in boxes} for _ in range(self.nop)]
            while True:
                newc = c - total
                Wm = np.zeros((n, 4 * newc))
                for b in boxes:
                    q = int(t.quad[b])
                    blk = self.probes(lev, b, total, newc)
                    Om[b] = np.concatenate([Om[b], blk], axis=1)
                    Wm[t.begin[b]:t.begin[b] + t.count[b], q * newc:(q + 1) * newc] = blk
                outs = self.applies(Wm)
                for op in range(self.nop):
                    B = outs[op] - self.lowrank_apply(op, Wm, lev)
                    for b in boxes:
                        rows = B[t.begin[b]:t.begin[b] + t.count[b]]
                        for q in range(4):
                            Yq[op][b][q] = np.concatenate([Yq[op][b][q], rows[:, q * newc:(q + 1) * newc]], axis=1)
                total = c
                need = False
                maxrank = 0
                for op in range(self.nop):
                    for (i, j) in pairs:
                        for (a, bb) in ((i, j), (j, i)):
                            Yab = Yq[op][a][int(t.quad[bb])]
                            k = orth(Yab, self.eps).shape[1]
                            maxrank = max(maxrank, k)
                            if k + OVERSAMPLE > total and total < t.count[bb]:
                                need = True
                if not need:
                    break
                c = grow_cols(total, maxrank)
            prev = maxrank
            peeled += 1
            self.cols[lev] = total
            self.ranks[lev] = maxrank
            for op in range(self.nop):
                blk = {}
                for (i, j) in pairs:
                    Yij = Yq[op][i][int(t.quad[j])]
                    Yji = Yq[op][j][int(t.quad[i])]
                    U1 = orth(Yij, self.eps)
                    U2 = orth(Yji, self.eps)
                    A1 = Om[i].T @ U1
                    C = Om[i].T @ Yij
                    A2 = U2.T @ Om[j]
                    M = np.linalg.pinv(A1) @ C @ np.linalg.pinv(A2)
                    blk[(i, j)] = (U1, M, U2)
                self.blocks[op].append(blk)
        # extraction at the leaves
        leaves = [int(b) for b in range(t.nbox) if t.is_leaf[b]]
        nL = int(max(t.count[b] for b in leaves))
        E = np.zeros((n, nL))
        for b in leaves:
            E[t.begin[b] + np.arange(t.count[b]), np.arange(t.count[b])] = 1.0
        outs = self.applies(E)
        traces = []
        for op in range(self.nop):
            H = outs[op] - self.lowrank_apply(op, E, t.max_depth + 1)
            tr = 0.0
            for b in leaves:
                tr += float(np.sum(H[t.begin[b] + np.arange(t.count[b]), np.arange(t.count[b])]))
            traces.append(tr)
        self.n_leaf_cols = nL
        return traces


def peel_traces(applies, tree, nop, eps_peel, seed):
    """Traces of nop symmetric operators given as one joint apply W -> [G_i W]."""
    return Peeler(tree, applies, nop, eps_peel, seed).run()
