"""Recursive skeletonization factorization, written out step by step
(oracle; TEST INFRASTRUCTURE ONLY).

This is the slow, plain reference for the approximation the HIP library
computes.  It follows Section 2 of the paper in order:

* Section 2.1: a quadtree over the observation locations; leaves hold at most
  ``leaf`` points (n_occ of Section 5).  Readings (the paper only says "equal
  subdomains" and "adaptive"): the root box is the square of side
  max(extent_x, extent_y) centred on the bounding-box midpoint; a box splits
  while it holds more than ``leaf`` points; a point with x >= cx goes east and
  y >= cy goes north; children are numbered NW, NE, SW, SE as in Fig. 1; inside
  a child the points keep their relative input order.  Empty children are not
  created.  Tree order lists the leaves depth first, so every box is a
  contiguous index range.

* Definition (interpolative decomposition): Householder QR with column
  pivoting on the compression matrix; at each step the pivot is the column
  with the largest residual norm (norms recomputed, ties to the lowest local
  index); the rank k is the number of steps taken before the largest residual
  norm drops to eps * |R_11| or below.  S = first k pivots, R = the rest, and
  T = R_11^-1 R_12.

* Section 2.3.1 (modified proxy trick): the compression matrix of a box B is
  [Sigma(N, I); M(Gamma, I)], N = active DOFs outside B whose distance to the
  centre of B is less than r_near * h (h = half-width of B), Gamma = proxy
  points on rings of radii between r_in * h and r_out * h (Fig. 3 draws
  r_near = 1.8, an annulus 1.75 .. 2.45 and several rings of equally spaced
  points).  Entries are kernel values; the active/active off-diagonal blocks
  are unmodified kernel entries (Section 2.2, the third bullet), so no
  modified entry ever enters a compression matrix.

* Section 2.1 (block elimination) with the partitioning [S, R] of I:
      X_sr = A_sr - A_ss T
      X_rr = A_rr - T^T X_sr - A_rs T
      X_rr = L L^T,  W = X_sr L^-T,  X_ss = A_ss - W W^T
  (the L_I and U_I operators), where A = the current diagonal block of box B:
  at a leaf the kernel block, at a parent the children's X_ss blocks on the
  diagonal and kernel entries between different children.

* Section 2.2 (eq. rskelf): levels are processed from the deepest to depth 1,
  every box of one depth seeing the active set as it was at the start of that
  depth; the remaining DOFs of the root are factored by a dense Cholesky.  A
  leaf shallower than the deepest level is skeletonized at its own depth.

* Section 2.4: F^-1, F, F^(1/2) and log|F| = 2 log|C| by sweeps over the
  per-box factors.

For the derivative matrix Sigma_rho the same compression is used in
multiply-only form (no inversion of the indefinite blocks): per box keep T,
X_sr and X_rr, and the parent's block is the unmodified kernel block.  This is
the same approximant as the Schur form, because the skeletons depend only on
the unmodified off-diagonal blocks.
"""
import numpy as np
import scipy.linalg as sla

from . import kernels as K

NEAR_RADIUS = 1.8
PROXY_R_IN = 1.75
PROXY_R_OUT = 2.45


class Tree:
    """Quadtree over points P (n x 2).  Box ids are in breadth-first order, so
    the boxes of one depth form a contiguous id range sorted by position."""

    def __init__(self, P, leaf, max_depth=40):
        P = np.asarray(P, dtype=np.float64)
        n = P.shape[0]
        self.n = n
        xmin, xmax = P[:, 0].min(), P[:, 0].max()
        ymin, ymax = P[:, 1].min(), P[:, 1].max()
        h = max(xmax - xmin, ymax - ymin) / 2.0
        if not h > 0.0:
            h = 0.5
        cx, cy = [(xmin + xmax) / 2.0], [(ymin + ymax) / 2.0]
        half, depth, parent, quad = [h], [0], [-1], [-1]
        begin, count = [0], [n]
        children = [[-1, -1, -1, -1]]
        perm = np.empty(n, dtype=np.int64)
        frontier = [(0, np.arange(n))]
        while frontier:
            nxt = []
            for b, idx in frontier:
                if idx.shape[0] > leaf and depth[b] < max_depth:
                    east = P[idx, 0] >= cx[b]
                    north = P[idx, 1] >= cy[b]
                    masks = [~east & north, east & north, ~east & ~north, east & ~north]
                    off = begin[b]
                    hh = half[b] / 2.0
                    for q in range(4):
                        sel = idx[masks[q]]
                        if sel.shape[0] == 0:
                            continue
                        c = len(cx)
                        cx.append(cx[b] + hh if q in (1, 3) else cx[b] - hh)
                        cy.append(cy[b] + hh if q in (0, 1) else cy[b] - hh)
                        half.append(hh)
                        depth.append(depth[b] + 1)
                        parent.append(b)
                        quad.append(q)
                        begin.append(off)
                        count.append(sel.shape[0])
                        children.append([-1, -1, -1, -1])
                        children[b][q] = c
                        off += sel.shape[0]
                        nxt.append((c, sel))
                else:
                    perm[begin[b]:begin[b] + count[b]] = idx
            frontier = nxt
        self.perm = perm
        self.cx = np.array(cx)
        self.cy = np.array(cy)
        self.half = np.array(half)
        self.depth = np.array(depth)
        self.parent = np.array(parent)
        self.quad = np.array(quad)
        self.begin = np.array(begin)
        self.count = np.array(count)
        self.children = np.array(children, dtype=np.int64).reshape(-1, 4)
        self.is_leaf = np.all(self.children < 0, axis=1)
        self.nbox = len(cx)
        self.max_depth = int(self.depth.max())
        self.levels = [np.nonzero(self.depth == d)[0] for d in range(self.max_depth + 1)]

    def kids(self, b):
        return [int(c) for c in self.children[b] if c >= 0]

    def dofs(self, b):
        return np.arange(self.begin[b], self.begin[b] + self.count[b])


def proxy_points(cx, cy, h, n_prox, rings, r_in=PROXY_R_IN, r_out=PROXY_R_OUT):
    """n_prox points on `rings` concentric rings around (cx, cy): ring q has
    radius h * (r_in + (r_out - r_in) (q + 1/2) / rings) and n_prox / rings
    equally spaced angles 2 pi (j + q / rings) / (n_prox / rings)."""
    per = n_prox // rings
    pts = []
    for q in range(rings):
        rad = h * (r_in + (r_out - r_in) * (q + 0.5) / rings)
        ang = 2.0 * np.pi * (np.arange(per) + q / rings) / per
        pts.append(np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], axis=1))
    return np.concatenate(pts, axis=0)


def cpqr_id(A, eps):
    """Interpolative decomposition of A (m x a) by Householder QR with column
    pivoting.  Returns (k, piv, T) with A[:, piv[k:]] ~= A[:, piv[:k]] @ T."""
    A = np.array(A, dtype=np.float64, copy=True)
    m, a = A.shape
    piv = np.arange(a)
    if a == 0:
        return 0, piv, np.zeros((0, 0))
    r11 = None
    k = 0
    for s in range(min(m, a)):
        norms = np.sqrt(np.sum(A[s:, s:] * A[s:, s:], axis=0))
        p = s + int(np.argmax(norms))  # argmax returns the first maximum
        nmax = norms[p - s]
        if r11 is None:
            r11 = nmax
        if not nmax > eps * r11 or nmax == 0.0:
            break
        if p != s:
            A[:, [s, p]] = A[:, [p, s]]
            piv[[s, p]] = piv[[p, s]]
        x = A[s:, s].copy()
        sigma = np.sqrt(np.dot(x, x))
        alpha = -sigma if x[0] >= 0 else sigma
        v = x
        v[0] = x[0] - alpha
        vtv = np.dot(v, v)
        A[s, s] = alpha
        A[s + 1:, s] = 0.0
        if s + 1 < a and vtv > 0:
            w = v @ A[s:, s + 1:]
            A[s:, s + 1:] -= np.outer(v, (2.0 / vtv) * w)
        k = s + 1
    R11 = np.triu(A[:k, :k])
    R12 = A[:k, k:]
    T = sla.solve_triangular(R11, R12, lower=False) if k > 0 else np.zeros((0, a))
    return k, piv, T


class Factor:
    """Recursive skeletonization factorization of Sigma (mode 'chol') or the
    multiply-only representation of Sigma_rho (mode 'mult')."""

    def __init__(self, P, theta, kernel, eps, leaf, alpha=1.0, n_prox=256, prox_rings=4,
                 mode="chol", r_near=NEAR_RADIUS, r_in=PROXY_R_IN, r_out=PROXY_R_OUT, tree=None, deriv=0):
        self.P = np.asarray(P, dtype=np.float64)
        self.tree = Tree(self.P, leaf) if tree is None else tree
        self.Pt = self.P[self.tree.perm]
        self.theta = tuple(float(t) for t in theta)
        self.kernel, self.alpha, self.eps = kernel, alpha, eps
        self.mode = mode
        self.deriv = deriv  # mode "mult": the parameter index of the derivative (0 = rho / theta_1, 1 = theta_2)
        self.n = self.P.shape[0]
        self._run(n_prox, prox_rings, r_near, r_in, r_out)

    # kernel entries between tree-order DOFs / arbitrary points
    def _entries(self, rows, cols):
        if self.mode == "chol":
            return K.cov_block(self.Pt, rows, cols, self.theta, self.kernel, self.alpha)
        return K.dcov_block(self.Pt, rows, cols, self.deriv, self.theta, self.kernel, self.alpha)

    def _proxy_entries(self, G, cols):
        if self.mode == "chol":
            return K.cross_cov(G, self.Pt[cols], self.theta, self.kernel, self.alpha)
        return K.cross_dcov(G, self.Pt[cols], self.deriv, self.theta, self.kernel, self.alpha)

    def _diag_block(self, b, I):
        """Current diagonal block of box b in the order of its active list I."""
        A = self._entries(I, I)
        t = self.tree
        if self.mode == "chol" and not t.is_leaf[b]:
            off = 0
            for c in t.kids(b):
                k = self.S[c].shape[0]
                A[off:off + k, off:off + k] = self.Xss[c]
                off += k
        return A

    def _active(self, b):
        t = self.tree
        if t.is_leaf[b]:
            return t.dofs(b)
        parts = [self.S[c] for c in t.kids(b)]
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)

    def _run(self, n_prox, prox_rings, r_near, r_in, r_out):
        t = self.tree
        self.S, self.R, self.T = {}, {}, {}
        self.L, self.W, self.Xss = {}, {}, {}
        self.Xsr, self.Xrr = {}, {}
        self.rank = {}
        self.logdet = 0.0
        Pt = self.Pt
        for lev in range(t.max_depth, 0, -1):
            boxes = t.levels[lev]
            act = {int(b): self._active(b) for b in boxes}
            # active DOFs at the start of this level: depth-lev boxes plus the
            # points of shallower leaves
            groups = list(act.items())
            for d in range(lev):
                for b in t.levels[d]:
                    if t.is_leaf[b]:
                        groups.append((int(b), t.dofs(b)))
            all_dofs = np.concatenate([g[1] for g in groups]) if groups else np.zeros(0, np.int64)
            owner = np.concatenate([np.full(g[1].shape[0], g[0]) for g in groups]) if groups else np.zeros(0, np.int64)
            for b in boxes:
                b = int(b)
                I = act[b]
                a = I.shape[0]
                if a == 0:
                    self.S[b], self.R[b], self.rank[b] = I, I, 0
                    self.T[b] = np.zeros((0, 0))
                    self.L[b], self.W[b], self.Xss[b] = np.zeros((0, 0)), np.zeros((0, 0)), np.zeros((0, 0))
                    self.Xsr[b], self.Xrr[b] = np.zeros((0, 0)), np.zeros((0, 0))
                    continue
                cx, cy, h = t.cx[b], t.cy[b], t.half[b]
                dx = Pt[all_dofs, 0] - cx
                dy = Pt[all_dofs, 1] - cy
                rr = r_near * h
                near = all_dofs[(dx * dx + dy * dy < rr * rr) & (owner != b)]
                G = proxy_points(cx, cy, h, n_prox, prox_rings, r_in, r_out)
                Aux = np.concatenate([self._entries(near, I), self._proxy_entries(G, I)], axis=0)
                k, piv, T = cpqr_id(Aux, self.eps)
                S, R = I[piv[:k]], I[piv[k:]]
                self.S[b], self.R[b], self.T[b], self.rank[b] = S, R, T, k
                A = self._diag_block(b, I)[np.ix_(piv, piv)]
                Ass, Asr, Ars, Arr = A[:k, :k], A[:k, k:], A[k:, :k], A[k:, k:]
                Xsr = Asr - Ass @ T
                Xrr = Arr - T.T @ Xsr - Ars @ T
                if self.mode == "chol":
                    if R.shape[0] > 0:
                        try:
                            L = sla.cholesky(Xrr, lower=True)
                        except np.linalg.LinAlgError as e:
                            raise RuntimeError("block not SPD at box %d" % b) from e
                        W = sla.solve_triangular(L, Xsr.T, lower=True).T
                        self.logdet += 2.0 * float(np.sum(np.log(np.diag(L))))
                    else:
                        L = np.zeros((0, 0))
                        W = np.zeros((k, 0))
                    self.L[b], self.W[b] = L, W
                    self.Xss[b] = Ass - W @ W.T
                else:
                    self.Xsr[b], self.Xrr[b] = Xsr, Xrr
        # root
        root = 0
        if t.max_depth == 0:
            Iroot = t.dofs(root)
        else:
            parts = [self.S[c] for c in t.kids(root)]
            Iroot = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        self.Iroot = Iroot
        Aroot = self._diag_block(root, Iroot) if t.max_depth > 0 else self._entries(Iroot, Iroot)
        if self.mode == "chol":
            if Iroot.shape[0] > 0:
                try:
                    self.Lroot = sla.cholesky(Aroot, lower=True)
                except np.linalg.LinAlgError as e:
                    raise RuntimeError("root block not SPD") from e
                self.logdet += 2.0 * float(np.sum(np.log(np.diag(self.Lroot))))
            else:
                self.Lroot = np.zeros((0, 0))
        else:
            self.Aroot = Aroot

    # ---- sweeps (vectors in tree order, shape (n,) or (n, c)) ----
    def _boxes_up(self):
        t = self.tree
        for lev in range(t.max_depth, 0, -1):
            for b in t.levels[lev]:
                yield int(b)

    def _boxes_down(self):
        t = self.tree
        for lev in range(1, t.max_depth + 1):
            for b in t.levels[lev]:
                yield int(b)

    def solve(self, bvec):
        """F^-1 b."""
        assert self.mode == "chol"
        x = np.array(bvec, dtype=np.float64, copy=True)
        for b in self._boxes_up():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            xr = x[R] - self.T[b].T @ x[S]
            cr = sla.solve_triangular(self.L[b], xr, lower=True)
            x[S] = x[S] - self.W[b] @ cr
            x[R] = cr
        I = self.Iroot
        if I.shape[0] > 0:
            x[I] = sla.cho_solve((self.Lroot, True), x[I])
        for b in self._boxes_down():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            xr = sla.solve_triangular(self.L[b], x[R] - self.W[b].T @ x[S], lower=True, trans="T")
            x[R] = xr
            x[S] = x[S] - self.T[b] @ xr
        return x

    def half_up(self, bvec):
        """B b for F^-1 = B^T B: the up sweep of solve() followed by
        L_root^-1 (the first half of the solve, Section 2.4).  B^T B = F^-1
        because each box's down step is the transpose of its up step."""
        assert self.mode == "chol"
        x = np.array(bvec, dtype=np.float64, copy=True)
        for b in self._boxes_up():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            xr = x[R] - self.T[b].T @ x[S]
            cr = sla.solve_triangular(self.L[b], xr, lower=True)
            x[S] = x[S] - self.W[b] @ cr
            x[R] = cr
        I = self.Iroot
        if I.shape[0] > 0:
            x[I] = sla.solve_triangular(self.Lroot, x[I], lower=True)
        return x

    def half_down(self, xvec):
        """B^T x: L_root^-T, then the down sweep of solve()."""
        assert self.mode == "chol"
        x = np.array(xvec, dtype=np.float64, copy=True)
        I = self.Iroot
        if I.shape[0] > 0:
            x[I] = sla.solve_triangular(self.Lroot, x[I], lower=True, trans="T")
        for b in self._boxes_down():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            xr = sla.solve_triangular(self.L[b], x[R] - self.W[b].T @ x[S], lower=True, trans="T")
            x[R] = xr
            x[S] = x[S] - self.T[b] @ xr
        return x

    def sqrt_t(self, xvec):
        """(F^(1/2))^T x."""
        x = np.array(xvec, dtype=np.float64, copy=True)
        out = np.zeros_like(x)
        for b in self._boxes_up():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            x[S] = x[S] + self.T[b] @ x[R]
            out[R] = self.L[b].T @ x[R] + self.W[b].T @ x[S]
        I = self.Iroot
        if I.shape[0] > 0:
            out[I] = self.Lroot.T @ x[I]
        return out

    def sqrt(self, yvec):
        """F^(1/2) y."""
        y = np.asarray(yvec, dtype=np.float64)
        v = np.array(y, copy=True)
        for b in self._boxes_up():
            R = self.R[b]
            if R.shape[0] > 0:
                v[R] = self.L[b] @ y[R]
        I = self.Iroot
        if I.shape[0] > 0:
            v[I] = self.Lroot @ y[I]
        for b in self._boxes_down():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            v[S] = v[S] + self.W[b] @ y[R]
            v[R] = v[R] + self.T[b].T @ v[S]
        return v

    def apply(self, xvec):
        """F x (for mode 'chol' F = F^(1/2) (F^(1/2))^T; for 'mult' the
        multiply-only sweep)."""
        if self.mode == "chol":
            return self.sqrt(self.sqrt_t(xvec))
        x = np.array(xvec, dtype=np.float64, copy=True)
        y = np.zeros_like(x)
        for b in self._boxes_up():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            x[S] = x[S] + self.T[b] @ x[R]
            y[R] = y[R] + self.Xrr[b] @ x[R] + self.Xsr[b].T @ x[S]
        I = self.Iroot
        if I.shape[0] > 0:
            y[I] = y[I] + self.Aroot @ x[I]
        # x[R] is final after the box's own up-step (coarser levels only touch
        # their active DOFs), so the X_sr x_R coupling can be added on the way
        # down, after the coarser levels' L operators have been applied to the
        # recursive part and before this level's own L operator.
        for b in self._boxes_down():
            S, R = self.S[b], self.R[b]
            if R.shape[0] == 0:
                continue
            y[S] = y[S] + self.Xsr[b] @ x[R]
            y[R] = y[R] + self.T[b].T @ y[S]
        return y

    # conversions between user order and tree order
    def to_tree(self, v):
        return np.asarray(v)[self.tree.perm]

    def from_tree(self, v):
        out = np.empty_like(np.asarray(v))
        out[self.tree.perm] = v
        return out


LOG2PI = float(np.log(2.0 * np.pi))


def profile_loglik_grad(P, z, theta, kernel, eps, leaf, eps_peel=None, seed=0, alpha=1.0, n_prox=256,
                        prox_rings=4):
    """The log profile likelihood of eq. prof and its gradient with the RSF:
    a = F^-1 z, b = F^-1 1, beta = (Sigma + 1 1^T)^-1 z = a - b (1^T a) / (1 + 1^T b)
    (Sherman-Morrison), z^T beta, and for the gradient beta^T Sigma_i beta with
    Sigma beta = z - 1 (1^T beta) and F_rho beta, the traces as in loglik_grad."""
    o = loglik_grad(P, z, theta, kernel, eps, leaf, eps_peel=eps_peel, seed=seed, alpha=alpha, n_prox=n_prox,
                    prox_rings=prox_rings)
    F, Fr = o["factor"], o["factor_rho"]
    n = F.tree.n
    rho, s2, nug = (float(v) for v in theta)
    zt = F.to_tree(np.asarray(z, dtype=np.float64))
    a = F.solve(zt)
    b = F.solve(np.ones(n))
    beta = a - b * (float(np.sum(a)) / (1.0 + float(np.sum(b))))
    zb = float(zt @ beta)
    ell = -0.5 * F.logdet - 0.5 * n * np.log(zb) + 0.5 * n * (np.log(n) - 1.0 - LOG2PI)
    sb = float(beta @ zt) - float(np.sum(beta)) ** 2       # beta^T Sigma beta
    bb = float(beta @ beta)
    quad = np.array([float(beta @ Fr.apply(beta)), (sb - nug * bb) / s2, bb])
    g = -0.5 * o["t"] + 0.5 * n * quad / zb
    return {"ell": ell, "g": g, "t": o["t"], "quad": quad, "zbeta": zb}


def conditional_mean(F, F22, z):
    """E[z' | z] = Sigma_12 Sigma_22^-1 z as in the remark after Algorithm 1:
    F factors the joint sites [x'; x] (the n1 prediction sites first), F22 the
    observed sites; Sigma_12 v is the first block of F [0; v] and
    Sigma_22^-1 b is F22^-1 b.  Vectors in caller order, (n2,) or (n2, k)."""
    n1 = F.tree.n - F22.tree.n
    z = np.asarray(z, dtype=np.float64)
    a = F22.from_tree(F22.solve(F22.to_tree(z)))
    v = np.concatenate([np.zeros((n1,) + a.shape[1:]), a])
    return F.from_tree(F.apply(F.to_tree(v)))[:n1]


def conditional_deviation(F, F22, xi):
    """S xi with S = [I, -Sigma_12 Sigma_22^-1] F^(1/2), so that S S^T is the
    conditional covariance Sigma_11 - Sigma_12 Sigma_22^-1 Sigma_12^T (the same
    remark); xi: (n,) or (n, k) standard normal draws, n = n1 + n2."""
    n1 = F.tree.n - F22.tree.n
    y = F.from_tree(F.sqrt(F.to_tree(np.asarray(xi, dtype=np.float64))))
    return y[:n1] - conditional_mean(F, F22, y[n1:])


def hutchinson_traces(F, Fr, nprobe, seed):
    """Hutchinson's estimator (eq. hutch) of Tr F^-1 and Tr F^-1 F_rho from
    nprobe Rademacher vectors u_j (oracle.philox.rademacher over the tree
    order): with w_j = B^T u_j (F^-1 = B^T B), u^T F^-1 u = |w|^2 and
    u^T B F_rho B^T u = w^T F_rho w, whose expectations are the two traces.
    Returns (t_inv, t_rho)."""
    from . import philox
    n = F.tree.n
    d = np.arange(n)[:, None]
    j = np.arange(nprobe)[None, :]
    U = philox.rademacher(d, j, seed)
    Wt = F.half_down(U)
    t_inv = float(np.sum(Wt * Wt)) / nprobe
    t_rho = float(np.sum(Wt * Fr.apply(Wt))) / nprobe
    return t_inv, t_rho


def loglik_grad(P, z, theta, kernel, eps, leaf, eps_peel=None, seed=0, alpha=1.0,
                n_prox=256, prox_rings=4, want_grad=True, hutch_probes=0, strong=False):
    """The paper's Algorithm 1 with the readings used throughout this package.

    l_hat = -1/2 z^T F^-1 z - 1/2 log|F| - (n/2) log 2 pi; for theta =
    (rho, sigma2, nugget):
      q_rho = 1/2 a^T F_rho a,  q_sigma2 = 1/2 (z^T a - nugget a^T a) / sigma2,
      q_nug = 1/2 a^T a            (a = F^-1 z, Sigma_sigma2 = (Sigma - nugget I) / sigma2)
      t_nug = Tr F^-1,  t_sigma2 = (n - nugget t_nug) / sigma2,
      t_rho = Tr F^-1 F_rho,  g_i = q_i - t_i / 2.
    Both traces are peeled from symmetric operators with the same traces
    (Section 3 allows any symmetrized form with the trace of F^-1 F_rho): with
    F^-1 = B^T B, Tr F^-1 = Tr B B^T and Tr F^-1 F_rho = Tr B F_rho B^T, and the
    two operators share the product B^T W.

    Anisotropic kernels (theta = (theta_1, theta_2, nugget)): q_i = 1/2 a^T F_i a
    and t_i = Tr F^-1 F_i for the derivative factorizations F_1, F_2 of
    Sigma_theta1, Sigma_theta2; the three operators B B^T, B F_1 B^T and
    B F_2 B^T are peeled jointly from one set of probes (as the two are for
    rho above); q_nug = 1/2 a^T a, t_nug = Tr F^-1.
    strong: the traces peeled in the strongly admissible format
    (oracle.peel_strong) instead of the weakly admissible one (oracle.peel).
    Returns a dict (user order for vectors)."""
    from . import peel
    eps_peel = eps if eps_peel is None else eps_peel
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    F = Factor(P, theta, kernel, eps, leaf, alpha=alpha, n_prox=n_prox, prox_rings=prox_rings)
    zt = F.to_tree(np.asarray(z, dtype=np.float64))
    a = F.solve(zt)
    za = float(zt @ a)
    ell = -0.5 * za - 0.5 * F.logdet - 0.5 * n * LOG2PI
    out = {"ell": ell, "logdet": F.logdet, "alpha": F.from_tree(a), "factor": F}
    if not want_grad:
        return out
    if K.is_aniso(kernel):
        return _loglik_grad_aniso(out, F, P, a, theta, kernel, eps, leaf, eps_peel, seed, alpha,
                                  n_prox, prox_rings, hutch_probes, strong)
    rho, s2, nug = (float(v) for v in theta)
    Peeler = peel.Peeler
    if strong:
        from .peel_strong import StrongPeeler as Peeler
    Fr = Factor(P, theta, kernel, eps, leaf, alpha=alpha, n_prox=n_prox, prox_rings=prox_rings,
                mode="mult", tree=F.tree)
    aa = float(a @ a)
    q = np.array([0.5 * float(a @ Fr.apply(a)), 0.5 * (za - nug * aa) / s2, 0.5 * aa])

    if hutch_probes > 0:
        t_inv, t_rho = hutchinson_traces(F, Fr, hutch_probes, seed)
        t = np.array([t_rho, (n - nug * t_inv) / s2, t_inv])
        out.update(q=q, t=t, g=q - 0.5 * t, factor_rho=Fr)
        return out

    def applies(Wm):
        H = F.half_down(Wm)
        return [F.half_up(H), F.half_up(Fr.apply(H))]

    pl = Peeler(F.tree, applies, 2, eps_peel, seed)
    t_inv, t_rho = pl.run()
    t = np.array([t_rho, (n - nug * t_inv) / s2, t_inv])
    out.update(q=q, t=t, g=q - 0.5 * t, factor_rho=Fr, peel_cols=pl.cols, peel_ranks=pl.ranks)
    return out


def _loglik_grad_aniso(out, F, P, a, theta, kernel, eps, leaf, eps_peel, seed, alpha,
                       n_prox, prox_rings, hutch_probes, strong=False):
    from . import peel
    Peeler = peel.Peeler
    if strong:
        from .peel_strong import StrongPeeler as Peeler
    Fs = [Factor(P, theta, kernel, eps, leaf, alpha=alpha, n_prox=n_prox, prox_rings=prox_rings,
                 mode="mult", tree=F.tree, deriv=w) for w in (0, 1)]
    aa = float(a @ a)
    q = np.array([0.5 * float(a @ Fs[0].apply(a)), 0.5 * float(a @ Fs[1].apply(a)), 0.5 * aa])
    if hutch_probes > 0:
        t_inv, t1 = hutchinson_traces(F, Fs[0], hutch_probes, seed)
        _, t2 = hutchinson_traces(F, Fs[1], hutch_probes, seed)
    else:
        def applies(Wm):
            H = F.half_down(Wm)
            return [F.half_up(H), F.half_up(Fs[0].apply(H)), F.half_up(Fs[1].apply(H))]

        pl = Peeler(F.tree, applies, 3, eps_peel, seed)
        t_inv, t1, t2 = pl.run()
        out.update(peel_cols=pl.cols, peel_ranks=pl.ranks)
    t = np.array([t1, t2, t_inv])
    out.update(q=q, t=t, g=q - 0.5 * t, factor_rho=Fs[0], factor_theta2=Fs[1])
    return out
