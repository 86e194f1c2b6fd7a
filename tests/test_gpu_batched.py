"""Batches of independent instances in one handle (one forest, one set of
launches per level) against the same instances factored one by one, against
the oracle's skeletons and against the dense definitions."""
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


def _instances():
    # uneven sizes, shapes and length scales; one instance smaller than a leaf
    inst = W.batch_instances(5, 7, n_lo=300, n_hi=2600)
    inst.append((W.uniform_points(40, 5), (0.2, 1.5, 1e-3)))
    return inst


@pytest.fixture(scope="module")
def batch():
    inst = _instances()
    print("batched factor of %d instances, n = %s" % (len(inst), [len(p) for p, _ in inst]), flush=True)
    B = R.BatchedFactor([_t(p) for p, _ in inst], [th for _, th in inst], kernel=K.MATERN32, eps=1e-7, leaf=64)
    zs = [dense.sample(p, W.gaussian(len(p), 100 + i), th, K.MATERN32) for i, (p, th) in enumerate(inst)]
    return inst, B, zs


def test_batched_matches_single_instances(batch):
    inst, B, zs = batch
    lds = B.logdets
    ls = B.loglik([_t(z) for z in zs])
    total = 0.0
    for i, ((P, th), z) in enumerate(zip(inst, zs)):
        F = R.Factor(_t(P), th, kernel=K.MATERN32, eps=1e-7, leaf=64)
        print("instance %d: n=%d logdet %.12e vs %.12e" % (i, len(P), lds[i], F.logdet), flush=True)
        assert lds[i] == pytest.approx(F.logdet, rel=1e-12, abs=1e-9)
        assert ls[i] == pytest.approx(F.loglik(_t(z)), rel=1e-11, abs=1e-8)
        total += ls[i]
        F.close()
    # the single-vector calls act on the block-diagonal operator
    zcat = _t(np.concatenate(zs))
    h = B._h
    out = R._lib.C.c_double()
    R._lib._check(R.load().rsf_loglik(h, R._lib.C.c_void_p(zcat.data_ptr()), R._lib.C.byref(out), None,
                                       R._lib._stream()))
    assert out.value == pytest.approx(total, rel=1e-12)


def test_batched_skeletons_match_oracle(batch):
    inst, B, zs = batch
    off = np.cumsum([0] + [len(p) for p, _ in inst])
    depth = B.tree_info()["depth"]
    want = {}
    for i, (P, th) in enumerate(inst):
        O = rsf.Factor(P, th, K.MATERN32, 1e-7, 64)
        for lev in range(1, O.tree.max_depth + 1):
            for b in O.tree.levels[lev]:
                want.setdefault(lev, []).append(off[i] + O.tree.perm[O.S[int(b)]])
    for lev in range(1, depth + 1):
        nb = R._lib.C.c_int32()
        lib = R.load()
        R._lib._check(lib.rsf_skeleton_export(B._h, lev, None, None, R._lib.C.byref(nb)))
        offs = (R._lib.C.c_int32 * (nb.value + 1))()
        R._lib._check(lib.rsf_skeleton_export(B._h, lev, offs, None, R._lib.C.byref(nb)))
        idx = (R._lib.C.c_int32 * max(1, offs[nb.value]))()
        R._lib._check(lib.rsf_skeleton_export(B._h, lev, offs, idx, R._lib.C.byref(nb)))
        got = [np.array(idx[offs[q]:offs[q + 1]]) for q in range(nb.value)]
        assert len(got) == len(want.get(lev, []))
        for g, w in zip(got, want[lev]):
            assert np.array_equal(g, w)


def test_batched_scores_against_dense(batch):
    inst, B, zs = batch
    eps_peel = 1e-6
    gs, info = B.grad([_t(z) for z in zs], eps_peel, 17)
    for i, ((P, th), z) in enumerate(zip(inst, zs)):
        d = dense.loglik_and_grad(P, z, th, K.MATERN32, want_terms=True)
        scale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
        err = np.abs(np.array(gs[i]) - d["g"]) / scale
        print("instance %d: g %s dense %s err/scale %s" % (i, np.array(gs[i]), d["g"], err), flush=True)
        assert np.all(err <= 1e3 * 1e-7 + 50 * eps_peel)
    # the single-instance score call is refused on a batch
    with pytest.raises(R.RsfError):
        g = (R._lib.C.c_double * 3)()
        R._lib._check(R.load().rsf_grad(B._h, R._lib.C.c_void_p(_t(np.zeros(sum(B.ns))).data_ptr()), 1e-6, 1, g,
                                        None, R._lib._stream()))


def test_batched_errors_name_the_instance():
    P = W.uniform_points(100, 3)
    Q = W.uniform_points(50, 4)
    Q[7] = Q[3]
    with pytest.raises(R.RsfError, match="instance 1"):
        R.BatchedFactor([_t(P), _t(Q)], [(0.1, 1.0, 1e-4)] * 2)


def test_c4_subset_smallest_and_largest_instances():
    """The 64-instance workload's two smallest instances and its largest
    (n = 2324, 2370 and 32253; aspect up to 4:1, eps 1e-6, leaf 64, 256
    proxies on 4 rings) in one batched handle: log-det, l and the score per
    instance against the same instances factored alone; the small instances'
    skeletons bit-exact against the oracle and their score against the dense
    definitions; sampled deepest-level skeletons of the large one computed one
    by one by the oracle."""
    spec = W.BATCHES["c4_batch64_matern32"]
    inst = W.batch_instances(spec["count"], spec["master_seed"])
    ns = np.array([len(p) for p, _ in inst])
    order = np.argsort(ns)
    pick = [int(order[0]), int(order[1]), int(order[-1])]
    sub = [inst[i] for i in pick]
    kw = dict(kernel=spec["kernel"], eps=spec["eps"], leaf=spec["leaf"], n_prox=spec["n_prox"],
              prox_rings=spec["prox_rings"])
    print("C4 subset: instances %s, n = %s" % (pick, [len(p) for p, _ in sub]), flush=True)
    rng = np.random.default_rng(spec["w_seed"])
    zs = []
    for i, (P, th) in enumerate(sub):
        F = R.Factor(_t(P), th, **kw)
        zs.append(F.apply_sqrt(_t(rng.standard_normal(len(P)))).cpu().numpy())
        F.close()
    B = R.BatchedFactor([_t(p) for p, _ in sub], [th for _, th in sub], **kw)
    lds = B.logdets
    ls = B.loglik([_t(z) for z in zs])
    gb, _ = B.grad([_t(z) for z in zs], spec["eps"], spec["peel_seed"])
    for i, ((P, th), z) in enumerate(zip(sub, zs)):
        F = R.Factor(_t(P), th, **kw)
        assert lds[i] == pytest.approx(F.logdet, rel=1e-12)
        assert ls[i] == pytest.approx(F.loglik(_t(z)), rel=1e-11)
        g1, i1 = F.grad(_t(z), spec["eps"], spec["peel_seed"])
        scale = np.abs(np.array(list(i1.q))) + 0.5 * np.abs(np.array(list(i1.t)))
        err = np.abs(np.array(gb[i]) - np.array(g1)) / scale
        print("  instance %d (n=%d): score vs alone %s of |q| + |t|/2" % (pick[i], len(P), ["%.1e" % v for v in err]),
              flush=True)
        # the batch draws its probes at its own tree-order rows: both are
        # eps_peel-accurate traces from different probes
        assert np.all(err <= 20 * spec["eps"])
        F.close()
    # skeletons of the two small instances against the oracle, in batch order
    off = np.cumsum([0] + [len(p) for p, _ in sub])
    lib = R.load()
    depth = B.tree_info()["depth"]
    want = {}
    oracle_factors = []
    for i, (P, th) in enumerate(sub[:2]):
        O = rsf.Factor(P, th, spec["kernel"], spec["eps"], spec["leaf"], n_prox=spec["n_prox"],
                       prox_rings=spec["prox_rings"])
        oracle_factors.append(O)
        for lev in range(1, O.tree.max_depth + 1):
            for b in O.tree.levels[lev]:
                want.setdefault(lev, []).append(off[i] + O.tree.perm[O.S[int(b)]])
    for lev in range(1, depth + 1):
        nb = R._lib.C.c_int32()
        R._lib._check(lib.rsf_skeleton_export(B._h, lev, None, None, R._lib.C.byref(nb)))
        offs = (R._lib.C.c_int32 * (nb.value + 1))()
        idx = (R._lib.C.c_int32 * max(1, 1 << 20))()
        R._lib._check(lib.rsf_skeleton_export(B._h, lev, offs, idx, R._lib.C.byref(nb)))
        got = [np.array(idx[offs[q]:offs[q + 1]]) for q in range(nb.value)]
        # boxes of a level are in instance order: the small instances' boxes come first
        w = want.get(lev, [])
        for g, x in zip(got[:len(w)], w):
            assert np.array_equal(g, x)
    # the small instances' scores against the dense definitions
    for i, ((P, th), z) in enumerate(zip(sub[:2], zs[:2])):
        d = dense.loglik_and_grad(P, z, th, spec["kernel"], want_terms=True)
        scale = np.abs(d["q"]) + 0.5 * np.abs(d["t"])
        assert np.all(np.abs(np.array(gb[i]) - d["g"]) <= (100 * spec["eps"] + 10 * spec["eps"]) * scale)
    # the large instance: sampled boxes of its deepest level, one by one
    P, th = sub[2]
    tree = rsf.Tree(P, spec["leaf"])
    D = tree.max_depth
    nb = R._lib.C.c_int32()
    R._lib._check(lib.rsf_skeleton_export(B._h, D, None, None, R._lib.C.byref(nb)))
    offs = (R._lib.C.c_int32 * (nb.value + 1))()
    idx = (R._lib.C.c_int32 * max(1, 1 << 20))()
    R._lib._check(lib.rsf_skeleton_export(B._h, D, offs, idx, R._lib.C.byref(nb)))
    boxes = tree.levels[D]
    first = nb.value - len(boxes)  # the large instance's boxes are the level's last ones
    Pt = P[tree.perm]
    pick_b = np.random.default_rng(5).choice(len(boxes), size=min(8, len(boxes)), replace=False)
    for q in pick_b:
        b = int(boxes[q])
        I = tree.dofs(b)
        cx, cy, h = tree.cx[b], tree.cy[b], tree.half[b]
        d2 = (Pt[:, 0] - cx) ** 2 + (Pt[:, 1] - cy) ** 2
        mask = d2 < (1.8 * h) ** 2
        mask[I] = False
        near = np.nonzero(mask)[0]
        G = rsf.proxy_points(cx, cy, h, spec["n_prox"], spec["prox_rings"])
        A = np.concatenate([K.cross_cov(Pt[near], Pt[I], th, spec["kernel"]),
                            K.cross_cov(G, Pt[I], th, spec["kernel"])], axis=0)
        k, piv, T = rsf.cpqr_id(A, spec["eps"])
        got = np.array(idx[offs[first + q]:offs[first + q + 1]])
        assert np.array_equal(got, off[2] + tree.perm[I[piv[:k]]])
    B.close()
