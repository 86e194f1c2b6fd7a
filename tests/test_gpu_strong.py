"""Strong-admissibility peeling on the GPU (rsf_opts.peeling = RSF_PEEL_STRONG)
against the oracle (oracle/peel_strong.py, the same Philox probes on counter
stream 2): on the oracle's probe schedule the traces agree to rounding, and
they lie within 20 eps_peel of the dense traces; a batch gives what its
instances give alone."""
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


def _schedule(o, depth):
    """The oracle's probe columns per level (levels without admissible blocks
    take any value) as the test-only override."""
    return ",".join(str(o["peel_cols"].get(lev, 8)) for lev in range(1, depth + 1))


@pytest.mark.parametrize("case", ["uniform_matern32", "grid_matern32_aniso"])
def test_strong_peeling_matches_oracle_and_dense(case, monkeypatch):
    if case == "uniform_matern32":
        P = W.uniform_points(1024, 11)
        kernel, theta, eps, leaf, n_prox, rings = K.MATERN32, (0.1, 1.0, 1e-4), 1e-9, 32, 64, 1
    else:
        P = W.grid_points(32)
        kernel, theta, eps, leaf, n_prox, rings = K.MATERN32_ANISO, (10.0, 7.0, 1e-4), 1e-9, 16, 64, 1
    n = P.shape[0]
    print("strong peeling case %s n=%d" % (case, n), flush=True)
    z = dense.sample(P, W.gaussian(n, 12), theta, kernel)
    eps_peel = 1e-6
    F = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=leaf, n_prox=n_prox, prox_rings=rings,
                 peeling="strong")
    g, info = F.grad(_t(z), eps_peel, 33)
    o = rsf.loglik_grad(P, z, theta, kernel, eps, leaf, eps_peel=eps_peel, seed=33, n_prox=n_prox,
                        prox_rings=rings, strong=True)
    depth = F.tree_info()["depth"]
    own = [info.peel_cols[lev] for lev in range(1, depth + 1)]
    print("  own probe schedule %s, oracle's %s" % (own, [o["peel_cols"].get(lev, 0) for lev in range(1, depth + 1)]),
          flush=True)
    for lev, r in o["peel_ranks"].items():
        assert abs(info.peel_rank[lev] - r) <= 2
    np.testing.assert_allclose(list(info.q), o["q"], rtol=1e-9)
    # rounding-level parity on the oracle's schedule
    monkeypatch.setenv("RSFGP_TEST_PEEL_COLS", _schedule(o, depth))
    gs, infs = F.grad(_t(z), eps_peel, 33)
    monkeypatch.delenv("RSFGP_TEST_PEEL_COLS")
    for lev, c in o["peel_cols"].items():
        assert infs.peel_cols[lev] == c
    terr = np.abs(np.array(list(infs.t)) - o["t"]) / np.abs(o["t"])
    print("  traces vs oracle on its schedule: %s" % ["%.1e" % v for v in terr], flush=True)
    np.testing.assert_allclose(list(infs.t), o["t"], rtol=1e-8)
    oscale = np.abs(o["q"]) + 0.5 * np.abs(o["t"])
    assert np.all(np.abs(np.array(gs) - o["g"]) <= 1e-8 * oscale)
    # the traces of F^-1 and F^-1 F_i against the dense ones
    d = dense.loglik_and_grad(P, z, theta, kernel, want_terms=True)
    derr = np.abs(np.array(list(info.t)) - d["t"]) / np.abs(d["t"])
    print("  traces vs dense: %s" % ["%.1e" % v for v in derr], flush=True)
    assert np.all(derr <= 20 * eps_peel)
    # weak and strong peeling of the same factorization agree to the tolerance
    Fw = R.Factor(_t(P), theta, kernel=kernel, eps=eps, leaf=leaf, n_prox=n_prox, prox_rings=rings)
    gw, iw = Fw.grad(_t(z), eps_peel, 33)
    np.testing.assert_allclose(list(info.t), list(iw.t), rtol=40 * eps_peel)
    assert list(info.q) == list(iw.q)


def test_strong_peeling_batch_equals_single():
    pts = [W.uniform_points(m, 60 + m) for m in (900, 1600)]
    zs = [W.gaussian(m, 70 + m) for m in (900, 1600)]
    th = [(0.06, 1.0, 1e-4), (0.09, 1.5, 1e-3)]
    kw = dict(kernel=K.MATERN32, eps=1e-7, leaf=32, peeling="strong")
    print("strong peeling batch of 2", flush=True)
    B = R.BatchedFactor([_t(p) for p in pts], th, **kw)
    gb, _ = B.grad([_t(z) for z in zs], 1e-6, 4)
    for i in range(2):
        Fi = R.Factor(_t(pts[i]), th[i], **kw)
        gi, ii = Fi.grad(_t(zs[i]), 1e-6, 4)
        scale = np.abs(np.array(list(ii.q))) + 0.5 * np.abs(np.array(list(ii.t)))
        assert np.all(np.abs(np.array(gb[i]) - np.array(gi)) <= 1e-9 * scale)


def test_strong_peeling_refuses_unknown_form():
    with pytest.raises(ValueError):
        R.Factor(_t(W.uniform_points(100, 1)), (0.1, 1.0, 1e-3), peeling="medium")
