"""Conditional mean and sampling (the remark after Algorithm 1) on the GPU:
against the oracle's compositions of the same factors (to rounding), and
against the dense conditional distribution (to the factorization accuracy)."""
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


def test_conditional_mean_and_sample_match_oracle():
    n1, n2 = 300, 4000
    print("conditional n1=%d n2=%d" % (n1, n2), flush=True)
    Pall = W.uniform_points(n1 + n2, 41)
    theta = (0.05, 1.0, 1e-3)
    kw = dict(kernel=K.MATERN32, eps=1e-8, leaf=64)
    F = R.Factor(_t(Pall), theta, **kw)
    F22 = R.Factor(_t(Pall[n1:]), theta, **kw)
    O = rsf.Factor(Pall, theta, K.MATERN32, 1e-8, 64)
    O22 = rsf.Factor(Pall[n1:], theta, K.MATERN32, 1e-8, 64)
    z = W.gaussian((n2, 3), 42)
    mu = R.cond_mean(F, F22, _t(z)).cpu().numpy()
    mu_o = rsf.conditional_mean(O, O22, z)
    _entrywise(mu, mu_o, 1e-9, "conditional mean")
    xi = W.gaussian((n1 + n2, 2), 43)
    dv = R.cond_sample(F, F22, _t(xi)).cpu().numpy()
    dv_o = rsf.conditional_deviation(O, O22, xi)
    _entrywise(dv, dv_o, 1e-6, "conditional deviation")
    # single vectors give the columns of the block calls
    m1 = R.cond_mean(F, F22, _t(z[:, 1])).cpu().numpy()
    assert np.allclose(m1, mu[:, 1], rtol=0, atol=1e-12 * np.abs(mu).max())


def test_conditional_covariance_against_dense():
    n1, n2 = 60, 700
    Pall = W.uniform_points(n1 + n2, 31)
    theta = (0.1, 1.0, 1e-3)
    kw = dict(kernel=K.MATERN32, eps=1e-10, leaf=32, n_prox=64, prox_rings=1)
    F = R.Factor(_t(Pall), theta, **kw)
    F22 = R.Factor(_t(Pall[n1:]), theta, **kw)
    S = dense.cov_matrix(Pall, theta, K.MATERN32)
    S11, S12, S22 = S[:n1, :n1], S[:n1, n1:], S[n1:, n1:]
    z = W.gaussian(n2, 33)
    mu = R.cond_mean(F, F22, _t(z)).cpu().numpy()
    mu_d = S12 @ np.linalg.solve(S22, z)
    _entrywise(mu, mu_d, 1e-6, "conditional mean vs dense")
    Sq = R.cond_sample(F, F22, _t(np.eye(n1 + n2))).cpu().numpy()
    C = Sq @ Sq.T
    C_d = S11 - S12 @ np.linalg.solve(S22, S12.T)
    _entrywise(C, C_d, 1e-6, "conditional covariance vs dense")


def test_conditional_errors():
    P = W.uniform_points(500, 5)
    F = R.Factor(_t(P), (0.1, 1.0, 1e-3), kernel=K.MATERN32)
    G = R.Factor(_t(P[100:]), (0.2, 1.0, 1e-3), kernel=K.MATERN32)
    with pytest.raises(R.RsfError):
        R.cond_mean(F, G, _t(np.zeros(400)))
    with pytest.raises(R.RsfError):
        R.cond_mean(G, F, _t(np.zeros(500)))
