"""The recorded log-likelihood graph: the first call on a handle runs eagerly,
the second records a HIP graph of the solve sweep and the dot products and
replays it, and later calls replay it.  Every replay,
with eager work and synchronisations in between, must give what the eager
path gives: alpha bitwise equal to rsf_solve (the same kernels), l equal to
the value assembled from it."""
import math

import numpy as np
import pytest
import torch

import paper_1603_08057_amd as R
from oracle import kernels as K
import workloads as W

pytestmark = pytest.mark.gpu


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n,leaf", [(6000, 64), (700, 32)])
def test_loglik_graph_replays_match_eager(n, leaf):
    print("graph case n=%d" % n, flush=True)
    P = W.uniform_points(n, 21)
    theta = (0.05, 1.0, 1e-4)
    F = R.Factor(_t(P), theta, kernel=K.MATERN32, eps=1e-7, leaf=leaf)
    zs = [_t(W.gaussian(n, 300 + i)) for i in range(4)]
    # eager references (rsf_solve takes the eager sweep)
    refs = []
    for z in zs:
        a = F.solve(z)
        ell = -0.5 * float(z @ a) - 0.5 * F.logdet - 0.5 * n * math.log(2 * math.pi)
        refs.append((ell, a.clone()))
    assert F.graph_state == 0
    ell0 = F.loglik(zs[0])  # eager: a handle used once records nothing
    assert ell0 == pytest.approx(refs[0][0], rel=1e-12)
    assert F.graph_state == 0
    ell1, a1 = F.loglik(zs[1], want_alpha=True)  # recorded, then replayed
    assert F.graph_state == 1
    assert torch.equal(a1, refs[1][1])
    assert ell1 == pytest.approx(refs[1][0], rel=1e-12)
    other = _t(W.gaussian(n, 999))
    for rep in range(3):
        for z, (ell_ref, a_ref) in zip(zs, refs):
            ell, a = F.loglik(z, want_alpha=True)
            assert torch.equal(a, a_ref)
            assert ell == pytest.approx(ell_ref, rel=1e-12)
            # eager work on the same stream between replays
            F.solve(other)
            torch.cuda.synchronize()
    F.close()
