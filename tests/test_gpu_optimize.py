"""The L-BFGS driver with GPU gradients: the same iterates as with the oracle's
gradients (complex128), and a monotone decrease of the infidelity."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from paper_2010_03598_amd import optimize
from tests.gpu_util import C128, dev_vec, xxz_of

pytestmark = pytest.mark.gpu


def test_lbfgs_iterates_match_oracle_driven_run():
    c = workloads.small()
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)

    def fg_oracle(u):
        r = grape.gradient_centred(ch, u, c.psi0, c.target, c.dt, c.m, True, krylov.default_tol())
        return 1.0 - r.F, -r.grad

    ref = optimize.lbfgs(fg_oracle, c.u, max_iter=4, df_min=0.0)
    out = optimize.optimize_controls(xxz_of(c), c.u, c.dt, kg.Krylov(c.m), dev_vec(c.psi0, C128),
                                     dev_vec(c.target, C128), I_target=-1.0, max_iter=4)
    assert out.iterations == ref.iterations == 4
    assert np.abs(np.array(out.history) - np.array(ref.history)).max() < 1e-9
    assert np.abs(out.x - ref.x).max() < 1e-7


@pytest.mark.parametrize("gradient", ["zeroth", "centred", "first_order", "quadrature"])
def test_infidelity_decreases(gradient):
    c = workloads.ascent()
    out = optimize.optimize_controls(xxz_of(c), c.u, c.dt, kg.Krylov(c.m), dev_vec(c.psi0, C128),
                                     dev_vec(c.target, C128), gradient=gradient, I_target=-1.0,
                                     max_iter=6, nodes=3)
    h = out.history
    assert all(b < a for a, b in zip(h, h[1:]))
    assert h[-1] < h[0]
