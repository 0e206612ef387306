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


def pe_task_vectors(t):
    from oracle import pe
    B = pe.PEBasis(t.L, t.K)
    e1 = np.zeros(B.dim, dtype=np.complex128)
    eD = np.zeros(B.dim, dtype=np.complex128)
    e1[B.index(np.array([t.e1_state]))[0]] = 1.0
    eD[B.index(np.array([t.eD_state]))[0]] = 1.0
    return e1, eD


@pytest.mark.parametrize("space", ["full", "reduced"])
@pytest.mark.parametrize("gradient", ["centred", "quadrature"])
def test_graph_replay_equals_eager(space, gradient):
    """A captured evaluation replayed for new controls gives the eager results bit
    for bit, on every replay, with eager work of the program in between."""
    if space == "full":
        c = workloads.small()
        h, N, dt, m = xxz_of(c), c.N, c.dt, c.m
        psi0, f = dev_vec(c.psi0, C128), dev_vec(c.target, C128)
        basis, u0 = None, c.u
    else:
        t = workloads.pe_paper(9, 3)
        e1, eD = pe_task_vectors(t)
        h = kg.XXZ(t.L, t.J, t.Delta, kg.KG_HC_SZ, t.hc_sites)
        N, dt, m, u0 = t.N, t.dt, t.m, t.u
        psi0, f = dev_vec(e1, C128), dev_vec(eD, C128)
        basis = kg.ReducedBasis(t.L, t.K)
    args = (h, N, dt, kg.Krylov(m), psi0, f, 7, gradient, 3, basis)
    eager = optimize.GradientEvaluator(*args, graph=False)
    graphed = optimize.GradientEvaluator(*args, graph=True)
    rng = np.random.default_rng(1)
    us = [u0, u0 + 0.1 * rng.standard_normal(N), u0 - 0.2 * rng.standard_normal(N), u0]
    for i, u in enumerate(us):
        Fg, gg = graphed(u)                    # call 0 eager, 1 captures, then replays
        Fe, ge = eager(u)
        torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work between replays
        assert Fg == Fe and np.array_equal(gg, ge), f"call {i}"


def test_transfer_task_reaches_the_target():
    """The task of Sec. III.B at D = 19 (M = 76 slices, dt = 0.5, m = 10): L-BFGS on
    the GPU's centred gradients, replayed from a graph, reaches I <= 1e-2 with the
    iterates of the oracle-driven run."""
    from oracle import pe
    t = workloads.pe_paper(7, 3)
    e1, eD = pe_task_vectors(t)
    ch = pe.PEChain(t.L, t.K, t.J, t.Delta, t.hc_sites)

    def fg_oracle(u):
        r = grape.gradient_centred(ch, u, e1, eD, t.dt, t.m, True, krylov.default_tol())
        return 1.0 - r.F, -r.grad

    ref = optimize.lbfgs(fg_oracle, t.u, f_target=1e-2, max_iter=60)
    h = kg.XXZ(t.L, t.J, t.Delta, kg.KG_HC_SZ, t.hc_sites)
    out = optimize.optimize_controls(h, t.u, t.dt, kg.Krylov(t.m), dev_vec(e1, C128),
                                     dev_vec(eD, C128), I_target=1e-2, max_iter=60,
                                     basis=kg.ReducedBasis(t.L, t.K), graph=True)
    assert out.reason == ref.reason == "f_target"
    assert out.f <= 1e-2
    assert out.iterations == ref.iterations
    assert np.abs(np.array(out.history) - np.array(ref.history)).max() < 1e-8
