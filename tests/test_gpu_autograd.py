"""The autograd adjoint form: torch.autograd.Function around grape_forward (with
sqrt(N) checkpoints) and the library's adjoint sweep.

Finite-difference protocol (the zeroth-order gradient of Eq. 5 differs from the
exact piecewise-constant gradient by O(dt) relative, so FD cannot check it to
rounding):
  (i)   central FD of the GPU FP64 forward vs the oracle's exact gradient
        (Gauss-Legendre quadrature of the natural gradient): 1e-6 relative;
  (ii)  GPU zeroth-order gradient vs the oracle's zeroth-order gradient:
        1e-10 (complex128) / 1e-4 (complex64);
  (iii) the O(dt) gap |g0 - g_exact| / |g_exact| is recorded and bounded.
"""

import json
import os

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, xxz_of

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        return json.load(fh)


def autograd_grad(c, dtype, ckpt_every):
    h = xxz_of(c)
    k = kg.Krylov(c.m)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda", requires_grad=True)
    F = kg.fidelity(u, h, c.dt, k, dev_vec(c.psi0, dtype), dev_vec(c.target, dtype), ckpt_every)
    F.backward()
    return float(F.detach().cpu()), host(u.grad)


def test_autograd_matches_oracle_and_adjoint_call():
    rng = np.random.default_rng(77)
    L, N = 10, 30
    c = workloads.Chain(L=L, J=1.0, Delta=0.5, hc_kind=0, hc_sites=1, N=N, dt=0.05, m=16,
                        u=rng.uniform(-1, 1, N), psi0=workloads.random_state(rng, 1 << L),
                        target=workloads.random_state(rng, 1 << L))
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    ref = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, True, krylov.default_tol())
    F, g = autograd_grad(c, C128, ckpt_every=6)
    assert abs(F - ref.F) / ref.F <= 1e-10
    assert rel_err(g, ref.grad) <= 1e-10
    # the same numbers as one grape_gradient call with the same checkpointing
    r = kg.grape_gradient(xxz_of(c), torch.tensor(c.u, device="cuda"), c.dt, kg.Krylov(c.m),
                          dev_vec(c.psi0), dev_vec(c.target), ckpt_every=6)
    assert np.array_equal(host(r.grad), g)
    F64, g64 = autograd_grad(c, C64, ckpt_every=6)
    assert abs(F64 - ref.F) / ref.F <= 1e-4 and rel_err(g64, ref.grad) <= 1e-4


@pytest.mark.parametrize("centred", [False, True])
def test_backward_twice_with_checkpoints(centred):
    """Backward runs twice on one graph (retain_graph) with 6 checkpoint segments,
    so the first sweep recomputes earlier segments into the segment buffers: the
    second gradient must be bit-identical to the first and to the oracle's."""
    rng = np.random.default_rng(91)
    L, N = 9, 17
    c = workloads.Chain(L=L, J=1.0, Delta=0.7, hc_kind=0, hc_sites=1, N=N, dt=0.05, m=12,
                        u=rng.uniform(-1, 1, N), psi0=workloads.random_state(rng, 1 << L),
                        target=workloads.random_state(rng, 1 << L))
    h = xxz_of(c)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda", requires_grad=True)
    F = kg.fidelity(u, h, c.dt, kg.Krylov(c.m), dev_vec(c.psi0), dev_vec(c.target), 3,
                    centred=centred)
    F.backward(retain_graph=True)
    g1 = host(u.grad).copy()
    u.grad = None
    F.backward()
    g2 = host(u.grad)
    assert np.array_equal(g1, g2)
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    fn = grape.gradient_centred if centred else grape.gradient
    ref = fn(ch, c.u, c.psi0, c.target, c.dt, c.m, True, krylov.default_tol())
    assert rel_err(g2, ref.grad) <= 1e-10


def short_chain():
    return workloads.adjoint(N=8)


@pytest.mark.parametrize("dtype,tol", [(C128, 1e-10), (C64, 1e-4)])
def test_zeroth_order_vs_oracle_L20(dtype, tol):
    """(ii): GPU zeroth-order gradient at the adjoint workload's size (L=20), 8 slices."""
    gold = load_golden("adjoint_short")
    c = short_chain()
    F, g = autograd_grad(c, dtype, ckpt_every=3)
    gref = np.array(gold["grad"])
    assert abs(F - gold["F"]) / gold["F"] <= tol
    assert rel_err(g, gref) <= tol
    assert np.abs(g - gref).max() / np.abs(gref).max() <= tol


def gpu_forward_F(c, u, dtype=C128):
    h = xxz_of(c)
    r = kg.grape_forward(h, torch.tensor(u, dtype=torch.float64, device="cuda"), c.dt,
                         kg.Krylov(c.m), dev_vec(c.psi0, dtype), dev_vec(c.target, dtype))
    return float(host(r.F))


def test_fd_of_forward_vs_exact_gradient_L20():
    """(i) and (iii) at L=20 on 8 slices."""
    gold = load_golden("adjoint_short")
    c = short_chain()
    hstep = 1e-4
    g_exact = np.array(gold["exact_grad"])
    fd = []
    for j in gold["exact_grad_slices"]:
        up = c.u.copy()
        up[j] += hstep
        um = c.u.copy()
        um[j] -= hstep
        fd.append((gpu_forward_F(c, up) - gpu_forward_F(c, um)) / (2 * hstep))
    fd = np.array(fd)
    assert rel_err(fd, g_exact) <= 1e-6
    gap = rel_err(np.array(gold["grad"]), g_exact)
    print(f"zeroth-order vs exact gradient at dt={c.dt}: {gap:.3e} (relative, l2)")
    assert 1e-4 <= gap <= 0.1


def test_full_size_adjoint_form():
    """The adjoint workload at full size (L=20, N=400, checkpoints every 20): mixed vs
    FP64 agreement at the stated error, and FD of the FP64 forward on the 8 chosen
    slices within the O(dt) gap of the zeroth-order gradient."""
    c = workloads.adjoint()
    ck = workloads.ADJOINT_CKPT_EVERY
    F128, g128 = autograd_grad(c, C128, ck)
    F64, g64 = autograd_grad(c, C64, ck)
    assert abs(F64 - F128) / F128 <= 1e-4
    assert rel_err(g64, g128) <= 1e-4
    slices = workloads.adjoint_fd_slices()
    hstep = 1e-4
    fd = []
    for j in slices:
        up = c.u.copy()
        up[j] += hstep
        um = c.u.copy()
        um[j] -= hstep
        fd.append((gpu_forward_F(c, up) - gpu_forward_F(c, um)) / (2 * hstep))
    fd = np.array(fd)
    gap = rel_err(g128[slices], fd)
    # the centred variant (App. B) closes most of the O(dt) gap
    h = xxz_of(c)
    rc = kg.grape_gradient(h, torch.tensor(c.u, device="cuda"), c.dt, kg.Krylov(c.m),
                           dev_vec(c.psi0, C128), dev_vec(c.target, C128), ckpt_every=ck,
                           centred=True)
    gap_c = rel_err(host(rc.grad)[slices], fd)
    print(f"full size: |g0 - FD| / |FD| on 8 slices = {gap:.3e}, centred {gap_c:.3e}; "
          f"mixed vs FP64 grad {rel_err(g64, g128):.2e}, F {abs(F64 - F128) / F128:.2e}")
    assert gap <= 0.1
    assert gap_c <= gap / 5
