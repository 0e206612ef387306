"""Operator control on a block of columns (grape_gradient_columns and its
reduced-basis form) against the oracle's column gradient, the single-state
path, checkpointing, and a whole-basis gate at its own propagator."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import exact, grape, krylov, model, pe
from oracle.model import HC_SX, HC_SZ
from tests.gpu_util import C64, C128, host, rel_err

pytestmark = pytest.mark.gpu

TOL = {C128: 1e-10, C64: 1e-4}


def cols(rng, n, D):
    return np.array([workloads.random_state(rng, D) for _ in range(n)])


def dev(a, dtype=C128):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def setup(seed, L=7, n=3, N=9, m=14, dt=0.15, kind=HC_SX, sites=1 << 2):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, N)
    P0, W = cols(rng, n, 1 << L), cols(rng, n, 1 << L)
    h = kg.XXZ(L, 1.0, 0.6, kind, sites)
    ch = model.Chain(L, 1.0, 0.6, kind, sites)
    return h, ch, u, P0, W, dt, m


@pytest.mark.parametrize("centred", [False, True])
@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n", [1, 2, 5])
def test_vs_oracle(centred, dtype, n):
    h, ch, u, P0, W, dt, m = setup(10 + n, n=n)
    ref = grape.gradient_columns(ch, u, P0, W, dt, m, True, krylov.default_tol(), centred=centred)
    r = kg.grape_gradient_columns(h, dev(u, torch.float64), dt, kg.Krylov(m), dev(P0, dtype),
                                  dev(W, dtype), centred=centred)
    assert abs(float(host(r.F)) - ref.F) <= TOL[dtype] * ref.F
    assert rel_err(host(r.grad), ref.grad) <= TOL[dtype]
    bc = host(r.beta_cols)
    ref_cols = [np.vdot(W[c], ref.psi_N[c]) for c in range(n)]
    assert rel_err(bc[:, 0] + 1j * bc[:, 1], ref_cols) <= TOL[dtype]


@pytest.mark.parametrize("centred", [False, True])
def test_one_column_is_the_state_transfer_path(centred):
    h, ch, u, P0, W, dt, m = setup(3, n=1)
    ud = dev(u, torch.float64)
    r = kg.grape_gradient_columns(h, ud, dt, kg.Krylov(m), dev(P0), dev(W), ckpt_every=4,
                                  centred=centred)
    s = kg.grape_gradient(h, ud, dt, kg.Krylov(m), dev(P0[0]), dev(W[0]), ckpt_every=4,
                          centred=centred)
    assert np.array_equal(host(r.grad), host(s.grad))
    assert float(host(r.F)) == float(host(s.F))


@pytest.mark.parametrize("ckpt", [1, 4, 9])
def test_checkpointed_is_bit_identical(ckpt):
    h, ch, u, P0, W, dt, m = setup(4, n=5)
    ud = dev(u, torch.float64)
    ref = kg.grape_gradient_columns(h, ud, dt, kg.Krylov(m), dev(P0, C64), dev(W, C64))
    r = kg.grape_gradient_columns(h, ud, dt, kg.Krylov(m), dev(P0, C64), dev(W, C64),
                                  ckpt_every=ckpt)
    assert np.array_equal(host(r.grad), host(ref.grad))
    assert np.array_equal(host(r.beta_cols), host(ref.beta_cols))


def test_whole_basis_gate_at_its_own_propagator():
    """All 16 columns of L=4 with W = e^{i phi} U(T) from dense propagators: F = 1 and
    a vanishing gradient (m = D makes each Krylov step exact)."""
    L, N, dt = 4, 5, 0.3
    D = 1 << L
    rng = np.random.default_rng(33)
    H0 = model.xxz_dense(L, 1.0, 0.5)
    Hc = model.hc_dense(L, HC_SX, 1 << 2)
    u = rng.uniform(-1, 1, N)
    U = np.eye(D, dtype=np.complex128)
    for uj in u:
        U = exact.propagator(H0 + uj * Hc, dt) @ U
    W = np.exp(0.7j) * U
    h = kg.XXZ(L, 1.0, 0.5, HC_SX, 1 << 2)
    r = kg.grape_gradient_columns(h, dev(u, torch.float64), dt, kg.Krylov(D), dev(np.eye(D)),
                                  dev(W.T))
    assert abs(float(host(r.F)) - 1.0) < 1e-12
    assert np.abs(host(r.grad)).max() < 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
def test_reduced_basis_columns_vs_oracle(dtype):
    t = workloads.pe_paper(9, 3)
    ch = pe.PEChain(t.L, t.K, t.J, t.Delta, t.hc_sites)
    rng = np.random.default_rng(8)
    n, N = 4, 40
    P0, W = cols(rng, n, ch.dim), cols(rng, n, ch.dim)
    u = t.u[:N]
    ref = grape.gradient_columns(ch, u, P0, W, t.dt, t.m, True, krylov.default_tol(), centred=True)
    h = kg.XXZ(t.L, t.J, t.Delta, HC_SZ, t.hc_sites)
    r = kg.grape_gradient_columns(h, dev(u, torch.float64), t.dt, kg.Krylov(t.m), dev(P0, dtype),
                                  dev(W, dtype), ckpt_every=7, centred=True,
                                  basis=kg.ReducedBasis(t.L, t.K))
    assert abs(float(host(r.F)) - ref.F) <= TOL[dtype] * ref.F
    assert rel_err(host(r.grad), ref.grad) <= TOL[dtype]


def test_gate_block_mixed_vs_fp64_L16():
    """Eight columns of an L=16 chain (65,536 amplitudes), 40 slices: complex64
    vectors with FP64 scalars against complex128."""
    h, ch, u, P0, W, dt, m = setup(9, L=16, n=8, N=40, m=16, dt=0.05)
    ud = dev(u, torch.float64)
    r128 = kg.grape_gradient_columns(h, ud, dt, kg.Krylov(m), dev(P0), dev(W), ckpt_every=7,
                                     centred=True)
    r64 = kg.grape_gradient_columns(h, ud, dt, kg.Krylov(m), dev(P0, C64), dev(W, C64),
                                    ckpt_every=7, centred=True)
    F128 = float(host(r128.F))
    assert abs(float(host(r64.F)) - F128) <= 1e-4 * F128
    assert rel_err(host(r64.grad), host(r128.grad)) <= 1e-4
