"""grape_forward / grape_gradient / grape_ascent_update on the GPU against the oracle."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from oracle.model import HC_SX, HC_SZ
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, xxz_of

pytestmark = pytest.mark.gpu


def run_gpu(c, dtype=C128, reorth=True, ckpt_every=0, m=None):
    h = xxz_of(c)
    k = kg.Krylov(c.m if m is None else m, reorth)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    r = kg.grape_gradient(h, u, c.dt, k, dev_vec(c.psi0, dtype), dev_vec(c.target, dtype),
                          ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    return r


def run_oracle(c, reorth=True, vec_eps=krylov.EPS_C128):
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    return grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m, reorth,
                          krylov.default_tol(vec_eps))


def errors(r, ref):
    F = float(host(r.F))
    g = host(r.grad)
    b = host(r.beta)
    eF = abs(F - ref.F) / abs(ref.F)
    eg = rel_err(g, ref.grad)
    eg_inf = float(np.abs(g - ref.grad).max() / np.abs(ref.grad).max())
    eb = abs(complex(b[0], b[1]) - ref.beta) / abs(ref.beta)
    return eF, eg, eg_inf, eb


@pytest.mark.parametrize("reorth", [True, False])
def test_small_workload_c128(reorth):
    c = workloads.small()
    ref = run_oracle(c, reorth)
    r = run_gpu(c, reorth=reorth)
    assert max(errors(r, ref)) <= 1e-10


def test_small_workload_c64():
    c = workloads.small()
    ref = run_oracle(c)
    r = run_gpu(c, dtype=C64)
    assert max(errors(r, ref)) <= 1e-4


def random_chain(L, N, dt, m, kind, sites, Delta, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    return workloads.Chain(L=L, J=1.0, Delta=Delta, hc_kind=kind, hc_sites=sites, N=N, dt=dt,
                           m=m, u=u, psi0=psi0, target=f)


@pytest.mark.parametrize("L,N,dt,m,kind,sites,Delta", [
    (2, 5, 0.3, 4, HC_SX, 2, 0.5), (5, 9, 0.2, 8, HC_SZ, 0b10001, 0.5),
    (7, 13, 0.1, 12, HC_SX, 1 << 3, 1.2), (10, 20, 0.05, 16, HC_SX, 1, 0.0),
    (12, 7, 0.5, 20, HC_SZ, 1 | (1 << 11), 0.5), (14, 6, 0.05, 24, HC_SX, 1, 1.0)])
def test_random_chains(L, N, dt, m, kind, sites, Delta):
    c = random_chain(L, N, dt, m, kind, sites, Delta, seed=L * 13 + N)
    ref = run_oracle(c)
    r = run_gpu(c)
    assert max(errors(r, ref)) <= 1e-10
    r64 = run_gpu(c, dtype=C64)
    assert max(errors(r64, ref)) <= 1e-4


@pytest.mark.parametrize("N,ckpt", [(17, 1), (17, 3), (17, 7), (17, 16), (17, 17), (40, 5),
                                    (40, 6), (41, 2)])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_checkpointed_is_bit_identical(N, ckpt, dtype):
    """Segment recomputation (paired with the costate sweep) reproduces the stored
    forward states exactly, so the gradient does not depend on the checkpointing."""
    c = random_chain(11, N, 0.05, 12, HC_SX, 1, 0.7, seed=ckpt)
    a = run_gpu(c, dtype=dtype, ckpt_every=0)
    b = run_gpu(c, dtype=dtype, ckpt_every=ckpt)
    assert np.array_equal(host(a.grad), host(b.grad))
    assert np.array_equal(host(a.beta), host(b.beta))
    assert float(host(a.F)) == float(host(b.F))


def test_forward_then_gradient_reuses_states():
    c = random_chain(12, 25, 0.05, 16, HC_SX, 1, 0.5, seed=5)
    h = xxz_of(c)
    k = kg.Krylov(c.m)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    psi0, f = dev_vec(c.psi0, C64), dev_vec(c.target, C64)
    fw = kg.grape_forward(h, u, c.dt, k, psi0, f, ckpt_every=5)
    g1 = kg.grape_gradient(h, u, c.dt, k, psi0, f, ckpt_every=5, states=fw.states,
                           states_valid=True, beta=fw.beta)
    g2 = kg.grape_gradient(h, u, c.dt, k, psi0, f, ckpt_every=5)
    assert np.array_equal(host(g1.grad), host(g2.grad))
    assert float(host(fw.F)) == float(host(g2.F))


def test_repeat_is_bit_identical():
    c = random_chain(15, 10, 0.05, 20, HC_SX, 1, 1.0, seed=9)
    a = run_gpu(c, dtype=C64)
    b = run_gpu(c, dtype=C64)
    assert np.array_equal(host(a.grad), host(b.grad))


def test_forward_state_is_unitary_image():
    c = random_chain(16, 12, 0.05, 16, HC_SX, 1, 0.5, seed=16)
    h = xxz_of(c)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    fw = kg.grape_forward(h, u, c.dt, kg.Krylov(16), dev_vec(c.psi0), dev_vec(c.target))
    D = 1 << c.L
    psi_N = host(fw.states[(c.N - 1) * D: c.N * D])
    assert abs(np.linalg.norm(psi_N) - 1.0) <= 1e-12


def test_ascent_update_matches_oracle():
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, 333)
    g = rng.standard_normal(333)
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    kg.grape_ascent_update(ud, torch.tensor(g, dtype=torch.float64, device="cuda"), 0.1)
    assert np.abs(host(ud) - grape.ascent_update(u, g, 0.1)).max() <= 1e-15
    kg.grape_ascent_update(ud, torch.zeros(333, dtype=torch.float64, device="cuda"), 0.1)
    assert np.abs(host(ud) - grape.ascent_update(u, g, 0.1)).max() <= 1e-15



@pytest.mark.parametrize("centred", [False, True])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_side_stream_recomputation_is_bit_identical(centred, dtype, monkeypatch):
    """Segment recomputation on the library's second stream gives exactly the
    results of the same calls made on the caller's stream (KG_ONE_STREAM)."""
    c = random_chain(12, 37, 0.05, 14, HC_SX, 1, 0.7, seed=21)
    h, k = xxz_of(c), kg.Krylov(c.m)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    args = (h, u, c.dt, k, dev_vec(c.psi0, dtype), dev_vec(c.target, dtype))
    two = kg.grape_gradient(*args, ckpt_every=5, centred=centred)
    g2, F2 = host(two.grad), float(host(two.F))
    monkeypatch.setenv("KG_ONE_STREAM", "1")
    one = kg.grape_gradient(*args, ckpt_every=5, centred=centred)
    g1, F1 = host(one.grad), float(host(one.F))
    monkeypatch.delenv("KG_ONE_STREAM")
    stored = kg.grape_gradient(*args, ckpt_every=0, centred=centred)
    assert np.array_equal(g1, g2) and F1 == F2
    assert np.array_equal(host(stored.grad), g2)


@pytest.mark.parametrize("dtype,tol", [(C128, 1e-10), (C64, 1e-4)])
def test_gradient_at_largest_krylov_dimension(dtype, tol):
    """m = 64 (the largest accepted) through the checkpointed sweeps: 4 segments, so
    the recomputation runs beside the costate propagation."""
    c = random_chain(10, 12, 0.2, 64, HC_SX, 1, 0.6, seed=64)
    eps = krylov.EPS_C128 if dtype == C128 else krylov.EPS_C64
    ref = run_oracle(c, vec_eps=eps)
    r = run_gpu(c, dtype=dtype, ckpt_every=3)
    assert max(errors(r, ref)) <= tol
    stored = run_gpu(c, dtype=dtype, ckpt_every=0)
    assert np.array_equal(host(stored.grad), host(r.grad))


@pytest.mark.parametrize("L", [23, 24])
def test_checkpointed_is_bit_identical_large(L):
    """At the large vector sizes (complex64 tiles of 2^11 amplitudes from L = 23)
    the checkpointed gradient with 3 segments equals the store-all one bit for bit."""
    c = random_chain(L, 7, 0.05, 8, HC_SX, 1, 0.5, seed=L)
    a = run_gpu(c, dtype=C64, ckpt_every=2)
    b = run_gpu(c, dtype=C64, ckpt_every=0)
    assert np.array_equal(host(a.grad), host(b.grad))
    assert float(host(a.F)) == float(host(b.F))
