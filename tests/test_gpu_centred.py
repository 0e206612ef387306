"""The centred gradient (grape_gradient_centred) on the GPU against the oracle's
centred gradient; its relation to the plain gradient's brackets; checkpointing."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, xxz_of

pytestmark = pytest.mark.gpu


def gpu(c, dtype, centred, ckpt_every=0):
    r = kg.grape_gradient(xxz_of(c), torch.tensor(c.u, dtype=torch.float64, device="cuda"), c.dt,
                          kg.Krylov(c.m), dev_vec(c.psi0, dtype), dev_vec(c.target, dtype),
                          ckpt_every=ckpt_every, centred=centred)
    torch.cuda.synchronize()
    return r


def oracle_centred(c, vec_eps):
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    return grape.gradient_centred(ch, c.u, c.psi0, c.target, c.dt, c.m, True,
                                  krylov.default_tol(vec_eps))


def random_chain(seed, L=9, N=23, m=12):
    rng = np.random.default_rng(seed)
    return workloads.Chain(L=L, J=1.0, Delta=0.8, hc_kind=0, hc_sites=1 << 3, N=N, dt=0.07, m=m,
                           u=rng.uniform(-1, 1, N), psi0=workloads.random_state(rng, 1 << L),
                           target=workloads.random_state(rng, 1 << L))


@pytest.mark.parametrize("dtype,eps,tol", [(C128, krylov.EPS_C128, 1e-10), (C64, krylov.EPS_C64, 1e-4)])
def test_small_workload_vs_oracle(dtype, eps, tol):
    c = workloads.small()
    r = gpu(c, dtype, True)
    ref = oracle_centred(c, eps)
    assert abs(float(host(r.F)) - ref.F) / ref.F <= tol
    assert rel_err(host(r.grad), ref.grad) <= tol
    assert np.abs(host(r.grad) - ref.grad).max() / np.abs(ref.grad).max() <= tol


@pytest.mark.parametrize("N", [1, 2, 1025, 2100])
def test_lengths_vs_oracle(N):
    """One slice, two slices, and lengths that cross the 1024-entry chunks of the
    in-place averaging."""
    c = random_chain(40 + N, L=6, N=N, m=8)
    r = gpu(c, C128, True)
    ref = oracle_centred(c, krylov.EPS_C128)
    assert rel_err(host(r.grad), ref.grad) <= 1e-10


def test_mean_of_plain_brackets():
    """Entries 2..N are the means of neighbouring entries of the plain gradient,
    bit for bit (the same bracket kernels on the same states)."""
    c = random_chain(3)
    g0 = host(gpu(c, C128, False).grad)
    gc = host(gpu(c, C128, True).grad)
    assert np.array_equal(gc[1:], 0.5 * (g0[:-1] + g0[1:]))


@pytest.mark.parametrize("ckpt", [1, 4, 7, 23])
def test_checkpointed_is_bit_identical(ckpt):
    c = random_chain(5)
    ref = host(gpu(c, C64, True).grad)
    assert np.array_equal(host(gpu(c, C64, True, ckpt).grad), ref)


def test_reuses_forward_states():
    c = random_chain(6)
    h, k = xxz_of(c), kg.Krylov(c.m)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda")
    p0, f = dev_vec(c.psi0), dev_vec(c.target)
    fw = kg.grape_forward(h, u, c.dt, k, p0, f, ckpt_every=5)
    r = kg.grape_gradient(h, u, c.dt, k, p0, f, ckpt_every=5, states=fw.states, states_valid=True,
                          beta=fw.beta, centred=True)
    assert np.array_equal(host(r.grad), host(gpu(c, C128, True, 5).grad))


def test_autograd_centred():
    c = random_chain(7)
    u = torch.tensor(c.u, dtype=torch.float64, device="cuda", requires_grad=True)
    F = kg.fidelity(u, xxz_of(c), c.dt, kg.Krylov(c.m), dev_vec(c.psi0), dev_vec(c.target), 4,
                    centred=True)
    F.backward()
    assert np.array_equal(host(u.grad), host(gpu(c, C128, True, 4).grad))
