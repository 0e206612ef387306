"""First order of the hierarchy of the time-averaged control operator
(grape_gradient_first_order) against the oracle's hierarchy at P = 1."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import grape, krylov, model
from oracle.model import HC_SX, HC_SZ
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, xxz_of

pytestmark = pytest.mark.gpu


def chain(seed, L=9, N=17, m=14, kind=HC_SX, sites=1 << 4):
    rng = np.random.default_rng(seed)
    return workloads.Chain(L=L, J=1.0, Delta=0.7, hc_kind=kind, hc_sites=sites, N=N, dt=0.08,
                           m=m, u=rng.uniform(-1, 1, N), psi0=workloads.random_state(rng, 1 << L),
                           target=workloads.random_state(rng, 1 << L))


def gpu(c, dtype=C128, ckpt_every=0):
    r = kg.grape_gradient(xxz_of(c), torch.tensor(c.u, dtype=torch.float64, device="cuda"), c.dt,
                          kg.Krylov(c.m), dev_vec(c.psi0, dtype), dev_vec(c.target, dtype),
                          ckpt_every=ckpt_every, first_order=True)
    torch.cuda.synchronize()
    return r


def oracle(c, eps):
    ch = model.Chain(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    return grape.gradient_hierarchy(ch, c.u, c.psi0, c.target, c.dt, c.m, 1, True,
                                    krylov.default_tol(eps))


@pytest.mark.parametrize("kind,sites", [(HC_SX, 1 << 4), (HC_SX, 1 << 8), (HC_SZ, 0b100000001)])
def test_vs_oracle(kind, sites):
    c = chain(1, kind=kind, sites=sites)
    ref = oracle(c, krylov.EPS_C128)
    r = gpu(c)
    assert abs(float(host(r.F)) - ref.F) / ref.F <= 1e-10
    assert rel_err(host(r.grad), ref.grad) <= 1e-10
    ref64 = oracle(c, krylov.EPS_C64)
    assert rel_err(host(gpu(c, C64).grad), ref64.grad) <= 1e-4


def test_small_workload():
    c = workloads.small()
    ref = oracle(c, krylov.EPS_C128)
    assert rel_err(host(gpu(c).grad), ref.grad) <= 1e-10


@pytest.mark.parametrize("ckpt", [1, 5, 17])
def test_checkpointed_is_bit_identical(ckpt):
    c = chain(2)
    assert np.array_equal(host(gpu(c, C128, ckpt).grad), host(gpu(c).grad))
