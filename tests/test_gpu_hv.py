"""H v on the GPU (xxz_apply) against the oracle: integer index maps and one-hot
columns bit-exact, random vectors to rounding, all tilings, the largest sizes."""

import numpy as np
import pytest
import torch

import paper_2010_03598_amd as kg
import workloads
from oracle import model
from oracle.model import HC_SX, HC_SZ
from tests.gpu_util import C64, C128, dev_vec, host, rel_err, tile_bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [2, 5, 8, 16, 24, 30])
def test_index_maps_bit_exact(L):
    D = 1 << L
    rng = np.random.default_rng(L)
    for s0, count in [(0, min(D, 4096)), (D - min(D, 1000), min(D, 1000)),
                      (int(rng.integers(0, max(1, D - 5000))), min(D, 5000))]:
        n_anti, pmask = kg.debug_index_map(L, s0, count)
        s = np.arange(s0, s0 + count, dtype=np.int64)
        assert np.array_equal(host(n_anti), model.n_antiparallel(L, s))
        assert np.array_equal(host(pmask).astype(np.int64) & 0xffffffff, model.partner_mask(L, s))


def dyadic_chain(L, kind, sites):
    return kg.XXZ(L, 1.0, 0.5, kind, sites)


CASES = [(HC_SX, lambda L: 1), (HC_SX, lambda L: 1 << (L // 2)), (HC_SX, lambda L: 1 << (L - 1)),
         (HC_SZ, lambda L: 1 | (1 << (L - 1))), (HC_SZ, lambda L: (1 << L) - 1)]


@pytest.mark.parametrize("L", [2, 3, 4, 6, 7, 9])
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", [C128, C64])
def test_columns_bit_exact_small(L, case, dtype):
    """H e_s for every s: each amplitude is one product of dyadic numbers, so exact."""
    kind, sites_of = CASES[case]
    sites = sites_of(L)
    h = dyadic_chain(L, kind, sites)
    u = 0.75
    Hk = model.xxz_dense(L, 1.0, 0.5) + u * model.hc_dense(L, kind, sites)
    D = 1 << L
    for s in range(D):
        e = torch.zeros(D, dtype=dtype, device="cuda")
        e[s] = 1.0
        col = host(kg.xxz_apply(h, u, e))
        assert np.array_equal(col.astype(np.complex128), Hk[:, s]), (L, s)


def expected_column(L, kind, sites, u, s):
    """Nonzero entries of column s of H0 + u Hc from the oracle's element rules."""
    out = {}
    sv = np.array([s], dtype=np.int64)
    d = float(model.diag_h0(L, 1.0, 0.5, sv)[0])
    if kind == HC_SZ:
        d += u * float(model.sz_control_diag(L, sites, sv)[0])
    out[s] = d
    pm = int(model.partner_mask(L, sv)[0])
    for p in range(L - 1):
        if (pm >> p) & 1:
            out[s ^ (3 << p)] = 0.5
    if kind == HC_SX:
        (i,) = model.hc_sites_list(L, sites)
        out[s ^ (1 << (L - i))] = out.get(s ^ (1 << (L - i)), 0.0) + 0.5 * u
    return out


@pytest.mark.parametrize("L", [13, 16, 20, 24])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_columns_bit_exact_sampled(L, dtype):
    D = 1 << L
    rng = np.random.default_rng(100 + L)
    u = 0.75
    for kind, sites in [(HC_SX, 1), (HC_SZ, 1 | (1 << (L - 1)))]:
        h = dyadic_chain(L, kind, sites)
        e = torch.zeros(D, dtype=dtype, device="cuda")
        for s in [0, D - 1, 0b0101 << (L - 4)] + [int(x) for x in rng.integers(0, D, 3)]:
            e.zero_()
            e[s] = 1.0
            col = kg.xxz_apply(h, u, e)
            want = expected_column(L, kind, sites, u, s)
            idx = torch.tensor(sorted(want), device="cuda")
            got = host(col[idx]).astype(np.complex128)
            assert np.array_equal(got, np.array([want[i] for i in sorted(want)])), (L, s)
            nz = int(torch.count_nonzero(col).item())
            assert nz == sum(1 for v in want.values() if v != 0.0)


@pytest.mark.parametrize("L", [2, 3, 5, 6, 8, 11, 12, 14, 16, 18])
@pytest.mark.parametrize("kind", [HC_SX, HC_SZ])
def test_random_vectors_c128(L, kind):
    rng = np.random.default_rng(L * 7 + kind)
    D = 1 << L
    sites = 1 << (L // 2) if kind == HC_SX else 1 | (1 << (L - 1))
    J, Delta, u = 0.9, 1.37, -0.61
    v = workloads.random_state(rng, D)
    ref = model.apply_h(L, J, Delta, kind, sites, u, v)
    out = host(kg.xxz_apply(kg.XXZ(L, J, Delta, kind, sites), u, dev_vec(v)))
    assert np.abs(out - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("L", [6, 10, 14, 17])
def test_random_vectors_c64(L):
    rng = np.random.default_rng(L)
    D = 1 << L
    v = workloads.random_state(rng, D).astype(np.complex64)
    ref = model.apply_h(L, 1.0, 0.5, HC_SX, 1, 0.3, v.astype(np.complex128))
    out = host(kg.xxz_apply(kg.XXZ(L, 1.0, 0.5), 0.3, dev_vec(v, C64)))
    assert np.abs(out - ref).max() <= 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("tb", [6, 7, 8, 9, 10, 11, 12, 13])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_every_tiling(tb, dtype):
    """Every (register, wavefront) split of the tile gives the same H v, for
    complex64 also the pair layout (tiles of 2^10 and more); S^x on the first
    site (a far partner), on site 11 (inside the wavefront) and on the last site
    (the other half of the thread's own pair in the pair layout)."""
    L = 14
    rng = np.random.default_rng(tb)
    v = workloads.random_state(rng, 1 << L)
    for kind, sites in [(HC_SX, 1), (HC_SX, 1 << 10), (HC_SX, 1 << (L - 1)),
                        (HC_SZ, 0b101 << 5)]:
        ref = model.apply_h(L, 1.0, 0.8, kind, sites, 0.45, v.astype(dtype_np(dtype)).astype(complex))
        with tile_bits(tb):
            out = host(kg.xxz_apply(kg.XXZ(L, 1.0, 0.8, kind, sites), 0.45, dev_vec(v, dtype)))
        tol = 1e-14 if dtype == C128 else 2e-6
        assert np.abs(out - ref).max() <= tol * np.abs(ref).max(), (tb, kind, sites)


def dtype_np(dtype):
    return np.complex128 if dtype == C128 else np.complex64


def test_hermitian():
    L = 15
    rng = np.random.default_rng(3)
    a = workloads.random_state(rng, 1 << L)
    b = workloads.random_state(rng, 1 << L)
    h = kg.XXZ(L, 1.0, 0.7, HC_SX, 1 << 3)
    Ha = host(kg.xxz_apply(h, 0.2, dev_vec(a)))
    Hb = host(kg.xxz_apply(h, 0.2, dev_vec(b)))
    assert abs(np.vdot(a, Hb) - np.conj(np.vdot(b, Ha))) < 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
def test_large_sampled_rows(dtype):
    """L=24 (the large workload's size): sampled output amplitudes from the oracle's rows."""
    L = 24
    D = 1 << L
    rng = np.random.default_rng(24)
    v = workloads.random_phase_state(rng, D)
    out = kg.xxz_apply(kg.XXZ(L, 1.0, 0.5), 0.37, dev_vec(v, dtype))
    rows = np.concatenate([np.arange(64), D - 1 - np.arange(64), rng.integers(0, D, 2000)])
    got = host(out[torch.tensor(rows, device="cuda")])
    vv = v.astype(dtype_np(dtype)).astype(np.complex128)
    ref = model.h_rows(L, 1.0, 0.5, HC_SX, 1, 0.37, vv, rows)
    scale = np.abs(ref).max()
    tol = 1e-14 if dtype == C128 else 2e-6
    assert np.abs(got - ref).max() <= tol * scale


def test_max_size_sampled():
    """L=30 (largest supported): 2^30 complex64 amplitudes in and out (16 GiB)."""
    L = 30
    D = 1 << L
    g = torch.Generator(device="cuda")
    g.manual_seed(30)
    v = torch.randn(D, dtype=C64, device="cuda", generator=g)
    out = kg.xxz_apply(kg.XXZ(L, 1.0, 0.5), -0.8, v)
    rng = np.random.default_rng(30)
    rows = np.concatenate([[0, 1, D - 2, D - 1], rng.integers(0, D, 200)])
    # the rows need v at s and its L partners only
    need = set()
    for s in rows:
        need.add(int(s))
        need.add(int(s) ^ (1 << (L - 1)))
        for p in range(L - 1):
            need.add(int(s) ^ (3 << p))
    need = np.array(sorted(need))
    vals = host(v[torch.tensor(need, device="cuda")]).astype(np.complex128)
    sparse = dict(zip(need.tolist(), vals.tolist()))

    class Lookup:
        def __getitem__(self, idx):
            idx = np.asarray(idx)
            return np.array([sparse[int(i)] for i in idx.ravel()]).reshape(idx.shape)

    ref = model.h_rows(L, 1.0, 0.5, HC_SX, 1, -0.8, Lookup(), rows)
    got = host(out[torch.tensor(rows, device="cuda")])
    assert np.abs(got - ref).max() <= 2e-6 * np.abs(ref).max()
    del v, out
    torch.cuda.empty_cache()
