"""Pins of the fixed-excitation, parity-even reduced basis (oracle/pe.py)."""

from math import comb

import numpy as np
import pytest

import workloads
from oracle import exact, grape, krylov, model, pe
from oracle.model import HC_SZ

EDGES = lambda L: 1 | (1 << (L - 1))          # sites 1 and L: the paper's control


def full_parts(L, J, Delta, sites):
    return model.xxz_dense(L, J, Delta), model.hc_dense(L, HC_SZ, sites)


@pytest.mark.parametrize("L,K", [(4, 2), (5, 2), (6, 3), (7, 2), (8, 4), (9, 3)])
def test_basis_counts_and_order(L, K):
    B = pe.PEBasis(L, K)
    assert B.dim == pe.sector_dim_count(L, K)
    assert np.all(np.diff(B.reps) > 0)
    # every sector state belongs to exactly one orbit
    st = pe.sector_states(L, K)
    assert st.size == comb(L, K)
    idx = B.index(st)
    assert np.array_equal(np.bincount(idx, minlength=B.dim), B.n)


@pytest.mark.parametrize("L,K", [(5, 2), (6, 3), (8, 3), (9, 4)])
def test_reduced_h_is_the_restriction_of_the_full_h(L, K):
    """y = P H_full E x for random x (E: embed, P: project), dyadic J, Delta, u."""
    J, Delta, u = 1.0, 0.5, 0.75
    B = pe.PEBasis(L, K)
    H0, Hc = full_parts(L, J, Delta, EDGES(L))
    rng = np.random.default_rng(L * 10 + K)
    x = rng.standard_normal(B.dim) + 1j * rng.standard_normal(B.dim)
    y_full = B.project((H0 + u * Hc) @ B.embed(x))
    y = pe.apply_h_pe(B, J, Delta, EDGES(L), u, x)
    assert np.abs(y - y_full).max() < 1e-13 * max(1.0, np.abs(y).max())
    # the embedding is an isometry onto a parity-even subspace
    X = B.embed(x)
    assert abs(np.linalg.norm(X) - np.linalg.norm(x)) < 1e-13
    assert np.abs(X - X[pe.reverse_bits(np.arange(1 << L), L)]).max() == 0.0


@pytest.mark.parametrize("L,K", [(6, 3), (7, 3), (8, 4)])
def test_paper_construction_gives_the_same_operator(L, K):
    """The paper's route: diagonalise Pi in the K-sector, keep the +1 eigenvectors Q,
    H_red = Q^dag H Q.  Same spectrum as the orbit basis, and the same subspace."""
    J, Delta, u = 1.0, 0.5, -0.3
    H0, Hc = full_parts(L, J, Delta, EDGES(L))
    H = H0 + u * Hc
    st = pe.sector_states(L, K)
    rev = pe.reverse_bits(st, L)
    pos = {int(s): i for i, s in enumerate(st)}
    Pi = np.zeros((st.size, st.size))
    for i, r in enumerate(rev):
        Pi[pos[int(r)], i] = 1.0
    w, V = np.linalg.eigh(Pi)
    Q = V[:, w > 0]
    Hs = H[np.ix_(st, st)]
    Hq = Q.T @ Hs @ Q
    B = pe.PEBasis(L, K)
    Hpe = pe.dense_pe(B, J, Delta, EDGES(L), u)
    assert np.abs(Hpe - Hpe.conj().T).max() < 1e-15
    assert np.allclose(np.linalg.eigvalsh(Hq), np.linalg.eigvalsh(Hpe), atol=1e-12)
    # subspace: the embedded basis vectors lie in span(Q)
    for c in range(B.dim):
        e = np.zeros(B.dim)
        e[c] = 1.0
        v = B.embed(e)[st]
        assert np.linalg.norm(v - Q @ (Q.T @ v)) < 1e-12


def test_task_states_are_the_example_orbits():
    L, K = 7, 2
    B = pe.PEBasis(L, K)
    e1, eD = B.task_states()
    X1, XD = B.embed(e1), B.embed(eD)
    # e_1: two up spins (0 bits) in the middle: down down up up down down down and its mirror
    a = int("1100111", 2)
    assert abs(X1[a]) > 0 and abs(X1[pe.reverse_bits(np.array([a]), L)[0]]) > 0
    # e_D: the up spins at one edge, in even superposition with the other edge
    left, right = int("0011111", 2), int("1111100", 2)
    assert abs(XD[left] - 2 ** -0.5) < 1e-15 and abs(XD[right] - 2 ** -0.5) < 1e-15
    assert abs(np.vdot(X1, XD)) == 0.0


def test_gradient_equals_full_space_gradient():
    """F and the exact PWC gradient of the transfer task are the same computed in the
    reduced basis and in the full 2^L space (dense propagators in both); the Krylov
    zeroth-order gradient on the reduced chain matches the full-space one."""
    L, K, N, dt = 7, 2, 6, 0.3
    J, Delta = 1.0, 0.5
    sites = EDGES(L)
    B = pe.PEBasis(L, K)
    e1, eD = B.task_states()
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, N)
    H0, Hc = full_parts(L, J, Delta, sites)
    Ff, gf = exact.exact_gradient_dense(H0, Hc, u, B.embed(e1), B.embed(eD), dt)
    H0r = pe.dense_pe(B, J, Delta, sites, 0.0)
    Hcr = np.diag(pe.hc_pe(B, sites)).astype(np.complex128)
    Fr, gr = exact.exact_gradient_dense(H0r, Hcr, u, e1, eD, dt)
    assert abs(Ff - Fr) < 1e-13 and np.abs(gf - gr).max() < 1e-13
    ch = pe.PEChain(L, K, J, Delta, sites)
    full = model.Chain(L, J, Delta, HC_SZ, sites)
    rk = grape.gradient(ch, u, e1, eD, dt, 12)
    rf = grape.gradient(full, u, B.embed(e1), B.embed(eD), dt, 12)
    assert abs(rk.F - rf.F) < 1e-12 and np.abs(rk.grad - rf.grad).max() < 1e-12


def test_control_sites_must_be_mirror_symmetric():
    with pytest.raises(ValueError):
        pe.PEChain(6, 3, 1.0, 0.5, 1)


@pytest.mark.parametrize("LK,D", sorted(workloads.PAPER_PE_DIMS.items()))
def test_dimensions_quoted_in_the_results(LK, D):
    """Sec. III.B quotes D = 10, 19, 44, 60, 146; each is the even-orbit count of a
    K = 3 sector (the (L, K) pairs are the workloads' reading)."""
    assert pe.sector_dim_count(*LK) == D
    assert pe.PEBasis(*LK).dim == D


def test_row_spot_check_equals_the_whole_product():
    B = pe.PEBasis(9, 4)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(B.dim) + 1j * rng.standard_normal(B.dim)
    y = pe.apply_h_pe(B, 2.0, 0.5, EDGES(9), 0.3, x)
    rows = [0, 5, B.dim // 2, B.dim - 1]
    assert np.abs(pe.apply_h_pe_rows(B, 2.0, 0.5, EDGES(9), 0.3, x, rows) - y[rows]).max() < 1e-14
