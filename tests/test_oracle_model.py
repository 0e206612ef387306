"""Pins of the oracle's Hamiltonian and Krylov propagator (CPU only).

Each check compares the oracle with something other than itself: a second
independent construction, a closed form, a symmetry of the model, or a library
routine on a case that reduces to it.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import krylov, model
from oracle.model import HC_SX, HC_SZ


def dense_h(L, J, Delta, kind, sites, u):
    return model.xxz_dense(L, J, Delta) + u * model.hc_dense(L, kind, sites)


# ---------------------------------------------------------------- Hamiltonian constructions

@pytest.mark.parametrize("L", [2, 3, 5, 8])
@pytest.mark.parametrize("kind,sites", [(HC_SX, 1), (HC_SX, 1 << 2), (HC_SZ, 1 | (1 << 1))])
def test_kronecker_equals_bit_construction_dyadic(L, kind, sites):
    """With dyadic J, Delta, u every matrix entry is exact in both constructions."""
    if sites.bit_length() > L:
        pytest.skip("site outside chain")
    J, Delta, u = 1.0, 0.5, 0.75
    Hk = dense_h(L, J, Delta, kind, sites, u)
    ch = model.Chain(L, J, Delta, kind, sites, matrix_free=False)
    Hs = (ch.H0 + u * ch.Hc).toarray()
    assert np.array_equal(Hk, Hs)
    # matrix-free apply and per-row evaluation on the identity columns
    D = 1 << L
    for s in range(D):
        e = np.zeros(D, complex)
        e[s] = 1.0
        col = model.apply_h(L, J, Delta, kind, sites, u, e)
        assert np.array_equal(col, Hk[:, s])
    v = workloads.random_state(np.random.default_rng(L), D)
    rows = np.arange(D)
    assert np.allclose(model.h_rows(L, J, Delta, kind, sites, u, v, rows), Hk @ v, atol=1e-14)


@pytest.mark.parametrize("L,Delta", [(4, 0.3), (6, 1.37), (7, 0.0)])
def test_constructions_agree_nondyadic(L, Delta):
    J, u = 0.9, -0.61
    Hk = dense_h(L, J, Delta, HC_SX, 1, u)
    ch = model.Chain(L, J, Delta, HC_SX, 1, matrix_free=False)
    assert np.allclose((ch.H0 + u * ch.Hc).toarray(), Hk, atol=1e-15, rtol=0)


@pytest.mark.parametrize("L", [3, 6])
def test_pauli_form_equals_spin_form(L):
    """Eq. 6 as printed, (J_p/2) sum sigma.sigma, is the S-form with J = 2 J_p, Delta = alpha_z."""
    Jp, az = 1.0, 0.5
    assert np.allclose(model.pauli_drift_dense(L, Jp, az), model.xxz_dense(L, 2 * Jp, az),
                       atol=1e-14, rtol=0)
    # the paper's control (J/2)(sigma^z_1 + sigma^z_L) = J_p (S^z_1 + S^z_L)
    sz = 2 * model.SZ
    paper_hc = (Jp / 2) * (model.site_op(L, 1, sz) + model.site_op(L, L, sz))
    ours = Jp * model.hc_dense(L, HC_SZ, 1 | (1 << (L - 1)))
    assert np.allclose(paper_hc, ours, atol=1e-15)


def test_basis_convention():
    """Up = bit 0, down = bit 1, site 1 most significant; S^z_1 reads the top bit."""
    L = 8
    assert workloads.basis_index("u" + "d" * 7) == 127
    assert workloads.basis_index("d" * 7 + "u") == 254
    sz1 = np.real(np.diag(model.site_op(L, 1, model.SZ)))
    assert sz1[127] == 0.5 and sz1[254] == -0.5
    szL = np.real(np.diag(model.site_op(L, L, model.SZ)))
    assert szL[254] == 0.5 and szL[127] == -0.5


@pytest.mark.parametrize("L", [4, 7])
def test_hermitian_and_symmetries(L):
    H0 = model.xxz_dense(L, 1.0, 0.5)
    assert np.array_equal(H0, H0.conj().T)
    sztot = sum(model.site_op(L, i, model.SZ) for i in range(1, L + 1))
    assert np.abs(H0 @ sztot - sztot @ H0).max() == 0.0          # Sec. III.A: [H_d, S^z] = 0
    D = 1 << L
    # parity: mirror the chain (bit b <-> bit L-1-b)
    P = np.zeros((D, D))
    for s in range(D):
        r = int(format(s, f"0{L}b")[::-1], 2)
        P[r, s] = 1.0
    assert np.abs(P @ H0 @ P - H0).max() < 1e-15
    hc = model.hc_dense(L, HC_SZ, 1 | (1 << (L - 1)))
    assert np.abs(P @ hc @ P - hc).max() == 0.0


def test_two_site_spectrum():
    """L=2: triplet m=+-1 at J Delta/4, m=0 doublet at +-J/2 - J Delta/4."""
    J, Delta = 1.3, 0.7
    ev = np.sort(np.linalg.eigvalsh(model.xxz_dense(2, J, Delta)))
    ref = np.sort([J * Delta / 4, J * Delta / 4, J / 2 - J * Delta / 4, -J / 2 - J * Delta / 4])
    assert np.allclose(ev, ref, atol=1e-15)


def test_index_maps_brute_force():
    L = 9
    s = np.arange(1 << L)
    pm = model.partner_mask(L, s)
    na = model.n_antiparallel(L, s)
    for x in [0, 1, 5, 127, 254, 300, 511]:
        bits = [(x >> b) & 1 for b in range(L)]
        want = sum(1 << p for p in range(L - 1) if bits[p] != bits[p + 1])
        assert pm[x] == want and na[x] == bin(want).count("1")


# ---------------------------------------------------------------- Krylov propagator

def krylov_prop(L, J, Delta, kind, sites, u, psi, t, m, reorth=True, tol=None):
    ch = model.Chain(L, J, Delta, kind, sites)
    return krylov.expv(lambda v: ch.apply(u, v), psi, t, m, reorth, tol, return_info=True)


def test_two_site_closed_form():
    """exp(-itH)|up,down> = e^{i J Delta t/4}(cos(Jt/2)|up,down> - i sin(Jt/2)|down,up>)."""
    J, Delta, t = 1.0, 0.5, 0.73
    psi = workloads.basis_state(2, workloads.basis_index("ud"))
    out, _ = krylov_prop(2, J, Delta, HC_SX, 1, 0.0, psi, t, 4)
    ref = np.zeros(4, complex)
    ph = np.exp(1j * J * Delta * t / 4)
    ref[workloads.basis_index("ud")] = ph * np.cos(J * t / 2)
    ref[workloads.basis_index("du")] = -1j * ph * np.sin(J * t / 2)
    assert np.abs(out - ref).max() < 1e-15


@pytest.mark.parametrize("L", [10, 14])
def test_single_magnon_xx_closed_form(L):
    """XX chain (Delta=0), one up spin at site 1 in a down background: textbook hopping."""
    J, t = 1.0, 0.4
    psi = workloads.basis_state(L, workloads.basis_index("u" + "d" * (L - 1)))
    out, lz = krylov_prop(L, J, 0.0, HC_SX, 1, 0.0, psi, t, 24)
    k = np.arange(1, L + 1)
    for n in range(1, L + 1):
        amp = np.sum(2.0 / (L + 1) * np.sin(np.pi * k / (L + 1)) * np.sin(np.pi * k * n / (L + 1))
                     * np.exp(-1j * J * np.cos(np.pi * k / (L + 1)) * t))
        idx = workloads.basis_index("d" * (n - 1) + "u" + "d" * (L - n))
        assert abs(out[idx] - amp) < 1e-12
    mask = np.ones(1 << L, bool)
    for n in range(1, L + 1):
        mask[workloads.basis_index("d" * (n - 1) + "u" + "d" * (L - n))] = False
    assert np.all(out[mask] == 0.0)


@pytest.mark.parametrize("L,m,t,u", [(6, 12, 0.1, 0.3), (8, 10, 0.1, -0.9), (10, 16, 0.25, 1.7),
                                     (8, 24, 0.5, 0.0)])
def test_krylov_matches_dense_expm(L, m, t, u):
    rng = np.random.default_rng(L * 100 + m)
    psi = workloads.random_state(rng, 1 << L)
    out, lz = krylov_prop(L, 1.0, 0.5, HC_SX, 1, u, psi, t, m)
    H = dense_h(L, 1.0, 0.5, HC_SX, 1, u)
    ref = sla.expm(-1j * t * H) @ psi
    assert np.linalg.norm(out - ref) < 1e-12
    # orthonormal basis and T = V H V^dagger
    V = lz.V
    assert np.abs(V.conj() @ V.T - np.eye(lz.m_eff)).max() < 1e-13
    T = V.conj() @ H @ V.T
    assert np.abs(np.diag(T).real - lz.alpha).max() < 1e-12
    assert np.abs(np.diag(T, -1) - lz.beta).max() < 1e-12


def test_tri_exp_against_library_expm():
    rng = np.random.default_rng(7)
    for m in [1, 2, 5, 13, 24]:
        a = rng.standard_normal(m) * 3
        b = np.abs(rng.standard_normal(m - 1)) + 0.1
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        for t in [0.05, -0.3, 2.0]:
            ref = sla.expm(-1j * t * T)[:, 0]
            assert np.abs(krylov.tri_exp_e1(a, b, t) - ref).max() < 1e-13


def test_unitarity_and_reversibility():
    L = 12
    rng = np.random.default_rng(3)
    psi = 0.7 * workloads.random_state(rng, 1 << L)
    out, lz = krylov_prop(L, 1.0, 1.0, HC_SX, 1, 0.8, psi, 0.05, 20)
    assert abs(np.linalg.norm(out) - 0.7) < 1e-12
    back, _ = krylov_prop(L, 1.0, 1.0, HC_SX, 1, 0.8, out, -0.05, 20)
    assert np.linalg.norm(back - psi) < 1e-12


def test_sz_sector_exact_zero_leakage_and_breakdown():
    """SZ control conserves S^z_tot: amplitudes outside the start sector stay exactly 0,
    and the Krylov space of a one-magnon start closes at the sector dimension L."""
    L = 8
    psi = workloads.basis_state(L, workloads.basis_index("u" + "d" * 7))
    out, lz = krylov_prop(L, 1.0, 0.5, HC_SZ, 1 | (1 << 7), 0.6, psi, 0.5, 12)
    assert lz.m_eff == 8
    sector = np.array([bin(s).count("1") == L - 1 for s in range(1 << L)])
    assert np.all(out[~sector] == 0.0)
    H = dense_h(L, 1.0, 0.5, HC_SZ, 1 | (1 << 7), 0.6)
    assert np.linalg.norm(out - sla.expm(-0.5j * H) @ psi) < 1e-12


def test_parity_conserved_with_paper_control():
    L = 7
    D = 1 << L
    rng = np.random.default_rng(11)
    v = workloads.random_state(rng, D)
    rev = np.array([int(format(s, f"0{L}b")[::-1], 2) for s in range(D)])
    even = v + v[rev]
    even /= np.linalg.norm(even)
    out, _ = krylov_prop(L, 1.0, 0.5, HC_SZ, 1 | (1 << (L - 1)), -0.4, even, 0.3, 16)
    assert np.linalg.norm(out[rev] - out) < 1e-12


def test_zero_vector():
    out, lz = krylov_prop(5, 1.0, 0.5, HC_SX, 1, 0.1, np.zeros(32, complex), 0.1, 6)
    assert lz.m_eff == 0 and np.all(out == 0)


def test_krylov_error_order():
    """App. A: for small steps the Krylov error behaves as O(dt^m)."""
    L = 8
    rng = np.random.default_rng(5)
    psi = workloads.random_state(rng, 1 << L)
    H = dense_h(L, 1.0, 0.5, HC_SX, 1, 0.3)
    lam, Q = np.linalg.eigh(H)
    for m in [3, 4, 5, 6]:
        dts = np.array([0.08, 0.04, 0.02])
        errs = []
        for dt in dts:
            out, _ = krylov_prop(L, 1.0, 0.5, HC_SX, 1, 0.3, psi, dt, m)
            ref = (Q * np.exp(-1j * lam * dt)) @ (Q.conj().T @ psi)
            errs.append(np.linalg.norm(out - ref))
        slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
        assert abs(slope - m) < 0.3, (m, slope, errs)


@pytest.mark.parametrize("L,m", [(8, 10), (10, 16)])
def test_plain_lanczos_window(L, m):
    """Without re-orthonormalisation (window of two vectors) the propagator is still
    accurate at these sizes and agrees with the full window to rounding."""
    rng = np.random.default_rng(L + m)
    psi = workloads.random_state(rng, 1 << L)
    a, la = krylov_prop(L, 1.0, 0.5, HC_SX, 1, 0.4, psi, 0.1, m, reorth=False)
    b, lb = krylov_prop(L, 1.0, 0.5, HC_SX, 1, 0.4, psi, 0.1, m, reorth=True)
    H = dense_h(L, 1.0, 0.5, HC_SX, 1, 0.4)
    ref = sla.expm(-0.1j * H) @ psi
    assert np.linalg.norm(a - ref) < 1e-12
    assert np.linalg.norm(a - b) < 1e-13
    assert np.abs(la.alpha - lb.alpha).max() < 1e-12
