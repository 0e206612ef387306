"""Pins of the oracle's GRAPE sweeps and gradients (CPU only).

The zeroth-order gradient of Eq. 5 is an approximation of the exact
piecewise-constant gradient (Eqs. B3-B5), so it is pinned three ways:
  * where it is exact (the control commutes with every slice Hamiltonian) it must
    equal the exact gradient, which is itself pinned against finite differences;
  * elsewhere its error against the exact gradient must shrink as dt^2;
  * a small step along it must raise the fidelity (sign).
The exact gradient is pinned by two independent derivative formulas and by
central finite differences of dense propagation.
"""

import numpy as np
import pytest

import workloads
from oracle import exact, grape, model
from oracle.model import HC_SX, HC_SZ


def dense_parts(L, J, Delta, kind, sites):
    return model.xxz_dense(L, J, Delta), model.hc_dense(L, kind, sites)


def chain_of(L, J, Delta, kind, sites):
    return model.Chain(L, J, Delta, kind, sites)


def test_small_workload_fidelity_matches_dense():
    c = workloads.small()
    ch = chain_of(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    r = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m)
    H0, Hc = dense_parts(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    Fd = exact.dense_fidelity(H0, Hc, c.u, c.psi0, c.target, c.dt)
    assert abs(r.F - Fd) < 1e-12
    assert abs(np.linalg.norm(r.psi_N) - 1.0) < 1e-12
    assert np.all(r.m_eff_fwd == c.m)


@pytest.mark.parametrize("L,N,dt", [(4, 5, 0.3), (5, 4, 0.7)])
def test_exact_derivative_two_formulas_and_fd(L, N, dt):
    rng = np.random.default_rng(L)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    for uj in u[:2]:
        H = H0 + uj * Hc
        assert np.abs(exact.dU_daleckii_krein(H, Hc, dt) - exact.dU_van_loan(H, Hc, dt)).max() < 1e-13
    F1, g1 = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt, method="dk")
    F2, g2 = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt, method="vanloan")
    assert np.abs(g1 - g2).max() < 1e-13
    fd = exact.fd_gradient(lambda uu: exact.dense_fidelity(H0, Hc, uu, psi0, f, dt), u,
                           range(N), h=1e-5)
    fdv = np.array([fd[j] for j in range(N)])
    assert np.abs(fdv - g1).max() < 1e-9 * max(1.0, np.abs(g1).max() * 1e3)
    assert np.abs(fdv - g1).max() / np.abs(g1).max() < 1e-7


def test_quadrature_exact_gradient_matches_dense():
    L, N, dt, m = 6, 6, 0.2, 20
    rng = np.random.default_rng(9)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    _, gd = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    _, gq = exact.exact_gradient_quadrature(ch, u, psi0, f, dt, m, slices=[0, 3, 5])
    for j in [0, 3, 5]:
        assert abs(gq[j] - gd[j]) < 1e-12


@pytest.mark.parametrize("case", ["no_drift", "total_sz"])
def test_zeroth_order_is_exact_when_control_commutes(case):
    """If [Hc, H_j] = 0 the time-averaged control operator (Eq. B6) is Hc itself,
    so the zeroth-order gradient equals the exact one."""
    L, N, dt = 5, 6, 0.4
    rng = np.random.default_rng(21)
    if case == "no_drift":
        J, kind, sites = 0.0, HC_SX, 1 << 2
    else:
        J, kind, sites = 1.0, HC_SZ, (1 << L) - 1
    H0, Hc = dense_parts(L, J, 0.5, kind, sites)
    assert np.abs(H0 @ Hc - Hc @ H0).max() < 1e-14
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    _, g_exact = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
    r = grape.gradient(chain_of(L, J, 0.5, kind, sites), u, psi0, f, dt, m=24)
    assert np.abs(r.grad - g_exact).max() < 1e-12 * max(1.0, np.abs(g_exact).max())
    assert np.abs(g_exact).max() > 1e-3   # the check is not vacuous


def test_zeroth_order_error_is_second_order_in_dt():
    """Error of Eq. 5 against the exact gradient falls ~4x per halving of dt.

    The control is one fixed smooth function of time sampled at slice midpoints on
    a fixed horizon T, so refining dt refines the same control problem."""
    L, T = 6, 0.8
    rng = np.random.default_rng(4)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    errs = []
    for dt in [0.1, 0.05, 0.025]:
        N = int(round(T / dt))
        t_mid = (np.arange(N) + 0.5) * dt
        u = np.sin(2.0 * t_mid) + 0.5 * np.cos(5.0 * t_mid)
        _, ge = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
        r = grape.gradient(ch, u, psi0, f, dt, m=24)
        errs.append(np.abs(r.grad - ge).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.5 < q < 4.5 for q in ratios), (errs, ratios)


def test_centred_error_is_third_order_in_dt():
    """The centred variant (App. B) falls ~8x per halving of dt on the same fixed-
    horizon problem on which Eq. 5 falls ~4x, and it is the more accurate of the two."""
    L, T = 6, 0.8
    rng = np.random.default_rng(4)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    errs, errs0 = [], []
    for dt in [0.1, 0.05, 0.025]:
        N = int(round(T / dt))
        t_mid = (np.arange(N) + 0.5) * dt
        u = np.sin(2.0 * t_mid) + 0.5 * np.cos(5.0 * t_mid)
        _, ge = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
        rc = grape.gradient_centred(ch, u, psi0, f, dt, m=24)
        r0 = grape.gradient(ch, u, psi0, f, dt, m=24)
        errs.append(np.abs(rc.grad - ge).max())
        errs0.append(np.abs(r0.grad - ge).max())
        assert abs(rc.F - r0.F) < 1e-14
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(7.0 < q < 9.0 for q in ratios), (errs, ratios)
    assert all(e < e0 / 5 for e, e0 in zip(errs, errs0)), (errs, errs0)


@pytest.mark.parametrize("case", ["no_drift", "conserved_sz"])
def test_centred_is_exact_when_control_commutes(case):
    """With [Hc, H_j] = 0 the bracket is the same at both ends of a slice, so the
    centred gradient, like Eq. 5, equals the exact one."""
    L, N, dt = 5, 6, 0.4
    rng = np.random.default_rng(22)
    if case == "no_drift":
        J, kind, sites = 0.0, HC_SX, 1 << 1
    else:
        J, kind, sites = 1.0, HC_SZ, (1 << L) - 1
    H0, Hc = dense_parts(L, J, 0.5, kind, sites)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    _, g_exact = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
    r = grape.gradient_centred(chain_of(L, J, 0.5, kind, sites), u, psi0, f, dt, m=24)
    assert np.abs(r.grad - g_exact).max() < 1e-12 * max(1.0, np.abs(g_exact).max())
    assert np.abs(g_exact).max() > 1e-3


def test_centred_single_slice_is_trapezoid_of_exact_integrand():
    """N = 1: the exact derivative is -i int_0^dt <e^{iH(dt-s)} f|Hc|e^{-iHs} psi0> ds
    (App. B, natural gradient); the centred value is the trapezoid rule of that
    integrand (end points s = 0 and s = dt), computed here from dense propagators."""
    L, dt = 5, 0.3
    rng = np.random.default_rng(23)
    H0, Hc = dense_parts(L, 1.0, 0.7, HC_SX, 1)
    u = np.array([0.4])
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    H = H0 + u[0] * Hc
    U = exact.propagator(H, dt)
    beta = np.vdot(f, U @ psi0)
    def integrand(s):
        a = exact.propagator(H, -(dt - s)) @ f      # e^{+iH(dt-s)} f
        b = exact.propagator(H, s) @ psi0          # e^{-iHs} psi0
        return 2.0 * (np.conj(beta) * (-1j) * np.vdot(a, Hc @ b)).real
    trap = 0.5 * dt * (integrand(0.0) + integrand(dt))
    r = grape.gradient_centred(chain_of(L, 1.0, 0.7, HC_SX, 1), u, psi0, f, dt, m=24)
    assert abs(r.grad[0] - trap) < 1e-12


def test_hierarchy_converges_to_exact_gradient():
    """The Taylor hierarchy of the time-averaged control operator (App. B) summed to
    high order reproduces the exact piecewise-constant gradient (Daleckii-Krein);
    order 0 is the zeroth-order gradient of Eq. 5."""
    L, N, dt = 5, 5, 0.25
    rng = np.random.default_rng(31)
    H0, Hc = dense_parts(L, 1.0, 0.6, HC_SX, 1 << 1)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    ch = chain_of(L, 1.0, 0.6, HC_SX, 1 << 1)
    _, ge = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
    r16 = grape.gradient_hierarchy(ch, u, psi0, f, dt, 24, P=16)
    assert np.abs(r16.grad - ge).max() < 1e-12 * max(1.0, np.abs(ge).max())
    r0 = grape.gradient_hierarchy(ch, u, psi0, f, dt, 24, P=0)
    g0 = grape.gradient(ch, u, psi0, f, dt, 24).grad
    assert np.abs(r0.grad - g0).max() < 1e-15


def test_first_order_hierarchy_error_is_third_order_in_dt():
    """Truncating after the first commutator leaves an O(dt^3) error per slice:
    ~8x per halving of dt on the fixed-horizon problem."""
    L, T = 6, 0.8
    rng = np.random.default_rng(4)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    errs = []
    for dt in [0.1, 0.05, 0.025]:
        N = int(round(T / dt))
        t_mid = (np.arange(N) + 0.5) * dt
        u = np.sin(2.0 * t_mid) + 0.5 * np.cos(5.0 * t_mid)
        _, ge = exact.exact_gradient_dense(H0, Hc, u, psi0, f, dt)
        r = grape.gradient_hierarchy(ch, u, psi0, f, dt, 24, P=1)
        errs.append(np.abs(r.grad - ge).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(7.0 < q < 9.0 for q in ratios), (errs, ratios)


def test_gradient_ascent_direction_raises_fidelity():
    c = workloads.small()
    ch = chain_of(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    r = grape.gradient(ch, c.u, c.psi0, c.target, c.dt, c.m)
    u2 = grape.ascent_update(c.u, r.grad, 0.05)
    F2 = grape.fidelity(ch, u2, c.psi0, c.target, c.dt, c.m)
    assert F2 > r.F
    # first-order prediction of the change, with the exact gradient within O(dt)
    H0, Hc = dense_parts(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    _, ge = exact.exact_gradient_dense(H0, Hc, c.u, c.psi0, c.target, c.dt)
    assert np.linalg.norm(r.grad - ge) / np.linalg.norm(ge) < 0.1


def test_costate_is_backward_propagated_target():
    """lambda_j = U_{j+1}^dag ... U_N^dag f, checked through <lambda_0|psi_0> = beta."""
    L, N, dt = 6, 7, 0.15
    rng = np.random.default_rng(8)
    u = rng.uniform(-1, 1, N)
    psi0 = workloads.random_state(rng, 1 << L)
    f = workloads.random_state(rng, 1 << L)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    from oracle import krylov
    lam = f.copy()
    for j in range(N, 0, -1):
        lam = krylov.expv(lambda v, uj=u[j - 1]: ch.apply(uj, v), lam, -dt, 24)
    r = grape.gradient(ch, u, psi0, f, dt, m=24)
    assert abs(np.vdot(lam, psi0) - r.beta) < 1e-12


def test_ascent_update():
    u = np.array([0.5, -0.25, 0.0])
    g = np.array([0.1, -0.4, 0.2])
    assert np.allclose(grape.ascent_update(u, g, 0.1), u + 0.1 * g / 0.4)
    assert np.array_equal(grape.ascent_update(u, np.zeros(3), 0.1), u)


# ---- operator control on a block of columns


def random_columns(rng, n, D):
    return np.array([workloads.random_state(rng, D) for _ in range(n)])


@pytest.mark.parametrize("centred", [False, True])
def test_columns_single_column_is_state_transfer(centred):
    c = workloads.small()
    ch = chain_of(c.L, c.J, c.Delta, c.hc_kind, c.hc_sites)
    u = c.u[:12]
    rc = grape.gradient_columns(ch, u, c.psi0[None], c.target[None], c.dt, c.m, centred=centred)
    fn = grape.gradient_centred if centred else grape.gradient
    r = fn(ch, u, c.psi0, c.target, c.dt, c.m)
    assert abs(rc.F - r.F) < 1e-15 and np.abs(rc.grad - r.grad).max() < 1e-15


@pytest.mark.parametrize("centred", [False, True])
def test_columns_exact_when_control_commutes(centred):
    """Total S^z commutes with the XXZ drift: the bracket sums are constant inside
    each slice and the column gradient equals the dense exact derivative of
    |Tr(W^dag U Psi0)/n|^2."""
    L, N, dt, n = 5, 6, 0.4, 3
    rng = np.random.default_rng(31)
    sites = (1 << L) - 1
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SZ, sites)
    u = rng.uniform(-1, 1, N)
    P0, W = random_columns(rng, n, 1 << L), random_columns(rng, n, 1 << L)
    F_exact, g_exact = exact.exact_operator_gradient_dense(H0, Hc, u, P0, W, dt)
    r = grape.gradient_columns(chain_of(L, 1.0, 0.5, HC_SZ, sites), u, P0, W, dt, m=24,
                               centred=centred)
    assert abs(r.F - F_exact) < 1e-13
    assert np.abs(r.grad - g_exact).max() < 1e-12 * max(1.0, np.abs(g_exact).max())
    assert np.abs(g_exact).max() > 1e-3


def test_columns_error_orders_in_dt():
    """Non-commuting control: at a fixed horizon the zeroth-order column gradient's
    error against the dense exact one falls ~4x per halving of dt and the centred
    one's ~8x, as for a single state."""
    L, T, n = 5, 0.8, 3
    rng = np.random.default_rng(32)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1)
    P0, W = random_columns(rng, n, 1 << L), random_columns(rng, n, 1 << L)
    ch = chain_of(L, 1.0, 0.5, HC_SX, 1)
    e0, ec = [], []
    for dt in [0.1, 0.05, 0.025]:
        N = int(round(T / dt))
        t_mid = (np.arange(N) + 0.5) * dt
        u = np.sin(2.0 * t_mid) + 0.5 * np.cos(5.0 * t_mid)
        _, ge = exact.exact_operator_gradient_dense(H0, Hc, u, P0, W, dt)
        e0.append(np.abs(grape.gradient_columns(ch, u, P0, W, dt, m=24).grad - ge).max())
        ec.append(np.abs(grape.gradient_columns(ch, u, P0, W, dt, m=24, centred=True).grad
                         - ge).max())
    r0 = [e0[0] / e0[1], e0[1] / e0[2]]
    rc = [ec[0] / ec[1], ec[1] / ec[2]]
    assert all(3.5 < q < 4.5 for q in r0), (e0, r0)
    assert all(7.0 < q < 9.0 for q in rc), (ec, rc)


def test_whole_basis_gate_at_its_own_propagator():
    """All 2^L columns (Psi0 = identity) with the target W = e^{i phi} U(T) of the
    same controls: F = 1 (phase-insensitive, m = D makes the Krylov step exact) and
    the gradient vanishes (a maximum)."""
    L, N, dt = 4, 5, 0.3
    D = 1 << L
    rng = np.random.default_rng(33)
    H0, Hc = dense_parts(L, 1.0, 0.5, HC_SX, 1 << 2)
    u = rng.uniform(-1, 1, N)
    U = np.eye(D, dtype=np.complex128)
    for uj in u:
        U = exact.propagator(H0 + uj * Hc, dt) @ U
    W = np.exp(0.7j) * U
    r = grape.gradient_columns(chain_of(L, 1.0, 0.5, HC_SX, 1 << 2), u, np.eye(D), W.T, dt, m=D)
    assert abs(r.F - 1.0) < 1e-12
    assert np.abs(r.grad).max() < 1e-12
