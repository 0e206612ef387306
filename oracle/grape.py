"""GRAPE sweeps with Krylov propagation (oracle; test infrastructure only).

Algorithm 1 with the propagators of Eq. B2 replaced by the Krylov propagator:
  forward   psi_0 = |i>,  psi_j = exp(-i H_j dt) psi_{j-1},  H_j = H0 + u_j Hc  (Eqs. 1, 4, B1, B2)
  overlap   beta = <f|psi_N>,  F = |beta|^2 = 1 - I                          (Eq. 2)
  backward  lambda_N = |f>,  lambda_{j-1} = exp(+i H_j dt) lambda_j
            (the paper's chi_j equals beta * lambda_j)
  gradient  dI/du_j ~ -2 dt Im<chi_j|Hc|psi_j>                                (Eq. 5)
            so dF/du_j = +2 dt Im(conj(beta) <lambda_j|Hc|psi_j>)
  ascent    u <- u + eta * g / max_j |g_j|  (plain steepest ascent; the paper's
            L-BFGS update of Algorithm 1 is not part of the hot path)
Slices are numbered j = 1..N in the paper and 0..N-1 in arrays here.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import krylov
from .model import Chain


@dataclasses.dataclass
class GradResult:
    F: float
    beta: complex
    grad: np.ndarray          # (N,) dF/du_j
    psi_N: np.ndarray
    m_eff_fwd: np.ndarray     # (N,) Krylov dimension reached per forward slice
    m_eff_bwd: np.ndarray     # (N,) per backward slice (entry 0 unused: no propagation at j=1)


def forward(chain: Chain, u, psi0, dt, m, reorth=True, tol=None, keep=True):
    """psi_0..psi_N (list) if ``keep`` else just psi_N, plus the m_eff per slice."""
    psi = np.asarray(psi0, dtype=np.complex128)
    states = [psi] if keep else None
    m_eff = np.zeros(len(u), dtype=np.int64)
    for j, uj in enumerate(u):
        psi, lz = krylov.expv(lambda v, uj=uj: chain.apply(uj, v), psi, dt, m, reorth, tol,
                              return_info=True)
        m_eff[j] = lz.m_eff
        if keep:
            states.append(psi)
    return (states if keep else psi), m_eff


def overlap(target, psi_N) -> complex:
    return complex(np.vdot(target, psi_N))


def fidelity(chain: Chain, u, psi0, target, dt, m, reorth=True, tol=None) -> float:
    psi_N, _ = forward(chain, u, psi0, dt, m, reorth, tol, keep=False)
    return abs(overlap(target, psi_N)) ** 2


def gradient(chain: Chain, u, psi0, target, dt, m, reorth=True, tol=None) -> GradResult:
    """Fidelity and zeroth-order gradient, store-all forward then one backward sweep."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    states, m_fwd = forward(chain, u, psi0, dt, m, reorth, tol, keep=True)
    beta = overlap(target, states[N])
    lam = np.asarray(target, dtype=np.complex128)
    g = np.zeros(N)
    m_bwd = np.zeros(N, dtype=np.int64)
    for j in range(N, 0, -1):                     # paper's slice index
        bracket = np.vdot(lam, chain.apply_hc(states[j]))
        g[j - 1] = 2.0 * dt * (np.conj(beta) * bracket).imag
        if j > 1:
            lam, lz = krylov.expv(lambda v, uj=u[j - 1]: chain.apply(uj, v), lam, -dt, m,
                                  reorth, tol, return_info=True)
            m_bwd[j - 1] = lz.m_eff
    return GradResult(F=abs(beta) ** 2, beta=beta, grad=g, psi_N=states[N], m_eff_fwd=m_fwd,
                      m_eff_bwd=m_bwd)


def gradient_centred(chain: Chain, u, psi0, target, dt, m, reorth=True, tol=None) -> GradResult:
    """Centred zeroth-order gradient (App. B, the centred variant of Eq. 5).

    The natural gradient is still taken constant over slice j, but evaluated at
    the slice centre, approximated by the mean of the Eq. 5 bracket at the two
    ends of the slice:
        G_j = 2 dt Im(conj(beta) <lambda_j|Hc|psi_j>),  j = 0..N,
        dF/du_j ~ (G_{j-1} + G_j) / 2,
    with lambda_0 = U_1^dagger lambda_1 (one backward propagation more than the
    plain gradient).  The paper states an error of O(dt^3) per slice instead of
    O(dt^2)."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    states, m_fwd = forward(chain, u, psi0, dt, m, reorth, tol, keep=True)
    beta = overlap(target, states[N])
    lam = np.asarray(target, dtype=np.complex128)
    G = np.zeros(N + 1)
    m_bwd = np.zeros(N, dtype=np.int64)
    for j in range(N, -1, -1):                    # paper's slice index, and j = 0
        bracket = np.vdot(lam, chain.apply_hc(states[j]))
        G[j] = 2.0 * dt * (np.conj(beta) * bracket).imag
        if j >= 1:
            lam, lz = krylov.expv(lambda v, uj=u[j - 1]: chain.apply(uj, v), lam, -dt, m,
                                  reorth, tol, return_info=True)
            m_bwd[j - 1] = lz.m_eff
    g = 0.5 * (G[:-1] + G[1:])
    return GradResult(F=abs(beta) ** 2, beta=beta, grad=g, psi_N=states[N], m_eff_fwd=m_fwd,
                      m_eff_bwd=m_bwd)


def gradient_hierarchy(chain: Chain, u, psi0, target, dt, m, P, reorth=True,
                       tol=None) -> GradResult:
    """Gradient from the truncated Taylor hierarchy of the time-averaged control
    operator (App. B): Hc_bar^[P] = sum_{p=0}^{P} (-i dt)^p / (p+1)! L^p Hc with the
    Liouvillian L = [H_j, .], and dF/du_j ~ 2 dt Im(conj(beta) <lambda_j|Hc_bar^[P]|psi_j>).
    P = 0 is Eq. 5.  Matrix-free: <lambda|L^p Hc|psi> = sum_k C(p,k) (-1)^k
    <H^(p-k) lambda| Hc |H^k psi> for Hermitian H."""
    from math import comb, factorial
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    states, m_fwd = forward(chain, u, psi0, dt, m, reorth, tol, keep=True)
    beta = overlap(target, states[N])
    lam = np.asarray(target, dtype=np.complex128)
    g = np.zeros(N)
    m_bwd = np.zeros(N, dtype=np.int64)
    for j in range(N, 0, -1):
        uj = u[j - 1]
        hp = [states[j]]                 # H^k psi_j
        hl = [lam]                       # H^k lambda_j
        for _ in range(P):
            hp.append(chain.apply(uj, hp[-1]))
            hl.append(chain.apply(uj, hl[-1]))
        val = 0.0 + 0.0j
        for p in range(P + 1):
            lp = sum(comb(p, k) * (-1) ** k * np.vdot(hl[p - k], chain.apply_hc(hp[k]))
                     for k in range(p + 1))
            val += (-1j * dt) ** p / factorial(p + 1) * lp
        g[j - 1] = 2.0 * dt * (np.conj(beta) * val).imag
        if j > 1:
            lam, lz = krylov.expv(lambda v, uj=uj: chain.apply(uj, v), lam, -dt, m, reorth, tol,
                                  return_info=True)
            m_bwd[j - 1] = lz.m_eff
    return GradResult(F=abs(beta) ** 2, beta=beta, grad=g, psi_N=states[N], m_eff_fwd=m_fwd,
                      m_eff_bwd=m_bwd)


def gradient_columns(chain: Chain, u, psi0s, targets, dt, m, reorth=True, tol=None,
                     centred=False) -> GradResult:
    """Operator control on a block of n columns (the generalisation named in the
    conclusions): the phase-insensitive subspace gate fidelity
        F = |beta|^2,  beta = (1/n) sum_c <w_c| U(T) |psi_c>,
    which is |Tr(W^dag U)/D|^2 when the columns are a whole basis.  Its
    zeroth-order gradient is Eq. 5 with the brackets of all columns summed:
        dF/du_j ~ 2 dt Im(conj(beta) (1/n) sum_c <lambda_{c,j}|Hc|psi_{c,j}>),
    lambda_{c,N} = w_c propagated backward per column; `centred` averages the
    bracket sums at the two ends of each slice as in gradient_centred.
    psi0s, targets: arrays of shape (n, D)."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    psi0s = np.atleast_2d(np.asarray(psi0s, dtype=np.complex128))
    targets = np.atleast_2d(np.asarray(targets, dtype=np.complex128))
    n = psi0s.shape[0]
    cols = [forward(chain, u, psi0s[c], dt, m, reorth, tol, keep=True)[0] for c in range(n)]
    beta = sum(overlap(targets[c], cols[c][N]) for c in range(n)) / n
    G = np.zeros(N + 1, dtype=np.complex128)        # (1/n) sum_c <lambda_c|Hc|psi_c> at j
    for c in range(n):
        lam = targets[c].copy()
        for j in range(N, -1 if centred else 0, -1):
            G[j] += np.vdot(lam, chain.apply_hc(cols[c][j])) / n
            if j >= (1 if centred else 2):
                lam = krylov.expv(lambda v, uj=u[j - 1]: chain.apply(uj, v), lam, -dt, m,
                                  reorth, tol)
    g_end = 2.0 * dt * (np.conj(beta) * G).imag
    g = 0.5 * (g_end[:-1] + g_end[1:]) if centred else g_end[1:]
    return GradResult(F=abs(beta) ** 2, beta=beta, grad=g, psi_N=np.array([s[N] for s in cols]),
                      m_eff_fwd=np.zeros(N, dtype=np.int64), m_eff_bwd=np.zeros(N, dtype=np.int64))


def ascent_update(u, g, eta):
    """u + eta * g / max|g| (no change when the gradient vanishes)."""
    gmax = float(np.max(np.abs(g)))
    if gmax == 0.0:
        return np.array(u, dtype=np.float64)
    return np.asarray(u, dtype=np.float64) + eta * np.asarray(g) / gmax
