"""Lanczos basis and Krylov propagator (oracle; test infrastructure only).

App. A describes the method:
  * Algorithm 2 builds an orthonormal basis v_0..v_{m-1} of the Krylov space
    span{psi, H psi, ..., H^{m-1} psi}.  Each candidate x_j = H v_{j-1} has its
    projections on basis vectors removed; all projection coefficients are taken
    against the same candidate x_j (classical Gram-Schmidt).  Plain Lanczos
    removes only the last two vectors; the full re-orthonormalisation the
    appendix mentions removes all previous vectors.  The projection on v_{j-1}
    is the diagonal entry of the tridiagonal T, the norm b_j of the remainder is
    its off-diagonal entry.
  * Eqs. A1-A3: psi(t) ~ V^dagger exp(-i T t) V psi; V psi = ||psi|| e_1.

Readings where the paper is silent (kept identical in the GPU library):
  * the loop runs to the requested dimension m (the printed loop has no bound);
  * breakdown: stop at m_eff = j when b_j <= tol * max(1, max_{i<j}(|alpha_i| + beta_i));
  * the input is scaled by its norm beta0 (the appendix assumes unit norm);
  * the small exponential is taken by diagonalising T (the appendix speaks of
    the effective Hamiltonian being diagonalised): exp(-itT) e_1 = S exp(-i theta t) S^T e_1.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

EPS_C128 = 2.0 ** -52
EPS_C64 = 2.0 ** -23


def default_tol(vec_eps: float = EPS_C128) -> float:
    return 64.0 * vec_eps


@dataclasses.dataclass
class LanczosResult:
    V: np.ndarray        # (m_eff, D) orthonormal basis
    alpha: np.ndarray    # (m_eff,) diagonal of T
    beta: np.ndarray     # (m_eff-1,) off-diagonal of T, beta[k] couples v_k and v_{k+1}
    beta0: float         # ||psi||
    m_eff: int


def lanczos(apply_h, psi: np.ndarray, m: int, reorth: bool = True,
            tol: float | None = None) -> LanczosResult:
    """Algorithm 2 with a projection window of the last two vectors (reorth=False)
    or of all previous vectors (reorth=True)."""
    tol = default_tol() if tol is None else tol
    D = psi.shape[0]
    beta0 = float(np.linalg.norm(psi))
    V = np.zeros((m, D), dtype=np.complex128)
    alpha = np.zeros(m)
    offd = np.zeros(m)           # offd[j] couples v_{j-1} and v_j; offd[0] = 0
    if beta0 == 0.0:
        return LanczosResult(V[:0], alpha[:0], offd[:0], 0.0, 0)
    V[0] = psi / beta0
    m_eff = m
    for j in range(1, m + 1):
        x = apply_h(V[j - 1])                     # candidate x_j = H v_{j-1}
        lo = 0 if reorth else max(0, j - 2)
        h = V[lo:j].conj() @ x                    # <v_k|x_j>, all against the same x_j
        alpha[j - 1] = h[-1].real                 # diagonal entry of T
        if j == m:
            break
        w = x - h @ V[lo:j]
        b = float(np.linalg.norm(w))
        scale = max(1.0, float(np.max(np.abs(alpha[:j]) + offd[:j])))
        if b <= tol * scale:                      # happy breakdown: K is invariant
            m_eff = j
            break
        offd[j] = b
        V[j] = w / b
    return LanczosResult(V[:m_eff].copy(), alpha[:m_eff].copy(), offd[1:m_eff].copy(), beta0,
                         m_eff)


def tri_exp_e1(alpha: np.ndarray, beta: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t T) e_1 for the real symmetric tridiagonal T = tridiag(beta, alpha, beta)."""
    if alpha.shape[0] == 1:
        return np.array([np.exp(-1j * t * alpha[0])])
    theta, S = sla.eigh_tridiagonal(alpha, beta)
    return S @ (np.exp(-1j * theta * t) * S[0, :])


def expv(apply_h, psi: np.ndarray, t: float, m: int, reorth: bool = True,
         tol: float | None = None, return_info: bool = False):
    """exp(-i t H) psi ~ ||psi|| V^T exp(-i t T) e_1  (Eqs. A1-A3)."""
    lz = lanczos(apply_h, psi, m, reorth=reorth, tol=tol)
    if lz.m_eff == 0:
        out = np.zeros_like(psi)
    else:
        c = tri_exp_e1(lz.alpha, lz.beta, t)
        out = lz.beta0 * (c @ lz.V)
    if return_info:
        return out, lz
    return out
