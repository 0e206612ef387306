"""Plain definitions that K-GRAPE approximates (oracle; test infrastructure only).

* Dense sub-propagators U_j = exp(-i H_j dt) by the spectral theorem (Eqs. B2, B12-B13).
* Exact piecewise-constant gradient (Eqs. B3-B5):
      dbeta/du_j = <lambda_j| dU_j/du_j |psi_{j-1}>,   dF/du_j = 2 Re(conj(beta) dbeta/du_j),
  with dU_j/du_j computed two independent ways:
      Daleckii-Krein:  Q [(Q^dag Hc Q) o Phi] Q^dag,
                       Phi_kl = (e^{-i l_k dt} - e^{-i l_l dt}) / (l_k - l_l), or -i dt e^{-i l_k dt} on ties
                       (the exact-derivative formula Eq. B14 is printed garbled; this is its
                       standard divided-difference form);
      Van Loan:        upper-right block of expm(-i dt [[H_j, Hc], [0, H_j]]).
* For sizes with no dense matrix: Gauss-Legendre quadrature of the natural gradient over
  each slice (Eqs. B6-B8):
      dbeta/du_j = -i int_0^dt <exp(+i H_j (dt-s)) lambda_j| Hc |exp(-i H_j s) psi_{j-1}> ds,
  with the node states from the oracle's Krylov propagator.
* Central finite differences of any fidelity function.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import krylov


def propagator(H: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t H) for Hermitian H by diagonalisation."""
    lam, Q = np.linalg.eigh(H)
    return (Q * np.exp(-1j * lam * t)) @ Q.conj().T


def dense_forward(H0, Hc, u, psi0, dt):
    states = [np.asarray(psi0, dtype=np.complex128)]
    for uj in u:
        states.append(propagator(H0 + uj * Hc, dt) @ states[-1])
    return states


def dense_fidelity(H0, Hc, u, psi0, target, dt) -> float:
    return abs(np.vdot(target, dense_forward(H0, Hc, u, psi0, dt)[-1])) ** 2


def dU_daleckii_krein(H: np.ndarray, Hc: np.ndarray, dt: float) -> np.ndarray:
    """Frechet derivative of exp(-i dt H) in the direction Hc, by divided differences."""
    lam, Q = np.linalg.eigh(H)
    e = np.exp(-1j * lam * dt)
    dl = lam[:, None] - lam[None, :]
    de = e[:, None] - e[None, :]
    ties = np.abs(dl) <= 1e-10 * max(1.0, float(np.max(np.abs(lam))))
    phi = np.where(ties, -1j * dt * e[:, None] * np.ones_like(dl), de / np.where(ties, 1.0, dl))
    Hct = Q.conj().T @ Hc @ Q
    return Q @ (Hct * phi) @ Q.conj().T


def dU_van_loan(H: np.ndarray, Hc: np.ndarray, dt: float) -> np.ndarray:
    """Same derivative from the block-triangular exponential."""
    D = H.shape[0]
    M = np.zeros((2 * D, 2 * D), dtype=np.complex128)
    M[:D, :D] = H
    M[D:, D:] = H
    M[:D, D:] = Hc
    E = sla.expm(-1j * dt * M)
    return E[:D, D:]


def exact_gradient_dense(H0, Hc, u, psi0, target, dt, method="dk"):
    """dF/du_j of the exact piecewise-constant propagation."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    states = dense_forward(H0, Hc, u, psi0, dt)
    beta = np.vdot(target, states[N])
    lam = np.asarray(target, dtype=np.complex128)
    g = np.zeros(N)
    for j in range(N, 0, -1):
        H = H0 + u[j - 1] * Hc
        dU = dU_daleckii_krein(H, Hc, dt) if method == "dk" else dU_van_loan(H, Hc, dt)
        dbeta = np.vdot(lam, dU @ states[j - 1])
        g[j - 1] = 2.0 * (np.conj(beta) * dbeta).real
        lam = propagator(H, dt).conj().T @ lam
    return abs(beta) ** 2, g


def exact_operator_gradient_dense(H0, Hc, u, psi0s, targets, dt):
    """F = |(1/n) Tr(W^dag U(T) Psi0)|^2 for the columns psi0s (n, D) and targets
    (n, D), and dF/du_j = 2 Re(conj(beta) dbeta/du_j) with the exact derivative
    of U_j (Daleckii-Krein), from dense propagators."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    P0 = np.asarray(psi0s, dtype=np.complex128).T          # D x n
    W = np.asarray(targets, dtype=np.complex128).T
    n = P0.shape[1]
    Us = [propagator(H0 + uj * Hc, dt) for uj in u]
    fwd = [P0]
    for U in Us:
        fwd.append(U @ fwd[-1])
    beta = np.trace(W.conj().T @ fwd[N]) / n
    g = np.zeros(N)
    lam = W
    for j in range(N, 0, -1):
        dU = dU_daleckii_krein(H0 + u[j - 1] * Hc, Hc, dt)
        dbeta = np.trace(lam.conj().T @ dU @ fwd[j - 1]) / n
        g[j - 1] = 2.0 * (np.conj(beta) * dbeta).real
        lam = Us[j - 1].conj().T @ lam
    return abs(beta) ** 2, g


def exact_gradient_quadrature(chain, u, psi0, target, dt, m, slices=None, nodes=8,
                              reorth=True):
    """dF/du_j for selected slices by Gauss-Legendre quadrature inside the slice.

    Forward states and costates come from the oracle's Krylov propagator (store-all);
    each node state is one further Krylov propagation over a partial step."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[0]
    slices = range(N) if slices is None else slices
    states = [np.asarray(psi0, dtype=np.complex128)]
    for uj in u:
        states.append(krylov.expv(lambda v, uj=uj: chain.apply(uj, v), states[-1], dt, m,
                                  reorth))
    beta = np.vdot(target, states[N])
    lams = {N: np.asarray(target, dtype=np.complex128)}
    lam = lams[N]
    for j in range(N, 1, -1):
        lam = krylov.expv(lambda v, uj=u[j - 1]: chain.apply(uj, v), lam, -dt, m, reorth)
        lams[j - 1] = lam
    x, w = np.polynomial.legendre.leggauss(nodes)
    svals = 0.5 * dt * (x + 1.0)
    wts = 0.5 * dt * w
    g = {}
    for jj in slices:
        j = jj + 1
        hj = (lambda v, uj=u[j - 1]: chain.apply(uj, v))
        acc = 0.0 + 0.0j
        for s, ws in zip(svals, wts):
            a = krylov.expv(hj, states[j - 1], s, m, reorth)          # e^{-iHs} psi_{j-1}
            b = krylov.expv(hj, lams[j], -(dt - s), m, reorth)        # e^{+iH(dt-s)} lambda_j
            acc += ws * np.vdot(b, chain.apply_hc(a))
        dbeta = -1j * acc
        g[jj] = 2.0 * (np.conj(beta) * dbeta).real
    return abs(beta) ** 2, g


def fd_gradient(fidelity_fn, u, slices, h=1e-5):
    """Central differences (F(u + h e_j) - F(u - h e_j)) / 2h."""
    u = np.asarray(u, dtype=np.float64)
    out = {}
    for j in slices:
        up = u.copy()
        up[j] += h
        um = u.copy()
        um[j] -= h
        out[j] = (fidelity_fn(up) - fidelity_fn(um)) / (2.0 * h)
    return out
