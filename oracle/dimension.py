"""Krylov dimension for a requested accuracy (oracle; test infrastructure only).

The paper leaves the Krylov dimension to the user and points to a-posteriori
error estimates for choosing it (App. A).  The batched form of the library
chooses it per chain from an a-priori bound instead; this module restates that
choice from its definitions so that the oracle can replay a batch with the
same dimensions:

* spectral radius of H = H0 + u Hc by Gershgorin's theorem on the matrix
  elements of Sec. III.A (S = sigma/2, open chain): each of the L-1 bonds adds
  at most |J|/2 off the diagonal (the hop) and |J Delta|/4 on it; S^x on one
  site adds 1/2 off the diagonal, a sum of S^z over n sites at most n/2 on it;
* Hochbruck & Lubich, SIAM J. Numer. Anal. 34 (1997), Theorem 2: for a
  skew-Hermitian A whose eigenvalues lie on an imaginary segment of length
  4 rho, the m-dimensional Lanczos approximation of exp(A) v (unit v) errs by
  at most 12 exp(-rho^2 / m) (e rho / m)^m once m >= 2 rho;
* the choice: the smallest m in [m_min, m_max] whose bound for A = -i dt H is
  at most tol / N (N slices, so that the errors of a sweep add up to tol);
  m_max when none is.
"""

from __future__ import annotations

import math


def gershgorin_norm(L: int, J: float, Delta: float, n_control_sites: int, umax: float) -> float:
    """Upper bound on the spectral radius of H0 + u Hc over |u| <= umax."""
    return (L - 1) * abs(J) * (0.5 + abs(Delta) / 4.0) + abs(umax) * 0.5 * n_control_sites


def hochbruck_lubich(rho: float, m: int) -> float:
    """Theorem 2 bound for a spectrum on a segment of length 4 rho (inf for m < 2 rho)."""
    if m < 2.0 * rho:
        return math.inf
    return 12.0 * math.exp(-rho * rho / m) * (math.e * rho / m) ** m


def krylov_dimension(L: int, J: float, Delta: float, n_control_sites: int, umax: float,
                     dt: float, N: int, tol: float = 1e-8, m_min: int = 8,
                     m_max: int = 24) -> int:
    """Smallest m in [m_min, m_max] with the bound <= tol / N for exp(-i dt H)."""
    # the spectrum of -i dt H lies on a segment of length 2 |dt| ||H|| = 4 rho
    rho = 0.5 * abs(dt) * gershgorin_norm(L, J, Delta, n_control_sites, umax)
    for m in range(m_min, m_max + 1):
        if hochbruck_lubich(rho, m) <= tol / N:
            return m
    return m_max
