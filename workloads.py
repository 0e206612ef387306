"""Seeded synthetic inputs for the K-GRAPE workloads.

This module only draws numbers: control amplitudes, random-phase states and
computational-basis states, plus the fixed parameters of each workload.  It
holds none of the method's arithmetic, so both the CPU oracle and the GPU path
can take their inputs from it without sharing any computation.

Conventions (paper Sec. III.A, ordering of the computational basis): spin up
is bit 0 and spin down is bit 1; reading a ket left to right gives a binary
number with site 1 as the most significant bit, so the index of a product
state is ``s = sum_i b_i 2**(L-i)``.

Workloads (all open XXZ chains, J = 1, control operator S^x on site 1):

* ``small``   L=8,  D=256,        N=50,  dt=0.1,  m=10, complex128
* ``ascent``  L=16, D=65,536,     N=200, dt=0.05, m=16, complex128, 20 ascent steps
* ``adjoint`` L=20, D=1,048,576,  N=400, dt=0.05, m=20, complex64 + FP64 scalars
* ``batched`` 64 chains, L in 10..16, N in 50..300, dt=0.05, complex64
* ``large``   L=24, D=16,777,216, N=500, dt=0.05, m=24, complex64 and complex128
* ``pe_task`` the transfer task of Sec. III.A in the fixed-excitation, even-parity
  basis (J=2, Delta=0.5, S^z control on sites 1 and L, dt=0.5, m=10);
  ``pe_large`` is L=25, K=12, N=200, dt=0.1

Random draws use ``numpy.random.default_rng(seed)``: first the controls, then
the phases of psi0, then the phases of the target, each phase vector
``U(0, 2*pi)**D`` giving the state ``exp(i*theta)/sqrt(D)``.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

HC_SX = 0
HC_SZ = 1


@dataclasses.dataclass(frozen=True)
class Chain:
    """One open XXZ chain and its control problem."""

    L: int
    J: float
    Delta: float
    hc_kind: int          # HC_SX or HC_SZ
    hc_sites: int         # bit (i-1) set <=> site i carries the control operator
    N: int                # number of piecewise-constant slices
    dt: float
    m: int                # Krylov dimension
    u: np.ndarray         # (N,) float64 control amplitudes
    psi0: np.ndarray      # (2**L,) complex128, unit norm
    target: np.ndarray    # (2**L,) complex128, unit norm

    @property
    def D(self) -> int:
        return 1 << self.L


def basis_index(spins: str) -> int:
    """Index of a product state written as a string of 'u'/'d' (site 1 first)."""
    s = 0
    for ch in spins:
        s = (s << 1) | (1 if ch == "d" else 0)
    return s


def basis_state(L: int, index: int) -> np.ndarray:
    v = np.zeros(1 << L, dtype=np.complex128)
    v[index] = 1.0
    return v


def random_phase_state(rng: np.random.Generator, D: int) -> np.ndarray:
    theta = rng.uniform(0.0, 2.0 * np.pi, D)
    return np.exp(1j * theta) / np.sqrt(D)


def random_state(rng: np.random.Generator, D: int) -> np.ndarray:
    """Gaussian complex vector scaled to unit norm (used by unit tests)."""
    v = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return v / np.linalg.norm(v)


def small(seed: int = 0) -> Chain:
    """L=8 chain, one up spin at site 1 moved to site 8 (product states)."""
    L = 8
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, 50)
    return Chain(L=L, J=1.0, Delta=0.5, hc_kind=HC_SX, hc_sites=1, N=50, dt=0.1, m=10, u=u,
                 psi0=basis_state(L, basis_index("u" + "d" * 7)),
                 target=basis_state(L, basis_index("d" * 7 + "u")))


def _random_chain(seed: int, L: int, Delta: float, N: int, dt: float, m: int,
                  urange: float) -> Chain:
    rng = np.random.default_rng(seed)
    D = 1 << L
    u = rng.uniform(-urange, urange, N)
    psi0 = random_phase_state(rng, D)
    target = random_phase_state(rng, D)
    return Chain(L=L, J=1.0, Delta=Delta, hc_kind=HC_SX, hc_sites=1, N=N, dt=dt, m=m, u=u,
                 psi0=psi0, target=target)


def ascent(seed: int = 1) -> Chain:
    """L=16 chain with random-phase states, controls U(-2,2)."""
    return _random_chain(seed, L=16, Delta=0.5, N=200, dt=0.05, m=16, urange=2.0)


ASCENT_STEPS = 20
ASCENT_ETA = 0.1


def adjoint(seed: int = 2, N: Optional[int] = None) -> Chain:
    """L=20 chain with random-phase states, controls U(-1,1).

    ``N`` truncates the slice count (same draws for the first N controls are
    not guaranteed; a truncated chain is a separate seeded instance)."""
    return _random_chain(seed, L=20, Delta=1.0, N=400 if N is None else N, dt=0.05, m=20,
                         urange=1.0)


def adjoint_fd_slices(seed: int = 2) -> np.ndarray:
    """The 8 slices (0-based) checked by finite differences for the L=20 chain."""
    rng = np.random.default_rng(seed)
    rng.uniform(-1.0, 1.0, 400)
    D = 1 << 20
    rng.uniform(0.0, 2.0 * np.pi, D)
    rng.uniform(0.0, 2.0 * np.pi, D)
    return np.sort(rng.choice(400, 8, replace=False))


def large(seed: int = 4, N: Optional[int] = None) -> Chain:
    """L=24 chain with random-phase states, controls U(-1,1), N=500."""
    return _random_chain(seed, L=24, Delta=0.5, N=500 if N is None else N, dt=0.05, m=24,
                         urange=1.0)


LARGE_CKPT_EVERY = 22
ADJOINT_CKPT_EVERY = 20


def batched(seed: int = 3, n_chains: int = 64, m: int = 16) -> List[Chain]:
    """64 independent chains of uneven length, anisotropy and slice count.

    ``m`` is a placeholder Krylov dimension; the autotuner replaces it per chain."""
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(n_chains):
        L = int(rng.integers(10, 17))
        Delta = float(rng.uniform(0.0, 1.5))
        N = int(rng.integers(50, 301))
        D = 1 << L
        u = rng.uniform(-1.0, 1.0, N)
        psi0 = random_phase_state(rng, D)
        target = random_phase_state(rng, D)
        chains.append(Chain(L=L, J=1.0, Delta=Delta, hc_kind=HC_SX, hc_sites=1, N=N, dt=0.05,
                            m=m, u=u, psi0=psi0, target=target))
    return chains


# ---------------------------------------------------------------- reduced basis

# Dimensions of the fixed-excitation, even-parity spaces studied in Sec. III.B
# (the figures quote D = 10, 19, 44, 60 and 146).  The (L, K) that give them
# with K = 3 excitations are this module's reading; the paper names D only.
PAPER_PE_DIMS = {(6, 3): 10, (7, 3): 19, (9, 3): 44, (10, 3): 60, (13, 3): 146}


@dataclasses.dataclass(frozen=True)
class PETask:
    """The transfer task e_1 -> e_D of Sec. III.A in the reduced basis of L spins
    with K excitations: the paper's drift (J_p = 1, alpha_z = 0.5, i.e. J = 2 and
    Delta = 0.5 in the S = sigma/2 form) and control J_p (S^z_1 + S^z_L).

    e1_state / eD_state are the product states (full-space indices) whose
    orbits are the task's basis vectors: K up spins in the middle of the chain,
    and K up spins at the left edge (its orbit also holds the right edge)."""

    L: int
    K: int
    J: float
    Delta: float
    hc_sites: int
    N: int
    dt: float
    m: int
    u: np.ndarray
    e1_state: int
    eD_state: int


def pe_task(L: int, K: int, N: int, seed: int = 5, dt: float = 0.5, m: int = 10) -> PETask:
    """Controls U(-1, 1) for N slices (the paper draws M = 4D of them), dt = 0.5,
    Krylov dimension 10 (Sec. III.B)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, N)
    left = (L - K) // 2
    e1 = basis_index("d" * left + "u" * K + "d" * (L - K - left))
    eD = basis_index("u" * K + "d" * (L - K))
    return PETask(L=L, K=K, J=2.0, Delta=0.5, hc_sites=1 | (1 << (L - 1)), N=N, dt=dt, m=m,
                  u=u, e1_state=e1, eD_state=eD)


def pe_paper(L: int, K: int, seed: int = 5) -> PETask:
    """A task of Sec. III.B at its own size: M = 4D slices."""
    return pe_task(L, K, 4 * PAPER_PE_DIMS[(L, K)], seed)


def pe_large(seed: int = 6, N: int = 200) -> PETask:
    """The transport task (odd L, even K) at L = 25, K = 12, N = 200 slices of
    dt = 0.1.  The spectral radius of this sector is about 20, so dt = 0.5 with
    10 Krylov vectors would sit outside the step sizes where the truncated
    propagator is accurate (the control window shrinks with D, Sec. III.B);
    dt = 0.1 keeps ||H|| dt near 2."""
    return pe_task(25, 12, N, seed, dt=0.1)


def scaled(chain: Chain, **changes) -> Chain:
    """A copy of ``chain`` with some fields replaced (e.g. a shorter N)."""
    if "N" in changes and "u" not in changes:
        changes["u"] = chain.u[: changes["N"]].copy()
    return dataclasses.replace(chain, **changes)
