"""Fixed-excitation, parity-even basis of the open XXZ chain (oracle; test
infrastructure only).

Sec. III.A: the drift and the control J_p (S^z_1 + S^z_L) conserve the number
K of excitations (up spins, bit 0) and the parity Pi, the mirror i -> L+1-i,
so a state that starts in the even-parity part of the K-excitation sector
stays there, and the computation can run in that reduced space.

Construction here, from the definitions: the sector is spanned by the product
states s with exactly K zero bits among L; Pi maps s to its bit reversal over
L bits.  Every orbit {s, Pi s} gives one even basis vector, (|s> + |Pi s>)/sqrt(2),
or |s> when Pi s = s.  An orbit is labelled by its smaller member r and the
basis is ordered by r ascending (the paper orders the reduced basis by the
binary number of the bit sequence, up = 0).  The paper reaches the same
subspace by diagonalising Pi inside the sector and keeping the +1
eigenvectors; a pin compares the two.

Reduced H v, matrix-free: with x the coordinates in this basis and X the
sector vector X(s) = x_a / sqrt(n_a) (n_a the orbit size of s), Y = H X is
again parity-even and y_b = sqrt(n_b) Y(r_b), so
    y_b = d(r_b) x_b + (J/2) sum_{bonds p of r_b} sqrt(n_b / n_a(p)) x_a(p),
a(p) the orbit of r_b with the antiparallel bits p, p+1 exchanged, and d the
diagonal of H0 + u Hc (Hc a sum of S^z over a mirror-symmetric set of sites).

Task states (the example following the control task, e_1 -> e_D): e_1 is the
orbit of K up spins in the middle of the chain (left block of down spins
floor((L-K)/2) long), e_D the orbit of K up spins at one edge.
"""

from __future__ import annotations

from math import comb

import numpy as np

from . import model


def reverse_bits(s: np.ndarray, L: int) -> np.ndarray:
    s = np.asarray(s, dtype=np.int64)
    r = np.zeros_like(s)
    for b in range(L):
        r |= ((s >> b) & 1) << (L - 1 - b)
    return r


def sector_states(L: int, K: int) -> np.ndarray:
    """All L-bit patterns with exactly K zero bits (K up spins), ascending."""
    s = np.arange(1 << L, dtype=np.int64)
    ones = np.zeros_like(s)
    for b in range(L):
        ones += (s >> b) & 1
    return s[ones == L - K]


class PEBasis:
    """Orbit representatives r (ascending), orbit sizes n, and the index map."""

    def __init__(self, L: int, K: int):
        self.L, self.K = L, K
        st = sector_states(L, K)
        rev = reverse_bits(st, L)
        self.reps = st[st <= rev]                       # orbit labels, ascending
        self.n = np.where(reverse_bits(self.reps, L) == self.reps, 1, 2)
        self.dim = self.reps.size
        self._pos = {int(r): i for i, r in enumerate(self.reps)}

    def index(self, s: np.ndarray) -> np.ndarray:
        """Basis index of the orbit of each sector state s."""
        s = np.asarray(s, dtype=np.int64)
        r = np.minimum(s, reverse_bits(s, self.L))
        return np.array([self._pos[int(v)] for v in r.ravel()], dtype=np.int64).reshape(s.shape)

    def embed(self, x: np.ndarray) -> np.ndarray:
        """Full-space vector (2^L amplitudes) of the reduced coordinates x."""
        X = np.zeros(1 << self.L, dtype=np.complex128)
        X[self.reps] = x / np.sqrt(self.n)
        X[reverse_bits(self.reps, self.L)] = x / np.sqrt(self.n)
        return X

    def project(self, X: np.ndarray) -> np.ndarray:
        """Reduced coordinates <b|X> of a full-space vector."""
        return (X[self.reps] + X[reverse_bits(self.reps, self.L)]) / np.sqrt(self.n) * \
            np.where(self.n == 1, 0.5, 1.0)

    def task_states(self):
        """(e_1, e_D) of the transfer task as reduced coordinate vectors."""
        L, K = self.L, self.K
        left = (L - K) // 2
        down = (1 << L) - 1
        mid = down & ~(((1 << K) - 1) << (L - left - K))   # K zero bits after `left` ones
        edge = (1 << (L - K)) - 1                          # K zero bits at the top (sites 1..K)
        e1 = np.zeros(self.dim, dtype=np.complex128)
        eD = np.zeros(self.dim, dtype=np.complex128)
        e1[self.index(np.array([mid]))[0]] = 1.0
        eD[self.index(np.array([edge]))[0]] = 1.0
        return e1, eD


def diag_pe(B: PEBasis, J: float, Delta: float, sz_sites: int, u: float) -> np.ndarray:
    d = model.diag_h0(B.L, J, Delta, B.reps).real.astype(np.float64)
    if sz_sites:
        d = d + u * model.sz_control_diag(B.L, sz_sites, B.reps).real
    return d


def apply_h_pe(B: PEBasis, J: float, Delta: float, sz_sites: int, u: float,
               x: np.ndarray) -> np.ndarray:
    """Reduced (H0 + u Hc) x, Hc = sum of S^z over `sz_sites` (mirror-symmetric)."""
    L = B.L
    y = diag_pe(B, J, Delta, sz_sites, u) * x
    for p in range(L - 1):
        active = (((B.reps >> p) ^ (B.reps >> (p + 1))) & 1) == 1
        rb = B.reps[active]
        a = B.index(rb ^ (3 << p))
        w = np.sqrt(B.n[active] / B.n[a])
        y[active] += 0.5 * J * w * x[a]
    return y


def apply_h_pe_rows(B: PEBasis, J: float, Delta: float, sz_sites: int, u: float,
                    x: np.ndarray, rows) -> np.ndarray:
    """Selected entries y_b of the reduced (H0 + u Hc) x, one row at a time
    (for spot checks at sizes where the whole product is too slow here)."""
    L = B.L
    out = np.zeros(len(rows), dtype=np.complex128)
    for i, b in enumerate(rows):
        r = int(B.reps[b])
        val = complex(diag_pe_rows(B, J, Delta, sz_sites, u, r)) * x[b]
        for p in range(L - 1):
            if ((r >> p) ^ (r >> (p + 1))) & 1:
                a = int(B.index(np.array([r ^ (3 << p)]))[0])
                val += 0.5 * J * np.sqrt(B.n[b] / B.n[a]) * x[a]
        out[i] = val
    return out


def diag_pe_rows(B: PEBasis, J: float, Delta: float, sz_sites: int, u: float, r: int) -> float:
    s = np.array([r], dtype=np.int64)
    d = float(model.diag_h0(B.L, J, Delta, s).real[0])
    if sz_sites:
        d += u * float(model.sz_control_diag(B.L, sz_sites, s).real[0])
    return d


def hc_pe(B: PEBasis, sz_sites: int) -> np.ndarray:
    """Diagonal of the reduced control operator."""
    return model.sz_control_diag(B.L, sz_sites, B.reps).real


def dense_pe(B: PEBasis, J: float, Delta: float, sz_sites: int, u: float) -> np.ndarray:
    """The reduced matrix, column by column from apply_h_pe (small dimensions)."""
    H = np.zeros((B.dim, B.dim), dtype=np.complex128)
    for c in range(B.dim):
        e = np.zeros(B.dim, dtype=np.complex128)
        e[c] = 1.0
        H[:, c] = apply_h_pe(B, J, Delta, sz_sites, u, e)
    return H


def is_mirror_symmetric(L: int, sites: int) -> bool:
    return all(((sites >> (i - 1)) & 1) == ((sites >> (L - i)) & 1) for i in range(1, L + 1))


class PEChain:
    """The reduced chain with the interface of model.Chain (apply, apply_hc), so
    the oracle's Krylov propagator and GRAPE sweeps run on it unchanged."""

    def __init__(self, L: int, K: int, J: float, Delta: float, sz_sites: int):
        if not is_mirror_symmetric(L, sz_sites):
            raise ValueError("the control sites must be mirror-symmetric to conserve parity")
        self.B = PEBasis(L, K)
        self.L, self.K, self.J, self.Delta, self.sz_sites = L, K, J, Delta, sz_sites
        self.dim = self.B.dim
        self._d0 = diag_pe(self.B, J, Delta, 0, 0.0)
        self._hc = hc_pe(self.B, sz_sites)

    def apply(self, u: float, v: np.ndarray) -> np.ndarray:
        return apply_h_pe(self.B, self.J, self.Delta, self.sz_sites, u, v)

    def apply_hc(self, v: np.ndarray) -> np.ndarray:
        return self._hc * v


def sector_dim_count(L: int, K: int) -> int:
    """Number of even orbits: (C(L,K) + palindromes) / 2."""
    st = sector_states(L, K)
    pal = int(np.sum(reverse_bits(st, L) == st))
    return (comb(L, K) + pal) // 2
