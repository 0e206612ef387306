"""Open XXZ spin chain and its control operators (oracle; test infrastructure only).

Model (Sec. III.A, Eq. 6; control operator Eq. 10):
    H0 = J * sum_{i=1}^{L-1} (Sx_i Sx_{i+1} + Sy_i Sy_{i+1} + Delta Sz_i Sz_{i+1}),  S = sigma/2.
The paper writes the drift with Pauli matrices and prefactor J_p/2 and anisotropy
alpha_z; with S = sigma/2 that is the same operator with J = 2 J_p, Delta = alpha_z
(pinned by ``pauli_drift_dense`` against ``xxz_dense``).

Control operators:
    SX(i):  S^x on one site i;
    SZ(A):  sum_{i in A} S^z_i  (the paper's control is J_p (S^z_1 + S^z_L), Eq. 10).

Basis (Sec. III.A, last paragraph of the model description): spin up = bit 0,
spin down = bit 1, site 1 is the most significant bit, so site i <-> bit L-i.

Three independent constructions:
    xxz_dense      Kronecker products of 2x2 spin matrices (small L);
    xxz_sparse     bit operations, assembled into scipy.sparse CSR;
    apply_h        matrix-free bit operations on a numpy vector;
and ``h_rows`` evaluates single output amplitudes (H v)[s] from the same
definition for sampled checks at sizes where no matrix can be built.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HC_SX = 0
HC_SZ = 1

# single-site spin-1/2 operators in the basis (up, down) = (bit 0, bit 1)
SX = np.array([[0.0, 0.5], [0.5, 0.0]], dtype=np.complex128)
SY = np.array([[0.0, -0.5j], [0.5j, 0.0]], dtype=np.complex128)
SZ = np.array([[0.5, 0.0], [0.0, -0.5]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def hc_sites_list(L: int, hc_sites: int):
    """Sites (1-based) whose bit is set in the ``hc_sites`` mask."""
    return [i for i in range(1, L + 1) if (hc_sites >> (i - 1)) & 1]


# --------------------------------------------------------------------------- dense (Kronecker)

def site_op(L: int, i: int, op: np.ndarray) -> np.ndarray:
    """op acting on site i (1-based) of an L-site chain; site 1 is the leftmost factor."""
    out = np.ones((1, 1), dtype=np.complex128)
    for k in range(1, L + 1):
        out = np.kron(out, op if k == i else I2)
    return out


def xxz_dense(L: int, J: float, Delta: float) -> np.ndarray:
    """Eq. 6 in the S = sigma/2 form, built from Kronecker products (L <= 12)."""
    D = 1 << L
    H = np.zeros((D, D), dtype=np.complex128)
    for i in range(1, L):
        H += J * (site_op(L, i, SX) @ site_op(L, i + 1, SX)
                  + site_op(L, i, SY) @ site_op(L, i + 1, SY)
                  + Delta * site_op(L, i, SZ) @ site_op(L, i + 1, SZ))
    return H


def pauli_drift_dense(L: int, Jp: float, alpha_z: float) -> np.ndarray:
    """Eq. 6 exactly as printed: (J_p/2) sum sigma.sigma with anisotropy alpha_z."""
    sx, sy, sz = 2 * SX, 2 * SY, 2 * SZ
    D = 1 << L
    H = np.zeros((D, D), dtype=np.complex128)
    for i in range(1, L):
        H += (Jp / 2.0) * (site_op(L, i, sx) @ site_op(L, i + 1, sx)
                           + site_op(L, i, sy) @ site_op(L, i + 1, sy)
                           + alpha_z * site_op(L, i, sz) @ site_op(L, i + 1, sz))
    return H


def hc_dense(L: int, hc_kind: int, hc_sites: int) -> np.ndarray:
    """Control operator from spin matrices: S^x on one site, or a sum of S^z."""
    sites = hc_sites_list(L, hc_sites)
    if hc_kind == HC_SX:
        assert len(sites) == 1
        return site_op(L, sites[0], SX)
    D = 1 << L
    H = np.zeros((D, D), dtype=np.complex128)
    for i in sites:
        H += site_op(L, i, SZ)
    return H


# --------------------------------------------------------------------------- bit definitions

def bit(s, b):
    return (s >> b) & 1


def n_antiparallel(L: int, s: np.ndarray) -> np.ndarray:
    """Number of nearest-neighbour bonds whose two spins differ, bond by bond."""
    n = np.zeros_like(s)
    for p in range(L - 1):
        n += bit(s, p) ^ bit(s, p + 1)
    return n


def diag_h0(L: int, J: float, Delta: float, s: np.ndarray) -> np.ndarray:
    """<s|H0|s> = J*Delta/4 * (#parallel bonds - #antiparallel bonds)."""
    c_zz = 0.25 * J * Delta
    return c_zz * (L - 1 - 2 * n_antiparallel(L, s)).astype(np.float64)


def sz_control_diag(L: int, hc_sites: int, s: np.ndarray) -> np.ndarray:
    """<s| sum_{i in A} S^z_i |s> = sum_{i in A} (1/2 - b_i)."""
    out = np.zeros(s.shape, dtype=np.float64)
    for i in hc_sites_list(L, hc_sites):
        out += 0.5 - bit(s, L - i)
    return out


def partner_mask(L: int, s: np.ndarray) -> np.ndarray:
    """Bit p set <=> bond (p, p+1) is antiparallel in s, i.e. s ^ (3 << p) is coupled to s."""
    m = np.zeros_like(s)
    for p in range(L - 1):
        m |= (bit(s, p) ^ bit(s, p + 1)) << p
    return m


# --------------------------------------------------------------------------- sparse (CSR)

def xxz_sparse(L: int, J: float, Delta: float) -> sp.csr_matrix:
    """H0 assembled element by element from the bit rules into CSR (L <= 22)."""
    D = 1 << L
    s = np.arange(D, dtype=np.int64)
    rows = [s]
    cols = [s]
    vals = [diag_h0(L, J, Delta, s).astype(np.complex128)]
    for p in range(L - 1):
        act = (bit(s, p) ^ bit(s, p + 1)).astype(bool)
        src = s[act]
        rows.append(src ^ (3 << p))
        cols.append(src)
        vals.append(np.full(src.shape, 0.5 * J, dtype=np.complex128))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(D, D))
    return H.tocsr()


def hc_sparse(L: int, hc_kind: int, hc_sites: int) -> sp.csr_matrix:
    D = 1 << L
    s = np.arange(D, dtype=np.int64)
    if hc_kind == HC_SX:
        sites = hc_sites_list(L, hc_sites)
        assert len(sites) == 1
        b = L - sites[0]
        return sp.csr_matrix((np.full(D, 0.5, dtype=np.complex128), (s ^ (1 << b), s)),
                             shape=(D, D))
    return sp.diags(sz_control_diag(L, hc_sites, s).astype(np.complex128)).tocsr()


# --------------------------------------------------------------------------- matrix-free

class Chain:
    """H(u) = H0 + u*Hc of an open XXZ chain, applied through whichever
    construction suits the size: CSR for L <= 22, matrix-free bits above."""

    def __init__(self, L: int, J: float, Delta: float, hc_kind: int, hc_sites: int,
                 matrix_free: bool | None = None):
        if hc_kind == HC_SX:
            assert len(hc_sites_list(L, hc_sites)) == 1, "SX control acts on exactly one site"
        self.L, self.J, self.Delta = L, J, Delta
        self.hc_kind, self.hc_sites = hc_kind, hc_sites
        self.D = 1 << L
        self.matrix_free = (L > 22) if matrix_free is None else matrix_free
        if not self.matrix_free:
            self.H0 = xxz_sparse(L, J, Delta)
            self.Hc = hc_sparse(L, hc_kind, hc_sites)

    def apply(self, u: float, v: np.ndarray) -> np.ndarray:
        if self.matrix_free:
            return apply_h(self.L, self.J, self.Delta, self.hc_kind, self.hc_sites, u, v)
        return self.H0 @ v + u * (self.Hc @ v)

    def apply_hc(self, v: np.ndarray) -> np.ndarray:
        if self.matrix_free:
            return apply_hc(self.L, self.hc_kind, self.hc_sites, v)
        return self.Hc @ v


def apply_hc(L: int, hc_kind: int, hc_sites: int, v: np.ndarray) -> np.ndarray:
    s = np.arange(1 << L, dtype=np.int64)
    if hc_kind == HC_SX:
        (i,) = hc_sites_list(L, hc_sites)
        return 0.5 * v[s ^ (1 << (L - i))]
    return sz_control_diag(L, hc_sites, s) * v


def apply_h(L, J, Delta, hc_kind, hc_sites, u, v):
    """(H0 + u Hc) v by bit operations, one bond at a time."""
    s = np.arange(1 << L, dtype=np.int64)
    w = diag_h0(L, J, Delta, s) * v
    for p in range(L - 1):
        act = (bit(s, p) ^ bit(s, p + 1)).astype(bool)
        w[act] += 0.5 * J * v[(s ^ (3 << p))[act]]
    if u != 0.0:
        w += u * apply_hc(L, hc_kind, hc_sites, v)
    return w


def h_rows(L, J, Delta, hc_kind, hc_sites, u, v, rows: np.ndarray) -> np.ndarray:
    """Selected amplitudes (H v)[s] for s in ``rows``, from the element definitions."""
    s = np.asarray(rows, dtype=np.int64)
    out = diag_h0(L, J, Delta, s) * v[s]
    for p in range(L - 1):
        act = bit(s, p) ^ bit(s, p + 1)
        out = out + np.where(act == 1, 0.5 * J * v[s ^ (3 << p)], 0.0)
    if hc_kind == HC_SX:
        (i,) = hc_sites_list(L, hc_sites)
        out = out + u * 0.5 * v[s ^ (1 << (L - i))]
    else:
        out = out + u * sz_control_diag(L, hc_sites, s) * v[s]
    return out
