/*
 * kgrape.h - C ABI of the MI355X (gfx950) K-GRAPE library (libkgrape.so).
 *
 * K-GRAPE (Larocca & Wisniacki, arXiv 2010.03598) is GRAPE with every
 * sub-propagator applied by a Krylov (Lanczos) approximation.  This library
 * runs its hot path on one GPU:
 *   xxz_apply       w = (H0 + u Hc) v                       (Sec. III.A, Eqs. 1, 6, 10)
 *   krylov_expv     v_out ~ exp(-i t (H0 + u Hc)) v_in      (App. A, Algorithm 2, Eqs. A1-A3)
 *   grape_forward   psi_j = U_j psi_{j-1}, beta = <f|psi_N>, F = |beta|^2
 *                                                           (Algorithm 1, Eqs. 2, 4, B1, B2)
 *   grape_gradient  dF/du_j = 2 dt Im(conj(beta) <lambda_j|Hc|psi_j>)
 *                   with lambda_N = f, lambda_{j-1} = U_j^dagger lambda_j   (Eq. 5, Algorithm 1)
 *   grape_gradient_centred  the same bracket at both ends of each slice, averaged
 *                   (the centred variant of App. B, error O(dt^3) per slice)
 *   grape_gradient_quadrature  exact piecewise-constant gradient by Gauss-Legendre
 *                   quadrature of the natural gradient inside each slice (App. B)
 *   grape_gradient_first_order  first order of the hierarchy of the time-averaged
 *                   control operator (one commutator with H_j, App. B)
 *   grape_ascent_update  u <- u + eta g / max|g|            (steepest ascent, Algorithm 1 update)
 *   grape_gradient_columns  operator control on a block of columns: the gradient of
 *                   |(1/n) sum_c <w_c|U(T)|psi_c>|^2 (the generalisation named in Sec. IV)
 *   xxz_pe_apply, krylov_expv_pe, grape_forward_pe, grape_gradient_pe
 *                   the same in the basis of fixed excitation number and even
 *                   mirror parity (Sec. III.A), for S^z controls on mirror-symmetric sites
 *
 * Model.  Open chain of L spins 1/2, S = sigma/2:
 *   H0 = J sum_{i=1}^{L-1} (Sx_i Sx_{i+1} + Sy_i Sy_{i+1} + Delta Sz_i Sz_{i+1}).
 * The paper's Pauli form (J_p/2) sum(sigma sigma + alpha_z sigma^z sigma^z) is
 * J = 2 J_p, Delta = alpha_z here.  Control operators: KG_HC_SX = S^x on one
 * site; KG_HC_SZ = sum of S^z over a set of sites (the paper's control is
 * J_p (S^z_1 + S^z_L), i.e. KG_HC_SZ on {1, L} with u scaled by J_p).
 *
 * Basis.  Spin up = bit 0, spin down = bit 1, site 1 is the most significant
 * bit: the amplitude of a product state sits at index s = sum_i b_i 2^(L-i)
 * (the paper's ordering of computational basis states, Sec. III.A).
 *
 * Data.  State vectors are D = 2^L complex amplitudes, interleaved (re, im),
 * contiguous: complex128 (16 B) for KG_C128, complex64 (8 B) for KG_C64.  All
 * vector, control, output and workspace pointers are DEVICE pointers owned by
 * the caller; vectors must be 16-byte aligned, workspaces 256-byte aligned.
 * Controls u and every scalar result (F, beta, gradient) are FP64.
 *
 * Precision KG_C64 keeps vectors in complex64 and applies H in FP32, while the
 * Lanczos scalars (alpha, beta, norms), every dot product (re-orthogonalisation
 * sums, overlap, gradient bracket), the small exponential and the basis
 * combination run in FP64 (one rounding to complex64 per stored vector).
 *
 * Conventions of every entry point.
 *   - Host-side validation runs first; on failure nothing is launched, the
 *     status is negative and kg_last_error() names the argument.
 *   - Nothing allocates device memory; scratch comes from the caller's
 *     workspace (size from kg_workspace_bytes).  No call synchronises the
 *     stream (kg_pe_build, which copies its tables synchronously, aside);
 *     results are ready when the stream reaches them.
 *   - `stream` is a hipStream_t (NULL = the default stream).  The gradient
 *     calls with checkpoints (more than two segments) run the recomputation of
 *     earlier segments on a second stream of the library's own (one per host
 *     thread and device, default priority), forked from `stream` with an event
 *     and joined back to it before any result is read, so the call stays
 *     ordered on `stream` and a capture of `stream` takes in both branches.
 *     Setting KG_ONE_STREAM in the environment keeps all work on `stream`.
 *   - Inputs are never renormalised: psi0 and the target should have unit norm.
 *   - Calls that share a workspace must not run concurrently.
 *   - Lanczos breakdown (an invariant Krylov space) is not an error: the call
 *     uses the reached dimension m_eff < m, reported through m_eff_dev.
 */
#ifndef KGRAPE_H
#define KGRAPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kg_status;
#define KG_OK 0
#define KG_EINVAL (-1)      /* bad argument: see kg_last_error() */
#define KG_EWORKSPACE (-3)  /* workspace or state buffer too small / misaligned */
#define KG_EDEVICE (-4)     /* a HIP runtime call failed (launch error, no device) */

#define KG_C128 0           /* complex128 vectors, FP64 everything */
#define KG_C64 1            /* complex64 vectors, FP64 scalars */

#define KG_HC_SX 0          /* S^x on exactly one site */
#define KG_HC_SZ 1          /* sum of S^z over a non-empty set of sites */

#define KG_MAX_M 64         /* largest Krylov dimension */
#define KG_MIN_L 2
#define KG_MAX_L 30

/* One open XXZ chain.  hc_sites: bit (i-1) set <=> site i (1..L) carries the
 * control operator; KG_HC_SX needs exactly one bit. */
typedef struct kg_xxz {
  int32_t L;
  int32_t hc_kind;
  double J;
  double Delta;
  uint64_t hc_sites;
} kg_xxz;

/* Krylov options.  m: dimension (1..KG_MAX_M).  reorth: 1 = each candidate
 * H v_k is orthogonalised against all previous basis vectors (full classical
 * Gram-Schmidt, App. A), 0 = against the last two only (plain Lanczos,
 * Algorithm 2).  breakdown_tol: relative threshold; the basis stops at step k
 * when ||w_{k+1}|| <= tol * max(1, max_{i<=k}(|alpha_i| + beta_i)); 0 selects
 * 64 * (unit roundoff of the vector type).  The projected exponential
 * exp(-i t T) e_1 is evaluated for |t| ||T||_inf <= 32768; beyond that, or for
 * a non-finite T (for example a non-finite control amplitude), the call's
 * output vector is NaN. */
typedef struct kg_krylov {
  int32_t m;
  int32_t reorth;
  double breakdown_tol;
} kg_krylov;

/* Thread-local description of the last failure in this thread ("" if none). */
const char* kg_last_error(void);

/* Library ABI version (monotonic integer). */
int32_t kg_version(void);

/* Bytes of workspace that krylov_expv, grape_forward and grape_gradient need
 * for this chain, Krylov dimension and precision: two Krylov slots (scalars,
 * reduction partials, m-1 basis vectors and one vector H v_k each; the
 * second slot advances the segment recomputation beside the backward sweep)
 * and one costate vector.
 * Returns 0 for invalid arguments. */
size_t kg_workspace_bytes(const kg_xxz* h, const kg_krylov* k, int32_t prec);

/* Bytes of the forward-state buffer of grape_forward/grape_gradient.
 * ckpt_every = 0 stores psi_1..psi_N (N vectors).  ckpt_every = c in 1..N
 * splits the slices into segments (q c, (q+1) c]; it stores psi_c, psi_2c, ...
 * below the last segment (ceil(N/c)-1 vectors) plus two segment buffers of c
 * vectors (one if there is a single segment).  The backward sweep recomputes
 * each earlier segment from its checkpoint beside the costate propagation of
 * the later one (sqrt(N) checkpointing when c ~ sqrt(N)).  Returns 0 for
 * invalid arguments. */
size_t kg_states_bytes(const kg_xxz* h, int32_t N, int32_t ckpt_every, int32_t prec);

/* w = (H0 + u Hc) v  (Eqs. 1, 6, 10; matrix-free).  v and w: D amplitudes of
 * type `prec`; they must not overlap.  Errors: KG_EINVAL, KG_EDEVICE. */
kg_status xxz_apply(const kg_xxz* h, double u, int32_t prec, const void* v, void* w,
                    void* stream);

/* v_out ~ exp(-i t (H0 + u Hc)) v_in by an m-dimensional Lanczos basis
 * (App. A, Algorithm 2) and the exponential of the tridiagonal projection
 * (Eqs. A1-A3): v_out = ||v_in|| V^T exp(-i t T) e_1.  v_out may equal v_in
 * (in place); otherwise they must not overlap.  A zero input gives a zero
 * output (m_eff = 0), an input with a non-finite amplitude a NaN output
 * (m_eff = 1).  m_eff_dev (nullable): device int32 that receives the
 * dimension reached.  Errors: KG_EINVAL, KG_EWORKSPACE, KG_EDEVICE. */
kg_status krylov_expv(const kg_xxz* h, double u, double t, const kg_krylov* k, int32_t prec,
                      const void* v_in, void* v_out, void* ws, size_t ws_bytes,
                      int32_t* m_eff_dev, void* stream);

/* krylov_expv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, kernels and results, with the scratch in a static device
 * array of kg_static_scratch_bytes() (64 MiB) that each GPU the library runs on
 * holds until the process ends, instead of a caller's workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine); the
 * caller still passes the vectors.  It needs one Krylov slot, 4.4 MB of
 * scalars and partials plus m vectors of 2^L amplitudes (for example L <= 18
 * with m <= 25 in complex64, L <= 17 with m <= 25 in complex128); larger
 * problems fail with KG_EWORKSPACE and a message.  Every call on a GPU shares
 * that GPU's array and leaves its contents there: calls that overlap on one
 * GPU (other streams, other host threads) race and must be serialised by the
 * caller.  Errors: KG_EINVAL, KG_EWORKSPACE, KG_EDEVICE. */
size_t kg_static_scratch_bytes(void);
kg_status krylov_expv_static(const kg_xxz* h, double u, double t, const kg_krylov* k, int32_t prec,
                             const void* v_in, void* v_out, int32_t* m_eff_dev, void* stream);

/* Forward sweep of Algorithm 1 (Eqs. 2, 4, B1, B2): psi_j = exp(-i dt H_j)
 * psi_{j-1}, H_j = H0 + u_j Hc, j = 1..N, with u_dev[j-1] = u_j.  Writes
 * beta = <target|psi_N> to beta_dev[0..1] (re, im) and F = |beta|^2 to
 * *F_dev.  `states` (kg_states_bytes) receives the stored forward states in
 * the layout of ckpt_every; psi_N is stored in it.  Errors: KG_EINVAL,
 * KG_EWORKSPACE, KG_EDEVICE. */
kg_status grape_forward(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                        const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                        double* F_dev, double* beta_dev, void* states, int32_t ckpt_every,
                        void* ws, size_t ws_bytes, void* stream);

/* Fidelity and zeroth-order GRAPE gradient (Eq. 5, Algorithm 1):
 *   grad_dev[j-1] = dF/du_j ~ 2 dt Im(conj(beta) <lambda_j|Hc|psi_j>),
 *   lambda_N = target, lambda_{j-1} = exp(+i dt H_j) lambda_j.
 * (The paper's infidelity gradient is -grad, its chi_j is beta lambda_j.)
 * states_valid = 1 reuses the states and beta of a preceding grape_forward
 * with the same arguments (no forward sweep); 0 runs the forward sweep first.
 * With ckpt_every > 0 the segments between checkpoints are recomputed; the
 * result is bit-identical to ckpt_every = 0.  With more than two segments
 * (N > 2 ckpt_every) the recomputation overwrites the segment buffers, so the
 * call uses the states up: a further gradient call on the same buffer needs
 * states_valid = 0 (every gradient variant below behaves the same way).
 * F_dev, beta_dev as in grape_forward.  Errors: KG_EINVAL, KG_EWORKSPACE,
 * KG_EDEVICE. */
kg_status grape_gradient(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                         const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                         double* F_dev, double* beta_dev, double* grad_dev, void* states,
                         int32_t ckpt_every, int32_t states_valid, void* ws, size_t ws_bytes,
                         void* stream);

/* Centred zeroth-order gradient (App. B, the centred variant of Eq. 5): the
 * natural gradient of slice j evaluated at the slice centre, approximated by
 * the mean of the Eq. 5 bracket at the two ends of the slice,
 *   dF/du_j ~ (G_{j-1} + G_j) / 2,  G_j = 2 dt Im(conj(beta) <lambda_j|Hc|psi_j>),
 * with G_0 from psi_0 and lambda_0 = U_1^dagger lambda_1 (one backward
 * propagation more than grape_gradient).  Its error against the exact
 * piecewise-constant gradient is O(dt^3) per slice instead of O(dt^2).
 * Arguments, buffers and errors as grape_gradient; states left by
 * grape_forward may be reused (states_valid = 1). */
kg_status grape_gradient_centred(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                 const kg_krylov* k, int32_t prec, const void* psi0,
                                 const void* target, double* F_dev, double* beta_dev,
                                 double* grad_dev, void* states, int32_t ckpt_every,
                                 int32_t states_valid, void* ws, size_t ws_bytes, void* stream);

/* Exact piecewise-constant gradient by Gauss-Legendre quadrature of the
 * natural gradient inside each slice (App. B): with nodes s_q in (0, dt) and
 * weights w_q of the n-point rule on [0, dt],
 *   dF/du_j = sum_q 2 w_q Im(conj(beta) <e^{+i H_j (dt - s_q)} lambda_j | Hc |
 *                                      e^{-i H_j s_q} psi_{j-1}>),
 * the node states from Krylov propagations over partial steps (2n per slice).
 * Its error is that of the n-point rule, O(dt^(2n+1)) per slice, plus the
 * Krylov error, so it is the derivative of the forward's F to that accuracy.
 * nodes: 1..KG_MAX_NODES.  The workspace must hold
 * kg_extended_workspace_bytes (two node vectors beyond kg_workspace_bytes).
 * Other arguments, buffers and errors as grape_gradient. */
#define KG_MAX_NODES 16
/* Workspace of grape_gradient_quadrature and grape_gradient_first_order:
 * kg_workspace_bytes plus two vectors.  Returns 0 for invalid arguments. */
size_t kg_extended_workspace_bytes(const kg_xxz* h, const kg_krylov* k, int32_t prec);
kg_status grape_gradient_quadrature(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                    const kg_krylov* k, int32_t prec, const void* psi0,
                                    const void* target, double* F_dev, double* beta_dev,
                                    double* grad_dev, void* states, int32_t ckpt_every,
                                    int32_t states_valid, int32_t nodes, void* ws,
                                    size_t ws_bytes, void* stream);

/* First order of the Taylor hierarchy of the time-averaged control operator
 * (App. B): Hc_bar^[1] = Hc - (i dt / 2) [H_j, Hc], and
 *   dF/du_j ~ 2 dt Im(conj(beta) <lambda_j| Hc_bar^[1] |psi_j>)
 *           = 2 dt Im(conj(beta) (<lambda|Hc psi> - (i dt/2)(<H lambda|Hc psi> - <lambda|Hc H psi>))),
 * two H v products per slice beyond Eq. 5.  Error O(dt^3) per slice.  The
 * workspace must hold kg_extended_workspace_bytes; other arguments as
 * grape_gradient. */
kg_status grape_gradient_first_order(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                     const kg_krylov* k, int32_t prec, const void* psi0,
                                     const void* target, double* F_dev, double* beta_dev,
                                     double* grad_dev, void* states, int32_t ckpt_every,
                                     int32_t states_valid, void* ws, size_t ws_bytes,
                                     void* stream);

/* Steepest-ascent update u_j <- u_j + eta * g_j / max_i |g_i| on the device
 * (u unchanged when g = 0).  N >= 1.  Errors: KG_EINVAL, KG_EDEVICE. */
kg_status grape_ascent_update(double* u_dev, const double* grad_dev, int32_t N, double eta,
                              void* stream);

/* ---------------------------------------------------------------- operator control
 * The conclusions name the control of operators (unitaries) as the method's
 * generalisation.  For a block of n columns psi_c -> w_c (all 2^L basis
 * vectors and W = the target unitary's columns give the whole gate) the
 * objective is the phase-insensitive subspace gate fidelity
 *   F = |beta|^2,  beta = (1/n) sum_c <w_c| U(T) |psi_c>   (= |Tr(W^dag U)/D|^2 for n = D),
 * and its zeroth-order gradient is Eq. 5 with the brackets of all columns:
 *   dF/du_j ~ 2 dt Im(conj(beta) (1/n) sum_c <lambda_{c,j}|Hc|psi_{c,j}>),
 * lambda_{c,N} = w_c propagated backward per column (centred = 1: the bracket
 * sums averaged over the two ends of each slice, as grape_gradient_centred).
 * Every column has its own Krylov spaces; the forward sweeps of two columns
 * share each launch.
 *   psi0s, targets  n_cols vectors of 2^L amplitudes each, column c at c * 2^L
 *   states          n_cols state buffers of kg_states_bytes(h, N, ckpt_every, prec)
 *                   bytes each, column c at c times that size
 *                   (kg_columns_states_bytes gives the total)
 *   beta_cols_dev   2 n_cols doubles: <w_c|psi_{c,N}> per column (output)
 *   F_dev (nullable), beta_dev (2 doubles), grad_dev (N doubles): F, beta, dF/du
 *   ws              kg_workspace_bytes, as for grape_gradient
 * Errors: KG_EINVAL, KG_EWORKSPACE, KG_EDEVICE. */
size_t kg_columns_states_bytes(const kg_xxz* h, int32_t n_cols, int32_t N, int32_t ckpt_every,
                               int32_t prec);
kg_status grape_gradient_columns(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                 const kg_krylov* k, int32_t prec, int32_t n_cols,
                                 const void* psi0s, const void* targets, double* F_dev,
                                 double* beta_dev, double* beta_cols_dev, double* grad_dev,
                                 void* states, int32_t ckpt_every, int32_t centred, void* ws,
                                 size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- reduced basis
 * Sec. III.A: H0 and an S^z control on a mirror-symmetric set of sites conserve
 * the number K of excitations (up spins, zero bits) and the mirror parity
 * Pi: site i <-> L+1-i, so a state that starts in the even-parity part of the
 * K-excitation sector stays there.  That part has one basis vector per orbit
 * {s, Pi s} of the sector's patterns s: (|s> + |Pi s>)/sqrt(2), or |s> when
 * Pi s = s.  Orbits are labelled by their smaller member and ordered by it
 * (ascending binary number, up = 0, the ordering of Sec. III.A); kg_pe_dim
 * gives their number, (C(L, K) + #palindromes) / 2.
 *
 * The _pe entry points take vectors of pe->dim amplitudes in this basis (same
 * element types and alignment as the full-space calls) and compute exactly
 * what their full-space counterparts compute on the embedded vectors: the
 * reduced H v is y_b = d(r_b) x_b + (J/2) sum_p sqrt(n_b / n_a) x_a over the
 * antiparallel bonds p of the label r_b (a the orbit of r_b with bits p, p+1
 * exchanged, n the orbit sizes, d the diagonal of H0 + u Hc).  L may reach
 * KG_PE_MAX_L here; the chain's control must be KG_HC_SZ with hc_sites
 * mirror-symmetric (KG_EINVAL otherwise). */
#define KG_PE_MAX_L 32

/* A built reduced basis.  tables: device memory of kg_pe_tables_bytes,
 * 256-byte aligned, owned by the caller and filled by kg_pe_build (binomial
 * coefficients, orbit labels, the orbit index of every sector pattern by its
 * combinatorial rank); it must stay allocated and unmodified while calls use it. */
typedef struct kg_pe {
  int32_t L;
  int32_t K;
  int64_t dim;
  const void* tables;
} kg_pe;

/* Number of basis vectors for L spins and K excitations (0 for invalid
 * arguments: 2 <= L <= KG_PE_MAX_L, 0 <= K <= L). */
int64_t kg_pe_dim(int32_t L, int32_t K);

/* Bytes of device tables of the basis (0 for invalid arguments). */
size_t kg_pe_tables_bytes(int32_t L, int32_t K);

/* The tables in HOST memory (no device call), kg_pe_tables_bytes long, with
 * R = 4 dim rounded up to a multiple of 256:
 *   byte 0:            binomial coefficients C(n, k), uint32 at [n * 33 + k], n, k <= 32;
 *   byte 4608:         the orbit labels, uint32, dim of them, ascending;
 *   byte 4608 + R:     the combinatorial rank of each label (uint32, dim);
 *   byte 4608 + 2 R:   the orbit index (int32) of every sector pattern s at
 *                      its combinatorial rank sum_i C(z_i, i) over the zero-bit
 *                      positions z_1 < z_2 < ... of s (C(L, K) entries);
 * then, for bases with S = ceil(dim / 64) slices of 64 rows and
 * S * 64 * (L - 1) <= 2^30 (every K up to L = 28), a neighbour table, each section
 * at the next 256-byte boundary:
 *   slot counts:       uint32 per slice, the largest number of antiparallel
 *                      bonds among its labels;
 *   neighbours:        uint32, L - 1 slots per row: slot j of row 64 s + l at
 *                      [(s (L - 1) + j) 64 + l] holds a | c << 30, a the orbit
 *                      reached through the label's j-th antiparallel bond
 *                      (ascending), c = 1, 2, 3 for sqrt(n_b / n_a) = 1,
 *                      sqrt 2, 1/sqrt 2; unused slots hold the row's own index
 *                      with c = 0 (rows past dim: 0).
 * The reduced H v gathers through the neighbour table when it is there and
 * forms the ranks itself otherwise, with the same sums either way.
 * A caller may copy this image to device memory itself and fill a kg_pe with
 * it.  Errors: KG_EINVAL, KG_EWORKSPACE. */
kg_status kg_pe_tables_host(int32_t L, int32_t K, void* tables_host, size_t tables_bytes);

/* kg_pe_tables_host into a host buffer, a synchronous host-to-device copy into
 * tables_dev, and *pe filled.  Errors: KG_EINVAL, KG_EWORKSPACE (tables_bytes
 * too small), KG_EDEVICE. */
kg_status kg_pe_build(int32_t L, int32_t K, void* tables_dev, size_t tables_bytes, kg_pe* pe);

/* Workspace bytes of krylov_expv_pe, grape_forward_pe and grape_gradient_pe:
 * the layout of kg_workspace_bytes with vectors of pe->dim amplitudes;
 * extended = 1 adds the two node vectors of the quadrature and first-order
 * gradients.  0 for invalid arguments. */
size_t kg_pe_workspace_bytes(const kg_pe* pe, const kg_krylov* k, int32_t prec, int32_t extended);

/* Bytes of the forward-state buffer (layout of kg_states_bytes, vectors of
 * pe->dim amplitudes).  0 for invalid arguments. */
size_t kg_pe_states_bytes(const kg_pe* pe, int32_t N, int32_t ckpt_every, int32_t prec);

/* w = (H0 + u Hc) v in the reduced basis (one gather per antiparallel bond).
 * v, w: pe->dim amplitudes, not overlapping.  Errors: KG_EINVAL, KG_EDEVICE. */
kg_status xxz_pe_apply(const kg_xxz* h, const kg_pe* pe, double u, int32_t prec, const void* v,
                       void* w, void* stream);

/* krylov_expv in the reduced basis.  Arguments, workspace rules and errors as
 * krylov_expv (workspace from kg_pe_workspace_bytes). */
kg_status krylov_expv_pe(const kg_xxz* h, const kg_pe* pe, double u, double t, const kg_krylov* k,
                         int32_t prec, const void* v_in, void* v_out, void* ws, size_t ws_bytes,
                         int32_t* m_eff_dev, void* stream);

/* grape_forward in the reduced basis (states from kg_pe_states_bytes). */
kg_status grape_forward_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev, int32_t N,
                           double dt, const kg_krylov* k, int32_t prec, const void* psi0,
                           const void* target, double* F_dev, double* beta_dev, void* states,
                           int32_t ckpt_every, void* ws, size_t ws_bytes, void* stream);

/* Gradients in the reduced basis.  variant selects the full-space entry point
 * it mirrors; nodes is the quadrature's node count (1..KG_MAX_NODES) and must
 * be 0 for the other variants.  The quadrature and first-order variants need
 * the extended workspace (kg_pe_workspace_bytes with extended = 1). */
#define KG_GRAD_ZEROTH 0       /* grape_gradient */
#define KG_GRAD_CENTRED 1      /* grape_gradient_centred */
#define KG_GRAD_FIRST_ORDER 2  /* grape_gradient_first_order */
#define KG_GRAD_QUADRATURE 3   /* grape_gradient_quadrature */
kg_status grape_gradient_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev, int32_t N,
                            double dt, const kg_krylov* k, int32_t prec, const void* psi0,
                            const void* target, double* F_dev, double* beta_dev, double* grad_dev,
                            void* states, int32_t ckpt_every, int32_t states_valid,
                            int32_t variant, int32_t nodes, void* ws, size_t ws_bytes,
                            void* stream);

/* Operator control in the reduced basis: grape_gradient_columns with vectors
 * of pe->dim amplitudes, n_cols state buffers of kg_pe_states_bytes each and
 * the workspace of kg_pe_workspace_bytes (extended = 0). */
kg_status grape_gradient_columns_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev,
                                    int32_t N, double dt, const kg_krylov* k, int32_t prec,
                                    int32_t n_cols, const void* psi0s, const void* targets,
                                    double* F_dev, double* beta_dev, double* beta_cols_dev,
                                    double* grad_dev, void* states, int32_t ckpt_every,
                                    int32_t centred, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- batched form
 * Many independent chains (different L, Delta, N, m) evaluated by one
 * persistent launch: for every chain the forward sweep, the overlap, the
 * backward sweep and the per-slice gradient of Eq. 5 (store-all), in
 * complex64 vectors with FP64 scalars.  Each chain is served by its own team
 * of workgroups [team_first, team_first + team_size); the teams of different
 * chains must not overlap and every team must lie in [0, n_blocks).  The
 * chain's data are addressed by element offsets into the packed arrays:
 *   u_all[off_u .. off_u+N), grad_all[off_u .. off_u+N)        controls, gradient
 *   psi0_all / target_all[off_vec .. off_vec+2^L)              complex64 states
 *   states_all[off_states .. off_states+N*2^L)                 forward states
 *   ws + off_ws (256-aligned), kg_batched_chain_ws_bytes(L, m, team_size) bytes
 * Supported: 10 <= L <= 20 and team_size <= 64. */
typedef struct kg_chain {
  kg_xxz h;
  int32_t N;
  int32_t m;
  int32_t reorth;
  int32_t team_first;
  int32_t team_size;
  int32_t pad_;
  double dt;
  double breakdown_tol;  /* 0: 64 * 2^-23 */
  int64_t off_u;
  int64_t off_vec;
  int64_t off_states;
  int64_t off_ws;
} kg_chain;

/* Scratch bytes of one chain of the batched form. 0 for invalid arguments. */
size_t kg_batched_chain_ws_bytes(int32_t L, int32_t m, int32_t team_size);

/* Sizes of the packed buffers of a planned batch. */
typedef struct kg_batch_plan {
  int64_t u_len;        /* doubles of u_all and grad_all */
  int64_t vec_len;      /* complex64 amplitudes of psi0_all and target_all */
  int64_t states_len;   /* complex64 amplitudes of states_all */
  uint64_t ws_bytes;    /* bytes of the workspace */
  int32_t blocks_used;  /* workgroups covered by the teams (<= n_blocks) */
  int32_t pad_;
} kg_batch_plan;

/* Host-only planning of a batch (no device call).  On input each chains[i]
 * holds h, N, dt, reorth and breakdown_tol, and m (0: choose it) and, with
 * keep_teams = 1, team_size.  The call fills in:
 *   m           where it was 0: the smallest m in [m_min, m_max] for which the
 *               a-priori error bound of the Lanczos approximation of
 *               exp(-i dt H) v (Hochbruck and Lubich, SIAM J. Numer. Anal. 34
 *               (1997), Theorem 2, for a skew-Hermitian argument), with the
 *               spectral radius of H0 + u Hc bounded by Gershgorin's theorem
 *               for |u| <= umax[i], is at most tol / N (m_max if none is).
 *               The paper leaves the dimension to the user and points to
 *               a-posteriori estimates for the choice (App. A);
 *   team_size   with keep_teams = 0: one workgroup per chain, then the chain
 *               with the largest modelled time, 2N m (5 + 0.65 (m + 6)/2
 *               ceil(tiles / team)) microseconds with tiles = 2^L / 1024 (the
 *               lowest index on ties), gets the smallest team that holds
 *               fewer tiles per member, while that stays within
 *               min(max_team, tiles) and the grid of n_blocks workgroups; any
 *               size from 1 to 64 can result;
 *   team_first, off_u, off_vec, off_states, off_ws
 *               the chains packed one after the other in order (workspace
 *               offsets 256-byte aligned);
 * and *plan with the buffer sizes grape_gradient_batched then needs.  umax may
 * be NULL when no m is 0.  Errors: KG_EINVAL. */
kg_status kg_batched_plan(kg_chain* chains, int32_t n_chains, const double* umax, int32_t n_blocks,
                          int32_t max_team, int32_t keep_teams, double tol, int32_t m_min,
                          int32_t m_max, kg_batch_plan* plan);

/* Autotuner of the team shapes: for each cap in caps[0..n_caps) it plans the
 * teams of the chains (kg_batched_plan with keep_teams = 0, max_team = cap and
 * the chains' m), copies the descriptors to chains_dev and times `reps`
 * launches of grape_gradient_batched after one warm-up launch on `stream`
 * (HIP events; ms_out[q] receives the mean time per launch of cap q,
 * nullable).  It then plans the fastest cap into chains_host and chains_dev,
 * writes it to *best_cap, and synchronises the stream before it returns (the
 * one synchronous call of the batched form).  The buffers are those of
 * grape_gradient_batched; ws must hold the plan of the largest cap.  The
 * results in F_all, beta_all and grad_all are those of the last timed launch.
 * Errors: KG_EINVAL, KG_EWORKSPACE, KG_EDEVICE. */
kg_status kg_batched_autotune(kg_chain* chains_host, kg_chain* chains_dev, int32_t n_chains,
                              int32_t n_blocks, const int32_t* caps, int32_t n_caps, int32_t reps,
                              const double* u_all, int64_t u_len, const void* psi0_all,
                              const void* target_all, int64_t vec_len, void* states_all,
                              int64_t states_len, double* F_all, double* beta_all,
                              double* grad_all, void* ws, size_t ws_bytes, int32_t* status_dev,
                              float* ms_out, int32_t* best_cap, void* stream);

/* F and dF/du for n_chains chains in one persistent launch.  chains_host holds
 * the descriptors for validation on the host; chains_dev is the same array in
 * device memory, read by the kernel (keep the two identical).  Array lengths:
 * u_len doubles in u_all and grad_all, vec_len amplitudes in psi0_all and
 * target_all, states_len amplitudes in states_all, ws_bytes in ws.  n_blocks
 * is the size of the persistent grid (at most the number of compute units, so
 * that every team is resident at once).  F_all[c] = |beta_c|^2, beta_all[2c],
 * beta_all[2c+1] = beta_c.  *status_dev becomes nonzero if a team barrier
 * timed out (the results are then invalid).  Errors: KG_EINVAL, KG_EWORKSPACE,
 * KG_EDEVICE. */
kg_status grape_gradient_batched(const kg_chain* chains_host, const kg_chain* chains_dev,
                                 int32_t n_chains, int32_t n_blocks, const double* u_all,
                                 int64_t u_len, const void* psi0_all, const void* target_all,
                                 int64_t vec_len, void* states_all, int64_t states_len,
                                 double* F_all, double* beta_all, double* grad_all, void* ws,
                                 size_t ws_bytes, int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------- diagnostics
 * Integer index maps of H0 for s = s0 .. s0+count-1 (L <= 30):
 *   n_anti[i]       = number of antiparallel nearest-neighbour bonds of s,
 *   partner_mask[i] = bit p set <=> bond (p, p+1) is antiparallel, i.e. the
 *                     hopping term couples s to s ^ (3 << p).
 * Device outputs.  Errors: KG_EINVAL, KG_EDEVICE. */
kg_status kg_debug_index_map(int32_t L, uint32_t s0, uint32_t count, int32_t* n_anti_dev,
                             uint32_t* partner_mask_dev, void* stream);

/* Sampled kernel timing, for benchmarks (not thread-safe, one session at a
 * time).  Between kg_profile_begin and kg_profile_end, every sample_every-th
 * Krylov call (and every sample_every-th overlap, bracket and xxz_apply
 * launch) records a pair of HIP events on its stream around each kernel, for
 * at most max_launches kernels.  kg_profile_end waits for the last event and
 * fills, per kernel class (KG_PROF_NCLASS entries each; NULL skips an array):
 * launches timed, summed duration in ms, and summed algorithmic bytes
 * (vectors each kernel must read and write once, no cache re-reads).
 * Errors: KG_EINVAL, KG_EDEVICE. */
#define KG_PROF_PASS_A 0    /* Lanczos pass A: H v_k and the projection dots */
#define KG_PROF_PASS_B 1    /* Lanczos pass B: new basis vector and its norm */
#define KG_PROF_COMBINE 2   /* v_out = beta0 V^T exp(-itT) e_1 */
#define KG_PROF_BRACKET 3   /* gradient bracket <lambda|Hc|psi> */
#define KG_PROF_OVERLAP 4   /* <f|psi_N> */
#define KG_PROF_HV 5        /* xxz_apply */
#define KG_PROF_NCLASS 6
kg_status kg_profile_begin(int32_t sample_every, int32_t max_launches);
kg_status kg_profile_end(int64_t* launches, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* KGRAPE_H */
