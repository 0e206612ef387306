// Internal interface between the C-ABI layer (kg_capi.cpp) and the HIP kernels
// (kg_kernels.hip).  Not installed; the public interface is include/kgrape.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace kg {

constexpr int kMaxM = 64;          // largest Krylov dimension
// reduction scalars per pass: two per window vector, two of the new vector,
// the norm carried from pass B to pass A
constexpr int kMaxScal = 2 * kMaxM + 3;
constexpr int kMaxGrid = 2048;     // largest grid of the reducing kernels
constexpr int kPartialRows = kMaxGrid + kMaxGrid / 64;  // block rows + group rows
// largest grid of the Lanczos passes: every block of pass B reads the pass A
// partials of all of them (32 bytes a row), so the grid stays at 512 blocks
// unless the vector has at least kLzManyTiles tiles, where kLzGridLarge blocks
// stream it faster (Krylov calls at L=23 and 24, complex64: 3 and 4.5 %)
constexpr int kLzGrid = 512;
// The Infinity Cache (memory-side cache) of the MI355X.  A Krylov basis of m
// vectors well beyond it is streamed from HBM at every step, and the
// streaming passes (pass B, the combination) then load it nontemporally.
// Timed forward sweeps per Krylov call, plain against nontemporal loads:
// complex64 m=20 L=22 (671 MB basis) 2.29 -> 2.21 ms, m=24 L=23 6.33 -> 5.87
// ms, L=24 12.75 -> 11.56 ms; complex128 L=22 4.48 -> 4.04 ms, m=24 L=24
// 24.4 -> 22.5 ms; but with a basis of 336 MB, partly held by the cache
// (complex64 L=21, complex128 L=20), 1.12 -> 1.17 and 1.08 -> 1.10 ms.
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;
inline bool streamed_past_cache(int m, uint32_t D, size_t amp_bytes) {
  return (size_t)m * D * amp_bytes > 2 * kInfinityCacheBytes;
}
constexpr int kLzGridLarge = 2048;
constexpr uint32_t kLzManyTiles = 4096;

struct cplx_d {                    // complex FP64 with a fixed layout
  double re, im;
};

// Scalars of one Krylov call, resident in device memory.  offd[k] couples
// v_{k-1} and v_k (offd[0] = 0); scale[k] = 1/||stored vector k||.  Fields
// that step k reads from step k-1 while step k's own values are written in
// the same launch are kept twice, by the parity of the step.
struct KState {
  double alpha[kMaxM];
  double offd[kMaxM + 1];
  double scale[kMaxM + 1];
  cplx_d coef[2][kMaxM];  // projection coefficients of step k (window order), at k & 1
  cplx_d dcomb[kMaxM];    // combination coefficients beta0 * c_j * scale_j
  // c^(i)_i and c^(i)_{i-1} of every step i (projection coefficients on the
  // stored vector itself and on its predecessor)
  cplx_d cdiag[kMaxM];
  cplx_d csub[kMaxM];
  cplx_d gcol[2][kMaxM];  // measured Gram columns <u_j|u_p>, by the parity of p
  double beta0;
  double normT[2];        // max_{i<=k}(|alpha_i| + offd_i), at k & 1
  int32_t m_eff;
  int32_t done;           // basis complete (normal end, breakdown or zero input)
  int32_t pad_[2];
  // GRAPE scalars
  cplx_d overlap;         // beta = <f|psi_N>
  double fid;
  double g0;              // centred gradient: the bracket at the start of slice 1
  uint32_t counters[kMaxGrid / 64 + 4];  // arrivals in the running grid reduction
  // totals of pass B(k-1)'s measurement columns (window order) and, after
  // them, of its norm column, summed by helper wavefronts of pass A(k)
  cplx_d colsum[kMaxScal];
};

struct HvArgs {            // the Hamiltonian H0 + u Hc of one chain
  int32_t L;
  int32_t hc_kind;         // 0: S^x on one site, 1: sum of S^z
  int32_t hc_bit;          // flipped bit of the S^x control (L - site)
  int32_t sz_count;        // number of S^z control sites
  uint32_t sz_mask;        // bits of the S^z control sites
  int32_t pad_;
  double half_J;           // J/2 (hopping amplitude)
  double c_zz;             // J*Delta/4 (diagonal unit)
  const double* u_ptr;     // control amplitude in device memory, or nullptr
  double u_val;            // control amplitude used when u_ptr == nullptr
};

struct Geo {               // tiling of one state vector
  int32_t L;
  int32_t TB;              // tile = 2^TB amplitudes, staged in LDS
  int32_t RB;              // 2^RB amplitudes per thread
  int32_t WB;              // 2^WB wavefronts per block
  uint32_t D;
  uint32_t ntiles;
  int32_t small;           // D < 2^TB: amplitudes past D are masked
  int32_t grid;            // blocks of the tiled kernels
};

// Tiling of a 2^L vector; grid_cap bounds the grid (kLzGrid for the Lanczos
// passes, kMaxGrid for a standalone H v); `standalone` allows the larger
// complex64 tile of the standalone H v.
Geo make_geo(int L, int prec, int tile_bits_override, int grid_cap = kLzGrid,
             bool standalone = false);
int stream_grid(uint32_t D);

struct Workspace {         // carved from the caller's workspace
  KState* st;
  cplx_d* partials;        // [kMaxScal][kPartialRows]: column major, one row per block
  void* basis;             // m-1 vectors (stored Krylov vectors 1..m-1)
  void* yk;                // one vector: y_k = H v_k of the running step
  void* lam;               // one vector (costate)
  void* node_a;            // quadrature workspaces only: psi at a node
  void* node_b;            //   and lambda at the node
};

size_t ws_fixed_bytes();
size_t vec_bytes(int L, int prec);

// ---- sampled kernel timing (kg_profile_begin / kg_profile_end)
enum ProfClass { kProfPassA = 0, kProfPassB, kProfCombine, kProfBracket, kProfOverlap, kProfHv, kProfN };
struct Profiler;
// Non-null while profiling is active and the current Krylov call is sampled.
Profiler* profiler_for_call();
Profiler* profiler_for_launch();
// profiler_start arms a pair of events for the next sampled launch, which
// takes them with profiler_take and passes them to the dispatch itself
// (hipExtLaunchKernel: the kernel's own start and end, as a kernel trace
// records them); profiler_stop files the record if a launch took them.
void profiler_start(Profiler* p, hipStream_t s);
void profiler_stop(Profiler* p, hipStream_t s, int cls, double bytes);
bool profiler_take(hipEvent_t* e0, hipEvent_t* e1);

// ---- launchers (kg_kernels.hip); all enqueue on `s` and return hipSuccess or the launch error
hipError_t launch_hv(int prec, const HvArgs& a, const Geo& g, const void* v, void* w, hipStream_t s);

// The fixed-excitation, parity-even basis (device tables built by kg_pe_build).
struct PeArgs {
  const uint32_t* reps;    // orbit representatives (bit patterns), ascending
  const uint32_t* ranks;   // combinatorial rank of each representative
  const int32_t* index;    // basis index of a sector state's orbit, by combinatorial rank
  const uint32_t* binom;   // C(n, k) at [n * kPeBinom + k], n, k <= 32
  // neighbour table (nullptr when the basis has none, see kPeNbrMaxEntries):
  // slot counts per slice of 64 rows, and slot j of row 64 s + l at
  // nbr[(s * nbr_slots + j) * 64 + l] = orbit | weight code << 30
  const uint32_t* scnt;
  const uint32_t* nbr;
  int32_t nbr_slots;       // L - 1 when the table is there
  int32_t L, K;
  uint32_t dim;
  uint32_t nsec;           // C(L, K): entries of `index`
};
constexpr int kPeBinom = 33;
// The neighbour table is built for bases whose table has at most this many
// slots (64 per slice and bond: 4 GiB); beyond, H v forms the ranks itself.
constexpr uint64_t kPeNbrMaxEntries = 1ull << 30;
// Algorithmic bytes of one reduced-basis H v on vectors of vb bytes.
double pe_gather_bytes(const PeArgs& p, double vb);

struct KrylovCall {
  HvArgs hv;
  Geo geo;
  const PeArgs* pe = nullptr;  // reduced basis (nullptr: full 2^L space)
  int prec;
  int m;
  int reorth;
  double t;
  double tol;
  const void* v_in;
  void* v_out;
  int32_t* m_eff_out;      // nullable
};
hipError_t launch_krylov(const KrylovCall& c, const Workspace& ws, hipStream_t s);
// Two independent calls of the same L, m, reorth and precision in the same launches.
hipError_t launch_krylov_pair(const KrylovCall& c0, const Workspace& w0, const KrylovCall& c1,
                              const Workspace& w1, hipStream_t s);

hipError_t launch_overlap(int prec, uint32_t D, const void* f, const void* psi, const Workspace& ws,
                          double* F_dev, double* beta_dev, hipStream_t s);
hipError_t launch_bracket(int prec, const HvArgs& a, uint32_t D, const void* lam, const void* psi,
                          double dt, const double* beta_dev, const Workspace& ws, double* grad_slot,
                          hipStream_t s, bool accumulate = false, double coef_im = 0.0,
                          const uint32_t* pe_reps = nullptr);
hipError_t launch_hv_pe(int prec, const HvArgs& a, const PeArgs& p, const void* v, void* w,
                        hipStream_t s);
hipError_t launch_init(KState* st, hipStream_t s);

// Scratch of krylov_expv_static (kg_static.hip): a device array of this many
// bytes per GPU; *ptr receives its device address on the current device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
hipError_t static_scratch(void** ptr);
hipError_t launch_ascent(double* u, const double* g, int N, double eta, hipStream_t s);
hipError_t launch_centre(double* g, int N, const double* g0, hipStream_t s);
hipError_t launch_mean_overlap(const double* beta_cols, int n, double* beta, double* F,
                               hipStream_t s);

// batched persistent form (kg_batched.hip); kg_chain comes from kgrape.h
}  // namespace kg
struct kg_chain;
namespace kg {
size_t batched_chain_ws_bytes(int L, int m, int team);
hipError_t launch_batched(const kg_chain* chains_dev, int n_chains, int n_blocks, const double* u_all,
                          const void* psi0_all, const void* target_all, void* states_all,
                          double* F_all, double* beta_all, double* grad_all, void* ws,
                          int32_t* status, hipStream_t s);
hipError_t launch_index_map(int L, uint32_t s0, uint32_t count, int32_t* n_anti, uint32_t* pmask,
                            hipStream_t s);

}  // namespace kg
