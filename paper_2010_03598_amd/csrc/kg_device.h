// Device helpers shared by the HIP translation units of libkgrape: wavefront
// and grid reductions, the tridiagonal exponential, and H v on a tile.
// Internal; included only by kg_kernels.hip and kg_batched.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "kg_internal.h"

namespace kg {
namespace {

template <typename R>
struct VT;
template <>
struct VT<float> {
  using T = float2;
};
template <>
struct VT<double> {
  using T = double2;
};

// ---------------------------------------------------------------------- helpers

// v read from another lane by a DPP move (both 32-bit halves); lanes outside
// ROW_MASK receive +0.0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same value in every lane.  DPP steps in a fixed
// order: pairs and quads (quad permutations), rows of 16 (row rotations by 4
// and 8), then the row broadcasts of lanes 15 and 31 carry the partial sums
// up to lane 63, whose value is broadcast.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);       // row_ror:4
  v += dpp_f64<0x128>(v);       // row_ror:8
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sums of four values over the 64 lanes of a wavefront at once; lane l
// returns the total of v[l mod 4].  Two halving exchanges within quads (the
// lane keeps the half its index bit selects and adds the partner's copy of
// it), then sums over the other index bits: rotations by 4 and 8 inside rows
// of 16 lanes (they keep l mod 4), then exchanges with lane l ^ 16 and
// l ^ 32.  The order of the additions is fixed.  About a third of the
// instructions of four wave_sum calls.
__device__ __forceinline__ double quad_sums_within_rows(double v0, double v1, double v2,
                                                        double v3) {
  const int lane = threadIdx.x & 63;
  // bit 1: lanes with the bit set keep values 2, 3
  const bool b1 = (lane >> 1) & 1;
  const double s0 = b1 ? v0 : v2, s1 = b1 ? v1 : v3;
  double k0 = (b1 ? v2 : v0) + dpp_f64<0x4E>(s0);   // quad_perm [2,3,0,1]
  double k1 = (b1 ? v3 : v1) + dpp_f64<0x4E>(s1);
  // bit 0: lanes with the bit set keep the second of the two
  const bool b0 = lane & 1;
  double t = (b0 ? k1 : k0) + dpp_f64<0xB1>(b0 ? k0 : k1);   // quad_perm [1,0,3,2]
  t += dpp_f64<0x124>(t);   // row_ror:4
  t += dpp_f64<0x128>(t);   // row_ror:8
  return t;
}

// The exchanges across rows through LDS permutes (ds_bpermute).
__device__ __forceinline__ double quad_sums(double v0, double v1, double v2, double v3) {
  double t = quad_sums_within_rows(v0, v1, v2, v3);
  t += __shfl_xor(t, 16, 64);
  t += __shfl_xor(t, 32, 64);
  return t;
}

// Two quad_sums with one exchange across rows: lane l returns the total of
// a[l mod 4] where bit 2 of l is clear and of b[l mod 4] where it is set
// (after the sums within rows every lane of a row holds its row's totals, so
// half of a row can carry b).  Faster in the batched kernel; in pass B of the
// tiled form it made the step slower.
__device__ __forceinline__ double quad_sums_pair(double a0, double a1, double a2, double a3,
                                                 double b0, double b1, double b2, double b3) {
  const double ta = quad_sums_within_rows(a0, a1, a2, a3);
  const double tb = quad_sums_within_rows(b0, b1, b2, b3);
  double t = ((threadIdx.x >> 2) & 1u) ? tb : ta;
  t += __shfl_xor(t, 16, 64);
  t += __shfl_xor(t, 32, 64);
  return t;
}

// v of lane l ^ 16 (l ^ 32) by the lane-swap instructions, no LDS.  Called
// with both operands equal, permlane16_swap returns {lanes of odd rows take
// the even row below, lanes of even rows keep theirs} and {even rows take the
// odd row above, odd rows keep theirs}; permlane32_swap the same with the
// wavefront's two halves.
__device__ __forceinline__ double xor_lanes_16(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const bool up = (threadIdx.x & 16) != 0;
  return __hiloint2double((int)(up ? b[0] : b[1]), (int)(up ? a[0] : a[1]));
}
__device__ __forceinline__ double xor_lanes_32(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const bool up = (threadIdx.x & 32) != 0;
  return __hiloint2double((int)(up ? b[0] : b[1]), (int)(up ? a[0] : a[1]));
}

// quad_sums with the exchanges across rows by lane swaps.  Faster in the
// one-block Krylov call; in the tiled passes it made the Lanczos step slower
// (the LDS-permute form stays there).
__device__ __forceinline__ double quad_sums_swap(double v0, double v1, double v2, double v3) {
  double t = quad_sums_within_rows(v0, v1, v2, v3);
  t += xor_lanes_16(t);
  t += xor_lanes_32(t);
  return t;
}

// p[s] when `ok`, else zero.  The load is always issued (at index 0 when not
// `ok`, so it stays in bounds) and the value masked afterwards.
template <typename V>
__device__ __forceinline__ V ld_masked(const V* p, uint32_t s, bool ok) {
  const V v = p[ok ? s : 0u];
  return ok ? v : V{0, 0};
}

// A nontemporal load of one amplitude (complex64 or complex128): for vectors
// streamed once per pass whose whole set does not fit in the Infinity Cache,
// so that they do not displace lines that will be read again.
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  if constexpr (sizeof(V) == 8) {
    typedef float e2 __attribute__((ext_vector_type(2)));
    const e2 t = __builtin_nontemporal_load(reinterpret_cast<const e2*>(p));
    V o;
    o.x = t.x;
    o.y = t.y;
    return o;
  } else {
    typedef double e2 __attribute__((ext_vector_type(2)));
    const e2 t = __builtin_nontemporal_load(reinterpret_cast<const e2*>(p));
    V o;
    o.x = t.x;
    o.y = t.y;
    return o;
  }
}

// The same for two neighbouring complex64 amplitudes (16 bytes, aligned).
__device__ __forceinline__ float4 ld_stream4(const float4* p) {
  typedef float e4 __attribute__((ext_vector_type(4)));
  const e4 t = __builtin_nontemporal_load(reinterpret_cast<const e4*>(p));
  return float4{t.x, t.y, t.z, t.w};
}

// The NR amplitudes p[s0 | r << 6] of a thread's slots in a tile.  `full`
// (the whole tile lies inside the vector) must be the same for the whole
// block: then the loads are plain and unconditional, so the compiler issues
// them together; a per-lane bound test around each load makes it wait for
// each one in turn.  Slots at or past D read as zero.
template <typename V, int NR>
__device__ __forceinline__ void load_slots(const V* p, uint32_t s0, bool full, uint32_t D,
                                           V (&out)[NR]) {
  if (full) {
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r] = p[s0 | ((uint32_t)r << 6)];
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t s = s0 | ((uint32_t)r << 6);
      out[r] = ld_masked(p, s, s < D);
    }
  }
}

// The value of lane l (a wavefront-uniform l), in every lane.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Maximum over the 64 lanes of values >= 0 (a lane outside a DPP source
// reads +0.0), the same value in every lane: the DPP steps of wave_sum.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x124>(v));
  v = fmax(v, dpp_f64<0x128>(v));
  v = fmax(v, dpp_f64<0x142, 0xA>(v));
  v = fmax(v, dpp_f64<0x143, 0xC>(v));
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Vector element loads and stores that are coherent across the XCDs' L2
// caches (device-scope atomics in 8-byte pieces): the channel through which
// the workgroups of a team exchange amplitudes inside one launch.
template <typename V>
__device__ __forceinline__ V ld_coh(const V* p) {
  static_assert(sizeof(V) == 8 || sizeof(V) == 16, "complex64 or complex128 amplitudes");
  const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
  uint64_t b[sizeof(V) / 8];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(V) / 8); ++i)
    b[i] = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  V v;
  __builtin_memcpy(&v, b, sizeof(V));
  return v;
}

template <typename V>
__device__ __forceinline__ void st_coh(V* p, const V& v) {
  uint64_t b[sizeof(V) / 8];
  __builtin_memcpy(b, &v, sizeof(V));
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(V) / 8); ++i)
    __hip_atomic_store(q + i, b[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A load of a partner amplitude: plain, or coherent when other workgroups of
// the same launch wrote it (kCoh).
template <bool kCoh, typename V>
__device__ __forceinline__ V ld_partner(const V* p) {
  if constexpr (kCoh) {
    return ld_coh(p);
  } else {
    return *p;
  }
}

__device__ __forceinline__ void st_agent_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Make this wavefront's device-coherent stores complete before what follows.
__device__ __forceinline__ void complete_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Columns j of a partials table summed over `cnt` rows.  The table is column
// major (column stride kPartialRows, one row per block): j < ns from `cols`,
// j == ns (when `xcol` is given) from `xcol`.  Columns j < c_plain and `xcol`
// were written by an earlier launch and are read with plain 16-byte loads;
// the others, written by blocks of this launch, with device-scope loads.
// Lane l adds rows l, l+64, ... in order, then a fixed butterfly; the block's
// wavefronts share the columns.  The loads of a batch of JB columns (RPL rows
// per lane each) are all issued before any is used: one memory round trip per
// batch.
template <int RPL, int JB>
__device__ void sum_rows_t(const cplx_d* cols, uint32_t cnt, int ns, const cplx_d* xcol,
                           int c_plain, cplx_d* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nc = ns + (xcol ? 1 : 0);
  for (int j0 = wv; j0 < nc; j0 += nw * JB) {
    double re[JB], im[JB];
#pragma unroll
    for (int c = 0; c < JB; ++c) re[c] = im[c] = 0.0;
    for (uint32_t b0 = 0; b0 < cnt; b0 += RPL * 64) {
      double pr[JB][RPL], pi[JB][RPL];
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        const int j = j0 + c * nw;
        const cplx_d* base = (j < ns) ? cols + (size_t)j * kPartialRows : xcol;
        const bool plain = j < c_plain || j == ns;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const uint32_t r = min(b0 + q * 64 + lane, cnt - 1);
          if (j >= nc) {
            pr[c][q] = pi[c][q] = 0.0;
          } else if (plain) {
            const cplx_d v = base[r];
            pr[c][q] = v.re;
            pi[c][q] = v.im;
          } else {
            pr[c][q] = ld_agent(&base[r].re);
            pi[c][q] = ld_agent(&base[r].im);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < JB; ++c) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const bool in = (b0 + q * 64 + lane) < cnt;
          re[c] += in ? pr[c][q] : 0.0;
          im[c] += in ? pi[c][q] : 0.0;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < JB; ++c) {
      const int j = j0 + c * nw;
      const double sr = wave_sum(re[c]);
      const double si = wave_sum(im[c]);
      if (j < nc && lane == 0) tot[j] = cplx_d{sr, si};
    }
  }
}

// sum_rows_t with the batch shape chosen for the row count: about 16 loads
// in flight per lane.
__device__ void sum_rows(const cplx_d* cols, uint32_t cnt, int ns, const cplx_d* xcol, int c_plain,
                         cplx_d* tot) {
  if (cnt <= 64) {
    sum_rows_t<1, 8>(cols, cnt, ns, xcol, c_plain, tot);
  } else if (cnt <= 128) {
    sum_rows_t<2, 4>(cols, cnt, ns, xcol, c_plain, tot);
  } else if (cnt <= 256) {
    sum_rows_t<4, 2>(cols, cnt, ns, xcol, c_plain, tot);
  } else {
    sum_rows_t<8, 1>(cols, cnt, ns, xcol, c_plain, tot);
  }
}

// Count this block's arrival; true in the block that arrives last of `cnt`.
__device__ bool arrive_last(uint32_t* counter, uint32_t cnt) {
  __shared__ int last;
  const int lane = threadIdx.x & 63;
  if ((threadIdx.x >> 6) == 0) {
    complete_stores();
    uint32_t prev = 0;
    if (lane == 0)
      prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = __shfl(prev, 0, 64);
    if (lane == 0) last = (prev == cnt - 1);
  }
  __syncthreads();
  if (!last) return false;
  if (threadIdx.x == 0) st_agent_u32(counter, 0u);
  return true;
}

// largest grid reduced in one level: one block summing 635 rows beat the
// two levels by 1.7 % per reduced-basis gradient (635 tiles); at 1024 rows
// the two levels were ahead
constexpr uint32_t kReduceFlat = 768;
constexpr uint32_t kGroup = 64;        // blocks per group of the two-level reduction

// Deterministic grid-wide sum of `ns` complex FP64 values.  Every block
// passes its block totals in `tot` (LDS); `b` is the block's index among the
// G blocks that reduce together.  Returns true in exactly one block, the last
// to arrive, with the grid totals in `tot`.  Up to kReduceFlat blocks the last
// block adds all partials; larger grids add groups of kGroup blocks first (the
// last block of each group), then the groups.  The order is fixed, so results
// do not depend on which block arrives last.  The partials table is column
// major: value (column j, block b) at partials[j * kPartialRows + b].  When
// `xcol` is given (one value per block, written by an earlier launch) its sum
// over the G blocks lands in tot[ns] by the same scheme.  With c0 > 0 this
// launch formed only columns [c0, ns): each block writes those, and columns
// [0, c0) were written by an earlier launch; the sums cover all columns.
//
// The partials of this launch travel only through device-scope (sc1) stores
// and loads, which are coherent across the XCDs' L2 caches; the stores are
// waited for before the arrival counter is incremented.  No device-wide fence
// is needed, so the L2 caches are never written back or invalidated here.
// counters[0] counts the top level, counters[1 + g] group g.
__device__ bool grid_reduce(cplx_d* tot, int ns, cplx_d* partials, uint32_t* counters, uint32_t b,
                            uint32_t G, const cplx_d* xcol = nullptr, int c0 = 0) {
  const int lane = threadIdx.x & 63;
  if (G == 1) {
    for (int j = threadIdx.x; j < c0; j += blockDim.x) tot[j] = partials[(size_t)j * kPartialRows];
    if (xcol && threadIdx.x == 0) tot[ns] = xcol[0];
    __syncthreads();
    return true;
  }
  if ((threadIdx.x >> 6) == 0) {
    for (int j = c0 + lane; j < ns; j += 64) {
      st_agent(&partials[(size_t)j * kPartialRows + b].re, tot[j].re);
      st_agent(&partials[(size_t)j * kPartialRows + b].im, tot[j].im);
    }
  }
  if (G <= kReduceFlat) {
    if (!arrive_last(&counters[0], G)) return false;
    sum_rows(partials, G, ns, xcol, c0, tot);
    __syncthreads();
    return true;
  }
  const uint32_t grp = b / kGroup, ngrp = (G + kGroup - 1) / kGroup;
  const uint32_t gsize = min(kGroup, G - grp * kGroup);
  if (!arrive_last(&counters[1 + grp], gsize)) return false;
  sum_rows(partials + (size_t)grp * kGroup, gsize, ns, xcol ? xcol + (size_t)grp * kGroup : nullptr,
           c0, tot);
  __syncthreads();
  // group totals (and the extra column's, in column ns) go to rows [G, G + ngrp)
  const int nc = ns + (xcol ? 1 : 0);
  if ((threadIdx.x >> 6) == 0) {
    for (int j = lane; j < nc; j += 64) {
      st_agent(&partials[(size_t)j * kPartialRows + G + grp].re, tot[j].re);
      st_agent(&partials[(size_t)j * kPartialRows + G + grp].im, tot[j].im);
    }
  }
  if (!arrive_last(&counters[0], ngrp)) return false;
  sum_rows(partials + G, ngrp, nc, nullptr, 0, tot);
  __syncthreads();
  return true;
}

// Sum the per-wavefront accumulators wacc[w * kMaxScal + j], j in [c0, ns), of
// a block in wavefront order.
__device__ void block_totals(const cplx_d* wacc, int ns, cplx_d* tot, int c0 = 0) {
  const int nw = blockDim.x >> 6;
  for (int j = c0 + (int)threadIdx.x; j < ns; j += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int q = 0; q < nw; ++q) {
      re += wacc[q * kMaxScal + j].re;
      im += wacc[q * kMaxScal + j].im;
    }
    tot[j] = cplx_d{re, im};
  }
  __syncthreads();
}

// exp(-i t T) e_1 for the real symmetric tridiagonal T held row by row in the
// lanes of one wavefront (lane i: diagonal a, couplings lo = T[i][i-1] and
// hi = T[i][i+1]; rows past the dimension are zero).  Scaled Taylor series:
// the step is split into nsub pieces with |t/nsub| ||T||_inf <= 1/2 and each
// piece uses 16 terms (remainder below 2^-17/17! relative).
// Beyond kMaxSubsteps pieces (|t| ||T||_inf > kMaxSubsteps / 2, or a
// non-finite T or t) the result is NaN: the loop stays bounded whatever the
// entries.
constexpr double kMaxSubsteps = 65536.0;
__device__ void tri_exp_wave(double a, double lo, double hi, double t, double& cr, double& ci) {
  const int lane = threadIdx.x & 63;
  const double nrm = wave_max(fabs(a) + lo + hi);
  const double want = ceil(fabs(t) * nrm * 2.0);
  if (!(want <= kMaxSubsteps)) {
    cr = ci = NAN;
    return;
  }
  const int nsub = want < 1.0 ? 1 : (int)want;
  const double tau = t / (double)nsub;
  double yr = (lane == 0) ? 1.0 : 0.0, yi = 0.0;
  for (int step = 0; step < nsub; ++step) {
    double tr = yr, ti = yi, ar = yr, ai = yi;
#pragma unroll 4
    for (int p = 1; p <= 16; ++p) {
      // neighbours by DPP wavefront shifts: lane i reads lane i-1 (wave_shr:1)
      // and lane i+1 (wave_shl:1); the lanes at the ends read 0, where the
      // matching off-diagonal entry is 0 anyway
      const double dr = dpp_f64<0x138>(tr), di = dpp_f64<0x138>(ti);
      const double ur = dpp_f64<0x130>(tr), ui = dpp_f64<0x130>(ti);
      const double zr = a * tr + lo * dr + hi * ur;
      const double zi = a * ti + lo * di + hi * ui;
      const double c = tau / (double)p;
      tr = c * zi;
      ti = -c * zr;
      ar += tr;
      ai += ti;
    }
    yr = ar;
    yi = ai;
  }
  cr = yr;
  ci = yi;
}

// ---------------------------------------------------------------------- Lanczos window dots

// KState values of the earlier steps that the scalar update of step k reads,
// staged in LDS by wavefront 0 (all written by earlier launches).
struct FinScalars {
  double alpha[kMaxM];
  double offd[kMaxM];
  double scale[kMaxM];
  cplx_d coef[kMaxM];    // step k-1's projection coefficients (window order)
  cplx_d gprev[kMaxM];   // the Gram column measured two steps back
  cplx_d cdiag[kMaxM];
  cplx_d csub[kMaxM];
  double normT, beta0;
};

// The window dots of step k, d_i = <u_i|H u_k> for i in [i0, k), on wavefront
// 0 (lane l: i = i0 + l), without reading a window vector.  u_i are the stored
// (unnormalised) vectors, s_i = 1/||u_i|| and c^(i) the projection
// coefficients of step i, so that pass B(i) stored
//   u_{i+1} = s_i y_i - sum_j c^(i)_j u_j,   y_i = H u_i.
// As H is Hermitian, d_i = <y_i|u_k> = (e_{i+1} + sum_j conj(c^(i)_j) e_j) / s_i
// with e_j = <u_j|u_k>; and with p = k-1,
//   e_j = s_p <u_j|y_p> - sum_l c^(p)_l G_jl,   e_k = ||u_k||^2,
// where G_jl = <u_j|u_l>.  Pass B(p) measured <u_j|y_p> (columns [0, nb)) and
// G_jp (columns [nb, 2nb)) on the stored vectors, and pass B(p-1) the column
// G_{j,p-1}.  In a re-orthogonalised basis the entries G_jl (j != l) and the
// coefficients c^(i)_j (j < i-1) are of the order of the rounding error, so
// the products of two of them are dropped: the sums keep l in {j, p-1, p} and
// j in {i-1, i}, which are all the terms of the three-term window.  In exact
// arithmetic the dots are exact either way (G is then diagonal).  k, i0 and
// i0p are the step and the first indices of its window and of step k-1's; the
// measured column G_jp goes to gcol_out[j] (nullable), for step k+1.
__device__ cplx_d window_dots(int k, int i0, int i0p, const FinScalars& fs, const cplx_d* tot,
                              int nb, double ekk, cplx_d* gcol_out) {
  const int lane = threadIdx.x & 63;
  const int p = k - 1, ip = i0p;
  const int j = ip + lane;
  const bool has_pm = p - 1 >= ip;
  // step p's coefficients and the stored scalars
  const cplx_d cp = fs.coef[p - ip];
  const cplx_d cpm = has_pm ? fs.coef[p - 1 - ip] : cplx_d{0.0, 0.0};
  const double sp = fs.scale[p];
  double er = 0.0, ei = 0.0;
  if (lane < nb) {
    const cplx_d cj = fs.coef[lane];
    const double sj = fs.scale[j];
    const cplx_d gjp = tot[nb + lane];
    cplx_d gjm{0.0, 0.0};   // G_{j,p-1}
    if (has_pm) {
      if (j == p) {
        gjm = tot[nb + (p - 1 - ip)];
        gjm.im = -gjm.im;
      } else if (j == p - 1) {
        gjm = cplx_d{1.0 / (sj * sj), 0.0};
      } else {
        gjm = fs.gprev[j];   // gcol[(p - 1) & 1], staged
      }
    }
    er = sp * tot[lane].re - (cp.re * gjp.re - cp.im * gjp.im) -
         (cpm.re * gjm.re - cpm.im * gjm.im);
    ei = sp * tot[lane].im - (cp.re * gjp.im + cp.im * gjp.re) -
         (cpm.re * gjm.im + cpm.im * gjm.re);
    if (j < p - 1) {
      const double gjj = 1.0 / (sj * sj);
      er -= cj.re * gjj;
      ei -= cj.im * gjj;
    }
    if (gcol_out) gcol_out[j] = gjp;   // for step k+1
  } else if (lane == nb) {
    er = ekk;   // j = k
  }
  // lane l: i = i0 + l takes e_{i+1}, e_i and e_{i-1} from lanes i+1-ip, i-ip, i-1-ip
  const int i = i0 + lane;
  const bool want = i < k;
  const int src = i - ip;
  const double e1r = __shfl(er, min(max(src + 1, 0), 63), 64);
  const double e1i = __shfl(ei, min(max(src + 1, 0), 63), 64);
  const double e0r = __shfl(er, min(max(src, 0), 63), 64);
  const double e0i = __shfl(ei, min(max(src, 0), 63), 64);
  const double emr = __shfl(er, min(max(src - 1, 0), 63), 64);
  const double emi = __shfl(ei, min(max(src - 1, 0), 63), 64);
  if (!want) return cplx_d{0.0, 0.0};
  const cplx_d cd = fs.cdiag[i];
  double dr = e1r + cd.re * e0r + cd.im * e0i;
  double di = e1i + cd.re * e0i - cd.im * e0r;
  if (i >= 1 && i - 1 >= ip) {
    const cplx_d cs = fs.csub[i];
    dr += cs.re * emr + cs.im * emi;
    di += cs.re * emi - cs.im * emr;
  }
  const double si = fs.scale[i];
  return cplx_d{dr / si, di / si};
}

// ---------------------------------------------------------------------- H v on a tile

template <typename R, int RB>
struct Tile {
  static constexpr int NR = 1 << RB;
  R xr[NR], xi[NR];  // stored vector at the thread's amplitudes
  R yr[NR], yi[NR];  // (H x) at the thread's amplitudes
};

__device__ __forceinline__ uint32_t tile_of(const Geo& g, uint32_t it, uint32_t b, uint32_t G) {
  if (G >= 8 && (G & 7u) == 0 && (g.ntiles & 7u) == 0) {
    const uint32_t per = G >> 3, xcd = b & 7u, j = b >> 3;
    return xcd * (g.ntiles >> 3) + j + it * per;
  }
  return b + it * G;
}

// Partner vectors fetched per round trip for the bonds that leave the tile:
// about 128 bytes of partner amplitudes per thread, at most 4 vectors.
template <typename R, int RB>
struct FarSlots {
  static constexpr int units = 16 / ((1 << RB) * (int)(sizeof(R) / 4));
  static constexpr int n = units > 8 ? 8 : (units < 1 ? 1 : units);
};

// Basis vectors fetched per round trip in the projection/update loops: about
// 128 bytes of amplitudes per thread, at most 8 vectors.
template <typename R, int RB>
struct WinSlots {
  static constexpr int units = 16 / ((1 << RB) * (int)(sizeof(R) / 4));
  static constexpr int n = units > 8 ? 8 : (units < 1 ? 1 : units);
};

// Take the next far bond from `glb` (or none) for one slot of a round trip.
template <typename R>
__device__ __forceinline__ void next_far(uint32_t& glb, R hJ, uint32_t& flip, R& coef) {
  if (glb) {
    const int p = __builtin_ctz(glb);
    glb &= glb - 1;
    flip = 3u << p;
    coef = hJ;
  } else {
    flip = 0u;   // reads the thread's own amplitude, weighted by zero
    coef = (R)0;
  }
}

// y = (H0 + u Hc) x on one tile (amplitudes base .. base + 2^TB - 1).  The
// tile's amplitudes, the S^x partners and the first far partners are requested
// in one round trip before anything waits (partners outside the tile with
// coherent loads when kCoh: other workgroups of the launch wrote them).
template <typename R, int RB, bool kCoh = false>
__device__ __forceinline__ void hv_tile(Tile<R, RB>& T, const HvArgs& a, const Geo& g,
                                        uint32_t tile, const typename VT<R>::T* __restrict__ x,
                                        typename VT<R>::T* lds, double u) {
  using V = typename VT<R>::T;
  constexpr int NR = 1 << RB;
  constexpr int NS = FarSlots<R, RB>::n;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = uniform_u32(threadIdx.x >> 6);
  const int L = g.L;
  const int TB = g.TB;
  const uint32_t base = tile << TB;
  const uint32_t eb = lane | (w << (6 + RB));
  const uint32_t sU = base | (w << (6 + RB));
  const uint32_t bondmask = (1u << (L - 1)) - 1u;
  const R hJ = (R)a.half_J;
  const R cu = (R)(0.5 * u);

  // bonds whose two bits are both wavefront or tile bits (p >= 6+RB): their
  // predicate is the same for every slot of the wavefront
  const int p0 = 6 + RB;
  uint32_t act = (sU ^ (sU >> 1)) & bondmask;
  act = (act >> p0) << p0;
  const uint32_t lds_bonds = (TB - 1 > p0) ? (act & ((1u << (TB - 1)) - 1u)) : 0u;
  uint32_t glb = g.small ? 0u : (act & ~lds_bonds);
  const bool sx_glb = (a.hc_kind == 0) && (a.hc_bit >= TB);

  // ---- round trip 1: own amplitudes, S^x partners, first far partners
  V own[NR];
  load_slots<V, NR>(x, base | eb, !g.small, g.D, own);
  uint32_t f[NS];
  R cf[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (j == 0 && sx_glb) {
      f[0] = 1u << a.hc_bit;
      cf[0] = cu;
    } else {
      next_far<R>(glb, hJ, f[j], cf[j]);
    }
  }
  V gq[NS][NR];
  if (!g.small) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
#pragma unroll
      for (int r = 0; r < NR; ++r) gq[j][r] = ld_partner<kCoh>(&x[(base | eb | ((uint32_t)r << 6)) ^ f[j]]);
    }
  }

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    lds[eb | ((uint32_t)r << 6)] = own[r];
    T.xr[r] = own[r].x;
    T.xi[r] = own[r].y;
  }
  __syncthreads();

  const R czz = (R)a.c_zz;
  const R uR = (R)u;

  // diagonal: J Delta/4 (L-1-2 n_anti) (+ u sum_{i in A}(1/2 - b_i) for the S^z control)
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t s = base | eb | ((uint32_t)r << 6);
    const int n = __popc((s ^ (s >> 1)) & bondmask);
    R d = czz * (R)(L - 1 - 2 * n);
    if (a.hc_kind == 1) d += uR * ((R)(0.5 * a.sz_count) - (R)__popc(s & a.sz_mask));
    T.yr[r] = d * T.xr[r];
    T.yi[r] = d * T.xi[r];
  }

  // bonds between two lane bits (p = 0..4): partner in LDS, per-lane coefficient
  const int pl = min(4, L - 2);
  for (int p = 0; p <= pl; ++p) {
    const R c = (((lane >> p) ^ (lane >> (p + 1))) & 1u) ? hJ : (R)0;
    const uint32_t pe = eb ^ (3u << p);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const V q = lds[pe | ((uint32_t)r << 6)];
      T.yr[r] += c * q.x;
      T.yi[r] += c * q.y;
    }
  }

  // bond p = 5 (lane bit 5 with bit 6): per-lane coefficient, loads issued together
  if (L - 2 >= 5) {
    const uint32_t flip = 3u << 5;
    V q[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = eb | ((uint32_t)r << 6);
      q[r] = (6 < TB) ? lds[e ^ flip] : ld_partner<kCoh>(&x[(base | e) ^ flip]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t s = base | eb | ((uint32_t)r << 6);
      const R c = (((s >> 5) ^ (s >> 6)) & 1u) ? hJ : (R)0;
      T.yr[r] += c * q[r].x;
      T.yi[r] += c * q[r].y;
    }
  }

  // bonds between two register bits (p = 6 .. 6+RB-2): compile-time predicates
#pragma unroll
  for (int q = 0; q + 1 < RB; ++q) {
    if (6 + q <= L - 2) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (((r >> q) ^ (r >> (q + 1))) & 1) {
          const int rp = r ^ (3 << q);
          T.yr[r] += hJ * T.xr[rp];
          T.yi[r] += hJ * T.xi[rp];
        }
      }
    }
  }

  // bond p = 6+RB-1 between the top register bit and the next bit (a wavefront
  // or tile bit): for a given wavefront, the active slots are the half whose top
  // register bit differs from that bit
  if constexpr (RB >= 1) {
   if (6 + RB - 1 <= L - 2) {
    constexpr int p = 6 + RB - 1;
    constexpr int NH = (NR / 2 > 0) ? NR / 2 : 1;
    const uint32_t flip = 3u << p;
    const bool in_lds = (p + 1 < TB);
    const uint32_t hi = (sU >> (p + 1)) & 1u;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if ((uint32_t)half != hi) {
        V q[NH];
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const int r = j | (half << (RB - 1));
          const uint32_t e = eb | ((uint32_t)r << 6);
          q[j] = in_lds ? lds[e ^ flip] : ld_partner<kCoh>(&x[(base | e) ^ flip]);
        }
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const int r = j | (half << (RB - 1));
          T.yr[r] += hJ * q[j].x;
          T.yi[r] += hJ * q[j].y;
        }
      }
    }
   }
  }

  // uniform bonds with the partner inside the tile: LDS
  {
    uint32_t lb = lds_bonds;
    while (lb) {
      const int p = __builtin_ctz(lb);
      lb &= lb - 1;
      const uint32_t flip = 3u << p;
      V q[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) q[r] = lds[(eb | ((uint32_t)r << 6)) ^ flip];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        T.yr[r] += hJ * q[r].x;
        T.yi[r] += hJ * q[r].y;
      }
    }
  }

  // far partners of round trip 1, then the remaining far bonds NS per round trip
  if (!g.small) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        T.yr[r] += cf[j] * gq[j][r].x;
        T.yi[r] += cf[j] * gq[j][r].y;
      }
    }
    while (glb) {
#pragma unroll
      for (int j = 0; j < NS; ++j) next_far<R>(glb, hJ, f[j], cf[j]);
#pragma unroll
      for (int j = 0; j < NS; ++j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) gq[j][r] = ld_partner<kCoh>(&x[(base | eb | ((uint32_t)r << 6)) ^ f[j]]);
      }
#pragma unroll
      for (int j = 0; j < NS; ++j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          T.yr[r] += cf[j] * gq[j][r].x;
          T.yi[r] += cf[j] * gq[j][r].y;
        }
      }
    }
  }

  // S^x control inside the tile: u/2 times the amplitude with that bit flipped
  if (a.hc_kind == 0 && !sx_glb) {
    const uint32_t flip = 1u << a.hc_bit;
    V q[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) q[r] = lds[(eb | ((uint32_t)r << 6)) ^ flip];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T.yr[r] += cu * q[r].x;
      T.yi[r] += cu * q[r].y;
    }
  }

}

// y = (H0 + u Hc) x on one full tile of complex64 amplitudes held in pairs, so
// that every global and LDS access moves 16 bytes: thread (lane, w) holds the
// pairs q in [0, 2^(RB-1)) with amplitudes
//   e = h | lane << 1 | q << 7 | w << (6+RB),   h = 0, 1.
// Bonds with a bit below 6+RB (inside the wavefront) and the active bonds
// between two wavefront bits read the partner pair from LDS; bonds reaching
// the tile-index bits read the partner tile's pairs from global memory (a
// predicate uniform over the wavefront), as hv_tile does.  A partner e ^ (3 << p)
// is in the same half of a pair unless p = 0 (bits 0 and 1), where it is the
// other half of the neighbouring pair.  Needs RB >= 2, 2^TB <= D and at least
// two wavefronts (6+RB < TB), and 16-byte aligned x.
template <int RB, bool kCoh = false>
__device__ __forceinline__ void hv_tile_pairs(Tile<float, RB>& T, const HvArgs& a, const Geo& g,
                                              uint32_t tile, const float2* __restrict__ x,
                                              float2* lds, double u) {
  static_assert(RB >= 2, "two pairs or more per thread");
  constexpr int NR = 1 << RB;
  constexpr int NP = NR / 2;
  constexpr int NS = FarSlots<float, RB>::n;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = uniform_u32(threadIdx.x >> 6);
  const int L = g.L;
  const int TB = g.TB;
  const uint32_t base = tile << TB;
  const uint32_t wb = w << (6 + RB);
  const uint32_t bondmask = (1u << (L - 1)) - 1u;
  const float hJ = (float)a.half_J;
  const float cu = (float)(0.5 * u);
  const float4* __restrict__ x4 = reinterpret_cast<const float4*>(x);
  float4* lds4 = reinterpret_cast<float4*>(lds);
  uint32_t ep[NP];   // first amplitude of pair q inside the tile
#pragma unroll
  for (int q = 0; q < NP; ++q) ep[q] = (lane << 1) | ((uint32_t)q << 7) | wb;

  // bonds between two wavefront or tile bits (p >= 6+RB): wavefront-uniform
  const int p0 = 6 + RB;
  const uint32_t sU = base | wb;
  uint32_t act = (sU ^ (sU >> 1)) & bondmask;
  act = (act >> p0) << p0;
  const uint32_t lds_bonds = act & ((1u << (TB - 1)) - 1u);
  uint32_t glb = act & ~lds_bonds;
  const bool sx_glb = (a.hc_kind == 0) && (a.hc_bit >= TB);

  // ---- round trip 1: own pairs, the S^x partner and the first far partners
  float4 own[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) own[q] = x4[(base | ep[q]) >> 1];
  uint32_t f[NS];
  float cf[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (j == 0 && sx_glb) {
      f[0] = 1u << a.hc_bit;
      cf[0] = cu;
    } else {
      next_far<float>(glb, hJ, f[j], cf[j]);
    }
  }
  float4 gq[NS][NP];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
#pragma unroll
    for (int q = 0; q < NP; ++q) gq[j][q] = ld_partner<kCoh>(&x4[((base | ep[q]) ^ f[j]) >> 1]);
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    lds4[ep[q] >> 1] = own[q];
    T.xr[2 * q] = own[q].x;
    T.xi[2 * q] = own[q].y;
    T.xr[2 * q + 1] = own[q].z;
    T.xi[2 * q + 1] = own[q].w;
  }
  __syncthreads();

  // ---- diagonal: J Delta/4 (L-1-2 n_anti) (+ u sum_{i in A}(1/2 - b_i) for S^z)
  const float czz = (float)a.c_zz;
  const float uR = (float)u;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t s = base | ep[r >> 1] | (uint32_t)(r & 1);
    const int n = __popc((s ^ (s >> 1)) & bondmask);
    float d = czz * (float)(L - 1 - 2 * n);
    if (a.hc_kind == 1) d += uR * ((float)(0.5 * a.sz_count) - (float)__popc(s & a.sz_mask));
    T.yr[r] = d * T.xr[r];
    T.yi[r] = d * T.xi[r];
  }

  // ---- bonds inside the tile: the partner pair from LDS
  uint32_t inb = ((1u << p0) - 1u) | lds_bonds;
  while (inb) {
    const int p = __builtin_ctz(inb);
    inb &= inb - 1;
    const uint32_t flip = 3u << p;
    float4 P[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) P[q] = lds4[(ep[q] ^ flip) >> 1];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t e = ep[q] | (uint32_t)h;
        const float c = (((e >> p) ^ (e >> (p + 1))) & 1u) ? hJ : 0.0f;
        const bool other = (p == 0) ? (h == 0) : (h == 1);   // the partner's half
        const float pr = other ? P[q].z : P[q].x;
        const float pi = other ? P[q].w : P[q].y;
        T.yr[2 * q + h] += c * pr;
        T.yi[2 * q + h] += c * pi;
      }
    }
  }

  // ---- far partners of round trip 1, then the remaining far bonds NS per round trip
#pragma unroll
  for (int j = 0; j < NS; ++j) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      T.yr[2 * q] += cf[j] * gq[j][q].x;
      T.yi[2 * q] += cf[j] * gq[j][q].y;
      T.yr[2 * q + 1] += cf[j] * gq[j][q].z;
      T.yi[2 * q + 1] += cf[j] * gq[j][q].w;
    }
  }
  while (glb) {
#pragma unroll
    for (int j = 0; j < NS; ++j) next_far<float>(glb, hJ, f[j], cf[j]);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
#pragma unroll
      for (int q = 0; q < NP; ++q) gq[j][q] = ld_partner<kCoh>(&x4[((base | ep[q]) ^ f[j]) >> 1]);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T.yr[2 * q] += cf[j] * gq[j][q].x;
        T.yi[2 * q] += cf[j] * gq[j][q].y;
        T.yr[2 * q + 1] += cf[j] * gq[j][q].z;
        T.yi[2 * q + 1] += cf[j] * gq[j][q].w;
      }
    }
  }

  // ---- S^x control inside the tile: u/2 times the amplitude with that bit flipped
  if (a.hc_kind == 0 && !sx_glb) {
    const uint32_t flip = 1u << a.hc_bit;
    float4 P[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) P[q] = lds4[(ep[q] ^ flip) >> 1];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool other = (flip & 1u) ? (h == 0) : (h == 1);
        T.yr[2 * q + h] += cu * (other ? P[q].z : P[q].x);
        T.yi[2 * q + h] += cu * (other ? P[q].w : P[q].y);
      }
    }
  }
}

// Whether a tiling of complex64 amplitudes runs hv_tile_pairs: whole tiles of
// at least two wavefronts with two pairs or more per thread.
__host__ __device__ inline bool pairs_tiling(const Geo& g) {
  return !g.small && g.RB >= 2 && g.TB > 6 + g.RB;
}

__device__ __forceinline__ double control_value(const HvArgs& a) {
  return a.u_ptr ? *a.u_ptr : a.u_val;
}

}  // namespace
}  // namespace kg
