// HIP kernels of the K-GRAPE hot path for gfx950 (MI355X).
//
// Memory-bound throughout, so no MFMA: every kernel streams state vectors
// through HBM (or the Infinity Cache) once per pass and keeps the arithmetic in
// registers.  Layout: a state vector is D = 2^L interleaved complex amplitudes.
//
// H v (Sec. III.A, Eqs. 6 and 10).  A block stages a tile of 2^TB consecutive
// amplitudes in LDS.  Inside the tile, amplitude index bits are assigned as
//   bits 0..5           lane of the wavefront,
//   bits 6..6+RB-1      register slot r of the thread (2^RB amplitudes per thread),
//   bits 6+RB..TB-1     wavefront of the block,
// so global loads are fully coalesced (a wavefront reads 64 consecutive
// amplitudes per slot).  The hopping term of bond p couples s and s^(3<<p)
// when bits p and p+1 of s differ.  Bonds between two register bits are
// resolved in registers with compile-time predicates; bonds inside the tile
// read the partner from LDS; bonds reaching bit TB or above read the partner
// tile from global memory (L2/Infinity Cache), with a predicate that is
// uniform across the wavefront, so the loads stay coalesced and inactive bonds
// cost one scalar branch.  The diagonal S^z S^z term is one popcount.
//
// Lanczos (App. A, Algorithm 2 with the full re-orthonormalisation it
// describes).  One basis step is two passes over the tile grid:
//   pass A(k): x = stored v_k; y = H x (recomputed from the tile);
//              h_i = <v_i|y> for the projection window, and <x|x>;
//   pass B(k): w = s_k y - sum_i (h_i s_i) v_i, stored unnormalised as v_{k+1},
//              and ||w||^2.
// Stored vectors are not rescaled: scale_k = 1/||stored_k|| lives in device
// memory and is folded into the coefficients.  Each pass ends with a
// deterministic two-level grid reduction in FP64 (fixed order, no
// floating-point atomics); the last block to finish applies the scalar update
// (alpha, beta, breakdown test) and, when the basis is complete, evaluates
// exp(-itT) e_1 on one wavefront in FP64.  A final streaming pass forms
// v_out = beta0 V^T exp(-itT) e_1 with FP64 accumulation.
//
// Blocks of the tiled kernels are mapped to tiles XCD by XCD: block b runs on
// XCD b%8, and the tiles of one XCD form one contiguous range, so partner tiles
// of the lower hopping bonds are read from the same L2.

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
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

__device__ __forceinline__ void st_agent_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Make this wavefront's device-coherent stores complete before what follows.
__device__ __forceinline__ void complete_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Deterministic grid-wide sum of `ns` complex FP64 values.  Every block
// passes its block totals in `tot` (LDS).  Returns true in exactly one block,
// the last to arrive, with the grid totals in `tot`.  Partials are combined
// in a fixed order: blocks of a group of kGroup, then groups.
//
// The partials travel only through device-scope (sc1) stores and loads, which
// are coherent across the XCDs' L2 caches; a store is waited for before the
// arrival counter is incremented.  No device-wide fence is needed, so the L2
// caches are never written back or invalidated here.
__device__ bool grid_reduce(cplx_d* tot, int ns, cplx_d* partials, cplx_d* gpartials,
                            uint32_t* counters) {
  __shared__ int last;
  const uint32_t b = blockIdx.x, G = gridDim.x;
  if (G == 1) return true;
  const uint32_t grp = b / kGroup, ngrp = (G + kGroup - 1) / kGroup;
  const uint32_t gsize = min((uint32_t)kGroup, G - grp * kGroup);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;

  if (wv == 0) {
    for (int j = lane; j < ns; j += 64) {
      st_agent(&partials[(size_t)b * kMaxScal + j].re, tot[j].re);
      st_agent(&partials[(size_t)b * kMaxScal + j].im, tot[j].im);
    }
    complete_stores();
    uint32_t prev = 0;
    if (lane == 0)
      prev = __hip_atomic_fetch_add(&counters[grp], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = __shfl(prev, 0, 64);
    if (lane == 0) last = (prev == gsize - 1);
  }
  __syncthreads();
  if (!last) return false;
  if (threadIdx.x == 0) st_agent_u32(&counters[grp], 0u);
  for (int j = wv; j < ns; j += nw) {
    double re = 0.0, im = 0.0;
    if ((uint32_t)lane < gsize) {
      const cplx_d* p = &partials[(size_t)(grp * kGroup + lane) * kMaxScal + j];
      re = ld_agent(&p->re);
      im = ld_agent(&p->im);
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (ngrp == 1) {
      if (lane == 0) tot[j] = cplx_d{re, im};
    } else if (lane == 0) {
      st_agent(&gpartials[(size_t)grp * kMaxScal + j].re, re);
      st_agent(&gpartials[(size_t)grp * kMaxScal + j].im, im);
    }
  }
  complete_stores();
  __syncthreads();
  if (ngrp == 1) return true;
  if (wv == 0) {
    uint32_t prev = 0;
    if (lane == 0)
      prev = __hip_atomic_fetch_add(&counters[kMaxGroups], 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    prev = __shfl(prev, 0, 64);
    if (lane == 0) last = (prev == ngrp - 1);
  }
  __syncthreads();
  if (!last) return false;
  if (threadIdx.x == 0) st_agent_u32(&counters[kMaxGroups], 0u);
  for (int j = wv; j < ns; j += nw) {
    double re = 0.0, im = 0.0;
    if ((uint32_t)lane < ngrp) {
      const cplx_d* p = &gpartials[(size_t)lane * kMaxScal + j];
      re = ld_agent(&p->re);
      im = ld_agent(&p->im);
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) tot[j] = cplx_d{re, im};
  }
  __syncthreads();
  return true;
}

// Sum the per-wavefront accumulators wacc[w * kMaxScal + j] of a block in
// wavefront order.
__device__ void block_totals(const cplx_d* wacc, int ns, cplx_d* tot) {
  const int nw = blockDim.x >> 6;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
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
__device__ void tri_exp_wave(double a, double lo, double hi, double t, double& cr, double& ci) {
  const int lane = threadIdx.x & 63;
  const double nrm = wave_max(fabs(a) + lo + hi);
  int nsub = (int)ceil(fabs(t) * nrm * 2.0);
  if (nsub < 1) nsub = 1;
  const double tau = t / (double)nsub;
  double yr = (lane == 0) ? 1.0 : 0.0, yi = 0.0;
  for (int step = 0; step < nsub; ++step) {
    double tr = yr, ti = yi, ar = yr, ai = yi;
#pragma unroll 4
    for (int p = 1; p <= 16; ++p) {
      const double dr = __shfl_up(tr, 1, 64), di = __shfl_up(ti, 1, 64);
      const double ur = __shfl_down(tr, 1, 64), ui = __shfl_down(ti, 1, 64);
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

// ---------------------------------------------------------------------- H v on a tile

template <typename R, int RB>
struct Tile {
  static constexpr int NR = 1 << RB;
  R xr[NR], xi[NR];  // stored vector at the thread's amplitudes
  R yr[NR], yi[NR];  // (H x) at the thread's amplitudes
};

__device__ __forceinline__ uint32_t tile_of(const Geo& g, uint32_t it) {
  const uint32_t G = gridDim.x, b = blockIdx.x;
  if (G >= 8 && (G & 7u) == 0 && (g.ntiles & 7u) == 0) {
    const uint32_t per = G >> 3, xcd = b & 7u, j = b >> 3;
    return xcd * (g.ntiles >> 3) + j + it * per;
  }
  return b + it * G;
}

template <typename R, int RB>
__device__ __forceinline__ void hv_tile(Tile<R, RB>& T, const HvArgs& a, const Geo& g,
                                        uint32_t tile, const typename VT<R>::T* __restrict__ x,
                                        typename VT<R>::T* lds, double u) {
  using V = typename VT<R>::T;
  constexpr int NR = 1 << RB;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = uniform_u32(threadIdx.x >> 6);
  const int L = g.L;
  const int TB = g.TB;
  const uint32_t base = tile << TB;
  const uint32_t eb = lane | (w << (6 + RB));
  const uint32_t sU = base | (w << (6 + RB));

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t e = eb | ((uint32_t)r << 6);
    const uint32_t s = base | e;
    V val;
    if (!g.small || s < g.D) {
      val = x[s];
    } else {
      val.x = (R)0;
      val.y = (R)0;
    }
    lds[e] = val;
    T.xr[r] = val.x;
    T.xi[r] = val.y;
  }
  __syncthreads();

  const R hJ = (R)a.half_J;
  const R czz = (R)a.c_zz;
  const uint32_t bondmask = (1u << (L - 1)) - 1u;
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
      q[r] = (6 < TB) ? lds[e ^ flip] : x[(base | e) ^ flip];
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
          q[j] = in_lds ? lds[e ^ flip] : x[(base | e) ^ flip];
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

  // bonds whose two bits are both wavefront or tile bits (p >= 6+RB): the
  // predicate is the same for every slot of the wavefront.  Partners inside the
  // tile come from LDS, the others from global memory; two active bonds are
  // loaded per round trip.
  {
    const int p0 = 6 + RB;
    uint32_t act = (sU ^ (sU >> 1)) & bondmask;
    act = (p0 >= 32) ? 0u : (act >> p0) << p0;
    const uint32_t lds_bonds = (TB - 1 > p0) ? (act & ((1u << (TB - 1)) - 1u)) : 0u;
    uint32_t glb_bonds = act & ~lds_bonds;
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
    while (glb_bonds) {
      const int p1 = __builtin_ctz(glb_bonds);
      glb_bonds &= glb_bonds - 1;
      const uint32_t f1 = 3u << p1;
      if (glb_bonds) {
        const int p2 = __builtin_ctz(glb_bonds);
        glb_bonds &= glb_bonds - 1;
        const uint32_t f2 = 3u << p2;
        V q1[NR], q2[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const uint32_t s = base | eb | ((uint32_t)r << 6);
          q1[r] = x[s ^ f1];
          q2[r] = x[s ^ f2];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          T.yr[r] += hJ * q1[r].x;
          T.yi[r] += hJ * q1[r].y;
          T.yr[r] += hJ * q2[r].x;
          T.yi[r] += hJ * q2[r].y;
        }
      } else {
        V q1[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) q1[r] = x[(base | eb | ((uint32_t)r << 6)) ^ f1];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          T.yr[r] += hJ * q1[r].x;
          T.yi[r] += hJ * q1[r].y;
        }
      }
    }
  }

  // S^x control on one site: u/2 times the amplitude with that bit flipped
  if (a.hc_kind == 0) {
    const R cu = (R)(0.5 * u);
    const uint32_t flip = 1u << a.hc_bit;
    V q[NR];
    if (a.hc_bit < TB) {
#pragma unroll
      for (int r = 0; r < NR; ++r) q[r] = lds[(eb | ((uint32_t)r << 6)) ^ flip];
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r) q[r] = x[(base | eb | ((uint32_t)r << 6)) ^ flip];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T.yr[r] += cu * q[r].x;
      T.yi[r] += cu * q[r].y;
    }
  }
}

__device__ __forceinline__ double control_value(const HvArgs& a) {
  return a.u_ptr ? *a.u_ptr : a.u_val;
}

// ---------------------------------------------------------------------- xxz_apply

template <typename R, int RB>
__global__ void __launch_bounds__(RB >= 3 ? 512 : 1024) k_hv(HvArgs a, Geo g, const typename VT<R>::T* __restrict__ v,
                                            typename VT<R>::T* __restrict__ w) {
  using V = typename VT<R>::T;
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const double u = control_value(a);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = uniform_u32(threadIdx.x >> 6);
  const uint32_t eb = lane | (wv << (6 + RB));
  const uint32_t iters = g.ntiles / gridDim.x;
  Tile<R, RB> T;
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t tile = tile_of(g, it);
    if (it) __syncthreads();
    hv_tile<R, RB>(T, a, g, tile, v, lds, u);
    const uint32_t base = tile << g.TB;
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
      const uint32_t s = base | eb | ((uint32_t)r << 6);
      if (!g.small || s < g.D) {
        V o;
        o.x = T.yr[r];
        o.y = T.yi[r];
        w[s] = o;
      }
    }
  }
}

// ---------------------------------------------------------------------- Lanczos passes

struct LzArgs {
  HvArgs hv;
  Geo geo;
  const void* slot0;  // stored vector 0: the input of the Krylov call
  void* basis;        // stored vectors 1..m-1
  int32_t k;          // basis step
  int32_t i0;         // first index of the projection window [i0, k]
  int32_t m;
  int32_t pad_;
  double t;
  double tol;
  KState* st;
  cplx_d* partials;
  cplx_d* gpartials;
};

template <typename V>
__device__ __forceinline__ const V* slot_ptr(const LzArgs& a, int i) {
  return i == 0 ? reinterpret_cast<const V*>(a.slot0)
                : reinterpret_cast<const V*>(a.basis) + (size_t)(i - 1) * a.geo.D;
}

// Scalar tail of a basis: exp(-itT) e_1 on wavefront 0 of the finishing block
// and the combination coefficients dcomb_j = beta0 c_j scale_j.  `fresh_alpha`
// replaces alpha[m_eff-1] when it was produced by this very kernel (NaN: read
// it from memory); `fresh_s0`/`fresh_b0` likewise for step 0.
__device__ void finish_basis(const LzArgs& a, int m_eff, double fresh_alpha, double fresh_b0,
                             double fresh_s0) {
  KState* st = a.st;
  const int i = threadIdx.x & 63;
  double ai = 0.0, lo = 0.0, hi = 0.0, sc = 0.0;
  if (i < m_eff) {
    ai = (i == m_eff - 1 && !isnan(fresh_alpha)) ? fresh_alpha : st->alpha[i];
    lo = (i > 0) ? st->offd[i] : 0.0;
    hi = (i + 1 < m_eff) ? st->offd[i + 1] : 0.0;
    sc = (i == 0 && !isnan(fresh_s0)) ? fresh_s0 : st->scale[i];
  }
  const double b0 = isnan(fresh_b0) ? st->beta0 : fresh_b0;
  double cr, ci;
  tri_exp_wave(ai, lo, hi, a.t, cr, ci);
  if (i < m_eff) st->dcomb[i] = cplx_d{b0 * cr * sc, b0 * ci * sc};
  if (i == 0) {
    st->m_eff = m_eff;
    st->done = 1;
  }
}

template <typename R, int RB>
__global__ void __launch_bounds__(RB >= 3 ? 512 : 1024) k_pass_a(LzArgs a) {
  using V = typename VT<R>::T;
  constexpr int NR = 1 << RB;
  if (a.k > 0 && a.st->done) return;
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  __shared__ cplx_d tot[kMaxScal];

  const int nwin = a.k - a.i0 + 1;
  const int ns = nwin + 1;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = uniform_u32(threadIdx.x >> 6);
  const uint32_t eb = lane | (wv << (6 + RB));
  // lane l accumulates window entry l across the tiles of this block
  double acc_re = 0.0, acc_im = 0.0, acc_nn = 0.0;

  const double u = control_value(a.hv);
  const V* x = slot_ptr<V>(a, a.k);
  const uint32_t iters = a.geo.ntiles / gridDim.x;
  Tile<R, RB> T;
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t tile = tile_of(a.geo, it);
    if (it) __syncthreads();
    hv_tile<R, RB>(T, a.hv, a.geo, tile, x, lds, u);
    const uint32_t base = tile << a.geo.TB;
    // window vectors other than v_k, two per round trip
    for (int i = a.i0; i < a.k; i += 2) {
      const bool two = (i + 1 < a.k);
      const V* v1 = slot_ptr<V>(a, i);
      const V* v2 = slot_ptr<V>(a, two ? i + 1 : i);
      V q1[NR], q2[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t s = base | eb | ((uint32_t)r << 6);
        const bool ok = !a.geo.small || s < a.geo.D;
        q1[r] = ok ? v1[s] : V{(R)0, (R)0};
        q2[r] = (ok && two) ? v2[s] : V{(R)0, (R)0};
      }
      double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double yr = T.yr[r], yi = T.yi[r];
        const double ar = q1[r].x, ai = q1[r].y, br = q2[r].x, bi = q2[r].y;
        s1r += ar * yr + ai * yi;
        s1i += ar * yi - ai * yr;
        s2r += br * yr + bi * yi;
        s2i += br * yi - bi * yr;
      }
      s1r = wave_sum(s1r);
      s1i = wave_sum(s1i);
      if ((int)lane == i - a.i0) {
        acc_re += s1r;
        acc_im += s1i;
      }
      if (two) {
        s2r = wave_sum(s2r);
        s2i = wave_sum(s2i);
        if ((int)lane == i + 1 - a.i0) {
          acc_re += s2r;
          acc_im += s2i;
        }
      }
    }
    {
      // v_k itself, from registers
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double vr = T.xr[r], vi = T.xi[r], yr = T.yr[r], yi = T.yi[r];
        sr += vr * yr + vi * yi;
        si += vr * yi - vi * yr;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if ((int)lane == a.k - a.i0) {
        acc_re += sr;
        acc_im += si;
      }
    }
    double nn = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double vr = T.xr[r], vi = T.xi[r];
      nn += vr * vr + vi * vi;
    }
    acc_nn += wave_sum(nn);
  }
  __syncthreads();
  cplx_d* wacc = reinterpret_cast<cplx_d*>(smem_raw);
  if ((int)lane < nwin) wacc[wv * kMaxScal + lane] = cplx_d{acc_re, acc_im};
  if (lane == 0) wacc[wv * kMaxScal + nwin] = cplx_d{acc_nn, 0.0};
  __syncthreads();
  block_totals(wacc, ns, tot);
  if (!grid_reduce(tot, ns, a.partials, a.gpartials, a.st->counters)) return;
  if (threadIdx.x >= 64) return;

  // ---- scalar update on wavefront 0 of the last block
  KState* st = a.st;
  const int lane0 = threadIdx.x;
  const int k = a.k;
  double sk, b0 = NAN, s0 = NAN;
  if (k == 0) {
    const double nn = tot[nwin].re;
    if (!(nn > 0.0)) {
      if (lane0 == 0) {
        st->beta0 = 0.0;
        st->normT = 0.0;
        st->m_eff = 0;
        st->done = 1;
      }
      return;
    }
    b0 = sqrt(nn);
    sk = 1.0 / b0;
    s0 = sk;
    if (lane0 == 0) {
      st->beta0 = b0;
      st->scale[0] = sk;
      st->offd[0] = 0.0;
      st->done = 0;
    }
  } else {
    sk = st->scale[k];
  }
  for (int l = lane0; l < nwin; l += 64) {
    const int i = a.i0 + l;
    const double si = (i == k) ? sk : st->scale[i];
    const double f = si * sk;
    st->coef[l] = cplx_d{tot[l].re * f * si, tot[l].im * f * si};
  }
  const double alpha = tot[nwin - 1].re * sk * sk;
  const double offk = (k == 0) ? 0.0 : st->offd[k];
  const double prevT = (k == 0) ? 0.0 : st->normT;
  const double normT = fmax(prevT, fabs(alpha) + offk);
  if (lane0 == 0) {
    st->alpha[k] = alpha;
    st->normT = normT;
  }
  if (k == a.m - 1) finish_basis(a, a.m, alpha, b0, s0);
}

template <typename R, int RB>
__global__ void __launch_bounds__(RB >= 3 ? 512 : 1024) k_pass_b(LzArgs a) {
  using V = typename VT<R>::T;
  constexpr int NR = 1 << RB;
  if (a.st->done) return;
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  __shared__ cplx_d tot[kMaxScal];

  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = uniform_u32(threadIdx.x >> 6);
  const uint32_t eb = lane | (wv << (6 + RB));
  double acc_nn = 0.0;

  const KState* st = a.st;
  const double sk = st->scale[a.k];
  const double u = control_value(a.hv);
  const V* x = slot_ptr<V>(a, a.k);
  V* out = reinterpret_cast<V*>(a.basis) + (size_t)a.k * a.geo.D;
  const uint32_t iters = a.geo.ntiles / gridDim.x;
  Tile<R, RB> T;
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t tile = tile_of(a.geo, it);
    if (it) __syncthreads();
    hv_tile<R, RB>(T, a.hv, a.geo, tile, x, lds, u);
    const uint32_t base = tile << a.geo.TB;
    double zr[NR], zi[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      zr[r] = sk * (double)T.yr[r];
      zi[r] = sk * (double)T.yi[r];
    }
    // window vectors other than v_k, two per round trip
    for (int i = a.i0; i < a.k; i += 2) {
      const bool two = (i + 1 < a.k);
      const cplx_d c1 = st->coef[i - a.i0];
      const cplx_d c2 = two ? st->coef[i + 1 - a.i0] : cplx_d{0.0, 0.0};
      const V* v1 = slot_ptr<V>(a, i);
      const V* v2 = slot_ptr<V>(a, two ? i + 1 : i);
      V q1[NR], q2[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t s = base | eb | ((uint32_t)r << 6);
        const bool ok = !a.geo.small || s < a.geo.D;
        q1[r] = ok ? v1[s] : V{(R)0, (R)0};
        q2[r] = (ok && two) ? v2[s] : V{(R)0, (R)0};
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double ar = q1[r].x, ai = q1[r].y, br = q2[r].x, bi = q2[r].y;
        zr[r] -= c1.re * ar - c1.im * ai;
        zi[r] -= c1.re * ai + c1.im * ar;
        zr[r] -= c2.re * br - c2.im * bi;
        zi[r] -= c2.re * bi + c2.im * br;
      }
    }
    {
      const cplx_d c = st->coef[a.k - a.i0];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const double vr = T.xr[r], vi = T.xi[r];
        zr[r] -= c.re * vr - c.im * vi;
        zi[r] -= c.re * vi + c.im * vr;
      }
    }
    double nn = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t s = base | eb | ((uint32_t)r << 6);
      V o;
      o.x = (R)zr[r];
      o.y = (R)zi[r];
      if (!a.geo.small || s < a.geo.D) {
        out[s] = o;
        nn += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
      }
    }
    acc_nn += wave_sum(nn);
  }
  __syncthreads();
  cplx_d* wacc = reinterpret_cast<cplx_d*>(smem_raw);
  if (lane == 0) wacc[wv * kMaxScal] = cplx_d{acc_nn, 0.0};
  __syncthreads();
  block_totals(wacc, 1, tot);
  if (!grid_reduce(tot, 1, a.partials, a.gpartials, a.st->counters)) return;
  if (threadIdx.x >= 64) return;

  KState* stw = a.st;
  const double b = sqrt(tot[0].re);
  const double normT = stw->normT;
  if (b <= a.tol * fmax(1.0, normT)) {
    finish_basis(a, a.k + 1, NAN, NAN, NAN);
  } else if (threadIdx.x == 0) {
    stw->offd[a.k + 1] = b;
    stw->scale[a.k + 1] = 1.0 / b;
  }
}

// ---------------------------------------------------------------------- streaming kernels

constexpr int kStreamBlock = 256;
constexpr int kStreamUnroll = 4;

template <typename R>
__global__ void __launch_bounds__(kStreamBlock)
    k_combine(const KState* __restrict__ st, uint32_t D, const typename VT<R>::T* slot0,
              const typename VT<R>::T* basis, typename VT<R>::T* out, int32_t* m_eff_out) {
  using V = typename VT<R>::T;
  const int me = st->m_eff;
  const uint32_t stride = gridDim.x * kStreamBlock;
  for (uint32_t s0 = blockIdx.x * kStreamBlock + threadIdx.x; s0 < D; s0 += stride * kStreamUnroll) {
    double ar[kStreamUnroll], ai[kStreamUnroll];
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) {
      ar[q] = 0.0;
      ai[q] = 0.0;
    }
    for (int j = 0; j < me; ++j) {
      const cplx_d c = st->dcomb[j];
      const V* vj = (j == 0) ? slot0 : basis + (size_t)(j - 1) * D;
      V v[kStreamUnroll];
#pragma unroll
      for (int q = 0; q < kStreamUnroll; ++q) {
        const uint32_t s = s0 + q * stride;
        if (s < D) {
          v[q] = vj[s];
        } else {
          v[q].x = (R)0;
          v[q].y = (R)0;
        }
      }
#pragma unroll
      for (int q = 0; q < kStreamUnroll; ++q) {
        const double vr = v[q].x, vi = v[q].y;
        ar[q] += c.re * vr - c.im * vi;
        ai[q] += c.re * vi + c.im * vr;
      }
    }
#pragma unroll
    for (int q = 0; q < kStreamUnroll; ++q) {
      const uint32_t s = s0 + q * stride;
      if (s < D) {
        V o;
        o.x = (R)ar[q];
        o.y = (R)ai[q];
        out[s] = o;
      }
    }
  }
  if (m_eff_out && blockIdx.x == 0 && threadIdx.x == 0) *m_eff_out = me;
}

// beta = <f|psi> (Eq. 2); the last block writes beta, F = |beta|^2.
template <typename R>
__global__ void __launch_bounds__(kStreamBlock)
    k_overlap(uint32_t D, const typename VT<R>::T* __restrict__ f, const typename VT<R>::T* __restrict__ psi,
              KState* st, cplx_d* partials, cplx_d* gpartials, double* F_dev, double* beta_dev) {
  __shared__ cplx_d wacc[(kStreamBlock / 64) * kMaxScal];
  __shared__ cplx_d tot[kMaxScal];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  double sr = 0.0, si = 0.0;
  const uint32_t stride = gridDim.x * kStreamBlock;
  for (uint32_t s = blockIdx.x * kStreamBlock + threadIdx.x; s < D; s += stride) {
    const double fr = f[s].x, fi = f[s].y, pr = psi[s].x, pi = psi[s].y;
    sr += fr * pr + fi * pi;
    si += fr * pi - fi * pr;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) wacc[wv * kMaxScal] = cplx_d{sr, si};
  __syncthreads();
  block_totals(wacc, 1, tot);
  if (!grid_reduce(tot, 1, partials, gpartials, st->counters)) return;
  if (threadIdx.x == 0) {
    const cplx_d b = tot[0];
    st->overlap = b;
    st->fid = b.re * b.re + b.im * b.im;
    if (beta_dev) {
      beta_dev[0] = b.re;
      beta_dev[1] = b.im;
    }
    if (F_dev) *F_dev = b.re * b.re + b.im * b.im;
  }
}

// g_j = 2 dt Im(conj(beta) <lambda|Hc|psi>)  (Eq. 5 with chi = beta lambda, sign of dF).
template <typename R>
__global__ void __launch_bounds__(kStreamBlock)
    k_bracket(HvArgs a, uint32_t D, const typename VT<R>::T* __restrict__ lam,
              const typename VT<R>::T* __restrict__ psi, double dt, const double* beta_dev,
              KState* st, cplx_d* partials, cplx_d* gpartials, double* grad_slot) {
  __shared__ cplx_d wacc[(kStreamBlock / 64) * kMaxScal];
  __shared__ cplx_d tot[kMaxScal];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  double sr = 0.0, si = 0.0;
  const uint32_t stride = gridDim.x * kStreamBlock;
  const uint32_t flip = (a.hc_kind == 0) ? (1u << a.hc_bit) : 0u;
  for (uint32_t s = blockIdx.x * kStreamBlock + threadIdx.x; s < D; s += stride) {
    double pr, pi;
    if (a.hc_kind == 0) {
      pr = 0.5 * (double)psi[s ^ flip].x;
      pi = 0.5 * (double)psi[s ^ flip].y;
    } else {
      const double dz = 0.5 * a.sz_count - (double)__popc(s & a.sz_mask);
      pr = dz * (double)psi[s].x;
      pi = dz * (double)psi[s].y;
    }
    const double lr = lam[s].x, li = lam[s].y;
    sr += lr * pr + li * pi;
    si += lr * pi - li * pr;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) wacc[wv * kMaxScal] = cplx_d{sr, si};
  __syncthreads();
  block_totals(wacc, 1, tot);
  if (!grid_reduce(tot, 1, partials, gpartials, st->counters)) return;
  if (threadIdx.x == 0) {
    const double br = beta_dev[0], bi = beta_dev[1];
    const cplx_d B = tot[0];
    *grad_slot = 2.0 * dt * (br * B.im - bi * B.re);
  }
}

// u <- u + eta g / max|g| in one block (deterministic max).
__global__ void __launch_bounds__(1024) k_ascent(double* u, const double* g, int N, double eta) {
  __shared__ double wmax[16];
  double m = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) m = fmax(m, fabs(g[j]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  double gm = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) gm = fmax(gm, wmax[q]);
  if (gm == 0.0) return;
  const double f = eta / gm;
  for (int j = threadIdx.x; j < N; j += blockDim.x) u[j] += f * g[j];
}

__global__ void k_index_map(int L, uint32_t s0, uint32_t count, int32_t* n_anti, uint32_t* pmask) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t s = s0 + i;
  const uint32_t m = (s ^ (s >> 1)) & ((1u << (L - 1)) - 1u);
  n_anti[i] = __popc(m);
  pmask[i] = m;
}

__global__ void k_init_state(KState* st) {
  const int i = threadIdx.x;
  if (i < kMaxGroups + 2) st->counters[i] = 0u;
  if (i == 0) {
    st->done = 0;
    st->m_eff = 0;
    st->normT = 0.0;
  }
}

// ---------------------------------------------------------------------- launch helpers

template <typename R>
size_t lds_bytes(const Geo& g) {
  const size_t tile = ((size_t)1 << g.TB) * sizeof(typename VT<R>::T);
  const size_t red = ((size_t)1 << g.WB) * kMaxScal * sizeof(cplx_d);
  return tile > red ? tile : red;
}

template <typename R, int RB>
hipError_t launch_hv_t(const HvArgs& a, const Geo& g, const void* v, void* w, hipStream_t s) {
  using V = typename VT<R>::T;
  hipLaunchKernelGGL((k_hv<R, RB>), dim3(g.grid), dim3(64 << g.WB), lds_bytes<R>(g), s, a, g,
                     reinterpret_cast<const V*>(v), reinterpret_cast<V*>(w));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_hv_r(const HvArgs& a, const Geo& g, const void* v, void* w, hipStream_t s) {
  switch (g.RB) {
    case 0: return launch_hv_t<R, 0>(a, g, v, w, s);
    case 1: return launch_hv_t<R, 1>(a, g, v, w, s);
    case 2: return launch_hv_t<R, 2>(a, g, v, w, s);
    default: return launch_hv_t<R, 3>(a, g, v, w, s);
  }
}

template <typename R, int RB>
hipError_t launch_pass(bool pass_a, const LzArgs& la, hipStream_t s) {
  const Geo& g = la.geo;
  if (pass_a) {
    hipLaunchKernelGGL((k_pass_a<R, RB>), dim3(g.grid), dim3(64 << g.WB), lds_bytes<R>(g), s, la);
  } else {
    hipLaunchKernelGGL((k_pass_b<R, RB>), dim3(g.grid), dim3(64 << g.WB), lds_bytes<R>(g), s, la);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pass_r(bool pass_a, const LzArgs& la, hipStream_t s) {
  switch (la.geo.RB) {
    case 0: return launch_pass<R, 0>(pass_a, la, s);
    case 1: return launch_pass<R, 1>(pass_a, la, s);
    case 2: return launch_pass<R, 2>(pass_a, la, s);
    default: return launch_pass<R, 3>(pass_a, la, s);
  }
}

template <typename R>
hipError_t launch_krylov_t(const KrylovCall& c, const Workspace& ws, hipStream_t s) {
  using V = typename VT<R>::T;
  LzArgs la;
  la.hv = c.hv;
  la.geo = c.geo;
  la.slot0 = c.v_in;
  la.basis = ws.basis;
  la.m = c.m;
  la.pad_ = 0;
  la.t = c.t;
  la.tol = c.tol;
  la.st = ws.st;
  la.partials = ws.partials;
  la.gpartials = ws.gpartials;
  Profiler* prof = profiler_for_call();
  const double vb = (double)c.geo.D * sizeof(V);
  hipError_t e;
  for (int k = 0; k < c.m; ++k) {
    const bool last = (k == c.m - 1);
    la.k = k;
    la.i0 = last ? k : (c.reorth ? 0 : (k > 0 ? k - 1 : 0));
    const int nwin = k - la.i0 + 1;
    if (prof) profiler_start(prof, s);
    if ((e = launch_pass_r<R>(true, la, s)) != hipSuccess) return e;
    // algorithmic bytes: the window vectors (v_k included) are read once
    if (prof) profiler_stop(prof, s, kProfPassA, nwin * vb);
    if (!last) {
      if (prof) profiler_start(prof, s);
      if ((e = launch_pass_r<R>(false, la, s)) != hipSuccess) return e;
      // the window vectors are read and v_{k+1} is written
      if (prof) profiler_stop(prof, s, kProfPassB, (nwin + 1) * vb);
    }
  }
  const uint32_t D = c.geo.D;
  if (prof) profiler_start(prof, s);
  hipLaunchKernelGGL((k_combine<R>), dim3(stream_grid(D)), dim3(kStreamBlock), 0, s,
                     (const KState*)ws.st, D, reinterpret_cast<const V*>(c.v_in),
                     reinterpret_cast<const V*>(ws.basis), reinterpret_cast<V*>(c.v_out), c.m_eff_out);
  e = hipGetLastError();
  // m basis vectors read (fewer after a breakdown), v_out written
  if (prof) profiler_stop(prof, s, kProfCombine, (c.m + 1) * vb);
  return e;
}

}  // namespace

// ---------------------------------------------------------------------- public launchers

int stream_grid(uint32_t D) {
  const uint64_t per = (uint64_t)kStreamBlock * kStreamUnroll;
  uint64_t g = (D + per - 1) / per;
  if (g < 1) g = 1;
  if (g > (uint64_t)kMaxGrid) g = kMaxGrid;
  return (int)g;
}

hipError_t launch_init(KState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(128), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_hv(int prec, const HvArgs& a, const Geo& g, const void* v, void* w, hipStream_t s) {
  return prec == 0 ? launch_hv_r<double>(a, g, v, w, s) : launch_hv_r<float>(a, g, v, w, s);
}

hipError_t launch_krylov(const KrylovCall& c, const Workspace& ws, hipStream_t s) {
  return c.prec == 0 ? launch_krylov_t<double>(c, ws, s) : launch_krylov_t<float>(c, ws, s);
}

hipError_t launch_overlap(int prec, uint32_t D, const void* f, const void* psi, const Workspace& ws,
                          double* F_dev, double* beta_dev, hipStream_t s) {
  const int grid = stream_grid(D);
  if (prec == 0) {
    hipLaunchKernelGGL(k_overlap<double>, dim3(grid), dim3(kStreamBlock), 0, s, D,
                       reinterpret_cast<const double2*>(f), reinterpret_cast<const double2*>(psi),
                       ws.st, ws.partials, ws.gpartials, F_dev, beta_dev);
  } else {
    hipLaunchKernelGGL(k_overlap<float>, dim3(grid), dim3(kStreamBlock), 0, s, D,
                       reinterpret_cast<const float2*>(f), reinterpret_cast<const float2*>(psi),
                       ws.st, ws.partials, ws.gpartials, F_dev, beta_dev);
  }
  return hipGetLastError();
}

hipError_t launch_bracket(int prec, const HvArgs& a, uint32_t D, const void* lam, const void* psi,
                          double dt, const double* beta_dev, const Workspace& ws, double* grad_slot,
                          hipStream_t s) {
  const int grid = stream_grid(D);
  if (prec == 0) {
    hipLaunchKernelGGL(k_bracket<double>, dim3(grid), dim3(kStreamBlock), 0, s, a, D,
                       reinterpret_cast<const double2*>(lam), reinterpret_cast<const double2*>(psi),
                       dt, beta_dev, ws.st, ws.partials, ws.gpartials, grad_slot);
  } else {
    hipLaunchKernelGGL(k_bracket<float>, dim3(grid), dim3(kStreamBlock), 0, s, a, D,
                       reinterpret_cast<const float2*>(lam), reinterpret_cast<const float2*>(psi),
                       dt, beta_dev, ws.st, ws.partials, ws.gpartials, grad_slot);
  }
  return hipGetLastError();
}

hipError_t launch_ascent(double* u, const double* g, int N, double eta, hipStream_t s) {
  hipLaunchKernelGGL(k_ascent, dim3(1), dim3(1024), 0, s, u, g, N, eta);
  return hipGetLastError();
}

hipError_t launch_index_map(int L, uint32_t s0, uint32_t count, int32_t* n_anti, uint32_t* pmask,
                            hipStream_t s) {
  const uint32_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_index_map, dim3(blocks), dim3(256), 0, s, L, s0, count, n_anti, pmask);
  return hipGetLastError();
}

}  // namespace kg
