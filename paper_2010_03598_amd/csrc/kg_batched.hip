// Batched form: many independent chains (different L, Delta, N, m) evaluated by
// one persistent launch.  Every chain is served by a team of workgroups that
// runs the chain's whole GRAPE gradient (Algorithm 1 with Krylov propagation,
// App. A): forward sweep, overlap, backward sweep and the per-slice brackets
// of Eq. 5, storing all forward states.  Vectors are complex64, every
// reduction, Lanczos scalar and the small exponential FP64.
//
// Inside a team the work is split by tiles of 1024 amplitudes (one amplitude
// per thread).  Reductions are finished redundantly by every member: each
// member publishes its block totals, waits at the team barrier and adds the
// members' totals in member order, so all members hold identical scalars and
// no member ever waits for a single "last" block.  A Lanczos step is one tile
// pass and one team reduction (team_krylov).  The barrier is one arrival word
// per member in global memory; its spin is bounded, and a timeout sets the
// status word, which makes every other waiting member leave as well, so every
// wavefront of the launch terminates.  Teams of one workgroup synchronise with
// __syncthreads only.
//
// Coherence without device-wide fences: every vector a member writes is stored
// with device-scope (L2 write-through) stores, and every amplitude a member
// reads from another member's tiles (H v partners, the S^x partner of a
// bracket) and every reduction partial is loaded with device-scope loads.  A
// member's own tiles are read with plain loads.  Before arriving at the
// barrier a member waits for its stores to complete; no L2 is ever written
// back or invalidated as a whole.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "kg_device.h"
#include "kg_internal.h"
#include "kgrape.h"

namespace kg {
namespace {

constexpr int kBTB = 10;  // tile bits
constexpr int kBRB = 0;   // one amplitude per thread
constexpr int kBWB = 4;   // 16 wavefronts
constexpr int kBThreads = 64 << kBWB;
constexpr uint32_t kSpinLimit = 1u << 24;

// One arrival word per team member (teams of at most 64): member r writes the
// number of barriers it has reached to flag[r].
struct TeamSync {
  uint32_t flag[64];
};

// Scratch of one chain at kg_chain::off_ws: arrival words, two partial
// buffers, the m-1 Krylov basis vectors, the costate vector, y = H u_k and
// two buffers for w'_k.
__host__ __device__ inline size_t bws_partials_off() { return 256; }
__host__ __device__ inline size_t bws_basis_off(int team) {
  const size_t p = 256 + 2 * (size_t)team * kMaxScal * sizeof(cplx_d);
  return (p + 255) / 256 * 256;
}

struct BCtx {
  HvArgs hv;
  Geo geo;
  uint32_t member, team;
  uint32_t gen;
  uint32_t red;       // reductions done (selects the partial buffer)
  TeamSync* sync;
  cplx_d* partials;   // [2][team][kMaxScal]
  float2* basis;
  float2* lam;
  float2* ybuf;       // y = H u_k of the running step (own tiles only)
  float2* wbuf;       // w'_k, two vectors by the parity of k (H v partners)
  int32_t* status;
};

// Team barrier: every member's device-coherent stores complete, then each
// member publishes its barrier count in its own arrival word and wavefront 0
// polls the team's words (one load per lane) until all have reached it.  No
// read-modify-write and no last-arriver broadcast: an arrival is seen by the
// others as soon as its store lands.  Bounded spin; a timeout or another
// team's failure sets or reads the status word and returns false.
__device__ bool team_barrier(BCtx& c) {
  __shared__ int ok;
  __syncthreads();
  // every wavefront's stores are complete before the block is counted
  complete_stores();
  __syncthreads();
  if (threadIdx.x < 64) {
    int good = 1;
    if (c.team > 1) {
      const uint32_t lane = threadIdx.x;
      const uint32_t target = c.gen + 1;
      if (lane == 0) st_agent_u32(&c.sync->flag[c.member], target);
      uint32_t it = 0;
      while (true) {
        const uint32_t v = (lane < c.team)
                               ? __hip_atomic_load(&c.sync->flag[lane], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)
                               : target;
        if (__all((int32_t)(v - target) >= 0)) break;
        if (__hip_atomic_load(c.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          good = 0;
          break;
        }
        if (++it > kSpinLimit) {
          if (lane == 0) __hip_atomic_store(c.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      c.gen = target;
    }
    if (threadIdx.x == 0) ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Block totals in `tot` -> team totals in `tot` (identical in every member).
__device__ bool team_reduce(BCtx& c, cplx_d* tot, int ns) {
  if (c.team == 1) return true;
  cplx_d* buf = c.partials + (size_t)(c.red & 1u) * c.team * kMaxScal;
  c.red++;
  if (threadIdx.x < 64) {
    for (int j = threadIdx.x; j < ns; j += 64) {
      st_agent(&buf[(size_t)c.member * kMaxScal + j].re, tot[j].re);
      st_agent(&buf[(size_t)c.member * kMaxScal + j].im, tot[j].im);
    }
  }
  if (!team_barrier(c)) return false;
  // lane r takes member r's part (team <= 64); a fixed butterfly adds them, so
  // every member obtains the same sums
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wv; j < ns; j += nw) {
    double re = 0.0, im = 0.0;
    if ((uint32_t)lane < c.team) {
      re = ld_agent(&buf[(size_t)lane * kMaxScal + j].re);
      im = ld_agent(&buf[(size_t)lane * kMaxScal + j].im);
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) tot[j] = cplx_d{re, im};
  }
  __syncthreads();
  return true;
}

// Scalars of the running Krylov call, held in LDS by every member (every member
// computes them from the same team sums, so all hold the same values).  The
// projection coefficients and the measured Gram columns are kept for two
// steps, by the parity of the step; cdiag/csub are step i's coefficients on
// the stored vector i itself and on vector i-1.
struct KScal {
  double alpha[kMaxM];
  double offd[kMaxM + 1];
  double scale[kMaxM + 1];
  cplx_d coef[2][kMaxM];
  cplx_d dcomb[kMaxM];
  cplx_d cdiag[kMaxM];
  cplx_d csub[kMaxM];
  cplx_d gcol[2][kMaxM];
  double beta0;
  double normT;
  int m_eff;
  int done;
};

__device__ __forceinline__ const float2* bslot(const BCtx& c, const float2* in, int i) {
  return i == 0 ? in : c.basis + (size_t)(i - 1) * c.geo.D;
}

// One Krylov call exp(-i t H) in -> out for the team (out may equal in).
//
// One tile pass and one team reduction per Lanczos step.  The newest
// projection coefficient of step k, c_k = s_k^3 <u_k|y_k>, needs a team sum of
// this step's own H v, so its subtraction is deferred: the pass of step k
// stores
//   w'_k = s_k y_k - sum_{i < k in the window} c^(k)_i u_i     (w'_0 = y_0)
// and the pass of step k+1 materialises the stored vector and its H v as
//   u_{k+1} = sig_k w'_k - c_k u_k,   y_{k+1} = sig_k H w'_k - c_k y_k,
// with sig_0 = s_0 = 1/||u_0|| and sig_k = 1 after (H is linear; y_k is the
// member's own tile, kept from the step before).  The team sums after step k
// give alpha_k and c_k, ||u_{k+1}||^2 = ||sig w'||^2 - 2 sig Re(conj(c_k)
// <u_k|w'>) + |c_k|^2 ||u_k||^2 from the pass's measurements, the breakdown
// test, and the window dots and coefficients of step k+1 (window_dots, from
// <u_i|y_k> and <u_i|u_k> measured on the stored vectors, as the
// single-chain passes derive them).  In exact arithmetic u_{k+1} is the
// vector of Algorithm 2 with every coefficient taken against the same y_k.
// w'_k is read by other members as H v partners (device-scope stores, two
// buffers by the parity of k); u_k and y_k only by their own member.
__device__ bool team_krylov(BCtx& c, const kg_chain& ch, double t, double tol, const float2* in,
                            float2* out, KScal& K, float2* lds, cplx_d* wacc, cplx_d* tot,
                            FinScalars& fs) {
  using V = float2;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = uniform_u32(threadIdx.x >> 6);
  const int m = ch.m;
  const double u = *c.hv.u_ptr;
  const uint32_t D = c.geo.D;
  Tile<float, kBRB> T;
  if (threadIdx.x == 0) {
    K.done = 0;
    K.normT = 0.0;
    K.m_eff = m;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const bool last = (k == m - 1);
    const int i0 = last ? k : (ch.reorth ? 0 : (k > 0 ? k - 1 : 0));
    const int nwin = k - i0 + 1;
    // measurement columns: <u_i|y_k> at i - i0, <u_i|u_k> at nwin + i - i0
    // (i in [i0, k]), ||w'||^2 at 2 nwin, <u_k|w'> at 2 nwin + 1
    const int ncol = 2 * nwin + 2;
    const float2* hsrc = (k == 0) ? in : c.wbuf + (size_t)((k - 1) & 1) * D;
    const double sig = (k == 1) ? K.scale[0] : 1.0;
    const cplx_d cl = (k >= 1) ? K.cdiag[k - 1] : cplx_d{0.0, 0.0};
    const double sk = (k >= 1) ? K.scale[k] : 1.0;
    const cplx_d* cf = K.coef[k & 1];
    float2* uk = (k >= 1) ? c.basis + (size_t)(k - 1) * D : nullptr;
    const float2* ul = (k >= 1) ? bslot(c, in, k - 1) : nullptr;
    float2* wk = c.wbuf + (size_t)(k & 1) * D;
    cplx_d* wrow = wacc + wv * kMaxScal;
    for (int j = (int)lane; j < ncol; j += 64) wrow[j] = cplx_d{0.0, 0.0};
    const auto add_quad = [&](int col0, int col1, double tq) {
      // lanes 0, 1: column col0 (re, im); lanes 2, 3: column col1
      if (lane < 4u) {
        cplx_d& d = wrow[lane < 2u ? col0 : col1];
        if (lane & 1u) {
          d.im += tq;
        } else {
          d.re += tq;
        }
      }
    };
    for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
      __syncthreads();
      hv_tile<float, kBRB, true>(T, c.hv, c.geo, tile, hsrc, lds, u);
      const uint32_t s = (tile << kBTB) | lane | (wv << 6);
      // u_k and y_k, rounded as stored
      V uo, yo;
      if (k == 0) {
        uo = V{T.xr[0], T.xi[0]};
        yo = V{T.yr[0], T.yi[0]};
      } else {
        const V up = ul[s], yp = c.ybuf[s];
        uo.x = (float)(sig * (double)T.xr[0] - (cl.re * up.x - cl.im * up.y));
        uo.y = (float)(sig * (double)T.xi[0] - (cl.re * up.y + cl.im * up.x));
        yo.x = (float)(sig * (double)T.yr[0] - (cl.re * yp.x - cl.im * yp.y));
        yo.y = (float)(sig * (double)T.yi[0] - (cl.re * yp.y + cl.im * yp.x));
        uk[s] = uo;
      }
      if (!last) c.ybuf[s] = yo;
      const double xr = uo.x, xi = uo.y, yr = yo.x, yi = yo.y;
      // <u_k|y_k>, ||u_k||^2
      add_quad(nwin - 1, 2 * nwin - 1, quad_sums(xr * yr + xi * yi, xr * yi - xi * yr, xr * xr + xi * xi, 0.0));
      double zr = sk * yr, zi = sk * yi;
      // the window before u_k, eight vectors per round trip
      for (int i = i0; i < k; i += 8) {
        V q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (i + j < k) q[j] = bslot(c, in, i + j)[s];
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          if (i + j < k) {
            double d4[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              d4[h][0] = d4[h][1] = d4[h][2] = d4[h][3] = 0.0;
              if (i + j + h < k) {
                const double vr = q[j + h].x, vi = q[j + h].y;
                const cplx_d cc = cf[i + j + h - i0];
                zr -= cc.re * vr - cc.im * vi;
                zi -= cc.re * vi + cc.im * vr;
                d4[h][0] = vr * yr + vi * yi;
                d4[h][1] = vr * yi - vi * yr;
                d4[h][2] = vr * xr + vi * xi;
                d4[h][3] = vr * xi - vi * xr;
              }
            }
            const double tq = quad_sums_pair(d4[0][0], d4[0][1], d4[0][2], d4[0][3], d4[1][0],
                                             d4[1][1], d4[1][2], d4[1][3]);
            // lanes 0..3: vector i + j; lanes 4..7: vector i + j + 1
            const int h = (int)((lane >> 2) & 1u);
            if (lane < 8u && i + j + h < k) {
              const uint32_t l4 = lane & 3u;
              const int w = i + j + h - i0;
              cplx_d& d = wrow[l4 < 2u ? w : nwin + w];
              if (l4 & 1u) {
                d.im += tq;
              } else {
                d.re += tq;
              }
            }
          }
        }
      }
      if (!last) {
        V o;
        o.x = (float)zr;
        o.y = (float)zi;
        st_coh(&wk[s], o);      // read by other members as H v partners
        const double orr = o.x, oi = o.y;
        add_quad(2 * nwin, 2 * nwin + 1,
                 quad_sums(orr * orr + oi * oi, 0.0, xr * orr + xi * oi, xr * oi - xi * orr));
      }
    }
    __syncthreads();
    block_totals(wacc, ncol, tot);
    if (!team_reduce(c, tot, ncol)) return false;
    // ---- scalars after step k (wavefront 0 of every member, the same values)
    if (threadIdx.x < 64) {
      const int l = threadIdx.x;
      fs.alpha[l] = K.alpha[l];
      fs.offd[l] = K.offd[l];
      fs.scale[l] = K.scale[l];
      fs.coef[l] = K.coef[k & 1][l];
      fs.gprev[l] = K.gcol[(k + 1) & 1][l];
      fs.cdiag[l] = K.cdiag[l];
      fs.csub[l] = K.csub[l];
      const cplx_d tkk = tot[nwin - 1];
      const double ukk = tot[2 * nwin - 1].re;
      bool go = true;
      double s = sk;
      if (k == 0) {
        if (!(ukk > 0.0)) {
          // a zero input gives a zero output; a non-finite one a NaN output
          go = false;
          if (l == 0) {
            K.beta0 = (ukk == 0.0) ? 0.0 : NAN;
            K.m_eff = (ukk == 0.0) ? 0 : 1;
            K.alpha[0] = 0.0;
            K.scale[0] = 1.0;
            K.done = 1;
          }
        } else {
          s = 1.0 / sqrt(ukk);
          if (l == 0) {
            K.beta0 = sqrt(ukk);
            K.scale[0] = s;
            K.offd[0] = 0.0;
          }
          fs.scale[0] = s;
        }
      }
      if (go) {
        // alpha_k and c^(k)_k
        const double alpha = tkk.re * s * s;
        const cplx_d ckk{tkk.re * s * s * s, tkk.im * s * s * s};
        const double normT = fmax(k == 0 ? 0.0 : K.normT, fabs(alpha) + (k == 0 ? 0.0 : K.offd[k]));
        if (l == k - i0) fs.coef[l] = ckk;
        if (l == k) fs.cdiag[l] = ckk;
        if (l == 0) {
          K.alpha[k] = alpha;
          K.coef[k & 1][k - i0] = ckk;
          K.cdiag[k] = ckk;
          K.normT = normT;
        }
        if (last) {
          if (l == 0) {
            K.m_eff = m;
            K.done = 1;
          }
        } else {
          // ||u_{k+1}||^2 of the deferred subtraction, or a breakdown (an
          // invariant Krylov space of dimension k + 1)
          const double sg = (k == 0) ? s : 1.0;
          const cplx_d pw = tot[2 * nwin + 1];
          double b2 = sg * sg * tot[2 * nwin].re - 2.0 * sg * (ckk.re * pw.re + ckk.im * pw.im) +
                      (ckk.re * ckk.re + ckk.im * ckk.im) * ukk;
          b2 = fmax(b2, 0.0);
          const double bk = sqrt(b2);
          if (bk <= tol * fmax(1.0, normT)) {
            if (l == 0) {
              K.m_eff = k + 1;
              K.done = 1;
            }
          } else {
            const double sn = 1.0 / bk;
            if (l == 0) {
              K.offd[k + 1] = bk;
              K.scale[k + 1] = sn;
            }
            // window dots and coefficients of step k + 1 (all but the newest)
            const int kn = k + 1;
            const int i0n = (kn == m - 1) ? kn : (ch.reorth ? 0 : kn - 1);
            const int nwn = kn - i0n + 1;
            if (nwn > 1) {
              const cplx_d d = window_dots(kn, i0n, i0, fs, tot, nwin, b2, K.gcol[k & 1]);
              if (l < nwn - 1) {
                const int i = i0n + l;
                const double si = fs.scale[i];
                const cplx_d cc{d.re * si * si * sn, d.im * si * si * sn};
                K.coef[kn & 1][l] = cc;
                if (i == k) K.csub[kn] = cc;
              }
            }
          }
        }
      }
    }
    __syncthreads();
    if (K.done) break;
  }
  // ---- exp(-itT) e_1 on wavefront 0 and the combination coefficients
  const int me = K.m_eff;
  if (threadIdx.x < 64) {
    const int i = threadIdx.x;
    double ai = 0.0, lo = 0.0, hi = 0.0;
    if (i < me) {
      ai = K.alpha[i];
      lo = (i > 0) ? K.offd[i] : 0.0;
      hi = (i + 1 < me) ? K.offd[i + 1] : 0.0;
    }
    double cr, ci;
    tri_exp_wave(ai, lo, hi, t, cr, ci);
    if (i < me) K.dcomb[i] = cplx_d{K.beta0 * cr * K.scale[i], K.beta0 * ci * K.scale[i]};
  }
  __syncthreads();
  // ---- combination v_out = sum_j dcomb_j v_j (FP64 accumulation)
  for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
    const uint32_t s = (tile << kBTB) | threadIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int j0 = 0; j0 < me; j0 += 8) {
      V q[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (j0 + jj < me) q[jj] = bslot(c, in, j0 + jj)[s];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        if (j0 + jj < me) {
          const cplx_d d = K.dcomb[j0 + jj];
          ar += d.re * (double)q[jj].x - d.im * (double)q[jj].y;
          ai += d.re * (double)q[jj].y + d.im * (double)q[jj].x;
        }
      }
    }
    V o;
    o.x = (float)ar;
    o.y = (float)ai;
    st_coh(&out[s], o);
  }
  return team_barrier(c);
}

// Team sum of sum_s conj(a[s]) * (op b)[s] with op = identity or Hc.
__device__ bool team_dot(BCtx& c, const float2* a, const float2* b, bool apply_hc, cplx_d* wacc,
                         cplx_d* tot, cplx_d& result) {
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  double sr = 0.0, si = 0.0;
  const uint32_t flip = (apply_hc && c.hv.hc_kind == 0) ? (1u << c.hv.hc_bit) : 0u;
  for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
    const uint32_t s = (tile << kBTB) | threadIdx.x;
    const float2 x = a[s];
    const float2 y = flip ? ld_coh(&b[s ^ flip]) : b[s];   // the S^x partner may be another member's
    double w = 1.0;
    if (apply_hc) {
      w = (c.hv.hc_kind == 0) ? 0.5 : 0.5 * c.hv.sz_count - (double)__popc(s & c.hv.sz_mask);
    }
    const double yr = w * (double)y.x, yi = w * (double)y.y;
    sr += (double)x.x * yr + (double)x.y * yi;
    si += (double)x.x * yi - (double)x.y * yr;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  __syncthreads();
  if (lane == 0) wacc[wv * kMaxScal] = cplx_d{sr, si};
  __syncthreads();
  block_totals(wacc, 1, tot);
  if (!team_reduce(c, tot, 1)) return false;
  result = tot[0];
  __syncthreads();
  return true;
}

__global__ void __launch_bounds__(kBThreads)
    k_batched(const kg_chain* __restrict__ chains, int n_chains, const double* u_all,
              const float2* psi0_all, const float2* target_all, float2* states_all, double* F_all,
              double* beta_all, double* grad_all, char* ws, int32_t* status) {
  extern __shared__ unsigned char smem_raw[];
  // the H v tile, then the per-wavefront accumulator rows (used together)
  float2* lds = reinterpret_cast<float2*>(smem_raw);
  cplx_d* wacc = reinterpret_cast<cplx_d*>(smem_raw + ((size_t)1 << kBTB) * sizeof(float2));
  __shared__ cplx_d tot[kMaxScal];
  __shared__ KScal K;
  __shared__ FinScalars fs;

  // the chain of this workgroup
  int cid = -1;
  for (int i = 0; i < n_chains; ++i) {
    const int f = chains[i].team_first, n = chains[i].team_size;
    if ((int)blockIdx.x >= f && (int)blockIdx.x < f + n) cid = i;
  }
  if (cid < 0) return;
  const kg_chain ch = chains[cid];
  const int L = ch.h.L;
  BCtx c;
  c.member = blockIdx.x - ch.team_first;
  c.team = ch.team_size;
  c.gen = 0;
  c.red = 0;
  char* cw = ws + ch.off_ws;
  c.sync = reinterpret_cast<TeamSync*>(cw);
  c.partials = reinterpret_cast<cplx_d*>(cw + bws_partials_off());
  c.basis = reinterpret_cast<float2*>(cw + bws_basis_off(ch.team_size));
  const uint32_t D = 1u << L;
  c.lam = c.basis + (size_t)(ch.m > 1 ? ch.m - 1 : 0) * D;
  c.ybuf = c.lam + D;
  c.wbuf = c.ybuf + D;
  c.status = status;
  c.geo.L = L;
  c.geo.TB = kBTB;
  c.geo.RB = kBRB;
  c.geo.WB = kBWB;
  c.geo.D = D;
  c.geo.ntiles = D >> kBTB;
  c.geo.small = 0;
  c.geo.grid = ch.team_size;
  c.hv.L = L;
  c.hv.hc_kind = ch.h.hc_kind;
  c.hv.hc_bit = 0;
  c.hv.sz_mask = 0;
  c.hv.sz_count = 0;
  if (ch.h.hc_kind == 0) {
    c.hv.hc_bit = L - (__builtin_ctzll(ch.h.hc_sites) + 1);
  } else {
    for (int i = 1; i <= L; ++i) {
      if ((ch.h.hc_sites >> (i - 1)) & 1ull) {
        c.hv.sz_mask |= 1u << (L - i);
        c.hv.sz_count++;
      }
    }
  }
  c.hv.pad_ = 0;
  c.hv.half_J = 0.5 * ch.h.J;
  c.hv.c_zz = 0.25 * ch.h.J * ch.h.Delta;
  c.hv.u_val = 0.0;
  const double tol = ch.breakdown_tol > 0.0 ? ch.breakdown_tol : 64.0 * ldexp(1.0, -23);

  const double* u = u_all + ch.off_u;
  const float2* psi0 = psi0_all + ch.off_vec;
  const float2* target = target_all + ch.off_vec;
  float2* states = states_all + ch.off_states;
  double* grad = grad_all + ch.off_u;

  // forward sweep: psi_j = exp(-i dt H_j) psi_{j-1}, stored as states[j-1]
  const float2* prev = psi0;
  for (int j = 1; j <= ch.N; ++j) {
    c.hv.u_ptr = u + (j - 1);
    float2* out = states + (size_t)(j - 1) * D;
    if (!team_krylov(c, ch, ch.dt, tol, prev, out, K, lds, wacc, tot, fs)) return;
    prev = out;
  }
  cplx_d beta;
  if (!team_dot(c, target, prev, false, wacc, tot, beta)) return;
  if (c.member == 0 && threadIdx.x == 0) {
    F_all[cid] = beta.re * beta.re + beta.im * beta.im;
    beta_all[2 * cid] = beta.re;
    beta_all[2 * cid + 1] = beta.im;
  }
  // backward sweep with the gradient brackets
  const float2* lam = target;
  for (int j = ch.N; j >= 1; --j) {
    cplx_d B;
    if (!team_dot(c, lam, states + (size_t)(j - 1) * D, true, wacc, tot, B)) return;
    if (c.member == 0 && threadIdx.x == 0) grad[j - 1] = 2.0 * ch.dt * (beta.re * B.im - beta.im * B.re);
    if (j > 1) {
      c.hv.u_ptr = u + (j - 1);
      if (!team_krylov(c, ch, -ch.dt, tol, lam, c.lam, K, lds, wacc, tot, fs)) return;
      lam = c.lam;
    }
  }
}

__global__ void k_batched_init(const kg_chain* chains, int n_chains, char* ws, int32_t* status) {
  const int i = blockIdx.x;
  if (i < n_chains && threadIdx.x < 64) {
    TeamSync* s = reinterpret_cast<TeamSync*>(ws + chains[i].off_ws);
    s->flag[threadIdx.x] = 0u;
  }
  if (i == 0 && threadIdx.x == 0) *status = 0;
}

}  // namespace

size_t batched_chain_ws_bytes(int L, int m, int team) {
  const size_t vb = ((size_t)1 << L) * sizeof(float2);
  // basis, costate, y, and the two w' buffers
  return bws_basis_off(team) + vb * (size_t)(m > 1 ? m - 1 : 0) + 4 * vb;
}

hipError_t launch_batched(const kg_chain* chains_dev, int n_chains, int n_blocks, const double* u_all,
                          const void* psi0_all, const void* target_all, void* states_all,
                          double* F_all, double* beta_all, double* grad_all, void* ws,
                          int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_batched_init, dim3(n_chains), dim3(64), 0, s, chains_dev, n_chains,
                     static_cast<char*>(ws), status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t tile = ((size_t)1 << kBTB) * sizeof(float2);
  const size_t red = ((size_t)kBThreads / 64) * kMaxScal * sizeof(cplx_d);
  hipLaunchKernelGGL(k_batched, dim3(n_blocks), dim3(kBThreads), tile + red, s,
                     chains_dev, n_chains, u_all, reinterpret_cast<const float2*>(psi0_all),
                     reinterpret_cast<const float2*>(target_all), reinterpret_cast<float2*>(states_all),
                     F_all, beta_all, grad_all, static_cast<char*>(ws), status);
  return hipGetLastError();
}

}  // namespace kg
