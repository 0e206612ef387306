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
// no member ever waits for a single "last" block.  The barrier is an arrival
// counter plus a generation word in global memory; its spin is bounded, and a
// timeout sets the status word, which makes every other waiting member leave as
// well, so every wavefront of the launch terminates.  Teams of one workgroup
// synchronise with __syncthreads only.
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

struct TeamSync {
  uint32_t count;
  uint32_t gen;
  uint32_t pad_[62];
};

// Scratch of one chain at kg_chain::off_ws: sync word, two partial buffers,
// the m-1 Krylov basis vectors, the costate vector and y = H v_k.
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
  float2* ybuf;       // y = H v_k of the running step (own tiles only)
  int32_t* status;
};

__device__ bool team_barrier(BCtx& c) {
  __shared__ int ok;
  __syncthreads();
  // every wavefront's stores are complete before the block is counted
  complete_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    if (c.team > 1) {
      const uint32_t target = c.gen + 1;
      const uint32_t arrived =
          __hip_atomic_fetch_add(&c.sync->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
      if (arrived == c.team) {
        __hip_atomic_store(&c.sync->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        complete_stores();   // the reset lands before the new generation is seen
        __hip_atomic_store(&c.sync->gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t it = 0;
        while (__hip_atomic_load(&c.sync->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
          if (__hip_atomic_load(c.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            good = 0;
            break;
          }
          if (++it > kSpinLimit) {
            __hip_atomic_store(c.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            good = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      c.gen = target;
    }
    ok = good;
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

// Scalars of the running Krylov call, held in LDS by every member.
struct KScal {
  double alpha[kMaxM];
  double offd[kMaxM + 1];
  double scale[kMaxM + 1];
  cplx_d coef[kMaxM];
  cplx_d dcomb[kMaxM];
  double beta0;
  double normT;
  int m_eff;
  int done;
};

__device__ __forceinline__ const float2* bslot(const BCtx& c, const float2* in, int i) {
  return i == 0 ? in : c.basis + (size_t)(i - 1) * c.geo.D;
}

// One Krylov call exp(-i t H) in -> out for the team (out may equal in).
__device__ bool team_krylov(BCtx& c, const kg_chain& ch, double t, double tol, const float2* in,
                            float2* out, KScal& K, float2* lds, cplx_d* wacc, cplx_d* tot) {
  using V = float2;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = uniform_u32(threadIdx.x >> 6);
  const int m = ch.m;
  const double u = *c.hv.u_ptr;
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
    const float2* x = bslot(c, in, k);
    // ---- pass A(k): y = H x, <v_i|y> over the window, <x|x>
    double acc_re = 0.0, acc_im = 0.0, acc_nn = 0.0;
    for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
      __syncthreads();
      hv_tile<float, kBRB, true>(T, c.hv, c.geo, tile, x, lds, u);
      const uint32_t s = (tile << kBTB) | lane | (wv << 6);
      const double yr = T.yr[0], yi = T.yi[0];
      if (!last) c.ybuf[s] = V{T.yr[0], T.yi[0]};   // for pass B of this member
      for (int i = i0; i < k; i += 8) {
        V q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (i + j < k) q[j] = bslot(c, in, i + j)[s];
        // two window vectors' dots per wavefront sum: quad_sums leaves value v
        // of {Re, Im of vector j, Re, Im of vector j+1} in lane v
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          if (i + j < k) {
            const bool two = i + j + 1 < k;
            const double s0 = (double)q[j].x * yr + (double)q[j].y * yi;
            const double s1 = (double)q[j].x * yi - (double)q[j].y * yr;
            const double s2 = two ? (double)q[j + 1].x * yr + (double)q[j + 1].y * yi : 0.0;
            const double s3 = two ? (double)q[j + 1].x * yi - (double)q[j + 1].y * yr : 0.0;
            const double t = quad_sums(s0, s1, s2, s3);
            if ((int)lane == i + j - i0) {
              acc_re += lane_value(t, 0);
              acc_im += lane_value(t, 1);
            }
            if (two && (int)lane == i + j + 1 - i0) {
              acc_re += lane_value(t, 2);
              acc_im += lane_value(t, 3);
            }
          }
        }
      }
      {
        const double xr = T.xr[0], xi = T.xi[0];
        const double t = quad_sums(xr * yr + xi * yi, xr * yi - xi * yr, xr * xr + xi * xi, 0.0);
        if ((int)lane == k - i0) {
          acc_re += lane_value(t, 0);
          acc_im += lane_value(t, 1);
        }
        acc_nn += lane_value(t, 2);
      }
    }
    __syncthreads();
    if ((int)lane < nwin) wacc[wv * kMaxScal + lane] = cplx_d{acc_re, acc_im};
    if (lane == 0) wacc[wv * kMaxScal + nwin] = cplx_d{acc_nn, 0.0};
    __syncthreads();
    block_totals(wacc, nwin + 1, tot);
    if (!team_reduce(c, tot, nwin + 1)) return false;
    if (threadIdx.x == 0) {
      double sk;
      bool zero = false;
      if (k == 0) {
        const double nn = tot[nwin].re;
        if (nn == 0.0) {
          zero = true;
          K.beta0 = 0.0;
          K.m_eff = 0;
          K.done = 1;
        } else if (!(nn > 0.0)) {
          // a non-finite input: exp(0) times NaN, so the output is NaN
          zero = true;
          K.beta0 = NAN;
          K.m_eff = 1;
          K.alpha[0] = 0.0;
          K.scale[0] = 1.0;
          K.done = 1;
        } else {
          K.beta0 = sqrt(nn);
          K.scale[0] = 1.0 / K.beta0;
          K.offd[0] = 0.0;
        }
      }
      if (!zero) {
        sk = K.scale[k];
        for (int l = 0; l < nwin; ++l) {
          const int i = i0 + l;
          const double si = K.scale[i];
          const double f = si * sk;
          K.coef[l] = cplx_d{tot[l].re * f * si, tot[l].im * f * si};
        }
        const double alpha = tot[nwin - 1].re * sk * sk;
        K.alpha[k] = alpha;
        K.normT = fmax(k == 0 ? 0.0 : K.normT, fabs(alpha) + (k == 0 ? 0.0 : K.offd[k]));
        if (last) {
          K.m_eff = m;
          K.done = 1;
        }
      }
    }
    __syncthreads();
    if (K.done) break;
    // ---- pass B(k): w = s_k y - sum_i coef_i v_i -> stored v_{k+1}, ||w||^2
    const double sk = K.scale[k];
    float2* vout = c.basis + (size_t)k * c.geo.D;
    double bnn = 0.0;
    for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
      const uint32_t s = (tile << kBTB) | lane | (wv << 6);
      const V yv = c.ybuf[s];
      const V xv = x[s];
      double zr = sk * (double)yv.x, zi = sk * (double)yv.y;
      for (int i = i0; i < k; i += 8) {
        V q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (i + j < k) q[j] = bslot(c, in, i + j)[s];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (i + j < k) {
            const cplx_d cc = K.coef[i + j - i0];
            zr -= cc.re * (double)q[j].x - cc.im * (double)q[j].y;
            zi -= cc.re * (double)q[j].y + cc.im * (double)q[j].x;
          }
        }
      }
      {
        const cplx_d cc = K.coef[k - i0];
        zr -= cc.re * (double)xv.x - cc.im * (double)xv.y;
        zi -= cc.re * (double)xv.y + cc.im * (double)xv.x;
      }
      V o;
      o.x = (float)zr;
      o.y = (float)zi;
      st_coh(&vout[s], o);      // read by other members as H v partners
      bnn += wave_sum((double)o.x * (double)o.x + (double)o.y * (double)o.y);
    }
    __syncthreads();
    if (lane == 0) wacc[wv * kMaxScal] = cplx_d{bnn, 0.0};
    __syncthreads();
    block_totals(wacc, 1, tot);
    if (!team_reduce(c, tot, 1)) return false;
    if (threadIdx.x == 0) {
      const double b = sqrt(tot[0].re);
      if (b <= tol * fmax(1.0, K.normT)) {
        K.m_eff = k + 1;
        K.done = 1;
      } else {
        K.offd[k + 1] = b;
        K.scale[k + 1] = 1.0 / b;
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
  float2* lds = reinterpret_cast<float2*>(smem_raw);
  cplx_d* wacc = reinterpret_cast<cplx_d*>(smem_raw);
  __shared__ cplx_d tot[kMaxScal];
  __shared__ KScal K;

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
    if (!team_krylov(c, ch, ch.dt, tol, prev, out, K, lds, wacc, tot)) return;
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
      if (!team_krylov(c, ch, -ch.dt, tol, lam, c.lam, K, lds, wacc, tot)) return;
      lam = c.lam;
    }
  }
}

__global__ void k_batched_init(const kg_chain* chains, int n_chains, char* ws, int32_t* status) {
  const int i = blockIdx.x;
  if (i < n_chains && threadIdx.x == 0) {
    TeamSync* s = reinterpret_cast<TeamSync*>(ws + chains[i].off_ws);
    s->count = 0;
    s->gen = 0;
  }
  if (i == 0 && threadIdx.x == 0) *status = 0;
}

}  // namespace

size_t batched_chain_ws_bytes(int L, int m, int team) {
  const size_t vb = ((size_t)1 << L) * sizeof(float2);
  return bws_basis_off(team) + vb * (size_t)(m > 1 ? m - 1 : 0) + 2 * vb;
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
  hipLaunchKernelGGL(k_batched, dim3(n_blocks), dim3(kBThreads), tile > red ? tile : red, s,
                     chains_dev, n_chains, u_all, reinterpret_cast<const float2*>(psi0_all),
                     reinterpret_cast<const float2*>(target_all), reinterpret_cast<float2*>(states_all),
                     F_all, beta_all, grad_all, static_cast<char*>(ws), status);
  return hipGetLastError();
}

}  // namespace kg
