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

// One arrival word per team member (teams of at most 64): member r writes the
// number of barriers it has reached to flag[r].
struct TeamSync {
  uint32_t flag[64];
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
  cplx_d bmeas[kMaxScal];   // this member's pass B measurements, for the next step's sums
  double beta0;
  double normT;
  int m_eff;
  int done;
};

__device__ __forceinline__ const float2* bslot(const BCtx& c, const float2* in, int i) {
  return i == 0 ? in : c.basis + (size_t)(i - 1) * c.geo.D;
}

// One Krylov call exp(-i t H) in -> out for the team (out may equal in).
// Each step k is two passes over the member's tiles, as in the single-chain
// kernels: pass A forms y = H v_k and only <v_k|y>, ||v_k||^2; the team sums
// them together with pass B(k-1)'s measurements, and every member runs the
// scalar update (breakdown test, window dots derived from the measurements,
// projection coefficients); pass B then reads the window once to form
// w = s_k y - sum_i c_i v_i and measures <v_j|y> and <v_j|v_k> for the next
// step's window dots.  A team barrier after pass B makes v_{k+1} visible to
// the members that read its tiles as H v partners.
__device__ bool team_krylov(BCtx& c, const kg_chain& ch, double t, double tol, const float2* in,
                            float2* out, KScal& K, float2* lds, cplx_d* wacc, cplx_d* tot,
                            FinScalars& fs) {
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
  int i0p = 0;
  for (int k = 0; k < m; ++k) {
    const bool last = (k == m - 1);
    const int i0 = last ? k : (ch.reorth ? 0 : (k > 0 ? k - 1 : 0));
    const int i0n = (k + 1 == m - 1) ? k + 1 : (ch.reorth ? 0 : k);
    const int nwin = k - i0 + 1;
    // window dots of step k come from pass B(k-1)'s measurements of nb vectors
    const int nb = (k > 0 && i0 < k) ? k - i0p : 0;
    const int ca = 2 * nb, ns = ca + 2;
    const float2* x = bslot(c, in, k);
    // ---- pass A(k): y = H x, <x|y> and <x|x>
    double acc = 0.0;
    for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
      __syncthreads();
      hv_tile<float, kBRB, true>(T, c.hv, c.geo, tile, x, lds, u);
      const uint32_t s = (tile << kBTB) | lane | (wv << 6);
      if (!last) c.ybuf[s] = V{T.yr[0], T.yi[0]};   // for pass B of this member
      const double xr = T.xr[0], xi = T.xi[0], yr = T.yr[0], yi = T.yi[0];
      acc += quad_sums(xr * yr + xi * yi, xr * yi - xi * yr, xr * xr + xi * xi, 0.0);
    }
    __syncthreads();
    if (lane < 4u) reinterpret_cast<double*>(&wacc[wv * kMaxScal + ca])[lane] = (lane < 3u) ? acc : 0.0;
    // pass B(k-1)'s block totals join the sums of this step
    for (int j = threadIdx.x; j < ca; j += blockDim.x) tot[j] = K.bmeas[j];
    if (k > 0 && threadIdx.x == 0) tot[ns] = K.bmeas[ca];
    __syncthreads();
    block_totals(wacc, ns, tot, ca);
    if (!team_reduce(c, tot, k > 0 ? ns + 1 : ns)) return false;
    // ---- scalar update of step k on wavefront 0 of every member
    if (threadIdx.x < 64) {
      const int l = threadIdx.x;
      if (k > 0) {
        // the earlier steps' scalars for the window dots, staged from K
        fs.alpha[l] = K.alpha[l];
        fs.offd[l] = K.offd[l];
        fs.scale[l] = K.scale[l];
        fs.coef[l] = K.coef[(k - 1) & 1][l];
        fs.gprev[l] = K.gcol[k & 1][l];
        fs.cdiag[l] = K.cdiag[l];
        fs.csub[l] = K.csub[l];
        if (l == 0) {
          fs.normT = K.normT;
          fs.beta0 = K.beta0;
        }
      }
      bool go = true;
      double sk = 0.0, bk = 0.0;
      if (k == 0) {
        const double nn = tot[ca + 1].re;
        if (!(nn > 0.0)) {
          // a zero input gives a zero output; a non-finite one a NaN output
          go = false;
          if (l == 0) {
            K.beta0 = (nn == 0.0) ? 0.0 : NAN;
            K.m_eff = (nn == 0.0) ? 0 : 1;
            K.alpha[0] = 0.0;
            K.scale[0] = 1.0;
            K.done = 1;
          }
        } else {
          sk = 1.0 / sqrt(nn);
          if (l == 0) {
            K.beta0 = sqrt(nn);
            K.scale[0] = sk;
            K.offd[0] = 0.0;
          }
        }
      } else {
        // ||w|| of pass B(k-1): the off-diagonal entry of step k, or a breakdown
        bk = sqrt(tot[ns].re);
        if (bk <= tol * fmax(1.0, fs.normT)) {
          go = false;
          if (l == 0) {
            K.m_eff = k;
            K.done = 1;
          }
        } else {
          sk = 1.0 / bk;
          if (l == 0) {
            K.offd[k] = bk;
            K.scale[k] = sk;
          }
        }
      }
      if (go) {
        const cplx_d d = (nb > 0) ? window_dots(k, i0, i0p, fs, tot, nb, tot[ns].re, K.gcol[(k - 1) & 1])
                                  : cplx_d{0.0, 0.0};
        if (l < nwin) {
          const int i = i0 + l;
          const double si = (i == k) ? sk : K.scale[i];
          const double f = si * sk;
          const cplx_d tt = (i == k) ? tot[ca] : d;
          const cplx_d cc{tt.re * f * si, tt.im * f * si};
          K.coef[k & 1][l] = cc;
          if (i == k) K.cdiag[k] = cc;
          if (i == k - 1) K.csub[k] = cc;
        }
        const double alpha = tot[ca].re * sk * sk;
        if (l == 0) {
          K.alpha[k] = alpha;
          K.normT = fmax(k == 0 ? 0.0 : fs.normT, fabs(alpha) + (k == 0 ? 0.0 : bk));
          if (last) {
            K.m_eff = m;
            K.done = 1;
          }
        }
      }
    }
    __syncthreads();
    i0p = i0;
    if (K.done) break;
    // ---- pass B(k): w = s_k y - sum_i c_i v_i -> stored v_{k+1}; ||w||^2 and,
    // when step k+1 has window dots, <v_j|y> (columns [0, nbo)) and <v_j|v_k>
    // (columns [nbo, 2nbo)) for the window vectors j
    const int nbo = (i0n <= k) ? nwin : 0;
    const double sk = K.scale[k];
    const cplx_d* cf = K.coef[k & 1];
    float2* vout = c.basis + (size_t)k * c.geo.D;
    cplx_d* wrow = wacc + wv * kMaxScal;
    for (int j = (int)lane; j < 2 * nbo; j += 64) wrow[j] = cplx_d{0.0, 0.0};
    double bnn = 0.0;
    const auto add_quad = [&](int w, double tq) {
      if (lane < 4u) {
        cplx_d& d = wrow[(lane < 2u ? 0 : nbo) + w];
        if (lane & 1u) {
          d.im += tq;
        } else {
          d.re += tq;
        }
      }
    };
    for (uint32_t tile = c.member; tile < c.geo.ntiles; tile += c.team) {
      const uint32_t s = (tile << kBTB) | lane | (wv << 6);
      const V yv = c.ybuf[s];
      const V xv = x[s];
      const double yr = yv.x, yi = yv.y, xr = xv.x, xi = xv.y;
      double zr, zi;
      {
        const cplx_d cc = cf[k - i0];
        zr = sk * yr - (cc.re * xr - cc.im * xi);
        zi = sk * yi - (cc.re * xi + cc.im * xr);
      }
      if (nbo) add_quad(k - i0, quad_sums(xr * yr + xi * yi, xr * yi - xi * yr, xr * xr + xi * xi, 0.0));
      for (int i = i0; i < k; i += 8) {
        V q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (i + j < k) q[j] = bslot(c, in, i + j)[s];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (i + j < k) {
            const cplx_d cc = cf[i + j - i0];
            const double vr = q[j].x, vi = q[j].y;
            zr -= cc.re * vr - cc.im * vi;
            zi -= cc.re * vi + cc.im * vr;
            if (nbo)
              add_quad(i + j - i0, quad_sums(vr * yr + vi * yi, vr * yi - vi * yr,
                                             vr * xr + vi * xi, vr * xi - vi * xr));
          }
        }
      }
      V o;
      o.x = (float)zr;
      o.y = (float)zi;
      st_coh(&vout[s], o);      // read by other members as H v partners
      bnn += wave_sum((double)o.x * (double)o.x + (double)o.y * (double)o.y);
    }
    if (lane == 0) wrow[2 * nbo] = cplx_d{bnn, 0.0};
    __syncthreads();
    block_totals(wacc, 2 * nbo + 1, K.bmeas);
    // v_{k+1} complete in every member before any member reads its partners
    if (!team_barrier(c)) return false;
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
