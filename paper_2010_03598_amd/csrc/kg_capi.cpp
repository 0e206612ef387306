// C ABI of libkgrape (declared in include/kgrape.h): argument validation,
// workspace carving and the orchestration of the GRAPE sweeps (Algorithm 1)
// on top of the kernels in kg_kernels.hip.  No entry point allocates device
// memory or synchronises the stream.

#include "kgrape.h"

#include <hip/hip_runtime_api.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kg_internal.h"

namespace kg {

namespace {

thread_local std::string g_last_error;

kg_status fail(kg_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

kg_status ok() {
  g_last_error.clear();
  return KG_OK;
}

kg_status hip_fail(hipError_t e, const char* where) {
  return fail(KG_EDEVICE, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

#define KG_CHECK(x)                                  \
  do {                                               \
    kg_status st_ = (x);                             \
    if (st_ != KG_OK) return st_;                    \
  } while (0)

#define KG_HIP(x, where)                             \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

kg_status check_xxz(const kg_xxz* h, int max_L = KG_MAX_L) {
  if (!h) return fail(KG_EINVAL, "h is NULL");
  if (h->L < KG_MIN_L || h->L > max_L)
    return fail(KG_EINVAL, "L=%d outside [%d, %d]", h->L, KG_MIN_L, max_L);
  if (!isfinite(h->J) || !isfinite(h->Delta)) return fail(KG_EINVAL, "J and Delta must be finite");
  if (h->hc_kind != KG_HC_SX && h->hc_kind != KG_HC_SZ)
    return fail(KG_EINVAL, "unknown hc_kind %d", h->hc_kind);
  if (h->hc_sites == 0) return fail(KG_EINVAL, "hc_sites is empty");
  if (h->hc_sites >> h->L) return fail(KG_EINVAL, "hc_sites names a site beyond L=%d", h->L);
  if (h->hc_kind == KG_HC_SX && __builtin_popcountll(h->hc_sites) != 1)
    return fail(KG_EINVAL, "KG_HC_SX needs exactly one site");
  return KG_OK;
}

kg_status check_krylov(const kg_krylov* k) {
  if (!k) return fail(KG_EINVAL, "k is NULL");
  if (k->m < 1 || k->m > KG_MAX_M) return fail(KG_EINVAL, "m=%d outside [1, %d]", k->m, KG_MAX_M);
  if (k->reorth != 0 && k->reorth != 1) return fail(KG_EINVAL, "reorth must be 0 or 1");
  if (!(k->breakdown_tol >= 0.0) || !isfinite(k->breakdown_tol))
    return fail(KG_EINVAL, "breakdown_tol must be finite and >= 0");
  return KG_OK;
}

kg_status check_prec(int32_t prec) {
  if (prec != KG_C128 && prec != KG_C64) return fail(KG_EINVAL, "unknown precision %d", prec);
  return KG_OK;
}

kg_status check_vec(const void* p, int32_t prec, const char* name) {
  if (!p) return fail(KG_EINVAL, "%s is NULL", name);
  const uintptr_t a = prec == KG_C128 ? 16 : 8;
  if ((uintptr_t)p % a) return fail(KG_EINVAL, "%s is not %d-byte aligned", name, (int)a);
  return KG_OK;
}

bool overlap(const void* a, const void* b, size_t n) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + n && y < x + n;
}

double default_tol(int32_t prec) { return 64.0 * (prec == KG_C128 ? ldexp(1.0, -52) : ldexp(1.0, -23)); }

HvArgs make_hv(const kg_xxz* h, const double* u_ptr, double u_val) {
  HvArgs a;
  memset(&a, 0, sizeof(a));
  a.L = h->L;
  a.hc_kind = h->hc_kind;
  if (h->hc_kind == KG_HC_SX) {
    const int site = __builtin_ctzll(h->hc_sites) + 1;
    a.hc_bit = h->L - site;
  } else {
    uint32_t mask = 0;
    int cnt = 0;
    for (int i = 1; i <= h->L; ++i) {
      if ((h->hc_sites >> (i - 1)) & 1ull) {
        mask |= 1u << (h->L - i);
        ++cnt;
      }
    }
    a.sz_mask = mask;
    a.sz_count = cnt;
  }
  a.half_J = 0.5 * h->J;
  a.c_zz = 0.25 * h->J * h->Delta;
  a.u_ptr = u_ptr;
  a.u_val = u_val;
  return a;
}

size_t vbytes(uint64_t D, int32_t prec) { return (size_t)D * (prec == KG_C128 ? 16 : 8); }

// A Krylov slot: scalars, reduction partials, basis vectors 1..m-1 and the
// vector y_k = H v_k of the running step.
size_t slot_bytes_d(uint64_t D, const kg_krylov* k, int32_t prec) {
  return ws_fixed_bytes() + align_up(vbytes(D, prec) * (size_t)(k->m - 1), 256) +
         align_up(vbytes(D, prec), 256);
}

// workspace of vectors of D amplitudes; `extended` adds the two node vectors
size_t ws_bytes_d(uint64_t D, const kg_krylov* k, int32_t prec, bool extended) {
  return 2 * slot_bytes_d(D, k, prec) + align_up(vbytes(D, prec), 256) +
         (extended ? 2 * align_up(vbytes(D, prec), 256) : 0);
}

// The workspace holds two Krylov slots (scalars, reduction partials, m-1
// basis vectors and the H v_k vector each) and one costate vector.  Slot 0 serves single calls and
// the backward sweep, slot 1 the segment recomputation advanced beside it.
size_t states_bytes_d(uint64_t D, int32_t N, int32_t ckpt_every, int32_t prec) {
  const size_t vb = vbytes(D, prec);
  if (ckpt_every == 0) return vb * (size_t)N;
  const int nseg = (N + ckpt_every - 1) / ckpt_every;
  const int nbuf = nseg > 1 ? 2 : 1;
  return vb * (size_t)(nseg - 1 + nbuf * ckpt_every);
}

kg_status carve_d(void* ws, size_t ws_bytes, uint64_t D, const kg_krylov* k, int32_t prec,
                  Workspace* out0, Workspace* out1, bool extended = false) {
  if (!ws) return fail(KG_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(KG_EWORKSPACE, "workspace is not 256-byte aligned");
  const size_t need = ws_bytes_d(D, k, prec, extended);
  if (ws_bytes < need)
    return fail(KG_EWORKSPACE, "workspace has %zu bytes, needs %zu%s", ws_bytes, need,
                extended ? " (extended)" : "");
  char* p = static_cast<char*>(ws);
  const size_t vb = align_up(vbytes(D, prec), 256);
  Workspace* outs[2] = {out0, out1};
  for (int i = 0; i < 2; ++i) {
    Workspace* o = outs[i];
    char* q = p + (size_t)i * slot_bytes_d(D, k, prec);
    if (!o) continue;
    o->st = reinterpret_cast<KState*>(q);
    q += align_up(sizeof(KState), 256);
    o->partials = reinterpret_cast<cplx_d*>(q);
    q += align_up(sizeof(cplx_d) * kPartialRows * kMaxScal, 256);
    o->basis = q;
    q += align_up(vbytes(D, prec) * (size_t)(k->m - 1), 256);
    o->yk = q;
    o->lam = p + 2 * slot_bytes_d(D, k, prec);
    o->node_a = extended ? static_cast<char*>(o->lam) + vb : nullptr;
    o->node_b = extended ? static_cast<char*>(o->lam) + 2 * vb : nullptr;
  }
  return KG_OK;
}


// Where the forward states live in the caller's state buffer.  With
// checkpoints every c slices, segment q holds slices (q c, (q+1) c]; psi_{(q+1)c}
// of every segment but the last is a checkpoint, the other states of segment q
// go to segment buffer (q mod 2).  The forward sweep therefore leaves the last
// two segments in the buffers, and during the backward sweep of segment q the
// other buffer receives the recomputation of segment q-1.
struct States {
  int N = 0, c = 0, nseg = 1, nbuf = 1;
  char* base = nullptr;
  size_t vb = 0;
  const void* psi0 = nullptr;

  void* ckpt(int q) const { return base + (size_t)(q - 1) * vb; }  // psi_{q c}, 1 <= q < nseg
  void* buf(int q, int i) const {
    const int b = (nbuf == 2) ? (q & 1) : 0;
    return base + (size_t)(nseg - 1 + b * c + i) * vb;
  }
  // slot of psi_j (j >= 1), in the forward sweep and after recomputation alike
  void* at(int j) const {
    if (c == 0) return base + (size_t)(j - 1) * vb;
    const int q = (j - 1) / c;
    if (j % c == 0 && q < nseg - 1) return ckpt(q + 1);
    return buf(q, j - q * c - 1);
  }
  const void* at0(int j) const { return j == 0 ? psi0 : at(j); }
};

States make_states(int N, int c, void* base, size_t vb, const void* psi0) {
  States s;
  s.N = N;
  s.c = c;
  s.base = static_cast<char*>(base);
  s.vb = vb;
  s.psi0 = psi0;
  if (c > 0) {
    s.nseg = (N + c - 1) / c;
    s.nbuf = s.nseg > 1 ? 2 : 1;
  }
  return s;
}

struct SweepArgs {
  const kg_xxz* h;
  const double* u_dev;
  int N;
  double dt;
  const kg_krylov* k;
  int prec;
  const void* psi0;
  const void* target;
  Geo geo;
  Workspace ws;    // slot 0: single calls and the backward sweep
  Workspace ws1;   // slot 1: recomputation beside the backward sweep
  hipStream_t stream;
  const PeArgs* pe = nullptr;   // reduced basis (nullptr: full space)
  size_t vb = 0;                // bytes of one vector
};

KrylovCall krylov_call(const SweepArgs& a, int j, double t, const void* in, void* out) {
  KrylovCall c;
  c.hv = make_hv(a.h, a.u_dev + (j - 1), 0.0);
  c.geo = a.geo;
  c.prec = a.prec;
  c.m = a.k->m;
  c.reorth = a.k->reorth;
  c.t = t;
  c.tol = a.k->breakdown_tol > 0.0 ? a.k->breakdown_tol : default_tol(a.prec);
  c.v_in = in;
  c.v_out = out;
  c.m_eff_out = nullptr;
  c.pe = a.pe;
  return c;
}

kg_status forward_sweep(const SweepArgs& a, const States& S, double* F_dev, double* beta_dev) {
  for (int j = 1; j <= a.N; ++j) {
    const KrylovCall c = krylov_call(a, j, a.dt, S.at0(j - 1), S.at(j));
    KG_HIP(launch_krylov(c, a.ws, a.stream), "forward sweep");
  }
  Profiler* prof = profiler_for_launch();
  if (prof) profiler_start(prof, a.stream);
  KG_HIP(launch_overlap(a.prec, a.geo.D, a.target, S.at(a.N), a.ws, F_dev, beta_dev, a.stream),
         "overlap");
  if (prof) profiler_stop(prof, a.stream, kProfOverlap, 2.0 * a.vb);
  return KG_OK;
}

// The backward sweep runs the segment recomputation on a second stream beside
// the costate propagation: the two chains of Krylov calls are independent
// inside a segment, and on separate streams one chain's reduction tails
// overlap the other's passes (paired launches, which put both calls in the
// same kernels, are no faster than two single ones).  Resources are created
// once per host thread and device, at the default priority; events fork the
// side stream off the caller's stream and join it back, so the work is
// ordered for the caller and a stream capture takes in both branches.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// nullptr: use paired launches on the caller's stream instead
const SideStream* side_stream(hipStream_t caller) {
  static thread_local SideStream per_device[64];
  if (getenv("KG_ONE_STREAM")) return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  SideStream& r = per_device[dev];
  if (!r.s) {
    // creating resources while the caller's stream is being captured is not
    // allowed everywhere: fall back to paired launches for that call
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(caller, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ef = nullptr, ej = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&ef, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ej, hipEventDisableTiming) != hipSuccess) {
      if (ef) (void)hipEventDestroy(ef);
      (void)hipStreamDestroy(st);
      return nullptr;
    }
    r.s = st;
    r.fork = ef;
    r.join = ej;
  }
  return &r;
}

// Nodes of the in-slice quadrature: times s_q in (0, dt) and weights w_q.
struct Quadrature {
  int n = 0;
  double s[KG_MAX_NODES];
  double w[KG_MAX_NODES];
};

// Costate sweep and brackets.  With `centred`, the sweep continues to
// lambda_0 = U_1^dagger lambda_1, takes the bracket with psi_0 into KState::g0
// and replaces every g_j by the mean of the brackets at the two ends of slice j.
// With a quadrature (Q.n > 0), slice j's entry is instead
//   sum_q 2 w_q Im(conj(beta) <e^{+iH_j(dt-s_q)} lambda_j| Hc |e^{-iH_j s_q} psi_{j-1}>),
// the node states coming from paired Krylov calls on the two workspace slots.
// With `first_order`, the bracket takes Hc - (i dt/2)[H_j, Hc]: H_j psi_j and
// H_j lambda_j go to the node vectors and two more brackets are added.
//
// Operator control runs one such sweep per column (col = 0..ncols-1): every
// bracket is scaled by 1/ncols, columns after the first add to the gradient,
// and the centred average is taken once, after the last column.
kg_status backward_sweep(const SweepArgs& a, const States& S, const double* beta_dev,
                         double* grad_dev, bool centred = false, const Quadrature* Q = nullptr,
                         bool first_order = false, int col = 0, int ncols = 1) {
  const HvArgs hc = make_hv(a.h, nullptr, 0.0);
  const double dt_b = a.dt / ncols;
  const bool acc = col > 0;
  const uint32_t* pe_reps = a.pe ? a.pe->reps : nullptr;
  const void* lam = a.target;
  // The quadrature's node states use both slots as well: psi to the node on
  // the caller's stream (slot 0, like the costate), lambda to the node on the
  // side stream (slot 1, like the recomputation), or both in paired launches
  // without a side stream.
  const SideStream* side = (S.c > 0 && S.nseg > 2) ? side_stream(a.stream) : nullptr;
  for (int q = S.nseg - 1; q >= 0; --q) {
    if (side) {
      // the recomputation of this segment's loop overwrites the buffer that the
      // previous segment's brackets read: start it after them
      KG_HIP(hipEventRecord(side->fork, a.stream), "backward sweep fork");
      KG_HIP(hipStreamWaitEvent(side->s, side->fork, 0), "backward sweep fork");
    }
    const int cs = (S.c == 0) ? 0 : q * S.c;
    const int len = (S.c == 0) ? a.N : ((a.N - cs < S.c) ? a.N - cs : S.c);
    // segment q-1 is recomputed beside this segment's backward sweep unless the
    // forward sweep left it in its buffer (the two last segments)
    const int rq = q - 1;
    const bool recompute = S.c > 0 && rq >= 0 && rq <= S.nseg - 3;
    const void* re_in = recompute ? (rq == 0 ? a.psi0 : S.ckpt(rq)) : nullptr;
    int re_i = 1;
    for (int j = cs + len; j > cs; --j) {
      if (Q && Q->n > 0) {
        for (int q = 0; q < Q->n; ++q) {
          const KrylovCall ca = krylov_call(a, j, Q->s[q], S.at0(j - 1), a.ws.node_a);
          const KrylovCall cb = krylov_call(a, j, -(a.dt - Q->s[q]), lam, a.ws.node_b);
          if (side) {
            // lambda's node state starts after the costate that made lambda and
            // the bracket that last read node_b; the bracket waits for it
            KG_HIP(hipEventRecord(side->fork, a.stream), "quadrature fork");
            KG_HIP(hipStreamWaitEvent(side->s, side->fork, 0), "quadrature fork");
            KG_HIP(launch_krylov(ca, a.ws, a.stream), "quadrature node state");
            KG_HIP(launch_krylov(cb, a.ws1, side->s), "quadrature node state");
            KG_HIP(hipEventRecord(side->join, side->s), "quadrature join");
            KG_HIP(hipStreamWaitEvent(a.stream, side->join, 0), "quadrature join");
          } else {
            KG_HIP(launch_krylov_pair(ca, a.ws, cb, a.ws1, a.stream), "quadrature node states");
          }
          KG_HIP(launch_bracket(a.prec, hc, a.geo.D, a.ws.node_b, a.ws.node_a, Q->w[q], beta_dev,
                                a.ws, grad_dev + (j - 1), a.stream, q > 0, 0.0, pe_reps),
                 "quadrature bracket");
        }
      } else {
        Profiler* prof = profiler_for_launch();
        if (prof) profiler_start(prof, a.stream);
        KG_HIP(launch_bracket(a.prec, hc, a.geo.D, lam, S.at(j), dt_b, beta_dev, a.ws,
                              grad_dev + (j - 1), a.stream, acc, 0.0, pe_reps),
               "gradient bracket");
        if (prof) profiler_stop(prof, a.stream, kProfBracket, 2.0 * a.vb);
        if (first_order) {
          const HvArgs hj = make_hv(a.h, a.u_dev + (j - 1), 0.0);
          const double c1 = 0.5 * a.dt * a.dt;
          if (a.pe) {
            KG_HIP(launch_hv_pe(a.prec, hj, *a.pe, S.at(j), a.ws.node_a, a.stream), "H psi_j");
            KG_HIP(launch_hv_pe(a.prec, hj, *a.pe, lam, a.ws.node_b, a.stream), "H lambda_j");
          } else {
            KG_HIP(launch_hv(a.prec, hj, a.geo, S.at(j), a.ws.node_a, a.stream), "H psi_j");
            KG_HIP(launch_hv(a.prec, hj, a.geo, lam, a.ws.node_b, a.stream), "H lambda_j");
          }
          // - (i dt^2/2) <H lambda|Hc psi> + (i dt^2/2) <lambda|Hc H psi>
          KG_HIP(launch_bracket(a.prec, hc, a.geo.D, a.ws.node_b, S.at(j), 0.0, beta_dev, a.ws,
                                grad_dev + (j - 1), a.stream, true, -c1, pe_reps),
                 "first-order bracket");
          KG_HIP(launch_bracket(a.prec, hc, a.geo.D, lam, a.ws.node_a, 0.0, beta_dev, a.ws,
                                grad_dev + (j - 1), a.stream, true, c1, pe_reps),
                 "first-order bracket");
        }
      }
      if (j > 1 || centred) {
        const KrylovCall cb = krylov_call(a, j, -a.dt, lam, a.ws.lam);
        if (recompute && re_i <= S.c - 1) {
          const int jr = rq * S.c + re_i;
          const KrylovCall cr = krylov_call(a, jr, a.dt, re_in, S.at(jr));
          if (side) {
            KG_HIP(launch_krylov(cb, a.ws, a.stream), "backward sweep");
            KG_HIP(launch_krylov(cr, a.ws1, side->s), "segment recomputation");
          } else {
            KG_HIP(launch_krylov_pair(cb, a.ws, cr, a.ws1, a.stream), "backward sweep");
          }
          re_in = S.at(jr);
          ++re_i;
        } else {
          KG_HIP(launch_krylov(cb, a.ws, a.stream), "backward sweep");
        }
        lam = a.ws.lam;
      }
    }
    for (; recompute && re_i <= S.c - 1; ++re_i) {
      const int jr = rq * S.c + re_i;
      const KrylovCall cr = krylov_call(a, jr, a.dt, re_in, S.at(jr));
      KG_HIP(launch_krylov(cr, a.ws1, side ? side->s : a.stream), "segment recomputation");
      re_in = S.at(jr);
    }
    if (side) {
      // the next segment's brackets read the states recomputed here
      KG_HIP(hipEventRecord(side->join, side->s), "backward sweep join");
      KG_HIP(hipStreamWaitEvent(a.stream, side->join, 0), "backward sweep join");
    }
  }
  if (centred) {
    KG_HIP(launch_bracket(a.prec, hc, a.geo.D, lam, a.psi0, dt_b, beta_dev, a.ws, &a.ws.st->g0,
                          a.stream, acc, 0.0, pe_reps),
           "gradient bracket at t = 0");
    if (col == ncols - 1)
      KG_HIP(launch_centre(grad_dev, a.N, &a.ws.st->g0, a.stream), "centred gradient");
  }
  return KG_OK;
}

kg_status check_sweep(const kg_xxz* h, const double* u_dev, int32_t N, double dt, const kg_krylov* k,
                      int32_t prec, const void* psi0, const void* target, void* states,
                      int32_t ckpt_every, int max_L = KG_MAX_L) {
  KG_CHECK(check_xxz(h, max_L));
  KG_CHECK(check_krylov(k));
  KG_CHECK(check_prec(prec));
  if (!u_dev) return fail(KG_EINVAL, "u_dev is NULL");
  if ((uintptr_t)u_dev % 8) return fail(KG_EINVAL, "u_dev is not 8-byte aligned");
  if (N < 1) return fail(KG_EINVAL, "N=%d must be >= 1", N);
  if (!isfinite(dt)) return fail(KG_EINVAL, "dt must be finite");
  if (ckpt_every < 0 || ckpt_every > N)
    return fail(KG_EINVAL, "ckpt_every=%d outside [0, N=%d]", ckpt_every, N);
  KG_CHECK(check_vec(psi0, prec, "psi0"));
  KG_CHECK(check_vec(target, prec, "target"));
  KG_CHECK(check_vec(states, prec, "states"));
  return KG_OK;
}

}  // namespace

// ---------------------------------------------------------------------- sampled kernel timing

struct Profiler {
  int sample_every = 1;
  long calls = 0;
  long launches = 0;
  std::vector<hipEvent_t> ev;
  int used = 0;
  int armed = -1;      // first of the armed event pair, or -1
  bool taken = false;  // a launch took the armed pair
  struct Rec {
    int cls;
    double bytes;
    int e0, e1;
  };
  std::vector<Rec> recs;
};

namespace {
Profiler* g_prof = nullptr;
}

Profiler* profiler_for_call() {
  if (!g_prof) return nullptr;
  const bool take = (g_prof->calls++ % g_prof->sample_every) == 0;
  return take ? g_prof : nullptr;
}

Profiler* profiler_for_launch() {
  if (!g_prof) return nullptr;
  const bool take = (g_prof->launches++ % g_prof->sample_every) == 0;
  return take ? g_prof : nullptr;
}

void profiler_start(Profiler* p, hipStream_t s) {
  (void)s;
  p->armed = -1;
  p->taken = false;
  if (p->used + 2 > (int)p->ev.size()) return;
  p->armed = p->used;
}

bool profiler_take(hipEvent_t* e0, hipEvent_t* e1) {
  Profiler* p = g_prof;
  if (!p || p->armed < 0 || p->taken) return false;
  *e0 = p->ev[p->armed];
  *e1 = p->ev[p->armed + 1];
  p->taken = true;
  return true;
}

void profiler_stop(Profiler* p, hipStream_t s, int cls, double bytes) {
  (void)s;
  if (p->armed >= 0 && p->taken) {
    p->recs.push_back(Profiler::Rec{cls, bytes, p->armed, p->armed + 1});
    p->used += 2;
  }
  p->armed = -1;
  p->taken = false;
}

size_t vec_bytes(int L, int prec) { return ((size_t)1 << L) * (prec == KG_C128 ? 16 : 8); }

size_t ws_fixed_bytes() {
  return align_up(sizeof(KState), 256) + align_up(sizeof(cplx_d) * kPartialRows * kMaxScal, 256);
}

// Tile of a standalone H v (xxz_apply), from graph-timed launches at
// L = 12..24 over tiles of 2^8..2^13: small tiles (more blocks per compute
// unit to hide the partner loads) up to L = 18, larger ones as the vector
// outgrows the caches (complex64 in the pair layout from 2^10).  The Krylov
// passes keep make_geo's tiles, which were timed as whole Krylov calls.
int hv_tile_bits(int L, int prec) {
  if (L <= 18) return 8;
  if (prec == KG_C128) return (L <= 20) ? 9 : (L <= 22 ? 11 : 12);
  return (L <= 21) ? 10 : (L == 22 ? 11 : 12);
}

Geo make_geo(int L, int prec, int tile_bits_override, int grid_cap, bool standalone) {
  Geo g;
  memset(&g, 0, sizeof(g));
  g.L = L;
  g.D = 1u << L;
  // complex64 tiles of 2^13 (eight amplitudes per thread, 1024 threads) only
  // for the standalone H v: the Lanczos passes keep at most 2^12
  const int tb_max = (standalone && prec == KG_C64) ? 13 : 12;
  // default tile, from timed gradients (m = 20, checkpointed): complex64
  // 2^9 amplitudes up to L = 17, 2^10 at L = 18 and 2^11 from L = 19 (2^11
  // against 2^12: 9, 2, 7 and 2 % faster at L = 19..22, 3-4.5 % per Krylov
  // call at L = 23, 24); complex128 2^9..2^11 up to L = 19 and 2^12 beyond
  int tb;
  if (prec == KG_C128) {
    tb = (L >= 20) ? 12 : std::min(std::max(L - 8, 9), 12);
  } else {
    tb = (L >= 19) ? 11 : (L == 18 ? 10 : 9);
  }
  if (tile_bits_override >= 6) tb = tile_bits_override;
  if (tb > tb_max) tb = tb_max;
  if (tb > L) tb = L;
  if (tb < 6) tb = 6;
  // amplitudes per thread (2^RB) grow with the tile until register pressure
  // limits them; the rest of the tile is spread over up to 16 wavefronts
  static const int rb_c64[14] = {0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 2, 2, 3};
  static const int rb_c128[14] = {0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 2, 3, 3};
  g.TB = tb;
  g.RB = (prec == KG_C128) ? rb_c128[tb] : rb_c64[tb];
  g.WB = tb - 6 - g.RB;
  g.small = (L < g.TB) ? 1 : 0;
  g.ntiles = g.small ? 1u : (1u << (L - g.TB));
  if (grid_cap == kLzGrid && g.ntiles >= kLzManyTiles) grid_cap = kLzGridLarge;
  g.grid = (int)(g.ntiles < (uint32_t)grid_cap ? g.ntiles : (uint32_t)grid_cap);
  return g;
}

int tile_override_from_env() {
  const char* e = getenv("KG_TILE_BITS");
  return e ? atoi(e) : 0;
}

}  // namespace kg

using namespace kg;

extern "C" {

const char* kg_last_error(void) { return g_last_error.c_str(); }

int32_t kg_version(void) { return 1; }

size_t kg_workspace_bytes(const kg_xxz* h, const kg_krylov* k, int32_t prec) {
  if (check_xxz(h) != KG_OK || check_krylov(k) != KG_OK || check_prec(prec) != KG_OK) return 0;
  return ws_bytes_d((uint64_t)1 << h->L, k, prec, false);
}

size_t kg_states_bytes(const kg_xxz* h, int32_t N, int32_t ckpt_every, int32_t prec) {
  if (check_xxz(h) != KG_OK || check_prec(prec) != KG_OK) return 0;
  if (N < 1 || ckpt_every < 0 || ckpt_every > N) {
    fail(KG_EINVAL, "bad N=%d or ckpt_every=%d", N, ckpt_every);
    return 0;
  }
  return states_bytes_d((uint64_t)1 << h->L, N, ckpt_every, prec);
}

kg_status xxz_apply(const kg_xxz* h, double u, int32_t prec, const void* v, void* w, void* stream) {
  KG_CHECK(check_xxz(h));
  KG_CHECK(check_prec(prec));
  if (!isfinite(u)) return fail(KG_EINVAL, "u must be finite");
  KG_CHECK(check_vec(v, prec, "v"));
  KG_CHECK(check_vec(w, prec, "w"));
  if (overlap(v, w, vec_bytes(h->L, prec))) return fail(KG_EINVAL, "v and w overlap");
  const int tb_env = tile_override_from_env();
  const Geo g = make_geo(h->L, prec, tb_env >= 6 ? tb_env : hv_tile_bits(h->L, prec), kMaxGrid,
                         true);
  const HvArgs a = make_hv(h, nullptr, u);
  Profiler* prof = profiler_for_launch();
  if (prof) profiler_start(prof, (hipStream_t)stream);
  KG_HIP(launch_hv(prec, a, g, v, w, (hipStream_t)stream), "xxz_apply");
  if (prof) profiler_stop(prof, (hipStream_t)stream, kProfHv, 2.0 * vec_bytes(h->L, prec));
  return ok();
}

namespace {

// The vector space of a sweep: the full 2^L space, or the reduced basis.
struct Space {
  Geo geo;
  const PeArgs* pe;   // nullptr: full space
};

kg_status expv_impl(const kg_xxz* h, const Space& sp, double u, double t, const kg_krylov* k,
                    int32_t prec, const void* v_in, void* v_out, void* ws, size_t ws_bytes,
                    int32_t* m_eff_dev, void* stream) {
  KG_CHECK(check_krylov(k));
  KG_CHECK(check_prec(prec));
  if (!isfinite(u) || !isfinite(t)) return fail(KG_EINVAL, "u and t must be finite");
  KG_CHECK(check_vec(v_in, prec, "v_in"));
  KG_CHECK(check_vec(v_out, prec, "v_out"));
  if (v_in != v_out && overlap(v_in, v_out, vbytes(sp.geo.D, prec)))
    return fail(KG_EINVAL, "v_in and v_out overlap without being equal");
  if (m_eff_dev && (uintptr_t)m_eff_dev % 4) return fail(KG_EINVAL, "m_eff_dev misaligned");
  Workspace W;
  KG_CHECK(carve_d(ws, ws_bytes, sp.geo.D, k, prec, &W, nullptr));
  const hipStream_t s = (hipStream_t)stream;
  KrylovCall c;
  c.hv = make_hv(h, nullptr, u);
  c.geo = sp.geo;
  c.pe = sp.pe;
  c.prec = prec;
  c.m = k->m;
  c.reorth = k->reorth;
  c.t = t;
  c.tol = k->breakdown_tol > 0.0 ? k->breakdown_tol : default_tol(prec);
  c.v_in = v_in;
  c.v_out = v_out;
  c.m_eff_out = m_eff_dev;
  KG_HIP(launch_init(W.st, s), "krylov_expv init");
  KG_HIP(launch_krylov(c, W, s), "krylov_expv");
  return ok();
}

kg_status forward_impl(const kg_xxz* h, const Space& sp, const double* u_dev, int32_t N, double dt,
                       const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                       double* F_dev, double* beta_dev, void* states, int32_t ckpt_every, void* ws,
                       size_t ws_bytes, void* stream, const char* name) {
  if (!F_dev || !beta_dev) return fail(KG_EINVAL, "F_dev and beta_dev are required");
  Workspace W, W1;
  KG_CHECK(carve_d(ws, ws_bytes, sp.geo.D, k, prec, &W, &W1));
  SweepArgs a{h, u_dev, N, dt, k, prec, psi0, target, sp.geo, W, W1, (hipStream_t)stream,
              sp.pe, vbytes(sp.geo.D, prec)};
  const States S = make_states(N, ckpt_every, states, a.vb, psi0);
  KG_HIP(launch_init(W.st, a.stream), name);
  KG_HIP(launch_init(W1.st, a.stream), name);
  KG_CHECK(forward_sweep(a, S, F_dev, beta_dev));
  return ok();
}

kg_status gradient_core(const kg_xxz* h, const Space& sp, const double* u_dev, int32_t N,
                        double dt, const kg_krylov* k, int32_t prec, const void* psi0,
                        const void* target, double* F_dev, double* beta_dev, double* grad_dev,
                        void* states, int32_t ckpt_every, int32_t states_valid, void* ws,
                        size_t ws_bytes, void* stream, bool centred, const char* name,
                        const Quadrature* Q, bool first_order) {
  if (!beta_dev || !grad_dev) return fail(KG_EINVAL, "beta_dev and grad_dev are required");
  if (states_valid != 0 && states_valid != 1) return fail(KG_EINVAL, "states_valid must be 0 or 1");
  Workspace W, W1;
  KG_CHECK(carve_d(ws, ws_bytes, sp.geo.D, k, prec, &W, &W1, Q != nullptr || first_order));
  SweepArgs a{h, u_dev, N, dt, k, prec, psi0, target, sp.geo, W, W1, (hipStream_t)stream,
              sp.pe, vbytes(sp.geo.D, prec)};
  const States S = make_states(N, ckpt_every, states, a.vb, psi0);
  KG_HIP(launch_init(W.st, a.stream), name);
  KG_HIP(launch_init(W1.st, a.stream), name);
  if (!states_valid) KG_CHECK(forward_sweep(a, S, F_dev, beta_dev));
  KG_CHECK(backward_sweep(a, S, beta_dev, grad_dev, centred, Q, first_order));
  return ok();
}

kg_status gradient_impl(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                        const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                        double* F_dev, double* beta_dev, double* grad_dev, void* states,
                        int32_t ckpt_every, int32_t states_valid, void* ws, size_t ws_bytes,
                        void* stream, bool centred, const char* name,
                        const Quadrature* Q = nullptr, bool first_order = false) {
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0, target, states, ckpt_every));
  const Space sp{make_geo(h->L, prec, tile_override_from_env()), nullptr};
  return gradient_core(h, sp, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev,
                       states, ckpt_every, states_valid, ws, ws_bytes, stream, centred, name, Q,
                       first_order);
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's iteration on P_n
// (three-term recurrence) from the starting values cos(pi (i + 3/4) / (n + 1/2)),
// weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int kk = 2; kk <= n; ++kk) {
        const double p2 = ((2.0 * kk - 1.0) * z * p1 - (kk - 1.0) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z) (P_0 = 1 when n = 1)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) <= 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Nodes and weights of the n-point rule on [0, dt].
kg_status make_quadrature(int32_t nodes, double dt, Quadrature* Q) {
  if (nodes < 1 || nodes > KG_MAX_NODES)
    return fail(KG_EINVAL, "nodes=%d outside [1, %d]", nodes, KG_MAX_NODES);
  Q->n = nodes;
  double x[KG_MAX_NODES], w[KG_MAX_NODES];
  gauss_legendre(nodes, x, w);
  for (int q = 0; q < nodes; ++q) {
    Q->s[q] = 0.5 * dt * (x[q] + 1.0);
    Q->w[q] = 0.5 * dt * w[q];
  }
  return KG_OK;
}

}  // namespace

kg_status krylov_expv(const kg_xxz* h, double u, double t, const kg_krylov* k, int32_t prec,
                      const void* v_in, void* v_out, void* ws, size_t ws_bytes, int32_t* m_eff_dev,
                      void* stream) {
  KG_CHECK(check_xxz(h));
  const Space sp{make_geo(h->L, prec, tile_override_from_env()), nullptr};
  return expv_impl(h, sp, u, t, k, prec, v_in, v_out, ws, ws_bytes, m_eff_dev, stream);
}

size_t kg_static_scratch_bytes(void) { return kStaticScratchBytes; }

kg_status krylov_expv_static(const kg_xxz* h, double u, double t, const kg_krylov* k, int32_t prec,
                             const void* v_in, void* v_out, int32_t* m_eff_dev, void* stream) {
  KG_CHECK(check_xxz(h));
  KG_CHECK(check_krylov(k));
  KG_CHECK(check_prec(prec));
  if (!isfinite(u) || !isfinite(t)) return fail(KG_EINVAL, "u and t must be finite");
  KG_CHECK(check_vec(v_in, prec, "v_in"));
  KG_CHECK(check_vec(v_out, prec, "v_out"));
  const Geo geo = make_geo(h->L, prec, tile_override_from_env());
  if (v_in != v_out && overlap(v_in, v_out, vbytes(geo.D, prec)))
    return fail(KG_EINVAL, "v_in and v_out overlap without being equal");
  if (m_eff_dev && (uintptr_t)m_eff_dev % 4) return fail(KG_EINVAL, "m_eff_dev misaligned");
  // one Krylov slot (scalars, partials, m-1 basis vectors and H v_k)
  const size_t need = slot_bytes_d(geo.D, k, prec);
  if (need > kStaticScratchBytes)
    return fail(KG_EWORKSPACE,
                "krylov_expv_static: L=%d, m=%d needs %zu bytes of scratch, the static "
                "scratch holds %zu (use krylov_expv with a workspace)",
                h->L, k->m, need, kStaticScratchBytes);
  void* base = nullptr;
  KG_HIP(static_scratch(&base), "krylov_expv_static scratch address");
  char* q = static_cast<char*>(base);
  Workspace W;
  memset(&W, 0, sizeof(W));
  W.st = reinterpret_cast<KState*>(q);
  q += align_up(sizeof(KState), 256);
  W.partials = reinterpret_cast<cplx_d*>(q);
  q += align_up(sizeof(cplx_d) * kPartialRows * kMaxScal, 256);
  W.basis = q;
  q += align_up(vbytes(geo.D, prec) * (size_t)(k->m - 1), 256);
  W.yk = q;
  const hipStream_t s = (hipStream_t)stream;
  KrylovCall c;
  c.hv = make_hv(h, nullptr, u);
  c.geo = geo;
  c.pe = nullptr;
  c.prec = prec;
  c.m = k->m;
  c.reorth = k->reorth;
  c.t = t;
  c.tol = k->breakdown_tol > 0.0 ? k->breakdown_tol : default_tol(prec);
  c.v_in = v_in;
  c.v_out = v_out;
  c.m_eff_out = m_eff_dev;
  KG_HIP(launch_init(W.st, s), "krylov_expv_static init");
  KG_HIP(launch_krylov(c, W, s), "krylov_expv_static");
  return ok();
}

kg_status grape_forward(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                        const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                        double* F_dev, double* beta_dev, void* states, int32_t ckpt_every, void* ws,
                        size_t ws_bytes, void* stream) {
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0, target, states, ckpt_every));
  const Space sp{make_geo(h->L, prec, tile_override_from_env()), nullptr};
  return forward_impl(h, sp, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, states,
                      ckpt_every, ws, ws_bytes, stream, "grape_forward");
}

kg_status grape_gradient(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                         const kg_krylov* k, int32_t prec, const void* psi0, const void* target,
                         double* F_dev, double* beta_dev, double* grad_dev, void* states,
                         int32_t ckpt_every, int32_t states_valid, void* ws, size_t ws_bytes,
                         void* stream) {
  return gradient_impl(h, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev, states,
                       ckpt_every, states_valid, ws, ws_bytes, stream, false, "grape_gradient");
}

size_t kg_extended_workspace_bytes(const kg_xxz* h, const kg_krylov* k, int32_t prec) {
  if (check_xxz(h) != KG_OK || check_krylov(k) != KG_OK || check_prec(prec) != KG_OK) return 0;
  return ws_bytes_d((uint64_t)1 << h->L, k, prec, true);
}

kg_status grape_gradient_quadrature(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                    const kg_krylov* k, int32_t prec, const void* psi0,
                                    const void* target, double* F_dev, double* beta_dev,
                                    double* grad_dev, void* states, int32_t ckpt_every,
                                    int32_t states_valid, int32_t nodes, void* ws,
                                    size_t ws_bytes, void* stream) {
  Quadrature Q;
  KG_CHECK(make_quadrature(nodes, dt, &Q));
  return gradient_impl(h, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev, states,
                       ckpt_every, states_valid, ws, ws_bytes, stream, false,
                       "grape_gradient_quadrature", &Q);
}

kg_status grape_gradient_first_order(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                     const kg_krylov* k, int32_t prec, const void* psi0,
                                     const void* target, double* F_dev, double* beta_dev,
                                     double* grad_dev, void* states, int32_t ckpt_every,
                                     int32_t states_valid, void* ws, size_t ws_bytes,
                                     void* stream) {
  return gradient_impl(h, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev, states,
                       ckpt_every, states_valid, ws, ws_bytes, stream, false,
                       "grape_gradient_first_order", nullptr, true);
}

kg_status grape_gradient_centred(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                 const kg_krylov* k, int32_t prec, const void* psi0,
                                 const void* target, double* F_dev, double* beta_dev,
                                 double* grad_dev, void* states, int32_t ckpt_every,
                                 int32_t states_valid, void* ws, size_t ws_bytes, void* stream) {
  return gradient_impl(h, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev, states,
                       ckpt_every, states_valid, ws, ws_bytes, stream, true,
                       "grape_gradient_centred");
}

kg_status grape_ascent_update(double* u_dev, const double* grad_dev, int32_t N, double eta,
                              void* stream) {
  if (!u_dev || !grad_dev) return fail(KG_EINVAL, "u_dev and grad_dev are required");
  if (N < 1) return fail(KG_EINVAL, "N must be >= 1");
  if (!isfinite(eta)) return fail(KG_EINVAL, "eta must be finite");
  KG_HIP(launch_ascent(u_dev, grad_dev, N, eta, (hipStream_t)stream), "grape_ascent_update");
  return ok();
}

size_t kg_batched_chain_ws_bytes(int32_t L, int32_t m, int32_t team_size) {
  if (L < 10 || L > 20 || m < 1 || m > KG_MAX_M || team_size < 1 || team_size > 64) return 0;
  return batched_chain_ws_bytes(L, m, team_size);
}

kg_status grape_gradient_batched(const kg_chain* chains_host, const kg_chain* chains_dev,
                                 int32_t n_chains, int32_t n_blocks, const double* u_all,
                                 int64_t u_len, const void* psi0_all, const void* target_all,
                                 int64_t vec_len, void* states_all, int64_t states_len,
                                 double* F_all, double* beta_all, double* grad_all, void* ws,
                                 size_t ws_bytes, int32_t* status_dev, void* stream) {
  if (!chains_host || !chains_dev) return fail(KG_EINVAL, "chain descriptors are required");
  if (n_chains < 1 || n_chains > 4096) return fail(KG_EINVAL, "n_chains=%d outside [1, 4096]", n_chains);
  int dev = 0, ncu = 0;
  KG_HIP(hipGetDevice(&dev), "grape_gradient_batched");
  KG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
         "grape_gradient_batched");
  if (n_blocks < 1 || n_blocks > ncu)
    return fail(KG_EINVAL, "n_blocks=%d outside [1, %d compute units]", n_blocks, ncu);
  if (!u_all || !grad_all || !F_all || !beta_all || !status_dev)
    return fail(KG_EINVAL, "u_all, grad_all, F_all, beta_all and status_dev are required");
  KG_CHECK(check_vec(psi0_all, KG_C64, "psi0_all"));
  KG_CHECK(check_vec(target_all, KG_C64, "target_all"));
  KG_CHECK(check_vec(states_all, KG_C64, "states_all"));
  if (!ws || (uintptr_t)ws % 256) return fail(KG_EWORKSPACE, "workspace missing or not 256-byte aligned");
  std::vector<int> owner(n_blocks, -1);
  std::vector<std::pair<int64_t, int64_t>> wsr;
  for (int i = 0; i < n_chains; ++i) {
    const kg_chain& c = chains_host[i];
    KG_CHECK(check_xxz(&c.h));
    if (c.h.L < 10 || c.h.L > 20) return fail(KG_EINVAL, "chain %d: L=%d outside [10, 20]", i, c.h.L);
    if (c.N < 1) return fail(KG_EINVAL, "chain %d: N=%d", i, c.N);
    if (c.m < 1 || c.m > KG_MAX_M) return fail(KG_EINVAL, "chain %d: m=%d", i, c.m);
    if (c.reorth != 0 && c.reorth != 1) return fail(KG_EINVAL, "chain %d: reorth", i);
    if (!isfinite(c.dt) || !(c.breakdown_tol >= 0.0) || !isfinite(c.breakdown_tol))
      return fail(KG_EINVAL, "chain %d: dt or breakdown_tol", i);
    if (c.team_size < 1 || c.team_size > 64 || c.team_first < 0 || c.team_first + c.team_size > n_blocks)
      return fail(KG_EINVAL, "chain %d: team [%d, %d) outside the grid of %d", i, c.team_first,
                  c.team_first + c.team_size, n_blocks);
    for (int b = c.team_first; b < c.team_first + c.team_size; ++b) {
      if (owner[b] >= 0) return fail(KG_EINVAL, "chains %d and %d share workgroup %d", owner[b], i, b);
      owner[b] = i;
    }
    const int64_t D = (int64_t)1 << c.h.L;
    if (c.off_u < 0 || c.off_u + c.N > u_len) return fail(KG_EINVAL, "chain %d: off_u out of range", i);
    if (c.off_vec < 0 || c.off_vec + D > vec_len)
      return fail(KG_EINVAL, "chain %d: off_vec out of range", i);
    if (c.off_states < 0 || c.off_states + (int64_t)c.N * D > states_len)
      return fail(KG_EINVAL, "chain %d: off_states out of range", i);
    const int64_t wb = (int64_t)batched_chain_ws_bytes(c.h.L, c.m, c.team_size);
    if (c.off_ws < 0 || c.off_ws % 256 || (size_t)(c.off_ws + wb) > ws_bytes)
      return fail(KG_EWORKSPACE, "chain %d: workspace range [%lld, %lld) invalid for %zu bytes", i,
                  (long long)c.off_ws, (long long)(c.off_ws + wb), ws_bytes);
    wsr.push_back({c.off_ws, c.off_ws + wb});
  }
  std::sort(wsr.begin(), wsr.end());
  for (size_t i = 1; i < wsr.size(); ++i)
    if (wsr[i].first < wsr[i - 1].second) return fail(KG_EWORKSPACE, "chain workspaces overlap");
  KG_HIP(launch_batched(chains_dev, n_chains, n_blocks, u_all, psi0_all, target_all, states_all,
                        F_all, beta_all, grad_all, ws, status_dev, (hipStream_t)stream),
         "grape_gradient_batched");
  return ok();
}

// ---------------------------------------------------------------------- batch planning

namespace {

constexpr int kBatchTile = 1024;   // amplitudes of a tile of the persistent kernel

// Upper bound on the spectral radius of H0 + u Hc for |u| <= umax (Gershgorin on
// the matrix elements of the open chain with S = sigma/2): each of the L-1 bonds
// adds at most |J|/2 off the diagonal and |J Delta|/4 on it; S^x on one site adds
// 1/2 off the diagonal, a sum of S^z over n sites at most n/2 on it.
double gershgorin_norm(const kg_xxz& h, double umax) {
  return (h.L - 1) * fabs(h.J) * (0.5 + fabs(h.Delta) / 4.0) +
         fabs(umax) * 0.5 * (double)__builtin_popcountll(h.hc_sites);
}

// Hochbruck & Lubich (SIAM J. Numer. Anal. 34, 1997), Theorem 2: the error of the
// m-dimensional Lanczos approximation of exp(A) v, A skew-Hermitian with its
// spectrum on an imaginary segment of length 4 rho, is at most
// 12 exp(-rho^2/m) (e rho/m)^m for m >= 2 rho.
double hochbruck_lubich(double rho, int m) {
  if (m < 2.0 * rho) return INFINITY;
  return 12.0 * exp(-rho * rho / m) * pow(M_E * rho / m, (double)m);
}

// The smallest m in [m_min, m_max] whose bound for A = -i dt H meets tol / N.
int krylov_dimension(const kg_xxz& h, double umax, double dt, int N, double tol, int m_min,
                     int m_max) {
  const double rho = 0.5 * fabs(dt) * gershgorin_norm(h, umax);
  for (int m = m_min; m <= m_max; ++m)
    if (hochbruck_lubich(rho, m) <= tol / N) return m;
  return m_max;
}

// Vector traffic of one chain's gradient in amplitude passes: 2N Krylov calls of
// about m^2 + 3m passes over 2^L amplitudes.
// Modelled time (us) of a chain on a team of T workgroups.  Each of its about
// 2 N m Lanczos steps costs a fixed part (the team barrier and the scalar
// update) and, for the busiest member, a part per tile it holds that grows
// with the window (about (m + 6) / 2 vectors on average).  The part per tile
// fits the heaviest chain of the 64-chain workload alone (L=16, m=11: 359,
// 180, 92, 49, 28, 17.7 and 13.6 us per step on 1, 2, 4, ..., 64
// workgroups).  The fixed part is the one that gave the fastest planned
// launches of that workload: 4-6 us all gave 127 ms; 0-3 us 132-140 ms,
// 7-8 us 130-131 ms, 12 us 138 ms and 16 us 152 ms (teams by doubling: 150 ms).
constexpr double kStepFixedUs = 5.0;
constexpr double kStepTileUs = 0.65;   // per tile and window vector

int64_t chain_tiles(const kg_chain& c) {
  return std::max<int64_t>(1, ((int64_t)1 << c.h.L) / kBatchTile);
}

double chain_time(const kg_chain& c, int team) {
  const int64_t per = (chain_tiles(c) + team - 1) / team;
  return 2.0 * c.N * c.m * (kStepFixedUs + kStepTileUs * 0.5 * (c.m + 6) * (double)per);
}

}  // namespace

kg_status kg_batched_plan(kg_chain* chains, int32_t n_chains, const double* umax, int32_t n_blocks,
                          int32_t max_team, int32_t keep_teams, double tol, int32_t m_min,
                          int32_t m_max, kg_batch_plan* plan) {
  if (!chains || !plan) return fail(KG_EINVAL, "chains and plan are required");
  if (n_chains < 1 || n_chains > 4096) return fail(KG_EINVAL, "n_chains=%d outside [1, 4096]", n_chains);
  if (n_blocks < n_chains)
    return fail(KG_EINVAL, "%d chains need at least %d workgroups, the grid has %d", n_chains,
                n_chains, n_blocks);
  if (max_team < 1 || max_team > 64) return fail(KG_EINVAL, "max_team=%d outside [1, 64]", max_team);
  if (keep_teams != 0 && keep_teams != 1) return fail(KG_EINVAL, "keep_teams must be 0 or 1");
  if (!(tol > 0.0) || !isfinite(tol)) return fail(KG_EINVAL, "tol must be finite and > 0");
  if (m_min < 1 || m_max > KG_MAX_M || m_min > m_max)
    return fail(KG_EINVAL, "Krylov range [%d, %d] outside [1, %d]", m_min, m_max, KG_MAX_M);
  for (int i = 0; i < n_chains; ++i) {
    kg_chain& c = chains[i];
    KG_CHECK(check_xxz(&c.h));
    if (c.h.L < 10 || c.h.L > 20) return fail(KG_EINVAL, "chain %d: L=%d outside [10, 20]", i, c.h.L);
    if (c.N < 1) return fail(KG_EINVAL, "chain %d: N=%d", i, c.N);
    if (!isfinite(c.dt)) return fail(KG_EINVAL, "chain %d: dt must be finite", i);
    if (c.m == 0) {
      if (!umax || !isfinite(umax[i]))
        return fail(KG_EINVAL, "chain %d: m = 0 needs a finite umax", i);
      c.m = krylov_dimension(c.h, umax[i], c.dt, c.N, tol, m_min, m_max);
    } else if (c.m < 1 || c.m > KG_MAX_M) {
      return fail(KG_EINVAL, "chain %d: m=%d", i, c.m);
    }
    if (keep_teams && (c.team_size < 1 || c.team_size > 64))
      return fail(KG_EINVAL, "chain %d: team_size=%d outside [1, 64]", i, c.team_size);
  }
  if (!keep_teams) {
    // greedy makespan balancing: one workgroup per chain, then give the chain
    // with the largest modelled time (the lowest index on ties) the smallest
    // team that holds fewer tiles per member, while its cap and the grid allow
    // it.  The slowest chain bounds the launch, so the loop ends when it cannot
    // be sped up.
    std::vector<int> cap(n_chains);
    int used = n_chains;
    for (int i = 0; i < n_chains; ++i) {
      chains[i].team_size = 1;
      cap[i] = (int)std::min<int64_t>(max_team, chain_tiles(chains[i]));
    }
    for (;;) {
      int best = 0;
      for (int i = 1; i < n_chains; ++i)
        if (chain_time(chains[i], chains[i].team_size) >
            chain_time(chains[best], chains[best].team_size))
          best = i;
      kg_chain& c = chains[best];
      const int64_t tiles = chain_tiles(c);
      const int64_t per = (tiles + c.team_size - 1) / c.team_size;
      if (per <= 1) break;
      const int next = (int)((tiles + per - 2) / (per - 1));   // ceil(tiles / (per - 1))
      if (next > cap[best] || used + (next - c.team_size) > n_blocks) break;
      used += next - c.team_size;
      c.team_size = next;
    }
  }
  int64_t off_u = 0, off_vec = 0, off_states = 0, off_ws = 0;
  int first = 0;
  for (int i = 0; i < n_chains; ++i) {
    kg_chain& c = chains[i];
    const int64_t D = (int64_t)1 << c.h.L;
    c.team_first = first;
    c.off_u = off_u;
    c.off_vec = off_vec;
    c.off_states = off_states;
    c.off_ws = off_ws;
    first += c.team_size;
    off_u += c.N;
    off_vec += D;
    off_states += (int64_t)c.N * D;
    off_ws += (int64_t)align_up(batched_chain_ws_bytes(c.h.L, c.m, c.team_size), 256);
  }
  if (first > n_blocks)
    return fail(KG_EINVAL, "the teams need %d workgroups, the grid has %d", first, n_blocks);
  plan->u_len = off_u;
  plan->vec_len = off_vec;
  plan->states_len = off_states;
  plan->ws_bytes = (uint64_t)off_ws;
  plan->blocks_used = first;
  plan->pad_ = 0;
  return ok();
}

kg_status kg_batched_autotune(kg_chain* chains_host, kg_chain* chains_dev, int32_t n_chains,
                              int32_t n_blocks, const int32_t* caps, int32_t n_caps, int32_t reps,
                              const double* u_all, int64_t u_len, const void* psi0_all,
                              const void* target_all, int64_t vec_len, void* states_all,
                              int64_t states_len, double* F_all, double* beta_all,
                              double* grad_all, void* ws, size_t ws_bytes, int32_t* status_dev,
                              float* ms_out, int32_t* best_cap, void* stream) {
  if (!chains_host || !chains_dev || !caps || !best_cap)
    return fail(KG_EINVAL, "chains, caps and best_cap are required");
  if (n_chains < 1 || n_chains > 4096) return fail(KG_EINVAL, "n_chains=%d outside [1, 4096]", n_chains);
  if (n_caps < 1 || n_caps > 16) return fail(KG_EINVAL, "n_caps=%d outside [1, 16]", n_caps);
  if (reps < 1 || reps > 100) return fail(KG_EINVAL, "reps=%d outside [1, 100]", reps);
  const hipStream_t s = (hipStream_t)stream;
  std::vector<kg_chain> trial(chains_host, chains_host + n_chains);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KG_HIP(hipEventCreate(&e0), "kg_batched_autotune");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(KG_EDEVICE, "kg_batched_autotune: event creation failed");
  }
  kg_status st = KG_OK;
  float best_ms = INFINITY;
  int best = -1;
  const size_t desc_bytes = sizeof(kg_chain) * (size_t)n_chains;
  for (int q = 0; q < n_caps && st == KG_OK; ++q) {
    kg_batch_plan plan;
    st = kg_batched_plan(trial.data(), n_chains, nullptr, n_blocks, caps[q], 0, 1.0, 1, KG_MAX_M,
                         &plan);
    if (st != KG_OK) break;
    if (plan.ws_bytes > ws_bytes) {
      st = fail(KG_EWORKSPACE, "cap %d needs %llu workspace bytes, %zu given", caps[q],
                (unsigned long long)plan.ws_bytes, ws_bytes);
      break;
    }
    hipError_t e = hipMemcpyAsync(chains_dev, trial.data(), desc_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      st = hip_fail(e, "kg_batched_autotune");
      break;
    }
    // one launch to warm up, then `reps` timed
    for (int r = 0; r <= reps && st == KG_OK; ++r) {
      if (r == 1 && (e = hipEventRecord(e0, s)) != hipSuccess) st = hip_fail(e, "kg_batched_autotune");
      if (st == KG_OK)
        st = grape_gradient_batched(trial.data(), chains_dev, n_chains, n_blocks, u_all, u_len,
                                    psi0_all, target_all, vec_len, states_all, states_len, F_all,
                                    beta_all, grad_all, ws, ws_bytes, status_dev, stream);
    }
    if (st != KG_OK) break;
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
      st = hip_fail(e, "kg_batched_autotune");
      break;
    }
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
      st = hip_fail(e, "kg_batched_autotune");
      break;
    }
    ms /= (float)reps;
    if (ms_out) ms_out[q] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = q;
    }
  }
  if (st == KG_OK) {
    kg_batch_plan plan;
    st = kg_batched_plan(chains_host, n_chains, nullptr, n_blocks, caps[best], 0, 1.0, 1, KG_MAX_M,
                         &plan);
    if (st == KG_OK) {
      hipError_t e = hipMemcpyAsync(chains_dev, chains_host, desc_bytes, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = hip_fail(e, "kg_batched_autotune");
    }
    if (st == KG_OK) *best_cap = caps[best];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st == KG_OK ? ok() : st;
}

kg_status kg_profile_begin(int32_t sample_every, int32_t max_launches) {
  if (g_prof) return fail(KG_EINVAL, "profiling is already active");
  if (sample_every < 1 || max_launches < 1 || max_launches > (1 << 22))
    return fail(KG_EINVAL, "sample_every >= 1 and 1 <= max_launches <= 2^22 required");
  Profiler* p = new Profiler();
  p->sample_every = sample_every;
  p->ev.resize(2 * (size_t)max_launches);
  for (auto& e : p->ev) {
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      for (auto& f : p->ev)
        if (f) hipEventDestroy(f);
      delete p;
      return hip_fail(r, "kg_profile_begin");
    }
  }
  g_prof = p;
  return ok();
}

kg_status kg_profile_end(int64_t* launches, double* ms, double* bytes) {
  if (!g_prof) return fail(KG_EINVAL, "profiling is not active");
  Profiler* p = g_prof;
  g_prof = nullptr;
  kg_status st = KG_OK;
  for (int c = 0; c < kProfN; ++c) {
    if (launches) launches[c] = 0;
    if (ms) ms[c] = 0.0;
    if (bytes) bytes[c] = 0.0;
  }
  if (!p->recs.empty()) {
    hipError_t r = hipEventSynchronize(p->ev[p->recs.back().e1]);
    if (r != hipSuccess) st = hip_fail(r, "kg_profile_end");
    for (const auto& rec : p->recs) {
      float t = 0.0f;
      if (st == KG_OK) {
        r = hipEventElapsedTime(&t, p->ev[rec.e0], p->ev[rec.e1]);
        if (r != hipSuccess) st = hip_fail(r, "kg_profile_end");
      }
      if (launches) launches[rec.cls] += 1;
      if (ms) ms[rec.cls] += t;
      if (bytes) bytes[rec.cls] += rec.bytes;
    }
  }
  for (auto& e : p->ev) hipEventDestroy(e);
  delete p;
  return st == KG_OK ? ok() : st;
}

// ---------------------------------------------------------------------- operator control

namespace {

// Forward sweeps of all columns (two per launch), the mean overlap, then one
// costate sweep per column adding its brackets.
kg_status columns_core(const kg_xxz* h, const Space& sp, const double* u_dev, int32_t N, double dt,
                       const kg_krylov* k, int32_t prec, int32_t n_cols, const void* psi0s,
                       const void* targets, double* F_dev, double* beta_dev, double* beta_cols_dev,
                       double* grad_dev, void* states, int32_t ckpt_every, int32_t centred,
                       void* ws, size_t ws_bytes, void* stream) {
  if (n_cols < 1) return fail(KG_EINVAL, "n_cols=%d must be >= 1", n_cols);
  if (!beta_dev || !beta_cols_dev || !grad_dev)
    return fail(KG_EINVAL, "beta_dev, beta_cols_dev and grad_dev are required");
  if ((uintptr_t)beta_cols_dev % 8) return fail(KG_EINVAL, "beta_cols_dev is not 8-byte aligned");
  if (centred != 0 && centred != 1) return fail(KG_EINVAL, "centred must be 0 or 1");
  Workspace W, W1;
  KG_CHECK(carve_d(ws, ws_bytes, sp.geo.D, k, prec, &W, &W1));
  const size_t vb = vbytes(sp.geo.D, prec);
  const size_t sb = states_bytes_d(sp.geo.D, N, ckpt_every, prec);
  const hipStream_t s = (hipStream_t)stream;
  auto col_args = [&](int c, const Workspace& w0, const Workspace& w1) {
    return SweepArgs{h, u_dev, N, dt, k, prec,
                     static_cast<const char*>(psi0s) + (size_t)c * vb,
                     static_cast<const char*>(targets) + (size_t)c * vb, sp.geo, w0, w1, s,
                     sp.pe, vb};
  };
  auto col_states = [&](int c) {
    return make_states(N, ckpt_every, static_cast<char*>(states) + (size_t)c * sb, vb,
                       static_cast<const char*>(psi0s) + (size_t)c * vb);
  };
  KG_HIP(launch_init(W.st, s), "grape_gradient_columns");
  KG_HIP(launch_init(W1.st, s), "grape_gradient_columns");
  for (int c = 0; c < n_cols; c += 2) {
    const SweepArgs a0 = col_args(c, W, W1);
    const States S0 = col_states(c);
    if (c + 1 < n_cols) {
      const SweepArgs a1 = col_args(c + 1, W1, W);
      const States S1 = col_states(c + 1);
      for (int j = 1; j <= N; ++j) {
        const KrylovCall k0 = krylov_call(a0, j, dt, S0.at0(j - 1), S0.at(j));
        const KrylovCall k1 = krylov_call(a1, j, dt, S1.at0(j - 1), S1.at(j));
        KG_HIP(launch_krylov_pair(k0, W, k1, W1, s), "column forward sweeps");
      }
      KG_HIP(launch_overlap(prec, sp.geo.D, a1.target, S1.at(N), W1, nullptr,
                            beta_cols_dev + 2 * (c + 1), s),
             "column overlap");
    } else {
      for (int j = 1; j <= N; ++j) {
        const KrylovCall k0 = krylov_call(a0, j, dt, S0.at0(j - 1), S0.at(j));
        KG_HIP(launch_krylov(k0, W, s), "column forward sweep");
      }
    }
    KG_HIP(launch_overlap(prec, sp.geo.D, a0.target, S0.at(N), W, nullptr, beta_cols_dev + 2 * c,
                          s),
           "column overlap");
  }
  KG_HIP(launch_mean_overlap(beta_cols_dev, n_cols, beta_dev, F_dev, s), "mean overlap");
  for (int c = 0; c < n_cols; ++c)
    KG_CHECK(backward_sweep(col_args(c, W, W1), col_states(c), beta_dev, grad_dev, centred != 0,
                            nullptr, false, c, n_cols));
  return ok();
}

}  // namespace

size_t kg_columns_states_bytes(const kg_xxz* h, int32_t n_cols, int32_t N, int32_t ckpt_every,
                               int32_t prec) {
  if (n_cols < 1) return 0;
  const size_t one = kg_states_bytes(h, N, ckpt_every, prec);
  return one * (size_t)n_cols;
}

kg_status grape_gradient_columns(const kg_xxz* h, const double* u_dev, int32_t N, double dt,
                                 const kg_krylov* k, int32_t prec, int32_t n_cols,
                                 const void* psi0s, const void* targets, double* F_dev,
                                 double* beta_dev, double* beta_cols_dev, double* grad_dev,
                                 void* states, int32_t ckpt_every, int32_t centred, void* ws,
                                 size_t ws_bytes, void* stream) {
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0s, targets, states, ckpt_every));
  const Space sp{make_geo(h->L, prec, tile_override_from_env()), nullptr};
  return columns_core(h, sp, u_dev, N, dt, k, prec, n_cols, psi0s, targets, F_dev, beta_dev,
                      beta_cols_dev, grad_dev, states, ckpt_every, centred, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------- reduced basis

namespace {

// Pascal's triangle up to n = 32 (exact in 64 bits).
struct Pascal {
  uint64_t c[kPeBinom][kPeBinom];
  Pascal() {
    memset(c, 0, sizeof(c));
    for (int n = 0; n < kPeBinom; ++n) {
      c[n][0] = 1;
      for (int k = 1; k <= n; ++k) c[n][k] = c[n - 1][k - 1] + (k < n ? c[n - 1][k] : 0);
    }
  }
};

const Pascal& pascal() {
  static const Pascal p;
  return p;
}

uint32_t reverse_bits(uint32_t s, int L) {
  uint32_t r = 0;
  for (int b = 0; b < L; ++b) r |= ((s >> b) & 1u) << (L - 1 - b);
  return r;
}

// Number of orbits {s, Pi s} among the L-bit patterns with K zero bits: the
// sector size plus its palindromes, halved.  A palindrome is fixed by its first
// floor(L/2) bits and (L odd) its middle bit, so it has an even number of zero
// bits outside the middle.
int64_t pe_dim(int L, int K) {
  const Pascal& P = pascal();
  const uint64_t sector = P.c[L][K];
  uint64_t pal = 0;
  if (L % 2 == 1 || K % 2 == 0) pal = P.c[L / 2][K / 2];
  return (int64_t)((sector + pal) / 2);
}

// Table layout in the caller's buffer: binomials (uint32, kPeBinom^2), orbit
// representatives (uint32, dim), their ranks (uint32, dim), index by
// combinatorial rank (int32, C(L,K)), each at a 256-byte boundary; then, for
// bases of at most kPeNbrMaxEntries neighbour slots, the slot count of each
// slice of 64 rows (uint32) and the neighbour slots (uint32, L - 1 per row).
struct PeLayout {
  size_t off_reps, off_ranks, off_index, off_scnt, off_nbr, total;
  uint64_t nslices;
  int nbr_slots;           // 0: no neighbour table
};

PeLayout pe_layout(int L, int K) {
  PeLayout o;
  const uint64_t dim = (uint64_t)pe_dim(L, K);
  o.off_reps = align_up(sizeof(uint32_t) * kPeBinom * kPeBinom, 256);
  o.off_ranks = o.off_reps + align_up(sizeof(uint32_t) * (size_t)dim, 256);
  o.off_index = o.off_ranks + align_up(sizeof(uint32_t) * (size_t)dim, 256);
  o.off_scnt = o.off_index + align_up(sizeof(int32_t) * (size_t)pascal().c[L][K], 256);
  o.nslices = (dim + 63) / 64;
  o.nbr_slots = (L >= 2 && o.nslices * 64 * (uint64_t)(L - 1) <= kPeNbrMaxEntries) ? L - 1 : 0;
  if (o.nbr_slots == 0) {
    o.off_nbr = o.total = o.off_scnt;
    return o;
  }
  o.off_nbr = o.off_scnt + align_up(sizeof(uint32_t) * (size_t)o.nslices, 256);
  o.total = o.off_nbr + sizeof(uint32_t) * (size_t)(o.nslices * 64 * (uint64_t)o.nbr_slots);
  return o;
}

// The bits of s (L of them) in reverse order: swaps of ever larger halves.
uint32_t reverse_bits_fast(uint32_t s, int L) {
  s = ((s >> 1) & 0x55555555u) | ((s & 0x55555555u) << 1);
  s = ((s >> 2) & 0x33333333u) | ((s & 0x33333333u) << 2);
  s = ((s >> 4) & 0x0F0F0F0Fu) | ((s & 0x0F0F0F0Fu) << 4);
  s = ((s >> 8) & 0x00FF00FFu) | ((s & 0x00FF00FFu) << 8);
  s = (s >> 16) | (s << 16);
  return s >> (32 - L);
}

kg_status check_pe_shape(int32_t L, int32_t K) {
  if (L < KG_MIN_L || L > KG_PE_MAX_L)
    return fail(KG_EINVAL, "L=%d outside [%d, %d]", L, KG_MIN_L, KG_PE_MAX_L);
  if (K < 0 || K > L) return fail(KG_EINVAL, "K=%d outside [0, L=%d]", K, L);
  return KG_OK;
}

kg_status check_pe(const kg_pe* pe) {
  if (!pe) return fail(KG_EINVAL, "pe is NULL");
  KG_CHECK(check_pe_shape(pe->L, pe->K));
  if (pe->dim != pe_dim(pe->L, pe->K))
    return fail(KG_EINVAL, "pe->dim=%lld is not the dimension %lld of L=%d, K=%d",
                (long long)pe->dim, (long long)pe_dim(pe->L, pe->K), pe->L, pe->K);
  if (!pe->tables || (uintptr_t)pe->tables % 256)
    return fail(KG_EINVAL, "pe->tables missing or not 256-byte aligned");
  return KG_OK;
}

// The chain must conserve the excitation number and the mirror parity: an
// S^z control on a mirror-symmetric set of sites.
kg_status check_pe_chain(const kg_xxz* h, const kg_pe* pe) {
  KG_CHECK(check_xxz(h, KG_PE_MAX_L));
  KG_CHECK(check_pe(pe));
  if (h->L != pe->L) return fail(KG_EINVAL, "h->L=%d differs from pe->L=%d", h->L, pe->L);
  if (h->hc_kind != KG_HC_SZ)
    return fail(KG_EINVAL, "the reduced basis needs an S^z control (KG_HC_SZ)");
  for (int i = 1; i <= h->L; ++i)
    if (((h->hc_sites >> (i - 1)) & 1ull) != ((h->hc_sites >> (h->L - i)) & 1ull))
      return fail(KG_EINVAL, "hc_sites is not mirror-symmetric (site %d vs %d)", i, h->L + 1 - i);
  return KG_OK;
}

PeArgs pe_args(const kg_pe* pe) {
  const PeLayout o = pe_layout(pe->L, pe->K);
  const char* t = static_cast<const char*>(pe->tables);
  PeArgs a;
  memset(&a, 0, sizeof(a));
  a.binom = reinterpret_cast<const uint32_t*>(t);
  a.reps = reinterpret_cast<const uint32_t*>(t + o.off_reps);
  a.ranks = reinterpret_cast<const uint32_t*>(t + o.off_ranks);
  a.index = reinterpret_cast<const int32_t*>(t + o.off_index);
  // KG_PE_NO_NEIGHBORS=1 keeps the rank-forming H v (the tests run both forms)
  const char* nn = getenv("KG_PE_NO_NEIGHBORS");
  if (o.nbr_slots > 0 && !(nn && nn[0] == '1')) {
    a.scnt = reinterpret_cast<const uint32_t*>(t + o.off_scnt);
    a.nbr = reinterpret_cast<const uint32_t*>(t + o.off_nbr);
    a.nbr_slots = o.nbr_slots;
  }
  a.L = pe->L;
  a.K = pe->K;
  a.dim = (uint32_t)pe->dim;
  a.nsec = (uint32_t)pascal().c[pe->L][pe->K];
  return a;
}

// Lanczos tiles of the reduced basis: four amplitudes per thread, tiles of
// 2^TB (TB = 8..12) amplitudes, the smallest TB that keeps the tile count at
// or below kLzGrid.  Beyond that, each block takes `it` tiles and the grid is
// the smallest multiple of 8 with grid * it >= the tile count; the count is
// padded to grid * it (the padded tail is masked like the ragged last tile).
Geo make_geo_pe(int L, uint64_t dim) {
  Geo g;
  memset(&g, 0, sizeof(g));
  g.L = L;
  g.D = (uint32_t)dim;
  int tb = 8;
  while (tb < 12 && ((dim + ((uint64_t)1 << tb) - 1) >> tb) > (uint64_t)kLzGrid) ++tb;
  uint64_t nt = (dim + ((uint64_t)1 << tb) - 1) >> tb;
  if (nt < 1) nt = 1;
  uint64_t grid = nt;
  if (nt > (uint64_t)kLzGrid) {
    const uint64_t it = (nt + kLzGrid - 1) / kLzGrid;
    grid = ((nt + it - 1) / it + 7) / 8 * 8;
    nt = grid * it;
  }
  g.TB = tb;
  g.RB = 2;
  g.WB = tb - 8;
  g.small = 1;
  g.ntiles = (uint32_t)nt;
  g.grid = (int)grid;
  return g;
}

}  // namespace

int64_t kg_pe_dim(int32_t L, int32_t K) {
  if (check_pe_shape(L, K) != KG_OK) return 0;
  return pe_dim(L, K);
}

size_t kg_pe_tables_bytes(int32_t L, int32_t K) {
  if (check_pe_shape(L, K) != KG_OK) return 0;
  return pe_layout(L, K).total;
}

kg_status kg_pe_tables_host(int32_t L, int32_t K, void* tables_host, size_t tables_bytes) {
  KG_CHECK(check_pe_shape(L, K));
  const PeLayout o = pe_layout(L, K);
  if (!tables_host) return fail(KG_EINVAL, "tables_host is NULL");
  if (tables_bytes < o.total)
    return fail(KG_EWORKSPACE, "tables have %zu bytes, need %zu", tables_bytes, o.total);
  const Pascal& P = pascal();
  const uint64_t sector = P.c[L][K];
  const int64_t dim = pe_dim(L, K);
  char* host = static_cast<char*>(tables_host);
  memset(host, 0, o.total);
  uint32_t* binom = reinterpret_cast<uint32_t*>(host);
  for (int n = 0; n < kPeBinom; ++n)
    for (int k = 0; k < kPeBinom; ++k) binom[n * kPeBinom + k] = (uint32_t)P.c[n][k];
  uint32_t* reps = reinterpret_cast<uint32_t*>(host + o.off_reps);
  uint32_t* ranks = reinterpret_cast<uint32_t*>(host + o.off_ranks);
  int32_t* index = reinterpret_cast<int32_t*>(host + o.off_index);
  const uint64_t full = (L == 32) ? 0xFFFFFFFFull : ((1ull << L) - 1ull);
  auto rank = [&](uint32_t s) {
    uint64_t z = ~(uint64_t)s & full, r = 0;
    for (int i = 1; z; ++i, z &= z - 1) r += P.c[__builtin_ctzll(z)][i];
    return r;
  };
  // the sector's patterns (L-K one bits) in ascending order; an orbit's
  // smaller member comes first and takes the next index
  const int ones = L - K;
  uint64_t v = ones ? ((1ull << ones) - 1ull) : 0ull;
  int64_t next = 0;
  uint64_t seen = 0;
  while (true) {
    const uint32_t s = (uint32_t)v;
    const uint32_t rs = reverse_bits(s, L);
    const uint64_t rk = rank(s);
    if (s <= rs) {
      reps[next] = s;
      ranks[next] = (uint32_t)rk;
      index[rk] = (int32_t)next;
      ++next;
    } else {
      index[rk] = index[rank(rs)];
    }
    ++seen;
    if (ones == 0) break;
    // next pattern with the same number of one bits (Gosper)
    const uint64_t c = v & (~v + 1ull);
    const uint64_t r = v + c;
    v = (((r ^ v) >> 2) / c) | r;
    if (v > full) break;
  }
  if (seen != sector || next != dim)
    return fail(KG_EINVAL, "internal: enumerated %llu states and %lld orbits, expected %llu, %lld",
                (unsigned long long)seen, (long long)next, (unsigned long long)sector,
                (long long)dim);
  if (o.nbr_slots > 0) {
    // neighbour table: the j-th antiparallel bond q (ascending) of label r
    // exchanges bits q, q+1; the rank moves by C(q, zeros below q), up when
    // the zero moves from q to q+1
    const int S = o.nbr_slots;
    uint32_t* scnt = reinterpret_cast<uint32_t*>(host + o.off_scnt);
    uint32_t* nbr = reinterpret_cast<uint32_t*>(host + o.off_nbr);
    const uint32_t bondmask = (L == 32) ? 0x7FFFFFFFu : ((1u << (L - 1)) - 1u);
    for (int64_t b = 0; b < dim; ++b) {
      const uint32_t r = reps[b];
      const uint64_t rk = ranks[b];
      const uint32_t zeros = ~r & (uint32_t)full;
      const bool nb2 = reverse_bits_fast(r, L) != r;
      uint32_t* row = nbr + (size_t)(b >> 6) * S * 64 + (b & 63);
      int j = 0;
      for (uint32_t act = (r ^ (r >> 1)) & bondmask; act; act &= act - 1u, ++j) {
        const int q = __builtin_ctz(act);
        const uint64_t dl = P.c[q][__builtin_popcount(zeros & ((1u << q) - 1u))];
        const uint64_t rk2 = ((r >> q) & 1u) ? rk - dl : rk + dl;
        const uint32_t s2 = r ^ (3u << q);
        const bool na2 = reverse_bits_fast(s2, L) != s2;
        const uint32_t code = (nb2 == na2) ? 1u : (nb2 ? 2u : 3u);
        if (rk2 >= sector || index[rk2] < 0 || index[rk2] >= dim)
          return fail(KG_EINVAL, "internal: neighbour of orbit %lld out of range", (long long)b);
        row[(size_t)j * 64] = (uint32_t)index[rk2] | (code << 30);
      }
      for (int i = j; i < S; ++i) row[(size_t)i * 64] = (uint32_t)b;
      uint32_t& c = scnt[b >> 6];
      if ((uint32_t)j > c) c = (uint32_t)j;
    }
  }
  return ok();
}

kg_status kg_pe_build(int32_t L, int32_t K, void* tables_dev, size_t tables_bytes, kg_pe* pe) {
  KG_CHECK(check_pe_shape(L, K));
  if (!pe) return fail(KG_EINVAL, "pe is NULL");
  if (!tables_dev || (uintptr_t)tables_dev % 256)
    return fail(KG_EINVAL, "tables_dev missing or not 256-byte aligned");
  const PeLayout o = pe_layout(L, K);
  if (tables_bytes < o.total)
    return fail(KG_EWORKSPACE, "tables have %zu bytes, need %zu", tables_bytes, o.total);
  std::vector<char> host(o.total);
  KG_CHECK(kg_pe_tables_host(L, K, host.data(), host.size()));
  KG_HIP(hipMemcpy(tables_dev, host.data(), o.total, hipMemcpyHostToDevice), "kg_pe_build");
  const int64_t dim = pe_dim(L, K);
  pe->L = L;
  pe->K = K;
  pe->dim = dim;
  pe->tables = tables_dev;
  return ok();
}

size_t kg_pe_workspace_bytes(const kg_pe* pe, const kg_krylov* k, int32_t prec, int32_t extended) {
  if (check_pe(pe) != KG_OK || check_krylov(k) != KG_OK || check_prec(prec) != KG_OK) return 0;
  return ws_bytes_d((uint64_t)pe->dim, k, prec, extended != 0);
}

size_t kg_pe_states_bytes(const kg_pe* pe, int32_t N, int32_t ckpt_every, int32_t prec) {
  if (check_pe(pe) != KG_OK || check_prec(prec) != KG_OK) return 0;
  if (N < 1 || ckpt_every < 0 || ckpt_every > N) {
    fail(KG_EINVAL, "bad N=%d or ckpt_every=%d", N, ckpt_every);
    return 0;
  }
  return states_bytes_d((uint64_t)pe->dim, N, ckpt_every, prec);
}

kg_status xxz_pe_apply(const kg_xxz* h, const kg_pe* pe, double u, int32_t prec, const void* v,
                       void* w, void* stream) {
  KG_CHECK(check_pe_chain(h, pe));
  KG_CHECK(check_prec(prec));
  if (!isfinite(u)) return fail(KG_EINVAL, "u must be finite");
  KG_CHECK(check_vec(v, prec, "v"));
  KG_CHECK(check_vec(w, prec, "w"));
  if (overlap(v, w, vbytes((uint64_t)pe->dim, prec))) return fail(KG_EINVAL, "v and w overlap");
  const PeArgs pa = pe_args(pe);
  KG_HIP(launch_hv_pe(prec, make_hv(h, nullptr, u), pa, v, w, (hipStream_t)stream), "xxz_pe_apply");
  return ok();
}

kg_status krylov_expv_pe(const kg_xxz* h, const kg_pe* pe, double u, double t, const kg_krylov* k,
                         int32_t prec, const void* v_in, void* v_out, void* ws, size_t ws_bytes,
                         int32_t* m_eff_dev, void* stream) {
  KG_CHECK(check_pe_chain(h, pe));
  const PeArgs pa = pe_args(pe);
  const Space sp{make_geo_pe(h->L, (uint64_t)pe->dim), &pa};
  return expv_impl(h, sp, u, t, k, prec, v_in, v_out, ws, ws_bytes, m_eff_dev, stream);
}

kg_status grape_forward_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev, int32_t N,
                           double dt, const kg_krylov* k, int32_t prec, const void* psi0,
                           const void* target, double* F_dev, double* beta_dev, void* states,
                           int32_t ckpt_every, void* ws, size_t ws_bytes, void* stream) {
  KG_CHECK(check_pe_chain(h, pe));
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0, target, states, ckpt_every, KG_PE_MAX_L));
  const PeArgs pa = pe_args(pe);
  const Space sp{make_geo_pe(h->L, (uint64_t)pe->dim), &pa};
  return forward_impl(h, sp, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, states,
                      ckpt_every, ws, ws_bytes, stream, "grape_forward_pe");
}

kg_status grape_gradient_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev, int32_t N,
                            double dt, const kg_krylov* k, int32_t prec, const void* psi0,
                            const void* target, double* F_dev, double* beta_dev, double* grad_dev,
                            void* states, int32_t ckpt_every, int32_t states_valid,
                            int32_t variant, int32_t nodes, void* ws, size_t ws_bytes,
                            void* stream) {
  KG_CHECK(check_pe_chain(h, pe));
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0, target, states, ckpt_every, KG_PE_MAX_L));
  Quadrature Q;
  const Quadrature* qp = nullptr;
  switch (variant) {
    case KG_GRAD_ZEROTH:
    case KG_GRAD_CENTRED:
    case KG_GRAD_FIRST_ORDER:
      if (nodes != 0) return fail(KG_EINVAL, "nodes must be 0 for variant %d", variant);
      break;
    case KG_GRAD_QUADRATURE:
      KG_CHECK(make_quadrature(nodes, dt, &Q));
      qp = &Q;
      break;
    default:
      return fail(KG_EINVAL, "unknown gradient variant %d", variant);
  }
  const PeArgs pa = pe_args(pe);
  const Space sp{make_geo_pe(h->L, (uint64_t)pe->dim), &pa};
  return gradient_core(h, sp, u_dev, N, dt, k, prec, psi0, target, F_dev, beta_dev, grad_dev,
                       states, ckpt_every, states_valid, ws, ws_bytes, stream,
                       variant == KG_GRAD_CENTRED, "grape_gradient_pe", qp,
                       variant == KG_GRAD_FIRST_ORDER);
}

kg_status grape_gradient_columns_pe(const kg_xxz* h, const kg_pe* pe, const double* u_dev,
                                    int32_t N, double dt, const kg_krylov* k, int32_t prec,
                                    int32_t n_cols, const void* psi0s, const void* targets,
                                    double* F_dev, double* beta_dev, double* beta_cols_dev,
                                    double* grad_dev, void* states, int32_t ckpt_every,
                                    int32_t centred, void* ws, size_t ws_bytes, void* stream) {
  KG_CHECK(check_pe_chain(h, pe));
  KG_CHECK(check_sweep(h, u_dev, N, dt, k, prec, psi0s, targets, states, ckpt_every, KG_PE_MAX_L));
  const PeArgs pa = pe_args(pe);
  const Space sp{make_geo_pe(h->L, (uint64_t)pe->dim), &pa};
  return columns_core(h, sp, u_dev, N, dt, k, prec, n_cols, psi0s, targets, F_dev, beta_dev,
                      beta_cols_dev, grad_dev, states, ckpt_every, centred, ws, ws_bytes, stream);
}

kg_status kg_debug_index_map(int32_t L, uint32_t s0, uint32_t count, int32_t* n_anti_dev,
                             uint32_t* partner_mask_dev, void* stream) {
  if (L < KG_MIN_L || L > KG_MAX_L) return fail(KG_EINVAL, "L=%d outside [%d, %d]", L, KG_MIN_L, KG_MAX_L);
  if (!n_anti_dev || !partner_mask_dev) return fail(KG_EINVAL, "outputs are required");
  if ((uint64_t)s0 + count > ((uint64_t)1 << L)) return fail(KG_EINVAL, "range exceeds 2^L");
  if (count == 0) return ok();
  KG_HIP(launch_index_map(L, s0, count, n_anti_dev, partner_mask_dev, (hipStream_t)stream),
         "kg_debug_index_map");
  return ok();
}

}  // extern "C"

namespace kg {

// Algorithmic bytes of one reduced-basis H v: x read and y written (2 vb), the
// orbit labels read, and either the labels' ranks (forming the neighbours'
// ranks in the kernel) or the neighbour slots the slices use (64 of 4 bytes per
// slot).  The slot total is counted once per (L, K) by enumerating the orbit
// labels in ascending order, as the table builder does.
double pe_gather_bytes(const PeArgs& p, double vb) {
  const double labels = 4.0 * (double)p.dim;
  if (!p.nbr) return 2.0 * vb + 2.0 * labels;
  static std::mutex mu;
  static std::map<std::pair<int, int>, uint64_t> slots;
  std::lock_guard<std::mutex> lock(mu);
  auto it = slots.find({p.L, p.K});
  if (it == slots.end()) {
    const int L = p.L, ones = L - p.K;
    const uint64_t full = (L == 32) ? 0xFFFFFFFFull : ((1ull << L) - 1ull);
    const uint32_t bondmask = (L == 32) ? 0x7FFFFFFFu : ((1u << (L - 1)) - 1u);
    uint64_t v = ones ? ((1ull << ones) - 1ull) : 0ull, row = 0, total = 0;
    uint32_t cmax = 0;
    while (true) {
      const uint32_t s = (uint32_t)v;
      if (s <= reverse_bits_fast(s, L)) {
        cmax = std::max(cmax, (uint32_t)__builtin_popcount((s ^ (s >> 1)) & bondmask));
        if ((++row & 63u) == 0u) { total += cmax; cmax = 0; }
      }
      if (ones == 0) break;
      const uint64_t c = v & (~v + 1ull);
      const uint64_t r = v + c;
      v = (((r ^ v) >> 2) / c) | r;
      if (v > full) break;
    }
    if (row & 63u) total += cmax;
    it = slots.emplace(std::make_pair(p.L, p.K), total).first;
  }
  return 2.0 * vb + labels + 256.0 * (double)it->second;
}

}  // namespace kg
