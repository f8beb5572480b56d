// C ABI of the LocalPower library: problem handle, workspace layout, the
// round driver (Algorithm 1 with sign-fixing / OPT alignment) and its hipGraph
// replay.  Host code only; the kernels live in k_local.hip and k_small.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "lp_internal.h"

namespace {

thread_local std::string g_err;

lp_status fail(lp_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define LP_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Free list of the sin theta result cells (shared by all devices: a cell index
// in use on one device is not handed out on another, which is only cautious).
std::mutex g_sin_mu;
uint64_t g_sin_busy = 0;

int take_sin_cell() {
  std::lock_guard<std::mutex> g(g_sin_mu);
  for (int c = 0; c < lp::kSinSlots; ++c)
    if (!(g_sin_busy >> c & 1)) {
      g_sin_busy |= uint64_t(1) << c;
      return c;
    }
  return -1;
}

void give_sin_cell(int c) {
  std::lock_guard<std::mutex> g(g_sin_mu);
  g_sin_busy &= ~(uint64_t(1) << c);
}

size_t elem_bytes(lp_dtype t) { return t == LP_F64 ? 8 : (t == LP_F32 ? 4 : 2); }

bool check_offsets(const int64_t* o, int32_t m, int64_t n, std::string* err) {
  if (o == nullptr || m < 1) {
    *err = "offsets must be non-NULL with m >= 1";
    return false;
  }
  if (o[0] != 0 || o[m] != n) {
    *err = "offsets[0] must be 0 and offsets[m] must be n";
    return false;
  }
  for (int i = 0; i < m; ++i)
    if (o[i + 1] <= o[i]) {
      *err = "offsets must increase strictly (every partition non-empty)";
      return false;
    }
  return true;
}

}  // namespace

namespace lp {

bool make_plan(lp_dtype dtype, int64_t n, int64_t d, const int64_t* offsets, int32_t m,
               int32_t k_max, Plan* P, std::string* err) {
  if (dtype != LP_F64 && dtype != LP_F32 && dtype != LP_BF16) {
    *err = "unknown dtype";
    return false;
  }
  if (n < 1 || d < 1) {
    *err = "need n >= 1 and d >= 1";
    return false;
  }
  if (k_max < 1 || k_max > kMaxK || k_max > d) {
    *err = "need 1 <= k_max <= min(d, 64)";
    return false;
  }
  if (!check_offsets(offsets, m, n, err)) return false;
  P->dtype = dtype;
  P->n = n;
  P->d = d;
  P->m = m;
  P->k_max = k_max;
  P->acc_bytes = dtype == LP_F64 ? 8 : 4;
  P->zw_bytes = dtype == LP_F64 ? 8 : 4;
  P->path = LocalPath::TwoPass;
  P->lda = 0;
  // about 512 work items (two resident workgroups per CU), 16-row granularity
  int64_t cr = (n + 511) / 512;
  cr = ((cr + 15) / 16) * 16;
  cr = std::max<int64_t>(16, std::min<int64_t>(cr, 4096));
  P->min_chunk_rows = cr;
  P->variant = 1;
  P->nt_loads = true;
  P->split_operands = false;
  P->valu = true;
  build_items(P, offsets, cr);
  P->n_gram_chunks = (int32_t)((d + kGramRows - 1) / kGramRows);
  const size_t dk = (size_t)d * k_max;
  const size_t mb = (size_t)std::max(m, 1);
  Layout& L = P->L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.Zi = take(mb * dk * 8);
  L.Zw = take(mb * dk * P->zw_bytes);
  L.Yi = take(mb * dk * 8);
  L.tmp = take(mb * dk * 8);
  L.Z = take(dk * 8);
  L.Zw_shared = take(dk * P->zw_bytes);
  L.Y = take(dk * 8);
  L.Uref = take(dk * 8);
  L.part = take(P->items.size() * dk * P->acc_bytes);
  L.tbuf = take((size_t)n * k_max * P->acc_bytes);
  L.gram = take(mb * P->n_gram_chunks * (size_t)k_max * k_max * 8);
  L.gram2 = take(mb * P->n_gram_chunks * (size_t)k_max * k_max * 8);
  L.rinv = take(mb * 2 * (size_t)k_max * k_max * 8);   // R^{-1} per matrix, then summed Grams
  L.omat = take(mb * (size_t)k_max * k_max * 8);
  L.sgn = take(mb * k_max);
  L.flags = take((mb + 2) * 4);
  L.items = take(P->items.size() * sizeof(WorkItem));
  L.slot_off = take((mb + 1) * 4);
  L.hist = take(kHistCap * 8);
  L.ctr = take(4);
  L.scal = take(64 * 8);
  L.rho = take(kHistCap * 8);
  L.rho_part = take(mb * 8);
  L.rho_ctr = take(4);
  L.sinw = take(sin_theta_scratch_doubles(d, k_max, k_max) * 8);   // per-round sin theta
  // start and end stamps of every workgroup of one two-pass local multiply at the
  // default work-item size (pass 1: items x 128-row blocks, pass 2: items x
  // 256-column blocks)
  P->stamp_cap = (int64_t)P->items.size() * ((cr + 127) / 128 + (d + 255) / 256);
  L.stamps = take((size_t)P->stamp_cap * 16);
  L.total = o;
  return true;
}

void build_items(Plan* P, const int64_t* offsets, int64_t cr) {
  P->chunk_rows = cr;
  P->items.clear();
  int32_t slot = 0;
  for (int i = 0; i < P->m; ++i) {
    for (int64_t r = offsets[i]; r < offsets[i + 1]; r += cr) {
      WorkItem it;
      it.part = i;
      it.slot = slot++;
      it.row0 = r;
      it.rows = std::min<int64_t>(cr, offsets[i + 1] - r);
      P->items.push_back(it);
    }
  }
}

hipError_t launch_local_multiply(const Plan& P, const void* A, int64_t lda, int k, const void* Zw,
                                 int64_t z_stride, void* tbuf, void* part,
                                 const WorkItem* items_dev, int nitems, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  if (P.valu && valu_eligible(P.dtype, P.d, lda, k, A))
    return launch_local_multiply_valu(P, A, lda, k, Zw, z_stride, part, items_dev, nitems, s);
  if (P.path == LocalPath::Mfma32 && mfma32_eligible(P.dtype, P.d, lda, k))
    return launch_local_multiply_mfma32(P, A, lda, k, Zw, z_stride, part, items_dev, nitems, s);
  if (P.path == LocalPath::MfmaBf16 && mfma16_eligible(P.dtype, P.d, lda, k, A, P.split_operands))
    return launch_local_multiply_mfma16(P, A, lda, k, Zw, z_stride, part, items_dev, nitems, s);
  if (gemm_eligible(P.dtype, P.d, lda, A)) {
    // without a named kernel: split operands on BF16 matrix cores for BF16 A (three
    // BF16 products, exact) and for k > 16 (where FP32 matrix cores bind)
    const bool split = P.split_products || (P.two_pass_auto && (P.dtype == LP_BF16 || k > 16));
    return split ? launch_local_multiply_gemm3(P, A, lda, k, Zw, z_stride, tbuf, part, items_dev, nitems, s)
                 : launch_local_multiply_gemm(P, A, lda, k, Zw, z_stride, tbuf, part, items_dev, nitems, s);
  }
  return launch_local_multiply_twopass(P, A, lda, k, Zw, z_stride, tbuf, part, items_dev, nitems, s);
}

hipError_t cholqr2_passes(int batch, int64_t d, int k, const double* Y, const double* gram,
                          double* gram2, double* tmp, double* rfac, double* Q, void* zw,
                          size_t zw_bytes, int32_t* flags, hipStream_t s) {
  const int nch = (int)((d + kGramRows - 1) / kGramRows);
  hipError_t e;
  // pass 1: R1 = chol(Y^T Y), Q1 = Y R1^{-1}, and the Gram partials of Q1
  if ((e = launch_chol_solve(batch, d, k, nch, Y, gram, rfac, tmp, nullptr, 0, gram2, flags, s)) !=
      hipSuccess)
    return e;
  // pass 2: R2 = chol(Q1^T Q1), Q = Q1 R2^{-1} (and the working copy)
  return launch_chol_solve(batch, d, k, chol_solve_chunks(d, k), tmp, gram2, rfac, Q, zw,
                           zw_bytes, nullptr, flags, s);
}

hipError_t cholqr2_from_gram(const Plan& P, char* ws, int batch, int64_t d, int k, const double* Y,
                             double* Q, void* zw, int32_t* flags, hipStream_t s, int b0) {
  const Layout& L = P.L;
  const int nch = (int)((d + kGramRows - 1) / kGramRows);
  const int64_t kk = (int64_t)k * k;
  double* gram = (double*)(ws + L.gram) + (int64_t)b0 * nch * kk;
  double* gram2 = (double*)(ws + L.gram2) + (int64_t)b0 * nch * kk;
  double* tmp = (double*)(ws + L.tmp) + (int64_t)b0 * d * k;
  double* rfac = (double*)(ws + L.rinv) + (int64_t)b0 * 2 * kk;
  return cholqr2_passes(batch, d, k, Y, gram, gram2, tmp, rfac, Q, zw, P.zw_bytes, flags, s);
}

hipError_t cholqr2(const Plan& P, char* ws, int batch, int64_t d, int k, const double* Y, double* Q,
                   void* zw, int32_t* flags, hipStream_t s) {
  const int64_t dk = d * k;
  hipError_t e = launch_cross_gram(batch, d, k, Y, dk, Y, dk, (double*)(ws + P.L.gram), s);
  if (e != hipSuccess) return e;
  return cholqr2_from_gram(P, ws, batch, d, k, Y, Q, zw, flags, s);
}

}  // namespace lp

using namespace lp;

namespace {

struct Ptrs {
  double *Zi, *Yi, *Z, *Y, *Uref, *gram, *omat, *hist, *rho, *rho_part, *sinw;
  void *Zw, *Zw_shared, *part, *tbuf;
  int8_t* sgn;
  int32_t *flags, *slot_off, *ctr, *rho_ctr;
  WorkItem* items;
};

Ptrs ptrs(lp_problem* P) {
  const Layout& L = P->plan.L;
  char* w = P->ws;
  Ptrs p;
  p.Zi = (double*)(w + L.Zi);
  p.Yi = (double*)(w + L.Yi);
  p.Z = (double*)(w + L.Z);
  p.Y = (double*)(w + L.Y);
  p.Uref = (double*)(w + L.Uref);
  p.gram = (double*)(w + L.gram);
  p.omat = (double*)(w + L.omat);
  p.hist = (double*)(w + L.hist);
  p.rho = (double*)(w + L.rho);
  p.rho_part = (double*)(w + L.rho_part);
  p.sinw = (double*)(w + L.sinw);
  p.rho_ctr = (int32_t*)(w + L.rho_ctr);
  p.Zw = w + L.Zw;
  p.Zw_shared = w + L.Zw_shared;
  p.part = w + L.part;
  p.tbuf = w + L.tbuf;
  p.sgn = (int8_t*)(w + L.sgn);
  p.flags = (int32_t*)(w + L.flags);
  p.slot_off = (int32_t*)(w + L.slot_off);
  p.ctr = (int32_t*)(w + L.ctr);
  p.items = (WorkItem*)(w + L.items);
  return p;
}

constexpr int kEvPairs = 256;

// Sum the durations of the recorded event pairs into P->ms_local.
hipError_t drain_timing(lp_problem* P) {
  if (P->ev_used == 0) return hipSuccess;
  hipError_t e = hipStreamSynchronize(P->stream);
  if (e != hipSuccess) return e;
  for (int j = 0; j < P->ev_used; ++j) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, P->ev_pool[2 * j], P->ev_pool[2 * j + 1]);
    if (e != hipSuccess) return e;
    P->ms_local += ms;
  }
  P->local_launches += P->ev_used;
  P->ev_used = 0;
  return hipSuccess;
}

// Add an event-record node to the graph being captured on `s`, after the nodes
// the stream's next operation would depend on, and make it the new dependency.
hipError_t capture_event_node(hipStream_t s, hipEvent_t ev) {
  hipStreamCaptureStatus st;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  hipError_t e = hipStreamGetCaptureInfo_v2(s, &st, &id, &g, &deps, &nd);
  if (e != hipSuccess) return e;
  if (st != hipStreamCaptureStatusActive || g == nullptr) return hipErrorInvalidValue;
  hipGraphNode_t node;
  if ((e = hipGraphAddEventRecordNode(&node, g, deps, nd, ev)) != hipSuccess) return e;
  return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
}

// One local iteration on every partition: Yi = A_i^T (A_i Z_i).  When this
// launch is timed, it is bracketed by a pair of events: external event nodes of
// the timed graph instance being captured, or plain event records.
// The local-Gram form splits the contraction of its multiply in two at k <= 16
// when the partial buffer holds two Y_i per partition; the reduction then reads
// the matching slot offsets.
int gram_split(const lp_problem* P, int k) { return (k <= 16 && P->gram_split2) ? 2 : 1; }
const int32_t* gram_slots(const lp_problem* P, int k) {
  return gram_split(P, k) == 2 ? P->gram_slot_off + P->m + 1 : P->gram_slot_off;
}

hipError_t local_iter(lp_problem* P, int k, const void* zsrc, int64_t zstride) {
  Ptrs p = ptrs(P);
  hipError_t e;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  const bool timed = P->timing_now;
  if (timed && P->timing_slot >= 0) {
    const int pair = P->timing_slot * kPairsPerSlot + P->timing_pair++;
    ev0 = P->ev_pool[2 * pair];
    ev1 = P->ev_pool[2 * pair + 1];
    if ((e = capture_event_node(P->stream, ev0)) != hipSuccess) return e;
  } else if (timed) {
    if (P->ev_used == kEvPairs && (e = drain_timing(P)) != hipSuccess) return e;
    ev0 = P->ev_pool[2 * P->ev_used];
    ev1 = P->ev_pool[2 * P->ev_used + 1];
    P->ev_used++;
    if ((e = hipEventRecord(ev0, P->stream)) != hipSuccess) return e;
  }
  if (P->gram_on)
    e = launch_gram_multiply(P->plan, P->gram_M, k, zsrc, zstride, p.tbuf, P->gram_items, P->m,
                             gram_split(P, k), P->stream);
  else
    e = launch_local_multiply(P->plan, P->A, P->lda, k, zsrc, zstride, p.tbuf, p.part, p.items,
                              (int)P->plan.items.size(), P->stream);
  if (e != hipSuccess) return e;
  if (ev1 != nullptr) {
    e = (P->timing_slot >= 0) ? capture_event_node(P->stream, ev1) : hipEventRecord(ev1, P->stream);
    if (e != hipSuccess) return e;
  }
  if (P->gram_on)  // Y_i itself, or its two contraction halves, as the FP32 partials
    return launch_reduce_gram(P->plan, k, p.tbuf, gram_slots(P, k), p.Yi, p.gram, 0, P->m,
                              P->stream);
  return launch_reduce_gram(P->plan, k, p.part, p.slot_off, p.Yi, p.gram, 0, P->m, P->stream);
}

// Bracket the next launch on stream s with the timing pair (ev0 before it) or
// close the bracket after it (ev1): external event nodes of the timed graph
// instance being captured, or plain event records.
hipError_t timing_mark(lp_problem* P, hipStream_t s, hipEvent_t ev) {
  return (P->timing_slot >= 0) ? capture_event_node(s, ev) : hipEventRecord(ev, s);
}

// Take the next pair of timing events (graph slot pair or plain pool pair).
hipError_t timing_pair(lp_problem* P, hipEvent_t* ev0, hipEvent_t* ev1) {
  if (P->timing_slot >= 0) {
    const int pair = P->timing_slot * kPairsPerSlot + P->timing_pair++;
    *ev0 = P->ev_pool[2 * pair];
    *ev1 = P->ev_pool[2 * pair + 1];
    return hipSuccess;
  }
  if (P->ev_used == kEvPairs) {
    hipError_t e = drain_timing(P);
    if (e != hipSuccess) return e;
  }
  *ev0 = P->ev_pool[2 * P->ev_used];
  *ev1 = P->ev_pool[2 * P->ev_used + 1];
  P->ev_used++;
  return hipSuccess;
}

// One communication round with the partitions in two halves on two streams
// (Algorithm 1; the same operations and the same arithmetic per partition as
// the one-stream round, only the order across partitions differs).  The local
// multiplies form one chain: half 0 then half 1 of step l, then half 0 of step
// l + 1, so each half's reduction, CholeskyQR2 and alignment run while the
// other half streams A.  Half 0 holds the base partition; half 1 aligns after
// the base's last local orthonormalisation.  The two halves join before the
// aggregation.  When the step is timed, one pair of events brackets both
// halves' local multiplies (back to back in the chain).
hipError_t enqueue_round_split(lp_problem* P, int k, int p, lp_agg mode, int hist) {
  Ptrs q = ptrs(P);
  const int64_t d = P->d;
  const int64_t dk = d * k;
  const int64_t kk = (int64_t)k * k;
  const int nch = P->plan.n_gram_chunks;
  const size_t zwb = P->plan.zw_bytes;
  const hipStream_t st[2] = {P->stream, P->stream2};
  hipError_t e;
#define LP_TRY(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
  LP_TRY(hipEventRecord(P->ev_fork, st[0]));
  LP_TRY(hipStreamWaitEvent(st[1], P->ev_fork, 0));
  const double* Zb = q.Zi + (int64_t)P->base * dk;
  for (int l = 1; l <= p; ++l) {
    const void* zsrc = (l == 1) ? q.Zw_shared : q.Zw;
    const int64_t zstride = (l == 1) ? 0 : dk;
    const bool timed = P->timing && (l == 1 || !P->timing_first_only);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (timed) LP_TRY(timing_pair(P, &ev0, &ev1));
    for (int h = 0; h < 2; ++h) {
      const Half& H = P->half[h];
      const hipStream_t s = st[h];
      double* Zi = q.Zi + (int64_t)H.b0 * dk;
      void* zw = (char*)q.Zw + (size_t)H.b0 * dk * zwb;
      double* gram = q.gram + (int64_t)H.b0 * nch * kk;
      if (l == p && p >= 2 && mode != LP_AGG_VANILLA) {
        if (h == 1) LP_TRY(hipStreamWaitEvent(s, P->ev_base, 0));
        if (mode == LP_AGG_SIGN) {
          LP_TRY(launch_diag_dot(H.nb, d, k, Zi, Zb, gram, s));
          LP_TRY(launch_sign_apply(H.nb, d, k, gram, Zi, zw, zwb, q.sgn + (int64_t)H.b0 * k, s));
        } else {
          double* O = q.omat + (int64_t)H.b0 * kk;
          LP_TRY(launch_cross_gram(H.nb, d, k, Zi, dk, Zb, 0, gram, s));
          LP_TRY(launch_procrustes(H.nb, nch, k, gram, O, q.flags + P->m + 1, s));
          LP_TRY(launch_right_mult(H.nb, d, k, Zi, O, kk, false, nullptr, zw, zwb, s));
        }
      }
      // the chain of local multiplies: after the other half's previous one
      if (l > 1 || h == 1) LP_TRY(hipStreamWaitEvent(s, P->ev_k1[1 - h], 0));
      if (timed && h == 0) LP_TRY(timing_mark(P, s, ev0));
      LP_TRY(launch_local_multiply(P->plan, P->A, P->lda, k, zsrc, zstride, q.tbuf, q.part,
                                   q.items + H.it0, H.nit, s));
      if (timed && h == 1) LP_TRY(timing_mark(P, s, ev1));
      LP_TRY(hipEventRecord(P->ev_k1[h], s));
      LP_TRY(launch_reduce_gram(P->plan, k, q.part, q.slot_off, q.Yi, q.gram, H.b0, H.nb, s));
      if (l < p) {
        LP_TRY(cholqr2_from_gram(P->plan, P->ws, H.nb, d, k, q.Yi + (int64_t)H.b0 * dk, Zi, zw,
                                 q.flags + H.b0, s, H.b0));
        if (h == 0 && l == p - 1) LP_TRY(hipEventRecord(P->ev_base, s));
      }
    }
  }
  LP_TRY(hipEventRecord(P->ev_join2, st[1]));
  LP_TRY(hipStreamWaitEvent(st[0], P->ev_join2, 0));
  const hipStream_t s = st[0];
  LP_TRY(launch_aggregate_gram(P->m, d, k, q.Yi, 1.0 / (double)P->n, q.Y, q.gram, s));
  LP_TRY(cholqr2_from_gram(P->plan, P->ws, 1, d, k, q.Y, q.Z, q.Zw_shared, q.flags + P->m, s));
  if (hist > 0) LP_TRY(launch_sin_theta_chunked(d, k, hist, q.Z, q.Uref, q.sinw, nullptr, q.hist, q.ctr, s));
#undef LP_TRY
  return hipSuccess;
}

// Enqueue one communication round with p local steps (only kernel launches, so
// the sequence can be captured into a graph).
hipError_t enqueue_round(lp_problem* P, int k, int p, lp_agg mode, int hist) {
  if (P->split_now) return enqueue_round_split(P, k, p, mode, hist);
  Ptrs q = ptrs(P);
  hipStream_t s = P->stream;
  const int m = P->m;
  const int64_t d = P->d;
  const int64_t dk = d * k;
  const int nch = P->plan.n_gram_chunks;
  hipError_t e;
  for (int l = 1; l <= p; ++l) {
    const void* zsrc = (l == 1) ? q.Zw_shared : q.Zw;
    const int64_t zstride = (l == 1) ? 0 : dk;
    if (l == p && p >= 2 && P->rho_now) {
      // residual error of the inputs of the last local step (before any alignment)
      if ((e = launch_rho(m, d, k, mode == LP_AGG_OPT, q.Zi, q.rho_part, q.rho, q.rho_ctr, s)) !=
          hipSuccess)
        return e;
    }
    if (l == p && p >= 2 && mode != LP_AGG_VANILLA) {
      // align the inputs of the last local step against the base node's
      const double* Zb = q.Zi + (int64_t)P->base * dk;
      if (mode == LP_AGG_SIGN) {
        if ((e = launch_diag_dot(m, d, k, q.Zi, Zb, q.gram, s)) != hipSuccess) return e;
        if ((e = launch_sign_apply(m, d, k, q.gram, q.Zi, q.Zw, P->plan.zw_bytes, q.sgn, s)) !=
            hipSuccess)
          return e;
      } else {
        if ((e = launch_cross_gram(m, d, k, q.Zi, dk, Zb, 0, q.gram, s)) != hipSuccess) return e;
        if ((e = launch_procrustes(m, nch, k, q.gram, q.omat, q.flags + m + 1, s)) != hipSuccess)
          return e;
        if ((e = launch_right_mult(m, d, k, q.Zi, q.omat, (int64_t)k * k, false, nullptr, q.Zw,
                                   P->plan.zw_bytes, s)) != hipSuccess)
          return e;
      }
    }
    P->timing_now = P->timing && (l == 1 || !P->timing_first_only);
    e = local_iter(P, k, zsrc, zstride);
    P->timing_now = false;
    if (e != hipSuccess) return e;
    if (l < p) {
      if ((e = cholqr2_from_gram(P->plan, P->ws, m, d, k, q.Yi, q.Zi, q.Zw, q.flags, s)) !=
          hipSuccess)
        return e;
    }
  }
  if (p == 1 && P->rho_now &&
      (e = launch_rho(0, d, k, false, q.Zi, q.rho_part, q.rho, q.rho_ctr, s)) != hipSuccess)
    return e;
  if ((e = launch_aggregate_gram(m, d, k, q.Yi, 1.0 / (double)P->n, q.Y, q.gram, s)) != hipSuccess)
    return e;
  if ((e = cholqr2_from_gram(P->plan, P->ws, 1, d, k, q.Y, q.Z, q.Zw_shared, q.flags + m, s)) !=
      hipSuccess)
    return e;
  if (hist > 0) {
    if ((e = launch_sin_theta_chunked(d, k, hist, q.Z, q.Uref, q.sinw, nullptr, q.hist, q.ctr, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// hist > 0: after the round, append sin theta of Z (d x k) against the first
// hist columns of the reference to the device history.
lp_status run_round(lp_problem* P, int k, int p, lp_agg mode, int hist, bool use_graph,
                    int slot) {
  if (!use_graph) {
    LP_HIP(enqueue_round(P, k, p, mode, hist));
    return LP_OK;
  }
  GraphKey key{k, p, (int)mode, hist, slot, slot >= 0 && P->timing_first_only ? 1 : 0,
               P->split_now ? 1 : 0, P->rho_now ? 1 : 0};
  auto it = P->graphs.find(key);
  if (it == P->graphs.end()) {
    hipGraph_t g = nullptr;
    LP_HIP(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
    P->timing_slot = slot;
    P->timing_pair = 0;
    hipError_t e = enqueue_round(P, k, p, mode, hist);
    P->timing_slot = -1;
    hipError_t e2 = hipStreamEndCapture(P->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return fail(LP_EDEVICE, std::string("capture: ") +
                                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(LP_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e3));
    it = P->graphs.emplace(key, ex).first;
  }
  LP_HIP(hipGraphLaunch(it->second, P->stream));
  return LP_OK;
}

// Sum the event pairs of the timed graph instances replayed since the last harvest.
hipError_t harvest_slots(lp_problem* P, std::vector<std::pair<int, int>>& pending) {
  if (pending.empty()) return hipSuccess;
  hipError_t e = hipStreamSynchronize(P->stream);
  if (e != hipSuccess) return e;
  for (auto& sp : pending) {
    for (int j = 0; j < sp.second; ++j) {
      const int pair = sp.first * kPairsPerSlot + j;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, P->ev_pool[2 * pair], P->ev_pool[2 * pair + 1]);
      if (e != hipSuccess) return e;
      P->ms_local += ms;
      P->local_launches++;
    }
  }
  pending.clear();
  return hipSuccess;
}

// Make the problem's own stream wait for the caller's stream.
// The fused kernel family this problem can use (TwoPass when none applies).
LocalPath fused_kind(const lp_problem* P) {
  // the fused matrix-core kernels take every rank up to their tile width
  if (mfma32_eligible(P->dtype, P->d, P->lda, 1)) return LocalPath::Mfma32;
  if (mfma16_eligible(P->dtype, P->d, P->lda, 1, P->A, false)) return LocalPath::MfmaBf16;
  return LocalPath::TwoPass;
}

// Whether a fused (single-pass) kernel handles this k.
bool fused_for_k(const lp_problem* P, int k) {
  if (P->plan.valu && valu_eligible(P->dtype, P->d, P->lda, k, P->A)) return true;
  switch (fused_kind(P)) {
    case LocalPath::Mfma32: return mfma32_eligible(P->dtype, P->d, P->lda, k);
    case LocalPath::MfmaBf16:
      return mfma16_eligible(P->dtype, P->d, P->lda, k, P->A, P->plan.split_operands);
    default: return false;
  }
}

lp_status join_in(lp_problem* P) {
  LP_HIP(hipEventRecord(P->ev_join_in, P->user_stream));
  LP_HIP(hipStreamWaitEvent(P->stream, P->ev_join_in, 0));
  return LP_OK;
}

// Make the caller's stream wait for the problem's own stream.
lp_status join_out(lp_problem* P) {
  LP_HIP(hipEventRecord(P->ev_join_out, P->stream));
  LP_HIP(hipStreamWaitEvent(P->user_stream, P->ev_join_out, 0));
  return LP_OK;
}

// Copy the work list and the per-partition slot prefix to the device (synchronous).
// The two-pass kernels write one d x k partial per work item, read back by the
// reduction; one workgroup per item matters only to the fused kernels.  When the
// problem's rank runs two-pass, items of 16 k acc / b rows keep the partials
// under 1/16 of A's bytes, as long as items x ceil(d / 256) pass-2 workgroups
// still cover the chip (512).  (At d = 4096, n = 65536, k = 64 in BF16 the
// default items wrote as many partial bytes as A holds.)  Returns whether the
// work list changed (it then needs an upload).
bool two_pass_items(lp_problem* P) {
  if (fused_for_k(P, P->k_max)) return false;
  const int64_t b = P->dtype == LP_F64 ? 8 : (P->dtype == LP_F32 ? 4 : 2);
  int64_t cr = std::min<int64_t>(16 * (int64_t)P->k_max * (int64_t)P->plan.acc_bytes / b,
                                 P->n * ((P->d + 255) / 256) / 512);
  cr = std::min<int64_t>(cr / 16 * 16, 4096);
  if (cr <= P->plan.chunk_rows) return false;
  build_items(&P->plan, P->offsets.data(), cr);
  return true;
}

lp_status upload_items(lp_problem* P) {
  const int m = P->m;
  std::vector<int32_t> slot_off(m + 1, 0);
  for (const WorkItem& it : P->plan.items) slot_off[it.part + 1]++;
  for (int i = 0; i < m; ++i) slot_off[i + 1] += slot_off[i];
  Ptrs p = ptrs(P);
  LP_HIP(hipMemcpyAsync(p.items, P->plan.items.data(), P->plan.items.size() * sizeof(WorkItem),
                        hipMemcpyHostToDevice, P->stream));
  LP_HIP(hipMemcpyAsync(p.slot_off, slot_off.data(), (m + 1) * sizeof(int32_t),
                        hipMemcpyHostToDevice, P->stream));
  LP_HIP(hipStreamSynchronize(P->stream));
  // halves for split rounds: cut where the rows reach half of n (at least one
  // partition on each side); half 0 is the side that holds the base partition
  P->can_split = m >= 2;
  if (P->can_split) {
    int cut = 1;
    while (cut < m - 1 && 2 * P->offsets[cut] < P->n) ++cut;
    int item_cut = 0;
    while (item_cut < (int)P->plan.items.size() && P->plan.items[item_cut].part < cut) ++item_cut;
    const Half lo{0, cut, 0, item_cut};
    const Half hi{cut, m - cut, item_cut, (int)P->plan.items.size() - item_cut};
    P->half[0] = P->base < cut ? lo : hi;
    P->half[1] = P->base < cut ? hi : lo;
  }
  return LP_OK;
}

lp_status check_k(lp_problem* P, int32_t k) {
  if (k < 1 || k > P->k_max) return fail(LP_EINVAL, "need 1 <= k <= k_max");
  for (int i = 0; i < P->m; ++i)
    if (P->offsets[i + 1] - P->offsets[i] < k)
      return fail(LP_EINVAL, "every partition needs at least k rows");
  return LP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Step-wise driving (the serving layer runs many problems one round at a time;
// everything is enqueued on the problem's own stream, nothing synchronises).
// ---------------------------------------------------------------------------
namespace lp {

lp_status drive_begin(lp_problem* P, int k, const double* Y0, bool orthonormal) {
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  Ptrs q = ptrs(P);
  hipStream_t s = P->stream;
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(launch_fill_i32(q.flags, P->m + 2, 0, s));
  LP_HIP(launch_fill_i32(q.ctr, 1, 0, s));
  if (orthonormal) {
    LP_HIP(hipMemcpyAsync(q.Z, Y0, (size_t)P->d * k * 8, hipMemcpyDeviceToDevice, s));
    LP_HIP(launch_to_working(P->plan, 1, P->d, k, q.Z, q.Zw_shared, s));
  } else {
    LP_HIP(cholqr2(P->plan, P->ws, 1, P->d, k, Y0, q.Z, q.Zw_shared, q.flags + P->m, s));
  }
  return LP_OK;
}

lp_status drive_round(lp_problem* P, int k, int p, lp_agg mode) {
  if (p < 1) return fail(LP_EINVAL, "p must be >= 1");
  P->split_now = false;   // served jobs keep to their own stream
  return run_round(P, k, p, mode, 0, true, -1);
}

const double* drive_z(lp_problem* P) { return ptrs(P).Z; }

hipError_t drive_change(lp_problem* P, int k, const double* Zprev, double* out) {
  Ptrs q = ptrs(P);
  return launch_sin_theta_chunked(P->d, k, k, q.Z, Zprev, q.sinw, out, nullptr, nullptr, P->stream);
}

lp_status report(lp_status s, const std::string& msg) { return fail(s, msg); }

hipStream_t drive_stream(lp_problem* P) { return P->stream; }

void drive_prefer_matrix_cores(lp_problem* P, int k) {
  const bool bf16 = P->dtype == LP_BF16 &&
                    mfma16_eligible(P->dtype, P->d, P->lda, k, P->A, P->plan.split_operands);
  const bool fp32 = P->dtype == LP_F32 && k >= 5 && mfma32_eligible(P->dtype, P->d, P->lda, k);
  if (k <= 8 && (bf16 || fp32)) P->plan.valu = false;
}

lp_status drive_split_operands(lp_problem* P, bool split) {
  P->plan.split_operands = split;
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  // split operands at k > 16, d = 2048 move the rank to the two-pass kernels
  return two_pass_items(P) ? upload_items(P) : LP_OK;
}

lp_status drive_breakdowns(lp_problem* P, int* breakdowns) {
  Ptrs q = ptrs(P);
  std::vector<int32_t> flags(P->m + 2, 0);
  LP_HIP(hipMemcpyAsync(flags.data(), q.flags, (P->m + 2) * 4, hipMemcpyDeviceToHost, P->stream));
  LP_HIP(hipStreamSynchronize(P->stream));
  int b = 0;
  for (int i = 0; i < P->m + 1; ++i) b += flags[i];
  *breakdowns = b;
  return LP_OK;
}

}  // namespace lp

extern "C" {

const char* lp_strerror(lp_status s) {
  switch (s) {
    case LP_OK: return "ok";
    case LP_EINVAL: return "invalid argument";
    case LP_ENOMEM: return "insufficient memory";
    case LP_EDEVICE: return "HIP device error";
    case LP_EBREAKDOWN: return "Cholesky breakdown (rank-deficient iterate)";
    case LP_ENOTCONV: return "not converged";
    case LP_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* lp_last_error(void) { return g_err.c_str(); }

lp_status lp_workspace_size(lp_dtype dtype, int64_t n, int64_t d, const int64_t* offsets, int32_t m,
                            int32_t k_max, size_t* bytes) {
  if (bytes == nullptr) return fail(LP_EINVAL, "bytes is NULL");
  Plan P;
  std::string err;
  if (!make_plan(dtype, n, d, offsets, m, k_max, &P, &err)) return fail(LP_EINVAL, err);
  *bytes = P.L.total;
  return LP_OK;
}

lp_status lp_create(lp_problem** out, const void* A, lp_dtype dtype, int64_t n, int64_t d,
                    int64_t lda, const int64_t* offsets, int32_t m, int32_t k_max, void* workspace,
                    size_t ws_bytes, void* stream) {
  if (out == nullptr) return fail(LP_EINVAL, "out is NULL");
  *out = nullptr;
  if (A == nullptr) return fail(LP_EINVAL, "A is NULL");
  if (((uintptr_t)A & 15) != 0) return fail(LP_EINVAL, "A must be 16-byte aligned");
  if (lda < d) return fail(LP_EINVAL, "need lda >= d");
  if (workspace == nullptr || ((uintptr_t)workspace & 255) != 0)
    return fail(LP_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  std::string err;
  lp_problem* P = new (std::nothrow) lp_problem();
  if (P == nullptr) return fail(LP_ENOMEM, "host allocation failed");
  if (!make_plan(dtype, n, d, offsets, m, k_max, &P->plan, &err)) {
    delete P;
    return fail(LP_EINVAL, err);
  }
  if (ws_bytes < P->plan.L.total) {
    size_t need = P->plan.L.total;
    delete P;
    return fail(LP_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  P->plan.lda = lda;
  P->A = A;
  P->dtype = dtype;
  P->n = n;
  P->d = d;
  P->lda = lda;
  P->m = m;
  P->k_max = k_max;
  P->plan.path = fused_kind(P);
  // untuned defaults: the fused variants the autotuner picks on the benchmark shapes
  // (FP32: direct-to-LDS, software-pipelined, public local_kernel 9; BF16: four
  // waves, one tile ahead, public 2)
  if (P->plan.path == LocalPath::Mfma32) P->plan.variant = 7;
  if (P->plan.path == LocalPath::MfmaBf16) P->plan.variant = 0;
  P->offsets.assign(offsets, offsets + m + 1);
  two_pass_items(P);
  P->base = 0;
  for (int i = 1; i < m; ++i)
    if (offsets[i + 1] - offsets[i] > offsets[P->base + 1] - offsets[P->base]) P->base = i;
  P->ws = (char*)workspace;
  P->ws_bytes = ws_bytes;
  P->user_stream = (hipStream_t)stream;
  hipError_t e = hipGetDevice(&P->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking);

  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&P->ev_t0);
  if (e == hipSuccess) e = hipEventCreate(&P->ev_t1);
  if (e != hipSuccess) {
    delete P;
    return fail(LP_EDEVICE, std::string("stream/event creation: ") + hipGetErrorString(e));
  }
  // The workspace belongs to the caller's stream: wait for it before the first
  // write, since its memory may have been handed back while kernels queued on
  // that stream still use it.
  lp_status ust = join_in(P);
  if (ust == LP_OK) ust = upload_items(P);
  if (ust != LP_OK) {
    std::string msg = g_err;
    lp_destroy(P);
    return fail(ust, "upload of the work list: " + msg);
  }
  *out = P;
  return LP_OK;
}

lp_status lp_destroy(lp_problem* P) {
  if (P == nullptr) return LP_OK;
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& ev : P->ev_pool)
    if (ev) (void)hipEventDestroy(ev);
  if (P->stream) {
    (void)hipStreamSynchronize(P->stream);
    (void)hipStreamDestroy(P->stream);
  }
  if (P->stream2) {
    (void)hipStreamSynchronize(P->stream2);
    (void)hipStreamDestroy(P->stream2);
  }
  for (hipEvent_t ev : {P->ev_fork, P->ev_join2, P->ev_base, P->ev_k1[0], P->ev_k1[1]})
    if (ev) (void)hipEventDestroy(ev);
  if (P->ev_join_in) (void)hipEventDestroy(P->ev_join_in);
  if (P->ev_join_out) (void)hipEventDestroy(P->ev_join_out);
  if (P->ev_t0) (void)hipEventDestroy(P->ev_t0);
  if (P->ev_t1) (void)hipEventDestroy(P->ev_t1);
  if (P->change_host) (void)hipHostFree(P->change_host);
  delete P;
  return LP_OK;
}

lp_status lp_set_tuning(lp_problem* P, const lp_tuning* t) {
  if (P == nullptr || t == nullptr || t->struct_size < (int32_t)sizeof(lp_tuning))
    return fail(LP_EINVAL, "problem/tuning is NULL or struct_size too small");
  if (t->local_kernel < 0 || t->local_kernel > 11) return fail(LP_EINVAL, "local_kernel out of range");
  const bool two_pass = t->local_kernel == 1 || t->local_kernel == 11;
  if (t->local_kernel > 5 && !two_pass && fused_kind(P) == LocalPath::MfmaBf16)
    return fail(LP_EINVAL, "the BF16 fused kernel has four variants (local_kernel 2 to 5)");
  int64_t cr = t->chunk_rows == 0 ? P->plan.min_chunk_rows : t->chunk_rows;
  if (cr % 16 != 0 || cr < P->plan.min_chunk_rows)
    return fail(LP_EINVAL, "chunk_rows must be a multiple of 16 and >= the default");
  lp_status jst = join_in(P);
  if (jst != LP_OK) return jst;
  LP_HIP(hipStreamSynchronize(P->stream));
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  const LocalPath fk = fused_kind(P);
  if (two_pass || (t->local_kernel >= 2 && fk == LocalPath::TwoPass)) {
    P->plan.path = LocalPath::TwoPass;
  } else if (fk == LocalPath::Mfma32) {
    P->plan.path = fk;
    P->plan.variant = t->local_kernel >= 2 ? t->local_kernel - 2 : 7;   // automatic: the default
  } else if (fk == LocalPath::MfmaBf16) {
    P->plan.path = fk;
    const bool w8 = P->d == 1024 || P->d == 2048;   // the eight-wave forms need these widths
    const bool ahead = t->local_kernel >= 4;        // two tiles in flight per wave
    const bool eight = (t->local_kernel == 3 || t->local_kernel == 5) && w8;
    P->plan.variant = (ahead ? 2 : 0) + (eight ? 1 : 0);
  }
  P->plan.nt_loads = t->cached_loads == 0;
  P->plan.split_operands = t->split_operands != 0;
  P->plan.valu = t->local_kernel == 0;   // ranks <= 8: the vector-ALU kernel unless a kernel is named
  P->plan.split_products = t->local_kernel == 11;
  P->plan.two_pass_auto = t->local_kernel == 0;
  build_items(&P->plan, P->offsets.data(), cr);
  return upload_items(P);
}

lp_status lp_get_tuning(lp_problem* P, lp_tuning* t) {
  if (P == nullptr || t == nullptr) return fail(LP_EINVAL, "NULL argument");
  t->struct_size = sizeof(lp_tuning);
  t->local_kernel = P->plan.path == LocalPath::TwoPass ? (P->plan.split_products ? 11 : 1)
                                                       : 2 + P->plan.variant;
  t->chunk_rows = P->plan.chunk_rows;
  t->cached_loads = P->plan.nt_loads ? 0 : 1;
  t->split_operands = P->plan.split_operands ? 1 : 0;
  return LP_OK;
}

}  // extern "C"

namespace {

std::string tune_key(lp_problem* P, int k) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream os;
  os << arch << "|" << (int)P->dtype << "|" << P->n << "|" << P->d << "|" << P->m << "|" << k << "|"
     << P->lda << "|" << (P->plan.split_operands ? 1 : 0);
  return os.str();
}

bool cache_lookup(const std::string& path, const std::string& key, int32_t split, lp_tuning* t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last entry for a key wins
    const size_t eq = line.find('=');
    if (eq == std::string::npos || line.substr(0, eq) != key) continue;
    int lk = 0, cached = 0;
    long long cr = 0;
    if (std::sscanf(line.c_str() + eq + 1, "%d,%lld,%d", &lk, &cr, &cached) == 3) {
      t->struct_size = sizeof(lp_tuning);
      t->local_kernel = lk;
      t->chunk_rows = cr;
      t->cached_loads = cached;
      t->split_operands = split;
      found = true;
    }
  }
  return found;
}

// Z_out = the current iterate, or with ritz_out its Rayleigh-Ritz rotation
// after one p = 1 pass: Y = M Z, H = Z^T Y, H = Q diag(lam) Q^T, Z <- Z Q.
hipError_t finish_z(lp_problem* P, int k, double* Z_out, double* ritz_out) {
  Ptrs q = ptrs(P);
  hipStream_t s = P->stream;
  const int64_t d = P->d, dk = d * k;
  hipError_t e;
  if (ritz_out == nullptr) return hipMemcpyAsync(Z_out, q.Z, dk * 8, hipMemcpyDeviceToDevice, s);
  if ((e = local_iter(P, k, q.Zw_shared, 0)) != hipSuccess) return e;
  if ((e = launch_aggregate(P->m, d, k, q.Yi, 1.0 / (double)P->n, q.Y, s)) != hipSuccess) return e;
  if ((e = launch_cross_gram(1, d, k, q.Z, dk, q.Y, dk, q.gram, s)) != hipSuccess) return e;
  if ((e = launch_sym_eig(P->plan.n_gram_chunks, k, q.gram, ritz_out, q.omat, s)) != hipSuccess)
    return e;
  return launch_right_mult(1, d, k, q.Z, q.omat, 0, false, Z_out, nullptr, 0, s);
}

void cache_store(const std::string& path, const std::string& key, const lp_tuning& t) {
  std::ofstream f(path, std::ios::app);
  if (f) f << key << "=" << t.local_kernel << "," << (long long)t.chunk_rows << "," << t.cached_loads << "\n";
}

}  // namespace

extern "C" {

lp_status lp_autotune(lp_problem* P, int32_t k, const char* cache_path, lp_tuning* chosen) {
  if (P == nullptr) return fail(LP_EINVAL, "problem is NULL");
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  std::string path = cache_path ? cache_path : "";
  if (path.empty()) {
    const char* env = std::getenv("LP_AUTOTUNE_CACHE");
    if (env != nullptr) path = env;
  }
  const std::string key = tune_key(P, k);
  lp_tuning best;
  std::memset(&best, 0, sizeof(best));
  best.struct_size = sizeof(lp_tuning);
  if (!path.empty() && cache_lookup(path, key, P->plan.split_operands ? 1 : 0, &best)) {
    if ((st = lp_set_tuning(P, &best)) != LP_OK) return st;
    if (chosen) *chosen = best;
    return LP_OK;
  }
  const int32_t split = P->plan.split_operands ? 1 : 0;   // kept: a choice of accuracy
  // candidates: the vector-ALU kernel (k <= 8), the fused matrix-core variants when
  // they take this rank, else the two forms of the two-pass kernel; each at three
  // work-item sizes
  const bool valu_k = valu_eligible(P->dtype, P->d, P->lda, k, P->A);
  const LocalPath fk = fused_kind(P);
  const bool mfma_k =
      (fk == LocalPath::Mfma32 && mfma32_eligible(P->dtype, P->d, P->lda, k)) ||
      (fk == LocalPath::MfmaBf16 && mfma16_eligible(P->dtype, P->d, P->lda, k, P->A, split != 0));
  const int lk_max = fk == LocalPath::Mfma32 ? 10 : 5;
  std::vector<lp_tuning> cand;
  const int64_t c0 = P->plan.min_chunk_rows;
  for (int64_t cr : {c0, 2 * c0, 4 * c0}) {
    if (valu_k) cand.push_back({(int32_t)sizeof(lp_tuning), 0, cr, 0, split});
    if (mfma_k) {
      for (int lk = 2; lk <= lk_max; ++lk)
        for (int cached = 0; cached <= 1; ++cached) cand.push_back({(int32_t)sizeof(lp_tuning), lk, cr, cached, split});
    } else {
      for (int lk : {1, 11}) cand.push_back({(int32_t)sizeof(lp_tuning), lk, cr, 0, split});
    }
  }
  if ((st = join_in(P)) != LP_OK) return st;
  Ptrs q = ptrs(P);
  LP_HIP(launch_fill_i32((int32_t*)q.Zw_shared, (int)(P->d * k * P->plan.zw_bytes / 4), 0, P->stream));
  hipEvent_t e0, e1;
  LP_HIP(hipEventCreate(&e0));
  LP_HIP(hipEventCreate(&e1));
  // average time of `reps` launches of candidate c after two untimed ones
  auto time_candidate = [&](const lp_tuning& c, int reps, double* ms_out) -> lp_status {
    lp_status cs = lp_set_tuning(P, &c);
    if (cs != LP_OK) return cs;
    hipError_t e = hipSuccess;
    for (int it = 0; it < 2 && e == hipSuccess; ++it)
      e = launch_local_multiply(P->plan, P->A, P->lda, k, q.Zw_shared, 0, q.tbuf, q.part, q.items,
                                (int)P->plan.items.size(), P->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, P->stream);
    for (int it = 0; it < reps && e == hipSuccess; ++it)
      e = launch_local_multiply(P->plan, P->A, P->lda, k, q.Zw_shared, 0, q.tbuf, q.part, q.items,
                                (int)P->plan.items.size(), P->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, P->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return fail(LP_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    *ms_out = ms / reps;
    return LP_OK;
  };
  // bring the clocks up before anything is compared
  double ms = 0.0;
  st = time_candidate(cand[0], 24, &ms);
  // first pass over every candidate, then the three fastest again
  std::vector<std::pair<double, size_t>> order;
  for (size_t ci = 0; ci < cand.size() && st == LP_OK; ++ci) {
    st = time_candidate(cand[ci], 6, &ms);
    order.emplace_back(ms, ci);
  }
  double best_ms = 1e300;
  if (st == LP_OK) {
    std::sort(order.begin(), order.end());
    for (size_t r = 0; r < std::min<size_t>(3, order.size()) && st == LP_OK; ++r) {
      st = time_candidate(cand[order[r].second], 12, &ms);
      if (st == LP_OK && ms < best_ms) {
        best_ms = ms;
        best = cand[order[r].second];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LP_OK) return st;
  if ((st = lp_set_tuning(P, &best)) != LP_OK) return st;
  if (!path.empty()) cache_store(path, key, best);
  if (chosen) *chosen = best;
  return join_out(P);
}

lp_status lp_run(lp_problem* P, int32_t k, const int32_t* p_sched, int32_t T, lp_agg mode,
                 const double* Y0, double* Z_out, double* ritz_out, const lp_run_opts* opts,
                 lp_run_stats* stats) {
  if (P == nullptr) return fail(LP_EINVAL, "problem is NULL");
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  if (T < 1 || p_sched == nullptr) return fail(LP_EINVAL, "need T >= 1 and a schedule");
  for (int r = 0; r < T; ++r)
    if (p_sched[r] < 1) return fail(LP_EINVAL, "every p_sched[r] must be >= 1");
  if (mode != LP_AGG_VANILLA && mode != LP_AGG_SIGN && mode != LP_AGG_OPT)
    return fail(LP_EINVAL, "unknown aggregation mode");
  if (Z_out == nullptr) return fail(LP_EINVAL, "Z_out is required");
  lp_run_opts o;
  std::memset(&o, 0, sizeof(o));
  o.use_graph = 1;
  if (opts != nullptr) {
    const size_t n = std::min<size_t>(sizeof(o), (size_t)std::max(opts->struct_size, 0));
    std::memcpy(&o, opts, n);
    if (n < offsetof(lp_run_opts, use_graph) + sizeof(int32_t)) o.use_graph = 1;
  }
  const bool hist = o.U_ref != nullptr && o.sin_hist != nullptr;
  if (o.k_ref < 0 || o.k_ref > k) return fail(LP_EINVAL, "k_ref must be 0 or in [1, k]");
  const int k_ref = o.k_ref > 0 ? o.k_ref : k;
  const int hist_k = hist ? k_ref : 0;
  if (o.time_local < 0 || o.time_local > 2) return fail(LP_EINVAL, "time_local must be 0, 1 or 2");
  if (o.split_rounds < 0 || o.split_rounds > 2) return fail(LP_EINVAL, "split_rounds must be 0, 1 or 2");
  bool split;
  {
    const bool fused =
        (P->plan.valu && valu_eligible(P->dtype, P->d, P->lda, k, P->A)) ||
        (P->plan.path == LocalPath::Mfma32 && mfma32_eligible(P->dtype, P->d, P->lda, k)) ||
        (P->plan.path == LocalPath::MfmaBf16 &&
         mfma16_eligible(P->dtype, P->d, P->lda, k, P->A, P->plan.split_operands));
    split = P->can_split && !P->gram_on && o.rho_out == nullptr &&
            (o.split_rounds == 1 || (o.split_rounds == 0 && !fused));
  }
  if (split && P->stream2 == nullptr) {
    // the second stream and its events exist only in problems that run split
    // rounds (an idle stream still takes a hardware queue slot from the others)
    hipError_t e = hipStreamCreateWithFlags(&P->stream2, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&P->ev_fork, &P->ev_join2, &P->ev_base, &P->ev_k1[0], &P->ev_k1[1]})
      if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(LP_EDEVICE, std::string("second stream/events: ") + hipGetErrorString(e));
  }
  const bool timing = o.time_local != 0;
  P->timing_first_only = o.time_local == 2;
  const bool graph = o.use_graph != 0;
  if (timing && P->ev_pool.empty()) {
    P->ev_pool.assign(2 * kEvPairs, nullptr);
    for (auto& ev : P->ev_pool) LP_HIP(hipEventCreate(&ev));
  }
  P->ev_used = 0;
  P->ms_local = 0.0;
  P->local_launches = 0;
  Ptrs q = ptrs(P);
  const int m = P->m;
  const int64_t d = P->d;
  const int64_t dk = d * k;
  hipStream_t s = P->stream;
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(launch_fill_i32(q.flags, m + 2, 0, s));
  LP_HIP(launch_fill_i32(q.ctr, 1, 0, s));
  LP_HIP(launch_fill_i32(q.rho_ctr, 1, 0, s));
  if (hist) LP_HIP(hipMemcpyAsync(q.Uref, o.U_ref, (size_t)d * k_ref * 8, hipMemcpyDeviceToDevice, s));
  // Z_0 = orth(Y_0) (Algorithm 1, initialisation); without Y0 the Gaussian
  // start is drawn from the seed into the (still unused) local-product buffer
  if (Y0 == nullptr) {
    if (o.z0_orthonormal) return fail(LP_EINVAL, "z0_orthonormal needs a Y0");
    LP_HIP(launch_gaussian(dk, o.seed, q.Yi, s));
    Y0 = q.Yi;
  }
  if (o.z0_orthonormal) {
    LP_HIP(hipMemcpyAsync(q.Z, Y0, dk * 8, hipMemcpyDeviceToDevice, s));
    LP_HIP(launch_to_working(P->plan, 1, d, k, q.Z, q.Zw_shared, s));
  } else {
    LP_HIP(cholqr2(P->plan, P->ws, 1, d, k, Y0, q.Z, q.Zw_shared, q.flags + m, s));
  }
  LP_HIP(hipEventRecord(P->ev_t0, s));
  int rounds = 0, iters = 0, hist_done = 0, rho_done = 0, graph_rounds = 0;
  P->timing = timing;
  P->split_now = split;
  P->rho_now = o.rho_out != nullptr;
  std::vector<std::pair<int, int>> pending;  // (slot, p) of timed graph rounds not yet harvested
  for (int r = 0; r < T; ++r) {
    const int p = p_sched[r];
    const bool timed_graph = timing && graph && P->timed_graphs_ok && p <= kPairsPerSlot;
    // the two timing forms share the event pool: finish one before using the other
    if (timed_graph && P->ev_used > 0) LP_HIP(drain_timing(P));
    if (!timed_graph && timing && !pending.empty()) LP_HIP(harvest_slots(P, pending));
    if (timed_graph) {
      const int slot = (int)pending.size();
      st = run_round(P, k, p, mode, hist_k, true, slot);
      if (st != LP_OK) {
        // the runtime refused the captured event records: time with plain launches
        // (the refusal stays readable through lp_last_error)
        P->timed_graphs_ok = false;
        LP_HIP(harvest_slots(P, pending));
        st = run_round(P, k, p, mode, hist_k, false, -1);
      } else {
        pending.emplace_back(slot, P->timing_first_only ? 1 : p);
        graph_rounds++;
      }
    } else {
      st = run_round(P, k, p, mode, hist_k, graph && !timing, -1);
      if (graph && !timing) graph_rounds++;
    }
    if (st != LP_OK) {
      P->timing = false;
      P->split_now = false;
      P->rho_now = false;
      return st;
    }
    if ((int)pending.size() == kTimedSlots || (r == T - 1 && !pending.empty()))
      LP_HIP(harvest_slots(P, pending));
    rounds++;
    iters += p;
    if (o.signs_out != nullptr) {
      int8_t* dst = o.signs_out + (size_t)r * m * k;
      if (p >= 2 && mode == LP_AGG_SIGN) {
        LP_HIP(hipMemcpyAsync(dst, q.sgn, (size_t)m * k, hipMemcpyDeviceToHost, s));
        LP_HIP(hipStreamSynchronize(s));
      } else {
        std::memset(dst, 0, (size_t)m * k);
      }
    }
    if (hist && (rounds - hist_done == kHistCap || r == T - 1)) {
      LP_HIP(hipMemcpyAsync(o.sin_hist + hist_done, q.hist, (size_t)(rounds - hist_done) * 8,
                            hipMemcpyDeviceToHost, s));
      LP_HIP(launch_fill_i32(q.ctr, 1, 0, s));
      LP_HIP(hipStreamSynchronize(s));
      hist_done = rounds;
    }
    if (P->rho_now && (rounds - rho_done == kHistCap || r == T - 1)) {
      LP_HIP(hipMemcpyAsync(o.rho_out + rho_done, q.rho, (size_t)(rounds - rho_done) * 8,
                            hipMemcpyDeviceToHost, s));
      LP_HIP(launch_fill_i32(q.rho_ctr, 1, 0, s));
      LP_HIP(hipStreamSynchronize(s));
      rho_done = rounds;
    }
  }
  P->split_now = false;
  P->rho_now = false;
  LP_HIP(hipEventRecord(P->ev_t1, s));
  if (timing) LP_HIP(drain_timing(P));
  P->timing = false;
  LP_HIP(finish_z(P, k, Z_out, ritz_out));
  std::vector<int32_t> flags(m + 2, 0);
  LP_HIP(hipMemcpyAsync(flags.data(), q.flags, (m + 2) * 4, hipMemcpyDeviceToHost, s));
  LP_HIP(hipStreamSynchronize(s));
  if ((st = join_out(P)) != LP_OK) return st;
  int breakdowns = 0;
  for (int i = 0; i < m + 1; ++i) breakdowns += flags[i];
  if (stats != nullptr) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, P->ev_t0, P->ev_t1);
    stats->rounds = rounds;
    stats->local_iters = iters;
    stats->breakdowns = breakdowns;
    stats->near_singular = flags[m + 1];
    stats->ms_total = ms;
    stats->bytes_A = (double)iters * (double)P->n * (double)P->d * (double)elem_bytes(P->dtype);
    stats->ms_local = P->ms_local;
    stats->local_launches = P->local_launches;
    stats->graph_rounds = graph_rounds;
    stats->split_rounds = split ? 1 : 0;
  }
  if (breakdowns) return fail(LP_EBREAKDOWN, "Cholesky breakdown in an orthonormalisation");
  return LP_OK;
}

lp_status lp_solve(lp_problem* P, int32_t k, lp_agg mode, const double* Y0, double* Z_out,
                   double* ritz_out, const lp_solve_opts* opts, lp_solve_stats* stats) {
  if (P == nullptr || Z_out == nullptr || opts == nullptr)
    return fail(LP_EINVAL, "problem, Z_out and opts are required");
  // callers built before the seed field existed pass the shorter struct
  if (opts->struct_size < (int32_t)offsetof(lp_solve_opts, seed))
    return fail(LP_EINVAL, "opts->struct_size too small");
  lp_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  std::memcpy(&o, opts, std::min<size_t>(sizeof(o), (size_t)opts->struct_size));
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  if (mode != LP_AGG_VANILLA && mode != LP_AGG_SIGN && mode != LP_AGG_OPT)
    return fail(LP_EINVAL, "unknown aggregation mode");
  if (o.p0 < 1 || !(o.target > 0.0) || o.max_rounds < 1)
    return fail(LP_EINVAL, "need p0 >= 1, target > 0 and max_rounds >= 1");
  if (P->change_host == nullptr) LP_HIP(hipHostMalloc((void**)&P->change_host, sizeof(double)));
  Ptrs q = ptrs(P);
  const int m = P->m;
  const int64_t dk = P->d * k;
  hipStream_t s = P->stream;
  if (Y0 == nullptr) {
    if (o.z0_orthonormal) return fail(LP_EINVAL, "z0_orthonormal needs a Y0");
    if ((st = join_in(P)) != LP_OK) return st;
    LP_HIP(launch_gaussian(dk, o.seed, q.Yi, s));
    Y0 = q.Yi;
  }
  if ((st = drive_begin(P, k, Y0, o.z0_orthonormal != 0)) != LP_OK) return st;
  // the previous iterate lives in the reference buffer (no reference here); the
  // change of a round goes to the first history cell
  LP_HIP(hipMemcpyAsync(q.Uref, q.Z, dk * 8, hipMemcpyDeviceToDevice, s));
  LP_HIP(hipEventRecord(P->ev_t0, s));
  StopRule rule;
  rule.p = o.p0;
  rule.target = o.target;
  int rounds = 0, iters = 0;
  bool settled = false, finite = true;
  P->split_now = false;
  while (rounds < o.max_rounds && !settled) {
    const int p = rule.p;
    if ((st = run_round(P, k, p, mode, 0, true, -1)) != LP_OK) return st;
    LP_HIP(launch_sin_theta_chunked(P->d, k, k, q.Z, q.Uref, q.sinw, q.hist, nullptr, nullptr, s));
    LP_HIP(hipMemcpyAsync(q.Uref, q.Z, dk * 8, hipMemcpyDeviceToDevice, s));
    LP_HIP(hipMemcpyAsync(P->change_host, q.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    LP_HIP(hipStreamSynchronize(s));
    const double c = *P->change_host;
    if (o.p_used != nullptr) o.p_used[rounds] = p;
    if (o.change_out != nullptr) o.change_out[rounds] = c;
    rounds++;
    iters += p;
    if (!std::isfinite(c)) {  // a breakdown left no valid iterate
      finite = false;
      break;
    }
    settled = rule.step(c);
  }
  LP_HIP(hipEventRecord(P->ev_t1, s));
  LP_HIP(finish_z(P, k, Z_out, ritz_out));
  std::vector<int32_t> flags(m + 2, 0);
  LP_HIP(hipMemcpyAsync(flags.data(), q.flags, (m + 2) * 4, hipMemcpyDeviceToHost, s));
  LP_HIP(hipStreamSynchronize(s));
  if ((st = join_out(P)) != LP_OK) return st;
  int breakdowns = 0;
  for (int i = 0; i < m + 1; ++i) breakdowns += flags[i];
  if (stats != nullptr) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, P->ev_t0, P->ev_t1);
    stats->rounds = rounds;
    stats->local_iters = iters;
    stats->breakdowns = breakdowns;
    stats->near_singular = flags[m + 1];
    stats->p_final = rule.p_run;
    stats->change = rule.change;
    stats->estimate = rule.estimate;
    stats->ms_total = ms;
  }
  if (breakdowns) return fail(LP_EBREAKDOWN, "Cholesky breakdown in an orthonormalisation");
  if (!finite) return fail(LP_ENOTCONV, "the change between rounds is not finite");
  if (!settled) return fail(LP_ENOTCONV, "not settled at p = 1 within max_rounds");
  return LP_OK;
}

lp_status lp_gram_bytes(const lp_problem* P, size_t* bytes) {
  if (P == nullptr || bytes == nullptr) return fail(LP_EINVAL, "NULL argument");
  const size_t d = (size_t)P->d, m = (size_t)P->m;
  *bytes = align256(m * d * d * 4) + align256(m * sizeof(WorkItem)) + align256(2 * (m + 1) * 4) +
           align256(eta_scratch_bytes(P->d, P->m));
  return LP_OK;
}

lp_status lp_gram_enable(lp_problem* P, void* buffer, size_t bytes) {
  if (P == nullptr || buffer == nullptr) return fail(LP_EINVAL, "NULL argument");
  if (((uintptr_t)buffer & 255) != 0) return fail(LP_EINVAL, "buffer must be 256-byte aligned");
  size_t need = 0;
  lp_gram_bytes(P, &need);
  if (bytes < need) return fail(LP_EINVAL, "buffer smaller than lp_gram_bytes");
  if (P->dtype != LP_F32 && P->dtype != LP_BF16)
    return fail(LP_EINVAL, "the Gram form takes FP32 or BF16 A");
  if (P->d % 4 != 0) return fail(LP_EINVAL, "the Gram form needs d % 4 == 0");
  if ((int64_t)P->m * P->d > P->n)
    return fail(LP_EINVAL, "the Gram form needs m d <= n (it would move more bytes than A)");
  const int64_t d = P->d;
  const int m = P->m;
  char* b = (char*)buffer;
  float* M = (float*)b;
  WorkItem* items = (WorkItem*)(b + align256((size_t)m * d * d * 4));
  int32_t* slot_off = (int32_t*)((char*)items + align256((size_t)m * sizeof(WorkItem)));
  char* eta = (char*)slot_off + align256(2 * (size_t)(m + 1) * 4);
  lp_status st;
  if ((st = join_in(P)) != LP_OK) return st;
  // M_i = A_i^T A_i on the FP32 matrix cores: the work list first holds the
  // partitions' row ranges for the Gram products, then the multiply's items
  std::vector<WorkItem> parts(m);
  for (int i = 0; i < m; ++i)
    parts[i] = WorkItem{i, i, P->offsets[i], P->offsets[i + 1] - P->offsets[i]};
  LP_HIP(hipMemcpyAsync(items, parts.data(), m * sizeof(WorkItem), hipMemcpyHostToDevice, P->stream));
  LP_HIP(launch_gram_products(P->plan, P->A, P->lda, items, m, M, P->stream));
  std::vector<WorkItem> hi(m);
  std::vector<int32_t> ho(2 * (m + 1));
  for (int i = 0; i < m; ++i) hi[i] = WorkItem{i, i, (int64_t)i * d, d};
  for (int i = 0; i <= m; ++i) {
    ho[i] = i;
    ho[m + 1 + i] = 2 * i;
  }
  LP_HIP(hipMemcpyAsync(items, hi.data(), m * sizeof(WorkItem), hipMemcpyHostToDevice, P->stream));
  LP_HIP(hipMemcpyAsync(slot_off, ho.data(), 2 * (m + 1) * 4, hipMemcpyHostToDevice, P->stream));
  LP_HIP(hipStreamSynchronize(P->stream));
  // captured rounds launch the other form's kernels
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  P->gram_M = M;
  P->gram_items = items;
  P->gram_slot_off = slot_off;
  P->gram_eta = eta;
  P->gram_split2 = 2 * (int64_t)m * d <= P->n;   // the partial buffer holds n x k_max values
  P->gram_on = true;
  return join_out(P);
}

lp_status lp_gram_disable(lp_problem* P) {
  if (P == nullptr) return fail(LP_EINVAL, "NULL argument");
  if (!P->gram_on) return LP_OK;
  LP_HIP(hipStreamSynchronize(P->stream));
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  P->gram_on = false;
  P->gram_M = nullptr;
  P->gram_items = nullptr;
  P->gram_slot_off = nullptr;
  P->gram_eta = nullptr;
  return LP_OK;
}

lp_status lp_eta(lp_problem* P, int32_t iters, double* eta_out, double* per_part_out) {
  if (P == nullptr || eta_out == nullptr) return fail(LP_EINVAL, "NULL argument");
  if (!P->gram_on) return fail(LP_EINVAL, "lp_eta needs the local-Gram form (lp_gram_enable)");
  if (iters < 1) return fail(LP_EINVAL, "need iters >= 1");
  const int m = P->m;
  const int nb = eta_start_vectors();
  std::vector<double> inv_s(m), est((size_t)(m + 1) * nb);
  for (int i = 0; i < m; ++i) inv_s[i] = 1.0 / (double)(P->offsets[i + 1] - P->offsets[i]);
  lp_status st;
  if ((st = join_in(P)) != LP_OK) return st;
  hipError_t e = launch_eta(P->d, m, P->n, P->gram_M, inv_s.data(), iters, P->gram_eta, est.data(),
                            P->stream);
  if (e != hipSuccess) return fail(LP_EDEVICE, std::string("eta: ") + hipGetErrorString(e));
  auto row_max = [&](int b) {
    double v = 0.0;
    for (int j = 0; j < nb; ++j) v = std::max(v, est[(size_t)b * nb + j]);
    return v;
  };
  const double mn = row_max(m);
  double eta = 0.0;
  for (int i = 0; i < m; ++i) {
    const double v = mn > 0.0 ? row_max(i) / mn : 0.0;
    if (per_part_out != nullptr) per_part_out[i] = v;
    eta = std::max(eta, v);
  }
  *eta_out = eta;
  return join_out(P);
}

lp_status lp_local_multiply(lp_problem* P, int32_t k, const double* Z, double* Y_out) {
  if (P == nullptr || Z == nullptr || Y_out == nullptr) return fail(LP_EINVAL, "NULL argument");
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  Ptrs q = ptrs(P);
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(launch_to_working(P->plan, 1, P->d, k, Z, q.Zw_shared, P->stream));
  if (P->gram_on) {
    LP_HIP(launch_gram_multiply(P->plan, P->gram_M, k, q.Zw_shared, 0, q.tbuf, P->gram_items, P->m,
                                gram_split(P, k), P->stream));
    LP_HIP(launch_reduce_partials(P->plan, k, q.tbuf, gram_slots(P, k), Y_out, P->stream));
    return join_out(P);
  }
  LP_HIP(launch_local_multiply(P->plan, P->A, P->lda, k, q.Zw_shared, 0, q.tbuf, q.part, q.items,
                               (int)P->plan.items.size(), P->stream));
  LP_HIP(launch_reduce_partials(P->plan, k, q.part, q.slot_off, Y_out, P->stream));
  return join_out(P);
}

lp_status lp_profile_local_multiply(lp_problem* P, int32_t k, const double* Z, double* wg_out,
                                     int32_t max_wg, int32_t* n_wg) {
  if (P == nullptr || Z == nullptr || n_wg == nullptr || (wg_out == nullptr && max_wg > 0))
    return fail(LP_EINVAL, "NULL argument");
  lp_status st = check_k(P, k);
  if (st != LP_OK) return st;
  if (P->gram_on || fused_for_k(P, k) || !gemm_eligible(P->dtype, P->d, P->lda, P->A))
    return fail(LP_EINVAL, "profiling covers the two-pass local multiply only");
  const int64_t nitems = (int64_t)P->plan.items.size();
  int64_t rw1 = 0, cw2 = 0;
  two_pass_geometry(P->plan, &rw1, &cw2);
  const int64_t g1 = nitems * ((P->plan.chunk_rows + rw1 - 1) / rw1);
  const int64_t g2 = nitems * ((P->d + cw2 - 1) / cw2);
  *n_wg = (int32_t)(g1 + g2);
  if (g1 + g2 > P->plan.stamp_cap)
    return fail(LP_EINVAL, "profile at the default work-item size (the stamp area is sized for it)");
  if (max_wg < g1 + g2) return fail(LP_EINVAL, "wg_out holds fewer rows than *n_wg");
  Ptrs q = ptrs(P);
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(launch_to_working(P->plan, 1, P->d, k, Z, q.Zw_shared, P->stream));
  P->plan.stamps = (unsigned long long*)(P->ws + P->plan.L.stamps);
  hipError_t e = launch_local_multiply(P->plan, P->A, P->lda, k, q.Zw_shared, 0, q.tbuf, q.part,
                                       q.items, (int)nitems, P->stream);
  P->plan.stamps = nullptr;
  if (e != hipSuccess) return fail(LP_EDEVICE, std::string("profiled launch: ") + hipGetErrorString(e));
  std::vector<unsigned long long> h((size_t)2 * (g1 + g2));
  LP_HIP(hipMemcpyAsync(h.data(), P->ws + P->plan.L.stamps, h.size() * 8, hipMemcpyDeviceToHost,
                        P->stream));
  LP_HIP(hipStreamSynchronize(P->stream));
  int khz = 0;
  LP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, P->device));
  if (khz <= 0) return fail(LP_EDEVICE, "wall clock rate unavailable");
  unsigned long long t0 = h[0];
  for (size_t j = 0; j < h.size(); j += 2) t0 = std::min(t0, h[j]);
  const double us_per_tick = 1e3 / (double)khz;
  for (int64_t wg = 0; wg < g1 + g2; ++wg) {
    const bool second = wg >= g1;
    const int64_t local = second ? wg - g1 : wg;
    double* o = wg_out + 4 * wg;
    o[0] = second ? 2.0 : 1.0;
    o[1] = (double)(local % nitems);
    o[2] = (double)(h[2 * wg] - t0) * us_per_tick;
    o[3] = (double)(h[2 * wg + 1] - t0) * us_per_tick;
  }
  return join_out(P);
}

lp_status lp_orth(lp_problem* P, int32_t k, int32_t batch, const double* Y, double* Q,
                  int32_t* flags) {
  if (P == nullptr || Y == nullptr || Q == nullptr) return fail(LP_EINVAL, "NULL argument");
  if (k < 1 || k > P->k_max) return fail(LP_EINVAL, "need 1 <= k <= k_max");
  if (batch < 1 || batch > std::max(P->m, 1)) return fail(LP_EINVAL, "need 1 <= batch <= m");
  lp_status st;
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(cholqr2(P->plan, P->ws, batch, P->d, k, Y, Q, nullptr, flags, P->stream));
  return join_out(P);
}

lp_status lp_align(lp_problem* P, int32_t k, int32_t batch, lp_agg mode, const double* Zi,
                   const double* Zb, void* out) {
  if (P == nullptr || Zi == nullptr || Zb == nullptr || out == nullptr)
    return fail(LP_EINVAL, "NULL argument");
  if (k < 1 || k > P->k_max) return fail(LP_EINVAL, "need 1 <= k <= k_max");
  if (batch < 1 || batch > std::max(P->m, 1)) return fail(LP_EINVAL, "need 1 <= batch <= m");
  if (mode != LP_AGG_SIGN && mode != LP_AGG_OPT) return fail(LP_EINVAL, "mode must be SIGN or OPT");
  Ptrs q = ptrs(P);
  const int64_t dk = P->d * k;
  lp_status st;
  if ((st = join_in(P)) != LP_OK) return st;
  LP_HIP(launch_cross_gram(batch, P->d, k, Zi, dk, Zb, 0, q.gram, P->stream));
  if (mode == LP_AGG_SIGN)
    LP_HIP(launch_sign_from_gram(batch, P->plan.n_gram_chunks, k, q.gram, (int8_t*)out, P->stream));
  else
    LP_HIP(launch_procrustes(batch, P->plan.n_gram_chunks, k, q.gram, (double*)out, nullptr,
                             P->stream));
  return join_out(P);
}

lp_status lp_bandwidth_probe(const void* buf, size_t bytes, int32_t iters, double* gbs_out,
                             void* stream) {
  if (buf == nullptr || gbs_out == nullptr || bytes < 16 || (bytes % 16) != 0 || iters < 1 ||
      ((uintptr_t)buf & 15) != 0)
    return fail(LP_EINVAL, "need a 16-byte aligned buffer, bytes a multiple of 16, iters >= 1");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  LP_HIP(hipEventCreate(&e0));
  LP_HIP(hipEventCreate(&e1));
  double best = 0.0;
  hipError_t err = hipSuccess;
  for (int it = 0; it < iters && err == hipSuccess; ++it) {
    err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = launch_stream_read(buf, bytes, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms > 0.f) best = std::max(best, (double)bytes / (ms * 1e-3) / 1e9);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(LP_EDEVICE, std::string("bandwidth probe: ") + hipGetErrorString(err));
  *gbs_out = best;
  return LP_OK;
}

lp_status lp_copy_probe(void* dst, const void* src, size_t bytes, int32_t iters, double* gbs_out,
                        void* stream) {
  if (dst == nullptr || src == nullptr || gbs_out == nullptr || bytes < 16 || (bytes % 16) != 0 ||
      iters < 1 || ((uintptr_t)dst & 15) != 0 || ((uintptr_t)src & 15) != 0)
    return fail(LP_EINVAL, "need 16-byte aligned buffers, bytes a multiple of 16, iters >= 1");
  const char* d0 = (const char*)dst;
  const char* s0 = (const char*)src;
  if (d0 < s0 + bytes && s0 < d0 + bytes) return fail(LP_EINVAL, "src and dst overlap");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  LP_HIP(hipEventCreate(&e0));
  LP_HIP(hipEventCreate(&e1));
  double best = 0.0;
  hipError_t err = hipSuccess;
  for (int it = 0; it < iters && err == hipSuccess; ++it) {
    err = hipEventRecord(e0, s);
    if (err == hipSuccess) err = launch_stream_copy(dst, src, bytes, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms > 0.f) best = std::max(best, 2.0 * (double)bytes / (ms * 1e-3) / 1e9);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(LP_EDEVICE, std::string("copy probe: ") + hipGetErrorString(err));
  *gbs_out = best;
  return LP_OK;
}

lp_status lp_generate(void* A, lp_dtype dtype, int64_t n, int64_t d, int64_t lda, int32_t k,
                      double gap, double decay, uint64_t seed, double* U_out, void* stream) {
  if (A == nullptr && U_out == nullptr) return fail(LP_EINVAL, "nothing to write (A and U_out NULL)");
  if (!truth_shape_ok(n, d))
    return fail(LP_EINVAL, "need d a power of two in [16, 8192] and n a positive multiple of d");
  if (k < 1 || k > d) return fail(LP_EINVAL, "need 1 <= k <= d");
  if (!(gap >= 1.0) || !(decay > 0.0 && decay <= 1.0))
    return fail(LP_EINVAL, "need gap >= 1 and 0 < decay <= 1");
  hipStream_t s = (hipStream_t)stream;
  if (A != nullptr) {
    if (dtype != LP_F32 && dtype != LP_BF16) return fail(LP_EINVAL, "A must be FP32 or BF16");
    const uintptr_t align = dtype == LP_F32 ? 16 : 8;
    if (lda < d || lda % 4 != 0 || ((uintptr_t)A % align) != 0)
      return fail(LP_EINVAL, "need lda >= d, lda % 4 == 0 and A aligned to 4 elements");
    LP_HIP(launch_truth_matrix(A, dtype, n, d, lda, k, gap, decay, seed, s));
  }
  if (U_out != nullptr) LP_HIP(launch_truth_basis(d, k, seed, U_out, s));
  return LP_OK;
}

lp_status lp_sin_theta(const double* Z, const double* U, int64_t d, int32_t k, double* out_host,
                       void* stream) {
  return lp_sin_theta_r(Z, k, U, k, d, out_host, stream);
}

lp_status lp_sin_theta_r(const double* Z, int32_t r, const double* U, int32_t k, int64_t d,
                         double* out_host, void* stream) {
  if (Z == nullptr || U == nullptr || out_host == nullptr) return fail(LP_EINVAL, "NULL argument");
  if (d < 1 || k < 1 || r < k || r > kMaxK || r > d)
    return fail(LP_EINVAL, "need 1 <= k <= r <= min(d, 64)");
  hipStream_t s = (hipStream_t)stream;
  double* cells = nullptr;
  LP_HIP(sin_slot_address(&cells));
  const int cell = take_sin_cell();
  if (cell < 0) return fail(LP_EBUSY, "more than 64 sin theta calls in flight");
  hipError_t e = launch_sin_theta(d, r, k, Z, U, cells + cell, nullptr, nullptr, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, cells + cell, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  give_sin_cell(cell);
  if (e != hipSuccess) return fail(LP_EDEVICE, std::string("sin theta: ") + hipGetErrorString(e));
  return LP_OK;
}

}  // extern "C"
