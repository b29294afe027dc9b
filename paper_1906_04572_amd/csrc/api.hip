// C ABI of libcorutv: contexts, workspace planning, the CoR-UTV pipeline
// (Sec. 3.1, Algorithm 1), the single-step entry points and the serving
// scheduler.  Every arithmetic step runs in the HIP kernels of this library;
// the host only validates, plans buffers and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <thread>
#include <vector>

#include "arena.hpp"
#include "internal.hpp"

using namespace corutv;

// ---------------------------------------------------------------------------
// workspace plan of one decomposition
namespace {

constexpr int kMaxQr = 64;  // status words (one per tall-skinny QR)
// Reduced-precision forms store every basis in FP32, so a CholeskyQR step
// whose orthogonality loss bound u l (||R||_F ||R^-1||_F)^2 is below the FP32
// unit roundoff needs no second step.
constexpr double kOneStepThr = 5.9604644775390625e-08;  // 2^-24
// Sketches with at most this many columns take the three-launch CholeskyQR2.
constexpr int kQr16Max = 16;

struct Plan {
  int64_t mm = 0, nn = 0;  // oriented problem: mm >= nn rows of Q1 / Q2
  int ell = 0, ellp = 0;
  int prec = 0;
  int64_t ldm = 0, ldn = 0, ldx = 0;
  int64_t part_elems = 0;
  int xsplits = 0;
  // byte offsets
  size_t o_wop = 0, o_qop = 0, o_part = 0, o_x0 = 0, o_x1 = 0, o_q1 = 0, o_q2 = 0, o_xp = 0,
         o_g = 0, o_r = 0, o_rinv = 0, o_core = 0, o_qt = 0, o_rt = 0, o_qw = 0, o_tt = 0,
         o_piv = 0, o_st = 0, o_res = 0, o_sum = 0, o_cw = 0, o_sbf = 0, o_stage = 0, o_hh = 0,
         o_q16 = 0;
  // host-resident A: panels of panel_rows storage rows, stage_ld elements each
  int64_t panel_rows = 0, stage_ld = 0;
  size_t stage_bytes = 0;  // one staging panel
  size_t total = 0;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// The partial-tile capacity of a shape takes tens of microseconds of host
// time (geometry scans over every grid size); every blocking call and every
// admitted request needs it, so it is kept per shape.
std::mutex g_cap_mu;
std::map<std::tuple<int64_t, int64_t, int, int>, int64_t> g_cap;

int64_t partials_capacity_cached(int64_t n_out, int64_t k_len, int ellp, int prec) {
  const auto key = std::make_tuple(n_out, k_len, ellp, prec);
  {
    std::lock_guard<std::mutex> lk(g_cap_mu);
    auto it = g_cap.find(key);
    if (it != g_cap.end()) return it->second;
  }
  const int64_t cap = partials_capacity(n_out, k_len, ellp, prec);
  std::lock_guard<std::mutex> lk(g_cap_mu);
  if (g_cap.size() > 4096) g_cap.clear();  // bounded for streams of many shapes
  g_cap[key] = cap;
  return cap;
}

bool make_plan(int64_t m, int64_t n, int k, int p, int q, int prec, Plan* pl) {
  (void)q;
  if (m < 1 || n < 1 || k < 1 || p < 0) return false;
  const int64_t ell = (int64_t)k + p;
  if (ell > std::min(m, n) || ell > 256) return false;
  if (prec < P_F64 || prec > P_BF16X3) return false;
  pl->mm = std::max(m, n);
  pl->nn = std::min(m, n);
  pl->ell = (int)ell;
  pl->ellp = pad_ell((int)ell);
  pl->prec = prec;
  pl->ldm = round_up(pl->mm, 64);
  pl->ldn = round_up(pl->nn, 64);
  pl->ldx = std::max(pl->ldm, pl->ldn);
  const int es = prec == P_F64 ? 8 : 4;  // path element size
  // partial tiles: the larger of the two pass orientations (gemm prec for
  // partial element size: BF16 forms accumulate in FP32 like F32)
  const int gp = prec == P_F64 ? P_F64 : P_F32;
  pl->part_elems = std::max(partials_capacity_cached(pl->mm, pl->nn, pl->ellp, gp),
                            partials_capacity_cached(pl->nn, pl->mm, pl->ellp, gp));
  pl->xsplits = std::max(xty_splits(pl->mm, pl->ell), xty_splits(pl->nn, pl->ell));
  const size_t l2 = (size_t)ell * ell * 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  pl->o_wop = take((size_t)pl->ellp * pl->ldn * es);
  pl->o_qop = take((size_t)pl->ellp * pl->ldm * es);
  pl->o_part = take((size_t)pl->part_elems * (prec == P_F64 ? 8 : 4));
  pl->o_x0 = take((size_t)pl->ellp * pl->ldx * 8);
  pl->o_x1 = take((size_t)pl->ellp * pl->ldx * 8);
  pl->o_q1 = take((size_t)pl->ellp * pl->ldm * 8);
  pl->o_q2 = take((size_t)pl->ellp * pl->ldn * 8);
  pl->o_xp = take((size_t)pl->xsplits * l2);
  pl->o_g = take(l2);
  pl->o_r = take(2 * l2);
  pl->o_rinv = take(l2);
  pl->o_core = take(l2);
  pl->o_qt = take(l2);
  pl->o_rt = take(l2);
  pl->o_qw = take(2 * l2 + 2 * (size_t)ell * 8);
  pl->o_tt = take(l2);
  pl->o_piv = take((size_t)ell * 4);
  pl->o_st = take(kMaxQr * 4);
  pl->o_res = take((size_t)residual_blocks(pl->mm) * 2 * 8);
  pl->o_sum = take(2 * 8);
  pl->o_cw = take(chol_work_bytes((int)ell));
  pl->o_hh = take(std::max(hh_work_bytes(pl->mm, (int)ell), hh_work_bytes(pl->nn, (int)ell)));
  if (prec == P_BF16 || prec == P_BF16X3) pl->o_sbf = take(sketch_bf16_bytes(pl->ellp, pl->ldx));
  if (ell <= kQr16Max) pl->o_q16 = take(qr16_work_bytes());
  pl->total = off;
  return true;
}

constexpr int kDefaultPanelRows = 4096;

// Add two staging panels for a host-resident A (storage rows of srow_len
// elements of es bytes; rows padded to 16 bytes so the passes can use vector
// loads).
bool plan_host_stages(int64_t nrows, int64_t srow_len, int es, int panel_rows, Plan* pl) {
  if (panel_rows < 0 || nrows < 1 || srow_len < 1) return false;
  pl->panel_rows = std::min<int64_t>(panel_rows ? panel_rows : kDefaultPanelRows, nrows);
  pl->stage_ld = round_up(srow_len, 16 / es);
  pl->stage_bytes = align256((size_t)pl->panel_rows * pl->stage_ld * es);
  pl->o_stage = pl->total;
  pl->total += 2 * pl->stage_bytes;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// context
struct Job;

struct corutv_ctx {
  int device = 0;
  int num_cu = 256;
  std::vector<hipStream_t> streams;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::atomic<bool> poisoned{false};
  std::atomic<int> inject_after{0};  // > 0: the n-th next launch check fails (test hook)
  std::mutex run_mu;  // serializes blocking calls on streams[0]
  // serving
  int max_queue = 4096;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> queue;
  std::map<uint64_t, Job*> jobs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread sched;
  bool sched_started = false;
  std::vector<int> slot_busy;
  Arena arena;               // workspace ranges in use (requests and blocking calls)
  int blocking_waiters = 0;  // blocking calls waiting for workspace: admissions pause
  int* host_status = nullptr;                    // pinned, kMaxQr per slot
  // pass timing (blocking decompositions only)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  int64_t t_passes = 0;
  double t_total = 0, t_min = 1e300, t_max = 0;
  // host-resident A: copy stream and its events (created on first use)
  hipStream_t copy_stream = nullptr;
  hipEvent_t stage_ev[5] = {};  // ready[2], free[2], start
  // start / end of a blocking decomposition (created on first use)
  hipEvent_t dec_ev[2] = {};
  // r_j of the last corutv_rpca call (Algorithm 2)
  std::vector<int32_t> rank_hist;
};

namespace {

// A launch check.  corutv_debug_inject_failure makes the n-th next check on a
// context fail as a HIP error would, so the error path can be tested without
// a real device fault.
bool inject_hit(corutv_ctx* c) {
  int v = c->inject_after.load();
  while (v > 0 && !c->inject_after.compare_exchange_weak(v, v - 1)) {
  }
  return v == 1;
}

#define HIPOK(expr)                                                    \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess || inject_hit(ctx)) return CORUTV_E_DEVICE;  \
  } while (0)

bool mat_ok(const corutv_mat* a) {
  if (!a || !a->ptr || a->rows < 1 || a->cols < 1) return false;
  if (a->dtype != CORUTV_F64 && a->dtype != CORUTV_F32) return false;
  if (a->layout == CORUTV_COL_MAJOR) return a->ld >= a->rows;
  if (a->layout == CORUTV_ROW_MAJOR) return a->ld >= a->cols;
  return false;
}

MatOut out_of(const corutv_mat* a) {
  MatOut o;
  o.ptr = a->ptr;
  o.ld = a->ld;
  o.dtype = a->dtype;
  o.layout = a->layout;
  return o;
}

// Arguments of one decomposition, validated.
struct DecArgs {
  corutv_mat A, U, V;
  double* T = nullptr;
  int64_t ldt = 0;
  // optional: T's transpose with the other triangle zeroed, written by the
  // same launch as T (ld ldt2)
  double* T2 = nullptr;
  int64_t ldt2 = 0;
  int32_t* piv = nullptr;
  int k = 0, p = 0, q = 0;
  uint64_t seed = 0;
  uint32_t sub = 0;
  corutv_opts opts{};
};

int validate(const DecArgs& d) {
  if (!mat_ok(&d.A) || !mat_ok(&d.U) || !mat_ok(&d.V) || !d.T) return CORUTV_E_INVAL;
  const int64_t m = d.A.rows, n = d.A.cols;
  const int64_t ell = (int64_t)d.k + d.p;
  if (d.k < 1 || d.p < 0 || d.q < 0 || d.q > 30) return CORUTV_E_INVAL;
  if (ell > std::min(m, n) || ell > 256) return CORUTV_E_INVAL;
  if (d.U.rows != m || d.U.cols != ell || d.V.rows != n || d.V.cols != ell) return CORUTV_E_INVAL;
  if (d.ldt < ell) return CORUTV_E_INVAL;
  const int prec = d.opts.prec;
  if (prec < P_F64 || prec > P_BF16X3) return CORUTV_E_INVAL;
  if (prec == P_F64 && d.A.dtype != CORUTV_F64) return CORUTV_E_INVAL;
  if (prec != P_F64 && d.A.dtype != CORUTV_F32) return CORUTV_E_INVAL;
  if (d.opts.tri < CORUTV_TRI_AUTO || d.opts.tri > CORUTV_TRI_LOWER) return CORUTV_E_INVAL;
  if ((uint32_t)d.opts.flags & ~(uint32_t)(CORUTV_FLAG_CORE_FROM_RZ | CORUTV_FLAG_A_HOST)) return CORUTV_E_INVAL;
  if (d.opts.flags & CORUTV_FLAG_A_HOST) {
    if (prec != P_F64 && prec != P_F32) return CORUTV_E_INVAL;
    if (d.opts.want_err || d.opts.panel_rows < 0) return CORUTV_E_INVAL;
  }
  return CORUTV_OK;
}

struct Enqueued {
  int nqr = 0;
  int* dev_status = nullptr;
  double* dev_sum = nullptr;
  int transposed = 0;
  int tri = CORUTV_TRI_UPPER;
  int passes = 0;
};

// Thin QR of the sketch held in the stream-K partials `pp` (rows x ell):
// CholeskyQR2 with FP64 Gram and Cholesky (sketches of at most 16 columns:
// the one- or three-launch form), Householder after a breakdown.
// Outputs: q64 (FP64, may be scratch) and, for the F32 path, q32.
// one_step: the first Cholesky may decide (status 4) that a second step is
// not needed; then Q = X R1^-1 goes straight to the outputs and the kernels
// of the second step return at once.
hipError_t qr_from_partials(const Plan& pl, char* ws, const Partials& pp, int64_t rows, int64_t ld,
                            double* q64, float* q32, int* st, hipStream_t s, double* rfac = nullptr,
                            bool one_step = false, bool summed = false) {
  const int ell = pl.ell;
  double* x0 = (double*)(ws + pl.o_x0);
  double* x1 = (double*)(ws + pl.o_x1);
  double* xp = (double*)(ws + pl.o_xp);
  double* G = (double*)(ws + pl.o_g);
  double* R = (double*)(ws + pl.o_r);
  double* Ri = (double*)(ws + pl.o_rinv);
  double* cw = (double*)(ws + pl.o_cw);
  const int64_t l2 = (int64_t)ell * ell;
  const int splits = xty_splits(rows, ell);
  hipError_t e;
  // summed: the sketch is already in x0 (passes over a host-resident A)
  if (!summed && (e = launch_sum_partials(pp, ell, pl.ellp, x0, nullptr, ld, s)) != hipSuccess) return e;
  if (ell <= kQr16Max) {
    bool covered = false;
    if ((e = launch_qr16(x0, ld, rows, ell, q64, q32, rfac, st, (double*)(ws + pl.o_q16),
                         one_step ? kOneStepThr : 0.0, s, x1, ld, (double*)(ws + pl.o_hh), &covered)) != hipSuccess)
      return e;
    if (covered) return hipSuccess;
    return launch_householder_qr(x0, ld, rows, ell, x1, ld, q64, ld, q32, ld, rfac, st,
                                 (double*)(ws + pl.o_hh), s);
  }
  if ((e = launch_xty(x0, ld, x0, ld, rows, ell, xp, splits, nullptr, s)) != hipSuccess) return e;
  if ((e = launch_reduce(xp, splits, l2, G, nullptr, s)) != hipSuccess) return e;
  if ((e = launch_chol(G, ell, R, Ri, st, nullptr, cw, s, one_step ? kOneStepThr : 0.0)) != hipSuccess)
    return e;
  MatOut ox1;
  ox1.ptr = x1;
  ox1.ld = ld;
  MatOut o1, o2;
  o1.ptr = q64;
  o1.ld = ld;
  if (q32) {
    o2.ptr = q32;
    o2.ld = ld;
    o2.dtype = CORUTV_F32;
  }
  // X R1^{-1}: the basis itself when one step is enough (status 4), else the
  // input of the second step (status 0); one launch either way
  if (one_step)
    e = launch_rowmat(x0, ld, rows, ell, Ri, ell, nullptr, o1, 1, o2, 1, st, s, true, 4, ox1, 1, 0);
  else
    e = launch_rowmat(x0, ld, rows, ell, Ri, ell, nullptr, ox1, 1, MatOut(), 0, st, s, true);
  if (e != hipSuccess) return e;
  if ((e = launch_xty(x1, ld, x1, ld, rows, ell, xp, splits, st, s)) != hipSuccess) return e;
  if ((e = launch_reduce(xp, splits, l2, G, st, s)) != hipSuccess) return e;
  double* R2 = R + l2;  // the second factor goes beside the first
  if ((e = launch_chol(G, ell, R2, Ri, st, st, cw, s)) != hipSuccess) return e;
  if ((e = launch_rowmat(x1, ld, rows, ell, Ri, ell, nullptr, o1, 1, o2, 1, st, s, true)) != hipSuccess)
    return e;
  // optional R factor: R2 R1 on the Cholesky route, the Householder R after a
  // breakdown (each kernel checks the status word)
  if (rfac && (e = launch_trprod(R2, R, ell, rfac, st, s)) != hipSuccess) return e;
  return launch_householder_qr(x0, ld, rows, ell, x1, ld, q64, ld, q32, ld, rfac, st,
                               (double*)(ws + pl.o_hh), s);
}

// Enqueue a whole decomposition on stream s using the workspace at ws.
int enqueue_decompose(corutv_ctx* ctx, const Plan& pl, char* ws, const DecArgs& d, hipStream_t s,
                      Enqueued* out, std::vector<hipEvent_t>* pass_ev = nullptr) {
  const int64_t m = d.A.rows, n = d.A.cols;
  const int ell = pl.ell, ellp = pl.ellp;
  const int prec = d.opts.prec;
  const bool f64 = prec == P_F64;
  const bool transposed = m < n;
  const int64_t mm = pl.mm, nn = pl.nn;
  // big row-major view of A
  const bool a_col = d.A.layout == CORUTV_COL_MAJOR;
  const int64_t Rb = a_col ? n : m, Cb = a_col ? m : n;
  // problem matrix P = A (or A^T when transposed); P X is trans tA on the big view
  const int tA = (a_col ? 1 : 0) ^ (transposed ? 1 : 0);
  const int tAt = 1 - tA;
  int tri = d.opts.tri;
  if (tri == CORUTV_TRI_AUTO) tri = transposed ? CORUTV_TRI_LOWER : CORUTV_TRI_UPPER;
  // the oriented problem factors P with its own triangle; transposing back flips it
  const bool lower_inner = transposed ? (tri == CORUTV_TRI_UPPER) : (tri == CORUTV_TRI_LOWER);

  void* wop = ws + pl.o_wop;  // nn x ellp, path dtype
  void* qop = ws + pl.o_qop;  // mm x ellp, path dtype
  void* part = ws + pl.o_part;
  double* q1 = (double*)(ws + pl.o_q1);
  double* q2 = (double*)(ws + pl.o_q2);
  double* x0 = (double*)(ws + pl.o_x0);
  double* x1 = (double*)(ws + pl.o_x1);
  double* xp = (double*)(ws + pl.o_xp);
  double* core = (double*)(ws + pl.o_core);
  double* qt = (double*)(ws + pl.o_qt);
  double* rt = (double*)(ws + pl.o_rt);
  double* qw = (double*)(ws + pl.o_qw);
  double* tt = (double*)(ws + pl.o_tt);
  int32_t* piv = (int32_t*)(ws + pl.o_piv);
  int* st = (int*)(ws + pl.o_st);
  const int64_t ldm = pl.ldm, ldn = pl.ldn;
  const int es = f64 ? 8 : 4;

  // status words, and the pass operands, whose padding columns and rows must
  // read as zero (one launch)
  // (every size is a whole number of 16-byte words: ld is a multiple of 64)
  static_assert(kMaxQr * sizeof(int) % 16 == 0, "status words fill 16-byte words");
  ZeroRanges z{};
  auto zero = [&](void* p, size_t bytes) {
    z.ptr[z.count] = p;
    z.words[z.count] = (int64_t)(bytes / 16);
    ++z.count;
  };
  zero(st, kMaxQr * sizeof(int));
  zero(wop, (size_t)ellp * ldn * es);
  if (!f64) zero(qop, (size_t)ellp * ldm * es);
  zero(q1, (size_t)ellp * ldm * 8);
  zero(q2, (size_t)ellp * ldn * 8);
  if (ell <= kQr16Max) zero(ws + pl.o_q16 + qr16_work_bytes() - 256, 256);  // block counter
  HIPOK(launch_zero_ranges(z, s));
  // F64 path: the FP64 bases are the pass operands themselves
  const void* qsrc = f64 ? (const void*)q1 : qop;
  const void* wsrc = f64 ? (const void*)q2 : wop;

  int nqr = 0;
  Partials pp;
  size_t evi = 0;
  auto mark = [&]() {
    if (pass_ev && evi < pass_ev->size()) hipEventRecord((*pass_ev)[evi++], s);
  };
  // Host-resident A: the big row-major view (Rb x Cb, pitch d.A.ld) goes
  // through two staging panels of pl.panel_rows rows.  A pass contracting
  // over Cb (trans 0) yields the rows of each panel's output directly; one
  // contracting over Rb (trans 1) adds the panels' products, in panel order.
  // The result lands summed in x0 (ld ldout); x1 holds a panel's product.
  const bool host_a = (d.opts.flags & CORUTV_FLAG_A_HOST) != 0;
  auto stream_pass = [&](int trans, const void* opnd, int64_t ldo, int64_t ldout) -> hipError_t {
    hipStream_t cs = ctx->copy_stream;
    hipEvent_t* ev = ctx->stage_ev;
    char* stage[2] = {ws + pl.o_stage, ws + pl.o_stage + pl.stage_bytes};
    const int64_t pr = pl.panel_rows, np = (Rb + pr - 1) / pr;
    hipError_t e;
    // the staging panels are free once everything queued so far has run
    if ((e = hipEventRecord(ev[4], s)) != hipSuccess || (e = hipStreamWaitEvent(cs, ev[4], 0)) != hipSuccess)
      return e;
    for (int64_t pi = 0; pi < np; ++pi) {
      const int b = (int)(pi & 1);
      const int64_t r0 = pi * pr, nr = std::min(pr, Rb - r0);
      if (pi >= 2 && (e = hipStreamWaitEvent(cs, ev[2 + b], 0)) != hipSuccess) return e;
      if ((e = hipMemcpy2DAsync(stage[b], (size_t)pl.stage_ld * es, (const char*)d.A.ptr + (size_t)r0 * d.A.ld * es,
                                (size_t)d.A.ld * es, (size_t)Cb * es, (size_t)nr, hipMemcpyHostToDevice, cs)) !=
          hipSuccess)
        return e;
      if ((e = hipEventRecord(ev[b], cs)) != hipSuccess || (e = hipStreamWaitEvent(s, ev[b], 0)) != hipSuccess)
        return e;
      if (trans == 0) {
        if ((e = launch_sketch(prec, 0, stage[b], pl.stage_ld, nr, Cb, opnd, ldo, ellp, part, pl.part_elems, &pp,
                               ctx->num_cu, s, nullptr)) != hipSuccess ||
            (e = launch_sum_partials(pp, ell, ellp, x0 + r0, nullptr, ldout, s)) != hipSuccess)
          return e;
      } else {
        const void* o = (const char*)opnd + (size_t)r0 * es;  // skinny rows r0..
        if ((e = launch_sketch(prec, 1, stage[b], pl.stage_ld, nr, Cb, o, ldo, ellp, part, pl.part_elems, &pp,
                               ctx->num_cu, s, nullptr)) != hipSuccess ||
            (e = launch_sum_partials(pp, ell, ellp, pi == 0 ? x0 : x1, nullptr, ldout, s)) != hipSuccess)
          return e;
        if (pi > 0 && (e = launch_add_cols(x0, x1, Cb, ellp, ldout, s)) != hipSuccess) return e;
      }
      if ((e = hipEventRecord(ev[2 + b], s)) != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // BF16: the sketches of the power loop run in BF16; the passes that give
  // the returned factors directly -- the second sketch Z = P^T Q1 (whose QR
  // is Q2) and the core pass P Q2 -- run in the split form (BF16X3), so the
  // core is accurate to FP32 level and only the captured subspace carries
  // the BF16 rounding of A.
  const int prec_final = prec == P_BF16 ? P_BF16X3 : prec;
  auto passA = [&](const void* opnd, int pr) {  // P X, X nn x ell -> mm x ell
    mark();
    hipError_t e = host_a ? stream_pass(tA, opnd, ldn, ldm)
                          : launch_sketch(pr, tA, d.A.ptr, d.A.ld, Rb, Cb, opnd, ldn, ellp, part,
                                          pl.part_elems, &pp, ctx->num_cu, s, ws + pl.o_sbf, x0, ldm, ell);
    mark();
    return e;
  };
  auto passAt = [&](const void* opnd, int pr) {  // P^T Y, Y mm x ell -> nn x ell
    mark();
    hipError_t e = host_a ? stream_pass(tAt, opnd, ldm, ldn)
                          : launch_sketch(pr, tAt, d.A.ptr, d.A.ld, Rb, Cb, opnd, ldm, ellp, part,
                                          pl.part_elems, &pp, ctx->num_cu, s, ws + pl.o_sbf, x0, ldn, ell);
    mark();
    return e;
  };
  // Omega (nn x ell), then Q1 = qf(P Omega)
  HIPOK(launch_omega(nn, ell, ellp, d.seed, d.sub, f64 ? (double*)wop : nullptr,
                     f64 ? nullptr : (float*)wop, ldn, s));
  HIPOK(passA(wop, prec));
  HIPOK(qr_from_partials(pl, ws, pp, mm, ldm, q1, f64 ? nullptr : (float*)qop, st + nqr++, s, nullptr, !f64,
                         host_a));
  for (int it = 0; it < d.q; ++it) {
    // W = qf(P^T Q1); Q1 = qf(P W)
    HIPOK(passAt(qsrc, prec));
    HIPOK(qr_from_partials(pl, ws, pp, nn, ldn, q2, f64 ? nullptr : (float*)wop, st + nqr++, s, nullptr, !f64,
                           host_a));
    HIPOK(passA(wsrc, prec));
    HIPOK(qr_from_partials(pl, ws, pp, mm, ldm, q1, f64 ? nullptr : (float*)qop, st + nqr++, s, nullptr, !f64,
                         host_a));
  }
  // Z = P^T Q1; Q2, R_Z = qf(Z)
  const bool core_rz = (d.opts.flags & CORUTV_FLAG_CORE_FROM_RZ) != 0;
  HIPOK(passAt(qsrc, prec_final));
  HIPOK(qr_from_partials(pl, ws, pp, nn, ldn, q2, f64 ? nullptr : (float*)wop, st + nqr++, s,
                         core_rz ? core : nullptr, !f64, host_a));
  if (core_rz) {
    // D = Q1^T P Q2 = R_Z^T (Q2 R_Z = Z = P^T Q1): no pass over A; the
    // QRCP of D reads R_Z transposed, the QRCP of D^T reads R_Z as is
    HIPOK(launch_qrcp(core, ell, lower_inner ? 0 : 1, ell, qt, rt, piv, qw, s));
  } else {
    // core D = Q1^T (P Q2)
    HIPOK(passA(wsrc, prec_final));
    if (!host_a) HIPOK(launch_sum_partials(pp, ell, ellp, x0, nullptr, ldm, s));
    const int sp = xty_splits(mm, ell);
    HIPOK(launch_xty(q1, ldm, x0, ldm, mm, ell, xp, sp, nullptr, s));
    HIPOK(launch_reduce(xp, sp, (int64_t)ell * ell, core, nullptr, s));
    // QRCP of D (upper) or of D^T (lower)
    HIPOK(launch_qrcp(core, ell, lower_inner ? 1 : 0, ell, qt, rt, piv, qw, s));
  }
  // lifts in the oriented problem: Uo (mm x ell), Vo (nn x ell), To
  //   upper: Uo = Q1 Qt, To = R, Vo = Q2[:, piv]
  //   lower: Uo = Q1[:, piv], To = R^T, Vo = Q2 Qt
  const corutv_mat* Udst = transposed ? &d.V : &d.U;
  const corutv_mat* Vdst = transposed ? &d.U : &d.V;
  MatOut ou = out_of(Udst), ov = out_of(Vdst);
  MatOut u64, v64;
  const bool want_err = d.opts.want_err != 0;
  if (want_err) {  // FP64 copies for the residual
    u64.ptr = x0;
    u64.ld = ldm;
    v64.ptr = x1;
    v64.ld = ldn;
  }
  if (!lower_inner) {
    HIPOK(launch_rowmat(q1, ldm, mm, ell, qt, ell, nullptr, ou, 0, u64, 0, nullptr, s));
    HIPOK(launch_rowmat(q2, ldn, nn, ell, nullptr, 0, piv, ov, 0, v64, 0, nullptr, s));
  } else {
    HIPOK(launch_rowmat(q1, ldm, mm, ell, nullptr, 0, piv, ou, 0, u64, 0, nullptr, s));
    HIPOK(launch_rowmat(q2, ldn, nn, ell, qt, ell, nullptr, ov, 0, v64, 0, nullptr, s));
  }
  // To (oriented) into tt; user T = To (not transposed) or To^T (transposed)
  const bool t_lower_user = transposed ? !lower_inner : lower_inner;
  {
    double* dst[3] = {tt, d.T, d.T2};
    const int64_t ld[3] = {ell, d.ldt, d.ldt2};
    const int tr[3] = {lower_inner ? 1 : 0, transposed ? 1 : 0, 1};
    const int up[3] = {lower_inner ? 0 : 1, t_lower_user ? 0 : 1, t_lower_user ? 1 : 0};
    HIPOK(launch_copy_tri_chain(rt, ell, d.T2 ? 3 : 2, dst, ld, tr, up, s));
  }
  if (d.piv) HIPOK(hipMemcpyAsync(d.piv, piv, (size_t)ell * 4, hipMemcpyDeviceToDevice, s));
  int passes = 2 * d.q + (core_rz ? 2 : 3);
  double* sum = (double*)(ws + pl.o_sum);
  if (want_err) {
    // residual of P ~ Uo To Vo^T on the big row-major view of A:
    //   tA == 0: big = P, rows mm:  B = Uo To,   V = Vo
    //   tA == 1: big = P^T, rows nn: B = Vo To^T, V = Uo
    double* res = (double*)(ws + pl.o_res);
    double* bm = (double*)(ws + pl.o_q1);  // Q1 no longer needed
    double* tmat = (double*)(ws + pl.o_g);
    MatOut ob;
    ob.ptr = bm;
    if (tA == 0) {
      ob.ld = ldm;
      HIPOK(launch_rowmat(x0, ldm, mm, ell, tt, ell, nullptr, ob, 0, MatOut(), 0, nullptr, s));
      HIPOK(launch_residual(d.A.ptr, d.A.dtype, d.A.ld, Rb, Cb, bm, ldm, x1, ldn, ell, res, s));
    } else {
      ob.ld = ldn;
      HIPOK(launch_copy_tri(tt, ell, 1, lower_inner ? 1 : 0, tmat, ell, s));  // To^T
      HIPOK(launch_rowmat(x1, ldn, nn, ell, tmat, ell, nullptr, ob, 0, MatOut(), 0, nullptr, s));
      HIPOK(launch_residual(d.A.ptr, d.A.dtype, d.A.ld, Rb, Cb, bm, ldn, x0, ldm, ell, res, s));
    }
    HIPOK(launch_reduce(res, residual_blocks(mm), 2, sum, nullptr, s));
    passes += 1;
  }
  out->nqr = nqr;
  out->dev_status = st;
  out->dev_sum = want_err ? sum : nullptr;
  out->transposed = transposed;
  out->tri = t_lower_user ? CORUTV_TRI_LOWER : CORUTV_TRI_UPPER;
  out->passes = passes;
  return CORUTV_OK;
}

int finish_info(const Enqueued& eq, const int* hst, const double* hsum, corutv_info* info) {
  int fallbacks = 0, numeric = 0, single = 0;
  for (int i = 0; i < eq.nqr; ++i) {
    if (hst[i] & 2) numeric = 1;
    if ((hst[i] & 3) == 1) ++fallbacks;
    if ((hst[i] & 7) == 4) ++single;
  }
  if (info) {
    info->ell = 0;
    info->transposed = eq.transposed;
    info->tri = eq.tri;
    info->qr_fallbacks = fallbacks;
    info->qr_one_step = single;
    info->passes = eq.passes;
    info->rel_err = -1.0;
    info->a_fro = -1.0;
    if (hsum) {
      info->a_fro = std::sqrt(hsum[1]);
      info->rel_err = hsum[1] > 0 ? std::sqrt(hsum[0] / hsum[1]) : 0.0;
    }
  }
  if (numeric) return CORUTV_E_NUMERIC;
  if (hsum && !(std::isfinite(hsum[0]) && std::isfinite(hsum[1]))) return CORUTV_E_NUMERIC;
  return CORUTV_OK;
}

int guard(corutv_ctx* ctx) {
  if (!ctx) return CORUTV_E_INVAL;
  if (ctx->poisoned.load()) return CORUTV_E_DEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return CORUTV_E_DEVICE;
  return CORUTV_OK;
}

int poison(corutv_ctx* ctx) {
  ctx->poisoned.store(true);
  return CORUTV_E_DEVICE;
}

// A blocking call's range of the workspace.  It is taken from the same arena
// as the serving requests' ranges (under the context mutex, waiting while
// requests in flight hold the space; the scheduler admits nothing new
// meanwhile), so a blocking call never overlaps a request's scratch, and is
// returned when the call ends.
struct WsLease {
  corutv_ctx* c = nullptr;
  size_t off = 0;
  bool held = false;
  char* base() const { return c->ws + off; }
  ~WsLease() {
    if (!held) return;
    std::lock_guard<std::mutex> lk(c->mu);
    c->arena.release(off);
    c->cv.notify_all();
  }
};

int lease_ws(corutv_ctx* c, size_t bytes, WsLease* l) {
  if (bytes > c->ws_bytes) return CORUTV_E_NOMEM;
  std::unique_lock<std::mutex> lk(c->mu);
  ++c->blocking_waiters;
  bool got = false;
  c->cv.wait(lk, [&] {
    if (c->poisoned.load()) return true;
    got = c->arena.alloc(bytes, &l->off);
    return got;
  });
  --c->blocking_waiters;
  c->cv.notify_all();
  if (!got) return CORUTV_E_DEVICE;
  l->c = c;
  l->held = true;
  return CORUTV_OK;
}

// ---------------------------------------------------------------------------
// Scratch of corutv_decompose_noalloc: a fixed array in the library's own
// device memory, one copy per device (the code object's data), held until
// the process ends.  Host code never passes `scratch` itself to a kernel --
// on the host that name is only a stand-in -- but the device address that
// hipGetSymbolAddress returns for it, looked up once per device at context
// creation with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu[kMaxDevices];  // one call at a time per device
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_init_mu;

// Called by corutv_create with `device` current.
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(g_scratch_init_mu);
  if (g_scratch_ptr[device]) return CORUTV_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CORUTV_E_DEVICE;
  g_scratch_ptr[device] = ptr;
  return CORUTV_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_init_mu);
  return g_scratch_ptr[device];
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char* corutv_strerror(int code) {
  switch (code) {
    case CORUTV_OK: return "ok";
    case CORUTV_PENDING: return "pending";
    case CORUTV_E_INVAL: return "invalid argument";
    case CORUTV_E_NOMEM: return "workspace too small";
    case CORUTV_E_BUSY: return "queue full";
    case CORUTV_E_NUMERIC: return "non-finite input or unrecoverable factorization";
    case CORUTV_E_DEVICE: return "device error (context poisoned)";
    case CORUTV_E_NOTFOUND: return "unknown ticket";
    default: return "unknown status";
  }
}

uint64_t corutv_workspace_bytes(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q, int32_t prec) {
  Plan pl;
  if (!make_plan(m, n, k, p, q, prec, &pl)) return 0;
  return pl.total;
}

uint64_t corutv_workspace_bytes_host(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q, int32_t prec,
                                     int32_t layout, int32_t panel_rows) {
  if (prec != P_F64 && prec != P_F32) return 0;
  if (layout != CORUTV_COL_MAJOR && layout != CORUTV_ROW_MAJOR) return 0;
  Plan pl;
  if (!make_plan(m, n, k, p, q, prec, &pl)) return 0;
  const bool col = layout == CORUTV_COL_MAJOR;
  if (!plan_host_stages(col ? n : m, col ? m : n, prec == P_F64 ? 8 : 4, panel_rows, &pl)) return 0;
  return pl.total;
}

int corutv_create(corutv_ctx** out, const corutv_config* cfg) {
  if (!out || !cfg) return CORUTV_E_INVAL;
  *out = nullptr;
  if (cfg->n_streams < 1 || !cfg->streams) return CORUTV_E_INVAL;
  // a null workspace only with zero bytes (a context for the allocation-free
  // entry point; every other call then reports E_NOMEM)
  if (!cfg->workspace && cfg->workspace_bytes != 0) return CORUTV_E_INVAL;
  if (((uintptr_t)cfg->workspace) % 256 != 0) return CORUTV_E_INVAL;
  corutv_ctx* c = new (std::nothrow) corutv_ctx();
  if (!c) return CORUTV_E_NOMEM;
  c->device = cfg->device;
  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return CORUTV_E_DEVICE;
  }
  if (int rs = scratch_setup(c->device)) {
    delete c;
    return rs;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
      cus > 0)
    c->num_cu = cus;
  for (int i = 0; i < cfg->n_streams; ++i) c->streams.push_back((hipStream_t)cfg->streams[i]);
  c->ws = (char*)cfg->workspace;
  c->ws_bytes = cfg->workspace_bytes;
  c->arena.reset(c->ws_bytes);
  c->max_queue = cfg->max_queue > 0 ? cfg->max_queue : 4096;
  const int slots = std::max(1, cfg->n_streams - 1);
  c->slot_busy.assign(slots, 0);
  if (hipHostMalloc((void**)&c->host_status, sizeof(int) * (kMaxQr + 8) * (slots + 1)) != hipSuccess) {
    delete c;
    return CORUTV_E_DEVICE;
  }
  // start / end events of blocking calls, made here so that the
  // allocation-free entry point creates nothing
  if (hipEventCreate(&c->dec_ev[0]) != hipSuccess || hipEventCreate(&c->dec_ev[1]) != hipSuccess) {
    corutv_destroy(c);
    return CORUTV_E_DEVICE;
  }
  *out = c;
  return CORUTV_OK;
}

int corutv_decompose_noalloc(corutv_ctx* ctx, const corutv_mat* A, int32_t k, int32_t p, int32_t q,
                             uint64_t seed, const corutv_opts* opts, corutv_mat* U, double* T, int64_t ldt,
                             corutv_mat* V, int32_t* piv, corutv_info* info) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!A || !U || !V || !opts) return CORUTV_E_INVAL;
  DecArgs d;
  d.A = *A;
  d.U = *U;
  d.V = *V;
  d.T = T;
  d.ldt = ldt;
  d.piv = piv;
  d.k = k;
  d.p = p;
  d.q = q;
  d.seed = seed;
  d.opts = *opts;
  if ((rc = validate(d)) != CORUTV_OK) return rc;
  if (opts->flags & CORUTV_FLAG_A_HOST) return CORUTV_E_INVAL;  // staging panels are not provided
  Plan pl;
  if (!make_plan(A->rows, A->cols, k, p, q, opts->prec, &pl)) return CORUTV_E_INVAL;
  if (pl.total > kScratchBytes) return CORUTV_E_NOMEM;
  char* ws = (char*)scratch_ptr(ctx->device);
  if (!ws) return CORUTV_E_DEVICE;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  std::lock_guard<std::mutex> lks(g_scratch_mu[ctx->device]);
  hipStream_t s = ctx->streams[0];
  hipEvent_t e0 = ctx->dec_ev[0], e1 = ctx->dec_ev[1];
  HIPOK(hipEventRecord(e0, s));
  Enqueued eq;
  rc = enqueue_decompose(ctx, pl, ws, d, s, &eq);
  if (rc == CORUTV_E_DEVICE) return poison(ctx);
  if (rc != CORUTV_OK) return rc;
  int* hst = ctx->host_status;  // pinned, written back without staging
  double* hsum = (double*)(ctx->host_status + kMaxQr);
  if (hipEventRecord(e1, s) != hipSuccess ||
      hipMemcpyAsync(hst, eq.dev_status, sizeof(int) * eq.nqr, hipMemcpyDeviceToHost, s) != hipSuccess)
    return poison(ctx);
  if (eq.dev_sum && hipMemcpyAsync(hsum, eq.dev_sum, 16, hipMemcpyDeviceToHost, s) != hipSuccess)
    return poison(ctx);
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  rc = finish_info(eq, hst, eq.dev_sum ? hsum : nullptr, info);
  if (info) {
    info->gpu_ms = ms;
    info->ell = pl.ell;
  }
  return rc;
}

int corutv_decompose(corutv_ctx* ctx, const corutv_mat* A, int32_t k, int32_t p, int32_t q,
                     uint64_t seed, const corutv_opts* opts, corutv_mat* U, double* T, int64_t ldt,
                     corutv_mat* V, int32_t* piv, corutv_info* info) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!A || !U || !V || !opts) return CORUTV_E_INVAL;
  DecArgs d;
  d.A = *A;
  d.U = *U;
  d.V = *V;
  d.T = T;
  d.ldt = ldt;
  d.piv = piv;
  d.k = k;
  d.p = p;
  d.q = q;
  d.seed = seed;
  d.opts = *opts;
  if ((rc = validate(d)) != CORUTV_OK) return rc;
  Plan pl;
  if (!make_plan(A->rows, A->cols, k, p, q, opts->prec, &pl)) return CORUTV_E_INVAL;
  const bool host_a = (opts->flags & CORUTV_FLAG_A_HOST) != 0;
  if (host_a) {
    const bool col = A->layout == CORUTV_COL_MAJOR;
    if (!plan_host_stages(col ? A->cols : A->rows, col ? A->rows : A->cols, opts->prec == P_F64 ? 8 : 4,
                          opts->panel_rows, &pl))
      return CORUTV_E_INVAL;
  }
  if (pl.total > ctx->ws_bytes) return CORUTV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  WsLease lease;
  if ((rc = lease_ws(ctx, pl.total, &lease)) != CORUTV_OK) return rc;
  hipStream_t s = ctx->streams[0];
  if (host_a && !ctx->copy_stream) {
    if (hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking) != hipSuccess) return poison(ctx);
    for (hipEvent_t& e : ctx->stage_ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return poison(ctx);
  }
  if (!ctx->dec_ev[0] &&
      (hipEventCreate(&ctx->dec_ev[0]) != hipSuccess || hipEventCreate(&ctx->dec_ev[1]) != hipSuccess))
    return poison(ctx);
  hipEvent_t e0 = ctx->dec_ev[0], e1 = ctx->dec_ev[1];
  hipEventRecord(e0, s);
  Enqueued eq;
  const int npass = 2 * q + ((opts->flags & CORUTV_FLAG_CORE_FROM_RZ) ? 2 : 3);
  if (ctx->timing) {
    while ((int)ctx->ev_pool.size() < 2 * npass) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return poison(ctx);
      ctx->ev_pool.push_back(e);
    }
  }
  std::vector<hipEvent_t> pev;
  if (ctx->timing) pev.assign(ctx->ev_pool.begin(), ctx->ev_pool.begin() + 2 * npass);
  rc = enqueue_decompose(ctx, pl, lease.base(), d, s, &eq, ctx->timing ? &pev : nullptr);
  if (rc == CORUTV_E_DEVICE) return poison(ctx);
  if (rc != CORUTV_OK) return rc;
  hipEventRecord(e1, s);
  int* hst = ctx->host_status;
  double hsum[2] = {0, 0};
  if (hipMemcpyAsync(hst, eq.dev_status, sizeof(int) * eq.nqr, hipMemcpyDeviceToHost, s) != hipSuccess)
    return poison(ctx);
  if (eq.dev_sum && hipMemcpyAsync(hsum, eq.dev_sum, 16, hipMemcpyDeviceToHost, s) != hipSuccess)
    return poison(ctx);
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  if (ctx->timing) {
    for (int i = 0; i < npass; ++i) {
      float pm = 0.f;
      if (hipEventElapsedTime(&pm, pev[2 * i], pev[2 * i + 1]) != hipSuccess) continue;
      ctx->t_passes++;
      ctx->t_total += pm;
      ctx->t_min = std::min(ctx->t_min, (double)pm);
      ctx->t_max = std::max(ctx->t_max, (double)pm);
    }
  }
  rc = finish_info(eq, hst, eq.dev_sum ? hsum : nullptr, info);
  if (info) {
    info->gpu_ms = ms;
    info->ell = pl.ell;
  }
  return rc;
}

int corutv_omega(corutv_ctx* ctx, int64_t n, int32_t ell, uint64_t seed, uint32_t sub, int32_t dtype,
                 void* out, int64_t ld) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (n < 1 || ell < 1 || !out || ld < n || (dtype != CORUTV_F64 && dtype != CORUTV_F32))
    return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  hipStream_t s = ctx->streams[0];
  HIPOK(launch_omega(n, ell, ell, seed, sub, dtype == CORUTV_F64 ? (double*)out : nullptr,
                     dtype == CORUTV_F32 ? (float*)out : nullptr, ld, s));
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  return CORUTV_OK;
}

int corutv_sketch(corutv_ctx* ctx, const corutv_mat* A, int32_t trans, int32_t prec, const void* X,
                  int64_t ldx, int32_t ell, void* Y, int64_t ldy) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!mat_ok(A) || !X || !Y || ell < 1 || ell > 256 || (trans != 0 && trans != 1))
    return CORUTV_E_INVAL;
  if (prec < P_F64 || prec > P_BF16X3) return CORUTV_E_INVAL;
  if ((prec == P_F64) != (A->dtype == CORUTV_F64)) return CORUTV_E_INVAL;
  const int64_t m = A->rows, n = A->cols;
  const int64_t klen = trans ? m : n, nout = trans ? n : m;
  if (ldx < klen || ldy < nout) return CORUTV_E_INVAL;
  const int ellp = pad_ell(ell);
  const int es = prec == P_F64 ? 8 : 4;
  const int64_t ldk = round_up(klen, 64);
  const bool a_col = A->layout == CORUTV_COL_MAJOR;
  const int64_t Rb = a_col ? n : m, Cb = a_col ? m : n;
  const int t = (a_col ? 1 : 0) ^ trans;
  const int64_t cap = partials_capacity_cached(nout, klen, ellp, prec);
  const bool bf = prec == P_BF16 || prec == P_BF16X3;
  const size_t need = align256((size_t)ellp * ldk * es) + align256((size_t)cap * es) +
                      (bf ? align256(sketch_bf16_bytes(ellp, ldk)) : 0);
  if (need > ctx->ws_bytes) return CORUTV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  WsLease lease;
  if ((rc = lease_ws(ctx, need, &lease)) != CORUTV_OK) return rc;
  hipStream_t s = ctx->streams[0];
  char* xs = lease.base();
  char* part = xs + align256((size_t)ellp * ldk * es);
  char* sbf = part + align256((size_t)cap * es);
  HIPOK(hipMemsetAsync(xs, 0, (size_t)ellp * ldk * es, s));
  HIPOK(hipMemcpy2DAsync(xs, ldk * es, X, ldx * es, klen * es, ell, hipMemcpyDeviceToDevice, s));
  Partials pp;
  HIPOK(launch_sketch(prec, t, A->ptr, A->ld, Rb, Cb, xs, ldk, ellp, part, cap, &pp, ctx->num_cu, s,
                      bf ? sbf : nullptr));
  HIPOK(launch_sum_partials(pp, ell, ell, prec == P_F64 ? (double*)Y : nullptr,
                            prec == P_F64 ? nullptr : (float*)Y, ldy, s));
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  return CORUTV_OK;
}

int corutv_tsqr(corutv_ctx* ctx, const double* X, int64_t rows, int32_t ell, int64_t ldx, double* Q,
                int64_t ldq, double* R, int64_t ldr, int32_t* fallback) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!X || !Q || rows < 1 || ell < 1 || ell > 256 || rows < ell || ldx < rows || ldq < rows)
    return CORUTV_E_INVAL;
  if (R && ldr < ell) return CORUTV_E_INVAL;
  const int64_t ld = round_up(rows, 64);
  const int ellp = pad_ell(ell);
  const size_t l2 = (size_t)ell * ell * 8;
  const int splits = xty_splits(rows, ell);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += align256(b);
    return o;
  };
  const size_t o_x0 = take((size_t)ellp * ld * 8), o_x1 = take((size_t)ellp * ld * 8),
               o_q = take((size_t)ellp * ld * 8), o_xp = take(splits * l2), o_g = take(l2),
               o_r1 = take(2 * l2), o_r2 = take(2 * l2), o_ri = take(l2), o_rh = take(l2),
               o_st = take(64), o_cw = take(chol_work_bytes(ell)), o_hh = take(hh_work_bytes(rows, ell));
  if (off > ctx->ws_bytes) return CORUTV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  WsLease lease;
  if ((rc = lease_ws(ctx, off, &lease)) != CORUTV_OK) return rc;
  hipStream_t s = ctx->streams[0];
  char* w = lease.base();
  double *x0 = (double*)(w + o_x0), *x1 = (double*)(w + o_x1), *qq = (double*)(w + o_q),
         *xp = (double*)(w + o_xp), *G = (double*)(w + o_g), *R1 = (double*)(w + o_r1),
         *R2 = (double*)(w + o_r2), *Ri = (double*)(w + o_ri), *Rh = (double*)(w + o_rh);
  int* st = (int*)(w + o_st);
  double* cw = (double*)(w + o_cw);
  HIPOK(launch_fill_int(st, 1, 0, s));
  HIPOK(hipMemcpy2DAsync(x0, ld * 8, X, ldx * 8, rows * 8, ell, hipMemcpyDeviceToDevice, s));
  const int64_t l2e = (int64_t)ell * ell;
  HIPOK(launch_xty(x0, ld, x0, ld, rows, ell, xp, splits, nullptr, s));
  HIPOK(launch_reduce(xp, splits, l2e, G, nullptr, s));
  HIPOK(launch_chol(G, ell, R1, Ri, st, nullptr, cw, s));
  MatOut ox1;
  ox1.ptr = x1;
  ox1.ld = ld;
  HIPOK(launch_rowmat(x0, ld, rows, ell, Ri, ell, nullptr, ox1, 1, MatOut(), 0, st, s, true));
  HIPOK(launch_xty(x1, ld, x1, ld, rows, ell, xp, splits, st, s));
  HIPOK(launch_reduce(xp, splits, l2e, G, st, s));
  HIPOK(launch_chol(G, ell, R2, Ri, st, st, cw, s));
  MatOut oq;
  oq.ptr = qq;
  oq.ld = ld;
  HIPOK(launch_rowmat(x1, ld, rows, ell, Ri, ell, nullptr, oq, 1, MatOut(), 0, st, s, true));
  HIPOK(launch_householder_qr(x0, ld, rows, ell, x1, ld, qq, ld, nullptr, 0, Rh, st, (double*)(w + o_hh), s));
  int hst = 0;
  HIPOK(hipMemcpyAsync(&hst, st, 4, hipMemcpyDeviceToHost, s));
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  if (hst & 2) return CORUTV_E_NUMERIC;
  const bool fb = (hst & 3) == 1;
  if (fallback) *fallback = fb ? 1 : 0;
  HIPOK(hipMemcpy2DAsync(Q, ldq * 8, qq, ld * 8, rows * 8, ell, hipMemcpyDeviceToDevice, s));
  if (R) {
    if (fb) {
      HIPOK(launch_copy_tri(Rh, ell, 0, 1, R, ldr, s));
    } else {
      MatOut orr;  // R = R2 R1
      orr.ptr = R;
      orr.ld = ldr;
      HIPOK(launch_rowmat(R2, ell, ell, ell, R1, ell, nullptr, orr, 0, MatOut(), 0, nullptr, s, true));
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  return CORUTV_OK;
}

int corutv_qrcp(corutv_ctx* ctx, int32_t ell, const double* D, int64_t ldd, double* Qt, double* R,
                int32_t* piv) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (ell < 1 || ell > 256 || !D || !Qt || !R || !piv || ldd < ell) return CORUTV_E_INVAL;
  const size_t need = ((size_t)2 * ell * ell + 2 * ell) * 8;
  if (need > ctx->ws_bytes) return CORUTV_E_NOMEM;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  WsLease lease;
  if ((rc = lease_ws(ctx, need, &lease)) != CORUTV_OK) return rc;
  hipStream_t s = ctx->streams[0];
  HIPOK(launch_qrcp(D, ldd, 0, ell, Qt, R, piv, (double*)lease.base(), s));
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  return CORUTV_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving: host queue + scheduler thread, slots = streams[1..] (or streams[0])
struct Job {
  uint64_t ticket = 0;
  DecArgs d;
  Plan pl;
  enum { QUEUED, RUNNING, DONE } state = QUEUED;
  int rc = CORUTV_PENDING;
  corutv_info info{};
  int slot = -1;
  size_t off = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // recorded on the context stream at submit: the request starts after the
  // work the caller had queued there (its inputs and zero-filled outputs)
  hipEvent_t ready = nullptr;
  Enqueued eq;
  ~Job() {
    if (ready) hipEventDestroy(ready);
  }
};

namespace {

int* slot_status(corutv_ctx* c, int slot) { return c->host_status + (size_t)(slot + 1) * (kMaxQr + 8); }
double* slot_sum(corutv_ctx* c, int slot) { return (double*)(slot_status(c, slot) + kMaxQr); }

hipStream_t slot_stream(corutv_ctx* c, int slot) {
  return c->streams.size() > 1 ? c->streams[1 + slot] : c->streams[0];
}

// Start the job on a free slot if memory allows (called with c->mu held).
bool try_start(corutv_ctx* c, Job* j) {
  int slot = -1;
  for (size_t i = 0; i < c->slot_busy.size(); ++i)
    if (!c->slot_busy[i]) {
      slot = (int)i;
      break;
    }
  if (slot < 0) return false;
  size_t off = 0;
  if (!c->arena.alloc(j->pl.total, &off)) return false;
  hipStream_t s = slot_stream(c, slot);
  j->slot = slot;
  j->off = off;
  c->slot_busy[slot] = 1;
  j->state = Job::RUNNING;
  int rc = CORUTV_OK;
  if (hipEventCreate(&j->e0) != hipSuccess || hipEventCreate(&j->e1) != hipSuccess) rc = CORUTV_E_DEVICE;
  if (rc == CORUTV_OK && j->ready && hipStreamWaitEvent(s, j->ready, 0) != hipSuccess) rc = CORUTV_E_DEVICE;
  if (rc == CORUTV_OK) hipEventRecord(j->e0, s);
  if (rc == CORUTV_OK) rc = enqueue_decompose(c, j->pl, c->ws + off, j->d, s, &j->eq);
  if (rc == CORUTV_OK) {
    hipEventRecord(j->e1, s);
    if (hipMemcpyAsync(slot_status(c, slot), j->eq.dev_status, sizeof(int) * j->eq.nqr,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = CORUTV_E_DEVICE;
    if (rc == CORUTV_OK && j->eq.dev_sum &&
        hipMemcpyAsync(slot_sum(c, slot), j->eq.dev_sum, 16, hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = CORUTV_E_DEVICE;
    if (rc == CORUTV_OK && hipEventRecord(j->e1, s) != hipSuccess) rc = CORUTV_E_DEVICE;
  }
  if (rc != CORUTV_OK) {
    if (rc == CORUTV_E_DEVICE) c->poisoned.store(true);
    j->rc = rc;
    j->state = Job::DONE;
    c->slot_busy[slot] = 0;
    c->arena.release(off);
  }
  return true;
}

void finish_job(corutv_ctx* c, Job* j) {
  float ms = 0.f;
  hipEventElapsedTime(&ms, j->e0, j->e1);
  j->rc = finish_info(j->eq, slot_status(c, j->slot), j->eq.dev_sum ? slot_sum(c, j->slot) : nullptr,
                      &j->info);
  j->info.gpu_ms = ms;
  j->info.ell = j->pl.ell;
  hipEventDestroy(j->e0);
  hipEventDestroy(j->e1);
  if (j->ready) hipEventDestroy(j->ready);
  j->ready = nullptr;
  c->slot_busy[j->slot] = 0;
  c->arena.release(j->off);
  j->state = Job::DONE;
}

void scheduler(corutv_ctx* c) {
  hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(c->mu);
  for (;;) {
    bool progress = false;
    // completions
    for (auto& kv : c->jobs) {
      Job* j = kv.second;
      if (j->state != Job::RUNNING) continue;
      const hipError_t q = hipEventQuery(j->e1);
      if (q == hipSuccess) {
        finish_job(c, j);
        progress = true;
      } else if (q != hipErrorNotReady) {
        c->poisoned.store(true);
        j->rc = CORUTV_E_DEVICE;
        j->state = Job::DONE;
        c->slot_busy[j->slot] = 0;
        c->arena.release(j->off);
        progress = true;
      }
    }
    // admissions, in arrival order (the head blocks later requests so that
    // large requests are not starved)
    // (paused while a blocking call waits for workspace, so it gets the
    // next range that frees up)
    bool blocked = false;
    while (!c->queue.empty()) {
      if (c->blocking_waiters > 0) {
        blocked = true;
        break;
      }
      Job* j = c->queue.front();
      if (c->poisoned.load()) {
        j->rc = CORUTV_E_DEVICE;
        j->state = Job::DONE;
        c->queue.pop_front();
        progress = true;
        continue;
      }
      if (!try_start(c, j)) {
        blocked = true;
        break;
      }
      c->queue.pop_front();
      progress = true;
    }
    if (progress) c->cv.notify_all();
    bool running = false;
    for (auto& kv : c->jobs)
      if (kv.second->state == Job::RUNNING) running = true;
    if (c->stop && c->queue.empty() && !running) break;
    // Every wait releases the lock.  Running requests are polled; otherwise
    // an admission blocked by a blocking call (waiting for workspace, or
    // holding it) waits for that call's notification -- a predicate that
    // is already true here would keep the lock and starve that call.
    if (running)
      c->cv.wait_for(lk, std::chrono::microseconds(20));
    else if (blocked)
      c->cv.wait(lk);
    else
      c->cv.wait(lk, [&] { return c->stop || !c->queue.empty(); });
  }
}

}  // namespace

extern "C" {

int corutv_submit(corutv_ctx* ctx, const corutv_request* req, uint64_t* ticket) {
  int rc = guard(ctx);
  if (rc) return rc;
  if (!req || !ticket) return CORUTV_E_INVAL;
  Job* j = new (std::nothrow) Job();
  if (!j) return CORUTV_E_NOMEM;
  j->d.A = req->A;
  j->d.U = req->U;
  j->d.V = req->V;
  j->d.T = req->T;
  j->d.ldt = req->ldt;
  j->d.piv = req->piv;
  j->d.k = req->k;
  j->d.p = req->p;
  j->d.q = req->q;
  j->d.seed = req->seed;
  j->d.opts = req->opts;
  if (req->opts.flags & CORUTV_FLAG_A_HOST) {  // blocking corutv_decompose only
    delete j;
    return CORUTV_E_INVAL;
  }
  if ((rc = validate(j->d)) != CORUTV_OK ||
      !make_plan(req->A.rows, req->A.cols, req->k, req->p, req->q, req->opts.prec, &j->pl)) {
    delete j;
    return rc ? rc : CORUTV_E_INVAL;
  }
  if (j->pl.total > ctx->ws_bytes) {
    delete j;
    return CORUTV_E_NOMEM;
  }
  if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(j->ready, ctx->streams[0]) != hipSuccess) {
    delete j;
    return poison(ctx);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if ((int)ctx->queue.size() >= ctx->max_queue) {
    delete j;
    return CORUTV_E_BUSY;
  }
  if (!ctx->sched_started) {
    ctx->sched = std::thread(scheduler, ctx);
    ctx->sched_started = true;
  }
  j->ticket = ctx->next_ticket++;
  ctx->jobs[j->ticket] = j;
  ctx->queue.push_back(j);
  *ticket = j->ticket;
  ctx->cv.notify_all();
  return CORUTV_OK;
}

int corutv_poll(corutv_ctx* ctx, uint64_t ticket, corutv_info* info) {
  if (!ctx) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(ticket);
  if (it == ctx->jobs.end()) return CORUTV_E_NOTFOUND;
  Job* j = it->second;
  if (j->state != Job::DONE) return CORUTV_PENDING;
  const int rc = j->rc;
  if (info) *info = j->info;
  ctx->jobs.erase(it);
  delete j;
  return rc;
}

int corutv_wait(corutv_ctx* ctx, uint64_t ticket, corutv_info* info) {
  if (!ctx) return CORUTV_E_INVAL;
  {
    std::unique_lock<std::mutex> lk(ctx->mu);
    auto it = ctx->jobs.find(ticket);
    if (it == ctx->jobs.end()) return CORUTV_E_NOTFOUND;
    Job* j = it->second;
    ctx->cv.wait(lk, [&] { return j->state == Job::DONE; });
  }
  return corutv_poll(ctx, ticket, info);
}

int corutv_cancel(corutv_ctx* ctx, uint64_t ticket) {
  if (!ctx) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(ticket);
  if (it == ctx->jobs.end()) return CORUTV_E_NOTFOUND;
  Job* j = it->second;
  if (j->state != Job::QUEUED) return CORUTV_E_BUSY;
  for (auto q = ctx->queue.begin(); q != ctx->queue.end(); ++q)
    if (*q == j) {
      ctx->queue.erase(q);
      break;
    }
  ctx->jobs.erase(it);
  delete j;
  return CORUTV_OK;
}

int corutv_debug_inject_failure(corutv_ctx* ctx, int32_t after_checks) {
  if (!ctx || after_checks < 0) return CORUTV_E_INVAL;
  ctx->inject_after.store(after_checks);
  return CORUTV_OK;
}

int corutv_pass_timing(corutv_ctx* ctx, int32_t enable, int32_t reset) {
  if (!ctx) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  ctx->timing = enable != 0;
  if (reset) {
    ctx->t_passes = 0;
    ctx->t_total = 0;
    ctx->t_min = 1e300;
    ctx->t_max = 0;
  }
  return CORUTV_OK;
}

int corutv_get_pass_stats(corutv_ctx* ctx, corutv_pass_stats* out) {
  if (!ctx || !out) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  out->passes = ctx->t_passes;
  out->total_ms = ctx->t_total;
  out->min_ms = ctx->t_passes ? ctx->t_min : 0.0;
  out->max_ms = ctx->t_max;
  return CORUTV_OK;
}

int corutv_destroy(corutv_ctx* ctx) {
  if (!ctx) return CORUTV_E_INVAL;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
    ctx->cv.notify_all();
  }
  if (ctx->sched_started) ctx->sched.join();
  for (auto& kv : ctx->jobs) delete kv.second;
  ctx->jobs.clear();
  if (ctx->host_status) hipHostFree(ctx->host_status);
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  for (hipEvent_t e : ctx->dec_ev)
    if (e) hipEventDestroy(e);
  if (ctx->copy_stream) {
    hipStreamSynchronize(ctx->copy_stream);
    for (hipEvent_t e : ctx->stage_ev)
      if (e) hipEventDestroy(e);
    hipStreamDestroy(ctx->copy_stream);
  }
  delete ctx;
  return CORUTV_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// ALM-CoRUTV (Sec. 4, Algorithm 2)
namespace {

// iterations whose r_j is recorded
constexpr int kRankHist = 4096;

struct RpcaPlan {
  Plan dec;
  int ell = 0;
  size_t o_y = 0, o_b = 0, o_u = 0, o_v = 0, o_t = 0, o_tt = 0, o_p = 0, o_q = 0, o_part = 0,
         o_sum = 0, o_flag = 0, o_hist = 0;
  size_t total = 0;
};

bool make_rpca_plan(int64_t m, int64_t n, int k, int p, int q, RpcaPlan* rp) {
  if (!make_plan(m, n, k, p, q, P_F64, &rp->dec)) return false;
  const int ell = k + p;
  rp->ell = ell;
  size_t off = rp->dec.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  rp->o_y = take((size_t)m * n * 8);
  rp->o_b = take((size_t)m * n * 8);
  rp->o_u = take((size_t)m * ell * 8);
  rp->o_v = take((size_t)n * ell * 8);
  rp->o_t = take((size_t)ell * ell * 8);
  rp->o_tt = take((size_t)ell * ell * 8);
  rp->o_p = take((size_t)m * ell * 8);
  rp->o_q = take((size_t)n * ell * 8);
  rp->o_part = take((size_t)rpca_partial_blocks() * 8);
  rp->o_sum = take(4 * 8);
  rp->o_flag = take(16);
  rp->o_hist = take(kRankHist * sizeof(int32_t));
  rp->total = off;
  return true;
}

}  // namespace

extern "C" int corutv_rpca_ranks(corutv_ctx* ctx, int32_t* ranks, int32_t n, int32_t* count) {
  if (!ctx || n < 0 || (n > 0 && !ranks)) return CORUTV_E_INVAL;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  const int32_t c = (int32_t)ctx->rank_hist.size();
  for (int32_t i = 0; i < std::min(n, c); ++i) ranks[i] = ctx->rank_hist[i];
  if (count) *count = c;
  return CORUTV_OK;
}

extern "C" uint64_t corutv_rpca_workspace_bytes(int64_t m, int64_t n, int32_t k, int32_t p, int32_t q) {
  RpcaPlan rp;
  if (!make_rpca_plan(m, n, k, p, q, &rp)) return 0;
  return rp.total;
}

extern "C" int corutv_rpca(corutv_ctx* ctx, const corutv_mat* M, double lambda, int32_t k, int32_t p,
                           int32_t q, int32_t max_iter, double tol, uint64_t seed,
                           const corutv_opts* opts, corutv_mat* L, corutv_mat* S,
                           corutv_rpca_info* info) {
  int rc = guard(ctx);
  if (rc) return rc;
  (void)opts;
  if (!mat_ok(M) || !mat_ok(S) || M->dtype != CORUTV_F32 || S->dtype != CORUTV_F32) return CORUTV_E_INVAL;
  const int64_t m = M->rows, n = M->cols;
  if (S->rows != m || S->cols != n) return CORUTV_E_INVAL;
  if (L && (!mat_ok(L) || L->dtype != CORUTV_F32 || L->rows != m || L->cols != n)) return CORUTV_E_INVAL;
  if (k < 1 || p < 0 || q < 0 || q > 30 || max_iter < 1 || (int64_t)k + p > std::min(m, n) || k + p > 256)
    return CORUTV_E_INVAL;
  RpcaPlan rp;
  if (!make_rpca_plan(m, n, k, p, q, &rp)) return CORUTV_E_INVAL;
  if (rp.total > ctx->ws_bytes) return CORUTV_E_NOMEM;
  if (!(lambda > 0)) lambda = 1.0 / std::sqrt((double)std::max(m, n));
  const int ell = rp.ell;
  std::lock_guard<std::mutex> lk(ctx->run_mu);
  WsLease lease;
  if ((rc = lease_ws(ctx, rp.total, &lease)) != CORUTV_OK) return rc;
  hipStream_t s = ctx->streams[0];
  char* ws = lease.base();
  double* Y = (double*)(ws + rp.o_y);
  double* B = (double*)(ws + rp.o_b);
  double* U = (double*)(ws + rp.o_u);
  double* V = (double*)(ws + rp.o_v);
  double* T = (double*)(ws + rp.o_t);
  double* Tt = (double*)(ws + rp.o_tt);
  double* Pm = (double*)(ws + rp.o_p);
  double* Qm = (double*)(ws + rp.o_q);
  double* part = (double*)(ws + rp.o_part);
  double* sum = (double*)(ws + rp.o_sum);
  int* sticky = (int*)(ws + rp.o_flag);  // OR of the loop's QR status words
  int* hist = (int*)(ws + rp.o_hist);     // r_j per iteration
  const int nb = rpca_partial_blocks();
  // Y and B share M's layout, packed
  const int lay = M->layout;
  const int64_t ldi = lay == CORUTV_COL_MAJOR ? m : n;
  if (ctx->timing) {
    while ((int)ctx->ev_pool.size() < 2 * max_iter) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return poison(ctx);
      ctx->ev_pool.push_back(e);
    }
  }
  // the context's start / end events (calls on one context are serialised)
  if (!ctx->dec_ev[0] &&
      (hipEventCreate(&ctx->dec_ev[0]) != hipSuccess || hipEventCreate(&ctx->dec_ev[1]) != hipSuccess))
    return poison(ctx);
  hipEvent_t e0 = ctx->dec_ev[0], e1 = ctx->dec_ev[1];
  hipEventRecord(e0, s);
  // Y = 0 (m n doubles: a whole number of 16-byte words when m n is even)
  if ((size_t)m * n % 2 == 0) {
    ZeroRanges zy{};
    zy.ptr[0] = Y;
    zy.words[0] = (int64_t)((size_t)m * n / 2);
    zy.count = 1;
    HIPOK(launch_zero_ranges(zy, s));
  } else {
    HIPOK(hipMemsetAsync(Y, 0, (size_t)m * n * 8, s));
  }
  HIPOK(launch_widen((const float*)M->ptr, lay, M->ld, m, n, B, ldi, s));
  HIPOK(launch_fill_int(sticky, 1, 0, s));
  // ||M||_F
  HIPOK(launch_sumsq((const float*)M->ptr, lay, M->ld, m, n, part, s));
  HIPOK(launch_reduce(part, nb, 1, sum, nullptr, s));
  // decomposition arguments shared by every CoR-UTV of the loop
  DecArgs d;
  d.U = corutv_mat{U, m, ell, m, CORUTV_F64, CORUTV_COL_MAJOR};
  d.V = corutv_mat{V, n, ell, n, CORUTV_F64, CORUTV_COL_MAJOR};
  d.T = T;
  d.ldt = ell;
  d.T2 = Tt;  // T^T for the rank-r factors below, from the same launch as T
  d.ldt2 = ell;
  d.k = k;
  d.p = p;
  d.q = q;
  d.seed = seed;
  d.opts.prec = P_F64;
  d.opts.tri = CORUTV_TRI_AUTO;
  Enqueued eq;
  corutv_mat Bm{B, m, n, ldi, CORUTV_F64, lay};
  // mu_0 = 1.25 / ||M||_2, with ||M||_2 estimated by T[0,0] of a CoR-UTV of M
  d.A = Bm;
  d.sub = 0xFFFF;
  rc = enqueue_decompose(ctx, rp.dec, ws, d, s, &eq);
  if (rc != CORUTV_OK) return rc == CORUTV_E_DEVICE ? poison(ctx) : rc;
  double h[2] = {0, 0};
  int hst[kMaxQr];
  HIPOK(hipMemcpyAsync(h, T, 8, hipMemcpyDeviceToHost, s));
  HIPOK(hipMemcpyAsync(h + 1, sum, 8, hipMemcpyDeviceToHost, s));
  HIPOK(hipMemcpyAsync(hst, eq.dev_status, sizeof(int) * eq.nqr, hipMemcpyDeviceToHost, s));
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  if (finish_info(eq, hst, nullptr, nullptr) != CORUTV_OK || !(h[0] > 0) || !std::isfinite(h[1]))
    return CORUTV_E_NUMERIC;
  const double normM = std::sqrt(h[1]);
  const double mu0 = 1.25 / h[0];
  const double mu_bar = 1e7 * mu0;
  const double rho = 1.5;
  double mu = mu0;
  const bool lower = m < n;  // AUTO orientation: lower T for the wide problem
  int iters = 0;
  double zeta = -1.0, mu_last = mu;
  for (int j = 0; j < max_iter; ++j) {
    d.A = Bm;
    d.sub = (uint32_t)j;
    rc = enqueue_decompose(ctx, rp.dec, ws, d, s, &eq);
    if (rc != CORUTV_OK) return rc == CORUTV_E_DEVICE ? poison(ctx) : rc;
    // rank-r factors: upper T -> P = U, Q = V T^T; lower T -> P = U T, Q = V
    MatOut o;
    o.ptr = lower ? Pm : Qm;
    o.ld = lower ? m : n;
    if (lower)
      HIPOK(launch_rowmat(U, m, m, ell, T, ell, nullptr, o, 0, MatOut(), 0, nullptr, s));
    else
      HIPOK(launch_rowmat(V, n, n, ell, Tt, ell, nullptr, o, 0, MatOut(), 0, nullptr, s));
    const double* P = lower ? Pm : U;
    const double* Q = lower ? V : Qm;
    const double mu_next = std::min(rho * mu, mu_bar);
    const bool last = j + 1 == max_iter;
    // L is an output only: written when this iteration may be the last
    const bool want_l = L && (last || tol > 0);
    if (ctx->timing) hipEventRecord(ctx->ev_pool[2 * j], s);
    HIPOK(launch_rpca_elementwise((const float*)M->ptr, lay, M->ld, (float*)S->ptr, S->layout, S->ld, Y,
                                  ldi, last ? nullptr : B, ldi, want_l ? (float*)L->ptr : nullptr,
                                  L ? L->layout : CORUTV_COL_MAJOR, L ? L->ld : 1, m, n, P, m, Q, n, T,
                                  ell, ell, mu, mu_next, lambda, part, eq.dev_status, eq.nqr, sticky,
                                  j < kRankHist ? hist + j : nullptr, s));
    if (ctx->timing) hipEventRecord(ctx->ev_pool[2 * j + 1], s);
    iters = j + 1;
    mu_last = mu;
    mu = mu_next;
    if (tol > 0 || last) {  // the residual is needed: sum the step's partials
      HIPOK(launch_reduce(part, nb, 1, sum, nullptr, s));
      double zs = 0;
      int flags = 0;
      HIPOK(hipMemcpyAsync(&zs, sum, 8, hipMemcpyDeviceToHost, s));
      HIPOK(hipMemcpyAsync(&flags, sticky, 4, hipMemcpyDeviceToHost, s));
      if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
      zeta = std::sqrt(zs) / normM;
      // a non-finite input to a QR of the loop (status bit 2) or residual
      if ((flags & 2) || !std::isfinite(zeta)) return CORUTV_E_NUMERIC;
      if (tol > 0 && zeta < tol) break;
    }
  }
  // final rank: diagonal entries of the last T above 1/mu_last
  std::vector<double> Th((size_t)ell * ell);
  HIPOK(hipMemcpyAsync(Th.data(), T, Th.size() * 8, hipMemcpyDeviceToHost, s));
  std::vector<int32_t> rh((size_t)std::min(iters, kRankHist));
  if (!rh.empty()) HIPOK(hipMemcpyAsync(rh.data(), hist, rh.size() * 4, hipMemcpyDeviceToHost, s));
  hipEventRecord(e1, s);
  if (hipStreamSynchronize(s) != hipSuccess) return poison(ctx);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  double step_ms = 0;
  if (ctx->timing) {
    for (int j = 0; j < iters; ++j) {
      float em = 0.f;
      if (hipEventElapsedTime(&em, ctx->ev_pool[2 * j], ctx->ev_pool[2 * j + 1]) == hipSuccess) step_ms += em;
    }
  }
  ctx->rank_hist.swap(rh);
  int r = 0;  // diagonal entries above the last threshold (eq. 12)
  for (int i = 0; i < ell; ++i) r += Th[(size_t)i * ell + i] > 1.0 / mu_last ? 1 : 0;
  if (info) {
    info->step_ms = step_ms;
    info->iters = iters;
    info->final_rank = r;
    info->zeta = zeta;
    info->mu0 = mu0;
    info->mu = mu;
    info->gpu_ms = ms;
  }
  return CORUTV_OK;
}
