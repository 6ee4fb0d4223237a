// Host runtime of libblrqr: the C ABI, device memory, and the launch plans
// of compression, the tiled BLR-QR (Alg. 4 with Section 3.4 of arXiv
// 2208.06194), the application of Q / Q^T (Alg. 5) and the least-squares
// solve.
//
// Planning.  Tile formats evolve only through OP1 (a low-rank target that
// receives a dense update becomes dense), which depends on formats alone, so
// the host simulates the format evolution once and knows every launch of the
// factorization before the first one is enqueued.  Ranks change on the device
// (rounded additions); low-rank slots have a fixed capacity rc (zero padded),
// so every product has a static shape and the device reads actual ranks only
// inside the recompression kernel.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <mutex>

namespace {
thread_local std::string g_last_error;

blr_status fail(blr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace

namespace blr {

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) throw Error(BLR_ERR_OOM, std::string(what) + ": out of device memory");
  throw Error(BLR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* Arena::alloc(size_t n) {
  if (n == 0) n = 256;
  n = (n + 255) & ~(size_t)255;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(BLR_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
  }
  blocks.push_back(p);
  bytes += (int64_t)n;
  return p;
}

void Arena::release() {
  for (void* p : blocks) (void)hipFree(p);
  blocks.clear();
  bytes = 0;
}

void* Workspace::alloc(size_t n) {
  if (n == 0) n = 256;
  n = (n + 255) & ~(size_t)255;
  for (; cur < chunks.size(); ++cur) {
    Chunk& c = chunks[cur];
    if (c.size - c.used >= n) {
      void* p = c.p + c.used;
      c.used += n;
      return p;
    }
  }
  // a new chunk: at least 64 MiB, so that small allocations share chunks
  const size_t sz = std::max<size_t>(n, (size_t)64 << 20);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(BLR_ERR_OOM, "hipMalloc of " + std::to_string(sz) + " bytes of workspace failed");
  }
  chunks.push_back(Chunk{(char*)p, sz, n});
  cur = chunks.size() - 1;
  bytes += (int64_t)sz;
  return p;
}

void Workspace::reset() {
  for (Chunk& c : chunks) c.used = 0;
  cur = 0;
}

void Workspace::release() {
  for (Chunk& c : chunks) (void)hipFree(c.p);
  chunks.clear();
  cur = 0;
  bytes = 0;
}

void Plan::gemm(double* C, int64_t ldc, const double* Cin, int64_t ldcin, double* D2, int64_t ldd2,
                int M, int N, double alpha, double beta, const double* A, int64_t lda,
                const double* B, int64_t ldb, int K, int segflags, int descflags) {
  if (M <= 0 || N <= 0) return;
  GemmDesc d{};
  d.C = C;
  d.ldc = ldc;
  d.Cin = Cin;
  d.ldcin = ldcin;
  d.D2 = D2;
  d.ldd2 = ldd2;
  d.M = M;
  d.N = N;
  d.alpha = alpha;
  d.beta = beta;
  d.seg_begin = (int)curseg.size();
  d.nseg = K > 0 ? 1 : 0;
  d.flags = descflags;
  if (K > 0) {
    GemmSeg s{};
    s.A = A;
    s.B = B;
    s.lda = lda;
    s.ldb = ldb;
    s.K = K;
    s.flags = segflags;
    curseg.push_back(s);
  }
  const bool tri = segflags & (SEG_A_UPPER | SEG_A_UNIT_LOWER);
  curflops += 2.0 * M * N * (double)K * (tri ? 0.5 : 1.0);
  cur.push_back(d);
}

void Plan::gemm_multi(double* C, int64_t ldc, const double* Cin, int64_t ldcin, int M, int N, double alpha,
                      double beta, const std::vector<GemmSeg>& sv) {
  if (M <= 0 || N <= 0) return;
  GemmDesc d{};
  d.C = C;
  d.ldc = ldc;
  d.Cin = Cin;
  d.ldcin = ldcin;
  d.M = M;
  d.N = N;
  d.alpha = alpha;
  d.beta = beta;
  d.seg_begin = (int)curseg.size();
  d.nseg = 0;
  for (const GemmSeg& sg : sv) {
    if (sg.K <= 0) continue;
    curseg.push_back(sg);
    d.nseg++;
    const bool tri = sg.flags & (SEG_A_UPPER | SEG_A_UNIT_LOWER);
    curflops += 2.0 * M * N * (double)sg.K * (tri ? 0.5 : 1.0);
  }
  cur.push_back(d);
}

void Plan::flush_gemm(int fp32, int prof, bool allow_fast) {
  if (cur.empty()) return;
  int mn = 1 << 30;
  int64_t tiles128 = 0;
  for (auto& d : cur) {
    mn = std::min(mn, std::min(d.M, d.N));
    tiles128 += (int64_t)((d.M + 127) / 128) * ((d.N + 127) / 128);
  }
  // 128 x 128 tiles when every product has at least one full tile and the
  // batch has enough of them to fill the chip; 64 x 64 tiles otherwise
  int big = (mn >= 256 || (mn >= 128 && tiles128 >= 128)) ? GEMM_BIG : GEMM_SMALL;
  if (big == GEMM_BIG && allow_fast) {
    // fast path: full tiles, single uniform segment, aligned, no masks
    bool ok = true;
    int tflags = -1;
    auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    for (auto& d : cur) {
      if (d.M % 128 || d.N % 128 || d.nseg < 1) { ok = false; break; }
      for (int si = 0; si < d.nseg && ok; ++si) {
        const GemmSeg& sg = curseg[d.seg_begin + si];
        const int tf = sg.flags & (SEG_TRANS_A | SEG_TRANS_B);
        if (tflags < 0) tflags = tf;
        if (tf != tflags || (sg.flags & (SEG_A_UNIT_LOWER | SEG_B_UNIT_LOWER)) ||
            sg.K % (fp32 ? kFastKStep32 : kFastKStep64) ||
            !al(sg.A) || !al(sg.B) || (sg.lda & 1) || (sg.ldb & 1))
          ok = false;
      }
      if (!ok) break;
    }
    if (ok) {
      const bool ta = tflags & SEG_TRANS_A, tb = tflags & SEG_TRANS_B;
      big = ta ? (tb ? GEMM_FAST_TT : GEMM_FAST_TN) : (tb ? GEMM_FAST_NT : GEMM_FAST_NN);
    }
  }
  // FP64 products with at most 16 columns (Q^T B, Q B, the back-substitution
  // sums, basis products with a few right-hand sides) take the skinny kernel
  if (!fp32) {
    bool sk = true;
    int ta = -1;
    for (auto& d : cur) {
      if (d.N > 16 || (d.flags & DESC_LOWER_ONLY)) { sk = false; break; }
      for (int si = 0; si < d.nseg && sk; ++si) {
        const int f = curseg[d.seg_begin + si].flags;
        const int t = (f & SEG_TRANS_A) ? 1 : 0;
        if ((f & (SEG_TRANS_B | SEG_B_UNIT_LOWER)) || (ta >= 0 && t != ta)) sk = false;
        ta = t;
      }
      if (!sk) break;
    }
    if (sk && ta >= 0) big = ta ? GEMM_SKINNY_T : GEMM_SKINNY_N;
  }
  const bool skinny = big == GEMM_SKINNY_N || big == GEMM_SKINNY_T;
  const int BM = (big == GEMM_SMALL || skinny) ? 64 : 128;
  const int BN = skinny ? 16 : BM;
  // FP32 products with long K sums accumulate in FP64 between K chunks
  if (fp32 && big >= GEMM_FAST_NN) {
    int64_t kmax = 0;
    for (auto& d : cur) {
      int64_t kt = 0;
      for (int si = 0; si < d.nseg; ++si) kt += curseg[d.seg_begin + si].K;
      kmax = std::max(kmax, kt);
    }
    if (kmax > 1024) fp32 = 2;
  }
  Op o;
  o.kind = Op::GEMM;
  o.off = (int)descs.size();
  o.n = (int)cur.size();
  o.big = big;
  o.fp32 = fp32;
  o.prof = prof;
  o.flops = curflops;
  const int segbase = (int)segs.size();
  int tiles = 0;
  for (auto& d : cur) {
    d.tilesM = (d.M + BM - 1) / BM;
    d.tile_begin = tiles;
    tiles += d.tilesM * ((d.N + BN - 1) / BN);
    d.seg_begin += segbase;
    descs.push_back(d);
  }
  segs.insert(segs.end(), curseg.begin(), curseg.end());
  o.ntiles = tiles;
  o.stream = cur_stream;
  o.prio = cur_prio;
  ops.push_back(o);
  cur.clear();
  curseg.clear();
  curflops = 0.0;
}

void Plan::flush_rc() {
  if (currc.empty()) return;
  Op o;
  o.kind = Op::RC;
  o.off = (int)rcs.size();
  o.n = (int)currc.size();
  o.stream = cur_stream;
  o.prio = cur_prio;
  rcs.insert(rcs.end(), currc.begin(), currc.end());
  ops.push_back(o);
  currc.clear();
}

namespace {
template <class T>
T* upload_array(const std::vector<T>& v, DevAlloc& a, HostKeep& keep, hipStream_t s) {
  if (v.empty()) return nullptr;
  const size_t n = v.size() * sizeof(T);
  T* d = (T*)a.alloc(n);
  keep.emplace_back((const char*)v.data(), (const char*)v.data() + n);
  HIPCHECK(hipMemcpyAsync(d, keep.back().data(), n, hipMemcpyHostToDevice, s));
  return d;
}
}  // namespace

void Plan::upload(DevAlloc& a, HostKeep& keep, hipStream_t s) {
  d_descs = upload_array(descs, a, keep, s);
  d_segs = upload_array(segs, a, keep, s);
  d_copies = upload_array(copies, a, keep, s);
  d_rcs = upload_array(rcs, a, keep, s);
  d_jobs = upload_array(jobs, a, keep, s);
  d_tjobs = upload_array(tjobs, a, keep, s);
  d_lincs = upload_array(lincs, a, keep, s);
  d_frobs = upload_array(frobs, a, keep, s);
  d_trees = upload_array(trees, a, keep, s);
  d_titems = upload_array(titems, a, keep, s);
}

size_t Plan::upload_bytes() const {
  size_t n = 0;
  auto add = [&n](size_t bytes) {
    if (bytes) n += (bytes + 255) & ~(size_t)255;
  };
  add(descs.size() * sizeof(GemmDesc));
  add(segs.size() * sizeof(GemmSeg));
  add(copies.size() * sizeof(CopyDesc));
  add(rcs.size() * sizeof(RcDesc));
  add(jobs.size() * sizeof(PanelJob));
  add(tjobs.size() * sizeof(TrsmJob));
  add(lincs.size() * sizeof(LincombDesc));
  add(frobs.size() * sizeof(Frob2Desc));
  add(trees.size() * sizeof(TsqrTree));
  add(titems.size() * sizeof(TsqrItem));
  return n;
}

void Plan::clear() { *this = Plan(); }

}  // namespace blr

using namespace blr;

namespace {

int round_up(int x, int a) { return (x + a - 1) / a * a; }

RcParams rc_params(blr_matrix h) {
  RcParams p;
  p.b = h->b;
  p.rc = h->rc;
  p.cap = h->cap;
  p.eps = h->tol;
  p.overflow_count = h->d_counters;
  p.max_dropped_bits = h->d_counters + 1;
  return p;
}

constexpr int kStreams = 4;
// block columns of the tiled factor in flight at once (one chain each; the
// chains are merged into one launch list)
constexpr int kTiledChains = 32;

// Calls on one handle.  Every call that enqueues work records h->idle on the
// caller's stream at its end (after the handle's own streams have been
// joined to it).  The next call waits for that event only (the host waits
// for this handle's work, never for the whole device) before it reuses the
// workspace and drops the host copies of the previous uploads.
void wait_idle(blr_matrix h) {
  if (h->idle_set) HIPCHECK(hipEventSynchronize(h->idle));
}

void begin_call(blr_matrix h) {
  wait_idle(h);
  h->keep.clear();
  h->work.reset();
}

void end_call(blr_matrix h, hipStream_t s) {
  if (!h->idle) HIPCHECK(hipEventCreateWithFlags(&h->idle, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(h->idle, s));
  h->idle_set = true;
}

// Reuse the workspace inside a call once the caller's stream s has been
// synchronised (everything the call enqueued so far ran on s or was joined
// to it).
void reset_work_after_sync(blr_matrix h) {
  h->keep.clear();
  h->work.reset();
}

// Stream-ordered upload of a host array into the workspace.
template <class T>
T* upload_vec(blr_matrix h, const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return nullptr;
  const size_t n = v.size() * sizeof(T);
  T* d = (T*)h->work.alloc(n);
  h->keep.emplace_back((const char*)v.data(), (const char*)v.data() + n);
  HIPCHECK(hipMemcpyAsync(d, h->keep.back().data(), n, hipMemcpyHostToDevice, s));
  return d;
}

// The caller's rows (rows x nrhs, ld ldx) copied into a workspace block of
// prows rows whose remaining rows are zero: a block of the caller's size
// extended to a ragged matrix's embedding.  Enqueued on s.
double* pad_rows(blr_matrix h, const double* X, int64_t ldx, int64_t rows, int64_t prows, int nrhs, hipStream_t s) {
  double* P = (double*)h->work.alloc((size_t)prows * nrhs * 8);
  HIPCHECK(hipMemsetAsync(P, 0, (size_t)prows * nrhs * 8, s));
  HIPCHECK(hipMemcpy2DAsync(P, prows * 8, X, ldx * 8, rows * 8, nrhs, hipMemcpyDeviceToDevice, s));
  return P;
}

void ensure_streams(blr_matrix h) {
  while ((int)h->streams.size() < kStreams) {
    hipStream_t st;
    HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    h->streams.push_back(st);
  }
}

// Enqueue a plan.  Ops name one of the handle's look-ahead streams; the
// caller's stream s is joined before the first op and after the last one.
// Enqueue one op on stream q (launches counted on h).  ev: the plan's events
// (used only by a plan on several streams).
void enqueue(blr_matrix h, const Plan& P, const Op& o, hipStream_t q, bool multi, std::vector<hipEvent_t>& ev) {
    switch (o.kind) {
      case Op::GEMM: {
        // the dominant kernel: k_gemm_fast<CT, false, false> (untransposed
        // 128x128 products), FP64 operands (fp32 == 0) or FP32 (fp32 == 1)
        const bool rec = h->prof_on && o.big == GEMM_FAST_NN && (o.fp32 == 0 || o.fp32 == 1);
        const int pk = o.fp32;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (rec) {
          HIPCHECK(hipEventCreate(&e0));
          HIPCHECK(hipEventCreate(&e1));
          HIPCHECK(hipEventRecord(e0, q));
        }
        HIPCHECK(launch_gemm(P.d_descs + o.off, o.n, P.d_segs, o.ntiles, o.big, o.fp32, q));
        if (rec) {
          HIPCHECK(hipEventRecord(e1, q));
          h->prof_ev[pk].push_back(e0);
          h->prof_ev[pk].push_back(e1);
          h->prof_flops[pk] += o.flops;
          h->prof_launches[pk] += 1;
        }
        h->launches += 1;
        break;
      }
      case Op::PANEL:
        HIPCHECK(launch_panel(o.panel, q));
        h->launches += 1;
        break;
      case Op::PANEL_APPLY:
        HIPCHECK(launch_panel_apply(o.panel, o.n, q));
        h->launches += 1;
        break;
      case Op::TBACK:
        HIPCHECK(launch_t_backsolve(o.tback, q));
        h->launches += 1;
        break;
      case Op::RC:
        HIPCHECK(launch_recompress(P.d_rcs + o.off, o.n, rc_params(h), q));
        h->launches += 1;
        break;
      case Op::TALL_APPLY:
        HIPCHECK(launch_tall_apply(o.panel, o.ntiles, o.n, o.buf, q));
        h->launches += 2;
        break;
      case Op::COPY:
        HIPCHECK(launch_copy_blocks(P.d_copies + o.off, o.n, o.maxel, q));
        h->launches += 1;
        break;
      case Op::PANEL_B:
        HIPCHECK(launch_panel_batch(P.d_jobs + o.off, o.n, o.ib, o.ext, q));
        h->launches += 1;
        break;
      case Op::PANEL_APPLY_B:
        HIPCHECK(launch_panel_apply_batch(P.d_jobs + o.off, o.n, o.ib, o.ext, q));
        h->launches += 1;
        break;
      case Op::TBACK_B:
        HIPCHECK(launch_t_backsolve_batch(P.d_jobs + o.off, o.n, o.ext, q));
        h->launches += 1;
        break;
      case Op::TALL_APPLY_B:
        HIPCHECK(launch_tall_apply_batch(P.d_jobs + o.off, o.n, o.ib, o.ext, o.ext2, q));
        h->launches += 2;
        break;
      case Op::TRSM: {
        const TrsmJob& J = o.trsm;
        if (o.n) HIPCHECK(launch_trsm_upper_t(J.R, J.ldr, J.n, J.X, J.ldx, J.nrhs, q));
        else HIPCHECK(launch_trsm_upper(J.R, J.ldr, J.n, J.X, J.ldx, J.nrhs, q));
        h->launches += 1;
        break;
      }
      case Op::TRSM_B:
        HIPCHECK(launch_trsm_batch(P.d_tjobs + o.off, o.n, o.first, o.ext, q));
        h->launches += 1;
        break;
      case Op::LINCOMB:
        HIPCHECK(launch_lincomb_batch(P.d_lincs + o.off, o.n, o.maxel, q));
        h->launches += 1;
        break;
      case Op::FROB2:
        HIPCHECK(launch_frob2(P.d_frobs + o.off, o.n, q));
        h->launches += 1;
        break;
      case Op::MGS_STACK:
        HIPCHECK(launch_mgs_stack(o.mgs.X, o.mgs.ldx, o.mgs.h, o.mgs.w, o.mgs.R, o.mgs.ldr, q));
        h->launches += 1;
        break;
      case Op::TSQR_QR:
        HIPCHECK(launch_tsqr_qr(P.d_trees, P.d_titems + o.off, o.n, o.ext, q));
        h->launches += 1;
        break;
      case Op::TSQR_FIN:
        HIPCHECK(launch_tsqr_final(P.d_trees, P.d_titems + o.off, o.n, o.ext, q));
        h->launches += 1;
        break;
      case Op::WAIT:
        if (multi) HIPCHECK(hipStreamWaitEvent(q, ev[o.event], 0));
        break;
      case Op::RECORD:
        if (multi) HIPCHECK(hipEventRecord(ev[o.event], q));
        break;
      default:
        break;
    }
}

void execute(blr_matrix h, Plan& P, hipStream_t s) {
  int nstreams = 1;
  for (const Op& o : P.ops) nstreams = std::max(nstreams, o.stream + 1);
  std::vector<hipStream_t> st(nstreams, s);
  std::vector<hipEvent_t> ev(P.n_events, nullptr);
  hipEvent_t join = nullptr;
  if (nstreams > 1) {
    ensure_streams(h);
    for (int a = 0; a < nstreams; ++a) st[a] = h->streams[a];
    HIPCHECK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(join, s));
    for (int a = 0; a < nstreams; ++a) HIPCHECK(hipStreamWaitEvent(st[a], join, 0));
    for (auto& e : ev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  for (const Op& o : P.ops) enqueue(h, P, o, st[o.stream], nstreams > 1, ev);
  if (nstreams > 1) {
    for (int a = 0; a < nstreams; ++a) {
      hipEvent_t e;
      HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      HIPCHECK(hipEventRecord(e, st[a]));
      HIPCHECK(hipStreamWaitEvent(s, e, 0));
      HIPCHECK(hipEventDestroy(e));
    }
    for (auto& e : ev) HIPCHECK(hipEventDestroy(e));
    HIPCHECK(hipEventDestroy(join));
  }
}

// Upload a plan's descriptors into the handle's workspace and enqueue it.
void run_plan(blr_matrix h, Plan& P, hipStream_t s) {
  P.upload(h->work, h->keep, s);
  execute(h, P, s);
}

// ---------------------------------------------------------------------------
// Workspace of one factorization / application (single stream: reused by
// every step, since the ops of consecutive steps are ordered on the stream).
struct Work {
  double *Wx, *Wx2, *Wg;                    // panel trailing updates, Gram matrix
  std::vector<double*> X, X2;               // per column j: b x b
  std::vector<double*> PU, WU, YWU, M2, Uw; // per j: b x rc
  std::vector<double*> S, S2, Vtw;          // per j: rc x b
  std::vector<double*> G, M1;               // per j: rc x rc
  std::vector<int*> rankw;                  // per j
  std::vector<double*> rcw;                 // recompression workspaces (2 per j)
};

// Device bytes make_work(h, nrhs_cols) takes.
size_t work_bytes(blr_matrix h, int nrhs_cols) {
  const size_t b = h->b, rc = h->rc, q = std::max(h->q, 1);
  const size_t wcols = std::max<size_t>(b, nrhs_cols);
  const size_t d = 2 * b * wcols + b * b + 2 * q * b * wcols + q * (5 * b * rc + 3 * rc * b + 2 * rc * rc) +
                   2 * q * rc_work_doubles((int)b, (int)rc);
  return d * 8 + q * sizeof(int);
}

Work make_work(blr_matrix h, int nrhs_cols) {
  Work w;
  const int b = h->b, rc = h->rc, q = std::max(h->q, 1);
  const int wcols = std::max(b, nrhs_cols);
  Workspace& A = h->work;
  w.Wx = (double*)A.alloc((size_t)b * wcols * 8);
  w.Wx2 = (double*)A.alloc((size_t)b * wcols * 8);
  w.Wg = (double*)A.alloc((size_t)b * b * 8);
  double* big = (double*)A.alloc((size_t)2 * q * b * wcols * 8);
  double* lr = (double*)A.alloc((size_t)q * (5 * (size_t)b * rc + 3 * (size_t)rc * b + 2 * (size_t)rc * rc) * 8);
  int* rk = (int*)A.alloc((size_t)q * sizeof(int));
  const size_t rcwd = rc_work_doubles(b, rc);
  double* rcw = (double*)A.alloc((size_t)2 * q * rcwd * 8);
  for (int j = 0; j < q; ++j) {
    w.X.push_back(big + (size_t)(2 * j) * b * wcols);
    w.X2.push_back(big + (size_t)(2 * j + 1) * b * wcols);
    double* base = lr + (size_t)j * (5 * (size_t)b * rc + 3 * (size_t)rc * b + 2 * (size_t)rc * rc);
    w.PU.push_back(base);
    w.WU.push_back(base + (size_t)b * rc);
    w.YWU.push_back(base + 2 * (size_t)b * rc);
    w.M2.push_back(base + 3 * (size_t)b * rc);
    w.Uw.push_back(base + 4 * (size_t)b * rc);
    double* b2 = base + 5 * (size_t)b * rc;
    w.S.push_back(b2);
    w.S2.push_back(b2 + (size_t)rc * b);
    w.Vtw.push_back(b2 + 2 * (size_t)rc * b);
    double* b3 = b2 + 3 * (size_t)rc * b;
    w.G.push_back(b3);
    w.M1.push_back(b3 + (size_t)rc * rc);
    w.rankw.push_back(rk + j);
    w.rcw.push_back(rcw + (size_t)(2 * j) * rcwd);
    w.rcw.push_back(rcw + (size_t)(2 * j + 1) * rcwd);
  }
  return w;
}

// From this order up the full T of a tile QR is built by doubling; below it
// one back-substitution launch is cheaper than the 2 log2(n / ib) products.
constexpr int kTDoublingMin = 512;

// The full upper triangular T (n x n, ld ldt) of n reflectors from its ib x ib
// diagonal blocks (already in T) and the Gram matrix G = Y^T Y (strictly lower
// part read, ld ldg), by recursive doubling on the matrix cores (the compact
// WY merge of Schreiber and Van Loan): for adjacent blocks B1, B2 of width s
// (B2 possibly narrower at the end) T(B1, B2) = -T(B1, B1) G(B1, B2) T(B2, B2),
// for s = ib, 2 ib, 4 ib, ...; every level is two batched products
// (G(B2, B1)^T T22 into Mb, then -T11 Mb).  Mb needs n * n / 4 doubles.  T11
// is read as upper triangular with the zeros stored below its diagonal, which
// T's storage keeps.

void plan_t_doubling(Plan& P, const double* G, int64_t ldg, double* T, int64_t ldt, int n, int ib, double* Mb) {
  for (int s = ib; s < n; s *= 2) {
    size_t off = 0;
    std::vector<std::pair<int, size_t>> pairs;
    for (int a = 0; a + s < n; a += 2 * s) {
      const int s2 = std::min(s, n - a - s);
      P.gemm(Mb + off, s, nullptr, 0, nullptr, 0, s, s2, 1.0, 0.0, G + (a + s) + (int64_t)a * ldg, ldg,
             T + (a + s) + (int64_t)(a + s) * ldt, ldt, s2, SEG_TRANS_A);
      pairs.push_back({a, off});
      off += (size_t)s * s2;
    }
    P.flush_gemm();
    for (auto [a, o] : pairs) {
      const int s2 = std::min(s, n - a - s);
      P.gemm(T + a + (int64_t)(a + s) * ldt, ldt, nullptr, 0, nullptr, 0, s, s2, -1.0, 0.0, T + a + (int64_t)a * ldt,
             ldt, Mb + o, s, s, SEG_A_UPPER);
    }
    P.flush_gemm();
  }
}

// Householder QR of one tile (GEQRT, Section 3.4.1) or of [R; B] (TPQRT,
// Section 3.4.3), with inner blocking ib: a panel kernel generates ib
// reflectors and their T block, three products update the rest of the tile,
// and at the end the off-diagonal blocks of the full T come from the Gram
// matrix of all reflectors (by doubling for large tiles, else by one
// back-substitution).
void plan_tile_qr(Plan& P, blr_matrix h, Work& w, bool tp, double* X, int64_t ldx, int hb, double* R,
                  double* T, double* tau) {
  const int b = h->b;
  const int rowsh = tp ? hb : b;
  int ib = (rowsh > 512) ? 16 : std::min(32, h->ib);   // register panels hold 32 columns up to 512 rows
  if (b % ib) ib = 16;
  ib = std::min(ib, b);
  for (int c0 = 0; c0 < b; c0 += ib) {
    PanelArgs a{};
    a.mode = tp ? PANEL_TPQRT : PANEL_GEQRT;
    a.ib = ib;
    a.T = T + c0 + (int64_t)c0 * b;
    a.ldt = b;
    a.tau = tau + c0;
    if (tp) {
      a.h = hb;
      a.X = X + (int64_t)c0 * ldx;
      a.ldx = ldx;
      a.R = R + c0 + (int64_t)c0 * b;
      a.ldr = b;
    } else {
      a.h = b - c0;
      a.X = X + c0 + (int64_t)c0 * ldx;
      a.ldx = ldx;
    }
    P.panel(a);
    P.ops.back().flops = 2.0 * a.h * ib * ib;
    const int nt = b - c0 - ib;
    if (nt > 0) {
      P.panel_apply(a, nt);
      P.ops.back().flops = 4.0 * a.h * ib * nt + (double)ib * ib * nt;
    }
  }
  if (b > ib) {
    if (!tp)
      P.gemm(w.Wg, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, X, ldx, X, ldx, b,
             SEG_TRANS_A | SEG_A_UNIT_LOWER | SEG_B_UNIT_LOWER, DESC_LOWER_ONLY);
    else
      P.gemm(w.Wg, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, X, ldx, X, ldx, hb, SEG_TRANS_A,
             DESC_LOWER_ONLY);
    P.flush_gemm();
    if (b >= kTDoublingMin) {
      plan_t_doubling(P, w.Wg, b, T, b, b, ib, w.Wx2);
    } else {
      TBackArgs t{};
      t.n = b;
      t.ib = ib;
      t.G = w.Wg;
      t.ldg = b;
      t.tau = tau;
      t.T = T;
      t.ldt = b;
      P.tback(t);
      P.ops.back().flops = (double)b * b * b / 3.0;
    }
  }
}

enum Case { C_DDD, C_LDL, C_DLD, C_DLL, C_LLD, C_LLL };

// Tiled BLR-QR plan (Alg. 4, Section 3.4).
// Look-ahead: block column k runs on stream k % kStreams.  Before touching
// tile row i it waits for event E(i, k-1), recorded after column k-1 applied
// its reflector (i, k-1) to that tile row; so the TPQRT chains of
// neighbouring columns overlap while every tile sees its updates in the
// order of Alg. 4.
void plan_tiled(blr_matrix h, Plan& P, std::vector<Work>& works, int kend, bool fp32) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  const int ns = (int)works.size();
  auto ev = [&](int i, int k) { return i * q + k; };
  for (int k = 0; k < kend; ++k) {
    P.cur_stream = k % ns;
    P.cur_prio = k;
    Work& w = works[k % ns];
    if (k > 0) P.wait(ev(k, k - 1));
    Tile& Dkk = h->t(k, k);
    double* Tkk = h->T[(size_t)k * q + k];
    // GEQRT(k)
    plan_tile_qr(P, h, w, false, Dkk.D, b, b, nullptr, Tkk, h->tau[(size_t)k * q + k]);
    // LARFB(k, j > k): A_kj <- Qkk^T A_kj (dense tile or U of a low-rank tile)
    if (k + 1 < q) {
      for (int j = k + 1; j < q; ++j) {
        Tile& t = h->t(k, j);
        const bool d = t.fmt == DENSE;
        P.gemm(w.X[j], b, nullptr, 0, nullptr, 0, b, d ? b : rc, 1.0, 0.0, Dkk.D, b, d ? t.D : t.U, b, b,
               SEG_TRANS_A | SEG_A_UNIT_LOWER);
      }
      P.flush_gemm(fp32);
      for (int j = k + 1; j < q; ++j) {
        const bool d = h->t(k, j).fmt == DENSE;
        P.gemm(w.X2[j], b, nullptr, 0, nullptr, 0, b, d ? b : rc, 1.0, 0.0, Tkk, b, w.X[j], b, b,
               SEG_TRANS_A | SEG_A_UPPER);
      }
      P.flush_gemm(fp32);
      for (int j = k + 1; j < q; ++j) {
        Tile& t = h->t(k, j);
        const bool d = t.fmt == DENSE;
        double* C = d ? t.D : t.U;
        P.gemm(C, b, C, b, nullptr, 0, b, d ? b : rc, -1.0, 1.0, Dkk.D, b, w.X2[j], b, b, SEG_A_UNIT_LOWER);
      }
      P.flush_gemm(fp32);
    }
    for (int i = k + 1; i < p; ++i) {
      if (k > 0 && i > k) P.wait(ev(i, k - 1));
      Tile& Aik = h->t(i, k);
      const size_t ik = (size_t)i * q + k;
      double* Tik = h->T[ik];
      const bool yd = Aik.fmt == DENSE;
      h->yfmt[ik] = Aik.fmt;
      // TPQRT(i,k): QR of [R_kk; A_ik] (dense) or [R_kk; V_ik^T] (low-rank)
      if (yd)
        plan_tile_qr(P, h, w, true, Aik.D, b, b, Dkk.D, Tik, h->tau[ik]);
      else
        plan_tile_qr(P, h, w, true, Aik.Vt, rc, rc, Dkk.D, Tik, h->tau[ik]);
      if (k + 1 >= q) continue;
      struct Rec {
        Plan& P;
        int e;
        bool on;
        ~Rec() {
          if (on) P.record(e);
        }
      } rec{P, ev(i, k), k + 1 < kend};
      double* Y = Aik.D;     // dense reflector block
      double* UY = Aik.U;    // low-rank: Ytilde = UY * Yl
      double* Yl = Aik.Vt;   // rc x b
      // classify j, densify targets that OP1 turns dense
      std::vector<int> cs(q, -1);
      for (int j = k + 1; j < q; ++j) {
        Tile& R = h->t(k, j);
        Tile& A = h->t(i, j);
        if (yd && R.fmt == LOWRANK && A.fmt == DENSE) {
          P.gemm(R.D, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, R.U, b, R.Vt, rc, rc, 0);
          R.fmt = DENSE;
          h->n_fill++;
        }
        if (yd && R.fmt == DENSE && A.fmt == LOWRANK) {
          P.gemm(A.D, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, A.U, b, A.Vt, rc, rc, 0);
          A.fmt = DENSE;
          h->n_fill++;
        }
        const bool rd = R.fmt == DENSE, ad = A.fmt == DENSE;
        if (yd) cs[j] = (rd && ad) ? C_DDD : C_LDL;  // remaining dense-Y case has R and A low-rank
        else cs[j] = rd ? (ad ? C_DLD : C_DLL) : (ad ? C_LLD : C_LLL);
      }
      P.flush_gemm();
      // S1: pre-products
      for (int j = k + 1; j < q; ++j) {
        Tile& A = h->t(i, j);
        switch (cs[j]) {
          case C_LDL:
            P.gemm(w.PU[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Y, b, A.U, b, b, SEG_TRANS_A);
            break;
          case C_DLD:
          case C_LLD:
            P.gemm(w.S[j], rc, nullptr, 0, nullptr, 0, rc, b, 1.0, 0.0, UY, b, A.D, b, b, SEG_TRANS_A);
            break;
          case C_DLL:
          case C_LLL:
            P.gemm(w.G[j], rc, nullptr, 0, nullptr, 0, rc, rc, 1.0, 0.0, UY, b, A.U, b, b, SEG_TRANS_A);
            break;
          default:
            break;
        }
      }
      P.flush_gemm();
      for (int j = k + 1; j < q; ++j)
        if (cs[j] == C_DLL || cs[j] == C_LLL)
          P.gemm(w.PU[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Yl, rc, w.G[j], rc, rc, SEG_TRANS_A);
      P.flush_gemm();
      // S2: dense W0 = R + Ytilde^T A into X_j
      for (int j = k + 1; j < q; ++j) {
        Tile& R = h->t(k, j);
        Tile& A = h->t(i, j);
        if (cs[j] == C_DDD)
          P.gemm(w.X[j], b, R.D, b, nullptr, 0, b, b, 1.0, 1.0, Y, b, A.D, b, b, SEG_TRANS_A);
        else if (cs[j] == C_DLD)
          P.gemm(w.X[j], b, R.D, b, nullptr, 0, b, b, 1.0, 1.0, Yl, rc, w.S[j], rc, rc, SEG_TRANS_A);
        else if (cs[j] == C_DLL)
          P.gemm(w.X[j], b, R.D, b, nullptr, 0, b, b, 1.0, 1.0, w.PU[j], b, A.Vt, rc, rc, 0);
      }
      P.flush_gemm(fp32, 1);
      // RC1: low-rank W0 = R + Ytilde^T A (rounded addition)
      for (int j = k + 1; j < q; ++j) {
        Tile& R = h->t(k, j);
        Tile& A = h->t(i, j);
        if (cs[j] != C_LDL && cs[j] != C_LLD && cs[j] != C_LLL) continue;
        RcDesc d{};
        d.nterm = 2;
        d.t[0] = RcTerm{R.U, R.Vt, R.rank, b, rc, 0, 0, 1.0};
        if (cs[j] == C_LLD)
          d.t[1] = RcTerm{Yl, w.S[j], Aik.rank, rc, rc, 0, 1, 1.0};
        else
          d.t[1] = RcTerm{w.PU[j], A.Vt, A.rank, b, rc, 0, 0, 1.0};
        d.Uout = w.Uw[j];
        d.Vtout = w.Vtw[j];
        d.rank_out = w.rankw[j];
        d.work = w.rcw[2 * j];
        P.rc(d);
      }
      P.flush_rc();
      // S3: W = T^T W0; dense: R -= W (W kept in X2_j); low-rank: WU = T^T Uw
      for (int j = k + 1; j < q; ++j) {
        Tile& R = h->t(k, j);
        if (cs[j] == C_DDD || cs[j] == C_DLD || cs[j] == C_DLL)
          P.gemm(R.D, b, R.D, b, w.X2[j], b, b, b, -1.0, 1.0, Tik, b, w.X[j], b, b, SEG_TRANS_A | SEG_A_UPPER);
        else
          P.gemm(w.WU[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Tik, b, w.Uw[j], b, b,
                 SEG_TRANS_A | SEG_A_UPPER);
      }
      P.flush_gemm(fp32, 1);
      // S4a
      for (int j = k + 1; j < q; ++j) {
        Tile& A = h->t(i, j);
        switch (cs[j]) {
          case C_DDD:
            P.gemm(A.D, b, A.D, b, nullptr, 0, b, b, -1.0, 1.0, Y, b, w.X2[j], b, b, 0);
            break;
          case C_DLD:
          case C_DLL:
            P.gemm(w.S2[j], rc, nullptr, 0, nullptr, 0, rc, b, 1.0, 0.0, Yl, rc, w.X2[j], b, b, 0);
            break;
          case C_LDL:
            P.gemm(w.YWU[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Y, b, w.WU[j], b, b, 0);
            break;
          case C_LLD:
          case C_LLL:
            P.gemm(w.M1[j], rc, nullptr, 0, nullptr, 0, rc, rc, 1.0, 0.0, Yl, rc, w.WU[j], b, b, 0);
            break;
        }
      }
      P.flush_gemm(fp32, 1);
      // S4b
      for (int j = k + 1; j < q; ++j) {
        Tile& A = h->t(i, j);
        if (cs[j] == C_DLD)
          P.gemm(A.D, b, A.D, b, nullptr, 0, b, b, -1.0, 1.0, UY, b, w.S2[j], rc, rc, 0);
        else if (cs[j] == C_LLD || cs[j] == C_LLL)
          P.gemm(w.M2[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, UY, b, w.M1[j], rc, rc, 0);
      }
      P.flush_gemm();
      // S4c
      for (int j = k + 1; j < q; ++j) {
        Tile& A = h->t(i, j);
        if (cs[j] == C_LLD)
          P.gemm(A.D, b, A.D, b, nullptr, 0, b, b, -1.0, 1.0, w.M2[j], b, w.Vtw[j], rc, rc, 0);
      }
      P.flush_gemm();
      // RC2: low-rank targets R_kj -= W, A_ij -= Ytilde W
      for (int j = k + 1; j < q; ++j) {
        Tile& R = h->t(k, j);
        Tile& A = h->t(i, j);
        const int c = cs[j];
        if (c == C_LDL || c == C_LLD || c == C_LLL) {
          RcDesc d{};
          d.nterm = 2;
          d.t[0] = RcTerm{R.U, R.Vt, R.rank, b, rc, 0, 0, 1.0};
          d.t[1] = RcTerm{w.WU[j], w.Vtw[j], w.rankw[j], b, rc, 0, 0, -1.0};
          d.Uout = R.U;
          d.Vtout = R.Vt;
          d.rank_out = R.rank;
          d.work = w.rcw[2 * j];
          P.rc(d);
        }
        if (c == C_DLL || c == C_LDL || c == C_LLL) {
          RcDesc d{};
          d.nterm = 2;
          d.t[0] = RcTerm{A.U, A.Vt, A.rank, b, rc, 0, 0, 1.0};
          if (c == C_DLL)
            d.t[1] = RcTerm{UY, w.S2[j], Aik.rank, b, rc, 0, 0, -1.0};
          else if (c == C_LDL)
            d.t[1] = RcTerm{w.YWU[j], w.Vtw[j], w.rankw[j], b, rc, 0, 0, -1.0};
          else
            d.t[1] = RcTerm{w.M2[j], w.Vtw[j], w.rankw[j], b, rc, 0, 0, -1.0};
          d.Uout = A.U;
          d.Vtout = A.Vt;
          d.rank_out = A.rank;
          d.work = w.rcw[2 * j + 1];
          P.rc(d);
        }
      }
      P.flush_rc();
    }
  }
}

// B <- Q^T B (trans = 0) or Q B (trans = 1) for the tiled factor (Alg. 5,
// update read as C <- (I - [I; Y] T [I; Y]^T) C).
Plan merge_streams(const Plan& P, blr_matrix h);
void merge_streams_into(const Plan& P, blr_matrix h, Plan& M);

// Q^T B (trans 0) or Q B (trans 1) from the tiled factor's reflectors
// (Alg. 5).  Step k applies the GEQRT reflector of (k,k) to B_k and the
// TPQRT reflectors of (i,k), i > k, to [B_k; B_i]: for each i, in factor
// order for Q^T and reversed for Q, c_i = Ytilde_ik^T B_i, then
// W_i = op(T_ik) (B_k + c_i) and B_k -= W_i in one two-segment launch (B_k
// ping-ponged between two buffers, since every workgroup of the launch reads
// all of it), then B_i -= Ytilde_ik W_i.  Every step is planned as a chain
// of its own; before it touches row i it waits for the event the previous
// step (k - 1 for Q^T, k + 1 for Q) recorded when it was done with that row,
// so step k + 1 works on row i as soon as step k has updated it.  The chains
// are merged into one launch list (each round advances every ready chain by
// one op, batched by kernel and shape), as the tiled factor's are.  Chains
// k and k + ns share a stream and a workspace; ns is chosen so that the
// workspaces fit in `budget` bytes.
void plan_apply_tiled(blr_matrix h, Plan& P, double* B, int64_t ldb, int nrhs, int trans, DevAlloc& al,
                      size_t budget) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  const int K = h->steps_done;
  if (K <= 0) return;
  const size_t bn = (size_t)b * nrhs, rn = (size_t)rc * nrhs;
  const size_t per = (6 * bn + rn) * 8;
  const int ns = (int)std::max<size_t>(1, std::min<size_t>(std::min(K, 64), budget / per));
  struct ChainWork { double *Wx, *Wx2, *C, *W, *X, *Pb[2]; };
  std::vector<ChainWork> cw(ns);
  for (auto& c : cw) {
    c.Wx = (double*)al.alloc(bn * 8);
    c.Wx2 = (double*)al.alloc(bn * 8);
    c.C = (double*)al.alloc(bn * 8);
    c.W = (double*)al.alloc(bn * 8);
    c.X = (double*)al.alloc(rn * 8);
    c.Pb[0] = (double*)al.alloc(bn * 8);
    c.Pb[1] = (double*)al.alloc(bn * 8);
  }
  const int tflag = (trans ? 0 : SEG_TRANS_A) | SEG_A_UPPER;
  auto ev = [&](int i, int k) { return i * q + k; };   // step k is done with row i
  Plan L;
  auto diag = [&](int k, ChainWork& c) {
    Tile& Dkk = h->t(k, k);
    double* Tkk = h->T[(size_t)k * q + k];
    double* Bk = B + (int64_t)k * b;
    L.gemm(c.Wx, b, nullptr, 0, nullptr, 0, b, nrhs, 1.0, 0.0, Dkk.D, b, Bk, ldb, b, SEG_TRANS_A | SEG_A_UNIT_LOWER);
    L.flush_gemm();
    L.gemm(c.Wx2, b, nullptr, 0, nullptr, 0, b, nrhs, 1.0, 0.0, Tkk, b, c.Wx, b, b, tflag);
    L.flush_gemm();
    L.gemm(Bk, ldb, Bk, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, Dkk.D, b, c.Wx2, b, b, SEG_A_UNIT_LOWER);
    L.flush_gemm();
  };
  for (int t = 0; t < K; ++t) {
    const int k = trans ? K - 1 - t : t;
    const int prev = trans ? k + 1 : k - 1;
    const bool has_prev = t > 0;
    L.cur_stream = t % ns;
    L.cur_prio = t;
    ChainWork& c = cw[t % ns];
    double* Bk = B + (int64_t)k * b;
    if (!trans) {
      if (has_prev) L.wait(ev(k, prev));
      diag(k, c);
    }
    const double* src = Bk;
    int64_t lds = ldb;
    int x = 0;
    for (int r = 0; r < p - 1 - k; ++r) {
      const int i = trans ? p - 1 - r : k + 1 + r;
      if (has_prev) L.wait(ev(i, prev));
      const size_t ik = (size_t)i * q + k;
      const bool yd = h->yfmt[ik] == DENSE;
      Tile& Y = h->t(i, k);
      double* Bi = B + (int64_t)i * b;
      // c_i = Ytilde_ik^T B_i
      if (yd) {
        L.gemm(c.C, b, nullptr, 0, nullptr, 0, b, nrhs, 1.0, 0.0, Y.D, b, Bi, ldb, b, SEG_TRANS_A);
      } else {
        L.gemm(c.X, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, Y.U, b, Bi, ldb, b, SEG_TRANS_A);
        L.flush_gemm();
        L.gemm(c.C, b, nullptr, 0, nullptr, 0, b, nrhs, 1.0, 0.0, Y.Vt, rc, c.X, rc, rc, SEG_TRANS_A);
      }
      L.flush_gemm();
      // W_i = op(T_ik) (B_k + c_i); B_k -= W_i
      double* dst = c.Pb[x & 1];
      GemmSeg s0{}, s1{};
      s0.A = h->T[ik]; s0.lda = b; s0.B = src; s0.ldb = lds; s0.K = b; s0.flags = tflag;
      s1.A = h->T[ik]; s1.lda = b; s1.B = c.C; s1.ldb = b; s1.K = b; s1.flags = tflag;
      L.gemm_multi(dst, b, src, lds, b, nrhs, -1.0, 1.0, {s0, s1});
      L.cur.back().D2 = c.W;
      L.cur.back().ldd2 = b;
      L.flush_gemm();
      src = dst;
      lds = b;
      ++x;
      // B_i -= Ytilde_ik W_i
      if (yd) {
        L.gemm(Bi, ldb, Bi, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, Y.D, b, c.W, b, b, 0);
      } else {
        L.gemm(c.X, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, Y.Vt, rc, c.W, b, b, 0);
        L.flush_gemm();
        L.gemm(Bi, ldb, Bi, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, Y.U, b, c.X, rc, rc, 0);
      }
      L.flush_gemm();
      L.record(ev(i, k));
    }
    if (x > 0) L.copy({CopyDesc{src, Bk, (int64_t)b, ldb, b, nrhs, 0, 0, 0}});
    if (trans) diag(k, c);
    L.record(ev(k, k));
  }
  merge_streams_into(L, h, P);
}


// ---------------------------------------------------------------------------
// Block-column BLR-QR (Alg. 2 with Section 3.3).  Step k: gather the stack
// [A_kk; Av_{k+1,k}; ...] (Av = A for dense tiles, V^T for low-rank tiles)
// into one column-major buffer, take its Householder QR (the tile panel
// kernels while it has at most 512/1024 rows, the tall-panel kernels
// otherwise), build T_k, scatter R_kk and the reflector rows Y_ik back into
// the tiles, then for every j > k form Z_j = sum_i Ytilde_ik^T A_ij,
// W_j = T_k^T Z_j and apply A_ij -= Ytilde_ik W_j with the OP1/OP2 rules:
// Z_j is dense if any term is dense, else the low-rank terms are summed by
// rounded additions of two terms at a time in a pairwise tree.

constexpr int kGramSlices = 16;
constexpr int kApplySlices = 64;
constexpr int kZSlices = 16;

struct BcSlot {
  double *Ua, *Ub;   // b x rc
  double *Sa;        // rc x b
  double *Sm;        // rc x rc
  double *rcw;       // recompression workspace
  int* rank;         // rank of a partial sum of Z_j kept in (Ub, Sa)
};

struct BcWork {
  double* stack = nullptr;      // m x b
  double* Yf[2] = {nullptr, nullptr};  // b x b explicit unit-lower Y_kk (steps alternate)
  double* gpart = nullptr;      // kGramSlices x b x b split-K Gram partials
  int64_t gpart_doubles = 0;
  double* wblk = nullptr;       // 128 x b: W of a block reflector
  double* wblk2 = nullptr;      // 128 x b: T^T W
  double* wpart = nullptr;      // kApplySlices x 128 x b split-K partials of W
  double* zpart = nullptr;      // kZSlices x b x b partial sums of the look-ahead column's Z
  double* applypart = nullptr;  // kTallApplySlices x ceil(b/32) x 32 x 32
  double* tsqr = nullptr;       // tree buffers of a tall panel (tsqr_doubles)
  std::vector<BcSlot> slots;
};

// Leaves and tree levels of a tall panel of h rows (TsqrTree in qr.h).
int tsqr_levels(int64_t h, int* count) {
  int L = 0;
  count[0] = (int)((h + kTsqrRows - 1) / kTsqrRows);
  while (count[L] > 1) {
    if (L == kTsqrMaxLevels) throw Error(BLR_ERR_INVALID, "tall panel exceeds the tree depth");
    count[L + 1] = (count[L] + kTsqrFan - 1) / kTsqrFan;
    ++L;
  }
  return L;
}

// Doubles of the tree buffers for panels of up to h rows.
size_t tsqr_doubles(int64_t h) {
  int count[kTsqrMaxLevels + 1];
  const int L = tsqr_levels(h, count);
  constexpr size_t blk = (size_t)kTsqrIB * kTsqrIB;
  size_t n = 2 * (size_t)count[0] * blk;
  for (int l = 1; l <= L; ++l) n += ((size_t)count[l - 1] + count[l]) * blk;
  return n;
}

// QR of a tall panel (X: pivot of kTsqrIB columns, h rows, ld ldx) as a tree:
// one QR launch per level, then the reconstruction of the panel's
// reflectors, T (ld ldt) and tau.  buf holds tsqr_doubles(h) doubles.
void plan_tsqr(Plan& P, double* buf, double* X, int64_t ldx, int h, double* T, int64_t ldt, double* tau,
               double flops) {
  TsqrTree t{};
  t.X = X;
  t.ldx = ldx;
  t.h = h;
  t.T = T;
  t.ldt = ldt;
  t.tau = tau;
  const int L = tsqr_levels(h, t.count);
  t.levels = L;
  constexpr size_t blk = (size_t)kTsqrIB * kTsqrIB;
  double* p = buf;
  t.Y1 = p;
  p += (size_t)t.count[0] * blk;
  t.Tn[0] = p;
  p += (size_t)t.count[0] * blk;
  for (int l = 1; l <= L; ++l) {
    t.S[l] = p;
    p += (size_t)t.count[l - 1] * blk;
    t.Tn[l] = p;
    p += (size_t)t.count[l] * blk;
  }
  const int idx = (int)P.trees.size();
  P.trees.push_back(t);
  for (int l = 0; l <= L; ++l) {
    Op o;
    o.kind = Op::TSQR_QR;
    o.off = (int)P.titems.size();
    o.n = 1;
    o.ext = t.count[l];
    o.flops = (L == 0) ? flops : 0.0;
    P.titems.push_back(TsqrItem{idx, l, 0, 0});
    P.push(o);
  }
  if (L > 0) {
    Op o;
    o.kind = Op::TSQR_FIN;
    o.off = (int)P.titems.size();
    o.n = 1;
    o.ext = t.count[0];
    o.flops = flops;
    P.titems.push_back(TsqrItem{idx, 0, 0, 0});
    P.push(o);
  }
}

// Is Z_j = sum_{i >= i0} Ytilde_ik^T A_ij dense (some term dense: OP1)?  The
// Householder step sums from i0 = k, the Gram-Schmidt step from i0 = 0; the
// diagonal tile's block is dense in both.
bool bc_zdense(blr_matrix h, const std::vector<int8_t>& f, int k, int j, int i0) {
  const int q = h->q;
  for (int i = i0; i < h->p; ++i)
    if ((i == k || f[(size_t)i * q + k] == DENSE) && f[(size_t)i * q + j] == DENSE) return true;
  return false;
}
bool bc_zdense(blr_matrix h, const std::vector<int8_t>& f, int k, int j) { return bc_zdense(h, f, k, j, k); }

// Low-rank tiles that the block-column factorization turns dense (OP1): a
// low-rank A_ij receiving a dense update Ytilde_ik W_j.  Also returns the
// largest number of (i, j) pairs of one step that need low-rank temporaries.
// mgs: the Gram-Schmidt steps, which span every block row.
std::vector<int> bc_simulate(blr_matrix h, int kend, int* max_pairs, bool mgs = false) {
  const int p = h->p, q = h->q;
  std::vector<int8_t> f((size_t)p * q);
  for (size_t t = 0; t < f.size(); ++t) f[t] = h->tiles[t].fmt;
  std::vector<int> need;
  int mp = 0;
  for (int k = 0; k < kend; ++k) {
    const int i0 = mgs ? 0 : k;
    int pairs = 0;
    for (int j = k + 1; j < q; ++j) {
      const bool zd = bc_zdense(h, f, k, j, i0);
      for (int i = i0; i < p; ++i) {
        const bool yd = i == k || f[(size_t)i * q + k] == DENSE;
        int8_t& A = f[(size_t)i * q + j];
        if (!(yd && A == DENSE && zd)) pairs++;
        if (zd && yd && A == LOWRANK) {
          A = DENSE;
          need.push_back(i * q + j);
        }
      }
    }
    mp = std::max(mp, pairs);
  }
  *max_pairs = mp;
  return need;
}

BcWork make_bc_work(blr_matrix h, int npairs) {
  BcWork bw;
  const int b = h->b, rc = h->rc;
  Workspace& A = h->work;
  bw.stack = (double*)A.alloc((size_t)h->m * b * 8);
  bw.Yf[0] = (double*)A.alloc((size_t)b * b * 8);
  bw.Yf[1] = (double*)A.alloc((size_t)b * b * 8);
  bw.gpart_doubles = (int64_t)kGramSlices * b * b;
  bw.gpart = (double*)A.alloc((size_t)bw.gpart_doubles * 8);
  bw.wblk = (double*)A.alloc((size_t)128 * b * 8);
  bw.wblk2 = (double*)A.alloc((size_t)128 * b * 8);
  bw.wpart = (double*)A.alloc((size_t)kApplySlices * 128 * b * 8);
  bw.zpart = (double*)A.alloc((size_t)kZSlices * b * b * 8);
  bw.applypart = (double*)A.alloc((size_t)kTallApplySlices * ((b + 31) / 32) * 32 * 32 * 8);
  bw.tsqr = (double*)A.alloc(tsqr_doubles(h->m) * 8);
  const size_t rcwd = rc_work_doubles(b, rc);
  const size_t per = 2 * (size_t)b * rc + (size_t)rc * b + (size_t)rc * rc + rcwd;
  if (npairs > 0) {
    double* base = (double*)A.alloc((size_t)npairs * per * 8);
    int* ranks = (int*)A.alloc((size_t)npairs * sizeof(int));
    for (int a = 0; a < npairs; ++a) {
      double* x = base + (size_t)a * per;
      BcSlot sl;
      sl.Ua = x;
      sl.Ub = x + (size_t)b * rc;
      sl.Sa = x + 2 * (size_t)b * rc;
      sl.Sm = sl.Sa + (size_t)rc * b;
      sl.rcw = sl.Sm + (size_t)rc * rc;
      sl.rank = ranks + a;
      bw.slots.push_back(sl);
    }
  }
  return bw;
}

// Householder QR of the hs x b stack (ld hs) into T (b x b) and tau.
// Gram matrix G = Y^T Y (lower triangle valid) of the nw reflectors whose
// pivot is X (unit lower in the first nw rows, h rows, ld ldx).  The unit-
// lower top block goes to the masked kernel; the rows below it are split
// into slices of full products on the fast kernel so that tall stacks fill
// the chip; one reduction sums the parts.
void plan_gram(Plan& P, BcWork& bw, const double* X, int64_t ldx, int h, int nw, double* G, int64_t ldg) {
  const int rest = h - nw;
  // narrow blocks take more, shorter slices (the partial buffer holds
  // kGramSlices full-width Gram matrices)
  const int cap = (int)std::min<int64_t>(nw <= 256 ? 64 : kGramSlices, bw.gpart_doubles / ((int64_t)nw * nw));
  const int S = rest > 0 ? std::min(cap - 1, std::max(1, rest / (nw <= 256 ? 2048 : 4096))) : 0;
  const int ks = S > 0 ? ((rest + S - 1) / S + 15) / 16 * 16 : 0;
  const bool direct = S == 0;
  P.gemm(direct ? G : bw.gpart, direct ? ldg : nw, nullptr, 0, nullptr, 0, nw, nw, 1.0, 0.0, X, ldx, X, ldx, nw,
         SEG_TRANS_A | SEG_A_UNIT_LOWER | SEG_B_UNIT_LOWER, DESC_LOWER_ONLY);
  P.flush_gemm();
  int ns = 1;
  for (int r0 = nw; r0 < h; r0 += ks, ++ns) {
    const int kk = std::min(ks, h - r0);
    P.gemm(bw.gpart + (size_t)ns * nw * nw, nw, nullptr, 0, nullptr, 0, nw, nw, 1.0, 0.0, X + r0, ldx, X + r0, ldx,
           kk, SEG_TRANS_A);
  }
  P.flush_gemm();
  if (!direct) P.copy({CopyDesc{bw.gpart, G, (int64_t)nw, ldg, nw, nw, 0, ns, (int64_t)nw * nw}});
}

// T of the nw reflectors at X (into T, ld ldt; its ib x ib diagonal blocks
// already hold the panel kernels' T blocks): Gram matrix and back-substitution.
void plan_block_t(Plan& P, Work& w, BcWork& bw, const double* X, int64_t ldx, int h, int nw, int ib,
                  const double* tau, double* T, int64_t ldt) {
  plan_gram(P, bw, X, ldx, h, nw, w.Wg, nw);
  TBackArgs t{};
  t.n = nw;
  t.ib = ib;
  t.G = w.Wg;
  t.ldg = nw;
  t.tau = tau;
  t.T = T;
  t.ldt = ldt;
  P.tback(t);
  P.ops.back().flops = (double)nw * nw * nw / 3.0;
}

// C <- (I - Y T Y^T)^T C for the nw reflectors Y at X (h rows, unit lower
// in the first nw rows) and the nt columns C (same rows, ld ldx):
// W = Y^T C split over row slices (masked first slice, fast full products
// after it, one reduction), W2 = T^T W, C -= Y W2 (the unit-lower top block
// on the masked kernel, the rows below on the fast kernel).
void plan_block_apply(Plan& P, BcWork& bw, const double* X, double* C, int64_t ldx, int h, int nw, int nt,
                      const double* T, int64_t ldt) {
  // W = Y^T C: the unit-lower top block on the masked kernel, the rows below
  // in slices on the fast kernel, one reduction
  const int rest = h - nw;
  const int S = rest > 0 ? std::min(kApplySlices - 1, std::max(1, rest / 2048)) : 0;
  const int ks = S > 0 ? ((rest + S - 1) / S + 15) / 16 * 16 : 0;
  const bool direct = S == 0;
  P.gemm(direct ? bw.wblk : bw.wpart, nw, nullptr, 0, nullptr, 0, nw, nt, 1.0, 0.0, X, ldx, C, ldx, nw,
         SEG_TRANS_A | SEG_A_UNIT_LOWER);
  P.flush_gemm();
  int ns = 1;
  for (int r0 = nw; r0 < h; r0 += ks, ++ns) {
    const int kk = std::min(ks, h - r0);
    P.gemm(bw.wpart + (size_t)ns * nw * nt, nw, nullptr, 0, nullptr, 0, nw, nt, 1.0, 0.0, X + r0, ldx, C + r0, ldx,
           kk, SEG_TRANS_A);
  }
  P.flush_gemm();
  if (!direct) P.copy({CopyDesc{bw.wpart, bw.wblk, (int64_t)nw, (int64_t)nw, nw, nt, 0, ns, (int64_t)nw * nt}});
  P.gemm(bw.wblk2, nw, nullptr, 0, nullptr, 0, nw, nt, 1.0, 0.0, T, ldt, bw.wblk, nw, nw, SEG_TRANS_A | SEG_A_UPPER);
  P.flush_gemm();
  // rows [0, nw): unit-lower Y block; the rows below in a 128-multiple bulk and a ragged rest
  const int bulk = rest / 128 * 128;
  P.gemm(C, ldx, C, ldx, nullptr, 0, nw, nt, -1.0, 1.0, X, ldx, bw.wblk2, nw, nw, SEG_A_UNIT_LOWER);
  if (rest > bulk)
    P.gemm(C + nw + bulk, ldx, C + nw + bulk, ldx, nullptr, 0, rest - bulk, nt, -1.0, 1.0, X + nw + bulk, ldx,
           bw.wblk2, nw, nw, 0);
  P.flush_gemm();
  if (bulk > 0) {
    P.gemm(C + nw, ldx, C + nw, ldx, nullptr, 0, bulk, nt, -1.0, 1.0, X + nw, ldx, bw.wblk2, nw, nw, 0);
    P.flush_gemm();
  }
}

// Householder QR of the hs x b stack (ld hs) into T (b x b) and tau.
// Stacks of up to 512 (ib 32) or 1024 (ib 16) rows stay in the registers of
// the one-workgroup panel kernel.  Taller stacks: 16-column sub-panels
// factored as a tree (TSQR, a few launches each, with the Householder
// vectors reconstructed), each applied within its 128-column block by the
// split-K sub-panel update; each finished 128-column block is applied to the
// rest of the stack as a block reflector on the matrix cores.
void plan_stack_qr(Plan& P, blr_matrix h, Work& w, BcWork& bw, int hs, double* T, double* tau) {
  const int b = h->b;
  double* X = bw.stack;
  const bool tall = hs > 1024;
  int ib = (hs > 512 && !tall) ? 16 : std::min(32, h->ib);
  if (tall) ib = kTsqrIB;   // 16-column sub-panels factored as a tree of 256-row blocks
  if (b % ib) ib = 16;
  ib = std::min(ib, b);
  const int OB = (tall && b % 128 == 0) ? 128 : b;   // outer block of the tall path
  for (int o0 = 0; o0 < b; o0 += OB) {
    const int oend = std::min(b, o0 + OB);
    for (int c0 = o0; c0 < oend; c0 += ib) {
      const int hl = hs - c0;
      const int nt = (tall ? oend : b) - c0 - ib;
      PanelArgs a{};
      a.mode = PANEL_GEQRT;
      a.ib = ib;
      a.h = hl;
      a.X = X + c0 + (int64_t)c0 * hs;
      a.ldx = hs;
      a.T = T + c0 + (int64_t)c0 * b;
      a.ldt = b;
      a.tau = tau + c0;
      if (!tall) {
        P.panel(a);
        P.ops.back().flops = 2.0 * hl * ib * ib;
        if (nt > 0) {
          P.panel_apply(a, nt);
          P.ops.back().flops = 4.0 * hl * ib * nt;
        }
      } else {
        plan_tsqr(P, bw.tsqr, a.X, hs, hl, a.T, b, a.tau, 4.0 * hl * ib * ib);
        if (nt > 0) {
          Op o;
          o.kind = Op::TALL_APPLY;
          o.panel = a;
          o.ntiles = nt;
          o.n = std::min(kTallApplySlices, std::max(1, hl / 512));
          o.buf = bw.applypart;
          o.flops = 4.0 * hl * ib * nt;
          P.push(o);
        }
      }
    }
    const int ntr = b - oend;
    if (tall && OB < b && ntr > 0) {
      const int ho = hs - o0;
      double* Xo = X + o0 + (int64_t)o0 * hs;
      plan_block_t(P, w, bw, Xo, hs, ho, OB, ib, tau + o0, T + o0 + (int64_t)o0 * b, b);
      plan_block_apply(P, bw, Xo, Xo + (int64_t)OB * hs, hs, ho, OB, ntr, T + o0 + (int64_t)o0 * b, b);
    }
  }
  if (b > ib) plan_block_t(P, w, bw, X, hs, hs, b, ib, tau, T, b);
}

// Panel of block-column step k (Section 3.3.1): gather the stack
// [A_kk; Av_{k+1,k}; ...] (Av = A for dense tiles, V^T for low-rank tiles)
// into one column-major buffer, take its Householder QR (the tile panel
// kernels while it has at most 1024 rows, the tree (TSQR) kernels otherwise),
// build T_k and scatter R_kk and the reflector rows Y_ik back into the tiles,
// with an explicit unit-lower copy of Y_kk.
void plan_bc_panel(blr_matrix h, Plan& P, Work& w, BcWork& bw, int k) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  // 1. gather the stack
  std::vector<int64_t> off(p, 0);
  std::vector<int> rows(p, 0);
  std::vector<bool> yd(p, true);
  int hs = 0;
  for (int i = k; i < p; ++i) {
    yd[i] = i == k || h->t(i, k).fmt == DENSE;
    rows[i] = yd[i] ? b : rc;
    off[i] = hs;
    hs += rows[i];
  }
  std::vector<CopyDesc> cp;
  for (int i = k; i < p; ++i) {
    Tile& t = h->t(i, k);
    cp.push_back(CopyDesc{yd[i] ? t.D : t.Vt, bw.stack + off[i], yd[i] ? (int64_t)b : (int64_t)rc, (int64_t)hs,
                          rows[i], b, 0, 0});
  }
  P.copy(cp);
  // 2. Householder QR of the stack, T_k
  double* Tk = h->T[(size_t)k * q + k];
  double* tauk = h->tau[(size_t)k * q + k];
  plan_stack_qr(P, h, w, bw, hs, Tk, tauk);
  // 3. scatter R_kk / Y back, explicit unit-lower Y_kk
  cp.clear();
  for (int i = k; i < p; ++i) {
    Tile& t = h->t(i, k);
    cp.push_back(CopyDesc{bw.stack + off[i], yd[i] ? t.D : t.Vt, (int64_t)hs, yd[i] ? (int64_t)b : (int64_t)rc,
                          rows[i], b, 0, 0});
    if (i > k) h->yfmt[(size_t)i * q + k] = yd[i] ? DENSE : LOWRANK;
  }
  cp.push_back(CopyDesc{bw.stack, bw.Yf[k & 1], (int64_t)hs, (int64_t)b, b, b, 1, 0});
  P.copy(cp);
}

// The Gram-Schmidt form of a block-column step (the comparison method):
// store(j, dense, Zd, Zl) is called once the plan has formed R_kj = Z_j
// (dense in Zd, b x b, ld b; or low-rank in the slot term Zl) and plans its
// copy into R's tile before anything reuses the slot; for a low-rank R_kj it
// returns that tile as a term (U ld b, V^T ld rc), the W of the update.
struct BcGs {
  std::function<RcTerm(int, bool, const double*, const RcTerm&)> store;
};

// Trailing update of the columns j in [j0, j1) by the reflectors of step k
// (Section 3.3.2): Z_j = sum_i Ytilde_ik^T A_ij, W_j = T_k^T Z_j and
// A_ij -= Ytilde_ik W_j with the OP1/OP2 rules: Z_j is dense if any term is
// dense, else the low-rank terms are summed by rounded additions of two terms
// at a time in a pairwise tree over the order i = k, k+1, ...  Z and W are
// formed for every column first; the updates A_ij -= Ytilde_ik W_j then run
// for the columns below jsplit, mid() is called (the look-ahead hook), and
// the remaining columns follow.
void plan_bc_update(blr_matrix h, Plan& P, Work& w, BcWork& bw, int k, int j0, int j1, bool fp32,
                    int jsplit, const std::function<void()>& mid, const BcGs* gs) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  if (j0 >= j1) return;
  // the Householder step works on block rows i >= k with W = T_k^T Z; the
  // Gram-Schmidt step (gs) on every block row with W = Z (R_kj = Z_j)
  const int i0 = gs ? 0 : k;
  std::vector<bool> yd(p, true);
  for (int i = i0; i < p; ++i)
    if (i != k) yd[i] = h->yfmt[(size_t)i * q + k] == DENSE;
  double* Tk = gs ? nullptr : h->T[(size_t)k * q + k];
  auto Yd = [&](int i) -> double* { return i == k ? (gs ? h->t(k, k).D : bw.Yf[k & 1]) : h->t(i, k).D; };
  std::vector<bool> zd(q, false);
  std::vector<int8_t> f((size_t)p * q);
  for (size_t t = 0; t < f.size(); ++t) f[t] = h->tiles[t].fmt;
  for (int j = j0; j < j1; ++j) zd[j] = bc_zdense(h, f, k, j, i0);
  // slots for the pairs that need low-rank temporaries
  std::vector<int> slot((size_t)p * q, -1);
  int ns = 0;
  for (int j = j0; j < j1; ++j)
    for (int i = i0; i < p; ++i)
      if (!(yd[i] && h->t(i, j).fmt == DENSE && zd[j])) slot[(size_t)i * q + j] = ns++;
  if (ns > (int)bw.slots.size()) throw Error(BLR_ERR_DEVICE, "internal: block-column slot count");
  auto S = [&](int i, int j) -> BcSlot& { return bw.slots[slot[(size_t)i * q + j]]; };
  // 4a. pre-products of the low-rank terms
  for (int j = j0; j < j1; ++j)
    for (int i = i0; i < p; ++i) {
      Tile& A = h->t(i, j);
      Tile& Y = h->t(i, k);
      const bool ad = A.fmt == DENSE;
      if (yd[i] && ad) continue;
      BcSlot& sl = S(i, j);
      if (yd[i]) P.gemm(sl.Ua, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Yd(i), b, A.U, b, b, SEG_TRANS_A);
      else if (ad) P.gemm(sl.Sa, rc, nullptr, 0, nullptr, 0, rc, b, 1.0, 0.0, Y.U, b, A.D, b, b, SEG_TRANS_A);
      else P.gemm(sl.Sm, rc, nullptr, 0, nullptr, 0, rc, rc, 1.0, 0.0, Y.U, b, A.U, b, b, SEG_TRANS_A);
    }
  P.flush_gemm();
  for (int j = j0; j < j1; ++j)
    for (int i = i0; i < p; ++i)
      if (!yd[i] && h->t(i, j).fmt == LOWRANK) {
        BcSlot& sl = S(i, j);
        P.gemm(sl.Ua, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, h->t(i, k).Vt, rc, sl.Sm, rc, rc, SEG_TRANS_A);
      }
  P.flush_gemm();
  // 4b. dense Z_j: low-rank contributions, then the dense sum on top
  std::vector<bool> zlr(q, false);
  for (int j = j0; j < j1; ++j) {
    if (!zd[j]) continue;
    std::vector<GemmSeg> sv;
    for (int i = i0; i < p; ++i) {
      Tile& A = h->t(i, j);
      if (yd[i] && A.fmt == DENSE) continue;
      GemmSeg g{};
      if (A.fmt == LOWRANK) {
        g.A = S(i, j).Ua; g.lda = b; g.B = A.Vt; g.ldb = rc; g.K = rc; g.flags = 0;
      } else {
        g.A = h->t(i, k).Vt; g.lda = rc; g.B = S(i, j).Sa; g.ldb = rc; g.K = rc; g.flags = SEG_TRANS_A;
      }
      sv.push_back(g);
    }
    if (!sv.empty()) {
      P.gemm_multi(w.X[j], b, nullptr, 0, b, b, 1.0, 0.0, sv);
      zlr[j] = true;
    }
  }
  P.flush_gemm();
  std::vector<CopyDesc> zred;
#ifndef BLR_MIXED_ZCHUNK
#define BLR_MIXED_ZCHUNK 8
#endif
  // the mixed form's long Z_j sums (FP32 products, FP64 accumulation) go in
  // launches of at most BLR_MIXED_ZCHUNK tile rows, each adding into the
  // previous one's FP64 result: their workgroups, which hold every register
  // of a SIMD, then retire often enough for the look-ahead panel's kernels
  // to find free slots (the FP64 products, whose update stream is the
  // critical path, lose more to the extra launches than the panel gains)
  std::vector<std::vector<GemmSeg>> zlong;
  std::vector<int> zlong_j;
  for (int j = j0; j < j1; ++j) {
    if (!zd[j]) continue;
    std::vector<GemmSeg> sv;
    for (int i = i0; i < p; ++i) {
      Tile& A = h->t(i, j);
      if (!(yd[i] && A.fmt == DENSE)) continue;
      GemmSeg g{};
      g.A = Yd(i); g.lda = b; g.B = A.D; g.ldb = b; g.K = b; g.flags = SEG_TRANS_A;
      sv.push_back(g);
    }
    // a single column (the look-ahead column) is on the panels' critical
    // path: its sum over the stack is split into partial products so that it
    // finishes in a fraction of one long K sweep
    const int ng = (j1 - j0 == 1) ? std::min<int>((int)sv.size(), kZSlices - 1) : 1;
    if (ng <= 1) {
      if (fp32 && (int)sv.size() > BLR_MIXED_ZCHUNK) {
        zlong.push_back(sv);
        zlong_j.push_back(j);
        continue;
      }
      P.gemm_multi(w.X[j], b, zlr[j] ? w.X[j] : nullptr, b, b, b, 1.0, zlr[j] ? 1.0 : 0.0, sv);
      continue;
    }
    const int per = ((int)sv.size() + ng - 1) / ng;
    int nd = 0;
    if (zlr[j]) {   // the low-rank contributions already in X_j join the reduction as slice 0
      P.copy({CopyDesc{w.X[j], bw.zpart, (int64_t)b, (int64_t)b, b, b, 0, 0}});
      nd = 1;
    }
    for (int g0 = 0; g0 < (int)sv.size(); g0 += per, ++nd) {
      std::vector<GemmSeg> part(sv.begin() + g0, sv.begin() + std::min<int>((int)sv.size(), g0 + per));
      P.gemm_multi(bw.zpart + (size_t)nd * b * b, b, nullptr, 0, b, b, 1.0, 0.0, part);
    }
    zred.push_back(CopyDesc{bw.zpart, w.X[j], (int64_t)b, (int64_t)b, b, b, 0, nd, (int64_t)b * b});
  }
  P.flush_gemm(fp32, 1);
  if (!zlong.empty()) {
    const int S = BLR_MIXED_ZCHUNK;
    size_t smax = 0;
    for (auto& v : zlong) smax = std::max(smax, v.size());
    for (size_t c0 = 0; c0 < smax; c0 += S) {
      for (size_t x = 0; x < zlong.size(); ++x) {
        const auto& v = zlong[x];
        if (c0 >= v.size()) continue;
        const int j = zlong_j[x];
        std::vector<GemmSeg> part(v.begin() + c0, v.begin() + std::min(v.size(), c0 + S));
        const bool acc = c0 > 0 || zlr[j];
        P.gemm_multi(w.X[j], b, acc ? w.X[j] : nullptr, b, b, b, 1.0, acc ? 1.0 : 0.0, part);
      }
      P.flush_gemm(fp32, 1);
    }
  }
  if (!zred.empty()) P.copy(zred);
  // 4c. low-rank Z_j: rounded additions of two terms at a time in a pairwise
  // tree whose leaves are the terms in order i = k, k+1, ...: at stride
  // s = 1, 2, 4, ... term x absorbs term x + s (x a multiple of 2s).  The sum
  // goes to the slot of the left term (U into Ub, V^T into Sa, in place from
  // the second level on; the recompression reads its inputs before it writes),
  // so every level is one batch of independent problems.
  const int nt = p - i0;
  std::vector<std::vector<RcTerm>> tv(q);
  for (int j = j0; j < j1; ++j) {
    if (zd[j]) continue;
    tv[j].resize(nt);
    for (int x = 0; x < nt; ++x) {
      Tile& A = h->t(i0 + x, j);
      tv[j][x] = A.fmt == LOWRANK ? RcTerm{S(i0 + x, j).Ua, A.Vt, A.rank, b, rc, 0, 0, 1.0}
                                  : RcTerm{h->t(i0 + x, k).Vt, S(i0 + x, j).Sa, h->t(i0 + x, k).rank, rc, rc, 0, 1, 1.0};
    }
  }
  for (int st = 1; st < nt; st *= 2) {
    for (int j = j0; j < j1; ++j) {
      if (zd[j]) continue;
      for (int x = 0; x + st < nt; x += 2 * st) {
        BcSlot& sl = S(i0 + x, j);
        RcDesc d{};
        d.nterm = 2;
        d.t[0] = tv[j][x];
        d.t[1] = tv[j][x + st];
        d.Uout = sl.Ub;
        d.Vtout = sl.Sa;
        d.rank_out = sl.rank;
        d.work = sl.rcw;
        P.rc(d);
        tv[j][x] = RcTerm{sl.Ub, sl.Sa, sl.rank, b, rc, 0, 0, 1.0};
      }
    }
    P.flush_rc();
  }
  std::vector<RcTerm> zterm(q);
  for (int j = j0; j < j1; ++j)
    if (!zd[j]) zterm[j] = tv[j][0];
  // 5. W_j = T_k^T Z_j (Gram-Schmidt: W_j = Z_j, which is R_kj)
  if (!gs) {
    for (int j = j0; j < j1; ++j) {
      if (zd[j]) P.gemm(w.X2[j], b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, Tk, b, w.X[j], b, b, SEG_TRANS_A | SEG_A_UPPER);
      else P.gemm(w.WU[j], b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Tk, b, zterm[j].U, zterm[j].ldu, b,
                  SEG_TRANS_A | SEG_A_UPPER);
    }
    P.flush_gemm(fp32, 1);
  }
  std::vector<RcTerm> wterm(q);   // Gram-Schmidt: W_j = R_kj as stored in R
  if (gs)
    for (int j = j0; j < j1; ++j) wterm[j] = gs->store(j, zd[j], w.X[j], zterm[j]);
  auto Wd = [&](int j) -> double* { return gs ? w.X[j] : w.X2[j]; };
  auto WU = [&](int j) -> const double* { return gs ? wterm[j].U : w.WU[j]; };
  // stages 6-7 for the columns [ja, jb)
  auto apply_cols = [&](int ja, int jb) {
    if (ja >= jb) return;
    // 6. fill-in: low-rank targets of a dense update become dense (OP1)
    for (int j = ja; j < jb; ++j)
      for (int i = i0; i < p; ++i) {
        Tile& A = h->t(i, j);
        if (zd[j] && yd[i] && A.fmt == LOWRANK) {
          P.gemm(A.D, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, A.U, b, A.Vt, rc, rc, 0);
          A.fmt = DENSE;
          h->n_fill++;
        }
      }
    P.flush_gemm(fp32);
    // 7. updates A_ij -= Ytilde_ik W_j
    for (int j = ja; j < jb; ++j)
      for (int i = i0; i < p; ++i)
        if (yd[i] && zd[j])
          P.gemm(h->t(i, j).D, b, h->t(i, j).D, b, nullptr, 0, b, b, -1.0, 1.0, Yd(i), b, Wd(j), b, b, 0);
    P.flush_gemm(fp32, 1);
    for (int j = ja; j < jb; ++j)
      for (int i = i0; i < p; ++i) {
        if (yd[i] && zd[j]) continue;
        BcSlot& sl = S(i, j);
        if (!yd[i] && zd[j])
          P.gemm(sl.Sa, rc, nullptr, 0, nullptr, 0, rc, b, 1.0, 0.0, h->t(i, k).Vt, rc, Wd(j), b, b, 0);
        else if (yd[i])
          P.gemm(sl.Ub, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Yd(i), b, WU(j), b, b, 0);
        else
          P.gemm(sl.Sm, rc, nullptr, 0, nullptr, 0, rc, rc, 1.0, 0.0, h->t(i, k).Vt, rc, WU(j), b, b, 0);
      }
    P.flush_gemm();
    for (int j = ja; j < jb; ++j)
      for (int i = i0; i < p; ++i)
        if (!yd[i] && !zd[j]) {
          BcSlot& sl = S(i, j);
          P.gemm(sl.Ub, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, h->t(i, k).U, b, sl.Sm, rc, rc, 0);
        }
    P.flush_gemm();
    for (int j = ja; j < jb; ++j)
      for (int i = i0; i < p; ++i) {
        if (yd[i] && zd[j]) continue;
        Tile& A = h->t(i, j);
        BcSlot& sl = S(i, j);
        // the update as a low-rank product Uu Vu^T
        const double* Uu;
        const double* Vu;
        const int* ru;
        if (!yd[i] && zd[j]) { Uu = h->t(i, k).U; Vu = sl.Sa; ru = h->t(i, k).rank; }
        else if (gs) { Uu = sl.Ub; Vu = wterm[j].Vt; ru = wterm[j].rank_ptr; }
        else { Uu = sl.Ub; Vu = zterm[j].Vt; ru = zterm[j].rank_ptr; }
        if (A.fmt == DENSE) {
          P.gemm(A.D, b, A.D, b, nullptr, 0, b, b, -1.0, 1.0, Uu, b, Vu, rc, rc, 0);
        } else {
          RcDesc d{};
          d.nterm = 2;
          d.t[0] = RcTerm{A.U, A.Vt, A.rank, b, rc, 0, 0, 1.0};
          d.t[1] = RcTerm{Uu, Vu, ru, b, rc, 0, 0, -1.0};
          d.Uout = A.U;
          d.Vtout = A.Vt;
          d.rank_out = A.rank;
          d.work = sl.rcw;
          P.rc(d);
        }
      }
    P.flush_gemm(fp32);
    P.flush_rc();
  };
  apply_cols(j0, std::min(jsplit, j1));
  if (mid) mid();
  apply_cols(std::max(jsplit, j0), j1);
}

// Block-column BLR-QR (Alg. 2 with Section 3.3).  Look-ahead: stream 0 runs
// the trailing updates, stream 1 the panels.  Step k forms Z_j and W_j for
// every column, updates column k + 1 and records E_col(k); the panel of
// column k + 1 waits for it and runs beside the rest of step k's update
// (short-lived workgroups, so the panel's small launches find free compute
// units); step k + 1 waits for E_panel(k + 1).  The two steps' explicit
// Y_kk copies alternate between two buffers.
void plan_blockcol(blr_matrix h, Plan& P, Work& w, BcWork& bw, int kend, bool fp32, bool lookahead) {
  const int q = h->q;
  auto e_panel = [&](int k) { return k; };
  auto e_col = [&](int k) { return q + k; };
  const int ps = lookahead ? 1 : 0;
  if (kend <= 0) return;
  P.cur_stream = ps;
  plan_bc_panel(h, P, w, bw, 0);
  P.record(e_panel(0));
  for (int k = 0; k < kend; ++k) {
    P.cur_stream = 0;
    P.wait(e_panel(k));
    if (k + 1 >= q) continue;
    auto next_panel = [&]() {
      if (k + 1 >= kend) return;
      P.record(e_col(k));
      P.cur_stream = ps;
      P.wait(e_col(k));
      plan_bc_panel(h, P, w, bw, k + 1);
      P.record(e_panel(k + 1));
      P.cur_stream = 0;
    };
    // the look-ahead column gets a pass of its own when its Z is dense (a
    // short split product); a low-rank Z would add a second sequential chain
    // of rounded additions, so then one pass covers every column
    std::vector<int8_t> f((size_t)h->p * q);
    for (size_t t = 0; t < f.size(); ++t) f[t] = h->tiles[t].fmt;
    if (bc_zdense(h, f, k, k + 1)) {
      plan_bc_update(h, P, w, bw, k, k + 1, k + 2, fp32, k + 2, next_panel, nullptr);
      plan_bc_update(h, P, w, bw, k, k + 2, q, fp32, q, nullptr, nullptr);
    } else {
      plan_bc_update(h, P, w, bw, k, k + 1, q, fp32, k + 2, next_panel, nullptr);
    }
  }
  P.cur_stream = 0;
}

// ---------------------------------------------------------------------------
// Batched factorization of independent matrices (the task graph of Section
// 4.3 taken over many BLR matrices of uneven sizes).  Every matrix gets its
// own single-stream block-column plan; the plans are then merged into one
// launch list.  Each round launches, as one batched kernel, the next op of
// every matrix whose next op runs the same kernel with the same compile-time
// shape; the round takes the kernel whose matrices have the most ops left in
// total, so long factorizations keep moving while short ones ride along.  A
// matrix's ops keep their order and the batch runs on one stream, so every
// dependency of the single-matrix plan holds, and each job is computed
// exactly as by its own launch (bit-identical factors).

struct OpSig {
  int kind = -1, a = 0, b = 0, c = 0;
  bool operator==(const OpSig& o) const { return kind == o.kind && a == o.a && b == o.b && c == o.c; }
};

// register-tile template of the panel kernel: chunks of 64 rows, rounded up to 1, 2, 4, 8, 16
int panel_bucket(int h) {
  const int rs = (h + 63) / 64;
  int bk = 1;
  while (bk < rs) bk *= 2;
  return bk;
}

// false for ops that launch nothing (the waits and records of a one-stream plan)
bool op_launches(const Op& o) {
  switch (o.kind) {
    case Op::GEMM:
    case Op::RC: return o.n > 0;
    case Op::COPY: return o.n > 0 && o.maxel > 0;
    case Op::PANEL: return true;
    case Op::TSQR_QR:
    case Op::TSQR_FIN: return o.n > 0 && o.ext > 0;
    case Op::PANEL_APPLY: return o.n > 0;
    case Op::TBACK: return o.tback.n > o.tback.ib;
    case Op::TALL_APPLY: return o.ntiles > 0;
    case Op::TRSM: return o.trsm.n > 0 && o.trsm.nrhs > 0;
    case Op::LINCOMB: return o.n > 0 && o.maxel > 0;
    case Op::FROB2: return o.n > 0;
    case Op::WAIT:
    case Op::RECORD: return false;
    default: throw Error(BLR_ERR_INVALID, "op kind cannot be batched");
  }
}

OpSig op_sig(const Op& o) {
  OpSig g;
  g.kind = (int)o.kind;
  switch (o.kind) {
    case Op::GEMM: g.a = o.big; g.b = o.fp32; g.c = o.prof; break;
    case Op::PANEL: g.a = o.panel.ib; g.b = panel_bucket(o.panel.h); break;
    case Op::PANEL_APPLY:
    case Op::TALL_APPLY: g.a = o.panel.ib; break;
    case Op::TRSM: g.a = o.n; break;
    default: break;
  }
  return g;
}

// One merged op from the ops src[a] = (plan, op index), all of one signature.
void emit_merged(Plan& M, const std::vector<const Plan*>& plans, const std::vector<blr_matrix>& hs,
                 const std::vector<std::pair<int, int>>& src) {
  const Op& o0 = plans[src[0].first]->ops[src[0].second];
  Op m;
  m.kind = o0.kind;
  m.stream = 0;
  const bool single = src.size() == 1;
  auto job = [&](PanelJob j) { M.jobs.push_back(j); };
  switch (o0.kind) {
    case Op::GEMM:
      m.big = o0.big;
      m.fp32 = o0.fp32;
      m.prof = o0.prof;
      m.off = (int)M.descs.size();
      for (auto& sp : src) {
        const Plan& S = *plans[sp.first];
        const Op& o = S.ops[sp.second];
        for (int d = o.off; d < o.off + o.n; ++d) {
          GemmDesc e = S.descs[d];
          const int sb = e.seg_begin;
          e.seg_begin = (int)M.segs.size();
          M.segs.insert(M.segs.end(), S.segs.begin() + sb, S.segs.begin() + sb + e.nseg);
          e.tile_begin += m.ntiles;
          M.descs.push_back(e);
        }
        m.n += o.n;
        m.ntiles += o.ntiles;
        m.flops += o.flops;
      }
      break;
    case Op::RC:
      m.off = (int)M.rcs.size();
      for (auto& sp : src) {
        const Plan& S = *plans[sp.first];
        const Op& o = S.ops[sp.second];
        for (int d = o.off; d < o.off + o.n; ++d) {
          RcDesc e = S.rcs[d];
          e.counters = hs[sp.first]->d_counters;
          M.rcs.push_back(e);
        }
        m.n += o.n;
        m.flops += o.flops;
      }
      break;
    case Op::COPY:
      m.off = (int)M.copies.size();
      for (auto& sp : src) {
        const Plan& S = *plans[sp.first];
        const Op& o = S.ops[sp.second];
        M.copies.insert(M.copies.end(), S.copies.begin() + o.off, S.copies.begin() + o.off + o.n);
        m.n += o.n;
        m.maxel = std::max(m.maxel, o.maxel);
      }
      break;
    case Op::LINCOMB:
      m.off = (int)M.lincs.size();
      for (auto& sp : src) {
        const Plan& S = *plans[sp.first];
        const Op& o = S.ops[sp.second];
        M.lincs.insert(M.lincs.end(), S.lincs.begin() + o.off, S.lincs.begin() + o.off + o.n);
        m.n += o.n;
        m.maxel = std::max(m.maxel, o.maxel);
      }
      break;
    case Op::FROB2:
      m.off = (int)M.frobs.size();
      for (auto& sp : src) {
        const Plan& S = *plans[sp.first];
        const Op& o = S.ops[sp.second];
        M.frobs.insert(M.frobs.end(), S.frobs.begin() + o.off, S.frobs.begin() + o.off + o.n);
        m.n += o.n;
      }
      break;
    case Op::TSQR_QR:
    case Op::TSQR_FIN: {
      // the items' trees are copied into the merged plan; workgroups are
      // numbered across all items
      m.off = (int)M.titems.size();
      int wg = 0;
      for (auto& sp : src) {
        const Plan& pl = *plans[sp.first];
        const Op& o = pl.ops[sp.second];
        for (int x = 0; x < o.n; ++x) {
          TsqrItem it = pl.titems[(size_t)o.off + x];
          M.trees.push_back(pl.trees[it.tree]);
          it.tree = (int)M.trees.size() - 1;
          it.wg_begin = wg;
          wg += o0.kind == Op::TSQR_QR ? M.trees.back().count[it.level] : M.trees.back().count[0];
          M.titems.push_back(it);
          m.n += 1;
        }
        m.flops += o.flops;
      }
      m.ext = wg;
      break;
    }
    case Op::TRSM:
      if (single) {
        m = o0;
        m.stream = 0;
        break;
      }
      m.kind = Op::TRSM_B;
      m.first = o0.n;   // transposed solves
      m.off = (int)M.tjobs.size();
      for (auto& sp : src) {
        const Op& o = plans[sp.first]->ops[sp.second];
        M.tjobs.push_back(o.trsm);
        m.n += 1;
        m.ext = std::max(m.ext, o.trsm.nrhs);
      }
      break;
    default: {
      if (single) {   // one job: the single-problem kernel
        m = o0;
        m.stream = 0;
        break;
      }
      m.off = (int)M.jobs.size();
      for (auto& sp : src) {
        const Op& o = plans[sp.first]->ops[sp.second];
        PanelJob j{};
        switch (o.kind) {
          case Op::PANEL:
            m.kind = Op::PANEL_B;
            j.a = o.panel;
            m.ib = o.panel.ib;
            m.ext = std::max(m.ext, o.panel.h);
            break;
          case Op::PANEL_APPLY:
            m.kind = Op::PANEL_APPLY_B;
            j.a = o.panel;
            j.nt = o.n;
            m.ib = o.panel.ib;
            m.ext = std::max(m.ext, o.n);
            break;
          case Op::TBACK:
            m.kind = Op::TBACK_B;
            j.tb = o.tback;
            m.ext = std::max(m.ext, o.tback.n);
            break;
          case Op::TALL_APPLY:
            m.kind = Op::TALL_APPLY_B;
            j.a = o.panel;
            j.nt = o.ntiles;
            j.groups = o.n;
            j.part = o.buf;
            m.ib = o.panel.ib;
            m.ext = std::max(m.ext, o.ntiles);
            m.ext2 = std::max(m.ext2, o.n);
            break;
          default:
            throw Error(BLR_ERR_INVALID, "op kind cannot be batched");
        }
        job(j);
        m.n += 1;
        m.flops += o.flops;
      }
      break;
    }
  }
  M.ops.push_back(m);
}

Plan merge_plans(const std::vector<Plan>& plans, const std::vector<blr_matrix>& hs) {
  const int nb = (int)plans.size();
  std::vector<std::vector<int>> chain(nb);
  for (int i = 0; i < nb; ++i)
    for (int x = 0; x < (int)plans[i].ops.size(); ++x) {
      const Op& o = plans[i].ops[x];
      if (o.stream != 0) throw Error(BLR_ERR_INVALID, "batched plans run on one stream");
      if (op_launches(o)) chain[i].push_back(x);
    }
  std::vector<size_t> head(nb, 0);
  std::vector<OpSig> hsig(nb);
  for (int i = 0; i < nb; ++i)
    if (!chain[i].empty()) hsig[i] = op_sig(plans[i].ops[chain[i][0]]);
  Plan M;
  std::vector<const Plan*> pp(nb);
  for (int i = 0; i < nb; ++i) pp[i] = &plans[i];
  std::vector<std::pair<OpSig, int64_t>> score;
  std::vector<std::pair<int, int>> src;
  for (;;) {
    score.clear();
    for (int i = 0; i < nb; ++i) {
      if (head[i] >= chain[i].size()) continue;
      const int64_t left = (int64_t)(chain[i].size() - head[i]);
      bool found = false;
      for (auto& e : score)
        if (e.first == hsig[i]) {
          e.second += left;
          found = true;
          break;
        }
      if (!found) score.push_back({hsig[i], left});
    }
    if (score.empty()) break;
    size_t best = 0;
    for (size_t e = 1; e < score.size(); ++e)
      if (score[e].second > score[best].second) best = e;
    const OpSig g = score[best].first;
    src.clear();
    for (int i = 0; i < nb; ++i)
      if (head[i] < chain[i].size() && hsig[i] == g) src.push_back({i, chain[i][head[i]]});
    emit_merged(M, pp, hs, src);
    for (auto& sp : src) {
      const int i = sp.first;
      if (++head[i] < chain[i].size()) hsig[i] = op_sig(plans[i].ops[chain[i][head[i]]]);
    }
  }
  return M;
}

// One launch list from a plan on several streams (the tiled factor's task
// graph): each stream's ops form a chain, and a wait on an event holds its
// chain until the op recording that event has been reached in the recording
// chain.  Each round advances every chain whose head is ready by one op: the
// ready ops are grouped by kernel and shape, and each group is one batched
// launch, the group holding the oldest block column (the critical path)
// first.  Rounds run in order on one stream, so every dependency of the plan
// holds, and every job is computed exactly as by its own launch.
Plan merge_streams(const Plan& P, blr_matrix h) {
  Plan M;
  merge_streams_into(P, h, M);
  return M;
}

// merge_streams appending the merged ops to M (whose own ops come first).
void merge_streams_into(const Plan& P, blr_matrix h, Plan& M) {
  if (!M.cur.empty()) throw Error(BLR_ERR_DEVICE, "internal: merge into a plan with an unflushed product");
  int ns = 1;
  for (const Op& o : P.ops) ns = std::max(ns, o.stream + 1);
  std::vector<std::vector<int>> chain(ns);
  for (int x = 0; x < (int)P.ops.size(); ++x) {
    const Op& o = P.ops[x];
    if (o.kind == Op::WAIT || o.kind == Op::RECORD || op_launches(o)) chain[o.stream].push_back(x);
  }
  std::vector<size_t> head(ns, 0);
  std::vector<char> rec(std::max(P.n_events, 1), 0);
  const std::vector<const Plan*> pp{&P};
  const std::vector<blr_matrix> hv{h};
  std::vector<std::pair<int, int>> src;
  std::vector<int> ready;
  for (;;) {
    // pass records and satisfied waits until nothing moves
    bool moved = true;
    while (moved) {
      moved = false;
      for (int c = 0; c < ns; ++c)
        while (head[c] < chain[c].size()) {
          const Op& o = P.ops[chain[c][head[c]]];
          if (o.kind == Op::RECORD) {
            rec[o.event] = 1;
          } else if (o.kind == Op::WAIT) {
            if (!rec[o.event]) break;
          } else {
            break;
          }
          ++head[c];
          moved = true;
        }
    }
    // the ready heads, grouped by kernel and shape, oldest group first
    ready.clear();
    bool blocked = false;
    for (int c = 0; c < ns; ++c) {
      if (head[c] >= chain[c].size()) continue;
      const Op& o = P.ops[chain[c][head[c]]];
      if (o.kind == Op::WAIT) blocked = true;
      else ready.push_back(c);
    }
    if (ready.empty()) {
      if (blocked) throw Error(BLR_ERR_DEVICE, "internal: merged plan waits on an event never recorded");
      break;
    }
    std::sort(ready.begin(), ready.end(), [&](int a, int b2) {
      const int pa = P.ops[chain[a][head[a]]].prio, pb = P.ops[chain[b2][head[b2]]].prio;
      return pa < pb || (pa == pb && a < b2);
    });
    std::vector<char> done(ready.size(), 0);
    for (size_t r = 0; r < ready.size(); ++r) {
      if (done[r]) continue;
      const OpSig g = op_sig(P.ops[chain[ready[r]][head[ready[r]]]]);
      src.clear();
      for (size_t t = r; t < ready.size(); ++t)
        if (!done[t] && op_sig(P.ops[chain[ready[t]][head[ready[t]]]]) == g) {
          src.push_back({0, chain[ready[t]][head[ready[t]]]});
          done[t] = 1;
        }
      emit_merged(M, pp, hv, src);
    }
    for (int c : ready) ++head[c];
  }
}

// Run the one-stream plans of independent matrices as a batch.  The members
// are split into two groups of about equal work (largest first, each to the
// lighter group; an op counts as its flops plus 2e8 for its launch latency);
// each group's plans are merged and the two launch lists are enqueued
// interleaved on two streams of hv[0], joined to s before and after, so that
// one group's panel and solve kernels overlap the other group's products.
// Launches are counted on hv[0].
void run_batch_plans(std::vector<Plan>& plans, const std::vector<blr_matrix>& hv, hipStream_t s) {
  const int nb = (int)plans.size();
  if (nb == 0) return;
  const int ng = nb >= 2 ? 2 : 1;
  std::vector<std::pair<double, int>> wt(nb);
  for (int i = 0; i < nb; ++i) {
    double w = 0.0;
    for (const Op& o : plans[i].ops) w += o.flops + 2e8;
    wt[i] = {w, i};
  }
  std::sort(wt.begin(), wt.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  std::vector<std::vector<int>> grp(ng);
  std::vector<double> load(ng, 0.0);
  for (auto& e : wt) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    grp[g].push_back(e.second);
    load[g] += e.first;
  }
  std::vector<Plan> M(ng);
  for (int g = 0; g < ng; ++g) {
    std::sort(grp[g].begin(), grp[g].end());
    std::vector<Plan> gp;
    std::vector<blr_matrix> gh;
    for (int i : grp[g]) {
      gp.push_back(std::move(plans[i]));
      gh.push_back(hv[i]);
    }
    M[g] = merge_plans(gp, gh);
    M[g].upload(gh[0]->work, gh[0]->keep, s);
  }
  blr_matrix h0 = hv[0];
  std::vector<hipEvent_t> none;
  if (ng == 1) {
    for (const Op& o : M[0].ops) enqueue(h0, M[0], o, s, false, none);
    return;
  }
  ensure_streams(h0);
  hipStream_t st[2] = {h0->streams[0], h0->streams[1]};
  hipEvent_t join;
  HIPCHECK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(join, s));
  for (int g = 0; g < 2; ++g) HIPCHECK(hipStreamWaitEvent(st[g], join, 0));
  HIPCHECK(hipEventDestroy(join));
  // interleave in proportion to the two lists' lengths
  const size_t n0 = M[0].ops.size(), n1 = M[1].ops.size();
  size_t a = 0, b = 0;
  while (a < n0 || b < n1) {
    const bool take0 = b >= n1 || (a < n0 && (double)a * (double)n1 <= (double)b * (double)n0);
    if (take0) enqueue(h0, M[0], M[0].ops[a++], st[0], false, none);
    else enqueue(h0, M[1], M[1].ops[b++], st[1], false, none);
  }
  for (int g = 0; g < 2; ++g) {
    hipEvent_t e;
    HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(e, st[g]));
    HIPCHECK(hipStreamWaitEvent(s, e, 0));
    HIPCHECK(hipEventDestroy(e));
  }
}

// B <- Q^T B or Q B for the block-column factor (Alg. 3): per step k,
// W = sum_i Ytilde_ik^T B_i, W = T_k^T W (or T_k W), B_i -= Ytilde_ik W.
void plan_apply_blockcol(blr_matrix h, Plan& P, Work& w, double* B, int64_t ldb, int nrhs, int trans,
                         double* Sbuf, double* Wpart) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  const int K = h->steps_done;
  auto step = [&](int k) {
    double* Tk = h->T[(size_t)k * q + k];
    for (int i = k + 1; i < p; ++i)
      if (h->yfmt[(size_t)i * q + k] == LOWRANK)
        P.gemm(Sbuf + (size_t)i * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, h->t(i, k).U, b,
               B + (int64_t)i * b, ldb, b, SEG_TRANS_A);
    P.flush_gemm();
    std::vector<GemmSeg> sv;
    for (int i = k; i < p; ++i) {
      GemmSeg g{};
      if (i == k) {
        g.A = h->t(k, k).D; g.lda = b; g.B = B + (int64_t)k * b; g.ldb = ldb; g.K = b;
        g.flags = SEG_TRANS_A | SEG_A_UNIT_LOWER;
      } else if (h->yfmt[(size_t)i * q + k] == DENSE) {
        g.A = h->t(i, k).D; g.lda = b; g.B = B + (int64_t)i * b; g.ldb = ldb; g.K = b; g.flags = SEG_TRANS_A;
      } else {
        g.A = h->t(i, k).Vt; g.lda = rc; g.B = Sbuf + (size_t)i * rc * nrhs; g.ldb = rc; g.K = rc;
        g.flags = SEG_TRANS_A;
      }
      sv.push_back(g);
    }
    // the sum over the block column's tiles in up to kApplySlices groups
    // (one partial product each, then one reduction), so that a few
    // right-hand sides still fill the chip
    const int ng = std::min<int>((int)sv.size(), kApplySlices);
    if (ng <= 1) {
      P.gemm_multi(w.Wx, b, nullptr, 0, b, nrhs, 1.0, 0.0, sv);
      P.flush_gemm();
    } else {
      const int per = ((int)sv.size() + ng - 1) / ng;
      int nd = 0;
      for (int g0 = 0; g0 < (int)sv.size(); g0 += per, ++nd) {
        std::vector<GemmSeg> part(sv.begin() + g0, sv.begin() + std::min<int>((int)sv.size(), g0 + per));
        P.gemm_multi(Wpart + (size_t)nd * b * nrhs, b, nullptr, 0, b, nrhs, 1.0, 0.0, part);
      }
      P.flush_gemm();
      P.copy({CopyDesc{Wpart, w.Wx, (int64_t)b, (int64_t)b, b, nrhs, 0, nd, (int64_t)b * nrhs}});
    }
    P.gemm(w.Wx2, b, nullptr, 0, nullptr, 0, b, nrhs, 1.0, 0.0, Tk, b, w.Wx, b, b,
           (trans ? 0 : SEG_TRANS_A) | SEG_A_UPPER);
    P.flush_gemm();
    for (int i = k; i < p; ++i) {
      double* Bi = B + (int64_t)i * b;
      if (i == k)
        P.gemm(Bi, ldb, Bi, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, h->t(k, k).D, b, w.Wx2, b, b, SEG_A_UNIT_LOWER);
      else if (h->yfmt[(size_t)i * q + k] == DENSE)
        P.gemm(Bi, ldb, Bi, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, h->t(i, k).D, b, w.Wx2, b, b, 0);
      else
        P.gemm(Sbuf + (size_t)i * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, h->t(i, k).Vt, rc,
               w.Wx2, b, b, 0);
    }
    P.flush_gemm();
    for (int i = k + 1; i < p; ++i)
      if (h->yfmt[(size_t)i * q + k] == LOWRANK) {
        double* Bi = B + (int64_t)i * b;
        P.gemm(Bi, ldb, Bi, ldb, nullptr, 0, b, nrhs, -1.0, 1.0, h->t(i, k).U, b, Sbuf + (size_t)i * rc * nrhs, rc,
               rc, 0);
      }
    P.flush_gemm();
  };
  if (!trans)
    for (int k = 0; k < K; ++k) step(k);
  else
    for (int k = K - 1; k >= 0; --k) step(k);
}

// Q^T B or Q B; the block-column form's temporaries come from a (the
// handle's workspace by default).
void plan_apply(blr_matrix h, Plan& P, Work& w, double* B, int64_t ldb, int nrhs, int trans,
                DevAlloc* a = nullptr) {
  DevAlloc& al = a ? *a : h->work;
  if (h->variant == BLR_BLOCK_COLUMN) {
    double* S = (double*)al.alloc((size_t)h->p * h->rc * std::max(nrhs, 1) * 8);
    double* Wpart = (double*)al.alloc((size_t)kApplySlices * h->b * std::max(nrhs, 1) * 8);
    plan_apply_blockcol(h, P, w, B, ldb, nrhs, trans, S, Wpart);
  } else {
    // without a caller's allocator the chains' workspaces may take up to
    // 256 MiB of the handle's workspace; the no-allocation entry keeps them
    // within 16 MiB of its static scratch
    plan_apply_tiled(h, P, B, ldb, nrhs, trans, al, a ? (16u << 20) : (256u << 20));
  }
}

// The part of a Work that plan_apply uses: Wx, Wx2 (b x nrhs) and X[0]
// (rc x nrhs), from a.
Work make_apply_work(blr_matrix h, DevAlloc& a, int nrhs) {
  Work w;
  const size_t cols = (size_t)std::max(nrhs, 1);
  w.Wx = (double*)a.alloc((size_t)h->b * cols * 8);
  w.Wx2 = (double*)a.alloc((size_t)h->b * cols * 8);
  w.Wg = nullptr;
  w.X.push_back((double*)a.alloc((size_t)h->rc * cols * 8));
  return w;
}

// Products with the stored matrix (eq. blr_matrix_def): A~ X, A~^T X (the
// tiles before the factorization, or the copy a factor with keep_a kept) and
// R X (eq. qr_fact; the upper triangles of the diagonal tiles and the R_kj
// tiles).  Dense tiles multiply directly, low-rank ones through the small
// products V^T X or U^T X; one multi-segment descriptor per block row.
void plan_matmul(blr_matrix h, Plan& P, int op, const double* X, int64_t ldx, double* Y, int64_t ldy, int nrhs) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  std::vector<Tile>& T = (op == BLR_MATMUL_R || h->state == BLR_STATE_COMPRESSED) ? h->tiles : h->acopy;
  auto tile = [&](int i, int j) -> Tile& { return T[(size_t)i * q + j]; };
  const int rows = op == BLR_MATMUL_R ? q : p;
  std::vector<int> slot((size_t)p * q, -1);
  int nlr = 0;
  for (int i = 0; i < rows; ++i)
    for (int j = (op == BLR_MATMUL_R ? i + 1 : 0); j < q; ++j)
      if (tile(i, j).fmt == LOWRANK) slot[(size_t)i * q + j] = nlr++;
  double* S = (double*)h->work.alloc((size_t)std::max(nlr, 1) * rc * nrhs * 8);
  double* Dg = nullptr;
  if (op == BLR_MATMUL_R) {
    Dg = (double*)h->work.alloc((size_t)q * b * b * 8);
    std::vector<CopyDesc> cp;
    for (int k = 0; k < q; ++k)
      cp.push_back(CopyDesc{tile(k, k).D, Dg + (size_t)k * b * b, (int64_t)b, (int64_t)b, b, b, 2, 0});
    P.copy(cp);
  }
  auto Sp = [&](int i, int j) { return S + (size_t)slot[(size_t)i * q + j] * rc * nrhs; };
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < q; ++j) {
      if (slot[(size_t)i * q + j] < 0) continue;
      Tile& t = tile(i, j);
      if (op == BLR_MATMUL_AT)
        P.gemm(Sp(i, j), rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.U, b, X + (int64_t)i * b, ldx, b,
               SEG_TRANS_A);
      else
        P.gemm(Sp(i, j), rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.Vt, rc, X + (int64_t)j * b, ldx, b, 0);
    }
  P.flush_gemm(0, 0, false);
  const int outs = op == BLR_MATMUL_A ? p : q;
  for (int o = 0; o < outs; ++o) {
    std::vector<GemmSeg> sv;
    if (op == BLR_MATMUL_AT) {
      for (int i = 0; i < p; ++i) {
        Tile& t = tile(i, o);
        GemmSeg g{};
        if (t.fmt == DENSE) {
          g.A = t.D; g.lda = b; g.B = X + (int64_t)i * b; g.ldb = ldx; g.K = b; g.flags = SEG_TRANS_A;
        } else {
          g.A = t.Vt; g.lda = rc; g.B = Sp(i, o); g.ldb = rc; g.K = rc; g.flags = SEG_TRANS_A;
        }
        sv.push_back(g);
      }
    } else {
      for (int j = (op == BLR_MATMUL_R ? o : 0); j < q; ++j) {
        Tile& t = tile(o, j);
        GemmSeg g{};
        if (op == BLR_MATMUL_R && j == o) {
          g.A = Dg + (size_t)o * b * b; g.lda = b; g.B = X + (int64_t)j * b; g.ldb = ldx; g.K = b; g.flags = 0;
        } else if (t.fmt == DENSE) {
          g.A = t.D; g.lda = b; g.B = X + (int64_t)j * b; g.ldb = ldx; g.K = b; g.flags = 0;
        } else {
          g.A = t.U; g.lda = b; g.B = Sp(o, j); g.ldb = rc; g.K = rc; g.flags = 0;
        }
        sv.push_back(g);
      }
    }
    P.gemm_multi(Y + (int64_t)o * b, ldy, nullptr, 0, b, nrhs, 1.0, 0.0, sv);
  }
  P.flush_gemm(0, 0, false);
}

// Block back-substitution X <- R^{-1} X (trans = 0) or forward substitution
// X <- R^{-T} X (trans = 1) through the BLR factor R, in place on the n x nrhs
// block X: per block row, the off-diagonal tiles' contributions as one
// multi-segment product (low-rank tiles through V^T X_j or U^T X_j), then a
// triangular solve with the diagonal tile.  Enqueued on s.
// Workspace of plan_rsolve: Sx (rc x nrhs per tile column) and Wp (split partial sums).
struct RsolveWork {
  double *Sx, *Wp;
};
RsolveWork make_rsolve_work(blr_matrix h, int nrhs) {
  RsolveWork r;
  r.Sx = (double*)h->work.alloc((size_t)h->q * h->rc * nrhs * 8);
  r.Wp = (double*)h->work.alloc((size_t)kApplySlices * h->b * std::min(nrhs, 64) * 8);
  return r;
}

void plan_rsolve(blr_matrix h, Plan& Q, const RsolveWork& rw, double* X, int64_t ldx, int nrhs, int trans) {
  const int b = h->b, q = h->q, rc = h->rc;
  double* Sx = rw.Sx;
  double* Wp = rw.Wp;
  for (int step = 0; step < q; ++step) {
    const int k = trans ? step : q - 1 - step;
    double* Xk = X + (int64_t)k * b;
    // the already solved blocks: j > k (R X) or j < k (R^T X)
    const int jb = trans ? 0 : k + 1, je = trans ? k : q;
    bool any_lr = false;
    for (int j = jb; j < je; ++j) {
      Tile& t = trans ? h->t(j, k) : h->t(k, j);
      if (t.fmt != LOWRANK) continue;
      if (trans)   // (U V^T)^T X_j = V (U^T X_j)
        Q.gemm(Sx + (size_t)j * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.U, b,
               X + (int64_t)j * b, ldx, b, SEG_TRANS_A);
      else
        Q.gemm(Sx + (size_t)j * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.Vt, rc,
               X + (int64_t)j * b, ldx, b, 0);
      any_lr = true;
    }
    if (any_lr) Q.flush_gemm(0, 0, false);
    if (je > jb) {
      std::vector<GemmSeg> sv;
      for (int j = jb; j < je; ++j) {
        Tile& t = trans ? h->t(j, k) : h->t(k, j);
        GemmSeg sg{};
        if (t.fmt == DENSE) {
          sg.A = t.D; sg.lda = b; sg.B = X + (int64_t)j * b; sg.ldb = ldx; sg.K = b; sg.flags = trans ? SEG_TRANS_A : 0;
        } else if (trans) {
          sg.A = t.Vt; sg.lda = rc; sg.B = Sx + (size_t)j * rc * nrhs; sg.ldb = rc; sg.K = rc; sg.flags = SEG_TRANS_A;
        } else {
          sg.A = t.U; sg.lda = b; sg.B = Sx + (size_t)j * rc * nrhs; sg.ldb = rc; sg.K = rc; sg.flags = 0;
        }
        sv.push_back(sg);
      }
      // X_k -= sum_j (...): split over up to kApplySlices groups of tiles
      // (partial products, then X_k and the partials summed in one pass)
      const int ng = std::min<int>((int)sv.size(), kApplySlices - 1);
      if (ng <= 1 || nrhs > 64) {
        Q.gemm_multi(Xk, ldx, Xk, ldx, b, nrhs, -1.0, 1.0, sv);
        Q.flush_gemm(0, 0, false);
      } else {
        const int per = ((int)sv.size() + ng - 1) / ng;
        Q.copy({CopyDesc{Xk, Wp, ldx, (int64_t)b, b, nrhs, 0, 0}});
        int nd = 1;
        for (int g0 = 0; g0 < (int)sv.size(); g0 += per, ++nd) {
          std::vector<GemmSeg> part(sv.begin() + g0, sv.begin() + std::min<int>((int)sv.size(), g0 + per));
          Q.gemm_multi(Wp + (size_t)nd * b * nrhs, b, nullptr, 0, b, nrhs, -1.0, 0.0, part);
        }
        Q.flush_gemm(0, 0, false);
        Q.copy({CopyDesc{Wp, Xk, (int64_t)b, ldx, b, nrhs, 0, nd, (int64_t)b * nrhs}});
      }
    }
    Op o;
    o.kind = Op::TRSM;
    o.n = trans;
    o.trsm = TrsmJob{h->t(k, k).D, (int64_t)b, Xk, ldx, b, nrhs};
    Q.push(o);
  }
}

void run_rsolve(blr_matrix h, double* X, int64_t ldx, int nrhs, int trans, hipStream_t s) {
  Plan Q;
  plan_rsolve(h, Q, make_rsolve_work(h, nrhs), X, ldx, nrhs, trans);
  run_plan(h, Q, s);
}

// Singularity check of a complete factor: min |R_jj| against n u ||R||_F.
// sing_launch enqueues the reductions and their copies to the host; after
// the stream is synchronised, sing_ok evaluates them.
struct SingCheck {
  std::vector<double> ho, hf;
};
SingCheck sing_launch(blr_matrix h, hipStream_t s) {
  const int b = h->b, q = h->q, rc = h->rc;
  SingCheck c;
  std::vector<DiagDesc> dd(q);
  for (int k = 0; k < q; ++k) {
    dd[k].R = h->t(k, k).D;
    dd[k].ncols = (int)std::min<int64_t>(b, h->nu - (int64_t)k * b);   // the embedding's columns excluded
  }
  DiagDesc* ddd = upload_vec(h, dd, s);
  double* out = (double*)h->work.alloc((size_t)2 * q * 8);
  HIPCHECK(launch_diag_absmin(ddd, q, b, out, s));
  std::vector<Frob2Desc> fr;
  double* fo = (double*)h->work.alloc((size_t)q * q * 8 + 8);
  for (int k = 0; k < q; ++k)
    for (int j = k + 1; j < q; ++j) {
      Tile& t = h->t(k, j);
      double* o = fo + fr.size();
      if (t.fmt == DENSE) fr.push_back(Frob2Desc{t.D, b, b, b, o});
      else fr.push_back(Frob2Desc{t.Vt, rc, rc, b, o});
    }
  if (!fr.empty()) {
    Frob2Desc* dfr = upload_vec(h, fr, s);
    HIPCHECK(launch_frob2(dfr, (int)fr.size(), s));
  }
  c.ho.resize(2 * q);
  c.hf.resize(fr.size());
  HIPCHECK(hipMemcpyAsync(c.ho.data(), out, 2 * q * 8, hipMemcpyDeviceToHost, s));
  if (!fr.empty()) HIPCHECK(hipMemcpyAsync(c.hf.data(), fo, fr.size() * 8, hipMemcpyDeviceToHost, s));
  return c;
}
bool sing_ok(blr_matrix h, const SingCheck& c) {
  double r2 = 0.0, mn = 1e300;
  for (int k = 0; k < h->q; ++k) {
    mn = std::min(mn, c.ho[2 * k]);
    r2 += c.ho[2 * k + 1];
  }
  for (double v : c.hf) r2 += v;
  const double thr = (double)h->nu * 2.220446049250313e-16 * std::sqrt(r2);
  return mn > thr;
}

// Per-column decision after one refinement step, from the squared norms
// hn[c] = ||dx_c||^2 and hn[nrhs + c] = ||x_c||^2 of the step's correction
// and of the current iterate.  A column still refining (active) takes its
// correction (take[c] = 1) only while the correction is at most half the
// previous one taken; a larger one means the iteration has reached the
// rounding noise of its residuals or diverges, so it is dropped and the
// column stops with its current iterate (the rule LAPACK's refinement
// routines use).  A column also stops after taking a correction at the
// rounding level of x (||dx|| <= 2u ||x||).  prev keeps the last correction
// taken.  Returns true when no column is still refining.
bool refine_decide(const std::vector<double>& hn, std::vector<double>& prev, std::vector<char>& active,
                   std::vector<char>& take, int nrhs, double u) {
  bool done = true;
  for (int c = 0; c < nrhs; ++c) {
    take[c] = 0;
    if (!active[c]) continue;
    const double dx = std::sqrt(hn[c]);
    if (!(dx <= 0.5 * prev[c])) {   // no longer halving (or not finite): drop it
      active[c] = 0;
      continue;
    }
    take[c] = 1;
    prev[c] = dx;
    if (dx <= 2.0 * u * std::sqrt(hn[nrhs + c])) active[c] = 0;
    done = done && !active[c];
  }
  return done;
}

// Column runs of the columns a refinement step takes: [c0, c1) pairs.
std::vector<std::pair<int, int>> take_runs(const std::vector<char>& take) {
  std::vector<std::pair<int, int>> runs;
  const int nrhs = (int)take.size();
  for (int c = 0; c < nrhs;) {
    if (!take[c]) { ++c; continue; }
    int e = c;
    while (e < nrhs && take[e]) ++e;
    runs.emplace_back(c, e);
    c = e;
  }
  return runs;
}

// Keep a device copy of A~ (all tiles and ranks) for products after the
// in-place factorization.
void keep_copy(blr_matrix h, hipStream_t s) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  h->acopy.assign(h->tiles.size(), Tile{});
  size_t nd = 0, nl = 0;
  for (auto& t : h->tiles) (t.fmt == DENSE ? nd : nl)++;
  double* dp = (double*)h->amem.alloc(std::max<size_t>(nd, 1) * b * b * 8);
  double* lp = (double*)h->amem.alloc(std::max<size_t>(nl, 1) * 2 * (size_t)b * rc * 8);
  int* rk = (int*)h->amem.alloc((size_t)p * q * sizeof(int));
  HIPCHECK(hipMemcpyAsync(rk, h->d_rank, (size_t)p * q * sizeof(int), hipMemcpyDeviceToDevice, s));
  Plan P;
  std::vector<CopyDesc> cp;
  size_t id = 0, il = 0;
  for (size_t a = 0; a < h->tiles.size(); ++a) {
    Tile& t = h->tiles[a];
    Tile& c = h->acopy[a];
    c.fmt = t.fmt;
    c.rank = rk + a;
    if (t.fmt == DENSE) {
      c.D = dp + (id++) * (size_t)b * b;
      cp.push_back(CopyDesc{t.D, c.D, (int64_t)b, (int64_t)b, b, b, 0, 0});
    } else {
      c.U = lp + (il++) * 2 * (size_t)b * rc;
      c.Vt = c.U + (size_t)b * rc;
      cp.push_back(CopyDesc{t.U, c.U, (int64_t)b, (int64_t)b, b, rc, 0, 0});
      cp.push_back(CopyDesc{t.Vt, c.Vt, (int64_t)rc, (int64_t)rc, rc, b, 0, 0});
    }
  }
  P.copy(cp);
  run_plan(h, P, s);
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

blr_status run_guarded(const std::function<void()>& f) {
  try {
    f();
    return BLR_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return BLR_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return BLR_ERR_DEVICE;
  }
}

void alloc_common(blr_matrix h) {
  const size_t nt = (size_t)h->p * h->q;
  h->tiles.assign(nt, Tile());
  h->yfmt.assign(nt, DENSE);
  h->T.assign(nt, nullptr);
  h->tau.assign(nt, nullptr);
  h->d_rank = (int*)h->mem.alloc(nt * sizeof(int));
  HIPCHECK(hipMemset(h->d_rank, 0, nt * sizeof(int)));
  h->d_counters = (unsigned long long*)h->mem.alloc(4 * sizeof(unsigned long long));
  HIPCHECK(hipMemset(h->d_counters, 0, 4 * sizeof(unsigned long long)));
  for (size_t t = 0; t < nt; ++t) h->tiles[t].rank = h->d_rank + t;
}

// Allocate low-rank slots for the given tiles (one pool).
void alloc_lowrank(blr_matrix h, const std::vector<int>& idx) {
  if (idx.empty()) return;
  const size_t per = 2 * (size_t)h->b * h->rc;
  double* pool = (double*)h->mem.alloc(idx.size() * per * 8);
  HIPCHECK(hipMemset(pool, 0, idx.size() * per * 8));
  for (size_t a = 0; a < idx.size(); ++a) {
    Tile& t = h->tiles[idx[a]];
    t.U = pool + a * per;
    t.Vt = t.U + (size_t)h->b * h->rc;
  }
}

void alloc_dense(blr_matrix h, const std::vector<int>& idx) {
  if (idx.empty()) return;
  const size_t per = (size_t)h->b * h->b;
  double* pool = (double*)h->mem.alloc(idx.size() * per * 8);
  for (size_t a = 0; a < idx.size(); ++a) h->tiles[idx[a]].D = pool + a * per;
}

blr_status validate_opts(const blr_compress_opts* o) {
  if (!o) return fail(BLR_ERR_INVALID, "opts is NULL");
  if (o->m < 1 || o->n < 1 || o->m < o->n) return fail(BLR_ERR_INVALID, "need m >= n >= 1");
  if (o->tile < 16 || o->tile > 1024 || o->tile % 16)
    return fail(BLR_ERR_INVALID, "tile must be a multiple of 16 in [16, 1024]");
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(BLR_ERR_INVALID, "tol must be > 0");
  if (o->max_rank < 1 || o->max_rank > o->tile || o->max_rank > 128)
    return fail(BLR_ERR_INVALID, "max_rank must be in [1, min(tile, 128)]");
  if (o->overflow != BLR_OVERFLOW_DENSE && o->overflow != BLR_OVERFLOW_TRUNCATE)
    return fail(BLR_ERR_INVALID, "bad overflow policy");
  if (o->m / o->tile + 2 > 1 << 15 || o->n / o->tile + 1 > 1 << 15) return fail(BLR_ERR_INVALID, "too many tiles");
  return BLR_OK;
}

// Set-up and launch plan of one factorization (Alg. 2 or Alg. 4): fill-in
// slots from the simulated formats, T and tau storage, workspaces, plan.
// Returns the number of steps planned.
int prepare_factor(blr_matrix h, const blr_factor_opts* o, hipStream_t s, Plan& P, bool lookahead) {
  const int b = h->b, p = h->p, q = h->q;
  const int kend = (o->stop_after_k < 0) ? q : std::min(q, o->stop_after_k);

  h->variant = o->variant;
  h->precision = o->precision;
  h->ib = o->ib > 0 ? o->ib : 32;
  h->fmt0.resize((size_t)p * q);
  for (size_t t = 0; t < h->fmt0.size(); ++t) h->fmt0[t] = h->tiles[t].fmt;
  if (o->keep_a) keep_copy(h, s);
  const bool bc = o->variant == BLR_BLOCK_COLUMN;
  int bc_pairs = 0;
  // fill-in: simulate formats to find the tiles that need a dense slot
  if (bc) {
    alloc_dense(h, bc_simulate(h, kend, &bc_pairs));
  } else {
    std::vector<int8_t> f((size_t)p * q);
    for (size_t t = 0; t < f.size(); ++t) f[t] = h->tiles[t].fmt;
    std::vector<int> need;
    for (int k = 0; k < kend; ++k)
      for (int i = k + 1; i < p; ++i) {
        const bool yd = f[(size_t)i * q + k] == DENSE;
        if (!yd) continue;
        for (int j = k + 1; j < q; ++j) {
          int8_t& R = f[(size_t)k * q + j];
          int8_t& A = f[(size_t)i * q + j];
          if (R == LOWRANK && A == DENSE) {
            R = DENSE;
            need.push_back(k * q + j);
          }
          if (R == DENSE && A == LOWRANK) {
            A = DENSE;
            need.push_back(i * q + j);
          }
        }
      }
    alloc_dense(h, need);
  }
  // T and tau storage for every (i,k), i >= k, k < kend
  {
    std::vector<int> idx;
    for (int k = 0; k < kend; ++k)
      for (int i = k; i < (bc ? k + 1 : p); ++i) idx.push_back(i * q + k);
    double* tp = (double*)h->mem.alloc(idx.size() * (size_t)b * b * 8);
    HIPCHECK(hipMemset(tp, 0, idx.size() * (size_t)b * b * 8));
    double* tu = (double*)h->mem.alloc(idx.size() * (size_t)b * 8);
    HIPCHECK(hipMemset(tu, 0, idx.size() * (size_t)b * 8));
    for (size_t a = 0; a < idx.size(); ++a) {
      h->T[idx[a]] = tp + a * (size_t)b * b;
      h->tau[idx[a]] = tu + a * (size_t)b;
    }
  }
  std::vector<Work> works;
  int nstreams = bc ? 1 : std::min(q, kTiledChains);
  if (!bc) {
    // each chain holds a workspace of two b x b blocks per tile column: keep
    // them within half of the free device memory
    size_t fr = 0, tot = 0;
    HIPCHECK(hipMemGetInfo(&fr, &tot));
    const size_t per = work_bytes(h, 0);
    while (nstreams > 4 && (size_t)nstreams * per > fr / 2) nstreams /= 2;
  }
  for (int a = 0; a < nstreams; ++a) works.push_back(make_work(h, 0));
  h->n_fill = 0;
  if (bc) {
    BcWork bw = make_bc_work(h, bc_pairs);
    plan_blockcol(h, P, works[0], bw, kend, o->precision == BLR_MIXED_FP32, lookahead);
  } else {
    plan_tiled(h, P, works, kend, o->precision == BLR_MIXED_FP32);
    P = merge_streams(P, h);
  }
  h->flops = 0.0;
  for (auto& op : P.ops) h->flops += op.flops;
  for (int k = 0; k < 2; ++k) {
    for (auto e : h->prof_ev[k]) (void)hipEventDestroy(e);
    h->prof_ev[k].clear();
    h->prof_flops[k] = 0.0;
    h->prof_launches[k] = 0;
  }
  h->launches = 0;
  return kend;
}

blr_matrix new_handle(const blr_compress_opts* o) {
  blr_matrix h = new blr_matrix_s();
  const int64_t b = o->tile;
  h->mu = o->m;
  h->nu = o->n;
  // the embedding: whole tiles, with room below A for the identity block of
  // the padded columns (one more tile row when the padded rows are too few)
  h->n = (o->n + b - 1) / b * b;
  h->m = (o->m + b - 1) / b * b;
  h->pu = (int)(h->m / b);
  if (h->m - o->m < h->n - o->n) h->m += b;
  h->b = (int)b;
  h->p = (int)(h->m / b);
  h->q = (int)(h->n / b);
  h->cap = o->max_rank;
  h->rc = std::min(round_up(o->max_rank, 16), o->tile);
  h->tol = o->tol;
  h->overflow = o->overflow;
  return h;
}

}  // namespace

extern "C" {

const char* blr_status_string(blr_status s) {
  switch (s) {
    case BLR_OK: return "ok";
    case BLR_ERR_INVALID: return "invalid argument";
    case BLR_ERR_STATE: return "invalid state";
    case BLR_ERR_OOM: return "out of memory";
    case BLR_ERR_DEVICE: return "device error";
    case BLR_ERR_NONFINITE: return "non-finite input";
    case BLR_ERR_SINGULAR: return "singular R";
  }
  return "unknown status";
}

const char* blr_last_error(void) { return g_last_error.c_str(); }

blr_status blr_compress(const blr_source* src, const blr_compress_opts* o, void* stream, blr_matrix* out) {
  if (!src || !out) return fail(BLR_ERR_INVALID, "NULL argument");
  blr_status st = validate_opts(o);
  if (st != BLR_OK) return st;
  *out = nullptr;
  const bool kern = src->kind == BLR_SRC_KERNEL;
  if (kern) {
    if (!src->x || !src->y) return fail(BLR_ERR_INVALID, "kernel source needs x and y");
    if (src->dim < 1 || src->dim > 3) return fail(BLR_ERR_INVALID, "dim must be 1, 2 or 3");
    if (src->kernel != BLR_KERNEL_LOG2D && src->kernel != BLR_KERNEL_INV_R)
      return fail(BLR_ERR_INVALID, "bad kernel");
  } else if (src->kind == BLR_SRC_DENSE) {
    if (!src->A || src->lda < o->m) return fail(BLR_ERR_INVALID, "dense source needs A and lda >= m");
    if (src->admissibility == BLR_ADM_ADJACENT || src->admissibility == BLR_ADM_DIST_GT_DIAM)
      return fail(BLR_ERR_INVALID, "geometric admissibility needs a kernel source");
  } else {
    return fail(BLR_ERR_INVALID, "bad source kind");
  }
  if (src->admissibility < 0 || src->admissibility > BLR_ADM_MASK)
    return fail(BLR_ERR_INVALID, "bad admissibility");
  if (src->admissibility == BLR_ADM_MASK && !src->mask) return fail(BLR_ERR_INVALID, "mask is NULL");
  blr_matrix h = new_handle(o);
  hipStream_t s = as_stream(stream);
  st = run_guarded([&] {
    alloc_common(h);
    const int b = h->b, p = h->p, q = h->q, rc = h->rc;
    // finiteness of the input
    int* flag = (int*)h->work.alloc(sizeof(int));
    HIPCHECK(hipMemsetAsync(flag, 0, sizeof(int), s));
    if (kern) {
      HIPCHECK(launch_nonfinite(src->x, h->mu * src->dim, 1, h->mu * src->dim, flag, s));
      HIPCHECK(launch_nonfinite(src->y, h->nu * src->dim, 1, h->nu * src->dim, flag, s));
    } else {
      HIPCHECK(launch_nonfinite(src->A, h->mu, h->nu, src->lda, flag, s));
    }
    int hflag = 0;
    HIPCHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (hflag) throw Error(BLR_ERR_NONFINITE, "input contains NaN or Inf");
    // admissibility mask (true = low-rank) over the tile rows of A; a tile
    // row that only the embedding adds is zero outside its identity entries
    std::vector<int8_t> lr((size_t)p * q, 0);
    const int pu = h->pu;
    if (src->admissibility == BLR_ADM_WEAK) {
      std::fill(lr.begin(), lr.end(), 1);
    } else if (src->admissibility == BLR_ADM_MASK) {
      for (size_t t = 0; t < (size_t)pu * q; ++t) lr[t] = src->mask[t] ? 1 : 0;
    } else {
      const int d = src->dim;
      double* bx = (double*)h->work.alloc((size_t)4 * (p + q) * d * 8);
      double *rlo = bx, *rhi = bx + (size_t)p * d, *clo = bx + (size_t)2 * p * d, *chi = clo + (size_t)q * d;
      HIPCHECK(launch_boxes(src->x, (int)h->mu, d, b, rlo, rhi, s));
      HIPCHECK(launch_boxes(src->y, (int)h->nu, d, b, clo, chi, s));
      std::vector<double> hb((size_t)2 * (p + q) * d);
      HIPCHECK(hipMemcpyAsync(hb.data(), bx, hb.size() * 8, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      const double *Rlo = hb.data(), *Rhi = Rlo + (size_t)p * d, *Clo = Rlo + (size_t)2 * p * d,
                   *Chi = Clo + (size_t)q * d;
      for (int i = 0; i < pu; ++i)
        for (int j = 0; j < q; ++j) {
          double g2 = 0.0, dr2 = 0.0, dc2 = 0.0;
          for (int c = 0; c < d; ++c) {
            const double g = std::max(0.0, std::max(Rlo[i * d + c] - Chi[j * d + c], Clo[j * d + c] - Rhi[i * d + c]));
            g2 += g * g;
            dr2 += (Rhi[i * d + c] - Rlo[i * d + c]) * (Rhi[i * d + c] - Rlo[i * d + c]);
            dc2 += (Chi[j * d + c] - Clo[j * d + c]) * (Chi[j * d + c] - Clo[j * d + c]);
          }
          const double gap = std::sqrt(g2);
          bool low;
          if (src->admissibility == BLR_ADM_ADJACENT) low = gap > 0.0;
          else low = gap > std::max(std::sqrt(dr2), std::sqrt(dc2));
          lr[(size_t)i * q + j] = low ? 1 : 0;
        }
    }
    for (int i = pu; i < p; ++i)
      for (int j = 0; j < q; ++j) lr[(size_t)i * q + j] = 1;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j)
        if (h->has_identity(i, j)) lr[(size_t)i * q + j] = 0;
    for (int k = 0; k < std::min(p, q); ++k) lr[(size_t)k * q + k] = 0;
    std::vector<int> cand;
    for (size_t t = 0; t < lr.size(); ++t)
      if (lr[t]) cand.push_back((int)t);
    alloc_lowrank(h, cand);
    TileFillParams fp{};
    fp.b = b;
    fp.src_dense = kern ? 0 : 1;
    fp.A = src->A;
    fp.lda = src->lda;
    fp.x = src->x;
    fp.y = src->y;
    fp.dim = src->dim;
    fp.kernel = src->kernel;
    fp.reg = src->reg;
    fp.mu = h->mu;
    fp.nu = h->nu;
    std::vector<int> status(lr.size(), 0);
    if (!cand.empty()) {
      const int l = std::min(b, rc + 16);
      const int NB = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cand.size(), (int64_t)(256LL << 20) / ((int64_t)b * b * 8)));
      Workspace& cw = h->work;
      double* Om = (double*)cw.alloc((size_t)b * l * 8);
      HIPCHECK(launch_gaussian(Om, (int64_t)b * l, o->seed, 4, s));
      double* As = (double*)cw.alloc((size_t)NB * b * b * 8);
      double* Ys = (double*)cw.alloc((size_t)NB * b * l * 8);
      double* Qs = (double*)cw.alloc((size_t)NB * b * l * 8);
      double* Bs = (double*)cw.alloc((size_t)NB * l * b * 8);
      double* nrm = (double*)cw.alloc((size_t)NB * 2 * 8);
      int* stat = (int*)cw.alloc((size_t)NB * sizeof(int));
      const size_t cwd = comp_work_doubles(b, l);
      double* wk = (double*)cw.alloc((size_t)NB * cwd * 8);
      TileFillDesc* dfd = (TileFillDesc*)cw.alloc((size_t)NB * sizeof(TileFillDesc));
      Frob2Desc* dfr = (Frob2Desc*)cw.alloc((size_t)NB * 2 * sizeof(Frob2Desc));
      CompDesc* dcd = (CompDesc*)cw.alloc((size_t)NB * sizeof(CompDesc));
      GemmDesc* dgd = (GemmDesc*)cw.alloc((size_t)NB * 3 * sizeof(GemmDesc));
      GemmSeg* dgs = (GemmSeg*)cw.alloc((size_t)NB * 3 * sizeof(GemmSeg));
      for (size_t c0 = 0; c0 < cand.size(); c0 += NB) {
        const int nb = (int)std::min<size_t>(NB, cand.size() - c0);
        std::vector<TileFillDesc> fd(nb);
        std::vector<Frob2Desc> fr(2 * nb);
        std::vector<CompDesc> cd(nb);
        Plan P;
        for (int a = 0; a < nb; ++a) {
          const int t = cand[c0 + a];
          Tile& T = h->tiles[t];
          double* A = As + (size_t)a * b * b;
          fd[a] = TileFillDesc{A, t / q, t % q};
          fr[a] = Frob2Desc{A, b, b, b, nrm + 2 * a};
          fr[nb + a] = Frob2Desc{A, b, b, b, nrm + 2 * a + 1};
          CompDesc& D = cd[a];
          D.A = A;
          D.Y = Ys + (size_t)a * b * l;
          D.Q = Qs + (size_t)a * b * l;
          D.B = Bs + (size_t)a * l * b;
          D.Uout = T.U;
          D.Vtout = T.Vt;
          D.rank_out = T.rank;
          D.status_out = stat + a;
          D.work = wk + (size_t)a * cwd;
          D.anorm2 = nrm + 2 * a;
          D.enorm2 = nrm + 2 * a + 1;
          P.gemm(D.Y, b, nullptr, 0, nullptr, 0, b, l, 1.0, 0.0, A, b, Om, b, b, 0);
        }
        // stream-ordered uploads; the host arrays live until the stream is
        // synchronised at the end of this chunk of tiles
        HIPCHECK(hipMemcpyAsync(dfd, fd.data(), nb * sizeof(TileFillDesc), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(dfr, fr.data(), 2 * nb * sizeof(Frob2Desc), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(dcd, cd.data(), nb * sizeof(CompDesc), hipMemcpyHostToDevice, s));
        P.flush_gemm(0, 0, false);
        for (int a = 0; a < nb; ++a)
          P.gemm(cd[a].B, l, nullptr, 0, nullptr, 0, l, b, 1.0, 0.0, cd[a].Q, b, cd[a].A, b, b, SEG_TRANS_A);
        P.flush_gemm(0, 0, false);
        for (int a = 0; a < nb; ++a)
          P.gemm(const_cast<double*>(cd[a].A), b, cd[a].A, b, nullptr, 0, b, b, -1.0, 1.0, cd[a].Q, b,
                 cd[a].B, l, l, 0);
        P.flush_gemm(0, 0, false);
        HIPCHECK(hipMemcpyAsync(dgd, P.descs.data(), P.descs.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(dgs, P.segs.data(), P.segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice, s));
        HIPCHECK(launch_fill_tiles(dfd, nb, fp, s));
        HIPCHECK(launch_frob2(dfr, nb, s));
        HIPCHECK(launch_gemm(dgd + P.ops[0].off, P.ops[0].n, dgs, P.ops[0].ntiles, P.ops[0].big, 0, s));
        HIPCHECK(launch_rangefinder(dcd, nb, b, l, s));
        HIPCHECK(launch_gemm(dgd + P.ops[1].off, P.ops[1].n, dgs, P.ops[1].ntiles, P.ops[1].big, 0, s));
        HIPCHECK(launch_gemm(dgd + P.ops[2].off, P.ops[2].n, dgs, P.ops[2].ntiles, P.ops[2].big, 0, s));
        HIPCHECK(launch_frob2(dfr + nb, nb, s));
        CompParams cp{b, rc, l, h->cap, h->tol, h->overflow == BLR_OVERFLOW_TRUNCATE ? 1 : 0};
        HIPCHECK(launch_comp_svd(dcd, nb, cp, s));
        std::vector<int> hs(nb);
        HIPCHECK(hipMemcpyAsync(hs.data(), stat, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        for (int a = 0; a < nb; ++a) status[cand[c0 + a]] = hs[a];
      }
    }
    std::vector<int> dense;
    for (size_t t = 0; t < lr.size(); ++t) {
      if (!lr[t] || status[t] == 1) {
        dense.push_back((int)t);
        h->tiles[t].fmt = DENSE;
        if (lr[t]) h->compress_overflow++;
      } else {
        h->tiles[t].fmt = LOWRANK;
        if (status[t] == 2) h->compress_overflow++;
      }
    }
    alloc_dense(h, dense);
    for (size_t c0 = 0; c0 < dense.size(); c0 += 4096) {
      const int nb = (int)std::min<size_t>(4096, dense.size() - c0);
      std::vector<TileFillDesc> fd(nb);
      for (int a = 0; a < nb; ++a) {
        const int t = dense[c0 + a];
        fd[a] = TileFillDesc{h->tiles[t].D, t / q, t % q};
      }
      TileFillDesc* dfd = upload_vec(h, fd, s);
      HIPCHECK(launch_fill_tiles(dfd, nb, fp, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    reset_work_after_sync(h);
  });
  if (st != BLR_OK) {
    delete h;
    return st;
  }
  *out = h;
  return BLR_OK;
}

blr_status blr_import(const blr_compress_opts* o, const blr_tiles_host* t, void* stream, blr_matrix* out) {
  if (!t || !out || !t->fmt || !t->rank) return fail(BLR_ERR_INVALID, "NULL argument");
  blr_compress_opts oo = *o;
  oo.overflow = BLR_OVERFLOW_DENSE;
  blr_status st = validate_opts(&oo);
  if (st != BLR_OK) return st;
  blr_matrix h = new_handle(&oo);
  hipStream_t s = as_stream(stream);
  st = run_guarded([&] {
    alloc_common(h);
    const int b = h->b, rc = h->rc, q = h->q;
    const size_t nt = (size_t)h->p * q;
    const size_t ntu = (size_t)h->pu * q;   // tiles the caller supplies
    // formats: the caller's for its tiles (a tile holding identity entries of
    // the embedding is stored dense); the added tile row is zero (rank 0)
    // outside its identity entries
    std::vector<int8_t> fmt(nt, LOWRANK);
    std::vector<int> dn, lo;
    for (size_t i = 0; i < nt; ++i) {
      const int ti = (int)(i / q), tj = (int)(i % q);
      if (i < ntu) {
        const int r = t->rank[i];
        if (t->fmt[i] == LOWRANK && (r < 0 || r > h->cap)) throw Error(BLR_ERR_INVALID, "rank out of range");
        if (t->fmt[i] == LOWRANK && ti == tj) throw Error(BLR_ERR_INVALID, "diagonal tiles must be dense");
        fmt[i] = t->fmt[i] == LOWRANK ? LOWRANK : DENSE;
      }
      if (h->has_identity(ti, tj) || ti == tj) fmt[i] = DENSE;
      (fmt[i] == LOWRANK ? lo : dn).push_back((int)i);
    }
    bool any_lr_in = false, any_dense_in = false;
    for (size_t i = 0; i < ntu; ++i) (t->fmt[i] == LOWRANK ? any_lr_in : any_dense_in) = true;
    if (any_lr_in && (!t->U || !t->V)) throw Error(BLR_ERR_INVALID, "U and V needed for low-rank tiles");
    if (any_dense_in && !t->dense) throw Error(BLR_ERR_INVALID, "dense tiles needed");
    alloc_dense(h, dn);
    alloc_lowrank(h, lo);
    // entries of tile (ti, tj) that belong to A (the rest is the embedding's)
    auto rows_in = [&](int ti) { return (int)std::max<int64_t>(0, std::min<int64_t>(b, h->mu - (int64_t)ti * b)); };
    auto cols_in = [&](int tj) { return (int)std::max<int64_t>(0, std::min<int64_t>(b, h->nu - (int64_t)tj * b)); };
    std::vector<double> Db((size_t)b * b);
    for (int i : dn) {
      Tile& T = h->tiles[i];
      T.fmt = DENSE;
      const int ti = i / q, tj = i % q, ri = rows_in(ti), cj = cols_in(tj);
      std::fill(Db.begin(), Db.end(), 0.0);
      if ((size_t)i < ntu && t->fmt[i] != LOWRANK) {
        const double* src = t->dense + (size_t)i * b * b;
        for (int c = 0; c < cj; ++c)
          for (int r = 0; r < ri; ++r) Db[r + (size_t)c * b] = src[r + (size_t)c * b];
      } else if ((size_t)i < ntu) {
        // a supplied low-rank tile that the embedding stores dense
        const int rk = t->rank[i];
        const double* U = t->U + (size_t)i * b * rc;
        const double* V = t->V + (size_t)i * b * rc;
        for (int c = 0; c < cj; ++c)
          for (int r = 0; r < ri; ++r) {
            double v = 0.0;
            for (int l = 0; l < rk; ++l) v += U[r + (size_t)l * b] * V[c + (size_t)l * b];
            Db[r + (size_t)c * b] = v;
          }
      }
      for (int64_t g = std::max<int64_t>(h->mu, (int64_t)ti * b); g < std::min<int64_t>(h->mu + (h->n - h->nu), (int64_t)(ti + 1) * b); ++g) {
        const int64_t gc = h->nu + (g - h->mu);
        if (gc >= (int64_t)tj * b && gc < (int64_t)(tj + 1) * b) Db[(g - (int64_t)ti * b) + (size_t)(gc - (int64_t)tj * b) * b] = 1.0;
      }
      for (double v : Db)
        if (!std::isfinite(v)) throw Error(BLR_ERR_NONFINITE, "non-finite dense tile");
      HIPCHECK(hipMemcpy(T.D, Db.data(), (size_t)b * b * 8, hipMemcpyHostToDevice));
    }
    std::vector<double> Ub((size_t)b * rc), Vtb((size_t)rc * b);
    std::vector<int> ranks(nt, 0);
    for (int i : lo) {
      Tile& T = h->tiles[i];
      T.fmt = LOWRANK;
      std::fill(Ub.begin(), Ub.end(), 0.0);
      std::fill(Vtb.begin(), Vtb.end(), 0.0);
      if ((size_t)i < ntu) {
        const int r = t->rank[i], ti = i / q, tj = i % q, ri = rows_in(ti), cj = cols_in(tj);
        ranks[i] = r;
        const double* U = t->U + (size_t)i * b * rc;
        const double* V = t->V + (size_t)i * b * rc;
        for (int l = 0; l < r; ++l) {
          for (int e = 0; e < ri; ++e) Ub[e + (size_t)l * b] = U[e + (size_t)l * b];
          for (int e = 0; e < cj; ++e) Vtb[l + (size_t)e * rc] = V[e + (size_t)l * b];
        }
      }
      for (double v : Ub)
        if (!std::isfinite(v)) throw Error(BLR_ERR_NONFINITE, "non-finite U");
      for (double v : Vtb)
        if (!std::isfinite(v)) throw Error(BLR_ERR_NONFINITE, "non-finite V");
      HIPCHECK(hipMemcpy(T.U, Ub.data(), Ub.size() * 8, hipMemcpyHostToDevice));
      HIPCHECK(hipMemcpy(T.Vt, Vtb.data(), Vtb.size() * 8, hipMemcpyHostToDevice));
    }
    HIPCHECK(hipMemcpy(h->d_rank, ranks.data(), nt * sizeof(int), hipMemcpyHostToDevice));
    (void)s;
  });
  if (st != BLR_OK) {
    delete h;
    return st;
  }
  *out = h;
  return BLR_OK;
}

blr_status blr_export(blr_matrix h, blr_tiles_host* t) {
  if (!h || !t) return fail(BLR_ERR_INVALID, "NULL argument");
  return run_guarded([&] {
    wait_idle(h);
    const int b = h->b, rc = h->rc, q = h->q;
    const size_t nt = (size_t)h->pu * h->q;   // the tile rows that hold rows of A
    std::vector<int> ranks(nt);
    HIPCHECK(hipMemcpy(ranks.data(), h->d_rank, nt * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<double> tmp((size_t)b * std::max(b, rc));
    for (size_t i = 0; i < nt; ++i) {
      Tile& T = h->tiles[i];
      if (t->fmt) t->fmt[i] = T.fmt;
      if (t->rank) t->rank[i] = T.fmt == LOWRANK ? ranks[i] : -1;
      if (T.fmt == DENSE || (h->state == BLR_STATE_FACTORED && T.D)) {
        if (t->dense && T.D) HIPCHECK(hipMemcpy(t->dense + i * b * b, T.D, (size_t)b * b * 8, hipMemcpyDeviceToHost));
      }
      if (T.fmt == LOWRANK) {
        if (t->U) HIPCHECK(hipMemcpy(t->U + i * b * rc, T.U, (size_t)b * rc * 8, hipMemcpyDeviceToHost));
        const int row = (int)(i / q), col = (int)(i % q);
        const bool holds_y = h->state == BLR_STATE_FACTORED && row > col && col < h->steps_done;
        if (holds_y) {
          if (t->Y) HIPCHECK(hipMemcpy(t->Y + i * rc * b, T.Vt, (size_t)rc * b * 8, hipMemcpyDeviceToHost));
        } else if (t->V) {
          HIPCHECK(hipMemcpy(tmp.data(), T.Vt, (size_t)rc * b * 8, hipMemcpyDeviceToHost));
          double* V = t->V + i * b * rc;
          for (int l = 0; l < rc; ++l)
            for (int e = 0; e < b; ++e) V[e + (size_t)l * b] = tmp[l + (size_t)e * rc];
        }
      }
      if (t->T && h->T[i]) HIPCHECK(hipMemcpy(t->T + i * b * b, h->T[i], (size_t)b * b * 8, hipMemcpyDeviceToHost));
    }
  });
}

blr_status blr_qr_factor(blr_matrix h, const blr_factor_opts* o, void* stream) {
  if (!h || !o) return fail(BLR_ERR_INVALID, "NULL argument");
  if (h->state != BLR_STATE_COMPRESSED) return fail(BLR_ERR_STATE, "matrix is already factored");
  if (o->variant != BLR_TILED && o->variant != BLR_BLOCK_COLUMN) return fail(BLR_ERR_INVALID, "bad variant");
  if (o->precision != BLR_FP64 && o->precision != BLR_MIXED_FP32) return fail(BLR_ERR_INVALID, "bad precision");
  if (o->ib != 0 && o->ib != 16 && o->ib != 32) return fail(BLR_ERR_INVALID, "ib must be 0, 16 or 32");
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    begin_call(h);
    Plan P;
    const int kend = prepare_factor(h, o, s, P, true);
    HIPCHECK(hipMemsetAsync(h->d_counters, 0, 4 * sizeof(unsigned long long), s));
    run_plan(h, P, s);
    end_call(h, s);
    h->steps_done = kend;
    h->state = BLR_STATE_FACTORED;
  });
}

blr_status blr_qr_factor_batch(blr_matrix* hs, int32_t count, const blr_factor_opts* o, void* stream) {
  if (!hs || !o || count < 1) return fail(BLR_ERR_INVALID, "NULL argument or count < 1");
  if (o->variant != BLR_BLOCK_COLUMN) return fail(BLR_ERR_INVALID, "the batched factor runs the block-column variant");
  if (o->precision != BLR_FP64 && o->precision != BLR_MIXED_FP32) return fail(BLR_ERR_INVALID, "bad precision");
  if (o->ib != 0 && o->ib != 16 && o->ib != 32) return fail(BLR_ERR_INVALID, "ib must be 0, 16 or 32");
  std::vector<blr_matrix> v(hs, hs + count);
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(BLR_ERR_INVALID, "NULL handle in the batch");
    if (v[i]->state != BLR_STATE_COMPRESSED) return fail(BLR_ERR_STATE, "a matrix of the batch is already factored");
    for (int j = 0; j < i; ++j)
      if (v[j] == v[i]) return fail(BLR_ERR_INVALID, "a handle appears twice in the batch");
    if (v[i]->b != v[0]->b || v[i]->rc != v[0]->rc || v[i]->cap != v[0]->cap || v[i]->tol != v[0]->tol)
      return fail(BLR_ERR_INVALID, "the matrices of a batch share tile size, rank cap and tolerance");
  }
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    for (int i = 0; i < count; ++i) begin_call(v[i]);
    std::vector<Plan> plans(count);
    std::vector<int> kend(count);
    for (int i = 0; i < count; ++i) kend[i] = prepare_factor(v[i], o, s, plans[i], false);
    for (int i = 0; i < count; ++i)
      HIPCHECK(hipMemsetAsync(v[i]->d_counters, 0, 4 * sizeof(unsigned long long), s));
    run_batch_plans(plans, v, s);
    plans.clear();
    for (int i = 0; i < count; ++i) end_call(v[i], s);
    for (int i = 0; i < count; ++i) {
      v[i]->launches = v[0]->launches;
      v[i]->steps_done = kend[i];
      v[i]->state = BLR_STATE_FACTORED;
    }
  });
}

blr_status blr_apply_qt(blr_matrix h, int32_t trans, double* B, int64_t ldb, int32_t nrhs, void* stream) {
  if (!h || !B) return fail(BLR_ERR_INVALID, "NULL argument");
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (ldb < h->m || nrhs < 0 || (trans != 0 && trans != 1)) return fail(BLR_ERR_INVALID, "bad B shape or trans");
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    begin_call(h);
    Work w = make_work(h, nrhs);
    Plan P;
    plan_apply(h, P, w, B, ldb, nrhs, trans);
    run_plan(h, P, s);
    end_call(h, s);
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Blocked modified Gram-Schmidt BLR-QR (Section 2.1 Alg. 1 with Section 3.2),
// the method the paper compares its Householder algorithms with.  Step j
// stacks the right factors of every tile of block column j (dense: the tile;
// low-rank: V^T), takes their MGS QR in one workgroup (k_mgs_stack), writes
// Q^B back (dense tiles: the b x b block; low-rank tiles: the rows as the new
// V^T, so Q_ij = U_ij Q^B_ij keeps its U) with R_jj into R, and then runs the
// block-column update over every block row with W = Z: R_jk = Q_j^T A_k and
// A_k -= Q_j R_jk (the OP1/OP2 rules of the Householder update).
void plan_mgs(blr_matrix h, blr_matrix R, Plan& P, Work& w, BcWork& bw) {
  const int b = h->b, rc = h->rc, p = h->p, q = h->q;
  for (int j = 0; j < q; ++j) {
    std::vector<int64_t> off(p, 0);
    std::vector<int> rows(p, 0);
    int hs = 0;
    for (int i = 0; i < p; ++i) {
      rows[i] = h->t(i, j).fmt == DENSE ? b : rc;
      off[i] = hs;
      hs += rows[i];
    }
    std::vector<CopyDesc> cp;
    for (int i = 0; i < p; ++i) {
      Tile& t = h->t(i, j);
      const bool d = t.fmt == DENSE;
      cp.push_back(CopyDesc{d ? t.D : t.Vt, bw.stack + off[i], d ? (int64_t)b : (int64_t)rc, (int64_t)hs,
                            rows[i], b, 0, 0, 0});
    }
    P.copy(cp);
    P.mgs_stack(bw.stack, hs, hs, b, R->t(j, j).D, b);
    cp.clear();
    for (int i = 0; i < p; ++i) {
      Tile& t = h->t(i, j);
      const bool d = t.fmt == DENSE;
      cp.push_back(CopyDesc{bw.stack + off[i], d ? t.D : t.Vt, (int64_t)hs, d ? (int64_t)b : (int64_t)rc,
                            rows[i], b, 0, 0, 0});
      if (i != j) h->yfmt[(size_t)i * q + j] = t.fmt;
    }
    P.copy(cp);
    if (j + 1 >= q) break;
    // R_jk = Z_k, copied out of the step's temporaries into R's tile (j, k)
    // as soon as it is formed; a low-rank R_jk is then the W of the update
    BcGs gs;
    gs.store = [&](int k, bool dense, const double* Zd, const RcTerm& Zl) -> RcTerm {
      Tile& t = R->t(j, k);
      if (dense) {
        alloc_dense(R, {j * q + k});
        t.fmt = DENSE;
        P.copy({CopyDesc{Zd, t.D, (int64_t)b, (int64_t)b, b, b, 0, 0, 0}});
        return RcTerm{};
      }
      alloc_lowrank(R, {j * q + k});
      t.fmt = LOWRANK;
      P.copy({CopyDesc{Zl.U, t.U, Zl.ldu, (int64_t)b, b, rc, 0, 0, 0},
              CopyDesc{Zl.Vt, t.Vt, Zl.ldvt, (int64_t)rc, rc, b, 0, 0, 0},
              CopyDesc{(const double*)Zl.rank_ptr, (double*)t.rank, 1, 1, 1, 1, 3, 0, 0}});
      return RcTerm{t.U, t.Vt, t.rank, (int64_t)b, (int64_t)rc, 0, 0, 1.0};
    };
    plan_bc_update(h, P, w, bw, j, j + 1, q, false, q, nullptr, &gs);
  }
}

// ---------------------------------------------------------------------------
// Q^T B / Q B with no device allocation: the temporaries and the launch
// descriptors of the call live in one static device array.  Every GPU the
// library runs on holds its own copy until the process ends; its device
// address comes from hipGetSymbolAddress once per device (the array's name
// is only a host-side stand-in).  All calls on one GPU share it.
static __device__ __align__(256) char scratch[BLR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

char* scratch_for_current_device() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(BLR_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = (char*)ptr;
  }
  return g_scratch_dev[dev];
}

// Bump allocation over the static array.  Offsets past the end are handed
// out but never used: the caller checks the total before enqueuing anything.
struct ScratchAlloc : DevAlloc {
  char* base = nullptr;
  size_t used = 0;
  void* alloc(size_t n) override {
    if (n == 0) n = 256;
    n = (n + 255) & ~(size_t)255;
    char* p = base + used;
    used += n;
    return p;
  }
};
}  // namespace

extern "C" {

blr_status blr_mgs_qr(blr_matrix h, void* stream, blr_matrix* r_out) {
  if (!h || !r_out) return fail(BLR_ERR_INVALID, "NULL argument");
  *r_out = nullptr;
  if (h->state != BLR_STATE_COMPRESSED) return fail(BLR_ERR_STATE, "matrix is not in the compressed state");
  if (h->ragged()) return fail(BLR_ERR_INVALID, "the Gram-Schmidt factorization needs b to divide m and n");
  hipStream_t s = as_stream(stream);
  blr_compress_opts ro{};
  ro.m = h->n;
  ro.n = h->n;
  ro.tile = h->b;
  ro.tol = h->tol;
  ro.max_rank = h->cap;
  ro.overflow = BLR_OVERFLOW_DENSE;
  blr_matrix R = new_handle(&ro);
  blr_status st = run_guarded([&] {
    begin_call(h);
    const int b = h->b, q = h->q;
    alloc_common(R);
    // R: dense diagonal tiles; the tiles below the diagonal are zero (rank 0)
    std::vector<int> diag, below;
    for (int i = 0; i < q; ++i)
      for (int k = 0; k < q; ++k) {
        if (i == k) diag.push_back(i * q + k);
        else if (i > k) below.push_back(i * q + k);
      }
    alloc_dense(R, diag);
    for (int t : diag) R->tiles[t].fmt = DENSE;
    alloc_lowrank(R, below);
    for (int t : below) R->tiles[t].fmt = LOWRANK;
    // fill-in slots and temporaries of the Gram-Schmidt steps
    int pairs = 0;
    alloc_dense(h, bc_simulate(h, q, &pairs, true));
    Work w = make_work(h, 0);
    BcWork bw = make_bc_work(h, pairs);
    h->n_fill = 0;
    Plan P;
    plan_mgs(h, R, P, w, bw);
    // tiles of R right of the diagonal that no step wrote (q = 1) stay absent
    for (int i = 0; i < q; ++i)
      for (int k = i + 1; k < q; ++k)
        if (!R->t(i, k).D && !R->t(i, k).U) {
          alloc_lowrank(R, {i * q + k});
          R->t(i, k).fmt = LOWRANK;
        }
    h->flops = 0.0;
    for (auto& op : P.ops) h->flops += op.flops;
    h->launches = 0;
    (void)b;
    run_plan(h, P, s);
    end_call(h, s);
    HIPCHECK(hipStreamSynchronize(s));
  });
  if (st != BLR_OK) {
    delete R;
    return st;
  }
  *r_out = R;
  return BLR_OK;
}

blr_status blr_apply_qt_noalloc(blr_matrix h, int32_t trans, double* B, int64_t ldb, int32_t nrhs,
                                void* stream) {
  if (!h || !B) return fail(BLR_ERR_INVALID, "NULL argument");
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (ldb < h->m || nrhs < 0 || (trans != 0 && trans != 1)) return fail(BLR_ERR_INVALID, "bad B shape or trans");
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    ScratchAlloc a;
    a.base = scratch_for_current_device();
    Work w = make_apply_work(h, a, nrhs);
    Plan P;
    plan_apply(h, P, w, B, ldb, nrhs, trans, &a);
    const size_t need = a.used + P.upload_bytes();
    if (need > (size_t)BLR_NOALLOC_SCRATCH_BYTES)
      throw Error(BLR_ERR_INVALID, "blr_apply_qt_noalloc needs " + std::to_string(need) +
                                       " bytes of scratch for this matrix and nrhs; the static scratch holds " +
                                       std::to_string((size_t)BLR_NOALLOC_SCRATCH_BYTES));
    begin_call(h);   // this handle's earlier work has finished with its uploads
    P.upload(a, h->keep, s);
    execute(h, P, s);
    end_call(h, s);
  });
}

blr_status blr_lstsq_solve(blr_matrix h, const double* B, int64_t ldb, double* X, int64_t ldx, int32_t nrhs,
                           int32_t max_refine, double* resid_norms, void* stream) {
  if (!h || !B || !X) return fail(BLR_ERR_INVALID, "NULL argument");
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (h->steps_done != h->q) return fail(BLR_ERR_STATE, "factorization is incomplete");
  if (ldb < h->mu || ldx < h->nu || nrhs < 0) return fail(BLR_ERR_INVALID, "bad B or X shape");
  if (max_refine < 0) return fail(BLR_ERR_INVALID, "max_refine must be >= 0");
  if (max_refine > 0 && h->acopy.empty())
    return fail(BLR_ERR_STATE, "refinement needs the copy of A~ kept by a factor with keep_a");
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    const int64_t m = h->m, n = h->n;
    begin_call(h);
    {
      SingCheck sc = sing_launch(h, s);
      HIPCHECK(hipStreamSynchronize(s));
      if (!sing_ok(h, sc)) throw Error(BLR_ERR_SINGULAR, "R is numerically singular");
      reset_work_after_sync(h);
    }
    // a ragged matrix solves its embedding for [B; 0]; X is the leading rows
    // of the embedding's solution
    const double* Bw = B;
    int64_t ldbw = ldb;
    double* Xw = X;
    int64_t ldxw = ldx;
    if (h->ragged()) {
      Bw = pad_rows(h, B, ldb, h->mu, h->m, nrhs, s);
      ldbw = h->m;
      Xw = (double*)h->work.alloc((size_t)h->n * nrhs * 8);
      ldxw = h->n;
    }
    Work w = make_work(h, nrhs);
    auto apply = [&](double* C, int trans) {
      Plan P;
      plan_apply(h, P, w, C, m, nrhs, trans);
      run_plan(h, P, s);
    };
    auto frob2 = [&](const double* C, int64_t ld, int64_t rows, double* out) {
      std::vector<Frob2Desc> fr(nrhs);
      for (int c = 0; c < nrhs; ++c) fr[c] = Frob2Desc{C + (int64_t)c * ld, ld, (int)rows, 1, out + c};
      Frob2Desc* dfr = upload_vec(h, fr, s);
      if (rows > 0) HIPCHECK(launch_frob2(dfr, nrhs, s));
      else HIPCHECK(hipMemsetAsync(out, 0, nrhs * 8, s));
    };
    // Q^T B, then X = R^{-1} (Q^T B)[0:n]
    double* C = (double*)h->work.alloc((size_t)m * nrhs * 8);
    HIPCHECK(hipMemcpy2DAsync(C, m * 8, Bw, ldbw * 8, m * 8, nrhs, hipMemcpyDeviceToDevice, s));
    apply(C, 0);
    if (resid_norms && max_refine == 0) frob2(C + n, m, m - n, resid_norms);
    HIPCHECK(hipMemcpy2DAsync(Xw, ldxw * 8, C, m * 8, n * 8, nrhs, hipMemcpyDeviceToDevice, s));
    run_rsolve(h, Xw, ldxw, nrhs, 0, s);
    if (max_refine > 0) {
      // iterative refinement of [I A~; A~^T 0][r; x] = [b; 0] with FP64 residuals
      double* r = (double*)h->work.alloc((size_t)m * nrhs * 8);     // residual b - A~ x
      double* f = (double*)h->work.alloc((size_t)m * nrhs * 8);
      double* g = (double*)h->work.alloc((size_t)n * nrhs * 8);
      double* dr = (double*)h->work.alloc((size_t)m * nrhs * 8);
      double* nrm = (double*)h->work.alloc((size_t)2 * nrhs * 8);
      // r = Q [0; (Q^T b)[n:m]]
      HIPCHECK(launch_lincomb(r, m, C, m, nullptr, 0, nullptr, 0, 0.0, 0.0, 0.0, (int)n, nrhs, s));
      HIPCHECK(launch_lincomb(r + n, m, C + n, m, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, (int)(m - n), nrhs, s));
      apply(r, 1);
      const double u = 2.220446049250313e-16;
      std::vector<double> hn(2 * nrhs), prev(nrhs, HUGE_VAL);
      std::vector<char> active(nrhs, 1), take(nrhs, 0);
      // one refinement step as one launch list, planned and uploaded once:
      // f = b - r - A~ x, g = -A~^T r; d = Q^T f; h = R^{-T} g;
      // dr = Q [h; d_2]; dx = R^{-1} (d_1 - h); the squared norms of dx and x
      auto lc = [](double* out, int64_t ldo, const double* x, int64_t lx, const double* y, int64_t ly,
                   const double* z, int64_t lz, double a, double b, double c, int64_t rows, int cols) {
        return LincombDesc{out, ldo, x, lx, y, ly, z, lz, a, b, c, (int32_t)rows, cols};
      };
      Plan RP;
      const RsolveWork rw = make_rsolve_work(h, nrhs);
      plan_matmul(h, RP, BLR_MATMUL_A, Xw, ldxw, f, m, nrhs);
      plan_matmul(h, RP, BLR_MATMUL_AT, r, m, g, n, nrhs);
      RP.lincomb(lc(f, m, Bw, ldbw, r, m, f, m, 1.0, -1.0, -1.0, m, nrhs));
      plan_apply(h, RP, w, f, m, nrhs, 0);
      RP.lincomb(lc(g, n, g, n, nullptr, 0, nullptr, 0, -1.0, 0.0, 0.0, n, nrhs));
      plan_rsolve(h, RP, rw, g, n, nrhs, 1);
      RP.lincomb(lc(dr, m, g, n, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, n, nrhs));
      RP.lincomb(lc(dr + n, m, f + n, m, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, m - n, nrhs));
      plan_apply(h, RP, w, dr, m, nrhs, 1);
      RP.lincomb(lc(f, m, f, m, g, n, nullptr, 0, 1.0, -1.0, 0.0, n, nrhs));
      plan_rsolve(h, RP, rw, f, m, nrhs, 0);
      {
        std::vector<Frob2Desc> fr(2 * nrhs);
        for (int c = 0; c < nrhs; ++c) {
          fr[c] = Frob2Desc{f + (int64_t)c * m, m, (int32_t)n, 1, nrm + c};
          fr[nrhs + c] = Frob2Desc{Xw + (int64_t)c * ldxw, ldxw, (int32_t)n, 1, nrm + nrhs + c};
        }
        RP.frob2(fr);
      }
      RP.upload(h->work, h->keep, s);
      // the step is captured into a graph on one of the handle's own streams
      // (capturing launches nothing; the caller's stream may be the legacy
      // default stream, which cannot be captured) and replayed on s; every
      // op is a kernel, so the graph holds kernel nodes only
      ensure_streams(h);
      hipGraph_t graph = nullptr;
      hipGraphExec_t gexec = nullptr;
      int64_t step_launches = 0;
      {
        const bool prof = h->prof_on;
        h->prof_on = false;
        const int64_t l0 = h->launches;
        hipStream_t cs = h->streams[0];
        HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        struct CaptureGuard {   // an error inside the capture still ends it
          hipStream_t st;
          bool open = true;
          ~CaptureGuard() {
            if (!open) return;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
          }
        } guard{cs};
        execute(h, RP, cs);
        guard.open = false;
        HIPCHECK(hipStreamEndCapture(cs, &graph));
        h->prof_on = prof;
        step_launches = h->launches - l0;
        h->launches = l0;
        HIPCHECK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      }
      for (int it = 0; it < max_refine; ++it) {
        HIPCHECK(hipGraphLaunch(gexec, s));
        h->launches += step_launches;
        HIPCHECK(hipMemcpyAsync(hn.data(), nrm, 2 * nrhs * 8, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        const bool done = refine_decide(hn, prev, active, take, nrhs, u);
        // x += dx, r += dr on the columns that take it
        for (auto [c0, c1] : take_runs(take)) {
          const int nc = c1 - c0;
          HIPCHECK(launch_lincomb(Xw + c0 * ldxw, ldxw, Xw + c0 * ldxw, ldxw, f + c0 * m, m, nullptr, 0, 1.0, 1.0, 0.0,
                                  (int)n, nc, s));
          HIPCHECK(launch_lincomb(r + c0 * m, m, r + c0 * m, m, dr + c0 * m, m, nullptr, 0, 1.0, 1.0, 0.0, (int)m,
                                  nc, s));
        }
        if (done) break;
      }
      HIPCHECK(hipGraphExecDestroy(gexec));
      HIPCHECK(hipGraphDestroy(graph));
      if (resid_norms) frob2(r, m, m, resid_norms);
    }
    if (Xw != X) HIPCHECK(hipMemcpy2DAsync(X, ldx * 8, Xw, ldxw * 8, h->nu * 8, nrhs, hipMemcpyDeviceToDevice, s));
    end_call(h, s);
    HIPCHECK(hipStreamSynchronize(s));
  });
}

blr_status blr_lstsq_solve_batch(blr_matrix* hs, int32_t count, const double* const* B, const int64_t* ldb,
                                 double* const* X, const int64_t* ldx, int32_t nrhs, int32_t max_refine,
                                 void* stream) {
  if (!hs || !B || !ldb || !X || !ldx || count < 1) return fail(BLR_ERR_INVALID, "NULL argument or count < 1");
  if (nrhs < 0 || max_refine < 0) return fail(BLR_ERR_INVALID, "nrhs and max_refine must be >= 0");
  std::vector<blr_matrix> v(hs, hs + count);
  for (int i = 0; i < count; ++i) {
    blr_matrix h = v[i];
    if (!h || !B[i] || !X[i]) return fail(BLR_ERR_INVALID, "NULL handle or pointer in the batch");
    for (int j = 0; j < i; ++j)
      if (v[j] == h) return fail(BLR_ERR_INVALID, "a handle appears twice in the batch");
    if (h->state != BLR_STATE_FACTORED || h->steps_done != h->q)
      return fail(BLR_ERR_STATE, "a matrix of the batch is not (fully) factored");
    if (ldb[i] < h->mu || ldx[i] < h->nu) return fail(BLR_ERR_INVALID, "bad B or X shape");
    if (max_refine > 0 && h->acopy.empty())
      return fail(BLR_ERR_STATE, "refinement needs the copy of A~ kept by a factor with keep_a");
  }
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    for (int i = 0; i < count; ++i) begin_call(v[i]);
    std::vector<SingCheck> sc(count);
    for (int i = 0; i < count; ++i) sc[i] = sing_launch(v[i], s);
    HIPCHECK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {
      if (!sing_ok(v[i], sc[i]))
        throw Error(BLR_ERR_SINGULAR, "R of batch member " + std::to_string(i) + " is numerically singular");
      reset_work_after_sync(v[i]);
    }
    // ragged members solve their embedding for [B; 0] (see blr_lstsq_solve)
    std::vector<const double*> Bw(B, B + count);
    std::vector<double*> Xw(X, X + count);
    std::vector<int64_t> ldbw(ldb, ldb + count), ldxw(ldx, ldx + count);
    for (int i = 0; i < count; ++i)
      if (v[i]->ragged()) {
        Bw[i] = pad_rows(v[i], B[i], ldb[i], v[i]->mu, v[i]->m, nrhs, s);
        ldbw[i] = v[i]->m;
        Xw[i] = (double*)v[i]->work.alloc((size_t)v[i]->n * nrhs * 8);
        ldxw[i] = v[i]->n;
      }
    struct Member {
      Work w;
      RsolveWork rw;
      double *C = nullptr, *r = nullptr, *f = nullptr, *g = nullptr, *dr = nullptr, *nrm = nullptr;
      std::vector<double> hn, prev;
      std::vector<char> cact, take;
      bool active = true;
    };
    std::vector<Member> mb(count);
    auto run = [&](std::vector<Plan>& plans) {
      std::vector<Plan> live;
      std::vector<blr_matrix> hv;
      for (int i = 0; i < count; ++i)
        if (!plans[i].ops.empty()) {
          live.push_back(std::move(plans[i]));
          hv.push_back(v[i]);
        }
      run_batch_plans(live, hv, s);
    };
    auto lc = [](double* out, int64_t ldo, const double* x, int64_t lx, const double* y, int64_t ly,
                 const double* z, int64_t lz, double a, double b, double c, int64_t rows, int cols) {
      return LincombDesc{out, ldo, x, lx, y, ly, z, lz, a, b, c, (int32_t)rows, cols};
    };
    // Q^T B, then X = R^{-1} (Q^T B)[0:n]; with refinement also r = Q [0; (Q^T b)[n:m]]
    std::vector<Plan> plans(count);
    for (int i = 0; i < count; ++i) {
      blr_matrix h = v[i];
      const int64_t m = h->m, n = h->n;
      Member& e = mb[i];
      Plan& P = plans[i];
      e.w = make_work(h, nrhs);
      e.rw = make_rsolve_work(h, nrhs);
      e.C = (double*)h->work.alloc((size_t)m * nrhs * 8);
      P.copy({CopyDesc{Bw[i], e.C, ldbw[i], m, (int32_t)m, nrhs, 0, 0, 0}});
      plan_apply(h, P, e.w, e.C, m, nrhs, 0);
      P.copy({CopyDesc{e.C, Xw[i], m, ldxw[i], (int32_t)n, nrhs, 0, 0, 0}});
      plan_rsolve(h, P, e.rw, Xw[i], ldxw[i], nrhs, 0);
      if (max_refine > 0) {
        e.r = (double*)h->work.alloc((size_t)m * nrhs * 8);
        e.f = (double*)h->work.alloc((size_t)m * nrhs * 8);
        e.g = (double*)h->work.alloc((size_t)n * nrhs * 8);
        e.dr = (double*)h->work.alloc((size_t)m * nrhs * 8);
        e.nrm = (double*)h->work.alloc((size_t)2 * nrhs * 8);
        e.hn.resize(2 * nrhs);
        e.prev.assign(nrhs, HUGE_VAL);
        e.cact.assign(nrhs, 1);
        e.take.assign(nrhs, 0);
        P.lincomb(lc(e.r, m, e.C, m, nullptr, 0, nullptr, 0, 0.0, 0.0, 0.0, n, nrhs));
        P.lincomb(lc(e.r + n, m, e.C + n, m, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, m - n, nrhs));
        plan_apply(h, P, e.w, e.r, m, nrhs, 1);
      }
    }
    run(plans);
    // refinement of [I A~; A~^T 0][r; x] = [b; 0] with FP64 residuals, the
    // steps of blr_lstsq_solve for every member still refining
    const double u = 2.220446049250313e-16;
    for (int it = 0; it < max_refine; ++it) {
      plans.assign(count, Plan());
      bool any = false;
      for (int i = 0; i < count; ++i) {
        Member& e = mb[i];
        if (!e.active) continue;
        any = true;
        blr_matrix h = v[i];
        const int64_t m = h->m, n = h->n;
        Plan& P = plans[i];
        plan_matmul(h, P, BLR_MATMUL_A, Xw[i], ldxw[i], e.f, m, nrhs);
        plan_matmul(h, P, BLR_MATMUL_AT, e.r, m, e.g, n, nrhs);
        P.lincomb(lc(e.f, m, Bw[i], ldbw[i], e.r, m, e.f, m, 1.0, -1.0, -1.0, m, nrhs));
        plan_apply(h, P, e.w, e.f, m, nrhs, 0);
        P.lincomb(lc(e.g, n, e.g, n, nullptr, 0, nullptr, 0, -1.0, 0.0, 0.0, n, nrhs));
        plan_rsolve(h, P, e.rw, e.g, n, nrhs, 1);
        P.lincomb(lc(e.dr, m, e.g, n, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, n, nrhs));
        P.lincomb(lc(e.dr + n, m, e.f + n, m, nullptr, 0, nullptr, 0, 1.0, 0.0, 0.0, m - n, nrhs));
        plan_apply(h, P, e.w, e.dr, m, nrhs, 1);
        P.lincomb(lc(e.f, m, e.f, m, e.g, n, nullptr, 0, 1.0, -1.0, 0.0, n, nrhs));
        plan_rsolve(h, P, e.rw, e.f, m, nrhs, 0);
        std::vector<Frob2Desc> fr(2 * nrhs);
        for (int c = 0; c < nrhs; ++c) {
          fr[c] = Frob2Desc{e.f + (int64_t)c * m, m, (int32_t)n, 1, e.nrm + c};
          fr[nrhs + c] = Frob2Desc{Xw[i] + (int64_t)c * ldxw[i], ldxw[i], (int32_t)n, 1, e.nrm + nrhs + c};
        }
        P.frob2(fr);
      }
      if (!any) break;
      run(plans);
      for (int i = 0; i < count; ++i)
        if (mb[i].active)
          HIPCHECK(hipMemcpyAsync(mb[i].hn.data(), mb[i].nrm, 2 * nrhs * 8, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      // x += dx, r += dr on the columns that take the step
      plans.assign(count, Plan());
      for (int i = 0; i < count; ++i) {
        Member& e = mb[i];
        if (!e.active) continue;
        if (refine_decide(e.hn, e.prev, e.cact, e.take, nrhs, u)) e.active = false;
        blr_matrix h = v[i];
        const int64_t m = h->m, n = h->n;
        for (auto [c0, c1] : take_runs(e.take)) {
          const int nc = c1 - c0;
          plans[i].lincomb(lc(Xw[i] + c0 * ldxw[i], ldxw[i], Xw[i] + c0 * ldxw[i], ldxw[i], e.f + c0 * m, m, nullptr, 0,
                              1.0, 1.0, 0.0, n, nc));
          plans[i].lincomb(lc(e.r + c0 * m, m, e.r + c0 * m, m, e.dr + c0 * m, m, nullptr, 0, 1.0, 1.0, 0.0, m, nc));
        }
      }
      run(plans);
    }
    for (int i = 0; i < count; ++i)
      if (Xw[i] != X[i])
        HIPCHECK(hipMemcpy2DAsync(X[i], ldx[i] * 8, Xw[i], ldxw[i] * 8, v[i]->nu * 8, nrhs, hipMemcpyDeviceToDevice,
                                  s));
    for (int i = 0; i < count; ++i) end_call(v[i], s);
    HIPCHECK(hipStreamSynchronize(s));
  });
}

blr_status blr_rsolve(blr_matrix h, int32_t trans, double* X, int64_t ldx, int32_t nrhs, void* stream) {
  if (!h || !X) return fail(BLR_ERR_INVALID, "NULL argument");
  if (trans != 0 && trans != 1) return fail(BLR_ERR_INVALID, "trans must be 0 or 1");
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (h->steps_done != h->q) return fail(BLR_ERR_STATE, "factorization is incomplete");
  if (ldx < h->nu || nrhs < 0) return fail(BLR_ERR_INVALID, "bad X shape");
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    begin_call(h);
    if (!h->ragged()) {
      run_rsolve(h, X, ldx, nrhs, trans, s);
    } else {
      // R = diag(R_A, -I): the embedding's solve of X padded by zero rows
      double* Xp = pad_rows(h, X, ldx, h->nu, h->n, nrhs, s);
      run_rsolve(h, Xp, h->n, nrhs, trans, s);
      HIPCHECK(hipMemcpy2DAsync(X, ldx * 8, Xp, h->n * 8, h->nu * 8, nrhs, hipMemcpyDeviceToDevice, s));
    }
    end_call(h, s);
  });
}

// Adjoint of X = argmin ||A~ X - B|| (full column rank): Z = R^{-1} R^{-T} Xbar,
// Rs = B - A~ X, Bbar = A~ Z, and dL/dA~ = Rs Z^T - Bbar X^T restricted to the
// stored tiles of A~ (dense: the b x b block; low-rank U V^T: dU = dA V and
// dV = dA^T U, formed from small products with the factors).
blr_status blr_lstsq_adjoint(blr_matrix h, const double* B, int64_t ldb, const double* X, int64_t ldx,
                             const double* Xbar, int64_t ldxb, int32_t nrhs, double* Bbar, int64_t ldbb,
                             double* dD, double* dU, double* dV, void* stream) {
  if (!h || !B || !X || !Xbar || !Bbar) return fail(BLR_ERR_INVALID, "NULL argument");
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (h->steps_done != h->q) return fail(BLR_ERR_STATE, "factorization is incomplete");
  if (h->acopy.empty()) return fail(BLR_ERR_STATE, "the adjoint needs the copy of A~ kept by a factor with keep_a");
  if (h->ragged()) return fail(BLR_ERR_INVALID, "the adjoint needs b to divide m and n");
  if (ldb < h->m || ldx < h->n || ldxb < h->n || ldbb < h->m || nrhs < 0)
    return fail(BLR_ERR_INVALID, "bad B, X, Xbar or Bbar shape");
  if (nrhs == 0) return BLR_OK;
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    const int b = h->b, rc = h->rc, p = h->p, q = h->q;
    const int64_t m = h->m, n = h->n;
    begin_call(h);
    double* Z = (double*)h->work.alloc((size_t)n * nrhs * 8);
    double* Rs = (double*)h->work.alloc((size_t)m * nrhs * 8);
    // Z = R^{-1} R^{-T} Xbar
    HIPCHECK(hipMemcpy2DAsync(Z, n * 8, Xbar, ldxb * 8, n * 8, nrhs, hipMemcpyDeviceToDevice, s));
    run_rsolve(h, Z, n, nrhs, 1, s);
    run_rsolve(h, Z, n, nrhs, 0, s);
    // Rs = B - A~ X, Bbar = A~ Z
    {
      Plan P;
      plan_matmul(h, P, BLR_MATMUL_A, X, ldx, Rs, m, nrhs);
      plan_matmul(h, P, BLR_MATMUL_A, Z, n, Bbar, ldbb, nrhs);
      run_plan(h, P, s);
    }
    HIPCHECK(launch_lincomb(Rs, m, B, ldb, Rs, m, nullptr, 0, 1.0, -1.0, 0.0, (int)m, nrhs, s));
    // tile gradients
    std::vector<Tile>& T = h->acopy;
    int nlr = 0;
    for (auto& t : T) nlr += t.fmt == LOWRANK;
    double* S = (double*)h->work.alloc((size_t)std::max(nlr, 1) * 4 * rc * nrhs * 8);
    Plan P;
    int l = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j) {
        Tile& t = T[(size_t)i * q + j];
        const double* Rsi = Rs + (int64_t)i * b;
        const double* Bbi = Bbar + (int64_t)i * b;
        const double* Zj = Z + (int64_t)j * b;
        const double* Xj = X + (int64_t)j * b;
        const size_t tix = (size_t)i * q + j;
        if (t.fmt == DENSE) {
          if (dD) P.gemm(dD + tix * b * b, b, nullptr, 0, nullptr, 0, b, b, 1.0, 0.0, Rsi, m, Zj, n, nrhs,
                         SEG_TRANS_B);
        } else if (dU || dV) {
          double* S1 = S + (size_t)l * 4 * rc * nrhs;   // V^T Z_j, V^T X_j, U^T Rs_i, U^T Bbar_i (rc x nrhs each)
          P.gemm(S1, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.Vt, rc, Zj, n, b, 0);
          P.gemm(S1 + (size_t)rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.Vt, rc, Xj, ldx, b, 0);
          P.gemm(S1 + (size_t)2 * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.U, b, Rsi, m, b,
                 SEG_TRANS_A);
          P.gemm(S1 + (size_t)3 * rc * nrhs, rc, nullptr, 0, nullptr, 0, rc, nrhs, 1.0, 0.0, t.U, b, Bbi, ldbb, b,
                 SEG_TRANS_A);
          ++l;
        }
      }
    P.flush_gemm(0, 0, false);
    l = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j) {
        Tile& t = T[(size_t)i * q + j];
        const double* Rsi = Rs + (int64_t)i * b;
        const double* Bbi = Bbar + (int64_t)i * b;
        const double* Zj = Z + (int64_t)j * b;
        const double* Xj = X + (int64_t)j * b;
        const size_t tix = (size_t)i * q + j;
        if (t.fmt == DENSE) {
          if (dD) {
            double* C = dD + tix * b * b;
            P.gemm(C, b, C, b, nullptr, 0, b, b, -1.0, 1.0, Bbi, ldbb, Xj, ldx, nrhs, SEG_TRANS_B);
          }
        } else if (dU || dV) {
          const double* S1 = S + (size_t)l * 4 * rc * nrhs;
          if (dU) {   // dU = Rs_i (V^T Z_j)^T - Bbar_i (V^T X_j)^T
            double* C = dU + tix * b * rc;
            P.gemm(C, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Rsi, m, S1, rc, nrhs, SEG_TRANS_B);
          }
          if (dV) {   // dV = Z_j (U^T Rs_i)^T - X_j (U^T Bbar_i)^T
            double* C = dV + tix * b * rc;
            P.gemm(C, b, nullptr, 0, nullptr, 0, b, rc, 1.0, 0.0, Zj, n, S1 + (size_t)2 * rc * nrhs, rc, nrhs,
                   SEG_TRANS_B);
          }
          ++l;
        }
      }
    P.flush_gemm(0, 0, false);
    l = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < q; ++j) {
        Tile& t = T[(size_t)i * q + j];
        if (t.fmt == DENSE || !(dU || dV)) continue;
        const double* Bbi = Bbar + (int64_t)i * b;
        const double* Xj = X + (int64_t)j * b;
        const size_t tix = (size_t)i * q + j;
        const double* S1 = S + (size_t)l * 4 * rc * nrhs;
        if (dU) {
          double* C = dU + tix * b * rc;
          P.gemm(C, b, C, b, nullptr, 0, b, rc, -1.0, 1.0, Bbi, ldbb, S1 + (size_t)rc * nrhs, rc, nrhs, SEG_TRANS_B);
        }
        if (dV) {
          double* C = dV + tix * b * rc;
          P.gemm(C, b, C, b, nullptr, 0, b, rc, -1.0, 1.0, Xj, ldx, S1 + (size_t)3 * rc * nrhs, rc, nrhs,
                 SEG_TRANS_B);
        }
        ++l;
      }
    P.flush_gemm(0, 0, false);
    run_plan(h, P, s);
    end_call(h, s);
  });
}

// Explicit Q~ (Section 3.3: Q~ is a BLR matrix with the structure of A~ and
// the same threshold): the thin Q [I; 0] is formed densely, a block of
// columns at a time, and compressed with A~'s tile formats as the mask.
blr_status blr_form_q(blr_matrix h, void* stream, blr_matrix* q_out) {
  if (!h || !q_out) return fail(BLR_ERR_INVALID, "NULL argument");
  *q_out = nullptr;
  if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
  if (h->steps_done != h->q) return fail(BLR_ERR_STATE, "factorization is incomplete");
  if (h->ragged()) return fail(BLR_ERR_INVALID, "the explicit Q needs b to divide m and n");
  hipStream_t s = as_stream(stream);
  blr_status inner = BLR_OK;
  blr_status st = run_guarded([&] {
    const int b = h->b, p = h->p, q = h->q;
    const int64_t m = h->m, n = h->n;
    // the dense m x n block is stream-ordered memory: allocated and freed on
    // s, so that neither waits for other work on the device
    struct DevBuf {
      double* p = nullptr;
      hipStream_t s = nullptr;
      ~DevBuf() {
        if (p) (void)hipFreeAsync(p, s);
      }
    } E;
    begin_call(h);
    E.s = s;
    HIPCHECK(hipMallocAsync((void**)&E.p, (size_t)m * n * 8, s));
    HIPCHECK(hipMemsetAsync(E.p, 0, (size_t)m * n * 8, s));
    {
      Plan P;   // the identity in the top n x n block (unit-lower copy of zeros, in place)
      P.copy({CopyDesc{E.p, E.p, m, m, (int)n, (int)n, 1, 0}});
      run_plan(h, P, s);
    }
    // Q [I; 0], a block of columns at a time; the workspace of one block is
    // reused for the next once the stream has finished it
    const int64_t nc = std::min<int64_t>(n, 4096);
    for (int64_t c0 = 0; c0 < n; c0 += nc) {
      const int cols = (int)std::min<int64_t>(nc, n - c0);
      HIPCHECK(hipStreamSynchronize(s));
      reset_work_after_sync(h);
      Work w = make_work(h, cols);
      Plan P;
      plan_apply(h, P, w, E.p + c0 * m, m, cols, 1);
      run_plan(h, P, s);
    }
    end_call(h, s);
    std::vector<int8_t> mask((size_t)p * q);
    for (size_t t = 0; t < mask.size(); ++t) mask[t] = h->fmt0[t] == LOWRANK ? 1 : 0;
    blr_source src{};
    src.kind = BLR_SRC_DENSE;
    src.A = E.p;
    src.lda = m;
    src.admissibility = BLR_ADM_MASK;
    src.mask = mask.data();
    blr_compress_opts co{};
    co.m = m;
    co.n = n;
    co.tile = b;
    co.tol = h->tol;
    co.max_rank = h->cap;
    co.overflow = BLR_OVERFLOW_DENSE;
    inner = blr_compress(&src, &co, stream, q_out);
    if (inner != BLR_OK) throw Error(inner, blr_last_error());
  });
  return st;
}

blr_status blr_morton_sort(const double* pts, int64_t n, int32_t dim, int64_t* perm, double* sorted,
                           void* stream) {
  if (!pts || !perm) return fail(BLR_ERR_INVALID, "NULL argument");
  if (n < 0 || dim < 1 || dim > 3) return fail(BLR_ERR_INVALID, "n must be >= 0 and dim in 1..3");
  return run_guarded([&] { HIPCHECK(morton_sort(pts, n, dim, perm, sorted, as_stream(stream))); });
}

blr_status blr_matmul(blr_matrix h, int32_t op, const double* X, int64_t ldx, double* Y, int64_t ldy,
                      int32_t nrhs, void* stream) {
  if (!h || !X || !Y) return fail(BLR_ERR_INVALID, "NULL argument");
  if (op != BLR_MATMUL_A && op != BLR_MATMUL_AT && op != BLR_MATMUL_R) return fail(BLR_ERR_INVALID, "bad op");
  if (op == BLR_MATMUL_R) {
    if (h->state != BLR_STATE_FACTORED) return fail(BLR_ERR_STATE, "matrix is not factored");
    if (h->steps_done != h->q) return fail(BLR_ERR_STATE, "factorization is incomplete");
  } else if (h->state != BLR_STATE_COMPRESSED && h->acopy.empty()) {
    return fail(BLR_ERR_STATE, "the factorization has overwritten A (factor with keep_a to keep a copy)");
  }
  const int64_t xr = op == BLR_MATMUL_AT ? h->mu : h->nu;
  const int64_t yr = op == BLR_MATMUL_A ? h->mu : h->nu;
  if (nrhs < 0 || ldx < xr || ldy < yr) return fail(BLR_ERR_INVALID, "bad X or Y shape");
  if (nrhs == 0) return BLR_OK;
  {
    const char* xb = (const char*)X;
    const char* yb = (const char*)Y;
    const char* xe = xb + ((nrhs - 1) * ldx + xr) * 8;
    const char* ye = yb + ((nrhs - 1) * ldy + yr) * 8;
    if (xb < ye && yb < xe) return fail(BLR_ERR_INVALID, "X and Y overlap");
  }
  hipStream_t s = as_stream(stream);
  return run_guarded([&] {
    begin_call(h);
    if (!h->ragged()) {
      Plan P;
      plan_matmul(h, P, op, X, ldx, Y, ldy, nrhs);
      run_plan(h, P, s);
    } else {
      // the embedding's product with X padded by zero rows; Y is its leading rows
      const int64_t xe = op == BLR_MATMUL_AT ? h->m : h->n;
      const int64_t ye = op == BLR_MATMUL_A ? h->m : h->n;
      const double* Xp = pad_rows(h, X, ldx, xr, xe, nrhs, s);
      double* Yp = (double*)h->work.alloc((size_t)ye * nrhs * 8);
      Plan P;
      plan_matmul(h, P, op, Xp, xe, Yp, ye, nrhs);
      run_plan(h, P, s);
      HIPCHECK(hipMemcpy2DAsync(Y, ldy * 8, Yp, ye * 8, yr * 8, nrhs, hipMemcpyDeviceToDevice, s));
    }
    end_call(h, s);
  });
}

blr_status blr_query(blr_matrix h, blr_info* info) {
  if (!h || !info) return fail(BLR_ERR_INVALID, "NULL argument");
  return run_guarded([&] {
    wait_idle(h);
    std::memset(info, 0, sizeof(*info));
    info->m = h->mu;
    info->n = h->nu;
    info->tile = h->b;
    info->p = h->pu;
    info->q = h->q;
    info->m_pad = h->m;
    info->n_pad = h->n;
    info->p_pad = h->p;
    info->max_rank = h->cap;
    info->rank_capacity = h->rc;
    info->state = h->state;
    info->variant = h->variant;
    info->precision = h->precision;
    info->ib = h->ib;
    for (auto& t : h->tiles) (t.fmt == DENSE ? info->n_dense : info->n_lowrank)++;
    info->n_fill_in = h->n_fill;
    info->device_bytes = h->mem.bytes + h->work.bytes;
    info->compress_overflow = h->compress_overflow;
    unsigned long long c[2] = {0, 0};
    HIPCHECK(hipMemcpy(c, h->d_counters, sizeof(c), hipMemcpyDeviceToHost));
    info->factor_overflow = (int64_t)c[0];
    double md;
    std::memcpy(&md, &c[1], sizeof(md));
    info->max_dropped_rel = md;
    info->flops_factor = h->flops;
    info->kernel_launches = h->launches;
  });
}

void blr_destroy(blr_matrix h) {
  if (!h) return;
  // the handle's own work must end before its memory is freed
  if (h->idle_set) (void)hipEventSynchronize(h->idle);
  for (auto st : h->streams) (void)hipStreamSynchronize(st);
  for (int k = 0; k < 2; ++k)
    for (auto e : h->prof_ev[k]) (void)hipEventDestroy(e);
  for (auto st : h->streams) (void)hipStreamDestroy(st);
  if (h->idle) (void)hipEventDestroy(h->idle);
  delete h;
}

blr_status blr_profile_enable(blr_matrix h, int32_t on) {
  if (!h) return fail(BLR_ERR_INVALID, "NULL argument");
  h->prof_on = on != 0;
  return BLR_OK;
}

blr_status blr_profile_read(blr_matrix h, int32_t kernel, int64_t* launches, double* total_ms,
                            double* total_flops) {
  if (!h || !launches || !total_ms || !total_flops) return fail(BLR_ERR_INVALID, "NULL argument");
  if (kernel != 0 && kernel != 1) return fail(BLR_ERR_INVALID, "kernel must be 0 (FP64) or 1 (FP32)");
  return run_guarded([&] {
    wait_idle(h);
    double ms = 0.0;
    const auto& ev = h->prof_ev[kernel];
    for (size_t a = 0; a + 1 < ev.size(); a += 2) {
      float t = 0.f;
      HIPCHECK(hipEventElapsedTime(&t, ev[a], ev[a + 1]));
      ms += t;
    }
    *launches = h->prof_launches[kernel];
    *total_ms = ms;
    *total_flops = h->prof_flops[kernel];
  });
}

}  // extern "C"

#include "../../include/blrqr_selftest.h"

extern "C" blr_status blr_selftest_gemm(int32_t flags, int32_t M, int32_t N, int32_t K, double alpha,
                                        const double* A, int64_t lda, const double* B, int64_t ldb,
                                        double beta, double* C, int64_t ldc, int32_t fp32, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 0) return fail(BLR_ERR_INVALID, "bad arguments");
  return run_guarded([&] {
    Arena ar;
    HostKeep keep;
    Plan P;
    P.gemm(C, ldc, C, ldc, nullptr, 0, M, N, alpha, beta, A, lda, B, ldb, K, flags);
    P.flush_gemm(fp32);
    if (P.ops.empty()) return;
    P.upload(ar, keep, as_stream(stream));
    HIPCHECK(launch_gemm(P.d_descs, P.ops[0].n, P.d_segs, P.ops[0].ntiles, P.ops[0].big, P.ops[0].fp32,
                         as_stream(stream)));
    HIPCHECK(hipStreamSynchronize(as_stream(stream)));
  });
}
