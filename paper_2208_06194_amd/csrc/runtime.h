// Host runtime of libblrqr: handle, device memory, launch plans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/blrqr.h"
#include "gemm.h"
#include "lowrank.h"
#include "misc.h"
#include "morton.h"
#include "qr.h"

namespace blr {

enum Fmt : int8_t { DENSE = 0, LOWRANK = 1 };

struct Error : std::runtime_error {
  blr_status code;
  Error(blr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what);
#define HIPCHECK(x) ::blr::hip_check((x), #x)

struct Tile {
  int8_t fmt = DENSE;
  double* D = nullptr;   // dense slot b x b (ld b)
  double* U = nullptr;   // low-rank slot b x rc (ld b)
  double* Vt = nullptr;  // low-rank slot rc x b (ld rc); after TPQRT of a low-rank tile it holds Y
  int* rank = nullptr;   // device rank
};

// Source of device memory for a plan's descriptor arrays.
struct DevAlloc {
  virtual void* alloc(size_t n) = 0;
  virtual ~DevAlloc() = default;
};

// Device arena: every allocation is released by the owner's destructor.
struct Arena : DevAlloc {
  std::vector<void*> blocks;
  int64_t bytes = 0;
  void* alloc(size_t n) override;
  void release();
  ~Arena() override { release(); }
};

// Grow-only device workspace of a handle: bump allocation over chunks that
// are kept across calls.  reset() makes every chunk free again without
// freeing it, so a call that repeats an earlier call's allocations allocates
// nothing; only a larger demand adds a chunk.  The caller resets only after
// the work that used the chunks has completed.
struct Workspace : DevAlloc {
  struct Chunk {
    char* p;
    size_t size, used;
  };
  std::vector<Chunk> chunks;
  size_t cur = 0;
  int64_t bytes = 0;
  void* alloc(size_t n) override;
  void reset();
  void release();
  ~Workspace() override { release(); }
};

// Host copies of uploaded descriptor arrays, kept until the handle's next
// call has waited for the copies (stream-ordered uploads read them late).
using HostKeep = std::vector<std::vector<char>>;

// One enqueued operation of a plan.
struct Op {
  enum Kind {
    GEMM, PANEL, PANEL_APPLY, TBACK, RC, TRSM, WAIT, RECORD, TALL_APPLY, COPY,
    // batched forms of the panel kernels (jobs [off, off + n) of the plan)
    PANEL_B, PANEL_APPLY_B, TBACK_B, TALL_APPLY_B,
    // solve steps: batched triangular solves, linear combinations, squared norms
    TRSM_B, LINCOMB, FROB2,
    // the Gram-Schmidt comparison method: QR of a stacked block column
    MGS_STACK,
    // tall panels as a tree: one level's QR launch, the reconstruction
    // (items [off, off + n) of the plan, ext workgroups)
    TSQR_QR, TSQR_FIN
  } kind;
  int off = 0, n = 0, ntiles = 0, big = 0, fp32 = 0, prof = 0;
  int ib = 0, ext = 0, ext2 = 0, first = 0;   // batched panel ops: width, largest extents, first column
  int stream = 0;   // index into the plan's streams
  int prio = 0;     // merge order of a multi-stream plan: lower goes first (the block column)
  int event = -1;   // WAIT / RECORD: event index
  double flops = 0.0;
  PanelArgs panel{};
  TBackArgs tback{};
  TrsmJob trsm{};         // TRSM: the solve (n: 1 = with R^T)
  double* buf = nullptr;   // TALL_APPLY: partial sums
  int64_t maxel = 0;       // COPY: largest block
  struct {                 // MGS_STACK: X (h x w, ld ldx) -> Q, R (ld ldr)
    double* X;
    int64_t ldx;
    int h, w;
    double* R;
    int64_t ldr;
  } mgs{};
};

// Launch list with host-side descriptor arrays, uploaded once.
struct Plan {
  std::vector<Op> ops;
  std::vector<GemmDesc> descs;
  std::vector<GemmSeg> segs;
  std::vector<RcDesc> rcs;
  std::vector<CopyDesc> copies;
  std::vector<PanelJob> jobs;
  std::vector<TrsmJob> tjobs;
  std::vector<LincombDesc> lincs;
  std::vector<Frob2Desc> frobs;
  std::vector<TsqrTree> trees;
  std::vector<TsqrItem> titems;
  TsqrTree* d_trees = nullptr;
  TsqrItem* d_titems = nullptr;
  CopyDesc* d_copies = nullptr;
  PanelJob* d_jobs = nullptr;
  TrsmJob* d_tjobs = nullptr;
  LincombDesc* d_lincs = nullptr;
  Frob2Desc* d_frobs = nullptr;
  GemmDesc* d_descs = nullptr;
  GemmSeg* d_segs = nullptr;
  RcDesc* d_rcs = nullptr;
  // building helpers
  std::vector<GemmDesc> cur;     // descriptors of the GEMM op being built
  std::vector<GemmSeg> curseg;
  double curflops = 0.0;
  std::vector<RcDesc> currc;
  int cur_stream = 0;
  int cur_prio = 0;
  int n_events = 0;

  // add one descriptor with a single K segment
  void gemm(double* C, int64_t ldc, const double* Cin, int64_t ldcin, double* D2, int64_t ldd2,
            int M, int N, double alpha, double beta, const double* A, int64_t lda, const double* B,
            int64_t ldb, int K, int segflags, int descflags = 0);
  // add one descriptor summing several K segments: C = alpha * sum_s op(A_s) op(B_s) + beta * Cin
  void gemm_multi(double* C, int64_t ldc, const double* Cin, int64_t ldcin, int M, int N, double alpha,
                  double beta, const std::vector<GemmSeg>& segs);
  // allow_fast = false keeps the batch on the generic kernels (used outside
  // the factorization, so that the fast kernels time only its products)
  void flush_gemm(int fp32 = 0, int prof = 0, bool allow_fast = true);
  void rc(const RcDesc& d) { currc.push_back(d); }
  void flush_rc();
  void push(Op o) {
    o.stream = cur_stream;
    o.prio = cur_prio;
    ops.push_back(o);
  }
  void panel(const PanelArgs& a) { Op o; o.kind = Op::PANEL; o.panel = a; push(o); }
  void panel_apply(const PanelArgs& a, int nt) { Op o; o.kind = Op::PANEL_APPLY; o.panel = a; o.n = nt; push(o); }
  void tback(const TBackArgs& a) { Op o; o.kind = Op::TBACK; o.tback = a; push(o); }
  void copy(const std::vector<CopyDesc>& v) {
    if (v.empty()) return;
    Op o;
    o.kind = Op::COPY;
    o.off = (int)copies.size();
    o.n = (int)v.size();
    for (auto& c : v) o.maxel = std::max<int64_t>(o.maxel, (int64_t)c.rows * c.cols);
    copies.insert(copies.end(), v.begin(), v.end());
    push(o);
  }
  // out = a x + b y + c z on a rows x cols block (one launch)
  void lincomb(const LincombDesc& d) {
    if ((int64_t)d.rows * d.cols <= 0) return;
    Op o;
    o.kind = Op::LINCOMB;
    o.off = (int)lincs.size();
    o.n = 1;
    o.maxel = (int64_t)d.rows * d.cols;
    lincs.push_back(d);
    push(o);
  }
  void frob2(const std::vector<Frob2Desc>& v) {
    if (v.empty()) return;
    Op o;
    o.kind = Op::FROB2;
    o.off = (int)frobs.size();
    o.n = (int)v.size();
    frobs.insert(frobs.end(), v.begin(), v.end());
    push(o);
  }
  void mgs_stack(double* X, int64_t ldx, int h, int w, double* R, int64_t ldr) {
    Op o;
    o.kind = Op::MGS_STACK;
    o.mgs = {X, ldx, h, w, R, ldr};
    o.flops = 2.0 * h * w * w;
    push(o);
  }
  void wait(int e) { Op o; o.kind = Op::WAIT; o.event = e; push(o); n_events = std::max(n_events, e + 1); }
  void record(int e) { Op o; o.kind = Op::RECORD; o.event = e; push(o); n_events = std::max(n_events, e + 1); }
  // copy the descriptor arrays to device memory from a, enqueued on s; the
  // host sources are copied into keep first
  void upload(DevAlloc& a, HostKeep& keep, hipStream_t s);
  // device bytes upload() takes from an allocator that rounds each array up
  // to 256 bytes
  size_t upload_bytes() const;
  void clear();
};

}  // namespace blr

struct blr_matrix_s {
  // m x n and p x q tiles of the matrix the kernels factor.  When b does not
  // divide the caller's mu or nu it is the embedding [A 0; 0 E] of A
  // (mu x nu): zero rows and columns pad A to whole tiles, and E holds an
  // identity block in the padded columns (rows mu .. mu + n - nu - 1), so
  // that the embedding has full column rank; R = diag(R_A, -I) up to signs.
  int64_t m = 0, n = 0;
  int64_t mu = 0, nu = 0;   // the caller's rows and columns
  int pu = 0;               // tile rows holding rows of A (p, or p - 1 when E needs one more)
  int b = 0, p = 0, q = 0, cap = 0, rc = 0;
  double tol = 0.0;
  int overflow = 0;
  int state = BLR_STATE_COMPRESSED;
  int variant = 0, precision = 0, ib = 32;
  int steps_done = 0;
  std::vector<blr::Tile> tiles;          // p*q, i*q + j
  std::vector<blr::Tile> acopy;          // copy of A~ kept by a factor with keep_a (else empty)
  blr::Arena amem;                       // storage of acopy
  std::vector<int8_t> yfmt;              // p*q: format of Ytilde_ik after the factor
  std::vector<int8_t> fmt0;              // p*q: tile formats of A~ when the factor started
  std::vector<double*> T;                // p*q: T of tile (tiled) or of column (block column, at (k,k))
  std::vector<double*> tau;              // p*q
  int* d_rank = nullptr;
  unsigned long long* d_counters = nullptr;  // [0] overflow count, [1] max dropped bits
  blr::Arena mem;                        // tiles, T, ranks
  blr::Workspace work;                   // workspaces and plans of the calls, reused
  blr::HostKeep keep;                    // host sources of the last call's uploads
  hipEvent_t idle = nullptr;             // recorded at the end of every call's work
  bool idle_set = false;
  int64_t compress_overflow = 0;
  int64_t n_fill = 0;
  double flops = 0.0;
  int64_t launches = 0;
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev[2];     // [0] FP64, [1] FP32 fast untransposed products
  std::vector<hipStream_t> streams;      // look-ahead streams (created on first use)
  double prof_flops[2] = {0.0, 0.0};
  int64_t prof_launches[2] = {0, 0};

  blr::Tile& t(int i, int j) { return tiles[(size_t)i * q + j]; }
  bool ragged() const { return m != mu || n != nu; }
  // does tile (i, j) hold entries of the identity block E?
  bool has_identity(int i, int j) const {
    const int64_t pc = n - nu;
    if (pc == 0 || j != q - 1) return false;
    return (int64_t)i * b < mu + pc && (int64_t)(i + 1) * b > mu;
  }
};
