// Internal declarations of the cib library (host runtime + HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/cib.h"

namespace cib {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  cib_status code;
  Error(cib_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

#define CIB_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::cib::Error(CIB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CIB_REQUIRE(cond, code, msg)                                               \
  do {                                                                             \
    if (!(cond)) throw ::cib::Error((code), (msg));                                \
  } while (0)

constexpr int kMaxWords = 3;     // 64-bit words per species (nmax <= 6)
constexpr int kMaxBlock = 16;    // LOBPCG block size limit
constexpr int kMaxSeg = 127;     // 2M_B segments (7 bits in tile info)

}  // namespace cib

// ------------------------------------------------------------------ context
struct cib_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cib_allocator user{};
  bool has_user = false;
  std::mutex mu;
  // cache of freed blocks (hipMalloc path): size -> pointers
  std::unordered_multimap<size_t, void *> cache;
  std::unordered_map<void *, size_t> sizes;
  int64_t live = 0, peak = 0, cached = 0;
  bool busy = false;
  void *pinned = nullptr;  // small pinned host staging buffer
  // Handles made on this context and not yet freed.  cib_destroy while some
  // are live only marks the context; the free of the last one releases it.
  std::mutex life_mu;
  int64_t handles = 0;
  bool destroyed = false;
  size_t pinned_bytes = 0;

  // per-kernel event timing (cib_profile_*)
  bool profiling = false;
  struct Mark { int kernel; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  std::unordered_map<int, std::pair<int64_t, double>> kernel_totals;

  void *alloc(size_t bytes);
  void free(void *p);
  void release_cache();
  void *pinned_buf(size_t bytes);
};

namespace cib {

// Hot kernels known to the profiler.
enum KernelId { K_SCREEN = 0, K_ROW_COUNT, K_SCAN, K_ROW_FILL, K_SPMM, K_GRAM, K_RR, K_UPDATE, K_COUNT, K_APPLY_FREE, K_NKERN };
extern const char *const kKernelNames[K_NKERN];

// Timer marks recorded so far, and dropping the marks from index `from` on
// (launches that turned out to do nothing: a solve's iterations queued past
// its convergence).
size_t profile_marks(cib_ctx *c);
void profile_drop_marks(cib_ctx *c, size_t from);
// Brackets one launch with events when profiling is on (RAII).
// A stage time measured by other events, added to the profile (when on)
// as one launch of that kernel.
void profile_add(cib_ctx *c, int kernel, double seconds);

struct KTimer {
  cib_ctx *ctx;
  int k;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(cib_ctx *c, int kernel, hipStream_t st);
  ~KTimer();
};

// Kernels queued on a stream may still use buffers that a throw releases on
// its way out: while an UnwindFence is alive on this thread, the first device
// buffer released during exception unwinding waits for its stream, so no
// block goes back to the allocator (or its cache, shared with the other
// threads of the context) while a kernel can still touch it.  Declare the
// fence before the buffers it protects (it is destroyed after them).
class UnwindFence {
 public:
  explicit UnwindFence(hipStream_t s);
  ~UnwindFence();
  UnwindFence(const UnwindFence &) = delete;
  UnwindFence &operator=(const UnwindFence &) = delete;
  static void wait_if_unwinding();

 private:
  hipStream_t s_;
  UnwindFence *prev_;
  int depth_;
  bool waited_ = false;
};

// Typed device buffer owned through the context allocator.
template <typename T>
struct DBuf {
  cib_ctx *ctx = nullptr;
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(cib_ctx *c, size_t count) { reset(c, count); }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : ctx(o.ctx), p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) { release(); ctx = o.ctx; p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void reset(cib_ctx *c, size_t count) {
    release();
    ctx = c;
    n = count;
    p = count ? static_cast<T *>(c->alloc(count * sizeof(T))) : nullptr;
  }
  void release() {
    if (p && ctx) {
      UnwindFence::wait_if_unwinding();
      ctx->free(p);
    }
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  void upload(const T *h, size_t count, hipStream_t s) {
    if (count) CIB_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// ------------------------------------------------------------------ planner
struct Orbs {
  int nmax = -1, n_orb = 0, words = 0;
  std::vector<int> n, twoj, twom;
};
Orbs make_orbs(int nmax);
int q_min(int N, const Orbs &o);

struct SubList {
  std::vector<uint64_t> bits;  // size * kMaxWords, state-major, zero padded
  std::vector<int32_t> m2, q;
  size_t size() const { return m2.size(); }
};

struct Plan {
  cib_basis_spec spec{};
  int ns = 1;
  Orbs oA, oB;
  int W = 1;           // kernel word count: max over species
  int WA = 1, WB = 0;  // real word counts
  int qmax = -1;       // -1: no truncation
  int qminB = 0;       // lowest Q of a B configuration
  int nlev = 1;        // Q levels of B configurations a truncation can cut at (cut + 1; 1 without one)
  SubList A, B;        // A: non-empty blocks, ascending integer; B: (2M, Q, integer)
  std::vector<int64_t> a_off;                     // nA + 1
  std::vector<int32_t> a_len, a_seg;              // nA
  std::vector<int32_t> b_seg;                     // nB: segment of each B configuration
  std::vector<int32_t> bseg_start, bseg_m2;       // nseg + 1, nseg
  int64_t D = 0;
  int nA() const { return (int)A.size(); }
  int nB() const { return (int)B.size(); }
  int nseg() const { return (int)bseg_m2.size(); }
};
void validate_spec(const cib_basis_spec &s);
void make_plan(const cib_basis_spec &s, Plan &p);

// Per-interaction device tables.
struct DevInter {
  int nA = 0, nB = 0;
  const double *epsA = nullptr, *epsB = nullptr;
  // per ordered orbital pair p = a * n2 + b of each table: pidx[p] = 2M-block
  // << 16 | index in the block (-1: not a stored pair), prow[p] = offset of
  // the pair's row of its block in v
  const int32_t *pidxA = nullptr, *pidxB = nullptr, *pidxAB = nullptr;
  const int64_t *prowA = nullptr, *prowB = nullptr, *prowAB = nullptr;
  const double *vA = nullptr, *vB = nullptr, *vAB = nullptr;
  const double *dab = nullptr;  // nA * nB: V^AB_{(x,y),(x,y)}
  // V^AB by orbital transitions: rows are the A transitions (a <- c), columns
  // the B transitions (b <- d), one dense block per 2m_a - 2m_c = -(2m_b - 2m_d),
  // so that V^AB_{(a,b),(c,d)} = vt[arb[a * nA + c] + bcol[b * nB + d]]: the
  // tile supplies the row base, the B adjacency entry the column, and the
  // value costs one memory access.
  const double *vt = nullptr;
  const int32_t *arb = nullptr, *bcol = nullptr;
};

}  // namespace cib

struct cib_basis {
  cib_ctx *ctx = nullptr;
  cib::Plan plan;
  // device copies
  cib::DBuf<uint64_t> a_bits, b_bits;   // SoA: word w of configuration k at [w * n + k]
  cib::DBuf<int32_t> a_m2, a_q, a_len, a_seg, b_m2, b_q, b_seg, bseg_start;
  cib::DBuf<int64_t> a_off;
  cib::DBuf<int32_t> row_a, row_p, row_b;   // per state: A-block, position in it, B configuration
  cib::DBuf<uint64_t> words;            // SoA: (WA + WB) words x D
};

// Block-diagonal preconditioner: blocks of states (runs of at most
// max_block states of one many-body basis orbital), their eigenvectors and
// eigenvalues.
struct cib_precond {
  cib_ctx *ctx = nullptr;
  int64_t D = 0, n_blocks = 0, n_groups = 0;
  int largest = 0, max_block = 0, max_sweeps = 0;
  cib::DBuf<int32_t> perm;          // D: states in block order
  cib::DBuf<int64_t> boff, qoff;    // n_blocks + 1: block starts in perm, in Q
  cib::DBuf<double> Q, lam;         // eigenvectors (s x s each), eigenvalues (D)
  mutable cib::DBuf<double> theta;  // shifts staged by each apply call (one call per ctx at a time)
  std::vector<int32_t> perm_h;
  std::vector<int64_t> boff_h;
};

struct cib_interaction {
  cib_ctx *ctx = nullptr;
  int nA = 0, nB = 0;
  cib::DBuf<double> epsA, epsB, vA, vB, vAB, dab, vt;
  cib::DBuf<int32_t> pidxA, pidxB, pidxAB, arb, bcol;
  cib::DBuf<int64_t> prowA, prowB, prowAB;
  cib::DevInter view() const;
};

struct cib_matrix {
  cib_ctx *ctx = nullptr;
  int64_t D = 0, nnz = 0;
  cib_dtype dtype = CIB_F64;
  cib::DBuf<int64_t> row_ptr;
  cib::DBuf<int32_t> col;
  cib::DBuf<double> val64;
  cib::DBuf<float> val32;
  // strictly lower triangle (transposed copy) read by the SpMM
  int64_t nnz_lower = 0;
  cib::DBuf<int64_t> lo_ptr;
  cib::DBuf<int32_t> lo_col;
  cib::DBuf<double> lo_val64;
  cib::DBuf<float> lo_val32;
  cib_build_stats stats{};
  // row ranges of equal stored entries (both triangles), one per XCD
  int64_t xcd_rows[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const void *lo_val() const { return dtype == CIB_F64 ? (const void *)lo_val64.p : (const void *)lo_val32.p; }
  const void *val() const { return dtype == CIB_F64 ? (const void *)val64.p : (const void *)val32.p; }
};

namespace cib {

// ------------------------------------------------------------------ kernels
// (launchers defined in the .hip files; all asynchronous on `s`)
void launch_expand_basis(const cib_basis &b, hipStream_t s);
void launch_substate_energy(const cib_basis &b, const DevInter &it, double *eA, double *eB,
                            hipStream_t s);
void launch_dab(const DevInter &it, double *dab, hipStream_t s);
// Transition blocks of vt: block g holds rows [a0, a0 + na) of the A
// transition list and columns [b0, b0 + nb) of the B transition list (each
// entry a << 16 | c), stored row-major from vt offset base.
struct VtBlock {
  int64_t base;
  int32_t a0, na, b0, nb;
};
void launch_build_vt(const DevInter &it, const VtBlock *blocks, int nblk, const int32_t *atr,
                     const int32_t *btr, int64_t total, double *vt, hipStream_t s);

// Exclusive scans of int32 counts into int64 offsets (n + 1 values each, the
// last one the total), up to kScanArrays independent arrays per call;
// scratch >= scan_scratch(sizes) int64 values.
constexpr int kScanArrays = 4;
struct ScanJob {
  const int32_t *in;
  int64_t n;
  int64_t *out;
};
size_t scan_scratch(const std::vector<int64_t> &ns);
void launch_scans(const std::vector<ScanJob> &jobs, int64_t *scratch, hipStream_t s);

// Build H on stream s.  reserve(stage, bytes), when given, runs on the host
// before each group of device allocations with the exact bytes the group
// takes (stage 0: the counting passes' arrays; 1: the screens' lists, row
// counts, diagonal and offsets, once their sizes are known; 2: the stored
// entries of both triangles); it may block or throw (the build then stops,
// and its buffers are released once the stream has drained).
using BuildReserve = std::function<void(int stage, size_t bytes)>;
void build_matrix(cib_ctx *ctx, const cib_basis &b, const cib_interaction &it, cib_dtype dt,
                  cib_matrix &H, hipStream_t s, const BuildReserve &reserve);
cib_basis *make_basis(cib_ctx *ctx, const cib_basis_spec &spec, hipStream_t s);
cib_basis *make_basis(cib_ctx *ctx, Plan &&plan, hipStream_t s);
// Device bytes the context allocator takes for n bytes, and the peak device
// bytes of make_basis and upload_interaction for a plan.
size_t dev_bytes(size_t n);
size_t basis_device_bytes(const Plan &p);
size_t interaction_device_bytes(const Plan &p);
cib_interaction *upload_interaction(cib_ctx *ctx, const cib_basis &b, const cib_tables &t,
                                    hipStream_t s);

// stop: optional device flag; the launched kernels return at once when it
// is nonzero (a solve's iterations queued past its convergence).
void spmm_sym(const cib_matrix &H, const void *X, int64_t ldx, void *Y, int64_t ldy, int nvec,
              hipStream_t s, const int32_t *stop = nullptr);
// float32 H and X, Y written as float64 (the eigensolver's widened H W):
// false, with nothing launched, when the vector kernel does not apply.
bool spmm_sym_widen(const cib_matrix &H, const float *X, int64_t ldx, double *Y, int64_t ldy, int nvec,
                    hipStream_t s, const int32_t *stop);
// Matrix-free Y = H X (nvec 8 or 16, 16-byte aligned rows of the dtype):
// the build's screens and values, then one row pass that multiplies every
// entry into X instead of storing it.  Returns when Y is written.
struct ApplyReq {
  const void *X;
  int64_t ldx;
  void *Y;
  int64_t ldy;
  int nvec;
};
void apply_matrix_free(cib_ctx *ctx, const cib_basis &b, const cib_interaction &it, cib_dtype dt,
                       const ApplyReq &a, hipStream_t s);
// State-counting test: per-state counts of states within two particle
// differences (device counts, optional) and their total (host).
void count_pairs(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int N, int method, int32_t *counts, int64_t *total,
                 hipStream_t s);
// The same test with no device allocation: scratch in a static device array
// (up to static_count_max_states() states), whose address on a device is set
// up once by static_scratch_init with that device current (the context's
// creation does it).
void static_scratch_init(int device);
int64_t static_count_max_states();
void count_pairs_static(int device, const uint16_t *mbs, int64_t n, int N, int method, int32_t *counts,
                        int64_t *total, hipStream_t s);
// Block-diagonal preconditioner: set-up (groups, blocks, eigenpairs) and
// W = M(theta)^-1 R for ncol <= 16 columns (theta on the device).
void precond_create(cib_ctx *ctx, const cib_basis &b, const cib_matrix &H, int max_block, cib_precond &P,
                    hipStream_t s);
void precond_apply(const cib_precond &P, const double *theta_dev, int ncol, const double *R, int64_t ldr, double *W,
                   int64_t ldw, float *w32, int64_t ld32, hipStream_t s);
// out[k * nvec + v] = x_v^T O_k x_v for the m operators ops (host result).
void observables(cib_ctx *ctx, const cib_basis &b, const cib_tables *ops, int m, cib_dtype dt, const void *X,
                 int64_t ldx, int nvec, double *out, hipStream_t s);

// Step-wise LOBPCG (used by the serving loop): all calls enqueue on the run's
// stream; the status block (kStatusLen doubles: converged count, b relative
// residuals, b Ritz values, and the number of the iteration that wrote them)
// is copied to host memory by lobpcg_copy_status.
constexpr int kStatusIter = 1 + 2 * kMaxBlock;
constexpr int kStatusLen = 2 + 2 * kMaxBlock;
struct LobpcgRun;
// Arguments of the SpMM row kernel for nvec 8 / 16 with 16-byte aligned rows.
struct VecArgs {
  int64_t D;
  const int64_t *rp;
  const int32_t *col;
  const void *val;
  const int64_t *lrp;
  const int32_t *lcol;
  const void *lval;
  const void *X;
  int64_t ldx;
  void *Y;
  int64_t ldy;
  int64_t xr[9];     // XCD x takes rows [xr[x], xr[x + 1]) (single launches only)
  const int32_t *stop = nullptr;   // a solve's stop flag: the launch does nothing once it is set
  double *Y64 = nullptr;           // float32 matrix only: rows of Y written widened to float64 here
  int64_t ldy64 = 0;
};
// false when the vector kernel does not apply (nvec, alignment); blocks =
// workgroups of the matrix in a grouped launch
bool spmm_vec_args(const cib_matrix &H, const void *X, int64_t ldx, void *Y, int64_t ldy, int nvec, VecArgs &a,
                   int &blocks);
void launch_spmm_group(cib_dtype dt, int nvec, const VecArgs *dev_args, const int32_t *dev_off, int njobs,
                       int total_blocks, hipStream_t s);

// Arguments of one Rayleigh-Ritz step (device pointers of one solve).
struct RRArgs {
  int ns, b;
  const double *gram;   // S^T S then S^T H S, each kNS x (kNS + 1) row-major (rows and columns < ns used)
  double *C;        // ns x 2b: [Cx | Cp]
  double *lam;      // b
  int32_t *flag;    // [0]: rank of the search space, [1]: fallback taken
  double drop_tol;
  const double *hlow;  // lower bound of the spectrum of H (Gershgorin)
  const int32_t *stop = nullptr;   // a solve's stop flag: nothing is done once it is set
};

// Per-stage arguments of one LOBPCG iteration (device pointers of one solve).
struct UpdArgs {
  int64_t D;
  int b, ns, ld;
  double *S, *HS;
  const double *C, *lam, *diag;
  float *w32;             // optional float32 copy of W (dense D x b)
  double *npart;          // per block: b residual sums, b |x|^2 sums
  int rows_per_blk;
  const int32_t *locked;  // per column: converged at the previous check (W = 0)
  const int32_t *stop = nullptr;   // a solve's stop flag: nothing is done once it is set
};
struct WidenArgs {
  int64_t D;
  int b;
  const float *in;
  double *out;
  int ldo;
};
struct GramArgs {
  int64_t D;
  int ns, ld;
  const double *S, *HS;
  int64_t rows_per_blk;
  double *partial;
};
struct SumArgs {   // out[g][e] = sum of in[q][e] over parts q of group g (groups of per)
  int nout, nparts, per;
  const double *in;
  double *out;
  int pad;          // > 0: one [S^T S | S^T H S] pair of row length 2 pad, written padded (Rayleigh-Ritz layout)
};
struct FinishArgs {
  int b, nev, nparts;
  const double *npart, *lam;
  double tol;
  double *status;
  int32_t *locked;
};

// One LOBPCG iteration of one solve, stage by stage, with each stage's
// workgroup count (the serving loop's grouped launches).
struct IterPlan {
  cib_dtype dt;
  int nvec;
  VecArgs spmm;
  int spmm_blocks;
  bool widen;
  WidenArgs wid;
  int widen_blocks;
  int T;
  GramArgs gram;
  int gram_blocks;
  SumArgs gs1, gs2;
  int gs1_blocks, gs2_blocks;
  RRArgs rr;
  int TN;
  UpdArgs upd;
  int upd_blocks;
  SumArgs us;
  int us_blocks;
  FinishArgs fin;
  const double *status;   // device status block the iteration ends with
};

// Runs one planned iteration of several solves: every stage is one launch
// over all of them (per kernel variant), arguments staged through pinned
// memory with one copy.
struct GroupRunner {
  cib_ctx *ctx = nullptr;
  char *host = nullptr;
  cib::DBuf<char> dev;
  size_t cap = 0;
  explicit GroupRunner(cib_ctx *c) : ctx(c) {}
  ~GroupRunner();
  void run(const std::vector<LobpcgRun *> &runs, const std::vector<IterPlan> &plans, hipStream_t s);
};

LobpcgRun *lobpcg_create(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, hipStream_t s);
// advances the solve by one iteration's plan; false: not eligible (nothing advanced)
bool lobpcg_plan_iteration(LobpcgRun *r, IterPlan &p);

void lobpcg_start(LobpcgRun *r);
void lobpcg_iterate(LobpcgRun *r);
void lobpcg_copy_status(LobpcgRun *r, double *host);
int lobpcg_iters(const LobpcgRun *r);
void lobpcg_destroy(LobpcgRun *r);
size_t lobpcg_bytes(int64_t D, int b, cib_dtype dt);

cib_status serve_run(cib_ctx *ctx, const cib_request *reqs, int n, const cib_serve_opts &o,
                     cib_result *results);

// Lowest k eigenpairs of the symmetric tridiagonal matrix (diagonal a[n],
// off-diagonal b[n-1]) on the host: values th[k] ascending, vectors S (n x k,
// S[j * k + c]) orthonormal.
void tri_lowest(const std::vector<double> &a, const std::vector<double> &b, int n, int k, std::vector<double> &th,
                std::vector<double> &S);
cib_status lanczos_solve(cib_ctx *ctx, const cib_matrix &H, int nev, int max_iter, double tol, uint64_t seed,
                         double *evals, double *evecs, int64_t ld_evecs, cib_lanczos_info *info, hipStream_t s);
cib_status lobpcg_solve(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, double *evals,
                        double *evecs, int64_t ld_evecs, cib_lobpcg_info *info);

}  // namespace cib
