// extern "C" entry points: argument checks, error translation, handle life.
#include <algorithm>
#include <chrono>
#include <memory>

#include "cib_internal.hpp"

namespace cib {
const char *last_error_cstr();
void profile_collect(cib_ctx *c);
}  // namespace cib

using namespace cib;

namespace {

template <typename F>
cib_status guarded(F &&f) {
  try {
    f();
    set_last_error("");
    return CIB_OK;
  } catch (const cib::Error &e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return CIB_E_NOMEM;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return CIB_E_DEVICE;
  } catch (...) {
    set_last_error("unknown error");
    return CIB_E_DEVICE;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    CIB_HIP(hipGetDevice(&prev));
    if (prev != dev) CIB_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

struct BusyGuard {
  cib_ctx *c;
  explicit BusyGuard(cib_ctx *ctx) : c(ctx) {
    CIB_REQUIRE(!c->busy, CIB_E_BUSY, "context is already inside a call");
    c->busy = true;
  }
  ~BusyGuard() { c->busy = false; }
};

}  // namespace

extern "C" {

const char *cib_last_error(void) { return last_error_cstr(); }

cib_status cib_create(int device, const cib_allocator *a, void *hip_stream, cib_ctx **out) {
  return guarded([&] {
    CIB_REQUIRE(out, CIB_E_INVALID, "out is NULL");
    int n = 0;
    CIB_HIP(hipGetDeviceCount(&n));
    CIB_REQUIRE(device >= 0 && device < n, CIB_E_INVALID, "no such device");
    if (a) CIB_REQUIRE(a->alloc && a->free, CIB_E_INVALID, "allocator needs alloc and free");
    std::unique_ptr<cib_ctx> c(new cib_ctx);
    c->device = device;
    DeviceGuard g(device);
    static_scratch_init(device);
    if (a) { c->user = *a; c->has_user = true; }
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      CIB_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    *out = c.release();
  });
}

cib_status cib_profile_enable(cib_ctx *ctx, int on) {
  return guarded([&] {
    CIB_REQUIRE(ctx, CIB_E_INVALID, "ctx is NULL");
    ctx->profiling = on != 0;
  });
}

cib_status cib_profile_reset(cib_ctx *ctx) {
  return guarded([&] {
    CIB_REQUIRE(ctx, CIB_E_INVALID, "ctx is NULL");
    DeviceGuard g(ctx->device);
    profile_collect(ctx);
    ctx->kernel_totals.clear();
  });
}

cib_status cib_profile_query(cib_ctx *ctx, const char *kernel, int64_t *launches, double *total_s) {
  return guarded([&] {
    CIB_REQUIRE(ctx && kernel, CIB_E_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    profile_collect(ctx);
    int64_t n = 0;
    double t = 0.0;
    for (int k = 0; k < K_NKERN; ++k)
      if (std::strcmp(kernel, kKernelNames[k]) == 0) {
        auto it = ctx->kernel_totals.find(k);
        if (it != ctx->kernel_totals.end()) { n = it->second.first; t = it->second.second; }
      }
    if (launches) *launches = n;
    if (total_s) *total_s = t;
  });
}

}  // extern "C"

namespace {

void ctx_teardown(cib_ctx *ctx) {
  try {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    profile_collect(ctx);
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    ctx->release_cache();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  } catch (...) {
  }
  delete ctx;
}

void handle_made(cib_ctx *ctx) {
  std::lock_guard<std::mutex> l(ctx->life_mu);
  ++ctx->handles;
}

// After a handle's own release: the context goes too if it was destroyed
// while this was its last handle.
void handle_freed(cib_ctx *ctx) {
  bool last;
  {
    std::lock_guard<std::mutex> l(ctx->life_mu);
    last = --ctx->handles == 0 && ctx->destroyed;
  }
  if (last) ctx_teardown(ctx);
}

}  // namespace

extern "C" {

void cib_destroy(cib_ctx *ctx) {
  if (!ctx) return;
  bool now;
  {
    std::lock_guard<std::mutex> l(ctx->life_mu);
    ctx->destroyed = true;
    now = ctx->handles == 0;
  }
  if (now) ctx_teardown(ctx);
}

cib_status cib_ctx_bytes(const cib_ctx *ctx, int64_t *live, int64_t *peak) {
  return guarded([&] {
    CIB_REQUIRE(ctx, CIB_E_INVALID, "ctx is NULL");
    if (live) *live = ctx->live;
    if (peak) *peak = ctx->peak;
  });
}

// ------------------------------------------------------------------ basis
cib_status cib_build_basis(cib_ctx *ctx, const cib_basis_spec *spec, cib_basis **out, int64_t *dim) {
  return guarded([&] {
    CIB_REQUIRE(ctx && spec && out, CIB_E_INVALID, "NULL argument");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    std::unique_ptr<cib_basis> b(make_basis(ctx, *spec, ctx->stream));
    const Plan &p = b->plan;
    if (dim) *dim = p.D;
    handle_made(ctx);
    *out = b.release();
  });
}

cib_status cib_basis_info(const cib_basis *b, int64_t *dim, int32_t words[2], int32_t n_orb[2],
                          int64_t *n_ablocks) {
  return guarded([&] {
    CIB_REQUIRE(b, CIB_E_INVALID, "basis is NULL");
    if (dim) *dim = b->plan.D;
    if (words) { words[0] = b->plan.WA; words[1] = b->plan.WB; }
    if (n_orb) { n_orb[0] = b->plan.oA.n_orb; n_orb[1] = b->plan.ns == 2 ? b->plan.oB.n_orb : 0; }
    if (n_ablocks) *n_ablocks = b->plan.nA();
  });
}

cib_status cib_basis_export(const cib_basis *b, uint64_t *host_words) {
  return guarded([&] {
    CIB_REQUIRE(b && host_words, CIB_E_INVALID, "NULL argument");
    DeviceGuard g(b->ctx->device);
    const Plan &p = b->plan;
    const int nw = p.WA + p.WB;
    std::vector<uint64_t> soa((size_t)nw * p.D);
    CIB_HIP(hipMemcpyAsync(soa.data(), b->words.p, soa.size() * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, b->ctx->stream));
    CIB_HIP(hipStreamSynchronize(b->ctx->stream));
    for (int64_t i = 0; i < p.D; ++i)
      for (int w = 0; w < nw; ++w) host_words[i * nw + w] = soa[(size_t)w * p.D + i];
  });
}

void cib_basis_free(cib_basis *b) {
  if (!b) return;
  cib_ctx *ctx = b->ctx;
  try {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  } catch (...) {
  }
  delete b;
  handle_freed(ctx);
}

// ------------------------------------------------------------ interaction
cib_status cib_upload_interaction(cib_ctx *ctx, const cib_basis *b, const cib_tables *t,
                                  cib_interaction **out) {
  return guarded([&] {
    CIB_REQUIRE(ctx && b && t && out, CIB_E_INVALID, "NULL argument");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    *out = upload_interaction(ctx, *b, *t, ctx->stream);
    handle_made(ctx);
  });
}

void cib_interaction_free(cib_interaction *it) {
  if (!it) return;
  cib_ctx *ctx = it->ctx;
  try {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  } catch (...) {
  }
  delete it;
  handle_freed(ctx);
}

// ---------------------------------------------------------------- build H
cib_status cib_build_H_resident(cib_ctx *ctx, const cib_basis *b, const cib_interaction *it,
                                cib_dtype dt, cib_matrix **out, int64_t *nnz) {
  return guarded([&] {
    CIB_REQUIRE(ctx && b && it && out, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(dt == CIB_F64 || dt == CIB_F32, CIB_E_INVALID, "dtype must be CIB_F64 or CIB_F32");
    CIB_REQUIRE(it->nA == b->plan.oA.n_orb && it->nB == (b->plan.ns == 2 ? b->plan.oB.n_orb : 0),
                CIB_E_INVALID, "interaction was uploaded for another orbital set");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    std::unique_ptr<cib_matrix> H(new cib_matrix);
    H->ctx = ctx;
    build_matrix(ctx, *b, *it, dt, *H, ctx->stream, nullptr);
    if (nnz) *nnz = H->nnz;
    handle_made(ctx);
    *out = H.release();
  });
}

cib_status cib_build_H(cib_ctx *ctx, const cib_basis *b, const cib_tables *t, cib_dtype dt,
                       cib_matrix **out, int64_t *nnz) {
  cib_interaction *it = nullptr;
  cib_status st = cib_upload_interaction(ctx, b, t, &it);
  if (st != CIB_OK) return st;
  st = cib_build_H_resident(ctx, b, it, dt, out, nnz);
  std::string err = st == CIB_OK ? "" : cib_last_error();
  cib_interaction_free(it);
  if (st != CIB_OK) set_last_error(err);
  return st;
}

cib_status cib_matrix_info(const cib_matrix *H, int64_t *dim, int64_t *nnz, cib_dtype *dt) {
  return guarded([&] {
    CIB_REQUIRE(H, CIB_E_INVALID, "matrix is NULL");
    if (dim) *dim = H->D;
    if (nnz) *nnz = H->nnz;
    if (dt) *dt = H->dtype;
  });
}

cib_status cib_matrix_stats(const cib_matrix *H, cib_build_stats *st) {
  return guarded([&] {
    CIB_REQUIRE(H && st, CIB_E_INVALID, "NULL argument");
    *st = H->stats;
  });
}

cib_status cib_matrix_export(const cib_matrix *H, int64_t *row_ptr, int32_t *col, void *val) {
  return guarded([&] {
    CIB_REQUIRE(H, CIB_E_INVALID, "matrix is NULL");
    DeviceGuard g(H->ctx->device);
    hipStream_t s = H->ctx->stream;
    if (row_ptr)
      CIB_HIP(hipMemcpyAsync(row_ptr, H->row_ptr.p, sizeof(int64_t) * (H->D + 1), hipMemcpyDeviceToHost, s));
    if (col) CIB_HIP(hipMemcpyAsync(col, H->col.p, sizeof(int32_t) * H->nnz, hipMemcpyDeviceToHost, s));
    if (val)
      CIB_HIP(hipMemcpyAsync(val, H->val(), (H->dtype == CIB_F64 ? 8 : 4) * (size_t)H->nnz,
                             hipMemcpyDeviceToHost, s));
    CIB_HIP(hipStreamSynchronize(s));
  });
}

cib_status cib_matrix_device(const cib_matrix *H, const int64_t **row_ptr, const int32_t **col,
                             const void **val) {
  return guarded([&] {
    CIB_REQUIRE(H, CIB_E_INVALID, "matrix is NULL");
    if (row_ptr) *row_ptr = H->row_ptr.p;
    if (col) *col = H->col.p;
    if (val) *val = H->val();
  });
}

void cib_matrix_free(cib_matrix *H) {
  if (!H) return;
  cib_ctx *ctx = H->ctx;
  try {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  } catch (...) {
  }
  delete H;
  handle_freed(ctx);
}

// ---------------------------------------------------------------- apply H
cib_status cib_apply_H(cib_ctx *ctx, const cib_matrix *H, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, int32_t nvec) {
  return guarded([&] {
    CIB_REQUIRE(ctx && H && X && Y, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(nvec >= 1 && nvec <= 64, CIB_E_INVALID, "nvec must be in 1..64");
    CIB_REQUIRE(ldx >= nvec && ldy >= nvec, CIB_E_INVALID, "leading dimension smaller than nvec");
    CIB_REQUIRE(H->ctx == ctx, CIB_E_INVALID, "matrix belongs to another context");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    spmm_sym(*H, X, ldx, Y, ldy, nvec, ctx->stream);
  });
}

// ----------------------------------------------------------- observables
cib_status cib_observables(cib_ctx *ctx, const cib_basis *b, const cib_tables *ops, int32_t m, cib_dtype dt,
                           const void *X, int64_t ldx, int32_t nvec, double *out) {
  return guarded([&] {
    CIB_REQUIRE(ctx && b && ops && X && out, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(m >= 1, CIB_E_INVALID, "m must be at least 1");
    CIB_REQUIRE(dt == CIB_F64 || dt == CIB_F32, CIB_E_INVALID, "dtype must be CIB_F64 or CIB_F32");
    CIB_REQUIRE(nvec >= 1 && nvec <= 64, CIB_E_INVALID, "nvec must be in 1..64");
    CIB_REQUIRE(ldx >= nvec, CIB_E_INVALID, "leading dimension smaller than nvec");
    CIB_REQUIRE(b->ctx == ctx, CIB_E_INVALID, "basis belongs to another context");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    observables(ctx, *b, ops, m, dt, X, ldx, nvec, out, ctx->stream);
  });
}

// -------------------------------------------------------- matrix-free H X
cib_status cib_apply_H_free(cib_ctx *ctx, const cib_basis *b, const cib_interaction *it, cib_dtype dt,
                            const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nvec) {
  return guarded([&] {
    CIB_REQUIRE(ctx && b && it && X && Y, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(dt == CIB_F64 || dt == CIB_F32, CIB_E_INVALID, "dtype must be CIB_F64 or CIB_F32");
    CIB_REQUIRE(nvec == 8 || nvec == 16, CIB_E_INVALID, "nvec must be 8 or 16");
    CIB_REQUIRE(ldx >= nvec && ldy >= nvec, CIB_E_INVALID, "leading dimension smaller than nvec");
    const size_t sv = dt == CIB_F64 ? 8 : 4;
    CIB_REQUIRE((uintptr_t)X % 16 == 0 && (uintptr_t)Y % 16 == 0 && (ldx * sv) % 16 == 0 && (ldy * sv) % 16 == 0,
                CIB_E_INVALID, "X and Y rows must be 16-byte aligned");
    CIB_REQUIRE(it->nA == b->plan.oA.n_orb && it->nB == (b->plan.ns == 2 ? b->plan.oB.n_orb : 0),
                CIB_E_INVALID, "interaction was uploaded for another orbital set");
    CIB_REQUIRE(b->ctx == ctx, CIB_E_INVALID, "basis belongs to another context");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    apply_matrix_free(ctx, *b, *it, dt, ApplyReq{X, ldx, Y, ldy, nvec}, ctx->stream);
  });
}

// -------------------------------------------------------- state counting
cib_status cib_count_states(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int32_t n_particles, int32_t n_sp,
                            int32_t method, int32_t *counts, int64_t *total) {
  return guarded([&] {
    CIB_REQUIRE(ctx && mbs && total, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(n >= 1 && n <= (int64_t(1) << 22), CIB_E_INVALID, "n must be in 1..2^22");
    CIB_REQUIRE(n_particles >= 1 && n_particles <= 20, CIB_E_INVALID, "n_particles must be in 1..20");
    CIB_REQUIRE(n_sp >= n_particles && n_sp <= 65534, CIB_E_INVALID, "n_sp must be in n_particles..65534");
    CIB_REQUIRE(method >= 0 && method <= 2, CIB_E_INVALID, "method must be 0, 1 or 2");
    CIB_REQUIRE(method != 2 || n_sp <= 128, CIB_E_INVALID, "method 2 needs n_sp <= 128");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    count_pairs(ctx, mbs, n, n_particles, method, counts, total, ctx->stream);
  });
}

cib_status cib_count_states_noalloc(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int32_t n_particles,
                                    int32_t n_sp, int32_t method, int32_t *counts, int64_t *total) {
  return guarded([&] {
    CIB_REQUIRE(ctx && mbs && total, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(n >= 1 && n <= static_count_max_states(), CIB_E_INVALID,
                "n must be in 1.." + std::to_string(static_count_max_states()) + " (the static scratch)");
    CIB_REQUIRE(n_particles >= 1 && n_particles <= 20, CIB_E_INVALID, "n_particles must be in 1..20");
    CIB_REQUIRE(n_sp >= n_particles && n_sp <= 65534, CIB_E_INVALID, "n_sp must be in n_particles..65534");
    CIB_REQUIRE(method >= 0 && method <= 2, CIB_E_INVALID, "method must be 0, 1 or 2");
    CIB_REQUIRE(method != 2 || n_sp <= 128, CIB_E_INVALID, "method 2 needs n_sp <= 128");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    count_pairs_static(ctx->device, mbs, n, n_particles, method, counts, total, ctx->stream);
  });
}

}  // extern "C"

// ---------------------------------------------------------------- LOBPCG
extern "C" cib_status cib_lobpcg(cib_ctx *ctx, const cib_matrix *H, const cib_lobpcg_opts *o,
                                 double *evals, double *evecs, int64_t ld_evecs,
                                 cib_lobpcg_info *info) {
  cib_status st = CIB_OK;
  cib_status rc = guarded([&] {
    CIB_REQUIRE(ctx && H && o && evals, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(H->ctx == ctx, CIB_E_INVALID, "matrix belongs to another context");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    st = lobpcg_solve(ctx, *H, *o, evals, evecs, ld_evecs, info);
  });
  if (rc != CIB_OK) return rc;
  if (st == CIB_E_NOT_CONVERGED) set_last_error("LOBPCG reached max_iter before the tolerance");
  return st;
}

// ---------------------------------------------------------------- preconditioner
cib_status cib_precond_create(cib_ctx *ctx, const cib_basis *b, const cib_matrix *H, int32_t max_block,
                              cib_precond **out) {
  return guarded([&] {
    CIB_REQUIRE(ctx && b && H && out, CIB_E_INVALID, "NULL argument");
    *out = nullptr;
    CIB_REQUIRE(max_block >= 1 && max_block <= 64, CIB_E_INVALID, "max_block must be in 1..64");
    CIB_REQUIRE(b->ctx == ctx && H->ctx == ctx, CIB_E_INVALID, "basis or matrix belongs to another context");
    CIB_REQUIRE(H->D == b->plan.D, CIB_E_INVALID, "matrix was not built on this basis");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    std::unique_ptr<cib_precond> P(new cib_precond);
    precond_create(ctx, *b, *H, max_block, *P, ctx->stream);
    handle_made(ctx);
    *out = P.release();
  });
}

cib_status cib_precond_info(const cib_precond *P, int64_t *n_blocks, int64_t *n_groups, int32_t *largest,
                            int32_t *max_sweeps) {
  return guarded([&] {
    CIB_REQUIRE(P, CIB_E_INVALID, "NULL argument");
    if (n_blocks) *n_blocks = P->n_blocks;
    if (n_groups) *n_groups = P->n_groups;
    if (largest) *largest = P->largest;
    if (max_sweeps) *max_sweeps = P->max_sweeps;
  });
}

cib_status cib_precond_export(const cib_precond *P, int32_t *perm, int64_t *block_off) {
  return guarded([&] {
    CIB_REQUIRE(P, CIB_E_INVALID, "NULL argument");
    if (perm) std::copy(P->perm_h.begin(), P->perm_h.end(), perm);
    if (block_off) std::copy(P->boff_h.begin(), P->boff_h.end(), block_off);
  });
}

cib_status cib_precond_apply(cib_ctx *ctx, const cib_precond *P, const double *theta, const double *R, int64_t ldr,
                             double *W, int64_t ldw, int32_t ncol) {
  return guarded([&] {
    CIB_REQUIRE(ctx && P && theta && R && W, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(ncol >= 1 && ncol <= 16, CIB_E_INVALID, "ncol must be in 1..16");
    CIB_REQUIRE(ldr >= ncol && ldw >= ncol, CIB_E_INVALID, "leading dimension smaller than ncol");
    CIB_REQUIRE(P->ctx == ctx, CIB_E_INVALID, "preconditioner belongs to another context");
    CIB_REQUIRE(R != W || ldr == ldw, CIB_E_INVALID, "in-place apply needs ldr == ldw");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    P->theta.upload(theta, (size_t)ncol, ctx->stream);
    precond_apply(*P, P->theta.p, ncol, R, ldr, W, ldw, nullptr, 0, ctx->stream);
    CIB_HIP(hipStreamSynchronize(ctx->stream));
  });
}

void cib_precond_free(cib_precond *P) {
  if (!P) return;
  cib_ctx *ctx = P->ctx;
  try {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  } catch (...) {
  }
  delete P;
  handle_freed(ctx);
}

// ---------------------------------------------------------------- Lanczos
extern "C" cib_status cib_lanczos(cib_ctx *ctx, const cib_matrix *H, const cib_lanczos_opts *o, double *evals,
                                  double *evecs, int64_t ld_evecs, cib_lanczos_info *info) {
  cib_status st = CIB_OK;
  cib_status rc = guarded([&] {
    CIB_REQUIRE(ctx && H && o && evals, CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(H->ctx == ctx, CIB_E_INVALID, "matrix belongs to another context");
    CIB_REQUIRE(o->nev >= 1 && o->nev <= 64 && o->nev <= H->D, CIB_E_INVALID, "nev must be in 1..min(64, D)");
    CIB_REQUIRE(o->max_iter >= o->nev && o->max_iter <= 4096, CIB_E_INVALID, "max_iter must be in nev..4096");
    CIB_REQUIRE(!evecs || ld_evecs >= o->nev, CIB_E_INVALID, "ld_evecs smaller than nev");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    st = lanczos_solve(ctx, *H, o->nev, o->max_iter, o->tol, o->seed, evals, evecs, ld_evecs, info, ctx->stream);
  });
  if (rc != CIB_OK) return rc;
  if (st == CIB_E_NOT_CONVERGED) set_last_error("Lanczos reached max_iter before the tolerance");
  return st;
}

extern "C" cib_status cib_tridiag_lowest(const double *a, const double *b, int32_t n, int32_t k, double *theta,
                                        double *S) {
  return guarded([&] {
    CIB_REQUIRE(a && theta && S && (n < 2 || b), CIB_E_INVALID, "NULL argument");
    CIB_REQUIRE(n >= 1 && k >= 1 && k <= n, CIB_E_INVALID, "need 1 <= k <= n");
    std::vector<double> av(a, a + n), bv(b, b + (n - 1)), th, Sv;
    tri_lowest(av, bv, n, k, th, Sv);
    std::copy(th.begin(), th.end(), theta);
    std::copy(Sv.begin(), Sv.end(), S);
  });
}

// ---------------------------------------------------------------- serve
extern "C" cib_status cib_serve(cib_ctx *ctx, const cib_request *reqs, int32_t n,
                                const cib_serve_opts *opts, cib_result *results) {
  return guarded([&] {
    CIB_REQUIRE(ctx && opts && n >= 0, CIB_E_INVALID, "bad argument");
    CIB_REQUIRE(n == 0 || (reqs && results), CIB_E_INVALID, "NULL requests or results");
    BusyGuard busy(ctx);
    DeviceGuard g(ctx->device);
    serve_run(ctx, reqs, n, *opts, results);
  });
}
