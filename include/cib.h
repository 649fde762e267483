/* cib.h -- configuration-interaction Hamiltonian engine for AMD MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of a configuration-interaction (CI)
 * calculation as described in "Accelerating quantum many-body configuration
 * interaction with directives" (Cook, Fasano, Maris, Yang, Oryspayev):
 *
 *   cib_build_basis  Slater-determinant bit-string basis (Sec. 2; Fig. 1 step 1)
 *   cib_build_H      pair screen by popcount(xor) <= 4, fermionic phase and
 *                    two-body matrix-element lookup, counts -> offsets -> fill
 *                    of a half-stored symmetric CSR (Sec. 2.1-2.3; Fig. 1
 *                    steps 2-14)
 *   cib_apply_H      symmetric SpMM Y = H X (Sec. 2: sparse matrix-matrix
 *                    products of the eigensolver; Fig. 2 'FMA' variant)
 *   cib_lobpcg       lowest eigenpairs by block LOBPCG (Fig. 1 step 15)
 *   cib_serve        continuous-batching loop over many eigensolve requests
 *
 * Conventions shared by every call
 * --------------------------------
 * Status: every call returns CIB_OK (0) or a negative cib_status.  Out
 *   parameters are written only on CIB_OK (cib_lobpcg also fills eigenvalues
 *   and residuals on CIB_E_NOT_CONVERGED).  cib_last_error() returns a
 *   message for the calling thread's most recent failure; the string stays
 *   valid until the thread's next cib_* call.  No C++ exception crosses the
 *   ABI.  Arguments are validated before any device work is launched.
 * Ownership: handles (cib_ctx, cib_basis, cib_matrix, cib_interaction) are
 *   owned by the library and released with the matching cib_*_free /
 *   cib_destroy.  Host arrays passed in are owned by the caller and are
 *   copied before the call returns.  Device pointers passed to cib_apply_H /
 *   cib_lobpcg are owned by the caller and must stay valid until the context
 *   stream has passed the call.
 * Streams: a context issues all of its device work on one HIP stream (the
 *   caller's, or one it creates).  Calls on one context are not thread-safe;
 *   use one context per host thread.
 * Integers: offsets and counts that can exceed 2^31 are int64 (row
 *   pointers, nonzero counts, dimensions).
 */
#ifndef CIB_H
#define CIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cib_status;
#define CIB_OK 0
#define CIB_E_INVALID (-1)       /* bad argument or spec                     */
#define CIB_E_NOMEM (-2)         /* allocator returned NULL / over budget    */
#define CIB_E_DEVICE (-3)        /* HIP runtime error                        */
#define CIB_E_NOT_CONVERGED (-4) /* max_iter reached before the tolerance    */
#define CIB_E_OVERFLOW (-5)      /* a count exceeds the index type           */
#define CIB_E_EMPTY_BASIS (-6)   /* the spec admits no state (D = 0)         */
#define CIB_E_BUSY (-7)          /* context already inside a call            */
#define CIB_E_CANCELLED (-8)     /* deadline reached                         */

typedef enum { CIB_F64 = 0, CIB_F32 = 1 } cib_dtype;

typedef struct cib_ctx cib_ctx;
typedef struct cib_basis cib_basis;
typedef struct cib_interaction cib_interaction;
typedef struct cib_matrix cib_matrix;
typedef struct cib_precond cib_precond;

/* Device-memory hooks.  alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL; free releases it.  NULL hooks: hipMalloc and
 * hipFree behind a per-context cache of freed blocks. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} cib_allocator;

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to issue
 * work on (NULL: the context creates its own default-priority stream). */
cib_status cib_create(int device, const cib_allocator *alloc, void *hip_stream, cib_ctx **out);
/* Release a context.  Handles made on it (basis, interaction, matrix,
 * preconditioner) may be freed before or after: while some are live the
 * context is only marked, and the free of the last one releases it, so the
 * stream and allocator given to cib_create must stay valid until then.  No
 * other call may use a destroyed context. */
void cib_destroy(cib_ctx *ctx);
const char *cib_last_error(void);
/* Device bytes currently held by the context's allocations (live, not cached). */
cib_status cib_ctx_bytes(const cib_ctx *ctx, int64_t *live_bytes, int64_t *peak_bytes);

/* Per-kernel device timing: when enabled, the library brackets every launch
 * of its hot kernels with HIP events on the launching stream.  Query sums the
 * elapsed times of all completed launches of one kernel since the last reset
 * (it synchronises those events).  Kernel names: "spmm_sym", "gram",
 * "rayleigh_ritz", "update", "state_count", "apply_free" (the matrix-free
 * product's row pass), and the stages of a build, one launch each per
 * cib_build_H, timed by the build's own stage events (the device time
 * between them): "screens" (the tile and adjacency screens with their
 * substate energies and scans), "row_count", "scan" (the row offsets),
 * "row_fill" (the row pass that fills both stored triangles).  Unknown
 * names report zero launches. */
cib_status cib_profile_enable(cib_ctx *ctx, int on);
cib_status cib_profile_reset(cib_ctx *ctx);
cib_status cib_profile_query(cib_ctx *ctx, const char *kernel, int64_t *launches, double *total_s);

/* ---------------------------------------------------------------- basis --
 * Sec. 2: many-body states are antisymmetrised products of single-particle
 * states.  Single-particle orbitals of one species are harmonic-oscillator
 * shells n = 0..nmax; shell n has levels 2j = 1..2n+1 (odd) and each level the
 * projections 2m = -2j..2j step 2, in ascending (n, 2j, 2m) order (orbital
 * index = position).  A state is an N_A-subset of species-A orbitals times an
 * N_B-subset of species-B orbitals with sum(2m) = two_M and, if cut >= 0,
 * sum over all particles of n <= Qmin(N_A) + Qmin(N_B) + cut (Qmin fills the
 * shells from n = 0).  n_species = 1: species B is absent (nmax[1] and
 * n_particles[1] are ignored).
 *
 * Bit string BIN(Phi) (Sec. 2.1): bit k of species s is orbital k of s.  Each
 * species occupies ceil(n_orb/64) little-endian 64-bit words (at most 3:
 * nmax <= 6).
 *
 * Canonical order of the basis: ascending (A bits as an unsigned integer,
 * summed quanta Q_B of species B, B bits as an unsigned integer).  Within the
 * states of one A configuration ("A-block", the grouping of Sec. 2 into
 * many-body basis orbitals) the B configurations therefore form a prefix of
 * one list per 2M_B ordered by (Q_B, B).
 */
typedef struct {
  int32_t n_species;      /* 1 or 2                                        */
  int32_t nmax[2];        /* highest shell per species, 0..6               */
  int32_t n_particles[2]; /* particles per species, 1..n_orb               */
  int32_t two_M;          /* twice the total projection                    */
  int32_t cut;            /* summed-quanta truncation above minimum; <0: none */
} cib_basis_spec;

/* Enumerate the basis on the device.  *dim receives D.  Errors:
 * CIB_E_INVALID (n_species not 1/2, nmax outside 0..6, N outside 1..n_orb,
 * two_M parity differs from N_A + N_B), CIB_E_EMPTY_BASIS (D = 0),
 * CIB_E_OVERFLOW (D >= 2^31). */
cib_status cib_build_basis(cib_ctx *ctx, const cib_basis_spec *spec, cib_basis **out, int64_t *dim);
/* D, words per species (species B: 0 when absent), orbitals per species, and
 * the number of non-empty A-blocks. */
cib_status cib_basis_info(const cib_basis *b, int64_t *dim, int32_t words[2], int32_t n_orb[2],
                          int64_t *n_ablocks);
/* Copy the basis to caller-owned host memory: D x (words[0] + words[1])
 * uint64, state-major, species A words first.  Synchronises the ctx stream. */
cib_status cib_basis_export(const cib_basis *b, uint64_t *host_words);
void cib_basis_free(cib_basis *b);

/* ----------------------------------------------------------- interaction --
 * H = sum_s sum_a eps^s_a n_a
 *   + sum_s sum_{a<b, c<d} V^s_{ab,cd} a+_a a+_b a_d a_c
 *   + sum_{a,c in A; b,d in B} V^AB_{ab,cd} a+_a b+_b b_d a_c
 * Table layout ("M-blocked"): pairs are grouped by 2M_pair = 2m_a + 2m_b in
 * ascending order; inside a block pairs are lexicographic in (a, b).
 * Same-species pairs have a < b; cross-species pairs are all (a in A, b in B).
 * Each block is a full n_M x n_M row-major matrix, blocks concatenated; the
 * value for creation pair p and annihilation pair q is block[p * n_M + q].
 * The library reads only what the operator needs and does not require the
 * blocks to be symmetric, but H is symmetric only if they are.
 * Sign convention: a creation or annihilation operator acting on global mode
 * k (species A orbital k, or species B orbital k + n_orb[0]) contributes
 * (-1)^(occupied modes below k). */
typedef struct {
  const double *eps[2];    /* one-body energies, n_orb[s] each              */
  const double *v_same[2]; /* same-species blocked tables                   */
  const double *v_ab;      /* cross-species blocked table; NULL for 1 species */
} cib_tables;

/* Upload the tables for `basis`'s orbital sets (host arrays, copied).
 * CIB_E_OVERFLOW when the cross-species table, regrouped by orbital
 * transitions, would hold 2^29 or more values (far beyond the bases of the
 * paper's workloads). */
cib_status cib_upload_interaction(cib_ctx *ctx, const cib_basis *basis, const cib_tables *t,
                                  cib_interaction **out);
void cib_interaction_free(cib_interaction *it);

/* -------------------------------------------------------------- build H --
 * H_ij = <Phi_i|H|Phi_j> stored as the upper triangle (j >= i, diagonal first)
 * in CSR: int64 row_ptr[D+1], int32 col[nnz_half] ascending within a row,
 * values float64 or float32 (float32 = round-to-nearest-even of the float64
 * value).  The stored pattern is structural: every pair whose bit strings
 * differ in at most four orbitals (Sec. 2.1), whether or not its value is
 * zero.  Counting pass, counts -> offsets prefix sum, and a filling pass
 * (Fig. 1 steps 6-14; Sec. 2.2-2.3) with a deterministic in-row order.
 * Host synchronisations: the screen totals and the nonzero total size the
 * allocations.  The matrix also keeps the strictly lower triangle (built by
 * the same row passes, over the transposed screens, bitwise the transpose for
 * symmetric tables) because the SpMM reads both triangles instead of
 * scattering the transposed half with atomics; cib_matrix_export returns
 * only the upper half. */
cib_status cib_build_H(cib_ctx *ctx, const cib_basis *basis, const cib_tables *t, cib_dtype dtype,
                       cib_matrix **out, int64_t *nnz_half);
/* Same, with tables already on the device. */
cib_status cib_build_H_resident(cib_ctx *ctx, const cib_basis *basis, const cib_interaction *it,
                                cib_dtype dtype, cib_matrix **out, int64_t *nnz_half);

/* Every stage builds the stored upper half and the strictly lower copy the
 * SpMM reads side by side, so each time below covers both. */
typedef struct {
  /* device time of each stage of the last build, from HIP events, seconds */
  double t_screen_s;  /* A-configuration tile screen + B-configuration adjacency */
  double t_count_s;   /* per-row counting pass                           */
  double t_scan_s;    /* counts -> offsets                               */
  double t_fill_s;    /* per-row filling pass (both stored triangles)    */
  double t_total_s;   /* sum of the above (host waits between stages excluded) */
  int64_t n_tiles;    /* A-configuration pairs kept by the screen        */
  int64_t n_adjacent; /* B-configuration pairs kept by the screen        */
} cib_build_stats;

cib_status cib_matrix_info(const cib_matrix *H, int64_t *dim, int64_t *nnz_half, cib_dtype *dtype);
cib_status cib_matrix_stats(const cib_matrix *H, cib_build_stats *stats);
/* Copy the CSR to caller-owned host arrays (any may be NULL to skip).
 * val receives nnz_half elements of the matrix dtype.  Synchronises. */
cib_status cib_matrix_export(const cib_matrix *H, int64_t *row_ptr, int32_t *col, void *val);
/* Device pointers of the CSR arrays (owned by the matrix). */
cib_status cib_matrix_device(const cib_matrix *H, const int64_t **row_ptr, const int32_t **col,
                             const void **val);
void cib_matrix_free(cib_matrix *H);

/* -------------------------------------------------------------- apply H --
 * Y = H X for nvec vectors (1..64).  X and Y are device arrays of the matrix
 * dtype, D rows, row-major: element (i, v) at X[i * ldx + v], ldx >= nvec
 * (same for Y).  Asynchronous on the context stream; Y is overwritten.  Each
 * output row is gathered from both stored triangles (no atomics), so every
 * call gives the same bits. */
cib_status cib_apply_H(cib_ctx *ctx, const cib_matrix *H, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, int32_t nvec);

/* ----------------------------------------------------- matrix-free H X --
 * Y = H X without storing H (the multiply variant of the generic loop of
 * Fig. 2: compare, compute, multiply with the vector elements), for bases
 * whose matrix does not fit: H is given by the basis and the interaction
 * uploaded for it, the screens and per-entry values are computed as by
 * cib_build_H_resident, and one row pass multiplies every entry into X.
 * Matrix values are rounded to `dtype` as the stored matrix's are; the sum
 * order differs from cib_apply_H, so the two agree to rounding.  X, Y:
 * device arrays of `dtype`, D rows, row-major, nvec = 8 or 16 columns,
 * rows 16-byte aligned (X, Y and ldx * size, ldy * size multiples of 16).
 * Device memory: the screens (a small fraction of the matrix).  Returns when
 * Y is written.  Errors: CIB_E_INVALID for NULL pointers, a bad dtype,
 * nvec, leading dimension or alignment, an interaction of another orbital
 * set or a basis of another context. */
cib_status cib_apply_H_free(cib_ctx *ctx, const cib_basis *basis, const cib_interaction *it, cib_dtype dtype,
                            const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nvec);

/* ---------------------------------------------------------- observables --
 * Expectation values after the eigensolve (Fig. 1 steps 16-20):
 * out[k * nvec + v] = x_v^T O_k x_v for the m operators O_k given by ops[k]
 * (host tables in the cib_tables layout, for `basis`'s orbital sets; a
 * one-body operator has zero two-body tables) and the nvec vectors x_v
 * (1..64): X is a device array of `dtype`, D rows, row-major, element
 * (i, v) at X[i * ldx + v], ldx >= nvec.  Each operator is applied once:
 * with nvec = 8 or 16 and 16-byte aligned rows by the matrix-free product
 * of cib_apply_H_free (device memory: the screens), otherwise built as a
 * half-stored matrix of `dtype` by the same passes as cib_build_H, applied,
 * and freed before the next (device memory: one operator's matrix), plus
 * D x nvec values.  The products are summed in float64 in a fixed order, so
 * results are deterministic.  out: host, m * nvec doubles.  Synchronous.
 * Errors: CIB_E_INVALID for NULL pointers, m < 1, nvec outside 1..64,
 * ldx < nvec, a bad dtype or a basis of another context; CIB_E_NOMEM when
 * an operator's matrix does not fit. */
cib_status cib_observables(cib_ctx *ctx, const cib_basis *basis, const cib_tables *ops, int32_t m,
                           cib_dtype dtype, const void *X, int64_t ldx, int32_t nvec, double *out);

/* ------------------------------------------------------- state counting --
 * The state-counting test (Sec. 2.1; Listing 2 as a description): for each
 * of n many-body states, the number of states of the same list (itself
 * included) that differ from it in at most two particles, i.e. the nonzeros
 * of its row for a two-body operator.  mbs: device, n x n_particles uint16
 * single-particle indices, state-major, each row strictly ascending and
 * below n_sp (the index-tuple representation).  method: 0 = hybrid (bit
 * string of the lowest 64 single-particle states as a prefilter, then
 * count_difference on the tuples), 1 = count_difference on the tuples only,
 * 2 = popcount of the full 128-bit bit strings (n_sp <= 128); all three give
 * the same counts.  counts: device int32[n] or NULL; total: host, the sum.
 * Synchronous.  Errors: CIB_E_INVALID for NULL mbs/total, n outside
 * 1..2^22, n_particles outside 1..20, n_sp outside n_particles..65534, a bad
 * method, or method 2 with n_sp > 128.  Rows that are not ascending or hold
 * repeated indices give meaningless counts (no other effect). */
cib_status cib_count_states(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int32_t n_particles, int32_t n_sp,
                            int32_t method, int32_t *counts, int64_t *total);
/* cib_count_states for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, with their scratch (the
 * encoded states, the counts when counts is NULL, the total) in one static
 * device array of about 7.9 MB that every device the library runs on holds
 * until the process ends.  No hipMalloc, hipFree or other allocation.  n is
 * limited to 1..131072 (2^17): larger n gives CIB_E_INVALID with the limit
 * in the message; the other arguments and errors are those of
 * cib_count_states.  Every call on one device uses that device's array
 * (clearing the counts first), so calls that overlap on one device race and
 * must be serialised by the caller.  Synchronous. */
cib_status cib_count_states_noalloc(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int32_t n_particles,
                                    int32_t n_sp, int32_t method, int32_t *counts, int64_t *total);

/* ------------------------------------------------------- preconditioner --
 * Block-diagonal LOBPCG preconditioner over many-body basis orbitals (Sec. 2:
 * the states whose particles have the same (n, l, j) values, any m, form a
 * group, and the groups give a block-diagonal preconditioner).  A state's
 * group is the pair of its species' level occupations (particles per (n, 2j)
 * level); groups are ordered by their lowest state, states ascending inside;
 * a group of more than max_block (1..64) states is cut into consecutive runs
 * of max_block, and each run is one block.  Set-up: the blocks of H (its
 * stored entries whose row and column share a block) and their eigenpairs
 * by cyclic Jacobi rotations in float64 on the device.  Apply, for column c:
 * W_c = Q diag(1 / g(lambda_j - theta_c)) Q^T R_c per block, g moving gaps
 * below 1e-2 in magnitude to +-1e-2; max_block = 1 is exactly the diagonal
 * preconditioner.  H must have been built on basis b (same D); the object
 * keeps no reference to either.  Device memory: D x (max_block + 4) doubles
 * at most.  Synchronous. */
cib_status cib_precond_create(cib_ctx *ctx, const cib_basis *b, const cib_matrix *H, int32_t max_block,
                              cib_precond **out);
/* blocks, groups, largest block, and the most Jacobi sweeps a block took */
cib_status cib_precond_info(const cib_precond *P, int64_t *n_blocks, int64_t *n_groups, int32_t *largest,
                            int32_t *max_sweeps);
/* Host copies of the blocks: perm (D int32: states in block order) and
 * block_off (n_blocks + 1 int64: start of each block in perm); either may be
 * NULL. */
cib_status cib_precond_export(const cib_precond *P, int32_t *perm, int64_t *block_off);
/* W = M(theta)^-1 R for ncol (1..16) columns: R, W device float64, D x ncol
 * row-major with leading dimensions ldr, ldw >= ncol (W may be R, with ldw ==
 * ldr; no other overlap); theta host,
 * ncol shifts.  Deterministic (fixed summation order).  Synchronous. */
cib_status cib_precond_apply(cib_ctx *ctx, const cib_precond *P, const double *theta, const double *R, int64_t ldr,
                             double *W, int64_t ldw, int32_t ncol);
void cib_precond_free(cib_precond *P);

/* --------------------------------------------------------------- LOBPCG --
 * Lowest nev eigenpairs of H (Fig. 1 step 15) by block LOBPCG with block size
 * `block` (nev <= block <= 16, 3*block <= D).  Search space [X, W, P]; all
 * dense work (Gram matrices, Rayleigh-Ritz, residual norms) in float64 on the
 * device; the SpMM runs in the matrix dtype.  Preconditioner: diagonal,
 * W = R / (diag(H) - lambda) with |diag - lambda| clamped below at 1e-2, or,
 * when `precond` is set, the block-diagonal one of cib_precond_create (same
 * guard on each block's eigenvalue gaps).
 * Converged when ||H x_k - lambda_k x_k|| <= tol * max(|lambda_k|, 1) for all
 * k < nev (tol <= 0: 1e-9 for float64 H; 1e-5 for float32 H, whose SpMM
 * rounding floors the residual near 1e-6 while the eigenvalue error, quadratic
 * in the residual, stays far below 1e-6).  Soft locking: a column whose
 * residual met tol at the previous iteration gets W = 0, so it leaves the
 * search space (its direction is dropped by the Cholesky) until it drifts out.
 * X0: unit vectors at the `block` smallest diagonal entries (ties: lower
 * index) plus 1e-3 * noise from a counter-based generator keyed by `seed`,
 * unless x0 (device, D x block float64 row-major) is given. */
typedef struct {
  int32_t nev, block, max_iter;
  double tol;
  uint64_t seed;
  const double *x0;
  const cib_precond *precond;   /* NULL: diagonal; else made for this H */
} cib_lobpcg_opts;

typedef struct {
  int32_t iters, n_converged;
  double resid[64];     /* relative residual per eigenpair                 */
  double t_total_s;     /* wall time of the call                           */
  double t_spmm_s;      /* device time in the SpMM (events)                */
  int64_t n_spmm;       /* SpMM launches                                   */
} cib_lobpcg_info;

/* evals: host, nev float64.  evecs: device, D x nev float64 row-major with
 * leading dimension ld_evecs (>= nev), or NULL. */
cib_status cib_lobpcg(cib_ctx *ctx, const cib_matrix *H, const cib_lobpcg_opts *opts, double *evals,
                      double *evecs, int64_t ld_evecs, cib_lobpcg_info *info);

/* -------------------------------------------------------------- Lanczos --
 * Lowest nev eigenpairs of H (Fig. 1 step 15; the eigensolver the paper
 * names beside LOBPCG) by Lanczos with full reorthogonalisation: each step
 * applies H to one vector (cib_apply_H's SpMM; a float32 H gets a float32
 * copy of the vector), orthogonalises against every kept vector by
 * classical Gram-Schmidt applied twice, and extends the tridiagonal matrix
 * T; T's lowest eigenvalues (bisection of Sturm counts) and vectors
 * (inverse iteration) are computed on the host every fourth step.  Stops
 * when every Ritz pair's residual beta_k |s_k| <= tol max(|theta|, 1).
 * Vectors are float64 on the device: (max_iter + 1) x D doubles. */
typedef struct {
  int32_t nev;       /* 1..64, <= D                                          */
  int32_t max_iter;  /* steps (kept vectors), nev..4096                      */
  double tol;        /* relative residual; 0: 1e-10 (float64 H), 1e-6 (float32 H) */
  uint64_t seed;     /* start vector: SplitMix64 of (seed, row)              */
} cib_lanczos_opts;

typedef struct {
  int32_t iters, n_converged;
  double resid[64];     /* relative residual per eigenpair                 */
  double t_total_s;     /* wall time of the call                           */
  double t_spmv_s;      /* device time in the products with H (events)     */
} cib_lanczos_info;

/* evals: host, nev float64.  evecs: device, D x nev float64 row-major with
 * leading dimension ld_evecs (>= nev), or NULL.  Returns
 * CIB_E_NOT_CONVERGED (with the current estimates in evals) when max_iter
 * steps do not reach the tolerance; CIB_E_INVALID for NULL arguments, nev,
 * max_iter or ld_evecs out of range, or a matrix of another context. */
cib_status cib_lanczos(cib_ctx *ctx, const cib_matrix *H, const cib_lanczos_opts *opts, double *evals,
                       double *evecs, int64_t ld_evecs, cib_lanczos_info *info);

/* The host step of cib_lanczos, on its own (no device): the lowest k
 * eigenpairs of the symmetric tridiagonal matrix with diagonal a[n] and
 * off-diagonal b[n-1] (b unused when n = 1), by bisection of Sturm counts
 * and inverse iteration (pivots kept at 2.2e-16 |T| or more), orthonormalised
 * in order.  theta: k values ascending; S: n x k row-major, column c the
 * vector of theta[c].  Host arrays.  Errors: CIB_E_INVALID for NULL
 * arguments or k outside 1..n. */
cib_status cib_tridiag_lowest(const double *a, const double *b, int32_t n, int32_t k, double *theta,
                              double *S);

/* ---------------------------------------------------------------- serve --
 * Continuous batching of eigensolve requests.  Requests arrive at arrival_s
 * (relative to the call start; replayed in real time when opts->realtime,
 * else all are available at once).  A request is admitted when a slot is free
 * (max_active) and its device footprint fits the HBM budget.  Four builder
 * threads, each on a stream of its own, take admitted requests through the
 * basis and the H build while the solver loop runs.  Each solver step starts
 * the solves of newly built requests (one of n_streams streams each) and
 * advances every iterating request by one LOBPCG iteration, one launch per
 * stage covering all of them (SpMM, Gram, partial sums, Rayleigh-Ritz,
 * update, residual sums, finish; the launch parameters of each request are
 * those of its own solve, so its iterates are the same bits as when it runs
 * alone; a request the grouped SpMM cannot take iterates on its own stream),
 * reads the convergence flags back, and retires finished requests,
 * releasing their memory. */
typedef struct {
  uint64_t id;
  double arrival_s;
  cib_basis_spec basis;
  const cib_tables *tables;  /* host, read during the call */
  cib_dtype dtype;
  cib_lobpcg_opts solve;     /* nev <= 16; x0 must be NULL */
} cib_request;

typedef struct {
  uint64_t id;
  cib_status status;         /* CIB_OK, CIB_E_NOT_CONVERGED, CIB_E_EMPTY_BASIS, ... */
  int64_t dim, nnz_half;
  int32_t iters;
  double evals[16], resid[16];
  double t_arrive, t_admit, t_done;  /* seconds since the call started */
} cib_result;

typedef struct {
  size_t hbm_budget_bytes;   /* 0: 90% of free device memory at the call   */
  int32_t max_active;        /* <= 0: 64                                    */
  int32_t realtime;          /* honour arrival_s in wall-clock time         */
  double deadline_s;         /* <= 0: none; later requests get CIB_E_CANCELLED */
  int32_t n_streams;         /* <= 0: 8                                     */
} cib_serve_opts;

/* results: caller-owned array of n.  The return value reports only
 * infrastructure failure; per-request outcome is in results[i].status. */
cib_status cib_serve(cib_ctx *ctx, const cib_request *reqs, int32_t n, const cib_serve_opts *opts,
                     cib_result *results);

#ifdef __cplusplus
}
#endif
#endif /* CIB_H */
