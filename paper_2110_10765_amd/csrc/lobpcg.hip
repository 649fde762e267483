// Block LOBPCG for the lowest eigenpairs of the half-stored H (Fig. 1 step 15
// of the paper: "lowest n eigenvalues ... using LOBPCG").
//
// Search space S = [X | W | P] (b columns each), kept row-interleaved: row i
// of S holds X_i, W_i, P_i contiguously (3b float64), and HS = H S likewise.
// Per iteration: W <- H W (SpMM in the matrix dtype), partial Gram matrices
// S^T S and S^T HS over row chunks, one workgroup that reduces them and does
// the Rayleigh-Ritz step in float64 (scaled Cholesky of S^T S with dropping
// of dependent directions, reduced matrix, Householder tridiagonalisation,
// multisection for the wanted eigenvalues, twisted-factorisation
// eigenvectors), then a
// row-parallel update X, P, HX, HP <- S C, HS C, the residual R = HX - X L,
// its norms and the preconditioned W = R / (diag(H) - lambda).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

constexpr int kNS = 3 * kMaxBlock;   // 48: largest search space
constexpr int kLd = kNS + 1;         // padded LDS row length

// ------------------------------------------------------------ small kernels
template <typename T>
__global__ __launch_bounds__(256) void k_diag(int64_t D, const int64_t *rp, const T *val, double *diag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D) diag[i] = (double)val[rp[i]];   // the diagonal is each row's first entry
}

// The b smallest diagonal entries (ties: lower index), one workgroup.
// One pass of the selection of the b smallest (value, index) pairs, ties to
// the lower index: each workgroup takes kSelChunk consecutive candidates
// into LDS and emits its own b smallest, in order, by b rounds of a block
// arg-min (a chosen candidate is set to +inf in LDS).  The host repeats the
// pass on the emitted candidates until one workgroup remains.
constexpr int kSelChunk = 4096;

__global__ __launch_bounds__(256) void k_select_pass(int64_t n, const double *__restrict__ val,
                                                     const int64_t *__restrict__ id, int b,
                                                     double *__restrict__ oval, int64_t *__restrict__ oid) {
  __shared__ double sv[kSelChunk];
  __shared__ int64_t si[kSelChunk];
  __shared__ double wv[4];
  __shared__ int wk[4];
  const int64_t c0 = (int64_t)blockIdx.x * kSelChunk;
  const int m = (int)min<int64_t>(kSelChunk, n - c0);
  for (int k = threadIdx.x; k < kSelChunk; k += blockDim.x) {
    sv[k] = k < m ? val[c0 + k] : INFINITY;
    si[k] = k < m ? (id ? id[c0 + k] : c0 + k) : INT64_MAX;
  }
  __syncthreads();
  for (int r = 0; r < b; ++r) {
    double best = INFINITY;
    int bk = -1;
    for (int k = threadIdx.x; k < kSelChunk; k += blockDim.x) {
      const double v = sv[k];
      if (bk < 0 || v < best || (v == best && si[k] < si[bk])) { best = v; bk = k; }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const double ov = __shfl_xor(best, d, kWave);
      const int ok = __shfl_xor(bk, d, kWave);
      if (ov < best || (ov == best && si[ok] < si[bk])) { best = ov; bk = ok; }
    }
    if (lane_id() == 0) { wv[threadIdx.x >> 6] = best; wk[threadIdx.x >> 6] = bk; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = wv[0];
      int bx = wk[0];
      for (int w = 1; w < 4; ++w)
        if (wv[w] < bv || (wv[w] == bv && si[wk[w]] < si[bx])) { bv = wv[w]; bx = wk[w]; }
      oval[(int64_t)blockIdx.x * b + r] = bv;
      oid[(int64_t)blockIdx.x * b + r] = si[bx];
      sv[bx] = INFINITY;
      si[bx] = INT64_MAX;
    }
    __syncthreads();
  }
}

// X0 = e_{idx[c]} + 1e-3 * N(0,1) (Box-Muller from two SplitMix64 uniforms).
__global__ __launch_bounds__(256) void k_init_x(int64_t D, int b, int ld, const int64_t *idx,
                                                uint64_t seed, double *S) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D * b) return;
  const int64_t i = k / b;
  const int c = (int)(k % b);
  const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * (uint64_t)k));
  const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * (uint64_t)k + 1));
  const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  S[i * ld + c] = (idx[c] == i ? 1.0 : 0.0) + 1e-3 * g;
}

__global__ __launch_bounds__(256) void k_copy_x0(int64_t D, int b, int ld, const double *x0, double *S) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * b) S[(k / b) * ld + (k % b)] = x0[k];
}

// float64 block (ld_in) <-> float32 block (dense D x b)
__global__ __launch_bounds__(256) void k_narrow(int64_t D, int b, const double *in, int ldi, float *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * b) out[k] = (float)in[(k / b) * ldi + (k % b)];
}
// stop (here and below): a solve's stop flag; nonzero once it has converged,
// so the launches of iterations queued past that point do nothing
__global__ __launch_bounds__(256) void k_widen(int64_t D, int b, const float *in, double *out, int ldo,
                                               const int32_t *stop) {
  if (*stop) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * b) out[(k / b) * ldo + (k % b)] = (double)in[k];
}
__global__ __launch_bounds__(256) void k_widen_group(const WidenArgs *__restrict__ as, const int32_t *__restrict__ off,
                                                     int njobs) {
  const int j = group_job(off, njobs, (int)blockIdx.x);
  const WidenArgs a = as[j];
  const int64_t k = (int64_t)(blockIdx.x - off[j]) * blockDim.x + threadIdx.x;
  if (k < a.D * a.b) a.out[(k / a.b) * a.ldo + (k % a.b)] = (double)a.in[k];
}

__global__ __launch_bounds__(256) void k_copy_cols(int64_t D, int n, const double *S, int lds, double *out,
                                                   int64_t ldo) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * n) out[(k / n) * ldo + (k % n)] = S[(k / n) * lds + (k % n)];
}

// ------------------------------------------------------------ Gram matrices
// partial[blk] = sum over the block's rows of S_i^T [S_i, HS_i] for the first
// ns columns, as its upper 16 x 16 tiles: first those of S^T S, then those
// of S^T HS (gram_tiles(ns) doubles, the final partial-sum pass mirrors them
// into the Rayleigh-Ritz layout).  This
// is a dense contraction over the rows, done on the float64 matrix cores:
// v_mfma_f64_16x16x4f64 multiplies a 16 x 4 by a 4 x 16 block.  Four
// consecutive rows form one step; lane l holds row (l / 16), column
// 16 t + (l % 16) of tile t, which is at once the lane's element of the left
// operand (S^T, 16 x 4) and of the right operand (S or HS, 4 x 16), so the
// rows go from global memory straight into the operands (coalesced 128-byte
// row pieces, no LDS).  Output tile (ti, tj): lane l, element v holds row
// 16 ti + 4 v + (l / 16), column 16 tj + (l % 16) (checked on the device).
// S^T S and S^T HS are symmetric (H is): only their tiles ti <= tj are
// formed (the Rayleigh-Ritz step symmetrises S^T HS anyway, so the tiles
// below the diagonal added nothing but rounding).  The four waves of a
// workgroup take alternate steps (the next step's rows load during the
// current one); waves 0 and 1 store their tiles in LDS, waves 2 and 3 add
// theirs, and the workgroup writes (w0 + w2) + (w1 + w3) with coalesced
// stores.  The main loop streams S and HS at about 5 TB/s; adding the four
// waves one after another in the full layout had cost 15 of the kernel's
// 50 us at ns = 48.
constexpr int kGramSteps = 4;   // rows per matrix-core step
// doubles of one workgroup's partial Gram matrices: the upper 16 x 16 tiles
// of S^T S and of S^T HS, each tile lane-major (element v * 64 + lane)
__host__ __device__ constexpr int gram_tiles(int ns) {
  return 2 * ((ns + 15) / 16) * ((ns + 15) / 16 + 1) / 2 * 256;
}
constexpr int kGramPad = 48;    // doubles allocated past the last row of S and HS
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int T>   // 16-column tiles per side: ns <= 16 T
__device__ __forceinline__ void gram_block(int64_t D, int ns, int ld, const double *__restrict__ S,
                                           const double *__restrict__ HS, int64_t rows_per_blk,
                                           double *__restrict__ partial, int blk) {
  constexpr int NG = T * (T + 1) / 2;   // upper tiles of S^T S (and of S^T HS)
  __shared__ double red[2][2 * NG * 256];
  const int wv = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int kr = lane >> 4, kc = lane & 15;
  const int64_t r0 = (int64_t)blk * rows_per_blk;
  const int64_t r1 = min(D, r0 + rows_per_blk);
  dbl4 ag[NG], ah[NG];
#pragma unroll
  for (int a = 0; a < NG; ++a) {
    ag[a] = dbl4{0.0, 0.0, 0.0, 0.0};
    ah[a] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  // loads from a valid address in every lane, then select: a load under a
  // branch would make the compiler wait for the prefetch as well.  Columns
  // up to 16 T - 1 are read unclamped (S and HS carry kGramPad doubles of
  // padding past the last row), so the tiles of a row sit at fixed offsets.
  auto fetch = [&](int64_t rb, double (&xs)[T], double (&xh)[T]) {
    const int64_t row = rb + kr;
    const bool rok = row < r1;
    const double *sp = S + (rok ? row : r0) * ld + kc, *hp = HS + (rok ? row : r0) * ld + kc;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const bool ok = rok && 16 * t + kc < ns;
      const double vs = sp[16 * t], vh = hp[16 * t];
      xs[t] = ok ? vs : 0.0;
      xh[t] = ok ? vh : 0.0;
    }
  };
  constexpr int kStride = 4 * kGramSteps;   // rows per round of the four waves
  double xs[T], xh[T], ys[T], yh[T];
  int64_t rb = r0 + (int64_t)wv * kGramSteps;
  fetch(rb, xs, xh);
  for (; rb < r1; rb += kStride) {
    fetch(rb + kStride, ys, yh);   // rows past the slab load as 0
    int g = 0;
#pragma unroll
    for (int a = 0; a < T; ++a) {
#pragma unroll
      for (int c = a; c < T; ++c, ++g) {
        ag[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[a], xs[c], ag[g], 0, 0, 0);
        ah[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[a], xh[c], ah[g], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      xs[t] = ys[t];
      xh[t] = yh[t];
    }
  }
  // waves 0 and 1 store their tiles, waves 2 and 3 add theirs: (w0 + w2) + (w1 + w3)
  double *rw = red[wv & 1];
  if (wv < 2) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rw[g * 256 + v * 64 + lane] = ag[g][v];
        rw[(NG + g) * 256 + v * 64 + lane] = ah[g][v];
      }
  }
  __syncthreads();
  if (wv >= 2) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rw[g * 256 + v * 64 + lane] += ag[g][v];
        rw[(NG + g) * 256 + v * 64 + lane] += ah[g][v];
      }
  }
  __syncthreads();
  double *out = partial + (int64_t)blk * (2 * NG * 256);
  for (int e = threadIdx.x; e < 2 * NG * 256; e += blockDim.x) out[e] = red[0][e] + red[1][e];
}

template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gram(
    int64_t D, int ns, int ld, const double *__restrict__ S, const double *__restrict__ HS,
    int64_t rows_per_blk, double *__restrict__ partial, const int32_t *stop) {
  if (*stop) return;
  gram_block<T>(D, ns, ld, S, HS, rows_per_blk, partial, blockIdx.x);
}

template <int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gram_group(
    const GramArgs *__restrict__ as, const int32_t *__restrict__ off, int njobs) {
  const int j = group_job(off, njobs, (int)blockIdx.x);
  const GramArgs a = as[j];
  gram_block<T>(a.D, a.ns, a.ld, a.S, a.HS, a.rows_per_blk, a.partial, blockIdx.x - off[j]);
}

// out[g][e] = sum of in[q][e] over the parts q of group g (grid.y = groups of
// `per` consecutive parts), in a fixed order.  One thread per output element
// (coalesced); all loads of a group are in flight together.  The Gram
// reduction runs it twice: groups of 32 partial matrices, then the group sums.
__device__ __forceinline__ void sum_parts_elem(int nout, int nparts, int per, const double *__restrict__ in,
                                               double *__restrict__ out, int e, int grp, int pad) {
  if (e >= nout) return;
  const int q0 = grp * per, q1 = min(nparts, q0 + per);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int q = q0;
  for (; q + 8 <= q1; q += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = in[(int64_t)(q + t) * nout + e];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t & 3] += v[t];
  }
  for (; q < q1; ++q) acc[q & 3] += in[(int64_t)q * nout + e];
  const double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (pad > 0) {   // the upper tiles of S^T S and S^T H S (pad = ns) into two kNS x kLd blocks, mirrored
    const int T = (pad + 15) / 16, NG = T * (T + 1) / 2;
    int tile = e >> 8;
    const int which = tile >= NG;
    if (which) tile -= NG;
    int a = 0, c = 0;   // the tile's (row, column) among the upper tiles, row by row
    for (int nrow = T; a < T; ++a, --nrow) {
      if (tile < nrow) {
        c = a + tile;
        break;
      }
      tile -= nrow;
    }
    const int r = e & 255, lane = r & 63;
    const int i = 16 * a + 4 * (r >> 6) + (lane >> 4), j = 16 * c + (lane & 15);
    if (i < pad && j < pad) {
      double *o = out + (which ? kNS * kLd : 0);
      o[i * kLd + j] = v;
      if (a < c) o[j * kLd + i] = v;
    }
  } else {
    out[(int64_t)grp * nout + e] = v;
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(int nout, int nparts, int per, const double *__restrict__ in,
                                                   double *__restrict__ out, int pad, const int32_t *stop) {
  if (*stop) return;
  sum_parts_elem(nout, nparts, per, in, out, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, pad);
}

// a job's workgroups cover (element block, group) as x + xblocks * group
__global__ __launch_bounds__(256) void k_sum_parts_group(const SumArgs *__restrict__ as,
                                                         const int32_t *__restrict__ off, int njobs) {
  const int j = group_job(off, njobs, (int)blockIdx.x);
  const SumArgs a = as[j];
  const int loc = blockIdx.x - off[j];
  const int xb = (a.nout + 255) / 256;
  sum_parts_elem(a.nout, a.nparts, a.per, a.in, a.out, (loc % xb) * 256 + threadIdx.x, loc / xb, a.pad);
}

// Gershgorin lower bound of H: min_i (H_ii - sum_{j != i} |H_ij|), both halves.
template <typename T>
__global__ __launch_bounds__(256) void k_gersh_rows(int64_t D, const int64_t *rp, const T *val, const int64_t *lrp,
                                                    const T *lval, double *out) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (i >= D) return;
  const int lane = lane_id();
  double sum = 0.0;
  for (int64_t k = rp[i] + 1 + lane; k < rp[i + 1]; k += kWave) sum += fabs((double)val[k]);
  for (int64_t k = lrp[i] + lane; k < lrp[i + 1]; k += kWave) sum += fabs((double)lval[k]);
  sum = wave_sum(sum);
  if (lane == 0) out[i] = (double)val[rp[i]] - sum;
}

__global__ __launch_bounds__(1024) void k_min(int64_t n, const double *in, double *out) {
  __shared__ double red[1024 / kWave];
  double m = INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, in[i]);
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmin(m, __shfl_xor(m, d, kWave));
  if (lane_id() == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmin(r, red[w]);
    out[0] = r;
  }
}

// ------------------------------------------------------------ Rayleigh-Ritz

#include "rayleigh_ritz.hpp"

__global__ __launch_bounds__(256) void k_rayleigh_ritz(RRArgs g) {
  if (g.stop && *g.stop) return;
  rayleigh_ritz(g);
}

// The Rayleigh-Ritz steps of several independent solves in one launch, one
// workgroup each (each on its own compute unit): the serving loop's batch.
__global__ __launch_bounds__(256) void k_rayleigh_ritz_group(const RRArgs *__restrict__ gs) {
  const RRArgs g = gs[blockIdx.x];
  rayleigh_ritz(g);
}


// ------------------------------------------------------------ update

// [X P] = S [Cx Cp] and [HX HP] = HS [Cx Cp] on the float64 matrix cores, then
// the residual R = HX - X diag(lambda), the preconditioned W and the new
// blocks written in place.  One wave per 16 rows: the contraction index k
// (a column of S) is split as k = KS (l / 16) + s, so lane l reads the KS
// consecutive columns of row 16 q + (l % 16) it needs (left operand
// A[i][k] = S[row i][k]) and keeps the matching rows of [Cx Cp] (right
// operand) in registers for every step s.  Output element v of lane l is row
// 4 v + (l / 16), column 16 t + (l % 16) of output tile t; the lane holding x
// also holds hx, so the residual needs no exchange.  All reads of a row come
// before its writes (the MFMAs consume every loaded value), so the update is
// in place.  Per-column sums of the squared residuals and |x|^2 are reduced
// over lanes and waves in a fixed order.
template <int TN>   // 16-column output tiles over the 2b columns of [Cx Cp]
__device__ __forceinline__ void update_block(const UpdArgs &g, int blk) {
  constexpr int KMAX = kNS / 4;   // steps of the contraction (ns <= 48)
  __shared__ double lam[kMaxBlock];
  __shared__ double red[2][4][64];
  __shared__ double Cs[kNS][16 * TN];   // [Cx Cp], zero past ns rows / 2b columns
  __shared__ double rows[4][2][16][kNS + 1];   // per wave: its 16 rows of S and HS (padded)
  const int b = g.b, ns = g.ns, ld = g.ld, nb2 = 2 * b;
  const int wv = uni((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int kr = lane >> 4, kc = lane & 15;
  const int KS = (ns + 3) / 4;
  if (threadIdx.x < b) lam[threadIdx.x] = g.lam[threadIdx.x];
  for (int e = threadIdx.x; e < kNS * 16 * TN; e += blockDim.x) {
    const int k = e / (16 * TN), j = e % (16 * TN);
    Cs[k][j] = (k < ns && j < nb2) ? g.C[k * nb2 + j] : 0.0;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blk * g.rows_per_blk;
  const int64_t r1 = min(g.D, r0 + g.rows_per_blk);
  double rs = 0.0, xs = 0.0;   // this lane's column kc (when kc < b)
  for (int64_t rb = r0 + 16 * (int64_t)wv; rb < r1; rb += 64) {
    // the 16 rows go to LDS with row-contiguous loads (lane = column), the
    // operands come back out in the MFMA layout (row stride kNS + 1 keeps
    // the 16 rows of one read in distinct banks).  All 32 loads are issued
    // before the first LDS store (four at a time, as before, cost four
    // memory round trips per tile: 90 -> 77 us at D = 198,912, b = 16)
    double vs[16], vh[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = rb + r;
      const int64_t off = (i < r1 ? i : r0) * ld + (lane < ns ? lane : 0);
      vs[r] = g.S[off];
      vh[r] = g.HS[off];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool ok = rb + r < r1 && lane < ns;
      if (lane < kNS) {
        rows[wv][0][r][lane] = ok ? vs[r] : 0.0;
        rows[wv][1][r][lane] = ok ? vh[r] : 0.0;
      }
    }
    wave_lds_sync();
    double as[KMAX], ah[KMAX];
#pragma unroll
    for (int st = 0; st < KMAX; ++st) {
      const int k = min(KS * kr + st, kNS - 1);
      const bool ok = st < KS && KS * kr + st < ns;
      as[st] = ok ? rows[wv][0][kc][k] : 0.0;
      ah[st] = ok ? rows[wv][1][kc][k] : 0.0;
    }
    wave_lds_sync();
    dbl4 xo[TN], ho[TN];
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      xo[t] = dbl4{0.0, 0.0, 0.0, 0.0};
      ho[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int st = 0; st < KMAX; ++st)
      if (st < KS)
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          const double cb = Cs[min(KS * kr + st, kNS - 1)][16 * t + kc];
          xo[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[st], cb, xo[t], 0, 0, 0);
          ho[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ah[st], cb, ho[t], 0, 0, 0);
        }
    // tile 0 holds the X columns (j < b) and, for b < 16, P columns; later
    // tiles hold P columns only (P = S Cp: column j - b of the third block)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = rb + 4 * v + kr;
      if (i >= r1 || kc >= nb2) continue;
      double *s = g.S + i * ld;
      double *h = g.HS + i * ld;
      const double x = xo[0][v], hx = ho[0][v];
      if (kc < b) {
        const double res = hx - lam[kc] * x;
        double w = res;   // no diagonal: the block preconditioner follows
        if (g.diag) {
          double den = g.diag[i] - lam[kc];
          if (fabs(den) < 1e-2) den = den < 0 ? -1e-2 : 1e-2;
          w = res / den;
        }
        if (g.locked[kc]) w = 0.0;   // soft locking
        s[kc] = x;
        s[b + kc] = w;
        h[kc] = hx;
        if (g.w32) g.w32[i * b + kc] = (float)w;
        rs += res * res;
        xs += x * x;
      } else {
        s[b + kc] = x;
        h[b + kc] = hx;
      }
    }
#pragma unroll
    for (int t = 1; t < TN; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = rb + 4 * v + kr;
        const int j = 16 * t + kc;
        if (i >= r1 || j >= nb2) continue;
        g.S[i * ld + b + j] = xo[t][v];
        g.HS[i * ld + b + j] = ho[t][v];
      }
  }
  // column kc: lanes kc, kc + 16, kc + 32, kc + 48 of each wave, then waves
  red[0][wv][lane] = rs;
  red[1][wv][lane] = xs;
  __syncthreads();
  if (threadIdx.x < 2 * b) {
    const int cc = threadIdx.x % b, which = threadIdx.x / b;
    double t = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 4; ++q) t += red[which][w][16 * q + cc];
    g.npart[(int64_t)blk * 2 * b + threadIdx.x] = t;
  }
}

template <int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_update(UpdArgs g) {
  if (g.stop && *g.stop) return;
  update_block<TN>(g, blockIdx.x);
}

template <int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_update_group(
    const UpdArgs *__restrict__ as, const int32_t *__restrict__ off, int njobs) {
  const int j = group_job(off, njobs, (int)blockIdx.x);
  const UpdArgs g = as[j];
  update_block<TN>(g, blockIdx.x - off[j]);
}

// Relative residual norms and the count of converged leading pairs.
__device__ __forceinline__ void finish_body(int b, int nev, int nparts, const double *npart, const double *lam,
                                            double tol, double *status, int32_t *locked, int iter = 0,
                                            int32_t *stop = nullptr) {
  // 16 slices of the partial sums per column, then a fixed-order sum
  __shared__ double ra[16][kMaxBlock], rx[16][kMaxBlock];
  __shared__ double rs[kMaxBlock];
  const int c = threadIdx.x & 15, sl = threadIdx.x >> 4;
  double a = 0.0, x = 0.0;
  if (c < b)
    for (int q = sl; q < nparts; q += 16) {
      a += npart[(int64_t)q * 2 * b + c];
      x += npart[(int64_t)q * 2 * b + b + c];
    }
  ra[sl][c] = a;
  rx[sl][c] = x;
  __syncthreads();
  if (threadIdx.x < b) {
    double sa = 0.0, sx = 0.0;
    for (int q = 0; q < 16; ++q) { sa += ra[q][c]; sx += rx[q][c]; }
    rs[c] = sqrt(sa) / (fmax(fabs(lam[c]), 1.0) * sqrt(fmax(sx, 1e-300)));
    locked[c] = rs[c] <= tol;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int conv = 0;
    for (int k = 0; k < nev; ++k) conv += rs[k] <= tol;
    status[0] = conv;
    for (int k = 0; k < b; ++k) { status[1 + k] = rs[k]; status[1 + kMaxBlock + k] = lam[k]; }
    status[kStatusIter] = iter;
    if (stop && conv >= nev) *stop = 1;   // the iterations queued after this one do nothing
  }
}

__global__ __launch_bounds__(256) void k_finish(int b, int nev, int nparts, const double *npart,
                                                const double *lam, double tol, double *status,
                                                int32_t *locked, int iter, int32_t *stop) {
  if (*stop) return;
  finish_body(b, nev, nparts, npart, lam, tol, status, locked, iter, stop);
}

__global__ __launch_bounds__(256) void k_finish_group(const FinishArgs *__restrict__ as) {
  const FinishArgs a = as[blockIdx.x];
  finish_body(a.b, a.nev, a.nparts, a.npart, a.lam, a.tol, a.status, a.locked);
}

// ------------------------------------------------------------ host driver
static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// rows per Gram block: about 512 blocks, a multiple of the staging chunk
constexpr int kSumGroup = 32;  // partial Gram matrices added per thread in the first pass
// iterations a single solve queues before it waits for the status (at most
// kIterBatch - 1 of them, each a few microseconds of launches that return at
// once, follow the converged one; waiting after every iteration cost ~31 us)
constexpr int kIterBatch = 8;

// rows per Gram workgroup: about three workgroups per CU (three waves per
// SIMD), a multiple of the 16 rows the four waves take per round
static int64_t gram_rows_for(int64_t D) {
  int64_t r = std::max<int64_t>((D + 767) / 768, 16);
  return (r + 15) / 16 * 16;
}

// rows per update workgroup
// rows per update workgroup: 64 to 256, about a thousand workgroups (each
// loads [Cx Cp] once; at D = 198,912, 256 rows measured 77 us against 83 us
// with 64)
static int64_t upd_rows_for(int64_t D) {
  return std::min<int64_t>(256, std::max<int64_t>(64, ((D + 1023) / 1024 + 63) / 64 * 64));
}

struct LobpcgRun {
  cib_ctx *ctx;
  const cib_matrix &H;
  hipStream_t s;
  int64_t D;
  int b, nev, ld, gram_blocks, upd_blocks, max_iter;
  int64_t gram_rows, upd_rows;
  double tol;
  cib_lobpcg_opts opts;
  DBuf<double> S, HS, diag, partial, partial2, gram, C, lam, npart, npart2, status, hlow;
  DBuf<float> x32, y32;
  DBuf<int64_t> idx, seli;
  DBuf<double> selv;
  int64_t sel_half = 0;
  DBuf<int32_t> flag, locked, stop;
  int iters = 0;
  double t_spmm = 0.0;
  int64_t n_spmm = 0;
  bool timing = false;
  hipEvent_t ev0[kIterBatch] = {}, ev1[kIterBatch] = {};   // SpMM of each iteration of a batch

  LobpcgRun(cib_ctx *c, const cib_matrix &h, const cib_lobpcg_opts &o, hipStream_t st, bool time_spmm)
      : ctx(c), H(h), s(st), D(h.D), b(o.block), nev(o.nev), max_iter(o.max_iter), opts(o),
        timing(time_spmm) {
    CIB_REQUIRE(nev >= 1 && nev <= b && b <= kMaxBlock, CIB_E_INVALID, "need 1 <= nev <= block <= 16");
    CIB_REQUIRE(3 * (int64_t)b <= H.D, CIB_E_INVALID, "need 3 * block <= D");
    CIB_REQUIRE(o.max_iter >= 1, CIB_E_INVALID, "max_iter must be >= 1");
    tol = o.tol > 0 ? o.tol : (H.dtype == CIB_F64 ? 1e-9 : 1e-5);
    ld = 3 * b;
    S.reset(ctx, (size_t)D * ld + kGramPad);
    HS.reset(ctx, (size_t)D * ld + kGramPad);
    diag.reset(ctx, D);
    gram_rows = gram_rows_for(D);
    gram_blocks = (int)((D + gram_rows - 1) / gram_rows);
    upd_rows = upd_rows_for(D);
    upd_blocks = (int)((D + upd_rows - 1) / upd_rows);
    partial.reset(ctx, (size_t)gram_blocks * gram_tiles(kNS));
    partial2.reset(ctx, (size_t)((gram_blocks + kSumGroup - 1) / kSumGroup) * gram_tiles(kNS));
    gram.reset(ctx, (size_t)2 * kNS * kLd);
    hlow.reset(ctx, 1);
    C.reset(ctx, kNS * 2 * kMaxBlock);
    lam.reset(ctx, kMaxBlock);
    npart.reset(ctx, (size_t)upd_blocks * 2 * kMaxBlock);
    npart2.reset(ctx, (size_t)((upd_blocks + kSumGroup - 1) / kSumGroup) * 2 * kMaxBlock);
    status.reset(ctx, kStatusLen);
    idx.reset(ctx, kMaxBlock);
    sel_half = std::max<int64_t>(1, (D + kSelChunk - 1) / kSelChunk) * b;
    seli.reset(ctx, 2 * sel_half);
    selv.reset(ctx, 2 * sel_half + kMaxBlock);
    flag.reset(ctx, 4);
    locked.reset(ctx, kMaxBlock);
    stop.reset(ctx, 1);
    if (H.dtype == CIB_F32) {
      x32.reset(ctx, (size_t)D * b);
      y32.reset(ctx, (size_t)D * b);
    }
    if (timing)
      for (int k = 0; k < kIterBatch; ++k) {
        // timing only: no system-scope fence at every record
        CIB_HIP(hipEventCreateWithFlags(&ev0[k], hipEventDisableSystemFence));
        CIB_HIP(hipEventCreateWithFlags(&ev1[k], hipEventDisableSystemFence));
      }
  }
  ~LobpcgRun() {
    for (int k = 0; k < kIterBatch; ++k) {
      if (ev0[k]) (void)hipEventDestroy(ev0[k]);
      if (ev1[k]) (void)hipEventDestroy(ev1[k]);
    }
  }

  // HS[:, slot] = H S[:, slot]; ev = the batch position of the iteration
  void spmm(int slot, bool w32_ready, int ev = 0) {
    if (timing) CIB_HIP(hipEventRecord(ev0[ev], s));
    if (H.dtype == CIB_F64) {
      spmm_sym(H, S.p + slot * b, ld, HS.p + slot * b, ld, b, s, stop.p);
    } else {
      if (!w32_ready)
        hipLaunchKernelGGL(k_narrow, dim3(nblk(D * b)), dim3(256), 0, s, D, b, S.p + slot * b, ld, x32.p);
      // H W in float32, rows stored widened into HS (or through y32 and a
      // widening pass where the vector kernel does not apply)
      if (!spmm_sym_widen(H, x32.p, b, HS.p + slot * b, ld, b, s, stop.p)) {
        spmm_sym(H, x32.p, b, y32.p, b, b, s, stop.p);
        hipLaunchKernelGGL(k_widen, dim3(nblk(D * b)), dim3(256), 0, s, D, b, y32.p, HS.p + slot * b, ld, stop.p);
      }
    }
    if (timing) CIB_HIP(hipEventRecord(ev1[ev], s));
  }

  void rr_update(int ns) {
    gram_step(ns);
    RRArgs ra = rr_args(ns);
    ra.stop = stop.p;
    { KTimer kt(ctx, K_RR, s); hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(256), 0, s, ra); }
    update_step(ns);
  }

  RRArgs rr_args(int ns) const {
    return RRArgs{ns, b, gram.p, C.p, lam.p, flag.p, H.dtype == CIB_F64 ? 1e-10 : 1e-7, hlow.p};
  }

  void gram_step(int ns) {
    {
      KTimer kt(ctx, K_GRAM, s);
      const int T = (ns + 15) / 16;
      if (T == 1)
        hipLaunchKernelGGL(k_gram<1>, dim3(gram_blocks), dim3(256), 0, s, D, ns, ld, S.p, HS.p, gram_rows, partial.p,
                           stop.p);
      else if (T == 2)
        hipLaunchKernelGGL(k_gram<2>, dim3(gram_blocks), dim3(256), 0, s, D, ns, ld, S.p, HS.p, gram_rows, partial.p,
                           stop.p);
      else
        hipLaunchKernelGGL(k_gram<3>, dim3(gram_blocks), dim3(256), 0, s, D, ns, ld, S.p, HS.p, gram_rows, partial.p,
                           stop.p);
      const int nout = gram_tiles(ns);
      const int groups = (gram_blocks + kSumGroup - 1) / kSumGroup;
      hipLaunchKernelGGL(k_sum_parts, dim3((nout + 255) / 256, groups), dim3(256), 0, s, nout, gram_blocks,
                         kSumGroup, partial.p, partial2.p, 0, stop.p);
      hipLaunchKernelGGL(k_sum_parts, dim3((nout + 255) / 256, 1), dim3(256), 0, s, nout, groups, groups,
                         partial2.p, gram.p, ns, stop.p);
    }
  }

  void update_step(int ns) {
    const cib_precond *P = opts.precond;
    float *w32 = H.dtype == CIB_F32 ? x32.p : nullptr;
    UpdArgs ua{D, b, ns, ld, S.p, HS.p, C.p, lam.p, P ? nullptr : diag.p, P ? nullptr : w32,
               npart.p, (int)upd_rows, locked.p, stop.p};
    {
      KTimer kt(ctx, K_UPDATE, s);
      if (2 * b <= 16) hipLaunchKernelGGL(k_update<1>, dim3(upd_blocks), dim3(256), 0, s, ua);
      else hipLaunchKernelGGL(k_update<2>, dim3(upd_blocks), dim3(256), 0, s, ua);
    }
    // block preconditioner: W (the residuals, zero where locked) in place
    if (P) precond_apply(*P, lam.p, b, S.p + b, ld, S.p + b, ld, w32, b, s);
    // per-block residual sums: groups of kSumGroup first, then k_finish
    const int ugroups = (upd_blocks + kSumGroup - 1) / kSumGroup;
    hipLaunchKernelGGL(k_sum_parts, dim3(1, ugroups), dim3(256), 0, s, 2 * b, upd_blocks, kSumGroup, npart.p,
                       npart2.p, 0, stop.p);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, b, nev, ugroups, npart2.p, lam.p, tol, status.p, locked.p,
                       iters, stop.p);
    CIB_HIP(hipGetLastError());
  }

  // idx[0..b) = indices of the b smallest diagonal entries (ties: lower index)
  void select_smallest() {
    int64_t n = D;
    const double *v = diag.p;
    const int64_t *id = nullptr;
    int pass = 0;
    for (;;) {
      const int64_t nb = (n + kSelChunk - 1) / kSelChunk;
      double *ov = nb == 1 ? selv.p + 2 * sel_half : selv.p + (pass & 1 ? 0 : sel_half);
      int64_t *oi = nb == 1 ? idx.p : seli.p + (pass & 1 ? 0 : sel_half);
      hipLaunchKernelGGL(k_select_pass, dim3((unsigned)nb), dim3(256), 0, s, n, v, id, b, ov, oi);
      CIB_HIP(hipGetLastError());
      if (nb == 1) break;
      n = nb * b;
      v = ov;
      id = oi;
      ++pass;
    }
  }

  // diagonal, spectrum bound, X0 and the Rayleigh-Ritz step on X0 alone
  void start() {
    CIB_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t) * 4, s));
    CIB_HIP(hipMemsetAsync(locked.p, 0, sizeof(int32_t) * kMaxBlock, s));
    CIB_HIP(hipMemsetAsync(stop.p, 0, sizeof(int32_t), s));
    const unsigned rb = (unsigned)((D + 3) / 4);
    if (H.dtype == CIB_F64) {
      hipLaunchKernelGGL(k_diag<double>, dim3(nblk(D)), dim3(256), 0, s, D, H.row_ptr.p, H.val64.p, diag.p);
      hipLaunchKernelGGL(k_gersh_rows<double>, dim3(rb), dim3(256), 0, s, D, H.row_ptr.p, H.val64.p,
                         H.lo_ptr.p, H.lo_val64.p, HS.p);
    } else {
      hipLaunchKernelGGL(k_diag<float>, dim3(nblk(D)), dim3(256), 0, s, D, H.row_ptr.p, H.val32.p, diag.p);
      hipLaunchKernelGGL(k_gersh_rows<float>, dim3(rb), dim3(256), 0, s, D, H.row_ptr.p, H.val32.p,
                         H.lo_ptr.p, H.lo_val32.p, HS.p);
    }
    hipLaunchKernelGGL(k_min, dim3(1), dim3(1024), 0, s, D, HS.p, hlow.p);   // HS is scratch here
    if (opts.x0) {
      hipLaunchKernelGGL(k_copy_x0, dim3(nblk(D * b)), dim3(256), 0, s, D, b, ld, opts.x0, S.p);
    } else {
      select_smallest();
      hipLaunchKernelGGL(k_init_x, dim3(nblk(D * b)), dim3(256), 0, s, D, b, ld, idx.p, opts.seed, S.p);
    }
    CIB_HIP(hipGetLastError());
    spmm(0, false);
    rr_update(b);
  }

  // ev: the iteration's position in a batch (its SpMM timer events)
  void iterate(int ev = 0) {
    ++iters;
    spmm(1, H.dtype == CIB_F32, ev);
    rr_update(iters == 1 ? 2 * b : 3 * b);
  }

  // One iteration as the arguments of each stage, for a caller that runs
  // the same stage of several solves as one launch (the launch parameters
  // are those of iterate(), so the results are the same bits).  False (and
  // nothing advanced) when the SpMM does not take the vector kernel.
  bool plan_iteration(IterPlan &p) {
    const bool f32 = H.dtype == CIB_F32;
    const void *X = f32 ? (const void *)x32.p : (const void *)(S.p + b);
    void *Y = f32 ? (void *)y32.p : (void *)(HS.p + b);
    const int64_t ldx = f32 ? b : ld;
    if (!spmm_vec_args(H, X, ldx, Y, ldx, b, p.spmm, p.spmm_blocks)) return false;
    ++iters;
    const int ns = iters == 1 ? 2 * b : 3 * b;
    step_ns = ns;
    p.dt = H.dtype;
    p.nvec = b;
    p.widen = f32;
    p.wid = WidenArgs{D, b, y32.p, HS.p + b, ld};
    p.widen_blocks = (int)nblk(D * b);
    p.T = (ns + 15) / 16;
    p.gram = GramArgs{D, ns, ld, S.p, HS.p, gram_rows, partial.p};
    p.gram_blocks = gram_blocks;
    const int nout = gram_tiles(ns), xb = (nout + 255) / 256;
    const int groups = (gram_blocks + kSumGroup - 1) / kSumGroup;
    p.gs1 = SumArgs{nout, gram_blocks, kSumGroup, partial.p, partial2.p, 0};
    p.gs1_blocks = xb * groups;
    p.gs2 = SumArgs{nout, groups, groups, partial2.p, gram.p, ns};
    p.gs2_blocks = xb;
    p.rr = rr_args(ns);
    p.TN = 2 * b <= 16 ? 1 : 2;
    p.upd = UpdArgs{D, b, ns, ld, S.p, HS.p, C.p, lam.p, diag.p, f32 ? x32.p : nullptr, npart.p, (int)upd_rows,
                    locked.p};
    p.upd_blocks = upd_blocks;
    const int ugroups = (upd_blocks + kSumGroup - 1) / kSumGroup;
    p.us = SumArgs{2 * b, upd_blocks, kSumGroup, npart.p, npart2.p, 0};
    p.us_blocks = ugroups;   // 2b <= 32 outputs: one element block per group
    p.fin = FinishArgs{b, nev, ugroups, npart2.p, lam.p, tol, status.p, nullptr};
    p.fin.locked = locked.p;
    p.status = status.p;
    return true;
  }

  int step_ns = 0;

  void copy_status(double *host) {
    CIB_HIP(hipMemcpyAsync(host, status.p, sizeof(double) * kStatusLen, hipMemcpyDeviceToHost, s));
  }

  // the SpMMs of the first n iterations of the batch just waited for
  void spmm_time_accumulate(int n) {
    n_spmm += n;
    if (!timing) return;
    for (int k = 0; k < n; ++k) {
      float ms = 0.f;
      CIB_HIP(hipEventElapsedTime(&ms, ev0[k], ev1[k]));
      t_spmm += ms * 1e-3;
    }
  }

  void copy_vectors(double *evecs, int64_t ld_evecs) {
    hipLaunchKernelGGL(k_copy_cols, dim3(nblk(D * nev)), dim3(256), 0, s, D, nev, S.p, ld, evecs, ld_evecs);
    CIB_HIP(hipGetLastError());
  }
};

// The device bytes of a LobpcgRun (its constructor's allocations, each as
// the context allocator rounds it).
size_t lobpcg_bytes(int64_t D, int b, cib_dtype dt) {
  const int64_t gram_rows = gram_rows_for(D);
  const int64_t gram_blocks = (D + gram_rows - 1) / gram_rows;
  const int64_t upd_rows = upd_rows_for(D);
  const int64_t upd_blocks = (D + upd_rows - 1) / upd_rows;
  const int64_t groups = (gram_blocks + kSumGroup - 1) / kSumGroup;
  const int64_t ugroups = (upd_blocks + kSumGroup - 1) / kSumGroup;
  const int64_t sel_half = std::max<int64_t>(1, (D + kSelChunk - 1) / kSelChunk) * b;
  auto d8 = [](int64_t n) { return dev_bytes((size_t)n * 8); };
  auto d4 = [](int64_t n) { return dev_bytes((size_t)n * 4); };
  size_t n = 2 * d8(D * 3 * b + kGramPad) + d8(D) + d8(gram_blocks * gram_tiles(kNS)) +
             d8(groups * gram_tiles(kNS)) + d8(2 * kNS * kLd) + d8(1) + d8(kNS * 2 * kMaxBlock) + d8(kMaxBlock) +
             d8(upd_blocks * 2 * kMaxBlock) + d8(ugroups * 2 * kMaxBlock) + d8(kStatusLen) + d8(kMaxBlock) +
             d8(2 * sel_half) + d8(2 * sel_half + kMaxBlock) + d4(4) + d4(kMaxBlock) + d4(1);
  if (dt == CIB_F32) n += 2 * d4(D * b);
  return n;
}

LobpcgRun *lobpcg_create(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, hipStream_t s) {
  return new LobpcgRun(ctx, H, o, s, false);
}
void lobpcg_start(LobpcgRun *r) { r->start(); }
bool lobpcg_plan_iteration(LobpcgRun *r, IterPlan &p) { return r->plan_iteration(p); }

// ------------------------------------------------------------ grouped iterations
// The stage arrays of one group (same dtype, block size and tile counts) and
// each stage's workgroup offsets, packed into one staging buffer.
namespace {
template <typename A>
size_t put(char *base, size_t &at, const A *src, size_t n) {
  at = (at + 255) / 256 * 256;
  const size_t o = at;
  if (base) std::memcpy(base + o, src, sizeof(A) * n);
  at += sizeof(A) * n;
  return o;
}
}  // namespace

GroupRunner::~GroupRunner() {
  if (host) (void)hipHostFree(host);
}

void GroupRunner::run(const std::vector<LobpcgRun *> &runs, const std::vector<IterPlan> &plans, hipStream_t s) {
  const int n = (int)runs.size();
  if (n == 0) return;
  // groups by kernel variant, in job order
  std::vector<std::vector<int>> groups;
  auto key = [&](const IterPlan &p) { return ((int)p.dt << 16) | (p.nvec << 8) | (p.T << 4) | p.TN; };
  for (int j = 0; j < n; ++j) {
    bool placed = false;
    for (auto &g : groups)
      if (key(plans[g[0]]) == key(plans[j])) { g.push_back(j); placed = true; break; }
    if (!placed) groups.push_back({j});
  }
  struct Layout {
    size_t spmm, ospmm, wid, owid, gram, ogram, gs1, ogs1, gs2, ogs2, rr, upd, oupd, us, ous, fin;
    int tspmm, twid, tgram, tgs1, tgs2, tupd, tus;
  };
  std::vector<Layout> lay(groups.size());
  // two passes: sizes, then the copy into the (grown) staging buffer
  for (int pass = 0; pass < 2; ++pass) {
    char *base = pass ? host : nullptr;
    size_t at = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const auto &g = groups[gi];
      const int m = (int)g.size();
      std::vector<VecArgs> a_sp(m);
      std::vector<WidenArgs> a_w(m);
      std::vector<GramArgs> a_g(m);
      std::vector<SumArgs> a_s1(m), a_s2(m), a_us(m);
      std::vector<RRArgs> a_rr(m);
      std::vector<UpdArgs> a_u(m);
      std::vector<FinishArgs> a_f(m);
      std::vector<int32_t> o_sp(m + 1, 0), o_w(m + 1, 0), o_g(m + 1, 0), o_s1(m + 1, 0), o_s2(m + 1, 0),
          o_u(m + 1, 0), o_us(m + 1, 0);
      for (int q = 0; q < m; ++q) {
        const IterPlan &p = plans[g[q]];
        a_sp[q] = p.spmm; a_w[q] = p.wid; a_g[q] = p.gram; a_s1[q] = p.gs1; a_s2[q] = p.gs2;
        a_rr[q] = p.rr; a_u[q] = p.upd; a_us[q] = p.us; a_f[q] = p.fin;
        o_sp[q + 1] = o_sp[q] + p.spmm_blocks;
        o_w[q + 1] = o_w[q] + p.widen_blocks;
        o_g[q + 1] = o_g[q] + p.gram_blocks;
        o_s1[q + 1] = o_s1[q] + p.gs1_blocks;
        o_s2[q + 1] = o_s2[q] + p.gs2_blocks;
        o_u[q + 1] = o_u[q] + p.upd_blocks;
        o_us[q + 1] = o_us[q] + p.us_blocks;
      }
      Layout &L = lay[gi];
      L.spmm = put(base, at, a_sp.data(), m); L.ospmm = put(base, at, o_sp.data(), m + 1);
      L.wid = put(base, at, a_w.data(), m); L.owid = put(base, at, o_w.data(), m + 1);
      L.gram = put(base, at, a_g.data(), m); L.ogram = put(base, at, o_g.data(), m + 1);
      L.gs1 = put(base, at, a_s1.data(), m); L.ogs1 = put(base, at, o_s1.data(), m + 1);
      L.gs2 = put(base, at, a_s2.data(), m); L.ogs2 = put(base, at, o_s2.data(), m + 1);
      L.rr = put(base, at, a_rr.data(), m);
      L.upd = put(base, at, a_u.data(), m); L.oupd = put(base, at, o_u.data(), m + 1);
      L.us = put(base, at, a_us.data(), m); L.ous = put(base, at, o_us.data(), m + 1);
      L.fin = put(base, at, a_f.data(), m);
      L.tspmm = o_sp[m]; L.twid = o_w[m]; L.tgram = o_g[m]; L.tgs1 = o_s1[m]; L.tgs2 = o_s2[m];
      L.tupd = o_u[m]; L.tus = o_us[m];
    }
    if (pass == 0 && at > cap) {
      if (host) (void)hipHostFree(host);
      host = nullptr;
      CIB_HIP(hipHostMalloc((void **)&host, at, hipHostMallocDefault));
      dev.reset(ctx, at);
      cap = at;
    }
    if (pass == 1) CIB_HIP(hipMemcpyAsync(dev.p, host, at, hipMemcpyHostToDevice, s));
  }
  const char *d = dev.p;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Layout &L = lay[gi];
    const int m = (int)groups[gi].size();
    const IterPlan &p0 = plans[groups[gi][0]];
    auto off = [&](size_t o) { return reinterpret_cast<const int32_t *>(d + o); };
    launch_spmm_group(p0.dt, p0.nvec, reinterpret_cast<const VecArgs *>(d + L.spmm), off(L.ospmm), m, L.tspmm, s);
    if (p0.widen)
      hipLaunchKernelGGL(k_widen_group, dim3(L.twid), dim3(256), 0, s, reinterpret_cast<const WidenArgs *>(d + L.wid),
                         off(L.owid), m);
    const GramArgs *ga = reinterpret_cast<const GramArgs *>(d + L.gram);
    if (p0.T == 1) hipLaunchKernelGGL(k_gram_group<1>, dim3(L.tgram), dim3(256), 0, s, ga, off(L.ogram), m);
    else if (p0.T == 2) hipLaunchKernelGGL(k_gram_group<2>, dim3(L.tgram), dim3(256), 0, s, ga, off(L.ogram), m);
    else hipLaunchKernelGGL(k_gram_group<3>, dim3(L.tgram), dim3(256), 0, s, ga, off(L.ogram), m);
    hipLaunchKernelGGL(k_sum_parts_group, dim3(L.tgs1), dim3(256), 0, s, reinterpret_cast<const SumArgs *>(d + L.gs1),
                       off(L.ogs1), m);
    hipLaunchKernelGGL(k_sum_parts_group, dim3(L.tgs2), dim3(256), 0, s, reinterpret_cast<const SumArgs *>(d + L.gs2),
                       off(L.ogs2), m);
    hipLaunchKernelGGL(k_rayleigh_ritz_group, dim3(m), dim3(256), 0, s, reinterpret_cast<const RRArgs *>(d + L.rr));
    const UpdArgs *ua = reinterpret_cast<const UpdArgs *>(d + L.upd);
    if (p0.TN == 1) hipLaunchKernelGGL(k_update_group<1>, dim3(L.tupd), dim3(256), 0, s, ua, off(L.oupd), m);
    else hipLaunchKernelGGL(k_update_group<2>, dim3(L.tupd), dim3(256), 0, s, ua, off(L.oupd), m);
    hipLaunchKernelGGL(k_sum_parts_group, dim3(L.tus), dim3(256), 0, s, reinterpret_cast<const SumArgs *>(d + L.us),
                       off(L.ous), m);
    hipLaunchKernelGGL(k_finish_group, dim3(m), dim3(256), 0, s, reinterpret_cast<const FinishArgs *>(d + L.fin));
    CIB_HIP(hipGetLastError());
  }
}

void lobpcg_iterate(LobpcgRun *r) { r->iterate(); }
void lobpcg_copy_status(LobpcgRun *r, double *host) { r->copy_status(host); }
int lobpcg_iters(const LobpcgRun *r) { return r->iters; }
void lobpcg_destroy(LobpcgRun *r) { delete r; }

cib_status lobpcg_solve(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, double *evals,
                        double *evecs, int64_t ld_evecs, cib_lobpcg_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  CIB_REQUIRE(!evecs || ld_evecs >= o.nev, CIB_E_INVALID, "ld_evecs < nev");
  CIB_REQUIRE(!o.precond || (o.precond->ctx == ctx && o.precond->D == H.D), CIB_E_INVALID,
              "preconditioner was not made for this matrix's basis and context");
  UnwindFence fence(ctx->stream);
  LobpcgRun L(ctx, H, o, ctx->stream, true);
  double *st = static_cast<double *>(ctx->pinned_buf(sizeof(double) * kStatusLen));
  L.start();
  L.copy_status(st);
  CIB_HIP(hipStreamSynchronize(L.s));
  L.spmm_time_accumulate(1);
  auto finite = [&] {
    for (int k = 0; k < L.b; ++k)
      if (!std::isfinite(st[1 + k]) || !std::isfinite(st[1 + kMaxBlock + k])) return false;
    return true;
  };
  int conv = (int)st[0];
  CIB_REQUIRE(finite(), CIB_E_DEVICE, "LOBPCG produced non-finite Ritz values");
  // Iterations are queued in batches without waiting for each one's status:
  // the iteration that converges sets the stop flag on the device, and every
  // launch of the iterations queued after it returns at once (their timer
  // marks are dropped, their SpMMs not counted).  The results are those of a
  // solve that waited after every iteration.  The block preconditioner's
  // kernels do not look at the flag, so with it every iteration is waited for.
  const int batch = o.precond ? 1 : kIterBatch;
  while (conv < L.nev && L.iters < L.max_iter) {
    const int first = L.iters + 1;
    const int nq = std::min(batch, L.max_iter - L.iters);
    size_t marks[kIterBatch];
    for (int k = 0; k < nq; ++k) {
      marks[k] = profile_marks(ctx);
      L.iterate(k);
    }
    L.copy_status(st);
    CIB_HIP(hipStreamSynchronize(L.s));
    const int last = (int)st[kStatusIter];   // the last iteration that ran
    const int ran = last - first + 1;
    CIB_REQUIRE(ran >= 1 && ran <= nq, CIB_E_DEVICE, "LOBPCG status does not match the queued iterations");
    if (ran < nq) profile_drop_marks(ctx, marks[ran]);
    L.iters = last;
    L.spmm_time_accumulate(ran);
    conv = (int)st[0];
    CIB_REQUIRE(finite(), CIB_E_DEVICE, "LOBPCG produced non-finite Ritz values");
  }
  for (int k = 0; k < L.nev; ++k) evals[k] = st[1 + kMaxBlock + k];
  if (evecs) L.copy_vectors(evecs, ld_evecs);
  CIB_HIP(hipStreamSynchronize(L.s));
  if (info) {
    info->iters = L.iters;
    info->n_converged = conv;
    for (int k = 0; k < 64; ++k) info->resid[k] = k < L.b ? st[1 + k] : 0.0;
    info->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_spmm_s = L.t_spmm;
    info->n_spmm = L.n_spmm;
  }
  return conv >= L.nev ? CIB_OK : CIB_E_NOT_CONVERGED;
}

}  // namespace cib
