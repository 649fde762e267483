// Block LOBPCG for the lowest eigenpairs of the half-stored H (Fig. 1 step 15
// of the paper: "lowest n eigenvalues ... using LOBPCG").
//
// Search space S = [X | W | P] (b columns each), kept row-interleaved: row i
// of S holds X_i, W_i, P_i contiguously (3b float64), and HS = H S likewise.
// Per iteration: W <- H W (SpMM in the matrix dtype), partial Gram matrices
// S^T S and S^T HS over row chunks, one workgroup that reduces them and does
// the Rayleigh-Ritz step in float64 (scaled Cholesky of S^T S with dropping
// of dependent directions, reduced matrix, parallel cyclic Jacobi), then a
// row-parallel update X, P, HX, HP <- S C, HS C, the residual R = HX - X L,
// its norms and the preconditioned W = R / (diag(H) - lambda).
#include <algorithm>
#include <chrono>
#include <cmath>

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
__global__ __launch_bounds__(1024) void k_select_smallest(int64_t D, const double *diag, int b,
                                                          int64_t *idx) {
  __shared__ double sv[1024 / kWave];
  __shared__ int64_t si[1024 / kWave];
  __shared__ int64_t chosen[kMaxBlock];
  for (int r = 0; r < b; ++r) {
    double best = INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= chosen[q] == i;
      const double v = diag[i];
      if (!taken && (v < best || (v == best && i < bi))) { best = v; bi = i; }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const double ov = __shfl_xor(best, d, kWave);
      const int64_t oi = __shfl_xor(bi, d, kWave);
      if (ov < best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane_id() == 0) { sv[threadIdx.x >> 6] = best; si[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = sv[0];
      int64_t bx = si[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (sv[w] < bv || (sv[w] == bv && si[w] < bx)) { bv = sv[w]; bx = si[w]; }
      chosen[r] = bx;
      idx[r] = bx;
    }
    __syncthreads();
  }
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
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
__global__ __launch_bounds__(256) void k_widen(int64_t D, int b, const float *in, double *out, int ldo) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * b) out[(k / b) * ldo + (k % b)] = (double)in[k];
}

__global__ __launch_bounds__(256) void k_copy_cols(int64_t D, int n, const double *S, int lds, double *out,
                                                   int64_t ldo) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < D * n) out[(k / n) * ldo + (k % n)] = S[(k / n) * lds + (k % n)];
}

// ------------------------------------------------------------ Gram matrices
// partial[blk] = sum over the block's rows of S_i^T [S_i, HS_i] for the first
// ns columns: an ns x 2ns matrix (left half S^T S, right half S^T HS).
constexpr int kGramRows = 32;

__global__ __launch_bounds__(256) void k_gram(int64_t D, int ns, int ld, const double *__restrict__ S,
                                              const double *__restrict__ HS, int64_t rows_per_blk,
                                              double *__restrict__ partial) {
  __shared__ double ts[kGramRows][kNS + 1];
  __shared__ double th[kGramRows][kNS + 1];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = min(D, r0 + rows_per_blk);
  const int nout = ns * 2 * ns;
  double acc[18];
#pragma unroll
  for (int q = 0; q < 18; ++q) acc[q] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kGramRows) {
    const int nr = (int)min<int64_t>(kGramRows, r1 - rb);
    for (int k = threadIdx.x; k < kGramRows * ns; k += blockDim.x) {
      const int r = k / ns, c = k % ns;
      const bool in = r < nr;
      ts[r][c] = in ? S[(rb + r) * ld + c] : 0.0;
      th[r][c] = in ? HS[(rb + r) * ld + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 18; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < nout) {
        const int i = e / (2 * ns), j = e % (2 * ns);
        double a = acc[q];
        if (j < ns) {
          for (int r = 0; r < kGramRows; ++r) a += ts[r][i] * ts[r][j];
        } else {
          for (int r = 0; r < kGramRows; ++r) a += ts[r][i] * th[r][j - ns];
        }
        acc[q] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < nout) partial[(int64_t)blockIdx.x * nout + e] = acc[q];
  }
}

// ------------------------------------------------------------ Rayleigh-Ritz
struct RRArgs {
  int ns, b, nparts;
  const double *partial;
  double *C;        // ns x 2b: [Cx | Cp]
  double *lam;      // b
  int32_t *flag;    // [0]: rank of the search space
  double drop_tol;
};

// Parallel cyclic Jacobi on the r x r symmetric matrix A (LDS, ld kLd);
// V receives the eigenvectors (columns).  Round-robin ordering: in each round
// the r/2 rotations touch disjoint index pairs, so each 2x2 block of A is
// transformed by one thread.
__device__ void jacobi_eig(double (*A)[kLd], double (*V)[kLd], int r, double *cs, int *pq,
                           double *red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = r + (r & 1);
  for (int k = tid; k < r * r; k += nt) V[k / r][k % r] = (k / r == k % r) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // off-diagonal and total Frobenius norms
    double off = 0.0, tot = 0.0;
    for (int k = tid; k < r * r; k += nt) {
      const double a = A[k / r][k % r];
      tot += a * a;
      if (k / r != k % r) off += a * a;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if (lane_id() == 0) { red[2 * (tid >> 6)] = off; red[2 * (tid >> 6) + 1] = tot; }
    __syncthreads();
    double so = 0.0, st = 0.0;
    for (int w = 0; w < nt / kWave; ++w) { so += red[2 * w]; st += red[2 * w + 1]; }
    __syncthreads();
    if (so <= 1e-32 * st || so == 0.0) break;
    for (int rd = 0; rd < m - 1; ++rd) {
      // pairs of this round
      for (int k = tid; k < m / 2; k += nt) {
        int p, q;
        if (k == 0) { p = 0; q = 1 + rd % (m - 1); }
        else {
          p = 1 + ((rd - k) % (m - 1) + (m - 1)) % (m - 1);
          q = 1 + (rd + k) % (m - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < r) {
          const double apq = A[p][q];
          if (apq != 0.0) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
      }
      __syncthreads();
      // A <- J^T A J, one 2x2 block (pair k1 rows, pair k2 columns) per item
      const int h = m / 2;
      for (int k = tid; k < h * h; k += nt) {
        const int k1 = k / h, k2 = k % h;
        const int p1 = pq[2 * k1], q1 = pq[2 * k1 + 1], p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
        if (q1 >= r || q2 >= r) {
          // a dummy index (odd r): rotate only the real one of each pair
          if (q1 >= r && q2 >= r) {
            // p1 and p2 are real, nothing rotates
          } else if (q1 >= r) {  // rows p1 only, columns (p2, q2)
            const double c2 = cs[2 * k2], s2 = cs[2 * k2 + 1];
            const double a = A[p1][p2], bq = A[p1][q2];
            A[p1][p2] = c2 * a - s2 * bq;
            A[p1][q2] = s2 * a + c2 * bq;
          } else {               // rows (p1, q1), column p2 only
            const double c1 = cs[2 * k1], s1 = cs[2 * k1 + 1];
            const double a = A[p1][p2], bq = A[q1][p2];
            A[p1][p2] = c1 * a - s1 * bq;
            A[q1][p2] = s1 * a + c1 * bq;
          }
          continue;
        }
        const double c1 = cs[2 * k1], s1 = cs[2 * k1 + 1], c2 = cs[2 * k2], s2 = cs[2 * k2 + 1];
        const double app = A[p1][p2], apq = A[p1][q2], aqp = A[q1][p2], aqq = A[q1][q2];
        // rows: new_p = c1 row_p - s1 row_q ; new_q = s1 row_p + c1 row_q
        const double bpp = c1 * app - s1 * aqp, bpq = c1 * apq - s1 * aqq;
        const double bqp = s1 * app + c1 * aqp, bqq = s1 * apq + c1 * aqq;
        // columns: new_p = c2 col_p - s2 col_q ; new_q = s2 col_p + c2 col_q
        A[p1][p2] = c2 * bpp - s2 * bpq;
        A[p1][q2] = s2 * bpp + c2 * bpq;
        A[q1][p2] = c2 * bqp - s2 * bqq;
        A[q1][q2] = s2 * bqp + c2 * bqq;
      }
      // V <- V J
      for (int k = tid; k < r * h; k += nt) {
        const int i = k / h, kk = k % h;
        const int p = pq[2 * kk], q = pq[2 * kk + 1];
        if (q >= r) continue;
        const double c = cs[2 * kk], s = cs[2 * kk + 1];
        const double vp = V[i][p], vq = V[i][q];
        V[i][p] = c * vp - s * vq;
        V[i][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_rayleigh_ritz(RRArgs g) {
  __shared__ double G[kNS][kLd], Hm[kNS][kLd], V[kNS][kLd];
  __shared__ double scale[kNS], cs[kNS], red[16], theta[kNS];
  __shared__ int keep[kNS], kidx[kNS], pq[kNS], order[kNS];
  __shared__ int rank_s;
  const int ns = g.ns, b = g.b, tid = threadIdx.x, nt = blockDim.x;
  const int nout = ns * 2 * ns;
  // 1. reduce the partial Gram matrices (fixed order: deterministic)
  for (int e = tid; e < nout; e += nt) {
    double s = 0.0;
    for (int q = 0; q < g.nparts; ++q) s += g.partial[(int64_t)q * nout + e];
    const int i = e / (2 * ns), j = e % (2 * ns);
    if (j < ns) G[i][j] = s; else Hm[i][j - ns] = s;
  }
  __syncthreads();
  // 2. symmetrise, scale to unit diagonal
  for (int i = tid; i < ns; i += nt) {
    const double d = G[i][i];
    scale[i] = d > 1e-300 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < ns * ns; e += nt) {
    const int i = e / ns, j = e % ns;
    if (i <= j) {
      const double si = scale[i] * scale[j];
      const double gv = 0.5 * (G[i][j] + G[j][i]) * si;
      const double hv = 0.5 * (Hm[i][j] + Hm[j][i]) * si;
      G[i][j] = gv; G[j][i] = gv;
      Hm[i][j] = hv; Hm[j][i] = hv;
    }
  }
  __syncthreads();
  // 3. right-looking Cholesky of G (lower, in place) with dropping of columns
  //    whose residual diagonal falls below drop_tol (dependent directions)
  for (int k = 0; k < ns; ++k) {
    if (tid == 0) {
      const double piv = G[k][k];
      keep[k] = (scale[k] > 0.0 && piv > g.drop_tol) ? 1 : 0;
      G[k][k] = keep[k] ? sqrt(piv) : 0.0;
    }
    __syncthreads();
    const double lkk = G[k][k];
    for (int i = k + 1 + tid; i < ns; i += nt) G[i][k] = keep[k] ? G[i][k] / lkk : 0.0;
    __syncthreads();
    if (keep[k]) {
      const int m = ns - k - 1;
      for (int e = tid; e < m * m; e += nt) {
        const int i = k + 1 + e / m, j = k + 1 + e % m;
        if (j <= i) G[i][j] -= G[i][k] * G[j][k];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    int r = 0;
    for (int k = 0; k < ns; ++k) if (keep[k]) kidx[r++] = k;
    rank_s = r;
  }
  __syncthreads();
  const int r = rank_s;
  // 4. reduced matrix M = L^-1 Hm L^-T over the kept indices.
  //    Z = L^-1 Hm: thread j solves for column j into V (forward substitution).
  for (int j = tid; j < r; j += nt) {
    const int cj = kidx[j];
    for (int a = 0; a < r; ++a) {
      const int ka = kidx[a];
      double s = Hm[ka][cj];
      for (int q = 0; q < a; ++q) s -= G[ka][kidx[q]] * V[q][j];
      V[a][j] = s / G[ka][ka];
    }
  }
  __syncthreads();
  //    M = L^-1 Z^T: column j has right-hand side row j of Z; written into Hm
  //    (no longer needed) in compressed indices.
  for (int j = tid; j < r; j += nt) {
    for (int a = 0; a < r; ++a) {
      const int ka = kidx[a];
      double s = V[j][a];
      for (int q = 0; q < a; ++q) s -= G[ka][kidx[q]] * Hm[q][j];
      Hm[a][j] = s / G[ka][ka];
    }
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int i = e / r, j = e % r;
    if (i < j) {
      const double v = 0.5 * (Hm[i][j] + Hm[j][i]);
      Hm[i][j] = v;
      Hm[j][i] = v;
    }
  }
  __syncthreads();
  // 5. eigen-decomposition of M
  jacobi_eig(Hm, V, r, cs, pq, red);
  __syncthreads();
  // 6. ascending order of the Ritz values
  for (int a = tid; a < r; a += nt) theta[a] = Hm[a][a];
  __syncthreads();
  if (tid == 0) {
    for (int a = 0; a < r; ++a) order[a] = a;
    for (int a = 1; a < r; ++a) {
      const int t = order[a];
      const double vt = theta[t];
      int q = a - 1;
      while (q >= 0 && theta[order[q]] > vt) { order[q + 1] = order[q]; --q; }
      order[q + 1] = t;
    }
    g.flag[0] = r;
  }
  __syncthreads();
  // 7. coefficients: C_x[:, c] = scale * L^-T y_c (back substitution into
  //    Hm[.][c]), dropped rows 0; C_p = C_x with the X rows zeroed.
  for (int c = tid; c < b; c += nt) {
    const int oc = c < r ? order[c] : 0;
    for (int a = r - 1; a >= 0; --a) {
      double s = c < r ? V[a][oc] : 0.0;
      for (int q = a + 1; q < r; ++q) s -= G[kidx[q]][kidx[a]] * Hm[q][c];
      Hm[a][c] = s / G[kidx[a]][kidx[a]];
    }
    for (int k = 0; k < ns; ++k) {
      g.C[k * 2 * b + c] = 0.0;
      g.C[k * 2 * b + b + c] = 0.0;
    }
    for (int a = 0; a < r; ++a) {
      const int k = kidx[a];
      const double v = c < r ? Hm[a][c] * scale[k] : 0.0;
      g.C[k * 2 * b + c] = v;
      g.C[k * 2 * b + b + c] = k < b ? 0.0 : v;
    }
    g.lam[c] = c < r ? theta[oc] : 0.0;
  }
}

// ------------------------------------------------------------ update
struct UpdArgs {
  int64_t D;
  int b, ns, ld;
  double *S, *HS;
  const double *C, *lam, *diag;
  float *w32;             // optional float32 copy of W (dense D x b)
  double *npart;          // per block: b residual sums, b |x|^2 sums
  int rows_per_blk;
};

// Threads (row, column c).  All reads of a row precede the barrier, all writes
// follow it, so the update is in place.
__global__ __launch_bounds__(256) void k_update(UpdArgs g) {
  __shared__ double Cs[kNS * 2 * kMaxBlock];
  __shared__ double lam[kMaxBlock];
  __shared__ double red[2 * kMaxBlock];
  const int b = g.b, ns = g.ns, ld = g.ld;
  for (int k = threadIdx.x; k < ns * 2 * b; k += blockDim.x) Cs[k] = g.C[k];
  if (threadIdx.x < b) lam[threadIdx.x] = g.lam[threadIdx.x];
  if (threadIdx.x < 2 * b) red[threadIdx.x] = 0.0;
  __syncthreads();
  const int rows_per_pass = blockDim.x / b;
  const int c = threadIdx.x % b, rr = threadIdx.x / b;
  const bool active = rr < rows_per_pass;
  const int64_t r0 = (int64_t)blockIdx.x * g.rows_per_blk;
  const int64_t r1 = min(g.D, r0 + g.rows_per_blk);
  double rs = 0.0, xs = 0.0;
  for (int64_t base = r0; base < r1; base += rows_per_pass) {
    const int64_t i = base + rr;
    const bool ok = active && i < r1;
    double x = 0.0, p = 0.0, hx = 0.0, hp = 0.0;
    if (ok) {
      const double *s = g.S + i * ld;
      const double *h = g.HS + i * ld;
      for (int k = 0; k < ns; ++k) {
        const double sk = s[k], hk = h[k];
        const double cx = Cs[k * 2 * b + c], cp = Cs[k * 2 * b + b + c];
        x += sk * cx;
        p += sk * cp;
        hx += hk * cx;
        hp += hk * cp;
      }
    }
    __syncthreads();
    if (ok) {
      const double res = hx - lam[c] * x;
      double den = g.diag[i] - lam[c];
      if (fabs(den) < 1e-2) den = den < 0 ? -1e-2 : 1e-2;
      const double w = res / den;
      double *s = g.S + i * ld;
      double *h = g.HS + i * ld;
      s[c] = x;
      s[b + c] = w;
      s[2 * b + c] = p;
      h[c] = hx;
      h[2 * b + c] = hp;
      if (g.w32) g.w32[i * b + c] = (float)w;
      rs += res * res;
      xs += x * x;
    }
    __syncthreads();
  }
  if (active) {
    atomicAdd(&red[c], rs);
    atomicAdd(&red[b + c], xs);
  }
  __syncthreads();
  if (threadIdx.x < 2 * b) g.npart[(int64_t)blockIdx.x * 2 * b + threadIdx.x] = red[threadIdx.x];
}

// Relative residual norms and the count of converged leading pairs.
__global__ void k_finish(int b, int nev, int nparts, const double *npart, const double *lam, double tol,
                         double *status) {
  __shared__ double rs[kMaxBlock], xs[kMaxBlock];
  const int c = threadIdx.x;
  if (c < b) {
    double a = 0.0, x = 0.0;
    for (int q = 0; q < nparts; ++q) {
      a += npart[(int64_t)q * 2 * b + c];
      x += npart[(int64_t)q * 2 * b + b + c];
    }
    rs[c] = sqrt(a) / (fmax(fabs(lam[c]), 1.0) * sqrt(fmax(x, 1e-300)));
    xs[c] = lam[c];
  }
  __syncthreads();
  if (c == 0) {
    int conv = 0;
    for (int k = 0; k < nev; ++k) conv += rs[k] <= tol;
    status[0] = conv;
    for (int k = 0; k < b; ++k) { status[1 + k] = rs[k]; status[1 + kMaxBlock + k] = xs[k]; }
  }
}

// ------------------------------------------------------------ host driver
static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

struct LobpcgRun {
  cib_ctx *ctx;
  const cib_matrix &H;
  hipStream_t s;
  int64_t D;
  int b, nev, ld, gram_blocks, upd_blocks, max_iter;
  int64_t gram_rows, upd_rows;
  double tol;
  cib_lobpcg_opts opts;
  DBuf<double> S, HS, diag, partial, C, lam, npart, status;
  DBuf<float> x32, y32;
  DBuf<int64_t> idx;
  DBuf<int32_t> flag;
  int iters = 0;
  double t_spmm = 0.0;
  int64_t n_spmm = 0;
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  LobpcgRun(cib_ctx *c, const cib_matrix &h, const cib_lobpcg_opts &o, hipStream_t st, bool time_spmm)
      : ctx(c), H(h), s(st), D(h.D), b(o.block), nev(o.nev), max_iter(o.max_iter), opts(o),
        timing(time_spmm) {
    CIB_REQUIRE(nev >= 1 && nev <= b && b <= kMaxBlock, CIB_E_INVALID, "need 1 <= nev <= block <= 16");
    CIB_REQUIRE(3 * (int64_t)b <= H.D, CIB_E_INVALID, "need 3 * block <= D");
    CIB_REQUIRE(o.max_iter >= 1, CIB_E_INVALID, "max_iter must be >= 1");
    tol = o.tol > 0 ? o.tol : (H.dtype == CIB_F64 ? 1e-9 : 1e-6);
    ld = 3 * b;
    S.reset(ctx, (size_t)D * ld);
    HS.reset(ctx, (size_t)D * ld);
    diag.reset(ctx, D);
    gram_rows = std::max<int64_t>(256, (D + 2047) / 2048);
    gram_blocks = (int)((D + gram_rows - 1) / gram_rows);
    upd_rows = std::max<int64_t>(64, (D + 4095) / 4096);
    upd_blocks = (int)((D + upd_rows - 1) / upd_rows);
    partial.reset(ctx, (size_t)gram_blocks * kNS * 2 * kNS);
    C.reset(ctx, kNS * 2 * kMaxBlock);
    lam.reset(ctx, kMaxBlock);
    npart.reset(ctx, (size_t)upd_blocks * 2 * kMaxBlock);
    status.reset(ctx, kStatusLen);
    idx.reset(ctx, kMaxBlock);
    flag.reset(ctx, 4);
    if (H.dtype == CIB_F32) {
      x32.reset(ctx, (size_t)D * b);
      y32.reset(ctx, (size_t)D * b);
    }
    if (timing) {
      CIB_HIP(hipEventCreate(&ev0));
      CIB_HIP(hipEventCreate(&ev1));
    }
  }
  ~LobpcgRun() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  // HS[:, slot] = H S[:, slot]
  void spmm(int slot, bool w32_ready) {
    if (timing) CIB_HIP(hipEventRecord(ev0, s));
    if (H.dtype == CIB_F64) {
      spmm_sym(H, S.p + slot * b, ld, HS.p + slot * b, ld, b, s);
    } else {
      if (!w32_ready)
        hipLaunchKernelGGL(k_narrow, dim3(nblk(D * b)), dim3(256), 0, s, D, b, S.p + slot * b, ld, x32.p);
      spmm_sym(H, x32.p, b, y32.p, b, b, s);
      hipLaunchKernelGGL(k_widen, dim3(nblk(D * b)), dim3(256), 0, s, D, b, y32.p, HS.p + slot * b, ld);
    }
    if (timing) CIB_HIP(hipEventRecord(ev1, s));
    ++n_spmm;
  }

  void rr_update(int ns) {
    { KTimer kt(ctx, K_GRAM, s); hipLaunchKernelGGL(k_gram, dim3(gram_blocks), dim3(256), 0, s, D, ns, ld, S.p, HS.p, gram_rows, partial.p); }
    RRArgs ra{ns, b, gram_blocks, partial.p, C.p, lam.p, flag.p, 1e-10};
    { KTimer kt(ctx, K_RR, s); hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(256), 0, s, ra); }
    UpdArgs ua{D, b, ns, ld, S.p, HS.p, C.p, lam.p, diag.p, H.dtype == CIB_F32 ? x32.p : nullptr,
               npart.p, (int)upd_rows};
    { KTimer kt(ctx, K_UPDATE, s); hipLaunchKernelGGL(k_update, dim3(upd_blocks), dim3(256), 0, s, ua); }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, b, nev, upd_blocks, npart.p, lam.p, tol, status.p);
    CIB_HIP(hipGetLastError());
  }

  // diagonal, X0 and the Rayleigh-Ritz step on X0 alone
  void start() {
    if (H.dtype == CIB_F64)
      hipLaunchKernelGGL(k_diag<double>, dim3(nblk(D)), dim3(256), 0, s, D, H.row_ptr.p, H.val64.p, diag.p);
    else
      hipLaunchKernelGGL(k_diag<float>, dim3(nblk(D)), dim3(256), 0, s, D, H.row_ptr.p, H.val32.p, diag.p);
    if (opts.x0) {
      hipLaunchKernelGGL(k_copy_x0, dim3(nblk(D * b)), dim3(256), 0, s, D, b, ld, opts.x0, S.p);
    } else {
      hipLaunchKernelGGL(k_select_smallest, dim3(1), dim3(1024), 0, s, D, diag.p, b, idx.p);
      hipLaunchKernelGGL(k_init_x, dim3(nblk(D * b)), dim3(256), 0, s, D, b, ld, idx.p, opts.seed, S.p);
    }
    CIB_HIP(hipGetLastError());
    spmm(0, false);
    rr_update(b);
  }

  void iterate() {
    ++iters;
    spmm(1, H.dtype == CIB_F32);
    rr_update(iters == 1 ? 2 * b : 3 * b);
  }

  void copy_status(double *host) {
    CIB_HIP(hipMemcpyAsync(host, status.p, sizeof(double) * kStatusLen, hipMemcpyDeviceToHost, s));
  }

  void spmm_time_accumulate() {
    if (!timing) return;
    float ms = 0.f;
    CIB_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    t_spmm += ms * 1e-3;
  }

  void copy_vectors(double *evecs, int64_t ld_evecs) {
    hipLaunchKernelGGL(k_copy_cols, dim3(nblk(D * nev)), dim3(256), 0, s, D, nev, S.p, ld, evecs, ld_evecs);
    CIB_HIP(hipGetLastError());
  }
};

size_t lobpcg_bytes(int64_t D, int b, cib_dtype dt) {
  const int64_t gram_rows = std::max<int64_t>(256, (D + 2047) / 2048);
  const int64_t gram_blocks = (D + gram_rows - 1) / gram_rows;
  const int64_t upd_rows = std::max<int64_t>(64, (D + 4095) / 4096);
  const int64_t upd_blocks = (D + upd_rows - 1) / upd_rows;
  size_t n = (size_t)D * 3 * b * 8 * 2 + (size_t)D * 8 + (size_t)gram_blocks * kNS * 2 * kNS * 8 +
             (size_t)upd_blocks * 2 * kMaxBlock * 8 + 64 * 1024;
  if (dt == CIB_F32) n += (size_t)D * b * 4 * 2;
  return n;
}

LobpcgRun *lobpcg_create(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, hipStream_t s) {
  return new LobpcgRun(ctx, H, o, s, false);
}
void lobpcg_start(LobpcgRun *r) { r->start(); }
void lobpcg_iterate(LobpcgRun *r) { r->iterate(); }
void lobpcg_copy_status(LobpcgRun *r, double *host) { r->copy_status(host); }
int lobpcg_iters(const LobpcgRun *r) { return r->iters; }
void lobpcg_destroy(LobpcgRun *r) { delete r; }

cib_status lobpcg_solve(cib_ctx *ctx, const cib_matrix &H, const cib_lobpcg_opts &o, double *evals,
                        double *evecs, int64_t ld_evecs, cib_lobpcg_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  CIB_REQUIRE(!evecs || ld_evecs >= o.nev, CIB_E_INVALID, "ld_evecs < nev");
  LobpcgRun L(ctx, H, o, ctx->stream, true);
  double *st = static_cast<double *>(ctx->pinned_buf(sizeof(double) * kStatusLen));
  L.start();
  L.copy_status(st);
  CIB_HIP(hipStreamSynchronize(L.s));
  L.spmm_time_accumulate();
  int conv = (int)st[0];
  while (conv < L.nev && L.iters < L.max_iter) {
    L.iterate();
    L.copy_status(st);
    CIB_HIP(hipStreamSynchronize(L.s));
    L.spmm_time_accumulate();
    conv = (int)st[0];
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
