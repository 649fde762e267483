// Lanczos with full reorthogonalisation: the paper's alternative eigensolver
// for the lowest eigenpairs (Fig. 1 step 15; Sec. 2 names LOBPCG or Lanczos).
//
// Step k: w = H v_k (the symmetric SpMM, one vector; a float32 matrix gets a
// float32 copy of v_k), then classical Gram-Schmidt against all kept vectors
// applied twice, h = V^T w, w -= V h (alpha_k = sum of the two h_k), beta_k =
// |w|, v_{k+1} = w / beta_k.  The vectors stay in float64 on the device (one
// column of D values each); the small tridiagonal T_k (alpha, beta) is solved
// on the host: its lowest eigenvalues by bisection of Sturm counts, their
// vectors by inverse iteration, orthogonalised in order.  The residual of a
// Ritz pair is beta_k |s_k| (the last entry of its T-eigenvector), exact with
// full reorthogonalisation; the run stops when all nev residuals are below
// tol max(|theta|, 1), and the Ritz vectors are formed as V S on the device.
//
// Device sums (the dot products of a step) are per-wave DPP sums of fixed
// row chunks added chunk by chunk in order, so a run is deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

constexpr int kLzChunk = 4096;   // rows per wave in the dot products

// part[c * ncol + j] = sum over the rows of chunk c of V[j][r] w[r]: a wave
// per (chunk, column), lanes stride the chunk.
__global__ __launch_bounds__(256) void k_lz_dots(int64_t D, int ncol, const double *__restrict__ V,
                                                 const double *__restrict__ w, double *__restrict__ part) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nchunk = (int)((D + kLzChunk - 1) / kLzChunk);
  if (wave >= (int64_t)nchunk * ncol) return;
  const int j = (int)(wave % ncol), c = (int)(wave / ncol);
  const int64_t r0 = (int64_t)c * kLzChunk, r1 = r0 + kLzChunk < D ? r0 + kLzChunk : D;
  const double *v = V + (int64_t)j * D;
  double acc = 0.0;
  for (int64_t r = r0 + lane_id(); r < r1; r += kWave) acc += v[r] * w[r];
  acc = wave_sum_dpp(acc);
  if (lane_id() == 0) part[(int64_t)c * ncol + j] = acc;
}

// h[j] = sum over chunks c, ascending, of part[c * ncol + j]
__global__ void k_lz_sum(int nchunk, int ncol, const double *__restrict__ part, double *__restrict__ h) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * ncol + j];
  h[j] = s;
}

// w[r] -= sum over j, ascending, of V[j][r] h[j]
__global__ __launch_bounds__(256) void k_lz_sub(int64_t D, int ncol, const double *__restrict__ V,
                                                const double *__restrict__ h, double *__restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  double s = 0.0;
  for (int j = 0; j < ncol; ++j) s += V[(int64_t)j * D + r] * h[j];
  w[r] -= s;
}

// v = w * inv (and its float32 copy)
__global__ __launch_bounds__(256) void k_lz_scale(int64_t D, const double *__restrict__ w, double inv,
                                                  double *__restrict__ v, float *__restrict__ v32) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const double x = w[r] * inv;
  v[r] = x;
  if (v32) v32[r] = (float)x;
}

__global__ __launch_bounds__(256) void k_lz_widen(int64_t D, const float *__restrict__ y, double *__restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < D) w[r] = (double)y[r];
}

// start vector: uniform(-1, 1) entries from SplitMix64 of (seed, row)
__global__ __launch_bounds__(256) void k_lz_start(int64_t D, uint64_t seed, double *__restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  const uint64_t x = splitmix64(seed ^ splitmix64((uint64_t)r));
  w[r] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Y[i * ld + c] = sum over j < n, ascending, of V[j][i] S[j * nev + c]
__global__ __launch_bounds__(256) void k_lz_ritz(int64_t D, int n, int nev, const double *__restrict__ V,
                                                 const double *__restrict__ S, double *__restrict__ Y, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D * nev) return;
  const int64_t i = e / nev;
  const int c = (int)(e % nev);
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += V[(int64_t)j * D + i] * S[(int64_t)j * nev + c];
  Y[i * ld + c] = s;
}

// ------------------------------------------------------------ host side
namespace {

// eigenvalues of the symmetric tridiagonal T (diagonal a, off-diagonal b)
// below x: the negative pivots of T - x I = L D L^T
int tri_count(const std::vector<double> &a, const std::vector<double> &b, int n, double x, double pivmin) {
  int c = 0;
  double q = 1.0;
  for (int i = 0; i < n; ++i) {
    q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
  }
  return c;
}

// solve (T - x I) y = r in place (Gaussian elimination with partial pivoting
// on the tridiagonal band; the fill-in is a second superdiagonal)
void tri_solve(const std::vector<double> &a, const std::vector<double> &b, int n, double x, double pivmin,
               std::vector<double> &r) {
  std::vector<double> d(n), u1(n, 0.0), u2(n, 0.0);
  // working rows: row i holds (d[i], u1[i], u2[i]) on columns i, i+1, i+2
  for (int i = 0; i < n; ++i) {
    d[i] = a[i] - x;
    u1[i] = i + 1 < n ? b[i] : 0.0;
  }
  std::vector<double> sub(n, 0.0);   // sub-diagonal entry below row i's pivot
  for (int i = 0; i + 1 < n; ++i) sub[i] = b[i];
  for (int i = 0; i + 1 < n; ++i) {
    // candidates for the pivot of column i: row i (d[i]) and row i+1 (sub[i])
    if (std::fabs(sub[i]) > std::fabs(d[i])) {
      // swap rows i and i+1 (row i+1: sub[i], d[i+1], u1[i+1] on columns i, i+1, i+2)
      std::swap(d[i], sub[i]);
      std::swap(u1[i], d[i + 1]);
      std::swap(u2[i], u1[i + 1]);
      std::swap(r[i], r[i + 1]);
    }
    if (std::fabs(d[i]) < pivmin) d[i] = pivmin;
    const double l = sub[i] / d[i];
    d[i + 1] -= l * u1[i];
    u1[i + 1] -= l * u2[i];
    r[i + 1] -= l * r[i];
  }
  if (std::fabs(d[n - 1]) < pivmin) d[n - 1] = pivmin;
  for (int i = n - 1; i >= 0; --i) {
    double s = r[i];
    if (i + 1 < n) s -= u1[i] * r[i + 1];
    if (i + 2 < n) s -= u2[i] * r[i + 2];
    r[i] = s / d[i];
  }
}

}  // namespace

// lowest k eigenpairs of T: values in th, vectors (n x k, column c at S[j * k + c])
void tri_lowest(const std::vector<double> &a, const std::vector<double> &b, int n, int k, std::vector<double> &th,
                std::vector<double> &S) {
  double lo = 1e300, hi = -1e300, tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double rad = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - rad);
    hi = std::max(hi, a[i] + rad);
  }
  tnorm = std::max(std::fabs(lo), std::fabs(hi));
  const double pivmin = std::max(1e-300, 1e-290 * std::max(tnorm, 1.0));
  lo -= 1e-14 * tnorm + pivmin;
  hi += 1e-14 * tnorm + pivmin;
  th.assign(k, 0.0);
  for (int c = 0; c < k; ++c) {   // the (c+1)-th smallest: the first x with count > c
    double l = lo, h = hi;
    for (int it = 0; it < 200 && h - l > 4e-16 * std::max(std::fabs(l), std::fabs(h)) + pivmin; ++it) {
      const double m = 0.5 * (l + h);
      if (tri_count(a, b, n, m, pivmin) > c) h = m;
      else l = m;
    }
    th[c] = 0.5 * (l + h);
  }
  S.assign((size_t)n * k, 0.0);
  std::vector<double> y(n);
  // pivots of the inverse-iteration solves kept at eps |T| or more: a shift
  // equal to an eigenvalue to the last bit makes a pivot vanish, and a
  // near-zero replacement would overflow the solution (growth stays below
  // 1 / eps per solve, and every solve is followed by a normalisation)
  const double pivsolve = std::max(pivmin, 2.2e-16 * tnorm);
  for (int c = 0; c < k; ++c) {
    for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.01 * ((i * 7919 + c * 104729) % 101) / 101.0;
    for (int it = 0; it < 3; ++it) {
      tri_solve(a, b, n, th[c], pivsolve, y);
      // orthogonalise against the vectors already found (clusters), normalise
      for (int q = 0; q < c; ++q) {
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += S[(size_t)i * k + q] * y[i];
        for (int i = 0; i < n; ++i) y[i] -= dot * S[(size_t)i * k + q];
      }
      // normalise, dividing by the largest entry first (a solve can return
      // entries near the overflow threshold; their squares would overflow)
      double big = 0.0;
      for (int i = 0; i < n; ++i) big = std::max(big, std::fabs(y[i]));
      if (!(big > 0.0) || !std::isfinite(big)) big = 1.0;
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) {
        y[i] /= big;
        nrm += y[i] * y[i];
      }
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0)) nrm = 1.0;
      for (int i = 0; i < n; ++i) y[i] /= nrm;
    }
    for (int i = 0; i < n; ++i) S[(size_t)i * k + c] = y[i];
  }
}

cib_status lanczos_solve(cib_ctx *ctx, const cib_matrix &H, int nev, int max_iter, double tol, uint64_t seed,
                         double *evals, double *evecs, int64_t ld_evecs, cib_lanczos_info *info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  UnwindFence fence(s);
  const int64_t D = H.D;
  const int m = (int)std::min<int64_t>(max_iter, D);
  const bool f32 = H.dtype == CIB_F32;
  if (tol <= 0) tol = f32 ? 1e-6 : 1e-10;
  const int nchunk = (int)((D + kLzChunk - 1) / kLzChunk);
  DBuf<double> V(ctx, (size_t)(m + 1) * D), w(ctx, D), part(ctx, (size_t)nchunk * (m + 1)),
      h(ctx, 2 * (size_t)(m + 2));
  DBuf<float> v32, y32;
  if (f32) {
    v32.reset(ctx, D);
    y32.reset(ctx, D);
  }
  const dim3 rows((unsigned)((D + 255) / 256)), t256(256);
  auto dots = [&](const double *Vp, int ncol, double *out) {
    const int64_t waves = (int64_t)nchunk * ncol;
    hipLaunchKernelGGL(k_lz_dots, dim3((unsigned)((waves + 3) / 4)), t256, 0, s, D, ncol, Vp, w.p, part.p);
    hipLaunchKernelGGL(k_lz_sum, dim3((unsigned)((ncol + 255) / 256)), t256, 0, s, nchunk, ncol, part.p, out);
  };
  auto read = [&](const double *dev, double *host, int n) {
    CIB_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
    CIB_HIP(hipStreamSynchronize(s));
  };
  // v_0 = random unit vector
  hipLaunchKernelGGL(k_lz_start, rows, t256, 0, s, D, seed, w.p);
  dots(w.p, 1, h.p);
  double nrm2 = 0.0;
  read(h.p, &nrm2, 1);
  CIB_REQUIRE(nrm2 > 0.0, CIB_E_DEVICE, "Lanczos start vector is zero");
  hipLaunchKernelGGL(k_lz_scale, rows, t256, 0, s, D, w.p, 1.0 / std::sqrt(nrm2), V.p, f32 ? v32.p : nullptr);

  std::vector<double> alpha, beta, th, S, hh(2 * (m + 2));
  int n = 0, conv = 0;
  double t_spmv = 0.0;
  hipEvent_t e0, e1;
  // timing only: no system-scope fence at every record
  CIB_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  CIB_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  std::vector<double> resid(nev, INFINITY);
  for (int k = 0; k < m; ++k) {
    double *vk = V.p + (int64_t)k * D;
    CIB_HIP(hipEventRecord(e0, s));
    {
      KTimer kt(ctx, K_SPMM, s);
      if (f32) {
        spmm_sym(H, v32.p, 1, y32.p, 1, 1, s);
        hipLaunchKernelGGL(k_lz_widen, rows, t256, 0, s, D, y32.p, w.p);
      } else {
        spmm_sym(H, vk, 1, w.p, 1, 1, s);
      }
    }
    CIB_HIP(hipEventRecord(e1, s));
    // classical Gram-Schmidt twice against v_0 .. v_k
    for (int pass = 0; pass < 2; ++pass) {
      dots(V.p, k + 1, h.p + pass * (m + 2));
      hipLaunchKernelGGL(k_lz_sub, rows, t256, 0, s, D, k + 1, V.p, h.p + pass * (m + 2), w.p);
    }
    dots(w.p, 1, h.p + 2 * (m + 2) - 1);
    CIB_HIP(hipMemcpyAsync(hh.data(), h.p, 2 * (m + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
    CIB_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    CIB_HIP(hipEventElapsedTime(&ms, e0, e1));
    t_spmv += ms * 1e-3;
    alpha.push_back(hh[k] + hh[(m + 2) + k]);
    const double b = std::sqrt(std::max(hh[2 * (m + 2) - 1], 0.0));
    n = k + 1;
    const bool last = k + 1 == m;
    const double scale = std::max(std::fabs(alpha.back()), 1.0);
    const bool invariant = b <= 1e-14 * scale;
    // convergence: every fourth step once n >= nev, and at the end
    if (n >= nev && ((k % 4) == 3 || last || invariant)) {
      tri_lowest(alpha, beta, n, nev, th, S);
      conv = 0;
      for (int c = 0; c < nev; ++c) {
        resid[c] = invariant ? 0.0 : b * std::fabs(S[(size_t)(n - 1) * nev + c]) / std::max(std::fabs(th[c]), 1.0);
        if (resid[c] <= tol) ++conv;
      }
      if (conv == nev) break;
    }
    if (invariant || last) break;
    beta.push_back(b);
    hipLaunchKernelGGL(k_lz_scale, rows, t256, 0, s, D, w.p, 1.0 / b, V.p + (int64_t)(k + 1) * D,
                       f32 ? v32.p : nullptr);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CIB_REQUIRE(n >= nev && (int)th.size() == nev, CIB_E_NOT_CONVERGED,
              "Lanczos stopped before the tridiagonal matrix reached nev rows");
  for (int c = 0; c < nev; ++c) evals[c] = th[c];
  if (evecs) {
    DBuf<double> Sd(ctx, (size_t)n * nev);
    Sd.upload(S.data(), S.size(), s);
    hipLaunchKernelGGL(k_lz_ritz, dim3((unsigned)((D * nev + 255) / 256)), t256, 0, s, D, n, nev, V.p, Sd.p,
                       evecs, ld_evecs);
    CIB_HIP(hipGetLastError());
    CIB_HIP(hipStreamSynchronize(s));
  }
  if (info) {
    info->iters = n;
    info->n_converged = conv;
    for (int c = 0; c < 64; ++c) info->resid[c] = c < nev ? resid[c] : 0.0;
    info->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_spmv_s = t_spmv;
  }
  return conv == nev ? CIB_OK : CIB_E_NOT_CONVERGED;
}

}  // namespace cib
