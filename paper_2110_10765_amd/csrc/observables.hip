// Observables after the eigensolve (Fig. 1 steps 16-20): for m operators O_k
// (one-body energies and two-body tables in the Hamiltonian's layout) and n
// vectors x_v, a[k][v] = x_v^T O_k x_v.
//
// Each operator is applied once: with 8 or 16 vectors by the matrix-free
// product (the build's screens and values multiplied into X, no CSR held),
// otherwise built as a half-stored matrix by the same passes as H and
// applied by the symmetric SpMM, then freed before the next operator.  The
// products x_v . (O_k x_v) are summed in float64 in a fixed order: per
// workgroup, each thread owns one column and a stride of rows, the
// workgroup's partial sums are added in thread order, and one pass adds the
// workgroups' sums in workgroup order (the register accumulators and
// fixed-order tree of the paper's scalar reductions, with no atomics).
#include <memory>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {

constexpr int kDotThreads = 256, kDotRows = 1024;   // rows per workgroup

// partial[blk * nvec + v] = sum over rows i of the workgroup of X[i][v] Y[i][v]
// (float64); nvec <= 64, so at least four threads share a column.
template <typename T>
__global__ __launch_bounds__(kDotThreads) void k_col_dots(int64_t D, int nvec, const T *__restrict__ X,
                                                          int64_t ldx, const T *__restrict__ Y, int64_t ldy,
                                                          double *__restrict__ partial) {
  __shared__ double s[kDotThreads];
  const int t = threadIdx.x;
  const int groups = kDotThreads / nvec;
  const int v = t % nvec, g = t / nvec;
  const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
  const int64_t r1 = r0 + kDotRows < D ? r0 + kDotRows : D;
  double acc = 0.0;
  if (g < groups)
    for (int64_t i = r0 + g; i < r1; i += groups) acc += (double)X[i * ldx + v] * (double)Y[i * ldy + v];
  s[t] = acc;
  __syncthreads();
  if (t < nvec) {
    double sum = 0.0;
    for (int q = 0; q < groups; ++q) sum += s[q * nvec + t];
    partial[(int64_t)blockIdx.x * nvec + t] = sum;
  }
}

// out[v] = sum over workgroups b (ascending) of partial[b * nvec + v]
__global__ void k_sum_cols(int nblk, int nvec, const double *__restrict__ partial, double *__restrict__ out) {
  const int v = threadIdx.x;
  if (v >= nvec) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * nvec + v];
  out[v] = s;
}

void observables(cib_ctx *ctx, const cib_basis &b, const cib_tables *ops, int m, cib_dtype dt, const void *X,
                 int64_t ldx, int nvec, double *out, hipStream_t s) {
  UnwindFence fence(s);
  const int64_t D = b.plan.D;
  const size_t sv = dt == CIB_F64 ? 8 : 4;
  const int nblk = (int)((D + kDotRows - 1) / kDotRows);
  // Y holds D x nvec values of the matrix dtype (16-byte aligned rows when
  // nvec * sv is, like the caller's X)
  DBuf<double> Y(ctx, (size_t)((D * nvec * sv + 7) / 8));
  DBuf<double> partial(ctx, (size_t)nblk * nvec), dout(ctx, (size_t)m * nvec);
  // waits for the stream before the buffers declared ahead of it are freed,
  // also when a step throws
  struct SyncFirst {
    hipStream_t s;
    ~SyncFirst() { (void)hipStreamSynchronize(s); }
  };
  // 8 or 16 vectors in 16-byte rows: the matrix-free product (the build's
  // screens and values, no CSR); otherwise the operator is built and applied
  const bool free_ok = (nvec == 8 || nvec == 16) && (uintptr_t)X % 16 == 0 && (ldx * sv) % 16 == 0;
  for (int k = 0; k < m; ++k) {
    std::unique_ptr<cib_interaction> it(upload_interaction(ctx, b, ops[k], s));
    cib_matrix H;
    H.ctx = ctx;
    SyncFirst sync{s};
    if (free_ok) {
      apply_matrix_free(ctx, b, *it, dt, ApplyReq{X, ldx, Y.p, (int64_t)nvec, nvec}, s);
    } else {
      build_matrix(ctx, b, *it, dt, H, s, nullptr);
      spmm_sym(H, X, ldx, Y.p, nvec, nvec, s);
    }
    if (dt == CIB_F64)
      hipLaunchKernelGGL(k_col_dots<double>, dim3(nblk), dim3(kDotThreads), 0, s, D, nvec,
                         static_cast<const double *>(X), ldx, Y.p, (int64_t)nvec, partial.p);
    else
      hipLaunchKernelGGL(k_col_dots<float>, dim3(nblk), dim3(kDotThreads), 0, s, D, nvec,
                         static_cast<const float *>(X), ldx, reinterpret_cast<const float *>(Y.p),
                         (int64_t)nvec, partial.p);
    hipLaunchKernelGGL(k_sum_cols, dim3(1), dim3(64), 0, s, nblk, nvec, partial.p, dout.p + (size_t)k * nvec);
    CIB_HIP(hipGetLastError());
  }
  CIB_HIP(hipMemcpyAsync(out, dout.p, (size_t)m * nvec * sizeof(double), hipMemcpyDeviceToHost, s));
  CIB_HIP(hipStreamSynchronize(s));
}

}  // namespace cib
