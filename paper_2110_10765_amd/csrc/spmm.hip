// Symmetric SpMM Y = H X from the half-stored CSR (upper triangle with the
// diagonal): y_i += sum_{j>=i} H_ij x_j (row gather) and y_j += H_ij x_i for
// j > i (transposed half, device atomics).  Sec. 2: sparse matrix-matrix
// products of the eigensolver; Fig. 2 line 5 ("FMA of H_ij with the i-th row
// and j-th column vector elements").
//
// Layout: X, Y row-major (D x nvec, leading dimensions ldx / ldy), so one
// vector row is one contiguous run of 8 or 16 values.  A wave handles one
// row; its 64 lanes are E = 64 / B entry slots times B vector columns, so a
// gather of x_j and an atomic update of y_j are each one contiguous segment.
#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T *Y, int64_t D, int64_t ldy, int nvec) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = k / nvec, c = k % nvec;
  if (r < D) Y[r * ldy + c] = T(0);
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_spmm_sym(int64_t D, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const T *__restrict__ val,
                                                  const T *__restrict__ X, int64_t ldx, T *Y,
                                                  int64_t ldy, int nvec, int v0) {
  constexpr int E = kWave / B;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (i >= D) return;
  const int lane = lane_id();
  const int e = lane / B, c = lane % B;
  const bool cv = c < nvec - v0 && c < B;
  const int vc = v0 + c;
  const T xi = cv ? X[i * ldx + vc] : T(0);
  T acc = T(0);
  const int64_t k1 = rp[i + 1];
  for (int64_t k = rp[i] + e; k < k1; k += E) {
    const int32_t j = col[k];
    const T h = val[k];
    if (cv) {
      acc += h * X[(int64_t)j * ldx + vc];
      if (j != i) unsafeAtomicAdd(&Y[(int64_t)j * ldy + vc], h * xi);
    }
  }
#pragma unroll
  for (int s = kWave / 2; s >= B; s >>= 1) acc += __shfl_down(acc, s, kWave);
  if (e == 0 && cv) unsafeAtomicAdd(&Y[i * ldy + vc], acc);
}

template <typename T>
static void spmm_t(const cib_matrix &H, const T *X, int64_t ldx, T *Y, int64_t ldy, int nvec,
                   hipStream_t s) {
  const int64_t D = H.D;
  const T *val = static_cast<const T *>(H.val());
  const int64_t nz = D * nvec;
  hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, Y, D, ldy, nvec);
  const unsigned nblk = (unsigned)((D + 3) / 4);
  for (int v0 = 0; v0 < nvec; v0 += 16) {
    KTimer kt(H.ctx, K_SPMM, s);
    if (nvec - v0 <= 8)
      hipLaunchKernelGGL((k_spmm_sym<T, 8>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p, H.col.p,
                         val, X, ldx, Y, ldy, nvec, v0);
    else
      hipLaunchKernelGGL((k_spmm_sym<T, 16>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p,
                         H.col.p, val, X, ldx, Y, ldy, nvec, v0);
  }
  CIB_HIP(hipGetLastError());
}

void spmm_sym(const cib_matrix &H, const void *X, int64_t ldx, void *Y, int64_t ldy, int nvec,
              hipStream_t s) {
  if (H.dtype == CIB_F64)
    spmm_t<double>(H, static_cast<const double *>(X), ldx, static_cast<double *>(Y), ldy, nvec, s);
  else
    spmm_t<float>(H, static_cast<const float *>(X), ldx, static_cast<float *>(Y), ldy, nvec, s);
}

}  // namespace cib
