// Symmetric SpMM Y = H X (Sec. 2: sparse matrix-matrix products of the
// eigensolver; Fig. 2 line 5, "FMA of H_ij with the i-th row and j-th column
// vector elements").  Row i gathers its upper half (the half-stored CSR,
// j >= i) and its strictly lower half (the transposed copy the build keeps),
// so every output row is written once by one wave: no atomics, no zeroing,
// and a fixed summation order (deterministic).
//
// Layout: X, Y row-major (D x nvec, leading dimensions ldx / ldy), so one
// vector row is one contiguous run of 8 or 16 values.  A wave handles one
// row; its 64 lanes are E = 64 / B entry slots times B vector columns, so a
// gather of x_j is one contiguous segment, and each lane keeps U entries in
// flight.
#include <type_traits>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

template <typename T, int B, int U>
__device__ __forceinline__ T row_dot(int64_t k0, int64_t k1, const int32_t *__restrict__ col,
                                     const T *__restrict__ val, const T *__restrict__ X, int64_t ldx,
                                     int vc, bool cv, int e) {
  constexpr int E = kWave / B;
  T acc = T(0);
  int64_t k = k0 + e;
  for (; k + (U - 1) * E < k1; k += U * E) {
    int32_t j[U];
    T h[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      j[u] = col[k + u * E];
      h[u] = val[k + u * E];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = cv ? X[(int64_t)j[u] * ldx + vc] : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += h[u] * x[u];
  }
  for (; k < k1; k += E) {
    const int32_t j = col[k];
    const T h = val[k];
    acc += h * (cv ? X[(int64_t)j * ldx + vc] : T(0));
  }
  return acc;
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_spmm_sym(int64_t D, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const T *__restrict__ val,
                                                  const int64_t *__restrict__ lrp,
                                                  const int32_t *__restrict__ lcol,
                                                  const T *__restrict__ lval,
                                                  const T *__restrict__ X, int64_t ldx, T *__restrict__ Y,
                                                  int64_t ldy, int nvec, int v0) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (i >= D) return;
  const int lane = lane_id();
  const int e = lane / B, c = lane % B;
  const bool cv = c < nvec - v0;
  const int vc = v0 + c;
  T acc = row_dot<T, B, 4>(lrp[i], lrp[i + 1], lcol, lval, X, ldx, vc, cv, e);
  acc += row_dot<T, B, 4>(rp[i], rp[i + 1], col, val, X, ldx, vc, cv, e);
#pragma unroll
  for (int s = kWave / 2; s >= B; s >>= 1) acc += __shfl_down(acc, s, kWave);
  if (e == 0 && cv) Y[i * ldy + vc] = acc;
}

// Wide variant for nvec == NV (8 or 16) with 16-byte aligned rows: one lane
// per stored entry, so col/val reads are coalesced across the wave, and the
// x_j row is fetched with 16-byte vector loads into NV register accumulators;
// the row total is a wave reduction per vector column.
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_spmm_wide(int64_t D, const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const T *__restrict__ val,
                                                   const int64_t *__restrict__ lrp,
                                                   const int32_t *__restrict__ lcol,
                                                   const T *__restrict__ lval,
                                                   const T *__restrict__ X, int64_t ldx, T *__restrict__ Y,
                                                   int64_t ldy) {
  constexpr int PER16 = 16 / sizeof(T);           // values per 16-byte load
  using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = blk * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (i >= D) return;
  const int lane = lane_id();
  T acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = T(0);
  auto part = [&](int64_t k0, int64_t k1, const int32_t *__restrict__ cc, const T *__restrict__ vv) {
    for (int64_t k = k0 + lane; k < k1; k += kWave) {
      const int32_t j = cc[k];
      const T h = vv[k];
      const V *xr = reinterpret_cast<const V *>(X + (int64_t)j * ldx);
#pragma unroll
      for (int q = 0; q < NV / PER16; ++q) {
        const V t = xr[q];
        if constexpr (sizeof(T) == 8) {
          acc[2 * q] += h * t.x;
          acc[2 * q + 1] += h * t.y;
        } else {
          acc[4 * q] += h * t.x;
          acc[4 * q + 1] += h * t.y;
          acc[4 * q + 2] += h * t.z;
          acc[4 * q + 3] += h * t.w;
        }
      }
    }
  };
  part(lrp[i], lrp[i + 1], lcol, lval);
  part(rp[i], rp[i + 1], col, val);
  // reduce each column over the wave; lane v ends with column v's total
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = wave_sum(acc[v]);
  T mine = acc[0];
#pragma unroll
  for (int v = 1; v < NV; ++v) mine = lane == v ? acc[v] : mine;
  if (lane < NV) Y[i * ldy + lane] = mine;
}

template <typename T>
static void spmm_t(const cib_matrix &H, const T *X, int64_t ldx, T *Y, int64_t ldy, int nvec,
                   hipStream_t s) {
  const int64_t D = H.D;
  const T *val = static_cast<const T *>(H.val());
  const T *lval = static_cast<const T *>(H.lo_val());
  const unsigned nblk = (unsigned)((D + 3) / 4);
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((ldx * sizeof(T)) % 16 == 0);
  if (aligned && (nvec == 8 || nvec == 16)) {
    KTimer kt(H.ctx, K_SPMM, s);
    if (nvec == 8)
      hipLaunchKernelGGL((k_spmm_wide<T, 8>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p, H.col.p, val,
                         H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy);
    else
      hipLaunchKernelGGL((k_spmm_wide<T, 16>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p, H.col.p, val,
                         H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy);
    CIB_HIP(hipGetLastError());
    return;
  }
  for (int v0 = 0; v0 < nvec; v0 += 16) {
    KTimer kt(H.ctx, K_SPMM, s);
    if (nvec - v0 <= 8)
      hipLaunchKernelGGL((k_spmm_sym<T, 8>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p, H.col.p,
                         val, H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy, nvec, v0);
    else
      hipLaunchKernelGGL((k_spmm_sym<T, 16>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p,
                         H.col.p, val, H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy, nvec, v0);
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
