// Symmetric SpMM Y = H X (Sec. 2: sparse matrix-matrix products of the
// eigensolver; Fig. 2, the FMA of H_ij with the vector elements of row j).
// Row i gathers its upper half (the half-stored CSR, j >= i) and its
// strictly lower half (the transposed copy the build keeps), so every output
// row is produced by gathers only: no atomics, no zeroing, and a fixed
// summation order (deterministic).
//
// Layout: X, Y row-major (D x nvec, leading dimensions ldx / ldy), so one
// vector row is one contiguous run of nvec values.
#include <algorithm>
#include <type_traits>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

// ------------------------------------------------------------ general path
// Any nvec, any alignment: a wave per row, 64 / B entry slots times B vector
// columns, so a gather of x_j is one contiguous segment.
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
                                                  int64_t ldy, int nvec, int v0, const int32_t *stop) {
  if (stop && *stop) return;   // a solve's iteration queued past its convergence
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

// ------------------------------------------------------------ vector path
// Rows per workgroup of the grouped (serving) launch: one count for both
// dtypes, since the workgroup offsets of a batch are made on the host.
constexpr int kGroupRows = 4;

// Butterfly reduce-scatter of N accumulators over the lane bits M, M/2, ...,
// G (the entry-slot bits): each exchange halves the values a lane keeps, so
// N values cost N - 1 + (remaining steps) shuffles instead of N per step.
template <typename T, int N, int M, int G>
struct Bfly {
  __device__ __forceinline__ static void run(T *acc, int lane) {
    if constexpr (M >= G) {
      if constexpr (N > 1) {
        const bool up = lane & M;
#pragma unroll
        for (int k = 0; k < N / 2; ++k) {
          const T keep = up ? acc[N / 2 + k] : acc[k];
          const T send = up ? acc[k] : acc[N / 2 + k];
          acc[k] = keep + __shfl_xor(send, M, kWave);
        }
        Bfly<T, N / 2, M / 2, G>::run(acc, lane);
      } else {
        acc[0] += __shfl_xor(acc[0], M, kWave);
        Bfly<T, 1, M / 2, G>::run(acc, lane);
      }
    }
  }
};

// nvec == NV (8 or 16) with 16-byte aligned rows of X.  One wave per row.
// The wave reads 64 consecutive entries of the row (lower part, then upper
// part) with one coalesced load of col and of val; the entries are handed to groups of G lanes by
// lane permutes, and each group gathers the NV values of x_j with one
// 16-byte load per lane.  The col/val loads of the next step are issued
// behind the gathers of the current one, so a step costs one memory round
// trip.  Columns are reduced over the entry slots at the end with a
// butterfly.
//
// The limit here is the number of L1 misses in flight per CU, not HBM:
// every entry gathers a row of X.  Neighbouring rows gather many of the
// same X rows (64 consecutive rows reference each 128-byte line of X about
// five times), but only if they walk their columns together do those lines
// stay in L1 in between: the rows of one workgroup therefore take their
// 64-entry steps in lockstep, with a workgroup barrier after every step (a
// row that has ended keeps joining the barriers until the longest row of
// the workgroup ends).  Measured at D ~ 2e5, b = 16: 18-20% faster than the
// same rows without the barriers, float32 and float64; a barrier every two
// or four steps gains less.  Splitting the columns into chunks, one per
// XCD, so that X stays in L2, and streaming col/val with non-temporal loads
// were both measured slower.
//
// The workgroup takes rows [i0, i0 + nrows), one per wave; a wave past the
// last row only joins the barriers.
template <typename T, int NV>
__device__ __forceinline__ void spmm_vec_rows(const VecArgs &a, int64_t i0, int nrows) {
  constexpr int PER16 = 16 / sizeof(T);  // values per 16-byte load
  constexpr int G = NV / PER16;          // lanes per entry
  constexpr int E = kWave / G;           // entries per gather instruction
  using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  const int32_t *__restrict__ col = a.col;
  const int32_t *__restrict__ lcol = a.lcol;
  const T *__restrict__ val = static_cast<const T *>(a.val);
  const T *__restrict__ lval = static_cast<const T *>(a.lval);
  const T *__restrict__ X = static_cast<const T *>(a.X);
  const int lane = lane_id();
  const int e = lane / G, g = lane % G;
  const int wv = uni((int)(threadIdx.x >> 6));
  const bool live = wv < nrows;
  const int64_t i = i0 + (live ? wv : 0);
  // longest row of the workgroup: the number of lockstep steps
  int most = 0;
  for (int r = 0; r < nrows; ++r)
    most = max(most, (int)((a.lrp[i0 + r + 1] - a.lrp[i0 + r]) + (a.rp[i0 + r + 1] - a.rp[i0 + r])));
  const int64_t lb = a.lrp[i], ub = a.rp[i];
  const int nl = live ? (int)(a.lrp[i + 1] - lb) : 0;
  const int n = live ? nl + (int)(a.rp[i + 1] - ub) : 0;
  // Loads are issued unconditionally (out-of-range lanes read a valid
  // address and discard it): loads under branches would make the compiler
  // wait for every outstanding load, the prefetch included.
  auto fetch = [&](int p, int32_t &j, T &h) {
    const bool ok = p < n;
    const bool lo = p < nl;
    const int64_t k = !ok ? ub : lo ? lb + p : ub + (p - nl);
    const int32_t *cp = ok && lo ? lcol : col;
    const T *vp = ok && lo ? lval : val;
    const int32_t jj = cp[k];
    const T hh = vp[k];
    j = ok ? jj : -1;
    h = ok ? hh : T(0);
  };
  T acc[PER16];
#pragma unroll
  for (int t = 0; t < PER16; ++t) acc[t] = T(0);
  int32_t jn;
  T hn;
  fetch(lane, jn, hn);
  for (int p0 = 0; p0 < most; p0 += kWave) {
    if (p0 < n) {   // uniform over the wave
      const int32_t jc = jn;
      const T hc = hn;
      V x[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int32_t j = __shfl(jc, u * E + e, kWave);
        x[u] = reinterpret_cast<const V *>(X + (int64_t)(j < 0 ? i : j) * a.ldx)[g];
      }
      fetch(p0 + kWave + lane, jn, hn);
#pragma unroll
      for (int u = 0; u < G; ++u) {
        // lane permutes first, with every lane active: a permute reading a
        // lane that has branched off returns garbage
        const T h = __shfl(hc, u * E + e, kWave);
        const bool used = __shfl(jc, u * E + e, kWave) >= 0;
        // an unused slot has j < 0 and h == 0; skip it so a non-finite x_i
        // cannot leak in
        if (!used) continue;
        if constexpr (sizeof(T) == 8) {
          acc[0] += h * x[u].x;
          acc[1] += h * x[u].y;
        } else {
          acc[0] += h * x[u].x;
          acc[1] += h * x[u].y;
          acc[2] += h * x[u].z;
          acc[3] += h * x[u].w;
        }
      }
    }
    __syncthreads();
  }
  Bfly<T, PER16, kWave / 2, G>::run(acc, lane);
  // after the exchanges, lane bits above log2(64 / PER16) select the column
  constexpr int SEL = kWave / PER16;
  T *Y = static_cast<T *>(a.Y);
  if (live && (lane & (SEL - 1) & ~(G - 1)) == 0) {
    const int c = g * PER16 + ((lane / SEL) & (PER16 - 1));
    if (sizeof(T) == 4 && a.Y64) a.Y64[i * a.ldy64 + c] = (double)acc[0];
    else Y[i * a.ldy + c] = acc[0];
  }
}

// Rows per workgroup of the lockstep kernels: 8 for float32, 4 for float64
// (measured best at D ~ 2e5, b = 16; 16 rows were slower for both).
template <typename T>
constexpr int vec_rows_per_block() {
  return sizeof(T) == 8 ? 4 : 8;
}

template <typename T, int NV>
__global__ __launch_bounds__(64 * vec_rows_per_block<T>()) void k_spmm_vec(const VecArgs a) {
  // workgroups go to the 8 XCDs round-robin; XCD x (block mod 8) walks its
  // own range of rows, the ranges holding equal numbers of stored entries
  constexpr int R = vec_rows_per_block<T>();
  if (a.stop && *a.stop) return;   // a solve's iteration queued past its convergence
  const int x = blockIdx.x & 7;
  const int64_t i0 = a.xr[x] + (int64_t)(blockIdx.x >> 3) * R;
  if (i0 >= a.xr[x + 1]) return;   // whole workgroup
  spmm_vec_rows<T, NV>(a, i0, (int)min<int64_t>(R, a.xr[x + 1] - i0));
}

// Several matrices in one launch (the serving loop's batch): off[j] is the
// first workgroup of job j (kGroupRows rows per workgroup, plain row order).
template <typename T, int NV>
__global__ __launch_bounds__(64 * kGroupRows) void k_spmm_vec_group(const VecArgs *__restrict__ as,
                                                                    const int32_t *__restrict__ off, int njobs) {
  const int j = group_job(off, njobs, (int)blockIdx.x);
  const VecArgs &a = as[j];
  const int64_t i0 = (int64_t)(blockIdx.x - off[j]) * kGroupRows;
  if (i0 >= a.D) return;   // whole workgroup
  spmm_vec_rows<T, NV>(a, i0, (int)min<int64_t>(kGroupRows, a.D - i0));
}

// ------------------------------------------------------------ host side
template <typename T>
static void spmm_t(const cib_matrix &H, const T *X, int64_t ldx, T *Y, int64_t ldy, int nvec,
                   hipStream_t s, const int32_t *stop) {
  const int64_t D = H.D;
  const T *val = static_cast<const T *>(H.val());
  const T *lval = static_cast<const T *>(H.lo_val());
  const unsigned nblk = (unsigned)((D + 3) / 4);
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((ldx * sizeof(T)) % 16 == 0);
  if (aligned && (nvec == 8 || nvec == 16)) {
    // Each XCD takes one contiguous range of rows holding an eighth of the
    // stored entries (both triangles): X rows gathered by nearby rows stay in
    // that XCD's L2, and the ranges are balanced.  Measured against plain
    // block order: 6-22% faster at D ~ 2e5, equal at D ~ 2e4; equal row
    // counts per XCD instead were up to 10% slower than plain order.
    VecArgs a{D, H.row_ptr.p, H.col.p, val, H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy, {}, stop};
    constexpr int R = vec_rows_per_block<T>();
    int64_t most = 0;
    for (int x = 0; x < 9; ++x) a.xr[x] = H.xcd_rows[x];
    for (int x = 0; x < 8; ++x) most = std::max<int64_t>(most, a.xr[x + 1] - a.xr[x]);
    const unsigned grid = (unsigned)std::max<int64_t>(8, 8 * ((most + R - 1) / R));
    KTimer kt(H.ctx, K_SPMM, s);
    if (nvec == 8) hipLaunchKernelGGL((k_spmm_vec<T, 8>), dim3(grid), dim3(64 * R), 0, s, a);
    else hipLaunchKernelGGL((k_spmm_vec<T, 16>), dim3(grid), dim3(64 * R), 0, s, a);
    CIB_HIP(hipGetLastError());
    return;
  }
  // B vector columns per wave step, the narrowest that covers the columns
  // left: one vector (the Lanczos product) gives 64 entry slots per step
  // instead of 8
  auto launch = [&](auto bc, int v0) {
    constexpr int B = decltype(bc)::value;
    hipLaunchKernelGGL((k_spmm_sym<T, B>), dim3(nblk), dim3(256), 0, s, D, H.row_ptr.p, H.col.p, val,
                       H.lo_ptr.p, H.lo_col.p, lval, X, ldx, Y, ldy, nvec, v0, stop);
  };
  for (int v0 = 0; v0 < nvec; v0 += 16) {
    KTimer kt(H.ctx, K_SPMM, s);
    const int left = nvec - v0;
    if (left == 1) launch(std::integral_constant<int, 1>{}, v0);
    else if (left == 2) launch(std::integral_constant<int, 2>{}, v0);
    else if (left <= 4) launch(std::integral_constant<int, 4>{}, v0);
    else if (left <= 8) launch(std::integral_constant<int, 8>{}, v0);
    else launch(std::integral_constant<int, 16>{}, v0);
  }
  CIB_HIP(hipGetLastError());
}

bool spmm_sym_widen(const cib_matrix &H, const float *X, int64_t ldx, double *Y, int64_t ldy, int nvec,
                    hipStream_t s, const int32_t *stop) {
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((ldx * sizeof(float)) % 16 == 0);
  if (H.dtype != CIB_F32 || !aligned || (nvec != 8 && nvec != 16)) return false;
  constexpr int R = vec_rows_per_block<float>();
  VecArgs a{H.D, H.row_ptr.p, H.col.p, H.val(), H.lo_ptr.p, H.lo_col.p, H.lo_val(), X, ldx, nullptr, 0, {}, stop,
            Y, ldy};
  int64_t most = 0;
  for (int x = 0; x < 9; ++x) a.xr[x] = H.xcd_rows[x];
  for (int x = 0; x < 8; ++x) most = std::max<int64_t>(most, a.xr[x + 1] - a.xr[x]);
  const unsigned grid = (unsigned)std::max<int64_t>(8, 8 * ((most + R - 1) / R));
  KTimer kt(H.ctx, K_SPMM, s);
  if (nvec == 8) hipLaunchKernelGGL((k_spmm_vec<float, 8>), dim3(grid), dim3(64 * R), 0, s, a);
  else hipLaunchKernelGGL((k_spmm_vec<float, 16>), dim3(grid), dim3(64 * R), 0, s, a);
  CIB_HIP(hipGetLastError());
  return true;
}

bool spmm_vec_args(const cib_matrix &H, const void *X, int64_t ldx, void *Y, int64_t ldy, int nvec, VecArgs &a,
                   int &blocks) {
  const size_t sv = H.dtype == CIB_F64 ? 8 : 4;
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((ldx * sv) % 16 == 0);
  if (!aligned || (nvec != 8 && nvec != 16)) return false;
  a = VecArgs{H.D, H.row_ptr.p, H.col.p, H.val(), H.lo_ptr.p, H.lo_col.p, H.lo_val(), X, ldx, Y, ldy, {}};
  blocks = (int)((H.D + kGroupRows - 1) / kGroupRows);
  return true;
}

void launch_spmm_group(cib_dtype dt, int nvec, const VecArgs *dev_args, const int32_t *dev_off, int njobs,
                       int total_blocks, hipStream_t s) {
  if (njobs <= 0 || total_blocks <= 0) return;
  const dim3 g((unsigned)total_blocks), t(64 * kGroupRows);
  if (dt == CIB_F64) {
    if (nvec == 8) hipLaunchKernelGGL((k_spmm_vec_group<double, 8>), g, t, 0, s, dev_args, dev_off, njobs);
    else hipLaunchKernelGGL((k_spmm_vec_group<double, 16>), g, t, 0, s, dev_args, dev_off, njobs);
  } else {
    if (nvec == 8) hipLaunchKernelGGL((k_spmm_vec_group<float, 8>), g, t, 0, s, dev_args, dev_off, njobs);
    else hipLaunchKernelGGL((k_spmm_vec_group<float, 16>), g, t, 0, s, dev_args, dev_off, njobs);
  }
  CIB_HIP(hipGetLastError());
}

void spmm_sym(const cib_matrix &H, const void *X, int64_t ldx, void *Y, int64_t ldy, int nvec,
              hipStream_t s, const int32_t *stop) {
  if (H.dtype == CIB_F64)
    spmm_t<double>(H, static_cast<const double *>(X), ldx, static_cast<double *>(Y), ldy, nvec, s, stop);
  else
    spmm_t<float>(H, static_cast<const float *>(X), ldx, static_cast<float *>(Y), ldy, nvec, s, stop);
}

}  // namespace cib
