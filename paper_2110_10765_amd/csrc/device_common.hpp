// Device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cib {
namespace dev {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Number of set lanes below the calling lane in a 64-bit ballot mask.
__device__ __forceinline__ int mask_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// A value equal in all lanes of the wave, moved to a scalar register.  The
// compiler treats anything derived from threadIdx.x as varying per lane, also
// threadIdx.x / 64, so per-wave indices and what is loaded through them would
// otherwise be computed lane by lane in vector registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint64_t uni(uint64_t v) { return (uint64_t)uni((int64_t)v); }

// Lane permutation within rows of 16 lanes through DPP (no LDS round trip).
// For the permutations used here every lane has a valid source, so no old
// value is needed (bound_ctrl).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)((uint64_t)hi << 32 | lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

// Sum over the 64 lanes, returned to every lane (all lanes must be active):
// DPP exchanges inside each row of 16 (xor 1, xor 2, mirrored halves,
// mirrored row), then the four row sums read as scalars, in a fixed order.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Orders LDS accesses between the lanes of one wave: LDS instructions of a
// wave execute in issue order, so only compiler code motion has to be
// stopped (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum of an int over the 64 lanes through DPP (all lanes
// active): shifts by 1, 2, 4, 8 inside each row of 16, then the last lane of
// a row is broadcast into the next row(s).  No LDS round trips.
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false); // row_bcast:15 -> rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false); // row_bcast:31 -> rows 2, 3
  return v;
}

// Inclusive prefix maximum of a non-negative int over the 64 lanes through
// DPP (all lanes active; lanes shifted in from outside a row read 0, the
// identity for non-negative values).
__device__ __forceinline__ int wave_incl_max_dpp(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true));   // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true));   // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true));   // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true));   // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false));  // row_bcast:15 -> rows 1, 3
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false));  // row_bcast:31 -> rows 2, 3
  return v;
}

// Inclusive and exclusive wave-wide prefix sums.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (l >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Job of workgroup b in a grouped launch (several independent problems in
// one grid): off[0..n) holds each job's first workgroup, ascending, off[0] = 0.
// The search reads the same entries in every lane.
__device__ __forceinline__ int group_job(const int32_t *off, int n, int b) {
  int lo = 0, hi = n;   // the last job whose first workgroup is <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Map a linear block index so that each XCD (blocks are dispatched to the 8
// XCDs round-robin) works on one contiguous range of logical blocks, which
// keeps the data those blocks share inside one XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t x = b & 7, k = b >> 3;
  const int64_t start = x * q + (x < r ? x : r);
  return start + k;
}

// ---- multiword bit strings (W little-endian 64-bit words) ----
template <int W>
__device__ __forceinline__ int popc_xor(const uint64_t *a, const uint64_t *b) {
  int d = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) d += __popcll(a[w] ^ b[w]);
  return d;
}

// number of set bits of s strictly below bit k
template <int W>
__device__ __forceinline__ int count_below(const uint64_t *s, int k) {
  int c = 0;
  const int kw = k >> 6;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t m = w < kw ? ~0ull : (w == kw ? ((1ull << (k & 63)) - 1ull) : 0ull);
    c += __popcll(s[w] & m);
  }
  return c;
}

// index of the lowest set bit among W words, -1 if none; clears it in a
// (straight-line over the words, so they stay in registers)
template <int W>
__device__ __forceinline__ int pop_lowest(uint64_t *a) {
  int res = -1;
  bool found = false;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const bool here = !found && a[w] != 0ull;
    const int k = __builtin_ctzll(a[w] | (here ? 0ull : 1ull));
    res = here ? w * 64 + k : res;
    a[w] = here ? (a[w] & (a[w] - 1ull)) : a[w];
    found = found || here;
  }
  return res;
}

// (every word is touched with a constant index, so the words stay in
// registers: a variable index would put the array in scratch memory)
template <int W>
__device__ __forceinline__ void clear_bit(uint64_t *s, int k) {
  const int kw = k >> 6;
  const uint64_t m = 1ull << (k & 63);
#pragma unroll
  for (int w = 0; w < W; ++w) s[w] &= w == kw ? ~m : ~0ull;
}
template <int W>
__device__ __forceinline__ void set_bit(uint64_t *s, int k) {
  const int kw = k >> 6;
  const uint64_t m = 1ull << (k & 63);
#pragma unroll
  for (int w = 0; w < W; ++w) s[w] |= w == kw ? m : 0ull;
}

// Phase of a+_p a_h acting on ket bits s (h occupied, p empty): each operator
// contributes (-1)^(occupied below its mode) in the state it acts on.
template <int W>
__device__ __forceinline__ int sign_single(const uint64_t *s, int p, int h) {
  uint64_t t[W];
#pragma unroll
  for (int w = 0; w < W; ++w) t[w] = s[w];
  int e = count_below<W>(t, h);
  clear_bit<W>(t, h);
  e += count_below<W>(t, p);
  return (e & 1) ? -1 : 1;
}

// Phase of a+_p1 a+_p2 a_h2 a_h1 on ket bits s (p1 < p2, h1 < h2).
template <int W>
__device__ __forceinline__ int sign_double(const uint64_t *s, int p1, int p2, int h1, int h2) {
  uint64_t t[W];
#pragma unroll
  for (int w = 0; w < W; ++w) t[w] = s[w];
  int e = count_below<W>(t, h1);
  clear_bit<W>(t, h1);
  e += count_below<W>(t, h2);
  clear_bit<W>(t, h2);
  e += count_below<W>(t, p2) + count_below<W>(t, p1);
  return (e & 1) ? -1 : 1;
}

}  // namespace dev
}  // namespace cib
