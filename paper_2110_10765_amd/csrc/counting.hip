// State-counting test (Sec. 2.1, Listing 2 as a description; the paper's
// counting experiment): for each of n many-body states of N particles, the
// number of states of the same list (itself included) that a two-body
// operator connects, i.e. that differ from it in at most two particles.
// Three methods, which must agree:
//   0  the hybrid representation: a bit string of the lowest 64
//      single-particle states as a prefilter (its xor popcount is a lower
//      bound of the full one, so > 4 rejects), then count_difference on the
//      index tuples for the pairs that pass;
//   1  count_difference on the index tuples for every pair;
//   2  popcount of the xor of the full 128-bit bit strings (n_sp <= 128).
// count_difference of two tuples of N distinct indices is 2 (N - |a ∩ b|)
// (what the merge of Listing 1 returns); the intersection is counted here by
// comparing every entry of one tuple with every entry of the other, fully
// unrolled, which has no data-dependent loop for a wave to diverge on.
//
// Layout: one thread per row state (kept in registers), the workgroup's
// columns staged through LDS 256 at a time and read by all lanes at the
// same address (broadcast); each workgroup covers a slab of 8192 columns so
// n = 2^17 gives 8192 workgroups.  Per-row counts are added with integer
// atomics (exact in any order).
#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {

constexpr int kCountMaxN = 20;      // particles per state
constexpr int kCountThreads = 256;  // row states per workgroup
constexpr int kCountSlab = 8192;    // column states per workgroup
constexpr int kCountChunk = 256;    // column states per LDS stage

struct CountState {
  uint64_t lo, hi;                  // bits of single-particle states 0..63, 64..127
  uint32_t m[kCountMaxN / 2];       // index tuple, two 16-bit entries per word
};

// Entries past N: 0xfffe in the stored tuples, 0xffff in a row's unpacked
// copy, so padding never matches (indices are below 0xfffe).
__global__ void k_count_encode(int64_t n, int N, const uint16_t *__restrict__ mbs, CountState *__restrict__ st) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  CountState s;
  s.lo = s.hi = 0;
  for (int w = 0; w < kCountMaxN / 2; ++w) s.m[w] = 0xfffefffeu;
  for (int k = 0; k < N; ++k) {
    const uint32_t x = mbs[i * N + k];
    if (x < 64) s.lo |= 1ull << x;
    else if (x < 128) s.hi |= 1ull << (x - 64);
    const int sh = 16 * (k & 1);
    s.m[k >> 1] = (s.m[k >> 1] & ~(0xffffu << sh)) | (x << sh);
  }
  st[i] = s;
}

// |a ∩ b| for a row tuple a (unpacked) and a column tuple b (packed), over
// the first NP entries of each.
template <int NP>
__device__ __forceinline__ int intersect(const uint32_t *a, const uint32_t *bw) {
  int c = 0;
#pragma unroll
  for (int w = 0; w < NP / 2; ++w) {
    const uint32_t b0 = bw[w] & 0xffffu, b1 = bw[w] >> 16;
#pragma unroll
    for (int k = 0; k < NP; ++k) c += (a[k] == b0) + (a[k] == b1);
  }
  return c;
}

template <int METHOD, int NP>
__global__ __launch_bounds__(kCountThreads) void k_count_pairs(int64_t n, int N, const CountState *__restrict__ st,
                                                               int32_t *__restrict__ counts) {
  __shared__ CountState cs[kCountChunk];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kCountThreads + t;
  const int64_t j0 = (int64_t)blockIdx.y * kCountSlab;
  const int64_t j1 = j0 + kCountSlab < n ? j0 + kCountSlab : n;
  const CountState me = st[i < n ? i : n - 1];
  uint32_t a[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const uint32_t x = (me.m[k >> 1] >> (16 * (k & 1))) & 0xffffu;
    a[k] = k < N ? x : 0xffffu;
  }
  int cnt = 0;
  for (int64_t c0 = j0; c0 < j1; c0 += kCountChunk) {
    __syncthreads();   // the previous stage has been read
    if (c0 + t < j1) cs[t] = st[c0 + t];
    __syncthreads();
    const int nc = (int)(j1 - c0 < kCountChunk ? j1 - c0 : kCountChunk);
    for (int c = 0; c < nc; ++c) {
      bool conn;
      if constexpr (METHOD == 2) {
        conn = __popcll(me.lo ^ cs[c].lo) + __popcll(me.hi ^ cs[c].hi) <= 4;
      } else {
        conn = false;
        if (METHOD == 1 || __popcll(me.lo ^ cs[c].lo) <= 4) conn = intersect<NP>(a, cs[c].m) >= N - 2;
      }
      cnt += conn;
    }
  }
  if (i < n && cnt) atomicAdd(&counts[i], cnt);
}

// total = sum of the n counts (one workgroup, integer sums)
__global__ __launch_bounds__(256) void k_count_total(int64_t n, const int32_t *__restrict__ counts,
                                                    int64_t *__restrict__ total) {
  __shared__ int64_t s[256];
  int64_t acc = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += counts[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = s[0];
}

template <int METHOD>
static void launch_count(int NP, dim3 g, hipStream_t s, int64_t n, int N, const CountState *st, int32_t *counts) {
  const dim3 b(kCountThreads);
  switch (NP) {
    case 4: hipLaunchKernelGGL((k_count_pairs<METHOD, 4>), g, b, 0, s, n, N, st, counts); break;
    case 8: hipLaunchKernelGGL((k_count_pairs<METHOD, 8>), g, b, 0, s, n, N, st, counts); break;
    case 12: hipLaunchKernelGGL((k_count_pairs<METHOD, 12>), g, b, 0, s, n, N, st, counts); break;
    case 16: hipLaunchKernelGGL((k_count_pairs<METHOD, 16>), g, b, 0, s, n, N, st, counts); break;
    default: hipLaunchKernelGGL((k_count_pairs<METHOD, 20>), g, b, 0, s, n, N, st, counts); break;
  }
}

// ---------------------------------------------------------- no allocation
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the same
// kernels with their scratch (encoded states, per-state counts, the total)
// in one static device array.  Host code never names the array in a launch
// or a copy: its address on each device is looked up once, with that device
// current, and kept per device.
constexpr int64_t kStaticCountStates = int64_t(1) << 17;
constexpr size_t kStaticCountBytes =
    (size_t)kStaticCountStates * sizeof(CountState) + (size_t)kStaticCountStates * sizeof(int32_t) + 256;
static __device__ __align__(256) unsigned char scratch[kStaticCountBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

void static_scratch_init(int device) {
  CIB_REQUIRE(device >= 0 && device < kMaxDevices, CIB_E_INVALID, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  int cur = -1;
  CIB_HIP(hipGetDevice(&cur));
  CIB_REQUIRE(cur == device, CIB_E_DEVICE, "static scratch set-up needs its device current");
  void *ptr = nullptr;
  CIB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  CIB_REQUIRE(ptr != nullptr, CIB_E_DEVICE, "hipGetSymbolAddress returned no address for the static scratch");
  g_scratch_ptr[device] = ptr;
}

__global__ void k_fill_i32(int64_t n, int32_t *__restrict__ p, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int64_t static_count_max_states() { return kStaticCountStates; }

void count_pairs_static(int device, const uint16_t *mbs, int64_t n, int N, int method, int32_t *counts,
                        int64_t *total, hipStream_t s) {
  CIB_REQUIRE(n <= kStaticCountStates, CIB_E_INVALID,
              "n exceeds the static scratch (" + std::to_string(kStaticCountStates) + " states)");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    base = device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
  }
  CIB_REQUIRE(base, CIB_E_DEVICE, "static scratch was not set up on this device");
  char *b = static_cast<char *>(base);
  CountState *st = reinterpret_cast<CountState *>(b);
  int32_t *own = reinterpret_cast<int32_t *>(b + (size_t)kStaticCountStates * sizeof(CountState));
  int64_t *tot = reinterpret_cast<int64_t *>(b + (size_t)kStaticCountStates * (sizeof(CountState) + sizeof(int32_t)));
  if (!counts) counts = own;
  const dim3 g256((unsigned)((n + 255) / 256));
  hipLaunchKernelGGL(k_count_encode, g256, dim3(256), 0, s, n, N, mbs, st);
  // every call starts from zero counts: the array keeps the last call's values
  hipLaunchKernelGGL(k_fill_i32, g256, dim3(256), 0, s, n, counts, 0);
  const int NP = (N + 3) / 4 * 4;
  const dim3 g((unsigned)((n + kCountThreads - 1) / kCountThreads), (unsigned)((n + kCountSlab - 1) / kCountSlab));
  if (method == 0) launch_count<0>(NP, g, s, n, N, st, counts);
  else if (method == 1) launch_count<1>(NP, g, s, n, N, st, counts);
  else launch_count<2>(NP, g, s, n, N, st, counts);
  hipLaunchKernelGGL(k_count_total, dim3(1), dim3(256), 0, s, n, counts, tot);
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipMemcpyAsync(total, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  CIB_HIP(hipStreamSynchronize(s));
}

void count_pairs(cib_ctx *ctx, const uint16_t *mbs, int64_t n, int N, int method, int32_t *counts, int64_t *total,
                 hipStream_t s) {
  UnwindFence fence(s);
  DBuf<CountState> st(ctx, (size_t)n);
  DBuf<int32_t> own;
  if (!counts) {
    own.reset(ctx, (size_t)n);
    counts = own.p;
  }
  DBuf<int64_t> tot(ctx, 1);
  hipLaunchKernelGGL(k_count_encode, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, N, mbs, st.p);
  CIB_HIP(hipMemsetAsync(counts, 0, (size_t)n * sizeof(int32_t), s));
  const int NP = (N + 3) / 4 * 4;
  const dim3 g((unsigned)((n + kCountThreads - 1) / kCountThreads), (unsigned)((n + kCountSlab - 1) / kCountSlab));
  {
    KTimer kt(ctx, K_COUNT, s);
    if (method == 0) launch_count<0>(NP, g, s, n, N, st.p, counts);
    else if (method == 1) launch_count<1>(NP, g, s, n, N, st.p, counts);
    else launch_count<2>(NP, g, s, n, N, st.p, counts);
  }
  hipLaunchKernelGGL(k_count_total, dim3(1), dim3(256), 0, s, n, counts, tot.p);
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipMemcpyAsync(total, tot.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  CIB_HIP(hipStreamSynchronize(s));
}

}  // namespace cib
