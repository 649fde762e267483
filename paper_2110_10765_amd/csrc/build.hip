// Hamiltonian construction on the device (Fig. 1 steps 1-14 of the paper).
//
// Two-level screen.  Every state is a pair (alpha, beta) of one species-A and
// one species-B configuration, and popcount(BIN_i ^ BIN_j) is the sum of the
// A and B popcounts, so the popcount(xor) <= 4 screen of Sec. 2.1 factorises:
//   * tiles: A-configuration pairs (alpha, alpha') with popcount <= 4
//     (kA = popcount/2 orbitals differ); the analogue of the tile screen over
//     many-body basis orbitals of Fig. 1 steps 2-5;
//   * adjacency: B-configuration pairs with popcount <= 4 in the same 2M_B
//     list (used inside an A-block) and popcount <= 2 in any list (used by
//     kA = 1 tiles); kA = 2 tiles pair each state with the same B position.
// Per-pair phases and matrix elements that depend on one species only are
// computed once per tile / adjacency entry; the per-row passes only combine
// them.  Counting pass -> exclusive scan -> filling pass, one wave per row,
// lanes over tiles, ballot/scan compaction: the columns of a row come out in
// ascending order without atomics (Sec. 2.2-2.3).
#include <algorithm>
#include <functional>
#include <initializer_list>
#include <type_traits>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {
using namespace dev;

// ------------------------------------------------------------ table access
// V_{(a,b),(c,d)} from the blocked layout; 0 across 2M blocks and for pairs
// the layout does not store.  The three table reads are independent, so the
// value costs two dependent memory accesses.
__device__ __forceinline__ double v_pair(const int32_t *pidx, const int64_t *prow, int n2,
                                         const double *v, int a, int b, int c, int d) {
  const int pk = pidx[a * n2 + b], qk = pidx[c * n2 + d];
  const int64_t rb = prow[a * n2 + b];
  if ((pk | qk) < 0 || (pk >> 16) != (qk >> 16)) return 0.0;
  return v[rb + (qk & 0xffff)];
}

// Antisymmetrised same-species element Vbar_{(a,x),(c,x)}: V stored for
// ordered pairs, one sign flip per pair that has to be reordered.
__device__ __forceinline__ double vbar_same(const int32_t *pidx, const int64_t *prow, int n,
                                            const double *v, int a, int x, int c) {
  int s = 1, p0 = a, p1 = x, q0 = c, q1 = x;
  if (a > x) { p0 = x; p1 = a; s = -s; }
  if (c > x) { q0 = x; q1 = c; s = -s; }
  return s * v_pair(pidx, prow, n, v, p0, p1, q0, q1);
}

__device__ __forceinline__ double vab(const DevInter &it, int a, int b, int c, int d) {
  return v_pair(it.pidxAB, it.prowAB, it.nB, it.vAB, a, b, c, d);
}

template <int W>
__device__ __forceinline__ void load_bits(const uint64_t *soa, int64_t n, int64_t k, uint64_t *out) {
#pragma unroll
  for (int w = 0; w < W; ++w) out[w] = soa[(int64_t)w * n + k];
}

// ------------------------------------------------------------ basis expansion
template <int W>
__global__ __launch_bounds__(256) void k_expand_basis(int64_t D, int nA, int nB, int WA, int WB,
                                                      const int64_t *__restrict__ a_off,
                                                      const int32_t *__restrict__ a_seg,
                                                      const int32_t *__restrict__ bseg_start,
                                                      const uint64_t *__restrict__ a_bits,
                                                      const uint64_t *__restrict__ b_bits,
                                                      uint64_t *__restrict__ words,
                                                      int32_t *__restrict__ row_a,
                                                      int32_t *__restrict__ row_p,
                                                      int32_t *__restrict__ row_b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  int lo = 0, hi = nA;  // largest alpha with a_off[alpha] <= i
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a_off[mid] <= i) lo = mid; else hi = mid;
  }
  const int p = (int)(i - a_off[lo]);
  const int beta = bseg_start[a_seg[lo]] + p;
  row_a[i] = lo;
  row_p[i] = p;
  row_b[i] = beta;
  for (int w = 0; w < WA; ++w) words[(int64_t)w * D + i] = a_bits[(int64_t)w * nA + lo];
  for (int w = 0; w < WB; ++w) words[(int64_t)(WA + w) * D + i] = b_bits[(int64_t)w * nB + beta];
}

// ------------------------------------------------------------ configuration energies
// E(config) = sum_a eps_a + sum_{a<b in config} V_{ab,ab} (diagonal of one species)
template <int W>
__global__ __launch_bounds__(256) void k_config_energy(int n, const uint64_t *__restrict__ bits,
                                                       const double *__restrict__ eps,
                                                       const int32_t *pidx, const int64_t *prow,
                                                       int norb, const double *v,
                                                       double *__restrict__ e) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint64_t s[W];
  load_bits<W>(bits, n, k, s);
  double acc = 0.0;
  uint64_t t[W];
#pragma unroll
  for (int w = 0; w < W; ++w) t[w] = s[w];
  for (int a = pop_lowest<W>(t); a >= 0; a = pop_lowest<W>(t)) {
    acc += eps[a];
    uint64_t u[W];
#pragma unroll
    for (int w = 0; w < W; ++w) u[w] = t[w];
    for (int b = pop_lowest<W>(u); b >= 0; b = pop_lowest<W>(u))
      acc += v_pair(pidx, prow, norb, v, a, b, a, b);
  }
  e[k] = acc;
}

__global__ void k_dab(DevInter it, double *dab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= it.nA * it.nB) return;
  const int x = k / it.nB, y = k % it.nB;
  dab[k] = vab(it, x, y, x, y);
}

// One thread per entry of the transition table: find the entry's block, its
// A transition (row) and B transition (column), read V^AB from the blocked
// pair table.
__global__ void k_build_vt(DevInter it, const VtBlock *blk, int nblk, const int32_t *atr,
                           const int32_t *btr, int64_t total, double *vt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  int g = 0;
  while (g + 1 < nblk && blk[g + 1].base <= e) ++g;
  const VtBlock B = blk[g];
  const int64_t r = e - B.base;
  const int32_t ta = atr[B.a0 + (int)(r / B.nb)], tb = btr[B.b0 + (int)(r % B.nb)];
  vt[e] = vab(it, ta >> 16, tb >> 16, ta & 0xffff, tb & 0xffff);
}

// V^AB_{(a,b),(c,d)} through the transition table (row base of a <- c from
// the tile, column of b <- d from the B adjacency entry).
// (a 32-bit byte offset: the load takes the scalar base and one vector
// register; the table holds far fewer than 2^29 elements)
__device__ __forceinline__ double vt_at(const DevInter &it, int32_t rb, int32_t col) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(it.vt) + (uint32_t)(rb + col) * 8u);
}

// Sum of f(k) over the set bits k of s (at most 64 * W), in ascending k, with
// the table reads of four terms issued before their additions.  Skipped terms
// are not added, so the result equals the plain ascending loop bit for bit.
template <int W, typename F>
__device__ __forceinline__ double sum_over_bits(const uint64_t *s, F f) {
  uint64_t t[W];
#pragma unroll
  for (int w = 0; w < W; ++w) t[w] = s[w];
  double sum = 0.0;
  for (;;) {
    const int k0 = pop_lowest<W>(t), k1 = pop_lowest<W>(t), k2 = pop_lowest<W>(t), k3 = pop_lowest<W>(t);
    const double v0 = k0 >= 0 ? f(k0) : 0.0, v1 = k1 >= 0 ? f(k1) : 0.0;
    const double v2 = k2 >= 0 ? f(k2) : 0.0, v3 = k3 >= 0 ? f(k3) : 0.0;
    if (k0 >= 0) sum += v0;
    if (k1 >= 0) sum += v1;
    if (k2 >= 0) sum += v2;
    if (k3 < 0) break;
    sum += v3;
  }
  return sum;
}

// Table offsets of the spectator sums of one row: for each occupied orbital
// x of a configuration, in ascending x, the diagonal transition x <- x in the
// table's row map (A) or column map (B).  Written once per row to the wave's
// LDS slots, so a sum then issues all its table reads at once.  Slots past
// the occupation hold map[0] (reads stay in bounds and are not added); more
// than kSpec occupied orbitals fall back to the loop over the bits.
constexpr int kSpec = 8;
struct SpecIdx {
  int n;
  const int32_t *r;   // LDS, kSpec slots, 16-byte aligned
};

template <int W>
__device__ __forceinline__ SpecIdx spec_idx(const uint64_t *bits, const int32_t *map, int nmap, int32_t *slot) {
  const int lane = lane_id();
  if (lane < kSpec) slot[lane] = map[0];
  int below = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const uint64_t t = uni(bits[w]);
    const int x = w * kWave + lane;
    const int rank = below + (int)__popcll(t & ((1ull << lane) - 1));
    if (x < nmap && ((t >> lane) & 1) && rank < kSpec) slot[rank] = map[x * (nmap + 1)];
    below += (int)__popcll(t);
  }
  wave_lds_sync();
  return SpecIdx{below, slot};
}

// sum over the occupied orbitals of f(offset), ascending, as sum_over_bits
template <int W, typename F>
__device__ __forceinline__ double spec_sum(const SpecIdx &s, const uint64_t *bits, const int32_t *map, int nmap,
                                           F f) {
  if (s.n > kSpec) return sum_over_bits<W>(bits, [&](int x) { return f(map[x * (nmap + 1)]); });
  double sum = 0.0;
#pragma unroll
  for (int k0 = 0; k0 < kSpec; k0 += 4) {
    if (k0 >= s.n) break;
    const int4 r = *reinterpret_cast<const int4 *>(s.r + k0);
    const double v0 = f(r.x), v1 = f(r.y), v2 = f(r.z), v3 = f(r.w);
    sum += v0;
    if (k0 + 1 < s.n) sum += v1;
    if (k0 + 2 < s.n) sum += v2;
    if (k0 + 3 < s.n) sum += v3;
  }
  return sum;
}

// Diagonal element of every state, E_A(alpha) + E_B(beta) + sum over the
// occupied pairs (x in alpha, y in beta) of V^AB_{(x,y),(x,y)}; one thread
// per state, added in the order the row pass used to add them.
template <int W>
__global__ __launch_bounds__(256) void k_state_diag(int64_t D, const int32_t *__restrict__ row_a,
                                                    const int32_t *__restrict__ row_p,
                                                    const int32_t *__restrict__ a_seg,
                                                    const int32_t *__restrict__ bseg_start,
                                                    const uint64_t *__restrict__ a_bits, int nA,
                                                    const uint64_t *__restrict__ b_bits, int nB,
                                                    const double *__restrict__ eA, const double *__restrict__ eB,
                                                    DevInter it, double *__restrict__ diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= D) return;
  const int alpha = row_a[i];
  const int beta = bseg_start[a_seg[alpha]] + row_p[i];
  double v = eB[beta];
  v += eA[alpha];
  if (it.nB > 0) {
    uint64_t ab[W], bb[W];
    load_bits<W>(a_bits, nA, alpha, ab);
    load_bits<W>(b_bits, nB, beta, bb);
    for (int x = pop_lowest<W>(ab); x >= 0; x = pop_lowest<W>(ab)) {
      uint64_t u[W];
#pragma unroll
      for (int w = 0; w < W; ++w) u[w] = bb[w];
      for (int y = pop_lowest<W>(u); y >= 0; y = pop_lowest<W>(u)) v += it.dab[x * it.nB + y];
    }
  }
  diag[i] = v;
}

// ------------------------------------------------------------ tile screen
// One wave per A configuration alpha; lanes over alpha' > alpha (or < alpha for
// the lower triangle).  Kept: kA = 1, or kA = 2 with equal 2M_A (a kA = 2 pair
// needs identical B configurations).  Tile data are computed with alpha as the
// bra (row) and alpha' as the ket (column).
// One tile (alpha, alpha') as the row passes read it: a single 16-byte load.
// off = first state of alpha' (a CSR column, so below 2^31), len = states of
// alpha', info and rb as written by k_tile_val.
struct alignas(16) TileRec {
  int32_t info, len, off, rb;
};

struct TileArgs {
  int nA;
  int nchunk;             // chunks of 64 candidate configurations (the tile lists' stride)
  int ngroup, gsz;        // groups of gsz <= 64 configurations alpha, one wave per (chunk, group)
  const uint64_t *a_bits;
  const int32_t *a_m2, *a_len, *a_seg;
  const int64_t *a_off;
  DevInter it;
  int32_t *tcnt;          // count pass: per unit
  const int64_t *t_ptr;   // fill pass: per unit
  TileRec *t_rec;         // fill pass: off and len of every tile
  int32_t *t_src, *t_dst;   // fill pass: (alpha, alpha') of every tile
};

// Phase, info and value of one tile, alpha the bra (row) and alpha' the ket
// (column): kA = 1 (p <- h, spectators in common): info = 1 | p << 2 | h << 10
// | phase bit << 18 | 2M list of alpha' << 19, value = phase x AA spectator
// sum, rb = row base of p <- h in the V^AB transition table; kA = 2: info 2,
// value = phase x pair element.
template <int W>
__global__ __launch_bounds__(256) void k_tile_val(int64_t n, const int32_t *__restrict__ src,
                                                  const int32_t *__restrict__ dst,
                                                  const uint64_t *__restrict__ a_bits, int nAc,
                                                  const int32_t *__restrict__ a_seg, DevInter it,
                                                  TileRec *__restrict__ t_rec, double *__restrict__ t_val,
                                                  const int32_t *__restrict__ a_q, int qcap) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int alpha = src[e], j = dst[e];
  uint64_t ra[W], ca[W], part[W], hole[W], common[W];
  load_bits<W>(a_bits, nAc, alpha, ra);
  load_bits<W>(a_bits, nAc, j, ca);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    part[w] = ra[w] & ~ca[w];
    hole[w] = ca[w] & ~ra[w];
    common[w] = ra[w] & ca[w];
  }
  const int p1 = pop_lowest<W>(part), h1 = pop_lowest<W>(hole);
  const int p2 = pop_lowest<W>(part), h2 = pop_lowest<W>(hole);
  int info, rb = 0;
  double val;
  if (p2 < 0) {  // kA = 1
    const int sg = sign_single<W>(ca, p1, h1);
    const double sum = sum_over_bits<W>(
        common, [&](int x) { return vbar_same(it.pidxA, it.prowA, it.nA, it.vA, p1, x, h1); });
    val = sg * sum;
    info = 1 | (p1 << 2) | (h1 << 10) | ((sg < 0) << 18) | (a_seg[j] << 19);
    rb = it.arb ? it.arb[p1 * it.nA + h1] : 0;
    // a kA = 1 tile keeps, in place of alpha''s length, the Q level its B
    // states stop at (qcap - Q_A(alpha'), qcap = qmax - qmin_B; 0 without a
    // truncation): its entries are the L1 entries of the row's B
    // configuration in alpha''s 2M_B list up to that level
    t_rec[e].len = qcap >= 0 ? qcap - a_q[j] : 0;
  } else {       // kA = 2
    const int sg = sign_double<W>(ca, p1, p2, h1, h2);
    val = sg * v_pair(it.pidxA, it.prowA, it.nA, it.vA, p1, p2, h1, h2);
    info = 2;
  }
  t_rec[e].info = info;
  t_rec[e].rb = rb;
  t_val[e] = val;
}

// One wave per (chunk of 64 candidate configurations alpha', group of up
// to 64 configurations alpha), restricted to alpha' > alpha (upper) or
// alpha' < alpha (LOWER): the lanes hold the candidates, the wave takes the
// group's configurations one after another (their bits and 2M read once,
// coalesced, and broadcast from a lane).  The count pass writes the count of
// every (alpha, chunk), alpha-major, so that their scan lists each
// alpha's tiles in ascending alpha' (alpha's tiles at [t_ptr[alpha *
// nchunk], t_ptr[(alpha + 1) * nchunk])).  (A wave per (alpha, 256
// candidates) instead waited on its setup reads.)
template <int W, bool FILL, bool LOWER>
__global__ __launch_bounds__(256) void k_tile_pass(TileArgs g) {
  const int64_t unit = blockIdx.x * (int64_t)(blockDim.x / kWave) + uni((int)(threadIdx.x >> 6));
  if (unit >= (int64_t)g.nchunk * g.ngroup) return;
  const int q = (int)(unit / g.ngroup), bg = (int)(unit % g.ngroup);
  const int lane = lane_id();
  const int j = q * kWave + lane;
  const bool jv = j < g.nA;
  const int a0 = bg * g.gsz, na = min(g.gsz, g.nA - a0);
  // lane k: alpha = a0 + k
  const int al = min(a0 + lane, g.nA - 1);
  const int64_t cell = (int64_t)al * g.nchunk + q;
  // no candidate of the chunk is on the wanted side of any alpha of the
  // group: zero counts (count pass) or nothing to write
  if (LOWER ? q * kWave >= a0 + na - 1 : q * kWave + kWave - 1 <= a0) {
    if (!FILL && lane < na) g.tcnt[cell] = 0;
    return;
  }
  uint64_t cb[W], vb[W];
  load_bits<W>(g.a_bits, g.nA, jv ? j : 0, cb);
  const int cm = g.a_m2[jv ? j : 0];
  load_bits<W>(g.a_bits, g.nA, al, vb);
  const int vm = g.a_m2[al];
  int64_t vo = 0;
  int32_t coff = 0, clen = 0;
  if (FILL) {
    vo = g.t_ptr[cell];
    coff = (int32_t)g.a_off[jv ? j : 0];
    clen = g.a_len[jv ? j : 0];
  }
  int my = 0;
  for (int k = 0; k < na; ++k) {
    const int alpha = a0 + k;
    uint64_t ra[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t lo32 = __builtin_amdgcn_readlane((int)(uint32_t)vb[w], k);
      const uint32_t hi32 = __builtin_amdgcn_readlane((int)(uint32_t)(vb[w] >> 32), k);
      ra[w] = (uint64_t)hi32 << 32 | lo32;
    }
    const int m = __builtin_amdgcn_readlane(vm, k);
    bool ok = false;
    if (jv && (LOWER ? j < alpha : j > alpha)) {
      const int d = popc_xor<W>(ra, cb);
      ok = d <= 2 || (d == 4 && cm == m);
    }
    const uint64_t msk = ballot(ok);
    if constexpr (!FILL) {
      if (lane == k) my = __popcll(msk);
    } else if (ok) {
      const int64_t o = readlane_i64(vo, k) + mask_rank(msk);
      g.t_rec[o].off = coff;
      g.t_rec[o].len = clen;
      g.t_src[o] = alpha;
      g.t_dst[o] = j;
    }
  }
  if (!FILL && lane < na) g.tcnt[cell] = my;
}

// ------------------------------------------------------------ B adjacency
// One wave per unit (beta, segment h).  Lsame(beta): beta' in beta's own 2M_B
// list with popcount <= 4, ascending position; carries the B-only value part.
// L1(beta): beta' in any list with popcount <= 2, grouped by list, ascending.
// A list whose 2M_B differs from beta's by more than one orbital change can
// shift it (max_dm) holds no L1 entry and is not scanned.  Entry info:
// orbitals changed (0, 1, 2) | phase bit << 2 | (one change b <- d) the column
// of b <- d in the V^AB transition table << 3.
// One B adjacency entry as the row passes read it (one 8-byte load): pos =
// position of beta' in its 2M_B list, info as written by k_adj_val.
struct alignas(8) AdjRec {
  int32_t pos, info;
};

struct AdjArgs {
  int nB, nseg, nchunk, ngroup, gsz;   // chunks of 64 configurations over all lists; groups of gsz <= 64 B configurations
  const uint64_t *b_bits;
  const int32_t *b_seg, *bseg_start;
  const int32_t *chunk_list, *coff;   // list of every chunk; first chunk of every list (nseg + 1)
  const int32_t *ls_base;             // first Lsame cell of every beta (its own list's chunks), nB + 1
  int32_t *ls_cnt, *l1_cnt;           // count pass: per (beta, own-list chunk); per (beta, chunk), beta-major
  const int64_t *ls_off, *l1_off;     // fill pass: their exclusive scans
  int32_t *ls_self;
  AdjRec *ls_rec, *l1_rec;                      // fill pass: pos of every entry
  int32_t *ls_src, *ls_dst, *l1_src, *l1_dst;   // (beta, beta') of every entry
};

// Phase, value and table column of one B adjacency entry (beta bra, beta'
// ket).  Entry info: orbitals changed (0, 1, 2) | phase bit << 2 | (one
// change b <- d) the column of b <- d in the V^AB transition table << 3.
// The value is the B-only part: E_B for beta' = beta, the spectator sum for
// one change, the pair element for two.
template <int W>
__global__ __launch_bounds__(256) void k_adj_val(int64_t n, const int32_t *__restrict__ src,
                                                 const int32_t *__restrict__ dst,
                                                 const uint64_t *__restrict__ b_bits, int nBc,
                                                 const double *__restrict__ eB, DevInter it,
                                                 AdjRec *__restrict__ rec_out, double *__restrict__ val_out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int beta = src[e], bj = dst[e];
  uint64_t rb[W], cb[W], part[W], hole[W], common[W];
  load_bits<W>(b_bits, nBc, beta, rb);
  load_bits<W>(b_bits, nBc, bj, cb);
  int d = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    part[w] = rb[w] & ~cb[w];
    hole[w] = cb[w] & ~rb[w];
    common[w] = rb[w] & cb[w];
    d += __popcll(part[w]);
  }
  const int p1 = pop_lowest<W>(part), h1 = pop_lowest<W>(hole);
  const int p2 = pop_lowest<W>(part), h2 = pop_lowest<W>(hole);
  int info = 0;
  double val = 0.0;
  if (d == 0) {
    val = eB[beta];
  } else if (d == 1) {
    const int sg = sign_single<W>(cb, p1, h1);
    info = 1 | ((sg < 0) << 2) | ((it.bcol ? it.bcol[p1 * it.nB + h1] : 0) << 3);
    if (val_out) {
      const double sum = sum_over_bits<W>(
          common, [&](int y) { return vbar_same(it.pidxB, it.prowB, it.nB, it.vB, p1, y, h1); });
      val = sg * sum;
    }
  } else {
    const int sg = sign_double<W>(cb, p1, p2, h1, h2);
    info = 2;
    if (val_out) val = sg * v_pair(it.pidxB, it.prowB, it.nB, it.vB, p1, p2, h1, h2);
  }
  rec_out[e].info = info;
  if (val_out) val_out[e] = val;
}

// lev_cnt[(beta * nseg + h) * nlev + t] = number of the L1 entries of B
// configuration beta in 2M_B list h whose Q_B is at most qmin_B + t (the
// list is ordered by Q_B, so they are a prefix of the segment).  One thread
// per entry: the last entry of each Q level writes the counts of the levels
// from its own up to the next entry's, the first entry of a segment the
// zeros below it (a segment without entries keeps the zeros it was cleared
// to).  The row passes read a kA = 1 tile's entry count here instead of
// searching the segment for the tile's length.
__global__ __launch_bounds__(256) void k_l1_levels(int64_t n, int nseg, int nlev, int qminB,
                                                   const int64_t *__restrict__ l1_seg,
                                                   const int32_t *__restrict__ l1_src,
                                                   const int32_t *__restrict__ l1_dst,
                                                   const int32_t *__restrict__ b_seg,
                                                   const int32_t *__restrict__ b_q, int32_t *__restrict__ lev_cnt,
                                                   int nB, int32_t *__restrict__ lev_t) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int dst = l1_dst[e];
  const int64_t u = (int64_t)l1_src[e] * nseg + b_seg[dst];
  const int64_t e0 = l1_seg[u], e1 = l1_seg[u + 1];
  const int lev = nlev > 1 ? b_q[dst] - qminB : 0;
  const int next = e + 1 < e1 ? (nlev > 1 ? b_q[l1_dst[e + 1]] - qminB : 0) : nlev;
  int32_t *out = lev_cnt + u * nlev;
  if (e == e0)
    for (int t = 0; t < lev; ++t) out[t] = 0;
  for (int t = lev; t < next; ++t) out[t] = (int32_t)(e - e0 + 1);
  if (lev_t) {   // the same counts bin-major: lev_t[((h * nlev) + t) * nB + beta]
    const int beta = l1_src[e], h = (int)(u - (int64_t)beta * nseg);
    int32_t *ot = lev_t + (int64_t)h * nlev * nB + beta;
    if (e == e0)
      for (int t = 0; t < lev; ++t) ot[(int64_t)t * nB] = 0;
    for (int t = lev; t < next; ++t) ot[(int64_t)t * nB] = (int32_t)(e - e0 + 1);
  }
}

// One wave per (chunk of 64 configurations of one 2M_B list, group of up to
// 64 B configurations beta): the lanes hold the chunk's candidates beta', and the
// wave takes the group's configurations one after another (their bits and
// lists read once, coalesced, and broadcast from a lane).  Lsame(beta):
// beta' in beta's own list with popcount <= 4; L1(beta): beta' in any list
// with popcount <= 2.  The count pass writes the L1 count of every (beta,
// chunk), beta-major, and the Lsame count of every chunk of beta's own
// list, so that their scans place every chunk's entries: the entries of
// beta come out grouped by list, ascending position.  (A wave per
// (beta, list) instead waited on its setup reads: 145 K short waves at D =
// 198,912.)
template <int W, bool FILL>
__global__ __launch_bounds__(256) void k_adj_pass(AdjArgs g) {
  const int64_t unit = blockIdx.x * (int64_t)(blockDim.x / kWave) + uni((int)(threadIdx.x >> 6));
  if (unit >= (int64_t)g.nchunk * g.ngroup) return;
  const int q = (int)(unit / g.ngroup), bg = (int)(unit % g.ngroup);
  const int lane = lane_id();
  const int h = uni(g.chunk_list[q]);
  const int lo = uni(g.bseg_start[h]), hi = uni(g.bseg_start[h + 1]);
  const int j = lo + (q - uni(g.coff[h])) * kWave + lane;
  const bool jv = j < hi;
  uint64_t cb[W];
  load_bits<W>(g.b_bits, g.nB, jv ? j : lo, cb);
  const int b0 = bg * g.gsz, nb = min(g.gsz, g.nB - b0);
  // lane k: the bits, list and (fill pass) output offsets of beta = b0 + k
  const int bl = min(b0 + lane, g.nB - 1);
  uint64_t vb[W];
  load_bits<W>(g.b_bits, g.nB, bl, vb);
  const int vseg = g.b_seg[bl];
  const int64_t cell = (int64_t)bl * g.nchunk + q;
  const int64_t lcell = g.ls_base[bl] + (q - uni(g.coff[h]));   // (a cell only where vseg == h)
  int64_t vls = 0, vl1 = 0;
  if (FILL) {
    vls = vseg == h ? g.ls_off[lcell] : 0;
    vl1 = g.l1_off[cell];
  }
  int my_ls = 0, my_l1 = 0;
  for (int k = 0; k < nb; ++k) {
    uint64_t rb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t lo32 = __builtin_amdgcn_readlane((int)(uint32_t)vb[w], k);
      const uint32_t hi32 = __builtin_amdgcn_readlane((int)(uint32_t)(vb[w] >> 32), k);
      rb[w] = (uint64_t)hi32 << 32 | lo32;
    }
    const bool own = __builtin_amdgcn_readlane(vseg, k) == h;
    const int d = jv ? popc_xor<W>(rb, cb) : 99;
    const bool in_ls = own && d <= 4, in_l1 = d <= 2;
    const uint64_t m_ls = ballot(in_ls), m_l1 = ballot(in_l1);
    if constexpr (!FILL) {
      if (lane == k) {
        my_ls = __popcll(m_ls);
        my_l1 = __popcll(m_l1);
      }
    } else {
      const int beta = b0 + k;
      if (in_ls) {
        const int64_t o = readlane_i64(vls, k) + mask_rank(m_ls);
        g.ls_rec[o].pos = j - lo;
        g.ls_src[o] = beta;
        g.ls_dst[o] = j;
        if (j == beta) g.ls_self[beta] = (int32_t)o;
      }
      if (in_l1) {
        const int64_t o = readlane_i64(vl1, k) + mask_rank(m_l1);
        g.l1_rec[o].pos = j - lo;
        g.l1_src[o] = beta;
        g.l1_dst[o] = j;
      }
    }
  }
  if (!FILL && lane < nb) {
    if (vseg == h) g.ls_cnt[lcell] = my_ls;
    g.l1_cnt[cell] = my_l1;
  }
}

// The per-(beta, list) starts of the L1 lists and the per-beta starts of the
// Lsame lists, from the per-(beta, chunk) scans (a list without chunks
// starts where the next one does).  Also zeroes the level-count tables that
// k_l1_levels and k_ls_levels fill later (nlev values per (beta, list), and
// per beta; lev_t and ls_lev may be null), so that no fill is queued
// between the build's kernels.
__global__ __launch_bounds__(256) void k_adj_offsets(int nB, int nseg, int nchunk, const int32_t *__restrict__ coff,
                                                     const int32_t *__restrict__ ls_base,
                                                     const int64_t *__restrict__ ls_off,
                                                     const int64_t *__restrict__ l1_off, int64_t *__restrict__ ls_ptr,
                                                     int64_t *__restrict__ l1_seg, int nlev,
                                                     int32_t *__restrict__ lev_cnt, int32_t *__restrict__ lev_t,
                                                     int32_t *__restrict__ ls_lev) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nB * nseg;
  if (e < n) {
    for (int t = 0; t < nlev; ++t) {
      lev_cnt[e * nlev + t] = 0;
      if (lev_t) lev_t[e * nlev + t] = 0;
    }
    if (ls_lev && e < nB)
      for (int t = 0; t < nlev; ++t) ls_lev[e * nlev + t] = 0;
    const int beta = (int)(e / nseg), h = (int)(e % nseg);
    l1_seg[e] = l1_off[(int64_t)beta * nchunk + coff[h]];
    if (h == 0) ls_ptr[beta] = ls_off[ls_base[beta]];
  } else if (e == n) {
    l1_seg[n] = l1_off[(int64_t)nB * nchunk];
    ls_ptr[nB] = ls_off[ls_base[nB]];
  }
}

// ------------------------------------------------------------ row counts
// A row's entry counts depend on its A configuration only through alpha's
// tiles, and on its B configuration only through the level tables:
//   kA = 1 tiles: sum over (2M_B list g, Q level t) of [alpha's kA = 1
//     tiles in (g, t)] x lev_cnt[beta][g][t];
//   kA = 2 tiles: alpha's kA = 2 tiles whose length exceeds the row's
//     position p in alpha's block;
//   Lsame: its entries up to alpha's Q level, split at beta itself (those
//     before it are the lower row's, the rest the upper row's).
// tile_hist[(alpha * nseg + g) * nlev + t] counts the first, k2len lists the
// lengths of alpha's kA = 2 tiles from alpha's first tile on (in tile
// order), k2n[alpha] how many.  One wave per alpha: the histogram is added
// up in LDS (integer adds: the result does not depend on their order) and
// written out once; the kA = 2 lengths are compacted with ballots.
constexpr int kHistBins = 2048;   // bins per wave in LDS (nseg x nlev at most this)
__global__ __launch_bounds__(256) void k_tile_hist(int nA, const int64_t *__restrict__ t_ptr, int tstride,
                                                   const TileRec *__restrict__ rec, int nlev, int nbin,
                                                   int32_t *__restrict__ hist, int32_t *__restrict__ k2len,
                                                   int32_t *__restrict__ k2n) {
  __shared__ int32_t h[4][kHistBins];
  const int wv = uni((int)(threadIdx.x >> 6));
  const int alpha = (int)blockIdx.x * 4 + wv;
  if (alpha >= nA) return;   // whole wave
  const int lane = lane_id();
  for (int k = lane; k < nbin; k += kWave) h[wv][k] = 0;
  wave_lds_sync();
  const int64_t t0 = uni(t_ptr[(int64_t)alpha * tstride]), t1 = uni(t_ptr[(int64_t)(alpha + 1) * tstride]);
  int n2 = 0;
  for (int64_t tb = t0; tb < t1; tb += kWave) {
    const int64_t t = tb + lane;
    int4 r = make_int4(0, 0, 0, 0);
    if (t < t1) r = reinterpret_cast<const int4 *>(rec)[t];
    const bool two = t < t1 && (r.x & 3) == 2;
    if (t < t1 && !two) atomicAdd(&h[wv][((r.x >> 19) & 0x7f) * nlev + r.y], 1);   // kA = 1: r.y is the Q level
    const uint64_t m = ballot(two);
    if (two) k2len[t0 + n2 + mask_rank(m)] = r.y;
    n2 += __popcll(m);
  }
  wave_lds_sync();
  for (int k = lane; k < nbin; k += kWave) hist[(int64_t)alpha * nbin + k] = h[wv][k];
  if (lane == 0) k2n[alpha] = n2;
}

// ls_lev[beta * nlev + t] = Lsame entries of beta with Q_B <= qmin_B + t (a
// prefix: the list is ordered by position), one thread per entry, written
// as k_l1_levels writes its table.
__global__ __launch_bounds__(256) void k_ls_levels(int64_t n, int nlev, int qminB, const int64_t *__restrict__ ls_ptr,
                                                   const int32_t *__restrict__ ls_src,
                                                   const int32_t *__restrict__ ls_dst,
                                                   const int32_t *__restrict__ b_q, int32_t *__restrict__ ls_lev) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int beta = ls_src[e];
  const int64_t e0 = ls_ptr[beta], e1 = ls_ptr[beta + 1];
  const int lev = nlev > 1 ? b_q[ls_dst[e]] - qminB : 0;
  const int next = e + 1 < e1 ? (nlev > 1 ? b_q[ls_dst[e + 1]] - qminB : 0) : nlev;
  int32_t *out = ls_lev + (int64_t)beta * nlev;
  if (e == e0)
    for (int t = 0; t < lev; ++t) out[t] = 0;
  for (int t = lev; t < next; ++t) out[t] = (int32_t)(e - e0 + 1);
}

struct CountArgs {
  int nA, nB, nseg, nlev, nbin, qcap, tstride;
  const int32_t *cstart;   // nA + 1: first wave of each A configuration (a wave per 64 rows)
  int64_t nwaves;
  const int64_t *a_off;
  const int32_t *a_len, *a_q, *a_seg, *bseg_start, *ls_self;
  const int64_t *ls_ptr, *t_ptr, *tl_ptr;
  const int32_t *lev_t, *ls_lev;
  const int32_t *hist_u, *hist_l, *k2len_u, *k2len_l, *k2n_u, *k2n_l;
  int32_t *rcnt, *rlcnt;
};

// One wave per (A configuration alpha, 64 rows of its block), a lane per
// row: row a_off[alpha] + p has B configuration bseg_start[a_seg[alpha]] + p,
// so the lanes' B configurations are consecutive and the bin-major level
// table is read coalesced.  alpha's histogram bins are walked in order (the
// empty ones skipped: a uniform branch), its kA = 2 lengths one by one.
constexpr int kCountBins = 4;   // histogram bins per lane kept in registers (nbin <= 256)
__global__ __launch_bounds__(256) void k_row_count_tab(CountArgs c) {
  __shared__ int32_t zb[4][kCountBins * kWave], zu[4][kCountBins * kWave], zl[4][kCountBins * kWave];
  const int wv = uni((int)(threadIdx.x >> 6));
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  if (w >= c.nwaves) return;   // whole wave
  // the A configuration of this wave: last alpha with cstart[alpha] <= w
  int lo = 0, hi = c.nA;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (uni(c.cstart[mid]) <= w) lo = mid; else hi = mid;
  }
  const int alpha = lo, chunk = (int)(w - uni(c.cstart[alpha]));
  const int len = uni(c.a_len[alpha]);
  const int lane = lane_id();
  const int p = chunk * kWave + lane;
  const bool live = p < len;
  const int64_t r0 = uni(c.a_off[alpha]);
  const int beta = uni(c.bseg_start[uni(c.a_seg[alpha])]) + (live ? p : 0);
  // alpha's non-empty bins, listed in LDS in bin order
  const int32_t *hu = c.hist_u + (int64_t)alpha * c.nbin, *hl = c.hist_l + (int64_t)alpha * c.nbin;
  int nz = 0;
#pragma unroll
  for (int q = 0; q < kCountBins; ++q) {
    const int k = q * kWave + lane;
    const int vu = k < c.nbin ? hu[k] : 0, vl = k < c.nbin ? hl[k] : 0;
    const bool use = (vu | vl) != 0;
    const uint64_t m = ballot(use);
    if (use) {
      const int o = nz + mask_rank(m);
      zb[wv][o] = k;
      zu[wv][o] = vu;
      zl[wv][o] = vl;
    }
    nz += __popcll(m);
  }
  wave_lds_sync();
  int su = 0, sl = 0;
  for (int t0 = 0; t0 < nz; t0 += 8) {   // eight table reads in flight, then the products
    int f[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = min(t0 + u, nz - 1);
      f[u] = c.lev_t[(int64_t)zb[wv][t] * c.nB + beta];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (t0 + u < nz) {
        su += zu[wv][t0 + u] * f[u];
        sl += zl[wv][t0 + u] * f[u];
      }
    }
  }
  // kA = 2 tiles: one entry each while p < the length of alpha'
  const int64_t bu = uni(c.t_ptr[(int64_t)alpha * c.tstride]), bl = uni(c.tl_ptr[(int64_t)alpha * c.tstride]);
  const int nu = uni(c.k2n_u[alpha]), nl = uni(c.k2n_l[alpha]);
  for (int k0 = 0; k0 < nu; k0 += kWave) {   // lane k0 + j holds length j; the row's count from a ballot
    const int k = k0 + lane;
    const int lk = k < nu ? c.k2len_u[bu + k] : 0;
    for (int j = 0; j < min(kWave, nu - k0); ++j) su += p < __builtin_amdgcn_readlane(lk, j);
  }
  for (int k0 = 0; k0 < nl; k0 += kWave) {
    const int k = k0 + lane;
    const int lk = k < nl ? c.k2len_l[bl + k] : 0;
    for (int j = 0; j < min(kWave, nl - k0); ++j) sl += p < __builtin_amdgcn_readlane(lk, j);
  }
  if (live) {
    // Lsame: the entries up to alpha's Q level, split at beta itself
    const int lev = c.qcap >= 0 ? c.qcap - uni(c.a_q[alpha]) : 0;
    const int before = (int)(c.ls_self[beta] - c.ls_ptr[beta]);
    c.rcnt[r0 + p] = su + c.ls_lev[(int64_t)beta * c.nlev + lev] - before;
    c.rlcnt[r0 + p] = sl + before;
  }
}

// ------------------------------------------------------------ row passes
struct RowArgs {
  int64_t D;
  int nA, nB, nseg;
  const int32_t *row_a, *row_p, *row_b, *a_seg, *a_len, *bseg_start;
  const int64_t *a_off;
  const uint64_t *a_bits, *b_bits;
  const double *eA;
  const int64_t *t_ptr;   // per tile unit: alpha's tiles at [alpha * tstride, (alpha + 1) * tstride]
  int tstride;
  const TileRec *t_rec;
  const double *t_val;
  const int64_t *ls_ptr, *l1_seg;
  const int32_t *ls_self;
  const AdjRec *ls_rec, *l1_rec;
  const int32_t *lev_cnt;   // k_l1_levels
  int nlev;
  const int32_t *b_q;       // fill pass: Q_B of every B configuration, and its minimum
  int qminB;
  const double *ls_val;
  const double *diag;       // fill pass: diagonal element of every state
  DevInter it;
  int32_t *rcnt;            // count pass
  const int64_t *row_ptr;   // fill pass
  int32_t *col;
  void *val;
};

// The lower triangle's own arrays: its tile lists (the transposed tiles) and
// its outputs.  Everything else it shares with the upper triangle's RowArgs;
// passing only these (and making the lower RowArgs on the device from the
// upper one) keeps one copy of the shared pointers in scalar registers
// instead of two, which the fill kernel could not hold at eight waves per
// SIMD without spilling them to vector lanes.
struct LowerArgs {
  const int64_t *t_ptr;
  const TileRec *t_rec;
  const double *t_val;
  int32_t *rcnt;
  const int64_t *row_ptr;
  int32_t *col;
  void *val;
};

__device__ __forceinline__ RowArgs lower_args(const RowArgs &g, const LowerArgs &l) {
  RowArgs r = g;
  r.t_ptr = l.t_ptr;
  r.t_rec = l.t_rec;
  r.t_val = l.t_val;
  r.rcnt = l.rcnt;
  r.row_ptr = l.row_ptr;
  r.col = l.col;
  r.val = l.val;
  return r;
}

// Where a fill pass sends each entry (column j, value v): NoAcc stores it in
// the CSR arrays; ApplyAcc multiplies it into row j of X (the matrix-free
// product, rounding v to T as the stored matrix would) and keeps the sums of
// the lane's entries in registers.
struct NoAcc {
  static constexpr bool kApply = false;
  __device__ __forceinline__ void add(int32_t, double) {}
};

template <typename T, int NV>
struct ApplyAcc {
  static constexpr bool kApply = true;
  using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  static constexpr int PER = 16 / sizeof(T), NL = NV / PER;   // values per load, loads per row
  const T *X;
  int64_t ldx;
  T a[NV];
  __device__ __forceinline__ void add(int32_t j, double v) {
    const T h = (T)v;
    const V *x = reinterpret_cast<const V *>(X + (int64_t)j * ldx);
    V xv[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) xv[l] = x[l];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if constexpr (sizeof(T) == 8) {
        a[2 * l] += h * xv[l].x;
        a[2 * l + 1] += h * xv[l].y;
      } else {
        a[4 * l] += h * xv[l].x;
        a[4 * l + 1] += h * xv[l].y;
        a[4 * l + 2] += h * xv[l].z;
        a[4 * l + 3] += h * xv[l].w;
      }
    }
  }
};

// Diagonal A-block part of a row: Lsame(beta) entries [e0, e1) in position
// order, kept while position < len(alpha) (a prefix).
template <int W, bool FILL, typename T, class Acc>
__device__ __forceinline__ void row_diag(const RowArgs &g, int64_t i, int64_t e0, int64_t e1, int alpha,
                                         int len_a, int64_t off_a, const uint64_t *ab, const SpecIdx &sa_idx,
                                         int64_t out, int64_t &cnt, Acc &acc) {
  const int lane = lane_id();
  T *val = static_cast<T *>(g.val);
  for (int64_t k0 = e0; k0 < e1; k0 += kWave) {
    const int64_t k = k0 + lane;
    const bool valid = k < e1;
    // all reads of the entry at once, at a clamped index
    const int64_t kq = valid ? k : e0;
    const int2 r = reinterpret_cast<const int2 *>(g.ls_rec)[kq];
    const int pos = r.x;
    const int info = FILL ? r.y : 0;
    const double lval = FILL ? g.ls_val[kq] : 0.0;
    const bool ok = valid && pos < len_a;
    const uint64_t m = ballot(ok);
    if (FILL && ok) {
      double v = lval;
      const int kb = info & 3;
      if (kb == 0) {  // diagonal: E_A + E_B + sum_{x in alpha, y in beta} V^AB_{xy,xy}
        v = g.diag[i];
      } else if (kb == 1) {  // B single: + s_B sum_{x in alpha} V^AB_{(x,b),(x,d)}
        const int32_t bc = info >> 3;
        const double s = (info >> 2) & 1 ? -1.0 : 1.0;
        v += s * spec_sum<W>(sa_idx, ab, g.it.arb, g.it.nA, [&](int32_t r) { return vt_at(g.it, r, bc); });
      }
      if constexpr (Acc::kApply) {
        acc.add((int32_t)(off_a + pos), v);
      } else {
        const uint32_t o = (uint32_t)(k - k0);   // from out + cnt, as a 32-bit byte offset below
        *reinterpret_cast<int32_t *>(reinterpret_cast<char *>(g.col + (out + cnt)) + o * 4u) = (int32_t)(off_a + pos);
        *reinterpret_cast<T *>(reinterpret_cast<char *>(val + (out + cnt)) + o * (uint32_t)sizeof(T)) = (T)v;
      }
    }
    cnt += __popcll(m);
    if (m != ballot(valid)) break;
  }
}

// beta's L1 list as one row pass sees it: either staged in LDS (segment
// offsets relative to the list's start) or read from global memory.
constexpr int kL1Stage = 512;   // entries of one configuration's L1 list kept in LDS

template <bool ST>
struct L1View {
  const int32_t *seg32;   // ST: nseg + 1 offsets relative to the list start
  const int64_t *seg64;   // !ST: absolute offsets of beta's segments
  int64_t base;           // !ST: absolute offset of the list start
  const int2 *rec;        // (pos, info), indexed relative to the list start
  __device__ __forceinline__ int seg(int h) const {
    if constexpr (ST) return seg32[h];
    else return (int)(seg64[h] - base);
  }
  __device__ __forceinline__ int pos(int k) const { return rec[k].x; }
};

// Tile part of a row: tiles [t0, t1) in ascending alpha'.  Lanes over tiles;
// a kA = 2 tile holds at most one entry (same B position), a kA = 1 tile the
// prefix of beta's L1 list for the tile's 2M_B list with position < len.
// kA = 1 entries are expanded over all lanes of the wave.
template <int W, bool FILL, typename T, bool ST, class Acc>
__device__ __forceinline__ void row_tiles(const RowArgs &g, int64_t t0, int64_t t1, int p, int seg_a, int lev_b,
                                          const uint64_t *bb, const SpecIdx &sb_idx, int64_t out, int64_t &cnt,
                                          const L1View<ST> &L, const int32_t *lev, int32_t *mark, Acc &acc) {
  const int lane = lane_id();
  T *val = static_cast<T *>(g.val);
  // the tile data of a batch of 64 is read together, one batch ahead of its
  // use (unconditional reads at a clamped index: a read under a branch would
  // make the compiler wait for the look-ahead as well)
  struct Batch {
    int info, len, off, rb;
    double val;
  };
  auto fetch = [&](int64_t tb, Batch &d) {
    const int64_t t = min(tb + lane, t1 - 1);
    const int4 r = reinterpret_cast<const int4 *>(g.t_rec)[t];
    d.info = r.x;
    d.len = r.y;
    if (FILL) {
      d.off = r.z;
      d.rb = r.w;
      d.val = g.t_val[t];
    }
  };
  // the kept window's per-lane entry data, and how to write one entry
  int rem = 0, w_il = 0, w_io = 0, w_coff = 0, w_orbs = 0;
  double w_bu = 0.0;
  auto emit = [&](bool on) {
    if (!on) return;
    const int orb = w_orbs & 0x7fffffff;
    const int2 lr = L.rec[w_il];
    const int li = lr.y, lp = lr.x;
    double v;
    if ((li & 3) == 0) {  // B unchanged: the tile's value, formed per tile below
      v = w_bu;
    } else {              // one A and one B orbital change: the two phases on the table element
      const uint64_t neg = (uint64_t)(((uint32_t)w_orbs >> 31) ^ ((uint32_t)li >> 2 & 1u)) << 63;
      v = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, vt_at(g.it, orb, li >> 3)) ^ neg);
    }
    if constexpr (Acc::kApply) {
      acc.add(w_coff + lp, v);
    } else {
      // byte offsets as 32-bit values: the stores take the scalar base
      // and a 32-bit vector offset (a row's outputs stay below 2^29)
      const uint32_t io = (uint32_t)w_io;
      *reinterpret_cast<int32_t *>(reinterpret_cast<char *>(g.col + out) + io * 4u) = w_coff + lp;
      *reinterpret_cast<T *>(reinterpret_cast<char *>(val + out) + io * (uint32_t)sizeof(T)) = (T)v;
    }
  };
  Batch nx;
  if (t0 < t1) fetch(t0, nx);
  for (int64_t tb = t0; tb < t1; tb += kWave) {
    const int64_t t = tb + lane;
    const Batch cur = nx;
    fetch(tb + kWave, nx);
    int ne = 0, info = 0, l0 = 0;
    if (t < t1) {
      info = cur.info;
      const int len = cur.len;
      if ((info & 3) == 2) {
        ne = p < len;
      } else {  // the segment's entries up to the tile's Q level (len holds the level)
        const int gt = (info >> 19) & 0x7f;
        l0 = L.seg(gt);
        ne = lev[gt * g.nlev + len];
      }
    }
    const int incl = wave_incl_scan_dpp(ne);
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    if (FILL) {
      const int orel = incl - ne;   // lane's first output, relative to out + cnt
      const bool two = (info & 3) == 2;
      const int32_t coff = ne ? cur.off : 0, rb = (!two && ne) ? cur.rb : 0;
      const double tv = ne ? cur.val : 0.0;
      // The value of the tile's entry that keeps beta, AA part + s_A sum_{y
      // in beta} V^AB_{(a,y),(c,y)}: a kA = 1 tile has one when its p <- h
      // keeps 2m (alpha' in alpha's 2M_B list) and its Q level reaches
      // beta's.  Formed once per tile here, with the batch's lanes together,
      // not once per window of entries; the entry's lane takes it by a lane
      // permute.
      double bu;
      {
        double sum = 0.0;
        if (!two && ne && g.it.nB > 0 && ((info >> 19) & 0x7f) == seg_a && cur.len >= lev_b)
          sum = spec_sum<W>(sb_idx, bb, g.it.bcol, g.it.nB, [&](int32_t c) { return vt_at(g.it, rb, c); });
        bu = tv + ((info >> 18) & 1 ? -sum : sum);
      }
      // this batch's outputs start at out + cnt (a matrix-free product
      // stores nothing)
      int32_t *const colb = Acc::kApply ? nullptr : g.col + (out + cnt);
      T *const valb = Acc::kApply ? nullptr : val + (out + cnt);
      if (two && ne) {
        if constexpr (Acc::kApply) {
          acc.add(coff + p, tv);
        } else {
          colb[(uint32_t)orel] = coff + p;
          valb[(uint32_t)orel] = (T)tv;
        }
      }
      // kA = 1 entries, spread over the lanes in windows of 64 that run on
      // from one batch of tiles into the next.  What an entry's lane needs of
      // its tile: list index = pl + k, output index (from the row's first
      // output) = po + k, the column base, the table row base with the
      // tile's phase bit on top (rb < 2^31) and the tile's value for the
      // entry that keeps beta.  A window the batch leaves short is kept in
      // registers (lanes [0, rem)) and completed by the next batch; the last
      // one is written after the last batch.
      const int n1 = two ? 0 : ne;
      const int incl1 = wave_incl_scan_dpp(n1);
      const int tot1 = __builtin_amdgcn_readlane(incl1, kWave - 1);
      const int st1 = incl1 - n1;
      const int pl = l0 - st1, po = (int)cnt + orel - st1;
      const int prb = (int)((uint32_t)rb | ((uint32_t)(info >> 18) & 1u) << 31);
      // Window [kb, kb + 64) of this batch's entries (kb from -rem: the kept
      // entries come first): each tile marks the slot where its entries
      // start (lane + 1), a prefix maximum spreads the marks, the owner of
      // the slot before the window covers the slots ahead of the first mark.
      // Every shuffle below runs with the whole wave active (uniform loop).
      int carry = 0;
      for (int kb = -rem; tot1 > 0 && kb < tot1; kb += kWave) {
        const int k = kb + lane;
        mark[lane] = 0;
        wave_lds_sync();
        if (n1 > 0 && st1 >= kb && st1 < kb + kWave) mark[st1 - kb] = lane + 1;
        wave_lds_sync();
        const int own = max(wave_incl_max_dpp(mark[lane]), carry) - 1;
        wave_lds_sync();
        carry = __builtin_amdgcn_readlane(own + 1, kWave - 1);
        const int nil = __shfl(pl, own, kWave) + k;
        const int nio = __shfl(po, own, kWave) + k;
        const int ncoff = __shfl(coff, own, kWave);
        const int norbs = __shfl(prb, own, kWave);
        const double nbu = __shfl(bu, own, kWave);
        if (k >= 0) {
          w_il = nil;
          w_io = nio;
          w_coff = ncoff;
          w_orbs = norbs;
          w_bu = nbu;
        }
        if (kb + kWave > tot1) {   // short: kept for the next batch
          rem = tot1 - kb;
          break;
        }
        emit(true);
        rem = 0;
      }
    }
    cnt += total;
  }
  if (FILL && rem > 0) emit(lane < rem);
}

// Body of the row passes (count, fill, matrix-free apply) for row i, wave wv
// of the workgroup; the kernels below describe the enumeration.
template <int W, bool FILL, typename T, class Acc>
__device__ __forceinline__ void row_pass(const RowArgs &g, const LowerArgs &lo, int64_t i, int wv, Acc &acc) {
  const RowArgs gl = lower_args(g, lo);
  __shared__ int2 s_rec[4][kL1Stage];
  __shared__ int32_t s_seg[4][kMaxSeg + 2];
  __shared__ int32_t s_mark[4][FILL ? kWave : 1];
  __shared__ __align__(16) int32_t s_spec[4][FILL ? 2 * kSpec : 1];
  const int lane = lane_id();
  const int alpha = uni(g.row_a[i]), p = uni(g.row_p[i]);
  const int beta = uni(g.row_b[i]);
  const int len_a = uni(g.a_len[alpha]);
  const int seg_a = FILL ? uni(g.a_seg[alpha]) : 0;   // alpha's 2M_B list
  const int lev_b = FILL && g.nlev > 1 ? uni(g.b_q[beta]) - g.qminB : 0;   // beta's Q level
  const int64_t off_a = uni(g.a_off[alpha]);
  uint64_t ab[W], bb[W];
  SpecIdx sa_idx{0, nullptr}, sb_idx{0, nullptr};
  if (FILL) {
    // (kept in vector registers: the table reads in the per-entry sums over
    // these bits then go through the vector memory path)
    load_bits<W>(g.a_bits, g.nA, alpha, ab);
    load_bits<W>(g.b_bits, g.nB, beta, bb);
    // spectator sums exist only with two species (one species has no
    // transition table: its maps are not allocated)
    if (g.it.nB > 0) {
      sa_idx = spec_idx<W>(ab, g.it.arb, g.it.nA, s_spec[wv]);
      sb_idx = spec_idx<W>(bb, g.it.bcol, g.it.nB, s_spec[wv] + kSpec);
    }
  }
  // the CSR offsets of the row (a matrix-free product stores nothing)
  constexpr bool kStore = FILL && !Acc::kApply;
  const int64_t out_u = kStore ? uni(g.row_ptr[i]) : 0;
  const int64_t l1b = (int64_t)beta * g.nseg;
  const int64_t base = uni(g.l1_seg[l1b]);
  const int64_t n1 = uni(g.l1_seg[l1b + g.nseg]) - base;
  const int64_t t0u = uni(g.t_ptr[(int64_t)alpha * g.tstride]), t1u = uni(g.t_ptr[(int64_t)(alpha + 1) * g.tstride]);
  const int32_t *const lev = g.lev_cnt + (int64_t)beta * g.nseg * g.nlev;   // beta's entry counts by list and level
  int64_t cu = 0, cl = 0;
  // The four parts in column order.  What only the lower parts use is read
  // after the upper parts (fewer values held in scalar registers across
  // them).  beta's Lsame list: [ls_lo, ls_me) before beta itself, [ls_me,
  // ls_hi) from it on.
  auto parts = [&](const auto &L) {
    constexpr bool ST = std::is_same<std::decay_t<decltype(L)>, L1View<true>>::value;
    const int64_t ls_me = uni((int64_t)g.ls_self[beta]), ls_hi = uni(g.ls_ptr[beta + 1]);
    row_diag<W, FILL, T>(g, i, ls_me, ls_hi, alpha, len_a, off_a, ab, sa_idx, out_u, cu, acc);
    row_tiles<W, FILL, T, ST>(g, t0u, t1u, p, seg_a, lev_b, bb, sb_idx, out_u, cu, L, lev, s_mark[wv], acc);
    const int64_t out_l = kStore ? uni(gl.row_ptr[i]) : 0;
    const int64_t t0l = uni(gl.t_ptr[(int64_t)alpha * gl.tstride]);
    const int64_t t1l = uni(gl.t_ptr[(int64_t)(alpha + 1) * gl.tstride]);
    row_tiles<W, FILL, T, ST>(gl, t0l, t1l, p, seg_a, lev_b, bb, sb_idx, out_l, cl, L, lev, s_mark[wv], acc);
    const int64_t ls_lo = uni(g.ls_ptr[beta]);
    row_diag<W, FILL, T>(gl, i, ls_lo, ls_me, alpha, len_a, off_a, ab, sa_idx, out_l, cl, acc);
  };
  if (n1 <= kL1Stage && g.nseg <= kMaxSeg + 1) {
    for (int64_t k = lane; k < n1; k += kWave) {
      s_rec[wv][k] = reinterpret_cast<const int2 *>(g.l1_rec)[base + k];
    }
    for (int h = lane; h <= g.nseg; h += kWave) s_seg[wv][h] = (int32_t)(g.l1_seg[l1b + h] - base);
    wave_lds_sync();
    parts(L1View<true>{s_seg[wv], nullptr, 0, s_rec[wv]});
  } else {
    parts(L1View<false>{nullptr, g.l1_seg + l1b, base, reinterpret_cast<const int2 *>(g.l1_rec) + base});
  }
  if (!FILL && lane == 0) {
    g.rcnt[i] = (int32_t)cu;
    gl.rcnt[i] = (int32_t)cl;
  }
}

// One wave per row i = (alpha, p), both stored triangles: g holds the upper
// tiles and outputs, gl the lower ones.  Upper row (j >= i): the diagonal
// A-block from beta itself on (positions < len(alpha)), then tiles
// alpha' > alpha.  Lower row (j < i): tiles alpha' < alpha, then the
// diagonal A-block entries before beta.  Both lists come out in ascending
// column order.  The row's preamble, its spectator slots and beta's L1 list
// (at most a few hundred entries for these bases, copied to LDS so the
// per-tile binary searches and the expansion read it there) serve both
// triangles; one pass over both measured 6-8% faster than one per triangle.
// Eight waves per SIMD (the most the hardware holds) are asked for
// explicitly: the pass waits on chains of dependent reads, and the scalar
// registers the compiler would otherwise keep cap it at seven (measured 12%
// slower).
template <int W, bool FILL, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_row_pass(RowArgs g, LowerArgs gl) {
  // plain block order: rows of very different lengths sit in runs, and
  // giving each XCD one contiguous range of rows (for L2 locality of the
  // tile lists) measured 30-40% slower from the imbalance between XCDs
  const int wv = uni((int)(threadIdx.x >> 6));
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
  if (i >= g.D) return;
  NoAcc acc;
  row_pass<W, FILL, T>(g, gl, i, wv, acc);
}

// Matrix-free product Y = H X (the FMA variant of Fig. 2: compare, compute
// and multiply without storing H): the fill pass's enumeration of row i,
// every entry multiplied into its row of X; the lanes' sums are combined by
// a fixed butterfly and lane 0 writes row i of Y.  X and Y rows of NV values
// (8 or 16), 16-byte aligned.
template <int W, typename T, int NV>
__global__ __launch_bounds__(256) void k_row_apply(RowArgs g, LowerArgs gl, const T *X, int64_t ldx, T *Y,
                                                   int64_t ldy) {
  const int wv = uni((int)(threadIdx.x >> 6));
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + wv;
  if (i >= g.D) return;
  ApplyAcc<T, NV> acc;
  acc.X = X;
  acc.ldx = ldx;
#pragma unroll
  for (int u = 0; u < NV; ++u) acc.a[u] = T(0);
  row_pass<W, true, T>(g, gl, i, wv, acc);
#pragma unroll
  for (int u = 0; u < NV; ++u)
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) acc.a[u] += __shfl_xor(acc.a[u], d, kWave);
  if (lane_id() == 0) {
    using V = typename ApplyAcc<T, NV>::V;
    V *y = reinterpret_cast<V *>(Y + i * ldy);
#pragma unroll
    for (int l = 0; l < ApplyAcc<T, NV>::NL; ++l) {
      if constexpr (sizeof(T) == 8) y[l] = V{acc.a[2 * l], acc.a[2 * l + 1]};
      else y[l] = V{acc.a[4 * l], acc.a[4 * l + 1], acc.a[4 * l + 2], acc.a[4 * l + 3]};
    }
  }
}

// ------------------------------------------------------------ exclusive scan
constexpr int kScanThreads = 256, kScanItems = 16, kScanTile = kScanThreads * kScanItems;

__device__ int64_t block_excl_scan(int64_t v, int64_t *lds, int64_t &total) {
  const int lane = lane_id(), wv = threadIdx.x >> 6;
  const int64_t incl = wave_incl_scan(v);
  if (lane == kWave - 1) lds[wv] = incl;
  __syncthreads();
  int64_t wbase = 0;
  total = 0;
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    if (k < wv) wbase += lds[k];
    total += lds[k];
  }
  __syncthreads();
  return wbase + incl - v;
}

// Several independent exclusive scans in one set of three launches: the
// tiles of all arrays form one grid (block -> array through blk0), the
// per-tile totals of each array are scanned by one block per array, and the
// down-sweep writes every array's offsets and its total.
struct ScanSet {
  int n_arrays;
  const int32_t *in[kScanArrays];
  int64_t *out[kScanArrays];
  int64_t n[kScanArrays];
  int64_t blk0[kScanArrays + 1];   // first tile of each array; blk0[n_arrays] = all tiles
};

__device__ __forceinline__ int scan_array_of(const ScanSet &S, int64_t b) {
  int k = 0;
  while (k + 1 < S.n_arrays && b >= S.blk0[k + 1]) ++k;
  return k;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(ScanSet S, int64_t *bsum) {
  __shared__ int64_t lds[kScanThreads / kWave];
  const int k = scan_array_of(S, blockIdx.x);
  const int32_t *in = S.in[k];
  const int64_t n = S.n[k];
  const int64_t base = (blockIdx.x - S.blk0[k]) * kScanTile;
  int64_t s = 0;
  for (int t = 0; t < kScanItems; ++t) {
    const int64_t idx = base + (int64_t)t * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  int64_t total;
  block_excl_scan(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// one block per array: exclusive scan of its tile totals, in place; the
// array's total goes to bsum[blk0[n_arrays] + k]
__global__ __launch_bounds__(kScanThreads) void k_scan_top(ScanSet S, int64_t *bsum) {
  __shared__ int64_t lds[kScanThreads / kWave];
  const int k = blockIdx.x;
  const int64_t b0 = S.blk0[k], nb = S.blk0[k + 1] - b0;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int64_t idx = c0 + threadIdx.x;
    const int64_t v = idx < nb ? bsum[b0 + idx] : 0;
    int64_t total;
    const int64_t ex = block_excl_scan(v, lds, total);
    if (idx < nb) bsum[b0 + idx] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[S.blk0[S.n_arrays] + k] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(ScanSet S, const int64_t *bsum) {
  __shared__ int64_t lds[kScanThreads / kWave];
  const int k = scan_array_of(S, blockIdx.x);
  const int32_t *in = S.in[k];
  int64_t *out = S.out[k];
  const int64_t n = S.n[k];
  const int64_t lb = blockIdx.x - S.blk0[k];
  const int64_t base = lb * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    v[t] = base + t < n ? in[base + t] : 0;
    s += v[t];
  }
  int64_t total;
  int64_t run = bsum[blockIdx.x] + block_excl_scan(s, lds, total);
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    if (base + t < n) out[base + t] = run;
    run += v[t];
  }
  if (blockIdx.x == S.blk0[k + 1] - 1 && threadIdx.x == 0) out[n] = bsum[S.blk0[S.n_arrays] + k];
}

size_t scan_scratch(const std::vector<int64_t> &ns) {
  size_t t = 0;
  for (int64_t n : ns) t += (size_t)std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  return t + ns.size();
}

void launch_scans(const std::vector<ScanJob> &jobs, int64_t *scratch, hipStream_t s) {
  CIB_REQUIRE(!jobs.empty() && jobs.size() <= (size_t)kScanArrays, CIB_E_INVALID, "scan batch size");
  ScanSet S{};
  S.n_arrays = (int)jobs.size();
  int64_t nb = 0;
  for (int k = 0; k < S.n_arrays; ++k) {
    S.in[k] = jobs[k].in;
    S.out[k] = jobs[k].out;
    S.n[k] = jobs[k].n;
    S.blk0[k] = nb;
    nb += std::max<int64_t>(1, (jobs[k].n + kScanTile - 1) / kScanTile);
  }
  S.blk0[S.n_arrays] = nb;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, S, scratch);
  hipLaunchKernelGGL(k_scan_top, dim3((unsigned)S.n_arrays), dim3(kScanThreads), 0, s, S, scratch);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, S, (const int64_t *)scratch);
  CIB_HIP(hipGetLastError());
}

// ------------------------------------------------------------ launchers
template <int W>
static void expand_w(const cib_basis &b, hipStream_t s) {
  const Plan &p = b.plan;
  const unsigned nblk = (unsigned)((p.D + 255) / 256);
  hipLaunchKernelGGL(k_expand_basis<W>, dim3(nblk), dim3(256), 0, s, p.D, p.nA(), p.nB(), p.WA,
                     p.WB, b.a_off.p, b.a_seg.p, b.bseg_start.p, b.a_bits.p, b.b_bits.p,
                     b.words.p, b.row_a.p, b.row_p.p, b.row_b.p);
}

void launch_expand_basis(const cib_basis &b, hipStream_t s) {
  switch (b.plan.W) {
    case 1: expand_w<1>(b, s); break;
    case 2: expand_w<2>(b, s); break;
    default: expand_w<3>(b, s); break;
  }
  CIB_HIP(hipGetLastError());
}

template <int W>
static void energy_w(const cib_basis &b, const DevInter &it, double *eA, double *eB, hipStream_t s) {
  const Plan &p = b.plan;
  hipLaunchKernelGGL(k_config_energy<W>, dim3((p.nA() + 255) / 256), dim3(256), 0, s, p.nA(),
                     b.a_bits.p, it.epsA, it.pidxA, it.prowA, it.nA, it.vA, eA);
  if (it.nB > 0)
    hipLaunchKernelGGL(k_config_energy<W>, dim3((p.nB() + 255) / 256), dim3(256), 0, s, p.nB(),
                       b.b_bits.p, it.epsB, it.pidxB, it.prowB, it.nB, it.vB, eB);
  else
    CIB_HIP(hipMemsetAsync(eB, 0, sizeof(double) * p.nB(), s));
}

void launch_substate_energy(const cib_basis &b, const DevInter &it, double *eA, double *eB,
                            hipStream_t s) {
  switch (b.plan.W) {
    case 1: energy_w<1>(b, it, eA, eB, s); break;
    case 2: energy_w<2>(b, it, eA, eB, s); break;
    default: energy_w<3>(b, it, eA, eB, s); break;
  }
  CIB_HIP(hipGetLastError());
}

void launch_build_vt(const DevInter &it, const VtBlock *blocks, int nblk, const int32_t *atr,
                     const int32_t *btr, int64_t total, double *vt, hipStream_t s) {
  if (total == 0 || nblk == 0) return;
  hipLaunchKernelGGL(k_build_vt, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, it, blocks, nblk,
                     atr, btr, total, vt);
  CIB_HIP(hipGetLastError());
}

void launch_dab(const DevInter &it, double *dab, hipStream_t s) {
  const int n = it.nA * it.nB;
  if (n == 0) return;
  hipLaunchKernelGGL(k_dab, dim3((n + 255) / 256), dim3(256), 0, s, it, dab);
  CIB_HIP(hipGetLastError());
}

// Copies up to 4 device int64 values (the totals of several scans) into one
// small device array, so the host reads them with a single synchronisation.
struct Gather4 {
  const int64_t *src[4];
};
__global__ void k_gather_i64(Gather4 g, int n, int64_t *out) {
  const int t = threadIdx.x;
  if (t < n) out[t] = *g.src[t];
}

static void read_totals(std::initializer_list<const int64_t *> src, int64_t *scratch, int64_t *host,
                        hipStream_t s) {
  Gather4 g{};
  int n = 0;
  for (const int64_t *q : src) g.src[n++] = q;
  hipLaunchKernelGGL(k_gather_i64, dim3(1), dim3(64), 0, s, g, n, scratch);
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipMemcpyAsync(host, scratch, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
  CIB_HIP(hipStreamSynchronize(s));
}

// out[x] = first row i with rp[i] + lrp[i] >= x / 8 of all stored entries
// (both triangles), x = 0 .. 8: row ranges of equal work for the 8 XCDs.
__global__ void k_xcd_rows(int64_t D, const int64_t *rp, const int64_t *lrp, int64_t *out) {
  const int x = threadIdx.x;
  if (x > 8) return;
  const int64_t total = rp[D] + lrp[D];
  const int64_t target = x == 8 ? total + 1 : (total / 8) * x + (total % 8) * x / 8;
  int64_t lo = 0, hi = D;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (rp[m] + lrp[m] < target) lo = m + 1;
    else hi = m;
  }
  out[x] = x == 8 ? D : lo;
}

struct Events {
  hipEvent_t e[8];
  // timing only: no system-scope fence at every record
  Events() { for (auto &x : e) CIB_HIP(hipEventCreateWithFlags(&x, hipEventDisableSystemFence)); }
  ~Events() { for (auto &x : e) (void)hipEventDestroy(x); }
  double ms(int a, int b) {
    float t = 0;
    CIB_HIP(hipEventElapsedTime(&t, e[a], e[b]));
    return t * 1e-3;
  }
};

// The upper half (the product) and the strictly lower copy (read by the
// SpMM) are built by the same passes side by side, so the host waits twice:
// once for the sizes of the screens' lists, once for the two nonzero counts.
template <int W, typename T, int NV>
static void launch_apply(unsigned rblk, const RowArgs &ra, const LowerArgs &rl, const ApplyReq &a, hipStream_t s) {
  hipLaunchKernelGGL((k_row_apply<W, T, NV>), dim3(rblk), dim3(256), 0, s, ra, rl, static_cast<const T *>(a.X),
                     a.ldx, static_cast<T *>(a.Y), a.ldy);
}

// The build (ap == nullptr): screens, counts, offsets, fill into H.  With
// ap: the screens, then the matrix-free product Y = H X instead of a matrix
// (H is not touched).
template <int W>
static void build_w(cib_ctx *ctx, const cib_basis &b, const cib_interaction &itr, cib_dtype dt,
                    cib_matrix &H, hipStream_t s, const BuildReserve &reserve, const ApplyReq *ap = nullptr) {
  UnwindFence fence(s);
  const Plan &p = b.plan;
  const DevInter it = itr.view();
  const int nA = p.nA(), nB = p.nB(), nseg = p.nseg();
  const int qcap = p.qmax >= 0 ? p.qmax - p.qminB : -1;   // Q_A + Q_B <= qmax as a cap on Q_A + (Q_B - qmin_B)
  // row counts from per-configuration tables (k_row_count_tab) unless the
  // per-A-configuration histograms would be large
  const int64_t nbin = (int64_t)nseg * p.nlev;
  const bool tab_count = nbin <= kCountBins * kWave && (int64_t)nA * nbin <= (int64_t(1) << 25) &&
                         (int64_t)nB * nbin <= (int64_t(1) << 28);
  Events ev;
  auto bytes = [](size_t count, size_t elem) { return dev_bytes(count * elem); };

  // ---- counting passes of the two screens (tiles of both triangles)
  // tile screen: chunks of 64 candidates, groups of 64 configurations per
  // wave, fewer where that would leave the grid short of eight waves per SIMD
  const int nchunk = (nA + kWave - 1) / kWave;
  int gsz_a = kWave;
  while (gsz_a > 16 && (int64_t)nchunk * ((nA + gsz_a - 1) / gsz_a) < 8192) gsz_a /= 2;
  const int ngroup_a = (nA + gsz_a - 1) / gsz_a;
  const int64_t nunit = (int64_t)nA * nchunk;   // (alpha, chunk) cells
  // the adjacency screen's chunks: 64 configurations of one 2M_B list each
  std::vector<int32_t> coff_h(nseg + 1, 0), chunk_list_h;
  for (int h = 0; h < nseg; ++h) {
    const int nc = (p.bseg_start[h + 1] - p.bseg_start[h] + kWave - 1) / kWave;
    coff_h[h + 1] = coff_h[h] + nc;
    for (int c = 0; c < nc; ++c) chunk_list_h.push_back(h);
  }
  // groups of 64 B configurations per wave, fewer where that would leave
  // the grid short of eight waves per SIMD
  const int nchunk_b = coff_h[nseg];
  int gsz_b = kWave;
  while (gsz_b > 16 && (int64_t)nchunk_b * ((nB + gsz_b - 1) / gsz_b) < 8192) gsz_b /= 2;
  const int ngroup_b = (nB + gsz_b - 1) / gsz_b;
  const int64_t ncell = (int64_t)nB * nchunk_b;
  std::vector<int32_t> ls_base_h(nB + 1, 0);   // Lsame cells: the chunks of each beta's own list
  for (int bb = 0; bb < nB; ++bb)
    ls_base_h[bb + 1] = ls_base_h[bb] + (coff_h[p.b_seg[bb] + 1] - coff_h[p.b_seg[bb]]);
  const int64_t nlcell = ls_base_h[nB];
  const int64_t nscr = std::max(scan_scratch({nunit, nunit, nlcell, ncell}), scan_scratch({p.D, p.D}));
  if (reserve)
    reserve(0, bytes(nA, 8) + bytes(nB, 8) + 2 * bytes(nunit, 4) + bytes(nlcell, 4) + bytes(ncell, 4) +
                   2 * bytes(nunit + 1, 8) + bytes(nlcell + 1, 8) + bytes(ncell + 1, 8) + bytes(nB + 1, 8) +
                   bytes((size_t)nB * nseg + 1, 8) + bytes(nscr, 8) + bytes(4, 8) +
                   bytes(std::max<size_t>(chunk_list_h.size(), 1), 4) + bytes(nseg + 1, 4) + bytes(nB + 1, 4) +
                   (tab_count ? 2 : 1) * bytes((size_t)nB * nseg * p.nlev, 4) +
                   (tab_count && !ap ? bytes((size_t)nB * p.nlev, 4) : 0));
  // (each stage's buffers are taken before its first event: host work inside
  // a timed interval would leave the device idle there)
  DBuf<double> eA(ctx, nA), eB(ctx, nB);
  DBuf<int32_t> tcnt(ctx, nunit), tlcnt(ctx, nunit), ls_cnt(ctx, nlcell), l1_cnt(ctx, ncell);
  DBuf<int64_t> t_ptr(ctx, nunit + 1), tl_ptr(ctx, nunit + 1), ls_off(ctx, nlcell + 1), l1_off(ctx, ncell + 1);
  DBuf<int64_t> ls_ptr(ctx, nB + 1), l1_seg(ctx, (size_t)nB * nseg + 1);
  DBuf<int64_t> scratch(ctx, nscr), totals(ctx, 4);
  DBuf<int32_t> chunk_list(ctx, std::max<size_t>(chunk_list_h.size(), 1)), coff(ctx, nseg + 1);
  DBuf<int32_t> ls_base(ctx, nB + 1);
  // level counts of the L1 lists (per (beta, list); also bin-major for the
  // table-driven row counts) and of the Lsame lists, zeroed by k_adj_offsets
  DBuf<int32_t> lev_cnt(ctx, (size_t)nB * nseg * p.nlev), lev_t, ls_lev;
  if (tab_count) lev_t.reset(ctx, (size_t)nB * nseg * p.nlev);
  if (tab_count && !ap) ls_lev.reset(ctx, (size_t)nB * p.nlev);
  chunk_list.upload(chunk_list_h.data(), chunk_list_h.size(), s);
  coff.upload(coff_h.data(), nseg + 1, s);
  ls_base.upload(ls_base_h.data(), nB + 1, s);
  CIB_HIP(hipEventRecord(ev.e[0], s));
  launch_substate_energy(b, it, eA.p, eB.p, s);
  TileArgs ta{};
  ta.nA = nA; ta.nchunk = nchunk; ta.ngroup = ngroup_a; ta.gsz = gsz_a; ta.a_bits = b.a_bits.p; ta.a_m2 = b.a_m2.p; ta.a_len = b.a_len.p;
  ta.a_seg = b.a_seg.p; ta.a_off = b.a_off.p; ta.it = it; ta.tcnt = tcnt.p;
  TileArgs tl = ta;
  tl.tcnt = tlcnt.p;
  const unsigned tblk = (unsigned)(((int64_t)nchunk * ngroup_a + 3) / 4);
  {
    hipLaunchKernelGGL((k_tile_pass<W, false, false>), dim3(tblk), dim3(256), 0, s, ta);
    hipLaunchKernelGGL((k_tile_pass<W, false, true>), dim3(tblk), dim3(256), 0, s, tl);
  }
  AdjArgs aa{};
  aa.nB = nB; aa.nseg = nseg; aa.nchunk = nchunk_b; aa.ngroup = ngroup_b; aa.gsz = gsz_b;
  aa.b_bits = b.b_bits.p; aa.b_seg = b.b_seg.p; aa.bseg_start = b.bseg_start.p;
  aa.chunk_list = chunk_list.p; aa.coff = coff.p; aa.ls_base = ls_base.p; aa.ls_cnt = ls_cnt.p;
  aa.l1_cnt = l1_cnt.p;
  const unsigned ablk = (unsigned)(((int64_t)nchunk_b * ngroup_b + 3) / 4);
  hipLaunchKernelGGL((k_adj_pass<W, false>), dim3(ablk), dim3(256), 0, s, aa);
  CIB_HIP(hipGetLastError());
  launch_scans({{tcnt.p, nunit, t_ptr.p}, {tlcnt.p, nunit, tl_ptr.p}, {ls_cnt.p, nlcell, ls_off.p},
                {l1_cnt.p, ncell, l1_off.p}},
               scratch.p, s);
  hipLaunchKernelGGL(k_adj_offsets, dim3((unsigned)(((int64_t)nB * nseg + 256) / 256)), dim3(256), 0, s, nB, nseg,
                     nchunk_b, coff.p, ls_base.p, ls_off.p, l1_off.p, ls_ptr.p, l1_seg.p, p.nlev, lev_cnt.p,
                     tab_count ? lev_t.p : nullptr, tab_count && !ap ? ls_lev.p : nullptr);
  CIB_HIP(hipEventRecord(ev.e[1], s));
  int64_t n4[4];
  read_totals({t_ptr.p + nunit, tl_ptr.p + nunit, ls_ptr.p + nB, l1_seg.p + (int64_t)nB * nseg}, totals.p, n4, s);
  const int64_t n_tiles = n4[0], n_lt = n4[1], n_ls = n4[2], n_l1 = n4[3];

  // ---- filling passes of the two screens
  auto at_least1 = [](int64_t n) { return (size_t)std::max<int64_t>(n, 1); };
  if (reserve) {
    const size_t nt = at_least1(n_tiles), nl = at_least1(n_lt), ns = at_least1(n_ls), n1 = at_least1(n_l1);
    // screens, row counts, diagonal and the two offset arrays
    reserve(1, (bytes(nt, 16) + 2 * bytes(nt, 4) + bytes(nt, 8)) + (bytes(nl, 16) + 2 * bytes(nl, 4) + bytes(nl, 8)) +
                   bytes(nB, 4) + bytes(ns, 8) + 2 * bytes(ns, 4) + bytes(n1, 8) + 2 * bytes(n1, 4) + bytes(ns, 8) +
                   (tab_count ? 2 * bytes((size_t)nA * nseg * p.nlev, 4) + bytes(nt, 4) + bytes(nl, 4) +
                                    bytes(nA + 1, 4) + 2 * bytes(nA, 4)
                              : 0) +
                   2 * bytes(p.D, 4) +
                   bytes(p.D, 8) + 2 * bytes(p.D + 1, 8));
  }
  DBuf<TileRec> t_rec(ctx, at_least1(n_tiles)), tl_rec(ctx, at_least1(n_lt));
  DBuf<int32_t> t_src(ctx, at_least1(n_tiles)), t_dst(ctx, at_least1(n_tiles));
  DBuf<int32_t> tl_src(ctx, at_least1(n_lt)), tl_dst(ctx, at_least1(n_lt));
  DBuf<double> t_val(ctx, at_least1(n_tiles)), tl_val(ctx, at_least1(n_lt));
  DBuf<int32_t> ls_self(ctx, nB);
  DBuf<AdjRec> ls_rec(ctx, at_least1(n_ls)), l1_rec(ctx, at_least1(n_l1));
  DBuf<int32_t> ls_src(ctx, at_least1(n_ls)), ls_dst(ctx, at_least1(n_ls));
  DBuf<int32_t> l1_src(ctx, at_least1(n_l1)), l1_dst(ctx, at_least1(n_l1));
  DBuf<double> ls_val(ctx, at_least1(n_ls));
  // the row-count stage's buffers and the row offsets
  DBuf<int32_t> rcnt(ctx, p.D), rlcnt(ctx, p.D);
  DBuf<double> diag(ctx, p.D);
  DBuf<int32_t> hist_u, hist_l, k2len_u, k2len_l, k2n_u, k2n_l, cstart;
  std::vector<int32_t> cstart_h(nA + 1, 0);   // waves of k_row_count_tab: one per 64 rows of each block
  if (tab_count && !ap) {
    for (int a2 = 0; a2 < nA; ++a2) cstart_h[a2 + 1] = cstart_h[a2] + (p.a_len[a2] + kWave - 1) / kWave;
    cstart.reset(ctx, nA + 1);
    cstart.upload(cstart_h.data(), nA + 1, s);
    hist_u.reset(ctx, (size_t)nA * nbin);
    hist_l.reset(ctx, (size_t)nA * nbin);
    k2len_u.reset(ctx, at_least1(n_tiles));
    k2len_l.reset(ctx, at_least1(n_lt));
    k2n_u.reset(ctx, nA);
    k2n_l.reset(ctx, nA);
  }
  if (!ap) {
    H.row_ptr.reset(ctx, p.D + 1);
    H.lo_ptr.reset(ctx, p.D + 1);
  }
  CIB_HIP(hipEventRecord(ev.e[2], s));
  ta.t_ptr = t_ptr.p; ta.t_rec = t_rec.p; ta.t_src = t_src.p; ta.t_dst = t_dst.p;
  tl.t_ptr = tl_ptr.p; tl.t_rec = tl_rec.p; tl.t_src = tl_src.p; tl.t_dst = tl_dst.p;
  auto nb256 = [](int64_t n) { return dim3((unsigned)std::max<int64_t>((n + 255) / 256, 1)); };
  {
    hipLaunchKernelGGL((k_tile_pass<W, true, false>), dim3(tblk), dim3(256), 0, s, ta);
    hipLaunchKernelGGL((k_tile_pass<W, true, true>), dim3(tblk), dim3(256), 0, s, tl);
    // phases and values, one thread per tile
    if (n_tiles)
      hipLaunchKernelGGL((k_tile_val<W>), nb256(n_tiles), dim3(256), 0, s, n_tiles, t_src.p, t_dst.p,
                         b.a_bits.p, nA, b.a_seg.p, it, t_rec.p, t_val.p, b.a_q.p, qcap);
    if (n_lt)
      hipLaunchKernelGGL((k_tile_val<W>), nb256(n_lt), dim3(256), 0, s, n_lt, tl_src.p, tl_dst.p,
                         b.a_bits.p, nA, b.a_seg.p, it, tl_rec.p, tl_val.p, b.a_q.p, qcap);
  }
  aa.ls_off = ls_off.p; aa.l1_off = l1_off.p; aa.ls_self = ls_self.p; aa.ls_rec = ls_rec.p;
  aa.l1_rec = l1_rec.p; aa.ls_src = ls_src.p; aa.ls_dst = ls_dst.p; aa.l1_src = l1_src.p; aa.l1_dst = l1_dst.p;
  {
    hipLaunchKernelGGL((k_adj_pass<W, true>), dim3(ablk), dim3(256), 0, s, aa);
    // phases, table columns and B-only values, one thread per entry
    if (n_ls)
      hipLaunchKernelGGL((k_adj_val<W>), nb256(n_ls), dim3(256), 0, s, n_ls, ls_src.p, ls_dst.p, b.b_bits.p,
                         nB, eB.p, it, ls_rec.p, ls_val.p);
    if (n_l1)
      hipLaunchKernelGGL((k_adj_val<W>), nb256(n_l1), dim3(256), 0, s, n_l1, l1_src.p, l1_dst.p, b.b_bits.p,
                         nB, eB.p, it, l1_rec.p, (double *)nullptr);
    if (n_l1)
      hipLaunchKernelGGL(k_l1_levels, nb256(n_l1), dim3(256), 0, s, n_l1, nseg, p.nlev, p.qminB, l1_seg.p,
                         l1_src.p, l1_dst.p, b.b_seg.p, b.b_q.p, lev_cnt.p, nB, tab_count ? lev_t.p : nullptr);
  }
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipEventRecord(ev.e[3], s));

  // ---- per-row counting passes (both triangles), offsets
  RowArgs ra{};
  ra.D = p.D; ra.nA = nA; ra.nB = nB; ra.nseg = nseg;
  ra.row_a = b.row_a.p; ra.row_p = b.row_p.p; ra.row_b = b.row_b.p; ra.a_seg = b.a_seg.p; ra.a_len = b.a_len.p;
  ra.bseg_start = b.bseg_start.p; ra.a_off = b.a_off.p; ra.a_bits = b.a_bits.p; ra.b_bits = b.b_bits.p;
  ra.eA = eA.p; ra.t_ptr = t_ptr.p; ra.tstride = nchunk; ra.t_rec = t_rec.p;
  ra.t_val = t_val.p; ra.ls_ptr = ls_ptr.p; ra.l1_seg = l1_seg.p; ra.ls_self = ls_self.p;
  ra.ls_rec = ls_rec.p; ra.l1_rec = l1_rec.p; ra.lev_cnt = lev_cnt.p; ra.nlev = p.nlev;
  ra.ls_val = ls_val.p; ra.it = it; ra.b_q = b.b_q.p; ra.qminB = p.qminB;
  ra.rcnt = rcnt.p;
  LowerArgs rl{tl_ptr.p, tl_rec.p, tl_val.p, rlcnt.p, nullptr, nullptr, nullptr};
  const unsigned rblk = (unsigned)((p.D + 3) / 4);
  if (ap) {
    hipLaunchKernelGGL((k_state_diag<W>), dim3((unsigned)((p.D + 255) / 256)), dim3(256), 0, s, p.D,
                       b.row_a.p, b.row_p.p, b.a_seg.p, b.bseg_start.p, b.a_bits.p, nA, b.b_bits.p, nB,
                       eA.p, eB.p, it, diag.p);
    ra.diag = diag.p;
    {
      KTimer kt(ctx, K_APPLY_FREE, s);
      if (dt == CIB_F64) {
        if (ap->nvec == 8) launch_apply<W, double, 8>(rblk, ra, rl, *ap, s);
        else launch_apply<W, double, 16>(rblk, ra, rl, *ap, s);
      } else {
        if (ap->nvec == 8) launch_apply<W, float, 8>(rblk, ra, rl, *ap, s);
        else launch_apply<W, float, 16>(rblk, ra, rl, *ap, s);
      }
    }
    CIB_HIP(hipGetLastError());
    CIB_HIP(hipStreamSynchronize(s));   // the screens are freed on return
    return;
  }
  {
    if (tab_count) {
      const unsigned ablk4 = (unsigned)((nA + 3) / 4);
      hipLaunchKernelGGL(k_tile_hist, dim3(ablk4), dim3(256), 0, s, nA, t_ptr.p, nchunk, t_rec.p, p.nlev, (int)nbin,
                         hist_u.p, k2len_u.p, k2n_u.p);
      hipLaunchKernelGGL(k_tile_hist, dim3(ablk4), dim3(256), 0, s, nA, tl_ptr.p, nchunk, tl_rec.p, p.nlev, (int)nbin,
                         hist_l.p, k2len_l.p, k2n_l.p);
      if (n_ls)
        hipLaunchKernelGGL(k_ls_levels, nb256(n_ls), dim3(256), 0, s, n_ls, p.nlev, p.qminB, ls_ptr.p, ls_src.p,
                           ls_dst.p, b.b_q.p, ls_lev.p);
      CountArgs ca{nA, nB, nseg, p.nlev, (int)nbin, qcap, nchunk, cstart.p, cstart_h[nA], b.a_off.p, b.a_len.p,
                   b.a_q.p,
                   b.a_seg.p, b.bseg_start.p, ls_self.p, ls_ptr.p, t_ptr.p, tl_ptr.p, lev_t.p, ls_lev.p,
                   hist_u.p, hist_l.p, k2len_u.p, k2len_l.p, k2n_u.p, k2n_l.p, rcnt.p, rlcnt.p};
      hipLaunchKernelGGL(k_row_count_tab, dim3((unsigned)((cstart_h[nA] + 3) / 4)), dim3(256), 0, s, ca);
    } else {
      hipLaunchKernelGGL((k_row_pass<W, false, double>), dim3(rblk), dim3(256), 0, s, ra, rl);
    }
    hipLaunchKernelGGL((k_state_diag<W>), dim3((unsigned)((p.D + 255) / 256)), dim3(256), 0, s, p.D,
                       b.row_a.p, b.row_p.p, b.a_seg.p, b.bseg_start.p, b.a_bits.p, nA, b.b_bits.p, nB,
                       eA.p, eB.p, it, diag.p);
  }
  ra.diag = diag.p;
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipEventRecord(ev.e[4], s));
  {
    launch_scans({{rcnt.p, p.D, H.row_ptr.p}, {rlcnt.p, p.D, H.lo_ptr.p}}, scratch.p, s);
  }
  CIB_HIP(hipEventRecord(ev.e[5], s));
  int64_t n2[2];
  read_totals({H.row_ptr.p + p.D, H.lo_ptr.p + p.D}, totals.p, n2, s);
  const int64_t nnz = n2[0], nlo = n2[1];
  const size_t sv = dt == CIB_F64 ? 8 : 4;
  if (reserve)
    reserve(2, bytes(at_least1(nnz), 4) + bytes(at_least1(nlo), 4) + bytes(at_least1(nnz), sv) +
                   bytes(at_least1(nlo), sv) + bytes(9, 8));

  // ---- filling passes
  H.col.reset(ctx, at_least1(nnz));
  H.lo_col.reset(ctx, at_least1(nlo));
  if (dt == CIB_F64) {
    H.val64.reset(ctx, at_least1(nnz));
    H.lo_val64.reset(ctx, at_least1(nlo));
  } else {
    H.val32.reset(ctx, at_least1(nnz));
    H.lo_val32.reset(ctx, at_least1(nlo));
  }
  ra.row_ptr = H.row_ptr.p;
  ra.col = H.col.p;
  ra.val = dt == CIB_F64 ? (void *)H.val64.p : (void *)H.val32.p;
  rl.row_ptr = H.lo_ptr.p;
  rl.col = H.lo_col.p;
  rl.val = dt == CIB_F64 ? (void *)H.lo_val64.p : (void *)H.lo_val32.p;
  CIB_HIP(hipEventRecord(ev.e[6], s));
  {
    if (dt == CIB_F64)
      hipLaunchKernelGGL((k_row_pass<W, true, double>), dim3(rblk), dim3(256), 0, s, ra, rl);
    else
      hipLaunchKernelGGL((k_row_pass<W, true, float>), dim3(rblk), dim3(256), 0, s, ra, rl);
  }
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipEventRecord(ev.e[7], s));
  DBuf<int64_t> xr(ctx, 9);
  hipLaunchKernelGGL(k_xcd_rows, dim3(1), dim3(64), 0, s, p.D, H.row_ptr.p, H.lo_ptr.p, xr.p);
  CIB_HIP(hipGetLastError());
  CIB_HIP(hipMemcpyAsync(H.xcd_rows, xr.p, sizeof(H.xcd_rows), hipMemcpyDeviceToHost, s));
  CIB_HIP(hipStreamSynchronize(s));

  H.D = p.D;
  H.nnz = nnz;
  H.nnz_lower = nlo;
  H.dtype = dt;
  H.stats.t_screen_s = ev.ms(0, 1) + ev.ms(2, 3);
  H.stats.t_count_s = ev.ms(3, 4);
  H.stats.t_scan_s = ev.ms(4, 5);
  H.stats.t_fill_s = ev.ms(6, 7);
  H.stats.t_total_s = H.stats.t_screen_s + H.stats.t_count_s + H.stats.t_scan_s + H.stats.t_fill_s;
  // the per-stage device times of the profile come from the stage events
  // above (timers of their own inside the stages would hold the device idle
  // while the host records them between the short kernels)
  profile_add(ctx, K_SCREEN, H.stats.t_screen_s);
  profile_add(ctx, K_ROW_COUNT, H.stats.t_count_s);
  profile_add(ctx, K_SCAN, H.stats.t_scan_s);
  profile_add(ctx, K_ROW_FILL, H.stats.t_fill_s);
  H.stats.n_tiles = n_tiles;
  H.stats.n_adjacent = n_ls + n_l1;
}

void apply_matrix_free(cib_ctx *ctx, const cib_basis &b, const cib_interaction &it, cib_dtype dt,
                       const ApplyReq &a, hipStream_t s) {
  cib_matrix unused;
  unused.ctx = ctx;
  switch (b.plan.W) {
    case 1: build_w<1>(ctx, b, it, dt, unused, s, nullptr, &a); break;
    case 2: build_w<2>(ctx, b, it, dt, unused, s, nullptr, &a); break;
    default: build_w<3>(ctx, b, it, dt, unused, s, nullptr, &a); break;
  }
}

void build_matrix(cib_ctx *ctx, const cib_basis &b, const cib_interaction &it, cib_dtype dt,
                  cib_matrix &H, hipStream_t s, const BuildReserve &reserve) {
  switch (b.plan.W) {
    case 1: build_w<1>(ctx, b, it, dt, H, s, reserve); break;
    case 2: build_w<2>(ctx, b, it, dt, H, s, reserve); break;
    default: build_w<3>(ctx, b, it, dt, H, s, reserve); break;
  }
}

}  // namespace cib
