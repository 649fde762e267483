// Block-diagonal preconditioner over many-body basis orbitals (Sec. 2: the
// states whose particles have the same (n, l, j) values, whatever their m,
// form a group, and the groups give LOBPCG a block-diagonal preconditioner).
//
// Set-up, once per matrix:
//   1  groups (host, from the basis plan): each species configuration is
//      reduced to its level occupations (particles per (n, 2j) level), a
//      state's group is the pair of its species' occupation classes; groups
//      are ordered by their lowest state, states ascending inside a group,
//      and a group of more than max_block states is cut into consecutive
//      runs of max_block;
//   2  k_pc_extract: the dense diagonal blocks of H from its upper half, one
//      wave per row (each unordered pair inside a block is stored once in
//      the half matrix, so every element is written once);
//   3  k_pc_jacobi: each block's eigenpairs by cyclic Jacobi rotations in
//      round-robin order (the n/2 rotations of a round touch disjoint rows
//      and columns and are applied together), one workgroup per block with
//      the block and its rotations in LDS, until the off-diagonal part is
//      below 1e-15 of the block's Frobenius norm.
// Application, per LOBPCG iteration: W[:, c] = Q diag(1 / g(lambda_j -
// theta_c)) Q^T R[:, c] per block, g the guard of the diagonal
// preconditioner (gaps below 1e-2 in magnitude move to +-1e-2), one
// workgroup per block; blocks of one state give exactly the diagonal
// preconditioner's bits.
#include <algorithm>
#include <map>
#include <vector>

#include "cib_internal.hpp"
#include "device_common.hpp"

namespace cib {

constexpr int kPcMax = 64;        // largest block
constexpr int kPcCols = 16;       // columns per application
constexpr int kPcSweeps = 40;     // Jacobi sweep limit

__device__ __forceinline__ double pc_gap(double x) {
  if (fabs(x) < 1e-2) x = x < 0 ? -1e-2 : 1e-2;
  return x;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pc_extract(int64_t D, const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const int32_t *__restrict__ blk, const int32_t *__restrict__ pos,
                                                    const int64_t *__restrict__ boff, const int64_t *__restrict__ qoff,
                                                    double *__restrict__ M) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= D) return;
  const int lane = threadIdx.x & 63;
  const int k = blk[i], pi = pos[i];
  const int s = (int)(boff[k + 1] - boff[k]);
  double *Mk = M + qoff[k];
  for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) {
    const int j = col[e];
    if (blk[j] != k) continue;
    const int pj = pos[j];
    const double v = (double)val[e];
    Mk[pi * s + pj] = v;
    Mk[pj * s + pi] = v;
  }
}

// In: M holds each block (s x s, row-major).  Out: M holds its eigenvectors
// (column j = eigenvector j) and lam[boff[k] + j] eigenvalue j; sweeps[k]
// the sweeps taken.  SM >= every block's size (LDS tiles of SM rows).
template <int SM>
__global__ __launch_bounds__(256) void k_pc_jacobi(const int64_t *__restrict__ boff, const int64_t *__restrict__ qoff,
                                                   double *__restrict__ M, double *__restrict__ lam,
                                                   int32_t *__restrict__ sweeps) {
  __shared__ double A[SM][SM + 1], V[SM][SM + 1];
  __shared__ double cs[SM / 2], sn[SM / 2];
  __shared__ int pp[SM / 2], qq[SM / 2];
  __shared__ double red[2][256];
  const int t = threadIdx.x, k = blockIdx.x;
  const int64_t o = boff[k];
  const int s = (int)(boff[k + 1] - o);
  const int n = s + (s & 1), m = n / 2;   // an odd size gets an idle zero row/column
  double *Mk = M + qoff[k];
  for (int e = t; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    A[r][c] = (r < s && c < s) ? Mk[r * s + c] : 0.0;
    V[r][c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < kPcSweeps && n > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = t; e < n * n; e += 256) {
      const int r = e / n, c = e % n;
      const double a2 = A[r][c] * A[r][c];
      tot += a2;
      if (r != c) off += a2;
    }
    red[0][t] = off;
    red[1][t] = tot;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) {
        red[0][t] += red[0][t + h];
        red[1][t] += red[1][t + h];
      }
      __syncthreads();
    }
    const bool done = red[0][0] <= 1e-30 * red[1][0];
    __syncthreads();   // red is rewritten by the next sweep's sums
    if (done) break;
    for (int rnd = 0; rnd < n - 1; ++rnd) {
      if (t < m) {
        // circle method: position 0 fixed, the others rotate by rnd
        const int a = t == 0 ? 0 : 1 + (t - 1 + rnd) % (n - 1);
        const int b = 1 + (n - 2 - t + rnd) % (n - 1);
        const int p = min(a, b), q = max(a, b);
        const double apq = A[p][q];
        double c = 1.0, sv = 0.0;
        if (apq != 0.0) {
          // the rotation that zeroes (p, q): t = sgn(tau) / (|tau| + sqrt(1 + tau^2))
          const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sv = tt * c;
        }
        pp[t] = p;
        qq[t] = q;
        cs[t] = c;
        sn[t] = sv;
      }
      __syncthreads();
      for (int e = t; e < m * n; e += 256) {   // rows p, q of J^T A
        const int i = e / n, x = e % n;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], sv = sn[i];
        const double ap = A[p][x], aq = A[q][x];
        A[p][x] = c * ap - sv * aq;
        A[q][x] = sv * ap + c * aq;
      }
      __syncthreads();
      for (int e = t; e < m * n; e += 256) {   // columns p, q of (J^T A) J and V J
        const int i = e / n, x = e % n;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], sv = sn[i];
        const double ap = A[x][p], aq = A[x][q];
        A[x][p] = c * ap - sv * aq;
        A[x][q] = sv * ap + c * aq;
        const double vp = V[x][p], vq = V[x][q];
        V[x][p] = c * vp - sv * vq;
        V[x][q] = sv * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int e = t; e < s * s; e += 256) Mk[e] = V[e / s][e % s];
  if (t < s) lam[o + t] = A[t][t];
  if (t == 0) sweeps[k] = sweep;
}

// W[perm rows of block k][c] = Q (Q^T R / g(lam - theta_c)); W may be R (each
// block reads all its rows before it writes them, and blocks share no rows).
template <int SM>
__global__ __launch_bounds__(256) void k_pc_apply(const int32_t *__restrict__ perm, const int64_t *__restrict__ boff,
                                                  const int64_t *__restrict__ qoff, const double *__restrict__ Q,
                                                  const double *__restrict__ lam, const double *__restrict__ theta,
                                                  int ncol, const double *R, int64_t ldr, double *W, int64_t ldw,
                                                  float *__restrict__ w32, int64_t ld32) {
  __shared__ double Qs[SM][SM + 1];
  __shared__ double Rs[SM][kPcCols + 1], Ts[SM][kPcCols + 1];
  __shared__ double th[kPcCols];
  const int t = threadIdx.x, k = blockIdx.x;
  const int64_t o = boff[k];
  const int s = (int)(boff[k + 1] - o);
  const double *Qk = Q + qoff[k];
  for (int e = t; e < s * s; e += 256) Qs[e / s][e % s] = Qk[e];
  for (int e = t; e < s * ncol; e += 256) {
    const int a = e / ncol, c = e % ncol;
    Rs[a][c] = R[(int64_t)perm[o + a] * ldr + c];
  }
  if (t < ncol) th[t] = theta[t];
  __syncthreads();
  for (int e = t; e < s * ncol; e += 256) {
    const int j = e / ncol, c = e % ncol;
    double acc = 0.0;
    for (int a = 0; a < s; ++a) acc += Qs[a][j] * Rs[a][c];
    Ts[j][c] = acc / pc_gap(lam[o + j] - th[c]);
  }
  __syncthreads();
  for (int e = t; e < s * ncol; e += 256) {
    const int a = e / ncol, c = e % ncol;
    double acc = 0.0;
    for (int j = 0; j < s; ++j) acc += Qs[a][j] * Ts[j][c];
    const int64_t row = perm[o + a];
    W[row * ldw + c] = acc;
    if (w32) w32[row * ld32 + c] = (float)acc;
  }
}

namespace {

// level-occupation class of each configuration of one species
std::vector<int32_t> occupation_classes(const SubList &L, const Orbs &o) {
  std::vector<int> level(o.n_orb);
  int nlev = 0;
  for (int a = 0; a < o.n_orb; ++a) {
    if (a > 0 && (o.n[a] != o.n[a - 1] || o.twoj[a] != o.twoj[a - 1])) ++nlev;
    level[a] = nlev;
  }
  ++nlev;
  std::map<std::vector<uint8_t>, int32_t> ids;
  std::vector<int32_t> cls(L.size());
  std::vector<uint8_t> occ(nlev);
  for (size_t k = 0; k < L.size(); ++k) {
    std::fill(occ.begin(), occ.end(), 0);
    for (int a = 0; a < o.n_orb; ++a)
      if ((L.bits[k * kMaxWords + a / 64] >> (a % 64)) & 1) ++occ[level[a]];
    auto it = ids.emplace(occ, (int32_t)ids.size()).first;
    cls[k] = it->second;
  }
  return cls;
}

}  // namespace

void precond_create(cib_ctx *ctx, const cib_basis &b, const cib_matrix &H, int max_block, cib_precond &P,
                    hipStream_t st) {
  const Plan &pl = b.plan;
  const int64_t D = pl.D;
  const std::vector<int32_t> ca = occupation_classes(pl.A, pl.oA);
  std::vector<int32_t> cb;
  if (pl.ns == 2) cb = occupation_classes(pl.B, pl.oB);
  const int64_t ncb = pl.ns == 2 ? (int64_t)*std::max_element(cb.begin(), cb.end()) + 1 : 1;
  // group of each state, numbered by first appearance in state order
  // (a direct table over the key range when it is small, else a map)
  const int64_t nca = *std::max_element(ca.begin(), ca.end()) + 1;
  const bool direct = nca * ncb <= (int64_t(1) << 22);
  std::vector<int32_t> table(direct ? nca * ncb : 0, -1);
  std::map<int64_t, int32_t> gid;
  int32_t ngi = 0;
  std::vector<int32_t> grp(D);
  for (int alpha = 0; alpha < pl.nA(); ++alpha)
    for (int64_t i = pl.a_off[alpha]; i < pl.a_off[alpha + 1]; ++i) {
      int64_t key = ca[alpha] * ncb;
      if (pl.ns == 2) key += cb[pl.bseg_start[pl.a_seg[alpha]] + (i - pl.a_off[alpha])];
      int32_t &slot = direct ? table[key] : gid.emplace(key, -1).first->second;
      if (slot < 0) slot = ngi++;
      grp[i] = slot;
    }
  const int64_t ng = ngi;
  std::vector<int64_t> gstart(ng + 1, 0);
  for (int64_t i = 0; i < D; ++i) ++gstart[grp[i] + 1];
  for (int64_t g = 0; g < ng; ++g) gstart[g + 1] += gstart[g];
  P.perm_h.assign(D, 0);
  {
    std::vector<int64_t> fill(gstart.begin(), gstart.end() - 1);
    for (int64_t i = 0; i < D; ++i) P.perm_h[fill[grp[i]]++] = (int32_t)i;
  }
  // runs of at most max_block inside each group
  P.boff_h.clear();
  for (int64_t g = 0; g < ng; ++g)
    for (int64_t x = gstart[g]; x < gstart[g + 1]; x += max_block) P.boff_h.push_back(x);
  P.boff_h.push_back(D);
  const int64_t nb = (int64_t)P.boff_h.size() - 1;
  std::vector<int64_t> qoff(nb + 1, 0);
  std::vector<int32_t> blk(D), pos(D);
  int largest = 0;
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t sk = P.boff_h[k + 1] - P.boff_h[k];
    largest = std::max(largest, (int)sk);
    qoff[k + 1] = qoff[k] + sk * sk;
    for (int64_t x = P.boff_h[k]; x < P.boff_h[k + 1]; ++x) {
      blk[P.perm_h[x]] = (int32_t)k;
      pos[P.perm_h[x]] = (int32_t)(x - P.boff_h[k]);
    }
  }
  P.ctx = ctx;
  P.D = D;
  P.n_blocks = nb;
  P.n_groups = ng;
  P.largest = largest;
  P.max_block = max_block;
  P.perm.reset(ctx, D);
  P.boff.reset(ctx, nb + 1);
  P.qoff.reset(ctx, nb + 1);
  P.Q.reset(ctx, qoff[nb]);
  P.lam.reset(ctx, D);
  P.theta.reset(ctx, kPcCols);
  DBuf<int32_t> dblk(ctx, D), dpos(ctx, D), sw(ctx, nb);
  // waits for the stream before the buffers above (and the caller's P, if a
  // step throws) are released
  struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
  } sync_on_exit{st};
  P.perm.upload(P.perm_h.data(), D, st);
  P.boff.upload(P.boff_h.data(), nb + 1, st);
  P.qoff.upload(qoff.data(), nb + 1, st);
  dblk.upload(blk.data(), D, st);
  dpos.upload(pos.data(), D, st);
  CIB_HIP(hipMemsetAsync(P.Q.p, 0, P.Q.bytes(), st));
  const dim3 ge((unsigned)((D + 3) / 4));
  if (H.dtype == CIB_F64)
    hipLaunchKernelGGL(k_pc_extract<double>, ge, dim3(256), 0, st, D, H.row_ptr.p, H.col.p, H.val64.p, dblk.p,
                       dpos.p, P.boff.p, P.qoff.p, P.Q.p);
  else
    hipLaunchKernelGGL(k_pc_extract<float>, ge, dim3(256), 0, st, D, H.row_ptr.p, H.col.p, H.val32.p, dblk.p,
                       dpos.p, P.boff.p, P.qoff.p, P.Q.p);
  const dim3 gj((unsigned)nb);
  if (largest <= 16) hipLaunchKernelGGL(k_pc_jacobi<16>, gj, dim3(256), 0, st, P.boff.p, P.qoff.p, P.Q.p, P.lam.p, sw.p);
  else if (largest <= 32) hipLaunchKernelGGL(k_pc_jacobi<32>, gj, dim3(256), 0, st, P.boff.p, P.qoff.p, P.Q.p, P.lam.p, sw.p);
  else hipLaunchKernelGGL(k_pc_jacobi<kPcMax>, gj, dim3(256), 0, st, P.boff.p, P.qoff.p, P.Q.p, P.lam.p, sw.p);
  CIB_HIP(hipGetLastError());
  std::vector<int32_t> swh(nb);
  CIB_HIP(hipMemcpyAsync(swh.data(), sw.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
  CIB_HIP(hipStreamSynchronize(st));
  P.max_sweeps = nb ? *std::max_element(swh.begin(), swh.end()) : 0;
}

void precond_apply(const cib_precond &P, const double *theta_dev, int ncol, const double *R, int64_t ldr, double *W,
                   int64_t ldw, float *w32, int64_t ld32, hipStream_t st) {
  const dim3 g((unsigned)P.n_blocks);
  if (P.largest <= 16)
    hipLaunchKernelGGL(k_pc_apply<16>, g, dim3(256), 0, st, P.perm.p, P.boff.p, P.qoff.p, P.Q.p, P.lam.p, theta_dev,
                       ncol, R, ldr, W, ldw, w32, ld32);
  else if (P.largest <= 32)
    hipLaunchKernelGGL(k_pc_apply<32>, g, dim3(256), 0, st, P.perm.p, P.boff.p, P.qoff.p, P.Q.p, P.lam.p, theta_dev,
                       ncol, R, ldr, W, ldw, w32, ld32);
  else
    hipLaunchKernelGGL(k_pc_apply<kPcMax>, g, dim3(256), 0, st, P.perm.p, P.boff.p, P.qoff.p, P.Q.p, P.lam.p,
                       theta_dev, ncol, R, ldr, W, ldw, w32, ld32);
  CIB_HIP(hipGetLastError());
}

}  // namespace cib
