// Rayleigh-Ritz step of block LOBPCG (Fig. 1 step 15): the lowest b
// eigenpairs of the pencil (S^T H S, S^T S) for the search space
// S = [X | W | P], in one workgroup of 256 threads (four waves).
//
// Included by lobpcg.hip inside namespace cib (it uses kNS, kLd, dbl4,
// RRArgs and the device helpers declared there).
//
// (1) reduce the partial Gram matrices; (2) scale both to the unit diagonal
// of S^T S; (3) Cholesky S^T S = L L^T, dropping columns whose residual
// pivot is at most drop_tol (directions already spanned); (4) the kept rows
// and columns compacted, Z = L^-1 and the reduced matrix M = Z (S^T H S) Z^T;
// (5) Householder reduction of M to a tridiagonal T; (6) the lowest b
// eigenvalues of T by multisection of Sturm counts; (7) their eigenvectors
// from twisted factorisations of T - theta I, re-orthogonalised inside
// clusters; (8) back to M's basis with the reflectors; (9) coefficients
// C_x = scale * Z^T y in S's columns and C_p = C_x with the X rows zeroed
// (P = W C_W + P C_P).
//
// Costs on the matrix cores' hosts: one wave issues a dependent float64
// operation every ~9 cycles and an independent one every ~5.6; an LDS read
// returns after ~60 cycles; a workgroup barrier costs ~10.  The sequential
// parts are therefore written as short runtime loops whose per-step
// dependent chain is one or two operations, with the wide work spread over
// the four waves, and without per-step division or square root.

// 1 / x from the hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Sum over each row of 16 lanes, returned to all 16 (the same bits in every
// lane: each stage adds the same two operands, in either order).
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}

// Minimum and maximum over the wave (all lanes active), in every lane.
__device__ __forceinline__ void wave_minmax(double &lo, double &hi) {
  lo = fmin(lo, dpp_f64<0xB1>(lo)); hi = fmax(hi, dpp_f64<0xB1>(hi));
  lo = fmin(lo, dpp_f64<0x4E>(lo)); hi = fmax(hi, dpp_f64<0x4E>(hi));
  lo = fmin(lo, dpp_f64<0x141>(lo)); hi = fmax(hi, dpp_f64<0x141>(hi));
  lo = fmin(lo, dpp_f64<0x140>(lo)); hi = fmax(hi, dpp_f64<0x140>(hi));
  lo = fmin(fmin(readlane_f64(lo, 0), readlane_f64(lo, 16)), fmin(readlane_f64(lo, 32), readlane_f64(lo, 48)));
  hi = fmax(fmax(readlane_f64(hi, 0), readlane_f64(hi, 16)), fmax(readlane_f64(hi, 32), readlane_f64(hi, 48)));
}

// Number of eigenvalues below x of the symmetric tridiagonal T with diagonal
// d and squared off-diagonal e2, T scaled so that its Gershgorin interval
// lies within [-2, 2] and every inner e2 >= 2^-100.  In LDS, read at the same
// address by every lane: d[0 .. n) and es[j] = e2_{j-1} (es[0] = 0), n a
// multiple of 8 <= 64, padded past the matrix with d = 4 > x and es = 0,
// which add no sign change.  The count is the number of sign changes of
// p_{-1} = 1, p_j = (d_j - x) p_{j-1} - e2_{j-1} p_{j-2} (the characteristic
// polynomials of the leading blocks), i.e. of negative pivots of
// T - x I = L D L^T.  One FMA per step is dependent; the sign bits are
// shifted into a 64-bit word and the changes counted at the end.  A zero p_j
// counts as positive, which with e2 > 0 gives the count of the pivot -0
// (p_{j+1} = -e2 p_{j-1} then carries the change).  p is rescaled by a power
// of two (exact) every 8 steps when it leaves [2^-200, 2^200]: within 8
// steps it grows at most 5^8-fold and shrinks at most 2^-400-fold.
__device__ __forceinline__ int sturm_lds(const double *d, const double *es, int n, double x) {
  double pm = 0.0, p = 1.0;
  uint32_t bhi = 0, blo = 0;
  for (int j0 = 0; j0 < n; j0 += 8) {
    double dv[8], ev[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      dv[t] = d[j0 + t];
      ev[t] = es[j0 + t];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const double pn = fma(dv[t] - x, p, -(ev[t] * pm));
      pm = p;
      p = pn;
      bhi = __builtin_amdgcn_alignbit(bhi, blo, 31);
      blo = __builtin_amdgcn_alignbit(blo, (uint32_t)(__builtin_bit_cast(uint64_t, p) >> 32), 31);
    }
    const double mx = fmax(fabs(p), fabs(pm));
    if (mx > 0x1p200 || mx < 0x1p-200) {
      const double s = ldexp(1.0, -ilogb(mx));
      p *= s;
      pm *= s;
    }
  }
  const uint64_t bits = ((uint64_t)bhi << 32) | blo;   // p_0 at bit n - 1, p_{n-1} at bit 0
  return __popcll(bits ^ (bits >> 1));
}

__device__ __forceinline__ void rayleigh_ritz(const RRArgs &g) {
  constexpr int kCW = kNS / 4;   // columns per wave in the Cholesky and Z steps
  __shared__ double GH[2][kNS][kLd], Z[kNS][kLd];
  double (&G)[kNS][kLd] = GH[0];    // S^T S, then L, then workspace
  double (&Hm)[kNS][kLd] = GH[1];   // S^T H S, then M and the reflectors
  __shared__ double scale[kNS], dd[kNS], ee[kNS], e2[kNS], beta[kNS], dinv[kNS];
  __shared__ double pw[4][kWave], hv[4][kWave], hw[4][kWave], sg[4], xb[kWave];   // Householder: partial products, v, w, next row and its norm
  __shared__ double colbuf[2][kWave];   // column k of L at Cholesky step k
  __shared__ double rowbuf[4][16];      // row q of a diagonal block of Z, per wave
  __shared__ double Tt[3][16][17];      // tile products while Z is formed
  __shared__ double theta[kMaxBlock], vnrm[kMaxBlock], bnd[4];
  __shared__ double dsc[kNS + 8], esc[kNS + 8];   // T for the Sturm counts, padded
  __shared__ int keep[kNS], kidx[kNS], twi[kMaxBlock];
  __shared__ int rank_s, retry_s;
  const int ns_full = g.ns, b = g.b, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & (kWave - 1), wv = uni((int)(tid >> 6));
  int ns = ns_full, r = 0, nb = 0;
  double drop_tol = g.drop_tol, sc = 1.0, tns = 1.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
  // -- phase 1
  // 1. S^T S and S^T H S, stored by the Gram reduction in this kernel's
  //    layout (two kNS x kLd blocks), copied as they are in 16-byte pieces;
  //    only rows and columns below ns are used (a retry keeps the leading
  //    [X W] blocks)
  {
    constexpr int kPieces = kNS * kLd;   // 16-byte pieces in both blocks
    constexpr int kPer = (kPieces + 255) / 256;
    const double2 *src = reinterpret_cast<const double2 *>(g.gram);
    double2 *dst = reinterpret_cast<double2 *>(&GH[0][0][0]);
    double2 v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = tid + 256 * t;
      v[t] = src[e < kPieces ? e : 0];
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t)
      if (tid + 256 * t < kPieces) dst[tid + 256 * t] = v[t];
  }
  __syncthreads();
  // -- phase 2
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
  // -- phase 3
  // 3. right-looking Cholesky with dropping over a 16 x 16 grid of threads:
  //    thread (i0, j0) holds rows i0 + 16 ra and columns j0 + 16 cb (ra, cb
  //    < 3) in registers.  Column k belongs to the 16 threads with j0 = k mod
  //    16 (one row of 16 lanes): they read the pivot from the lane holding
  //    (k, k), form the column (1/sqrt from the hardware estimate and one
  //    Newton step; zero when dropped) and publish it in LDS; after one
  //    barrier every thread subtracts l_ik l_jk from its nine elements.  The
  //    multipliers of rows and columns up to k are zero, so the factor's
  //    columns stay as formed; only the lower triangle and the diagonal are
  //    read afterwards.
  {
    const int i0 = tid & 15, j0 = tid >> 4;
    const uint64_t okm = __ballot(lane < ns && scale[lane < kNS ? lane : 0] > 0.0);   // nonzero columns
    double a[3][3];
#pragma unroll
    for (int ra = 0; ra < 3; ++ra)
#pragma unroll
      for (int cb = 0; cb < 3; ++cb) {
        const int i = i0 + 16 * ra, j = j0 + 16 * cb;
        a[ra][cb] = (i < ns && j < ns) ? G[i][j] : 0.0;
      }
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)   // the column block: the owners' registers are fixed
#pragma unroll 1
      for (int km = 0; km < 16; ++km) {
        const int k = 16 * kb + km;
        if (k >= ns) break;
        if (j0 == km) {
          const int src = ((tid & 63) & ~15) | km;   // the lane of this row of 16 that holds (k, k)
          const uint64_t u = __builtin_bit_cast(uint64_t, a[kb][kb]);
          const double piv = __builtin_bit_cast(
              double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src) << 32) |
                          (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src));
          const bool kk = ((okm >> k) & 1ull) && piv > drop_tol;   // every owner decides the same
          const double pv = kk ? piv : 1.0;
          double y = __builtin_amdgcn_rsq(pv);
          y = y * fma(-0.5 * pv * y, y, 1.5);
#pragma unroll
          for (int ra = 0; ra < 3; ++ra) {
            const int i = i0 + 16 * ra;
            const double c = a[ra][kb];
            const double l = (kk && i > k && i < ns) ? c * y : 0.0;
            a[ra][kb] = i > k ? l : (i == k ? (kk ? piv * y : 0.0) : c);
            colbuf[k & 1][i] = l;
          }
          if (i0 == 0) keep[k] = kk;
        }
        __syncthreads();
        double lr[3], lc[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          lr[m] = colbuf[k & 1][i0 + 16 * m];
          lc[m] = colbuf[k & 1][j0 + 16 * m];
        }
#pragma unroll
        for (int ra = 0; ra < 3; ++ra)
#pragma unroll
          for (int cb = 0; cb < 3; ++cb) a[ra][cb] -= lr[ra] * lc[cb];
      }
#pragma unroll
    for (int ra = 0; ra < 3; ++ra)
#pragma unroll
      for (int cb = 0; cb < 3; ++cb) {
        const int i = i0 + 16 * ra, j = j0 + 16 * cb;
        if (i < ns && j < ns) G[i][j] = a[ra][cb];
      }
  }
  __syncthreads();
  // -- phase 4
  // 4a. compact L (G) and S^T H S (Hm) to the kept rows and columns, in
  //     place: kidx increases, so every source lies at or after its target
  //     in both indices, and a batch's loads precede its stores
  if (tid < kWave) {
    const int i = tid;
    const bool kp = i < ns && keep[i];
    const uint64_t km = __ballot(kp);
    if (kp) kidx[mask_rank(km)] = i;
    if (i == 0) rank_s = (int)__popcll(km);
    wave_lds_sync();
    const int rr = rank_s;
    if (rr < ns && i < rr) {
      const int ka = kidx[i];
      for (int q0 = 0; q0 < rr; q0 += 8) {
        double lv[8], hv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int kq = kidx[min(q0 + t, rr - 1)];
          lv[t] = G[ka][kq];
          hv[t] = Hm[ka][kq];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (q0 + t < rr) {
            G[i][q0 + t] = lv[t];
            Hm[i][q0 + t] = hv[t];
          }
      }
    }
    wave_lds_sync();
    if (i < rr) dinv[i] = 1.0 / G[i][i];
  }
  __syncthreads();
  r = rank_s;
  // -- phase 10
  // 4b. Z = L^-1 by 16 x 16 blocks, L taken as the identity past r.  The
  //     three diagonal blocks are inverted at once (wave w: lanes = the rows
  //     of block w, the block's columns in registers; at step q lane q
  //     publishes its row and every row below subtracts L_aq / L_qq times
  //     it; rows scaled by 1 / L_aa at the end).  The blocks below the
  //     diagonal follow from tile products on the matrix cores:
  //     Z10 = -Z11 (L10 Z00), Z21 = -Z22 (L21 Z11), Z20 = -Z22 (L20 Z00 + L21 Z10).
  for (int e = tid; e < kNS * kLd; e += nt) (&Z[0][0])[e] = 0.0;
  __syncthreads();
  if (wv < 3) {
    const int a = lane & 15, ga = 16 * wv + a;   // lanes 16..63 shadow lanes 0..15
    double zr[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) zr[m] = a == m ? 1.0 : 0.0;
#pragma unroll 1
    for (int q = 0; q < 16; ++q) {
      const int gq = 16 * wv + q;
      const double laq = (a > q && ga < r) ? G[ga][gq] * dinv[gq] : 0.0;
      if (lane == q)
#pragma unroll
        for (int m = 0; m < 16; ++m) rowbuf[wv][m] = zr[m];
      wave_lds_sync();
#pragma unroll
      for (int m = 0; m < 16; ++m) zr[m] -= laq * rowbuf[wv][m];
      wave_lds_sync();
    }
    const double da = ga < r ? dinv[ga] : 1.0;
    if (lane < 16)
#pragma unroll
      for (int m = 0; m < 16; ++m) Z[ga][16 * wv + m] = zr[m] * da;
  }
  __syncthreads();
  {
    // one 16 x 16 tile product per wave and stage; L's blocks below the
    // diagonal are read as zero past r
    const int kr = lane >> 4, kc = lane & 15;
    auto lmat = [&](int i, int j) { return (i < r && j < r) ? G[i][j] : 0.0; };
    auto tile = [&](auto A, int ra, auto B, int cb, int ka, dbl4 acc) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = ka + 4 * s4 + kr;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A(ra + kc, k), B(k, cb + kc), acc, 0, 0, 0);
      }
      return acc;
    };
    auto zmat = [&](int i, int j) { return Z[i][j]; };
    auto tmat = [&](int i, int j) { return Tt[wv][i & 15][j & 15]; };
    auto store_t = [&](int slot, dbl4 acc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Tt[slot][4 * v + kr][kc] = acc[v];
    };
    const dbl4 z4 = {0.0, 0.0, 0.0, 0.0};
    // stage 1: T10 = L10 Z00 (wave 0), T21 = L21 Z11 (wave 1), T20 = L20 Z00 (wave 2)
    if (wv == 0) store_t(0, tile(lmat, 16, zmat, 0, 0, z4));
    else if (wv == 1) store_t(1, tile(lmat, 32, zmat, 16, 16, z4));
    else if (wv == 2) store_t(2, tile(lmat, 32, zmat, 0, 0, z4));
    __syncthreads();
    // stage 2: Z10 = -Z11 T10 (wave 0), Z21 = -Z22 T21 (wave 1)
    if (wv < 2) {
      const int d = 16 * (wv + 1);   // the diagonal block multiplying
      const dbl4 acc = tile(zmat, d, tmat, 0, d, z4);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[d + 4 * v + kr][16 * wv + kc] = -acc[v];
    }
    __syncthreads();
    // stage 3: T20 += L21 Z10 (wave 0; T20 in slot 2)
    if (wv == 0) {
      dbl4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = Tt[2][4 * v + kr][kc];
      store_t(2, tile(lmat, 32, zmat, 0, 16, acc));
    }
    __syncthreads();
    // stage 4: Z20 = -Z22 T20 (wave 0)
    if (wv == 0) {
      auto t2 = [&](int i, int j) { return Tt[2][i & 15][j & 15]; };
      const dbl4 acc = tile(zmat, 32, t2, 0, 32, z4);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[32 + 4 * v + kr][kc] = -acc[v];
    }
  }
  __syncthreads();
  // -- phase 11
  // 4c. T1 = A Z^T into G, then M = Z T1 into Hm (A = compacted S^T H S,
  //     zero outside r x r), as 3 x 3 tiles of 16 x 16 on the matrix cores:
  //     wave w takes tiles w, w + 4, w + 8, their products interleaved
  //     (independent accumulators); Z is block lower triangular, which
  //     bounds the k-steps of the second product.
  {
    const int kr = lane >> 4, kc = lane & 15;
    dbl4 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int s4 = 0; s4 < kNS / 4; ++s4) {
      const int ka = 4 * s4 + kr;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int tile = wv + 4 * t;
        if (tile < 9) {
          const int ra = 16 * (tile / 3) + kc, cq = 16 * (tile % 3) + kc;
          const double av = (ra < r && ka < r) ? Hm[ra][ka] : 0.0;
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Z[cq][ka], acc[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int tile = wv + 4 * t;
      if (tile < 9)
#pragma unroll
        for (int v = 0; v < 4; ++v) G[16 * (tile / 3) + 4 * v + kr][16 * (tile % 3) + kc] = acc[t][v];
      acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 2
    for (int s4 = 0; s4 < kNS / 4; ++s4) {
      const int ka = 4 * s4 + kr;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int tile = wv + 4 * t, ta = tile / 3;
        if (tile < 9 && s4 < 4 * (ta + 1))
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Z[16 * ta + kc][ka], G[ka][16 * (tile % 3) + kc], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int tile = wv + 4 * t;
      if (tile < 9)
#pragma unroll
        for (int v = 0; v < 4; ++v) Hm[16 * (tile / 3) + 4 * v + kr][16 * (tile % 3) + kc] = acc[t][v];
    }
  }
  __syncthreads();
  // -- phase 16
  for (int e = tid; e < r * r; e += nt) {
    const int i = e / r, j = e % r;
    if (i < j) {
      const double v = 0.5 * (Hm[i][j] + Hm[j][i]);
      Hm[i][j] = v;
      Hm[j][i] = v;
    }
  }
  __syncthreads();
  // -- phase 5
  // 5. Householder tridiagonalisation of M (r x r), kept symmetric in
  //    registers: lane i of wave w holds row i, columns [kCW w, kCW w + kCW).
  //    Step k: x = row k right of the diagonal (published in LDS by lane k
  //    of every wave when it finished the previous step, with the partial
  //    squared norms of its columns); the reflector v and its scale (every
  //    wave alike, so the same bits); p = beta A v over each wave's columns,
  //    summed in LDS in wave order; w = p - K v with K = beta v.p / 2; A -= v
  //    w^T + w v^T.  v and w are zero outside (k, r), so no product needs a
  //    test; each wave keeps its own copy of them in LDS, read back at one
  //    address by all lanes.  Reflector k is kept in column k of Hm below
  //    the subdiagonal, its scale in beta[k]; Hm's diagonal and last
  //    subdiagonal entry are written back at the end.
  {
    const int i = lane;
    const int ic = i < kNS ? i : kNS - 1;
    const int jw = kCW * wv;
    double ar[kCW];
#pragma unroll
    for (int q = 0; q < kCW; ++q) ar[q] = (i < r && jw + q < r) ? Hm[ic][jw + q] : 0.0;
    if (wv == 0) {
      const double x = (i > 0 && i < r) ? Hm[0][ic] : 0.0;
      if (i < kNS) xb[i] = x;
      const double s0 = wave_sum_dpp(x * x);
      if (i < 4) sg[i] = i == 0 ? s0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k + 2 < r; ++k) {
      const bool act = i < r && i > k;
      const double xi = act ? xb[ic] : 0.0;
      const double sigma = (sg[0] + sg[1]) + (sg[2] + sg[3]);
      const double x0 = xb[k + 1];
      const double tail = sigma - x0 * x0;
      const bool refl = tail > 1e-300;
      double alpha = x0, bk = 0.0;
      if (refl) {   // every lane alike
        double y = __builtin_amdgcn_rsq(sigma);
        y = y * fma(-0.5 * sigma * y, y, 1.5);
        alpha = -copysign(sigma * y, x0);
        bk = 2.0 * rcp_f64(tail + (x0 - alpha) * (x0 - alpha));
      }
      const double vi = i == k + 1 ? x0 - alpha : xi;
      hv[wv][i] = vi;
      wave_lds_sync();
      double vv[kCW];
#pragma unroll
      for (int q = 0; q < kCW; ++q) vv[q] = hv[wv][jw + q];
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < kCW; q += 2) {
        a0 = fma(ar[q], vv[q], a0);
        a1 = fma(ar[q + 1], vv[q + 1], a1);
      }
      pw[wv][i] = act ? a0 + a1 : 0.0;
      __syncthreads();
      const double pi = bk * ((pw[0][i] + pw[1][i]) + (pw[2][i] + pw[3][i]));
      const double K = 0.5 * bk * wave_sum_dpp(vi * pi);
      const double wi = pi - K * vi;
      hw[wv][i] = wi;
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < kCW; ++q) ar[q] = fma(-wi, vv[q], fma(-vi, hw[wv][jw + q], ar[q]));
      // squared norm of the next row right of its diagonal (columns past r
      // hold zeros); only the wave holding column k + 1 needs a mask
      double s2 = 0.0;
      if (jw > k + 1) {
#pragma unroll
        for (int q = 0; q < kCW; ++q) s2 = fma(ar[q], ar[q], s2);
      } else if (jw + kCW > k + 2) {
#pragma unroll
        for (int q = 0; q < kCW; ++q) s2 = jw + q > k + 1 ? fma(ar[q], ar[q], s2) : s2;
      }
      if (i == k + 1) {   // the next row, for the next step
#pragma unroll
        for (int q = 0; q < kCW; ++q) xb[jw + q] = ar[q];
        sg[wv] = s2;
      }
      if (wv == 0 && act) Hm[i][k] = vi;
      if (tid == 0) {
        beta[k] = bk;
        ee[k] = alpha;
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kCW; ++q) {
      const int j = jw + q;
      if (i < r && (j == i || (i == r - 1 && j == r - 2))) Hm[i][j] = ar[q];
    }
  }
  __syncthreads();
  for (int i = tid; i < r; i += nt) {
    dd[i] = Hm[i][i];
    if (i == r - 2) ee[i] = Hm[r - 1][r - 2];
  }
  __syncthreads();
  // -- phase 6
  // 6. lowest nb eigenvalues of T by multisection.  T is scaled by the power
  //    of two sc that brings its Gershgorin bound tns into [1, 2) (d, e and
  //    theta are kept scaled from here on).  gsz threads per eigenvalue (32
  //    when nb <= 8, else 16), each round cutting the interval into gsz + 1
  //    parts, until (gsz + 1)^rounds > 2^53.
  nb = b < r ? b : r;
  if (tid < kWave) {
    const int i = tid;
    double lo = INFINITY, hi = -INFINITY;
    if (i < r) {
      const double rad = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < r ? fabs(ee[i]) : 0.0);
      lo = dd[i] - rad;
      hi = dd[i] + rad;
    }
    wave_minmax(lo, hi);
    if (i == 0) {
      bnd[0] = lo;
      bnd[1] = hi;
    }
  }
  __syncthreads();
  {
    const double tn = fmax(fabs(bnd[0]), fabs(bnd[1]));
    sc = tn > 0.0 && tn < INFINITY ? ldexp(1.0, -ilogb(tn)) : 1.0;
    tns = tn * sc;
  }
  for (int i = tid; i < r; i += nt) {
    dd[i] *= sc;
    if (i + 1 < r) {
      ee[i] *= sc;
      e2[i] = ee[i] * ee[i];
    }
  }
  __syncthreads();
  const int n8 = (r + 7) & ~7;
  for (int j = tid; j < n8; j += nt) {
    dsc[j] = j < r ? dd[j] : 4.0;
    esc[j] = (j > 0 && j < r) ? fmax(e2[j - 1], 0x1p-100) : 0.0;
  }
  __syncthreads();
  {
    const double gl = bnd[0] * sc - 0x1p-48 * tns, gu = bnd[1] * sc + 0x1p-48 * tns;
    const int gsz = nb <= 8 ? 32 : 16;
    const int rounds = gsz == 32 ? 11 : 14;
    const double inv = 1.0 / (gsz + 1);
    const int grp = tid / gsz, t = tid % gsz;
    double lo = gl, hi = gu;
    for (int round = 0; round < rounds; ++round) {
      const double x = lo + (t + 1) * (hi - lo) * inv;
      const bool above = grp < nb ? sturm_lds(dsc, esc, n8, x) > grp : true;
      const uint64_t m = __ballot(above);
      const uint64_t gm = (m >> (lane & ~(gsz - 1))) & ((1ull << gsz) - 1ull);
      const int first = __builtin_ctzll(gm | (1ull << gsz));  // first sub-point with count > grp
      const double nlo = first == 0 ? lo : lo + first * (hi - lo) * inv;
      const double nhi = first == gsz ? hi : lo + (first + 1) * (hi - lo) * inv;
      lo = nlo;
      hi = nhi;
    }
    if (t == 0 && grp < nb) theta[grp] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // a Ritz value below the spectrum of H means a numerically dependent
  // direction spoiled the reduced matrix: redo without P and a looser drop
  if (tid == 0) {
    const double lowb = g.hlow ? g.hlow[0] : -INFINITY;
    const double t0 = theta[0] / sc;
    retry_s = attempt == 0 && nb > 0 && (!(t0 == t0) || t0 < lowb - 1e-6 * fmax(1.0, fabs(lowb)));
  }
  __syncthreads();
  if (!retry_s) break;
  ns = min(ns_full, 2 * b);
  drop_tol = fmax(drop_tol * 1e4, 1e-6);
  if (tid == 0) g.flag[1] = 1;
  __syncthreads();
  }
  // -- phase 7
  // 7. eigenvectors of T (scaled) by twisted factorisation, in wave 0:
  //    lane c runs the top-down pivots D+ of T - theta_c I, lane 16 + c the
  //    bottom-up pivots D-; the twist k minimises |D+_k + D-_k - (d_k -
  //    theta)| (the first minimum); from z_k = 1 the vector grows outward
  //    with the ratios -e / D (lane c upwards, lane 16 + c downwards).
  //    Workspace in G (free after step 4): D+, D- and the vectors, [c][i].
  double *DP = &G[0][0], *DM = DP + kMaxBlock * kNS, *Y = DM + kMaxBlock * kNS;
  static_assert(3 * kMaxBlock * kNS <= kNS * kLd, "workspace fits in G");
  const double pivmin = 0x1p-900;
  if (tid < 2 * kMaxBlock) {
    const int c = tid & 15, dir = tid >> 4;
    const bool act = c < nb;
    const double th = theta[act ? c : 0];
    double *D = (dir ? DM : DP) + c * kNS;
    if (act) {
      const int i0 = dir ? r - 1 : 0;
      double q = dd[i0] - th;
      D[i0] = q;
#pragma unroll 4
      for (int m = 1; m < r; ++m) {
        const int i = dir ? r - 1 - m : m;
        const double ev = e2[dir ? i : i - 1];
        const double di = dd[i];
        const double qg = fabs(q) < pivmin ? -pivmin : q;
        q = (di - th) - ev * rcp_f64(qg);
        D[i] = q;
      }
    }
    // -- phase 12
    wave_lds_sync();
    int tw = 0;
    double best = 1e300;
    if (act) {
      const int h = (r + 1) / 2, k0 = dir ? h : 0, k1 = dir ? r : h;
      tw = k0;
#pragma unroll 4
      for (int k = k0; k < k1; ++k) {
        const double gam = fabs(DP[c * kNS + k] + DM[c * kNS + k] - (dd[k] - th));
        if (gam < best) {
          best = gam;
          tw = k;
        }
      }
    }
    const double ob = __shfl_xor(best, 16, kWave);
    const int otw = __shfl_xor(tw, 16, kWave);
    const double blo = dir ? ob : best, bhi = dir ? best : ob;
    const int tlo = dir ? otw : tw, thi = dir ? tw : otw;
    if (act && dir == 0) twi[c] = bhi < blo ? thi : tlo;
  }
  __syncthreads();
  // the ratios -e / D for every vector and index, in place (all threads):
  // DP[c][i] <- -e_i / D+_i (i + 1 < r), DM[c][i] <- -e_{i-1} / D-_i (i > 0).
  // A pivot is kept away from zero (|D| >= 1e-280 (1 + |e|)).
  for (int e = tid; e < nb * kNS; e += nt) {
    const int i = e % kNS;
    if (i < r) {
      if (i + 1 < r) {
        const double q = DP[e], ev = ee[i], qmin = 1e-280 * (1.0 + fabs(ev));
        DP[e] = -(ev * rcp_f64(fabs(q) < qmin ? (q < 0 ? -qmin : qmin) : q));
      }
      if (i > 0) {
        const double q = DM[e], ev = ee[i - 1], qmin = 1e-280 * (1.0 + fabs(ev));
        DM[e] = -(ev * rcp_f64(fabs(q) < qmin ? (q < 0 ? -qmin : qmin) : q));
      }
    }
  }
  __syncthreads();
  // from z_twist = 1 outward: lane c upwards (z_i = F_i z_{i+1}), lane 16 + c
  // downwards (z_i = G_i z_{i-1}); the partial vector is rescaled when an
  // entry passes 1e10, so a nearly split T cannot overflow
  if (tid < 2 * kMaxBlock) {
    const int c = tid & 15, dir = tid >> 4;
    const bool act = c < nb;
    const int tw = act ? twi[c] : 0;
    const double *R = (dir ? DM : DP) + c * kNS;
    double *Yc = Y + c * kNS;
    double sl = 1.0;   // this lane's rescaling so far
    if (act) {
      double z = 1.0;
      const int n = dir ? r - 1 - tw : tw;
#pragma unroll 4
      for (int m = 1; m <= n; ++m) {
        const int i = dir ? tw + m : tw - m;
        z *= R[i];
        Yc[i] = z;
        if (fabs(z) > 1e10) {
          const double s = 1.0 / fabs(z);
          for (int j = dir ? tw + 1 : i; j <= (dir ? i : tw - 1); ++j) Yc[j] *= s;
          z *= s;
          sl *= s;
        }
      }
    }
    // both halves to the smaller of the two scales (z_k = 1 in each)
    const double osl = __shfl_xor(sl, 16, kWave);
    const double f = fmin(sl, osl);
    if (act) {
      if (f != sl) {
        const double s = f / sl;
        if (dir) for (int i = tw + 1; i < r; ++i) Yc[i] *= s;
        else for (int i = 0; i < tw; ++i) Yc[i] *= s;
      }
      if (dir == 0) Yc[tw] = f;
    }
    wave_lds_sync();
    // -- phase 13
    // norms (lane c): a vector that is not finite becomes the twist's unit vector
    if (tid < kMaxBlock && act) {
      double s0 = 0.0, s1 = 0.0;
      int i = 0;
#pragma unroll 4
      for (; i + 1 < r; i += 2) {
        s0 = fma(Yc[i], Yc[i], s0);
        s1 = fma(Yc[i + 1], Yc[i + 1], s1);
      }
      if (i < r) s0 = fma(Yc[i], Yc[i], s0);
      const double s = s0 + s1;
      if (!(s > 0.0) || !(s < INFINITY)) {
        for (int j = 0; j < r; ++j) Yc[j] = j == tw ? 1.0 : 0.0;
        vnrm[c] = 1.0;
      } else {
        vnrm[c] = 1.0 / sqrt(s);
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < nb * kNS; e += nt)
    if (e % kNS < r) Y[e] *= vnrm[e / kNS];
  __syncthreads();
  // -- phase 14
  // re-orthogonalise inside clusters of close eigenvalues (theta ascending:
  // a cluster is a run of neighbours closer than cl), wave 0, in order
  if (tid < kWave) {
    const double cl = 1e-5 * tns;
    const bool near = tid > 0 && tid < nb && theta[tid] - theta[tid - 1] <= cl;
    if (__ballot(near) != 0ull) {
      for (int c = 1; c < nb; ++c) {
        bool any = false;
        for (int j = 0; j < c; ++j) {
          if (fabs(theta[c] - theta[j]) > cl) continue;
          any = true;
          double dot = 0.0;
          for (int i = tid; i < r; i += kWave) dot += Y[c * kNS + i] * Y[j * kNS + i];
          dot = wave_sum(dot);
          for (int i = tid; i < r; i += kWave) Y[c * kNS + i] -= dot * Y[j * kNS + i];
        }
        if (any) {
          double nrm = 0.0;
          for (int i = tid; i < r; i += kWave) nrm += Y[c * kNS + i] * Y[c * kNS + i];
          nrm = wave_sum(nrm);
          nrm = 1.0 / sqrt(nrm);
          for (int i = tid; i < r; i += kWave) Y[c * kNS + i] *= nrm;
        }
        wave_lds_sync();
      }
    }
  }
  __syncthreads();
  // -- phase 8
  // 8. y <- Q y with the reflectors (last one first): wave w takes vectors
  //    4 w .. 4 w + 3, 16 lanes each; lane t holds rows t, t + 16, t + 32 in
  //    registers and the dot products are summed in the row of 16 by DPP
  {
    const int c = 4 * wv + (lane >> 4), t = lane & 15;
    const bool act = c < nb;
    double y[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int i = t + 16 * m;
      y[m] = (act && i < r) ? Y[c * kNS + i] : 0.0;
    }
    for (int k = r - 3; k >= 0; --k) {
      const double bk = beta[k];
      double rv[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int i = t + 16 * m;
        rv[m] = (i > k && i < r) ? Hm[i][k] : 0.0;
      }
      const double dot = row_sum16(fma(rv[2], y[2], fma(rv[1], y[1], rv[0] * y[0])));
      const double f = bk * dot;
#pragma unroll
      for (int m = 0; m < 3; ++m) y[m] -= f * rv[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int i = t + 16 * m;
      if (act && i < r) Y[c * kNS + i] = y[m];
    }
  }
  __syncthreads();
  // -- phase 9
  // 9. coefficients z = Z^T y of the kept columns: thread (a0, c) forms rows
  //    a0, a0 + 16, a0 + 32 of vector c; C_x = scale * z, C_p = C_x with the
  //    X rows zeroed; dropped columns and unused vectors get zeros
  if (tid == 0) g.flag[0] = r;
  {
    const int a0 = tid & 15, c = tid >> 4;
    if (c < nb) {
      double z0 = 0.0, z1 = 0.0, z2 = 0.0;
      for (int i = 0; i < r; ++i) {
        const double yv = Y[c * kNS + i];
        z0 = fma(Z[i][a0], yv, z0);
        z1 = fma(Z[i][a0 + 16], yv, z1);
        z2 = fma(Z[i][a0 + 32], yv, z2);
      }
      const double zz[3] = {z0, z1, z2};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int a = a0 + 16 * m;
        if (a < r) {
          const int k = kidx[a];
          const double v = zz[m] * scale[k];
          g.C[k * 2 * b + c] = v;
          g.C[k * 2 * b + b + c] = k < b ? 0.0 : v;
        }
      }
    }
  }
  for (int e = tid; e < ns_full * b; e += nt) {
    const int k = e / b, c = e % b;
    if (!(c < nb && k < ns && keep[k])) {
      g.C[k * 2 * b + c] = 0.0;
      g.C[k * 2 * b + b + c] = 0.0;
    }
  }
  for (int c = tid; c < b; c += nt) g.lam[c] = c < nb ? theta[c] / sc : 0.0;
}
