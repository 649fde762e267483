/* CPU ORACLE -- test infrastructure only, never linked into the GPU library.
 *
 * Plain C + OpenMP.  Two brute-force routines that are too slow in Python at
 * the larger workload sizes:
 *
 *  oracle_apply_columns  applies the second-quantised Hamiltonian (Sec. 2 of
 *      the paper: one-body energies plus a two-body interaction) to ket bit
 *      strings, one creation/annihilation operator at a time, and looks the
 *      resulting bra up in a hash map of the basis.  This is the definition
 *      H_ij = <Phi_i|H|Phi_j> written out; it shares nothing with the XOR /
 *      popcount Slater-Condon route of the GPU path.
 *
 *  oracle_pattern_rows   lists, for each requested row i, every j >= i whose
 *      bit string differs from row i's in at most four single-particle states
 *      (Sec. 2.1: popcount(BIN_i xor BIN_j) <= 4 for a two-body operator),
 *      comparing against every state.
 *
 * State representation: one concatenated bit string of up to 256 bits per
 * state (species A modes at global positions 0..nA-1, species B at nA..),
 * held as 4 little-endian 64-bit words.  Operator sign convention: an
 * annihilator or creator acting on global mode k contributes (-1)^(number of
 * occupied modes below k) in the state it acts on.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define MAXW 4

typedef struct { uint64_t w[MAXW]; } st_t;

typedef struct {
  int32_t n1, n2;          /* orbitals of the two pair members' species      */
  const int32_t *pp;       /* n1*n2: pair id of (a,b), -1 if not a valid pair */
  const int32_t *pblk;     /* pair id -> block                               */
  const int32_t *pstart;   /* block -> first pair id (nblk+1 entries)        */
  const int32_t *plist;    /* pair id -> (a, b), 2 entries per pair          */
  const int64_t *vbase;    /* block -> offset of its n x n matrix in v       */
  const double *v;         /* blocked symmetric matrices, row-major          */
} pairtab_t;

/* ---------------- bit helpers ---------------- */
static int getbit(const st_t *s, int k) { return (int)((s->w[k >> 6] >> (k & 63)) & 1u); }
static void flipbit(st_t *s, int k) { s->w[k >> 6] ^= (uint64_t)1 << (k & 63); }
static int count_below(const st_t *s, int k) {
  /* number of occupied modes q < k */
  int c = 0;
  for (int w = 0; w < (k >> 6); ++w) c += __builtin_popcountll(s->w[w]);
  if (k & 63) c += __builtin_popcountll(s->w[k >> 6] & (((uint64_t)1 << (k & 63)) - 1));
  return c;
}
/* a_k: returns 0 if mode k is empty, else +-1 and updates s */
static int op_annihilate(st_t *s, int k) {
  if (!getbit(s, k)) return 0;
  int sg = (count_below(s, k) & 1) ? -1 : 1;
  flipbit(s, k);
  return sg;
}
/* a^dagger_k: returns 0 if mode k is occupied, else +-1 and updates s */
static int op_create(st_t *s, int k) {
  if (getbit(s, k)) return 0;
  int sg = (count_below(s, k) & 1) ? -1 : 1;
  flipbit(s, k);
  return sg;
}

/* ---------------- basis hash map: state -> index ---------------- */
typedef struct { int64_t cap; int64_t *idx; const st_t *st; } smap_t;

/* the 64-bit finaliser fmix64 of MurmurHash3 (Appleby), published constants */
static uint64_t mix64(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33; return x;
}
static uint64_t st_hash(const st_t *s) {
  uint64_t h = 0x9e3779b97f4a7c15ULL;
  for (int w = 0; w < MAXW; ++w) h = mix64(h ^ s->w[w]) + (uint64_t)w;
  return h;
}
static int st_eq(const st_t *a, const st_t *b) { return memcmp(a, b, sizeof(st_t)) == 0; }

static int smap_build(smap_t *m, const st_t *st, int64_t D) {
  int64_t cap = 16;
  while (cap < 2 * D + 16) cap <<= 1;
  m->cap = cap; m->st = st;
  m->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
  if (!m->idx) return -1;
  for (int64_t i = 0; i < cap; ++i) m->idx[i] = -1;
  for (int64_t i = 0; i < D; ++i) {
    uint64_t h = st_hash(&st[i]) & (uint64_t)(cap - 1);
    while (m->idx[h] >= 0) {
      if (st_eq(&st[m->idx[h]], &st[i])) return -2;  /* duplicate state */
      h = (h + 1) & (uint64_t)(cap - 1);
    }
    m->idx[h] = i;
  }
  return 0;
}
static int64_t smap_find(const smap_t *m, const st_t *s) {
  uint64_t h = st_hash(s) & (uint64_t)(m->cap - 1);
  while (m->idx[h] >= 0) {
    if (st_eq(&m->st[m->idx[h]], s)) return m->idx[h];
    h = (h + 1) & (uint64_t)(m->cap - 1);
  }
  return -1;
}

/* ---------------- per-column accumulator: row -> Neumaier sum ---------------- */
typedef struct { int64_t cap, n; int64_t *key; double *sum, *comp; } acc_t;

static void acc_init(acc_t *a) {
  a->cap = 1024; a->n = 0;
  a->key = (int64_t *)malloc(sizeof(int64_t) * (size_t)a->cap);
  a->sum = (double *)malloc(sizeof(double) * (size_t)a->cap);
  a->comp = (double *)malloc(sizeof(double) * (size_t)a->cap);
  for (int64_t i = 0; i < a->cap; ++i) a->key[i] = -1;
}
static void acc_free(acc_t *a) { free(a->key); free(a->sum); free(a->comp); }
static void acc_clear(acc_t *a) {
  for (int64_t i = 0; i < a->cap; ++i) a->key[i] = -1;
  a->n = 0;
}
static void acc_add(acc_t *a, int64_t row, double x);
static void acc_grow(acc_t *a) {
  acc_t b; b.cap = a->cap * 2; b.n = 0;
  b.key = (int64_t *)malloc(sizeof(int64_t) * (size_t)b.cap);
  b.sum = (double *)malloc(sizeof(double) * (size_t)b.cap);
  b.comp = (double *)malloc(sizeof(double) * (size_t)b.cap);
  for (int64_t i = 0; i < b.cap; ++i) b.key[i] = -1;
  for (int64_t i = 0; i < a->cap; ++i) {
    if (a->key[i] < 0) continue;
    uint64_t h = mix64((uint64_t)a->key[i]) & (uint64_t)(b.cap - 1);
    while (b.key[h] >= 0) h = (h + 1) & (uint64_t)(b.cap - 1);
    b.key[h] = a->key[i]; b.sum[h] = a->sum[i]; b.comp[h] = a->comp[i]; b.n++;
  }
  acc_free(a); *a = b;
}
static void acc_add(acc_t *a, int64_t row, double x) {
  if (2 * (a->n + 1) > a->cap) acc_grow(a);
  uint64_t h = mix64((uint64_t)row) & (uint64_t)(a->cap - 1);
  while (a->key[h] >= 0 && a->key[h] != row) h = (h + 1) & (uint64_t)(a->cap - 1);
  if (a->key[h] < 0) { a->key[h] = row; a->sum[h] = 0.0; a->comp[h] = 0.0; a->n++; }
  /* Neumaier compensated summation */
  double s = a->sum[h], t = s + x;
  if (fabs(s) >= fabs(x)) a->comp[h] += (s - t) + x; else a->comp[h] += (x - t) + s;
  a->sum[h] = t;
}

/* ---------------- the Hamiltonian applied to one ket ---------------- */
typedef struct {
  int nA, nB;                    /* modes of species A and B (nB = 0: one species) */
  const double *epsA, *epsB;
  const pairtab_t *tA, *tB, *tAB;
  const int32_t *qmode;          /* shell quantum n of each global mode */
  int32_t qmax;                  /* < 0: no truncation */
} ham_t;

static int64_t lost_ok(const ham_t *h, const st_t *s) {
  /* an image outside the basis must break the truncation, else closure fails */
  if (h->qmax < 0) return 1;
  int q = 0;
  for (int k = 0; k < h->nA + h->nB; ++k) if (getbit(s, k)) q += h->qmode[k];
  return q > h->qmax;
}

static void apply_one(const ham_t *h, const smap_t *map, const st_t *ket, int64_t ket_idx,
                      acc_t *acc, int64_t *n_bad) {
  /* one-body part: sum_a eps_a n_a (diagonal) */
  for (int a = 0; a < h->nA; ++a) if (getbit(ket, a)) acc_add(acc, ket_idx, h->epsA[a]);
  for (int b = 0; b < h->nB; ++b) if (getbit(ket, h->nA + b)) acc_add(acc, ket_idx, h->epsB[b]);

  /* same-species two-body part: sum_{a<b, c<d} V_{ab,cd} a+_a a+_b a_d a_c */
  for (int sp = 0; sp < 2; ++sp) {
    const pairtab_t *t = sp == 0 ? h->tA : h->tB;
    int n = sp == 0 ? h->nA : h->nB, off = sp == 0 ? 0 : h->nA;
    if (n == 0 || t == NULL) continue;
    for (int c = 0; c < n; ++c) {
      if (!getbit(ket, off + c)) continue;
      for (int d = c + 1; d < n; ++d) {
        if (!getbit(ket, off + d)) continue;
        int32_t pid = t->pp[c * t->n2 + d];
        int32_t blk = t->pblk[pid];
        int32_t p0 = t->pstart[blk], nb = t->pstart[blk + 1] - p0;
        int32_t col = pid - p0;
        for (int32_t r = 0; r < nb; ++r) {
          int a = t->plist[2 * (p0 + r)], b = t->plist[2 * (p0 + r) + 1];
          double v = t->v[t->vbase[blk] + (int64_t)r * nb + col];
          st_t s = *ket; int sg = 1, x;
          x = op_annihilate(&s, off + c); if (!x) continue; sg *= x;
          x = op_annihilate(&s, off + d); if (!x) continue; sg *= x;
          x = op_create(&s, off + b);     if (!x) continue; sg *= x;
          x = op_create(&s, off + a);     if (!x) continue; sg *= x;
          int64_t i = smap_find(map, &s);
          if (i < 0) { if (!lost_ok(h, &s)) (*n_bad)++; continue; }
          acc_add(acc, i, sg * v);
        }
      }
    }
  }
  /* cross-species part: sum_{a,c in A; b,d in B} V^AB_{ab,cd} a+_a b+_b b_d a_c */
  if (h->nB > 0 && h->tAB != NULL) {
    const pairtab_t *t = h->tAB;
    for (int c = 0; c < h->nA; ++c) {
      if (!getbit(ket, c)) continue;
      for (int d = 0; d < h->nB; ++d) {
        if (!getbit(ket, h->nA + d)) continue;
        int32_t pid = t->pp[c * t->n2 + d];
        int32_t blk = t->pblk[pid];
        int32_t p0 = t->pstart[blk], nb = t->pstart[blk + 1] - p0;
        int32_t col = pid - p0;
        for (int32_t r = 0; r < nb; ++r) {
          int a = t->plist[2 * (p0 + r)], b = t->plist[2 * (p0 + r) + 1];
          double v = t->v[t->vbase[blk] + (int64_t)r * nb + col];
          st_t s = *ket; int sg = 1, x;
          x = op_annihilate(&s, c);           if (!x) continue; sg *= x;
          x = op_annihilate(&s, h->nA + d);   if (!x) continue; sg *= x;
          x = op_create(&s, h->nA + b);       if (!x) continue; sg *= x;
          x = op_create(&s, a);               if (!x) continue; sg *= x;
          int64_t i = smap_find(map, &s);
          if (i < 0) { if (!lost_ok(h, &s)) (*n_bad)++; continue; }
          acc_add(acc, i, sg * v);
        }
      }
    }
  }
}

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Apply H to the kets cols[0..ncols).  Column c's image is written as rows
 * out_row[out_ptr[c] .. out_ptr[c+1]) (ascending) with values out_val.
 * Call with out_row == NULL to get the per-column counts in out_ptr[c+1].
 * Returns 0, or <0 on error.  n_bad receives the number of operator images
 * that fell outside the basis without breaking the truncation (must be 0). */
int oracle_apply_columns(int nw, int64_t D, const uint64_t *words,
                         int nA, int nB, const double *epsA, const double *epsB,
                         const pairtab_t *tA, const pairtab_t *tB, const pairtab_t *tAB,
                         const int32_t *qmode, int32_t qmax,
                         int64_t ncols, const int64_t *cols,
                         int64_t *out_ptr, int64_t *out_row, double *out_val,
                         int64_t *n_bad) {
  if (nw < 1 || nw > MAXW) return -1;
  st_t *st = (st_t *)calloc((size_t)D + 1, sizeof(st_t));
  if (!st) return -2;
  for (int64_t i = 0; i < D; ++i)
    for (int w = 0; w < nw; ++w) st[i].w[w] = words[i * nw + w];
  smap_t map;
  if (smap_build(&map, st, D) != 0) { free(st); return -3; }
  ham_t h = {nA, nB, epsA, epsB, tA, tB, tAB, qmode, qmax};
  int64_t bad_total = 0;
  int err = 0;
#pragma omp parallel reduction(+ : bad_total)
  {
    acc_t acc; acc_init(&acc);
    int64_t *rows = NULL; int64_t rows_cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < ncols; ++c) {
      int64_t j = cols[c];
      if (j < 0 || j >= D) { err = 1; continue; }
      acc_clear(&acc);
      apply_one(&h, &map, &st[j], j, &acc, &bad_total);
      if (out_row == NULL) { out_ptr[c + 1] = acc.n; continue; }
      if (rows_cap < acc.n) { free(rows); rows_cap = acc.n * 2; rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)rows_cap); }
      int64_t m = 0;
      for (int64_t q = 0; q < acc.cap; ++q) if (acc.key[q] >= 0) rows[m++] = acc.key[q];
      qsort(rows, (size_t)m, sizeof(int64_t), cmp_i64);
      int64_t o = out_ptr[c];
      if (out_ptr[c + 1] - o != m) { err = 2; continue; }
      for (int64_t q = 0; q < m; ++q) {
        uint64_t hh = mix64((uint64_t)rows[q]) & (uint64_t)(acc.cap - 1);
        while (acc.key[hh] != rows[q]) hh = (hh + 1) & (uint64_t)(acc.cap - 1);
        out_row[o + q] = rows[q];
        out_val[o + q] = acc.sum[hh] + acc.comp[hh];
      }
    }
    free(rows); acc_free(&acc);
  }
  free(map.idx); free(st);
  *n_bad = bad_total;
  return err ? -4 - err : 0;
}

/* Brute-force pattern: for each requested row i, every j >= i with
 * popcount(state_i xor state_j) <= 4, ascending.  Two-pass like above. */
int oracle_pattern_rows(int nw, int64_t D, const uint64_t *words, int64_t nrows,
                        const int64_t *rows, int64_t *out_ptr, int32_t *out_col) {
  if (nw < 1 || nw > MAXW) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    const uint64_t *wi = words + i * nw;
    int64_t m = 0, o = out_col ? out_ptr[r] : 0;
    for (int64_t j = i; j < D; ++j) {
      const uint64_t *wj = words + j * nw;
      int diff = 0;
      for (int w = 0; w < nw; ++w) diff += __builtin_popcountll(wi[w] ^ wj[w]);
      if (diff <= 4) { if (out_col) out_col[o + m] = (int32_t)j; m++; }
    }
    if (!out_col) out_ptr[r + 1] = m;
  }
  return 0;
}
