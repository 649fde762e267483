"""CPU ORACLE (test infrastructure only) -- plain statements of each step.

Every function names the passage of the paper it follows.  Nothing here is
tuned; where a loop is slow it is meant to be read, not timed.  The C helpers
in ci_oracle.c (built with gcc, loaded through ctypes) do the same brute-force
work for bases too large for Python loops.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from collections import defaultdict

import numpy as np

__all__ = [
    "orbital_list", "shell_capacity", "q_min", "q_max", "Basis",
    "Interaction", "annihilate", "create", "apply_H", "dense_H",
    "pattern_rows", "half_csr", "half_csr_rows", "exclusive_scan",
    "count_difference", "popcount", "dim_generating_function",
    "nnz_class_count", "trace_generating_function", "spmm_half",
    "eigs_dense", "eigs_sparse", "full_from_half", "residual_audit",
    "load_clib", "build_clib", "apply_columns", "observables", "count_connected",
    "level_occupations", "mb_orbital_groups", "clamped_shift", "block_precond_apply",
]


# ---------------------------------------------------------------------------
# Single-particle space.  Sec. 2: single-particle states carry (n, l, j, m);
# here harmonic-oscillator shells n = 0..nmax, each with levels
# 2j = 1, 3, ..., 2n+1 and 2j+1 projections 2m = -2j..2j (step 2).
# ---------------------------------------------------------------------------
def orbital_list(nmax):
    """[(n, 2j, 2m), ...] in ascending (n, 2j, 2m) order; index = orbital."""
    out = []
    for n in range(nmax + 1):
        for twoj in range(1, 2 * n + 2, 2):
            for twom in range(-twoj, twoj + 1, 2):
                out.append((n, twoj, twom))
    return out


def shell_capacity(n):
    """Orbitals in shell n: sum over 2j = 1..2n+1 of (2j + 1) = (n+1)(n+2)."""
    return sum(twoj + 1 for twoj in range(1, 2 * n + 2, 2))


def q_min(N, nmax):
    """Smallest summed shell quanta of N particles: fill shells from n = 0."""
    q, left = 0, N
    for n in range(nmax + 1):
        take = min(left, shell_capacity(n))
        q += take * n
        left -= take
    if left:
        raise ValueError("more particles than orbitals")
    return q


def q_max(spec):
    """Truncation: summed quanta of all particles <= minimum + cut (None: no cut)."""
    if spec.cut < 0:
        return None
    return sum(q_min(spec.n_particles[s], spec.nmax[s]) for s in range(spec.n_species)) + spec.cut


def popcount(x):
    return bin(x).count("1")


# ---------------------------------------------------------------------------
# Many-body basis (Sec. 2: antisymmetrised products of single-particle states,
# represented by the occupation bit string BIN(Phi), Sec. 2.1).  Brute force:
# all N-subsets of each species, paired under the total-2M and truncation
# constraints, then sorted by the canonical key (A as integer, Q_B, B as
# integer).
# ---------------------------------------------------------------------------
class Basis:
    def __init__(self, spec):
        self.spec = spec
        ns = spec.n_species
        self.orbs = [orbital_list(spec.nmax[0]),
                     orbital_list(spec.nmax[1]) if ns == 2 else []]
        self.n_orb = [len(self.orbs[0]), len(self.orbs[1])]
        NA = spec.n_particles[0]
        NB = spec.n_particles[1] if ns == 2 else 0
        self.N = [NA, NB]
        if NA > self.n_orb[0] or NB > self.n_orb[1]:
            raise ValueError("more particles than orbitals")
        qmx = q_max(spec)
        self.qmax = qmx
        subs = []
        for s in range(2):
            orbs, N = self.orbs[s], self.N[s]
            lst = []
            for occ in itertools.combinations(range(len(orbs)), N):
                q = sum(orbs[k][0] for k in occ)
                if qmx is not None and q > qmx:
                    continue
                m = sum(orbs[k][2] for k in occ)
                bits = 0
                for k in occ:
                    bits |= 1 << k
                lst.append((bits, m, q))
            subs.append(lst)
        by_m = defaultdict(list)
        for (b, m, q) in subs[1]:
            by_m[m].append((b, q))
        states = []
        for (a, ma, qa) in subs[0]:
            for (b, qb) in by_m.get(spec.two_M - ma, []):
                if qmx is not None and qa + qb > qmx:
                    continue
                states.append((a, qb, b))
        states.sort()                    # key (A integer, Q_B, B integer)
        self.A = [t[0] for t in states]
        self.B = [t[2] for t in states]
        self.glob = [a | (b << self.n_orb[0]) for a, b in zip(self.A, self.B)]
        self.index = {g: i for i, g in enumerate(self.glob)}
        self.D = len(states)

    def __len__(self):
        return self.D

    # word layouts used only to compare with what the GPU library exports
    def species_words(self):
        """State-major uint64 words: species A words then species B words,
        each species padded to ceil(n_orb/64) little-endian words."""
        wa = max(1, -(-self.n_orb[0] // 64))
        wb = -(-self.n_orb[1] // 64) if self.spec.n_species == 2 else 0
        out = np.zeros((self.D, wa + wb), dtype=np.uint64)
        mask = (1 << 64) - 1
        for i, (a, b) in enumerate(zip(self.A, self.B)):
            for w in range(wa):
                out[i, w] = (a >> (64 * w)) & mask
            for w in range(wb):
                out[i, wa + w] = (b >> (64 * w)) & mask
        return out

    def global_words(self, nw=4):
        """State-major uint64 words of the concatenated bit string."""
        out = np.zeros((self.D, nw), dtype=np.uint64)
        mask = (1 << 64) - 1
        for i, g in enumerate(self.glob):
            for w in range(nw):
                out[i, w] = (g >> (64 * w)) & mask
        return out

    def qmode(self):
        return [o[0] for o in self.orbs[0]] + [o[0] for o in self.orbs[1]]


# ---------------------------------------------------------------------------
# Interaction: the oracle's own reading of the documented table layout
# (pairs grouped by 2M_pair ascending, lexicographic inside a block, each
# block a full symmetric row-major matrix, blocks concatenated).
# ---------------------------------------------------------------------------
class _PairTable:
    def __init__(self, pairs_with_m, v):
        blocks = defaultdict(list)
        for (a, b, m) in pairs_with_m:
            blocks[m].append((a, b))
        self.blocks = []          # (2M, [pairs], base)
        self.pos = {}             # pair -> (block number, index)
        base = 0
        for k, m in enumerate(sorted(blocks)):
            prs = sorted(blocks[m])
            self.blocks.append((m, prs, base))
            for i, p in enumerate(prs):
                self.pos[p] = (k, i)
            base += len(prs) ** 2
        if v is not None and base != len(v):
            raise ValueError("table size %d does not match layout %d" % (len(v), base))
        self.v = v

    def value(self, p, q):
        """V_{p,q}: zero when the pairs sit in different 2M blocks."""
        (bp, ip), (bq, iq) = self.pos[p], self.pos[q]
        if bp != bq:
            return 0.0
        _, prs, base = self.blocks[bp]
        return float(self.v[base + ip * len(prs) + iq])

    def partners(self, q):
        """All (p, V_{p,q}) with p in the same 2M block as q."""
        bq, iq = self.pos[q]
        _, prs, base = self.blocks[bq]
        n = len(prs)
        for ip, p in enumerate(prs):
            yield p, float(self.v[base + ip * n + iq])


class Interaction:
    """H = sum_s sum_a eps^s_a n_a
         + sum_s sum_{a<b, c<d} V^s_{ab,cd} a+_a a+_b a_d a_c
         + sum_{a,c in A; b,d in B} V^AB_{ab,cd} a+_a b+_b b_d a_c."""

    def __init__(self, basis, tables):
        self.basis = basis
        self.eps = [np.asarray(e, dtype=np.float64) for e in tables.eps]
        self.same = []
        for s in range(basis.spec.n_species):
            orbs = basis.orbs[s]
            prs = [(a, b, orbs[a][2] + orbs[b][2])
                   for a in range(len(orbs)) for b in range(a + 1, len(orbs))]
            self.same.append(_PairTable(prs, tables.v_same[s]))
        self.cross = None
        if basis.spec.n_species == 2:
            oa, ob = basis.orbs
            prs = [(a, b, oa[a][2] + ob[b][2]) for a in range(len(oa)) for b in range(len(ob))]
            self.cross = _PairTable(prs, tables.v_ab)

    # flat arrays for the C helper
    def _c_table(self, t, n1, n2):
        pp = -np.ones(n1 * n2, dtype=np.int32)
        pblk, pstart, plist, vbase = [], [0], [], []
        pid = 0
        for k, (_, prs, base) in enumerate(t.blocks):
            vbase.append(base)
            for (a, b) in prs:
                pp[a * n2 + b] = pid
                pblk.append(k)
                plist += [a, b]
                pid += 1
            pstart.append(pid)
        return dict(n1=n1, n2=n2, pp=pp, pblk=np.asarray(pblk, np.int32),
                    pstart=np.asarray(pstart, np.int32),
                    plist=np.asarray(plist, np.int32),
                    vbase=np.asarray(vbase, np.int64),
                    v=np.ascontiguousarray(t.v, dtype=np.float64))


# ---------------------------------------------------------------------------
# Second quantisation on bit strings.  Global mode k: species A orbital k, or
# species B orbital k - n_A.  Convention: a_k and a+_k acting on a state pick
# up (-1) ** (number of occupied modes below k), counted one by one.
# ---------------------------------------------------------------------------
def _occupied_below(state, k):
    c = 0
    for q in range(k):
        if (state >> q) & 1:
            c += 1
    return c


def annihilate(state, k):
    if not (state >> k) & 1:
        return 0, None
    return (-1) ** _occupied_below(state, k), state ^ (1 << k)


def create(state, k):
    if (state >> k) & 1:
        return 0, None
    return (-1) ** _occupied_below(state, k), state | (1 << k)


def _apply_string(state, ops):
    """ops applied in list order (the rightmost operator of the product first)."""
    sign = 1
    for kind, k in ops:
        s, state = (annihilate if kind == "a" else create)(state, k)
        if state is None:
            return 0, None
        sign *= s
    return sign, state


def apply_H(ket, inter):
    """H|ket> as {bra: value}, every term of the operator applied one by one
    (Sec. 2; Fig. 1 step 14 'compute the nonzero matrix entry').  Values are
    exactly-rounded sums (math.fsum) of the contributing terms."""
    b = inter.basis
    nA = b.n_orb[0]
    terms = defaultdict(list)
    for s in range(b.spec.n_species):
        off = 0 if s == 0 else nA
        for k in range(b.n_orb[s]):
            if (ket >> (off + k)) & 1:
                terms[ket].append(float(inter.eps[s][k]))
    for s in range(b.spec.n_species):
        off = 0 if s == 0 else nA
        occ = [k for k in range(b.n_orb[s]) if (ket >> (off + k)) & 1]
        for (c, d) in itertools.combinations(occ, 2):
            for (a, bb), v in inter.same[s].partners((c, d)):
                sg, bra = _apply_string(ket, [("a", off + c), ("a", off + d),
                                              ("c", off + bb), ("c", off + a)])
                if bra is not None:
                    terms[bra].append(sg * v)
    if b.spec.n_species == 2:
        occa = [k for k in range(nA) if (ket >> k) & 1]
        occb = [k for k in range(b.n_orb[1]) if (ket >> (nA + k)) & 1]
        for c in occa:
            for d in occb:
                for (a, bb), v in inter.cross.partners((c, d)):
                    sg, bra = _apply_string(ket, [("a", c), ("a", nA + d),
                                                  ("c", nA + bb), ("c", a)])
                    if bra is not None:
                        terms[bra].append(sg * v)
    return {bra: math.fsum(t) for bra, t in terms.items()}


def _state_q(basis, g):
    q = 0
    for k, qn in enumerate(basis.qmode()):
        if (g >> k) & 1:
            q += qn
    return q


def dense_H(basis, inter, check_closure=True):
    """Dense H_ij = <Phi_i|H|Phi_j>, column j from H|Phi_j> (small D only)."""
    D = basis.D
    H = np.zeros((D, D))
    for j, ket in enumerate(basis.glob):
        for bra, v in apply_H(ket, inter).items():
            i = basis.index.get(bra)
            if i is None:
                if check_closure and (basis.qmax is None or _state_q(basis, bra) <= basis.qmax):
                    raise AssertionError("operator image outside the basis")
                continue
            H[i, j] = v
    return H


# ---------------------------------------------------------------------------
# Sparsity (Sec. 2.1): H_ij can be nonzero only if popcount(BIN_i xor BIN_j)
# <= 4 for a two-body operator.  Structural pattern = all such pairs.
# ---------------------------------------------------------------------------
def pattern_rows(basis, rows=None):
    """{i: ascending array of j >= i with popcount(BIN_i xor BIN_j) <= 4}."""
    lib = load_clib()
    words = np.ascontiguousarray(basis.global_words(4))
    rows = np.arange(basis.D, dtype=np.int64) if rows is None else np.asarray(rows, np.int64)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    _chk(lib.oracle_pattern_rows(4, basis.D, _p(words), len(rows), _p(rows), _p(ptr), None))
    ptr = np.cumsum(ptr)
    cols = np.zeros(int(ptr[-1]), dtype=np.int32)
    _chk(lib.oracle_pattern_rows(4, basis.D, _p(words), len(rows), _p(rows), _p(ptr), _p(cols)))
    return ptr, cols


def exclusive_scan(x):
    """Sec. 2.2: y_1 = 0, y_{i+1} = y_i + x_i.  Returns n+1 values (the last
    is the total, which a CSR row pointer needs)."""
    y = [0] * (len(x) + 1)
    for i in range(len(x)):
        y[i + 1] = y[i] + int(x[i])
    return np.asarray(y, dtype=np.int64)


def count_difference(s1, s2):
    """Sec. 2.1 (count_difference of two index tuples, Listing 1 as a
    description): with c entries common to both tuples, each side holds
    len - c entries the other lacks; the result is twice the larger side."""
    c = len(set(s1) & set(s2))
    return 2 * max(len(s1) - c, len(s2) - c)


def count_connected(mbs, n_sp, rows=None):
    """The state-counting test (Sec. 2.1, Listing 2 as a description): for
    each state i of the list, the number of states j (j = i included) that a
    two-body operator connects, i.e. that differ from it in at most two
    particles: popcount(BIN_i xor BIN_j) <= 4 with BIN the full bit string
    of the state over all n_sp single-particle states.  mbs: (n, N) index
    tuples; rows: the states to count for (default all), each against the
    whole list.  Returns int64 counts (numpy, blocks of rows)."""
    mbs = np.asarray(mbs, dtype=np.int64)
    n = mbs.shape[0]
    nw = max(1, -(-n_sp // 64))
    words = np.zeros((n, nw), dtype=np.uint64)
    for k in range(mbs.shape[1]):
        w, b = mbs[:, k] // 64, (mbs[:, k] % 64).astype(np.uint64)
        for q in range(nw):
            sel = w == q
            words[sel, q] |= np.left_shift(np.uint64(1), b[sel])
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    counts = np.zeros(len(rows), dtype=np.int64)
    for i0 in range(0, len(rows), 256):
        r = rows[i0:i0 + 256]
        d = np.zeros((len(r), n), dtype=np.int64)
        for q in range(nw):
            d += np.bitwise_count(words[r, q][:, None] ^ words[None, :, q])
        counts[i0:i0 + 256] = (d <= 4).sum(axis=1)
    return counts


# ---------------------------------------------------------------------------
# The C helpers
# ---------------------------------------------------------------------------
_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_ci_oracle.so")


class _CPairTab(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("pp", ctypes.c_void_p), ("pblk", ctypes.c_void_p),
                ("pstart", ctypes.c_void_p), ("plist", ctypes.c_void_p),
                ("vbase", ctypes.c_void_p), ("v", ctypes.c_void_p)]


def build_clib(force=False):
    """Compile ci_oracle.c with gcc (the oracle's own build step)."""
    src = os.path.join(_HERE, "ci_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def load_clib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO):
            build_clib()
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_apply_columns.argtypes = [ctypes.c_int, i64, vp, ctypes.c_int, ctypes.c_int,
                                             vp, vp, vp, vp, vp, vp, i32, i64, vp, vp, vp, vp, vp]
        lib.oracle_apply_columns.restype = ctypes.c_int
        lib.oracle_pattern_rows.argtypes = [ctypes.c_int, i64, vp, i64, vp, vp, vp]
        lib.oracle_pattern_rows.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _chk(rc):
    if rc != 0:
        raise RuntimeError("oracle C helper failed: %d" % rc)


def apply_columns(basis, inter, cols):
    """H|Phi_j> for each j in cols via the C helper: (ptr, rows, vals);
    column c's image occupies rows[ptr[c]:ptr[c+1]] (ascending)."""
    lib = load_clib()
    b = basis
    nA, nB = b.n_orb
    words = np.ascontiguousarray(b.global_words(4))
    keep = []

    def tab(t, n1, n2):
        d = inter._c_table(t, n1, n2)
        keep.append(d)
        return _CPairTab(n1, n2, _p(d["pp"]).value, _p(d["pblk"]).value,
                         _p(d["pstart"]).value, _p(d["plist"]).value,
                         _p(d["vbase"]).value, _p(d["v"]).value)

    tA = tab(inter.same[0], nA, nA)
    tB = tab(inter.same[1], nB, nB) if b.spec.n_species == 2 else None
    tAB = tab(inter.cross, nA, nB) if b.spec.n_species == 2 else None
    epsA = np.ascontiguousarray(inter.eps[0])
    epsB = np.ascontiguousarray(inter.eps[1]) if b.spec.n_species == 2 else np.zeros(1)
    qmode = np.asarray(b.qmode() + [0], dtype=np.int32)
    qmax = -1 if b.qmax is None else int(b.qmax)
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    ptr = np.zeros(len(cols) + 1, dtype=np.int64)
    bad = np.zeros(1, dtype=np.int64)
    ref = lambda t: None if t is None else ctypes.byref(t)
    args = [4, b.D, _p(words), nA, nB if b.spec.n_species == 2 else 0, _p(epsA), _p(epsB),
            ref(tA), ref(tB), ref(tAB), _p(qmode), qmax, len(cols), _p(cols)]
    _chk(lib.oracle_apply_columns(*args, _p(ptr), None, None, _p(bad)))
    ptr = np.cumsum(ptr)
    rows = np.zeros(int(ptr[-1]), dtype=np.int64)
    vals = np.zeros(int(ptr[-1]), dtype=np.float64)
    _chk(lib.oracle_apply_columns(*args, _p(ptr), _p(rows), _p(vals), _p(bad)))
    if bad[0]:
        raise AssertionError("%d operator images left the basis without breaking the cut" % bad[0])
    return ptr, rows, vals


# ---------------------------------------------------------------------------
# Half-stored CSR (upper triangle incl. diagonal, ascending columns, int64 row
# pointers via the counts-to-offsets scan of Sec. 2.2; Fig. 1 steps 6-14).
# ---------------------------------------------------------------------------
def half_csr(basis, inter):
    """Full half-CSR: structure from the brute-force pattern, values
    H_ij = <Phi_i|H|Phi_j> read from the image of ket j.  A pattern entry that
    no operator term reaches is an exact 0.0; an operator entry outside the
    pattern is an error."""
    pptr, pcol = pattern_rows(basis)
    counts = np.diff(pptr)
    row_ptr = exclusive_scan(counts)
    cptr, crow, cval = apply_columns(basis, inter, np.arange(basis.D))
    # entry (i, j) from column j; keep the upper triangle i <= j
    colidx = np.repeat(np.arange(basis.D, dtype=np.int64), np.diff(cptr))
    up = crow <= colidx
    i_u, j_u, v_u = crow[up], colidx[up], cval[up]
    order = np.lexsort((j_u, i_u))
    i_u, j_u, v_u = i_u[order], j_u[order], v_u[order]
    # locate each operator entry in the pattern (both key lists ascending)
    D = basis.D
    pkey = np.repeat(np.arange(D, dtype=np.int64), counts) * D + pcol.astype(np.int64)
    okey = i_u * D + j_u
    pos = np.searchsorted(pkey, okey)
    inside = (pos < len(pkey)) & (pkey[np.minimum(pos, len(pkey) - 1)] == okey)
    if not inside.all():
        raise AssertionError("operator entry outside the popcount<=4 pattern")
    val = np.zeros(len(pcol), dtype=np.float64)
    val[pos] = v_u
    return row_ptr, pcol, val


def half_csr_rows(basis, inter, rows):
    """Selected rows of the half-CSR: structure by brute force over all j >= i,
    values from the image of ket i (H is symmetric, so H_ij = <Phi_j|H|Phi_i>).
    Returns {i: (cols, vals)}."""
    rows = np.asarray(rows, dtype=np.int64)
    pptr, pcol = pattern_rows(basis, rows)
    cptr, crow, cval = apply_columns(basis, inter, rows)
    out = {}
    for k, i in enumerate(rows):
        cols = pcol[pptr[k]:pptr[k + 1]].astype(np.int64)
        img = dict(zip(crow[cptr[k]:cptr[k + 1]].tolist(), cval[cptr[k]:cptr[k + 1]].tolist()))
        in_pattern = set(cols.tolist())
        for j in img:
            if j >= i and j not in in_pattern:
                raise AssertionError("operator entry outside the pattern")
        out[int(i)] = (cols, np.asarray([img.get(int(j), 0.0) for j in cols]))
    return out


# ---------------------------------------------------------------------------
# Counting pins that avoid enumerating state pairs.
# ---------------------------------------------------------------------------
def _species_poly(orbs, N):
    """Coefficients c[N', 2M + off, Q] of prod_orbitals (1 + x t^{2m} q^n),
    truncated at N particles: a plain dynamic programme over orbitals."""
    mmax = sum(sorted((abs(o[2]) for o in orbs), reverse=True)[:N]) if orbs else 0
    qtop = sum(sorted((o[0] for o in orbs), reverse=True)[:N]) if orbs else 0
    off = mmax
    c = np.zeros((N + 1, 2 * mmax + 1, qtop + 1), dtype=object)
    c[0, off, 0] = 1
    for (n, _, m) in orbs:
        new = c.copy()
        for k in range(N):
            for mi in range(2 * mmax + 1):
                mj = mi + m
                if mj < 0 or mj > 2 * mmax:
                    continue
                for q in range(qtop + 1 - n):
                    if c[k, mi, q]:
                        new[k + 1, mj, q + n] += c[k, mi, q]
        c = new
    return c[N], off


def dim_generating_function(spec):
    """D = sum over 2M_A + 2M_B = 2M and Q_A + Q_B <= Qmax of the product of
    the per-species generating-function coefficients."""
    qmx = q_max(spec)
    cA, oA = _species_poly(orbital_list(spec.nmax[0]), spec.n_particles[0])
    if spec.n_species == 2:
        cB, oB = _species_poly(orbital_list(spec.nmax[1]), spec.n_particles[1])
    else:
        cB, oB = np.array([[1]], dtype=object), 0
    D = 0
    for ma in range(cA.shape[0]):
        for qa in range(cA.shape[1]):
            if not cA[ma, qa]:
                continue
            mb = spec.two_M - (ma - oA) + oB
            if mb < 0 or mb >= cB.shape[0]:
                continue
            for qb in range(cB.shape[1]):
                if qmx is not None and qa + qb > qmx:
                    continue
                D += cA[ma, qa] * cB[mb, qb]
    return int(D)


def nnz_class_count(spec):
    """Count pattern entries without listing state pairs (Sec. 2.1 rule):
    group each species' substates by (2M, Q); for each ordered pair of A
    classes and of B classes, count substate pairs at distance k (popcount of
    the XOR = 2k) and combine sum_{kA + kB <= 2} nA * nB over the class pairs
    that both lie in the basis.  Returns (nnz_full, nnz_half)."""
    qmx = q_max(spec)

    def classes(orbs, N):
        cl = defaultdict(list)
        for occ in itertools.combinations(range(len(orbs)), N):
            q = sum(orbs[k][0] for k in occ)
            if qmx is not None and q > qmx:
                continue
            m = sum(orbs[k][2] for k in occ)
            bits = 0
            for k in occ:
                bits |= 1 << k
            cl[(m, q)].append(bits)
        return cl

    def pair_counts(cl):
        keys = sorted(cl)
        arrs = {}
        for key in keys:
            ints = cl[key]
            nw = 2
            a = np.zeros((len(ints), nw), dtype=np.uint64)
            for i, x in enumerate(ints):
                a[i, 0] = x & ((1 << 64) - 1)
                a[i, 1] = x >> 64
            arrs[key] = a
        out = {}
        for k1 in keys:
            for k2 in keys:
                x = arrs[k1][:, None, :] ^ arrs[k2][None, :, :]
                d = np.bitwise_count(x).sum(axis=2)
                out[(k1, k2)] = [int((d == 0).sum()), int((d == 2).sum()), int((d == 4).sum())]
        return out

    clA = classes(orbital_list(spec.nmax[0]), spec.n_particles[0])
    if spec.n_species == 2:
        clB = classes(orbital_list(spec.nmax[1]), spec.n_particles[1])
    else:
        clB = {(0, 0): [0]}
    pA, pB = pair_counts(clA), pair_counts(clB)
    pairs = [(ka, kb) for ka in clA for kb in clB
             if ka[0] + kb[0] == spec.two_M and (qmx is None or ka[1] + kb[1] <= qmx)]
    full = 0
    for (a1, b1) in pairs:
        for (a2, b2) in pairs:
            na, nb = pA[(a1, a2)], pB[(b1, b2)]
            for ka in range(3):
                for kb in range(3 - ka):
                    full += na[ka] * nb[kb]
    D = sum(len(clA[a]) * len(clB[b]) for (a, b) in pairs)
    return full, (full + D) // 2


def trace_generating_function(spec, tables):
    """Tr H without enumerating states: sum_a eps_a * #(states with a occupied)
    + sum_{a<b} V_{ab,ab} * #(states with a, b occupied) (same species)
    + sum_{a in A, b in B} V^AB_{ab,ab} * #(states with a and b occupied).
    The counts come from the per-species generating functions with the fixed
    orbitals removed."""
    qmx = q_max(spec)
    ns = spec.n_species
    orbs = [orbital_list(spec.nmax[0]), orbital_list(spec.nmax[1]) if ns == 2 else []]
    N = [spec.n_particles[0], spec.n_particles[1] if ns == 2 else 0]

    def table(s, fixed):
        """{(2M, Q): count} of species-s substates containing all `fixed`."""
        rest = [o for k, o in enumerate(orbs[s]) if k not in fixed]
        n_left = N[s] - len(fixed)
        if n_left < 0:
            return {}
        c, off = _species_poly(rest, n_left)
        m0 = sum(orbs[s][k][2] for k in fixed)
        q0 = sum(orbs[s][k][0] for k in fixed)
        out = {}
        for mi in range(c.shape[0]):
            for q in range(c.shape[1]):
                if c[mi, q]:
                    out[(mi - off + m0, q + q0)] = int(c[mi, q])
        return out

    def combine(ta, tb):
        tot = 0
        for (ma, qa), ca in ta.items():
            for (mb, qb), cb in tb.items():
                if ma + mb == spec.two_M and (qmx is None or qa + qb <= qmx):
                    tot += ca * cb
        return tot

    full = [table(0, ()), table(1, ()) if ns == 2 else {(0, 0): 1}]
    inter_same = [None, None]
    tr = 0.0
    terms = []
    for s in range(ns):
        other = full[1 - s]
        for a in range(len(orbs[s])):
            t = table(s, (a,))
            cnt = combine(t, other) if s == 0 else combine(other, t)
            terms.append(float(tables.eps[s][a]) * cnt)
    # diagonal same-species elements V_{ab,ab}
    for s in range(ns):
        lay = _PairTable([(a, b, orbs[s][a][2] + orbs[s][b][2])
                          for a in range(len(orbs[s])) for b in range(a + 1, len(orbs[s]))],
                         tables.v_same[s])
        inter_same[s] = lay
        other = full[1 - s]
        for a in range(len(orbs[s])):
            for b in range(a + 1, len(orbs[s])):
                t = table(s, (a, b))
                cnt = combine(t, other) if s == 0 else combine(other, t)
                if cnt:
                    terms.append(lay.value((a, b), (a, b)) * cnt)
    if ns == 2:
        lay = _PairTable([(a, b, orbs[0][a][2] + orbs[1][b][2])
                          for a in range(len(orbs[0])) for b in range(len(orbs[1]))], tables.v_ab)
        for a in range(len(orbs[0])):
            ta = table(0, (a,))
            for b in range(len(orbs[1])):
                cnt = combine(ta, table(1, (b,)))
                if cnt:
                    terms.append(lay.value((a, b), (a, b)) * cnt)
    tr = math.fsum(terms)
    return tr


# ---------------------------------------------------------------------------
# SpMM and eigenvalues (Fig. 1 step 15; Fig. 2 'FMA with vector elements').
# ---------------------------------------------------------------------------
def full_from_half(row_ptr, col, val, D):
    """scipy CSR of the full symmetric matrix U + U^T - diag(U)."""
    import scipy.sparse as sp
    U = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col, dtype=np.int64),
                       np.asarray(row_ptr, dtype=np.int64)), shape=(D, D))
    return (U + U.T - sp.diags(U.diagonal())).tocsr()


def spmm_half(row_ptr, col, val, X):
    """Y = H X in float64 with H given by its upper half (library sparse matmul
    on the expanded matrix).  Also returns |H| |X| for error bounds."""
    D = len(row_ptr) - 1
    H = full_from_half(row_ptr, col, val, D)
    X = np.asarray(X, dtype=np.float64)
    return H @ X, abs(H) @ np.abs(X)


def observables(basis, tables_list, X):
    """Expectation values of several operators in several vectors, the
    step after the eigensolve (Fig. 1 steps 16-20): a[k, v] = sum_ij
    X[i, v] (O_k)_ij X[j, v], where O_k is the many-body operator defined by
    tables_list[k] (one-body energies and two-body tables in the layout of
    the Hamiltonian's).  Each O_k is formed as its half-stored matrix from
    the operator image (half_csr), expanded, and applied in float64."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((len(tables_list), X.shape[1]))
    for k, t in enumerate(tables_list):
        rp, col, val = half_csr(basis, Interaction(basis, t))
        Y = full_from_half(rp, col, val, basis.D) @ X
        out[k] = np.sum(X * Y, axis=0)
    return out


def eigs_dense(H, k):
    """Lowest k eigenvalues of a dense symmetric matrix (LAPACK via numpy)."""
    w = np.linalg.eigvalsh(np.asarray(H, dtype=np.float64))
    return w[:k]


def eigs_sparse(row_ptr, col, val, k, tol=1e-13):
    """Lowest k eigenpairs of the half-stored matrix (ARPACK via scipy)."""
    import scipy.sparse.linalg as sla
    D = len(row_ptr) - 1
    H = full_from_half(row_ptr, col, val, D)
    w, v = sla.eigsh(H, k=k, which="SA", tol=tol)
    order = np.argsort(w)
    return w[order], v[:, order]


def residual_audit(row_ptr, col, val, lam, X):
    """||H x - lam x|| / (max(|lam|, 1) ||x||) per column, float64."""
    Y, _ = spmm_half(row_ptr, col, val, X)
    X = np.asarray(X, dtype=np.float64)
    r = np.linalg.norm(Y - X * np.asarray(lam)[None, :], axis=0)
    return r / (np.maximum(np.abs(lam), 1.0) * np.linalg.norm(X, axis=0))


# ---------------------------------------------------------------------------
# Block-diagonal preconditioner over many-body basis orbitals (Sec. 2: states
# with the same (n, l, j) values of their particles and any m values form a
# group; the grouping gives LOBPCG a block-diagonal preconditioner).
# ---------------------------------------------------------------------------
def level_occupations(orbs, bits):
    """Particles in each (n, 2j) level of one species' bit string, levels in
    the orbital order."""
    occ = {}
    for k, (n, twoj, _) in enumerate(orbs):
        occ.setdefault((n, twoj), 0)
        if (bits >> k) & 1:
            occ[(n, twoj)] += 1
    return tuple(occ[key] for key in sorted(occ))


def mb_orbital_groups(basis, max_block):
    """Blocks of the preconditioner as lists of state indices.

    The many-body basis orbital of a state is its pair of level-occupation
    tuples (species A, species B).  Groups are ordered by their lowest state;
    a group's states are ascending; a group of more than max_block states is
    cut into consecutive runs of max_block (the last shorter)."""
    groups = {}
    order = []
    for i in range(basis.D):
        key = (level_occupations(basis.orbs[0], basis.A[i]),
               level_occupations(basis.orbs[1], basis.B[i]) if basis.spec.n_species == 2 else ())
        if key not in groups:
            groups[key] = []
            order.append(key)
        groups[key].append(i)
    blocks = []
    for key in order:
        g = groups[key]
        for s in range(0, len(g), max_block):
            blocks.append(g[s:s + max_block])
    return blocks


def clamped_shift(x, floor=1e-2):
    """x moved away from zero to magnitude floor, sign kept (zero goes up):
    the guard of the diagonal preconditioner (diag - lambda)^-1."""
    if abs(x) >= floor:
        return x
    return -floor if x < 0 else floor


def block_precond_apply(row_ptr, col, val, blocks, R, theta, floor=1e-2):
    """W[:, c] = M_c^-1 R[:, c] with M_c the block diagonal of H - theta_c I
    over the given blocks, each block inverted through its eigenpairs
    (numpy's eigh) with eigenvalue gaps clamped like the diagonal
    preconditioner's: M_c^-1 = Q diag(1 / clamp(lambda_j - theta_c)) Q^T.
    float64 throughout."""
    D = len(row_ptr) - 1
    Hf = full_from_half(row_ptr, col, val, D)
    R = np.asarray(R, dtype=np.float64)
    W = np.zeros_like(R)
    for idx in blocks:
        idx = np.asarray(idx, dtype=np.int64)
        lam, Q = np.linalg.eigh(Hf[idx][:, idx].toarray())
        T = Q.T @ R[idx]
        for c, th in enumerate(theta):
            T[:, c] /= np.array([clamped_shift(l - th, floor) for l in lam])
        W[idx] = Q @ T
    return W
