"""Pins of the oracle's Hamiltonian (CPU only).

The oracle applies operator strings to bit strings.  It is pinned by:
* Jordan-Wigner Fock-space matrices: a_k built as Kronecker products, checked
  for the canonical anticommutation relations, H assembled by sparse matrix
  products from the generator's own table layout, then restricted to the
  basis -- an independent construction of the same second-quantised H;
* closed forms (two particles of one species; one particle of each species;
  V = 0; a completely filled species);
* the trace from generating functions (no state enumeration);
* symmetry H = H^T, with both triangles built from different kets.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import cigen
import oracle as O


def _tables(spec, seed=7, v_scale=1.0):
    return cigen.make_tables(spec, seed, v_scale)


def _dense(spec, tables):
    b = O.Basis(spec)
    return b, O.dense_H(b, O.Interaction(b, tables))


# ------------------------------------------------------------ Jordan-Wigner
def _jw_ops(K):
    """a_k for modes k = 0..K-1 on the 2^K Fock space; Fock index bit k is
    the occupation of mode k.  Kronecker factor order puts mode K-1 first."""
    I = sp.identity(2, format="csr")
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    lower = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    ops = []
    for k in range(K):
        m = sp.identity(1, format="csr")
        for q in range(K - 1, -1, -1):
            f = I if q > k else (lower if q == k else Z)
            m = sp.kron(m, f, format="csr")
        ops.append(m)
    return ops


def _jw_hamiltonian(spec, tables):
    nA = cigen.orbitals(spec.nmax[0]).shape[0]
    nB = cigen.orbitals(spec.nmax[1]).shape[0] if spec.n_species == 2 else 0
    K = nA + nB
    a = _jw_ops(K)
    ad = [x.T.tocsr() for x in a]
    H = sp.csr_matrix((2 ** K, 2 ** K))
    for k in range(nA):
        H = H + tables.eps[0][k] * (ad[k] @ a[k])
    for k in range(nB):
        H = H + tables.eps[1][k] * (ad[nA + k] @ a[nA + k])
    # same-species blocks, read with the generator's own layout description
    for s in range(spec.n_species):
        off = 0 if s == 0 else nA
        base = 0
        for (_, pa, pb) in cigen.same_pair_layout(spec.nmax[s]):
            n = len(pa)
            blk = tables.v_same[s][base:base + n * n].reshape(n, n)
            for p in range(n):
                for q in range(n):
                    aa, bb, cc, dd = off + pa[p], off + pb[p], off + pa[q], off + pb[q]
                    H = H + blk[p, q] * (ad[aa] @ ad[bb] @ a[dd] @ a[cc])
            base += n * n
    if spec.n_species == 2:
        base = 0
        for (_, pa, pb) in cigen.cross_pair_layout(spec.nmax[0], spec.nmax[1]):
            n = len(pa)
            blk = tables.v_ab[base:base + n * n].reshape(n, n)
            for p in range(n):
                for q in range(n):
                    aa, bb, cc, dd = pa[p], nA + pb[p], pa[q], nA + pb[q]
                    H = H + blk[p, q] * (ad[aa] @ ad[bb] @ a[dd] @ a[cc])
            base += n * n
    return H.tocsr(), a


def test_jw_anticommutation():
    a = _jw_ops(5)
    ad = [x.T.tocsr() for x in a]
    eye = sp.identity(32, format="csr")
    for i in range(5):
        for j in range(5):
            acomm = (a[i] @ ad[j] + ad[j] @ a[i]) - (eye if i == j else 0 * eye)
            assert abs(acomm).max() == 0
            assert abs(a[i] @ a[j] + a[j] @ a[i]).max() == 0


@pytest.mark.parametrize("spec", [
    cigen.BasisSpec.one(1, 2, 0, -1),
    cigen.BasisSpec.one(1, 3, 1, -1),
    cigen.BasisSpec.one(1, 4, 0, 1),
    cigen.BasisSpec.two(1, 2, 0, 1, 1, -1),
    cigen.BasisSpec.two(0, 1, 1, 2, 1, -1),
    cigen.BasisSpec.two(1, 2, 1, 1, 1, 1),
], ids=str)
def test_oracle_equals_jordan_wigner(spec):
    t = _tables(spec, seed=17)
    b, H = _dense(spec, t)
    Hf, _ = _jw_hamiltonian(spec, t)
    idx = np.asarray(b.glob, dtype=np.int64)
    ref = Hf[idx][:, idx].toarray()
    assert np.abs(H - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    # the Fock-space H conserves particle number: no coupling out of the basis
    # sector except through the truncation
    if spec.cut < 0:
        col = Hf[:, idx]
        inside = np.zeros(Hf.shape[0], dtype=bool)
        inside[idx] = True
        rows_hit = np.unique(col.nonzero()[0])
        assert inside[rows_hit].all()


# ------------------------------------------------------------ closed forms
def test_two_particles_one_species():
    """N = 2: H_(ab),(cd) = (eps_a + eps_b) delta + V_ab,cd with every phase +1."""
    spec = cigen.BasisSpec.one(2, 2, 0, -1)
    t = _tables(spec, seed=3)
    b, H = _dense(spec, t)
    lay = {}
    base = 0
    for (_, pa, pb) in cigen.same_pair_layout(2):
        n = len(pa)
        for p in range(n):
            lay[(int(pa[p]), int(pb[p]))] = (base, n, p)
        base += n * n
    pairs = [tuple(k for k in range(20) if (g >> k) & 1) for g in b.glob]
    for i, (a1, b1) in enumerate(pairs):
        for j, (c1, d1) in enumerate(pairs):
            bi, n, p = lay[(a1, b1)]
            bj, _, q = lay[(c1, d1)]
            want = t.v_same[0][bi + p * n + q] if bi == bj else 0.0
            if i == j:
                want += t.eps[0][a1] + t.eps[0][b1]
            assert H[i, j] == pytest.approx(want, abs=1e-14)


def test_one_particle_each_species():
    """1A + 1B: H_(ab),(cd) = (eps^A_a + eps^B_b) delta + V^AB_ab,cd."""
    spec = cigen.BasisSpec.two(2, 1, 2, 1, 0, -1)
    t = _tables(spec, seed=4)
    b, H = _dense(spec, t)
    lay = {}
    base = 0
    for (_, pa, pb) in cigen.cross_pair_layout(2, 2):
        n = len(pa)
        for p in range(n):
            lay[(int(pa[p]), int(pb[p]))] = (base, n, p)
        base += n * n
    st = [((a).bit_length() - 1, (bb).bit_length() - 1) for a, bb in zip(b.A, b.B)]
    for i, (a1, b1) in enumerate(st):
        for j, (c1, d1) in enumerate(st):
            bi, n, p = lay[(a1, b1)]
            bj, _, q = lay[(c1, d1)]
            want = t.v_ab[bi + p * n + q] if bi == bj else 0.0
            if i == j:
                want += t.eps[0][a1] + t.eps[1][b1]
            assert H[i, j] == pytest.approx(want, abs=1e-14)


def test_zero_interaction_is_diagonal():
    spec = cigen.BasisSpec.two(2, 2, 2, 2, 0, 2)
    t = _tables(spec, seed=5, v_scale=0.0)
    b, H = _dense(spec, t)
    assert np.count_nonzero(H - np.diag(np.diag(H))) == 0
    want = []
    for a, bb in zip(b.A, b.B):
        e = sum(t.eps[0][k] for k in range(b.n_orb[0]) if (a >> k) & 1)
        e += sum(t.eps[1][k] for k in range(b.n_orb[1]) if (bb >> k) & 1)
        want.append(e)
    assert np.allclose(np.diag(H), want, rtol=0, atol=1e-13)
    # eigenvalues are the sorted sums of occupied energies
    assert np.allclose(O.eigs_dense(H, 6), np.sort(want)[:6], atol=1e-12)


def test_filled_species():
    """N = n_orb (D = 1): E = sum eps + sum_{a<b} V_ab,ab."""
    spec = cigen.BasisSpec.one(1, 8, 0, -1)
    t = _tables(spec, seed=6)
    b, H = _dense(spec, t)
    assert b.D == 1
    e = math.fsum(t.eps[0])
    base = 0
    for (_, pa, pb) in cigen.same_pair_layout(1):
        n = len(pa)
        e += math.fsum(t.v_same[0][base + p * n + p] for p in range(n))
        base += n * n
    assert H[0, 0] == pytest.approx(e, abs=1e-12)


# ------------------------------------------------------------ trace, symmetry
@pytest.mark.parametrize("spec", [
    cigen.BasisSpec.one(2, 4, 0, -1),
    cigen.BasisSpec.two(2, 2, 2, 2, 0, 2),
    cigen.BasisSpec.two(1, 2, 2, 2, 0, -1),
], ids=str)
def test_trace_from_generating_functions(spec):
    t = _tables(spec, seed=8)
    b, H = _dense(spec, t)
    tr = O.trace_generating_function(spec, t)
    assert np.trace(H) == pytest.approx(tr, rel=1e-13, abs=1e-11)


def test_symmetry_and_c_helper_agree():
    spec = cigen.BasisSpec.two(2, 2, 2, 2, 0, 2)
    t = _tables(spec, seed=9)
    b, H = _dense(spec, t)
    assert np.abs(H - H.T).max() <= 1e-13
    rp, col, val = O.half_csr(b, O.Interaction(b, t))
    U = O.full_from_half(rp, col, val, b.D).toarray()
    assert np.abs(U - H).max() <= 1e-13
    # row sampler (values from the image of ket i) agrees with the full build
    rows = [0, b.D // 2, b.D - 1]
    R = O.half_csr_rows(b, O.Interaction(b, t), rows)
    for i in rows:
        c, v = R[i]
        assert np.array_equal(c, col[rp[i]:rp[i + 1]])
        assert np.abs(v - val[rp[i]:rp[i + 1]]).max() <= 1e-13


# ------------------------------------------------------------ C helper, several words
# The C helper (operator application on the concatenated bit string held as
# 64-bit words, with a hash map from state to index) computes every expected
# value at full size.  Its sign rule counts occupied modes below k across word
# boundaries; here it is checked against the Python operator application
# (pinned above by the Jordan-Wigner construction) on bases whose global modes
# span two, three and four words: 40 + 40 modes (species B straddles the first
# boundary), 168 modes of one species, 112 + 112 modes.  The sampled kets
# include those with two or more particles inside one word above the first,
# where the count of a partial word decides the sign.
def _upper_word_pairs(g):
    return any(bin((g >> (64 * w)) & ((1 << 64) - 1)).count("1") >= 2 for w in range(1, 4))


@pytest.mark.parametrize("spec", [
    cigen.BasisSpec.two(3, 2, 3, 2, 0, 6),
    cigen.BasisSpec.one(6, 3, 1, 10),
    cigen.BasisSpec.two(5, 2, 5, 2, 0, 4),
], ids=str)
def test_c_helper_across_words(spec):
    b = O.Basis(spec)
    inter = O.Interaction(b, _tables(spec, seed=11))
    assert sum(b.n_orb) > 64
    rng = np.random.default_rng(3)
    multi = [j for j, g in enumerate(b.glob) if _upper_word_pairs(g)]
    assert len(multi) >= 10
    pick = set(rng.choice(multi, min(40, len(multi)), replace=False).tolist())
    pick |= set(rng.choice(b.D, 40, replace=False).tolist())
    cols = np.array(sorted(pick), dtype=np.int64)
    ptr, rows, vals = O.apply_columns(b, inter, cols)
    for k, j in enumerate(cols):
        want = {}
        for bra, v in O.apply_H(b.glob[j], inter).items():
            i = b.index.get(bra)
            if i is not None:
                want[i] = v
        got = dict(zip(rows[ptr[k]:ptr[k + 1]].tolist(), vals[ptr[k]:ptr[k + 1]].tolist()))
        assert set(got) == set(want), "column %d: image rows differ" % j
        for i, v in want.items():
            assert got[i] == pytest.approx(v, rel=1e-14, abs=1e-14), (j, i)
