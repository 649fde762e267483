"""GPU parity of the basis and of the half-stored Hamiltonian (through the C ABI).

Bar: basis words, row pointers and column indices bit-exact; values of
double-difference entries (one operator term: +-V) bit-exact in float64 and
equal to the float32 rounding of the oracle value; diagonal and single-
difference entries (several terms summed in another order) within
64 * 2^-53 * S, S = 2^8 bounding the sum of |terms| of these workloads
(<= 40 terms of |eps| <= 6, |V| <= 6); float32 values within one float32 ulp
of the oracle's float64 value.
"""
import os

import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import (EPS32, EPS64, GOLDEN, golden, gpu_ctx, oracle_basis, oracle_csr,
                          oracle_tables, xor_popcount_rows)

pytestmark = pytest.mark.gpu

SMALL = {
    "sp1_n2_N4": cigen.WORKLOADS["sp1_n2_N4"],
    "ab_n3_3p3_cut4": cigen.WORKLOADS["ab_n3_3p3_cut4"],
    "ragged_1sp": cigen.Workload("ragged_1sp", cigen.BasisSpec.one(3, 3, 1, 2), 21, 4, 8, "f64"),
    "ragged_2sp": cigen.Workload("ragged_2sp", cigen.BasisSpec.two(2, 2, 3, 3, 1, 3), 22, 4, 8, "f64"),
    "tiny_2sp": cigen.Workload("tiny_2sp", cigen.BasisSpec.two(1, 1, 1, 1, 0, -1), 23, 2, 2, "f64"),
    # two species with no truncation (a single Q level: every kA = 1 tile that
    # keeps 2m holds its row's own B configuration), D = 6,040 over many
    # 64-tile batches and entry windows
    "nocut_2sp": cigen.Workload("nocut_2sp", cigen.BasisSpec.two(2, 2, 2, 2, 0, -1), 27, 4, 8, "f64"),
    "one_state": cigen.Workload("one_state", cigen.BasisSpec.one(1, 8, 0, -1), 24, 1, 1, "f64"),
    # the largest orbital sets: n <= 6 is 168 orbitals, three 64-bit words;
    # N = 2 connects every pair (a dense H), and a mixed basis has three
    # words for A and one for B
    "w3_1sp_dense": cigen.Workload("w3_1sp_dense", cigen.BasisSpec.one(6, 2, 0, -1), 25, 4, 8, "f64"),
    "w3_2sp_mixed": cigen.Workload("w3_2sp_mixed", cigen.BasisSpec.two(6, 1, 2, 2, 1, 3), 26, 4, 8, "f64"),
}
TOL_ABS = 64 * EPS64 * 2.0 ** 8


def _gpu_basis_and_H(w, dtype):
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    print("case", w.name, dtype, flush=True)
    b = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, b, oracle_tables(w.spec, w.seed), dtype)
    return b, H


def _check_values(words, rp, col, val_gpu, val_ref, dtype):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    d = xor_popcount_rows(words, rows, col)
    assert set(np.unique(d).tolist()) <= {0, 2, 4}
    dd = d == 4
    if dtype == "f64":
        assert np.array_equal(val_gpu[dd], val_ref[dd])
        assert np.abs(val_gpu[~dd] - val_ref[~dd]).max(initial=0) <= TOL_ABS
    else:
        assert np.array_equal(val_gpu[dd], val_ref[dd].astype(np.float32))
        ulp = np.spacing(np.abs(val_ref.astype(np.float32)))
        assert np.all(np.abs(val_gpu.astype(np.float64) - val_ref) <= ulp)


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_basis_and_H_full(name, dtype):
    w = SMALL[name]
    ob = oracle_basis(w.spec)
    b, H = _gpu_basis_and_H(w, dtype)
    assert b.dim == ob.D == O.dim_generating_function(w.spec)
    words = b.export()
    assert np.array_equal(words, ob.species_words())
    rp_r, col_r, val_r = oracle_csr(w.spec, w.seed)
    rp, col, val = H.export()
    assert H.nnz == int(rp_r[-1])
    assert np.array_equal(rp, rp_r)
    assert np.array_equal(col, col_r)
    _check_values(words, rp, col, val, val_r, dtype)
    st = H.stats()
    assert st["t_total_s"] > 0


@pytest.mark.parametrize("name", ["ab_n3_3p3_cut6", "ab_n5_4p4_cut4"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_H_full_size_sampled_rows(name, dtype):
    """Full-size workloads: nnz against the stored oracle count, structural
    invariants of every row, and 48 sampled rows element by element."""
    w = cigen.WORKLOADS[name]
    if not os.path.exists(os.path.join(GOLDEN, name + ".json")):
        pytest.skip("stored oracle values for %s not generated" % name)
    g = golden(name)
    b, H = _gpu_basis_and_H(w, dtype)
    assert b.dim == g["D"]
    assert H.nnz == g["nnz_half"]
    rp, col, val = H.export()
    D = b.dim
    assert rp[0] == 0 and rp[-1] == H.nnz and np.all(np.diff(rp) >= 1)
    first = col[rp[:-1]]
    assert np.array_equal(first, np.arange(D))           # diagonal first
    rows = np.repeat(np.arange(D, dtype=np.int64), np.diff(rp))
    assert np.all(col >= rows)
    inner = np.ones(len(col), dtype=bool)
    inner[rp[:-1]] = False
    assert np.all(np.diff(col.astype(np.int64))[inner[1:]] > 0)   # ascending in a row
    words = b.export()
    d = xor_popcount_rows(words, rows, col)
    assert d.max() <= 4
    rng = np.random.default_rng(5)
    sample = np.unique(np.concatenate([[0, 1, D // 2, D - 2, D - 1], rng.integers(0, D, 43)]))
    ob = oracle_basis(w.spec)
    assert np.array_equal(words[sample], ob.species_words()[sample])
    ref = O.half_csr_rows(ob, O.Interaction(ob, oracle_tables(w.spec, w.seed)), sample)
    for i in sample:
        c_ref, v_ref = ref[int(i)]
        lo, hi = rp[i], rp[i + 1]
        assert np.array_equal(col[lo:hi], c_ref), i
        dd = xor_popcount_rows(words, np.full(hi - lo, i), col[lo:hi]) == 4
        if dtype == "f64":
            assert np.array_equal(val[lo:hi][dd], v_ref[dd]), i
            assert np.abs(val[lo:hi] - v_ref).max() <= TOL_ABS, i
        else:
            assert np.array_equal(val[lo:hi][dd], v_ref[dd].astype(np.float32)), i
            ulp = np.spacing(np.abs(v_ref.astype(np.float32)))
            assert np.all(np.abs(val[lo:hi].astype(np.float64) - v_ref) <= ulp), i


def test_invalid_specs_are_rejected():
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    bad = [cigen.BasisSpec(3, (2, 2), (2, 2), 0, -1),         # n_species
           cigen.BasisSpec.one(7, 2, 0, -1),                   # nmax > 6
           cigen.BasisSpec.one(1, 9, 1, -1),                   # N > n_orb
           cigen.BasisSpec.two(2, 2, 2, 1, 0, -1)]             # 2M parity
    for s in bad:
        with pytest.raises(cib.CibError) as e:
            cib.build_basis(ctx, s)
        assert e.value.code == cib.CIB_E_INVALID
    with pytest.raises(cib.CibError) as e:
        cib.build_basis(ctx, cigen.BasisSpec.one(1, 2, 40, -1))   # no state reaches 2M = 40
    assert e.value.code == cib.CIB_E_EMPTY_BASIS
