"""GPU parity of the matrix-free product Y = H X (cib_apply_H_free: the
build's screens and values multiplied into X without storing H) against the
oracle, in the bar of the SpMM tests: |Y - Y_ref| <= gamma_k |H| |X| with
k = 2 (max row length) + 2 and the unit roundoff of the dtype (the float32
reference rounds the oracle's matrix and X to float32).  Small workloads
are compared in full; at D = 198,912 and 173,624, 64 sampled rows are
compared with rows the oracle computes one by one, and the whole product
with the stored-matrix SpMM."""
import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import EPS32, EPS64, gpu_ctx, oracle_basis, oracle_csr, oracle_tables

pytestmark = pytest.mark.gpu


def _gamma(k, u):
    return k * u / (1 - k * u)


@pytest.mark.parametrize("name", ["sp1_n2_N4", "ab_n3_3p3_cut4"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nvec", [8, 16])
def test_apply_free_matches_oracle(name, dtype, nvec):
    import torch
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS[name]
    ctx = gpu_ctx()
    print("case", name, dtype, nvec, flush=True)
    b = cib.build_basis(ctx, w.spec)
    inter = cib.upload_interaction(ctx, b, oracle_tables(w.spec, w.seed))
    rp, col, val = oracle_csr(w.spec, w.seed)
    X = np.random.default_rng(nvec).standard_normal((b.dim, nvec))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
        val = val.astype(np.float32).astype(np.float64)
    Y = cib.apply_H_free(ctx, b, inter, torch.tensor(X, dtype=tdt, device="cuda:0"))
    torch.cuda.synchronize()
    Yref, absHX = O.spmm_half(rp, col, val, X)
    k = 2 * int(np.diff(rp).max()) + 2
    u = EPS64 if dtype == "f64" else EPS32
    assert np.all(np.abs(Y.cpu().numpy().astype(np.float64) - Yref) <= _gamma(k, u) * absHX + 1e-300)


@pytest.mark.parametrize("name,nvec", [("ab_n3_3p3_cut6", 16), ("ab_n5_4p4_cut4", 8)])
def test_apply_free_full_size(name, nvec):
    import torch
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS[name]
    ctx = gpu_ctx()
    print("case", name, nvec, flush=True)
    b = cib.build_basis(ctx, w.spec)
    tables = oracle_tables(w.spec, w.seed)
    inter = cib.upload_interaction(ctx, b, tables)
    D = b.dim
    rng = np.random.default_rng(12)
    X = rng.standard_normal((D, nvec)).astype(np.float32).astype(np.float64)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda:0")
    Y = cib.apply_H_free(ctx, b, inter, Xd).cpu().numpy().astype(np.float64)
    # the stored matrix, same values, other summation order
    H = cib.build_H(ctx, b, inter, "f32")
    Ys = cib.apply_H(ctx, H, Xd).cpu().numpy().astype(np.float64)
    H.free()
    sample = np.unique(np.concatenate([[0, 1, D // 2, D - 2, D - 1], rng.integers(0, D, 59)]))
    ob = oracle_basis(w.spec)
    ptr, rows, vals = O.apply_columns(ob, O.Interaction(ob, tables), sample)
    for c, i in enumerate(sample):
        rr, vv = rows[ptr[c]:ptr[c + 1]], vals[ptr[c]:ptr[c + 1]].astype(np.float32).astype(np.float64)
        yref = vv @ X[rr]
        absHX = np.abs(vv) @ np.abs(X[rr])
        tol = _gamma(len(rr) + 2, EPS32) * absHX + 1e-300
        assert np.all(np.abs(Y[i] - yref) <= tol), (i, Y[i], yref)
    # whole product against the stored-matrix SpMM: both within the bound of
    # the exact product, so within twice that of each other; |H| |X| is
    # bounded below by |H X| only, so compare in a norm
    assert np.linalg.norm(Y - Ys) <= 1e-5 * np.linalg.norm(Ys)


def test_apply_free_rejects_bad_arguments():
    import torch
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["sp1_n2_N4"]
    ctx = gpu_ctx()
    b = cib.build_basis(ctx, w.spec)
    inter = cib.upload_interaction(ctx, b, oracle_tables(w.spec, w.seed))
    with pytest.raises(cib.CibError):
        cib.apply_H_free(ctx, b, inter, torch.zeros((b.dim, 4), dtype=torch.float64, device="cuda:0"))
    X = torch.zeros((b.dim, 9), dtype=torch.float64, device="cuda:0")[:, :8]   # ld 9: rows not 16-byte aligned
    with pytest.raises(cib.CibError):
        cib.apply_H_free(ctx, b, inter, X)
    other = cib.build_basis(ctx, cigen.WORKLOADS["ab_n3_3p3_cut4"].spec)
    with pytest.raises(cib.CibError):
        cib.apply_H_free(ctx, other, inter, torch.zeros((other.dim, 8), dtype=torch.float64, device="cuda:0"))


@pytest.mark.parametrize("spec,seed", [(cigen.BasisSpec.one(6, 2, 0, -1), 25),
                                       (cigen.BasisSpec.two(6, 1, 2, 2, 1, 3), 26)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_free_three_words(spec, seed, dtype):
    """168 orbitals (three 64-bit words per configuration), against the oracle."""
    import torch
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    print("case", spec, dtype, flush=True)
    b = cib.build_basis(ctx, spec)
    inter = cib.upload_interaction(ctx, b, oracle_tables(spec, seed))
    rp, col, val = oracle_csr(spec, seed)
    X = np.random.default_rng(seed).standard_normal((b.dim, 8))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        X = X.astype(np.float32).astype(np.float64)
        val = val.astype(np.float32).astype(np.float64)
    Y = cib.apply_H_free(ctx, b, inter, torch.tensor(X, dtype=tdt, device="cuda:0"))
    torch.cuda.synchronize()
    Yref, absHX = O.spmm_half(rp, col, val, X)
    k = 2 * int(np.diff(rp).max()) + 2
    u = EPS64 if dtype == "f64" else EPS32
    assert np.all(np.abs(Y.cpu().numpy().astype(np.float64) - Yref) <= _gamma(k, u) * absHX + 1e-300)
