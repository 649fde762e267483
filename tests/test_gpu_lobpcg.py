"""GPU parity of the LOBPCG eigenvalues (cib_lobpcg) against the oracle.

Bar (relative error |lam - lam_ref| / max(|lam_ref|, 1)):
* float64 H: 1e-10 against LAPACK / ARPACK on the oracle's matrix;
* float32 H (SpMM in float32, Rayleigh-Ritz in float64): 1e-6 against the
  oracle's float64 eigenvalues.
Eigenvectors are checked through the oracle's residual ||Hx - lam x|| /
(max(|lam|,1) ||x||) and their orthonormality, never entry by entry (they are
defined only up to sign and rotation within degenerate subspaces).
"""
import os

import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import golden, gpu_ctx, oracle_csr, oracle_tables

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(b), 1.0)


def _solve(w, dtype, nev=None, block=None, **kw):
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    print("case", w.name, dtype, flush=True)
    b = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, b, oracle_tables(w.spec, w.seed), dtype)
    return cib.lobpcg(ctx, H, nev or w.nev, block=block or w.block, **kw)


@pytest.mark.parametrize("name", ["sp1_n2_N4", "ab_n3_3p3_cut4"])
def test_lobpcg_f64(name):
    w = cigen.WORKLOADS[name]
    g = golden(name)
    ev, info, vec = _solve(w, "f64", want_vectors=True, max_iter=800)
    assert info["status"] == 0, info
    ref = np.asarray(g.get("evals_f64_lapack", g["evals_f64"]))[:w.nev]
    assert _rel(ev, ref).max() <= 1e-10, (ev, ref)
    X = vec.cpu().numpy()
    assert np.abs(X.T @ X - np.eye(w.nev)).max() <= 1e-8
    rp, col, val = oracle_csr(w.spec, w.seed)
    assert O.residual_audit(rp, col, val, ev, X).max() <= 1e-8


@pytest.mark.parametrize("name", ["sp1_n2_N4", "ab_n3_3p3_cut4"])
def test_lobpcg_f32(name):
    w = cigen.WORKLOADS[name]
    g = golden(name)
    ev, info, _ = _solve(w, "f32", max_iter=800)
    assert info["status"] == 0, info
    assert _rel(ev, np.asarray(g["evals_f64"])[:w.nev]).max() <= 1e-6


@pytest.mark.parametrize("name,dtype", [("ab_n3_3p3_cut6", "f32"), ("ab_n5_4p4_cut4", "f32"),
                                        ("ab_n3_3p3_cut6", "f64"), ("ab_n5_4p4_cut4", "f64")])
def test_lobpcg_full_size(name, dtype):
    if not os.path.exists(os.path.join(GOLD, name + ".json")):
        pytest.skip("stored oracle eigenvalues not generated")
    w = cigen.WORKLOADS[name]
    g = golden(name)
    ev, info, _ = _solve(w, dtype, max_iter=1000)
    assert info["status"] == 0, info
    tol = 1e-6 if dtype == "f32" else 1e-10
    assert _rel(ev, np.asarray(g["evals_f64"])[:w.nev]).max() <= tol, (ev, g["evals_f64"][:w.nev])


@pytest.mark.parametrize("name", ["ab_n5_4p4_cut4", "ab_n3_3p3_cut6"])
def test_lobpcg_f32_against_f64_same_gpu(name):
    """The float32-H solve against the float64-H solve of the same basis on
    the same device: every requested eigenvalue within 1e-6 relative."""
    w = cigen.WORKLOADS[name]
    ev64, info64, _ = _solve(w, "f64", max_iter=1000)
    ev32, info32, _ = _solve(w, "f32", max_iter=1000)
    assert info64["status"] == 0 and info32["status"] == 0
    assert _rel(ev32, ev64).max() <= 1e-6, (ev32, ev64)


def test_lobpcg_block_sizes_and_small_basis():
    """block = nev, block = 16, and a basis only a few blocks wide."""
    spec = cigen.BasisSpec.two(1, 2, 2, 1, 1, -1)
    w = cigen.Workload("small", spec, 31, 3, 3, "f64")
    b = O.Basis(spec)
    H = O.dense_H(b, O.Interaction(b, oracle_tables(spec, 31)))
    ref = O.eigs_dense(H, 6)
    for nev, block in [(3, 3), (4, 8), (6, 16)]:
        if 3 * block > b.D:
            continue
        ev, info, _ = _solve(w, "f64", nev=nev, block=block, max_iter=500)
        assert info["status"] == 0
        assert _rel(ev, ref[:nev]).max() <= 1e-10, (nev, block)


def test_lobpcg_not_converged_and_invalid():
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["ab_n3_3p3_cut4"]
    ev, info, _ = _solve(w, "f64", max_iter=1)
    assert info["status"] == cib.CIB_E_NOT_CONVERGED
    assert info["iters"] == 1 and np.all(np.isfinite(ev)) and np.all(info["resid"] > 0)
    with pytest.raises(cib.CibError) as e:
        _solve(w, "f64", nev=9, block=8)
    assert e.value.code == cib.CIB_E_INVALID
    tiny = cigen.Workload("t", cigen.BasisSpec.two(1, 1, 1, 1, 0, -1), 3, 2, 8, "f64")  # D = 12 < 24
    with pytest.raises(cib.CibError) as e:
        _solve(tiny, "f64")
    assert e.value.code == cib.CIB_E_INVALID


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lobpcg_batched_iterations(dtype):
    """A single solve queues its iterations in batches and the converging one
    stops the rest on the device.  The count it reports must be the count
    that ran: max_iter one short of it stops there unconverged (a count that
    is not a multiple of the batch), max_iter equal to it gives the same bits,
    and the SpMM launches timed (queued-but-skipped ones dropped) and counted
    are one per iteration plus the start."""
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["sp1_n2_N4"]
    ctx = gpu_ctx()
    b = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, b, oracle_tables(w.spec, w.seed), dtype)
    ctx.profile(True)
    ev, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=800)
    n_launch, _ = ctx.kernel_time("spmm_sym")
    ctx.profile(False)
    n = info["iters"]
    assert info["status"] == 0 and n > 9, info
    assert n_launch == n + 1 and info["n_spmm"] == n + 1, (n_launch, info)
    ev_short, info_short, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=n - 1)
    assert info_short["status"] == cib.CIB_E_NOT_CONVERGED and info_short["iters"] == n - 1, info_short
    assert info_short["n_spmm"] == n, info_short
    ev_same, info_same, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=n)
    assert info_same["status"] == 0 and info_same["iters"] == n, info_same
    assert np.array_equal(ev_same, ev)
    assert _rel(ev, np.asarray(golden(w.name)["evals_f64"])[:w.nev]).max() <= (1e-10 if dtype == "f64" else 1e-6)
