"""Failure handling, allocator hooks and determinism (GPU).

* Allocation failure: a user allocator that returns NULL on its k-th call,
  for every k a cib_build_H makes: each call returns CIB_E_NOMEM and leaves
  the context's live device bytes where they were; a build afterwards gives
  the oracle's half CSR.  In cib_serve the k-th allocation of a builder
  thread fails: that request alone reports CIB_E_NOMEM, every other result
  has the same bits as in a clean run, and the live bytes return.
* The torch caching-allocator hook carries a build, a product and a solve.
* Determinism: two builds give byte-identical CSR arrays; two products, and
  two solves, give identical bits (fixed summation orders throughout).
* The serving budget bounds the context's device memory: its peak stays
  within the budget plus the serving loop's own small buffers.
* A context destroyed while handles made on it are live stays usable by
  their frees (the cyclic garbage collector finalizes in any order).
"""
import ctypes
import threading

import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import golden, gpu_ctx, oracle_csr, oracle_tables

pytestmark = pytest.mark.gpu


class FailingAllocator:
    """torch's caching allocator behind a switch: with fail_at = k the k-th
    counted call (1-based) returns NULL; only_other_threads counts calls made
    on threads other than the one that armed it."""

    def __init__(self, device=0):
        import torch
        self.calls, self.fail_at, self.failed = 0, None, False
        self.only_other_threads, self.owner = False, threading.get_ident()
        self.lock = threading.Lock()

        def alloc(n):
            with self.lock:
                count = not self.only_other_threads or threading.get_ident() != self.owner
                if count:
                    self.calls += 1
                    if self.fail_at is not None and self.calls == self.fail_at:
                        self.failed = True
                        return None
            return torch.cuda.caching_allocator_alloc(int(n), device)

        def free(p):
            torch.cuda.caching_allocator_delete(p)

        self.hooks = (alloc, free)

    def arm(self, k, only_other_threads=False):
        with self.lock:
            self.calls, self.fail_at, self.failed = 0, k, False
            self.only_other_threads, self.owner = only_other_threads, threading.get_ident()


def _csr(H):
    rp, col, val = H.export()
    return rp, col, val


def test_build_nomem_at_every_allocation():
    from paper_2110_10765_amd import cib
    fa = FailingAllocator()
    ctx = cib.Context(0, allocator=fa.hooks)
    w = cigen.WORKLOADS["ab_n3_3p3_cut4"]
    tables = oracle_tables(w.spec, w.seed)
    b = cib.build_basis(ctx, w.spec)
    live0 = ctx.bytes()[0]
    fa.arm(None)
    H = cib.build_H(ctx, b, tables, "f64")
    n_alloc = fa.calls
    H.free()
    assert ctx.bytes()[0] == live0 and n_alloc > 10
    for k in range(1, n_alloc + 1):
        print("fail at allocation", k, "of", n_alloc, flush=True)
        fa.arm(k)
        with pytest.raises(cib.CibError) as e:
            cib.build_H(ctx, b, tables, "f64")
        assert e.value.code == cib.CIB_E_NOMEM and fa.failed
        assert ctx.bytes()[0] == live0, (k, ctx.bytes()[0], live0)
    fa.arm(None)
    H = cib.build_H(ctx, b, tables, "f64")
    rp, col, val = _csr(H)
    rp_r, col_r, val_r = oracle_csr(w.spec, w.seed)
    assert np.array_equal(rp, rp_r) and np.array_equal(col, col_r)
    assert np.abs(val - val_r).max() <= 1e-12


def test_destroy_before_handles():
    import gc
    import torch
    from paper_2110_10765_amd import cib
    lib = cib.load()
    ctx = cib.Context(0, torch_allocator=True)
    w = cigen.WORKLOADS["ab_n3_3p3_cut4"]
    b = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, b, oracle_tables(w.spec, w.seed), "f64")
    rp_r, col_r, val_r = oracle_csr(w.spec, w.seed)
    lib.cib_destroy(ctx.h)  # the context is kept while b and H live
    ctx.h = None
    rp, col, val = _csr(H)
    assert np.array_equal(rp, rp_r) and np.array_equal(col, col_r)
    H.free()
    b.free()  # the last handle: the context goes with it
    # a cycle holding a context and its handles, collected in one pass
    ctx2 = cib.Context(0, torch_allocator=True)
    b2 = cib.build_basis(ctx2, w.spec)
    H2 = cib.build_H(ctx2, b2, oracle_tables(w.spec, w.seed), "f32")
    cycle = [ctx2, b2, H2]
    cycle.append(cycle)
    del ctx2, b2, H2, cycle
    gc.collect()
    torch.cuda.synchronize()


def test_torch_allocator_build_product_solve():
    import torch
    from paper_2110_10765_amd import cib
    ctx = cib.Context(0, torch_allocator=True)
    w = cigen.WORKLOADS["ab_n3_3p3_cut4"]
    b = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, b, oracle_tables(w.spec, w.seed), "f64")
    rp, col, val = _csr(H)
    rp_r, col_r, val_r = oracle_csr(w.spec, w.seed)
    assert np.array_equal(rp, rp_r) and np.array_equal(col, col_r)
    X = torch.randn(b.dim, 8, dtype=torch.float64, device="cuda:0")
    Y = cib.apply_H(ctx, H, X)
    Yr, absHX = O.spmm_half(rp_r, col_r, val_r, X.cpu().numpy())
    k = 2 * int(np.diff(rp_r).max()) + 2
    u = 2.0 ** -53
    assert np.all(np.abs(Y.cpu().numpy() - Yr) <= k * u / (1 - k * u) * absHX + 1e-300)
    ev, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=800)
    ref = np.asarray(golden(w.name)["evals_f64"])[:w.nev]
    assert info["status"] == 0
    assert np.max(np.abs(ev - ref) / np.maximum(np.abs(ref), 1)) <= 1e-10


@pytest.mark.parametrize("name,dtype,nvec", [("ab_n3_3p3_cut4", "f64", 8), ("ab_n3_3p3_cut4", "f32", 16),
                                             ("sp1_n2_N4", "f64", 8), ("ab_n3_3p3_cut4", "f32", 5)])
def test_determinism(name, dtype, nvec):
    import torch
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    w = cigen.WORKLOADS[name]
    b = cib.build_basis(ctx, w.spec)
    tables = oracle_tables(w.spec, w.seed)
    H1 = cib.build_H(ctx, b, tables, dtype)
    H2 = cib.build_H(ctx, b, tables, dtype)
    for a, c in zip(_csr(H1), _csr(H2)):
        assert a.dtype == c.dtype and a.tobytes() == c.tobytes()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = torch.randn(b.dim, nvec, dtype=tdt, device="cuda:0")
    Y1 = cib.apply_H(ctx, H1, X)
    Y2 = cib.apply_H(ctx, H1, X)
    Y3 = cib.apply_H(ctx, H2, X)
    assert torch.equal(Y1, Y2) and torch.equal(Y1, Y3)
    e1, i1, _ = cib.lobpcg(ctx, H1, w.nev, block=w.block, max_iter=800)
    e2, i2, _ = cib.lobpcg(ctx, H2, w.nev, block=w.block, max_iter=800)
    assert i1["iters"] == i2["iters"] and np.array_equal(e1, e2)


def _serve_reqs(n, dtype="f64"):
    out = []
    for r in cigen.request_trace(n, trace_seed=5):
        s = r["spec"]
        spec = cigen.BasisSpec.two(min(s.nmax[0], 3), s.n_particles[0], min(s.nmax[1], 3), s.n_particles[1],
                                   s.two_M, s.cut)
        out.append(dict(r, spec=spec, dtype=dtype, tol=0.0, max_iter=800, tables=oracle_tables(spec, r["seed"])))
    return out


def test_serve_builder_nomem_fails_one_request():
    from paper_2110_10765_amd import cib
    fa = FailingAllocator()
    ctx = cib.Context(0, allocator=fa.hooks)
    reqs = _serve_reqs(12)
    live0 = ctx.bytes()[0]
    fa.arm(None)
    clean = cib.serve(ctx, reqs, max_active=8)
    assert ctx.bytes()[0] == live0
    for k in (1, 7, 40):
        print("serve: builder allocation", k, "fails", flush=True)
        fa.arm(k, only_other_threads=True)
        res = cib.serve(ctx, reqs, max_active=8)
        assert fa.failed
        assert ctx.bytes()[0] == live0
        bad = [r for r in res if r["status"] == cib.CIB_E_NOMEM]
        assert len(bad) == 1, [r["status"] for r in res]
        for a, r in zip(clean, res):
            if r["status"] == cib.CIB_E_NOMEM:
                continue
            assert r["status"] == a["status"]
            if a["status"] == 0:
                assert r["iters"] == a["iters"] and np.array_equal(r["evals"], a["evals"])


def test_serve_budget_bounds_device_memory():
    from paper_2110_10765_amd import cib
    ctx = cib.Context(0)
    reqs = _serve_reqs(24, dtype="f32")
    live0, peak0 = ctx.bytes()
    full = cib.serve(ctx, reqs)
    ok = [r for r in full if r["status"] == 0]
    budget = 96 << 20
    ctx2 = cib.Context(0)
    live0, _ = ctx2.bytes()
    res = cib.serve(ctx2, reqs, hbm_budget_bytes=budget)
    live1, peak1 = ctx2.bytes()
    assert live1 == live0
    # the serving loop's own buffers (grouped launch arguments) sit outside
    # the budget: at most 1 MiB
    assert peak1 - live0 <= budget + (1 << 20), (peak1 - live0, budget)
    n_ok = 0
    for a, r in zip(full, res):
        if r["status"] == 0:
            n_ok += 1
            assert a["status"] == 0 and r["iters"] == a["iters"] and np.array_equal(r["evals"], a["evals"])
        else:
            assert r["status"] in (cib.CIB_E_NOMEM, cib.CIB_E_EMPTY_BASIS), r
    assert n_ok >= len(ok) // 2
