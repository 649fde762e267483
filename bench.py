#!/usr/bin/env python
"""Benchmark of the configuration-interaction hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole path on one synthetic problem (by default
the D = 198,912 two-species basis with float32 H, block 16, lowest 10
eigenpairs) with the interaction tables already resident in HBM: Slater-determinant basis, half-
stored H (popcount screen, phases, matrix elements, counts -> offsets ->
fill), and block LOBPCG to convergence (every iteration one symmetric SpMM,
float64 Gram / Rayleigh-Ritz / update).  Printed as one JSON line:

  value            H nonzeros built per second: nnz_half over the device time
                   of the build (HIP events around its kernels, both stored
                   triangles, tables resident), mean over the timed steps;
                   the rate over the wall time of the call is a submetric
  submetrics       H build rate per dtype, SpMM nnz*vec/s per dtype (kernel
                   time from HIP events), solves/s of the step, the same
                   numbers for the larger workloads, and the serving loop
                   (solves/s, p50/p99 latency) over the 512-request stream
  roofline         the kernel that dominates the step, its algorithmic bytes
                   per launch over its mean HIP-event duration vs 8 TB/s
                   (also: expectation values of 16 operators in 16 vectors,
                   the state-counting test's comparisons per second, and the
                   same eigenpairs by Lanczos)
  cpu_baseline     the CPU oracle (operator application + hashing) on a
                   bounded sample of the same workload, nnz per second; under
                   "serve", the serving stream through CPU worker processes
                   running the oracle, over a 20 s window; under "phases",
                   the oracle's basis, half CSR, SpMM and eigensolve on the
                   D = 20,004 workload
  host_nproc       host CPUs of the machine that ran it
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H nnz built/s; SpMM nnz·vec/s (FP64 vs FP32); solves/s + p99 latency"
HBM_PEAK_GBS = 8000.0


def _progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON line)."""
    print("bench: %s (%.0f s)" % (msg, time.perf_counter() - _T0), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def _sync():
    import torch
    torch.cuda.synchronize()


def _spmm_bytes(nnz_half, D, b, sv):
    return nnz_half * (4 + sv) + 8 * (D + 1) + 2 * D * b * sv


def _fill_bytes(nnz_half, D, sv):
    """Bytes the fill writes: both stored triangles (the upper half and the
    strictly lower copy the SpMM reads) and their row offsets."""
    return (2 * nnz_half - D) * (4 + sv) + 16 * (D + 1)


def _gram_bytes(D, b):
    return 2 * D * 3 * b * 8


def _update_bytes(D, b, f32):
    return 2 * D * 3 * b * 8 + 5 * D * b * 8 + (D * b * 4 if f32 else 0)


def _traffic(kernel, workload, dtype, block):
    """HBM bytes per launch of `kernel` from the committed counter profile
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counts), or None when
    there is none for this case or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "spmm_vec_ab_n3_3p3_cut6_traffic.json")
    src = os.path.join(ROOT, "paper_2110_10765_amd", "csrc", "spmm.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_id") != kernel or rec.get("workload") != workload or rec.get("dtype") != dtype
            or rec.get("block") != block or rec.get("source_sha256") != digest):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def measure_spmm(cib, ctx, H, b, reps):
    """Kernel-only SpMM time (HIP events inside the library) over `reps` applies."""
    import torch
    dt = torch.float64 if H.dtype == "f64" else torch.float32
    X = torch.randn(H.dim, b, dtype=dt, device="cuda:0")
    Y = torch.empty_like(X)
    for _ in range(3):
        cib.apply_H(ctx, H, X, Y)
    _sync()
    ctx.profile(True)
    for _ in range(reps):
        cib.apply_H(ctx, H, X, Y)
    _sync()
    n, t = ctx.kernel_time("spmm_sym")
    ctx.profile(False)
    return t / max(n, 1)


def measure_apply_free(cib, ctx, basis, inter, dtype, b, reps=5):
    """Matrix-free Y = H X (screens + values + apply pass, nothing stored):
    wall time per call, and the HIP-event time of the apply pass alone."""
    import torch
    dt = torch.float64 if dtype == "f64" else torch.float32
    X = torch.randn(basis.dim, b, dtype=dt, device="cuda:0")
    Y = torch.empty_like(X)
    cib.apply_H_free(ctx, basis, inter, X, Y)
    _sync()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        cib.apply_H_free(ctx, basis, inter, X, Y)
    _sync()
    wall = (time.perf_counter() - t0) / reps
    n, t = ctx.kernel_time("apply_free")
    ctx.profile(False)
    return wall, t / max(n, 1)


def measure_copy_gbs(reps=5):
    """Device-to-device copy of 1 GiB (torch), bytes read + written per
    second: the measured bandwidth the HBM fractions are also quoted against."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def workload_rates(cib, ctx, cigen, name, b, reps=20, copy_gbs=None):
    """Build and SpMM rates of one workload in both dtypes."""
    w = cigen.WORKLOADS[name]
    tables = cigen.make_tables(w.spec, w.seed)
    basis = cib.build_basis(ctx, w.spec)
    inter = cib.upload_interaction(ctx, basis, tables)
    out = {"D": basis.dim}
    for dt in ("f64", "f32"):
        sv = 8 if dt == "f64" else 4
        H = cib.build_H(ctx, basis, inter, dt)   # warm
        H.free()
        _sync()
        t0 = time.perf_counter()
        H = cib.build_H(ctx, basis, inter, dt)
        t_wall = time.perf_counter() - t0
        st = H.stats()
        t_spmm = measure_spmm(cib, ctx, H, b, reps)
        nnz_full = 2 * H.nnz - H.dim
        out["nnz_half"] = H.nnz
        out[dt] = {
            "build_nnz_per_s": H.nnz / st["t_total_s"],
            "build_wall_nnz_per_s": H.nnz / t_wall,
            "build_device_s": st["t_total_s"],
            "build_fill_s": st["t_fill_s"],
            "fill_hbm_frac": _fill_bytes(H.nnz, H.dim, sv) / st["t_fill_s"] / 1e9 / HBM_PEAK_GBS,
            "spmm_block": b,
            "spmm_nnz_vec_per_s": nnz_full * b / t_spmm,
            "spmm_kernel_s": t_spmm,
            "spmm_hbm_frac": _spmm_bytes(H.nnz, H.dim, b, sv) / t_spmm / 1e9 / HBM_PEAK_GBS,
            # the paper's counting metric: candidate state pairs (j >= i, what a
            # brute-force screen compares) per second of screen + count
            "screen_pairs_per_s": H.dim * (H.dim + 1) / 2 / (st["t_screen_s"] + st["t_count_s"]),
        }
        if b in (8, 16):
            wall, tpass = measure_apply_free(cib, ctx, basis, inter, dt, b)
            out[dt]["apply_free_wall_s"] = wall
            out[dt]["apply_free_pass_s"] = tpass
            out[dt]["apply_free_nnz_vec_per_s"] = nnz_full * b / wall
        if copy_gbs:
            out[dt]["fill_copy_frac"] = _fill_bytes(H.nnz, H.dim, sv) / st["t_fill_s"] / 1e9 / copy_gbs
            out[dt]["spmm_copy_frac"] = _spmm_bytes(H.nnz, H.dim, b, sv) / t_spmm / 1e9 / copy_gbs
        H.free()
    inter.free()
    basis.free()
    return out


def observables_rate(cib, ctx, cigen, name, nnz_half, m=16, nvec=16):
    """Expectation values of m random two-body operators (tables seeds
    2000 + k) in nvec vectors on the workload's basis: wall time of one
    cib_observables call (each operator applied once by the matrix-free
    product at 8 or 16 vectors)."""
    import torch
    w = cigen.WORKLOADS[name]
    basis = cib.build_basis(ctx, w.spec)
    tabs = [cigen.make_tables(w.spec, 2000 + k) for k in range(m)]
    tdt = torch.float64 if w.dtype == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(3)
    X = torch.randn(basis.dim, nvec, generator=g, dtype=torch.float64).to(tdt).to("cuda:0")
    cib.observables(ctx, basis, tabs[:1], X)   # warm
    _sync()
    t0 = time.perf_counter()
    cib.observables(ctx, basis, tabs, X)
    t = time.perf_counter() - t0
    nnz_full = 2 * nnz_half - basis.dim
    basis.free()
    return {"operators": m, "vectors": nvec, "dtype": w.dtype, "wall_s": t, "per_operator_s": t / m,
            "pair_vec_per_s": m * nnz_full * nvec / t}


def lanczos_rate(cib, ctx, cigen, w, inter, max_iter=1000):
    """The workload's lowest nev eigenpairs by Lanczos with full
    reorthogonalisation (the same H build, tolerance and nev as the LOBPCG
    step): steps, wall time of the solve, device time of its products."""
    basis = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, basis, inter, w.dtype)
    cib.lanczos(ctx, H, w.nev, max_iter=max_iter)           # warm
    _sync()
    t0 = time.perf_counter()
    ev, info, _ = cib.lanczos(ctx, H, w.nev, max_iter=max_iter)
    wall = time.perf_counter() - t0
    H.free()
    basis.free()
    return {"nev": w.nev, "steps": info["iters"], "status": info["status"], "solve_s": wall,
            "spmv_s": info["t_spmv_s"], "lowest_eigenvalues": ev.tolist()}


def precond_rates(cib, ctx, cigen, w, inter, caps=(16, 32, 64), max_iter=1000):
    """LOBPCG on the step's workload with the block-diagonal preconditioner
    over many-body basis orbitals (blocks of at most cap states) against the
    diagonal one: set-up wall time (groups, blocks, Jacobi eigenpairs),
    iterations and solve wall time."""
    basis = cib.build_basis(ctx, w.spec)
    H = cib.build_H(ctx, basis, inter, w.dtype)
    cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=max_iter)        # warm
    _sync()
    t0 = time.perf_counter()
    _, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=max_iter)
    out = {"diagonal": {"iters": info["iters"], "status": info["status"],
                        "solve_s": time.perf_counter() - t0}}
    for cap in caps:
        cib.Precond(ctx, basis, H, cap).free()                       # warm
        _sync()
        t0 = time.perf_counter()
        P = cib.Precond(ctx, basis, H, cap)
        setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=max_iter, precond=P)
        out["block_%d" % cap] = {"iters": info["iters"], "status": info["status"],
                                 "solve_s": time.perf_counter() - t0, "setup_s": setup,
                                 "blocks": P.n_blocks, "groups": P.n_groups, "largest": P.largest,
                                 "max_jacobi_sweeps": P.max_sweeps}
        P.free()
    H.free()
    basis.free()
    return out


def counting_rates(cib, ctx, cigen, n=1 << 17, N=8, reps=3):
    """The state-counting test at the paper's density: n biased random states
    of N particles in 128 single-particle states; state comparisons per second
    (n^2 over the kernel's HIP-event time) for the three methods."""
    import numpy as np
    mbs = cigen.counting_states(n, n_particles=N, n_sp=128, tau=36.0, seed=8)
    total, counts = cib.count_states(ctx, mbs, 128, 0)
    out = {"n": n, "particles": N, "n_sp": 128, "tau": 36.0, "connected_pairs": total,
           "median_density": float(np.median(counts)) / n}
    for m, name in ((0, "hybrid"), (1, "tuples_only"), (2, "bits128")):
        cib.count_states(ctx, mbs, 128, m, want_counts=False)     # warm
        ctx.profile(True)
        for _ in range(reps):
            tot, _ = cib.count_states(ctx, mbs, 128, m, want_counts=False)
            assert tot == total
        k, t = ctx.kernel_time("state_count")
        ctx.profile(False)
        out[name] = {"comparisons_per_s": n * n / (t / k), "kernel_s": t / k}
    return out


def serve_run(cib, ctx, cigen, dtype, n_req, budget=0, rate=math.inf):
    """The 512-request stream (trace seed 5).  rate = inf: all requests at
    t = 0 (closed loop, capacity); finite: Poisson arrivals replayed in real
    time, latency = t_done - t_arrive."""
    reqs = []
    for r in cigen.request_trace(n_req, rate=rate):
        r = dict(r)
        r["tables"] = cigen.make_tables(r["spec"], r["seed"])
        r["dtype"] = dtype
        r["tol"] = 0.0   # library default per dtype
        reqs.append(r)
    t0 = time.perf_counter()
    res = cib.serve(ctx, reqs, hbm_budget_bytes=budget, realtime=not math.isinf(rate))
    wall = time.perf_counter() - t0
    import numpy as np
    ok = [x for x in res if x["status"] == 0]
    lat = np.asarray([x["t_done"] - x["t_arrive"] for x in ok])
    wait = np.asarray([x["t_admit"] - x["t_arrive"] for x in ok])
    out = {"requests": n_req, "ok": len(ok),
           "empty_basis": sum(1 for x in res if x["status"] == cib.CIB_E_EMPTY_BASIS),
           "nomem": sum(1 for x in res if x["status"] == cib.CIB_E_NOMEM),
           "solves_per_s": len(ok) / wall, "makespan_s": wall,
           "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
           "admit_wait_p99_s": float(np.percentile(wait, 99)) if len(wait) else None}
    err = serve_sample_errors(res)
    if err:
        out["eval_rel_err_vs_oracle_f64"] = err
    if not math.isinf(rate):
        out["arrival_rate_per_s"] = rate
    if budget:
        out["hbm_budget_bytes"] = budget
    return out


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _rel_err(ev, ref):
    import numpy as np
    ev, ref = np.asarray(ev, dtype=float), np.asarray(ref, dtype=float)
    return (np.abs(ev - ref) / np.maximum(np.abs(ref), 1.0)).tolist()


def serve_sample_errors(res):
    """Eigenvalue error of each result in the stored sample of the trace
    (oracle float64 eigenvalues, tests/golden/serve_sample.json), relative
    to max(|lambda|, 1): per request id and the largest."""
    g = _golden("serve_sample")
    if not g:
        return None
    ref = {r["id"]: r["evals_f64"] for r in g["requests"]}
    per = {}
    for x in res:
        if x["status"] == 0 and x["id"] in ref:
            k = len(ref[x["id"]])
            per[str(x["id"])] = max(_rel_err(list(x["evals"])[:k], ref[x["id"]]))
    if not per:
        return None
    return {"max": max(per.values()), "per_request": per}


def small_case_us(cib, ctx, cigen, name="sp1_n2_N4", reps=20):
    """The D = 849 one-species workload (launch-latency bound): device time of
    the build (HIP events around its kernels), of one SpMM at its block, and
    the wall time of cib_lobpcg, in microseconds; eigenvalue error against
    the stored oracle (LAPACK) values."""
    w = cigen.WORKLOADS[name]
    basis = cib.build_basis(ctx, w.spec)
    inter = cib.upload_interaction(ctx, basis, cigen.make_tables(w.spec, w.seed))
    H = cib.build_H(ctx, basis, inter, w.dtype)
    H.free()
    builds = []
    for _ in range(reps):
        H = cib.build_H(ctx, basis, inter, w.dtype)
        builds.append(H.stats()["t_total_s"])
        H.free()
    H = cib.build_H(ctx, basis, inter, w.dtype)
    t_spmm = measure_spmm(cib, ctx, H, w.block, reps)
    cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=1000)
    _sync()
    t0 = time.perf_counter()
    for _ in range(5):
        ev, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=1000)
    solve = (time.perf_counter() - t0) / 5
    out = {"D": H.dim, "nnz_half": H.nnz, "dtype": w.dtype, "block": w.block,
           "build_device_us": 1e6 * sum(builds) / len(builds), "spmm_kernel_us": 1e6 * t_spmm,
           "lobpcg_wall_us": 1e6 * solve, "lobpcg_iters": info["iters"]}
    g = _golden(name)
    if g:
        ref = g.get("evals_f64_lapack", g["evals_f64"])[:w.nev]
        out["eval_rel_err_vs_oracle_f64"] = max(_rel_err(ev, ref))
    H.free()
    inter.free()
    basis.free()
    return out


def serve_suite(cib, ctx, cigen, n_req, sweep=True):
    """Closed-loop capacity C per dtype; with sweep, Poisson replays of the
    same trace at 0.5, 0.8, 0.95 C (float32) and 0.8 C (float64), and the
    closed loop under 2 GiB and 8 GiB HBM budgets (admission queueing)."""
    sub = {}
    for dt in ("f32", "f64"):
        sub["serve_" + dt] = serve_run(cib, ctx, cigen, dt, n_req)
        _progress("serving stream %s done" % dt)
    if not sweep:
        return sub
    for dt, fracs in (("f32", (0.5, 0.8, 0.95)), ("f64", (0.8,))):
        cap = sub["serve_" + dt]["solves_per_s"]
        for f in fracs:
            sub["serve_%s_poisson_%02d" % (dt, round(100 * f))] = serve_run(cib, ctx, cigen, dt, n_req,
                                                                             rate=f * cap)
            _progress("serving stream %s at %.2f of capacity done" % (dt, f))
    for dt in ("f32", "f64"):
        for gib in (2, 8):
            sub["serve_%s_budget_%dgib" % (dt, gib)] = serve_run(cib, ctx, cigen, dt, n_req,
                                                                 budget=gib << 30)
            _progress("serving stream %s under %d GiB done" % (dt, gib))
    return sub


def cpu_baseline(cigen, name, seconds=15.0):
    """The CPU oracle applying H to a bounded sample of kets of the workload."""
    import numpy as np
    import oracle as O
    w = cigen.WORKLOADS[name]
    b = O.Basis(w.spec)
    inter = O.Interaction(b, cigen.make_tables(w.spec, w.seed))
    rng = np.random.default_rng(0)
    n = 256
    total_nnz, total_t, cols_done = 0, 0.0, 0
    while total_t < seconds:
        cols = rng.integers(0, b.D, size=n)
        t0 = time.perf_counter()
        ptr, rows, vals = O.apply_columns(b, inter, cols)
        total_t += time.perf_counter() - t0
        total_nnz += int(ptr[-1])
        cols_done += len(cols)
        n = min(2 * n, 1 << 16)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # nnz_full entries produced -> nnz_half-equivalent rate (each stored entry once)
    return {"value": total_nnz / total_t * 0.5 * (1 + 1.0 / max(1, total_nnz / cols_done)),
            "unit": "nnz/s", "cores": threads, "kind": "oracle",
            "sample": "%d random kets of %s (D=%d): H applied by operator strings + hash lookup, "
                      "%.1f s; stored half-entries per second" % (cols_done, name, b.D, total_t)}


def cpu_phase_baseline(cigen, name="ab_n3_3p3_cut4", b=8, seconds=2.0):
    """The oracle's other phases on the D = 20,004 workload (the largest whose
    whole half CSR the oracle builds in seconds): basis, half CSR, half-CSR
    SpMM at block b in both dtypes (the oracle expands the half and also forms
    |H| |X| on every call), and the lowest 5 eigenvalues by ARPACK."""
    import numpy as np
    import oracle as O
    w = cigen.WORKLOADS[name]
    t0 = time.perf_counter()
    basis = O.Basis(w.spec)
    t1 = time.perf_counter()
    rp, col, val = O.half_csr(basis, O.Interaction(basis, cigen.make_tables(w.spec, w.seed)))
    t2 = time.perf_counter()
    nnz_full = 2 * len(col) - basis.D
    X = np.random.default_rng(0).standard_normal((basis.D, b))
    out = {"workload": name, "D": basis.D, "nnz_half": len(col), "basis_s": t1 - t0,
           "half_csr_s": t2 - t1, "half_csr_nnz_per_s": len(col) / (t2 - t1)}
    for dt, npt in (("f64", np.float64), ("f32", np.float32)):
        v, Xd = val.astype(npt), X.astype(npt)
        n, ts = 0, time.perf_counter()
        while time.perf_counter() - ts < seconds:
            O.spmm_half(rp, col, v, Xd)
            n += 1
        out["spmm_%s_nnz_vec_per_s" % dt] = nnz_full * b / ((time.perf_counter() - ts) / n)
    ts = time.perf_counter()
    O.eigs_sparse(rp, col, val, 5, tol=1e-10)
    out["eigensolve_s"] = time.perf_counter() - ts
    out["spmm_block"] = b
    return out


def _cpu_solve(req):
    """One request of the serving stream solved by the CPU oracle: basis, the
    half-stored H from the operator image, and its lowest eigenvalues (dense
    LAPACK up to D = 600, else ARPACK).  Runs in a worker process."""
    sys.path.insert(0, ROOT)
    import cigen
    import oracle as O
    t0 = time.perf_counter()
    b = O.Basis(req["spec"])
    if b.D > 0:
        inter = O.Interaction(b, cigen.make_tables(req["spec"], req["seed"]))
        rp, col, val = O.half_csr(b, inter)
        k = min(req["nev"], b.D)
        if b.D <= 600:
            O.eigs_dense(O.full_from_half(rp, col, val, b.D).toarray(), k)
        else:
            O.eigs_sparse(rp, col, val, k, tol=1e-10)
    return req["id"], b.D, time.perf_counter() - t0


def cpu_serve_baseline(n_req, seconds=20.0):
    """The serving stream through a pool of CPU worker processes running the
    oracle, closed loop in trace order, over a window of `seconds`: requests
    finished inside the window per second (the window cuts off the requests
    still running, so large ones are under-represented)."""
    import multiprocessing as mp
    import cigen
    workers = max(1, min(16, os.cpu_count() or 1))
    reqs = cigen.request_trace(n_req)
    done = []
    # spawned workers: fresh interpreters that never touch the GPU
    pool = mp.get_context("spawn").Pool(workers)
    try:
        t0 = time.perf_counter()
        it = pool.imap_unordered(_cpu_solve, reqs, chunksize=1)
        while True:
            left = seconds - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                done.append(it.next(timeout=left))
            except mp.TimeoutError:
                break
            except StopIteration:
                break
        window = min(seconds, time.perf_counter() - t0)
    finally:
        pool.terminate()
        pool.join()
    dims = sorted(d for _, d, _ in done)
    return {"value": len(done) / window, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": "%d of the %d requests of the serving stream finished within a %.0f s window "
                      "(closed loop, trace order, %d worker processes; D of the finished ones %s-%s): "
                      "basis, half CSR from the operator image, lowest 4 eigenvalues (LAPACK for D <= "
                      "600, else ARPACK)" % (len(done), n_req, window, workers,
                                            dims[0] if dims else "-", dims[-1] if dims else "-")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ab_n3_3p3_cut6")
    ap.add_argument("--extra", default="ab_n3_3p3_cut4:8,ab_n5_4p4_cut4:8")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-serve-sweep", action="store_true",
                    help="serving: closed loop only (no Poisson replays, no budget runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the observables, Lanczos and state-counting measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB five times (scale factor for the HBM byte counters)")
    ap.add_argument("--precond-only", action="store_true",
                    help="only the block-diagonal preconditioner measurement (JSON line)")
    ap.add_argument("--spmm-only", default="",
                    help="NAME:block:dtype -- only build H and run 10 SpMMs (for counter runs)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the closed-loop serving runs, float32 and float64 H (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU; --gpus %d is not supported (multi-GPU sharding "
              "is a design note only)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import cigen
    from paper_2110_10765_amd import cib

    if args.calibrate_copy:
        n = 1 << 27                          # 2^27 float64 = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        _sync()
        print(json.dumps({"calibrate_copy_bytes_each_way": n * 8, "launches": 5}))
        return
    if args.spmm_only:
        name, bb, dt = args.spmm_only.split(":")
        wl = cigen.WORKLOADS[name]
        ctx = cib.Context(0)
        basis = cib.build_basis(ctx, wl.spec)
        H = cib.build_H(ctx, basis, cigen.make_tables(wl.spec, wl.seed), dt)
        t = measure_spmm(cib, ctx, H, int(bb), 10)
        sv = 8 if dt == "f64" else 4
        print(json.dumps({"workload": name, "dtype": dt, "block": int(bb), "D": H.dim,
                          "nnz_half": H.nnz, "spmm_kernel_s": t,
                          "algorithmic_bytes": _spmm_bytes(H.nnz, H.dim, int(bb), sv)}))
        return

    if args.serve_only:
        ctx = cib.Context(0)
        print(json.dumps({"serve": serve_suite(cib, ctx, cigen, args.serve_requests, sweep=False)}))
        return

    if args.precond_only:
        # the block-diagonal preconditioner's set-up and LOBPCG runs with it
        # on the step's workload, alone (for kernel traces)
        w = cigen.WORKLOADS[args.workload]
        ctx = cib.Context(0)
        b0 = cib.build_basis(ctx, w.spec)
        inter = cib.upload_interaction(ctx, b0, cigen.make_tables(w.spec, w.seed))
        print(json.dumps({"workload": w.name, "block_precond": precond_rates(cib, ctx, cigen, w, inter)}))
        return

    w = cigen.WORKLOADS[args.workload]
    ctx = cib.Context(0)
    tables = cigen.make_tables(w.spec, w.seed)
    basis0 = cib.build_basis(ctx, w.spec)
    inter = cib.upload_interaction(ctx, basis0, tables)    # tables resident before timing

    def step(record=None):
        t0 = time.perf_counter()
        b = cib.build_basis(ctx, w.spec)
        t1 = time.perf_counter()
        H = cib.build_H(ctx, b, inter, w.dtype)
        t2 = time.perf_counter()
        ev, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=1000)
        t3 = time.perf_counter()
        if record is not None:
            record.append(dict(basis=t1 - t0, build=t2 - t1, solve=t3 - t2, nnz=H.nnz,
                               build_device=H.stats()["t_total_s"],
                               iters=info["iters"], status=info["status"], ev=ev.tolist()))
        H.free()
        b.free()

    for _ in range(args.warmup):
        step()
    _sync()
    _progress("warm-up steps done")
    ctx.profile(True)
    rec = []
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    _sync()
    elapsed = time.perf_counter() - t0
    _progress("timed steps done")
    kernels = {}
    for k in ("screens", "row_count", "scan", "row_fill", "spmm_sym", "gram",
              "rayleigh_ritz", "update"):
        n, t = ctx.kernel_time(k)
        kernels[k] = {"launches": n, "total_s": t, "mean_s": t / n if n else None}
    ctx.profile(False)

    D, nnz = basis0.dim, rec[0]["nnz"]
    sv = 8 if w.dtype == "f64" else 4
    b = w.block
    algo = {"spmm_sym": _spmm_bytes(nnz, D, b, sv), "row_fill": _fill_bytes(nnz, D, sv),
            "gram": _gram_bytes(D, b), "update": _update_bytes(D, b, w.dtype == "f32")}
    dom = max(kernels, key=lambda k: kernels[k]["total_s"])
    roof = None
    if dom in algo and kernels[dom]["launches"]:
        mean = kernels[dom]["mean_s"]
        ach = algo[dom] / mean / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": _traffic(dom, w.name, w.dtype, b),
                "bytes_per_launch": algo[dom], "mean_launch_s": mean}
    else:
        roof = {"kernel": dom, "bound": "latency", "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None, "mean_launch_s": kernels[dom]["mean_s"]}

    build_t = sum(r["build"] for r in rec) / len(rec)
    build_dev = sum(r["build_device"] for r in rec) / len(rec)
    g = _golden(w.name)
    step_err = None
    if g:
        step_err = _rel_err(rec[-1]["ev"], g["evals_f64"][:w.nev])
    sub = {
        "step_eval_rel_err_vs_oracle_f64": {"max": max(step_err), "per_eigenvalue": step_err} if step_err else None,
        "step_breakdown_s": {k: sum(r[k] for r in rec) / len(rec) for k in ("basis", "build", "solve")},
        "build_device_s": build_dev,
        "build_wall_nnz_per_s": nnz / build_t,
        "lobpcg_iters": [r["iters"] for r in rec],
        "lowest_eigenvalues": rec[-1]["ev"],
        "solves_per_s": args.steps / elapsed,
        "kernels": kernels,
    }
    copy_gbs = measure_copy_gbs()
    sub["hbm_copy_gbs"] = copy_gbs
    if roof.get("achieved"):
        roof["copy_frac"] = roof["achieved"] / copy_gbs
    ws = {}
    for item in filter(None, [args.workload + ":%d" % w.block] + args.extra.split(",")):
        name, bb = item.split(":")
        ws[name] = workload_rates(cib, ctx, cigen, name, int(bb), copy_gbs=copy_gbs)
    sub["workloads"] = ws
    _progress("workload rates done")
    sub["small_case"] = small_case_us(cib, ctx, cigen)
    if not args.no_next:
        sub["observables"] = observables_rate(cib, ctx, cigen, w.name, nnz)
        sub["lanczos"] = lanczos_rate(cib, ctx, cigen, w, inter)
        _progress("observables and Lanczos done")
        sub["block_precond"] = precond_rates(cib, ctx, cigen, w, inter)
        sub["state_count"] = counting_rates(cib, ctx, cigen)
        _progress("preconditioner and state counting done")
    if not args.no_serve:
        try:
            sub.update(serve_suite(cib, ctx, cigen, args.serve_requests, sweep=not args.no_serve_sweep))
        except cib.CibError as e:
            sub["serve"] = {"error": str(e)}
    line = {
        "metric": METRIC, "value": nnz / build_dev, "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": w.dtype,
        "dtype_note": "H values and SpMM in %s; Gram, Rayleigh-Ritz, residuals in f64" % w.dtype,
        "data": "synthetic (seeded eps ~ n + U(-0.1,0.1), V ~ N(0,1) m-conserving)",
        "config": {"workload": w.name, "D": D, "nnz_half": nnz, "nev": w.nev, "block": w.block,
                   "parallelism": "1 GPU"},
        "roofline": roof, "submetrics": sub, "host_nproc": os.cpu_count(),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cigen, w.name)
        line["cpu_baseline"]["phases"] = cpu_phase_baseline(cigen)
        _progress("CPU oracle baseline done")
        if not args.no_serve:
            line["cpu_baseline"]["serve"] = cpu_serve_baseline(args.serve_requests)
            _progress("CPU serving baseline done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
