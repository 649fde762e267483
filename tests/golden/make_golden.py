"""Write the stored expected values used by the full-size GPU parity tests.

Every number here is computed by the CPU oracle (oracle/) from the seeded
inputs (cigen); nothing comes from the GPU library.  Run from the repository
root:  python tests/golden/make_golden.py [workload ...]

Per workload it stores the basis dimension, the nonzero counts (from the
brute-force pattern, cross-checked against the class-pair count), and the
lowest eigenvalues of H in float64 and of the float32-rounded H (both by
ARPACK on the oracle's half-stored matrix, D <= 2e4 also by dense LAPACK).
"serve_sample" writes the lowest eigenvalues (float64 H and float32-rounded
H) of a fixed sample of the serving trace's requests.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cigen  # noqa: E402
import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def make(name):
    w = cigen.WORKLOADS[name]
    t0 = time.time()
    b = O.Basis(w.spec)
    tables = cigen.make_tables(w.spec, w.seed)
    inter = O.Interaction(b, tables)
    rp, col, val = O.half_csr(b, inter)
    full, half = O.nnz_class_count(w.spec)
    assert half == int(rp[-1]), (half, int(rp[-1]))
    k = max(w.nev, 10) + 3
    ev64, _ = O.eigs_sparse(rp, col, val, k)
    val32 = val.astype(np.float32).astype(np.float64)
    ev32, _ = O.eigs_sparse(rp, col, val32, k)
    out = dict(workload=name, spec=dict(n_species=w.spec.n_species, nmax=list(w.spec.nmax),
                                        n_particles=list(w.spec.n_particles),
                                        two_M=w.spec.two_M, cut=w.spec.cut),
               seed=w.seed, D=b.D, nnz_half=half, nnz_full=full,
               evals_f64=ev64[:k - 3].tolist(), evals_f32H=ev32[:k - 3].tolist(),
               diag_first=val[rp[:-1][:8]].tolist(),
               method="ARPACK eigsh(which='SA', tol=1e-13) on the oracle half CSR",
               source="tests/golden/make_golden.py (oracle/ and cigen/ only)")
    if b.D <= 20100:
        H = O.full_from_half(rp, col, val, b.D).toarray()
        out["evals_f64_lapack"] = O.eigs_dense(H, k - 3).tolist()
    out["seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, b.D, half, out["seconds"], "s", flush=True)


# A fixed sample of the 512-request serving trace (trace seed 5): shells up
# to 2, 3 and 4 (one and two 64-bit words per species), D from 67 to 59,462.
SERVE_SAMPLE = (0, 1, 3, 5, 7, 12, 14, 19, 22, 25, 27, 29, 30, 37)


def make_serve_sample():
    trace = cigen.request_trace(512, trace_seed=5)
    out = dict(trace_seed=5, n_requests=512, requests=[],
               method="dense LAPACK (D <= 4000) or ARPACK eigsh(which='SA', tol=1e-13) on the oracle half CSR",
               source="tests/golden/make_golden.py (oracle/ and cigen/ only)")
    for i in SERVE_SAMPLE:
        r = trace[i]
        t0 = time.time()
        b = O.Basis(r["spec"])
        rp, col, val = O.half_csr(b, O.Interaction(b, cigen.make_tables(r["spec"], r["seed"])))
        k = r["nev"]
        val32 = val.astype(np.float32).astype(np.float64)
        if b.D <= 4000:
            ev64 = O.eigs_dense(O.full_from_half(rp, col, val, b.D).toarray(), k)
            ev32 = O.eigs_dense(O.full_from_half(rp, col, val32, b.D).toarray(), k)
        else:
            ev64 = O.eigs_sparse(rp, col, val, k + 3)[0][:k]
            ev32 = O.eigs_sparse(rp, col, val32, k + 3)[0][:k]
        s = r["spec"]
        out["requests"].append(dict(id=i, seed=r["seed"], D=b.D, nnz_half=int(rp[-1]),
                                    spec=dict(nmax=list(s.nmax), n_particles=list(s.n_particles),
                                              two_M=s.two_M, cut=s.cut),
                                    evals_f64=list(map(float, ev64)), evals_f32H=list(map(float, ev32))))
        print("request", i, b.D, round(time.time() - t0, 1), "s", flush=True)
    with open(os.path.join(HERE, "serve_sample.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    names = sys.argv[1:] or list(cigen.WORKLOADS) + ["serve_sample"]
    for n in names:
        if n == "serve_sample":
            make_serve_sample()
        else:
            make(n)
