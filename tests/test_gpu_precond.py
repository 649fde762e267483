"""GPU parity of the block-diagonal preconditioner over many-body basis
orbitals (cib_precond_*, Sec. 2) and of LOBPCG run with it.

* Blocks (perm, offsets): bit-exact against the oracle's grouping.
* Application W = M(theta)^-1 R: the device eigenpairs come from Jacobi
  rotations stopped at an off-diagonal norm of 1e-15 of the block's Frobenius
  norm, the oracle's from LAPACK; both are backward stable, so a block's
  result moves by at most about |f'| ||E|| ||r|| + |f| ||r|| n u with
  f = 1 / g(lambda - theta), |f| <= 1/delta, |f'| <= 1/delta^2, delta the
  smallest guarded gap and ||E|| <= (1e-15 + n u) ||B||_F.  The bar is
  1e-12 (||B||_F / delta^2 + 1 / delta) ||r_k|| per block.  Shifts are kept
  1e-6 away from every block eigenvalue, where the guard's sign would be
  decided by rounding.
* Blocks of one state: R / g(diag - theta), one division on both sides, the
  diagonals equal up to the build's rounding; exact where the gap is guarded;
  and the whole LOBPCG solve bit-identical to the diagonal run.
* LOBPCG with the preconditioner: the eigenvalue bars of the diagonal runs.
"""
import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import EPS64, golden, gpu_ctx, oracle_basis, oracle_csr, oracle_tables

pytestmark = pytest.mark.gpu

SMALL = {
    "tiny": (cigen.BasisSpec.two(1, 1, 1, 1, 0, -1), 3),
    "one_species": (cigen.WORKLOADS["sp1_n2_N4"].spec, 1),
    "mixed": (cigen.BasisSpec.two(2, 2, 2, 3, 1, 2), 5),
    "cut4": (cigen.WORKLOADS["ab_n3_3p3_cut4"].spec, 1),
    # configurations over two and three 64-bit words (112 and 168 orbitals)
    "w3_1sp": (cigen.BasisSpec.one(6, 2, 0, -1), 25),
    "w3_2sp": (cigen.BasisSpec.two(6, 1, 2, 2, 1, 3), 26),
    "w2_b": (cigen.BasisSpec.two(4, 2, 5, 2, 0, 2), 27),
}


def _setup(spec, seed, dtype, cap):
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    b = cib.build_basis(ctx, spec)
    H = cib.build_H(ctx, b, oracle_tables(spec, seed), dtype)
    P = cib.Precond(ctx, b, H, cap)
    return ctx, b, H, P


def _flat(blocks):
    perm = np.asarray([i for g in blocks for i in g], dtype=np.int32)
    off = np.cumsum([0] + [len(g) for g in blocks]).astype(np.int64)
    return perm, off


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("cap", [1, 7, 64])
def test_blocks_match_oracle(name, cap):
    spec, seed = SMALL[name]
    print("case blocks", name, cap, flush=True)
    _, _, _, P = _setup(spec, seed, "f64", cap)
    groups = O.mb_orbital_groups(oracle_basis(spec), 10 ** 9)
    perm, off = P.blocks()
    rp, ro = _flat(O.mb_orbital_groups(oracle_basis(spec), cap))
    np.testing.assert_array_equal(perm, rp)
    np.testing.assert_array_equal(off, ro)
    assert P.n_groups == len(groups) and P.n_blocks == len(ro) - 1
    assert P.largest == int(np.diff(ro).max()) and P.max_sweeps < 40


def _block_tol(Hf, idx, theta, r):
    B = Hf[idx][:, idx].toarray()
    lam = np.linalg.eigvalsh(B)
    fro = np.linalg.norm(B)
    tol = np.zeros(len(theta))
    for c, t in enumerate(theta):
        gaps = np.abs([O.clamped_shift(l - t) for l in lam])
        assert np.abs(lam - t).min() > 1e-6, "shift too close to a block eigenvalue"
        d = gaps.min()
        tol[c] = 1e-12 * (fro / d ** 2 + 1 / d) * np.linalg.norm(r[:, c])
    return tol


@pytest.mark.parametrize("name", ["mixed", "cut4", "w3_1sp", "w2_b"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ncol", [1, 5, 16])
def test_apply_matches_oracle(name, dtype, ncol):
    import torch
    spec, seed = SMALL[name]
    print("case apply", name, dtype, ncol, flush=True)
    _, _, H, P = _setup(spec, seed, dtype, 64)
    rp, col, val = oracle_csr(spec, seed)
    if dtype == "f32":
        val = np.asarray(val).astype(np.float32).astype(np.float64)
    D = len(rp) - 1
    rng = np.random.default_rng(ncol)
    R = rng.standard_normal((D, ncol))
    d = np.asarray(val)[np.asarray(rp)[:-1]]
    theta = rng.uniform(d.min() - 1.0, d.min() + 2.0, ncol)
    blocks = O.mb_orbital_groups(oracle_basis(spec), 64)
    Hf = O.full_from_half(rp, col, val, D)
    ref = O.block_precond_apply(rp, col, val, blocks, R, theta)
    Rd = torch.from_numpy(R).to("cuda:0")
    W = P.apply(Rd, theta).cpu().numpy()
    W2 = P.apply(Rd.clone(), theta, W=None)
    np.testing.assert_array_equal(W2.cpu().numpy(), W)                 # deterministic
    Rin = Rd.clone()
    P.apply(Rin, theta, W=Rin)                                          # in place
    np.testing.assert_array_equal(Rin.cpu().numpy(), W)
    for idx in blocks:
        tol = _block_tol(Hf, idx, theta, R[idx])
        err = np.linalg.norm(W[idx] - ref[idx], axis=0)
        assert np.all(err <= tol), (idx[:4], err, tol)


def test_blocks_of_one_state_are_exact():
    import torch
    spec, seed = SMALL["cut4"]
    print("case singleton blocks", flush=True)
    _, _, _, P = _setup(spec, seed, "f64", 1)
    rp, col, val = oracle_csr(spec, seed)
    d = np.asarray(val)[np.asarray(rp)[:-1]]
    R = np.random.default_rng(8).standard_normal((len(d), 3))
    # two gaps inside the guard (+-5e-3, moved to +-1e-2), one far from it
    theta = [d[11] + 5e-3, d[500] - 5e-3, d.min() - 0.25]
    W = P.apply(torch.from_numpy(R).to("cuda:0"), theta).cpu().numpy()
    den = np.array([[O.clamped_shift(x - t) for t in theta] for x in d])
    E = R / den
    assert W[11, 0] == R[11, 0] / -1e-2 and W[500, 1] == R[500, 1] / 1e-2
    # the library's diagonal is the oracle's up to rounding (its own
    # summation order): one division on each side plus that difference
    # through 1 / gap
    tol = 4 * EPS64 * np.abs(E) + 1e-13 * np.maximum(np.abs(d), 1)[:, None] * np.abs(R) / den ** 2
    assert np.all(np.abs(W - E) <= tol)


@pytest.mark.parametrize("name,dtype,cap", [("sp1_n2_N4", "f64", 64), ("ab_n3_3p3_cut4", "f64", 64),
                                            ("ab_n3_3p3_cut4", "f64", 16), ("ab_n3_3p3_cut4", "f32", 64)])
def test_lobpcg_with_block_preconditioner(name, dtype, cap):
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS[name]
    g = golden(name)
    print("case lobpcg block precond", name, dtype, cap, flush=True)
    ctx, _, H, P = _setup(w.spec, w.seed, dtype, cap)
    ev, info, vec = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=600, precond=P, want_vectors=True)
    assert info["status"] == 0, info
    if dtype == "f64":
        ref = np.asarray(g.get("evals_f64_lapack", g["evals_f64"]))[:w.nev]
        assert (np.abs(ev - ref) / np.maximum(np.abs(ref), 1)).max() <= 1e-10, (ev, ref)
        rp, col, val = oracle_csr(w.spec, w.seed)
        assert O.residual_audit(rp, col, val, ev, vec.cpu().numpy()).max() <= 1e-8
    else:
        ref = np.asarray(g["evals_f64"])[:w.nev]
        assert (np.abs(ev - ref) / np.maximum(np.abs(ref), 1)).max() <= 1e-6, (ev, ref)


def test_lobpcg_blocks_of_one_state_match_diagonal_run():
    """max_block = 1 applies the diagonal preconditioner's exact bits, so the
    whole solve (iterates, iterations, eigenvalues) is the diagonal run's."""
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["ab_n3_3p3_cut4"]
    print("case lobpcg singleton blocks", flush=True)
    ctx, _, H, P = _setup(w.spec, w.seed, "f64", 1)
    e1, i1, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=600, precond=P)
    e0, i0, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=600)
    assert i1["iters"] == i0["iters"]
    np.testing.assert_array_equal(e1, e0)


def test_full_size_sampled_blocks():
    """D = 198,912: blocks equal the oracle's grouping; 12 blocks (the
    largest and a seeded sample) against the oracle's rows of H; LOBPCG with
    the preconditioner reaches the stored eigenvalues."""
    import torch
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["ab_n3_3p3_cut6"]
    print("case full size", w.name, flush=True)
    ctx, _, H, P = _setup(w.spec, w.seed, "f32", 64)
    ob = oracle_basis(w.spec)
    blocks = O.mb_orbital_groups(ob, 64)
    perm, off = P.blocks()
    rp, ro = _flat(blocks)
    np.testing.assert_array_equal(perm, rp)
    np.testing.assert_array_equal(off, ro)
    rng = np.random.default_rng(12)
    big = max(range(len(blocks)), key=lambda k: len(blocks[k]))
    pick = [big] + list(rng.choice(len(blocks), 11, replace=False))
    ncol = 4
    R = rng.standard_normal((ob.D, ncol))
    theta = np.array([-77.0, -75.5, -10.0, 1.5])
    W = P.apply(torch.from_numpy(R).to("cuda:0"), theta).cpu().numpy()
    inter = O.Interaction(ob, oracle_tables(w.spec, w.seed))
    for k in pick:
        idx = np.asarray(blocks[k])
        rows = O.half_csr_rows(ob, inter, idx)
        where = {int(i): a for a, i in enumerate(idx)}
        s = len(idx)
        B = np.zeros((s, s))
        for i in idx:
            cols, vals = rows[int(i)]
            for j, v in zip(cols, vals):
                if int(j) in where:
                    v32 = float(np.float32(v))
                    B[where[int(i)], where[int(j)]] = B[where[int(j)], where[int(i)]] = v32
        lam, Q = np.linalg.eigh(B)
        fro = np.linalg.norm(B)
        for c, t in enumerate(theta):
            assert np.abs(lam - t).min() > 1e-6
            gap = np.array([O.clamped_shift(x - t) for x in lam])
            ref = Q @ ((Q.T @ R[idx, c]) / gap)
            d = np.abs(gap).min()
            tol = 1e-12 * (fro / d ** 2 + 1 / d) * np.linalg.norm(R[idx, c])
            assert np.linalg.norm(W[idx, c] - ref) <= tol, (k, c)
    ev, info, _ = cib.lobpcg(ctx, H, w.nev, block=w.block, max_iter=600, precond=P)
    assert info["status"] == 0, info
    ref = np.asarray(golden(w.name)["evals_f64"])[:w.nev]
    assert (np.abs(ev - ref) / np.maximum(np.abs(ref), 1)).max() <= 1e-6, (ev, ref)


def test_precond_rejects_bad_arguments():
    import torch
    from paper_2110_10765_amd import cib
    spec, seed = SMALL["mixed"]
    ctx, b, H, P = _setup(spec, seed, "f64", 8)
    for cap in (0, 65):
        with pytest.raises(cib.CibError):
            cib.Precond(ctx, b, H, cap)
    R = torch.zeros(H.dim, 17, dtype=torch.float64, device="cuda:0")
    with pytest.raises(cib.CibError):
        P.apply(R, np.zeros(17))
    b2 = cib.build_basis(ctx, SMALL["tiny"][0])
    H2 = cib.build_H(ctx, b2, oracle_tables(SMALL["tiny"][0], 3), "f64")
    with pytest.raises(cib.CibError):
        cib.Precond(ctx, b2, H, 8)                                     # H not built on b2
    with pytest.raises(cib.CibError):
        cib.lobpcg(ctx, H2, 2, block=2, precond=P)                     # made for another basis
