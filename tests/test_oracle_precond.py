"""Pins of the oracle's block-diagonal preconditioner over many-body basis
orbitals (Sec. 2: states sharing the (n, l, j) values of their particles form
a group; the groups give LOBPCG a block-diagonal preconditioner).

The grouping is checked against level occupations counted a second way
(popcount of per-level orbital masks) and against what the grouping implies
(a partition; equal summed shell quanta inside a group).  The application is
checked against a linear solve (LU, not the eigendecomposition the oracle
uses) with one block over the whole space, against the diagonal
preconditioner with blocks of one state, and for block locality."""
import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import oracle_tables

SPECS = [
    cigen.BasisSpec.two(1, 1, 1, 1, 0, -1),
    cigen.BasisSpec.one(2, 4, 0, -1),
    cigen.BasisSpec.two(2, 2, 2, 3, 1, 2),
    cigen.WORKLOADS["ab_n3_3p3_cut4"].spec,
]


def _masks(nmax):
    orbs = O.orbital_list(nmax)
    levels = sorted({(n, j) for n, j, _ in orbs})
    return [sum(1 << k for k, (n, j, _) in enumerate(orbs) if (n, j) == lv) for lv in levels]


def _key(b, i):
    ka = tuple(O.popcount(b.A[i] & m) for m in _masks(b.spec.nmax[0]))
    kb = tuple(O.popcount(b.B[i] & m) for m in _masks(b.spec.nmax[1])) if b.spec.n_species == 2 else ()
    return ka, kb


@pytest.mark.parametrize("si", range(len(SPECS)))
def test_groups_partition_by_level_occupation(si):
    b = O.Basis(SPECS[si])
    groups = O.mb_orbital_groups(b, 10 ** 9)
    flat = sorted(i for g in groups for i in g)
    assert flat == list(range(b.D))
    keys = [_key(b, g[0]) for g in groups]
    assert len(set(keys)) == len(groups)                   # distinct groups differ
    nq = [n for n, _, _ in O.orbital_list(b.spec.nmax[0])]
    nqb = [n for n, _, _ in O.orbital_list(b.spec.nmax[1])] if b.spec.n_species == 2 else []
    for g, k in zip(groups, keys):
        assert g == sorted(g)
        assert all(_key(b, i) == k for i in g)            # one key per group
        q = {sum(nq[t] for t in range(len(nq)) if b.A[i] >> t & 1)
             + sum(nqb[t] for t in range(len(nqb)) if b.B[i] >> t & 1) for i in g}
        assert len(q) == 1                                 # same summed shell quanta
    assert [g[0] for g in groups] == sorted(g[0] for g in groups)


@pytest.mark.parametrize("cap", [1, 3, 7, 64])
def test_groups_cut_into_runs(cap):
    b = O.Basis(SPECS[2])
    whole = O.mb_orbital_groups(b, 10 ** 9)
    runs = O.mb_orbital_groups(b, cap)
    assert all(1 <= len(r) <= cap for r in runs)
    rebuilt = []
    for g in whole:
        n = -(-len(g) // cap)
        part, runs = runs[:n], runs[n:]
        assert sum(part, []) == g and all(len(p) == cap for p in part[:-1])
        rebuilt.append(g)
    assert not runs and rebuilt == whole


def _half(spec, seed):
    b = O.Basis(spec)
    rp, col, val = O.half_csr(b, O.Interaction(b, oracle_tables(spec, seed)))
    return b, rp, col, val


def test_one_block_is_a_shifted_solve():
    b, rp, col, val = _half(SPECS[0], 3)
    H = O.full_from_half(rp, col, val, b.D).toarray()
    lam = np.linalg.eigvalsh(H)
    theta = [lam[0] - 0.5, 0.5 * (lam[0] + lam[1]), lam[-1] + 1.0]
    assert min(abs(l - t) for l in lam for t in theta) > 1e-2
    R = np.random.default_rng(1).standard_normal((b.D, 3))
    W = O.block_precond_apply(rp, col, val, [list(range(b.D))], R, theta)
    for c, t in enumerate(theta):
        ref = np.linalg.solve(H - t * np.eye(b.D), R[:, c])
        np.testing.assert_allclose(W[:, c], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_blocks_of_one_state_are_the_diagonal_preconditioner():
    b, rp, col, val = _half(SPECS[2], 5)
    d = np.asarray(val)[np.asarray(rp)[:-1]]                 # each row's first entry is its diagonal
    H = O.full_from_half(rp, col, val, b.D)
    np.testing.assert_array_equal(d, H.diagonal())
    R = np.random.default_rng(2).standard_normal((b.D, 2))
    theta = [d[7], d.min() - 3.0]                            # a zero gap, clamped to 1e-2
    W = O.block_precond_apply(rp, col, val, O.mb_orbital_groups(b, 1), R, theta)
    den = np.array([[O.clamped_shift(x - t) for t in theta] for x in d])
    np.testing.assert_allclose(W, R / den, rtol=1e-14)
    assert W[7, 0] == pytest.approx(R[7, 0] / 1e-2, rel=1e-14)


def test_blocks_act_independently():
    b, rp, col, val = _half(SPECS[3], 1)
    blocks = O.mb_orbital_groups(b, 16)
    R = np.random.default_rng(4).standard_normal((b.D, 2))
    theta = [-3.0, 0.7]
    W = O.block_precond_apply(rp, col, val, blocks, R, theta)
    k = max(range(len(blocks)), key=lambda j: len(blocks[j]))
    R2 = R.copy()
    R2[blocks[k]] += 1.0
    W2 = O.block_precond_apply(rp, col, val, blocks, R2, theta)
    changed = np.flatnonzero(np.any(W2 != W, axis=1))
    assert set(changed) <= set(blocks[k]) and len(changed) > 0
    # each block solves its own shifted system where no gap is clamped
    H = O.full_from_half(rp, col, val, b.D)
    idx = np.asarray(blocks[k])
    Bk = H[idx][:, idx].toarray()
    if np.abs(np.linalg.eigvalsh(Bk) - theta[0]).min() > 1e-2:
        np.testing.assert_allclose((Bk - theta[0] * np.eye(len(idx))) @ W[idx, 0], R[idx, 0], atol=1e-9)
