"""Pins of the oracle's basis enumeration (CPU only).

The oracle lists Slater determinants by brute force over particle subsets.  It
is pinned here by (a) generating-function coefficients, integer polynomial
arithmetic that never lists a state, (b) the binomial identity summed over all
2M, and (c) the conservation laws every listed state must obey.
"""
import itertools
import math

import numpy as np
import pytest

import cigen
import oracle as O


SPECS = [
    cigen.BasisSpec.one(2, 4, 0, -1),          # 1 species, 20 orbitals, N = 4
    cigen.BasisSpec.two(3, 3, 3, 3, 0, 4),     # 3 + 3, cut 4
    cigen.BasisSpec.two(1, 2, 2, 1, 1, -1),    # unequal shells
    cigen.BasisSpec.one(1, 3, 1, 1),
    cigen.BasisSpec.two(2, 2, 2, 2, 0, 2),
]


@pytest.mark.parametrize("spec", SPECS, ids=str)
def test_dimension_equals_generating_function(spec):
    assert O.Basis(spec).D == O.dim_generating_function(spec)


def test_dimensions_of_the_workloads():
    # D of every workload from the generating function alone (no enumeration)
    want = {"sp1_n2_N4": 849, "ab_n3_3p3_cut4": 20004, "ab_n3_3p3_cut6": 198912,
            "ab_n5_4p4_cut4": 173624}
    for name, d in want.items():
        assert O.dim_generating_function(cigen.WORKLOADS[name].spec) == d, name


@pytest.mark.parametrize("nmax,N", [(1, 3), (2, 2), (2, 4)])
def test_binomial_identity(nmax, N):
    """Summed over every reachable 2M, one species without a cut holds all
    C(n_orb, N) subsets."""
    n_orb = len(O.orbital_list(nmax))
    tot = 0
    for twoM in range(-60, 61):
        if (twoM - N) % 2:
            continue
        tot += O.Basis(cigen.BasisSpec.one(nmax, N, twoM, -1)).D
    assert tot == math.comb(n_orb, N)


def test_orbital_counts():
    # shell n holds (n+1)(n+2) states; 20 / 40 / 70 / 112 orbitals up to n = 2..5
    for nmax, want in [(2, 20), (3, 40), (4, 70), (5, 112)]:
        orbs = O.orbital_list(nmax)
        assert len(orbs) == want
        for n in range(nmax + 1):
            assert sum(1 for o in orbs if o[0] == n) == (n + 1) * (n + 2)
    # and the input generator lists the same orbitals in the same order
    for nmax in range(6):
        assert [tuple(r) for r in cigen.orbitals(nmax).tolist()] == O.orbital_list(nmax)


def test_qmin():
    # shells hold 2, 6, 12, ...: 3 particles -> 2 at n=0, 1 at n=1
    assert O.q_min(1, 3) == 0 and O.q_min(2, 3) == 0
    assert O.q_min(3, 3) == 1 and O.q_min(4, 5) == 2
    assert O.q_min(8, 3) == 6 and O.q_min(9, 3) == 8


@pytest.mark.parametrize("spec", SPECS, ids=str)
def test_conservation_and_order(spec):
    b = O.Basis(spec)
    nA = b.n_orb[0]
    qmx = O.q_max(spec)
    keys = []
    for a, bb in zip(b.A, b.B):
        assert O.popcount(a) == spec.n_particles[0]
        if spec.n_species == 2:
            assert O.popcount(bb) == spec.n_particles[1]
        else:
            assert bb == 0
        m = sum(b.orbs[0][k][2] for k in range(nA) if (a >> k) & 1)
        m += sum(b.orbs[1][k][2] for k in range(b.n_orb[1]) if (bb >> k) & 1)
        assert m == spec.two_M
        q = sum(b.orbs[0][k][0] for k in range(nA) if (a >> k) & 1)
        qb = sum(b.orbs[1][k][0] for k in range(b.n_orb[1]) if (bb >> k) & 1)
        if qmx is not None:
            assert q + qb <= qmx
        keys.append((a, qb, bb))
    assert keys == sorted(keys)
    assert len(set(b.glob)) == b.D


def test_nested_prefix_property():
    """Within A-blocks of equal 2M_A the B-lists, ordered by (Q_B, B), are
    prefixes of one another (the canonical order makes this hold)."""
    b = O.Basis(cigen.WORKLOADS["ab_n3_3p3_cut4"].spec)
    lists = {}
    for a, bb in zip(b.A, b.B):
        lists.setdefault(a, []).append(bb)
    by_m = {}
    for a, lst in lists.items():
        ma = sum(b.orbs[0][k][2] for k in range(b.n_orb[0]) if (a >> k) & 1)
        by_m.setdefault(ma, []).append(lst)
    for lsts in by_m.values():
        longest = max(lsts, key=len)
        for l in lsts:
            assert longest[:len(l)] == l
