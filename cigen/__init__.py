"""Seeded synthetic inputs for the configuration-interaction hot path.

This module only *draws* inputs: the single-particle orbital list that fixes
the table layout, the one-body energies, the two-body matrix-element tables and
the request traces of the serving workload.  It holds none of the method's
arithmetic (no basis, no phases, no Hamiltonian), so both the CPU oracle and
the GPU library can consume what it produces without sharing any code.

Input law (the paper leaves the interaction unspecified; these are synthetic
stand-ins with the shapes of a shell-model calculation, Sec. 2 of the paper):

* Orbitals of one species: harmonic-oscillator shells n = 0..nmax; shell n has
  levels 2j = 1, 3, ..., 2n+1 and each level the states 2m = -2j..2j step 2.
  Orbital index = position in that (n, 2j, 2m) ascending order.
* One-body energies: eps_a = n_a + U(-0.1, 0.1), one array per species.
* Two-body tables, "M-blocked": pairs are grouped by 2M_pair = 2m_a + 2m_b in
  ascending order; inside a block pairs are in lexicographic (a, b) order.
  Same-species pairs have a < b; cross-species pairs are all (a in A, b in B).
  Each block is a full symmetric n_M x n_M matrix stored row-major, and the
  blocks are concatenated.  Entries are N(0, 1), drawn for the upper triangle
  (p <= q, row-major) and mirrored, so V_{pq} = V_{qp}.
* Draw order from numpy Generator(PCG64(seed)): eps of species A, eps of
  species B, V^AA blocks, V^BB blocks, V^AB blocks.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "BasisSpec", "Workload", "Tables", "orbitals", "same_pair_layout",
    "cross_pair_layout", "make_tables", "WORKLOADS", "request_trace",
    "random_spec_small",
]


@dataclasses.dataclass(frozen=True)
class BasisSpec:
    """Many-body basis definition.

    n_species   1 or 2
    nmax        highest oscillator shell per species
    n_particles particles per species
    two_M       twice the total angular-momentum projection
    cut         summed-shell-quanta truncation above the minimum; < 0: none
    """
    n_species: int
    nmax: tuple
    n_particles: tuple
    two_M: int = 0
    cut: int = -1

    @staticmethod
    def one(nmax: int, n: int, two_M: int = 0, cut: int = -1) -> "BasisSpec":
        return BasisSpec(1, (nmax, 0), (n, 0), two_M, cut)

    @staticmethod
    def two(nmax_a: int, n_a: int, nmax_b: int, n_b: int, two_M: int = 0,
            cut: int = -1) -> "BasisSpec":
        return BasisSpec(2, (nmax_a, nmax_b), (n_a, n_b), two_M, cut)


@dataclasses.dataclass
class Tables:
    """One-body energies and M-blocked two-body tables (float64, host)."""
    eps: List[np.ndarray]            # per species
    v_same: List[np.ndarray]         # per species, flat blocked layout
    v_ab: Optional[np.ndarray]       # flat blocked layout, None for 1 species


def orbitals(nmax: int) -> np.ndarray:
    """(n, 2j, 2m) rows in the canonical orbital order, int32 array [n_orb, 3]."""
    rows = []
    for n in range(nmax + 1):
        for twoj in range(1, 2 * n + 2, 2):
            for twom in range(-twoj, twoj + 1, 2):
                rows.append((n, twoj, twom))
    return np.asarray(rows, dtype=np.int32).reshape(-1, 3)


def _blocks(pairs_a: np.ndarray, pairs_b: np.ndarray, m2: np.ndarray):
    order = np.lexsort((pairs_b, pairs_a, m2))
    pa, pb, pm = pairs_a[order], pairs_b[order], m2[order]
    blocks = []
    if pm.size:
        cuts = np.flatnonzero(np.diff(pm)) + 1
        starts = np.concatenate(([0], cuts))
        ends = np.concatenate((cuts, [pm.size]))
        for s, e in zip(starts, ends):
            blocks.append((int(pm[s]), pa[s:e].copy(), pb[s:e].copy()))
    return blocks


def same_pair_layout(nmax: int):
    """Blocks of same-species pairs a < b: list of (2M_pair, a[], b[])."""
    o = orbitals(nmax)
    a, b = np.triu_indices(o.shape[0], k=1)
    return _blocks(a.astype(np.int32), b.astype(np.int32), o[a, 2] + o[b, 2])


def cross_pair_layout(nmax_a: int, nmax_b: int):
    """Blocks of cross-species pairs (a in A, b in B): list of (2M_pair, a[], b[])."""
    oa, ob = orbitals(nmax_a), orbitals(nmax_b)
    a, b = np.meshgrid(np.arange(oa.shape[0], dtype=np.int32),
                       np.arange(ob.shape[0], dtype=np.int32), indexing="ij")
    a, b = a.ravel(), b.ravel()
    return _blocks(a, b, oa[a, 2] + ob[b, 2])


def _draw_blocks(rng: np.random.Generator, blocks) -> np.ndarray:
    total = sum(len(pa) ** 2 for _, pa, _ in blocks)
    out = np.zeros(total, dtype=np.float64)
    base = 0
    for _, pa, _ in blocks:
        n = len(pa)
        z = rng.standard_normal(n * (n + 1) // 2)
        m = np.zeros((n, n))
        m[np.triu_indices(n)] = z
        m = m + m.T - np.diag(np.diag(m))
        out[base:base + n * n] = m.ravel()
        base += n * n
    return out


def make_tables(spec: BasisSpec, seed: int, v_scale: float = 1.0) -> Tables:
    """Draw eps and V for `spec` from PCG64(seed).  v_scale = 0 gives V = 0
    with the same eps draws (the random stream is consumed identically)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = spec.n_species
    eps = []
    for s in range(ns):
        o = orbitals(spec.nmax[s])
        eps.append(o[:, 0].astype(np.float64) + rng.uniform(-0.1, 0.1, o.shape[0]))
    v_same = [_draw_blocks(rng, same_pair_layout(spec.nmax[s])) * v_scale
              for s in range(ns)]
    v_ab = None
    if ns == 2:
        v_ab = _draw_blocks(rng, cross_pair_layout(spec.nmax[0], spec.nmax[1])) * v_scale
    return Tables(eps=eps, v_same=v_same, v_ab=v_ab)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    spec: BasisSpec
    seed: int
    nev: int
    block: int
    dtype: str          # "f64" or "f32": precision of the stored H and the SpMM


# The five synthetic workloads (shells, particles, truncation, interaction seed,
# eigenpairs wanted and LOBPCG block size).
WORKLOADS = {
    "sp1_n2_N4": Workload("sp1_n2_N4", BasisSpec.one(2, 4, 0, -1), 1, 5, 8, "f64"),
    "ab_n3_3p3_cut4": Workload("ab_n3_3p3_cut4", BasisSpec.two(3, 3, 3, 3, 0, 4), 2, 5, 8, "f64"),
    "ab_n5_4p4_cut4": Workload("ab_n5_4p4_cut4", BasisSpec.two(5, 4, 5, 4, 0, 4), 3, 5, 8, "f32"),
    "ab_n3_3p3_cut6": Workload("ab_n3_3p3_cut6", BasisSpec.two(3, 3, 3, 3, 0, 6), 4, 10, 16, "f32"),
}


def request_trace(n: int = 512, trace_seed: int = 5, rate: float = math.inf,
                  nev: int = 4, block: int = 8):
    """Serving stream: per request (id, arrival_s, spec, interaction seed).

    Each request draws nmax in {2,3,4} (both species), N_A and N_B in {2,3,4}
    and cut in {2,4} independently and uniformly; 2M = (N_A + N_B) mod 2 and
    the interaction seed is 1000 + id.  Arrivals are a Poisson process of the
    given rate (inf: all at t = 0).
    """
    rng = np.random.Generator(np.random.PCG64(trace_seed))
    nmax = rng.integers(2, 5, size=n)
    na = rng.integers(2, 5, size=n)
    nb = rng.integers(2, 5, size=n)
    cut = rng.choice(np.array([2, 4]), size=n)
    gaps = rng.exponential(1.0, size=n)
    if math.isinf(rate):
        arrival = np.zeros(n)
    else:
        arrival = np.cumsum(gaps) / rate
        arrival -= arrival[0]
    out = []
    for i in range(n):
        spec = BasisSpec.two(int(nmax[i]), int(na[i]), int(nmax[i]), int(nb[i]),
                             int((na[i] + nb[i]) % 2), int(cut[i]))
        out.append(dict(id=i, arrival_s=float(arrival[i]), spec=spec,
                        seed=1000 + i, nev=nev, block=block))
    return out


def counting_states(n: int, n_particles: int = 8, n_sp: int = 128, tau: float = 36.0,
                    seed: int = 0) -> np.ndarray:
    """Random many-body states for the state-counting test: n states, each
    n_particles distinct single-particle states out of n_sp, drawn without
    replacement with weights exp(-k / tau) (biased towards the lowest states;
    the Gumbel top-k draw).  tau = 36 at 8 particles out of 128 gives two
    random states a probability of about 6e-6 to differ in at most two
    particles, the median density of nonzeros the paper quotes for its test.
    Returns an (n, n_particles) uint16 array, each row ascending."""
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = -np.arange(n_sp) / tau + rng.gumbel(size=(n, n_sp))
    idx = np.argpartition(-keys, n_particles - 1, axis=1)[:, :n_particles]
    return np.sort(idx, axis=1).astype(np.uint16)


def random_spec_small(rng: np.random.Generator) -> BasisSpec:
    """A tiny random spec (for property tests): D stays in the hundreds."""
    if rng.random() < 0.3:
        nmax = int(rng.integers(1, 3))
        n = int(rng.integers(1, 4))
        return BasisSpec.one(nmax, n, int(n % 2), int(rng.choice([-1, 1, 2])))
    nmax = int(rng.integers(1, 3))
    na = int(rng.integers(1, 3))
    nb = int(rng.integers(1, 3))
    return BasisSpec.two(nmax, na, nmax, nb, int((na + nb) % 2),
                         int(rng.choice([-1, 1, 2])))
