"""Pins of the oracle's observables (CPU only): a[k, v] = x_v^T O_k x_v, the
step after the eigensolve (Fig. 1 steps 16-20).

The oracle forms each operator as its half-stored matrix from the operator
image.  It is pinned by:
* the number operator of one species (eps = 1 on that species, everything
  else 0): a = N_s |x|^2, a closed form;
* the quadratic form with the dense operator built ket by ket from operator
  strings (dense_H), a path that shares nothing with the half-stored matrix:
  a dropped triangle, a doubled diagonal or a transposed operand fails it;
* eigenvectors of the dense H: a = the eigenvalue for unit vectors;
* linearity in the tables.
"""
import numpy as np
import pytest

import cigen
import oracle as O

SPECS = {
    "one_species": cigen.WORKLOADS["sp1_n2_N4"].spec,
    "two_species": cigen.BasisSpec.two(1, 3, 2, 2, 1, 4),
}


def _number_tables(spec, species):
    t = cigen.make_tables(spec, 1, v_scale=0.0)
    eps = [np.zeros_like(e) for e in t.eps]
    eps[species][:] = 1.0
    return cigen.Tables(eps=eps, v_same=[np.zeros_like(v) for v in t.v_same],
                        v_ab=None if t.v_ab is None else np.zeros_like(t.v_ab))


def _x(D, n, seed=0):
    return np.random.default_rng(seed).standard_normal((D, n))


@pytest.mark.parametrize("name", sorted(SPECS))
def test_number_operator_closed_form(name):
    spec = SPECS[name]
    b = O.Basis(spec)
    X = _x(b.D, 3)
    for s in range(spec.n_species):
        a = O.observables(b, [_number_tables(spec, s)], X)[0]
        np.testing.assert_allclose(a, spec.n_particles[s] * np.sum(X * X, axis=0), rtol=1e-13)


@pytest.mark.parametrize("name", sorted(SPECS))
def test_quadratic_form_of_dense_operator(name):
    spec = SPECS[name]
    b = O.Basis(spec)
    tabs = [cigen.make_tables(spec, seed) for seed in (3, 4)]
    X = _x(b.D, 4, seed=1)
    a = O.observables(b, tabs, X)
    for k, t in enumerate(tabs):
        Dm = O.dense_H(b, O.Interaction(b, t))
        ref = np.einsum("iv,ij,jv->v", X, Dm, X)
        bound = np.einsum("iv,ij,jv->v", np.abs(X), np.abs(Dm), np.abs(X))
        assert np.all(np.abs(a[k] - ref) <= 1e-12 * bound)


def test_eigenvectors_give_eigenvalues():
    spec = SPECS["two_species"]
    b = O.Basis(spec)
    t = cigen.make_tables(spec, 5)
    w, V = np.linalg.eigh(O.dense_H(b, O.Interaction(b, t)))
    a = O.observables(b, [t], V[:, :4])[0]
    np.testing.assert_allclose(a, w[:4], rtol=0, atol=1e-10 * max(1.0, np.abs(w).max()))


def test_linear_in_the_tables():
    spec = SPECS["two_species"]
    b = O.Basis(spec)
    t1, t2 = cigen.make_tables(spec, 6), cigen.make_tables(spec, 7)
    tsum = cigen.Tables(eps=[x + y for x, y in zip(t1.eps, t2.eps)],
                        v_same=[x + y for x, y in zip(t1.v_same, t2.v_same)], v_ab=t1.v_ab + t2.v_ab)
    X = _x(b.D, 2, seed=2)
    a = O.observables(b, [t1, t2, tsum], X)
    np.testing.assert_allclose(a[2], a[0] + a[1], rtol=1e-12, atol=1e-12 * np.abs(a).max())
