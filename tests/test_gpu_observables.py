"""GPU parity of the observables a[k, v] = x_v^T O_k x_v (cib_observables,
Fig. 1 steps 16-20) against the oracle.

Small bases are compared in full with the oracle's quadratic forms of its
own half-stored operators; at the D = 198,912 size the number operator of a
species (eps = 1 on it, everything else 0) must give N_s |x_v|^2, which holds
at any size.

Bar (Higham's bound): |a - a_ref| <= gamma |x|^T |O| |x| with gamma for the
row length k = 2 (max stored row length) + 2 in the operator's dtype plus D
float64 terms of the final sums.  The float32 reference uses the oracle's
float64 operator rounded to float32 and the same float32 X, so the bound
covers only the arithmetic.
"""
import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import EPS32, EPS64, gpu_ctx

pytestmark = pytest.mark.gpu

SPECS = {
    "one_species": cigen.WORKLOADS["sp1_n2_N4"].spec,
    "two_species": cigen.BasisSpec.two(1, 3, 2, 2, 1, 4),
    # configurations over three 64-bit words (168 orbitals)
    "three_words": cigen.BasisSpec.one(6, 2, 0, -1),
}


def _gamma(k, u):
    return k * u / (1 - k * u)


def _number_tables(spec, species):
    t = cigen.make_tables(spec, 1, v_scale=0.0)
    eps = [np.zeros_like(e) for e in t.eps]
    eps[species][:] = 1.0
    return cigen.Tables(eps=eps, v_same=[np.zeros_like(v) for v in t.v_same],
                        v_ab=None if t.v_ab is None else np.zeros_like(t.v_ab))


@pytest.mark.parametrize("name", sorted(SPECS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nvec", [5, 8, 16])
def test_observables_match_oracle(name, dtype, nvec):
    import torch
    from paper_2110_10765_amd import cib
    spec = SPECS[name]
    ctx = gpu_ctx()
    print("case", name, dtype, nvec, flush=True)
    tabs = [cigen.make_tables(spec, 1), cigen.make_tables(spec, 9), _number_tables(spec, 0)]
    ob = O.Basis(spec)
    npt = np.float64 if dtype == "f64" else np.float32
    X = np.random.default_rng(nvec).standard_normal((ob.D, nvec)).astype(npt)
    basis = cib.build_basis(ctx, spec)
    assert basis.dim == ob.D
    Xd = torch.from_numpy(X).to("cuda:0")
    a = cib.observables(ctx, basis, tabs, Xd)
    torch.cuda.synchronize()
    Xf = X.astype(np.float64)
    u = EPS64 if dtype == "f64" else EPS32
    for k, t in enumerate(tabs):
        rp, col, val = O.half_csr(ob, O.Interaction(ob, t))
        Hs = O.full_from_half(rp, col, val.astype(npt).astype(np.float64), ob.D)
        ref = np.sum(Xf * (Hs @ Xf), axis=0)
        bound = np.sum(np.abs(Xf) * (abs(Hs) @ np.abs(Xf)), axis=0)
        kmax = 2 * int(np.diff(rp).max()) + 2
        tol = (_gamma(kmax, u) + _gamma(ob.D + 8, EPS64)) * bound
        assert np.all(np.abs(a[k] - ref) <= tol), (k, a[k], ref, tol)


def test_number_operator_full_size():
    """D = 198,912, float32 operator, 16 vectors: a = N_s |x|^2 for each species.
    The operator row is N_s on the diagonal and stored zeros elsewhere, so
    (O x)_i = fl(N_s x_i), one float32 rounding, and the float64 sum adds
    far less: |a - N_s |x|^2| <= 2^-24 N_s |x|^2 (with margin for the sum)."""
    import torch
    from paper_2110_10765_amd import cib
    w = cigen.WORKLOADS["ab_n3_3p3_cut6"]
    ctx = gpu_ctx()
    print("case number operator", w.name, flush=True)
    basis = cib.build_basis(ctx, w.spec)
    g = torch.Generator(device="cpu").manual_seed(11)
    X = torch.randn(basis.dim, 16, generator=g, dtype=torch.float32)
    a = cib.observables(ctx, basis, [_number_tables(w.spec, 0), _number_tables(w.spec, 1)], X.to("cuda:0"))
    sq = (X.double() ** 2).sum(dim=0).numpy()
    for s in range(2):
        np.testing.assert_allclose(a[s], w.spec.n_particles[s] * sq, rtol=2 * EPS32)


def test_observables_rejects_bad_arguments():
    import torch
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    spec = SPECS["one_species"]
    basis = cib.build_basis(ctx, spec)
    X = torch.zeros(basis.dim, 65, dtype=torch.float64, device="cuda:0")
    with pytest.raises(cib.CibError):
        cib.observables(ctx, basis, [cigen.make_tables(spec, 1)], X)
    with pytest.raises(cib.CibError):
        cib.observables(ctx, basis, [], X[:, :4])
