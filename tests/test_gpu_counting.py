"""GPU parity of the state-counting test (cib_count_states; Sec. 2.1,
Listing 2 as a description) against the oracle: per-state counts of the
states within two particle differences, bit-exact, for the three methods
(hybrid 64-bit prefilter + count_difference, count_difference only, 128-bit
popcount).  Small lists are compared in full; at n = 2^17 the three methods
must give the same counts and 64 sampled states are counted by the oracle
one by one."""
import numpy as np
import pytest

import cigen
import oracle as O
from tests.common import gpu_ctx

pytestmark = pytest.mark.gpu

# (particles, bias scale tau, n): from dense (tau = 4) to the paper's sparse
# regime (tau = 36), 2..20 particles, n not a multiple of 256
CASES = [(8, 36.0, 3000), (6, 4.0, 2500), (4, 8.0, 1000), (12, 12.0, 1500), (16, 20.0, 1000),
         (20, 30.0, 700), (2, 36.0, 900), (1, 10.0, 300)]


@pytest.mark.parametrize("N,tau,n", CASES)
@pytest.mark.parametrize("method", [0, 1, 2])
def test_counts_match_oracle(N, tau, n, method):
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    print("case", N, tau, n, method, flush=True)
    mbs = cigen.counting_states(n, n_particles=N, n_sp=128, tau=tau, seed=N)
    ref = O.count_connected(mbs, 128)
    total, c = cib.count_states(ctx, mbs, 128, method)
    assert np.array_equal(c, ref) and total == ref.sum()


@pytest.mark.parametrize("method", [0, 1])
def test_large_single_particle_space(method):
    """n_sp = 300 (five 64-bit words in the oracle): the tuple methods."""
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    mbs = cigen.counting_states(2000, n_particles=10, n_sp=300, tau=12.0, seed=5)
    ref = O.count_connected(mbs, 300)
    total, c = cib.count_states(ctx, mbs, 300, method)
    assert np.array_equal(c, ref) and total == ref.sum()


def test_two_column_slabs_ragged():
    """n = 8449: two slabs of 8192 columns, a ragged last row block."""
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    mbs = cigen.counting_states(8449, n_particles=8, n_sp=128, tau=6.0, seed=7)
    ref = O.count_connected(mbs, 128)
    for method in (0, 1, 2):
        total, c = cib.count_states(ctx, mbs, 128, method)
        assert np.array_equal(c, ref), method


def test_full_size_methods_agree_and_sampled_rows():
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    n = 1 << 17
    mbs = cigen.counting_states(n, n_particles=8, n_sp=128, tau=36.0, seed=8)
    res = [cib.count_states(ctx, mbs, 128, m) for m in (0, 1, 2)]
    assert res[0][0] == res[1][0] == res[2][0]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][1], res[2][1])
    assert np.all(res[0][1] >= 1)
    rows = np.random.default_rng(0).choice(n, 64, replace=False)
    assert np.array_equal(res[0][1][rows], O.count_connected(mbs, 128, rows=rows))


def test_rejects_bad_arguments():
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    mbs = cigen.counting_states(100, n_particles=4, n_sp=200, tau=10.0, seed=1)
    with pytest.raises(cib.CibError):
        cib.count_states(ctx, mbs, 200, 2)          # 128-bit strings need n_sp <= 128
    with pytest.raises(cib.CibError):
        cib.count_states(ctx, mbs, 200, 3)
    with pytest.raises(cib.CibError):
        cib.count_states(ctx, np.zeros((10, 21), dtype=np.uint16), 200, 0)
