"""cib_count_states_noalloc (the state-counting test with its scratch in a
static device array, for callers that cannot allocate) against
cib_count_states on the same inputs: per-state counts and totals bit for
bit, on two calls in a row, the second with a smaller input (the array keeps
the first call's values), with and without a caller counts array; and the
size limit is refused with CIB_E_INVALID."""
import numpy as np
import pytest

import cigen
from tests.common import gpu_ctx

pytestmark = pytest.mark.gpu


def _pair(ctx, mbs, method, want_counts):
    from paper_2110_10765_amd import cib
    ref = cib.count_states(ctx, mbs, 128, method, want_counts=want_counts)
    got = cib.count_states(ctx, mbs, 128, method, want_counts=want_counts, noalloc=True)
    return ref, got


@pytest.mark.parametrize("method", [0, 1, 2])
def test_noalloc_matches_allocating_entry_point(method):
    ctx = gpu_ctx()
    # a large list (two column slabs and more, ragged) and then a smaller one
    for n, N, tau, seed in ((20011, 8, 12.0, 3), (2999, 6, 4.0, 4)):
        print("noalloc case n=%d N=%d method=%d" % (n, N, method), flush=True)
        mbs = cigen.counting_states(n, n_particles=N, n_sp=128, tau=tau, seed=seed)
        (t_ref, c_ref), (t_got, c_got) = _pair(ctx, mbs, method, True)
        assert t_got == t_ref
        assert np.array_equal(c_got, c_ref)
        (t_ref2, _), (t_got2, none) = _pair(ctx, mbs, method, False)
        assert none is None and t_got2 == t_ref2 == t_ref


def test_noalloc_full_static_size_then_small():
    ctx = gpu_ctx()
    n_max = 1 << 17
    for n in (n_max, 513):
        print("noalloc size n=%d" % n, flush=True)
        mbs = cigen.counting_states(n, n_particles=8, n_sp=128, tau=36.0, seed=11)
        (t_ref, c_ref), (t_got, c_got) = _pair(ctx, mbs, 0, True)
        assert t_got == t_ref and np.array_equal(c_got, c_ref)


def test_noalloc_refuses_beyond_static_size():
    from paper_2110_10765_amd import cib
    ctx = gpu_ctx()
    mbs = cigen.counting_states((1 << 17) + 1, n_particles=4, n_sp=128, tau=36.0, seed=2)
    with pytest.raises(cib.CibError) as e:
        cib.count_states(ctx, mbs, 128, 0, noalloc=True)
    assert e.value.code == -1 and "131072" in str(e.value)
