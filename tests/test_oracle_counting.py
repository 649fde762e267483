"""Pins of the oracle's state-counting test (CPU only): for each state, the
number of states of the list (itself included) that differ from it in at
most two particles (Sec. 2.1, Listing 2 as a description).

The oracle counts with popcounts of full bit strings.  It is pinned by:
* brute force over pairs with count_difference (Listing 1 restated on index
  tuples, itself pinned to popcount elsewhere);
* the closed form for the complete list of C(M, N) states: every state is
  connected to 1 + N (M - N) + C(N, 2) C(M - N, 2) states;
* a state set straddling the 64-orbital word boundary.
"""
import itertools
import math

import numpy as np
import pytest

import cigen
import oracle as O


def test_brute_force_count_difference():
    mbs = cigen.counting_states(300, n_particles=6, n_sp=128, tau=4.0, seed=3)
    c = O.count_connected(mbs, 128)
    ref = [sum(O.count_difference(list(a), list(b)) <= 4 for b in mbs) for a in mbs]
    assert np.array_equal(c, ref)
    assert c.sum() > 300        # the bias makes some states connected


@pytest.mark.parametrize("M,N", [(9, 3), (12, 4), (10, 1), (8, 8)])
def test_complete_set_closed_form(M, N):
    mbs = np.array(list(itertools.combinations(range(M), N)), dtype=np.uint16)
    c = O.count_connected(mbs, M)
    per = 1 + N * (M - N) + math.comb(N, 2) * math.comb(M - N, 2)
    assert np.all(c == per)


def test_word_boundary():
    # orbitals 60..69 straddle the first and second 64-bit word
    mbs = np.array(list(itertools.combinations(range(60, 70), 3)), dtype=np.uint16)
    c = O.count_connected(mbs, 128)
    assert np.all(c == 1 + 3 * 7 + 3 * math.comb(7, 2))
