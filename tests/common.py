"""Shared helpers for the test-suite: cached oracle results and GPU context."""
import functools
import json
import os

import numpy as np

import cigen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


@functools.lru_cache(maxsize=None)
def oracle_basis(spec):
    return O.Basis(spec)


@functools.lru_cache(maxsize=None)
def oracle_tables(spec, seed):
    return cigen.make_tables(spec, seed)


@functools.lru_cache(maxsize=None)
def oracle_csr(spec, seed):
    b = oracle_basis(spec)
    return O.half_csr(b, O.Interaction(b, oracle_tables(spec, seed)))


def xor_popcount_rows(words, rows, cols):
    """popcount(BIN_i xor BIN_j) for parallel index arrays (state-major words)."""
    x = words[rows] ^ words[cols]
    return np.bitwise_count(x).sum(axis=1)


_CTX = None


def gpu_ctx():
    """One library context per test process (device 0)."""
    global _CTX
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    from paper_2110_10765_amd import cib
    if _CTX is None:
        _CTX = cib.Context(0)
    return _CTX
