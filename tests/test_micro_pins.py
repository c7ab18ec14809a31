"""Pins of the branch-divergence micro benchmark's oracle (CPU only)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import micro


def _py_round(v: int, k: int) -> int:
    """One mixing step written with Python integers (an independent path)."""
    m = (micro.M0 + 2 * k) % (1 << 64)
    return (((v ^ (v >> 29)) * m) + k + 1) % (1 << 64)


@pytest.mark.parametrize("k", [0, 1, 7, 31])
def test_closed_forms_from_zero(k):
    # from v = 0 one round gives k + 1; two rounds give (k + 1) M_k + k + 1,
    # since k + 1 < 2^29 has no bits above 29
    z = np.zeros(1, np.uint64)
    assert int(micro.mix_rounds(z, k, 1)[0]) == k + 1
    assert int(micro.mix_rounds(z, k, 2)[0]) == ((k + 1) * (micro.M0 + 2 * k) + k + 1) % (1 << 64)
    assert int(micro.mix_rounds(z, k, 0)[0]) == 0


def test_rounds_match_python_integers():
    rng = np.random.default_rng(3)
    vals = rng.integers(0, 2**63, 50, dtype=np.int64).astype(np.uint64)
    vals[:3] = [0, 2**64 - 1, 2**63]
    for k in (0, 5, 30):
        got = micro.mix_rounds(vals, k, 37)
        for v, g in zip(vals, got):
            w = int(v)
            for _ in range(37):
                w = _py_round(w, k)
            assert int(g) == w


def test_execute_touches_each_tuple_with_its_type():
    rng = np.random.default_rng(4)
    t = rng.integers(0, 9, 400).astype(np.int32)
    t[:5] = 99                                   # no such type: unchanged
    tup = rng.integers(-2**62, 2**62, 400, dtype=np.int64)
    out = micro.execute(t, tup, 9, 1)
    assert np.array_equal(out[:5], tup[:5])
    for i in range(5, 400, 37):
        w = int(tup[i]) % (1 << 64)
        for _ in range(100):
            w = _py_round(w, int(t[i]))
        assert int(out[i].view(np.uint64)) == w


def _splits(types, tbits, gbits):
    """Stable 1-bit splits, lowest of the top gbits bits first (pure Python)."""
    order = list(range(len(types)))
    for b in range(gbits):
        bit = tbits - gbits + b
        zeros = [i for i in order if not (types[i] >> bit) & 1]
        ones = [i for i in order if (types[i] >> bit) & 1]
        order = zeros + ones
    return order


@pytest.mark.parametrize("n_types,groups", [(16, 1), (16, 2), (16, 4), (16, 16), (5, 4), (32, 8)])
def test_grouped_order_is_the_stable_radix_partition(n_types, groups):
    rng = np.random.default_rng(n_types * 10 + groups)
    t = rng.integers(0, n_types, 300).astype(np.int32)
    got = micro.grouped_order(t, n_types, groups)
    tbits = int(n_types - 1).bit_length()
    gbits = int(groups - 1).bit_length()
    assert got.tolist() == _splits(t.tolist(), tbits, gbits)
    key = t[got] >> (tbits - gbits) if gbits else np.zeros(300, np.int64)
    assert np.all(np.diff(key) >= 0)             # grouped
    assert len(set(got.tolist())) == 300          # a permutation
