"""Oracle of the branch-divergence micro benchmark -- TEST INFRASTRUCTURE.

Section 6.2's micro benchmark: each transaction reads one tuple, computes on
it according to its type (one case of a switch per type) and writes the
result back; transactions are independent.  The paper's computation is
100 x calls of a transcendental function per transaction; this benchmark's
is 100 x rounds of an exact integer mixing step per transaction, with
constants of the type's own:

    v <- (v xor (v >> 29)) * M_k + (k + 1)  (mod 2^64),
    M_k = 0x9E3779B97F4A7C15 + 2 k.

Grouping (Appendix D): the transaction order is radix-partitioned on the type
id so that lanes of one wave run one case; with p groups the partition uses
the top log2 p bits of the type id and keeps the input order within a group.
"""
from __future__ import annotations

import numpy as np

M0 = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def mix_rounds(v: np.ndarray, k: int, rounds: int) -> np.ndarray:
    """``rounds`` mixing steps of type k on uint64 values (numpy wraps mod 2^64)."""
    v = v.astype(np.uint64, copy=True)
    m = np.uint64((M0 + 2 * k) & MASK)
    add = np.uint64(k + 1)
    s = np.uint64(29)
    with np.errstate(over="ignore"):
        for _ in range(rounds):
            v = (v ^ (v >> s)) * m + add
    return v


def execute(type_arr: np.ndarray, tuples: np.ndarray, n_types: int, x: int) -> np.ndarray:
    """Final tuples after every transaction ran once (order is irrelevant:
    transaction i touches tuple i only); types outside [0, n_types) leave
    their tuple unchanged."""
    out = tuples.astype(np.int64, copy=True)
    for k in range(n_types):
        sel = np.flatnonzero(type_arr == k)
        if sel.size:
            out[sel] = mix_rounds(tuples[sel].view(np.uint64), k, 100 * x).view(np.int64)
    return out


def grouped_order(type_arr: np.ndarray, n_types: int, groups: int) -> np.ndarray:
    """Transaction indices grouped on the top log2(groups) bits of the type
    id, input order kept within a group."""
    tbits = max(int(n_types - 1).bit_length(), 0)
    gbits = int(groups - 1).bit_length()
    key = type_arr.astype(np.int64) >> (tbits - gbits) if gbits else np.zeros_like(type_arr, np.int64)
    return np.argsort(key, kind="stable").astype(np.int32)
