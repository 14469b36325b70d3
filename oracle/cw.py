"""Oracle (test infrastructure only): constant-weight codes (Sec. 3.2, Sec. 4.1).

CW-Encode with the perfect mapping: the paper defers to an algorithm of its
reference [Mahdavi, Kerschbaum 2022] that it does not reproduce.  The reading
used here is the combinatorial number system (colex order): the value v in
[0, C(l, h)) maps to the positions c_h > ... > c_1 >= 0 with
    v = C(c_h, h) + C(c_{h-1}, h-1) + ... + C(c_1, 1),
found greedily: c_r = max{ c : C(c, r) <= v_r }.  The codeword has bit j set
iff j is one of the positions.  A dummy encodes to the all-zero word (Sec. 4.1).
"""
from __future__ import annotations

import math

import numpy as np

NO_POS = 0xFFFF


def encode_one(v: int, ell: int, h: int) -> list[int]:
    """Positions (descending) of the weight-h codeword of value v."""
    if not 0 <= v < math.comb(ell, h):
        raise ValueError("value out of range for CW(l, h)")
    pos = []
    for r in range(h, 0, -1):
        c = r - 1
        while math.comb(c + 1, r) <= v:
            c += 1
        pos.append(c)
        v -= math.comb(c, r)
    return pos


def encode_many(values: np.ndarray, ell: int, h: int) -> np.ndarray:
    """Vectorised encode_one: uint16 positions [len(values)][h], descending."""
    values = np.asarray(values, dtype=np.int64).copy()
    if values.size and (values.min() < 0 or int(values.max()) >= math.comb(ell, h)):
        raise ValueError("value out of range for CW(l, h)")
    out = np.empty((values.shape[0], h), dtype=np.uint16)
    for col, r in enumerate(range(h, 0, -1)):
        table = np.array([math.comb(c, r) for c in range(ell)], dtype=np.int64)  # nondecreasing in c
        c = np.searchsorted(table, values, side="right") - 1                    # max c: C(c,r) <= v
        out[:, col] = c
        values -= table[c]
    return out


def positions_table(table: np.ndarray, valid: np.ndarray, ell: int, h: int) -> np.ndarray:
    """Codeword positions of a binned table: [..., h] uint16 with NO_POS for dummies."""
    flat_t = table.reshape(-1)
    flat_v = valid.reshape(-1).astype(bool)
    out = np.full((flat_t.shape[0], h), NO_POS, dtype=np.uint16)
    if flat_v.any():
        out[flat_v] = encode_many(flat_t[flat_v], ell, h)
    return out.reshape(table.shape + (h,))


def planes(positions: np.ndarray, ell: int) -> np.ndarray:
    """Bit planes [l][b] of a client table's positions [b][h]: plane j, slot k = [j in cw(T[k])]."""
    b, h = positions.shape
    out = np.zeros((ell, b), dtype=np.uint32)
    for r in range(h):
        p = positions[:, r]
        ok = p != NO_POS
        out[p[ok].astype(np.int64), np.nonzero(ok)[0]] = 1
    return out
