"""Oracle (test infrastructure only): the protocol around the server computation.

Client preparation (Alg. 6 ClientDataPrep, gamma = 1): cuckoo table -> CW
positions -> one slot vector per codeword bit j -> encode -> encrypt.
Server preparation (Alg. 6 ServerDataPrep): simple hashing -> CW positions,
kept as a [mu][b][h] table of positions (the plaintexts pt_s[i'][j] are the
bit planes of this table).
Extraction (Alg. 3 and Alg. 5 ExtractPSISum): decrypt, read the indicator or
sum the slots mod t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cw, hashing
from . import params as P
from .core import Context


@dataclass
class Config:
    n: int               # ring degree N (= number of bins b)
    L: int               # ciphertext primes
    h: int               # Hamming weight
    item_bits: int       # lambda_bar (no PBH: the full element length)
    mu: int              # server maximum bin load
    hash_seed: int = 0x5EED
    n_hash: int = 3
    max_evictions: int = 500

    @property
    def ell(self) -> int:
        return P.code_length(self.item_bits, self.h)


def client_prepare(cfg: Config, items):
    table, valid = hashing.cuckoo_table(items, cfg.n, cfg.hash_seed, cfg.n_hash, cfg.max_evictions)
    pos = cw.positions_table(table, valid, cfg.ell, cfg.h)          # [b][h]
    return table, valid, pos, cw.planes(pos, cfg.ell)               # planes [l][b]


def server_prepare(cfg: Config, items):
    table, valid, max_load = hashing.simple_table(items, cfg.n, cfg.mu, cfg.hash_seed, cfg.n_hash)
    pos = cw.positions_table(table, valid, cfg.ell, cfg.h)          # [mu][b][h]
    return table, valid, pos, max_load


def encrypt_planes(ctx: Context, sk, planes, a, e):
    """a: [l][L][N] uniform residues, e: [l][N] errors -> cts [l][2][L][N]."""
    return ctx.encrypt_many(sk, ctx.encode_many(planes), a, e)


def plaintext_membership(client_table, client_valid, server_table, server_valid):
    """Indicator [b]: 1 iff the client's bin-k element occurs in the server's bin k."""
    b = client_table.shape[0]
    out = np.zeros(b, dtype=np.uint32)
    for k in range(b):
        if client_valid[k]:
            col = server_table[:, k][server_valid[:, k].astype(bool)]
            out[k] = 1 if (col == client_table[k]).any() else 0
    return out


def extract_cardinality(slots, t: int = P.T_PLAIN) -> int:
    return int(np.asarray(slots, dtype=np.int64).sum() % t)
