"""Oracle (test infrastructure only): the protocol around the server computation.

Client preparation (Alg. 6 ClientDataPrep, gamma = 1): cuckoo table -> CW
positions -> one slot vector per codeword bit j -> encode -> encrypt.
Server preparation (Alg. 6 ServerDataPrep): simple hashing -> CW positions,
kept as a [mu][b][h] table of positions (the plaintexts pt_s[i'][j] are the
bit planes of this table).
Server values (Alg. 4 labelled PSI, Alg. 5 PSI-Sum): val_s[i'] is the batch-encoded
plaintext whose slot k is the value of the server element at entry (i', k) of T_s.
Extraction (Alg. 3, Alg. 4 ExtractLabels and Alg. 5 ExtractPSISum): decrypt, read the
indicator or the labels, or sum the slots mod t.
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
    item_bits: int       # lambda, the element length
    mu: int              # server maximum bin load
    hash_seed: int = 0x5EED
    n_hash: int = 3
    max_evictions: int = 500
    pbh: bool = False    # permutation-based hashing (Sec. 3.3)

    @property
    def effective_bits(self) -> int:
        """lambda_bar: the length of the stored values.  Without PBH the element itself; with
        PBH lambda - log2(b) plus the bits that name the hash function."""
        if not self.pbh:
            return self.item_bits
        return self.item_bits - (self.n.bit_length() - 1) + (self.n_hash - 1).bit_length()

    @property
    def ell(self) -> int:
        return P.code_length(self.effective_bits, self.h)

    @property
    def pbh_bits(self):
        return self.item_bits if self.pbh else None


def client_prepare(cfg: Config, items):
    table, valid = hashing.cuckoo_table(items, cfg.n, cfg.hash_seed, cfg.n_hash, cfg.max_evictions,
                                        pbh_bits=cfg.pbh_bits)
    pos = cw.positions_table(table, valid, cfg.ell, cfg.h)          # [b][h]
    return table, valid, pos, cw.planes(pos, cfg.ell)               # planes [l][b]


def server_prepare(cfg: Config, items):
    table, valid, max_load = hashing.simple_table(items, cfg.n, cfg.mu, cfg.hash_seed, cfg.n_hash,
                                                  pbh_bits=cfg.pbh_bits)
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


def extract_sum(slots, t: int = P.T_PLAIN) -> int:
    """Alg. 5 ExtractPSISum: the sum of all slots mod t."""
    return int(np.asarray(slots, dtype=np.int64).sum() % t)


def server_values(cfg: Config, items, values):
    """val_s as a [mu][b] table: entry (i', k) = the value of the server element at (i', k)
    of T_s (Alg. 6 layout), 0 for dummies.  values[e] belongs to items[e]; values < t."""
    values = np.asarray(values, dtype=np.uint64)
    assert values.shape == np.asarray(items).shape and (values < P.T_PLAIN).all()
    _, valid, _, index = hashing.simple_table(items, cfg.n, cfg.mu, cfg.hash_seed, cfg.n_hash,
                                              pbh_bits=cfg.pbh_bits, with_index=True)
    out = np.zeros(valid.shape, dtype=np.uint32)
    sel = valid.astype(bool)
    out[sel] = values[index[sel]].astype(np.uint32)
    return out


def plaintext_labels(client_table, client_valid, server_table, server_valid, vals_table):
    """Alg. 4 in the clear: slot k = the value of the server element equal to the client's
    bin-k element (at most one, the sets have distinct elements), 0 if there is none."""
    hit = (server_table == client_table[None, :]) & server_valid.astype(bool) & \
        client_valid.astype(bool)[None, :]
    return (vals_table.astype(np.int64) * hit).sum(axis=0).astype(np.uint32)


def plaintext_sum(client_items, server_items, values, t: int = P.T_PLAIN) -> int:
    """Alg. 5 in the clear: the sum of the values of the common elements, mod t."""
    server_items = np.asarray(server_items, dtype=np.uint64)
    common = np.isin(server_items, np.asarray(client_items, dtype=np.uint64))
    return int(np.asarray(values, dtype=np.int64)[common].sum() % t)
