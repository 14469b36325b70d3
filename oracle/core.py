"""Oracle (test infrastructure only): ctypes binding of the C core.

Arrays are numpy, C-contiguous, in the layouts documented in csrc/oracle.h.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import params as P

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        L = C.CDLL(path)
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        u64, i = C.c_uint64, C.c_int
        sig = {
            "or_mulmod": (u64, [u64, u64, u64]),
            "or_poly_mul_schoolbook": (None, [u64p, u64p, u64p, i, u64]),
            "or_poly_eval_point": (u64, [u64p, i, u64, u64]),
            "or_eval_fwd": (None, [u64p, i, u64, u64]),
            "or_eval_inv": (None, [u64p, i, u64, u64]),
            "or_poly_mul_eval": (None, [u64p, u64p, u64p, i, u64, u64]),
            "or_ctx_create": (vp, [i, i, u64p, u64p, u64, u64]),
            "or_ctx_destroy": (None, [vp]),
            "or_ctx_delta": (None, [vp, u64p, C.POINTER(C.c_int), C.POINTER(C.c_uint64)]),
            "or_encode": (None, [vp, u32p, u32p]),
            "or_decode": (None, [vp, u32p, u32p]),
            "or_encrypt": (None, [vp, i8p, u32p, u64p, i32p, u64p]),
            "or_decrypt_poly": (None, [vp, i8p, u64p, u32p]),
            "or_encode_many": (None, [vp, u32p, i, u32p]),
            "or_encrypt_many": (None, [vp, i8p, u32p, u64p, i32p, i, u64p]),
            "or_noise_budget": (i, [vp, i8p, u64p]),
            "or_keygen_relin": (None, [vp, i8p, u64p, i32p, u64p]),
            "or_mul_plain": (None, [vp, u64p, u32p, u64p]),
            "or_add_plain_const": (None, [vp, u64p, C.c_uint32]),
            "or_add_plain": (None, [vp, u64p, u32p]),
            "or_mul_const": (None, [vp, u64p, C.c_uint32]),
            "or_multiply": (None, [vp, u64p, u64p, u64p]),
            "or_relin": (None, [vp, u64p, u64p, u64p]),
            "or_select_sum": (None, [vp, i, i, u64p, u16p, u64p]),
            "or_server_batch": (None, [vp, i, i, u64p, u16p, u64p, u64p]),
            "or_server_eval": (None, [vp, i, i, i, i, u64p, u16p, u64p, vp, vp, i, u64p]),
            "or_chacha_quarter": (None, [C.POINTER(C.c_uint32)] * 4),
            "or_chacha20_block": (None, [u32p, C.c_uint32, u32p, u32p]),
            "or_expand_uniform": (None, [vp, C.c_char_p, i, i, u64p, C.c_size_t]),
            "or_mod_switch": (None, [vp, u64p, u64p]),
            "or_num_threads": (i, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Context:
    """Scheme parameters: ring degree n, the L ciphertext primes, t = 65537."""

    def __init__(self, n: int, primes, t: int = P.T_PLAIN):
        self.n, self.t = n, t
        self.primes = [int(q) for q in primes]
        self.L = len(self.primes)
        self.psis = [P.primitive_root_2n(q, n) for q in self.primes]
        self.psi_t = P.primitive_root_2n(t, n)
        self.Q = 1
        for q in self.primes:
            self.Q *= q
        self.delta = self.Q // t
        self._h = lib().or_ctx_create(n, self.L, _c(self.primes, np.uint64),
                                      _c(self.psis, np.uint64), t, self.psi_t)
        if not self._h:
            raise ValueError("bad oracle context")

    @classmethod
    def standard(cls, n: int, L: int):
        return cls(n, P.select_primes(n, L))

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.or_ctx_destroy(self._h)
            self._h = None

    # shapes
    def ct_shape(self, k: int = 2):
        return (k, self.L, self.n)

    def zeros_ct(self, k: int = 2):
        return np.zeros(self.ct_shape(k), dtype=np.uint64)

    # batching
    def encode(self, slots):
        out = np.zeros(self.n, dtype=np.uint32)
        lib().or_encode(self._h, _c(slots, np.uint32), out)
        return out

    def decode(self, poly):
        out = np.zeros(self.n, dtype=np.uint32)
        lib().or_decode(self._h, _c(poly, np.uint32), out)
        return out

    # FV
    def encrypt(self, sk, m_poly, a, e):
        ct = self.zeros_ct()
        lib().or_encrypt(self._h, _c(sk, np.int8), _c(m_poly, np.uint32), _c(a, np.uint64),
                         _c(e, np.int32), ct)
        return ct

    def encode_many(self, slots):
        slots = _c(slots, np.uint32)
        out = np.zeros_like(slots)
        lib().or_encode_many(self._h, slots, slots.shape[0], out)
        return out

    def encrypt_many(self, sk, m_polys, a, e):
        m_polys = _c(m_polys, np.uint32)
        out = np.zeros((m_polys.shape[0], 2, self.L, self.n), dtype=np.uint64)
        lib().or_encrypt_many(self._h, _c(sk, np.int8), m_polys, _c(a, np.uint64), _c(e, np.int32),
                              m_polys.shape[0], out)
        return out

    def decrypt_poly(self, sk, ct):
        out = np.zeros(self.n, dtype=np.uint32)
        lib().or_decrypt_poly(self._h, _c(sk, np.int8), _c(ct, np.uint64), out)
        return out

    def decrypt_slots(self, sk, ct):
        return self.decode(self.decrypt_poly(sk, ct))

    def noise_budget(self, sk, ct) -> int:
        return int(lib().or_noise_budget(self._h, _c(sk, np.int8), _c(ct, np.uint64)))

    def keygen_relin(self, sk, a, e):
        rlk = np.zeros((self.L, 2, self.L, self.n), dtype=np.uint64)
        lib().or_keygen_relin(self._h, _c(sk, np.int8), _c(a, np.uint64), _c(e, np.int32), rlk)
        return rlk

    def mul_plain(self, ct, p_poly):
        out = self.zeros_ct()
        lib().or_mul_plain(self._h, _c(ct, np.uint64), _c(p_poly, np.uint32), out)
        return out

    def add_plain_const(self, ct, kappa: int):
        ct = _c(ct, np.uint64).copy()
        lib().or_add_plain_const(self._h, ct, kappa % self.t)
        return ct

    def add_plain(self, ct, p_poly):
        ct = _c(ct, np.uint64).copy()
        lib().or_add_plain(self._h, ct, _c(p_poly, np.uint32))
        return ct

    def mul_const(self, ct, k: int):
        ct = _c(ct, np.uint64).copy()
        lib().or_mul_const(self._h, ct, k % self.t)
        return ct

    def multiply(self, x, y):
        out = self.zeros_ct(3)
        lib().or_multiply(self._h, _c(x, np.uint64), _c(y, np.uint64), out)
        return out

    def relin(self, ct3, rlk):
        out = self.zeros_ct()
        lib().or_relin(self._h, _c(ct3, np.uint64), _c(rlk, np.uint64), out)
        return out

    # server computation
    def select_sum(self, cts, cw_batch, h: int):
        out = self.zeros_ct()
        cts = _c(cts, np.uint64)
        lib().or_select_sum(self._h, cts.shape[0], h, cts, _c(cw_batch, np.uint16), out)
        return out

    def server_batch(self, cts, cw_batch, rlk, h: int):
        out = self.zeros_ct()
        cts = _c(cts, np.uint64)
        lib().or_server_batch(self._h, cts.shape[0], h, cts, _c(cw_batch, np.uint16),
                              _c(rlk, np.uint64), out)
        return out

    def server_eval(self, cts, cw_table, rlk, h: int, mask=None, finalize=True,
                    begin: int = 0, end: int | None = None, vals=None):
        """Alg. 2 / 5 over server batches [begin, end); vals [mu][N] (values < t, one per table
        entry) multiplies each batch's equality ciphertext by its server values (Alg. 4 / 5)."""
        out = self.zeros_ct()
        cts = _c(cts, np.uint64)
        cw_table = _c(cw_table, np.uint16)
        end = cw_table.shape[0] if end is None else end
        m = None
        if mask is not None:
            m = _c(mask, np.uint32)
        v = None
        if vals is not None:
            v = _c(vals, np.uint32)
            assert v.shape == cw_table.shape[:2]
        lib().or_server_eval(self._h, cts.shape[0], h, begin, end, cts, cw_table,
                             _c(rlk, np.uint64), None if m is None else m.ctypes.data,
                             None if v is None else v.ctypes.data, 1 if finalize else 0, out)
        return out

    def expand_uniform(self, seed: bytes, first: int, count: int):
        """a_j, j in [first, first + count), [count][L][N], from a 32-byte seed (ChaCha20)."""
        assert len(seed) == 32
        out = np.zeros((count, self.L, self.n), dtype=np.uint64)
        lib().or_expand_uniform(self._h, seed, first, count, out, self.L * self.n)
        return out

    def mod_switch(self, ct):
        """[round(q_0 X / Q)]_{q_0} of every coefficient of ct [2][L][N] -> [2][N]."""
        out = np.zeros((2, self.n), dtype=np.uint64)
        lib().or_mod_switch(self._h, _c(ct, np.uint64), out)
        return out

    # integer views used by the pins
    def residues_to_int(self, res):
        """CRT of one coefficient's residues (list of L ints) -> integer in [0, Q)."""
        x = 0
        for q, r in zip(self.primes, res):
            Qi = self.Q // q
            x += (int(r) * pow(Qi, -1, q) % q) * Qi
        return x % self.Q

    def poly_to_ints(self, poly):
        """limb-major [L][n] -> list of integers in [0, Q)."""
        poly = np.asarray(poly)
        return [self.residues_to_int([int(poly[l, i]) for l in range(self.L)]) for i in range(self.n)]

    def ints_to_poly(self, ints):
        out = np.zeros((self.L, self.n), dtype=np.uint64)
        for l, q in enumerate(self.primes):
            out[l] = [int(v) % q for v in ints]
        return out


def chacha_quarter(a: int, b: int, c: int, d: int):
    v = [C.c_uint32(x) for x in (a, b, c, d)]
    lib().or_chacha_quarter(*[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def chacha20_block(key_words, counter: int, nonce_words):
    out = np.zeros(16, dtype=np.uint32)
    lib().or_chacha20_block(_c(key_words, np.uint32), counter, _c(nonce_words, np.uint32), out)
    return out


def num_threads() -> int:
    """Threads the oracle's parallel regions use (OpenMP)."""
    return int(lib().or_num_threads())
