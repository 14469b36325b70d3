"""Python binding of libpepsi.so: the gfx950 server computation of PEPSI PSI-cardinality.

Argument marshalling only: every step runs in the library's HIP kernels.  Device
buffers are torch tensors on the current HIP device (torch is used for device
memory and streams); host buffers are numpy arrays.  Names follow include/pepsi.h
without the ``pepsi_`` prefix.  The library is loaded from this directory; if it
is missing, importing the binding raises (there is no other implementation).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpepsi.so")

PEPSI_PARAMS_PBH = 1
PEPSI_SERVER_CACHE_PLAINTEXTS = 1
PEPSI_SERVER_PLANES_ONLY = 2
MAX_PRIMES = 17


class PepsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pepsi error {code}: {msg}")
        self.code = code


class ParamsDesc(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("h", C.c_uint32),
                ("item_bits", C.c_uint32), ("mu", C.c_uint32), ("n_hash", C.c_uint32),
                ("max_evictions", C.c_uint32), ("flags", C.c_uint32),
                ("hash_seed", C.c_uint64)]


class ParamsInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_q", C.c_uint32), ("n_aux", C.c_uint32),
                ("h", C.c_uint32), ("ell", C.c_uint32), ("mu", C.c_uint32),
                ("item_bits", C.c_uint32), ("n_hash", C.c_uint32), ("t", C.c_uint64),
                ("primes", C.c_uint64 * MAX_PRIMES), ("psi", C.c_uint64 * MAX_PRIMES),
                ("psi_t", C.c_uint32), ("q_bits", C.c_uint32),
                ("query_bytes", C.c_uint64), ("ct_bytes", C.c_uint64),
                ("rlk_bytes", C.c_uint64), ("cache_bytes", C.c_uint64),
                ("effective_bits", C.c_uint32), ("flags", C.c_uint32)]


class ServerInfo(C.Structure):
    _fields_ = [("mu", C.c_uint32), ("max_load", C.c_uint32), ("cached", C.c_uint32),
                ("cached_batches", C.c_uint32), ("device_bytes", C.c_uint64),
                ("plane_groups", C.c_uint32)]


class Schedule(C.Structure):
    _fields_ = [("tile_batches", C.c_uint32), ("select_kernel", C.c_uint32), ("graph", C.c_uint32),
                ("run", C.c_uint32), ("source", C.c_uint32), ("tuned_ms_per_query", C.c_double)]

    def as_dict(self) -> dict:
        return {"tile_batches": self.tile_batches,
                "select_kernel": {1: "int8 matrix cores (digit planes)", 2: "64-bit VALU"}.get(self.select_kernel,
                                                                                          "automatic"),
                "graph": {1: "captured HIP graph", 2: "eager launches"}.get(self.graph, "automatic"),
                "run": {1: "one select-and-sum launch per run of tiles", 2: "one per tile"}.get(self.run, "automatic"),
                "source": {0: "default rule", 1: "tuned table", 2: "caller"}.get(self.source, "?"),
                "tuned_ms_per_query": self.tuned_ms_per_query or None}


SELECT_PLANES, SELECT_VALU = 1, 2
GRAPH_ON, GRAPH_OFF = 1, 2
RUN_ON, RUN_OFF = 1, 2


class ReqStats(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("slot", C.c_uint32), ("done", C.c_uint32)]


class ServeInfo(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("tiles", C.c_uint32), ("active", C.c_uint32), ("queued", C.c_uint32),
                ("steps", C.c_uint64), ("completed", C.c_uint64), ("slot_bytes", C.c_uint64)]


class Timing(C.Structure):
    _fields_ = [("select_sum_launches", C.c_uint64), ("select_sum_bytes", C.c_uint64),
                ("select_sum_ms", C.c_double), ("evals", C.c_uint64), ("eval_ms", C.c_double),
                ("ntt_fwd_launches", C.c_uint64), ("ntt_fwd_rows", C.c_uint64), ("ntt_fwd_ms", C.c_double),
                ("ntt_inv_launches", C.c_uint64), ("ntt_inv_rows", C.c_uint64), ("ntt_inv_ms", C.c_double),
                ("rescale_launches", C.c_uint64), ("rescale_products", C.c_uint64), ("rescale_ms", C.c_double),
                ("ext_launches", C.c_uint64), ("ext_products", C.c_uint64), ("ext_ms", C.c_double)]


_SIGS = {
    "pepsi_last_error": (C.c_char_p, []),
    "pepsi_params_create": (C.c_int, [C.POINTER(ParamsDesc), C.POINTER(C.c_void_p)]),
    "pepsi_params_get_info": (C.c_int, [C.c_void_p, C.POINTER(ParamsInfo)]),
    "pepsi_params_destroy": (None, [C.c_void_p]),
    "pepsi_exact_path_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "pepsi_client_table": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "pepsi_codeword_planes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pepsi_client_table64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "pepsi_codeword_planes64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pepsi_large_element_bits": (C.c_int, [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                           C.POINTER(C.c_uint32)]),
    "pepsi_hash_elements": (C.c_int, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "pepsi_server_create64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                        C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pepsi_encrypt": (C.c_int, [C.c_void_p] * 5 + [C.c_uint32, C.c_void_p, C.c_void_p]),
    "pepsi_keygen_relin": (C.c_int, [C.c_void_p] * 6),
    "pepsi_decrypt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "pepsi_noise_budget": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "pepsi_server_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    "pepsi_server_create_with_values": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                                  C.c_void_p, C.POINTER(C.c_void_p)]),
    "pepsi_server_create_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                         C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pepsi_server_get_info": (C.c_int, [C.c_void_p, C.POINTER(ServerInfo)]),
    "pepsi_server_codewords": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pepsi_server_destroy": (None, [C.c_void_p]),
    "pepsi_server_eval": (C.c_int, [C.c_void_p] * 6),
    "pepsi_server_timing": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(Timing)]),
    "pepsi_server_eval_batch": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p]),
    "pepsi_clock": (C.c_double, []),
    "pepsi_probe_valu": (C.c_int, [C.c_uint32, C.POINTER(C.c_double)]),
    "pepsi_server_set_schedule": (C.c_int, [C.c_void_p, C.POINTER(Schedule)]),
    "pepsi_server_get_schedule": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(Schedule)]),
    "pepsi_expand_uniform": (C.c_int, [C.c_void_p, C.c_char_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_uint64,
                                       C.c_void_p]),
    "pepsi_mod_switch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pepsi_serve_create": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint64, C.POINTER(C.c_void_p)]),
    "pepsi_serve_submit": (C.c_int, [C.c_void_p] * 5 + [C.POINTER(C.c_uint64)]),
    "pepsi_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(ReqStats)]),
    "pepsi_serve_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(ReqStats)]),
    "pepsi_serve_get_info": (C.c_int, [C.c_void_p, C.POINTER(ServeInfo)]),
    "pepsi_serve_destroy": (None, [C.c_void_p]),
    "pepsi_server_eval_range": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                                          C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pepsi_ntt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                            C.c_void_p]),
    "pepsi_encode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "pepsi_decode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "pepsi_select_sum": (C.c_int, [C.c_void_p] * 5),
    "pepsi_multiply": (C.c_int, [C.c_void_p] * 5),
    "pepsi_multiply_noalloc": (C.c_int, [C.c_void_p] * 5),
    "pepsi_relin": (C.c_int, [C.c_void_p] * 5),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2310_14565_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc: int):
    if rc != 0:
        raise PepsiError(rc, lib().pepsi_last_error().decode())


def _dev(t):
    """Device pointer of a contiguous torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _host(a):
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return C.c_void_p(a.ctypes.data)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Params:
    """A parameter set on the current HIP device (pepsi_params_*)."""

    def __init__(self, log_n: int, n_q: int, h: int, item_bits: int, mu: int, n_hash: int = 3,
                 max_evictions: int = 500, hash_seed: int = 0x5EED, pbh: bool = False):
        """pbh: permutation-based hashing (stored values of lambda - log_n + ceil(log2 k) bits)."""
        d = ParamsDesc(log_n, n_q, h, item_bits, mu, n_hash, max_evictions, PEPSI_PARAMS_PBH if pbh else 0,
                       hash_seed)
        h_ = C.c_void_p()
        _check(lib().pepsi_params_create(C.byref(d), C.byref(h_)))
        self._h = h_
        info = ParamsInfo()
        _check(lib().pepsi_params_get_info(self._h, C.byref(info)))
        self.info = info
        self.n, self.L, self.K = info.n, info.n_q, info.n_aux
        self.h, self.ell, self.mu = info.h, info.ell, info.mu
        self.primes = [int(info.primes[i]) for i in range(self.L + self.K)]
        self.effective_bits, self.pbh = info.effective_bits, bool(info.flags & PEPSI_PARAMS_PBH)
        self.q_primes = self.primes[:self.L]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().pepsi_params_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def exact_path_count(self) -> int:
        v = C.c_uint64()
        _check(lib().pepsi_exact_path_count(self._h, C.byref(v)))
        return int(v.value)

    @property
    def wide(self) -> bool:
        """Elements or stored values above 32 bits: the 64-bit client and server calls."""
        return self.info.item_bits > 32 or self.effective_bits > 32

    # client preparation (host numpy)
    def client_table(self, items: np.ndarray):
        """Cuckoo table of the client's elements: (table, valid); uint64 values for wide parameters."""
        dt = np.uint64 if self.wide else np.uint32
        items = np.ascontiguousarray(items, dtype=dt)
        table = np.zeros(self.n, dt)
        valid = np.zeros(self.n, np.uint8)
        f = lib().pepsi_client_table64 if self.wide else lib().pepsi_client_table
        _check(f(self._h, _host(items), items.shape[0], _host(table), _host(valid)))
        return table, valid

    def codeword_planes(self, table: np.ndarray, valid: np.ndarray):
        planes = np.zeros((self.ell, self.n), np.uint32)
        dt = np.uint64 if self.wide else np.uint32
        f = lib().pepsi_codeword_planes64 if self.wide else lib().pepsi_codeword_planes
        _check(f(self._h, _host(np.ascontiguousarray(table, dt)), _host(np.ascontiguousarray(valid, np.uint8)),
                 _host(planes)))
        return planes

    # device operations (torch tensors)
    def encrypt(self, sk, slots, a, e, out, stream=None):
        _check(lib().pepsi_encrypt(self._h, _dev(sk), _dev(slots), _dev(a), _dev(e), slots.shape[0],
                                   _dev(out), _stream(stream)))

    def keygen_relin(self, sk, a, e, out, stream=None):
        _check(lib().pepsi_keygen_relin(self._h, _dev(sk), _dev(a), _dev(e), _dev(out), _stream(stream)))

    def decrypt(self, sk, ct, out_slots, stream=None):
        count = ct.shape[0] if ct.dim() == 4 else 1
        _check(lib().pepsi_decrypt(self._h, _dev(sk), _dev(ct), count, _dev(out_slots), _stream(stream)))

    def expand_uniform(self, seed: bytes, first: int, count: int, out, out_stride: int | None = None,
                       offset_words: int = 0, stream=None):
        """a_j for j in [first, first + count) from a 32-byte seed (ChaCha20) into the device tensor
        out, at word offset_words + j * out_stride (default a plain [count][L][N] array; pass
        out_stride = 2 L N and offset_words = L N to fill the c1 halves of a request)."""
        if len(seed) != 32:
            raise ValueError("seed must be 32 bytes")
        stride = self.L * self.n if out_stride is None else out_stride
        if offset_words + (count - 1) * stride + self.L * self.n > out.numel() and count > 0:
            raise ValueError("output tensor too small")
        ptr = C.c_void_p(_dev(out).value + 8 * offset_words)
        _check(lib().pepsi_expand_uniform(self._h, seed, first, count, ptr, stride, _stream(stream)))

    def mod_switch(self, ct, out, stream=None):
        """out [2][N] = the response ct [2][L][N] switched to the first prime."""
        _check(lib().pepsi_mod_switch(self._h, _dev(ct), _dev(out), _stream(stream)))

    def noise_budget(self, sk, ct, stream=None) -> int:
        b = C.c_int32()
        _check(lib().pepsi_noise_budget(self._h, _dev(sk), _dev(ct), C.byref(b), _stream(stream)))
        return int(b.value)

    def ntt(self, data, rows: int, first_prime: int, n_primes: int, inverse: bool, stream=None):
        _check(lib().pepsi_ntt(self._h, _dev(data), rows, first_prime, n_primes, 1 if inverse else 0,
                               _stream(stream)))

    def encode(self, slots, out, stream=None):
        _check(lib().pepsi_encode(self._h, _dev(slots), slots.shape[0], _dev(out), _stream(stream)))

    def decode(self, poly, out, stream=None):
        _check(lib().pepsi_decode(self._h, _dev(poly), poly.shape[0], _dev(out), _stream(stream)))

    def select_sum(self, cts, cw, out, stream=None):
        _check(lib().pepsi_select_sum(self._h, _dev(cts), _dev(cw), _dev(out), _stream(stream)))

    def multiply(self, x, y, out, stream=None):
        _check(lib().pepsi_multiply(self._h, _dev(x), _dev(y), _dev(out), _stream(stream)))

    def multiply_noalloc(self, x, y, out, stream=None):
        """pepsi_multiply without device allocation (scratch in the library's fixed array)."""
        _check(lib().pepsi_multiply_noalloc(self._h, _dev(x), _dev(y), _dev(out), _stream(stream)))

    def relin(self, ct3, rlk, out, stream=None):
        _check(lib().pepsi_relin(self._h, _dev(ct3), _dev(rlk), _dev(out), _stream(stream)))


class Server:
    """The server's prepared set on the device (pepsi_server_*)."""

    def __init__(self, params: Params, items: np.ndarray, cache_plaintexts: bool = False, stream=None,
                 values: np.ndarray | None = None, max_cached: int = 0, planes_only: bool = False):
        """values (one per item, < t) make every evaluation PSI-Sum (with a mask) or labelled
        PSI (without); None is PSI-cardinality / the indicator.  max_cached bounds the cached
        batches (0: as many as fit); planes_only keeps the cache only as int8 digit planes."""
        wide = params.wide
        items = np.ascontiguousarray(items, dtype=np.uint64 if wide else np.uint32)
        h_ = C.c_void_p()
        flags = PEPSI_SERVER_CACHE_PLAINTEXTS if cache_plaintexts else 0
        if planes_only:
            flags |= PEPSI_SERVER_PLANES_ONLY
        vp = None
        if values is not None:
            values = np.ascontiguousarray(values, dtype=np.uint32)
            if values.shape != items.shape:
                raise ValueError("one value per item")
            vp = _host(values)
        if not 0 <= max_cached < 2**32:
            raise ValueError("max_cached out of range")
        create = lib().pepsi_server_create64 if wide else lib().pepsi_server_create_ex
        _check(create(params.handle, _host(items), vp, items.shape[0], flags, max_cached, _stream(stream),
                      C.byref(h_)))
        self._h = h_
        self.params = params
        info = ServerInfo()
        _check(lib().pepsi_server_get_info(self._h, C.byref(info)))
        self.max_load, self.cached, self.device_bytes = info.max_load, bool(info.cached), info.device_bytes
        self.cached_batches = info.cached_batches
        self.plane_groups = info.plane_groups

    def close(self):
        if getattr(self, "_h", None):
            lib().pepsi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def codewords(self) -> np.ndarray:
        p = self.params
        out = np.zeros((p.mu, p.n, p.h), np.uint16)
        _check(lib().pepsi_server_codewords(self._h, _host(out)))
        return out

    def eval(self, cts, rlk, mask, out, stream=None):
        _check(lib().pepsi_server_eval(self._h, _dev(cts), _dev(rlk), _dev(mask), _dev(out), _stream(stream)))

    def eval_batch(self, cts, rlks, masks, outs, stream=None):
        """cts, rlks, outs: lists of device tensors (one per query); masks: list of tensors or None."""
        nq = len(cts)
        arr = C.c_void_p * nq
        c_ = arr(*[t.data_ptr() for t in cts])
        r_ = arr(*[t.data_ptr() for t in rlks])
        o_ = arr(*[t.data_ptr() for t in outs])
        m_ = None if masks is None else arr(*[0 if m is None else m.data_ptr() for m in masks])
        _check(lib().pepsi_server_eval_batch(self._h, nq, c_, r_, m_, o_, _stream(stream)))

    def set_schedule(self, tile_batches: int = 0, select_kernel: int = 0, graph: int = 0, run: int = 0,
                     reset: bool = False):
        """Force the batched schedule (0 = automatic); reset returns to the automatic schedule."""
        if reset:
            _check(lib().pepsi_server_set_schedule(self._h, None))
            return
        sch = Schedule(tile_batches, select_kernel, graph, run, 0, 0.0)
        _check(lib().pepsi_server_set_schedule(self._h, C.byref(sch)))

    def schedule(self, nq: int) -> Schedule:
        sch = Schedule()
        _check(lib().pepsi_server_get_schedule(self._h, nq, C.byref(sch)))
        return sch

    def timing(self, enable: bool, reset: bool = False) -> Timing:
        t = Timing()
        _check(lib().pepsi_server_timing(self._h, 1 if enable else 0, 1 if reset else 0, C.byref(t)))
        return t

    def eval_range(self, cts, rlk, begin: int, end: int, finalize: bool, mask, out, stream=None):
        _check(lib().pepsi_server_eval_range(self._h, _dev(cts), _dev(rlk), begin, end,
                                             1 if finalize else 0, _dev(mask), _dev(out), _stream(stream)))


def large_element_bits(n_bins: int, mu_client: int, mu_server: int, alpha: int = 40) -> int:
    """lambda = alpha + ceil(log2(b mu_c mu_s)) (pepsi_large_element_bits)."""
    v = C.c_uint32()
    _check(lib().pepsi_large_element_bits(n_bins, mu_client, mu_server, alpha, C.byref(v)))
    return int(v.value)


def hash_elements(elements, bits: int) -> np.ndarray:
    """Byte strings -> their first `bits` bits of SHA-256 (pepsi_hash_elements), uint64.  elements:
    a list of bytes, or a uint8 [count][length] array of equal-length elements."""
    if isinstance(elements, np.ndarray) and elements.ndim == 2 and elements.dtype == np.uint8:
        count, length = elements.shape
        data = np.ascontiguousarray(elements).reshape(-1)
        offsets = np.arange(count + 1, dtype=np.uint64) * np.uint64(length)
    else:
        blobs = [bytes(e) for e in elements]
        count = len(blobs)
        offsets = np.zeros(count + 1, np.uint64)
        offsets[1:] = np.cumsum([len(b) for b in blobs], dtype=np.uint64)
        data = np.frombuffer(b"".join(blobs), dtype=np.uint8)
    if data.size == 0:
        data = np.zeros(1, np.uint8)
    out = np.zeros(count, np.uint64)
    _check(lib().pepsi_hash_elements(bits, _host(data), _host(offsets), count, _host(out)))
    return out


VALU_KINDS = ("v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_add_u32", "v_mad_u32_u24", "v_fma_f64")
MFMA_INT8_KIND = 6          # pepsi_probe_valu kind of v_mfma_i32_16x16x64_i8, in int8 operations/s


def probe_valu(kind: int) -> float:
    """Measured lane operations per second of one VALU instruction kind (pepsi_probe_valu)."""
    v = C.c_double()
    _check(lib().pepsi_probe_valu(kind, C.byref(v)))
    return float(v.value)


def probe_mfma_int8() -> float:
    """Measured int8 operations per second of the matrix instruction v_mfma_i32_16x16x64_i8."""
    return probe_valu(MFMA_INT8_KIND)


def clock() -> float:
    return float(lib().pepsi_clock())


class Serve:
    """Continuous-batching serving loop over a prepared server (pepsi_serve_*)."""

    def __init__(self, server: Server, max_active: int = 0, hbm_budget: int = 0):
        h_ = C.c_void_p()
        _check(lib().pepsi_serve_create(server._h, max_active, hbm_budget, C.byref(h_)))
        self._h = h_
        self.server = server
        self._keep = {}

    def submit(self, cts, rlk, mask, out) -> int:
        rid = C.c_uint64()
        _check(lib().pepsi_serve_submit(self._h, _dev(cts), _dev(rlk), _dev(mask), _dev(out), C.byref(rid)))
        self._keep[rid.value] = (cts, rlk, mask, out)       # buffers must outlive the request
        return int(rid.value)

    def poll(self, rid: int):
        done = C.c_int()
        st = ReqStats()
        _check(lib().pepsi_serve_poll(self._h, rid, C.byref(done), C.byref(st)))
        return bool(done.value), st

    def wait(self, rid: int) -> ReqStats:
        st = ReqStats()
        _check(lib().pepsi_serve_wait(self._h, rid, C.byref(st)))
        self._keep.pop(rid, None)
        return st

    def info(self) -> ServeInfo:
        i = ServeInfo()
        _check(lib().pepsi_serve_get_info(self._h, C.byref(i)))
        return i

    def close(self):
        if getattr(self, "_h", None):
            lib().pepsi_serve_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
