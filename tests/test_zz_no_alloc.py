"""The allocation-free ciphertext product (pepsi_multiply_noalloc): its scratch is a fixed device
array of the library, so the call allocates nothing.  Through the C-ABI, two calls in a row -- the
second with a smaller input -- equal pepsi_multiply (and the oracle's textbook product) bit for bit;
a parameter set whose product needs more scratch than the array holds is refused before any device
work."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import empty, to_dev, to_host
from oracle.core import Context
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc():
    import paper_2310_14565_amd as pk
    f = pk.lib().pepsi_multiply_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p] * 5
    return f


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("shapes", [((13, 4), (10, 2)), ((12, 3), (11, 3))])
def test_noalloc_product_equals_multiply(shapes):
    import torch
    import paper_2310_14565_amd as pk
    f = _noalloc()
    for call, (log_n, L) in enumerate(shapes):
        n = 1 << log_n
        gp = pk.Params(log_n, L, 2, 16, 4)
        x = W.uniform_residues((2,), gp.q_primes, n, 100 + call, "na-x")
        y = W.uniform_residues((2,), gp.q_primes, n, 200 + call, "na-y")
        dx, dy = to_dev(x), to_dev(y)
        ref = empty((3, L, n), np.uint64)
        gp.multiply(dx, dy, ref)
        got = empty((3, L, n), np.uint64)
        got.fill_(-1)
        rc = f(gp.handle, C.c_void_p(dx.data_ptr()), C.c_void_p(dy.data_ptr()), C.c_void_p(got.data_ptr()), _stream())
        assert rc == 0, pk.lib().pepsi_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"call {call}: N={n} L={L}"
        if log_n <= 11:
            ctx = Context(n, gp.q_primes)
            assert (to_host(got, np.uint64) == ctx.multiply(x, y)).all()


def test_noalloc_refuses_beyond_its_scratch():
    import paper_2310_14565_amd as pk
    f = _noalloc()
    gp = pk.Params(14, 8, 2, 16, 4)                # 15.6 MB of scratch needed, 8 MiB held
    x = empty((2, 8, 1 << 14), np.uint64)
    out = empty((3, 8, 1 << 14), np.uint64)
    rc = f(gp.handle, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), _stream())
    assert rc == -1
    assert "scratch" in pk.lib().pepsi_last_error().decode()
