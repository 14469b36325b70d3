"""The C-ABI library loads and exports every entry point the header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pepsi.h")
LIB = os.path.join(ROOT, "paper_2310_14565_amd", "libpepsi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pepsi_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def library():
    if not os.path.exists(LIB):
        from paper_2310_14565_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_protocol_calls():
    names = declared()
    for must in ("pepsi_params_create", "pepsi_client_table", "pepsi_codeword_planes", "pepsi_encrypt",
                 "pepsi_keygen_relin", "pepsi_server_create", "pepsi_server_eval", "pepsi_decrypt"):
        assert must in names


def test_every_declared_symbol_is_exported(library):
    for name in declared():
        assert hasattr(library, name), name


def test_binding_covers_the_header():
    import paper_2310_14565_amd as pk
    assert sorted(pk.exported_symbols()) == declared()


def test_last_error_is_callable_without_a_device(library):
    f = library.pepsi_last_error
    f.restype = ctypes.c_char_p
    assert f() == b""
