"""CPU-side checks of the C ABI: the library loads, exports every function
include/pc2.h declares, and rejects bad arguments synchronously (these paths
return before any device work, so they run without a GPU)."""
from __future__ import annotations

import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "pc2.h"


def declared_functions() -> list[str]:
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pc2_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def pc2():
    from paper_2601_14980_amd import pc2 as mod
    return mod


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pc2_quantize", "pc2_dequantize", "pc2_encrypt", "pc2_decrypt",
                     "pc2_hom_add", "pc2_hom_scalar_mul", "pc2_hom_sum", "pc2_enc_sum_dec"):
        assert required in names


def test_library_exports_every_declared_symbol(pc2):
    lib = ctypes.CDLL(str(ROOT / "paper_2601_14980_amd" / "libpc2.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing
    # the binding wires every declared symbol
    assert sorted(pc2.EXPORTS) == declared_functions()


def test_strerror(pc2):
    assert pc2.strerror(0) == "ok"
    assert pc2.strerror(-2) == "input value out of range"
    assert pc2.strerror(12345) == "unknown status"


def test_null_arguments_rejected(pc2):
    lib = pc2.lib
    INVAL = pc2.PC2_E_INVAL
    q = pc2.pc2_qparams(20, 1 << 23, 1 << 24)
    assert lib.pc2_ctx_create(0, None) == INVAL
    assert lib.pc2_ctx_destroy(None) == INVAL
    assert lib.pc2_ctx_sync(None, None) == INVAL
    assert lib.pc2_quantize(None, ctypes.byref(q), None, None, 1, None) == INVAL
    assert lib.pc2_dequantize(None, ctypes.byref(q), None, 2, 1, None, 1, None) == INVAL
    assert lib.pc2_encrypt(None, None, 2, None, None, 1, None) == INVAL
    assert lib.pc2_decrypt(None, None, None, 1, None) == INVAL
    assert lib.pc2_hom_add(None, None, None, None, 1, None) == INVAL
    assert lib.pc2_hom_scalar_mul(None, None, None, None, 1, None) == INVAL
    assert lib.pc2_hom_sum(None, None, 2, None, 1, None) == INVAL
    assert lib.pc2_enc_sum_dec(None, None, None, 2, 2, None, 1, None) == INVAL
    assert lib.pc2_pk_create(None, 256, None, None) == INVAL
    assert lib.pc2_sk_create(None, 256, None, None, None) == INVAL
    assert lib.pc2_pk_destroy(None) == INVAL
    assert lib.pc2_sk_destroy(None) == INVAL
    assert lib.pc2_pk_info(None, None, None) == INVAL
    assert lib.pc2_pk_context(None, None, None) == INVAL
    assert lib.pc2_sk_public(None) is None
    h = ctypes.c_void_p()
    assert lib.pc2_server_create(None, None, 0, 8, 8, ctypes.byref(h)) == INVAL
    rid = ctypes.c_uint64()
    done = ctypes.c_int()
    n = ctypes.c_size_t()
    assert lib.pc2_serve_submit(None, None, ctypes.byref(rid)) == INVAL
    assert lib.pc2_serve_poll(None, 1, ctypes.byref(done)) == INVAL
    assert lib.pc2_serve_progress(None, None) == INVAL
    assert lib.pc2_serve_completed(None, None, 0, ctypes.byref(n)) == INVAL
    assert lib.pc2_server_stats(None, None, None, None) == INVAL
    assert lib.pc2_server_set_policy(None, pc2.PC2_SERVE_SHORTEST, 1.0) == INVAL
    assert lib.pc2_server_destroy(None) == INVAL


def test_context_without_gpu(pc2):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert pc2.lib.pc2_ctx_create(0, ctypes.byref(h)) == pc2.PC2_E_DEVICE
    assert pc2.lib.pc2_ctx_create(-1, ctypes.byref(h)) == pc2.PC2_E_DEVICE
