"""Thin ctypes binding of libpc2 (include/pc2.h).

Argument marshalling only: every function below checks tensor shapes and
dtypes, takes device pointers and the current HIP stream from torch, and calls
the C function of the same name.  All arithmetic runs in the library's HIP
kernels.  Importing this module fails if libpc2.so has not been built.

Limb arrays are torch tensors of dtype int32 holding the bit patterns of
little-endian uint32 limbs; uint64 arrays (quantized values, scalars) are int64
tensors holding the bit patterns.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t
from ctypes import c_uint32, c_uint64, c_void_p
from pathlib import Path
from typing import Optional, Sequence

import numpy as np
import torch

_LIB_PATH = Path(__file__).resolve().parent / "libpc2.so"

PC2_OK = 0
PC2_E_INVAL = -1
PC2_E_RANGE = -2
PC2_E_NOMEM = -3
PC2_E_DEVICE = -4
PC2_E_UNSUPPORTED = -5
PC2_E_BUSY = -6
PC2_OPT_WINDOW = 1
PC2_OPT_MODMUL = 2
PC2_OPT_TILE = 3
PC2_TILE_AUTO = 0
PC2_TILE_WIDE = 1
PC2_MODMUL_VALU = 0
PC2_MODMUL_MFMA = 1
PC2_MODMUL_AUTO = 2
PC2_OP_ENCRYPT = 1
PC2_OP_HOM_SUM = 2
PC2_OP_DECRYPT = 3
PC2_SERVE_FAIR = 0
PC2_SERVE_SHORTEST = 1

EXPORTS = [
    "pc2_ctx_create", "pc2_ctx_destroy", "pc2_ctx_sync", "pc2_ctx_take_error",
    "pc2_ctx_reserve", "pc2_ctx_set_option", "pc2_ctx_get_option", "pc2_strerror",
    "pc2_pk_create", "pc2_sk_create", "pc2_sk_public", "pc2_pk_destroy", "pc2_sk_destroy",
    "pc2_pk_info", "pc2_quantize", "pc2_dequantize", "pc2_encrypt", "pc2_encrypt_sk",
    "pc2_decrypt", "pc2_decrypt_static",
    "pc2_hom_add", "pc2_hom_scalar_mul", "pc2_hom_sum", "pc2_enc_sum_dec",
    "pc2_matvec_create", "pc2_matvec_info", "pc2_matvec_load", "pc2_matvec_apply",
    "pc2_matvec_destroy", "pc2_colsplit_create", "pc2_colsplit_set_scale",
    "pc2_colsplit_iterate", "pc2_colsplit_destroy",
    "pc2_batch_create", "pc2_batch_run", "pc2_batch_destroy", "pc2_autotune",
    "pc2_runner_create", "pc2_runner_group_size", "pc2_runner_launch", "pc2_runner_destroy",
    "pc2_pk_context", "pc2_server_create", "pc2_serve_submit", "pc2_serve_poll",
    "pc2_serve_progress", "pc2_serve_completed", "pc2_server_stats", "pc2_server_destroy",
    "pc2_server_set_policy",
    "pc2_admm_create", "pc2_admm_local", "pc2_admm_consensus", "pc2_admm_destroy",
]


class PC2Error(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


class pc2_qparams(ctypes.Structure):
    _fields_ = [("log2_scale", c_int32), ("offset", c_uint64), ("delta", c_uint64)]


class pc2_job(ctypes.Structure):
    _fields_ = [("op", c_int), ("pk", c_void_p), ("sk", c_void_p), ("in0", c_void_p),
                ("in1", c_void_p), ("m_limbs", c_uint32), ("out", c_void_p),
                ("count", c_size_t), ("K", c_uint32), ("inputs", c_void_p),
                ("lengths", c_void_p)]


def _load() -> ctypes.CDLL:
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2601_14980_amd.build`")
    lib = ctypes.CDLL(str(_LIB_PATH))
    P = c_void_p
    sig = {
        "pc2_ctx_create": (c_int, [c_int, POINTER(P)]),
        "pc2_ctx_destroy": (c_int, [P]),
        "pc2_ctx_sync": (c_int, [P, P]),
        "pc2_ctx_take_error": (c_int, [P]),
        "pc2_ctx_reserve": (c_int, [P, c_uint32]),
        "pc2_ctx_set_option": (c_int, [P, c_int, c_int64]),
        "pc2_ctx_get_option": (c_int, [P, c_int, POINTER(c_int64)]),
        "pc2_strerror": (c_char_p, [c_int]),
        "pc2_pk_create": (c_int, [P, c_uint32, P, POINTER(P)]),
        "pc2_sk_create": (c_int, [P, c_uint32, P, P, POINTER(P)]),
        "pc2_sk_public": (P, [P]),
        "pc2_pk_destroy": (c_int, [P]),
        "pc2_sk_destroy": (c_int, [P]),
        "pc2_pk_info": (c_int, [P, POINTER(c_uint32), POINTER(c_uint32)]),
        "pc2_pk_context": (c_int, [P, POINTER(P), POINTER(c_int)]),
        "pc2_quantize": (c_int, [P, POINTER(pc2_qparams), P, P, c_size_t, P]),
        "pc2_dequantize": (c_int, [P, POINTER(pc2_qparams), P, c_uint32, c_uint64, P,
                                   c_size_t, P]),
        "pc2_encrypt": (c_int, [P, P, c_uint32, P, P, c_size_t, P]),
        "pc2_encrypt_sk": (c_int, [P, P, c_uint32, P, P, c_size_t, P]),
        "pc2_decrypt": (c_int, [P, P, P, c_size_t, P]),
        "pc2_decrypt_static": (c_int, [P, P, P, c_size_t, P]),
        "pc2_hom_add": (c_int, [P, P, P, P, c_size_t, P]),
        "pc2_hom_scalar_mul": (c_int, [P, P, P, P, c_size_t, P]),
        "pc2_hom_sum": (c_int, [P, POINTER(P), c_uint32, P, c_size_t, P]),
        "pc2_enc_sum_dec": (c_int, [P, POINTER(P), POINTER(P), c_uint32, c_uint32, P,
                                    c_size_t, P]),
        "pc2_matvec_create": (c_int, [P, c_size_t, c_uint32, c_uint32, c_size_t, POINTER(P)]),
        "pc2_matvec_info": (c_int, [P, POINTER(c_uint32), POINTER(c_size_t)]),
        "pc2_matvec_load": (c_int, [P, P, P]),
        "pc2_matvec_apply": (c_int, [P, P, P, P, c_size_t, P]),
        "pc2_matvec_destroy": (c_int, [P]),
        "pc2_colsplit_create": (c_int, [P, P, P, c_uint32, c_uint32, c_uint32, c_double,
                                        c_uint32, P, c_size_t, P, POINTER(P)]),
        "pc2_colsplit_set_scale": (c_int, [P, c_uint32, P]),
        "pc2_colsplit_iterate": (c_int, [P, c_double, c_int, P, P, P, P]),
        "pc2_colsplit_destroy": (c_int, [P]),
        "pc2_batch_create": (c_int, [P, POINTER(pc2_job), c_size_t, POINTER(P)]),
        "pc2_batch_run": (c_int, [P, P]),
        "pc2_batch_destroy": (c_int, [P]),
        "pc2_autotune": (c_int, [P, P, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
        "pc2_runner_create": (c_int, [P, c_int, c_uint32, c_size_t, c_size_t, POINTER(P)]),
        "pc2_runner_group_size": (c_int, [P, c_int, POINTER(c_uint32)]),
        "pc2_runner_launch": (c_int, [P, POINTER(pc2_job), POINTER(c_size_t), POINTER(c_size_t),
                                      c_size_t, P]),
        "pc2_runner_destroy": (c_int, [P]),
        "pc2_server_create": (c_int, [P, P, c_size_t, c_size_t, c_size_t, POINTER(P)]),
        "pc2_serve_submit": (c_int, [P, POINTER(pc2_job), POINTER(c_uint64)]),
        "pc2_serve_poll": (c_int, [P, c_uint64, POINTER(c_int)]),
        "pc2_serve_progress": (c_int, [P, POINTER(c_size_t)]),
        "pc2_serve_completed": (c_int, [P, POINTER(c_uint64), c_size_t, POINTER(c_size_t)]),
        "pc2_server_stats": (c_int, [P, POINTER(c_uint64), POINTER(c_size_t), POINTER(c_size_t)]),
        "pc2_server_set_policy": (c_int, [P, c_int, c_double]),
        "pc2_server_destroy": (c_int, [P]),
        "pc2_admm_create": (c_int, [P, P, P, c_uint32, c_uint32, c_uint32, c_double, P,
                                    POINTER(P)]),
        "pc2_admm_local": (c_int, [P, P, P, P, P, P]),
        "pc2_admm_consensus": (c_int, [P, P, P, c_double, P, P, P]),
        "pc2_admm_destroy": (c_int, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def strerror(status: int) -> str:
    return lib.pc2_strerror(status).decode()


def _check(status: int, what: str) -> None:
    if status != PC2_OK:
        raise PC2Error(status, what)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev_ptr(t: torch.Tensor, dtype: torch.dtype, what: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    return t.data_ptr()


def limbs_to_host_array(x: int, nlimbs: int) -> np.ndarray:
    """int -> uint32 numpy array of nlimbs little-endian limbs."""
    return np.frombuffer(int(x).to_bytes(4 * nlimbs, "little"), dtype="<u4").astype(np.uint32)


# ------------------------------------------------------------------ handles
class Context:
    """A libpc2 context bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = c_void_p()
        _check(lib.pc2_ctx_create(device, byref(h)), "pc2_ctx_create")
        self.handle = h
        self.device = device

    def close(self) -> None:
        if self.handle:
            lib.pc2_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None) -> int:
        """Wait for the stream and return the latched data status (0 or PC2_E_RANGE)."""
        st = lib.pc2_ctx_sync(self.handle, _stream(stream))
        if st not in (PC2_OK, PC2_E_RANGE):
            raise PC2Error(st, "pc2_ctx_sync")
        return st

    def reserve(self, max_nbits: int) -> None:
        _check(lib.pc2_ctx_reserve(self.handle, max_nbits), "pc2_ctx_reserve")

    def set_option(self, option: int, value: int) -> None:
        _check(lib.pc2_ctx_set_option(self.handle, option, value), "pc2_ctx_set_option")

    def get_option(self, option: int) -> int:
        v = c_int64()
        _check(lib.pc2_ctx_get_option(self.handle, option, byref(v)), "pc2_ctx_get_option")
        return v.value


class PublicKey:
    def __init__(self, ctx: Context, nbits: int, n: int):
        self.ctx, self.nbits, self.n = ctx, nbits, n
        self.L = (nbits + 31) // 32
        arr = limbs_to_host_array(n, self.L)
        h = c_void_p()
        _check(lib.pc2_pk_create(ctx.handle, nbits, arr.ctypes.data, byref(h)), "pc2_pk_create")
        self.handle = h
        self._owned = True

    def close(self) -> None:
        if self.handle and self._owned:
            lib.pc2_pk_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SecretKey:
    def __init__(self, ctx: Context, nbits: int, p: int, q: int):
        self.ctx, self.nbits, self.p, self.q = ctx, nbits, p, q
        self.n = p * q
        self.L = (nbits + 31) // 32
        pa, qa = limbs_to_host_array(p, self.L), limbs_to_host_array(q, self.L)
        h = c_void_p()
        _check(lib.pc2_sk_create(ctx.handle, nbits, pa.ctypes.data, qa.ctypes.data, byref(h)),
               "pc2_sk_create")
        self.handle = h
        pub = PublicKey.__new__(PublicKey)
        pub.ctx, pub.nbits, pub.n, pub.L = ctx, nbits, self.n, self.L
        pub.handle = c_void_p(lib.pc2_sk_public(h))
        pub._owned = False
        self.public = pub

    def close(self) -> None:
        if self.handle:
            lib.pc2_sk_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- data calls
def _rows(t: torch.Tensor, width: int, what: str) -> int:
    if t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{what}: expected shape [count, {width}], got {tuple(t.shape)}")
    return t.shape[0]


def pc2_quantize(ctx: Context, log2_scale: int, offset: int, delta: int, x: torch.Tensor,
                 m: torch.Tensor, stream=None) -> None:
    """m (int64 bit patterns of uint64) <- rint(x 2^k) + offset for x in the
    common interval [-offset, delta - offset) / 2^k."""
    if x.shape != m.shape or x.dim() != 1:
        raise ValueError("x and m must be 1-D tensors of equal length")
    q = pc2_qparams(log2_scale, offset, delta)
    _check(lib.pc2_quantize(ctx.handle, byref(q), _dev_ptr(x, torch.float64, "x"),
                            _dev_ptr(m, torch.int64, "m"), x.numel(), _stream(stream)),
           "pc2_quantize")


def pc2_dequantize(ctx: Context, log2_scale: int, offset: int, m: torch.Tensor, weight: int,
                   x: torch.Tensor, stream=None) -> None:
    """x <- (M - weight*offset) / 2^k for M given as int32 limb rows [count, m_limbs]."""
    count = m.shape[0]
    if m.dim() != 2 or x.shape != (count,):
        raise ValueError("m must be [count, m_limbs] and x [count]")
    q = pc2_qparams(log2_scale, offset, offset)  # delta is not read by dequantize
    _check(lib.pc2_dequantize(ctx.handle, byref(q), _dev_ptr(m, torch.int32, "m"), m.shape[1],
                              weight, _dev_ptr(x, torch.float64, "x"), count, _stream(stream)),
           "pc2_dequantize")


def pc2_encrypt(pk: PublicKey, m: torch.Tensor, r: torch.Tensor, c: torch.Tensor,
                stream=None) -> None:
    count = _rows(r, pk.L, "r")
    if m.dim() != 2 or m.shape[0] != count:
        raise ValueError("m must be [count, m_limbs]")
    _rows(c, 2 * pk.L, "c")
    _check(lib.pc2_encrypt(pk.handle, _dev_ptr(m, torch.int32, "m"), m.shape[1],
                           _dev_ptr(r, torch.int32, "r"), _dev_ptr(c, torch.int32, "c"), count,
                           _stream(stream)), "pc2_encrypt")


def pc2_encrypt_sk(sk: SecretKey, m: torch.Tensor, r: torch.Tensor, c: torch.Tensor,
                   stream=None) -> None:
    count = _rows(r, sk.L, "r")
    if m.dim() != 2 or m.shape[0] != count:
        raise ValueError("m must be [count, m_limbs]")
    _rows(c, 2 * sk.L, "c")
    _check(lib.pc2_encrypt_sk(sk.handle, _dev_ptr(m, torch.int32, "m"), m.shape[1],
                              _dev_ptr(r, torch.int32, "r"), _dev_ptr(c, torch.int32, "c"), count,
                              _stream(stream)), "pc2_encrypt_sk")


def pc2_decrypt(sk: SecretKey, c: torch.Tensor, m: torch.Tensor, stream=None) -> None:
    count = _rows(c, 2 * sk.L, "c")
    _rows(m, sk.L, "m")
    if m.shape[0] != count:
        raise ValueError("m and c must have the same count")
    _check(lib.pc2_decrypt(sk.handle, _dev_ptr(c, torch.int32, "c"),
                           _dev_ptr(m, torch.int32, "m"), count, _stream(stream)), "pc2_decrypt")


def pc2_decrypt_static(sk: SecretKey, c: torch.Tensor, m: torch.Tensor, stream=None) -> None:
    """pc2_decrypt with the library's static device scratch: allocates nothing."""
    count = _rows(c, 2 * sk.L, "c")
    _rows(m, sk.L, "m")
    if m.shape[0] != count:
        raise ValueError("m and c must have the same count")
    _check(lib.pc2_decrypt_static(sk.handle, _dev_ptr(c, torch.int32, "c"),
                                  _dev_ptr(m, torch.int32, "m"), count, _stream(stream)),
           "pc2_decrypt_static")


def pc2_hom_add(pk: PublicKey, c1: torch.Tensor, c2: torch.Tensor, out: torch.Tensor,
                stream=None) -> None:
    count = _rows(c1, 2 * pk.L, "c1")
    _rows(c2, 2 * pk.L, "c2")
    _rows(out, 2 * pk.L, "out")
    _check(lib.pc2_hom_add(pk.handle, _dev_ptr(c1, torch.int32, "c1"),
                           _dev_ptr(c2, torch.int32, "c2"), _dev_ptr(out, torch.int32, "out"),
                           count, _stream(stream)), "pc2_hom_add")


def pc2_hom_scalar_mul(pk: PublicKey, c: torch.Tensor, k: torch.Tensor, out: torch.Tensor,
                       stream=None) -> None:
    count = _rows(c, 2 * pk.L, "c")
    _rows(out, 2 * pk.L, "out")
    if k.shape != (count,):
        raise ValueError("k must be [count]")
    _check(lib.pc2_hom_scalar_mul(pk.handle, _dev_ptr(c, torch.int32, "c"),
                                  _dev_ptr(k, torch.int64, "k"),
                                  _dev_ptr(out, torch.int32, "out"), count, _stream(stream)),
           "pc2_hom_scalar_mul")


def pc2_hom_sum(pk: PublicKey, cs: Sequence[torch.Tensor], out: torch.Tensor,
                stream=None) -> None:
    count = _rows(out, 2 * pk.L, "out")
    ptrs = (c_void_p * len(cs))()
    for i, c in enumerate(cs):
        if _rows(c, 2 * pk.L, f"c[{i}]") != count:
            raise ValueError("all inputs must have the output's count")
        ptrs[i] = _dev_ptr(c, torch.int32, f"c[{i}]")
    _check(lib.pc2_hom_sum(pk.handle, ptrs, len(cs), _dev_ptr(out, torch.int32, "out"), count,
                           _stream(stream)), "pc2_hom_sum")


def pc2_enc_sum_dec(sk: SecretKey, ms: Sequence[torch.Tensor], rs: Sequence[torch.Tensor],
                    m_out: torch.Tensor, stream=None) -> None:
    count = _rows(m_out, sk.L, "m_out")
    if len(ms) != len(rs) or not ms:
        raise ValueError("need K >= 1 plaintext and randomness arrays")
    m_limbs = ms[0].shape[1]
    mp, rp = (c_void_p * len(ms))(), (c_void_p * len(rs))()
    for i, (m, r) in enumerate(zip(ms, rs)):
        if _rows(m, m_limbs, f"m[{i}]") != count or _rows(r, sk.L, f"r[{i}]") != count:
            raise ValueError("all inputs must have the output's count")
        mp[i] = _dev_ptr(m, torch.int32, f"m[{i}]")
        rp[i] = _dev_ptr(r, torch.int32, f"r[{i}]")
    _check(lib.pc2_enc_sum_dec(sk.handle, mp, rp, len(ms), m_limbs,
                               _dev_ptr(m_out, torch.int32, "m_out"), count, _stream(stream)),
           "pc2_enc_sum_dec")


# -------------------------------------------------------- ciphertext mat-vec
class MatVec:
    """Plan of the ciphertext matrix-vector product (pc2_matvec):
    out_i = alpha_i * prod_j c_j^(B_ij) mod n^2 over fixed-base tables of c."""

    def __init__(self, pk: PublicKey, cols: int, ebits: int = 64, window: int = 0,
                 rows_hint: int = 0):
        h = c_void_p()
        _check(lib.pc2_matvec_create(pk.handle, cols, ebits, window, rows_hint, byref(h)),
               "pc2_matvec_create")
        self.handle = h
        self.pk = pk
        self.cols = cols
        w, nb = c_uint32(), c_size_t()
        _check(lib.pc2_matvec_info(h, byref(w), byref(nb)), "pc2_matvec_info")
        self.window = w.value
        self.table_bytes = nb.value

    def load(self, c: torch.Tensor, stream=None) -> None:
        if _rows(c, 2 * self.pk.L, "c") != self.cols:
            raise ValueError("c must hold one ciphertext per column")
        _check(lib.pc2_matvec_load(self.handle, _dev_ptr(c, torch.int32, "c"), _stream(stream)),
               "pc2_matvec_load")

    def apply(self, B: torch.Tensor, out: torch.Tensor, alpha: Optional[torch.Tensor] = None,
              stream=None) -> None:
        rows = _rows(out, 2 * self.pk.L, "out")
        if B.dim() != 2 or B.shape[0] != rows or B.shape[1] != self.cols:
            raise ValueError("B must be [rows][cols]")
        a = None
        if alpha is not None:
            if _rows(alpha, 2 * self.pk.L, "alpha") != rows:
                raise ValueError("alpha must have one ciphertext per row")
            a = _dev_ptr(alpha, torch.int32, "alpha")
        _check(lib.pc2_matvec_apply(self.handle, _dev_ptr(B, torch.int64, "B"), a,
                                    _dev_ptr(out, torch.int32, "out"), rows, _stream(stream)),
               "pc2_matvec_apply")

    def close(self) -> None:
        if self.handle:
            lib.pc2_matvec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------- batches
def _make_jobs(jobs: Sequence[dict], keep: list):
    """dicts (op, pk / sk, m, r, c, inputs, lengths, out) -> pc2_job array."""
    arr = (pc2_job * len(jobs))()
    for i, j in enumerate(jobs):
        op = j["op"]
        d = arr[i]
        d.op = op
        out = j["out"]
        d.out = _dev_ptr(out, torch.int32, "out")
        d.count = out.shape[0]
        if op == PC2_OP_ENCRYPT:
            d.pk = j["pk"].handle
            d.in0 = _dev_ptr(j["m"], torch.int32, "m")
            d.in1 = _dev_ptr(j["r"], torch.int32, "r")
            d.m_limbs = j["m"].shape[1]
        elif op == PC2_OP_DECRYPT:
            d.sk = j["sk"].handle
            d.in0 = _dev_ptr(j["c"], torch.int32, "c")
        elif op == PC2_OP_HOM_SUM:
            d.pk = j["pk"].handle
            ins = j["inputs"]
            ptrs = (c_void_p * len(ins))(*[_dev_ptr(t, torch.int32, "input") for t in ins])
            d.K = len(ins)
            d.inputs = ctypes.cast(ptrs, c_void_p)
            keep.append(ptrs)
            if j.get("lengths") is not None:
                lens = (c_size_t * len(ins))(*[int(v) for v in j["lengths"]])
                d.lengths = ctypes.cast(lens, c_void_p)
                keep.append(lens)
        else:
            raise ValueError(f"unknown op {op}")
    return arr


class Batch:
    """A planned persistent launch over many jobs of one operation.

    jobs: list of dicts with the fields of pc2_job -- op, pk / sk, m, r (encrypt),
    c (decrypt), inputs and optional lengths (hom_sum), out -- with tensors for
    the data arrays.  The tensors must outlive the batch.
    """

    def __init__(self, ctx: Context, jobs: Sequence[dict]):
        self.ctx = ctx
        self._keep: list = []
        arr = _make_jobs(jobs, self._keep)
        h = c_void_p()
        _check(lib.pc2_batch_create(ctx.handle, arr, len(jobs), byref(h)), "pc2_batch_create")
        self.handle = h

    def run(self, stream=None) -> None:
        """Run on a stream (torch's current one by default): the first run on a
        non-null stream is captured in a HIP graph, later runs replay it.
        stream=0 launches on the null stream without a graph."""
        st = _stream(stream) if stream != 0 else None
        _check(lib.pc2_batch_run(self.handle, st), "pc2_batch_run")

    def close(self) -> None:
        if self.handle:
            lib.pc2_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Runner:
    """Reusable persistent launcher (pc2_runner): one launch per call over
    element-group ranges of several jobs."""

    def __init__(self, ctx: Context, op: int, max_nbits: int, max_jobs: int, max_groups: int):
        h = c_void_p()
        _check(lib.pc2_runner_create(ctx.handle, op, max_nbits, max_jobs, max_groups, byref(h)),
               "pc2_runner_create")
        self.handle = h
        self.ctx = ctx

    def launch(self, jobs: Sequence[dict], first: Sequence[int], ngroups: Sequence[int],
               stream=None) -> None:
        keep: list = []
        arr = _make_jobs(jobs, keep)
        f = (c_size_t * len(jobs))(*first)
        g = (c_size_t * len(jobs))(*ngroups)
        _check(lib.pc2_runner_launch(self.handle, arr, f, g, len(jobs), _stream(stream)),
               "pc2_runner_launch")

    def close(self) -> None:
        if self.handle:
            lib.pc2_runner_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server for continuous batching under one key (pc2_server).

    submit() takes a job dict as for Batch (op, pk / sk, m, r, c, inputs,
    lengths, out); its tensors are held here until the request is reported
    done by poll() or completed()."""

    def __init__(self, ctx: Context, sk: SecretKey, hbm_budget: int = 0,
                 tick_groups: int = 2048, max_requests: int = 1024):
        h = c_void_p()
        _check(lib.pc2_server_create(ctx.handle, sk.handle, hbm_budget, tick_groups,
                                     max_requests, byref(h)), "pc2_server_create")
        self.handle = h
        self.ctx = ctx
        self._held: dict[int, tuple] = {}
        self._ids = (c_uint64 * max_requests)()

    def submit(self, job: dict) -> int:
        keep: list = []
        arr = _make_jobs([job], keep)
        rid = c_uint64()
        _check(lib.pc2_serve_submit(self.handle, arr, byref(rid)), "pc2_serve_submit")
        self._held[rid.value] = (job, keep)
        return rid.value

    def poll(self, rid: int) -> bool:
        done = c_int()
        _check(lib.pc2_serve_poll(self.handle, rid, byref(done)), "pc2_serve_poll")
        if done.value:
            self._held.pop(rid, None)
        return bool(done.value)

    def progress(self) -> int:
        pending = c_size_t()
        _check(lib.pc2_serve_progress(self.handle, byref(pending)), "pc2_serve_progress")
        return pending.value

    def completed(self) -> list[int]:
        n = c_size_t()
        _check(lib.pc2_serve_completed(self.handle, self._ids, len(self._ids), byref(n)),
               "pc2_serve_completed")
        ids = list(self._ids[:n.value])
        for rid in ids:
            self._held.pop(rid, None)
        return ids

    def set_policy(self, policy: int, max_age_s: float = 1.0) -> None:
        _check(lib.pc2_server_set_policy(self.handle, policy, max_age_s), "pc2_server_set_policy")

    def stats(self) -> dict:
        launches, mx, used = c_uint64(), c_size_t(), c_size_t()
        _check(lib.pc2_server_stats(self.handle, byref(launches), byref(mx), byref(used)),
               "pc2_server_stats")
        return dict(launches=launches.value, max_bytes=mx.value, used_bytes=used.value)

    def close(self) -> None:
        if self.handle:
            lib.pc2_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def runner_group_size(pk: PublicKey, op: int) -> int:
    v = c_uint32()
    _check(lib.pc2_runner_group_size(pk.handle, op, byref(v)), "pc2_runner_group_size")
    return v.value


def pc2_autotune(sk: SecretKey, stream=None) -> tuple[int, int, int]:
    """Tune the encryption tile and the exponentiation windows of this key's
    class; returns (w_enc, w_dec, lanes per ciphertext in encryption)."""
    we, wd, te = c_int(), c_int(), c_int()
    _check(lib.pc2_autotune(sk.handle, _stream(stream), byref(we), byref(wd), byref(te)),
           "pc2_autotune")
    return we.value, wd.value, te.value


# ---------------------------------------------------------------- marshalling
def to_device_limbs(arr: np.ndarray, device="cuda") -> torch.Tensor:
    """uint32 [count][limbs] numpy array -> int32 CUDA tensor (same bits)."""
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


def from_device_limbs(t: torch.Tensor) -> np.ndarray:
    """int32 tensor -> uint32 numpy array (same bits)."""
    return t.detach().cpu().numpy().view(np.uint32)
