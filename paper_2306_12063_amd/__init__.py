"""Python binding of libldpc, the MI355X QC-LDPC encoder/decoder library.

The functions below carry the names of the C entry points declared in
include/ldpc.h and only marshal arguments: base matrices travel as host
int16 arrays, data as torch tensors on the GPU (PyTorch provides device
memory and the current stream), and every step runs in the library's HIP
kernels. There is no CPU fallback: if libldpc.so is missing the import of a
function fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

__all__ = [
    "LdpcError", "lib", "ldpc_code_info", "ldpc_encode", "ldpc_decode_f32", "ldpc_decode_i8",
    "ldpc_quantize_i8", "ldpc_quantize_weights", "ldpc_autotune_decode", "ldpc_decode_layouts",
    "ldpc_set_decode_layout", "ldpc_nms_ckpt_bytes", "ldpc_nms_fwd", "ldpc_nms_bwd",
    "ldpc_random_bits", "ldpc_frame_stats", "ldpc_fallback_f32", "ldpc_fallback_i8", "Codeset", "ldpc_lds_probe",
    "ldpc_decode_flood_f32", "ldpc_decode_flood_i8", "ldpc_decode_q16", "ldpc_quantize_q16",
    "ldpc_encode_packed", "ldpc_shift_packed", "ldpc_decode_f32_packed", "ldpc_decode_i8_packed", "ldpc_awgn_llr", "ldpc_last_error", "ldpc_cache_clear",
    "EXPORTS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpc.so")

LDPC_OK, LDPC_EINVAL, LDPC_ESTRUCT, LDPC_ERANGE, LDPC_EDEVICE, LDPC_ENOMEM = 0, -1, -2, -3, -4, -5

_p, _i32, _i64, _u64, _f32 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_float
# name -> (argtypes, restype); every entry point of include/ldpc.h
EXPORTS = {
    "ldpc_code_info": ([_p, _i32, _i32, _i32, _p], _i32),
    "ldpc_encode": ([_p, _i32, _i32, _i32, _p, _p, _i64, _p], _i32),
    "ldpc_decode_f32": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _f32, _i32, _p, _p, _p, _p, _p, _p], _i32),
    "ldpc_decode_i8": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _i32, _i32, _p, _i32, _p, _p, _p, _p, _p], _i32),
    "ldpc_random_bits": ([_u64, _p, _i64, _i64, _p, _p], _i32),
    "ldpc_awgn_llr": ([_u64, _p, _p, _i64, _i64, _f32, _f32, _p, _p, _p, _p], _i32),
    "ldpc_frame_stats": ([_p, _p, _p, _p, _i64, _i64, _i64, _p, _p], _i32),
    "ldpc_lds_probe": ([_i32, _i32, _p, _p], _i32),
    "ldpc_fallback_f32": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _f32, _p, _p, _p, _p, _p, _p], _i32),
    "ldpc_fallback_i8": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _i32, _i32, _p, _p, _p, _p, _p, _p], _i32),
    "ldpc_quantize_i8": ([_p, _p, _i64, _f32, _p], _i32),
    "ldpc_quantize_weights": ([_p, _p, _i64, _p], _i32),
    "ldpc_autotune_decode": ([_p, _i32, _i32, _i32, _i32, _i32, _i64, _p, _p, _p], _i32),
    "ldpc_nms_ckpt_bytes": ([_p, _i32, _i32, _i32, _i64, _i32], C.c_size_t),
    "ldpc_nms_fwd": ([_p, _i32, _i32, _i32, _p, _p, _i64, _i32, _p, _p, C.c_size_t, _p, _p, _p], _i32),
    "ldpc_nms_bwd": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _p, _p, C.c_size_t, _p, _p, _p], _i32),
    "ldpc_codeset_create": ([_p, _p, _p, _p, _i32, _p], _i32),
    "ldpc_codeset_destroy": ([_p], None),
    "ldpc_codeset_info": ([_p, _i32, _p], _i32),
    "ldpc_batch_work_bytes": ([_p, _i64], C.c_size_t),
    "ldpc_decode_batch_f32": ([_p, _p, _p, _p, _i64, _i64, _i32, _f32, _i32, _p, _p, _p, _p, _p, C.c_size_t, _p],
                              _i32),
    "ldpc_decode_batch_i8": ([_p, _p, _p, _p, _i64, _i64, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p, C.c_size_t,
                              _p], _i32),
    "ldpc_decode_batch_f32_noalloc": ([_p, _p, _p, _p, _i64, _i64, _i32, _f32, _i32, _p, _p, _p, _p, _p], _i32),
    "ldpc_codeset_set_layout": ([_p, _i32, _i32, _i32], _i32),
    "ldpc_decode_layouts": ([_p, _i32, _i32, _i32, _i32, _p, _i32], _i32),
    "ldpc_set_decode_layout": ([_p, _i32, _i32, _i32, _i32, _p], _i32),
    "ldpc_codeset_autotune": ([_p, _i32, _p, _p, _p, _i64, _i64, _i32, _p, _p, _p, C.c_size_t, _p, _p, _p], _i32),
    "ldpc_decode_flood_f32": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _f32, _i32, _p, _p, _p, _p, _p], _i32),
    "ldpc_decode_flood_i8": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p], _i32),
    "ldpc_decode_q16": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p], _i32),
    "ldpc_quantize_q16": ([_p, _p, _i64, _f32, _i32, _p], _i32),
    "ldpc_encode_packed": ([_p, _i32, _i32, _i32, _p, _p, _i64, _p], _i32),
    "ldpc_shift_packed": ([_p, _p, _i64, _i32, _i32, _p], _i32),
    "ldpc_decode_f32_packed": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _f32, _i32, _p, _p, _p, _p, _p, _p], _i32),
    "ldpc_decode_i8_packed": ([_p, _i32, _i32, _i32, _p, _i64, _i32, _i32, _i32, _p, _i32, _p, _p, _p, _p, _p],
                              _i32),
    "ldpc_last_error": ([], C.c_char_p),
    "ldpc_cache_clear": ([], None),
}

_lock = threading.Lock()
_lib = None


class LdpcError(RuntimeError):
    def __init__(self, code, name, msg):
        super().__init__(f"{name} failed with status {code}: {msg}")
        self.code = code


def lib():
    """Loads libldpc.so (built in-tree by __graft_entry__.build())."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"libldpc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
            # torch ships its own HIP runtime under the same soname; loading
            # it first makes the library bind to that one copy. Opened the
            # other way round, the process would hold two HIP runtimes and
            # device pointers from torch would be foreign to the library.
            _torch()
            L = C.CDLL(LIB_PATH)
            for name, (args, res) in EXPORTS.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
            _lib = L
    return _lib


def ldpc_last_error() -> str:
    return lib().ldpc_last_error().decode()


def ldpc_cache_clear() -> None:
    lib().ldpc_cache_clear()


def _check(rc, name):
    if rc != LDPC_OK:
        raise LdpcError(rc, name, ldpc_last_error())


def _hbm(hbm):
    h = np.ascontiguousarray(np.asarray(hbm), dtype=np.int16)
    if h.ndim != 2:
        raise ValueError("base matrix must be 2-D [Mb][Nb]")
    return h


def _hptr(h):
    return h.ctypes.data_as(C.c_void_p)


def _torch():
    import torch
    return torch


def _dev(t, dtype, name, shape=None):
    """Checks a device tensor argument and returns its address."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _opt(t, dtype, name, shape=None):
    return None if t is None else _dev(t, dtype, name, shape)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def ldpc_code_info(hbm, Z):
    """Host-only description of a code: dict with N, K, M, E, dmax, enc_y."""
    h = _hbm(hbm)
    out = np.zeros(8, np.int64)
    _check(lib().ldpc_code_info(_hptr(h), h.shape[0], h.shape[1], Z, out.ctypes.data_as(C.c_void_p)),
           "ldpc_code_info")
    return dict(N=int(out[0]), K=int(out[1]), M=int(out[2]), E=int(out[3]), dmax=int(out[4]),
                enc_y=int(out[5]), Mb=int(out[6]), Nb=int(out[7]))


def ldpc_encode(hbm, Z, info, cw=None, stream=None):
    """Direct encoder: info u8 [F][K] (GPU) -> codewords u8 [F][N] (GPU)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F = info.shape[0]
    K, N = (Nb - Mb) * Z, Nb * Z
    ip = _dev(info, torch.uint8, "info", (F, K))
    if cw is None:
        cw = torch.empty((F, N), dtype=torch.uint8, device=info.device)
    cp = _dev(cw, torch.uint8, "cw", (F, N))
    _check(lib().ldpc_encode(_hptr(h), Mb, Nb, Z, ip, cp, F, _stream(stream)), "ldpc_encode")
    return cw


def ldpc_decode_f32(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True, w=None, bits=None, post=None,
                    iters=None, ok=None, want_post=True, stream=None):
    """FP32 layered min-sum. Returns (bits u8, post f32 or None, iters i32, ok u8)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    lp = _dev(llr, torch.float32, "llr", (F, Nb * Z))
    wp = _opt(w, torch.float32, "w", (max_iter, Mb, Nb))
    bits = torch.empty((F, N), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.float32, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_f32(_hptr(h), Mb, Nb, Z, lp, F, int(max_iter), float(alpha), int(bool(early_term)), wp,
                                 _dev(bits, torch.uint8, "bits", (F, N)), _opt(post, torch.float32, "post", (F, N)),
                                 _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)),
                                 _stream(stream)), "ldpc_decode_f32")
    return bits, post, iters, ok


def ldpc_decode_i8(hbm, Z, llr, max_iter=10, offset=1, wq=0, wq_table=None, early_term=True, bits=None,
                   post=None, iters=None, ok=None, want_post=True, stream=None):
    """Saturating int8/int16 layered min-sum. Returns (bits u8, post i16 or None, iters i32, ok u8)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    lp = _dev(llr, torch.int8, "llr", (F, Nb * Z))
    tp = _opt(wq_table, torch.uint8, "wq_table", (max_iter, Mb, Nb))
    bits = torch.empty((F, N), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.int16, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_i8(_hptr(h), Mb, Nb, Z, lp, F, int(max_iter), int(offset), int(wq), tp,
                                int(bool(early_term)), _dev(bits, torch.uint8, "bits", (F, N)),
                                _opt(post, torch.int16, "post", (F, N)), _dev(iters, torch.int32, "iters", (F,)),
                                _opt(ok, torch.uint8, "ok", (F,)), _stream(stream)), "ldpc_decode_i8")
    return bits, post, iters, ok


def ldpc_decode_f32_packed(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True, w=None, bits=None, post=None,
                           iters=None, ok=None, want_post=False, stream=None):
    """ldpc_decode_f32 with hard bits packed eight per byte (u8 [F][ceil(N/8)])."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    nb8 = (N + 7) // 8
    bits = torch.empty((F, nb8), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.float32, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_f32_packed(_hptr(h), Mb, Nb, Z, _dev(llr, torch.float32, "llr", (F, Nb * Z)), F,
                                        int(max_iter), float(alpha), int(bool(early_term)),
                                        _opt(w, torch.float32, "w", (max_iter, Mb, Nb)),
                                        _dev(bits, torch.uint8, "bits", (F, nb8)),
                                        _opt(post, torch.float32, "post", (F, N)),
                                        _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)),
                                        _stream(stream)), "ldpc_decode_f32_packed")
    return bits, post, iters, ok


def ldpc_decode_i8_packed(hbm, Z, llr, max_iter=10, offset=1, wq=0, wq_table=None, early_term=True, bits=None,
                          post=None, iters=None, ok=None, want_post=False, stream=None):
    """ldpc_decode_i8 with hard bits packed eight per byte (u8 [F][ceil(N/8)])."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    nb8 = (N + 7) // 8
    bits = torch.empty((F, nb8), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.int16, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_i8_packed(_hptr(h), Mb, Nb, Z, _dev(llr, torch.int8, "llr", (F, Nb * Z)), F,
                                       int(max_iter), int(offset), int(wq),
                                       _opt(wq_table, torch.uint8, "wq_table", (max_iter, Mb, Nb)),
                                       int(bool(early_term)), _dev(bits, torch.uint8, "bits", (F, nb8)),
                                       _opt(post, torch.int16, "post", (F, N)), _dev(iters, torch.int32, "iters", (F,)),
                                       _opt(ok, torch.uint8, "ok", (F,)), _stream(stream)), "ldpc_decode_i8_packed")
    return bits, post, iters, ok


def ldpc_decode_flood_f32(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True, bits=None, post=None, iters=None,
                          ok=None, want_post=True, stream=None):
    """Flooding (two-phase) normalised min-sum, FP32. Returns (bits, post or None, iters, ok)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    bits = torch.empty((F, N), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.float32, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_flood_f32(_hptr(h), Mb, Nb, Z, _dev(llr, torch.float32, "llr", (F, Nb * Z)), F,
                                       int(max_iter), float(alpha), int(bool(early_term)),
                                       _dev(bits, torch.uint8, "bits", (F, N)), _opt(post, torch.float32, "post", (F, N)),
                                       _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)),
                                       _stream(stream)), "ldpc_decode_flood_f32")
    return bits, post, iters, ok


def ldpc_decode_flood_i8(hbm, Z, llr, max_iter=10, offset=1, wq=0, early_term=True, bits=None, post=None, iters=None,
                         ok=None, want_post=True, stream=None):
    """Flooding schedule on the saturating int8/int16 path. Returns (bits, post i16 or None, iters, ok)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    bits = torch.empty((F, N), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.int16, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_flood_i8(_hptr(h), Mb, Nb, Z, _dev(llr, torch.int8, "llr", (F, Nb * Z)), F,
                                      int(max_iter), int(offset), int(wq), int(bool(early_term)),
                                      _dev(bits, torch.uint8, "bits", (F, N)), _opt(post, torch.int16, "post", (F, N)),
                                      _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)),
                                      _stream(stream)), "ldpc_decode_flood_i8")
    return bits, post, iters, ok


def ldpc_encode_packed(hbm, Z, info, out=None, stream=None):
    """Direct encoder on packed bits (LSB-first bytes): info u8 [F][ceil(K/8)]
    -> codewords u8 [F][ceil(N/8)]."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F = info.shape[0]
    N, K = Nb * Z, (Nb - Mb) * Z
    out = torch.empty((F, (N + 7) // 8), dtype=torch.uint8, device=info.device) if out is None else out
    _check(lib().ldpc_encode_packed(_hptr(h), Mb, Nb, Z, _dev(info, torch.uint8, "info", (F, (K + 7) // 8)),
                                    _dev(out, torch.uint8, "out", (F, (N + 7) // 8)), F, _stream(stream)),
           "ldpc_encode_packed")
    return out


def ldpc_shift_packed(blocks, Z, s, out=None, stream=None):
    """Cyclic shift of packed Z-bit blocks u8 [F][ceil(Z/8)]: out[r] = in[(r + s) mod Z]."""
    torch = _torch()
    F = blocks.shape[0]
    out = torch.empty_like(blocks) if out is None else out
    _check(lib().ldpc_shift_packed(_dev(blocks, torch.uint8, "blocks", (F, (Z + 7) // 8)),
                                   _dev(out, torch.uint8, "out", (F, (Z + 7) // 8)), F, int(Z), int(s),
                                   _stream(stream)), "ldpc_shift_packed")
    return out


def ldpc_quantize_q16(llr, scale=16.0, qmax=1023, out=None, stream=None):
    """Q_B-bit LLRs in int16 (Q_B = 10: qmax = 1023): clamp(rint(scale * llr), +-qmax)."""
    torch = _torch()
    out = torch.empty(llr.shape, dtype=torch.int16, device=llr.device) if out is None else out
    _check(lib().ldpc_quantize_q16(_dev(llr, torch.float32, "llr"), _dev(out, torch.int16, "out", tuple(llr.shape)),
                                   llr.numel(), float(scale), int(qmax), _stream(stream)), "ldpc_quantize_q16")
    return out


def ldpc_decode_q16(hbm, Z, llr, max_iter=10, wq=12, wrap=True, early_term=True, bits=None, post=None, iters=None,
                    ok=None, want_post=True, stream=None):
    """The paper's int16 fixed point (wrap-around, or saturating with wrap=False).
    Returns (bits, post i16 or None, iters, ok)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    dev = llr.device
    bits = torch.empty((F, N), dtype=torch.uint8, device=dev) if bits is None else bits
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.int16, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
    ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
    _check(lib().ldpc_decode_q16(_hptr(h), Mb, Nb, Z, _dev(llr, torch.int16, "llr", (F, Nb * Z)), F, int(max_iter),
                                 int(wq), int(bool(wrap)), int(bool(early_term)),
                                 _dev(bits, torch.uint8, "bits", (F, N)), _opt(post, torch.int16, "post", (F, N)),
                                 _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)),
                                 _stream(stream)), "ldpc_decode_q16")
    return bits, post, iters, ok


# tuning paths: the two arithmetic paths, and each with a weight table
_TUNE_PATHS = {"f32": 0, "i8": 1, "f32w": 2, "i8w": 3}


def ldpc_autotune_decode(hbm, Z, path="f32", max_iter=10, F=16384, stream=None):
    """Times candidate decode layouts for this code and keeps the fastest;
    path "f32" / "i8", or "f32w" / "i8w" for the kernels with a weight table.
    Returns dict(G, KF, FWp, threads, hoist, h2, waves, ms); h2 = 1: two
    frames per lane in packed FP16 (fixed point), G frame pairs per
    workgroup; waves: occupancy target the kernel was compiled for (0: none)."""
    h = _hbm(hbm)
    out = np.zeros(7, np.int32)
    ms = np.zeros(1, np.float32)
    p = _TUNE_PATHS[path]
    _check(lib().ldpc_autotune_decode(_hptr(h), h.shape[0], h.shape[1], Z, p, int(max_iter), int(F),
                                      out.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p),
                                      _stream(stream)), "ldpc_autotune_decode")
    return dict(G=int(out[0]), KF=int(out[1]), FWp=int(out[2]), threads=int(out[3]), hoist=int(out[4]),
                h2=int(out[5]), waves=int(out[6]), ms=float(ms[0]))


_LAYOUT_KEYS = ("G", "KF", "FWp", "threads", "hoist", "h2", "waves")


def ldpc_decode_layouts(hbm, Z, path="f32"):
    """Every layout the decode autotuner times for this code and path, as
    dicts with the keys of ldpc_autotune_decode (compiles each candidate)."""
    h = _hbm(hbm)
    p = _TUNE_PATHS[path]
    n = lib().ldpc_decode_layouts(_hptr(h), h.shape[0], h.shape[1], Z, p, None, 0)
    if n < 0:
        _check(n, "ldpc_decode_layouts")
    out = np.zeros((max(n, 1), 7), np.int32)
    m = lib().ldpc_decode_layouts(_hptr(h), h.shape[0], h.shape[1], Z, p, out.ctypes.data_as(C.c_void_p), n)
    if m < 0:
        _check(m, "ldpc_decode_layouts")
    return [dict(zip(_LAYOUT_KEYS, (int(v) for v in row))) for row in out[:n]]


def ldpc_set_decode_layout(hbm, Z, path, layout):
    """Makes `layout` (a dict with the keys of ldpc_autotune_decode, or None
    for the default) the decode layout of this code and path."""
    h = _hbm(hbm)
    p = _TUNE_PATHS[path]
    arr = None
    if layout is not None:
        arr = np.array([int(layout[k]) for k in _LAYOUT_KEYS], np.int32)
    _check(lib().ldpc_set_decode_layout(_hptr(h), h.shape[0], h.shape[1], Z, p,
                                        None if arr is None else arr.ctypes.data_as(C.c_void_p)),
           "ldpc_set_decode_layout")


def ldpc_quantize_i8(llr, scale=4.0, out=None, stream=None):
    torch = _torch()
    out = torch.empty(llr.shape, dtype=torch.int8, device=llr.device) if out is None else out
    _check(lib().ldpc_quantize_i8(_dev(llr, torch.float32, "llr"), _dev(out, torch.int8, "q", llr.shape),
                                  llr.numel(), float(scale), _stream(stream)), "ldpc_quantize_i8")
    return out


def ldpc_quantize_weights(w, out=None, stream=None):
    """1/16-step weights of the fixed-point decoder: u8 clamp(rint(16 w), 0, 31)."""
    torch = _torch()
    out = torch.empty(w.shape, dtype=torch.uint8, device=w.device) if out is None else out
    _check(lib().ldpc_quantize_weights(_dev(w, torch.float32, "w"), _dev(out, torch.uint8, "wq", w.shape), w.numel(),
                                       _stream(stream)), "ldpc_quantize_weights")
    return out


def _seed(seed):
    """(host seed, device seed address): `seed` is an int, or a GPU int64
    tensor of one element whose bits the kernel reads as the u64 seed."""
    torch = _torch()
    if isinstance(seed, torch.Tensor):
        return 0, _dev(seed, torch.int64, "seed", (1,))
    return int(seed) & 0xFFFFFFFFFFFFFFFF, None


def ldpc_random_bits(seed, F, K, out=None, device="cuda", stream=None):
    """Seeded information bits [F][K]; seed is an int or a one-element GPU
    int64 tensor read by the kernel (graph replays with new seeds)."""
    torch = _torch()
    out = torch.empty((F, K), dtype=torch.uint8, device=device) if out is None else out
    hs, ds = _seed(seed)
    _check(lib().ldpc_random_bits(hs, ds, F, K, _dev(out, torch.uint8, "info", (F, K)), _stream(stream)),
           "ldpc_random_bits")
    return out


def ldpc_awgn_llr(seed, cw, sigma, scale, out=None, stream=None):
    """BPSK/AWGN channel LLRs for codewords cw [F][N]. sigma and scale are
    floats, or GPU float32 tensors [F] of per-frame values; seed as for
    ldpc_random_bits."""
    torch = _torch()
    F, N = cw.shape
    out = torch.empty((F, N), dtype=torch.float32, device=cw.device) if out is None else out
    sf = cf = None
    if isinstance(sigma, torch.Tensor):
        sf, cf = _dev(sigma, torch.float32, "sigma", (F,)), _dev(scale, torch.float32, "scale", (F,))
        sigma = scale = 0.0
    hs, ds = _seed(seed)
    _check(lib().ldpc_awgn_llr(hs, ds, _dev(cw, torch.uint8, "cw", (F, N)), F, N, float(sigma), float(scale),
                               sf, cf, _dev(out, torch.float32, "llr", (F, N)), _stream(stream)), "ldpc_awgn_llr")
    return out


def ldpc_frame_stats(bits, info, iters=None, ok=None, counters=None, stream=None):
    """Adds (info-bit errors, frame errors, iterations, failed syndromes) of a
    decoded batch to int64 device counters [4]; returns the counters."""
    torch = _torch()
    F, N = bits.shape
    K = info.shape[1]
    if counters is None:
        counters = torch.zeros(4, dtype=torch.int64, device=bits.device)
    _check(lib().ldpc_frame_stats(_dev(bits, torch.uint8, "bits", (F, N)), _dev(info, torch.uint8, "info", (F, K)),
                                  _opt(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)), F, N, K,
                                  _dev(counters, torch.int64, "counters", (4,)), _stream(stream)), "ldpc_frame_stats")
    return counters


def ldpc_lds_probe(blocks, rounds, out=None, stream=None):
    """LDS read bandwidth probe (blocks * 256 * rounds * 128 bytes read);
    returns the checksum buffer f32 [blocks * 256]."""
    torch = _torch()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda") if out is None else out
    _check(lib().ldpc_lds_probe(int(blocks), int(rounds), _dev(out, torch.float32, "out", (blocks * 256,)),
                                _stream(stream)), "ldpc_lds_probe")
    return out


def _work(F, device):
    return _torch().empty(F + 1, dtype=_torch().int64, device=device)


def ldpc_fallback_f32(hbm, Z, llr, bits, iters, ok, post=None, max_iter=20, alpha=0.75, work=None, stream=None):
    """Re-decodes frames with ok == 0 by plain FP32 NMS (in place)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    work = _work(F, llr.device) if work is None else work
    _check(lib().ldpc_fallback_f32(_hptr(h), Mb, Nb, Z, _dev(llr, torch.float32, "llr", (F, Nb * Z)), F,
                                   int(max_iter), float(alpha), _dev(bits, torch.uint8, "bits", (F, N)),
                                   _opt(post, torch.float32, "post", (F, N)), _dev(iters, torch.int32, "iters", (F,)),
                                   _dev(ok, torch.uint8, "ok", (F,)), _dev(work, torch.int64, "work", (F + 1,)),
                                   _stream(stream)), "ldpc_fallback_f32")
    return bits, post, iters, ok


def ldpc_fallback_i8(hbm, Z, llr, bits, iters, ok, post=None, max_iter=20, offset=0, wq=12, work=None, stream=None):
    """Re-decodes frames with ok == 0 by plain fixed-point min-sum (in place)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    work = _work(F, llr.device) if work is None else work
    _check(lib().ldpc_fallback_i8(_hptr(h), Mb, Nb, Z, _dev(llr, torch.int8, "llr", (F, Nb * Z)), F, int(max_iter),
                                  int(offset), int(wq), _dev(bits, torch.uint8, "bits", (F, N)),
                                  _opt(post, torch.int16, "post", (F, N)), _dev(iters, torch.int32, "iters", (F,)),
                                  _dev(ok, torch.uint8, "ok", (F,)), _dev(work, torch.int64, "work", (F + 1,)),
                                  _stream(stream)), "ldpc_fallback_i8")
    return bits, post, iters, ok


def ldpc_nms_ckpt_bytes(hbm, Z, F, T):
    h = _hbm(hbm)
    n = lib().ldpc_nms_ckpt_bytes(_hptr(h), h.shape[0], h.shape[1], Z, int(F), int(T))
    if n == 0:
        raise LdpcError(LDPC_EINVAL, "ldpc_nms_ckpt_bytes", "invalid code or sizes")
    return int(n)


def ldpc_nms_fwd(hbm, Z, llr, cw, w, ckpt=None, post=None, want_post=False, stream=None):
    """Training forward of the learned decoder (T = w.shape[0] iterations).
    Returns (loss [T] f32 on the device, checkpoint buffer u8, post or None)."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = llr.shape
    T = w.shape[0]
    nbytes = ldpc_nms_ckpt_bytes(h, Z, F, T)
    if ckpt is None:
        ckpt = torch.empty(nbytes, dtype=torch.uint8, device=llr.device)
    if post is None and want_post:
        post = torch.empty((F, N), dtype=torch.float32, device=llr.device)
    loss = torch.empty(T, dtype=torch.float32, device=llr.device)
    _check(lib().ldpc_nms_fwd(_hptr(h), Mb, Nb, Z, _dev(llr, torch.float32, "llr", (F, Nb * Z)),
                              _dev(cw, torch.uint8, "cw", (F, N)), F, T, _dev(w, torch.float32, "w", (T, Mb, Nb)),
                              _dev(ckpt, torch.uint8, "ckpt"), ckpt.numel(), _dev(loss, torch.float32, "loss"),
                              _opt(post, torch.float32, "post", (F, N)), _stream(stream)), "ldpc_nms_fwd")
    return loss, ckpt, post


def ldpc_nms_bwd(hbm, Z, cw, w, ckpt, dloss, grad_w=None, stream=None):
    """Adjoint of ldpc_nms_fwd: gradient of sum_t dloss[t] * loss[t] w.r.t. w."""
    torch = _torch()
    h = _hbm(hbm)
    Mb, Nb = h.shape
    F, N = cw.shape
    T = w.shape[0]
    if grad_w is None:
        grad_w = torch.empty((T, Mb, Nb), dtype=torch.float32, device=cw.device)
    _check(lib().ldpc_nms_bwd(_hptr(h), Mb, Nb, Z, _dev(cw, torch.uint8, "cw", (F, N)), F, T,
                              _dev(w, torch.float32, "w", (T, Mb, Nb)), _dev(ckpt, torch.uint8, "ckpt"), ckpt.numel(),
                              _dev(dloss, torch.float32, "dloss", (T,)),
                              _dev(grad_w, torch.float32, "grad_w", (T, Mb, Nb)), _stream(stream)), "ldpc_nms_bwd")
    return grad_w


class Codeset:
    """Several codes decoded together by the batched persistent kernel
    (ldpc_codeset_create / ldpc_decode_batch_*). codes: list of (hbm, Z)."""

    def __init__(self, codes):
        self._h = [_hbm(h) for h, _ in codes]
        n = len(self._h)
        ptrs = (C.c_void_p * n)(*[h.ctypes.data for h in self._h])
        Mb = (C.c_int * n)(*[h.shape[0] for h in self._h])
        Nb = (C.c_int * n)(*[h.shape[1] for h in self._h])
        Zs = (C.c_int * n)(*[int(z) for _, z in codes])
        handle = C.c_void_p()
        _check(lib().ldpc_codeset_create(ptrs, Mb, Nb, Zs, n, C.byref(handle)), "ldpc_codeset_create")
        self._cs = handle
        self.n = n
        self.info = []
        out = np.zeros(8, np.int64)
        for c in range(n):
            _check(lib().ldpc_codeset_info(self._cs, c, out.ctypes.data_as(C.c_void_p)), "ldpc_codeset_info")
            self.info.append(dict(N=int(out[0]), K=int(out[1]), M=int(out[2]), E=int(out[3]), dmax=int(out[4]),
                                  cls=int(out[5]), G=int(out[6]), nclass=int(out[7])))

    def __del__(self):
        cs, self._cs = getattr(self, "_cs", None), None
        if cs and _lib is not None:
            _lib.ldpc_codeset_destroy(cs)

    def work_bytes(self, F):
        return int(lib().ldpc_batch_work_bytes(self._cs, int(F)))

    def _decode(self, name, code_id, off, llr, total, F, args_mid, bits, post, iters, ok, work, stream, llr_dtype,
                post_dtype, want_post):
        torch = _torch()
        dev = llr.device
        if work is None:
            work = torch.empty(self.work_bytes(F), dtype=torch.uint8, device=dev)
        bits = torch.empty(total, dtype=torch.uint8, device=dev) if bits is None else bits
        if post is None and want_post:
            post = torch.empty(total, dtype=post_dtype, device=dev)
        iters = torch.empty(F, dtype=torch.int32, device=dev) if iters is None else iters
        ok = torch.empty(F, dtype=torch.uint8, device=dev) if ok is None else ok
        fn = getattr(lib(), name)
        _check(fn(self._cs, _dev(code_id, torch.int32, "code_id", (F,)), _dev(off, torch.int64, "off", (F,)),
                  _dev(llr, llr_dtype, "llr", (total,)), total, F, *args_mid, _dev(bits, torch.uint8, "bits", (total,)),
                  _opt(post, post_dtype, "post", (total,)), _dev(iters, torch.int32, "iters", (F,)),
                  _opt(ok, torch.uint8, "ok", (F,)), _dev(work, torch.uint8, "work"), work.numel(),
                  _stream(stream)), name)
        return bits, post, iters, ok

    def decode_f32(self, code_id, off, llr, max_iter=10, alpha=0.75, early_term=True, bits=None, post=None,
                   iters=None, ok=None, work=None, want_post=True, stream=None):
        """Ragged batch: frame f of code code_id[f] occupies llr[off[f] : off[f] + N]."""
        torch = _torch()
        return self._decode("ldpc_decode_batch_f32", code_id, off, llr, llr.numel(), code_id.numel(),
                            (int(max_iter), float(alpha), int(bool(early_term))), bits, post, iters, ok, work, stream,
                            torch.float32, torch.float32, want_post)

    def decode_f32_noalloc(self, code_id, off, llr, bits, iters, post=None, ok=None, max_iter=10, alpha=0.75,
                           early_term=True, stream=None):
        """ldpc_decode_batch_f32_noalloc: as decode_f32, into the caller's
        output tensors (bits, iters; post and ok optional), with the work list
        in the library's static device scratch; neither the binding nor the
        library allocates device memory."""
        torch = _torch()
        F, total = code_id.numel(), llr.numel()
        _check(lib().ldpc_decode_batch_f32_noalloc(
            self._cs, _dev(code_id, torch.int32, "code_id", (F,)), _dev(off, torch.int64, "off", (F,)),
            _dev(llr, torch.float32, "llr", (total,)), total, F, int(max_iter), float(alpha), int(bool(early_term)),
            _dev(bits, torch.uint8, "bits", (total,)), _opt(post, torch.float32, "post", (total,)),
            _dev(iters, torch.int32, "iters", (F,)), _opt(ok, torch.uint8, "ok", (F,)), _stream(stream)),
            "ldpc_decode_batch_f32_noalloc")
        return bits, post, iters, ok

    def autotune(self, path, code_id, off, llr, max_iter=10, work=None, stream=None):
        """Times the batch layouts on this batch (ldpc_codeset_autotune) and keeps
        the fastest for `path` ("f32" or "i8"). Returns dict(threads, divisor, ms)."""
        torch = _torch()
        F = code_id.numel()
        p = {"f32": 0, "i8": 1}[path]
        dev = llr.device
        work = torch.empty(self.work_bytes(F), dtype=torch.uint8, device=dev) if work is None else work
        bits = torch.empty(llr.numel(), dtype=torch.uint8, device=dev)
        iters = torch.empty(F, dtype=torch.int32, device=dev)
        out = np.zeros(2, np.int32)
        ms = C.c_float()
        _check(lib().ldpc_codeset_autotune(self._cs, p, _dev(code_id, torch.int32, "code_id", (F,)),
                                           _dev(off, torch.int64, "off", (F,)),
                                           _dev(llr, torch.float32 if p == 0 else torch.int8, "llr"),
                                           llr.numel(), F, int(max_iter), _dev(bits, torch.uint8, "bits"),
                                           _dev(iters, torch.int32, "iters"), _dev(work, torch.uint8, "work"),
                                           work.numel(), out.ctypes.data_as(C.c_void_p), C.byref(ms),
                                           _stream(stream)), "ldpc_codeset_autotune")
        return dict(threads=int(out[0]), divisor=int(out[1]), ms=float(ms.value))

    def set_layout(self, path, threads, divisor=1):
        """Makes one of the batch autotuner's layouts (threads, divisor) the
        layout of later batched decodes of `path` (ldpc_codeset_set_layout)."""
        p = {"f32": 0, "i8": 1}[path]
        _check(lib().ldpc_codeset_set_layout(self._cs, p, int(threads), int(divisor)), "ldpc_codeset_set_layout")

    def decode_i8(self, code_id, off, llr, max_iter=10, offset=1, wq=0, early_term=True, bits=None, post=None,
                  iters=None, ok=None, work=None, want_post=True, stream=None):
        torch = _torch()
        return self._decode("ldpc_decode_batch_i8", code_id, off, llr, llr.numel(), code_id.numel(),
                            (int(max_iter), int(offset), int(wq), int(bool(early_term))), bits, post, iters, ok,
                            work, stream, torch.int8, torch.int16, want_post)
