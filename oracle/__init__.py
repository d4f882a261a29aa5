"""CPU oracle for the QC-LDPC direct encoder and layered min-sum decoder.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers. The product library never imports,
links or runs anything from this package. The arithmetic lives in the plain C
file next to this one (oracle.c); this module only marshals numpy arrays.

Each function names the part of the paper it follows; see oracle.c for the
definitions written out.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lock = threading.Lock()
_lib = None

ORC_OK, ORC_EINVAL, ORC_ESTRUCT, ORC_ENOMEM = 0, -1, -2, -5


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def lib():
    """Loads liboracle.so, building it first if it is not there."""
    global _lib
    with _lock:
        if _lib is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
            L = C.CDLL(path)
            p = C.c_void_p
            i32, i64, f32, f64, u64 = C.c_int, C.c_int64, C.c_float, C.c_double, C.c_uint64
            sig = {
                "orc_code_edges": [p, i32, i32, i32, p, p],
                "orc_encode": [p, i32, i32, i32, p, p, i64],
                "orc_syndrome_ok": [p, i32, i32, i32, p, i64, p],
                "orc_decode_f32": [p, i32, i32, i32, p, i64, i32, f32, i32, p, p, p, p, p],
                "orc_decode_f64": [p, i32, i32, i32, p, i64, i32, f64, i32, p, p, p, p, p],
                "orc_decode_i8": [p, i32, i32, i32, p, i64, i32, i32, i32, p, i32, p, p, p, p],
                "orc_decode_flood_f32": [p, i32, i32, i32, p, i64, i32, f32, i32, p, p, p, p],
                "orc_decode_flood_f64": [p, i32, i32, i32, p, i64, i32, f64, i32, p, p, p, p],
                "orc_decode_flood_i8": [p, i32, i32, i32, p, i64, i32, i32, i32, i32, p, p, p, p],
                "orc_quantize_i8": [p, p, i64, f32],
                "orc_quantize_weights": [p, p, i64],
                "orc_decode_q16": [p, i32, i32, i32, p, i64, i32, i32, i32, i32, p, p, p, p],
                "orc_quantize_q16": [p, p, i64, f32, i32],
                "orc_shift_packed": [p, p, i64, i32, i32],
                "orc_encode_packed": [p, i32, i32, i32, p, p, i64],
                "orc_nms_train": [p, i32, i32, i32, p, p, i64, i32, p, i32, p, p, p],
                "orc_frame_bits": [u64, i64, i64, p],
                "orc_frame_noise": [u64, i64, i64, p],
                "orc_channel": [p, p, i64, f32, f32, p],
            }
            for name, args in sig.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = C.c_int
            L.orc_philox4x32_10.argtypes = [p, p, p]
            L.orc_philox4x32_10.restype = None
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _hbm(hbm):
    h = np.ascontiguousarray(hbm, dtype=np.int16)
    if h.ndim != 2:
        raise ValueError("base matrix must be 2-D")
    return h


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(rc, what)


def code_edges(hbm, Z):
    """(E, max block-row degree) of the expanded code (Sec. 1)."""
    h = _hbm(hbm)
    e = np.zeros(1, np.int64)
    d = np.zeros(1, np.int32)
    _check(lib().orc_code_edges(_ptr(h), h.shape[0], h.shape[1], Z, _ptr(e), _ptr(d)), "code_edges")
    return int(e[0]), int(d[0])


def encode(hbm, Z, info):
    """Direct encoder, eqs. (12)-(15): info u8 [F][K] -> codeword u8 [F][N]."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    info = np.ascontiguousarray(info, dtype=np.uint8)
    F = info.shape[0]
    if info.shape[1] != (Nb - Mb) * Z:
        raise ValueError("info has the wrong length")
    cw = np.zeros((F, Nb * Z), np.uint8)
    _check(lib().orc_encode(_ptr(h), Mb, Nb, Z, _ptr(info), _ptr(cw), F), "encode")
    return cw


def syndrome_ok(hbm, Z, bits):
    """1 where H x = 0 for the hard-bit vector x of each frame (eq. 21)."""
    h = _hbm(hbm)
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    ok = np.zeros(bits.shape[0], np.uint8)
    _check(lib().orc_syndrome_ok(_ptr(h), h.shape[0], h.shape[1], Z, _ptr(bits), bits.shape[0], _ptr(ok)),
           "syndrome_ok")
    return ok


def _decode_fp(fn, dtype, hbm, Z, llr, max_iter, alpha, early_term, w):
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=dtype)
    F, N = llr.shape
    if N != Nb * Z:
        raise ValueError("llr has the wrong length")
    if w is not None:
        w = np.ascontiguousarray(w, dtype=dtype)
        if w.shape != (max_iter, Mb, Nb):
            raise ValueError("weight table must be [max_iter][Mb][Nb]")
    bits = np.zeros((F, N), np.uint8)
    post = np.zeros((F, N), dtype)
    iters = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    _check(fn(_ptr(h), Mb, Nb, Z, _ptr(llr), F, max_iter, alpha, int(bool(early_term)), _ptr(w),
              _ptr(bits), _ptr(post), _ptr(iters), _ptr(ok)), "decode")
    return bits, post, iters, ok


def decode_f32(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True, w=None):
    """Layered normalised min-sum in float (Sec. 4, eqs. 20-23).
    Returns (bits u8 [F][N], posteriors f32 [F][N], iterations i32 [F], ok u8 [F])."""
    return _decode_fp(lib().orc_decode_f32, np.float32, hbm, Z, llr, max_iter, alpha, early_term, w)


def decode_f64(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True, w=None):
    """The same decoder evaluated in double."""
    return _decode_fp(lib().orc_decode_f64, np.float64, hbm, Z, llr, max_iter, alpha, early_term, w)


def decode_i8(hbm, Z, llr, max_iter=10, offset=1, wq=0, wq_table=None, early_term=True):
    """Saturating fixed-point layered min-sum: int8 LLRs and messages, int16
    posteriors. wq = 0 selects offset min-sum, wq > 0 the weight wq/16.
    Returns (bits u8, posteriors i16, iterations i32, ok u8)."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=np.int8)
    F, N = llr.shape
    if N != Nb * Z:
        raise ValueError("llr has the wrong length")
    if wq_table is not None:
        wq_table = np.ascontiguousarray(wq_table, dtype=np.uint8)
        if wq_table.shape != (max_iter, Mb, Nb):
            raise ValueError("weight table must be [max_iter][Mb][Nb]")
    bits = np.zeros((F, N), np.uint8)
    post = np.zeros((F, N), np.int16)
    iters = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    _check(lib().orc_decode_i8(_ptr(h), Mb, Nb, Z, _ptr(llr), F, max_iter, offset, wq, _ptr(wq_table),
                               int(bool(early_term)), _ptr(bits), _ptr(post), _ptr(iters), _ptr(ok)),
           "decode_i8")
    return bits, post, iters, ok


def _flood_fp(fn, dtype, hbm, Z, llr, max_iter, alpha, early_term):
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=dtype)
    F, N = llr.shape
    if N != Nb * Z:
        raise ValueError("llr has the wrong length")
    bits = np.zeros((F, N), np.uint8)
    post = np.zeros((F, N), dtype)
    iters = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    _check(fn(_ptr(h), Mb, Nb, Z, _ptr(llr), F, max_iter, alpha, int(bool(early_term)), _ptr(bits), _ptr(post),
              _ptr(iters), _ptr(ok)), "decode_flood")
    return bits, post, iters, ok


def decode_flood_f32(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True):
    """Flooding (two-phase) normalised min-sum in float (Sec. 4, eqs. 18-23
    without layering). Returns (bits, posteriors f32, iterations, ok)."""
    return _flood_fp(lib().orc_decode_flood_f32, np.float32, hbm, Z, llr, max_iter, alpha, early_term)


def decode_flood_f64(hbm, Z, llr, max_iter=10, alpha=0.75, early_term=True):
    """The flooding decoder evaluated in double."""
    return _flood_fp(lib().orc_decode_flood_f64, np.float64, hbm, Z, llr, max_iter, alpha, early_term)


def decode_flood_i8(hbm, Z, llr, max_iter=10, offset=1, wq=0, early_term=True):
    """Flooding schedule on the saturating fixed-point path (int8 LLRs and
    messages, int16 posteriors). Returns (bits, posteriors i16, iterations, ok)."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=np.int8)
    F, N = llr.shape
    if N != Nb * Z:
        raise ValueError("llr has the wrong length")
    bits = np.zeros((F, N), np.uint8)
    post = np.zeros((F, N), np.int16)
    iters = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    _check(lib().orc_decode_flood_i8(_ptr(h), Mb, Nb, Z, _ptr(llr), F, max_iter, offset, wq,
                                     int(bool(early_term)), _ptr(bits), _ptr(post), _ptr(iters), _ptr(ok)),
           "decode_flood_i8")
    return bits, post, iters, ok


def decode_q16(hbm, Z, llr, max_iter=10, wq=12, wrap=True, early_term=True):
    """The paper's fixed point (Sec. 5): layered min-sum on int16 values with
    wrap-around (wrap=True) or symmetric saturating arithmetic, normalisation
    wq/16. llr: int16 [F][N] (Q_B-bit values). Returns (bits, posteriors i16,
    iterations, ok)."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=np.int16)
    F, N = llr.shape
    if N != Nb * Z:
        raise ValueError("llr has the wrong length")
    bits = np.zeros((F, N), np.uint8)
    post = np.zeros((F, N), np.int16)
    iters = np.zeros(F, np.int32)
    ok = np.zeros(F, np.uint8)
    _check(lib().orc_decode_q16(_ptr(h), Mb, Nb, Z, _ptr(llr), F, max_iter, wq, int(bool(wrap)),
                                int(bool(early_term)), _ptr(bits), _ptr(post), _ptr(iters), _ptr(ok)), "decode_q16")
    return bits, post, iters, ok


def quantize_q16(llr, scale=16.0, qmax=1023):
    """Q_B-bit quantiser (Q_B = 10: qmax = 1023): clamp(rint(scale * llr), +-qmax)."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    q = np.zeros(llr.shape, np.int16)
    _check(lib().orc_quantize_q16(_ptr(llr), _ptr(q), llr.size, scale, qmax), "quantize_q16")
    return q


def shift_packed(blocks, Z, s):
    """Cyclic shift of packed Z-bit blocks (LSB-first bytes, [F][ceil(Z/8)]):
    out[r] = in[(r + s) mod Z]."""
    blocks = np.ascontiguousarray(blocks, dtype=np.uint8)
    out = np.zeros_like(blocks)
    _check(lib().orc_shift_packed(_ptr(blocks), _ptr(out), blocks.shape[0], Z, s), "shift_packed")
    return out


def encode_packed(hbm, Z, info_packed):
    """Direct encoder on packed bits (LSB-first): info [F][ceil(K/8)] -> cw [F][ceil(N/8)]."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    info_packed = np.ascontiguousarray(info_packed, dtype=np.uint8)
    F = info_packed.shape[0]
    cw = np.zeros((F, (Nb * Z + 7) // 8), np.uint8)
    _check(lib().orc_encode_packed(_ptr(h), Mb, Nb, Z, _ptr(info_packed), _ptr(cw), F), "encode_packed")
    return cw


def quantize_weights(w):
    """1/16-step weights of the fixed-point decoder: clamp(rint(16 w), 0, 31),
    half to even; NaN -> 0 (oracle.c orc_quantize_weights)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    q = np.zeros(w.shape, np.uint8)
    _check(lib().orc_quantize_weights(_ptr(w), _ptr(q), w.size), "quantize_weights")
    return q


def quantize_i8(llr, scale=4.0):
    """q = clamp(rint(scale * llr), -127, 127), half to even."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    q = np.zeros(llr.shape, np.int8)
    _check(lib().orc_quantize_i8(_ptr(llr), _ptr(q), llr.size, scale), "quantize_i8")
    return q


def nms_train(hbm, Z, llr, cw, w, fwd_f32=False, grad=True, post=False):
    """Learned normalised min-sum: loss summed over iterations (per-iteration
    shares returned) and, if grad, its gradient w.r.t. w [T][Mb][Nb].
    Returns (loss_per_iter [T], grad [T][Mb][Nb] or None, post [F][N] or None)."""
    h = _hbm(hbm)
    Mb, Nb = h.shape
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    cw = np.ascontiguousarray(cw, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float64)
    T = w.shape[0]
    if w.shape != (T, Mb, Nb) or llr.shape != cw.shape or llr.shape[1] != Nb * Z:
        raise ValueError("shape mismatch")
    F = llr.shape[0]
    loss = np.zeros(T, np.float64)
    g = np.zeros((T, Mb, Nb), np.float64) if grad else None
    pl = np.zeros(llr.shape, np.float64) if post else None
    _check(lib().orc_nms_train(_ptr(h), Mb, Nb, Z, _ptr(llr), _ptr(cw), F, T, _ptr(w), int(bool(fwd_f32)),
                               _ptr(loss), _ptr(g), _ptr(pl)), "nms_train")
    return loss, g, pl


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def frame_bits(seed, F, K):
    """Seeded information bits u8 [F][K] drawn from Philox4x32-10."""
    out = np.zeros((F, K), np.uint8)
    _check(lib().orc_frame_bits(seed, F, K, _ptr(out)), "frame_bits")
    return out


def frame_noise(seed, F, N):
    """Seeded standard normals f64 [F][N] (Philox4x32-10 + Box-Muller)."""
    out = np.zeros((F, N), np.float64)
    _check(lib().orc_frame_noise(seed, F, N, _ptr(out)), "frame_noise")
    return out


def channel(cw, z, sigma, scale):
    """BPSK over AWGN and the LLR, eqs. (16)-(17), in float:
    LLR = ((1 - 2x) + sigma z) * scale with scale = 2 / sigma^2."""
    cw = np.ascontiguousarray(cw, dtype=np.uint8)
    z = np.ascontiguousarray(z, dtype=np.float32)
    if cw.shape != z.shape:
        raise ValueError("shape mismatch")
    out = np.zeros(cw.shape, np.float32)
    _check(lib().orc_channel(_ptr(cw), _ptr(z), cw.size, np.float32(sigma), np.float32(scale), _ptr(out)),
           "channel")
    return out


def llr_frames(hbm, Z, F, ebn0_db, seed, info=None):
    """Convenience: encode seeded info bits and pass them through the channel.
    Returns (info, cw, llr f32). Noise comes from the shared input generator."""
    import synth
    h = _hbm(hbm)
    N, K, _ = synth.code_dims(h, Z)
    if info is None:
        info = synth.info_bits(F, K, seed)
    cw = encode(h, Z, info)
    s2 = synth.sigma2_from_ebn0(ebn0_db, K / N)
    z = synth.std_normal(F, N, seed + 7777)
    sigma = np.float32(np.sqrt(s2))
    scale = np.float32(2.0 / s2)
    return info, cw, channel(cw, z, sigma, scale)
