"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every entry point include/ldpc.h declares, code descriptions are
right, and invalid arguments are rejected before anything is enqueued."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
import paper_2306_12063_amd as P
from helpers import dense_h

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ldpc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*(ldpc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_entry_point():
    names = _declared()
    assert "ldpc_decode_f32" in names and "ldpc_encode" in names
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(P.EXPORTS) == names


def test_code_info_matches_definition():
    for rate in synth.WIFI_RATES:
        h = synth.wifi_code(rate, 81)
        info = P.ldpc_code_info(h, 81)
        H = dense_h(h, 81)
        assert info["N"] == H.shape[1] and info["M"] == H.shape[0]
        assert info["K"] == H.shape[1] - H.shape[0]
        assert info["E"] == int(H.sum())
        assert info["dmax"] == int(H.sum(axis=1).max())
        assert info["enc_y"] == (h.shape[0] - 1) // 2
    g = synth.wifi_code("1/2", 27)
    g[0, 12] = 3
    assert P.ldpc_code_info(g, 27)["enc_y"] == -1


def _call_decode(h, Z, F=0, max_iter=10):
    h = np.ascontiguousarray(h, np.int16)
    Mb, Nb = h.shape
    rc = P.lib().ldpc_decode_f32(h.ctypes.data_as(C.c_void_p), Mb, Nb, Z, None, F, max_iter, 0.75, 1, None,
                                 None, None, None, None, None)
    return rc, P.ldpc_last_error()


def test_validation_errors_without_gpu():
    h = synth.wifi_code("1/2", 27)
    assert _call_decode(h, 27, F=0)[0] == P.LDPC_OK          # empty batch is a no-op
    bad = h.copy()
    bad[2, 3] = 27
    rc, msg = _call_decode(bad, 27)
    assert rc == P.LDPC_EINVAL and "outside" in msg
    rc, _ = _call_decode(h, 27, max_iter=0)
    assert rc == P.LDPC_EINVAL
    rc, _ = _call_decode(h, 27, F=-1)
    assert rc == P.LDPC_EINVAL
    deg1 = np.full((2, 4), -1, np.int16)
    deg1[0, :2] = 0
    deg1[1, 2] = 0
    rc, msg = _call_decode(deg1, 3)
    assert rc == P.LDPC_EINVAL and "degree" in msg
    rc, _ = _call_decode(np.zeros((3, 3), np.int16), 5)      # Nb <= Mb
    assert rc == P.LDPC_EINVAL
    rc, _ = _call_decode(np.zeros((2, 40), np.int16), 5)     # too many block columns
    assert rc == P.LDPC_ERANGE
    rc, _ = _call_decode(np.zeros((2, 4), np.int16), 300)    # Z beyond the kernel limit
    assert rc == P.LDPC_ERANGE
    # the limits themselves are accepted (F = 0: validation only), one beyond is not
    assert _call_decode(np.zeros((2, 4), np.int16), 256, F=0)[0] == P.LDPC_OK
    assert _call_decode(np.zeros((2, 4), np.int16), 257, F=0)[0] == P.LDPC_ERANGE
    assert _call_decode(synth.limit_code(16, 32, 8, 18, 6, 1), 8, F=0)[0] == P.LDPC_OK
    assert _call_decode(np.zeros((17, 40), np.int16)[:, :32], 8, F=0)[0] == P.LDPC_ERANGE   # 17 block rows
    assert _call_decode(synth.limit_code(6, 32, 8, 26, 6, 1), 8, F=0)[0] == P.LDPC_OK
    deg27 = synth.limit_code(5, 32, 8, 26, 6, 1)
    deg27[0, :] = 0                                          # a block row of check degree 32
    rc, msg = _call_decode(deg27, 8, F=0)
    assert rc == P.LDPC_ERANGE and "more than 26" in msg
    L = P.lib()
    assert L.ldpc_lds_probe(0, 1, None, None) == P.LDPC_EINVAL    # the LDS probe validates on the host too
    assert L.ldpc_lds_probe(1, 1, None, None) == P.LDPC_EINVAL


def test_null_device_pointers_rejected():
    h = np.ascontiguousarray(synth.wifi_code("1/2", 27), np.int16)
    rc = P.lib().ldpc_decode_f32(h.ctypes.data_as(C.c_void_p), 12, 24, 27, None, 5, 10, 0.75, 1, None,
                                 None, None, None, None, None)
    assert rc == P.LDPC_EINVAL and "null" in P.ldpc_last_error()
    rc = P.lib().ldpc_decode_i8(h.ctypes.data_as(C.c_void_p), 12, 24, 27, None, 5, 10, 200, 0, None, 1,
                                None, None, None, None, None)
    assert rc == P.LDPC_EINVAL and "offset" in P.ldpc_last_error()
    rc = P.lib().ldpc_decode_batch_f32_noalloc(None, None, None, None, 0, 5, 10, 0.75, 1, None, None, None, None,
                                               None)
    assert rc == P.LDPC_EINVAL and "null code set" in P.ldpc_last_error()


def test_encoder_structure_rejected_without_gpu():
    h = synth.wifi_code("2/3", 27)
    h[7, 16] = 2          # h_b: bottom entry differs from the top one
    h = np.ascontiguousarray(h, np.int16)
    rc = P.lib().ldpc_encode(h.ctypes.data_as(C.c_void_p), 8, 24, 27, None, None, 4, None)
    assert rc == P.LDPC_ESTRUCT


def test_ebn0_at_fer_interpolation():
    from paper_2306_12063_amd.learned import ebn0_at_fer
    pts = [dict(ebn0=1.0, fer=1e-1), dict(ebn0=2.0, fer=1e-2), dict(ebn0=3.0, fer=1e-4)]
    assert ebn0_at_fer(pts) == pytest.approx(2.5)
    assert ebn0_at_fer(pts, target=1e-2) == pytest.approx(2.0)
    assert ebn0_at_fer(pts[:2]) is None


@pytest.mark.parametrize("code,Z,G", [(("wimax", "1/2"), 96, 2), (("wifi", "5/6"), 81, 3), (("wifi", "1/2"), 27, 7)])
def test_nms_checkpoint_size(code, Z, G):
    # the training buffer: per iteration and frame L (N floats) and the raw
    # row state (3 M), the per-frame loss terms (T F), and the adjoint's
    # per-workgroup partial gradients (T Mb Nb per workgroup of G frames; G
    # fills the most lanes of whole waves: 2 x 96 = 192, 3 x 81 = 243 of 256,
    # 7 x 27 = 189 of 192)
    h = synth.wimax_code(code[1], Z) if code[0] == "wimax" else synth.wifi_code(code[1], Z)
    Mb, Nb = h.shape
    N, M = Nb * Z, Mb * Z
    for F, T in [(4096, 10), (37, 4), (1, 1)]:
        want = 4 * (T * F * (N + 3 * M) + T * F + ((F + G - 1) // G) * T * Mb * Nb)
        assert P.ldpc_nms_ckpt_bytes(h, Z, F, T) == want


def test_no_cpu_fallback_for_host_tensors():
    # every step runs in the library's kernels: host tensors are refused
    # before any call, never decoded on the CPU
    import torch
    h = synth.wifi_code("1/2", 27)
    calls = [lambda: P.ldpc_decode_f32(h, 27, torch.zeros((4, 648))),
             lambda: P.ldpc_decode_i8(h, 27, torch.zeros((4, 648), dtype=torch.int8)),
             lambda: P.ldpc_encode(h, 27, torch.zeros((4, 324), dtype=torch.uint8)),
             lambda: P.ldpc_quantize_i8(torch.zeros(16)),
             lambda: P.ldpc_nms_fwd(h, 27, torch.zeros((4, 648)), torch.zeros((4, 648), dtype=torch.uint8),
                                    torch.full((3, 12, 24), 0.75))]
    for call in calls:
        with pytest.raises(TypeError, match="GPU tensor"):
            call()


def test_missing_library_fails_loudly(tmp_path):
    # a copy of the binding without libldpc.so: the first library call raises
    # (there is no fallback implementation to drop to)
    import shutil
    import subprocess
    import sys
    src = os.path.join(os.path.dirname(HEADER), "..", "paper_2306_12063_amd")
    dst = tmp_path / "paper_2306_12063_amd"
    dst.mkdir()
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), dst / f)
    code = ("import paper_2306_12063_amd as P\n"
            "try:\n    P.lib()\nexcept ImportError as e:\n    print('raised:', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert "raised:" in out.stdout and "not built" in out.stdout, out.stdout + out.stderr


def test_weight_quantizer_validation_without_gpu():
    L = P.lib()
    assert L.ldpc_quantize_weights(None, None, 0, None) == P.LDPC_OK    # empty: no-op
    assert L.ldpc_quantize_weights(None, None, -1, None) == P.LDPC_EINVAL
    assert L.ldpc_quantize_weights(None, None, 4, None) == P.LDPC_EINVAL
    assert "null" in P.ldpc_last_error()
