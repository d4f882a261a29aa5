"""Pins for the oracle's learned normalised min-sum: the loss against a
direct evaluation from truncated plain decodes, and the adjoint gradient
against central finite differences in double precision."""
import numpy as np
import pytest

import oracle
import synth


def _setup(rate, Z, F, T, ebn0, seed):
    h = synth.wifi_code(rate, Z)
    info, cw, llr = oracle.llr_frames(h, Z, F, ebn0, seed)
    Mb, Nb = h.shape
    return h, cw, llr.astype(np.float64), np.full((T, Mb, Nb), 0.75)


def _softplus(z):
    return np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z)))


def test_loss_equals_direct_evaluation():
    # With every weight equal to alpha the unrolled decoder is plain NMS, so
    # L after iteration t is the posterior of a plain decode truncated at t.
    h, cw, llr, w = _setup("1/2", 27, 12, 5, 1.5, 3)
    T = w.shape[0]
    loss, _, post = oracle.nms_train(h, 27, llr, cw, w, grad=False, post=True)
    F, N = llr.shape
    x = 1.0 - 2.0 * cw
    for t in range(1, T + 1):
        _, pt, _, _ = oracle.decode_f64(h, 27, llr, max_iter=t, alpha=0.75, early_term=False)
        direct = _softplus(-x * pt).sum() / (T * F * N)
        assert loss[t - 1] == pytest.approx(direct, rel=1e-12)
        if t == T:
            assert np.array_equal(post, pt)


def test_float_forward_matches_float_decoder():
    h, cw, llr, w = _setup("2/3", 27, 10, 4, 2.0, 5)
    llr32 = llr.astype(np.float32)
    _, _, post = oracle.nms_train(h, 27, llr32.astype(np.float64), cw, w, fwd_f32=True, grad=False, post=True)
    _, p32, _, _ = oracle.decode_f32(h, 27, llr32, max_iter=4, alpha=0.75, early_term=False)
    assert np.array_equal(post.astype(np.float32), p32)


def _fd_check(h, Z, llr, cw, w, idx, steps=(1e-6, 1e-7, 1e-8)):
    """Central differences at successively smaller steps. A component is
    compared once two consecutive steps agree to 1e-4 (no sign or argmin
    switch lies within the step); components that never settle sit on a
    kink and are skipped."""
    loss0, g, _ = oracle.nms_train(h, Z, llr, cw, w, grad=True)
    checked = 0

    def loss_at(t, i, j, delta):
        wd = w.copy()
        wd[t, i, j] += delta
        return oracle.nms_train(h, Z, llr, cw, wd, grad=False)[0].sum()

    for k in idx:
        t, i, j = np.unravel_index(k, w.shape)
        if h[i, j] < 0:
            assert g[t, i, j] == 0.0
            continue
        prev = None
        for rel in steps:
            step = rel * max(1.0, abs(w[t, i, j]))
            fd = (loss_at(t, i, j, step) - loss_at(t, i, j, -step)) / (2 * step)
            if prev is not None and abs(fd - prev) <= 1e-4 * abs(prev) + 1e-12:
                assert abs(g[t, i, j] - fd) <= 1e-3 * abs(fd) + 1e-9, (t, i, j, g[t, i, j], fd)
                checked += 1
                break
            prev = fd
    return g, checked


def test_adjoint_matches_finite_differences_small_code():
    # Every weight component of a small code: T = 3 iterations, Z = 8.
    h, cw, llr, w = _setup("1/2", 8, 6, 3, 1.0, 17)
    rng = np.random.default_rng(0)
    w = w + rng.uniform(-0.1, 0.1, w.shape)
    g, checked = _fd_check(h, 8, llr, cw, w, range(w.size))
    assert checked >= 0.9 * int((h >= 0).sum()) * w.shape[0]
    assert np.abs(g).max() > 0


def test_adjoint_matches_finite_differences_wifi_shape():
    # The training code (Z = 81, rate 1/2, 10 iterations) on a 64-frame
    # batch, for a sample of weight components.
    h, cw, llr, w = _setup("1/2", 81, 64, 10, 2.0, 23)
    rng = np.random.default_rng(1)
    active = np.flatnonzero(np.broadcast_to(h >= 0, w.shape))
    idx = rng.choice(active, 12, replace=False)
    g, checked = _fd_check(h, 81, llr, cw, w, idx)
    assert checked >= 9
    inactive = np.broadcast_to(h < 0, w.shape)
    assert (g[inactive] == 0).all()
