"""Pins of the learned-denoiser oracle: rounding, convolution, adjoints, head
gradient and whole-network backward against finite differences."""
import numpy as np
import pytest
import torch
from scipy import signal

from oracle import cnn_oracle as cnn
from oracle import oracle as plain
from synth import scenes


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)
    # ties go to even
    assert cnn.bf16(1.0 + 2 ** -8) == 1.0
    assert cnn.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_conv_is_textbook_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 11, 13))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    out = cnn.conv3x3(x, w, b)
    for o in range(4):
        ref = sum(signal.correlate2d(x[i], w[o, i], mode="same", boundary="fill")
                  for i in range(3)) + b[o]
        np.testing.assert_allclose(out[o], ref, atol=1e-12)


def test_conv_adjoints():
    """<conv(x, w), g> = <x, input_grad(g, w)> = <w, weight_grad(x, g)>."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 9, 7))
    w = rng.normal(size=(6, 5, 3, 3))
    g = rng.normal(size=(6, 9, 7))
    lhs = (cnn.conv3x3(x, w) * g).sum()
    np.testing.assert_allclose((x * cnn.conv3x3_input_grad(g, w)).sum(), lhs, rtol=1e-12)
    np.testing.assert_allclose((w * cnn.conv3x3_weight_grad(x, g)).sum(), lhs, rtol=1e-12)


def test_untrained_network_returns_lsq_filter():
    sc = scenes.planes_scene(width=40, height=30, f=100.0, seed=2)
    params = cnn.init_params(0)
    Dt = cnn.forward(sc.disp, params)
    ref = cnn.f32(plain.denoise(sc.disp.astype(np.float64), 3))
    np.testing.assert_array_equal(np.isnan(Dt), np.isnan(ref))
    m = np.isfinite(ref)
    np.testing.assert_array_equal(Dt[m], ref[m])


def test_head_normals_match_plain_oracle():
    sc = scenes.planes_scene(width=60, height=45, f=120.0, seed=3, sigma=0.3)
    Dt = plain.denoise(sc.disp.astype(np.float64), 3)
    L, n, use = cnn.normal_loss(Dt, sc.normal, sc.cam, ng=5, need_grad=False)
    a1, a2, d = plain.affine(Dt, 5)
    nref = plain.normals(Dt, a1, a2, d, sc.cam)
    assert np.array_equal(use, d & np.isfinite(sc.normal[..., 0]))
    np.testing.assert_allclose(n[d], nref[d], atol=1e-12)
    ref_loss = np.mean(1.0 - (nref[use] * sc.normal[use]).sum(-1))
    assert abs(L - ref_loss) < 1e-12


def test_head_gradient_finite_differences():
    sc = scenes.planes_scene(width=14, height=12, f=40.0, seed=4, sigma=0.4, invalid_frac=0.1)
    Dt = plain.denoise(sc.disp.astype(np.float64), 3)
    L, n, use, grad = cnn.normal_loss(Dt, sc.normal, sc.cam, ng=5)
    rng = np.random.default_rng(0)
    idx = np.flatnonzero(np.isfinite(Dt))
    for j in rng.choice(idx, 25, replace=False):
        h = 1e-6
        Dp = Dt.copy(); Dp.flat[j] += h
        Dm = Dt.copy(); Dm.flat[j] -= h
        fd = (cnn.normal_loss(Dp, sc.normal, sc.cam, 5, need_grad=False)[0]
              - cnn.normal_loss(Dm, sc.normal, sc.cam, 5, need_grad=False)[0]) / (2 * h)
        assert abs(fd - grad.flat[j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (j, fd, grad.flat[j])


def test_network_backward_finite_differences():
    sc = scenes.planes_scene(width=10, height=9, f=30.0, seed=5, sigma=0.5, invalid_frac=0.1)
    rng = np.random.default_rng(1)
    params = cnn.init_params(3)
    params = [(w + rng.normal(0, 0.05, w.shape), b + rng.normal(0, 0.05, b.shape))
              for w, b in params]
    gup = rng.normal(size=sc.disp.shape)

    def objective(p):
        Dt = cnn.forward(sc.disp, p, emulate_bf16=False)
        return float(np.nansum(Dt * gup))

    grads = cnn.backward(sc.disp, params, gup, emulate_bf16=False)
    for k in (0, 2, 5):
        w, b = params[k]
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            h = 1e-6
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[k][0][idx] += h
            wm[k][0][idx] -= h
            fd = (objective(wp) - objective(wm)) / (2 * h)
            assert abs(fd - grads[k][0][idx]) <= 1e-5 * max(1.0, abs(fd)), (k, idx)
        j = int(rng.integers(0, b.size))
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[k][1][j] += 1e-6
        bm[k][1][j] -= 1e-6
        fd = (objective(bp) - objective(bm)) / 2e-6
        assert abs(fd - grads[k][1][j]) <= 1e-5 * max(1.0, abs(fd))


def test_fidelity_term_closed_form_and_gradient():
    """A constant offset c on the valid pixels gives L_f = c^2 exactly; the
    gradient matches central differences; invalid D~ and missing clean values
    are excluded."""
    rng = np.random.default_rng(6)
    clean = rng.uniform(5, 50, (9, 11))
    clean[0, 0] = np.nan
    Dt = clean + 0.75
    Dt[3, 4] = np.nan
    Dt[5, 5] = -1.0
    L, n, g = cnn.fidelity_loss(Dt, clean)
    assert n == 9 * 11 - 3
    assert abs(L - 0.75 ** 2) < 1e-12
    Dt = clean + rng.normal(0, 0.5, clean.shape)
    L, n, g = cnn.fidelity_loss(Dt, clean)
    for j in rng.choice(np.flatnonzero(np.isfinite(clean)), 10, replace=False):
        Dp = Dt.copy(); Dp.flat[j] += 1e-6
        Dm = Dt.copy(); Dm.flat[j] -= 1e-6
        fd = (cnn.fidelity_loss(Dp, clean)[0] - cnn.fidelity_loss(Dm, clean)[0]) / 2e-6
        assert abs(fd - g.flat[j]) < 1e-8


def test_backward_rounding_replay():
    """Scale of the GPU's backward rounding (bfloat16 gradients, FP32 sums)
    against the FP64 oracle backward, on the GPU gradient test's inputs: the
    roundings alone move each layer's gradient by under 1 %, visibly so on every
    layer before the last; FP32 summation order in the forward (bfloat16 flips
    of single activations) and the backward adds at most 1.5 % on top.  The GPU
    test's per-layer bound is 3x the sum of the two, computed on its inputs."""
    from tests import cnn_replay
    rng = np.random.default_rng(2)
    p = cnn.init_params(2)
    p = [(w + rng.normal(0, 0.05, w.shape) * (k == 5), b + rng.normal(0, 0.02, b.shape))
         for k, (w, b) in enumerate(p)]
    p32 = [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
           for w, b in p]
    nrm = np.linalg.norm
    sizes = [lw.size + lb.size for lw, lb in p32]
    for i in range(2):
        c = scenes.training_crop(i, crop=48)
        Dt = cnn.forward(c.disp, p32, True)
        _, _, _, dDt = cnn.normal_loss(Dt, c.normal, c.cam, 5)
        ora = cnn_replay.flat(cnn.backward(c.disp, p32, dDt, True))
        r64 = cnn_replay.flat(cnn_replay.replay(c.disp, p32, dDt))
        r32 = [cnn_replay.flat(cnn_replay.replay(c.disp, p32, dDt,
                                                 order=np.random.default_rng(s)))
               for s in range(3)]
        off = 0
        for k, n in enumerate(sizes):
            o, q = ora[off:off + n], r64[off:off + n]
            rel = nrm(q - o) / nrm(o)
            assert rel < 1e-2, (i, k, rel)
            if k < 5:
                assert rel > 1e-5, (i, k, rel)      # the roundings are visible
            for r in r32:
                spread = nrm(r[off:off + n] - q) / nrm(q)
                assert spread <= 1.5e-2, (i, k, spread)
            off += n
