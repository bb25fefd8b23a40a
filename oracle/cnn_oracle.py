"""FP64 oracle of the learned denoiser and of its normal-loss training step.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU-baseline leg of the
benchmark).  Plain numpy, no code shared with the GPU path.

Model (a learned stand-in for the hand-tuned filter; the paper notes its method
is differentiable and convolution-like, Sec. 1 contribution paragraph):
  mu  = the LSQ plane-fit filter of the disparity (window 3) at valid pixels,
        rounded to float32 (the filter's output type; the network sees the
        same float32 image a caller of the filter gets)
  x0  = (D - mu) / s at valid pixels, 0 at invalid ones;  x1 = validity (0/1)
  a_1 = relu(conv(W1, [x0, x1]) + b1)            2 -> 32 channels
  a_k = relu(conv(Wk, a_{k-1}) + bk)             32 -> 32, k = 2..5
  y   = conv(W6, a_5) + b6                       32 -> 1
  D~  = mu + s * y at valid pixels, NaN at invalid ones
conv is a 3x3 cross-correlation with zero padding: out[o, v, u] =
sum_{i, dy, dx} W[o, i, dy+1, dx+1] * in[i, v+dy, u+dx].
Weights and activations are bfloat16 (round to nearest even) with float32
accumulation on the GPU; `emulate_bf16=True` rounds at the same points (FP64 sum
rounded to float32, then to bfloat16).  With emulate_bf16=False everything is
FP64 (used for finite-difference pins).

Training loss (normals supervise the denoiser through the method's own
gradient and normal steps, Sec. 3.1-3.3):
  L_n = sum over pixels c with a defined normal and a ground-truth normal g_c of
        (1 - n_c . g_c) / N
with n_c the unit normal from the anchored masked LSQ slope of D~ (window n_g),
N the number of such pixels; optionally plus w * L_f with the fidelity term
  L_f = mean over pixels with a valid D~ and a finite clean disparity of
        (D~ - clean)^2.
"""
from __future__ import annotations

import numpy as np

from . import oracle as plain

S_SCALE = 1.0          # disparity scale of the network input / output (px)
CH = 32
LAYERS = [(2, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, 1)]


# ---------------------------------------------------------------- numerics
def bf16(x):
    """Round to bfloat16 (nearest even) via float32; returns float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def conv3x3(x, w, b=None):
    """Cross-correlation, zero padding.  x (Ci, H, W), w (Co, Ci, 3, 3)."""
    Ci, H, W = x.shape
    xp = np.zeros((Ci, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], H, W))
    for dy in range(3):
        for dx in range(3):
            out += np.tensordot(w[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + W], axes=(1, 0))
    if b is not None:
        out += b[:, None, None]
    return out


def conv3x3_input_grad(g, w):
    """d(conv3x3(x, w))/dx applied to upstream g (Co, H, W) -> (Ci, H, W)."""
    Co, H, W = g.shape
    gp = np.zeros((Co, H + 2, W + 2))
    gp[:, 1:-1, 1:-1] = g
    out = np.zeros((w.shape[1], H, W))
    # x[i, v, u] feeds out[o, v-dy', u-dx'] with weight w[o, i, dy'+1, dx'+1]
    for dy in range(3):
        for dx in range(3):
            out += np.tensordot(w[:, :, dy, dx], gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W],
                                axes=(0, 0))
    return out


def conv3x3_weight_grad(x, g):
    """d(sum g * conv3x3(x, w))/dw -> (Co, Ci, 3, 3)."""
    Ci, H, W = x.shape
    xp = np.zeros((Ci, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((g.shape[0], Ci, 3, 3))
    for dy in range(3):
        for dx in range(3):
            dw[:, :, dy, dx] = np.tensordot(g, xp[:, dy:dy + H, dx:dx + W], axes=([1, 2], [1, 2]))
    return dw


# ---------------------------------------------------------------- model
def init_params(seed=0):
    """He-style initialisation; the last layer starts at zero so that the
    untrained network returns the LSQ filter unchanged."""
    rng = np.random.default_rng(seed)
    params = []
    for k, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci))
        w = rng.normal(0.0, std, (co, ci, 3, 3))
        if k == len(LAYERS) - 1:
            w[:] = 0.0
        params.append((w, np.zeros(co)))
    return params


def features(D, nf_mu=3, s=S_SCALE):
    D = np.asarray(D, dtype=np.float64)
    valid = np.isfinite(D) & (D > 0)
    mu = f32(plain.denoise(D, nf_mu))
    x0 = np.where(valid, (np.where(valid, D, 0.0) - np.where(valid, mu, 0.0)) / s, 0.0)
    return mu, valid, np.stack([x0, valid.astype(np.float64)])


def forward(D, params, emulate_bf16=True, nf_mu=3, s=S_SCALE, keep=False):
    """Returns D~ (and the per-layer tensors when keep=True)."""
    mu, valid, x = features(D, nf_mu, s)
    rnd = bf16 if emulate_bf16 else (lambda t: t)
    acc = f32 if emulate_bf16 else (lambda t: t)
    a = rnd(x)
    acts = [a]
    pre = []
    for k, (w, b) in enumerate(params):
        z = acc(conv3x3(a, rnd(w), b))
        pre.append(z)
        if k < len(params) - 1:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
    y = z[0]
    Dt = np.where(valid, mu + s * y, np.nan)
    if keep:
        return Dt, dict(mu=mu, valid=valid, acts=acts, pre=pre, y=y)
    return Dt


# ---------------------------------------------------------------- loss head
def _offsets(r):
    return [(dx, dy) for dy in range(-r, r + 1) for dx in range(-r, r + 1) if dx or dy]


def _shift(a, dx, dy, fill):
    """out[v, u] = a[v + dy, u + dx] (fill outside)."""
    H, W = a.shape
    out = np.full((H, W), fill, dtype=a.dtype)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[ys:ye, xs:xe] = a[ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def normal_loss(Dt, n_gt, cam, ng=9, min_support=None, need_grad=True):
    """Loss of the normals of D~ against n_gt and (optionally) dL/dD~.

    The slope is the anchored masked LSQ of Sec. 3.2-3.3 written as
    g_u = sum_i wu_i (D_i - D_c), g_v = sum_i wv_i (D_i - D_c) with
    wu_i = (gamma v_ix - beta v_iy)/det, wv_i = (-beta v_ix + alpha v_iy)/det;
    m = (f_x g_u, f_y g_v, D_c - (u-u0) g_u - (v-v0) g_v), n = -m/|m|."""
    Dt = np.asarray(Dt, dtype=np.float64)
    H, W = Dt.shape
    r = ng // 2
    need = int(np.ceil(ng * ng / 2.0)) if min_support is None else min_support
    valid = np.isfinite(Dt) & (Dt > 0)
    Dz = np.where(valid, Dt, 0.0)
    al = np.zeros((H, W)); be = np.zeros((H, W)); ga = np.zeros((H, W))
    cnt = np.zeros((H, W)); Sx = np.zeros((H, W)); Sy = np.zeros((H, W))
    P1 = np.zeros((H, W)); P2 = np.zeros((H, W))
    for dx, dy in _offsets(r):
        m = _shift(valid, dx, dy, False)
        d = _shift(Dz, dx, dy, 0.0)
        cnt += m; Sx += m * dx; Sy += m * dy
        al += m * dx * dx; be += m * dx * dy; ga += m * dy * dy
        P1 += m * dx * d; P2 += m * dy * d
    det = al * ga - be * be
    defined = valid & (cnt >= need) & (det > 0)
    sdet = np.where(defined, det, 1.0)
    S1 = P1 - Sx * Dz
    S2 = P2 - Sy * Dz
    gu = (ga * S1 - be * S2) / sdet
    gv = (-be * S1 + al * S2) / sdet
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    mx = cam.fx * gu
    my = cam.fy * gv
    mz = Dz - (u - cam.u0) * gu - (v - cam.v0) * gv
    mn = np.sqrt(mx * mx + my * my + mz * mz)
    mn = np.where(defined, mn, 1.0)
    n = -np.stack([mx, my, mz], -1) / mn[..., None]
    use = defined & np.isfinite(n_gt[..., 0])
    N = max(int(use.sum()), 1)
    dots = (n * np.nan_to_num(n_gt)).sum(-1)
    L = float(np.where(use, 1.0 - dots, 0.0).sum() / N)
    if not need_grad:
        return L, n, use
    g = np.nan_to_num(n_gt)
    # dL/dm = (g - n (n.g)) / (N |m|)  on used pixels
    Gm = (g - n * dots[..., None]) / (N * mn[..., None])
    Gm = np.where(use[..., None], Gm, 0.0)
    Gu = Gm[..., 0] * cam.fx - Gm[..., 2] * (u - cam.u0)
    Gv = Gm[..., 1] * cam.fy - Gm[..., 2] * (v - cam.v0)
    A = (ga * Gu - be * Gv) / sdet
    B = (-be * Gu + al * Gv) / sdet
    A = np.where(use, A, 0.0)
    B = np.where(use, B, 0.0)
    grad = np.where(use, Gm[..., 2] - (A * Sx + B * Sy), 0.0)
    for dx, dy in _offsets(r):
        # centre c = j + (dx, dy) has j at offset (-dx, -dy)
        grad += valid * -(_shift(A, dx, dy, 0.0) * dx + _shift(B, dx, dy, 0.0) * dy)
    grad = np.where(valid, grad, 0.0)
    return L, n, use, grad


# ---------------------------------------------------------------- backward
def backward(D, params, dL_dDt, emulate_bf16=True, nf_mu=3, s=S_SCALE):
    """Parameter gradients of sum(dL_dDt * D~) through the network."""
    Dt, st = forward(D, params, emulate_bf16, nf_mu, s, keep=True)
    rnd = bf16 if emulate_bf16 else (lambda t: t)
    valid = st["valid"]
    g = np.where(valid, np.nan_to_num(dL_dDt), 0.0)[None] * s    # dL/dy
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        w, b = params[k]
        a_in = st["acts"][k]
        grads[k] = (conv3x3_weight_grad(a_in, g), g.sum(axis=(1, 2)))
        if k > 0:
            gin = conv3x3_input_grad(g, rnd(w))
            g = gin * (st["acts"][k] > 0)      # relu of the previous layer
    return grads


def fidelity_loss(Dt, clean):
    """Mean squared difference between D~ and the clean disparity over pixels
    where D~ is valid and the clean value finite; returns (L_f, count, dL_f/dD~)."""
    Dt = np.asarray(Dt, dtype=np.float64)
    clean = np.asarray(clean, dtype=np.float64)
    m = np.isfinite(Dt) & (Dt > 0) & np.isfinite(clean)
    n = int(m.sum())
    r = np.where(m, np.where(m, Dt, 0.0) - np.where(m, clean, 0.0), 0.0)
    nn = max(n, 1)
    return float((r * r).sum() / nn), n, 2.0 * r / nn


def loss_and_grads(D, params, n_gt, cam, ng=9, emulate_bf16=True, nf_mu=3, s=S_SCALE,
                   clean=None, w=0.0):
    Dt = forward(D, params, emulate_bf16, nf_mu, s)
    L, n, use, dDt = normal_loss(Dt, n_gt, cam, ng)
    if clean is not None:
        Lf, _, dF = fidelity_loss(Dt, clean)
        L, dDt = L + w * Lf, dDt + w * dF
    return L, backward(D, params, dDt, emulate_bf16, nf_mu, s)
