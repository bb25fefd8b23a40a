"""Replay of the learned denoiser's backward pass with the GPU kernels' rounding
points, used to derive the gradient tolerances of the GPU tests.

The oracle's backward (oracle/cnn_oracle.py) keeps every gradient in FP64.  The
GPU training kernels instead
  * take dL/dy as float32 and round it to bfloat16 for the backward-data pass
    of the last layer,
  * round every backward-data result (an FP32 MFMA sum) to bfloat16, then apply
    the ReLU mask of the layer below, and feed that bfloat16 gradient both to
    the next backward-data pass and to the weight gradient,
  * sum weight gradients in FP32 per 16x16 pixel tile (partials then reduced in
    FP64).
`replay` applies the same roundings with FP64 sums (order=None) or with FP32
sums in a random order (order = a numpy Generator; then the forward pass is
also summed in FP32 in a random order, so that, as on the GPU, an occasional
activation rounds to the neighbouring bfloat16 value), so the difference between
the replay and the oracle is what those roundings alone cause, and the spread
over orders is what FP32 summation order adds on top.  Test infrastructure only.
"""
import numpy as np

from oracle import cnn_oracle as cnn


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _input_grad32(g, w, rng):
    """conv3x3_input_grad with float32 sums, taps in a random order."""
    Co, H, W = g.shape
    gp = np.zeros((Co, H + 2, W + 2), np.float32)
    gp[:, 1:-1, 1:-1] = g
    out = np.zeros((w.shape[1], H, W), np.float32)
    taps = [(dy, dx) for dy in range(3) for dx in range(3)]
    for i in rng.permutation(9):
        dy, dx = taps[i]
        out += np.tensordot(w[:, :, dy, dx].astype(np.float32),
                            gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W], axes=(0, 0))
    return out.astype(np.float64)


def _weight_grad32(x, g, rng):
    """conv3x3_weight_grad with float32 sums over pixels in a random order."""
    Ci, H, W = x.shape
    xp = np.zeros((Ci, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    perm = rng.permutation(H * W)
    gg = g.reshape(g.shape[0], -1)[:, perm].astype(np.float32)
    dw = np.zeros((g.shape[0], Ci, 3, 3))
    for dy in range(3):
        for dx in range(3):
            xs = xp[:, dy:dy + H, dx:dx + W].reshape(Ci, -1)[:, perm].astype(np.float32)
            dw[:, :, dy, dx] = (gg @ xs.T).astype(np.float64)
    return dw


def _forward32(D, params, rng):
    """The network's activations with the GPU's rounding points, each layer
    summed in FP32 from the bias, taps in a random order."""
    mu, valid, x = cnn.features(D)
    a = cnn.bf16(x)
    acts = [a]
    for k, (w, b) in enumerate(params):
        Ci, H, W = a.shape
        ap = np.zeros((Ci, H + 2, W + 2), np.float32)
        ap[:, 1:-1, 1:-1] = a
        wb = cnn.bf16(w).astype(np.float32)
        z = np.broadcast_to(b.astype(np.float32)[:, None, None], (w.shape[0], H, W)).copy()
        for t in rng.permutation(9):
            dy, dx = divmod(int(t), 3)
            z += np.tensordot(wb[:, :, dy, dx], ap[:, dy:dy + H, dx:dx + W], axes=(1, 0))
        if k < len(params) - 1:
            a = cnn.bf16(np.maximum(z.astype(np.float64), 0.0))
            acts.append(a)
    return acts, valid


def replay(D, params, dL_dDt, order=None):
    """Parameter gradients of sum(dL_dDt * D~) with the GPU's rounding points;
    same layout as cnn_oracle.backward."""
    if order is None:
        _, st = cnn.forward(D, params, True, keep=True)
        acts, valid = st["acts"], st["valid"]
    else:
        acts, valid = _forward32(D, params, order)
    g = _f32(np.where(valid, np.nan_to_num(dL_dDt), 0.0))[None] * cnn.S_SCALE
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        w, _ = params[k]
        dw = (cnn.conv3x3_weight_grad(acts[k], g) if order is None
              else _weight_grad32(acts[k], g, order))
        grads[k] = (dw, g.sum(axis=(1, 2)))
        if k > 0:
            gb, wb = cnn.bf16(g), cnn.bf16(w)
            gin = (cnn.conv3x3_input_grad(gb, wb) if order is None
                   else _input_grad32(gb, wb, order))
            g = cnn.bf16(gin) * (acts[k] > 0)
    return grads


def flat(grads):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in grads])
