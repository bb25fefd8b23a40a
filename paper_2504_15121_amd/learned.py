"""Training and inference driver of the learned residual denoiser.

All arithmetic runs in the HIP kernels behind snx_cnn_train_step /
snx_cnn_denoise; this module only owns device buffers, builds batches from the
seeded crop generator, steps the learning-rate schedule and reads/writes
checkpoints.

Checkpoint: a .npz file with the FP32 parameters, the Adam moments, the step
count, the seed and a CRC32 of the parameter and moment bytes.  It is written to
a temporary file and renamed, so a checkpoint on disk is always complete;
loading checks the version and the CRC.
"""
from __future__ import annotations

import os
import zlib

import numpy as np

from . import _lib

CKPT_VERSION = 1
LAYERS = [(2, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, zero last layer (the untrained network
    returns the LSQ filter unchanged).  Flat float32 in the ABI's layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(LAYERS):
        w = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), (co, ci, 3, 3))
        if k == len(LAYERS) - 1:
            w[:] = 0.0
        parts += [w.ravel(), np.zeros(co)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == _lib.snx_cnn_param_count()
    return flat


def crop_batch(indices, crop=256):
    """Seeded training crops: disparity (B, H, W), normals (B, 3, H, W), cameras."""
    from synth import scenes
    scs = [scenes.training_crop(int(i), crop=crop) for i in indices]
    D = np.stack([s.disp for s in scs]).astype(np.float32)
    N = np.stack([np.moveaxis(s.normal, -1, 0) for s in scs]).astype(np.float32)
    return D, N, [s.cam for s in scs]


class Trainer:
    def __init__(self, device="cuda:0", crop=256, batch=8, normal_window=9, lr=1e-3,
                 seed=0, params=None):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.crop, self.batch, self.normal_window = crop, batch, normal_window
        self.lr, self.seed = lr, seed
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p.copy()).to(self.dev)
        n = self.params.numel()
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.packed = torch.empty(_lib.snx_cnn_packed_bytes() // 2, dtype=torch.int16,
                                  device=self.dev)
        self.loss = torch.zeros(2, dtype=torch.float64, device=self.dev)
        self.ws = torch.empty(_lib.snx_cnn_workspace_size(crop, crop, batch, True),
                              dtype=torch.uint8, device=self.dev)
        self.step = 0
        _lib.snx_cnn_pack(self.params, self.packed)

    def train_step(self, D, N, cams, lr=None, apply=True):
        """One Adam step on a batch (numpy or device tensors); returns the loss."""
        torch = self.torch
        D = torch.as_tensor(D, device=self.dev)
        N = torch.as_tensor(N, device=self.dev)
        step = self.step + 1 if apply else 0
        _lib.snx_cnn_train_step(D, N, cams, self.params, self.packed, self.grad, self.m, self.v,
                                step, self.lr if lr is None else lr, self.loss, self.ws,
                                normal_window=self.normal_window)
        if apply:
            self.step += 1
        return float(self.loss[0].item())

    def fit(self, n_steps, pool, log_every=0, lr_final=None):
        """Train on crops cycled from `pool` (D, N, cams); cosine learning-rate decay
        to lr_final (default lr / 10)."""
        D, N, cams = pool
        lr_final = self.lr / 10 if lr_final is None else lr_final
        losses = []
        n = D.shape[0]
        Dd = self.torch.as_tensor(D, device=self.dev)
        Nd = self.torch.as_tensor(N, device=self.dev)
        for k in range(n_steps):
            idx = [(k * self.batch + j) % n for j in range(self.batch)]
            lr = lr_final + 0.5 * (self.lr - lr_final) * (1 + np.cos(np.pi * k / max(1, n_steps)))
            loss = self.train_step(Dd[idx], Nd[idx], [cams[i] for i in idx], lr=lr)
            losses.append(loss)
            if log_every and (k + 1) % log_every == 0:
                print(f"step {self.step} loss {loss:.5f} lr {lr:.2e}", flush=True)
        return losses

    def model(self, workspace):
        return _lib.cnn_model(self.params, self.packed, workspace)

    # -------------------------------------------------------------- checkpoint
    def state(self):
        p = self.params.cpu().numpy()
        m = self.m.cpu().numpy()
        v = self.v.cpu().numpy()
        crc = zlib.crc32(p.tobytes() + m.tobytes() + v.tobytes())
        return dict(version=CKPT_VERSION, params=p, m=m, v=v, step=self.step, seed=self.seed,
                    crc=crc)

    def save(self, path):
        tmp = path + ".tmp.npz"
        np.savez(tmp, **self.state())
        os.replace(tmp, path)

    def load(self, path):
        st = load_checkpoint(path)
        self.params.copy_(self.torch.from_numpy(st["params"]))
        self.m.copy_(self.torch.from_numpy(st["m"]))
        self.v.copy_(self.torch.from_numpy(st["v"]))
        self.step = int(st["step"])
        self.seed = int(st["seed"])
        _lib.snx_cnn_pack(self.params, self.packed)


class CheckpointError(ValueError):
    pass


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as z:
        st = {k: z[k] for k in z.files}
    if int(st.get("version", -1)) != CKPT_VERSION:
        raise CheckpointError(f"{path}: unsupported checkpoint version")
    p, m, v = (np.ascontiguousarray(st[k], np.float32) for k in ("params", "m", "v"))
    if p.size != _lib.snx_cnn_param_count() or m.size != p.size or v.size != p.size:
        raise CheckpointError(f"{path}: wrong parameter count")
    if zlib.crc32(p.tobytes() + m.tobytes() + v.tobytes()) != int(st["crc"]):
        raise CheckpointError(f"{path}: CRC mismatch")
    st.update(params=p, m=m, v=v)
    return st
