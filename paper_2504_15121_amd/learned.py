"""Training and inference driver of the learned residual denoiser.

All arithmetic runs in the HIP kernels behind snx_cnn_train_step /
snx_cnn_denoise; this module only owns device buffers, builds batches from the
seeded crop generator, steps the learning-rate schedule and reads/writes
checkpoints.

Checkpoint: the library's model file (snx_model_save / snx_model_load: FP32
parameters, Adam moments, step, seed, training window and fidelity weight, a
version and a CRC-32), written to a temporary file and renamed, so a checkpoint
on disk is always complete; loading checks the version, the size and the CRC.
"""
from __future__ import annotations

import os

import numpy as np

from . import _lib

MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "denoiser_ng9.snxm")
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


def _one_crop(args):
    """Crop i of the training mix: a road-like crop when the running count of road
    crops, floor((i + 1) * road_frac), steps at i, else a Voronoi-plane crop."""
    from synth import scenes
    i, crop = args[0], args[1]
    road_frac = args[2] if len(args) > 2 else 0.0
    if np.floor((i + 1) * road_frac) > np.floor(i * road_frac):
        s = scenes.road_crop(int(i), crop=crop)
    else:
        s = scenes.training_crop(int(i), crop=crop)
    return (np.ascontiguousarray(s.disp, np.float32),
            np.ascontiguousarray(np.moveaxis(s.normal, -1, 0), np.float32), s.cam,
            np.ascontiguousarray(s.clean, np.float32))


def crop_batch(indices, crop=256, pool=None, road_frac=0.0):
    """Seeded training crops: disparity (B, H, W), normals (B, 3, H, W), cameras,
    clean disparity (B, H, W).  `pool` (a multiprocessing pool) spreads the
    generation over processes."""
    work = [(int(i), crop, road_frac) for i in indices]
    res = pool.map(_one_crop, work, chunksize=8) if pool is not None else list(map(_one_crop, work))
    D = np.ascontiguousarray(np.stack([r[0] for r in res]))
    N = np.ascontiguousarray(np.stack([r[1] for r in res]))
    Cl = np.ascontiguousarray(np.stack([r[3] for r in res]))
    return D, N, [r[2] for r in res], Cl


class Trainer:
    def __init__(self, device="cuda:0", crop=256, batch=8, normal_window=9, lr=1e-3,
                 seed=0, params=None, fidelity=0.0):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.crop, self.batch, self.normal_window = crop, batch, normal_window
        self.lr, self.seed, self.fidelity = lr, seed, fidelity
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p.copy()).to(self.dev)
        n = self.params.numel()
        self.grad = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.packed = torch.empty(_lib.snx_cnn_packed_bytes() // 2, dtype=torch.int16,
                                  device=self.dev)
        self.loss = torch.zeros(4, dtype=torch.float64, device=self.dev)
        self.ws = torch.empty(_lib.snx_cnn_workspace_size(crop, crop, batch, True),
                              dtype=torch.uint8, device=self.dev)
        self.step = 0
        _lib.snx_cnn_pack(self.params, self.packed)

    def train_step(self, D, N, cams, lr=None, apply=True, clean=None):
        """One Adam step on a batch (numpy or device tensors); returns the loss."""
        torch = self.torch
        D = torch.as_tensor(D, device=self.dev).contiguous()
        N = torch.as_tensor(N, device=self.dev).contiguous()
        if clean is not None and self.fidelity > 0:
            clean = torch.as_tensor(clean, device=self.dev).contiguous()
        else:
            clean = None
        step = self.step + 1 if apply else 0
        _lib.snx_cnn_train_step(D, N, cams, self.params, self.packed, self.grad, self.m, self.v,
                                step, self.lr if lr is None else lr, self.loss, self.ws,
                                normal_window=self.normal_window, clean=clean,
                                fidelity=self.fidelity)
        if apply:
            self.step += 1
        return float(self.loss[0].item())

    def fit(self, n_steps, pool, log_every=0, lr_final=None):
        """Train on crops cycled from `pool` (D, N, cams[, clean]); cosine
        learning-rate decay to lr_final (default lr / 10)."""
        D, N, cams = pool[:3]
        Cl = pool[3] if len(pool) > 3 else None
        lr_final = self.lr / 10 if lr_final is None else lr_final
        losses = []
        n = D.shape[0]
        Dd = self.torch.as_tensor(D, device=self.dev)
        Nd = self.torch.as_tensor(N, device=self.dev)
        Cd = None if Cl is None else self.torch.as_tensor(Cl, device=self.dev)
        for k in range(n_steps):
            idx = [(k * self.batch + j) % n for j in range(self.batch)]
            lr = lr_final + 0.5 * (self.lr - lr_final) * (1 + np.cos(np.pi * k / max(1, n_steps)))
            loss = self.train_step(Dd[idx], Nd[idx], [cams[i] for i in idx], lr=lr,
                                   clean=None if Cd is None else Cd[idx])
            losses.append(loss)
            if log_every and (k + 1) % log_every == 0:
                print(f"step {self.step} loss {loss:.5f} lr {lr:.2e}", flush=True)
        return losses

    def model(self, workspace):
        return _lib.cnn_model(self.params, self.packed, workspace)

    # -------------------------------------------------------------- checkpoint
    def save(self, path):
        _lib.model_save(path, self.params.cpu().numpy(), self.m.cpu().numpy(),
                        self.v.cpu().numpy(), step=self.step, normal_window=self.normal_window,
                        seed=self.seed, fidelity=self.fidelity)

    def load(self, path):
        st = load_checkpoint(path)
        if st["m"] is None:
            raise CheckpointError(f"{path}: no Adam state to resume from")
        self.params.copy_(self.torch.from_numpy(st["params"]))
        self.m.copy_(self.torch.from_numpy(st["m"]))
        self.v.copy_(self.torch.from_numpy(st["v"]))
        self.step = int(st["step"])
        self.seed = int(st["seed"])
        _lib.snx_cnn_pack(self.params, self.packed)


class CheckpointError(ValueError):
    pass


def load_checkpoint(path):
    """The model file's contents (see _lib.model_load); CheckpointError if the
    file is missing, corrupt or of another version."""
    try:
        return _lib.model_load(path)
    except _lib.SnxError as e:
        raise CheckpointError(str(e)) from None


# ------------------------------------------------------------------ training CLI
def train_main(argv=None):
    """Train the denoiser on seeded crops and write a checkpoint.

    Crops are generated in chunks by a process pool while the GPU trains on the
    previous chunk; each chunk is used for `--passes` passes in shuffled batches."""
    import argparse
    import multiprocessing as mp
    import time

    ap = argparse.ArgumentParser(prog="python -m paper_2504_15121_amd.learned")
    ap.add_argument("--crops", type=int, default=20000)
    ap.add_argument("--chunk", type=int, default=1000)
    ap.add_argument("--passes", type=int, default=1)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--normal-window", type=int, default=9)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--road-frac", type=float, default=0.5,
                    help="fraction of road-like crops in the training mix")
    ap.add_argument("--fidelity", type=float, default=0.1,
                    help="weight of the (D~ - clean)^2 term (px^-2)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--resume", default=None)
    a = ap.parse_args(argv)

    _lib.load()
    t = Trainer(crop=a.crop, batch=a.batch, normal_window=a.normal_window, lr=a.lr, seed=a.seed,
                fidelity=a.fidelity)
    if a.resume:
        t.load(a.resume)
    rng = np.random.default_rng(a.seed)
    n_chunks = (a.crops + a.chunk - 1) // a.chunk
    total_steps = n_chunks * a.passes * (a.chunk // a.batch)
    k = 0
    t0 = time.time()
    ctx = mp.get_context("spawn")
    with ctx.Pool(a.workers) as pool:
        nxt = pool.map_async(_one_crop, [(i, a.crop, a.road_frac)
                                         for i in range(min(a.chunk, a.crops))], chunksize=8)
        for c in range(n_chunks):
            res = nxt.get()
            lo = (c + 1) * a.chunk
            if lo < a.crops:
                nxt = pool.map_async(_one_crop, [(i, a.crop, a.road_frac)
                                                 for i in range(lo, min(lo + a.chunk, a.crops))],
                                     chunksize=8)
            D = t.torch.from_numpy(np.ascontiguousarray(np.stack([r[0] for r in res]))).to(t.dev)
            N = t.torch.from_numpy(np.ascontiguousarray(np.stack([r[1] for r in res]))).to(t.dev)
            cams = [r[2] for r in res]
            Cl = t.torch.from_numpy(np.ascontiguousarray(np.stack([r[3] for r in res]))).to(t.dev)
            losses = []
            for _ in range(a.passes):
                order = rng.permutation(len(res))
                for j in range(0, len(res) - a.batch + 1, a.batch):
                    idx = order[j:j + a.batch]
                    lr = a.lr_final + 0.5 * (a.lr - a.lr_final) * (1 + np.cos(np.pi * k / total_steps))
                    ii = t.torch.from_numpy(idx).to(t.dev)
                    losses.append(t.train_step(D[ii], N[ii], [cams[i] for i in idx], lr=lr,
                                               clean=Cl[ii]))
                    k += 1
            ln, lf = t.loss[2].item(), t.loss[3].item()
            print(f"chunk {c + 1}/{n_chunks} step {t.step} loss {np.mean(losses):.5f} "
                  f"(last: normal {ln:.4f}, fidelity {lf:.4f} px^2) lr {lr:.2e} "
                  f"{time.time() - t0:.1f} s", flush=True)
            t.save(a.out)
    return t


if __name__ == "__main__":
    train_main()
