"""What the trained denoiser gains over the method without it, on held-out seeds.

The committed checkpoint was trained on crops with seeds 10^6 + i; these scenes
use other seeds.  The learned path (network in place of the 3x3 LSQ filter) must
give a lower mean angular error than the plain path at the same gradient window,
on the training distribution's held-out crops and on full road frames.
Trained weights are not pinned by any oracle: only this gain is tested.
"""
import os

import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _mean_err(pts, gt):
    n = pts[..., 3:6].astype(np.float64)
    ok = np.isfinite(n[..., 0]) & np.isfinite(gt[..., 0])
    cr = np.linalg.norm(np.cross(n[ok], gt[ok]), axis=-1)
    dt = np.abs((n[ok] * gt[ok]).sum(-1))
    return float(np.degrees(np.arctan2(cr, dt)).mean()), int(ok.sum())


def _run(snx, sc, model, ng):
    H, W = sc.disp.shape
    d = torch.from_numpy(sc.disp).to(DEV)
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    pts = torch.empty((H, W, 8), device=DEV)
    ws = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_pipeline(d, sc.cam, lab, pts, ws, filter_window=3, normal_window=ng, cnn=model)
    torch.cuda.synchronize()
    return _mean_err(pts.cpu().numpy(), sc.normal)


@pytest.fixture(scope="module")
def trained():
    snx = _snx()
    from paper_2504_15121_amd import learned
    if not os.path.exists(learned.DEFAULT_MODEL):
        pytest.skip("no trained checkpoint in the package")
    st = learned.load_checkpoint(learned.DEFAULT_MODEL)
    P = torch.from_numpy(st["params"]).to(DEV)
    packed = torch.empty(snx.snx_cnn_packed_bytes() // 2, dtype=torch.int16, device=DEV)
    snx.snx_cnn_pack(P, packed)
    ws = torch.empty(snx.snx_cnn_workspace_size(2048, 1024, 1, 0), dtype=torch.uint8, device=DEV)
    return snx, snx.cnn_model(P, packed, ws), (P, packed, ws)


def test_gain_on_held_out_crops(trained):
    snx, model, _ = trained
    print("case learned gain crops", flush=True)
    plain, learned_ = [], []
    for i in range(12):
        sc = scenes.training_crop(5_000_000 + i, crop=256)
        plain.append(_run(snx, sc, None, 9))
        learned_.append(_run(snx, sc, model, 9))
    ep = sum(e * n for e, n in plain) / sum(n for _, n in plain)
    el = sum(e * n for e, n in learned_) / sum(n for _, n in learned_)
    print(f"held-out crops, n_g = 9: plain {ep:.3f} deg, learned {el:.3f} deg", flush=True)
    assert el < ep, (el, ep)


@pytest.mark.parametrize("ng", [9, 15])
def test_gain_on_road_frames(trained, ng):
    snx, model, _ = trained
    print(f"case learned gain road ng={ng}", flush=True)
    for seed in (5100, 5101):
        sc = scenes.road_scene(seed=seed)
        ep, n1 = _run(snx, sc, None, ng)
        el, n2 = _run(snx, sc, model, ng)
        print(f"road seed {seed}, n_g = {ng}: plain {ep:.3f} deg ({n1} px), "
              f"learned {el:.3f} deg ({n2} px)", flush=True)
        assert el < ep, (seed, el, ep)
