"""GPU parity of the compacted point cloud: the defined records of the GPU's own
dense cloud, packed in raster order, bit-exact against the oracle's plain
compaction of the same records; the count exact."""
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


def _compact(snx, pts):
    H, W = pts.shape[0], pts.shape[1]
    out = torch.full((max(H * W, 1), 8), -3.0, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = torch.empty(max(1, snx.snx_compact_points_workspace_size(W, H)), dtype=torch.uint8,
                     device=DEV)
    snx.snx_compact_points(pts, out, cnt, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(cnt.item())


def _check(oracle, snx, pts):
    out, n = _compact(snx, pts)
    ref = oracle.compact_points(pts.cpu().numpy())
    assert n == ref.shape[0]
    assert np.array_equal(out[:n].view(np.uint32), ref.view(np.uint32))
    # nothing written past the count
    assert np.all(out[n:] == -3.0)
    return n


@pytest.mark.parametrize("W,H", [(1920, 1080), (64, 64), (4097, 1), (1, 1), (130, 70),
                                 (77, 53)])
def test_compact_matches_oracle(oracle, W, H):
    snx = _snx()
    print(f"case compact {W}x{H}", flush=True)
    sc = scenes.planes_quadrics_scene(width=max(W, 8), height=max(H, 8), f=300.0, n_planes=6,
                                      n_spheres=2, seed=W + 7 * H)
    D = np.ascontiguousarray(sc.disp[:H, :W])
    d = torch.from_numpy(D).to(DEV)
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    pts = torch.empty((H, W, 8), device=DEV)
    ws = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_pipeline(d, sc.cam, lab, pts, ws, filter_window=3, normal_window=9)
    torch.cuda.synchronize()
    n = _check(oracle, snx, pts)
    if min(W, H) >= 9:          # a 9x9 slope needs rows and columns on both sides
        assert 0 < n < W * H


def test_compact_none_and_all_defined(oracle):
    snx = _snx()
    print("case compact none / all", flush=True)
    H, W = 33, 250
    rec = np.random.default_rng(5).normal(size=(H, W, 8)).astype(np.float32)
    rec[..., 7] = np.full((H, W), 2, np.uint32).view(np.float32)        # none defined
    assert _check(oracle, snx, torch.from_numpy(rec).to(DEV)) == 0
    rec[..., 7] = np.full((H, W), 3, np.uint32).view(np.float32)        # all defined
    assert _check(oracle, snx, torch.from_numpy(rec).to(DEV)) == H * W
    # alternating pattern across chunk and wave boundaries
    f = np.where((np.arange(H * W) % 3) == 1, 1, 0).astype(np.uint32).reshape(H, W)
    rec[..., 7] = f.view(np.float32)
    assert _check(oracle, snx, torch.from_numpy(rec).to(DEV)) == int(f.sum())


def test_compact_many_chunks_and_repeated_calls(oracle):
    """6 M records (about 1500 chunks of 4096: more count workgroups than fit
    on the chip at once, and chunk offsets summed over many earlier chunks),
    with the defined records' density changing from region to region (long
    empty and long full stretches); then the same workspace reused by calls on
    smaller and larger inputs, each bit-exact."""
    snx = _snx()
    rng = np.random.default_rng(11)
    H, W = 2000, 3000
    print(f"case compact many chunks {W}x{H}", flush=True)
    rec = rng.normal(size=(H, W, 8)).astype(np.float32)
    dens = np.repeat(rng.choice([0.0, 0.02, 0.5, 0.97, 1.0], size=H // 50), 50)
    f = ((rng.random((H, W)) < dens[:, None]).astype(np.uint32)
         | (rng.random((H, W)) < 0.5).astype(np.uint32) * np.uint32(2))
    rec[..., 7] = f.view(np.float32)
    pts = torch.from_numpy(rec).to(DEV)
    assert _check(oracle, snx, pts) == int((f & 1).sum())
    ws = torch.empty(snx.snx_compact_points_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    for h, w in [(7, 300), (H, W), (1, 1), (1000, 1500)]:
        print(f"case compact reuse {w}x{h}", flush=True)
        sub = pts[:h, :w].contiguous()
        out = torch.full((h * w, 8), -3.0, device=DEV)
        cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        snx.snx_compact_points(sub, out, cnt, ws)
        torch.cuda.synchronize()
        ref = oracle.compact_points(rec[:h, :w])
        n = int(cnt.item())
        assert n == ref.shape[0]
        o = out.cpu().numpy()
        assert np.array_equal(o[:n].view(np.uint32), ref.view(np.uint32))
        assert np.all(o[n:] == -3.0)
