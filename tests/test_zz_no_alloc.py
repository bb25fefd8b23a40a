"""The allocation-free compaction (snx_compact_points_noalloc, the library's
static device scratch) against snx_compact_points with a caller workspace: two
calls in a row on the same GPU, the second on a smaller frame, each output
bit-identical (count, records, and nothing written past the count)."""
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


def _records(snx, W, H, seed):
    """Dense records of the pipeline on a planes+quadrics frame."""
    sc = scenes.planes_quadrics_scene(width=W, height=H, f=0.7 * W, n_planes=10, n_spheres=3,
                                      seed=seed)
    d = torch.from_numpy(sc.disp).to(DEV)
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    pts = torch.empty((H, W, 8), device=DEV)
    ws = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_pipeline(d, sc.cam, lab, pts, ws, filter_window=3, normal_window=9)
    return pts


def _compact_both(snx, pts):
    H, W = pts.shape[:2]
    n = H * W
    ref = torch.full((n, 8), -3.0, device=DEV)
    got = torch.full((n, 8), -3.0, device=DEV)
    cr = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    cg = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_compact_points_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_compact_points(pts, ref, cr, ws)
    snx.snx_compact_points_noalloc(pts, got, cg)
    torch.cuda.synchronize()
    return ref, got, int(cr.item()), int(cg.item())


def test_noalloc_matches_workspace_call_twice():
    snx = _snx()
    for k, (W, H) in enumerate([(1920, 1080), (300, 170)]):
        print(f"case compact noalloc call {k + 1}: {W}x{H}", flush=True)
        pts = _records(snx, W, H, 40 + k)
        ref, got, cr, cg = _compact_both(snx, pts)
        flags = pts.view(torch.int32)[..., 7].cpu().numpy()
        assert cr == cg == int(((flags & 1) != 0).sum())
        assert 0 < cg < W * H
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32))


def test_noalloc_after_a_larger_call_and_edge_sizes():
    """The scratch keeps the previous call's contents: a smaller frame after a
    larger one, a one-chunk frame, one record, and none defined."""
    snx = _snx()
    big = _records(snx, 1280, 720, 50)
    _compact_both(snx, big)
    for W, H in [(64, 64), (1, 1), (4097, 1)]:
        print(f"case compact noalloc {W}x{H}", flush=True)
        pts = _records(snx, W, H, 51)
        ref, got, cr, cg = _compact_both(snx, pts)
        assert cr == cg
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
    none = torch.zeros((33, 129, 8), device=DEV)      # flags 0: nothing defined
    ref, got, cr, cg = _compact_both(snx, none)
    assert cr == cg == 0
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))


def test_noalloc_refuses_frames_over_its_limit():
    snx = _snx()
    pts = torch.zeros((1, 1, 8), device=DEV)
    out = torch.zeros((1, 8), device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    from paper_2504_15121_amd import _lib
    st = _lib.load().snx_compact_points_noalloc(pts.data_ptr(), 8192, 4097, out.data_ptr(),
                                                cnt.data_ptr(), None)
    assert st == 2
    assert b"allocation-free limit" in _lib.load().snx_last_error()
