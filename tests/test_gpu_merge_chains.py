"""Component labels where the seam merge builds long hook chains, against the
oracle's flood fill (bit-exact labels, minimum pixel index per component, and
counts), through snx_components and through the pipeline's two parts.

* a serpentine corridor two rows thick that winds through every tile row of a
  700 x 420 frame (11 x 14 component tiles), joined alternately at the left and
  right edges: one component whose tile roots are hooked across every
  horizontal and vertical seam;
* one constant plane over the whole frame with 20 % random holes: every tile
  root of the frame ends in the same tree;
* random 4-level disparities over 1.6 % invalid on a 1001 x 517 frame (ragged
  tiles in both directions), many small components touching the seams.
"""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _serpentine(H, W):
    y, x = np.mgrid[0:H, 0:W]
    m = (y % 4) < 2
    m |= (x == 0) & (y % 8 >= 2) & (y % 8 < 4)
    m |= (x == W - 1) & (y % 8 >= 6)
    D = np.full((H, W), 20.0, np.float32)
    D[~m] = np.nan
    return D


def _plane_with_holes(H, W, rng):
    D = np.full((H, W), 35.0, np.float32)
    D[rng.random((H, W)) < 0.2] = np.nan
    return D


def _levels(H, W, rng):
    D = (10.0 + 0.9 * rng.integers(0, 4, (H, W))).astype(np.float32)
    D[rng.random((H, W)) < 0.016] = np.nan
    return D


def _gpu_labels(snx, D, k_rel, t_abs):
    H, W = D.shape
    d = torch.from_numpy(D).to(DEV)
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_components_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_components(d, lab, ws, num_components=cnt, k_rel=k_rel, t_abs=t_abs)
    lab2 = torch.empty((H, W), dtype=torch.int32, device=DEV)
    cnt2 = torch.zeros(1, dtype=torch.int32, device=DEV)
    pts = torch.empty((H, W, 8), device=DEV)
    ws2 = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    cam = scenes.Camera(500.0, 500.0, 0.1, 0.5 * (W - 1), 0.5 * (H - 1))
    snx.snx_pipeline_part(d, cam, lab2, pts, ws2, parts=snx.PART_FOREST, num_components=cnt2,
                          filter_window=3, normal_window=9, k_rel=k_rel, t_abs=t_abs)
    snx.snx_pipeline_part(d, cam, lab2, pts, ws2, parts=snx.PART_POINTS, num_components=cnt2,
                          filter_window=3, normal_window=9, k_rel=k_rel, t_abs=t_abs)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(cnt.item()), lab2.cpu().numpy(), int(cnt2.item())


@pytest.mark.parametrize("case", ["serpentine", "plane_with_holes", "levels"])
def test_long_merge_chains(oracle, case):
    import paper_2504_15121_amd as snx
    snx.load()
    rng = np.random.default_rng(41)
    if case == "serpentine":
        D, k_rel, t_abs = _serpentine(420, 700), 0.1, 1.0
    elif case == "plane_with_holes":
        D, k_rel, t_abs = _plane_with_holes(420, 700, rng), 0.1, 1.0
    else:
        D, k_rel, t_abs = _levels(517, 1001, rng), 0.0, 1.0
    print(f"case merge chains {case} {D.shape}", flush=True)
    lab, cnt, lab2, cnt2 = _gpu_labels(snx, D, k_rel, t_abs)
    ref, nref = oracle.components(D, k_rel, t_abs)
    if case == "serpentine":
        assert nref == 1
    assert np.array_equal(lab, ref), (lab != ref).sum()
    assert cnt == nref
    assert np.array_equal(lab2, ref), (lab2 != ref).sum()
    assert cnt2 == nref


@pytest.mark.parametrize("shape", [(37, 70), (33, 65), (64, 128), (32, 64), (1, 200), (200, 1),
                                   (97, 193)])
def test_pipeline_seam_records(oracle, shape):
    """With the 3x3 filter the front decides every tile-seam pair from its halo
    and writes seam records for the merge: labels against the oracle on seam-
    crossing random-level frames (exact multiples of the tile, ragged, single
    row and column), with the label forest in the labels and, with a padded
    label stride, in the workspace."""
    import paper_2504_15121_amd as snx
    snx.load()
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    cam = scenes.Camera(500.0, 500.0, 0.1, 0.5 * (W - 1), 0.5 * (H - 1))
    for rep in range(6):
        D = _levels(H, W, rng)
        D[rng.random((H, W)) < (0.05, 0.3)[rep % 2]] = np.nan
        pad = 3 * (rep % 2)
        print(f"case seam records {shape} rep {rep} pad {pad}", flush=True)
        d = torch.from_numpy(D).to(DEV)
        lab = torch.full((H, W + pad), -9, dtype=torch.int32, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        pts = torch.empty((H, W, 8), device=DEV)
        ws = torch.empty(snx.snx_pipeline_workspace_size(W, H), dtype=torch.uint8, device=DEV)
        snx.snx_pipeline(d, cam, lab[:, :W], pts, ws, num_components=cnt, filter_window=3,
                         normal_window=3, k_rel=0.0, t_abs=1.0)
        torch.cuda.synchronize()
        ref, nref = oracle.components(D, 0.0, 1.0)
        got = lab[:, :W].cpu().numpy()
        assert np.array_equal(got, ref), (rep, (got != ref).sum())
        assert int(cnt.item()) == nref
