"""Component labels on many tiny and seam-crossing frames at once, through one
batch plan, against the oracle's flood fill frame by frame (bit-exact labels and
counts).

* every one of the 4096 validity masks of a 4 x 3 frame, with disparities drawn
  from levels 0.9 px apart (t_abs = 1, k_rel = 0: neighbours one level apart are
  joined, two levels apart are not), so that masks and edge patterns vary
  together;
* 256 frames of 70 x 37 (2 x 2 component tiles, so every frame has vertical and
  horizontal tile seams) with the same level construction and 25 % invalid, with
  filter windows 1 and 3 (the latter through the front's seam records);
* through the edge-graph hook (snx_components_from_edges), every one of the
  2^17 edge subsets of a 3 x 4 grid (all pixels present, and with random pixels
  absent), and random edge graphs on ragged frames, against the oracle's
  labelling of the same graph.
"""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _frames(shape, n, rng, masks=None, invalid=0.25):
    H, W = shape
    out = []
    for i in range(n):
        lv = rng.integers(0, 4, (H, W))
        D = (10.0 + 0.9 * lv).astype(np.float32)
        if masks is not None:
            m = np.array([(masks[i] >> k) & 1 for k in range(H * W)], bool).reshape(H, W)
        else:
            m = rng.random((H, W)) >= invalid
        D[~m] = np.nan
        out.append(D)
    return out


def _run(snx, Ds, filter_window=1):
    cam = scenes.Camera(100.0, 100.0, 0.1, 1.0, 1.0)
    bufs = []
    for D in Ds:
        H, W = D.shape
        bufs.append(dict(disp=torch.from_numpy(D).to(DEV), cam=cam,
                         labels=torch.empty((H, W), dtype=torch.int32, device=DEV),
                         points=torch.empty((H, W, 8), device=DEV),
                         disp_dn=torch.empty((H, W), device=DEV),
                         num_components=torch.zeros(1, dtype=torch.int32, device=DEV)))
    plan = snx.Plan(bufs, filter_window=filter_window, normal_window=3, k_rel=0.0, t_abs=1.0)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    return ([b["labels"].cpu().numpy() for b in bufs],
            [int(b["num_components"].item()) for b in bufs])


def _check(oracle, Ds, labs, cnts):
    for i, (D, lab, cnt) in enumerate(zip(Ds, labs, cnts)):
        ref, nref = oracle.components(D, 0.0, 1.0)
        assert np.array_equal(lab, ref), (i, D, lab, ref)
        assert cnt == nref, (i, cnt, nref)


def test_every_validity_mask_of_a_4x3_frame(oracle):
    import paper_2504_15121_amd as snx
    snx.load()
    print("case 4096 masks of 4x3", flush=True)
    rng = np.random.default_rng(12)
    Ds = _frames((3, 4), 4096, rng, masks=np.arange(4096))
    labs, cnts = _run(snx, Ds)
    _check(oracle, Ds, labs, cnts)


@pytest.mark.parametrize("filter_window", [1, 3])
def test_seam_crossing_frames(oracle, filter_window):
    """With the 3x3 filter the batch front writes seam records and the merge
    reads them; with window 1 the merge decides the pairs itself."""
    import paper_2504_15121_amd as snx
    snx.load()
    print(f"case 256 frames of 70x37, filter {filter_window}", flush=True)
    rng = np.random.default_rng(13)
    Ds = _frames((37, 70), 256, rng)
    labs, cnts = _run(snx, Ds, filter_window)
    _check(oracle, Ds, labs, cnts)


# ---------------------------------------------------------------------------
# Every edge pattern of a 3x4 grid, independently of validity, through the
# labelling's edge-graph hook (snx_components_from_edges), against the oracle's
# breadth-first labelling of the same graph.
_GRID_EDGES = ([(r, c, 2) for r in range(3) for c in range(1, 4)] +     # to the left
               [(r, c, 4) for r in range(1, 3) for c in range(4)])     # upwards


def _all_graphs(present_frac, seed, per_row=40):
    """All 2^17 edge subsets of a 3x4 grid as 3x4 blocks of one image: block k at
    rows 3 (k // per_row), columns 2 + 4 (k % per_row).  The two empty columns on
    the left make blocks straddle the vertical tile seams (x = 64, 128) and the
    3-row blocks straddle the horizontal seams every 32 rows.  No edge joins two
    blocks.  present_frac < 1 removes random pixels (their edge bits stay set and
    must be ignored)."""
    n = 1 << 17
    k = np.arange(n)
    blocks = np.ones((n, 3, 4), np.uint8)
    for e, (r, c, bit) in enumerate(_GRID_EDGES):
        blocks[:, r, c] |= (((k >> e) & 1) * bit).astype(np.uint8)
    if present_frac < 1.0:
        rng = np.random.default_rng(seed)
        blocks &= np.where(rng.random((n, 3, 4)) < present_frac, 0xFF, 0xFE).astype(np.uint8)
    rows = (n + per_row - 1) // per_row
    img = np.zeros((3 * rows, 2 + 4 * per_row), np.uint8)
    for j in range(n):
        y, x = 3 * (j // per_row), 2 + 4 * (j % per_row)
        img[y:y + 3, x:x + 4] = blocks[j]
    return img


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _labels_from_edges(flags, pad=0):
    snx = _snx()
    H, W = flags.shape
    f = torch.zeros((H, W + 3), dtype=torch.uint8, device=DEV)
    f[:, :W] = torch.from_numpy(flags).to(DEV)
    lab = torch.full((H, W + pad), -7, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_components_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_components_from_edges(f[:, :W], lab[:, :W], ws, num_components=cnt)
    torch.cuda.synchronize()
    return lab[:, :W].cpu().numpy(), int(cnt.item())


@pytest.mark.parametrize("present_frac,pad", [(1.0, 0), (0.8, 5)])
def test_every_3x4_edge_graph(oracle, present_frac, pad):
    print(f"case all 2^17 edge graphs of a 3x4 grid, present {present_frac}, label pad {pad}",
          flush=True)
    flags = _all_graphs(present_frac, seed=7)
    lab, cnt = _labels_from_edges(flags, pad)
    ref, cref = oracle.components_edges(flags)
    assert np.array_equal(lab, ref), int((lab != ref).sum())
    assert cnt == cref


@pytest.mark.parametrize("H,W,p_edge", [(517, 1001, 0.7), (1080, 1920, 0.55), (33, 65, 0.9),
                                        (1, 300, 0.8), (300, 1, 0.8)])
def test_random_edge_graphs(oracle, H, W, p_edge):
    """Random presence and edge bits everywhere (bits on the image border too,
    which must be ignored) on ragged frames; near the percolation threshold the
    components are long and wind across many tile seams."""
    print(f"case random edge graph {W}x{H} p={p_edge}", flush=True)
    rng = np.random.default_rng(H * 7 + W)
    flags = (rng.random((H, W)) < 0.95).astype(np.uint8)
    flags |= (rng.random((H, W)) < p_edge).astype(np.uint8) << 1
    flags |= (rng.random((H, W)) < p_edge).astype(np.uint8) << 2
    flags |= (rng.random((H, W)) < 0.5).astype(np.uint8) << 5      # an unused bit
    lab, cnt = _labels_from_edges(flags)
    ref, cref = oracle.components_edges(flags)
    assert np.array_equal(lab, ref), int((lab != ref).sum())
    assert cnt == cref


def test_edge_graph_hook_rejects_bad_arguments():
    snx = _snx()
    f = torch.zeros((4, 4), dtype=torch.uint8, device=DEV)
    lab = torch.zeros((4, 4), dtype=torch.int32, device=DEV)
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(snx.SnxError) as ei:
        snx.snx_components_from_edges(f, lab, small)
    assert ei.value.status == 3
