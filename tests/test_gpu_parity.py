"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Stage-wise protocol: the filter is compared with the oracle's filter on the raw
input; gradients, A, normals and points are compared with the oracle run on the
GPU's own float32 denoised disparity, so each stage's error is isolated.

Tolerances (derived from the arithmetic):
  denoised   the GPU solves in FP64 and rounds once to FP32, so it is within
             one float32 ulp of the exact value: |err| <= 2^-22 |D|
  A          FP64 solve rounded to FP32: |err| <= 2^-22 |a| + 1e-12
  normals    <= 1e-4 rad (required bound); definedness must match exactly
             (both sides take it from exact integer tests on the same input)
  points     relative error <= 1e-5 on x, y, z; labels and flags exact
  labels     bit-exact, component count exact
"""
import math

import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAN = float("nan")


def _cam32(cam):
    f = lambda x: float(np.float32(x))
    return scenes.Camera(f(cam.fx), f(cam.fy), f(cam.baseline), f(cam.u0), f(cam.v0))


def _alloc(H, W, pad=0):
    ld = W + pad
    return dict(
        dn=torch.full((H, ld), NAN, device=DEV),
        aff=torch.full((2, H, ld), NAN, device=DEV),
        nrm=torch.full((3, H, ld), NAN, device=DEV),
        lab=torch.full((H, ld), -7, dtype=torch.int32, device=DEV),
        cnt=torch.full((1,), -1, dtype=torch.int32, device=DEV),
        pts=torch.full((max(H, 1), max(W, 1), 8), NAN, device=DEV),
        ws=torch.empty(max(1, _snx().snx_pipeline_workspace_size(W, H)), dtype=torch.uint8,
                       device=DEV),
    )


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _to_dev(D, pad=0):
    H, W = D.shape
    t = torch.full((H, W + pad), NAN, device=DEV)
    t[:, :W] = torch.from_numpy(np.ascontiguousarray(D))
    return t[:, :W]


def run_separate(D, cam, nf, ng, k=0.1, t=1.0, pad=0, ms_g=0):
    snx = _snx()
    H, W = D.shape
    o = _alloc(H, W, pad)
    d = _to_dev(D, pad)
    snx.snx_denoise(d, o["dn"][:, :W], window=nf)
    snx.snx_affine_normals(o["dn"][:, :W], cam, affine=o["aff"], normals=o["nrm"], window=ng,
                           min_support=ms_g)
    snx.snx_components(d, o["lab"][:, :W], o["ws"], num_components=o["cnt"], k_rel=k, t_abs=t)
    snx.snx_point_cloud(o["dn"][:, :W], o["nrm"], o["lab"][:, :W], cam, o["pts"])
    torch.cuda.synchronize()
    return _host(o, H, W)


def run_fused(D, cam, nf, ng, k=0.1, t=1.0, pad=0, ms_g=0):
    snx = _snx()
    H, W = D.shape
    o = _alloc(H, W, pad)
    d = _to_dev(D, pad)
    snx.snx_pipeline(d, cam, o["lab"][:, :W], o["pts"], o["ws"], num_components=o["cnt"],
                     disp_dn=o["dn"][:, :W], affine=o["aff"], normals=o["nrm"],
                     filter_window=nf, normal_window=ng, normal_min_support=ms_g,
                     k_rel=k, t_abs=t)
    torch.cuda.synchronize()
    return _host(o, H, W)


def run_oriented(D, cam, nf, ng, k=0.1, t=1.0, pad=0, ms_g=0):
    """snx_components then the fused filter+gradient+records call."""
    snx = _snx()
    H, W = D.shape
    o = _alloc(H, W, pad)
    d = _to_dev(D, pad)
    snx.snx_components(d, o["lab"][:, :W], o["ws"], num_components=o["cnt"], k_rel=k, t_abs=t)
    snx.snx_oriented_point_cloud(d, cam, o["pts"], labels=o["lab"][:, :W], disp_dn=o["dn"][:, :W],
                                 affine=o["aff"], normals=o["nrm"], filter_window=nf,
                                 normal_window=ng, normal_min_support=ms_g)
    torch.cuda.synchronize()
    return _host(o, H, W)


def run_parts(D, cam, nf, ng, k=0.1, t=1.0, pad=0, ms_g=0):
    """snx_pipeline_part(forest) then snx_pipeline_part(points)."""
    snx = _snx()
    H, W = D.shape
    o = _alloc(H, W, pad)
    d = _to_dev(D, pad)
    for part in (snx.PART_FOREST, snx.PART_POINTS):
        snx.snx_pipeline_part(d, cam, o["lab"][:, :W], o["pts"], o["ws"], parts=part,
                              num_components=o["cnt"], disp_dn=o["dn"][:, :W], affine=o["aff"],
                              normals=o["nrm"], filter_window=nf, normal_window=ng,
                              normal_min_support=ms_g, k_rel=k, t_abs=t)
    torch.cuda.synchronize()
    return _host(o, H, W)


def _host(o, H, W):
    return dict(dn=o["dn"][:, :W].cpu().numpy(), aff=o["aff"][:, :, :W].cpu().numpy(),
                nrm=o["nrm"][:, :, :W].cpu().numpy(), lab=o["lab"][:, :W].cpu().numpy(),
                cnt=int(o["cnt"].item()),
                pts=o["pts"].cpu().numpy()[:H, :W] if H and W else np.zeros((H, W, 8), np.float32))


def check_parity(oracle, D, cam, nf, ng, g, k=0.1, t=1.0, ms_g=None):
    """Stage-wise comparison; returns the maximum normal angle in radians."""
    H, W = D.shape
    # filter on the raw input
    ref = oracle.denoise(D.astype(np.float64), nf)
    assert np.array_equal(np.isnan(ref), np.isnan(g["dn"]))
    m = np.isfinite(ref)
    err = np.abs(g["dn"][m].astype(np.float64) - ref[m])
    assert np.all(err <= 2.0 ** -22 * np.abs(ref[m])), err.max()
    # gradients, A, normals on the GPU's own denoised disparity
    dn64 = g["dn"].astype(np.float64)
    a1, a2, dfn = oracle.affine(dn64, ng, ms_g)
    nref = oracle.normals(dn64, a1, a2, dfn, cam)
    gdef = np.isfinite(g["nrm"][0])
    assert np.array_equal(gdef, dfn), (gdef != dfn).sum()
    assert np.all(np.isnan(g["aff"][:, ~dfn])) and np.all(np.isnan(g["nrm"][:, ~dfn]))
    for gp, rp in ((g["aff"][0], a1), (g["aff"][1], a2)):
        e = np.abs(gp[dfn].astype(np.float64) - rp[dfn])
        assert np.all(e <= 2.0 ** -22 * np.abs(rp[dfn]) + 1e-12), e.max()
    ng_ = np.moveaxis(g["nrm"], 0, -1).astype(np.float64)[dfn]
    nr = nref[dfn]
    ang = np.arctan2(np.linalg.norm(np.cross(ng_, nr), axis=-1), (ng_ * nr).sum(-1))
    max_ang = float(ang.max()) if ang.size else 0.0
    assert max_ang <= 1e-4, max_ang
    # labels on the raw input
    lab, cnt = oracle.components(D, k, t)
    assert np.array_equal(g["lab"], lab)
    assert g["cnt"] == cnt
    # point records
    pref = oracle.point_cloud(dn64, nref, cam)
    P = g["pts"]
    xyz = P[..., :3].astype(np.float64)
    assert np.all(np.isnan(xyz[~dfn]))
    rel = np.abs(xyz[dfn] - pref[..., :3][dfn]) / np.maximum(np.abs(pref[..., :3][dfn]), 1e-6)
    assert rel.size == 0 or rel.max() <= 1e-5, rel.max()
    np.testing.assert_array_equal(P[..., 3:6][dfn], np.moveaxis(g["nrm"], 0, -1)[dfn])
    li = P.view(np.int32)
    np.testing.assert_array_equal(li[..., 6], lab)
    flags = dfn.astype(np.int32) * 1 + (lab >= 0).astype(np.int32) * 2
    np.testing.assert_array_equal(li[..., 7], flags)
    return max_ang


def _same(a, b):
    for k in a:
        if k == "cnt":
            assert a[k] == b[k]
        else:
            assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), k


def test_planes_640x480_separate_and_fused(oracle):
    sc = scenes.workload("planes_640x480")
    cam = _cam32(sc.cam)
    print("case planes_640x480 nf=3 ng=9", flush=True)
    g = run_separate(sc.disp, cam, 3, 9)
    ang = check_parity(oracle, sc.disp, cam, 3, 9, g)
    print("max normal angle (rad)", ang)
    f = run_fused(sc.disp, cam, 3, 9)
    _same(g, f)
    _same(g, run_oriented(sc.disp, cam, 3, 9))
    _same(g, run_parts(sc.disp, cam, 3, 9))


@pytest.mark.parametrize("H,W,nf,ng,nanfrac,pad", [
    (1, 1, 3, 3, 0.0, 0),
    (1, 37, 3, 3, 0.0, 0),
    (37, 1, 1, 3, 0.0, 3),
    (5, 3, 3, 5, 0.1, 0),
    (70, 130, 3, 9, 0.05, 5),
    (17, 65, 5, 9, 0.3, 0),
    (33, 200, 1, 5, 0.0, 0),
    (64, 64, 9, 15, 0.08, 1),
    (100, 90, 3, 31, 0.05, 0),
    (19, 23, 3, 9, 1.0, 0),      # all invalid
])
def test_sizes_and_edges(oracle, H, W, nf, ng, nanfrac, pad):
    print(f"case H={H} W={W} nf={nf} ng={ng} nan={nanfrac} pad={pad}", flush=True)
    rng = np.random.default_rng(H * 1000 + W)
    cam = scenes.Camera.centred(W, H, 300.0, 0.125)
    v, u = np.mgrid[0:H, 0:W]
    D = (30.0 + 0.2 * u - 0.1 * v + rng.normal(0, 0.4, (H, W))).astype(np.float32)
    D[rng.random((H, W)) < nanfrac] = np.nan
    if H * W > 4:
        D.reshape(-1)[rng.integers(0, H * W, 2)] = -1.0    # non-positive = invalid
    g = run_separate(D, cam, nf, ng, pad=pad)
    check_parity(oracle, D, cam, nf, ng, g)
    f = run_fused(D, cam, nf, ng, pad=pad)
    _same(g, f)
    _same(g, run_oriented(D, cam, nf, ng, pad=pad))


@pytest.mark.parametrize("nf,ng", [(3, 45), (5, 45), (1, 61), (5, 61), (9, 23)])
def test_large_windows(oracle, nf, ng):
    """Gradient windows up to 61: the pipeline filters in a pass of its own when
    filter and gradient do not fit one tile; the one-kernel call refuses such
    windows with SNX_ERR_UNSUPPORTED instead."""
    snx = _snx()
    H, W = 150, 131
    print(f"case large windows nf={nf} ng={ng}", flush=True)
    rng = np.random.default_rng(ng * 10 + nf)
    cam = scenes.Camera.centred(W, H, 300.0, 0.125)
    v, u = np.mgrid[0:H, 0:W]
    D = (40.0 + 0.15 * u - 0.12 * v + rng.normal(0, 0.4, (H, W))).astype(np.float32)
    D[rng.random((H, W)) < 0.07] = np.nan
    g = run_separate(D, cam, nf, ng)
    check_parity(oracle, D, cam, nf, ng, g)
    _same(g, run_fused(D, cam, nf, ng))
    _same(g, run_parts(D, cam, nf, ng))
    try:
        o = run_oriented(D, cam, nf, ng)
    except snx.SnxError as e:
        assert e.status == 2, e
    else:
        _same(g, o)


def test_planes_quadrics_1920x1080_fused(oracle):
    sc = scenes.workload("planes_quadrics_1920x1080")
    cam = _cam32(sc.cam)
    print("case planes_quadrics_1920x1080 nf=3 ng=9 fused", flush=True)
    g = run_fused(sc.disp, cam, 3, 9)
    ang = check_parity(oracle, sc.disp, cam, 3, 9, g)
    print("max normal angle (rad)", ang)


def test_uneven_frames_small(oracle):
    frames = scenes.uneven_batch(n_frames=4, seed=3, size_scale=0.15)
    for i, sc in enumerate(frames):
        cam = _cam32(sc.cam)
        H, W = sc.disp.shape
        print(f"case uneven frame {i} {W}x{H}", flush=True)
        g = run_fused(sc.disp, cam, 3, 9)
        check_parity(oracle, sc.disp, cam, 3, 9, g)


def test_min_support_override(oracle):
    sc = scenes.planes_scene(width=150, height=100, f=250.0, seed=9, invalid_frac=0.3)
    cam = _cam32(sc.cam)
    print("case min_support 12", flush=True)
    g = run_separate(sc.disp, cam, 3, 7, ms_g=12)
    check_parity(oracle, sc.disp, cam, 3, 7, g, ms_g=12)


def test_deterministic_repeat():
    sc = scenes.planes_quadrics_scene(width=700, height=300, f=600.0, n_planes=12, n_spheres=4,
                                      seed=21)
    cam = _cam32(sc.cam)
    print("case determinism", flush=True)
    a = run_fused(sc.disp, cam, 3, 9)
    b = run_fused(sc.disp, cam, 3, 9)
    _same(a, b)


def test_road_1024_closed_form_accuracy(oracle):
    """Noise-free piecewise-planar input: GPU normals equal the analytic plane
    normals wherever the footprint lies inside one plane (float32 input)."""
    sc = scenes.road_scene(width=1024, height=512, f=1130.0, sigma=0.0, seed=4)
    cam = _cam32(sc.cam)
    D = sc.clean.astype(np.float32)
    D[~np.isfinite(sc.disp)] = np.nan
    print("case road noise-free", flush=True)
    g = run_fused(D, cam, 3, 9)
    from scipy import ndimage
    lo = ndimage.minimum_filter(sc.patch, size=11, mode="constant", cval=-5)
    hi = ndimage.maximum_filter(sc.patch, size=11, mode="constant", cval=-5)
    n = np.moveaxis(g["nrm"], 0, -1).astype(np.float64)
    inside = (lo == hi) & (sc.patch >= 0) & np.isfinite(n[..., 0])
    assert inside.sum() > 100000
    gt = sc.normal[inside]
    ang = np.arctan2(np.linalg.norm(np.cross(n[inside], gt), axis=-1), (n[inside] * gt).sum(-1))
    # float32 quantisation of the input only (the FP64 oracle gives the same)
    assert np.percentile(ang, 99.9) < 1e-5, np.percentile(ang, 99.9)


def _labels_gpu(D, pad):
    snx = _snx()
    H, W = D.shape
    d = _to_dev(D, pad)
    lab = torch.full((H, W + pad), -7, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_components_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_components(d, lab[:, :W], ws, num_components=cnt)
    torch.cuda.synchronize()
    return lab[:, :W].cpu().numpy(), int(cnt.item())


def _serpentine(H, W):
    D = np.full((H, W), np.nan, np.float32)
    for r in range(0, H, 4):
        D[r:r + 2, :] = 10.0
        c = W - 2 if (r // 4) % 2 == 0 else 0
        D[r:r + 4, c:c + 2] = 10.0
    return D


@pytest.mark.parametrize("kind", ["serpentine", "checker", "levels", "stripes"])
@pytest.mark.parametrize("pad", [0, 7])
def test_components_adversarial(oracle, kind, pad):
    print(f"case components {kind} pad={pad}", flush=True)
    rng = np.random.default_rng(len(kind) + pad)
    if kind == "serpentine":
        D = _serpentine(998, 701)
    elif kind == "checker":
        v, u = np.mgrid[0:300, 0:517]
        D = np.where((u + v) % 2 == 0, 10.0, 50.0).astype(np.float32)
    elif kind == "levels":
        D = rng.choice([5.0, 5.4, 6.0, 9.0, 9.9, 10.9, 20.0], size=(555, 777)).astype(np.float32)
        D += rng.normal(0, 0.05, D.shape).astype(np.float32)
        D[rng.random(D.shape) < 0.1] = np.nan
    else:
        v, u = np.mgrid[0:260, 0:640]
        D = np.where((u // 64) % 2 == 0, 10.0, 40.0).astype(np.float32)
        D[(v % 32) == 0] = np.nan
    lab, cnt = _labels_gpu(D, pad)
    ref, n = oracle.components(D, 0.1, 1.0)
    assert np.array_equal(lab, ref), (lab != ref).sum()
    assert cnt == n


def test_tile_heights_do_not_change_outputs():
    """Every compiled tile height (and the autotuner's choice) gives bitwise
    identical results."""
    snx = _snx()
    sc = scenes.planes_quadrics_scene(width=700, height=333, f=600.0, n_planes=12, n_spheres=4,
                                      seed=31)
    cam = _cam32(sc.cam)
    H, W = sc.disp.shape
    print("case tile heights", flush=True)
    ref = run_fused(sc.disp, cam, 3, 9)
    ref_o = run_oriented(sc.disp, cam, 3, 9)
    for th in (8, 16, 32):
        snx.snx_tune_set(W, H, 1, 9, th)
        snx.snx_tune_set(W, H, 3, 9, th)
        _same(ref, run_fused(sc.disp, cam, 3, 9))
        _same(ref, run_oriented(sc.disp, cam, 3, 9))
    snx.snx_tune_set(W, H, 1, 9, 0)
    snx.snx_tune_set(W, H, 3, 9, 0)
    chosen = snx.snx_autotune(W, H, 3, 9)
    assert chosen[0] in (8, 16, 32) and chosen[1] in (8, 16, 32)
    _same(ref, run_fused(sc.disp, cam, 3, 9))
    _same(ref_o, run_oriented(sc.disp, cam, 3, 9))
    snx.snx_tune_set(W, H, 1, 9, 0)
    snx.snx_tune_set(W, H, 3, 9, 0)


@pytest.mark.parametrize("ng", [21, 31, 45, 61])
def test_large_window_tile_heights(oracle, ng):
    """The large gradient windows run in tall tiles (one workgroup a CU): every
    compiled tile height of the gradient pass gives bitwise identical results,
    the tallest one checked against the oracle too; and a batch plan on the
    same frame with each tile height (its persistent back stage) equals the
    single-frame pipeline."""
    from tests.test_gpu_batch import _check
    snx = _snx()
    H, W = 150, 131
    rng = np.random.default_rng(ng)
    cam = scenes.Camera.centred(W, H, 300.0, 0.125)
    v, u = np.mgrid[0:H, 0:W]
    D = (40.0 + 0.15 * u - 0.12 * v + rng.normal(0, 0.4, (H, W))).astype(np.float32)
    D[rng.random((H, W)) < 0.07] = np.nan
    ref = run_separate(D, cam, 1, ng)
    tallest = None
    try:
        for th in (4, 8, 16, 32):
            try:
                snx.snx_tune_set(W, H, 1, ng, th)
            except snx.SnxError as e:
                assert e.status == 2, e
                continue
            print(f"case large window ng={ng} tile height {th}", flush=True)
            g = run_separate(D, cam, 1, ng)
            _same(ref, g)
            tallest = th
            f = dict(disp=torch.from_numpy(D).to(DEV), cam=cam,
                     labels=torch.empty((H, W), dtype=torch.int32, device=DEV),
                     points=torch.empty((H, W, 8), device=DEV),
                     disp_dn=torch.empty((H, W), device=DEV),
                     num_components=torch.zeros(1, dtype=torch.int32, device=DEV))
            g2 = dict(f, disp=torch.from_numpy(D[::-1].copy()).to(DEV),
                      labels=torch.empty((H, W), dtype=torch.int32, device=DEV),
                      points=torch.empty((H, W, 8), device=DEV),
                      disp_dn=torch.empty((H, W), device=DEV),
                      num_components=torch.zeros(1, dtype=torch.int32, device=DEV))
            plan = snx.Plan([f, g2], filter_window=1, normal_window=ng)
            plan.run()
            torch.cuda.synchronize()
            _check(snx, [f, g2], 1, ng)
            plan.close()
        assert tallest is not None
        snx.snx_tune_set(W, H, 1, ng, tallest)
        check_parity(oracle, D, cam, 1, ng, run_separate(D, cam, 1, ng))
    finally:
        snx.snx_tune_set(W, H, 1, ng, 0)
