"""GPU parity of the component-restricted gradient window (the n_g window keeps
only the valid pixels carrying the centre's component label) through the C ABI
against the FP64 oracle, with the same labels handed to both sides (the
oracle's components of the raw disparity).

Definedness must match exactly (support counts and alpha*gamma - beta^2 are
exact integers on both sides); A and normals carry the square-window
tolerances: |err| <= 2^-22 |a| + 1e-12, normals <= 1e-4 rad.
"""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NAN = float("nan")


def _snx():
    import paper_2504_15121_amd as snx
    snx.load()
    return snx


def _cam32(cam):
    f = lambda x: float(np.float32(x))
    return scenes.Camera(f(cam.fx), f(cam.fy), f(cam.baseline), f(cam.u0), f(cam.v0))


def _check(oracle, D, lab, cam, ng, ms=None, pad=0):
    snx = _snx()
    H, W = D.shape
    ld = W + pad
    d = torch.full((max(H, 1), ld), NAN, device=DEV)
    d[:H, :W] = torch.from_numpy(np.ascontiguousarray(D, np.float32))
    lb = torch.full((max(H, 1), ld), -5, dtype=torch.int32, device=DEV)
    lb[:H, :W] = torch.from_numpy(np.ascontiguousarray(lab, np.int32))
    aff = torch.full((2, H, ld), NAN, device=DEV)
    nrm = torch.full((3, H, ld), NAN, device=DEV)
    snx.snx_affine_normals_labels(d[:H, :W], lb[:H, :W], cam, affine=aff, normals=nrm, window=ng,
                                  min_support=0 if ms is None else ms)
    torch.cuda.synchronize()
    ga, gn = aff[:, :, :W].cpu().numpy(), nrm[:, :, :W].cpu().numpy()
    D64 = D.astype(np.float64)
    a1, a2, dfn = oracle.affine_labels(D64, lab, ng, ms)
    gdef = np.isfinite(gn[0])
    assert np.array_equal(gdef, dfn), (gdef != dfn).sum()
    assert np.all(np.isnan(ga[:, ~dfn])) and np.all(np.isnan(gn[:, ~dfn]))
    for gp, rp in ((ga[0], a1), (ga[1], a2)):
        e = np.abs(gp[dfn].astype(np.float64) - rp[dfn])
        assert np.all(e <= 2.0 ** -22 * np.abs(rp[dfn]) + 1e-12), e.max()
    nref = oracle.normals(D64, a1, a2, dfn, cam)
    g = np.moveaxis(gn, 0, -1).astype(np.float64)[dfn]
    r = nref[dfn]
    ang = np.arctan2(np.linalg.norm(np.cross(g, r), axis=-1), (g * r).sum(-1))
    assert ang.size == 0 or ang.max() <= 1e-4, ang.max()
    return ga, int(dfn.sum())


@pytest.mark.parametrize("W,H,ng,ms,pad", [
    (160, 120, 9, None, 0), (130, 70, 3, None, 2), (100, 90, 5, 6, 0), (200, 50, 15, None, 0),
    (70, 40, 21, 30, 1), (64, 16, 31, 100, 0), (90, 33, 7, None, 0), (1, 1, 9, None, 0),
    (5, 3, 3, 1, 0), (67, 19, 11, 20, 0),
])
def test_restricted_matches_oracle(oracle, W, H, ng, ms, pad):
    print(f"case restricted {W}x{H} ng {ng} ms {ms} pad {pad}", flush=True)
    sc = scenes.planes_quadrics_scene(width=max(W, 8), height=max(H, 8), f=300.0, n_planes=6,
                                      n_spheres=2, seed=W * 17 + H)
    D = np.ascontiguousarray(sc.disp[:H, :W])
    lab, _ = oracle.components(D, 0.1, 1.0)
    _, n = _check(oracle, D, lab, _cam32(sc.cam), ng, ms, pad)
    if W * H >= 1000:
        assert n > 0


def test_restricted_two_planes(oracle):
    print("case restricted two planes", flush=True)
    H, W = 30, 70
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    D = np.where(u < 33, 20.0 + 0.0625 * u, 40.0 - 0.03125 * v).astype(np.float32)
    lab, n = oracle.components(D, 0.1, 1.0)
    assert n == 2
    cam = scenes.Camera(300.0, 300.0, 0.2, 35.0, 15.0)
    ga, _ = _check(oracle, D, lab, cam, 9)
    d = np.isfinite(ga[0])
    L, R = d & (u < 33), d & (u >= 33)
    assert np.abs(ga[0][L] - (1 - 0.0625)).max() <= 2e-7
    assert np.abs(ga[0][R] - 1.0).max() <= 1e-7 and np.abs(ga[1][R] - 0.03125).max() <= 1e-7


def test_restricted_one_component_equals_plain_window(oracle):
    # one label everywhere: the restricted window is the plain window
    snx = _snx()
    print("case restricted = plain on one component", flush=True)
    sc = scenes.planes_quadrics_scene(width=96, height=64, f=300.0, n_planes=4, n_spheres=1,
                                      seed=3)
    D = np.ascontiguousarray(sc.disp)
    lab = np.where(np.isfinite(D) & (D > 0), 0, -1).astype(np.int32)
    cam = _cam32(sc.cam)
    ga, _ = _check(oracle, D, lab, cam, 9)
    d = torch.from_numpy(D).to(DEV)
    aff = torch.empty((2,) + D.shape, device=DEV)
    snx.snx_affine_normals(d, cam, affine=aff, window=9)
    torch.cuda.synchronize()
    pa = aff.cpu().numpy()
    assert np.array_equal(np.isnan(pa), np.isnan(ga))
    m = np.isfinite(pa)
    assert np.abs(pa[m].astype(np.float64) - ga[m]).max() <= 2.0 ** -21 * np.abs(pa[m]).max()


def test_restricted_uniform_and_mixed_bands(oracle):
    """Each wave of the kernel owns four output rows of a 64 x 16 tile and takes
    the separable route where every valid pixel its windows reach carries one
    label; the rows of the other bands are shared among the tile's waves.  One
    plane, one label, with single pixels of a second label placed so that tiles
    hold one, two, three or all four mixed bands, and a block of valid pixels
    labelled -1 (no component: undefined outputs there): every route and every
    sharing of rows against the oracle."""
    print("case restricted uniform and mixed bands", flush=True)
    H, W = 64, 260
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    D = (30.0 + 0.05 * u - 0.03 * v).astype(np.float32)
    D[5, 7] = np.nan
    lab = np.zeros((H, W), np.int32)
    # foreign labels in tile columns 0-3; with windows 3, 9 and 15 the tiles
    # hold from none to all four mixed bands
    lab[1, 20] = 7
    lab[2, 80] = 7
    lab[9, 90] = 7
    lab[24, 150] = 9
    lab[32, 200:205] = 11
    # valid pixels without a component
    lab[48:60, 230:250] = -1
    cam = scenes.Camera(300.0, 300.0, 0.2, 130.0, 32.0)
    for ng in (3, 9, 15):
        _check(oracle, D, lab, cam, ng)
