"""GPU parity of the adaptive star-fill support (Sec. 3.4, Adaptive Region
Estimation) through the C ABI against the FP64 oracle, on the same float32
input.

The supports are integer decisions: both sides take every stopping decision in
binary64 from the same float32 values (the covered-depth products are exact,
the Laplacian is summed in the same order), so definedness must match exactly.
A and the normals then carry the tolerances of the square-window path: FP64
solve rounded once to FP32, |err| <= 2^-22 |a| + 1e-12, normals <= 1e-4 rad.
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


def _laplacian_threshold(D, cam, q):
    """A depth-Laplacian threshold at quantile q of |L| over the frame (only to
    pick a threshold that stops some rays and not others)."""
    z = cam.fx * cam.baseline / np.where(D > 0, D, np.nan).astype(np.float64)
    L = (z[1:-1, 2:] + z[1:-1, :-2]) + (z[2:, 1:-1] + z[:-2, 1:-1]) - 4 * z[1:-1, 1:-1]
    L = np.abs(L[np.isfinite(L)])
    return float(np.quantile(L, q)) if L.size else 1.0


def _run(D, cam, dirs, steps, stop, thr, ms=0, pad=0):
    snx = _snx()
    H, W = D.shape
    d = torch.full((max(H, 1), W + pad), NAN, device=DEV)
    d[:H, :W] = torch.from_numpy(np.ascontiguousarray(D, np.float32))
    ld = W + pad
    aff = torch.full((2, H, ld), NAN, device=DEV)
    nrm = torch.full((3, H, ld), NAN, device=DEV)
    snx.snx_affine_normals_star(d[:H, :W], cam, affine=aff, normals=nrm, directions=dirs,
                                steps=steps, stop=stop, threshold=thr, min_support=ms)
    torch.cuda.synchronize()
    return aff[:, :, :W].cpu().numpy(), nrm[:, :, :W].cpu().numpy()


def _check(oracle, D, cam, dirs, steps, stop, thr, ms=0, pad=0):
    ga, gn = _run(D, cam, dirs, steps, stop, thr, ms, pad)
    D64 = D.astype(np.float64)
    a1, a2, dfn = oracle.star_affine(D64, dirs, steps, stop, thr, cam=cam, min_support=ms)
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
    return int(dfn.sum())


CASES = [
    # W, H, directions, steps, rule, threshold (CD: k; ST: quantile of |L|), min_support, pad
    (160, 120, 8, 10, "cd", 0.05, 0, 0),
    (160, 120, 4, 6, "cd", 0.02, 0, 3),
    (130, 70, 8, 10, "st", 0.8, 0, 0),
    (130, 70, 4, 3, "st", 0.95, 0, 1),
    (200, 150, 8, 32, "cd", 0.1, 0, 0),
    (67, 19, 8, 1, "cd", 0.5, 0, 0),
    (90, 40, 8, 12, "cd", 0.2, 30, 0),
    (1, 1, 8, 5, "cd", 0.05, 0, 0),
    (5, 3, 4, 2, "st", 0.8, 0, 0),
    (64, 16, 8, 32, "st", 0.9, 0, 0),
    (160, 120, 16, 10, "cd", 0.05, 0, 0),
    (130, 70, 16, 10, "st", 0.8, 0, 2),
    (200, 150, 16, 30, "cd", 0.1, 0, 0),
    (67, 19, 16, 1, "cd", 0.5, 8, 0),        # one step: at most 8 distinct pixels
    (90, 40, 16, 12, "cd", 0.2, 60, 0),
    (5, 3, 16, 2, "st", 0.8, 0, 0),
    (64, 16, 16, 32, "st", 0.9, 0, 0),
]


@pytest.mark.parametrize("W,H,dirs,steps,rule,thr,ms,pad", CASES)
def test_star_matches_oracle(oracle, W, H, dirs, steps, rule, thr, ms, pad):
    snx = _snx()
    print(f"case star {W}x{H} dirs {dirs} steps {steps} {rule} {thr} ms {ms} pad {pad}",
          flush=True)
    sc = scenes.planes_quadrics_scene(width=max(W, 8), height=max(H, 8), f=300.0, n_planes=6,
                                      n_spheres=2, seed=W * 131 + H)
    D = np.ascontiguousarray(sc.disp[:H, :W])
    cam = _cam32(sc.cam)
    stop = snx.STOP_CD if rule == "cd" else snx.STOP_ST
    t = thr if rule == "cd" else _laplacian_threshold(D, cam, thr)
    n = _check(oracle, D, cam, dirs, steps, stop, t, ms, pad)
    if W * H >= 1000:
        assert n > 0


def test_star_keeps_a_step_edge_apart(oracle):
    snx = _snx()
    print("case star step edge", flush=True)
    H, W = 30, 70
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    D = np.where(u < 33, 20.0 + 0.0625 * u, 40.0 - 0.03125 * v).astype(np.float32)
    cam = scenes.Camera(300.0, 300.0, 0.2, 35.0, 15.0)
    ga, gn = _run(D, cam, 8, 8, snx.STOP_CD, 0.1)
    d = np.isfinite(ga[0])
    L, R = d & (u < 33), d & (u >= 33)
    assert L.sum() > 500 and R.sum() > 500
    assert np.abs(ga[0][L] - (1 - 0.0625)).max() <= 2e-7
    assert np.abs(ga[1][L]).max() <= 1e-7
    assert np.abs(ga[0][R] - 1.0).max() <= 1e-7
    assert np.abs(ga[1][R] - 0.03125).max() <= 1e-7
    _check(oracle, D, cam, 8, 8, snx.STOP_CD, 0.1)


def test_star_all_invalid():
    snx = _snx()
    print("case star all invalid", flush=True)
    D = np.full((20, 70), np.nan, np.float32)
    cam = scenes.Camera(300.0, 300.0, 0.2, 35.0, 10.0)
    ga, gn = _run(D, cam, 8, 4, snx.STOP_CD, 0.1)
    assert np.all(np.isnan(ga)) and np.all(np.isnan(gn))
