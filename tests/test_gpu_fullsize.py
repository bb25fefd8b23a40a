"""Full-size checks in the configurations bench.py times, on the 1920x1080
planes+quadrics frame, at sampled pixels whose reference the oracle computes on
a crop holding everything the pixel depends on:

* star-fill support (8 directions x 10 steps and 16 directions x 30 steps,
  covered depth and ST t = 2): a pixel's rays reach `steps` px and the depth
  Laplacian one more, so a crop of radius steps + 1 (cut at the image border)
  gives its exact support;
* component-restricted 9x9 window: radius 4, with the frame's labels.

Definedness must agree exactly; A within the square-window tolerance."""
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


def _cam32(cam):
    f = lambda x: float(np.float32(x))
    return scenes.Camera(f(cam.fx), f(cam.fy), f(cam.baseline), f(cam.u0), f(cam.v0))


def _samples(H, W, n=64, seed=3):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (H - 1, W - 1), (15, 63), (16, 64), (H - 1, 640), (540, W - 1)]
    return pts + [(int(v), int(u)) for v, u in zip(rng.integers(0, H, n), rng.integers(0, W, n))]


def _cmp(a_gpu, a_ref, d_ref, v, u):
    gdef = np.isfinite(a_gpu[0, v, u])
    assert gdef == bool(d_ref), (v, u)
    if gdef:
        for k in range(2):
            e = abs(float(a_gpu[k, v, u]) - a_ref[k])
            assert e <= 2.0 ** -22 * abs(a_ref[k]) + 1e-12, (v, u, k, e)


@pytest.fixture(scope="module")
def frame():
    snx = _snx()
    sc = scenes.workload("planes_quadrics_1920x1080")
    H, W = sc.disp.shape
    d = torch.from_numpy(sc.disp).to(DEV)
    dn = torch.empty((H, W), device=DEV)
    snx.snx_denoise(d, dn, window=3)
    lab = torch.empty((H, W), dtype=torch.int32, device=DEV)
    ws = torch.empty(snx.snx_components_workspace_size(W, H), dtype=torch.uint8, device=DEV)
    snx.snx_components(d, lab, ws)
    torch.cuda.synchronize()
    return sc, d, dn, lab


@pytest.mark.parametrize("dirs,steps,stop,thr", [(8, 10, 0, 0.05), (8, 10, 1, 2.0),
                                                  (16, 30, 0, 0.1), (16, 30, 1, 2.0)])
def test_star_full_frame_sampled(oracle, frame, dirs, steps, stop, thr):
    """Also the paper's own adaptive configurations, 16 directions x 30 steps
    (Sec. 4, the 1024x720 timing table): crop radius steps + 1."""
    snx = _snx()
    sc, _, dn, _ = frame
    print(f"case star full frame {dirs} dirs {steps} steps stop {stop} thr {thr}", flush=True)
    cam = _cam32(sc.cam)
    H, W = dn.shape
    aff = torch.empty((2, H, W), device=DEV)
    snx.snx_affine_normals_star(dn, cam, affine=aff, directions=dirs, steps=steps, stop=stop,
                                threshold=thr)
    torch.cuda.synchronize()
    a = aff.cpu().numpy()
    D = dn.cpu().numpy().astype(np.float64)
    rr = steps + 1
    for v, u in _samples(H, W):
        v0, v1, u0, u1 = max(0, v - rr), min(H, v + rr + 1), max(0, u - rr), min(W, u + rr + 1)
        r1, r2, rd = oracle.star_affine(D[v0:v1, u0:u1], dirs, steps, stop, thr, cam=cam)
        _cmp(a, (r1[v - v0, u - u0], r2[v - v0, u - u0]), rd[v - v0, u - u0], v, u)


def test_restricted_full_frame_sampled(oracle, frame):
    snx = _snx()
    sc, _, dn, lab = frame
    print("case restricted window full frame", flush=True)
    cam = _cam32(sc.cam)
    H, W = dn.shape
    aff = torch.empty((2, H, W), device=DEV)
    snx.snx_affine_normals_labels(dn, lab, cam, affine=aff, window=9)
    torch.cuda.synchronize()
    a = aff.cpu().numpy()
    D = dn.cpu().numpy().astype(np.float64)
    L = lab.cpu().numpy()
    for v, u in _samples(H, W, seed=4):
        v0, v1, u0, u1 = max(0, v - 4), min(H, v + 5), max(0, u - 4), min(W, u + 5)
        r1, r2, rd = oracle.affine_labels(D[v0:v1, u0:u1], L[v0:v1, u0:u1], 9)
        _cmp(a, (r1[v - v0, u - u0], r2[v - v0, u - u0]), rd[v - v0, u - u0], v, u)
