"""Pins of the oracle's normal (Sec. 3.1) and of the whole plain pipeline."""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

from synth import scenes
from conftest import angle_deg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inside_one_patch(patch, size):
    lo = ndimage.minimum_filter(patch, size=size, mode="constant", cval=-5)
    hi = ndimage.maximum_filter(patch, size=size, mode="constant", cval=-5)
    return (lo == hi) & (patch >= 0)


@pytest.mark.parametrize("nf,ng", [(1, 3), (3, 5), (5, 9)])
def test_noise_free_planes_recover_ground_truth(oracle, nf, ng):
    """On noise-free piecewise-planar input the disparity is affine in (u, v), so
    every pixel whose combined footprint lies inside one plane gets the plane's
    normal (closed form, Sec. 2 eq. affine_mtx inverted by Sec. 3.1)."""
    sc = scenes.planes_scene(width=200, height=150, f=400.0, n_planes=4,
                             sigma=0.0, invalid_frac=0.0, seed=11 + nf)
    r = oracle.pipeline(sc.clean, sc.cam, nf=nf, ng=ng)
    Dt = oracle.denoise(sc.clean, nf)          # FP64 input (no float32 rounding)
    a1, a2, d = oracle.affine(Dt, ng)
    n = oracle.normals(Dt, a1, a2, d, sc.cam)
    inside = _inside_one_patch(sc.patch, nf + ng - 1) & d
    assert inside.sum() > 10000
    err = np.radians(angle_deg(n, sc.normal, signed=True))[inside]
    assert err.max() < 1e-9
    # the float32 pipeline on the same scene is within float32 quantisation
    err32 = np.radians(angle_deg(r["normals"], sc.normal, signed=True))[inside & r["defined"]]
    assert err32.max() < 5e-4


def test_fronto_parallel_plane(oracle):
    cam = scenes.Camera.centred(40, 30, 250.0, 0.1)
    D = np.full((30, 40), 12.5)
    a1, a2, d = oracle.affine(D, 5)
    n = oracle.normals(D, a1, a2, d, cam)
    np.testing.assert_allclose(n[d], np.tile([0.0, 0.0, -1.0], (d.sum(), 1)), atol=1e-15)


def test_normals_face_the_camera(oracle):
    sc = scenes.planes_quadrics_scene(width=320, height=200, f=300.0, n_planes=6,
                                      n_spheres=3, sigma=0.8, seed=3)
    r = oracle.pipeline(sc.disp, sc.cam, nf=3, ng=5)
    n, pts, d = r["normals"], r["points"], r["defined"]
    dots = (n * pts[..., :3]).sum(-1)
    assert d.sum() > 20000
    assert np.all(dots[d] < 0)
    np.testing.assert_allclose(np.linalg.norm(n[d], axis=-1), 1.0, atol=1e-14)


def test_printed_sign_of_b_would_fail(oracle):
    """The constraint-vector cross product gives -b f_x in the third component;
    the +b printed in the paper's closed form is tens of degrees off on a
    slanted plane.  Guards the reading against regressions."""
    cam = scenes.Camera.centred(64, 48, 300.0, 0.2)
    n_true = np.array([0.4, -0.3, -np.sqrt(1 - 0.25)])
    v, u = np.mgrid[0:48, 0:64].astype(np.float64)
    rays = np.stack([(u - cam.u0) / cam.fx, (v - cam.v0) / cam.fy, np.ones_like(u)], -1)
    z = -5.0 / (rays @ n_true)
    D = cam.fx * cam.baseline / z
    a1, a2, d = oracle.affine(D, 5)
    n = oracle.normals(D, a1, a2, d, cam)
    err = angle_deg(n, n_true[None, None, :], signed=True)[d]
    assert err.max() < 1e-8
    # printed form: [f_x z (a1-1), f_y z a2, -f_x x (a1-1) - f_y y a2 + b f_x]
    X = np.stack([(u - cam.u0) * z / cam.fx, (v - cam.v0) * z / cam.fy, z], -1)
    pr = np.stack([cam.fx * z * (a1 - 1), cam.fy * z * a2,
                   -cam.fx * X[..., 0] * (a1 - 1) - cam.fy * X[..., 1] * a2
                   + cam.baseline * cam.fx], -1)
    pr /= np.linalg.norm(pr, axis=-1, keepdims=True)
    assert angle_deg(pr, n_true[None, None, :])[d].mean() > 5.0


def test_sphere_table_soft_pin(oracle):
    """The paper's sphere table (Sec. 4, Table noise-compare, Affine rows):
    plain n x n affine estimator, no pre-filter, mean over 8 noise draws.
    Tolerance 0.15 deg for n <= 9 and 0.2 deg for n = 15.  The paper's figure is
    one noise draw: over seeds the mean of one draw spreads by 0.01-0.08 deg
    (standard deviation), so a single draw lies within about 0.15 deg of the
    expectation; the focal length (not stated, 500 px assumed) and the handling
    of the sphere's rim add a small systematic part (at n = 15, sigma = 0.2 the
    paper's 0.97 deg against 0.89 deg here)."""
    tab = json.load(open(os.path.join(GOLDEN, "sphere_noise_table.json")))
    for key, sigma in (("sigma_0.2", 0.2), ("sigma_1.0", 1.0)):
        ours = {n: [] for n in tab["window"]}
        for seed in range(8):
            sc = scenes.sphere_scene(sigma=sigma, seed=seed)
            D = sc.disp.astype(np.float64)
            for n in tab["window"]:
                a1, a2, d = oracle.affine(D, n)
                nrm = oracle.normals(D, a1, a2, d, sc.cam)
                m = d & np.isfinite(sc.normal[..., 0])
                ours[n].append(angle_deg(nrm, sc.normal)[m].mean())
        for n, paper in zip(tab["window"], tab[key]):
            tol = 0.15 if n <= 9 else 0.2
            mean = float(np.mean(ours[n]))
            assert abs(mean - paper) <= tol, (sigma, n, mean, paper)


def test_point_cloud_reprojects(oracle):
    """X of each point projects back through Pi_1 to its pixel, and
    Pi_1u(X) - Pi_2u(X) equals the filtered disparity (Sec. 2 projections)."""
    sc = scenes.planes_scene(width=96, height=64, f=200.0, sigma=0.3, seed=4)
    r = oracle.pipeline(sc.disp, sc.cam, nf=3, ng=5)
    P, d, Dt = r["points"], r["defined"], r["denoised"]
    cam = sc.cam
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    v, u = np.mgrid[0:64, 0:96].astype(np.float64)
    p1u = (cam.fx * x + cam.u0 * z) / z
    p1v = (cam.fy * y + cam.v0 * z) / z
    p2u = (cam.fx * (x - cam.baseline) + cam.u0 * z) / z
    np.testing.assert_allclose(p1u[d], u[d], atol=1e-9)
    np.testing.assert_allclose(p1v[d], v[d], atol=1e-9)
    np.testing.assert_allclose((p1u - p2u)[d], Dt[d], rtol=1e-12)
    assert np.all(np.isnan(P[~d]))
    np.testing.assert_array_equal(P[..., 3:][d], r["normals"][d])
