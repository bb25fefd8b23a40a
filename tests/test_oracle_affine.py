"""Pins of the oracle's affine parameters a1, a2 (Sec. 2, Sec. 3.2-3.3)."""
import numpy as np
import pytest

from synth import scenes


def test_kernel_layout_3x3(oracle):
    """A unit disparity bump at offset v recovers -s_1(v) and -s_2(v) of the full
    3x3 window (alpha = gamma = 6, beta = 0 by hand count), laid out as in the
    paper's 3x3 kernel figure: row -1 on top, column -1 on the left."""
    k1 = np.zeros((3, 3))
    k2 = np.zeros((3, 3))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            D = np.full((5, 5), 50.0)
            D[2 + dy, 2 + dx] += 1.0
            a1, a2, d = oracle.affine(D, 3)
            assert d[2, 2]
            # d_i - d_c = -1 at the bump (paper's d = -D), so a1 - 1 = -s_1
            k1[dy + 1, dx + 1] = -(a1[2, 2] - 1.0)
            k2[dy + 1, dx + 1] = -a2[2, 2]
    np.testing.assert_allclose(k1, np.array([[-1, 0, 1]] * 3) / 6.0, atol=1e-15)
    np.testing.assert_allclose(k2, np.array([[-1, -1, -1], [0, 0, 0], [1, 1, 1]]) / 6.0,
                               atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 9, 15])
def test_full_window_alpha_closed_form(oracle, n):
    """alpha = sum of v_x^2 over the full n x n window = n r (r+1) (2r+1) / 3."""
    r = n // 2
    alpha = n * r * (r + 1) * (2 * r + 1) // 3
    assert {3: 6, 5: 50, 9: 540, 15: 4200}[n] == alpha
    D = np.full((n + 4, n + 4), 20.0)
    c = (n + 4) // 2
    D[c, c + 1] += 1.0
    a1, a2, d = oracle.affine(D, n)
    assert d[c, c]
    assert abs(-1.0 / (a1[c, c] - 1.0) - alpha) < 1e-9 * alpha
    assert abs(a2[c, c]) < 1e-15


@pytest.mark.parametrize("ng", [3, 5, 9])
def test_exact_on_affine_disparity_with_masks(oracle, ng):
    rng = np.random.default_rng(ng)
    v, u = np.mgrid[0:20, 0:27].astype(np.float64)
    p, q = 0.37, -0.21
    D = 60.0 + p * u + q * v
    D[rng.random(D.shape) < 0.25] = np.nan
    a1, a2, d = oracle.affine(D, ng, min_support=3)
    assert d.sum() > 100
    np.testing.assert_allclose(a1[d], 1.0 - p, atol=1e-12)
    np.testing.assert_allclose(a2[d], -q, atol=1e-12)


def _affine_from_normal(n, X, cam):
    """The paper's closed form (eq. affine_mtx) from a normal and a 3-D point."""
    b, fx, fy = cam.baseline, cam.fx, cam.fy
    nX = n[0] * X[0] + n[1] * X[1] + n[2] * X[2]
    a1 = (n[0] * (X[0] - b) + n[1] * X[1] + n[2] * X[2]) / nX
    a2 = -b * fx * n[1] / (fy * nX)
    return a1, a2


def test_matches_closed_form_from_ground_truth_normals(oracle):
    sc = scenes.planes_scene(width=160, height=120, f=300.0, n_planes=3,
                             sigma=0.0, invalid_frac=0.0, seed=7)
    D = sc.clean
    ng = 5
    a1, a2, d = oracle.affine(D, ng)
    cam = sc.cam
    # pixels whose whole window lies inside one patch (and inside the image)
    from scipy import ndimage
    lo = ndimage.minimum_filter(sc.patch, size=ng, mode="constant", cval=-5)
    hi = ndimage.maximum_filter(sc.patch, size=ng, mode="constant", cval=-5)
    same = lo == hi
    vv, uu = np.nonzero(same & d)
    assert len(vv) > 5000
    z = cam.fx * cam.baseline / D[vv, uu]
    X = np.stack([(uu - cam.u0) * z / cam.fx, (vv - cam.v0) * z / cam.fy, z], 1)
    n = sc.normal[vv, uu]
    ref1, ref2 = _affine_from_normal(n.T, X.T, cam)
    np.testing.assert_allclose(a1[vv, uu], ref1, atol=1e-9)
    np.testing.assert_allclose(a2[vv, uu], ref2, atol=1e-9)


def _proj1(X, cam):
    return np.array([cam.fx * X[0] / X[2] + cam.u0, cam.fy * X[1] / X[2] + cam.v0])


def _proj2(X, cam):
    return np.array([cam.fx * (X[0] - cam.baseline) / X[2] + cam.u0,
                     cam.fy * X[1] / X[2] + cam.v0])


def _grad(f, X, h=1e-6):
    g = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[:, k] = (f(X + e) - f(X - e)) / (2 * h)
    return g


def test_general_formula_reduces_to_rectified_form():
    """eq. affine-matrix-general with w1..w5 from numerically differentiated
    projections gives a3 = 0, a4 = 1 and the rectified a1, a2 (Sec. 2)."""
    cam = scenes.Camera(700.0, 650.0, 0.25, 320.0, 240.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        X = np.array([rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(3, 9)])
        n = scenes.cone_normal(rng, 50.0)
        g1 = _grad(lambda Y: _proj1(Y, cam), X)
        g2 = _grad(lambda Y: _proj2(Y, cam), X)
        P1u, P1v, P2u, P2v = g1[0], g1[1], g2[0], g2[1]
        w1 = np.cross(P1v, P2u)
        w2 = np.cross(P2u, P1u)
        w3 = np.cross(P1v, P2v)
        w4 = np.cross(P2v, P1u)
        w5 = np.cross(P1v, P1u)
        A = np.array([[n @ w1, n @ w2], [n @ w3, n @ w4]]) / (n @ w5)
        a1, a2 = _affine_from_normal(n, X, cam)
        np.testing.assert_allclose(A, [[a1, a2], [0.0, 1.0]], atol=1e-6)


def _brute_force_affine(D, ng, need):
    H, W = D.shape
    r = ng // 2
    a = np.full((H, W, 2), np.nan)
    for v in range(H):
        for u in range(W):
            dc = D[v, u]
            if not (np.isfinite(dc) and dc > 0):
                continue
            V, d = [], []
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    if dx == 0 and dy == 0:
                        continue
                    uu, vv = u + dx, v + dy
                    if 0 <= uu < W and 0 <= vv < H and np.isfinite(D[vv, uu]) and D[vv, uu] > 0:
                        V.append([dx, dy])
                        d.append(-D[vv, uu] + dc)   # d_i - d_c with d = -D
            V = np.array(V, float).reshape(-1, 2)
            if len(V) < need or np.linalg.matrix_rank(V) < 2:
                continue
            a[v, u] = np.linalg.lstsq(V, np.array(d), rcond=None)[0]
    return a


@pytest.mark.parametrize("ng,frac", [(3, 0.2), (5, 0.35)])
def test_brute_force_lstsq(oracle, ng, frac):
    rng = np.random.default_rng(20 + ng)
    D = 25.0 + rng.normal(0, 1.5, (16, 16))
    D[rng.random(D.shape) < frac] = np.nan
    need = 4
    a1, a2, d = oracle.affine(D, ng, min_support=need)
    ref = _brute_force_affine(D, ng, need)
    assert np.array_equal(d, np.isfinite(ref[..., 0]))
    np.testing.assert_allclose(a1[d] - 1.0, ref[..., 0][d], atol=1e-11)
    np.testing.assert_allclose(a2[d], ref[..., 1][d], atol=1e-11)


def test_noise_law_full_window(oracle):
    """With i.i.d. N(0, sigma) noise and a full window, a1 - 1 ~ N(0, sigma^2/alpha)."""
    rng = np.random.default_rng(5)
    sigma, ng = 0.25, 9
    D = 40.0 + rng.normal(0, sigma, (260, 260))
    a1, a2, d = oracle.affine(D, ng)
    inner = (slice(4, -4), slice(4, -4))
    # neighbouring estimates overlap; use every 9th pixel in both directions
    s1 = (a1[inner][::9, ::9] - 1.0).ravel()
    s2 = a2[inner][::9, ::9].ravel()
    pred = sigma / np.sqrt(540.0)
    assert abs(s1.std() / pred - 1.0) < 0.1
    assert abs(s2.std() / pred - 1.0) < 0.1


def test_definedness_rules(oracle):
    D = np.full((7, 7), np.nan)
    D[3, :] = 10.0                      # neighbours only in the centre row: gamma = 0
    a1, a2, d = oracle.affine(D, 3, min_support=1)
    assert not d[3, 3]
    E = np.full((7, 7), 10.0)
    a1, a2, d = oracle.affine(E, 3)     # default min support 5 of 8
    assert d[1:-1].all() and d[:, 1:-1].all()
    assert not d[0, 0] and not d[-1, -1]   # image corners keep only 3 neighbours
    E[2, 2] = E[2, 3] = E[2, 4] = E[3, 2] = np.nan   # 4 of 8 neighbours left
    a1, a2, d = oracle.affine(E, 3)
    assert not d[3, 3]
    a1, a2, d = oracle.affine(E, 3, min_support=4)
    assert d[3, 3]
