"""Pins of the oracle's adaptive star-fill support (Sec. 3.4, Adaptive Region
Estimation) against facts fixed independently of its code:

* the LSQ over any support of an exact plane returns the plane's slope;
* across a large disparity jump the covered-depth rule keeps every support on
  its own side, so each side gets its own plane's slope exactly (a plain
  window mixes the two);
* supports of hand-built cases, worked out by hand from the stopping rules
  (an invalid pixel, a covered-depth crossing, a depth-Laplacian spike);
* the exact step at which the covered-depth rule stops a ray on a ramp;
* 16 directions: the support drawn by hand from the ray reading (directions
  2 pi m / 16 scaled to a unit larger component, offsets rounded to the
  nearest pixel; neighbouring rays share their first pixel, which counts once).
"""
import numpy as np
import pytest

from oracle import oracle

CD, ST = oracle.STOP_CD, oracle.STOP_ST


class _Cam:
    def __init__(self, fx, b):
        self.fx, self.fy, self.baseline, self.u0, self.v0 = fx, fx, b, 0.0, 0.0


def _plane(W, H, d0, gu, gv):
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return d0 + gu * u + gv * v


@pytest.mark.parametrize("dirs", [4, 8, 16])
@pytest.mark.parametrize("steps,stop,thr", [(3, CD, 0.5), (7, CD, 0.01), (5, ST, 1e9), (6, CD, 0.02)])
def test_plane_slope_exact_on_any_support(dirs, steps, stop, thr):
    gu, gv = 0.125, -0.0625                     # exact binary fractions
    D = _plane(40, 36, 30.0, gu, gv)
    a1, a2, d = oracle.star_affine(D, dirs, steps, stop, thr, cam=_Cam(100.0, 1.0))
    assert d.sum() > 0.5 * d.size
    # Sec. 2: a1 = 1 - g_u, a2 = -g_v for the positive disparity D
    assert np.abs(a1[d] - (1.0 - gu)).max() < 1e-12
    assert np.abs(a2[d] - (-gv)).max() < 1e-12


def test_step_edge_support_stays_on_its_side():
    H, W = 30, 40
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    left = 20.0 + 0.05 * u
    right = 40.0 - 0.03 * v
    D = np.where(u < 20, left, right)
    a1, a2, d = oracle.star_affine(D, 8, 8, CD, 0.1)
    L, R = d & (u < 20), d & (u >= 20)
    assert L.sum() > 200 and R.sum() > 200
    assert np.abs(a1[L] - (1.0 - 0.05)).max() < 1e-12 and np.abs(a2[L]).max() < 1e-12
    assert np.abs(a1[R] - 1.0).max() < 1e-12 and np.abs(a2[R] - 0.03).max() < 1e-12
    # a plain 9x9 window next to the jump mixes the two planes
    w1, _, wd = oracle.affine(D, 9)
    near = wd & (np.abs(u - 19.5) < 3)
    assert np.abs(w1[near] - np.where(u[near] < 20, 0.95, 1.0)).max() > 0.1


def _expected(steps, taken):
    side = 2 * steps + 1
    m = np.zeros((side, side), bool)
    for (ex, ey), n in taken.items():
        for k in range(1, n + 1):
            m[k * ey + steps, k * ex + steps] = True
    return m


def test_mask_hand_case_invalid_and_cd():
    D = np.full((11, 11), 10.0)
    c = 5
    D[c, c + 2] = np.nan          # ray (1, 0): second pixel invalid -> takes k = 1
    D[c + 2, c] = 12.0            # ray (0, 1): 10 * 2 > 0.05 * 10 * 12 -> stops at k = 2
    D[c + 2, c + 2] = 10.4        # ray (1, 1): 10 * 0.4 <= 0.05 * 10 * 10.4 -> continues
    m8 = oracle.star_mask(D, c, c, 8, 3, CD, 0.05)
    taken = {(1, 0): 1, (1, 1): 3, (0, 1): 1, (-1, 1): 3,
             (-1, 0): 3, (-1, -1): 3, (0, -1): 3, (1, -1): 3}
    assert np.array_equal(m8, _expected(3, taken))
    m4 = oracle.star_mask(D, c, c, 4, 3, CD, 0.05)
    assert np.array_equal(m4, _expected(3, {(1, 0): 1, (0, 1): 1, (-1, 0): 3, (0, -1): 3}))
    # an invalid centre has no support
    D[c, c] = np.nan
    assert oracle.star_mask(D, c, c, 8, 3, CD, 0.05) is None


def test_cd_crossing_on_a_ramp():
    # along +u from the centre: D = 10 + 0.5 k.  With k_cd = 0.1 the ray takes
    # k = 1, 2 (10 * 1.0 <= 0.1 * 10 * 11) and stops at k = 3
    # (10 * 1.5 > 0.1 * 10 * 11.5).
    D = np.full((9, 15), 10.0)
    c = 3
    for k in range(1, 12 - c):
        D[4, c + k] = 10.0 + 0.5 * k
    m = oracle.star_mask(D, c, 4, 4, 6, CD, 0.1)
    assert m[6, 6 + 1] and m[6, 6 + 2] and not m[6, 6 + 3]


def test_st_depth_laplacian_spike():
    # flat depth z = fxb / 10 = 10 with one spike pixel (D = 5, z = 20) three
    # pixels below the centre: the Laplacian at the pixel above the spike is
    # z_spike - z = 10 > t = 1, so the downward ray takes k = 1 only; the
    # Laplacian is zero wherever no neighbour is the spike.
    cam = _Cam(100.0, 1.0)
    D = np.full((21, 21), 10.0)
    c = 10
    D[c + 3, c] = 5.0
    m = oracle.star_mask(D, c, c, 8, 5, ST, 1.0, cam=cam)
    taken = {(1, 0): 5, (1, 1): 5, (0, 1): 1, (-1, 1): 5,
             (-1, 0): 5, (-1, -1): 5, (0, -1): 5, (1, -1): 5}
    assert np.array_equal(m, _expected(5, taken))
    # next to the image border the Laplacian is undefined: the ray to the
    # right from (17, 10) takes k = 1, 2 (u = 18, 19) and stops at u = 20
    m = oracle.star_mask(D, 17, 10, 4, 5, ST, 1.0, cam=cam)
    assert m[5, 5 + 1] and m[5, 5 + 2] and not m[5, 5 + 3]


def test_min_support_default_and_override():
    D = np.full((7, 7), 10.0)
    D[3, 4] = np.nan               # centre (3, 3) loses its right neighbour
    _, _, d = oracle.star_affine(D, 4, 1, CD, 0.5)        # default: 4 pixels
    assert not d[3, 3] and d[2, 3]
    _, _, d = oracle.star_affine(D, 4, 1, CD, 0.5, min_support=3)
    assert d[3, 3]


def test_cd_is_a_depth_range_not_a_disparity_range():
    # centre D = 10 with a nearer-disparity neighbour on the right: the depth
    # range is f B (1/a - 1/b).  D = 6: 1/6 - 1/10 = 0.067 > 0.5/10, so the
    # ray stops at once although the disparity range 4 is below 0.5 * 10;
    # D = 7: 1/7 - 1/10 = 0.043 <= 0.05, so the pixel is taken.
    for d1, taken in ((6.0, False), (7.0, True)):
        D = np.full((5, 5), 10.0)
        D[2, 3] = d1
        m = oracle.star_mask(D, 2, 2, 4, 1, CD, 0.5)
        assert m[1, 1 + 1] == taken, d1


# The 16-direction star of 3 steps on a full window, drawn by hand: the 8
# compass rays (axes, diagonals) take 3 pixels each; the 8 rays in between
# (tan 22.5 deg = 0.414: offsets (1, 0), (2, 1), (3, 1) for the first one, the
# rest by symmetry) share their first pixel with an axis ray, so they add 2
# each: 24 + 16 = 40 pixels.  Rows are v = -3 .. 3, columns u = -3 .. 3.
STAR16_3 = ["#.###.#",
            ".#####.",
            "#######",
            "###.###",
            "#######",
            ".#####.",
            "#.###.#"]


def test_star16_mask_by_hand():
    # the hand drawing above, derived ray by ray
    want = np.zeros((7, 7), np.uint8)
    dirs8 = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    for dx, dy in dirs8:
        for k in (1, 2, 3):
            want[3 + k * dy, 3 + k * dx] = 1
    # the in-between rays: major component k, minor round(0.414 k) = 0, 1, 1
    for sx in (-1, 1):
        for sy in (-1, 1):
            for k, r in ((2, 1), (3, 1)):
                want[3 + sy * r, 3 + sx * k] = 1          # near the u axis
                want[3 + sy * k, 3 + sx * r] = 1          # near the v axis
    drawn = np.array([[c == "#" for c in row] for row in STAR16_3], np.uint8)
    np.testing.assert_array_equal(want, drawn)
    assert int(want.sum()) == 40
    D = _plane(21, 21, 30.0, 0.0, 0.0)
    mask = oracle.star_mask(D, 10, 10, dirs=16, steps=3, stop=CD, thr=0.5)
    np.testing.assert_array_equal(mask, want.astype(bool))
    # 8 directions are the compass subset of the same reading
    m8 = oracle.star_mask(D, 10, 10, dirs=8, steps=3, stop=CD, thr=0.5)
    assert m8.sum() == 24 and not np.any(m8 & ~want.astype(bool))


def test_star16_shared_first_pixel():
    """An invalid pixel right of the centre stops the u+ axis ray and both
    in-between rays next to it at their first step (they would share it)."""
    D = _plane(21, 21, 30.0, 0.0, 0.0)
    D[10, 11] = np.nan
    mask = oracle.star_mask(D, 10, 10, dirs=16, steps=3, stop=CD, thr=0.5)
    want = np.array([[c == "#" for c in row] for row in STAR16_3], bool)
    want[3, 4:] = False               # the u+ axis ray: (1,0), (2,0), (3,0)
    want[2, 5:] = False               # the ray at -22.5 deg: (2,-1), (3,-1)
    want[4, 5:] = False               # the ray at +22.5 deg: (2,1), (3,1)
    np.testing.assert_array_equal(mask, want)
    assert mask.sum() == 40 - 3 - 2 - 2
