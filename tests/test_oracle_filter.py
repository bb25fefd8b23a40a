"""Pins of the oracle's denoising filter (masked LSQ plane-fit intercept).

The filter is the over-determined LSQ of Sec. 3.2 with a constant column added,
so it is pinned by what a least-squares plane fit must do regardless of how it
is coded: reproduce planes exactly under any mask of rank 3, reduce to the box
mean on a full window, reduce to the identity on a 1x1 window, and agree with
numpy's SVD least squares pixel by pixel.
"""
import numpy as np
import pytest
from scipy import ndimage


def _affine_map(H, W, rng, c=40.0, p=0.3, q=-0.2):
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return c + p * u + q * v


@pytest.mark.parametrize("nf", [3, 5, 9])
def test_plane_is_preserved_under_masks(oracle, nf):
    rng = np.random.default_rng(nf)
    D = _affine_map(24, 31, rng)
    D[rng.random(D.shape) < 0.3] = np.nan
    out = oracle.denoise(D, nf)
    valid = np.isfinite(D)
    assert np.all(np.isnan(out[~valid]))
    np.testing.assert_allclose(out[valid], D[valid], rtol=0, atol=1e-10)


def test_full_window_is_box_mean(oracle):
    rng = np.random.default_rng(1)
    D = 20.0 + rng.normal(0, 1.0, (30, 40))
    for nf in (3, 5, 7):
        r = nf // 2
        ref = ndimage.uniform_filter(D, size=nf, mode="constant")
        out = oracle.denoise(D, nf)
        np.testing.assert_allclose(out[r:-r, r:-r], ref[r:-r, r:-r], rtol=0, atol=1e-11)


def test_window_one_is_identity(oracle):
    rng = np.random.default_rng(2)
    D = 5.0 + rng.random((9, 13))
    D[rng.random(D.shape) < 0.2] = np.nan
    D[0, 0] = -1.0  # non-positive disparity is invalid
    out = oracle.denoise(D, 1)
    ok = np.isfinite(D) & (D > 0)
    np.testing.assert_array_equal(out[ok], D[ok])
    assert np.all(np.isnan(out[~ok]))


def _brute_force_filter(D, nf, need=3):
    H, W = D.shape
    r = nf // 2
    out = np.full(D.shape, np.nan)
    for v in range(H):
        for u in range(W):
            dc = D[v, u]
            if not (np.isfinite(dc) and dc > 0):
                continue
            rows, rhs = [], []
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    uu, vv = u + dx, v + dy
                    if 0 <= uu < W and 0 <= vv < H:
                        di = D[vv, uu]
                        if np.isfinite(di) and di > 0:
                            rows.append([1.0, dx, dy])
                            rhs.append(di)
            A = np.array(rows).reshape(-1, 3)
            if len(rows) < need or np.linalg.matrix_rank(A) < 3:
                out[v, u] = dc
                continue
            sol = np.linalg.lstsq(A, np.array(rhs), rcond=None)[0]
            out[v, u] = sol[0]
    return out


@pytest.mark.parametrize("nf,frac", [(3, 0.25), (5, 0.4)])
def test_brute_force_lstsq(oracle, nf, frac):
    rng = np.random.default_rng(10 + nf)
    D = 30.0 + rng.normal(0, 2.0, (16, 16))
    D[rng.random(D.shape) < frac] = np.nan
    out = oracle.denoise(D, nf)
    ref = _brute_force_filter(D, nf)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    m = np.isfinite(ref)
    np.testing.assert_allclose(out[m], ref[m], rtol=0, atol=1e-10)


def test_collinear_support_passes_through(oracle):
    # only one row of the 3x3 window is valid: rank 2, the centre is returned
    D = np.full((3, 3), np.nan)
    D[1, :] = [10.0, 17.0, 11.0]
    out = oracle.denoise(D, 3)
    assert out[1, 1] == 17.0
    # min_support larger than the support also passes through
    E = np.arange(1.0, 26.0).reshape(5, 5) + 3.0
    E[2, 2] += 5.0
    out = oracle.denoise(E, 3, min_support=10)
    np.testing.assert_array_equal(out, E)
