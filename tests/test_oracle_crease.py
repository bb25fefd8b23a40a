"""Pins of the oracle's crease-aware components: the covered-depth predicate plus
n_p . n_q >= cos_min on every 4-neighbour edge (binary64 from float32 normals),
checked on cases worked out by hand."""
import numpy as np

from oracle import oracle


def _roof(H=10, W=40, split=20):
    """A depth-continuous roof: the disparity rises to the ridge at u = split and
    falls after it, with one unit normal per side."""
    u = np.arange(W, dtype=np.float64)[None, :].repeat(H, 0)
    D = np.where(u < split, 20.0 + 0.25 * u, 20.0 + 0.25 * split - 0.25 * (u - split))
    nl = np.array([-0.6, 0.0, -0.8], np.float32)
    nr = np.array([0.6, 0.0, -0.8], np.float32)
    n = np.where((u < split)[None], nl[:, None, None], nr[:, None, None]).astype(np.float32)
    return D.astype(np.float32), n


def test_roof_is_one_covered_depth_component_and_two_crease_components():
    D, n = _roof()
    lab, c = oracle.components(D, 0.1, 1.0)
    assert c == 1 and np.all(lab == 0)
    # n_l . n_r = -0.36 + 0.64 = 0.28 < 0.9: the ridge splits the roof
    lab, c = oracle.components_crease(D, n, 0.1, 1.0, 0.9)
    assert c == 2
    assert np.all(lab[:, :20] == 0) and np.all(lab[:, 20:] == 20)
    # a loose threshold keeps it whole
    lab, c = oracle.components_crease(D, n, 0.1, 1.0, 0.25)
    assert c == 1


def test_undefined_normals_impose_nothing():
    D, n = _roof()
    n[:, :, 19] = np.nan          # the column left of the ridge has no normal
    lab, c = oracle.components_crease(D, n, 0.1, 1.0, 0.9)
    assert c == 1


def test_threshold_is_inclusive():
    D = np.full((1, 2), 10.0, np.float32)
    n = np.zeros((3, 1, 2), np.float32)
    n[:, 0, 0] = [1.0, 0.0, 0.0]
    n[:, 0, 1] = [0.5, 0.75, 0.25]        # dot = 0.5 exactly
    assert oracle.components_crease(D, n, 0.1, 1.0, 0.5)[1] == 1
    assert oracle.components_crease(D, n, 0.1, 1.0, np.nextafter(0.5, 1.0))[1] == 2


def test_covered_depth_still_applies():
    D, n = _roof()
    D[:, 30:] += 50.0             # a jump: covered depth splits it whatever the normals
    n[:] = np.array([0.0, 0.0, -1.0], np.float32)[:, None, None]
    lab, c = oracle.components_crease(D, n, 0.1, 1.0, 0.0)
    assert c == 2 and np.all(lab[:, 30:] == 30)
