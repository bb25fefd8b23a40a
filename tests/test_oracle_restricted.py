"""Pins of the oracle's component-restricted window (the n_g window keeps only
the pixels of the centre's surface component) against facts fixed
independently of its code:

* two planes meeting at a disparity jump are two components: with the window
  restricted, every pixel gets its own plane's slope exactly, while the plain
  window mixes the planes next to the jump;
* the support of hand-built label patterns, counted by hand through the
  min-support threshold;
* a centre without a label is undefined.
"""
import numpy as np

from oracle import oracle


def test_two_planes_keep_their_slopes():
    H, W = 30, 40
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    D = np.where(u < 20, 20.0 + 0.0625 * u, 40.0 - 0.03125 * v)
    lab, n = oracle.components(D.astype(np.float32), 0.1, 1.0)
    assert n == 2
    a1, a2, d = oracle.affine_labels(D, lab, 9)
    L, R = d & (u < 20), d & (u >= 20)
    assert L.sum() > 400 and R.sum() > 400
    assert np.abs(a1[L] - (1 - 0.0625)).max() < 1e-12 and np.abs(a2[L]).max() < 1e-12
    assert np.abs(a1[R] - 1.0).max() < 1e-12 and np.abs(a2[R] - 0.03125).max() < 1e-12
    # the pixels next to the jump keep enough support (half the window or more)
    assert d[5:25, 17:23].all()
    w1, _, wd = oracle.affine(D, 9)
    near = wd & (np.abs(u - 19.5) < 3)
    assert np.abs(w1[near] - np.where(u[near] < 20, 1 - 0.0625, 1.0)).max() > 0.1


def test_support_count_by_hand():
    # 5x5 frame, window 3x3 around the centre (2, 2): label 7 on the centre and
    # on 4 of its 8 neighbours (N, S, E, NE); the rest label 9
    D = np.full((5, 5), 10.0)
    lab = np.full((5, 5), 9, np.int32)
    for (y, x) in ((2, 2), (1, 2), (3, 2), (2, 3), (1, 3)):
        lab[y, x] = 7
    # support 4 >= 4: defined; with min_support 5: undefined
    _, _, d = oracle.affine_labels(D, lab, 3, min_support=4)
    assert d[2, 2]
    _, _, d = oracle.affine_labels(D, lab, 3, min_support=5)
    assert not d[2, 2]
    # only N and S: alpha = 0 -> singular, undefined even with min_support 1
    lab[2, 3] = lab[1, 3] = 9
    _, _, d = oracle.affine_labels(D, lab, 3, min_support=1)
    assert not d[2, 2]


def test_unlabelled_centre_is_undefined():
    D = np.full((7, 7), 10.0)
    lab = np.zeros((7, 7), np.int32)
    lab[3, 3] = -1
    _, _, d = oracle.affine_labels(D, lab, 3)
    assert not d[3, 3] and d[2, 2]
