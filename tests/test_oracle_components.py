"""Pins of the oracle's connected surface components (pairwise covered depth)."""
from fractions import Fraction

import numpy as np
import pytest

from synth import scenes


def _exact_edges(D, k_rel, t_abs):
    """Per-pixel edge bits of the covered-depth predicate in exact rational
    arithmetic: bit 0 valid, bit 1 joined to the left, bit 2 joined above."""
    H, W = D.shape
    valid = np.isfinite(D) & (D > 0)
    flags = valid.astype(np.uint8)
    kq, tq = Fraction(float(np.float32(k_rel))), Fraction(float(np.float32(t_abs)))
    for v in range(H):
        for u in range(W):
            for du, dv, bit in ((1, 0, 2), (0, 1, 4)):
                uu, vv = u + du, v + dv
                if uu >= W or vv >= H or not (valid[v, u] and valid[vv, uu]):
                    continue
                a, b = Fraction(float(D[v, u])), Fraction(float(D[vv, uu]))
                if abs(a - b) <= max(tq, kq * min(a, b)):
                    flags[vv, uu] |= bit
    return flags


def _closure_from_flags(flags):
    """Min-index labels from the transitive closure of the 4-neighbour graph
    given by edge bits (bit 0 present, bit 1 edge left, bit 2 edge up; an edge
    counts between two present pixels)."""
    H, W = flags.shape
    N = H * W
    present = (flags & 1).astype(bool).reshape(-1)
    adj = np.eye(N, dtype=bool) & present[:, None]
    for v in range(H):
        for u in range(W):
            q = v * W + u
            for bit, p in ((2, q - 1), (4, q - W)):
                if flags[v, u] & bit and (bit == 2 and u > 0 or bit == 4 and v > 0) \
                        and present[p] and present[q]:
                    adj[p, q] = adj[q, p] = True
    reach = adj.copy()
    while True:
        nxt = (reach.astype(np.uint8) @ reach.astype(np.uint8)) > 0
        if np.array_equal(nxt, reach):
            break
        reach = nxt
    lab = np.full(N, -1, np.int32)
    for p in range(N):
        if present[p]:
            lab[p] = np.flatnonzero(reach[p])[0]
    return lab.reshape(H, W), int(len(set(lab[lab >= 0].tolist())))


def _closure_labels(D, k_rel, t_abs):
    """Min-index labels from the transitive closure of the 4-neighbour edge
    relation, with the predicate evaluated in exact rational arithmetic."""
    return _closure_from_flags(_exact_edges(D, k_rel, t_abs))


@pytest.mark.parametrize("seed", range(6))
def test_against_transitive_closure(oracle, seed):
    rng = np.random.default_rng(seed)
    H, W = rng.integers(3, 9, 2)
    # values clustered so that many pairs sit near the thresholds
    D = rng.choice([5.0, 5.4, 6.0, 9.0, 9.9, 10.9, 20.0], size=(H, W)) \
        + rng.normal(0, 0.05, (H, W))
    D = D.astype(np.float32)
    D[rng.random((H, W)) < 0.15] = np.nan
    lab, n = oracle.components(D, 0.1, 0.5)
    ref, nref = _closure_labels(D, 0.1, 0.5)
    np.testing.assert_array_equal(lab, ref)
    assert n == nref


def test_predicate_matches_exact_arithmetic(oracle):
    """The binary64 sequence equals the real-number predicate on float32 input:
    checked on pairs straddling the relative and absolute thresholds."""
    rng = np.random.default_rng(9)
    k, t = np.float32(0.1), np.float32(1.0)
    for _ in range(300):
        a = np.float32(rng.uniform(0.5, 280.0))
        rel = float(k) * float(a)
        gap = max(float(t), rel) * (1.0 + rng.choice([-1, 1]) * 10.0 ** rng.uniform(-8, -5))
        b = np.float32(a + gap) if rng.random() < 0.5 else np.float32(max(a - gap, 0.3))
        D = np.array([[a, b]], np.float32)
        lab, n = oracle.components(D, float(k), float(t))
        A, B = Fraction(float(a)), Fraction(float(b))
        exact = abs(A - B) <= max(Fraction(float(t)), Fraction(float(k)) * min(A, B))
        assert (lab[0, 0] == lab[0, 1]) == exact


def test_invariants_on_scene(oracle):
    sc = scenes.planes_quadrics_scene(width=300, height=200, f=300.0, n_planes=8,
                                      n_spheres=3, sigma=0.5, seed=2)
    D = sc.disp
    lab, n = oracle.components(D, 0.1, 1.0)
    H, W = D.shape
    idx = np.arange(H * W).reshape(H, W)
    valid = np.isfinite(D) & (D > 0)
    assert np.all(lab[~valid] == -1)
    assert np.all(lab[valid] <= idx[valid])
    flat = lab.reshape(-1)
    assert np.all(flat[flat[valid.reshape(-1)]] == flat[valid.reshape(-1)])
    assert n == int(np.sum(flat == np.arange(H * W)))
    # neighbours joined by the predicate share a label
    a, b = D[:, :-1].astype(np.float64), D[:, 1:].astype(np.float64)
    e = valid[:, :-1] & valid[:, 1:] & (np.abs(a - b) <= np.maximum(1.0, np.float64(np.float32(0.1)) * np.minimum(a, b)))
    assert np.all(lab[:, :-1][e] == lab[:, 1:][e])


def test_depth_and_disparity_forms_agree():
    """|z_p - z_q| <= k min(z) holds exactly when |D_p - D_q| <= k min(D) for
    z = F / D, so the covered-depth rule may be evaluated on disparities."""
    rng = np.random.default_rng(1)
    F = Fraction(497)
    k = Fraction(1, 10)
    for _ in range(2000):
        a = Fraction(float(rng.uniform(1, 200)))
        b = a * (1 + k * Fraction(float(rng.uniform(-1.2, 1.2))))
        za, zb = F / a, F / b
        assert (abs(za - zb) <= k * min(za, zb)) == (abs(a - b) <= k * min(a, b))


def test_all_invalid_and_empty_rows(oracle):
    D = np.full((4, 5), np.nan, np.float32)
    lab, n = oracle.components(D)
    assert n == 0 and np.all(lab == -1)
    D = np.full((1, 7), 3.0, np.float32)
    lab, n = oracle.components(D)
    assert n == 1 and np.all(lab == 0)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", [None, (9, 1), (1, 9), (2, 2)])
def test_edge_graph_bfs_against_transitive_closure(oracle, seed, shape):
    """The oracle's labelling of an explicitly given edge graph (the exhaustive
    GPU test's reference) against the transitive closure of the same graph:
    random presence and edge bits, including bits on absent pixels and on the
    image border (which must be ignored); single-column and single-row frames,
    where the index step to the neighbour below equals the step to the right."""
    rng = np.random.default_rng(100 + seed)
    H, W = rng.integers(1, 9, 2) if shape is None else shape
    flags = (rng.random((H, W)) < 0.8).astype(np.uint8)
    flags |= (rng.random((H, W)) < 0.6).astype(np.uint8) << 1
    flags |= (rng.random((H, W)) < 0.6).astype(np.uint8) << 2
    lab, n = oracle.components_edges(flags)
    ref, nref = _closure_from_flags(flags)
    np.testing.assert_array_equal(lab, ref)
    assert n == nref


@pytest.mark.parametrize("seed", range(3))
def test_edge_graph_of_the_predicate_equals_components(oracle, seed):
    """Posing the covered-depth predicate's own edges as an explicit graph gives
    the disparity labelling back."""
    rng = np.random.default_rng(200 + seed)
    D = rng.choice([5.0, 5.4, 6.0, 9.0, 9.9, 20.0], size=(12, 17)) + rng.normal(0, 0.05, (12, 17))
    D = D.astype(np.float32)
    D[rng.random(D.shape) < 0.1] = np.nan
    lab, n = oracle.components(D, 0.1, 0.5)
    lab_e, n_e = oracle.components_edges(_exact_edges(D, 0.1, 0.5))
    np.testing.assert_array_equal(lab, lab_e)
    assert n == n_e
