"""Pins for the post hoc reconstruction oracle (Eq. (1), Eq. (2)) and the
accuracy metric (Eq. (5), Eq. (6)): the paper's own identity of Eq. (2) on
random lines, exact reconstruction of affine flow maps (linear interpolation
reproduces them whatever the hole pattern), the axis order of the passes, and
small hand-computed values."""

import numpy as np
import pytest

from oracle import reconstruct as rc


def test_eq1_weights_hand_values():
    vals = np.array([[0.0, 10.0, -3.0], [9.0, 9.0, 9.0], [9.0, 9.0, 9.0], [3.0, 4.0, 0.0]])
    known = np.array([True, False, False, True])
    out, filled = rc.fill_line(vals, known)
    assert filled.tolist() == [False, True, True, False]
    # x1 = 1: (1/3) f(3) + (2/3) f(0); x1 = 2: (2/3) f(3) + (1/3) f(0)
    np.testing.assert_allclose(out[1], [1.0, 8.0, -2.0], atol=1e-15)
    np.testing.assert_allclose(out[2], [2.0, 6.0, -1.0], atol=1e-15)


def test_eq2_identity_interpolating_rebuilt_values_equals_nearest_known():
    """Eq. (2): post hoc linear interpolation at any x through the rebuilt
    lattice equals linear interpolation between the closest known entries."""
    rng = np.random.default_rng(3)
    for trial in range(50):
        m = int(rng.integers(5, 40))
        vals = rng.normal(size=(m, 3))
        known = rng.random(m) < 0.5
        known[0] = known[-1] = True
        out, _ = rc.fill_line(vals, known)
        kidx = np.nonzero(known)[0]
        for x in rng.uniform(0, m - 1, 20):
            # through the rebuilt lattice: the two lattice entries around x
            i = min(int(np.floor(x)), m - 2)
            t = x - i
            rebuilt = (1 - t) * out[i] + t * out[i + 1]
            # directly from the closest known entries x0 <= x <= x2
            j = np.searchsorted(kidx, x, side="right") - 1
            j = min(j, len(kidx) - 2)
            x0, x2 = kidx[j], kidx[j + 1]
            direct = (x - x0) / (x2 - x0) * vals[x2] + (x2 - x) / (x2 - x0) * vals[x0]
            np.testing.assert_allclose(rebuilt, direct, atol=1e-12)


def _affine(m, A, c):
    k, j, i = np.meshgrid(np.arange(m[2]), np.arange(m[1]), np.arange(m[0]), indexing="ij")
    p = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(float)
    return p @ A.T + c, p


def test_affine_flow_maps_are_rebuilt_exactly():
    rng = np.random.default_rng(8)
    m = (9, 7, 6)
    A = rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    f, p = _affine(m, A, c)
    known = rng.random(f.shape[0]) < 0.6
    out, st = rc.reconstruct(f, known, m)
    assert np.all(st[known] == rc.KNOWN)
    rebuilt = st == rc.REBUILT
    assert rebuilt.sum() > 0.3 * (~known).sum()
    np.testing.assert_allclose(out[rebuilt], f[rebuilt], atol=1e-12)
    np.testing.assert_array_equal(out[known], f[known])
    assert np.all(np.isnan(out[st == rc.MISSING]))


def test_pass_order_x_then_y_then_z():
    m = (3, 3, 3)
    f, p = _affine(m, np.eye(3), np.zeros(3))
    known = np.ones(27, dtype=bool)
    ijk = p.astype(int)
    # the whole x-line y=1, z=1 is unknown: only the y pass (or z) can fill it
    line = (ijk[:, 1] == 1) & (ijk[:, 2] == 1)
    known[line] = False
    # an entry whose y and z lines have no known pair, x line does
    lone = (ijk[:, 0] == 1) & (ijk[:, 1] == 0) & (ijk[:, 2] == 0)
    known[lone] = False
    out, st = rc.reconstruct(f, known, m)
    assert np.all(st[line] == rc.REBUILT) and st[lone] == rc.REBUILT
    np.testing.assert_allclose(out[line | lone], f[line | lone], atol=1e-15)
    # no known pair on any axis: stays missing
    known2 = np.zeros(27, dtype=bool)
    known2[0] = True
    out2, st2 = rc.reconstruct(f, known2, m)
    assert st2[0] == rc.KNOWN and np.all(st2[1:] == rc.MISSING)
    # entries rebuilt in one pass bracket entries in the next: the z pass uses
    # x-pass values when the z line's known entries are themselves rebuilt
    known3 = np.zeros(27, dtype=bool)
    ends_x = (ijk[:, 0] != 1) & (ijk[:, 1] == 1) & (ijk[:, 2] != 1)
    known3[ends_x] = True      # (0|2, 1, 0|2): x pass fills (1, 1, 0|2)
    out3, st3 = rc.reconstruct(f, known3, m)
    centre = (ijk[:, 0] == 1) & (ijk[:, 1] == 1) & (ijk[:, 2] == 1)
    assert st3[centre] == rc.REBUILT   # by the z pass from (1, 1, 0) and (1, 1, 2)
    np.testing.assert_allclose(out3[centre], f[centre], atol=1e-15)


def test_accuracy_metric_hand_values():
    b = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 3.0, 4.0], [7.0, 7, 7]])
    bs = np.array([rc.KNOWN, rc.REBUILT, rc.KNOWN, rc.MISSING], dtype=np.uint8)
    m = np.zeros((4, 3))
    mf = np.array([0, 0, 1, 0], dtype=np.uint8)  # the third left the domain in m
    r = rc.flowmap_error(b, bs, m, mf, cell=2.0)
    assert r["n"] == 2 and r["uncovered"] == 1
    assert r["mean_l2"] == pytest.approx(0.5) and r["max_l2"] == pytest.approx(1.0)
    assert r["accuracy_pct"] == pytest.approx(75.0)
