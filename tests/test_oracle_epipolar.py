"""Pins of the epipolar-check oracle (oracle.epipolar) against two-view
geometry: exact projections of 3D points give the closed-form fundamental
matrix K^-T [t]x R K^-1 from any 8 samples (also under forward motion, where
F33 = 0); point-to-line distances against a geometric construction; planted
offsets along the line normal; planted outliers; a planar scene (rank 6) and
repeated samples give no model; ties go to the lowest index."""
import importlib.util
import os
import sys

import numpy as np
import pytest

if os.environ.get("LKO_EPI_SRC"):
    # the mutation tests point this at a planted copy of oracle/epipolar.py
    _spec = importlib.util.spec_from_file_location("oracle._epi_planted", os.environ["LKO_EPI_SRC"])
    E = importlib.util.module_from_spec(_spec)
    sys.modules[_spec.name] = E
    _spec.loader.exec_module(E)
else:
    from oracle import epipolar as E

INTR = (420.0, 410.0, 376.0, 240.0)


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return rz @ ry @ rx


def kmat(fx, fy, cx, cy):
    return np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1.0]])


def skew(t):
    return np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])


def two_views(n, R, t, seed, planar=False):
    """Points X in camera-1 coordinates, camera 2 = R X + t; pixel projections."""
    rng = np.random.default_rng(seed)
    if planar:
        xy = rng.uniform(-2, 2, (n, 2))
        X = np.column_stack([xy, 6.0 + 0.3 * xy[:, 0] - 0.2 * xy[:, 1]])
    else:
        X = np.column_stack([rng.uniform(-3, 3, n), rng.uniform(-2, 2, n), rng.uniform(4, 12, n)])
    K = kmat(*INTR)
    x1 = (K @ X.T).T
    X2 = (R @ X.T).T + t
    x2 = (K @ X2.T).T
    return x1[:, :2] / x1[:, 2:], x2[:, :2] / x2[:, 2:]


def f_true(R, t):
    ki = np.linalg.inv(kmat(*INTR))
    f = ki.T @ skew(t) @ R @ ki
    return f / np.linalg.norm(f)


def same_up_to_sign(a, b, tol):
    return min(np.abs(a - b).max(), np.abs(a + b).max()) <= tol


POSES = [(rot(0.02, -0.03, 0.01), np.array([0.3, -0.1, 0.05])),
         (rot(0.0, 0.0, 0.0), np.array([0.0, 0.0, 1.0])),            # forward motion: F33 = 0
         (rot(-0.05, 0.04, 0.1), np.array([-0.2, 0.25, -0.4]))]


@pytest.mark.parametrize("k", range(len(POSES)))
def test_model_is_the_true_fundamental_matrix(k):
    R, t = POSES[k]
    p, q = two_views(60, R, t, seed=k)
    ft = f_true(R, t)
    rng = np.random.default_rng(10 + k)
    for _ in range(5):
        s = rng.choice(60, 8, replace=False)
        f = E.model(p, q, s, INTR)
        assert f is not None and same_up_to_sign(f, ft, 1e-7)
    if k == 1:
        assert abs(ft[2, 2]) < 1e-12                 # c^T [t]x c = 0 for the principal point c
    best, counts, mask, _ = E.check(p, q, [rng.choice(60, 8, replace=False)], INTR)
    assert best == 0 and counts[0] == 60 and mask.all()


def test_errors_against_a_geometric_construction():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(3, 3))
    p = rng.uniform(0, 700, (40, 2))
    q = rng.uniform(0, 450, (40, 2))
    e = E.errors(f, p, q)
    for i in range(40):
        a, b, c = f @ np.array([p[i, 0], p[i, 1], 1.0])
        # two points on the line a x + b y + c = 0, then |cross| / |direction|
        if abs(b) > abs(a):
            u0, u1 = np.array([0.0, -c / b]), np.array([1.0, -(a + c) / b])
        else:
            u0, u1 = np.array([-c / a, 0.0]), np.array([-(b + c) / a, 1.0])
        d = u1 - u0
        w = q[i] - u0
        assert abs(e[i] - abs(d[0] * w[1] - d[1] * w[0]) / np.linalg.norm(d)) <= 1e-9 * max(1.0, e[i])


def test_planted_offsets_along_the_line_normal():
    R, t = POSES[0]
    p, q = two_views(50, R, t, seed=5)
    ft = f_true(R, t)
    q2 = q.copy()
    offs = np.zeros(50)
    offs[:10] = 0.5
    offs[10:20] = 1.5
    offs[20:25] = 0.999
    offs[25:30] = 1.001
    l = E.hom(p) @ ft.T
    nrm = l[:, :2] / np.linalg.norm(l[:, :2], axis=1, keepdims=True)
    q2 += offs[:, None] * nrm
    e = E.errors(ft, p, q2)
    assert np.allclose(e, offs, atol=1e-9)
    # hypotheses from untouched points recover the true model, the mask follows the offsets
    samples = [list(range(30, 38)), list(range(38, 46))]
    best, counts, mask, _ = E.check(p, q2, samples, INTR)
    assert best == 0 and counts[0] == counts[1] == 50 - 10 - 5     # ties: the lower index
    assert np.array_equal(mask, offs <= 1.0)


def test_outliers_and_contaminated_hypotheses():
    R, t = POSES[2]
    p, q = two_views(100, R, t, seed=7)
    ft = f_true(R, t)
    rng = np.random.default_rng(8)
    bad = rng.choice(100, 30, replace=False)
    l = E.hom(p) @ ft.T
    nrm = l[:, :2] / np.linalg.norm(l[:, :2], axis=1, keepdims=True)
    q = q.copy()
    q[bad] += (rng.uniform(20, 50, 30) * rng.choice([-1, 1], 30))[:, None] * nrm[bad]
    good = np.setdiff1d(np.arange(100), bad)
    samples = [np.concatenate([good[:7], bad[:1]]), good[10:18], np.concatenate([good[20:26], bad[1:3]])]
    best, counts, mask, _ = E.check(p, q, samples, INTR)
    assert best == 1 and counts[1] == 70
    assert np.array_equal(np.flatnonzero(mask), good)
    assert counts[0] < 70 and counts[2] < 70


def test_degenerate_hypotheses_give_no_model():
    R, t = POSES[0]
    p, q = two_views(40, R, t, seed=9, planar=True)
    assert E.model(p, q, list(range(8)), INTR) is None                 # a plane: rank 6
    p2, q2 = two_views(40, R, t, seed=9)
    samples = [[0, 1, 2, 3, 4, 5, 6, 6], [0, 1, 2, 3, 4, 5, 6, 40], [0, 1, 2]]
    best, counts, mask, errs = E.check(p2, q2, samples, INTR)
    assert best == -1 and counts.tolist() == [-1, -1, -1] and not mask.any() and errs == [None, None, None]
    best, counts, mask, _ = E.check(p2, q2, [], INTR)
    assert best == -1 and len(counts) == 0
