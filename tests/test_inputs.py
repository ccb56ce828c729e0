"""Input generators: mesh recipes and quadrature tables (no GPU)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from inputs import square_mesh, gauss7, paper7, centroid1, collapsed, batched_meshes
from inputs.rules import polygon_dirs
from inputs.workloads import small_constant, inv_dist_jittered, peridynamic, c_frac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dofs(mesh):
    M = mesh.n_vertices
    om = np.zeros(M, bool)
    di = np.zeros(M, bool)
    om[mesh.elements[mesh.labels == 1].ravel()] = True
    di[mesh.elements[mesh.labels == 2].ravel()] = True
    return om & ~di


@pytest.mark.parametrize("n,delta,K,M,dofs", [
    (16, 0.1, 800, 441, 225),
    (64, 0.05, 10368, 5329, 3969),
    (256, 0.02, 143648, 72361, 65025),
    (128, 3.0 / 128, 35912, 18225, 16129),
])
def test_mesh_counts(n, delta, K, M, dofs):
    m = square_mesh(n, delta=delta)
    assert m.n_elements == K and m.n_vertices == M
    assert int(_dofs(m).sum()) == dofs
    # layer at least delta wide
    assert m.m * m.h >= delta - 1e-12


def test_mesh_orientation_and_area():
    for jit in (0.0, 0.2):
        m = square_mesh(24, delta=0.1, jitter=jit, seed=0)
        v = m.vertices[m.elements]
        d = (v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - \
            (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1])
        assert np.all(d > 0)
        side = 1.0 + 2 * m.m * m.h
        assert abs(0.5 * d.sum() - side * side) < 1e-12
        om = m.labels == 1
        assert abs(0.5 * d[om].sum() - 1.0) < 1e-12


def test_jitter_keeps_lines():
    m = square_mesh(32, delta=0.1, jitter=0.2, seed=0)
    ref = square_mesh(32, delta=0.1)
    moved = np.any(m.vertices != ref.vertices, axis=1)
    assert moved.sum() > 0.5 * m.n_vertices
    N = m.n + 2 * m.m
    ii, jj = np.divmod(np.arange(m.n_vertices), N + 1)
    lines = {0, m.m, m.m + m.n, N}
    on = np.array([(a in lines) or (b in lines) for a, b in zip(ii, jj)])
    assert not moved[on].any()
    # seeded: same draw twice
    m2 = square_mesh(32, delta=0.1, jitter=0.2, seed=0)
    assert np.array_equal(m.vertices, m2.vertices)


def _tri_monomial(a, b):
    """Exact integral of xi1^a xi2^b over the reference triangle."""
    return Fraction(math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))


def _degree(rule, maxdeg=12, tol=1e-14):
    deg = -1
    for d in range(maxdeg + 1):
        ok = True
        for a in range(d + 1):
            b = d - a
            q = np.sum(rule.w * rule.xi[:, 0] ** a * rule.xi[:, 1] ** b)
            if abs(q - float(_tri_monomial(a, b))) > tol:
                ok = False
        if not ok:
            return deg
        deg = d
    return deg


def test_rule_degrees():
    # Radon's 7-point rule: degree 5; paper's rule: degree 3; centroid: 1
    assert _degree(gauss7()) == 5
    assert _degree(paper7()) == 3
    assert _degree(centroid1()) == 1
    for n in (2, 3, 4):
        assert _degree(collapsed(n)) == 2 * n - 1
    for r in (gauss7(), paper7(), centroid1(), collapsed(3)):
        assert abs(r.w.sum() - 0.5) < 1e-15
        assert np.all(r.xi >= -1e-15) and np.all(r.xi.sum(axis=1) <= 1 + 1e-15)


def test_paper7_matches_footnote():
    rows = []
    with open(os.path.join(GOLDEN, "paper7_rule.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, w = line.split()
            rows.append((float(Fraction(a)), float(Fraction(b)), int(w) / 120.0))
    g = np.array(rows)
    r = paper7()
    assert np.allclose(r.xi, g[:, :2], atol=0, rtol=0)
    assert np.allclose(r.w, g[:, 2], atol=1e-17)


def test_kernel_constants():
    # c_{s,delta} = (2-2s)/(pi delta^(2-2s)): s=-1 -> 4/(pi d^4); s=-1/2 -> 3/(pi d^3)
    for d in (0.1, 0.05, 0.02):
        assert abs(c_frac(-1.0, d) - 4 / (math.pi * d ** 4)) < 1e-9 * c_frac(-1.0, d)
        assert abs(c_frac(-0.5, d) - 3 / (math.pi * d ** 3)) < 1e-9 * c_frac(-0.5, d)
    w = small_constant()
    assert abs(w["c"] - 12732.395447351628) < 1e-6
    w = inv_dist_jittered()
    assert abs(w["c"] - 7639.437268410976) < 1e-6
    w = peridynamic()
    assert abs(w["c"] - 6 / (math.pi * w["delta"] ** 3)) < 1e-9 * w["c"]


def test_polygon_dirs():
    d = polygon_dirs(32)
    assert d.shape == (32, 2)
    assert np.allclose(np.hypot(d[:, 0], d[:, 1]), 1.0, atol=1e-15)
    assert d[0, 0] == 1.0 and d[0, 1] == 0.0
    ang = np.arctan2(d[:, 1], d[:, 0]) % (2 * np.pi)
    assert np.all(np.diff(ang) > 0)


def test_batched_recipe():
    probs = batched_meshes(64)
    assert len(probs) == 64
    ns = [p[0].n for p in probs]
    assert min(ns) >= 32 and max(ns) <= 160
    for mesh, delta, kind in probs:
        assert mesh.m == round(delta / mesh.h)
        assert mesh.m in (2, 3, 4, 5)
    assert [p[2] for p in probs[:2]] == ["constant", "inv_dist"]
