"""Published quadrature tables on the reference triangle.

Reference triangle: {xi >= 0, xi_1 + xi_2 <= 1}; points are reference
coordinates (xi_1, xi_2) and the weights sum to its area 1/2.  The rules are
inputs of the assembly (the paper passes outer and inner rules to the
assembler, Sec. 2.4.1), so they live here next to the meshes.

* ``gauss7``  - Radon's 7-point rule of degree 5 (centroid plus two
  (a, a, b) orbits with a = (6 -+ sqrt 15)/21).
* ``paper7``  - the 7-point rule of the paper's experiments: centroid,
  vertices and edge midpoints with weights 27/60, 3/60, 8/60 (footnote in
  Sec. 3.1), degree 3.
* ``centroid1`` - one point, degree 1.
* ``collapsed(n)`` - Stroud's conical product rule with n^2 points built
  from Gauss-Legendre and Gauss-Jacobi(1,0) nodes, degree 2n - 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Rule:
    name: str
    xi: np.ndarray   # float64 [P, 2]
    w: np.ndarray    # float64 [P], sum = 1/2

    @property
    def n(self) -> int:
        return int(self.w.shape[0])


def _orbit(a: float, b: float):
    # barycentric (a, a, b), (a, b, a), (b, a, a) -> reference (l1, l2)
    return [(a, b), (b, a), (a, a)]


def gauss7() -> Rule:
    s = math.sqrt(15.0)
    a1, b1 = (6.0 - s) / 21.0, (9.0 + 2.0 * s) / 21.0
    a2, b2 = (6.0 + s) / 21.0, (9.0 - 2.0 * s) / 21.0
    w1, w2 = (155.0 - s) / 1200.0, (155.0 + s) / 1200.0
    pts = [(1.0 / 3.0, 1.0 / 3.0)] + _orbit(a1, b1) + _orbit(a2, b2)
    wts = [9.0 / 40.0] + [w1] * 3 + [w2] * 3
    return Rule("gauss7", np.array(pts, dtype=np.float64),
                0.5 * np.array(wts, dtype=np.float64))


def paper7() -> Rule:
    pts = [(1.0 / 3.0, 1.0 / 3.0),
           (0.0, 0.0), (1.0, 0.0), (0.0, 1.0),
           (0.5, 0.0), (0.5, 0.5), (0.0, 0.5)]
    wts = [27.0 / 60.0] + [3.0 / 60.0] * 3 + [8.0 / 60.0] * 3
    return Rule("paper7", np.array(pts, dtype=np.float64),
                0.5 * np.array(wts, dtype=np.float64))


def centroid1() -> Rule:
    return Rule("centroid1", np.array([(1.0 / 3.0, 1.0 / 3.0)]),
                np.array([0.5]))


def collapsed(n: int) -> Rule:
    """Conical product rule: xi_1 = u, xi_2 = (1 - u) v with u from the
    Gauss-Jacobi rule of weight (1 - u) on [0, 1] and v Gauss-Legendre."""
    from scipy.special import roots_jacobi
    xg, wg = np.polynomial.legendre.leggauss(n)
    v = 0.5 * (xg + 1.0)
    wv = 0.5 * wg
    xj, wj = roots_jacobi(n, 1.0, 0.0)   # weight (1 - x) on [-1, 1]
    u = 0.5 * (xj + 1.0)
    wu = 0.25 * wj                       # (1-x) dx -> 2(1-u) * 2 du
    pts, wts = [], []
    for a, wa in zip(u, wu):
        for b, wb in zip(v, wv):
            pts.append((a, (1.0 - a) * b))
            wts.append(wa * wb)
    return Rule(f"collapsed{n}", np.array(pts), np.array(wts))


def polygon_dirs(n: int) -> np.ndarray:
    """Unit directions (cos 2 pi j/n, sin 2 pi j/n), j = 0..n-1, of a regular
    n-gon inscribed in the unit circle, counter-clockwise, vertex 0 at angle
    0.  Scaled by delta around an outer point they give the polygonal ball."""
    t = 2.0 * np.pi * np.arange(n) / n
    return np.ascontiguousarray(np.stack([np.cos(t), np.sin(t)], axis=1))
