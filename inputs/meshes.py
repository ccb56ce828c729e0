"""Seeded triangulations of the square test geometry.

The paper's experiments use a square domain Omega surrounded by an
interaction layer Omega_D of width delta, both meshed by the same uniform
grid of right-isosceles triangles (Sec. 3, problem setup; Fig. 2.1 for the
labelling).  The recipe here:

* Omega = [0,1]^2, h = 1/n, layer of m = ceil(delta/h - 1e-9) whole cells,
  so the base domain is [-m h, 1 + m h]^2 and is meshed by N = n + 2m cells
  per side.
* node (i, j) sits at ((i - m) h, (j - m) h) and has id i*(N+1) + j.
* cell (i, j) is split along its (v00, v11) diagonal into the elements
  2*(i*N + j) + 0 = (v00, v10, v11) and 2*(i*N + j) + 1 = (v00, v11, v01).
* label 1 (Omega) for cells inside [0,1]^2, label 2 (Omega_D) otherwise.
* optional jitter: every node is moved by a uniform offset in [-a h, a h]^2
  drawn from numpy's default_rng(seed), except nodes lying on one of the grid
  lines x or y in {-m h, 0, 1, 1 + m h}; those stay put so that Omega and the
  outer boundary remain exact squares.  For a < 0.25 every triangle keeps its
  orientation.

Nothing here evaluates the nonlocal operator.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray   # float64 [M, 2]
    elements: np.ndarray   # int32   [K, 3]
    labels: np.ndarray     # int32   [K]  (1 = Omega, 2 = Omega_D)
    h: float
    n: int                 # cells per side of Omega
    m: int                 # layer width in cells
    materials: np.ndarray | None = None   # int32 [K] material ids of a label-dependent kernel

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.elements.shape[0])


def layer_cells(n: int, delta: float, side: float = 1.0) -> int:
    """Number of whole cells needed for a layer of width >= delta."""
    h = side / n
    return int(math.ceil(delta / h - 1e-9))


def square_mesh(n: int, delta: float | None = None, m: int | None = None,
                jitter: float = 0.0, seed: int = 0,
                neumann: bool = False, side: float = 1.0) -> Mesh:
    """Uniform right-isosceles mesh of [0,1]^2 plus an interaction layer.

    ``n`` cells per side of Omega; the layer width is ``m`` cells (derived
    from ``delta`` when not given).  ``jitter`` is the relative amplitude a
    of the seeded node perturbation.  With ``neumann=True`` every element is
    labelled Omega (the pure-interaction case, base domain = Omega).
    ``side`` scales the geometry: Omega = [0, side]^2 and h = side / n (the
    numerical section's square is side = 0.5).
    """
    if m is None:
        if delta is None:
            raise ValueError("give delta or m")
        m = layer_cells(n, delta, side)
    h = side / n
    N = n + 2 * m
    ii, jj = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    ii = ii.reshape(-1)
    jj = jj.reshape(-1)
    verts = np.stack([(ii - m) * h, (jj - m) * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=verts.shape)
        fixed_lines = np.array([0, m, m + n, N])
        on_line = np.isin(ii, fixed_lines) | np.isin(jj, fixed_lines)
        d[on_line] = 0.0
        verts = verts + d

    ci, cj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ci = ci.reshape(-1)
    cj = cj.reshape(-1)
    v00 = ci * (N + 1) + cj
    v10 = (ci + 1) * (N + 1) + cj
    v11 = (ci + 1) * (N + 1) + cj + 1
    v01 = ci * (N + 1) + cj + 1
    elems = np.empty((2 * N * N, 3), dtype=np.int32)
    elems[0::2] = np.stack([v00, v10, v11], axis=1)
    elems[1::2] = np.stack([v00, v11, v01], axis=1)
    inside = (ci >= m) & (ci < m + n) & (cj >= m) & (cj < m + n)
    lab_cell = np.where(inside, 1, 2).astype(np.int32)
    labels = np.repeat(lab_cell, 2)
    if neumann:
        labels[:] = 1
    return Mesh(vertices=np.ascontiguousarray(verts),
                elements=np.ascontiguousarray(elems),
                labels=np.ascontiguousarray(labels), h=h, n=n, m=m)


def boundary_triangles_to_layer(mesh: Mesh, side: float = 1.0) -> Mesh:
    """The same mesh with every Omega triangle whose three vertices lie on
    the boundary of [0, side]^2 labelled 2 (two corner triangles on the
    uniform mesh).  This is the labelling the printed dof counts of the
    paper's discontinuous-Galerkin studies imply: 3 (2 n^2 - 2) unknowns per
    component for n cells per side; continuous problems are unchanged by it
    (those triangles carry no degree of freedom)."""
    V, E = mesh.vertices, mesh.elements
    p = V[E]
    on = (np.isclose(p[..., 0], 0.0) | np.isclose(p[..., 0], side) |
          np.isclose(p[..., 1], 0.0) | np.isclose(p[..., 1], side))
    labels = mesh.labels.copy()
    labels[(labels == 1) & on.all(axis=1)] = 2
    return Mesh(vertices=V, elements=E, labels=np.ascontiguousarray(labels), h=mesh.h, n=mesh.n, m=mesh.m,
                materials=mesh.materials)


def batched_meshes(count: int = 64, seed: int = 0, n_lo: int = 32,
                   n_hi: int = 160, ratios=(2, 3, 4, 5)):
    """Seeded list of (mesh, delta, kernel_kind) for the batched workload.

    Problem i draws n_i uniformly from [n_lo, n_hi] (h = 1/n_i) and
    r_i = delta/h from ``ratios``; even i use the constant kernel, odd i the
    weakly singular 1/|z| kernel.  No jitter.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        r = int(rng.choice(np.asarray(ratios)))
        h = 1.0 / n
        delta = r * h
        mesh = square_mesh(n, m=r)
        kind = "constant" if i % 2 == 0 else "inv_dist"
        out.append((mesh, delta, kind))
    return out
