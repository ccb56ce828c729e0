"""Workload recipes: mesh, kernel, horizon, rules and forcing per test case.

Each recipe is a plain dictionary of inputs.  Kernel constants follow the
paper's scalings: c_{s,delta} = (2 - 2s) / (pi delta^(2-2s)) for the
fractional-type family (Sec. 3.1, eq. for c_{s,delta}); s = -1 gives the
constant kernel 4/(pi delta^4), s = -1/2 the 1/|z| kernel 3/(pi delta^3).
The peridynamic case uses c = 6/(pi delta^3) for c (x-y)(x-y)^T/|x-y|^3.
"""
from __future__ import annotations

import math

from .meshes import square_mesh, batched_meshes
from .rules import gauss7


def c_frac(s: float, delta: float) -> float:
    return (2.0 - 2.0 * s) / (math.pi * delta ** (2.0 - 2.0 * s))


def _scalar(name, n, delta, kernel, approach="bary", jitter=0.0,
            singular_n=0, precision="fp64", polygon_n=32, seed=0):
    mesh = square_mesh(n, delta=delta, jitter=jitter, seed=seed)
    c = c_frac(-1.0, delta) if kernel == "constant" else c_frac(-0.5, delta)
    return dict(name=name, mesh=mesh, kernel=kernel, c=c, delta=delta,
                approach=approach, polygon_n=polygon_n, outer=gauss7(),
                inner=gauss7(), singular_n=singular_n, precision=precision,
                f=(-4.0,), ncomp=1)


def small_constant():
    """h = 1/16, delta = 0.1, constant kernel, barycentre inclusion, FP64;
    about 800 triangles."""
    return _scalar("const_h16_d0.1", 16, 0.1, "constant")


def inv_dist_jittered(n=64, delta=0.05, precision="mixed"):
    """1/|z| kernel, delta = 0.05, h = 1/64 with seeded jitter 0.2 h, Duffy
    quadrature on touching pairs; about 10k triangles."""
    return _scalar(f"invdist_h{n}_d{delta}_jit0.2", n, delta, "inv_dist",
                   jitter=0.2, singular_n=5, precision=precision)


def constant_polygon(n=256, delta=0.02, precision="mixed"):
    """Constant kernel, 32-gon ball approximation clipped in FP64, h = 1/256,
    delta = 0.02; about 144k triangles."""
    return _scalar(f"const_poly32_h{n}_d{delta}", n, delta, "constant",
                   approach="poly", precision=precision)


def peridynamic(n=128, ratio=3, precision="mixed"):
    """Bond-based peridynamics, vector P1, h = 1/128, delta = 3h, jitter
    0.15 h, Duffy quadrature on touching pairs."""
    h = 1.0 / n
    delta = ratio * h
    mesh = square_mesh(n, delta=delta, jitter=0.15, seed=0)
    return dict(name=f"peri_h{n}_r{ratio}_jit0.15", mesh=mesh,
                kernel="peridynamic", c=6.0 / (math.pi * delta ** 3),
                delta=delta, approach="bary", polygon_n=32, outer=gauss7(),
                inner=gauss7(), singular_n=5, precision=precision,
                f=None, f_affine=((-1.0, -2.0, 0.0), (0.0, 0.0, -1.0)),
                ncomp=2)


def batched(count=64, precision="mixed"):
    """64 problems, h in 1/32..1/160, delta/h in {2,3,4,5}; even problems
    constant kernel, odd problems 1/|z| with Duffy quadrature."""
    probs = []
    for i, (mesh, delta, kind) in enumerate(batched_meshes(count)):
        c = c_frac(-1.0, delta) if kind == "constant" else c_frac(-0.5, delta)
        probs.append(dict(name=f"batch{i}", mesh=mesh, kernel=kind, c=c,
                          delta=delta, approach="bary", polygon_n=32,
                          outer=gauss7(), inner=gauss7(),
                          singular_n=(5 if kind == "inv_dist" else 0),
                          precision=precision, f=(-4.0,), ncomp=1))
    return probs


WORKLOADS = {
    "const_h16": small_constant,
    "invdist_h64": inv_dist_jittered,
    "poly32_h256": constant_polygon,
    "peri_h128": peridynamic,
    "batched64": batched,
}


def workload(name: str, **kw):
    return WORKLOADS[name](**kw)
