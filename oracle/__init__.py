"""CPU oracle for nonlocal P1 stiffness assembly (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls into it.

The arithmetic lives in ``oracle.c`` (plain FP64 C, OpenMP over outer
elements, ``-ffp-contract=off``).  This module compiles and loads it, derives
the Gauss-Legendre nodes for the touching-pair transforms from numpy's
``leggauss``, and builds the CSR pattern with numpy from the pair list:
row n*i + c exists for degrees of freedom i (vertices of some Omega element
and of no Omega_D element, Fig. 2.1), and its columns are the union of the
vertex sets of all listed pairs whose vertices include i (eq. biFormApprox,
summed over all ordered pairs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KERNELS = {"constant": 0, "inv_dist": 1, "peridynamic": 2, "frac_half": 3}
APPROACHES = {"bary": 0, "poly": 1, "inf": 2, "nocaps": 3, "approxcaps": 4}   # Def. 2.5, 2.3, 2.4
FAR, VERTEX, EDGE, IDENT = 0, 1, 2, 3


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_elements", C.c_int64),
                ("vertices", C.c_void_p), ("elements", C.c_void_p),
                ("labels", C.c_void_p), ("materials", C.c_void_p)]


class _Cfg(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("ncomp", C.c_int32),
                ("c", C.c_double), ("delta", C.c_double),
                ("approach", C.c_int32), ("polygon_n", C.c_int32),
                ("polygon_dirs", C.c_void_p),
                ("P", C.c_int32), ("pxi", C.c_void_p), ("pw", C.c_void_p),
                ("Q", C.c_int32), ("qxi", C.c_void_p), ("qw", C.c_void_p),
                ("singular_n", C.c_int32), ("gl_x", C.c_void_p),
                ("gl_w", C.c_void_p), ("dg", C.c_int32),
                ("n_materials", C.c_int32), ("material_c", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.orc_pairs.restype = i64
        L.orc_pairs.argtypes = [vp, vp, vp, vp, vp, vp, i64]
        L.orc_pairs_bfs.restype = i64
        L.orc_pairs_bfs.argtypes = [vp, vp, vp, vp, vp, i64]
        L.orc_local.restype = C.c_int
        L.orc_local.argtypes = [vp, vp, i32, i32, C.c_int, vp, vp]
        L.orc_assemble.restype = C.c_int
        L.orc_assemble.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_rhs.restype = C.c_int
        L.orc_rhs.argtypes = [vp, vp, vp, vp, vp]
        L.orc_duffy_samples.restype = i64
        L.orc_duffy_samples.argtypes = [C.c_int, C.c_int, vp, vp, vp, vp, vp, i64]
        L.orc_clip_area.restype = C.c_double
        L.orc_clip_area.argtypes = [vp, vp, vp, i32, vp]
        L.orc_num_threads.restype = C.c_int
        L.orc_inner_moments.restype = C.c_int
        L.orc_inner_moments.argtypes = [vp, vp, vp, i32, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule on [0, 1] (numpy's leggauss, mapped)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return np.ascontiguousarray(0.5 * (x + 1.0)), np.ascontiguousarray(0.5 * w)


class Problem:
    """Holds the numpy arrays a ctypes call points into."""

    def __init__(self, mesh, cfg):
        from inputs.rules import polygon_dirs
        self.mesh = mesh
        self.cfg = cfg
        self.V = np.ascontiguousarray(mesh.vertices, dtype=np.float64)
        self.E = np.ascontiguousarray(mesh.elements, dtype=np.int32)
        self.lab = np.ascontiguousarray(mesh.labels, dtype=np.int32)
        self.n = int(cfg.get("ncomp", 1))
        # discontinuous P1: unknowns 3 k + local vertex of every element
        self.dg = cfg.get("ansatz", "cg") == "dg"
        outer, inner = cfg["outer"], cfg["inner"]
        self.pxi = np.ascontiguousarray(outer.xi, dtype=np.float64)
        self.pw = np.ascontiguousarray(outer.w, dtype=np.float64)
        self.qxi = np.ascontiguousarray(inner.xi, dtype=np.float64)
        self.qw = np.ascontiguousarray(inner.w, dtype=np.float64)
        ns = int(cfg.get("singular_n", 0))
        if ns > 0:
            self.glx, self.glw = gauss_legendre01(ns)
        else:
            self.glx = self.glw = np.zeros(1)
        pn = int(cfg.get("polygon_n", 32))
        self.pdirs = polygon_dirs(pn)
        # label-dependent kernel: material ids per element and the table
        # material_c[m(x)][m(y)] that scales the kernel
        mat = getattr(mesh, "materials", None)
        self.mat = None if mat is None else np.ascontiguousarray(mat, dtype=np.int32)
        mc = cfg.get("material_c")
        self.mc = None if mc is None else np.ascontiguousarray(mc, dtype=np.float64)
        if self.mc is not None and self.mat is None:
            raise ValueError("a material table needs mesh.materials")
        self.cm = _Mesh(self.V.shape[0], self.E.shape[0], _ptr(self.V),
                        _ptr(self.E), _ptr(self.lab), None if self.mat is None else _ptr(self.mat))
        self.cc = _Cfg(KERNELS[cfg["kernel"]], self.n, float(cfg["c"]),
                       float(cfg["delta"]), APPROACHES[cfg.get("approach", "bary")],
                       pn, _ptr(self.pdirs),
                       self.pw.shape[0], _ptr(self.pxi), _ptr(self.pw),
                       self.qw.shape[0], _ptr(self.qxi), _ptr(self.qw),
                       ns, _ptr(self.glx), _ptr(self.glw), 1 if self.dg else 0,
                       0 if self.mc is None else self.mc.shape[0],
                       None if self.mc is None else _ptr(self.mc))

    @property
    def n_unknowns(self):
        """Scalar unknowns per component: vertices (CG) or 3 per element (DG)."""
        return 3 * self.E.shape[0] if self.dg else self.V.shape[0]

    def unknowns_of(self, k):
        """Unknown ids of the vertices of elements k ([len(k), 3])."""
        k = np.asarray(k)
        if self.dg:
            return (3 * k.astype(np.int64))[:, None] + np.arange(3)[None, :]
        return self.E[k]

    # -- pairs -------------------------------------------------------
    def pairs(self, elem_mask=None):
        L = lib()
        mk = None if elem_mask is None else np.ascontiguousarray(elem_mask, dtype=np.uint8)
        total = L.orc_pairs(C.byref(self.cm), C.byref(self.cc), _ptr(mk), None, None, None, 0)
        if total < 0:
            raise MemoryError("oracle pair count failed")
        k = np.empty(total, np.int32)
        l = np.empty(total, np.int32)
        c = np.empty(total, np.int8)
        if total:
            L.orc_pairs(C.byref(self.cm), C.byref(self.cc), _ptr(mk), _ptr(k), _ptr(l), _ptr(c), total)
        return k, l, c

    def pairs_bfs(self):
        L = lib()
        cap = 64 * max(1, self.E.shape[0])
        while True:
            k = np.empty(cap, np.int32)
            l = np.empty(cap, np.int32)
            c = np.empty(cap, np.int8)
            total = L.orc_pairs_bfs(C.byref(self.cm), C.byref(self.cc), _ptr(k), _ptr(l), _ptr(c), cap)
            if total <= cap:
                return k[:total], l[:total], c[:total]
            cap = total

    # -- local matrices ------------------------------------------------
    def local(self, k, l, cls):
        L = lib()
        nodes = np.zeros(6, np.int32)
        mat = np.zeros((12 * 12,), np.float64)
        nu = L.orc_local(C.byref(self.cm), C.byref(self.cc), int(k), int(l), int(cls),
                         _ptr(nodes), _ptr(mat))
        d = nu * self.n
        return nodes[:nu].copy(), mat[:d * d].reshape(d, d).copy()

    # -- degrees of freedom and pattern --------------------------------
    def isdof(self):
        if self.dg:
            # the three unknowns of every Omega element
            return np.repeat(self.lab == 1, 3)
        M = self.V.shape[0]
        in_omega = np.zeros(M, bool)
        in_dir = np.zeros(M, bool)
        in_omega[self.E[self.lab == 1].reshape(-1)] = True
        in_dir[self.E[self.lab == 2].reshape(-1)] = True
        return in_omega & ~in_dir

    def pattern(self, k, l, rowsel=None):
        """CSR pattern (row_ptr int64 [nM+1], col int32) of the listed pairs."""
        M = self.n_unknowns
        n = self.n
        isdof = self.isdof()
        if rowsel is not None:
            isdof = isdof & rowsel
        keys = []
        chunk = 1 << 18
        for s in range(0, len(k), chunk):
            nodes = np.concatenate([self.unknowns_of(k[s:s + chunk]), self.unknowns_of(l[s:s + chunk])], axis=1)
            rows = np.repeat(nodes, 6, axis=1).reshape(-1)
            cols = np.tile(nodes, (1, 6)).reshape(-1)
            ok = isdof[rows]
            keys.append(np.unique(rows[ok].astype(np.int64) * M + cols[ok]))
        keys = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
        ri = keys // M
        cj = keys % M
        # expand node pairs (i, j) to components: row n i + c, cols n j + d
        cnt = np.bincount(ri, minlength=M)          # node-level row lengths
        nptr = np.zeros(M + 1, np.int64)
        np.cumsum(cnt, out=nptr[1:])
        row_len = np.repeat(cnt * n, n)              # each component row has n*len entries
        row_ptr = np.zeros(n * M + 1, np.int64)
        np.cumsum(row_len, out=row_ptr[1:])
        col = np.empty(int(row_ptr[-1]), np.int32)
        for c in range(n):
            for d in range(n):
                # position of (n i + c, n j + d): row_ptr[n i + c] + n * (rank of j in row i) + d
                rank = np.arange(len(keys)) - nptr[ri]
                pos = row_ptr[n * ri + c] + n * rank + d
                col[pos] = (n * cj + d).astype(np.int32)
        return row_ptr, col

    # -- assembly --------------------------------------------------------
    def assemble(self, pairs=None, rowsel=None):
        """Full (or row-restricted) stiffness matrix as CSR arrays."""
        if pairs is None:
            pairs = self.pairs()
        k, l, c = [np.ascontiguousarray(a) for a in pairs]
        row_ptr, col = self.pattern(k, l, rowsel)
        val = np.zeros(col.shape[0], np.float64)
        isdof = self.isdof().astype(np.uint8)
        rs = None if rowsel is None else np.ascontiguousarray(rowsel, dtype=np.uint8)
        rc = lib().orc_assemble(C.byref(self.cm), C.byref(self.cc), len(k), _ptr(k), _ptr(l),
                                _ptr(c), _ptr(isdof), _ptr(rs), _ptr(row_ptr), _ptr(col), _ptr(val))
        if rc != 0:
            raise RuntimeError("oracle assembly hit an entry outside the pattern")
        return row_ptr, col, val

    def assemble_rows(self, rows):
        """Rows of the matrix for the given node (DG: unknown) ids only
        (sampled check)."""
        M = self.n_unknowns
        rowsel = np.zeros(M, bool)
        rowsel[np.asarray(rows)] = True
        elem_mask = rowsel[self.unknowns_of(np.arange(self.E.shape[0]))].any(axis=1)
        pairs = self.pairs(elem_mask=elem_mask)
        return self.assemble(pairs=pairs, rowsel=rowsel)

    def inner_moments(self, x, l):
        """[area, int phi_a, int phi_a phi_b] of T_l n B(x) by the oracle's
        inner quadrature (ball approximation of the configuration)."""
        out = np.zeros(13)
        xx = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        lib().orc_inner_moments(C.byref(self.cc), C.byref(self.cm), _ptr(xx), int(l), _ptr(out))
        return out[0], out[1:4].copy(), out[4:].reshape(3, 3).copy()

    def clip_area(self, x, l):
        cnt = C.c_int32(0)
        xx = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        a = lib().orc_clip_area(C.byref(self.cc), _ptr(xx), C.byref(self.cm), int(l), C.byref(cnt))
        return a, cnt.value

    def rhs(self, f_const=None, f_affine=None, f_qp=None):
        n = self.n
        b = np.zeros(n * self.n_unknowns, np.float64)
        if f_qp is not None:
            fq = np.ascontiguousarray(f_qp, dtype=np.float64)
            aff = None
        else:
            if f_affine is None:
                f_affine = [(float(v), 0.0, 0.0) for v in f_const]
            aff = np.ascontiguousarray(np.asarray(f_affine, dtype=np.float64).reshape(-1))
            fq = None
        lib().orc_rhs(C.byref(self.cm), C.byref(self.cc), _ptr(fq), _ptr(aff), _ptr(b))
        return b


def duffy_samples(cls: int, n: int):
    """(xi, eta, weight) samples of the oracle's 4D rule for one class."""
    glx, glw = gauss_legendre01(n)
    L = lib()
    total = L.orc_duffy_samples(cls, n, _ptr(glx), _ptr(glw), None, None, None, 0)
    xi = np.empty((total, 2))
    eta = np.empty((total, 2))
    w = np.empty(total)
    L.orc_duffy_samples(cls, n, _ptr(glx), _ptr(glw), _ptr(xi), _ptr(eta), _ptr(w), total)
    return xi, eta, w


def num_threads() -> int:
    return int(lib().orc_num_threads())
