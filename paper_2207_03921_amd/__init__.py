"""Python binding of libnlfem (gfx950 nonlocal P1 stiffness assembly).

Thin ctypes layer over the C ABI declared in ``include/nlfem.h``: every
function here has the name of the C entry point it marshals arguments for.
PyTorch supplies device memory and the current HIP stream; all arithmetic
runs in the library's kernels.  There is no fallback: if ``libnlfem.so`` is
missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlfem.so")

NLFEM_OK = 0
ERRORS = {-1: "E_INVALID", -2: "E_MESH", -3: "E_NOMEM", -4: "E_HIP", -5: "E_OVERFLOW",
          -6: "E_MISMATCH", -7: "E_NODEVICE"}
K_CONSTANT, K_INV_DIST, K_PERIDYNAMIC, K_FRAC_HALF = 0, 1, 2, 3
A_NOCAPS_BARY, A_APPROXCAPS_POLY, A_INF_BALL, A_NOCAPS, A_APPROXCAPS = 0, 1, 2, 3, 4
P_FP64, P_MIXED = 0, 1
C_FAR, C_VERTEX, C_EDGE, C_IDENT = 0, 1, 2, 3

KERNELS = {"constant": K_CONSTANT, "inv_dist": K_INV_DIST, "peridynamic": K_PERIDYNAMIC, "frac_half": K_FRAC_HALF}
APPROACHES = {"bary": A_NOCAPS_BARY, "poly": A_APPROXCAPS_POLY, "inf": A_INF_BALL, "nocaps": A_NOCAPS,
              "approxcaps": A_APPROXCAPS}
PRECISIONS = {"fp64": P_FP64, "mixed": P_MIXED}
ANSATZ = {"cg": 0, "dg": 1}


class NlfemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_elements", C.c_int64),
                ("vertices", C.c_void_p), ("elements", C.c_void_p), ("labels", C.c_void_p),
                ("materials", C.c_void_p)]


class _Rule(C.Structure):
    _fields_ = [("n", C.c_int32), ("xi", C.c_void_p), ("w", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("c", C.c_double), ("delta", C.c_double),
                ("approach", C.c_int32), ("polygon_n", C.c_int32), ("polygon_dirs", C.c_void_p),
                ("outer", _Rule), ("inner", _Rule), ("singular_n", C.c_int32),
                ("precision", C.c_int32), ("ansatz", C.c_int32), ("n_materials", C.c_int32),
                ("material_c", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_pairs", "n_far", "n_vertex", "n_edge", "n_ident",
                                         "n_dof", "n_rows", "nnz", "n_upper_far", "n_upper_touch", "n_nbr",
                                         "rebuild", "skipped")]


ABI_VERSION = 5   # layout of the structs below
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_lib = None
_hooks = []   # every callback pair ever installed: blocks keep their free function
# until they are released, so no pair may be collected before the process ends


def lib():
    """Loads libnlfem.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NlfemError(-4, f"{LIB_PATH} not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int
        L.nlfem_version.restype = C.c_int32
        if L.nlfem_version() != ABI_VERSION:
            raise NlfemError(-4, f"{LIB_PATH} has ABI {L.nlfem_version()}, the binding expects {ABI_VERSION}")
        L.nlfem_last_error.restype = C.c_char_p
        L.nlfem_build_pairs.argtypes = [vp, vp, C.POINTER(vp), vp]
        L.nlfem_build_pairs.restype = i32
        L.nlfem_pairs_info.argtypes = [vp, vp]
        L.nlfem_pairs_info.restype = i32
        L.nlfem_pairs_export.argtypes = [vp, vp, vp, vp, vp]
        L.nlfem_pairs_export.restype = i32
        L.nlfem_csr_pattern.argtypes = [vp, vp, vp, vp]
        L.nlfem_csr_pattern.restype = i32
        L.nlfem_assemble.argtypes = [vp, vp, vp, vp, vp]
        L.nlfem_assemble.restype = i32
        L.nlfem_rhs.argtypes = [vp, vp, vp, vp, vp, vp]
        L.nlfem_rhs.restype = i32
        L.nlfem_pairs_free.argtypes = [vp]
        L.nlfem_pairs_free.restype = None
        L.nlfem_timing_enable.argtypes = [C.c_int]
        L.nlfem_timing_enable.restype = i32
        L.nlfem_timing_read.argtypes = [vp, vp, C.c_int]
        L.nlfem_timing_read.restype = i32
        L.nlfem_batch_create.argtypes = [C.c_int32, vp, vp, vp, vp, C.c_char_p, C.c_int32, C.POINTER(vp), vp]
        L.nlfem_batch_create.restype = i32
        L.nlfem_batch_assemble.argtypes = [vp, vp]
        L.nlfem_batch_assemble.restype = i32
        L.nlfem_batch_launch_graph.argtypes = [vp, vp]
        L.nlfem_batch_launch_graph.restype = i32
        L.nlfem_batch_info.argtypes = [vp, vp, vp]
        L.nlfem_batch_info.restype = i32
        L.nlfem_batch_free.argtypes = [vp]
        L.nlfem_batch_free.restype = None
        L.nlfem_assemble_batched.argtypes = [C.c_int32, vp, vp, vp, vp, C.c_char_p, vp]
        L.nlfem_assemble_batched.restype = i32
        L.nlfem_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
        L.nlfem_set_allocator.restype = i32
        L.nlfem_set_capacity.argtypes = [C.c_int64]
        L.nlfem_set_capacity.restype = i32
        L.nlfem_assemble_batched_noalloc.argtypes = [C.c_int32, vp, vp, vp, vp, vp]
        L.nlfem_assemble_batched_noalloc.restype = i32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != NLFEM_OK:
        raise NlfemError(rc, lib().nlfem_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t.data_ptr()


@dataclass
class DeviceMesh:
    """Device copies of a mesh (vertices float64 [M,2], elements int32 [K,3],
    labels int32 [K], optional materials int32 [K])."""
    vertices: object
    elements: object
    labels: object
    materials: object = None

    @classmethod
    def from_numpy(cls, mesh, device="cuda"):
        import torch
        mat = getattr(mesh, "materials", None)
        return cls(torch.as_tensor(np.ascontiguousarray(mesh.vertices, np.float64), device=device),
                   torch.as_tensor(np.ascontiguousarray(mesh.elements, np.int32), device=device),
                   torch.as_tensor(np.ascontiguousarray(mesh.labels, np.int32), device=device),
                   None if mat is None else torch.as_tensor(np.ascontiguousarray(mat, np.int32), device=device))

    def c_struct(self):
        import torch
        return _Mesh(self.vertices.shape[0], self.elements.shape[0],
                     _dev_ptr(self.vertices, torch.float64, "vertices"),
                     _dev_ptr(self.elements, torch.int32, "elements"),
                     _dev_ptr(self.labels, torch.int32, "labels"),
                     None if self.materials is None else _dev_ptr(self.materials, torch.int32, "materials"))


@dataclass
class Config:
    """Mirror of nlfem_config; host tables are kept alive by this object."""
    kernel: str
    c: float
    delta: float
    outer_xi: np.ndarray
    outer_w: np.ndarray
    inner_xi: np.ndarray
    inner_w: np.ndarray
    approach: str = "bary"
    polygon_dirs: np.ndarray | None = None
    singular_n: int = 0
    precision: str = "fp64"
    ansatz: str = "cg"
    material_c: np.ndarray | None = None   # [n][n]: Psi(x, y) = material_c[m(x)][m(y)] Psi0
    _keep: list = field(default_factory=list, repr=False)

    @property
    def ncomp(self) -> int:
        return 2 if self.kernel == "peridynamic" else 1

    def c_struct(self):
        # reused while no field was rebound and every table is already a
        # contiguous float64 array (the struct then points at the caller's
        # arrays, so changes made in place are seen)
        key = (self.kernel, self.c, self.delta, self.approach, self.singular_n, self.precision, self.ansatz,
               id(self.outer_xi), id(self.outer_w), id(self.inner_xi), id(self.inner_w), id(self.polygon_dirs),
               id(self.material_c))
        cached = self.__dict__.get("_cs")
        if cached is not None and cached[0] == key:
            return cached[1]
        arrs = [np.ascontiguousarray(a, np.float64) for a in
                (self.outer_xi, self.outer_w, self.inner_xi, self.inner_w)]
        dirs = None if self.polygon_dirs is None else np.ascontiguousarray(self.polygon_dirs, np.float64)
        mc = None if self.material_c is None else np.ascontiguousarray(self.material_c, np.float64)
        self._keep = arrs + [dirs, mc]
        oxi, ow, ixi, iw = arrs
        cs = _Config(KERNELS[self.kernel], float(self.c), float(self.delta),
                     APPROACHES[self.approach], 0 if dirs is None else dirs.shape[0],
                     None if dirs is None else dirs.ctypes.data,
                     _Rule(ow.shape[0], oxi.ctypes.data, ow.ctypes.data),
                     _Rule(iw.shape[0], ixi.ctypes.data, iw.ctypes.data),
                     int(self.singular_n), PRECISIONS[self.precision], ANSATZ[self.ansatz],
                     0 if mc is None else mc.shape[0], None if mc is None else mc.ctypes.data)
        src = (self.outer_xi, self.outer_w, self.inner_xi, self.inner_w)
        if all(a is b for a, b in zip(arrs, src)) and (dirs is None or dirs is self.polygon_dirs) and \
                (mc is None or mc is self.material_c):
            self.__dict__["_cs"] = (key, cs)
        return cs


class Pairs:
    """Owner of an nlfem_pairs handle."""

    def __init__(self, ptr: C.c_void_p, ncomp: int, n_vertices: int, n_unknowns: int | None = None):
        self.ptr = ptr
        self.ncomp = ncomp
        self.n_vertices = n_vertices
        # scalar unknowns per component: vertices (continuous) or 3 per element
        self.n_unknowns = n_vertices if n_unknowns is None else n_unknowns

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value and _lib is not None:
            _lib.nlfem_pairs_free(self.ptr)
            self.ptr = C.c_void_p(None)


def nlfem_version() -> int:
    return int(lib().nlfem_version())


def nlfem_last_error() -> str:
    return lib().nlfem_last_error().decode()


def nlfem_build_pairs(mesh: DeviceMesh, cfg: Config, pairs: Pairs | None = None, stream=None) -> Pairs:
    cm, cc = mesh.c_struct(), cfg.c_struct()
    h = C.c_void_p(None if pairs is None else pairs.ptr.value)
    _check(lib().nlfem_build_pairs(C.byref(cm), C.byref(cc), C.byref(h), _stream(stream)))
    nunk = 3 * int(mesh.elements.shape[0]) if cfg.ansatz == "dg" else int(mesh.vertices.shape[0])
    if pairs is not None:
        pairs.ptr = h
        pairs.ncomp = cfg.ncomp
        pairs.n_vertices = int(mesh.vertices.shape[0])
        pairs.n_unknowns = nunk
        return pairs
    return Pairs(h, cfg.ncomp, int(mesh.vertices.shape[0]), nunk)


def nlfem_pairs_info(pairs: Pairs) -> dict:
    info = _Info()
    _check(lib().nlfem_pairs_info(pairs.ptr, C.byref(info)))
    return {n: int(getattr(info, n)) for n, _ in _Info._fields_}


def nlfem_pairs_export(pairs: Pairs, stream=None):
    import torch
    n = nlfem_pairs_info(pairs)["n_pairs"]
    k = torch.empty(n, dtype=torch.int32, device="cuda")
    l = torch.empty(n, dtype=torch.int32, device="cuda")
    c = torch.empty(n, dtype=torch.int8, device="cuda")
    _check(lib().nlfem_pairs_export(pairs.ptr, C.c_void_p(k.data_ptr()), C.c_void_p(l.data_ptr()),
                                    C.c_void_p(c.data_ptr()), _stream(stream)))
    return k, l, c


def nlfem_csr_pattern(pairs: Pairs, stream=None):
    import torch
    info = nlfem_pairs_info(pairs)
    rp = torch.empty(pairs.ncomp * pairs.n_unknowns + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(max(info["nnz"], 1), dtype=torch.int32, device="cuda")
    _check(lib().nlfem_csr_pattern(pairs.ptr, C.c_void_p(rp.data_ptr()), C.c_void_p(col.data_ptr()),
                                   _stream(stream)))
    return rp, col[:info["nnz"]]


def nlfem_assemble(mesh: DeviceMesh, cfg: Config, pairs: Pairs, val=None, stream=None):
    import torch
    if val is None:
        nnz = nlfem_pairs_info(pairs)["nnz"]
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda")
    cm, cc = mesh.c_struct(), cfg.c_struct()
    _check(lib().nlfem_assemble(C.byref(cm), C.byref(cc), pairs.ptr,
                                C.c_void_p(_dev_ptr(val, torch.float64, "val")), _stream(stream)))
    return val


def nlfem_rhs(mesh: DeviceMesh, cfg: Config, f_qp=None, f_affine=None, b=None, stream=None):
    import torch
    n = cfg.ncomp
    if b is None:
        nunk = 3 * mesh.elements.shape[0] if cfg.ansatz == "dg" else mesh.vertices.shape[0]
        b = torch.empty(n * nunk, dtype=torch.float64, device="cuda")
    cm, cc = mesh.c_struct(), cfg.c_struct()
    fq = None if f_qp is None else C.c_void_p(_dev_ptr(f_qp, torch.float64, "f_qp"))
    aff = None
    if f_affine is not None:
        aff = np.ascontiguousarray(np.asarray(f_affine, np.float64).reshape(-1))
    _check(lib().nlfem_rhs(C.byref(cm), C.byref(cc), fq, None if aff is None else aff.ctypes.data,
                           C.c_void_p(_dev_ptr(b, torch.float64, "b")), _stream(stream)))
    return b


TIMING_PHASES = ("geometry", "pairs", "lists", "csr", "far", "touch", "rows", "rhs", "diag")


def nlfem_timing_enable(phases=True):
    """True: time every phase; False/None: off; an iterable of phase names:
    time only those."""
    if phases is True:
        mask = (1 << len(TIMING_PHASES)) - 1
    elif not phases:
        mask = 0
    else:
        mask = 0
        for p in phases:
            mask |= 1 << TIMING_PHASES.index(p)
    _check(lib().nlfem_timing_enable(mask))


def nlfem_timing_read(reset: bool = True) -> dict:
    ms = np.zeros(len(TIMING_PHASES), np.float64)
    n = np.zeros(len(TIMING_PHASES), np.int64)
    _check(lib().nlfem_timing_read(ms.ctypes.data, n.ctypes.data, 1 if reset else 0))
    return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(TIMING_PHASES)}


def nlfem_set_allocator(alloc=None, free=None, ctx=None):
    """Installs device-allocation hooks: alloc(nbytes, stream) -> int device
    pointer (0 = failure) and free(ptr, stream), both called with plain ints.
    Both None restores hipMalloc/hipFree.  A Python exception inside a hook
    counts as a failed allocation (alloc) or is ignored (free)."""
    if (alloc is None) != (free is None):
        raise ValueError("give both allocator functions or neither")
    if alloc is None:
        _check(lib().nlfem_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def _a(nbytes, stream, _ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:   # noqa: BLE001 - reported by the library as E_NOMEM
            return None

    def _f(ptr, stream, _ctx):
        try:
            free(int(ptr), int(stream or 0))
        except Exception:   # noqa: BLE001 - nothing to report to
            pass

    hooks = (ALLOC_FN(_a), FREE_FN(_f))
    _hooks.append(hooks)
    _check(lib().nlfem_set_allocator(hooks[0], hooks[1], None))


def torch_allocator():
    """(alloc, free) hooks that take device memory from torch's caching
    allocator on the library's stream."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def nlfem_set_capacity(max_entries: int = 0):
    _check(lib().nlfem_set_capacity(int(max_entries)))


def nlfem_pairs_free(pairs: Pairs):
    if pairs.ptr.value:
        lib().nlfem_pairs_free(pairs.ptr)
        pairs.ptr = C.c_void_p(None)


def assemble(mesh: DeviceMesh, cfg: Config, f_affine=None, stream=None):
    """Builds the pairs, assembles and returns (torch sparse CSR matrix, b)."""
    import torch
    pairs = nlfem_build_pairs(mesh, cfg, stream=stream)
    rp, col = nlfem_csr_pattern(pairs, stream=stream)
    val = nlfem_assemble(mesh, cfg, pairs, stream=stream)
    nnz = col.shape[0]
    N = cfg.ncomp * (3 * mesh.elements.shape[0] if cfg.ansatz == "dg" else mesh.vertices.shape[0])
    A = torch.sparse_csr_tensor(rp, col, val[:nnz], size=(N, N))
    if f_affine is None:
        f_affine = [(0.0, 0.0, 0.0)] * cfg.ncomp
    b = nlfem_rhs(mesh, cfg, f_affine=f_affine, stream=stream)
    return A, b


# ---------------------------------------------------------------- batches

class Batch:
    """Owner of an nlfem_batch; keeps the inputs it refers to alive."""

    def __init__(self, ptr, keep):
        self.ptr = ptr
        self._keep = keep

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value and _lib is not None:
            _lib.nlfem_batch_free(self.ptr)
            self.ptr = C.c_void_p(None)


def _batch_arrays(meshes, cfgs, pairs, vals):
    import torch
    n = len(meshes)
    if not (len(cfgs) == len(pairs) == len(vals) == n):
        raise ValueError("meshes, cfgs, pairs and vals must have the same length")
    cm = (_Mesh * n)(*[m.c_struct() for m in meshes])
    structs, tables = [], []
    for c in cfgs:   # a config may appear several times: keep every table set alive
        structs.append(c.c_struct())
        tables.append(list(c._keep))
    cc = (_Config * n)(*structs)
    ph = (C.c_void_p * n)(*[p.ptr.value for p in pairs])
    vp = (C.c_void_p * n)(*[_dev_ptr(v, torch.float64, "val") for v in vals])
    cc._tables = tables
    return n, cm, cc, ph, vp


def nlfem_batch_create(meshes, cfgs, pairs, vals, tune_cache=None, tune=0, stream=None) -> Batch:
    n, cm, cc, ph, vp = _batch_arrays(meshes, cfgs, pairs, vals)
    h = C.c_void_p(None)
    path = None if tune_cache is None else os.fsencode(tune_cache)
    _check(lib().nlfem_batch_create(n, cm, cc, ph, vp, path, int(tune), C.byref(h), _stream(stream)))
    return Batch(h, (list(meshes), list(cfgs), list(pairs), list(vals), cm, cc, ph, vp))


def nlfem_batch_assemble(batch: Batch, stream=None):
    _check(lib().nlfem_batch_assemble(batch.ptr, _stream(stream)))


def nlfem_batch_launch_graph(batch: Batch, stream=None):
    _check(lib().nlfem_batch_launch_graph(batch.ptr, _stream(stream)))


def nlfem_batch_info(batch: Batch) -> dict:
    g = C.c_int32(0)
    sh = (C.c_int32 * 8)()
    _check(lib().nlfem_batch_info(batch.ptr, C.byref(g), sh))
    names = ("far", "touch", "diag", "rows")
    return {"groups": int(g.value),
            "shape": {nm: {"chunk": int(sh[2 * i]), "per_cu": int(sh[2 * i + 1])} for i, nm in enumerate(names)}}


def nlfem_batch_free(batch: Batch):
    if batch.ptr.value:
        lib().nlfem_batch_free(batch.ptr)
        batch.ptr = C.c_void_p(None)


def nlfem_assemble_batched(meshes, cfgs, pairs, vals, tune_cache=None, stream=None):
    n, cm, cc, ph, vp = _batch_arrays(meshes, cfgs, pairs, vals)
    path = None if tune_cache is None else os.fsencode(tune_cache)
    _check(lib().nlfem_assemble_batched(n, cm, cc, ph, vp, path, _stream(stream)))
    return vals


def nlfem_assemble_batched_noalloc(meshes, cfgs, pairs, vals, stream=None):
    """The one-shot batch with its tables in the library's static device
    array: no device allocation."""
    n, cm, cc, ph, vp = _batch_arrays(meshes, cfgs, pairs, vals)
    _check(lib().nlfem_assemble_batched_noalloc(n, cm, cc, ph, vp, _stream(stream)))
    return vals
