"""Parity of the HIP path with the CPU oracle (MI355X only).

Pair lists and CSR patterns must match bit for bit; values within 1e-12
relative Frobenius norm in FP64 and 1e-5 in the mixed FP32/FP64 form (the
FP32 far-field error bound: relative coordinates keep z accurate to a few
1e-7 of delta, accumulation over 49 terms adds < 1e-6).
"""
import numpy as np
import pytest

from inputs import square_mesh, gauss7, paper7, collapsed, centroid1
from inputs.meshes import Mesh
from inputs.workloads import small_constant, inv_dist_jittered, peridynamic, constant_polygon, c_frac
from _gpu import gpu_run, to_sparse, rel_frob, entrywise, f_affine_of

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def _w(kernel, mesh, delta, rule=None, inner=None, singular_n=None, approach="bary", **kw):
    rule = rule or gauss7()
    if kernel == "constant":
        c = c_frac(-1.0, delta)
    elif kernel == "inv_dist":
        c = c_frac(-0.5, delta)
    elif kernel == "frac_half":
        c = c_frac(0.5, delta)
    else:
        c = 6.0 / (np.pi * delta ** 3)
    if singular_n is None:
        singular_n = 0 if kernel == "constant" else 5
    d = dict(name="adhoc", mesh=mesh, kernel=kernel, c=c, delta=delta, approach=approach,
             polygon_n=32, outer=rule, inner=inner or rule, singular_n=singular_n,
             precision="fp64", f=(-4.0,), ncomp=2 if kernel == "peridynamic" else 1)
    if kernel == "peridynamic":
        d["f"] = None
        d["f_affine"] = ((-1.0, -2.0, 0.0), (0.0, 0.0, -1.0))
    d.update(kw)
    return d


def _cases():
    return {
        "const_h16": small_constant(),
        "invdist_h24": inv_dist_jittered(n=24, delta=0.1, precision="fp64"),
        "peri_h20": peridynamic(n=20, ratio=3, precision="fp64"),
        "const_paper7": _w("constant", square_mesh(12, delta=0.15, jitter=0.1, seed=5), 0.15, rule=paper7()),
        "invdist_rule9": _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.15, seed=6), 0.2,
                            rule=collapsed(3)),
        "const_outer_ne_inner": _w("constant", square_mesh(10, delta=0.2, jitter=0.15, seed=7), 0.2,
                                   rule=gauss7(), inner=paper7()),
        "invdist_neumann": _w("inv_dist", square_mesh(12, delta=0.2, jitter=0.2, seed=8, neumann=True), 0.2),
        # constant kernel, barycentre ball: far blocks from the status masks
        # with 1 and 4 outer points (one nibble), and with 9 outer points
        # (more than the mask form takes: far records)
        "const_outer1_inner7": _w("constant", square_mesh(10, delta=0.2, jitter=0.15, seed=60), 0.2,
                                  rule=centroid1(), inner=gauss7()),
        "const_outer4_inner7": _w("constant", square_mesh(10, delta=0.2, jitter=0.15, seed=61), 0.2,
                                  rule=collapsed(2), inner=paper7()),
        "const_rule9": _w("constant", square_mesh(10, delta=0.2, jitter=0.15, seed=62), 0.2, rule=collapsed(3)),
        "const_duffy": _w("constant", square_mesh(12, delta=0.15, jitter=0.2, seed=9), 0.15, singular_n=4),
        # inscribed 32-gon: straddling points are clipped and fan-triangulated
        "const_poly_h16": _w("constant", square_mesh(16, delta=0.1), 0.1, approach="poly"),
        "const_poly_small_delta": _w("constant", square_mesh(8, delta=0.1, jitter=0.1, seed=12), 0.1,
                                     approach="poly"),
        "invdist_poly": _w("inv_dist", square_mesh(12, delta=0.15, jitter=0.2, seed=11), 0.15, approach="poly"),
        "peri_poly": _w("peridynamic", square_mesh(10, delta=0.25, jitter=0.1, seed=13), 0.25, approach="poly"),
        "const_poly_outer_ne_inner": _w("constant", square_mesh(10, delta=0.15, jitter=0.15, seed=14), 0.15,
                                        rule=gauss7(), inner=paper7(), approach="poly"),
        # outer and inner rules of different sizes (7 and 4 points; 7 and 1)
        "const_poly_p7_q4": _w("constant", square_mesh(10, delta=0.15, jitter=0.1, seed=15), 0.15,
                               rule=gauss7(), inner=collapsed(2), approach="poly"),
        "invdist_p7_q1": _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.15, seed=16), 0.2,
                            rule=gauss7(), inner=centroid1()),
        # infinity-norm ball (Def. 2.5): the square clipped exactly
        "const_inf_h16": _w("constant", square_mesh(16, delta=0.1), 0.1, approach="inf",
                            c=3.0 / (4.0 * 0.1 ** 4)),
        "const_inf_paper7_jit": _w("constant", square_mesh(10, delta=0.15, jitter=0.2, seed=19), 0.15,
                                   rule=paper7(), approach="inf", c=3.0 / (4.0 * 0.15 ** 4)),
        "invdist_inf": _w("inv_dist", square_mesh(12, delta=0.15, jitter=0.2, seed=20), 0.15, approach="inf"),
        "peri_inf": _w("peridynamic", square_mesh(10, delta=0.25, jitter=0.1, seed=21), 0.25, approach="inf"),
        # fractional-type kernel c/|z|^3 (s = 1/2, Sec. 3.1): hypersingular
        # touching pairs through the transforms with d = -1
        "frac_h16": _w("frac_half", square_mesh(16, delta=0.15, jitter=0.2, seed=24), 0.15),
        "frac_poly": _w("frac_half", square_mesh(12, delta=0.15, jitter=0.15, seed=25), 0.15, approach="poly"),
        "frac_inf_paper7": _w("frac_half", square_mesh(10, delta=0.2, jitter=0.1, seed=26), 0.2, approach="inf",
                              rule=paper7()),
        # the paper's balls (Def. 2.3 nocaps, Def. 2.4 approximate caps); the
        # uniform meshes with the vertex rule put points exactly on circles
        "const_nocaps_h16": _w("constant", square_mesh(16, delta=0.1, jitter=0.1, seed=27), 0.1, approach="nocaps"),
        "const_nocaps_uniform_paper7": _w("constant", square_mesh(12, delta=0.25), 0.25, approach="nocaps",
                                          rule=paper7()),
        "invdist_approxcaps": _w("inv_dist", square_mesh(12, delta=0.15, jitter=0.2, seed=28), 0.15,
                                 approach="approxcaps"),
        "frac_approxcaps_table2": _w("frac_half", square_mesh(10, delta=0.2, side=0.5), 0.2, approach="approxcaps",
                                     rule=paper7()),
        "peri_approxcaps": _w("peridynamic", square_mesh(10, delta=0.25, jitter=0.1, seed=29), 0.25,
                              approach="approxcaps"),
        # weakly singular kernels with the standard rule on touching pairs
        # (Table 1, singular_n = 0): the vertex rule puts points of both
        # elements on shared vertices and mid-sides, which are skipped
        "invdist_nozerodiv_paper7": _w("inv_dist", square_mesh(12, delta=0.15, jitter=0.2, seed=40), 0.15,
                                       rule=paper7(), singular_n=0),
        "peri_nozerodiv_approxcaps_table4": _w("peridynamic", square_mesh(10, delta=0.1, side=0.5), 0.1,
                                               approach="approxcaps", rule=paper7(), singular_n=0),
        "invdist_nozerodiv_poly": _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.1, seed=41), 0.2,
                                     approach="poly", rule=paper7(), singular_n=0),
    }


def _fan_mesh(nseg=72, r=0.1):
    """A node of valence nseg: nseg Omega triangles around the origin, closed
    by a ring of 2 nseg Omega_D triangles out to radius 2r (only the centre
    is a degree of freedom)."""
    ang = 2 * np.pi * np.arange(nseg) / nseg
    inner = np.stack([r * np.cos(ang), r * np.sin(ang)], 1)
    outer = np.stack([2 * r * np.cos(ang + np.pi / nseg), 2 * r * np.sin(ang + np.pi / nseg)], 1)
    V = np.vstack([[[0.0, 0.0]], inner, outer])
    E, L = [], []
    for i in range(nseg):
        j = (i + 1) % nseg
        E.append([0, 1 + i, 1 + j])
        L.append(1)
        E.append([1 + i, 1 + nseg + i, 1 + j])
        E.append([1 + j, 1 + nseg + i, 1 + nseg + j])
        L += [2, 2]
    return Mesh(V, np.array(E, np.int32), np.array(L, np.int32), r, 1, 1)


def _long_path_cases():
    """Meshes whose lists and rows exceed the short-list kernels' sizes: a
    horizon of 9-10 mesh sizes (neighbour lists above 256 entries: bitonic
    sort; CSR rows above 256 columns: bitonic row sort), and a node of
    valence 72 (more than one batch of 64 elements in the row gather, and
    more than 256 touching entries queued in one batch: the queue is flushed
    before the batch ends)."""
    return {
        "invdist_delta_10h": _w("inv_dist", square_mesh(8, delta=1.25, jitter=0.1, seed=17), 1.25),
        "peri_delta_9h": _w("peridynamic", square_mesh(6, delta=1.5, jitter=0.1, seed=18), 1.5),
        "invdist_fan72": _w("inv_dist", _fan_mesh(72), 0.3),
        # 16 mesh sizes: hash tables of 8192 ids, two rows per workgroup in
        # the symbolic pass
        "invdist_delta_16h": _w("inv_dist", square_mesh(6, delta=16.0 / 6.0, jitter=0.1, seed=32), 16.0 / 6.0),
    }


def _ignored_labels_case():
    mesh = square_mesh(12, delta=0.2, jitter=0.1, seed=10)
    lab = mesh.labels.copy()
    lab[::7] = 3            # elements outside the discretisation
    mesh = Mesh(mesh.vertices, mesh.elements, lab, mesh.h, mesh.n, mesh.m)
    return _w("inv_dist", mesh, 0.2)


def _compare_full(oracle_lib, w, precision):
    mesh = w["mesh"]
    P = oracle_lib.Problem(mesh, w)
    k, l, c = P.pairs()
    rp, col, val = P.assemble((k, l, c))
    g = gpu_run(mesh, w, precision=precision)
    gk, gl, gc = g["pairs"]
    assert np.array_equal(gk, k) and np.array_equal(gl, l) and np.array_equal(gc, c), "pair list"
    assert np.array_equal(g["row_ptr"], rp) and np.array_equal(g["col"], col), "CSR pattern"
    n = P.n * P.n_unknowns
    A = to_sparse(rp, col, val, n)
    G = to_sparse(g["row_ptr"], g["col"], g["val"], n)
    err = rel_frob(G, A)
    assert err <= TOL[precision], err
    ew = entrywise(G, A)
    assert ew <= TOL[precision], ew
    b = P.rhs(f_affine=f_affine_of(w))
    assert np.abs(g["b"] - b).max() <= 1e-13 * max(1.0, np.abs(b).max())
    info = g["info"]
    assert info["n_pairs"] == len(k)
    assert info["n_far"] == int((c == 0).sum())
    assert info["n_vertex"] == int((c == 1).sum()) and info["n_edge"] == int((c == 2).sum())
    assert info["n_ident"] == int((c == 3).sum())
    assert info["nnz"] == len(col)
    assert info["n_dof"] == int(P.isdof().sum())
    return err


@pytest.mark.parametrize("name", list(_long_path_cases()))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_long_lists_and_rows(oracle_lib, name, precision):
    w = _long_path_cases()[name]
    mesh = w["mesh"]
    print(f"case {name} {precision} K={mesh.n_elements}", flush=True)
    P = oracle_lib.Problem(mesh, w)
    k, l, c = P.pairs()
    rp, col = P.pattern(k, l)
    seg = np.bincount(np.concatenate([k, l]), minlength=mesh.n_elements)   # >= |S(e)|
    if name == "invdist_fan72":
        centre_elems = np.flatnonzero((mesh.elements == 0).any(axis=1))
        assert len(centre_elems) > 64                                    # two element batches
        touch_centre = np.isin(k, centre_elems) & (c != 0)
        assert touch_centre.sum() > 2 * 256                              # touching queue flushed
    else:
        assert np.diff(rp).max() > 256 * P.n                             # bitonic row sort
        assert (seg // 2).max() > 256                                    # bitonic list sort
    if name == "invdist_delta_16h":
        assert (seg // 2).max() > 1100                                   # hash tables of 8192 ids
    _compare_full(oracle_lib, w, precision)


def _dg_cases():
    """Discontinuous P1 ansatz (three unknowns per element): far pairs of
    every ball, touching pairs of singular kernels by the 4D transforms."""
    return {
        "dg_const_bary": _w("constant", square_mesh(10, delta=0.2, jitter=0.2, seed=33), 0.2, ansatz="dg"),
        "dg_invdist": _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.2, seed=34), 0.2, ansatz="dg"),
        "dg_peri": _w("peridynamic", square_mesh(8, delta=0.3, jitter=0.1, seed=35), 0.3, ansatz="dg"),
        "dg_const_poly": _w("constant", square_mesh(10, delta=0.15, jitter=0.1, seed=36), 0.15, approach="poly",
                            ansatz="dg"),
        "dg_invdist_approxcaps": _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.15, seed=37), 0.2,
                                    approach="approxcaps", ansatz="dg", rule=paper7()),
        "dg_const_duffy": _w("constant", square_mesh(8, delta=0.25, jitter=0.2, seed=38), 0.25, singular_n=4,
                             ansatz="dg"),
        # s = 1/2: the edge-touching integrals of jumping functions are the
        # Gauss rule's (log-divergent integrand), the same rule on both sides
        "dg_frac_approxcaps": _w("frac_half", square_mesh(10, delta=0.2, jitter=0.15, seed=39), 0.2,
                                 approach="approxcaps", ansatz="dg", rule=paper7()),
        "dg_peri_nozerodiv": _w("peridynamic", square_mesh(10, delta=0.1, jitter=0.1, seed=42, side=0.5), 0.1,
                                approach="approxcaps", ansatz="dg", rule=paper7(), singular_n=0),
    }


@pytest.mark.parametrize("name", list(_dg_cases()))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_dg(oracle_lib, name, precision):
    w = _dg_cases()[name]
    print(f"case {name} {precision}", flush=True)
    _compare_full(oracle_lib, w, precision)


@pytest.mark.parametrize("name", list(_cases()))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_small(oracle_lib, name, precision):
    w = _cases()[name]
    print(f"case {name} {precision}", flush=True)
    _compare_full(oracle_lib, w, precision)


def test_parity_ignored_labels(oracle_lib):
    _compare_full(oracle_lib, _ignored_labels_case(), "fp64")


def test_single_element_and_tiny_delta(oracle_lib):
    V = np.array([[0.0, 0.0], [1.0, 0.0], [0.2, 0.9]])
    mesh = Mesh(V, np.array([[0, 1, 2]], np.int32), np.array([1], np.int32), 1.0, 1, 0)
    _compare_full(oracle_lib, _w("inv_dist", mesh, 0.5), "fp64")
    # delta below every point-to-barycentre distance except the centroid's:
    # only self pairs for the constant kernel
    mesh = square_mesh(8, delta=0.2, jitter=0.1, seed=11)
    w = _w("constant", mesh, 1e-6)
    _compare_full(oracle_lib, w, "fp64")


def test_all_pairs_interact(oracle_lib):
    mesh = square_mesh(6, m=1, jitter=0.2, seed=12)
    _compare_full(oracle_lib, _w("inv_dist", mesh, 10.0), "fp64")


def test_no_dof_mesh():
    import paper_2207_03921_amd as nl
    mesh = square_mesh(4, m=1)
    lab = np.full_like(mesh.labels, 2)
    mesh = Mesh(mesh.vertices, mesh.elements, lab, mesh.h, mesh.n, mesh.m)
    w = _w("constant", mesh, 0.3)
    g = gpu_run(mesh, w)
    assert g["info"]["n_pairs"] == 0 and g["info"]["nnz"] == 0
    assert np.all(g["row_ptr"] == 0)


def test_mesh_errors():
    import torch
    import paper_2207_03921_amd as nl
    from _gpu import make_config
    mesh = square_mesh(4, m=1)
    w = _w("constant", mesh, 0.3)
    E = mesh.elements.copy()
    E[3] = [0, 1, 1]                # zero area
    dm = nl.DeviceMesh(torch.as_tensor(mesh.vertices, device="cuda"),
                       torch.as_tensor(E, device="cuda"), torch.as_tensor(mesh.labels, device="cuda"))
    with pytest.raises(nl.NlfemError) as ei:
        nl.nlfem_build_pairs(dm, make_config(w))
    assert ei.value.code == -2
    E = mesh.elements.copy()
    E[5, 1] = mesh.n_vertices + 3   # out of range
    dm = nl.DeviceMesh(torch.as_tensor(mesh.vertices, device="cuda"),
                       torch.as_tensor(E, device="cuda"), torch.as_tensor(mesh.labels, device="cuda"))
    with pytest.raises(nl.NlfemError) as ei:
        nl.nlfem_build_pairs(dm, make_config(w))
    assert ei.value.code == -2


def test_assemble_rejects_other_config():
    import paper_2207_03921_amd as nl
    from _gpu import make_config
    mesh = square_mesh(6, delta=0.2)
    w = _w("inv_dist", mesh, 0.2)
    dm = nl.DeviceMesh.from_numpy(mesh)
    pairs = nl.nlfem_build_pairs(dm, make_config(w))
    with pytest.raises(nl.NlfemError) as ei:
        nl.nlfem_assemble(dm, make_config(w, delta=0.25), pairs)
    assert ei.value.code == -6
    # c and precision may change
    nl.nlfem_assemble(dm, make_config(w, c=2.0, precision="mixed"), pairs)


def test_determinism_and_handle_reuse(oracle_lib):
    import torch
    import paper_2207_03921_amd as nl
    from _gpu import make_config
    w = inv_dist_jittered(n=24, delta=0.1, precision="fp64")
    mesh = w["mesh"]
    dm = nl.DeviceMesh.from_numpy(mesh)
    cfg = make_config(w)
    pairs = nl.nlfem_build_pairs(dm, cfg)
    v1 = nl.nlfem_assemble(dm, cfg, pairs).clone()
    v2 = nl.nlfem_assemble(dm, cfg, pairs).clone()
    torch.cuda.synchronize()
    d = (v1 - v2).abs().max().item() / v1.abs().max().item()
    assert d < 1e-14
    # rebuild the same handle for another horizon, compare with a fresh one
    cfg2 = make_config(w, delta=0.13)
    pairs = nl.nlfem_build_pairs(dm, cfg2, pairs=pairs)
    fresh = nl.nlfem_build_pairs(dm, cfg2)
    assert nl.nlfem_pairs_info(pairs) == nl.nlfem_pairs_info(fresh)
    r1, c1 = nl.nlfem_csr_pattern(pairs)
    r2, c2 = nl.nlfem_csr_pattern(fresh)
    assert torch.equal(r1, r2) and torch.equal(c1, c2)
    a1 = nl.nlfem_assemble(dm, cfg2, pairs)
    a2 = nl.nlfem_assemble(dm, cfg2, fresh)
    torch.cuda.synchronize()
    assert (a1 - a2).abs().max().item() <= 1e-14 * a2.abs().max().item()


# ---------------------------------------------------------------------------
# full-size workloads: complete pair lists, sampled rows, invariants

def _sample_rows(P, n_rows=48, seed=0):
    dof = np.flatnonzero(P.isdof())
    rng = np.random.default_rng(seed)
    pick = rng.choice(dof, size=min(n_rows, len(dof)), replace=False)
    # always include the first and last dof (boundary-adjacent rows)
    return np.unique(np.concatenate([pick, dof[:2], dof[-2:]]))


def _approxcaps_h128():
    """1/|z| kernel on the approximate-caps ball (Def. 2.4), h = 1/128,
    delta = 0.03 (about 37k triangles)."""
    return _w("inv_dist", square_mesh(128, delta=0.03, jitter=0.15, seed=30), 0.03, approach="approxcaps",
              precision="mixed")


def _inf_h96():
    """Constant kernel 3/(4 delta^4) on the infinity-norm ball, h = 1/96,
    delta = 0.05 (about 44k triangles)."""
    return _w("constant", square_mesh(96, delta=0.05, jitter=0.1, seed=23), 0.05, approach="inf",
              c=3.0 / (4.0 * 0.05 ** 4), precision="mixed")


@pytest.mark.parametrize("name", ["invdist_h64", "peri_h128", "poly32_h256", "inf_h96", "approxcaps_h128"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_full_size_sampled(oracle_lib, name, precision):
    w = {"invdist_h64": inv_dist_jittered, "peri_h128": peridynamic, "poly32_h256": constant_polygon,
         "inf_h96": _inf_h96, "approxcaps_h128": _approxcaps_h128}[name]()
    mesh = w["mesh"]
    print(f"full {name} {precision} K={mesh.n_elements}", flush=True)
    P = oracle_lib.Problem(mesh, w)
    g = gpu_run(mesh, w, precision=precision)
    rows = _sample_rows(P, n_rows=48)
    if precision == "fp64":
        gk, gl, gc = g["pairs"]
        if name in ("poly32_h256", "inf_h96", "approxcaps_h128"):
            # all pairs that meet the sampled rows' elements
            rowsel = np.zeros(mesh.n_vertices, bool)
            rowsel[rows] = True
            emask = rowsel[mesh.elements].any(axis=1)
            k, l, c = P.pairs(elem_mask=emask)
            keep = emask[gk] | emask[gl]
            gk, gl, gc = gk[keep], gl[keep], gc[keep]
        else:
            k, l, c = P.pairs()
        assert np.array_equal(gk, k) and np.array_equal(gl, l) and np.array_equal(gc, c)
    elif name in ("poly32_h256", "inf_h96", "approxcaps_h128"):
        # the mixed form decides inclusion in FP64 too: the same pairs meet the
        # sampled rows' elements
        gk, gl, gc = g["pairs"]
        rowsel = np.zeros(mesh.n_vertices, bool)
        rowsel[rows] = True
        emask = rowsel[mesh.elements].any(axis=1)
        k, l, c = P.pairs(elem_mask=emask)
        keep = emask[gk] | emask[gl]
        assert np.array_equal(gk[keep], k) and np.array_equal(gl[keep], l) and np.array_equal(gc[keep], c)
    rp, col, val = P.assemble_rows(rows)
    n = P.n
    G = to_sparse(g["row_ptr"], g["col"], g["val"], n * mesh.n_vertices)
    A = to_sparse(rp, col, val, n * mesh.n_vertices)
    sel = np.concatenate([n * rows + cc for cc in range(n)])
    Gs, As = G[sel], A[sel]
    assert np.array_equal(Gs.indptr, As.indptr) and np.array_equal(Gs.indices, As.indices)
    err = rel_frob(Gs, As)
    assert err <= TOL[precision], err
    ew = entrywise(Gs, As)
    assert ew <= TOL[precision], ew
    # invariants on the whole GPU matrix
    dofm = np.repeat(P.isdof(), n)
    B = G[dofm][:, dofm]
    asym = abs(B - B.T).max() / abs(B).max()
    assert asym <= (1e-14 if precision == "fp64" else 1e-6)
    ones = np.ones(n * mesh.n_vertices) if n == 1 else None
    if n == 1:
        r = G @ ones
        scale = abs(G) @ ones
        assert np.all(np.abs(r[dofm]) <= (1e-13 if precision == "fp64" else 1e-6) * scale[dofm])


_NONSYM = np.array([[1.0, 0.3], [2.5, 0.7]])
_SYM = np.array([[1.0, 0.4], [0.4, 2.0]])


def _mat(mesh, cut=0.45):
    """Material 1 for elements whose barycentre has x1 > cut, else 0."""
    import dataclasses
    bx = mesh.vertices[mesh.elements].mean(axis=1)[:, 0]
    return dataclasses.replace(mesh, materials=(bx > cut).astype(np.int32))


def _material_cases():
    """Label-dependent kernels C[m(x)][m(y)] Psi0: a symmetric table scales
    each pair's records; a non-symmetric one scales the columns of each
    element and takes the touching edge/vertex pairs through the 4D form."""
    return {
        "mat_const_bary_nonsym": dict(_w("constant", _mat(square_mesh(10, delta=0.2, jitter=0.2, seed=50)), 0.2),
                                      material_c=_NONSYM),
        "mat_invdist_sym": dict(_w("inv_dist", _mat(square_mesh(10, delta=0.2, jitter=0.2, seed=51)), 0.2),
                                material_c=_SYM),
        "mat_invdist_nonsym": dict(_w("inv_dist", _mat(square_mesh(10, delta=0.2, jitter=0.2, seed=52)), 0.2),
                                   material_c=_NONSYM),
        "mat_peri_nonsym": dict(_w("peridynamic", _mat(square_mesh(8, delta=0.3, jitter=0.1, seed=53)), 0.3),
                                material_c=_NONSYM),
        "mat_const_poly_nonsym": dict(_w("constant", _mat(square_mesh(10, delta=0.15, jitter=0.1, seed=54)), 0.15,
                                         approach="poly"), material_c=_NONSYM),
        "mat_frac_sym_approxcaps": dict(_w("frac_half", _mat(square_mesh(10, delta=0.2, jitter=0.1, seed=55)),
                                           0.2, approach="approxcaps", rule=paper7()), material_c=_SYM),
        "mat_invdist_nozerodiv_nonsym": dict(_w("inv_dist", _mat(square_mesh(10, delta=0.2, jitter=0.1, seed=56)),
                                                0.2, rule=paper7(), singular_n=0), material_c=_NONSYM),
        "mat_dg_invdist_nonsym": dict(_w("inv_dist", _mat(square_mesh(10, delta=0.2, jitter=0.2, seed=57)), 0.2,
                                         ansatz="dg"), material_c=_NONSYM),
        "mat_dg_peri_sym": dict(_w("peridynamic", _mat(square_mesh(8, delta=0.3, jitter=0.1, seed=58)), 0.3,
                                   ansatz="dg"), material_c=_SYM),
    }


@pytest.mark.parametrize("name", list(_material_cases()))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_materials(oracle_lib, name, precision):
    w = _material_cases()[name]
    print(f"case {name} {precision}", flush=True)
    _compare_full(oracle_lib, w, precision)


def test_material_table_validation():
    """Tables: 1..4 materials, finite, non-symmetric ones not with the s = 1/2
    kernel; the mesh needs materials with a table; ids outside the table are
    E_MESH at the build."""
    import torch
    import paper_2207_03921_amd as nl
    from _gpu import make_config
    mesh = _mat(square_mesh(6, delta=0.3))
    dm = nl.DeviceMesh.from_numpy(mesh)
    w = _w("inv_dist", mesh, 0.3)
    for table, msg in [(np.ones((5, 5)), "n_materials"), (np.array([[1.0, np.inf], [1.0, 1.0]]), "finite")]:
        with pytest.raises(nl.NlfemError) as e:
            nl.nlfem_build_pairs(dm, make_config(dict(w, material_c=table)))
        assert e.value.code == -1 and msg in str(e.value)
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_build_pairs(dm, make_config(dict(_w("frac_half", mesh, 0.3), material_c=_NONSYM)))
    assert e.value.code == -1 and "non-symmetric" in str(e.value)
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_build_pairs(nl.DeviceMesh(dm.vertices, dm.elements, dm.labels), make_config(dict(w, material_c=_SYM)))
    assert e.value.code == -1 and "materials" in str(e.value)
    bad = nl.DeviceMesh(dm.vertices, dm.elements, dm.labels, torch.full_like(dm.labels, 2))
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_build_pairs(bad, make_config(dict(w, material_c=_SYM)))
    assert e.value.code == -2 and "material" in str(e.value)
