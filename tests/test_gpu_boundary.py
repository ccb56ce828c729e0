"""The boundary's failure paths and hooks on the device (MI355X only):
allocator hooks (torch's caching allocator, a failing allocator), the
capacity limit, a non-conforming mesh, and the load vector from values at the
quadrature points."""
import numpy as np
import pytest

from inputs.workloads import inv_dist_jittered, small_constant
from _gpu import make_config, gpu_run, to_sparse

pytestmark = pytest.mark.gpu


@pytest.fixture
def nl():
    import paper_2207_03921_amd as nl
    yield nl
    nl.nlfem_set_allocator()   # every test leaves the default allocator
    nl.nlfem_set_capacity(0)


def _assemble(nl, w, cfg=None):
    import torch
    cfg = cfg or make_config(w)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, cfg)
    info = nl.nlfem_pairs_info(pairs)
    rp, col = nl.nlfem_csr_pattern(pairs)
    val = nl.nlfem_assemble(dm, cfg, pairs)
    torch.cuda.synchronize()
    return pairs, info, rp.cpu().numpy(), col.cpu().numpy(), val[:info["nnz"]].cpu().numpy()


def _same_values(a, b):
    # the row gather sums in LDS in arrival order: equal up to rounding
    return np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_torch_allocator_hook(nl):
    """Every handle and batch buffer comes from the hook and goes back to it;
    the results equal those of hipMalloc'd buffers."""
    import torch
    w = inv_dist_jittered(n=16, delta=0.15, precision="fp64")
    ref = _assemble(nl, w)
    nl.nlfem_pairs_free(ref[0])
    alloc, free = nl.torch_allocator()
    live = {}
    calls = {"alloc": 0, "free": 0}

    def a(n, s):
        p = alloc(n, s)
        calls["alloc"] += 1
        live[p] = n
        return p

    def f(p, s):
        calls["free"] += 1
        assert live.pop(p, None) is not None
        free(p, s)

    nl.nlfem_set_allocator(a, f)
    pairs, info, rp, col, val = _assemble(nl, w)
    held = [pairs]   # freed below even when an assertion fails
    try:
        _check_hooked(nl, w, ref, calls, live, info, rp, col, val, held)
    finally:
        for p in held:
            nl.nlfem_pairs_free(p)
    assert not live and calls["free"] == calls["alloc"]


def _check_hooked(nl, w, ref, calls, live, info, rp, col, val, held):
    import torch
    assert calls["alloc"] > 10 and live
    assert info == ref[1]
    assert np.array_equal(rp, ref[2]) and np.array_equal(col, ref[3])
    assert _same_values(val, ref[4])
    # a batch's tables come from the hook too
    cfg = make_config(w)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs2 = nl.nlfem_build_pairs(dm, cfg)
    held.append(pairs2)
    out = torch.zeros(info["nnz"], dtype=torch.float64, device="cuda")
    n_before = calls["alloc"]
    b = nl.nlfem_batch_create([dm], [cfg], [pairs2], [out], tune=0)
    assert calls["alloc"] == n_before + 1
    nl.nlfem_batch_assemble(b)
    torch.cuda.synchronize()
    assert _same_values(out.cpu().numpy(), ref[4])
    nl.nlfem_batch_free(b)


def test_failing_allocator(nl):
    """An allocator that fails after some blocks makes the build return
    E_NOMEM (no handle is returned, nothing leaks); with the default restored
    the same build succeeds."""
    import torch
    w = small_constant()
    alloc, free = nl.torch_allocator()
    for budget in (0, 5, 20):
        live = {}

        def a(n, s, left=[budget]):
            if left[0] <= 0:
                return 0
            left[0] -= 1
            p = alloc(n, s)
            live[p] = n
            return p

        def f(p, s):
            live.pop(p)
            free(p, s)

        nl.nlfem_set_allocator(a, f)
        dm = nl.DeviceMesh.from_numpy(w["mesh"])
        with pytest.raises(nl.NlfemError) as e:
            nl.nlfem_build_pairs(dm, make_config(w))
        assert e.value.code == -3, str(e.value)
        assert "allocator" in str(e.value)
        torch.cuda.synchronize()
        assert not live, f"{len(live)} blocks leaked after a failed build"
    nl.nlfem_set_allocator()
    pairs, info, *_ = _assemble(nl, w)
    assert info["n_pairs"] == 12906
    nl.nlfem_pairs_free(pairs)


def test_capacity_limit(nl):
    w = small_constant()
    pairs, info, *_ = _assemble(nl, w)
    nl.nlfem_pairs_free(pairs)
    nl.nlfem_set_capacity(info["n_nbr"] - 1)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_build_pairs(dm, make_config(w))
    assert e.value.code == -5 and "capacity" in str(e.value)
    nl.nlfem_set_capacity(info["n_nbr"])
    pairs = nl.nlfem_build_pairs(dm, make_config(w))
    assert nl.nlfem_pairs_info(pairs)["n_nbr"] == info["n_nbr"]
    nl.nlfem_pairs_free(pairs)


@pytest.mark.parametrize("label", [1, 2, 0])
def test_non_conforming_mesh(nl, label):
    """A third labelled element on an existing edge is E_MESH (Sec. 2.2,
    Assumption 2); with a label outside {1, 2} the element is ignored."""
    import copy
    w = small_constant()
    mesh = copy.deepcopy(w["mesh"])
    # the diagonal (v00, v11) of the first cell, shared by its two elements
    a, b = mesh.elements[0, 0], mesh.elements[0, 2]
    assert b in mesh.elements[1]
    pa, pb = mesh.vertices[a], mesh.vertices[b]
    # a new vertex mirrored across the edge (a, b) from the element's third one
    c = mesh.vertices[mesh.elements[0, 1]]
    mid = 0.5 * (pa + pb)
    d = pb - pa
    t = np.dot(c - pa, d) / np.dot(d, d)
    foot = pa + t * d
    new_v = foot - 0.5 * (c - foot) + 0.1 * (mid - foot)
    mesh.vertices = np.vstack([mesh.vertices, new_v])
    mesh.elements = np.vstack([mesh.elements, [[a, b, mesh.vertices.shape[0] - 1]]]).astype(np.int32)
    mesh.labels = np.append(mesh.labels, label).astype(np.int32)
    dm = nl.DeviceMesh.from_numpy(mesh)
    cfg = make_config(w)
    if label in (1, 2):
        with pytest.raises(nl.NlfemError) as e:
            nl.nlfem_build_pairs(dm, cfg)
        assert e.value.code == -2 and "edge" in str(e.value)
    else:
        pairs = nl.nlfem_build_pairs(dm, cfg)
        assert nl.nlfem_pairs_info(pairs)["n_pairs"] == 12906
        nl.nlfem_pairs_free(pairs)


@pytest.mark.parametrize("kind", ["scalar", "peridynamic"])
def test_rhs_from_quadrature_point_values(nl, oracle_lib, kind):
    """b from values at the outer quadrature points: f sampled from an affine
    function gives the affine result, and an arbitrary (seeded) table gives
    the oracle's result for the same table."""
    import torch
    from inputs.workloads import peridynamic
    w = inv_dist_jittered(n=16, delta=0.15, precision="fp64") if kind == "scalar" else \
        peridynamic(n=16, ratio=3, precision="fp64")
    mesh = w["mesh"]
    n = w["ncomp"]
    aff = np.array(w["f_affine"] if w.get("f_affine") is not None else [(-4.0, 0.7, -1.3)], np.float64)
    xi = w["outer"].xi
    V, E = mesh.vertices, mesh.elements
    v0 = V[E[:, 0]]
    J = np.stack([V[E[:, 1]] - v0, V[E[:, 2]] - v0], axis=2)   # [K, 2, 2]
    X = v0[:, None, :] + np.einsum("kij,pj->kpi", J, xi)           # [K, P, 2]
    fq = np.stack([aff[c, 0] + aff[c, 1] * X[..., 0] + aff[c, 2] * X[..., 1] for c in range(n)], axis=-1)
    cfg = make_config(w)
    dm = nl.DeviceMesh.from_numpy(mesh)
    b_aff = nl.nlfem_rhs(dm, cfg, f_affine=aff)
    b_qp = nl.nlfem_rhs(dm, cfg, f_qp=torch.as_tensor(np.ascontiguousarray(fq), device="cuda"))
    rng = np.random.default_rng(3)
    fr = rng.standard_normal(fq.shape)
    b_rand = nl.nlfem_rhs(dm, cfg, f_qp=torch.as_tensor(fr, device="cuda"))
    torch.cuda.synchronize()
    scale = np.abs(b_aff.cpu().numpy()).max()
    assert np.abs(b_qp.cpu().numpy() - b_aff.cpu().numpy()).max() <= 1e-14 * scale
    P = oracle_lib.Problem(mesh, w)
    ob = P.rhs(f_qp=fr)
    assert np.abs(b_rand.cpu().numpy() - ob).max() <= 1e-14 * np.abs(ob).max()


@pytest.mark.parametrize("kind", ["dg", "no_zero_division"])
def test_batch_rejects_single_problem_only_configs(nl, kind):
    """Batches take continuous problems whose singular kernels use the
    transforms; a discontinuous problem, or a weakly singular kernel with
    the standard rule on touching pairs (singular_n = 0), is refused with
    E_INVALID before anything runs (the single-problem path assembles it)."""
    import torch
    from inputs import square_mesh
    w = inv_dist_jittered(n=8, delta=0.25, precision="fp64")
    w = dict(w, mesh=square_mesh(8, delta=0.25))
    if kind == "dg":
        w["ansatz"] = "dg"
    else:
        w["singular_n"] = 0
    cfg = make_config(w)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, cfg)
    nnz = nl.nlfem_pairs_info(pairs)["nnz"]
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_batch_create([dm], [cfg], [pairs], [val])
    assert e.value.code == -1
    assert ("continuous" in str(e.value)) if kind == "dg" else ("singular_n" in str(e.value))
    nl.nlfem_assemble(dm, cfg, pairs, val)
    torch.cuda.synchronize()
    assert torch.isfinite(val).all() and float(val.abs().max()) > 0.0
    nl.nlfem_pairs_free(pairs)


def test_batch_material_tables(nl):
    """A symmetric material table runs in batches, bit-identical to the
    single-problem assembly; a non-symmetric one is refused there."""
    import dataclasses
    import torch
    from inputs import square_mesh
    mesh = square_mesh(10, delta=0.2, jitter=0.1, seed=60)
    bx = mesh.vertices[mesh.elements].mean(axis=1)[:, 0]
    mesh = dataclasses.replace(mesh, materials=(bx > 0.5).astype(np.int32))
    w = dict(inv_dist_jittered(n=10, delta=0.2, precision="fp64"), mesh=mesh,
             material_c=np.array([[1.0, 0.4], [0.4, 2.0]]))
    cfg = make_config(w)
    dm = nl.DeviceMesh.from_numpy(mesh)
    pairs = nl.nlfem_build_pairs(dm, cfg)
    ref = nl.nlfem_assemble(dm, cfg, pairs)
    nnz = nl.nlfem_pairs_info(pairs)["nnz"]
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    b = nl.nlfem_batch_create([dm], [cfg], [pairs], [val])
    nl.nlfem_batch_assemble(b)
    torch.cuda.synchronize()
    assert _same_values(val.cpu().numpy(), ref[:nnz].cpu().numpy())
    del b
    bad = make_config(dict(w, material_c=np.array([[1.0, 0.3], [2.5, 0.7]])))
    pairs2 = nl.nlfem_build_pairs(dm, bad)
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_batch_create([dm], [bad], [pairs2], [torch.zeros(nl.nlfem_pairs_info(pairs2)["nnz"],
                                                                    dtype=torch.float64, device="cuda")])
    assert e.value.code == -1 and "symmetric" in str(e.value)
    nl.nlfem_pairs_free(pairs)
    nl.nlfem_pairs_free(pairs2)
