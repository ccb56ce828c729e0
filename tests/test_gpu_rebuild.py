"""Rebuilding a pairs handle in place (MI355X only).

A rebuild of a handle whose last build had the same sizes and configuration
runs with the last build's sizes without waiting; device-side checks gate its
kernels, and the next call on the handle checks its read-back and runs the
plain build when the counts differ.  Every rebuild must give what a fresh
handle gives: the same counts, pairs and CSR pattern, and values equal up to
the order of floating-point sums (fp64 here), whichever call finishes the
check.
"""
import numpy as np
import pytest

from inputs import square_mesh
from inputs.workloads import inv_dist_jittered, peridynamic, constant_polygon
from _gpu import make_config

pytestmark = pytest.mark.gpu


def _result(nl, dm, cfg, pairs):
    import torch
    info = dict(nl.nlfem_pairs_info(pairs))
    rb = info.pop("rebuild")
    skipped = info.pop("skipped")
    rp, col = nl.nlfem_csr_pattern(pairs)
    val = nl.nlfem_assemble(dm, cfg, pairs)
    k, l, c = nl.nlfem_pairs_export(pairs)
    torch.cuda.synchronize()
    _result.skipped = skipped
    return dict(info=info, rebuild=rb, skipped=skipped, rp=rp.cpu().numpy(), col=col.cpu().numpy(),
                val=val[:info["nnz"]].cpu().numpy(), pairs=(k.cpu().numpy(), l.cpu().numpy(), c.cpu().numpy()))


def _assert_same(a, b):
    assert a["info"] == b["info"]
    assert np.array_equal(a["rp"], b["rp"]) and np.array_equal(a["col"], b["col"])
    for x, y in zip(a["pairs"], b["pairs"]):
        assert np.array_equal(x, y)
    scale = max(np.abs(b["val"]).max(), 1e-300)
    assert np.abs(a["val"] - b["val"]).max() <= 1e-13 * scale


def _result_assemble_first(nl, dm, cfg, pairs, nnz_before, path):
    """The same, with the assembly as the first call after the rebuild.  The
    assembly never waits: when the rebuild kept its sizes it writes the
    result; when it found other sizes its kernels skip their work (val keeps
    its contents) and the next nlfem_pairs_info counts the skipped call."""
    import torch
    val = torch.full((max(nnz_before, 1),), float("nan"), dtype=torch.float64, device="cuda")
    nl.nlfem_assemble(dm, cfg, pairs, val=val)
    skipped_before = _result.skipped
    r = _result(nl, dm, cfg, pairs)
    torch.cuda.synchronize()
    got = val.cpu().numpy()
    if path == 1:
        assert r["info"]["nnz"] == nnz_before
        assert np.array_equal(got, r["val"]) or np.abs(got - r["val"]).max() <= 1e-13 * max(np.abs(r["val"]).max(), 1e-300)
        assert r["skipped"] == skipped_before
    else:
        assert np.isnan(got).all()
        assert r["skipped"] == skipped_before + 1
    return r


def _fresh(nl, mesh, cfg):
    dm = nl.DeviceMesh.from_numpy(mesh)
    return _result(nl, dm, cfg, nl.nlfem_build_pairs(dm, cfg))


def test_rebuild_same_and_changed_meshes():
    import torch
    import paper_2207_03921_amd as nl
    w = inv_dist_jittered(n=24, delta=0.1, precision="fp64")
    A = w["mesh"]
    cfg = make_config(w)
    # B: the same vertices with part of the domain relabelled 1 -> 2 (same
    # box and radii, other pair and dof counts)
    B = square_mesh(24, delta=0.1, jitter=0.2, seed=0)
    B.vertices[:] = A.vertices
    B.elements[:] = A.elements
    B.labels[:] = A.labels
    bx = A.vertices[A.elements].mean(axis=1)
    B.labels[(B.labels == 1) & (bx[:, 0] < 0.4)] = 2
    # C: another jitter of the same grid (same sizes, other geometry)
    C = square_mesh(24, delta=0.1, jitter=0.2, seed=7)
    assert C.elements.shape == A.elements.shape and C.vertices.shape == A.vertices.shape
    ref = {name: _fresh(nl, m, cfg) for name, m in (("A", A), ("B", B), ("C", C))}
    assert ref["A"]["info"] != ref["B"]["info"]

    dm = {name: nl.DeviceMesh.from_numpy(m) for name, m in (("A", A), ("B", B), ("C", C))}
    pairs = nl.nlfem_build_pairs(dm["A"], cfg)
    r = _result(nl, dm["A"], cfg, pairs)
    assert r["rebuild"] == 0
    # (mesh, expected path): 1 = held with the last sizes, 2 = fell back
    for name, path in (("A", 1), ("A", 1), ("B", 2), ("B", 1), ("C", 2), ("A", 2), ("A", 1)):
        print("rebuild with", name, flush=True)
        pairs = nl.nlfem_build_pairs(dm[name], cfg, pairs=pairs)
        r = _result(nl, dm[name], cfg, pairs)
        assert r["rebuild"] == path, (name, r["rebuild"])
        _assert_same(r, ref[name])
    # the same sequence with the assembly as the first call after each rebuild
    for name, path in (("B", 2), ("B", 1), ("A", 2), ("A", 1)):
        print("rebuild with", name, "assembly first", flush=True)
        nnz_before = r["info"]["nnz"]
        pairs = nl.nlfem_build_pairs(dm[name], cfg, pairs=pairs)
        r = _result_assemble_first(nl, dm[name], cfg, pairs, nnz_before, path)
        assert r["rebuild"] == path, (name, r["rebuild"])
        _assert_same(r, ref[name])
    # an unchecked rebuild that found other sizes, replaced by a newer build
    # before any call checked it: its assembly skipped, the newer build plain
    skipped = r["skipped"]
    pairs = nl.nlfem_build_pairs(dm["B"], cfg, pairs=pairs)
    val = torch.full((max(r["info"]["nnz"], 1),), float("nan"), dtype=torch.float64, device="cuda")
    nl.nlfem_assemble(dm["B"], cfg, pairs, val=val)
    pairs = nl.nlfem_build_pairs(dm["B"], cfg, pairs=pairs)
    r = _result(nl, dm["B"], cfg, pairs)
    assert r["rebuild"] == 0 and r["skipped"] == skipped + 1
    assert torch.isnan(val).all().item()
    _assert_same(r, ref["B"])
    # a new device copy of the same mesh (other pointers, same values)
    dA2 = nl.DeviceMesh.from_numpy(A)
    pairs = nl.nlfem_build_pairs(dA2, cfg, pairs=pairs)   # B's sizes: falls back
    assert nl.nlfem_pairs_info(pairs)["rebuild"] == 2
    pairs = nl.nlfem_build_pairs(dA2, cfg, pairs=pairs)
    r = _result(nl, dA2, cfg, pairs)
    assert r["rebuild"] == 1
    _assert_same(r, ref["A"])
    nl.nlfem_pairs_free(pairs)


def test_batch_sees_rebuilds():
    """A batch stays valid across rebuilds that keep the sizes and reports a
    plain rebuild of one of its handles."""
    import torch
    import paper_2207_03921_amd as nl
    w = inv_dist_jittered(n=16, delta=0.12, precision="fp64")
    cfg = make_config(w)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, cfg)
    single = nl.nlfem_assemble(dm, cfg, pairs).clone()
    nnz = nl.nlfem_pairs_info(pairs)["nnz"]
    val = torch.full((nnz,), float("nan"), dtype=torch.float64, device="cuda")
    b = nl.nlfem_batch_create([dm], [cfg], [pairs], [val], tune=0)
    pairs = nl.nlfem_build_pairs(dm, cfg, pairs=pairs)   # same sizes: no wait
    nl.nlfem_batch_assemble(b)
    torch.cuda.synchronize()
    assert nl.nlfem_pairs_info(pairs)["rebuild"] == 1
    scale = single.abs().max().item()
    assert (val - single[:nnz]).abs().max().item() <= 1e-13 * scale
    pairs = nl.nlfem_build_pairs(dm, make_config(w, delta=0.13), pairs=pairs)   # plain
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_batch_assemble(b)
    assert e.value.code == -6
    nl.nlfem_batch_free(b)
    nl.nlfem_pairs_free(pairs)


def test_rebuild_after_config_change_is_plain():
    import paper_2207_03921_amd as nl
    w = inv_dist_jittered(n=16, delta=0.12, precision="fp64")
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, make_config(w))
    pairs = nl.nlfem_build_pairs(dm, make_config(w, delta=0.15), pairs=pairs)
    assert nl.nlfem_pairs_info(pairs)["rebuild"] == 0
    pairs = nl.nlfem_build_pairs(dm, make_config(w, delta=0.15), pairs=pairs)
    assert nl.nlfem_pairs_info(pairs)["rebuild"] == 1
    nl.nlfem_pairs_free(pairs)


@pytest.mark.parametrize("kind", ["peridynamic", "polygon"])
def test_rebuild_vector_and_polygon(kind):
    import paper_2207_03921_amd as nl
    if kind == "peridynamic":
        w = peridynamic(n=16, ratio=3, precision="fp64")
    else:
        w = constant_polygon(n=24, delta=0.08, precision="fp64")
    cfg = make_config(w)
    ref = _fresh(nl, w["mesh"], cfg)
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, cfg)
    for it in range(3):
        print(kind, "rebuild", it, flush=True)
        pairs = nl.nlfem_build_pairs(dm, cfg, pairs=pairs)
        r = _result(nl, dm, cfg, pairs)
        assert r["rebuild"] == 1
        _assert_same(r, ref)
    nl.nlfem_pairs_free(pairs)


def test_scans_by_direct_sums(monkeypatch):
    """The prefix sums of a build take, past a bounded wait for the tiles
    before them, the direct sum of the inputs before their tile.  Forcing that
    path everywhere (NLFEM_SCAN_SPIN=-1, read at every launch) must give the
    same build as the chained look-back, plainly built and rebuilt."""
    import paper_2207_03921_amd as nl
    w = inv_dist_jittered(n=48, delta=0.05, precision="fp64")
    cfg = make_config(w)
    assert w["mesh"].elements.shape[0] > 4 * 1024   # several tiles per scan
    ref = _fresh(nl, w["mesh"], cfg)
    monkeypatch.setenv("NLFEM_SCAN_SPIN", "-1")
    dm = nl.DeviceMesh.from_numpy(w["mesh"])
    pairs = nl.nlfem_build_pairs(dm, cfg)
    for path in (0, 1):
        r = _result(nl, dm, cfg, pairs)
        assert r["rebuild"] == path
        _assert_same(r, ref)
        pairs = nl.nlfem_build_pairs(dm, cfg, pairs=pairs)
    nl.nlfem_pairs_free(pairs)
