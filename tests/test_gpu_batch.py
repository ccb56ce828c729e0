"""Batched assembly (persistent launches over a global work queue, HIP graph
replay, tuned launch shapes) against the single-problem path and the oracle
(MI355X only).

The batched kernels run the same per-item functions as the single-problem
kernels, so every value must be bit-identical to nlfem_assemble of the same
problem; the single-problem path is itself checked against the oracle in
test_gpu_parity.py, and two full-size batch members are sampled against the
oracle here as well.
"""
import os

import numpy as np
import pytest

from inputs import square_mesh, gauss7, paper7, collapsed
from inputs.workloads import batched, inv_dist_jittered, peridynamic, c_frac
from _gpu import make_config, to_sparse, rel_frob, entrywise

pytestmark = pytest.mark.gpu


def _w(kernel, mesh, delta, precision, rule=None, inner=None, singular_n=None, approach="bary"):
    rule = rule or gauss7()
    c = {"constant": c_frac(-1.0, delta), "inv_dist": c_frac(-0.5, delta)}.get(kernel, 6.0 / (np.pi * delta ** 3))
    if singular_n is None:
        singular_n = 0 if kernel == "constant" else 5
    return dict(mesh=mesh, kernel=kernel, c=c, delta=delta, approach=approach, polygon_n=32, outer=rule,
                inner=inner or rule, singular_n=singular_n, precision=precision)


def _mixed_set():
    """Problems of every specialisation: kernels, precisions, rules, ball."""
    return [
        _w("constant", square_mesh(12, delta=0.15, jitter=0.1, seed=1), 0.15, "fp64"),
        _w("inv_dist", square_mesh(14, delta=0.12, jitter=0.2, seed=2), 0.12, "mixed"),
        _w("inv_dist", square_mesh(10, delta=0.2, jitter=0.2, seed=3), 0.2, "fp64"),
        _w("peridynamic", square_mesh(10, delta=0.3, jitter=0.15, seed=4), 0.3, "mixed"),
        _w("constant", square_mesh(9, delta=0.2, jitter=0.1, seed=5), 0.2, "mixed", rule=paper7()),
        _w("constant", square_mesh(8, delta=0.25, jitter=0.1, seed=6), 0.25, "fp64", rule=gauss7(), inner=paper7()),
        _w("inv_dist", square_mesh(8, delta=0.2, jitter=0.15, seed=7), 0.2, "fp64", rule=collapsed(3)),
        _w("constant", square_mesh(10, delta=0.12), 0.12, "mixed", approach="poly"),
        _w("constant", square_mesh(16, delta=0.1, jitter=0.05, seed=8), 0.1, "mixed"),
        _w("peridynamic", square_mesh(8, delta=0.3, jitter=0.1, seed=9), 0.3, "fp64"),
        _w("constant", square_mesh(6, delta=0.4, neumann=True), 0.4, "fp64", singular_n=3),
    ]


def _build(ws):
    import torch
    import paper_2207_03921_amd as nl
    out = []
    for w in ws:
        dm = nl.DeviceMesh.from_numpy(w["mesh"])
        cfg = make_config(w)
        pairs = nl.nlfem_build_pairs(dm, cfg)
        nnz = nl.nlfem_pairs_info(pairs)["nnz"]
        single = nl.nlfem_assemble(dm, cfg, pairs)
        val = torch.full((max(nnz, 1),), float("nan"), dtype=torch.float64, device="cuda")
        out.append(dict(dm=dm, cfg=cfg, pairs=pairs, nnz=nnz, single=single, val=val))
    torch.cuda.synchronize()
    return out


def _assert_same(probs):
    import torch
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        n = p["nnz"]
        assert torch.equal(p["val"][:n], p["single"][:n]), f"problem {i} differs from its single assembly"


def test_batch_matches_single_assembly():
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set())
    print("batch of", len(probs), flush=True)
    b = nl.nlfem_batch_create([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
                              [p["val"] for p in probs])
    info = nl.nlfem_batch_info(b)
    assert info["groups"] >= 8
    nl.nlfem_batch_assemble(b)
    _assert_same(probs)
    # a second run overwrites with identical values
    for p in probs:
        p["val"].fill_(float("nan"))
    nl.nlfem_batch_assemble(b)
    _assert_same(probs)
    nl.nlfem_batch_free(b)


def test_batch_graph_replays():
    import torch
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set()[:6])
    b = nl.nlfem_batch_create([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
                              [p["val"] for p in probs])
    for rep in range(4):
        print("replay", rep, flush=True)
        for p in probs:
            p["val"].fill_(float("nan"))
        x = torch.randn(1 << 16, device="cuda")
        _ = (x * x).sum()   # eager work between replays
        torch.cuda.synchronize()
        nl.nlfem_batch_launch_graph(b)
        _assert_same(probs)
    nl.nlfem_batch_free(b)


def test_batch_tuning_and_cache(tmp_path):
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set()[:5])
    cache = str(tmp_path / "tune.txt")
    args = ([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
            [p["val"] for p in probs])
    b1 = nl.nlfem_batch_create(*args, tune_cache=cache, tune=1)
    _assert_same(probs)   # tuning runs the assembly
    s1 = nl.nlfem_batch_info(b1)["shape"]
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("gfx950")
    b2 = nl.nlfem_batch_create(*args, tune_cache=cache, tune=1)   # read back, no new line
    assert nl.nlfem_batch_info(b2)["shape"] == s1
    assert len(open(cache).read().splitlines()) == 1
    for p in probs:
        p["val"].fill_(float("nan"))
    nl.nlfem_batch_assemble(b2)
    _assert_same(probs)


def test_batch_per_problem_shapes(tmp_path):
    """Every phase as one launch per problem (shape {0, 0}, forced through
    the tune cache): the values are those of the single-problem path."""
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set()[:5])
    cache = str(tmp_path / "tune.txt")
    args = ([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
            [p["val"] for p in probs])
    nl.nlfem_batch_free(nl.nlfem_batch_create(*args, tune_cache=cache, tune=1))
    key = open(cache).read().splitlines()[0].rsplit(" ", 8)[0]   # the line without its 8 shape numbers
    open(cache, "w").write(key + " 0 0 0 0 0 0 0 0\n")
    b = nl.nlfem_batch_create(*args, tune_cache=cache, tune=1)
    shape = nl.nlfem_batch_info(b)["shape"]
    assert all(v == {"chunk": 0, "per_cu": 0} for v in shape.values()), shape
    for p in probs:
        p["val"].fill_(float("nan"))
    nl.nlfem_batch_assemble(b)
    _assert_same(probs)
    for p in probs:
        p["val"].fill_(float("nan"))
    nl.nlfem_batch_launch_graph(b)
    _assert_same(probs)
    nl.nlfem_batch_free(b)


def test_batch_rejects_bad_input():
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set()[:2])
    dms = [p["dm"] for p in probs]
    cfgs = [p["cfg"] for p in probs]
    vals = [p["val"] for p in probs]
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_batch_create(dms, cfgs, [probs[0]["pairs"], probs[0]["pairs"]], vals)
    assert e.value.code == -1 or e.value.code == -6
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_batch_create(dms, cfgs[::-1], [p["pairs"] for p in probs], vals)
    assert e.value.code == -6


def test_assemble_batched_one_shot():
    import paper_2207_03921_amd as nl
    probs = _build(_mixed_set()[:4])
    nl.nlfem_assemble_batched([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
                              [p["val"] for p in probs])
    _assert_same(probs)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_full_size_64_problems(oracle_lib, precision):
    """The 64-problem workload (h from 1/32 to 1/160, delta/h in 2..5, half
    constant, half 1/|z|): every problem bit-identical to its single
    assembly, eight problems (both kernels, small to large meshes) sampled
    against the oracle, row by row and entry by entry."""
    import torch
    import paper_2207_03921_amd as nl
    ws = batched(64, precision=precision)
    print("building 64 problems", precision, flush=True)
    probs = _build(ws)
    b = nl.nlfem_batch_create([p["dm"] for p in probs], [p["cfg"] for p in probs], [p["pairs"] for p in probs],
                              [p["val"] for p in probs], tune=0)
    nl.nlfem_batch_launch_graph(b)
    _assert_same(probs)
    for i in (1, 2, 13, 22, 35, 44, 57, 62):   # 1/|z| (odd) and constant-kernel (even) members
        w = ws[i]
        P = oracle_lib.Problem(w["mesh"], w)
        dof = np.flatnonzero(P.isdof())
        rows = np.unique(np.random.default_rng(i).choice(dof, 12, replace=False))
        rp, col, val = P.assemble_rows(rows)
        rpg, colg = nl.nlfem_csr_pattern(probs[i]["pairs"])
        nv = w["mesh"].n_vertices
        G = to_sparse(rpg.cpu().numpy(), colg.cpu().numpy(), probs[i]["val"][:probs[i]["nnz"]].cpu().numpy(), nv)
        A = to_sparse(rp, col, val, nv)
        Gs, As = G[rows], A[rows]
        assert np.array_equal(Gs.indptr, As.indptr) and np.array_equal(Gs.indices, As.indices)
        tol = 1e-12 if precision == "fp64" else 1e-5
        assert rel_frob(Gs, As) <= tol
        assert entrywise(Gs, As) <= tol
    nl.nlfem_batch_free(b)
