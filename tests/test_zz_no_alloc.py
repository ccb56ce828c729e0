"""The allocation-free batched assembly (MI355X only): same results as the
allocating one-shot batch, on two calls in a row (the second with a smaller
batch), with no allocation through the library's allocator hooks."""
import numpy as np
import pytest

from inputs.workloads import inv_dist_jittered, small_constant, peridynamic
from _gpu import make_config

pytestmark = pytest.mark.gpu


def _problems(nl, specs):
    import torch
    out = []
    for w in specs:
        cfg = make_config(w)
        dm = nl.DeviceMesh.from_numpy(w["mesh"])
        pairs = nl.nlfem_build_pairs(dm, cfg)
        nnz = nl.nlfem_pairs_info(pairs)["nnz"]
        out.append((dm, cfg, pairs, nnz))
    torch.cuda.synchronize()
    return out


def _run(nl, probs, fn):
    import torch
    vals = [torch.full((max(nnz, 1),), float("nan"), dtype=torch.float64, device="cuda")
            for _, _, _, nnz in probs]
    fn([p[0] for p in probs], [p[1] for p in probs], [p[2] for p in probs], vals)
    torch.cuda.synchronize()
    return [v[:nnz].cpu().numpy() for v, (_, _, _, nnz) in zip(vals, probs)]


def test_noalloc_batch_matches_allocating_batch():
    import paper_2207_03921_amd as nl
    big = _problems(nl, [inv_dist_jittered(n=24, delta=0.1, precision="fp64"),
                         small_constant(),
                         inv_dist_jittered(n=16, delta=0.15, precision="mixed"),
                         peridynamic(n=16, ratio=3, precision="fp64")])
    small = _problems(nl, [small_constant(), inv_dist_jittered(n=12, delta=0.2, precision="fp64")])
    calls = {"n": 0}
    alloc, free = nl.torch_allocator()

    def counting_alloc(n, s):
        calls["n"] += 1
        return alloc(n, s)

    try:
        for probs in (big, small):
            print("problems", len(probs), "nnz", [p[3] for p in probs], flush=True)
            ref = _run(nl, probs, nl.nlfem_assemble_batched)
            nl.nlfem_set_allocator(counting_alloc, free)
            got = _run(nl, probs, nl.nlfem_assemble_batched_noalloc)
            nl.nlfem_set_allocator()
            assert calls["n"] == 0
            for (_, cfg, _, _), a, b in zip(probs, got, ref):
                assert not np.isnan(a).any()
                tol = 1e-12 if cfg.precision == "fp64" else 1e-6
                assert np.abs(a - b).max() <= tol * np.abs(b).max()
    finally:
        nl.nlfem_set_allocator()
    for probs in (big, small):
        for _, _, pairs, _ in probs:
            nl.nlfem_pairs_free(pairs)


def test_noalloc_batch_rejects_unchecked_rebuild():
    import torch
    import paper_2207_03921_amd as nl
    (dm, cfg, pairs, nnz), = _problems(nl, [small_constant()])
    pairs = nl.nlfem_build_pairs(dm, cfg, pairs=pairs)   # same sizes: unchecked
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NlfemError) as e:
        nl.nlfem_assemble_batched_noalloc([dm], [cfg], [pairs], [val])
    assert e.value.code == -1 and "unchecked" in str(e.value)
    assert nl.nlfem_pairs_info(pairs)["rebuild"] == 1
    nl.nlfem_assemble_batched_noalloc([dm], [cfg], [pairs], [val])
    torch.cuda.synchronize()
    nl.nlfem_pairs_free(pairs)
