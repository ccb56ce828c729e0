"""Benchmark: nonlocal P1 stiffness assembly on one MI355X.

Default workload: the 64-problem batch (h from 1/32 to 1/160, delta/h in
{2,3,4,5}, half the constant kernel, half 1/|z| with the regularising
transforms on touching pairs; 1.6 M triangles, 1.5e8 interacting pairs) in
the plain FP64 form.  One step = the whole hot path over the batch: the 64
pair structures rebuilt in place (geometry, pair search, lists, CSR pattern:
nlfem_build_pairs on each handle), the batched assembly of all 64 matrices
(nlfem_batch_assemble: persistent launches over the global work queue) and
the 64 load vectors (nlfem_rhs).  Inputs are resident in HBM before the timed
region.  value = ordered interacting pairs of the batch x steps / wall time
of the timed steps.

Also reported: the mixed FP32/FP64 batch, the batch replayed from a HIP
graph, the 64 problems assembled one after the other, the error of each form
against the oracle on a sample of problems, the oracle's throughput on the
same sample, and the roofline of the step's dominant kernel (algorithmic
work per the per-unit model below / its HIP-event time in the timed steps).

`--workload` selects one of the single-problem workloads instead.  Prints
ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = ("batched64", "invdist_h64", "const_h16", "peri_h128", "poly32_h256")
METRIC = "element-pair interactions assembled/sec"

# ---------------------------------------------------------------- work model
#
# Algorithmic work per unit (FMA = 2 flops, a reciprocal square root 1):
#  - far (non-touching) ordered pair with P x Q point pairs: per point pair
#    the kernel value (constant 2, 1/|z| 8, peridynamic 20 flops) and the
#    contraction Phi^T diag(w gamma) Phi (672 flops per 49 point pairs and
#    kernel component; 1, 1, 3 components): 770 / 1,064 / 3,000 flops for
#    the 7 x 7 rule;
#  - touching ordered pair: 45 flops per point of the reduced transform
#    rules (identical 6n, edge 4n^2, vertex 2n^3 points; n = 5: 30, 100,
#    250 points), 2.5 times that for peridynamics;
#  - bytes of an assembly: 9 per ordered pair (pair list entry), 8 per
#    stored matrix entry (written once), 200 per element (geometry).
# Peaks of MI355X: HBM 8 TB/s; vector FP64 78.6 TFLOP/s and FP32
# 157.3 TFLOP/s (256 CUs x 2.4 GHz x 128 and 256 flops per clock).
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
_KERNEL_FLOPS = {"constant": (2.0, 1), "inv_dist": (8.0, 1), "peridynamic": (20.0, 3)}


def far_pair_flops(kernel, p, q):
    kv, nk = _KERNEL_FLOPS[kernel]
    return p * q * (kv + nk * 672.0 / 49.0)


def touch_pair_flops(kernel, n):
    per_point = 45.0 * (2.5 if kernel == "peridynamic" else 1.0)
    return {"ident": 6 * n * per_point, "edge": 4 * n * n * per_point, "vertex": 2 * n ** 3 * per_point}


def work_of(info, w):
    """(far flops, touching flops, assembly bytes) of one problem."""
    p, q = len(w["outer"].w), len(w["inner"].w)
    far = info["n_far"] * far_pair_flops(w["kernel"], p, q)
    touch = 0.0
    n = int(w.get("singular_n", 0))
    if n > 0:
        t = touch_pair_flops(w["kernel"], n)
        touch = info["n_ident"] * t["ident"] + info["n_edge"] * t["edge"] + info["n_vertex"] * t["vertex"]
    nbytes = info["n_pairs"] * 9 + info["nnz"] * 8 + w["mesh"].n_elements * 200
    return far, touch, nbytes


def roofline_of(phase, ms, far, touch, nbytes, precision, kernels):
    """Roofline entry of the dominant phase: flops against the vector peak of
    its precision for the quadrature phases, bytes against HBM otherwise."""
    if phase == "far":
        fp32 = precision == "mixed"
        peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
        ach = far / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": None, "kernel": kernels, "phase": "far", "dtype": "f32" if fp32 else "f64",
                "algorithmic_flops": far, "launch_ms": ms}
    if phase == "touch":
        ach = touch / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_PEAK_TFLOPS, "traffic": None, "kernel": kernels, "phase": "touch",
                "dtype": "f64", "algorithmic_flops": touch, "launch_ms": ms}
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernels, "phase": phase, "algorithmic_bytes": nbytes, "launch_ms": ms}


PHASE_KERNELS = {
    "batched": {"far": "kb_far (one launch per kernel specialisation)", "touch": "kb_touch (one launch per class)",
                "diag": "kb_diag", "rows": "kb_rows", "geometry": "k_geometry, k_bucket_count/fill, scans",
                "pairs": "k_pairs", "lists": "k_sort_lists", "csr": "k_csr_rows, k_csr_pack", "rhs": "k_rhs"},
    "single": {"far": "k_far_rec", "touch": "k_touch_rec", "diag": "k_elem_diag", "rows": "k_rows",
               "geometry": "k_geometry, k_bucket_count/fill, scans", "pairs": "k_pairs", "lists": "k_sort_lists",
               "csr": "k_csr_rows, k_csr_pack", "rhs": "k_rhs"},
}


def source_digest():
    """Digest of the library's kernel sources: a committed counter summary
    holds the digest of the sources it was taken on."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2207_03921_amd", "csrc")
    for fn in sorted(os.listdir(src)):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(src, fn), "rb") as fh:
                h.update(fn.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, phase):
    """HBM bytes per step of the dominant phase's kernels from the committed
    counter summary, or None when it is missing or the sources changed."""
    path = os.path.join(ROOT, "profiles", f"traffic_{phase}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------- helpers

def _config(w, precision):
    import paper_2207_03921_amd as nl
    from inputs.rules import polygon_dirs
    return nl.Config(kernel=w["kernel"], c=float(w["c"]), delta=float(w["delta"]),
                     outer_xi=w["outer"].xi, outer_w=w["outer"].w, inner_xi=w["inner"].xi,
                     inner_w=w["inner"].w, approach=w.get("approach", "bary"),
                     polygon_dirs=polygon_dirs(32) if w.get("approach") == "poly" else None,
                     singular_n=int(w.get("singular_n", 0)), precision=precision)


def _f_affine(w):
    if w.get("f_affine") is not None:
        return w["f_affine"]
    return [(float(v), 0.0, 0.0) for v in w["f"]]


def _sparse(rp, col, val, n):
    import scipy.sparse as sp
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def _errors(G, A):
    """(relative Frobenius error, largest entry error relative to its row's
    largest entry)."""
    D = (G - A).tocsr()
    fro = float(np.sqrt(D.multiply(D).sum() / A.multiply(A).sum()))
    dmax = np.asarray(abs(D).max(axis=1).todense()).ravel()
    amax = np.asarray(abs(A).max(axis=1).todense()).ravel()
    ok = amax > 0
    return fro, float((dmax[ok] / amax[ok]).max()) if ok.any() else 0.0


def _timing_mask_all():
    import paper_2207_03921_amd as nl
    nl.nlfem_timing_enable(True)
    nl.nlfem_timing_read(reset=True)


def _phases_per_step(steps):
    import paper_2207_03921_amd as nl
    ph = nl.nlfem_timing_read(reset=True)
    nl.nlfem_timing_enable(False)
    return {k: v[0] / steps for k, v in ph.items()}


def cpu_sample(ws, idx, pairs_of, f_affine_of):
    """The oracle as it stands (brute-force pair search, assembly, load
    vector) on the sample problems, one run each: pairs/s and the matrices
    (for the error of each GPU form)."""
    import oracle
    oracle.build(force=False)
    total_pairs, total_t, mats = 0, 0.0, {}
    for i in idx:
        w = ws[i]
        P = oracle.Problem(w["mesh"], w)
        t0 = time.perf_counter()
        k, l, c = P.pairs()
        rp, col, val = P.assemble((k, l, c))
        P.rhs(f_affine=f_affine_of(w))
        total_t += time.perf_counter() - t0
        total_pairs += len(k)
        mats[i] = _sparse(rp, col, val, P.n * w["mesh"].n_vertices)
    return total_pairs / total_t, total_t, total_pairs, oracle.num_threads(), mats


# ---------------------------------------------------------------- batched

def bench_batched(args):
    import torch
    import paper_2207_03921_amd as nl
    from inputs import workloads as W
    torch.cuda.set_device(0)
    prec = args.precision
    ws = W.batched(64, precision=prec)
    dms = [nl.DeviceMesh.from_numpy(w["mesh"]) for w in ws]
    cfgs = [_config(w, prec) for w in ws]
    cfg64 = [_config(w, "fp64") for w in ws]
    cfgmx = [_config(w, "mixed") for w in ws]
    affs = [_f_affine(w) for w in ws]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = [nl.nlfem_build_pairs(d, c) for d, c in zip(dms, cfgs)]
    torch.cuda.synchronize()
    t_plain_build = time.perf_counter() - t0
    infos = [nl.nlfem_pairs_info(p) for p in pairs]
    n_pairs = sum(i["n_pairs"] for i in infos)
    vals = [torch.empty(max(i["nnz"], 1), dtype=torch.float64, device="cuda") for i in infos]
    bs = [torch.empty(c.ncomp * d.vertices.shape[0], dtype=torch.float64, device="cuda") for c, d in zip(cfgs, dms)]
    cache = os.path.join(ROOT, "paper_2207_03921_amd", "tune_cache.txt")
    batch = nl.nlfem_batch_create(dms, cfgs, pairs, vals, tune_cache=cache, tune=1)
    # The handles are independent: their rebuilds (and load vectors) run on
    # several streams at once, the largest problems spread first over the
    # least loaded stream; events order them against the batched assembly
    # on the default stream (a rebuild rewrites what the last assembly read).
    n_str = max(1, args.build_streams)
    streams = [torch.cuda.Stream() for _ in range(n_str)]
    load = [0] * n_str
    lane = [0] * len(ws)
    for i in sorted(range(len(ws)), key=lambda i: -infos[i]["n_pairs"]):
        s = min(range(n_str), key=load.__getitem__)
        lane[i] = s
        load[s] += infos[i]["n_pairs"]
    main_stream = torch.cuda.current_stream()

    def fan_out(work, spread=True):
        if not spread:   # everything on the default stream
            for i in range(len(ws)):
                work(i, main_stream)
            return
        ev = torch.cuda.Event()
        ev.record(main_stream)
        for s in streams:
            s.wait_event(ev)
        for i in range(len(ws)):
            work(i, streams[lane[i]])
        for s in streams:
            e = torch.cuda.Event()
            e.record(s)
            main_stream.wait_event(e)

    def rebuilds(spread=True):
        fan_out(lambda i, s: nl.nlfem_build_pairs(dms[i], cfgs[i], pairs=pairs[i], stream=s), spread)

    def step(spread=True):
        rebuilds(spread)
        nl.nlfem_batch_assemble(batch)
        fan_out(lambda i, s: nl.nlfem_rhs(dms[i], cfgs[i], f_affine=affs[i], b=bs[i], stream=s), spread)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # one untimed step with every phase timed, on one stream so that the
    # phase times are those of the kernels alone: the dominant phase
    _timing_mask_all()
    step(spread=False)
    torch.cuda.synchronize()
    phase_ms = _phases_per_step(1)
    dominant = max(phase_ms, key=phase_ms.get)
    # the timed steps, with HIP events around the dominant phase's launches
    # on the streams they run on
    nl.nlfem_timing_enable([dominant])
    nl.nlfem_timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    dom_ms = _phases_per_step(args.steps)[dominant]
    assert all(nl.nlfem_pairs_info(p)["rebuild"] == 1 for p in pairs), "a rebuild changed sizes"

    def timed(fn, steps, warmup=1):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    reps = max(3, args.steps // 2)
    # parts of the step
    t_build = timed(rebuilds, reps)
    for p in pairs:
        nl.nlfem_pairs_info(p)   # finishes the rebuilds' checks
    t_asm = timed(lambda: nl.nlfem_batch_assemble(batch), reps)
    t_graph = timed(lambda: nl.nlfem_batch_launch_graph(batch), reps)
    ref_vals = [v[:i["nnz"]].clone() for v, i in zip(vals, infos)]   # this form's result
    # the other precision form and the sequential plain FP64 assemblies
    vals_mx = [torch.empty_like(v) for v in vals]
    bmx = nl.nlfem_batch_create(dms, cfgmx, pairs, vals_mx, tune_cache=cache, tune=1)
    t_mixed = timed(lambda: nl.nlfem_batch_launch_graph(bmx), reps)
    vals_seq = [torch.empty_like(v) for v in vals]

    def sequential():
        for d, c, p, v in zip(dms, cfg64, pairs, vals_seq):
            nl.nlfem_assemble(d, c, p, val=v)

    t_seq = timed(sequential, reps)
    torch.cuda.synchronize()

    # accuracy of every form against the oracle, and the oracle's speed, on
    # the twenty smallest problems (both kernels; delta/h 2..5)
    order = sorted(range(len(ws)), key=lambda i: ws[i]["mesh"].n_elements)
    sample = sorted(order[:20])
    accuracy = None
    cpu = None
    if not args.no_cpu_baseline:
        rate, t_cpu, sp_pairs, threads, mats = cpu_sample(ws, sample, None, _f_affine)
        cpu = {"value": rate, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"problems {sample} of the batch (the twenty smallest, {sp_pairs} ordered pairs): "
                         f"brute-force pair search, assembly and load vector, one run each, {t_cpu:.1f} s"}
        accuracy = {}
        forms = [(f"{prec}_batched", ref_vals)] + ([("mixed_batched", vals_mx)] if prec == "fp64" else []) + \
            [("fp64_sequential", vals_seq)]
        for name, vv in forms:
            worst = [0.0, 0.0]
            for i in sample:
                rp, col = nl.nlfem_csr_pattern(pairs[i])
                nnz = infos[i]["nnz"]
                G = _sparse(rp.cpu().numpy(), col.cpu().numpy(), vv[i][:nnz].cpu().numpy(), mats[i].shape[0])
                fro, ent = _errors(G, mats[i])
                worst = [max(worst[0], fro), max(worst[1], ent)]
            accuracy[name] = {"rel_frobenius": worst[0], "max_entry_rel_row": worst[1]}

    far = touch = nbytes = 0.0
    for i, w in zip(infos, ws):
        f, t, b = work_of(i, w)
        far, touch, nbytes = far + f, touch + t, nbytes + b
    # a phase the tuner runs as one launch per problem uses the single-problem kernels
    shape = nl.nlfem_batch_info(batch)["shape"]
    kname = PHASE_KERNELS["batched"][dominant]
    if dominant in shape and shape[dominant]["chunk"] == 0:
        kname = PHASE_KERNELS["single"][dominant] + " (one launch per problem)"
    roof = roofline_of(dominant, dom_ms, far, touch, nbytes, prec, kname)
    roof["traffic"] = measured_traffic("batched64_" + prec, dominant)
    out = {
        "metric": METRIC,
        "value": n_pairs / t_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched64: 64 scalar problems, h 1/32..1/160, delta/h 2..5, constant and "
                               "1/|z| kernels, barycentre ball, gauss7 x gauss7, 5-point transforms",
                   "triangles": int(sum(w["mesh"].n_elements for w in ws)), "ordered_pairs": n_pairs,
                   "touching_pairs": int(sum(i["n_vertex"] + i["n_edge"] + i["n_ident"] for i in infos)),
                   "nnz": int(sum(i["nnz"] for i in infos)), "precision": prec,
                   "step": "64 rebuilds + batched assembly + 64 load vectors",
                   "build_streams": n_str},
        "roofline": roof,
        "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
        "parts_ms": {"rebuilds_64": t_build * 1e3, "batched_assembly": t_asm * 1e3,
                     "batched_assembly_graph": t_graph * 1e3, "plain_builds_64_first": t_plain_build * 1e3},
        "forms_assembly_ms": {f"{prec}_batched_graph": t_graph * 1e3, "mixed_batched_graph": t_mixed * 1e3,
                              "fp64_sequential_64": t_seq * 1e3,
                              "speedup_batched_vs_sequential_fp64": t_seq / t_asm if prec == "fp64" else None,
                              "speedup_mixed_vs_fp64_batched": (t_graph / t_mixed) if prec == "fp64" else None},
        "accuracy_vs_oracle": accuracy,
        "tuned_shape": nl.nlfem_batch_info(batch)["shape"],
        "launch_groups": nl.nlfem_batch_info(batch)["groups"],
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.copy_probe_mib > 0:
        out["copy_probe_bytes"] = _copy_probe(args.copy_probe_mib)
    print(json.dumps(out))
    nl.nlfem_batch_free(bmx)
    nl.nlfem_batch_free(batch)


def _copy_probe(mib):
    """One device copy of a known size (counter calibration)."""
    import torch
    n = mib << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return n


# ---------------------------------------------------------------- single

def _workload(name, precision):
    from inputs import workloads as W
    if name == "invdist_h64":
        return W.inv_dist_jittered(precision=precision)
    if name == "const_h16":
        w = W.small_constant()
        w["precision"] = precision
        return w
    if name == "peri_h128":
        return W.peridynamic(precision=precision)
    if name == "poly32_h256":
        return W.constant_polygon(precision=precision)
    raise SystemExit(f"unknown workload {name}")


def bench_single(args):
    import torch
    import paper_2207_03921_amd as nl
    torch.cuda.set_device(0)
    prec = args.precision
    w = _workload(args.workload, prec)
    mesh = w["mesh"]
    dm = nl.DeviceMesh.from_numpy(mesh)
    cfg = _config(w, prec)
    other = _config(w, "mixed" if prec == "fp64" else "fp64")
    aff = _f_affine(w)
    pairs = nl.nlfem_build_pairs(dm, cfg)
    info = nl.nlfem_pairs_info(pairs)
    val = torch.empty(max(info["nnz"], 1), dtype=torch.float64, device="cuda")
    val2 = torch.empty_like(val)
    b = torch.empty(cfg.ncomp * mesh.n_vertices, dtype=torch.float64, device="cuda")

    def step(c, v):
        nl.nlfem_build_pairs(dm, c, pairs=pairs)
        nl.nlfem_assemble(dm, c, pairs, val=v)
        nl.nlfem_rhs(dm, c, f_affine=aff, b=b)

    for _ in range(args.warmup):
        step(cfg, val)
    torch.cuda.synchronize()
    _timing_mask_all()
    step(cfg, val)
    torch.cuda.synchronize()
    phase_ms = _phases_per_step(1)
    dominant = max(phase_ms, key=phase_ms.get)
    nl.nlfem_timing_enable([dominant])
    nl.nlfem_timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(cfg, val)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    dom_ms = _phases_per_step(args.steps)[dominant]
    rebuild = nl.nlfem_pairs_info(pairs)["rebuild"]
    reps = max(3, args.steps // 2)
    for _ in range(2):
        step(other, val2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step(other, val2)
    torch.cuda.synchronize()
    t_other = (time.perf_counter() - t0) / reps
    far, touch, nbytes = work_of(info, w)
    roof = roofline_of(dominant, dom_ms, far, touch, nbytes, prec, PHASE_KERNELS["single"][dominant])
    roof["traffic"] = measured_traffic(f"{args.workload}_{prec}", dominant)
    out = {
        "metric": METRIC,
        "value": info["n_pairs"] / t_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} ({w['name']})", "triangles": mesh.n_elements,
                   "vertices": mesh.n_vertices, "ordered_pairs": info["n_pairs"],
                   "touching_pairs": info["n_vertex"] + info["n_edge"] + info["n_ident"],
                   "nnz": info["nnz"], "precision": prec, "step": "rebuild + assembly + load vector"},
        "roofline": roof,
        "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
        "rebuild": rebuild,
        "other_form": {"precision": other.precision, "ms_per_step": t_other * 1e3,
                       "value": info["n_pairs"] / t_other},
    }
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.Problem(mesh, w)
        t0 = time.perf_counter()
        k, l, c = P.pairs()
        rp, col, v = P.assemble((k, l, c))
        P.rhs(f_affine=aff)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(k) / dt, "unit": "pairs/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"whole workload ({len(k)} ordered pairs), one run, {dt:.2f} s"}
        A = _sparse(rp, col, v, P.n * mesh.n_vertices)
        torch.cuda.synchronize()
        acc = {}
        rpg, colg = nl.nlfem_csr_pattern(pairs)
        for name, vv in ((prec, val), (other.precision, val2)):
            G = _sparse(rpg.cpu().numpy(), colg.cpu().numpy(), vv[:info["nnz"]].cpu().numpy(), A.shape[0])
            fro, ent = _errors(G, A)
            acc[name] = {"rel_frobenius": fro, "max_entry_rel_row": ent}
        out["accuracy_vs_oracle"] = acc
    if args.copy_probe_mib > 0:
        out["copy_probe_bytes"] = _copy_probe(args.copy_probe_mib)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched64", choices=WORKLOADS)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--build-streams", type=int, default=4,
                    help="streams the batched workload's rebuilds and load vectors are spread over")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}); independent problems shard across GPUs "
              "with no communication, a single mesh by row ownership with a halo.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched64":
        bench_batched(args)
    else:
        bench_single(args)


if __name__ == "__main__":
    main()
