"""Benchmark: nonlocal P1 stiffness assembly on one MI355X.

One step = the whole hot path on one synthetic workload: element geometry,
pair search, CSR pattern (nlfem_build_pairs, reusing the handle's device
memory), the stiffness values (nlfem_assemble) and the load vector
(nlfem_rhs).  The metric is element-pair interactions assembled per second:
ordered interacting pairs of the workload x steps / wall time of the timed
steps, inputs resident in HBM.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = ("invdist_h64", "const_h16", "peri_h128", "poly32_h256", "batched64")


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


def cpu_baseline(w, runs=3):
    """The oracle as it stands on the host cores: the whole workload
    (brute-force pair search, assembly, load vector), median of `runs`."""
    import oracle
    oracle.build(force=False)
    P = oracle.Problem(w["mesh"], w)
    times, n = [], 0
    for _ in range(runs):
        t0 = time.perf_counter()
        k, l, c = P.pairs()
        P.assemble((k, l, c))
        P.rhs(f_affine=_f_affine(w))
        times.append(time.perf_counter() - t0)
        n = len(k)
    dt = sorted(times)[len(times) // 2]
    return {"value": n / dt, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"whole workload ({n} ordered pairs), median of {runs} runs of {dt:.2f} s"}


# ---------------------------------------------------------------- roofline
#
# Dominant kernel of the step: the row gather (phase "rows", one launch per
# assembly).  Its algorithmic bytes are what the row-owner gather must move
# at least once: every pair record and neighbour-list entry read once, the
# pattern read once and every value written once.
HBM_PEAK_GBS = 8000.0


def rows_algorithmic_bytes(info, n_vertices, n_elements, ncomp, precision):
    tr = 4 if precision == "mixed" else 8        # far records are FP32 in the mixed form
    nk = 1 if ncomp == 1 else 3
    far_stride = 21 * nk                         # X (9 blocks), De and Df (6 blocks each)
    touch_stride = (5 * ncomp) * (5 * ncomp + 1) // 2
    K, M = n_elements, n_vertices
    nnz_node = info["nnz"] // (ncomp * ncomp)
    return (info["n_upper_far"] * far_stride * tr       # non-touching records
            + info["n_upper_touch"] * touch_stride * 8  # touching records
            + K * 6 * nk * 8                            # per-element diagonal sums
            + info["n_nbr"] * (4 + 1 + 4)               # neighbour lists: id, flags, record index
            + K * 3 * 4 + 3 * K * 4                     # element vertices, node->element incidence
            + 2 * (M + 1) * 8 + M * 4                   # row and incidence pointers, node flags
            + nnz_node * 4                              # column ids
            + info["nnz"] * 8)                          # values, written once


# Vector-ALU peaks of MI355X (256 CUs at 2.4 GHz): FP32 157.3 TFLOP/s counts
# packed FP32 (two lanes per operation), which this build does not emit, so
# FP32 arithmetic here can reach at most half of it; FP64 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

# Kernel values Psi(z) after |z|^2: flops (a reciprocal square root counts
# one) and components
_KV = {"constant": (0, 1), "inv_dist": (2, 1), "peridynamic": (10, 3)}


def far_flops(info, kernel, p, q):
    """Flops of the non-touching records: per (outer, inner) point pair the
    difference (2), |z|^2 (3), Psi, the weight w_p|J_e| w_q|J_f| (s_p + t_q)
    (3) and per component the product, the row/column sums and three basis
    products (9); per outer point the X and D_e updates (36 per component)
    and its mapping (6); per inner point the D_f update (18 per component)
    and its mapping (6).  Equal rules take one pass for both orders of a
    pair, different rules two."""
    kv, nk = _KV[kernel]
    one = p * q * (8 + kv + 9 * nk) + p * (36 * nk + 6) + q * (18 * nk + 6)
    return info["n_upper_far"] * (one if p == q else 2 * one)


def touch_flops(info, kernel, n, ncomp):
    """Flops of the touching records: per quadrature point of the
    regularising transforms (identical 6n, edge 4n^2, vertex 2n^3 points) the
    difference (4), |z|^2 (3), Psi, the weighted kernel (one per component)
    and the outer product g g^T of the D = (3, 4 or 5) * ncomp local basis
    differences (D products, D (D + 1) / 2 multiply-adds)."""
    kv, nk = _KV[kernel]
    total = 0
    for pairs, pts, nu in ((info["n_ident"], 6 * n, 3), (info["n_edge"] // 2, 4 * n * n, 4),
                           (info["n_vertex"] // 2, 2 * n ** 3, 5)):
        d = nu * ncomp
        total += pairs * pts * (7 + kv + nk + d + d * (d + 1))
    return total


# The source of the row gather: its section of assemble_items.h (from the
# "phase 2: row gather" banner to the "plans" banner) and the k_rows kernel
# in assemble.hip.  A counter summary holds the digest of this text from
# when the counters were taken.
ROW_SECTIONS = (("assemble_items.h", "phase 2: row gather", "-- plans"),
                ("assemble.hip", "k_rows(RowArgs a)", "\n}\n"))


def row_gather_digest():
    import hashlib
    h = hashlib.sha256()
    for fn, start, end in ROW_SECTIONS:
        with open(os.path.join(ROOT, "paper_2207_03921_amd", "csrc", fn)) as fh:
            text = fh.read()
        a = text.index(start)
        b = text.index(end, a + len(start))
        h.update(text[a:b].encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the row gather from the committed counter
    summary, or None when it is missing or the kernel source has changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_rows_{workload}_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != row_gather_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_batched(args):
    """64 independent problems (h from 1/32 to 1/160, delta/h in 2..5, half
    constant, half 1/|z| with the regularising transforms).  The pair
    structures are built once (their build time is reported); a step is the
    assembly of all 64 problems: the batched form replays one HIP graph of
    persistent launches, the baseline assembles the problems one after the
    other in plain FP64."""
    import torch
    import paper_2207_03921_amd as nl
    from inputs import workloads as W
    torch.cuda.set_device(0)
    ws = W.batched(64, precision=args.precision)
    dms = [nl.DeviceMesh.from_numpy(w["mesh"]) for w in ws]
    cfgs = [_config(w, args.precision) for w in ws]
    cfg64 = [_config(w, "fp64") for w in ws]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = [nl.nlfem_build_pairs(d, c) for d, c in zip(dms, cfgs)]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    infos = [nl.nlfem_pairs_info(p) for p in pairs]
    n_pairs = sum(i["n_pairs"] for i in infos)
    vals = [torch.empty(max(i["nnz"], 1), dtype=torch.float64, device="cuda") for i in infos]
    cache = os.path.join(ROOT, "paper_2207_03921_amd", "tune_cache.txt")
    batch = nl.nlfem_batch_create(dms, cfgs, pairs, vals, tune_cache=cache, tune=1)
    batch64 = nl.nlfem_batch_create(dms, cfg64, pairs, vals, tune_cache=cache, tune=1)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    t_graph = timed(lambda: nl.nlfem_batch_launch_graph(batch), args.steps, args.warmup)
    t_graph64 = timed(lambda: nl.nlfem_batch_launch_graph(batch64), args.steps, args.warmup)

    def sequential():
        for d, c, p, v in zip(dms, cfg64, pairs, vals):
            nl.nlfem_assemble(d, c, p, val=v)

    t_seq = timed(sequential, max(3, args.steps // 2), 1)
    out = {
        "metric": "element-pair interactions assembled/sec",
        "value": n_pairs / t_graph,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_graph * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "batched64 (64 problems, h 1/32..1/160, delta/h 2..5, constant and 1/|z|)",
                   "triangles": int(sum(w["mesh"].n_elements for w in ws)), "ordered_pairs": n_pairs,
                   "touching_pairs": int(sum(i["n_vertex"] + i["n_edge"] + i["n_ident"] for i in infos)),
                   "nnz": int(sum(i["nnz"] for i in infos)), "precision": args.precision,
                   "launch_groups": nl.nlfem_batch_info(batch)["groups"]},
        "roofline": None,
        "build_ms_all_problems": t_build * 1e3,
        "batched_fp64_graph": {"ms_per_step": t_graph64 * 1e3, "value": n_pairs / t_graph64},
        "sequential_fp64_plain": {"ms_per_step": t_seq * 1e3, "value": n_pairs / t_seq},
        "speedup_vs_sequential_fp64": t_seq / t_graph,
        "tuned_shape": nl.nlfem_batch_info(batch)["shape"],
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="invdist_h64", choices=WORKLOADS)
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not run.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched64":
        bench_batched(args)
        return

    import torch
    import paper_2207_03921_amd as nl

    torch.cuda.set_device(0)
    w = _workload(args.workload, args.precision)
    mesh = w["mesh"]
    dm = nl.DeviceMesh.from_numpy(mesh)
    cfg = _config(w, args.precision)
    cfg64 = _config(w, "fp64")
    aff = _f_affine(w)
    stream = torch.cuda.current_stream()
    pairs = nl.nlfem_build_pairs(dm, cfg)
    info = nl.nlfem_pairs_info(pairs)
    val = torch.empty(max(info["nnz"], 1), dtype=torch.float64, device="cuda")
    b = torch.empty(cfg.ncomp * mesh.n_vertices, dtype=torch.float64, device="cuda")

    def step(c):
        nl.nlfem_build_pairs(dm, c, pairs=pairs)
        nl.nlfem_assemble(dm, c, pairs, val=val)
        nl.nlfem_rhs(dm, c, f_affine=aff, b=b)

    def timed(c, steps, warmup):
        for _ in range(warmup):
            step(c)
        torch.cuda.synchronize()
        # the row gather is timed by the library's HIP events on the stream
        # it is launched on, over exactly the timed steps
        nl.nlfem_timing_enable(["rows"])
        nl.nlfem_timing_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(c)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rows = nl.nlfem_timing_read(reset=True)["rows"]
        nl.nlfem_timing_enable(False)
        return dt, rows[0] / max(rows[1], 1)

    t_step, t_rows = timed(cfg, args.steps, args.warmup)
    rebuild = nl.nlfem_pairs_info(pairs)["rebuild"]

    # assemble alone (HIP events on the library's stream)
    def assemble_ms(c, reps=20):
        for _ in range(3):
            nl.nlfem_assemble(dm, c, pairs, val=val)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            nl.nlfem_assemble(dm, c, pairs, val=val)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # per-phase times per step, all phases timed (separate, untimed loop)
    nl.nlfem_timing_enable(True)
    nl.nlfem_timing_read(reset=True)
    for _ in range(args.steps):
        step(cfg)
    torch.cuda.synchronize()
    phases = nl.nlfem_timing_read(reset=True)
    nl.nlfem_timing_enable(False)
    phase_ms = {k: v[0] / args.steps for k, v in phases.items()}

    t_asm = assemble_ms(cfg)
    t_asm64 = assemble_ms(cfg64)
    t_step64, _ = timed(cfg64, max(3, args.steps // 2), 1)
    n_pairs = info["n_pairs"]
    alg = rows_algorithmic_bytes(info, mesh.n_vertices, mesh.n_elements, cfg.ncomp, args.precision)
    achieved = alg / (t_rows * 1e-3) / 1e9
    # the quadrature kernels against the vector-ALU peaks (per-phase loop)
    quad = {}
    if phase_ms.get("far", 0) > 0:
        fl = far_flops(info, w["kernel"], len(w["outer"].w), len(w["inner"].w))
        tf = fl / (phase_ms["far"] * 1e-3) / 1e12
        pk = FP32_PEAK_TFLOPS if args.precision == "mixed" else FP64_PEAK_TFLOPS
        quad["far"] = {"bound": "alu", "dtype": "f32" if args.precision == "mixed" else "f64",
                       "achieved": tf, "peak": pk, "unit": "TFLOP/s", "frac": tf / pk,
                       "flops": fl, "launch_ms": phase_ms["far"], "kernel": "k_far_rec"}
    if phase_ms.get("touch", 0) > 0 and int(w.get("singular_n", 0)) > 0:
        fl = touch_flops(info, w["kernel"], int(w["singular_n"]), cfg.ncomp)
        tf = fl / (phase_ms["touch"] * 1e-3) / 1e12
        quad["touch"] = {"bound": "alu", "dtype": "f64", "achieved": tf, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS, "flops": fl,
                         "launch_ms": phase_ms["touch"], "kernel": "k_touch_rec"}
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(args.workload, args.precision),
                "kernel": "k_rows (row gather)", "algorithmic_bytes": alg, "launch_ms": t_rows}
    out = {
        "metric": "element-pair interactions assembled/sec",
        "value": n_pairs / t_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} ({w['name']})", "triangles": mesh.n_elements,
                   "vertices": mesh.n_vertices, "ordered_pairs": n_pairs,
                   "touching_pairs": info["n_vertex"] + info["n_edge"] + info["n_ident"],
                   "nnz": info["nnz"], "precision": args.precision},
        "roofline": roofline,
        "build": {0: "plain build (three host synchronisations)",
                  1: "rebuild with the sizes of the previous build (one host synchronisation)",
                  2: "rebuild fell back to a plain build"}[rebuild],
        "roofline_quadrature": quad,
        "assemble_ms": t_asm,
        "phase_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "assemble_pairs_per_s": n_pairs / (t_asm * 1e-3),
        "fp64_plain": {"ms_per_step": t_step64 * 1e3, "value": n_pairs / t_step64,
                       "assemble_ms": t_asm64},
    }
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = n
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
