#!/usr/bin/env python3
"""Benchmark: converged linear-scaling ground-state solve on one MI355X.

Workload: 4096-atom diamond Si (8x8x8 cells, box 43.44 A, periodic), 9 orbitals
per atom, FP64 blocks; H/S cutoff 6 A, L cutoff 10 A, S^-1 cutoff 8 A.
One step = one pass of the whole hot path: Hotelling S^-1 (to stagnation),
the initial L from Z, and LNV iterations until |dE| < 1e-8 Ha.  Inputs are
seeded synthetic Si-like matrices standing in for the paper's Si runs; they are
resident on the GPU and the patterns and product plans are built before the
timed region (their build times are reported separately).

value = algorithmic block-product flops of the timed steps / timed wall time
(2 b^3 per block triple actually present; no zero fill counted).

Prints progress to stderr and one JSON line to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-sparse GFLOP/s + s per converged LNV solve, 4096-atom 9-orb, vs FP64 oracle"
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (= FP64 matrix) peak
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="si4096_b9",
                    choices=["si4096_b9", "si64_b4", "batch64", "si4096_b9_mixed", "guess", "invsqrt", "forces",
                             "contract"],
                    help="si64_b4: 64 atoms, 4 orbitals: one L S L product, 10 Hotelling steps and 20 LNV "
                         "iterations, the oracle doing the same; batch64: 64 uneven systems (512-4096 atoms, b = 4 and 9), the 16 A x 16 A -> 16 A "
                         "product of each, per-product launches against one tuned persistent launch; "
                         "si4096_b9_mixed: the solve with BF16 then FP32 products and 3 FP64 steps against "
                         "the FP64 solve; guess: networks trained on 4096-atom displaced frames, held-out 4096- and 32768-atom "
                         "displaced frame solved from the learned and from the plain starts; invsqrt: "
                         "truncated S^-1/2 and S^1/2 of the 4096-atom overlap (coupled Newton-Schulz); forces: "
                         "forces of a converged 4096-atom displaced frame; contract: the 4096-atom system "
                         "contracted to 4 on-site support functions per atom and solved, against the 9-orbital solve")
    ap.add_argument("--guess-train", type=int, default=48, help="training frames of the guess workload")
    ap.add_argument("--guess-train-cells", type=int, default=8,
                    help="cells per side of the guess training frames (8: 4096 atoms)")
    ap.add_argument("--guess-sample-frac", type=float, default=0.25,
                    help="fraction of each training frame's pair samples kept")
    ap.add_argument("--guess-cells", type=int, default=16,
                    help="cells per side of the large guess test frame (16: 32768 atoms); a frame of the "
                         "training size is also compared")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--max-lnv", type=int, default=300)
    ap.add_argument("--tol-e", type=float, default=1e-8)
    ap.add_argument("--cpu-rows", type=int, default=1024,
                    help="rows of the 16 A x 16 A product the oracle computes for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=-1,
                    help="product kernel variant for --mode product (-1: the library default)")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"],
                    help="operand precision of the --mode product and --mode classes launches")
    ap.add_argument("--rows", type=int, default=0,
                    help="rows per tile for --mode product (0: the library default)")
    ap.add_argument("--column-order", type=int, default=-1, choices=[-1, 0, 1],
                    help="tile column order for --mode product (-1: the library default)")
    ap.add_argument("--pair", action="store_true",
                    help="--mode product: the paired launch W = X X, U = Y X (two products sharing B) "
                         "instead of X X alone")
    ap.add_argument("--mode", default="solve", choices=["solve", "product", "classes"],
                    help="product: only the dominant 16 A x 16 A -> 16 A product, --steps launches, plus a "
                         "2 GiB device copy (for hardware-counter runs and their byte calibration); classes: "
                         "every product class of the 4096-atom solve under each tile setting (rows per "
                         "tile, direct or transposed plan, column order), --steps launches each")
    return ap.parse_args()


def product_mode(args):
    """The dominant product class alone, in the launch the solve uses, for counter runs."""
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    n, b = (8, 9) if args.workload == "si4096_b9" else (2, 4)
    s = synth.si4096_b9() if args.workload == "si4096_b9" else synth.si64_b4()
    rx = s.cutoffs["L"] + s.cutoffs["S"]
    ctx = bsm.Context(0)
    ctx.set_product_variant(args.variant)
    ctx.set_rows_per_wave(args.rows)
    if args.column_order >= 0:
        ctx.set_column_order(args.column_order)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    P = bsm.Pattern(ctx, pos, s.box, rx, b)
    g = torch.Generator(device=ctx.device)
    g.manual_seed(7)
    X = bsm.Matrix(P, torch.rand((P.nnzb, b, b), dtype=torch.float64, device=ctx.device, generator=g) - 0.5)
    C = bsm.Matrix(P)
    flops = bsm.product_flops(P, P, P)
    prec = {"f64": bsm.F64, "f32": bsm.F32, "bf16": bsm.BF16}[args.prec]
    if args.pair:
        if prec != bsm.F64:
            raise SystemExit("--pair runs FP64 products")
        Y = bsm.Matrix(P, torch.rand((P.nnzb, b, b), dtype=torch.float64, device=ctx.device, generator=g) - 0.5)
        C2 = bsm.Matrix(P)
        flops *= 2
    ctx.set_profiling(True)
    for k in range(args.steps):
        if args.pair:
            bsm.multiply_truncate_pair(1.0, X, Y, X, 0.0, C, C2)
        else:
            bsm.multiply_truncate_prec(prec, 1.0, X, X, 0.0, C)
        torch.cuda.synchronize()
        log(f"[product] launch {k}")
    st = ctx.product_stats()[0]
    src = torch.empty(1 << 28, dtype=torch.float64, device=ctx.device).fill_(1.0)   # 2 GiB
    log(f"[product] kernel {kernel_name(st)}, sources {kernel_sources_sha()}")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ms = st["ms"] / st["launches"]
    print(json.dumps({"mode": "product", "pair": args.pair, "precision": args.prec, "column_order": args.column_order,
                      "kernel": kernel_name(st),
                      "sources_sha256_16": kernel_sources_sha(),
                      "flops_per_launch": flops, "avg_ms": ms,
                      "tflops": flops / (ms * 1e-3) / 1e12, "blocks": P.nnzb,
                      "algorithmic_bytes": (5 if args.pair else 3) * P.nnzb * b * b * 8,
                      "copy_bytes": 2 * src.numel() * 8}),
          flush=True)


FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector peak

# (r_A, r_B, r_C) of the products in the 4096-atom solve: X = L S, Z G, S U and the like,
# M(G)'s second product, T = Z S, the Hotelling update, W = X X
SOLVE_CLASSES = [(10, 6, 16), (8, 10, 18), (6, 16, 10), (18, 8, 10), (8, 6, 14), (14, 8, 8), (16, 16, 16)]


def small_mode(args):
    """The 64-atom, 4-orbital system: one L S L product (L S on P(r_L + r_S), then times L on
    P(2 r_L + r_S)), 10 Hotelling steps and 20 LNV iterations from L0 = c mask_L(Z)."""
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    s = synth.si64_b4()
    cut = s.cutoffs
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    PS = bsm.Pattern(ctx, pos, s.box, cut["S"], s.b)
    PZ = bsm.Pattern(ctx, pos, s.box, cut["Z"], s.b)
    PL = bsm.Pattern(ctx, pos, s.box, cut["L"], s.b)
    PX = bsm.Pattern(ctx, pos, s.box, cut["L"] + cut["S"], s.b)
    PK = bsm.Pattern(ctx, pos, s.box, 2 * cut["L"] + cut["S"], s.b)
    S, H, Z, L = bsm.Matrix(PS), bsm.Matrix(PS), bsm.Matrix(PZ), bsm.Matrix(PL)
    X, K = bsm.Matrix(PX), bsm.Matrix(PK)
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)
    lnv = None

    def run():
        nonlocal lnv
        hr = bsm.hotelling_inverse(S, Z, max_iter=10, tol=0.0)
        if lnv is None:
            lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=0.0, init_from_z=True)
        else:
            lnv.reset(init_from_z=True)
        bsm.multiply_truncate(1.0, L, S, 0.0, X)
        bsm.multiply_truncate(1.0, X, L, 0.0, K)
        res = [lnv.step() for _ in range(20)]
        torch.cuda.synchronize()
        return hr, res

    for _ in range(max(args.warmup, 1)):
        run()
    t = time.perf_counter()
    for _ in range(args.steps):
        hr, res = run()
    dt = (time.perf_counter() - t) / args.steps
    log(f"[si64_b4] 10 Hotelling steps, L S L, 20 LNV iterations: {dt * 1e3:.2f} ms, E = {res[-1].E:.10f}")
    out = {"metric": "s per 64-atom 4-orb L S L product + 10 Hotelling steps + 20 LNV iterations",
           "value": round(dt, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": max(args.warmup, 1),
           "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "si64_b4: 64 atoms (2 x 2 x 2 cells), 4 orbitals, S = H = 6, L = Z = 8 A",
                      "natoms": s.natoms, "orbitals_per_atom": s.b},
           "hotelling_residuals": [hr.residuals[0], hr.residuals[-1]],
           "E_Ha": [r.E for r in res], "N": [r.N for r in res]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = small_cpu_baseline(s, out["E_Ha"])
    print(json.dumps(out), flush=True)


def small_cpu_baseline(s, E_gpu):
    """The oracle doing the same work (10 Hotelling steps, L S L, 20 LNV iterations), timed."""
    import numpy as np
    import oracle as O
    cut = s.cutoffs
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    t = time.perf_counter()
    PS = O.create_pattern(s.positions, s.box, cut["S"])
    PZ = O.create_pattern(s.positions, s.box, cut["Z"])
    PL = O.create_pattern(s.positions, s.box, cut["L"])
    PX = O.create_pattern(s.positions, s.box, cut["L"] + cut["S"])
    PK = O.create_pattern(s.positions, s.box, 2 * cut["L"] + cut["S"])
    S = O.from_blocks(PS, s.b, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(PS, s.b, s.H.rows, s.H.cols, s.H.blocks)
    hr = O.hotelling_inverse(S, PZ, max_iter=10, tol=0.0)
    st = O.lnv_init(S, H, hr.Z, PL, s.n_electrons, tol_E=0.0)
    O.product(O.product(st.L, S, PX), st.L, PK)
    E = [O.lnv_step(st).E for _ in range(20)]
    dt = time.perf_counter() - t
    rel = float(np.max(np.abs(np.array(E) - np.array(E_gpu)) / np.abs(np.array(E))))
    return {"value": round(dt, 3), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": "the whole workload (patterns, 10 Hotelling steps, L S L, 20 LNV iterations)",
            "cpu": host_cpu(), "max_rel_dE_per_iteration_vs_gpu": rel}


def classes_mode(args):
    """Each product class of the 4096-atom, b = 9 solve on random blocks, timed with HIP events
    on the library stream under every tile setting (operands in --prec); every setting must give
    the same bits (BF16 on the matrix cores: the same values within FP32 rounding)."""
    import itertools
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    s = synth.si4096_b9()
    prec = {"f64": bsm.F64, "f32": bsm.F32, "bf16": bsm.BF16}[args.prec]
    ctx = bsm.Context(0)
    dev = ctx.device
    pos = torch.tensor(s.positions, dtype=torch.float64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    pats, mats = {}, {}
    for r in sorted({r for c in SOLVE_CLASSES for r in c}):
        pats[r] = bsm.Pattern(ctx, pos, s.box, float(r), s.b)
    out = []
    for ra, rb, rc in SOLVE_CLASSES:
        for r in (ra, rb):
            if r not in mats:
                mats[r] = bsm.Matrix(pats[r], torch.rand((pats[r].nnzb, s.b, s.b), dtype=torch.float64,
                                                         device=dev, generator=g) - 0.5)
        A, B, C = mats[ra], mats[rb], bsm.Matrix(pats[rc])
        flops = bsm.product_flops(pats[ra], pats[rb], pats[rc])
        ref, rows_out = None, []
        # the same-pattern class has no transposed plan
        for rows, tmode, corder in itertools.product((4, 8), (0, 1, 2) if ra != rb else (0,), (0, 1)):
            ctx.set_rows_per_wave(rows)
            ctx.set_transposed_plans(tmode)
            ctx.set_column_order(corder)
            bsm.multiply_truncate_prec(prec, 1.0, A, B, 0.0, C)   # builds the plan
            torch.cuda.synchronize()
            if ref is None:
                ref = C.blocks.clone()
            elif prec != bsm.BF16 and not torch.equal(ref, C.blocks):
                raise RuntimeError(f"class {(ra, rb, rc)}: setting {(rows, tmode, corder)} changed the result")
            elif prec == bsm.BF16 and float((ref - C.blocks).abs().max()) > 1e-5 * float(ref.abs().max()):
                # the matrix cores sum each pair of entries in their own order: equal within FP32 rounding
                raise RuntimeError(f"class {(ra, rb, rc)}: setting {(rows, tmode, corder)} changed the result")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(ctx.stream):
                e0.record()
                for _ in range(args.steps):
                    bsm.multiply_truncate_prec(prec, 1.0, A, B, 0.0, C)
                e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            rows_out.append({"rows": rows, "transposed_plans": tmode, "column_order": corder,
                             "ms": round(ms, 3), "tflops": round(flops / ms / 1e9, 2)})
            log(f"[classes] P{ra} x P{rb} -> P{rc}: rows {rows}, transposed {tmode}, column order "
                f"{corder}: {ms:.3f} ms, {flops / ms / 1e9:.2f} TFLOP/s")
        default = [r for r in rows_out if r["rows"] == 8 and r["transposed_plans"] == (1 if ra != rb else 0)
                   and r["column_order"] == 1][0]
        best = min(rows_out, key=lambda r: r["ms"])
        out.append({"class": [ra, rb, rc], "flops": flops, "default": default, "best": best,
                    "default_frac": round(default["tflops"] / FP64_PEAK_TFLOPS, 4) if prec == bsm.F64 else None,
                    "settings": rows_out})
        del C
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "classes", "precision": args.prec, "workload": "si4096_b9", "steps": args.steps,
                      "sources_sha256_16": kernel_sources_sha(), "classes": out}), flush=True)


def batch_mode(args):
    """Many independent systems: the dominant product class of each, launched per product and
    as one persistent launch whose schedule the library's autotuner picks, in FP64 and FP32."""
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    cells = synth.batch_cells(count=args.batch_count)
    ctx = bsm.Context(0)
    dev = ctx.device
    rx = 16.0
    mats = []
    t0 = time.perf_counter()
    for n, (c, b) in enumerate(cells):
        pos, box, _ = synth.diamond_positions(c)
        P = bsm.Pattern(ctx, torch.tensor(pos, dtype=torch.float64, device=dev), box, rx, b)
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + n)
        X = bsm.Matrix(P, torch.rand((P.nnzb, b, b), dtype=torch.float64, device=dev, generator=g) - 0.5)
        mats.append((X, X, bsm.Matrix(P)))
    torch.cuda.synchronize()
    natoms = sum(len(synth.diamond_positions(c)[0]) for c, _ in cells)
    blocks = sum(m[2].pattern.nnzb for m in mats)
    log(f"[batch] {len(cells)} systems, {natoms} atoms, {blocks} blocks per matrix set, "
        f"setup {time.perf_counter() - t0:.1f} s, device memory {torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    def checksums():
        return [float(m[2].blocks.sum()) for m in mats]

    res = {}
    for prec, name in ((bsm.F64, "f64"), (bsm.F32, "f32")):
        flops = sum(bsm.product_flops(A.pattern, B.pattern, C.pattern) for A, B, C in mats)
        for A, B, C in mats:                                    # plans + warm-up
            bsm.multiply_truncate_prec(prec, 1.0, A, B, 0.0, C)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(args.steps):
            for A, B, C in mats:
                bsm.multiply_truncate_prec(prec, 1.0, A, B, 0.0, C)
        torch.cuda.synchronize()
        sep_s = (time.perf_counter() - t) / args.steps
        ref = checksums()
        log(f"[batch {name}] per-product launches: {sep_s * 1e3:.1f} ms, {flops / sep_s / 1e12:.2f} TFLOP/s")
        batch = bsm.Batch(ctx, mats, alpha=1.0, beta=0.0, precision=prec)
        t = time.perf_counter()
        cfg, tune_ms = batch.tune(reps=1)
        tune_s = time.perf_counter() - t
        log(f"[batch {name}] tuned in {tune_s:.1f} s: {cfg}, {tune_ms:.1f} ms")
        for w in range(args.warmup):
            batch.run()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream(dev)
        t = time.perf_counter()
        ev0.record(stream)
        for k in range(args.steps):
            batch.run()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall_s = (time.perf_counter() - t) / args.steps
        dev_ms = ev0.elapsed_time(ev1) / args.steps
        same = checksums() == ref
        log(f"[batch {name}] persistent launch: {dev_ms:.1f} ms, {flops / (dev_ms * 1e-3) / 1e12:.2f} TFLOP/s, "
            f"matches per-product launches: {same}")
        res[name] = dict(flops=flops, separate_ms=sep_s * 1e3, batch_ms=dev_ms, wall_s=wall_s, tuned=cfg,
                         tune_s=tune_s, same=same)
        batch.close()
    r64, r32 = res["f64"], res["f32"]
    achieved = r64["flops"] / (r64["batch_ms"] * 1e-3) / 1e12
    out = {
        "metric": "block-sparse GFLOP/s, 64 uneven systems in one persistent launch",
        "value": round(r64["flops"] / r64["wall_s"] / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r64["wall_s"] * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(cells)} diamond-Si systems, {natoms} atoms, b = 4 and 9, "
                               f"16 A x 16 A -> 16 A product each", "systems": len(cells), "natoms": natoms,
                   "b9_systems": sum(1 for _, b in cells if b == 9)},
        "f64": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r64.items()},
        "f32": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r32.items()},
        "f32_gflops": round(r32["flops"] / (r32["batch_ms"] * 1e-3) / 1e9, 2),
        "batch_speedup_vs_separate_f64": round(r64["separate_ms"] / r64["batch_ms"], 3),
        "batch_speedup_vs_separate_f32": round(r32["separate_ms"] / r32["batch_ms"], 3),
        "roofline": {"bound": "alu", "kernel": "k_product_batch (FP64)", "achieved": round(achieved, 3),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": None, "avg_launch_ms": round(r64["batch_ms"], 3)},
    }
    print(json.dumps(out), flush=True)



def _solver(ctx, s):
    import torch
    import paper_2205_08941_amd as bsm
    dev = ctx.device
    pos = torch.tensor(s.positions, dtype=torch.float64, device=dev)
    P = {k: bsm.Pattern(ctx, pos, s.box, s.cutoffs[k], s.b) for k in ("S", "Z", "L")}
    S, H, Z, L = bsm.Matrix(P["S"]), bsm.Matrix(P["S"]), bsm.Matrix(P["Z"]), bsm.Matrix(P["L"])
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)
    return P, S, H, Z, L


def mixed_mode(args):
    """Time to the converged energy: FP64 products against BF16 -> FP32 -> 3 x FP64 stages
    (and BF16 -> 5 x FP64)."""
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    s = synth.si4096_b9()
    ctx = bsm.Context(0)
    P, S, H, Z, L = _solver(ctx, s)
    bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
    lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=args.tol_e, init_from_z=True)
    # BF16 products until the energy stops falling, FP32 to |dE| < 1e-4 Ha, then 3 FP64 steps; and the
    # shortest schedule measured to stay within 1e-6 Ha/atom: BF16, then 5 FP64 steps
    stages = [(bsm.BF16, 30, 0.0, True), (bsm.F32, 60, 1e-4, True), (bsm.F64, 3, 0.0, False)]
    short = [(bsm.BF16, 30, 0.0, True), (bsm.F64, 5, 0.0, False)]
    out = {}
    for tag, sched in (("f64", [(bsm.F64, args.max_lnv, args.tol_e, False)]), ("mixed", stages), ("bf16_f64x5", short)):
        for rep in range(args.warmup + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
            lnv.reset(init_from_z=True)
            r = lnv.solve(sched)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
        e_idem = lnv.idempotency_error()
        out[tag] = dict(seconds=round(dt, 3), E=r["E"], iterations=r["iterations"], converged=r["converged"],
                        status=r["status"], idempotency_error=e_idem, hotelling=hr.iterations)
        log(f"[mixed] {tag}: {dt:.2f} s, iterations {r['iterations']}, E {r['E']:.10f}, e_idem {e_idem:.3e}")
    dE = abs(out["mixed"]["E"] - out["f64"]["E"]) / s.natoms
    out["bf16_f64x5"]["dE_per_atom_Ha"] = abs(out["bf16_f64x5"]["E"] - out["f64"]["E"]) / s.natoms
    res = {"metric": "s per converged LNV solve, 4096-atom 9-orb, mixed-precision products",
           "value": out["mixed"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
           "ms_per_step": out["mixed"]["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16/f32 products, f64 traces", "data": "synthetic",
           "config": {"workload": "si4096_b9: Hotelling + LNV, BF16 (matrix cores, until E rises) -> FP32 "
                                  "(to |dE| < 1e-4 Ha) -> 3 FP64 steps"},
           "f64": out["f64"], "mixed": out["mixed"], "dE_per_atom_Ha": dE,
           "speedup_vs_f64": round(out["f64"]["seconds"] / out["mixed"]["seconds"], 3),
           "bf16_f64x5": out["bf16_f64x5"],
           "bf16_f64x5_speedup_vs_f64": round(out["f64"]["seconds"] / out["bf16_f64x5"]["seconds"], 3)}
    g = stored_oracle_solve("si4096_b9")
    if g is not None:
        Eo = g["lnv"]["E_final"]
        for tag in out:
            out[tag]["dE_oracle_per_atom_Ha"] = abs(out[tag]["E"] - Eo) / s.natoms
            out[tag]["within_1e-6_Ha_per_atom_of_oracle"] = out[tag]["dE_oracle_per_atom_Ha"] <= 1e-6
        res["oracle"] = {"E_Ha": Eo, "idempotency_error": g["lnv"].get("idempotency_error"),
                         "lnv_iterations": len(g["lnv"]["iterations"]),
                         "source": "tests/golden/lnv_si4096_b9.json (FP64 CPU oracle, same seeded system)"}
        for tag in out:
            log(f"[oracle] {tag}: |E - E_oracle| / N = {out[tag]['dE_oracle_per_atom_Ha']:.3e} Ha")
    print(json.dumps(res), flush=True)


def invsqrt_mode(args):
    """S^-1/2 and S^1/2 of the 4096-atom, b = 9 overlap on the 8 A pattern by the truncated
    coupled Newton-Schulz iteration (bsm_inverse_sqrt), run to its truncation floor."""
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    s = synth.si4096_b9()
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    PS = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], s.b)
    PZ = bsm.Pattern(ctx, pos, s.box, s.cutoffs["Z"], s.b)
    S, Z, Y = bsm.Matrix(PS), bsm.Matrix(PZ), bsm.Matrix(PZ)
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    for _ in range(args.warmup):   # builds the patterns' plans
        bsm.inverse_sqrt(S, Z, Y, max_iter=100, tol=1e-12)
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t = time.perf_counter()
    for _ in range(args.steps):
        r = bsm.inverse_sqrt(S, Z, Y, max_iter=100, tol=1e-12)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    stats = ctx.product_stats()
    ctx.set_profiling(False)
    flops = sum(st["flops"] for st in stats) / args.steps
    top = max(stats, key=lambda st: st["ms"])
    top_ms = top["ms"] / top["launches"]
    top_tf = top["flops"] / top["launches"] / (top_ms * 1e-3) / 1e12
    log(f"[invsqrt] {r.iterations} updates, residual {r.residuals[0]:.3e} -> {r.residuals[-1]:.3e}, "
        f"{dt:.3f} s, {flops / dt / 1e12:.2f} TFLOP/s over the products")
    res = {"metric": "s per truncated S^-1/2 (coupled Newton-Schulz), 4096-atom 9-orb", "value": round(dt, 4),
           "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "si4096_b9 overlap (S on 6 A), S^-1/2 and S^1/2 on 8 A, to the truncation floor",
                      "natoms": len(s.positions), "orbitals_per_atom": s.b},
           "updates": r.iterations, "residuals": [r.residuals[0], r.residuals[-1]],
           "product_gflops": round(flops / dt / 1e9, 1),
           "roofline": {"bound": "alu", "kernel": f"{kernel_name(top)}: P{top['cutoffs'][0]:g} x "
                                                  f"P{top['cutoffs'][1]:g} -> P{top['cutoffs'][2]:g}",
                        "achieved": round(top_tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(top_tf / FP64_PEAK_TFLOPS, 4), "traffic": None,
                        "avg_launch_ms": round(top_ms, 3), "launches": top["launches"]}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = invsqrt_cpu_baseline(s, r.iterations)
    print(json.dumps(res), flush=True)


def forces_mode(args):
    """Forces of a converged 4096-atom, b = 9 displaced frame (geometry-smooth S and H):
    one converged solve, then lnv_forces timed."""
    import numpy as np
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    t = time.perf_counter()
    s = synth.make_system("si4096_b9_frame", 8, 9, synth.BIG_CUTOFFS, 10000, displacement_sigma=0.05,
                          smooth=True, derivatives=True)
    log(f"[forces] frame and derivative blocks generated in {time.perf_counter() - t:.1f} s")
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    P6 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], s.b)
    PZ = bsm.Pattern(ctx, pos, s.box, s.cutoffs["Z"], s.b)
    PL = bsm.Pattern(ctx, pos, s.box, s.cutoffs["L"], s.b)

    def filled(bl):
        m = bsm.Matrix(P6)
        bsm.fill_blocks(m, bl.rows, bl.cols, bl.blocks)
        return m
    S, H = filled(s.S), filled(s.H)
    dS, dH = [filled(d) for d in s.dS], [filled(d) for d in s.dH]
    Z, L = bsm.Matrix(PZ), bsm.Matrix(PL)
    torch.cuda.synchronize()
    t = time.perf_counter()
    hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
    lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=args.tol_e)
    r = lnv.solve([(bsm.F64, args.max_lnv, args.tol_e, False)])
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t
    for _ in range(args.warmup):
        lnv.forces(dS, dH)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        F, mu = lnv.forces(dS, dH)
    dt = (time.perf_counter() - t) / args.steps
    stats = ctx.product_stats()
    ctx.set_profiling(False)
    flops = sum(st["flops"] for st in stats) / args.steps
    top = max(stats, key=lambda st: st["ms"])
    top_ms = top["ms"] / top["launches"]
    top_tf = top["flops"] / top["launches"] / (top_ms * 1e-3) / 1e12
    log(f"[forces] solve {t_solve:.2f} s ({hr.iterations} Hotelling, {r['iterations']} LNV), forces {dt:.3f} s, "
        f"max |F| {np.abs(F).max():.4f} Ha/A, |sum F| {np.abs(F.sum(0)).max():.1e}")
    res = {"metric": "s per force evaluation at the converged density matrix, 4096-atom 9-orb frame",
           "value": round(dt, 4), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "4096-atom b = 9 displaced frame (sigma 0.05 A, geometry-smooth S and H), "
                                  "converged LNV, then F = -dOmega/dR", "natoms": s.natoms, "orbitals_per_atom": s.b},
           "solve_s": round(t_solve, 3), "lnv_iterations": r["iterations"], "mu": mu,
           "max_abs_force": float(np.abs(F).max()), "abs_sum_force": float(np.abs(F.sum(0)).max()),
           "product_gflops": round(flops / dt / 1e9, 1),
           "roofline": {"bound": "alu", "kernel": f"{kernel_name(top)}: P{top['cutoffs'][0]:g} x "
                                                  f"P{top['cutoffs'][1]:g} -> P{top['cutoffs'][2]:g}",
                        "achieved": round(top_tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(top_tf / FP64_PEAK_TFLOPS, 4), "traffic": None,
                        "avg_launch_ms": round(top_ms, 3), "launches": top["launches"]}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = forces_cpu_baseline(s, L, Z, mu)
    print(json.dumps(res), flush=True)


def onsite_coefficients(s, bc):
    """The bc lowest eigenvectors of every on-site H block (input preparation on the host)."""
    import numpy as np
    on = s.H.rows == s.H.cols
    order = np.argsort(s.H.rows[on])
    return np.stack([np.linalg.eigh(blk)[1][:, :bc] for blk in s.H.blocks[on][order]])


def contract_mode(args):
    """The 4096-atom, b = 9 system contracted to 4 on-site support functions per atom
    (bsm_contract) and solved at b = 4, against the 9-orbital solve in the same run."""
    import numpy as np
    import torch
    import synth
    import paper_2205_08941_amd as bsm
    s = synth.si4096_b9()
    bc = 4
    coef = onsite_coefficients(s, bc)
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    cut = s.cutoffs
    P9 = bsm.Pattern(ctx, pos, s.box, cut["S"], 9)
    S9, H9 = bsm.Matrix(P9), bsm.Matrix(P9)
    bsm.fill_blocks(S9, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H9, s.H.rows, s.H.cols, s.H.blocks)
    ct = torch.tensor(coef, dtype=torch.float64, device=ctx.device).contiguous()

    def solve(b, contracted):
        P6 = P9 if b == 9 else bsm.Pattern(ctx, pos, s.box, cut["S"], b)
        Z = bsm.Matrix(bsm.Pattern(ctx, pos, s.box, cut["Z"], b))
        L = bsm.Matrix(bsm.Pattern(ctx, pos, s.box, cut["L"], b))
        out = None
        for rep in range(args.warmup + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            if contracted:
                S, H = bsm.Matrix(P6), bsm.Matrix(P6)
                bsm.contract(S9, ct, S)
                bsm.contract(H9, ct, H)
            else:
                S, H = S9, H9
            if rep == args.warmup:
                ctx.set_profiling(True)
            hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
            lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=args.tol_e)
            r = lnv.solve([(bsm.F64, args.max_lnv, args.tol_e, False)])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            out = dict(seconds=round(dt, 3), E=r["E"], lnv=r["iterations"][0], hotelling=hr.iterations,
                       converged=r["converged"])
        stats = ctx.product_stats()
        ctx.set_profiling(False)
        return out, stats

    full, _ = solve(9, False)
    con, stats = solve(bc, True)
    dE = (con["E"] - full["E"]) / s.natoms
    top = max(stats, key=lambda st: st["ms"])
    top_ms = top["ms"] / top["launches"]
    top_tf = top["flops"] / top["launches"] / (top_ms * 1e-3) / 1e12
    log(f"[contract] 9 orbitals: {full['seconds']:.2f} s, E {full['E']:.6f}; {bc} support functions: "
        f"{con['seconds']:.2f} s, E {con['E']:.6f}, dE/N {dE:.3e} Ha")
    res = {"metric": "s per converged LNV solve, 4096-atom system contracted to 4 on-site support functions",
           "value": con["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
           "ms_per_step": con["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "si4096_b9 contracted to 4 support functions per atom (lowest on-site H "
                                  "eigenvectors), contraction + Hotelling + LNV at b = 4",
                      "natoms": s.natoms, "orbitals_per_atom": 9, "support_functions_per_atom": bc},
           "contracted": con, "full_9_orbitals": full, "dE_per_atom_Ha": dE,
           "speedup_vs_9_orbitals": round(full["seconds"] / con["seconds"], 3),
           "roofline": {"bound": "alu", "kernel": f"{kernel_name(top)}: P{top['cutoffs'][0]:g} x "
                                                  f"P{top['cutoffs'][1]:g} -> P{top['cutoffs'][2]:g}",
                        "achieved": round(top_tf, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(top_tf / FP64_PEAK_TFLOPS, 4), "traffic": None,
                        "avg_launch_ms": round(top_ms, 3), "launches": top["launches"]}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = contract_cpu_baseline(s, coef, con["lnv"])
    print(json.dumps(res), flush=True)


def contract_cpu_baseline(s, coef, lnv_iterations):
    """The oracle on the same contracted workload: contraction, Hotelling and the first
    LNV step timed, the step extrapolated linearly to the GPU run's LNV iteration count."""
    import oracle as O
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    t = time.perf_counter()
    S = O.contract(O.from_blocks(P6, s.b, s.S.rows, s.S.cols, s.S.blocks), coef)
    H = O.contract(O.from_blocks(P6, s.b, s.H.rows, s.H.cols, s.H.blocks), coef)
    Z = O.hotelling_inverse(S, O.create_pattern(s.positions, s.box, s.cutoffs["Z"]), max_iter=100).Z
    st = O.lnv_init(S, H, Z, O.create_pattern(s.positions, s.box, s.cutoffs["L"]), s.n_electrons)
    t_setup = time.perf_counter() - t
    t = time.perf_counter()
    O.lnv_step(st)
    t_step = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    return {"value": round(t_setup + lnv_iterations * t_step, 2), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"the same contracted {s.natoms}-atom workload: contraction + Hotelling + L0 {t_setup:.1f} s "
                      f"and one LNV step {t_step:.1f} s timed, extrapolated to {lnv_iterations} steps"}


def forces_cpu_baseline(s, L, Z, mu):
    """The oracle's force assembly on the same frame, at the GPU-converged L and mu (its own
    chemical-potential step, which needs two more 2 TFLOP products, skipped)."""
    import oracle as O
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    So = O.from_blocks(P6, s.b, s.S.rows, s.S.cols, s.S.blocks)
    Ho = O.from_blocks(P6, s.b, s.H.rows, s.H.cols, s.H.blocks)
    Zo = O.Matrix(O.create_pattern(s.positions, s.box, s.cutoffs["Z"]), s.b, Z.blocks.cpu().numpy())
    PLo = O.create_pattern(s.positions, s.box, s.cutoffs["L"])
    st = O.lnv_init(So, Ho, Zo, PLo, s.n_electrons, L0=O.Matrix(PLo, s.b, L.blocks.cpu().numpy()))
    dS = [O.from_blocks(P6, s.b, d.rows, d.cols, d.blocks) for d in s.dS]
    dH = [O.from_blocks(P6, s.b, d.rows, d.cols, d.blocks) for d in s.dH]
    t = time.perf_counter()
    O.lnv_forces(st, dS, dH, mu=mu)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    return {"value": round(dt, 2), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"the oracle's force assembly (K, Q, row sums) on the same {s.natoms}-atom frame at the "
                      f"GPU-converged L and mu, {dt:.1f} s"}


def invsqrt_cpu_baseline(s, updates):
    """The oracle on the same workload (its P(2 r_Z) pattern build included), timed for
    its start and for 2 updates, and extrapolated linearly to the GPU run's number of
    updates."""
    import oracle as O
    PSo = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    So = O.from_blocks(PSo, s.b, s.S.rows, s.S.cols, s.S.blocks)
    PZo = O.create_pattern(s.positions, s.box, s.cutoffs["Z"])
    t = time.perf_counter()
    O.inverse_sqrt(So, PZo, max_iter=0, tol=0.0)
    t0 = time.perf_counter() - t
    t = time.perf_counter()
    O.inverse_sqrt(So, PZo, max_iter=2, tol=0.0)
    t2 = time.perf_counter() - t
    per = (t2 - t0) / 2
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    return {"value": round(t0 + updates * per, 2), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"the same {len(s.positions)}-atom workload: start {t0:.1f} s and 2 updates {t2 - t0:.1f} s timed, "
                      f"extrapolated to {updates} updates"}


def guess_mode(args):
    """Learned starts: networks trained on plain solves of displaced frames (one solver state
    alive at a time), then held-out frames solved from the learned and from the plain starts."""
    import functools
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    import synth
    nt = args.guess_train_cells
    # the frames' S and H are generated on the host by worker processes, started before this
    # process loads the GPU library or touches the GPU (the workers never do) and kept ahead of
    # the solves
    pool = ProcessPoolExecutor(max_workers=8, mp_context=multiprocessing.get_context("spawn"))
    gen = functools.partial(synth.displaced_frame, (nt, nt, nt), 9)
    futures = [pool.submit(gen, seed=10000 + k) for k in range(args.guess_train)]
    big = pool.submit(functools.partial(synth.displaced_frame, (args.guess_cells,) * 3, 9), seed=20000)
    import torch
    import paper_2205_08941_amd as bsm
    from paper_2205_08941_amd import guess
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    ctx = bsm.Context(0)
    t = time.perf_counter()

    def frame(k):
        return lambda: guess.Frame(ctx, futures[k].result())

    netZ, netL, info = guess.train_guess(ctx, [frame(k) for k in range(args.guess_train)], epochs=30, batch=4096,
                                         lr=1e-3, log=log, sample_frac=args.guess_sample_frac, close_frames=True)
    train_s = time.perf_counter() - t
    gen_s = sum(r["seconds"] for r in info["solves"])
    torch.cuda.empty_cache()
    log(f"[guess] trained in {train_s:.1f} s ({gen_s:.1f} s of solves)")

    def compare(n, seed):
        sy = big.result() if n == args.guess_cells else synth.displaced_frame((n, n, n), 9, seed=seed)
        f = guess.Frame(ctx, sy)
        # a 32768-atom LNV state (~220 GB) and Hotelling's temporaries do not fit together:
        # every solve of such a frame starts by releasing the previous one's state (both the
        # plain and the learned start pay the allocation)
        fresh = f.sys.natoms > 4096
        log(f"[guess] test frame {f.sys.natoms} atoms: plain solve (plans)")
        f.solve_plain(tol_E=args.tol_e, fresh_state=fresh)            # warm-up: patterns, plans
        log(f"[guess] test frame {f.sys.natoms} atoms: plain solve (timed)")
        p = f.solve_plain(tol_E=args.tol_e, fresh_state=fresh)
        log(f"[guess] test frame {f.sys.natoms} atoms: learned start (timed)")
        g = f.solve_guess(netZ, netL, tol_E=args.tol_e, precision=bsm.BF16, fresh_state=fresh)
        log(f"[guess] {f.sys.natoms} atoms: plain {p['hotelling']} + {p['lnv']} in {p['seconds']:.2f} s; learned "
            f"{g['hotelling']} + {g['lnv']} in {g['seconds']:.2f} s; dE {g['E'] - p['E']:.2e} Ha")
        natoms = f.sys.natoms
        both = None
        if natoms <= 4096:
            # the two extensions together: the mixed-precision schedule of the si4096_b9_mixed
            # workload (BF16 matrix-core products until the energy rises, FP32 to |dE| < 1e-4 Ha,
            # 3 FP64 steps), from the plain and from the learned start
            sched = [(bsm.BF16, 30, 0.0, True), (bsm.F32, 60, 1e-4, True), (bsm.F64, 3, 0.0, False)]
            f.solve_plain(tol_E=args.tol_e, schedule=sched)     # warm-up: BF16 plans and scratch
            pm = f.solve_plain(tol_E=args.tol_e, schedule=sched)
            gm = f.solve_guess(netZ, netL, tol_E=args.tol_e, precision=bsm.BF16, schedule=sched)
            both = {"schedule": "BF16 products until E rises, FP32 to |dE| < 1e-4 Ha, 3 FP64 steps",
                    "plain": pm, "learned": gm,
                    "dE_per_atom_Ha_vs_fp64_plain": {"plain": abs(pm["E"] - p["E"]) / natoms,
                                                    "learned": abs(gm["E"] - p["E"]) / natoms},
                    "speedup_vs_fp64_plain": {"plain": round(p["seconds"] / pm["seconds"], 3),
                                              "learned": round(p["seconds"] / gm["seconds"], 3)}}
            log(f"[guess] {natoms} atoms, BF16 -> FP32 -> 3 x FP64: plain {pm['seconds']:.2f} s, learned {gm['seconds']:.2f} s; "
                f"dE/N {both['dE_per_atom_Ha_vs_fp64_plain']['plain']:.2e} / "
                f"{both['dE_per_atom_Ha_vs_fp64_plain']['learned']:.2e} Ha")
        f.close()
        del f
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out = dict(natoms=natoms, plain=p, learned=g, dE_per_atom_Ha=abs(g["E"] - p["E"]) / natoms,
                   speedup_vs_plain=round(p["seconds"] / g["seconds"], 3), state_released_per_solve=fresh)
        if both is not None:
            out["mixed_precision"] = both
        return out

    results = {}
    # the large frame first: it needs nearly all device memory, and the smaller frame's
    # reduced-precision products leave their operand scratch allocated in the context
    for n in sorted({nt, args.guess_cells}, reverse=True):
        try:
            results[8 * n ** 3] = compare(n, 20000)
        except Exception as e:   # e.g. device memory: reported, not hidden
            log(f"[guess] {8 * n ** 3}-atom comparison failed: {e}")
            results[8 * n ** 3] = {"unmeasured": str(e)[:300]}
    pool.shutdown()
    large = results[8 * args.guess_cells ** 3]
    head = large if "learned" in large else results[8 * nt ** 3]
    res = {"metric": f"s per converged LNV solve, {head['natoms']}-atom 9-orb displaced frame, learned start",
           "value": round(head["learned"]["seconds"], 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": round(head["learned"]["seconds"] * 1e3, 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 solve, bf16 network", "data": "synthetic",
           "config": {"workload": f"train on {args.guess_train} {8 * nt ** 3}-atom frames (sigma 0.05 A, "
                                  f"{args.guess_sample_frac:g} of each frame's pair samples), test on "
                                  f"{sorted(results)} atoms", "train_samples_L": info["samples_L"],
                      "train_samples_Z": info["samples_Z"]},
           "tests": {str(k): v for k, v in results.items()},
           "train_seconds": round(train_s, 2), "train_solve_seconds": round(gen_s, 2),
           "train_iterations": [[r["hotelling"], r["lnv"]] for r in info["solves"]],
           "loss_L": [info["losses_L"][0], info["losses_L"][-1]], "loss_Z": [info["losses_Z"][0], info["losses_Z"][-1]]}
    print(json.dumps(res), flush=True)


def cpu_baseline(args):
    """The FP64 oracle timed on a bounded sample: rows of the dominant product class."""
    import numpy as np
    import oracle as O
    import synth
    n = 8 if args.workload == "si4096_b9" else 2
    b = 9 if args.workload == "si4096_b9" else 4
    rx = 16.0 if args.workload == "si4096_b9" else 14.0
    pos, box, _ = synth.diamond_positions((n, n, n))
    P = O.create_pattern(pos, box, rx)
    rng = np.random.default_rng(7)
    X = O.Matrix(P, b, rng.uniform(-1, 1, (P.nnz, b, b)))
    C = O.Matrix(P, b)
    nrows = min(args.cpu_rows, P.natoms)
    tri = O.count_triples(P, P, P)
    flops = 2.0 * b ** 3 * float(tri[:nrows].sum())
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    t0 = time.perf_counter()
    O.multiply_truncate(1.0, X, X, 0.0, C, 0, nrows)     # OpenMP over the rows
    dt = time.perf_counter() - t0
    out = {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"output block-rows 0..{nrows - 1} of {P.natoms} of the {rx:g} A x {rx:g} A -> {rx:g} A "
                     f"product (the class holding ~90% of LNV flops), random FP64 blocks, "
                     f"{flops / 1e9:.1f} GFLOP in {dt:.1f} s",
           "cpu": host_cpu(), "nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)),
           "w_class_product_s_est": round(dt * float(tri.sum()) / float(tri[:nrows].sum()), 2)}
    g = stored_oracle_solve(args.workload)
    if g is not None:
        t = g["timing"]
        out["converged_solve"] = {
            "s": round(t["solve_s"], 1), "lnv_iteration_s_mean": round(t["lnv_s"] / len(t["lnv_step_s"]), 1),
            "hotelling_s": round(t["hotelling_s"], 1), "threads": t["threads"], "cpu": t["cpu"],
            "note": "the full oracle solve of the same system, measured once on the build host "
                    "(tests/golden/make_lnv_golden.py), not on this machine"}
    return out


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stored_oracle_solve(workload: str):
    """The stored FP64 oracle solve of the benchmarked system (tests/golden), if present."""
    path = os.path.join(ROOT, "tests", "golden", f"lnv_{workload}.json")
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


KERNEL_SOURCES = ("paper_2205_08941_amd/csrc/product.hip", "paper_2205_08941_amd/csrc/tiles.h")


def kernel_sources_sha() -> str:
    """First 16 hex digits of the SHA-256 of the product kernels' sources."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def kernel_name(st) -> str:
    b, g, v, p = st["b"], st["rows"], st["variant"], st.get("precision", 0)
    if st.get("products", 1) == 2:
        return f"k_product_ring_pair<{b}, {2 * g}> (2 products sharing an operand, one {g}-row plan)"
    if p == 2 and b == 9 and g in (4, 8) and v in (3, 4):
        return f"k_product_mfma_bf16<{g}>"
    depth = 3 if v == 3 and g <= 4 else 2   # 8-row ring tiles run 1 entry ahead in both ring variants
    name = {0: f"k_product_sgpr<{b}, {g}>", 1: f"k_product_f64_dpp<{b}, {g}>", 2: f"k_product_wg<{b}>",
            3: f"k_product_ring<{b}, {g}, {depth}>", 4: f"k_product_ring<{b}, {g}, 2>",
            5: f"k_product_ring<{b}, {g}, 2, 2 waves>", 6: f"k_product_mfma_f64<{g}>"}.get(v, f"variant {v}")
    return name if p == 0 else name + (" (FP32)" if p == 1 else " (BF16-rounded, FP32)")


def measured_traffic(name: str):
    """HBM bytes per launch of the dominant kernel from the committed counter summary
    profiles/<name>, or None when the kernel sources have changed since the counters
    were taken."""
    try:
        d = json.load(open(os.path.join(ROOT, "profiles", name)))
        if d.get("sources_sha256_16") != kernel_sources_sha():
            return None
        return d["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU domain "
              "decomposition is designed but not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "guess" and args.mode == "solve":
        guess_mode(args)   # starts host worker processes before the GPU library is loaded
        return
    import numpy as np
    import torch
    import synth
    import paper_2205_08941_amd as bsm

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.mode == "product":
        product_mode(args)
        return
    if args.mode == "classes":
        classes_mode(args)
        return
    if args.workload == "batch64":
        batch_mode(args)
        return
    if args.workload == "si64_b4":
        small_mode(args)
        return
    if args.workload == "si4096_b9_mixed":
        mixed_mode(args)
        return
    if args.workload == "invsqrt":
        invsqrt_mode(args)
        return
    if args.workload == "forces":
        forces_mode(args)
        return
    if args.workload == "contract":
        contract_mode(args)
        return
    s = synth.si4096_b9() if args.workload == "si4096_b9" else synth.si64_b4()
    cut = s.cutoffs
    ctx = bsm.Context(0)
    dev = ctx.device
    t0 = time.perf_counter()
    pos = torch.tensor(s.positions, dtype=torch.float64, device=dev)
    PS = bsm.Pattern(ctx, pos, s.box, cut["S"], s.b)
    PZ = bsm.Pattern(ctx, pos, s.box, cut["Z"], s.b)
    PL = bsm.Pattern(ctx, pos, s.box, cut["L"], s.b)
    torch.cuda.synchronize()
    pattern_s = time.perf_counter() - t0
    S, H, Z, L = bsm.Matrix(PS), bsm.Matrix(PS), bsm.Matrix(PZ), bsm.Matrix(PL)
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)
    torch.cuda.synchronize()
    log(f"[setup] {s.name}: {s.natoms} atoms, b={s.b}, patterns {pattern_s:.3f} s")

    t0 = time.perf_counter()
    hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
    lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=args.tol_e, init_from_z=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[setup] derived patterns + plans + first Hotelling: {setup_s:.2f} s")

    def solve(tag):
        t = time.perf_counter()
        hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
        flops = hr.product_flops
        flops += lnv.reset(init_from_z=True)
        it, res = 0, None
        for it in range(1, args.max_lnv + 1):
            res = lnv.step()
            flops += res.product_flops
            if res.status != 0:
                raise RuntimeError(f"LNV step {it} failed with status {res.status}")
            if it % 5 == 0 or res.converged:
                log(f"[{tag}] LNV {it:3d}  E={res.E:.10f}  dE={res.dE:+.3e}  N={res.N:.8f}  "
                    f"{time.perf_counter() - t:.1f} s")
            if res.converged:
                break
        torch.cuda.synchronize()
        if res is None or not res.converged:
            raise RuntimeError(f"[{tag}] LNV did not converge to |dE| < {args.tol_e:g} Ha in {it} iterations")
        return dict(seconds=time.perf_counter() - t, flops=flops, lnv_iterations=it,
                    hotelling_iterations=hr.iterations, E=res.E, N=res.N, converged=res.converged)

    warm = []
    for w in range(args.warmup):
        r = solve(f"warmup {w}")
        warm.append(r)
        log(f"[warmup {w}] {r['seconds']:.2f} s, {r['lnv_iterations']} LNV iterations")

    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [solve(f"step {k}") for k in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = ctx.product_stats()
    ctx.set_profiling(False)

    flops = sum(r["flops"] for r in runs)
    value = flops / elapsed / 1e9
    top = stats[0]
    per_launch_flops = top["flops"] / top["launches"]
    avg_ms = top["ms"] / top["launches"]
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12
    prod_ms = sum(st["ms"] for st in stats)
    prod_flops = sum(st["flops"] for st in stats)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: converged Hotelling + LNV solve", "natoms": s.natoms,
                   "orbitals_per_atom": s.b, "cutoffs_A": cut, "tol_E_Ha": args.tol_e, "seed": s.seed},
        "s_per_solve": round(elapsed / args.steps, 3),
        "lnv_iterations": runs[-1]["lnv_iterations"],
        "hotelling_iterations": runs[-1]["hotelling_iterations"],
        "E_Ha": runs[-1]["E"],
        "E_per_atom_Ha": runs[-1]["E"] / s.natoms,
        "converged": runs[-1]["converged"],
        "product_device_gflops": round(prod_flops / (prod_ms * 1e-3) / 1e9, 2),
        "product_share_of_time": round(prod_ms * 1e-3 / elapsed, 3),
        "pattern_build_s": round(pattern_s, 3),
        # outside the timed steps: derived patterns, Hotelling plans and the first Hotelling;
        # then the first solve, which also builds the LNV plans
        "setup_s": round(setup_s, 3),
        "first_solve_s": round(warm[0]["seconds"], 3) if warm else None,
        "roofline": {
            "bound": "alu",
            "kernel": f"{kernel_name(top)}: P{top['cutoffs'][0]:g} x P{top['cutoffs'][1]:g} -> "
                      f"P{top['cutoffs'][2]:g}",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": (measured_traffic("k_product_pair_si4096_b9_traffic.json" if top.get("products", 1) == 2
                                         else "k_product_si4096_b9_traffic.json") if s.b == 9 else None),
            "avg_launch_ms": round(avg_ms, 3),
            "launches": top["launches"],
            "flops_per_launch": per_launch_flops,
        },
        "product_classes": [
            {"cutoffs": st["cutoffs"], "kernel": kernel_name(st), "launches": st["launches"],
             "tflops": round(st["flops"] / (st["ms"] * 1e-3) / 1e12, 3), "ms": round(st["ms"], 2)}
            for st in stats],
    }
    g = stored_oracle_solve(args.workload)
    if g is not None:
        Eo = g["lnv"]["E_final"]
        out["oracle"] = {"E_Ha": Eo, "abs_dE_Ha": abs(runs[-1]["E"] - Eo),
                         "rel_dE": abs(runs[-1]["E"] - Eo) / abs(Eo),
                         "lnv_iterations": len(g["lnv"]["iterations"]),
                         "hotelling_iterations": g["hotelling"]["iterations"],
                         "source": f"tests/golden/lnv_{args.workload}.json (FP64 CPU oracle, same seeded system)"}
        log(f"[oracle] E = {Eo:.10f} Ha, |dE| = {out['oracle']['abs_dE_Ha']:.3e} Ha")
    if not args.no_cpu_baseline:
        log("[cpu] timing the oracle on a sample of the dominant product")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
