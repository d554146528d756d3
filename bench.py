#!/usr/bin/env python3
"""Benchmark of the per-rank, column-based SpMM path on one MI355X.

A step is one pass of the whole path over the workload: select (the
selection kernels, re-run on the device), pack_B, spmm (all column blocks in
one launch) and spmm_backward (the gradients autograd needs: A^T dY
written into the selected rows of a zero-filled dB, and dvals),
captured once in a HIP graph and replayed.  Inputs are resident in HBM
before timing starts.  The metric counts 2*nnz*N flops for each of the three
products of a step (Y, dBpacked, dvals).

Default workload: panel 0 of a 2^24-vertex R-MAT (a/b/c/d .57/.19/.19/.05,
32 samples per row) split into P = 128 column blocks, N = 128, float32.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME] [--N 128]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_VECTOR_PEAK_GFLOPS = 157300.0  # MI355X FP32 vector, published (no MFMA on this path)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="rmat24_p128_panel0",
                    choices=["rmat24_p128_panel0", "er24_p128_panel0", "rmat12_ef16", "rmat22_ef64",
                             "gcn_rmat21_ef25"])
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the per-block, bf16, flushed, N-sweep and autograd extras")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-sample-rows", type=int, default=None)
    return ap.parse_args()


def make_workload(name, dev):
    import synth

    if name == "rmat24_p128_panel0":
        return synth.config2(device=dev), 128
    if name == "er24_p128_panel0":
        return synth.config3_er(device=dev), 128
    if name == "rmat12_ef16":
        return synth.config1(device=dev), 32
    if name == "rmat22_ef64":
        return synth.config4(device=dev), 256
    if name == "gcn_rmat21_ef25":
        return synth.config5(device=dev), 128
    raise KeyError(name)


def src_hash():
    """Short hash of what fixes the kernels' behaviour: every library source
    and header (the hash stamped into the library) and the tuning table."""
    from paper_2512_20178_amd import build

    h = hashlib.sha256(build.source_hash().encode())
    with open(os.path.join(ROOT, "paper_2512_20178_amd", "tuning_mi355x.txt"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: the per-rank path has no collectives; "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    # the committed tuning table (autotuner results on MI355X) unless overridden
    os.environ.setdefault("SHIRO_TUNE_CACHE", os.path.join(ROOT, "paper_2512_20178_amd", "tuning_mi355x.txt"))
    import paper_2512_20178_amd as shiro
    import synth

    shiro._lib.check_build()  # a library built from other sources would time other kernels
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    A, N0 = make_workload(args.workload, dev)
    N = args.N or N0
    tdt = torch.float32 if args.dtype == "f32" else torch.bfloat16
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev).to(tdt)
    torch.cuda.synchronize()
    log(f"workload {args.workload}: n={A.n_rows} nnz={A.nnz} P={A.P} N={N} generated in {time.perf_counter() - t0:.1f}s")

    # ---- setup: partition + select (pattern-only, reused by every step) ----
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan = shiro.partition(A.row_ptr, A.col, A.n_rows, A.n_cols, A.P, A.p)
    t_part = time.perf_counter() - t
    t = time.perf_counter()
    U, Uq = shiro.select_rows(plan)
    t_sel = time.perf_counter() - t
    info = plan.info()
    M, nnz = info["rows"], info["nnz"]
    G = synth.dense(M, N, 0, synth.STREAM_DY, device=dev).to(tdt)
    log(f"plan: rows={M} nnz={nnz} U={U}; partition {t_part * 1e3:.1f} ms, select {t_sel * 1e3:.1f} ms")

    if not args.no_autotune:
        t = time.perf_counter()
        shiro.autotune(plan, N, tdt, ops=("spmm", "backward"))
        log(f"autotune {time.perf_counter() - t:.1f}s: spmm {shiro.get_tuning(plan, 'spmm', N, tdt)} "
            f"spmm_t {shiro.get_tuning(plan, 'spmm_t', N, tdt)} sddmm {shiro.get_tuning(plan, 'sddmm', N, tdt)}")
    shiro.prepare(plan, N, tdt, ops=("spmm", "backward", "per_block"))

    vals = A.vals
    Bp = torch.empty(U, N, dtype=tdt, device=dev)
    Y = torch.empty(M, N, dtype=tdt, device=dev)
    dB = torch.zeros(A.n_cols, N, dtype=tdt, device=dev)
    dvals = torch.zeros(A.nnz, dtype=torch.float32, device=dev)

    def step():
        shiro.refresh_selection(plan)
        shiro.pack_B(plan, B, out=Bp)
        shiro.spmm(plan, vals, Bp, out=Y)
        shiro.spmm_backward(plan, vals, G, Bp, dB=dB, dvals=dvals, dB_overwrite=True)

    # ---- capture one step as a HIP graph ----
    cs = torch.cuda.Stream()
    torch.cuda.synchronize()
    with plan.capture(cs) as gid_holder:
        step()
    gid = gid_holder[0]
    torch.cuda.synchronize()

    with torch.cuda.stream(cs):
        for _ in range(args.warmup):
            plan.replay(gid, stream=cs)
        cs.synchronize()
        torch.cuda.synchronize()  # barrier (single rank) + device sync
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        w0 = time.perf_counter()
        evs[0].record(cs)
        for i in range(args.steps):
            plan.replay(gid, stream=cs)
            evs[i + 1].record(cs)
        cs.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    per_step = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    flops_step = 3 * 2.0 * nnz * N
    gflops = flops_step / (ms_step * 1e-3) / 1e9
    log(f"step {ms_step * 1e3:.1f} us (wall {wall / args.steps * 1e6:.1f} us) -> {gflops:.1f} GFLOP/s")

    # ---- sampled outputs of the timed step (the oracle checks them in the
    # CPU leg): rows of Y, columns of dB and the value gradients of those rows
    samples = sample_outputs(A, info, np, torch)
    step_out = {tdt: take_samples(samples, Y, dB, dvals)}
    bnz = shiro.block_nnz(plan).cpu().numpy()

    # ---- per-kernel durations on the launch stream (HIP events) ----
    sz = 4 if tdt == torch.float32 else 2
    rp = A.row_ptr[info["row_begin"]: info["row_begin"] + M + 1]
    R_nonempty = int((rp[1:] != rp[:-1]).sum().item())
    # algorithmic bytes: every B / Bpacked / dY row read once, every output row
    # written once, 4 bytes per index and per value touched
    alg = {
        "select": 8 * nnz + 4 * U + 2 * ((A.n_cols + 7) // 8),
        "pack_B": 2 * U * N * sz,
        "spmm": 8 * (M + 1) + 8 * nnz + U * N * sz + M * N * sz,
        # A^T dY written into the U selected rows of dB, and dvals, in one
        # pass over the transposed pattern: row pointers, row ids, CSR
        # positions, values read, dvals written; dY rows and Bpacked read once
        "backward": 8 * (U + 1) + 16 * nnz + R_nonempty * N * sz + U * N * sz + U * N * sz,
    }
    ops = {
        "select": lambda: shiro.refresh_selection(plan),
        "pack_B": lambda: shiro.pack_B(plan, B, out=Bp),
        "spmm": lambda: shiro.spmm(plan, vals, Bp, out=Y),
        "backward": lambda: shiro.spmm_backward(plan, vals, G, Bp, dB=dB, dvals=dvals, dB_overwrite=True),
    }
    reps = 20
    kern_us, kern_stats, kern_flushed = {}, {}, {}
    # a 1 GiB write between calls evicts L2 and the MALL (for the flushed timings)
    scratch = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    s = torch.cuda.current_stream()
    for name, fn in ops.items():
        fn()
        torch.cuda.synchronize()
        evs_op = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs_op:
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        d = np.array([a.elapsed_time(b) for a, b in evs_op]) * 1e3
        kern_us[name] = float(d.mean())
        kern_stats[name] = {"mean": round(float(d.mean()), 2), "median": round(float(np.median(d)), 2),
                            "min": round(float(d.min()), 2)}
        if not args.no_extras:
            evs_op = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
            for a, b in evs_op:
                scratch.fill_(1.0)
                a.record(s)
                fn()
                b.record(s)
            torch.cuda.synchronize()
            kern_flushed[name] = round(float(np.mean([a.elapsed_time(b) for a, b in evs_op]) * 1e3), 2)
    del scratch
    log("per-call us: " + ", ".join(f"{k}={v:.1f}" for k, v in kern_us.items()))
    alg_step = sum(alg.values())

    dom = max(("pack_B", "spmm", "backward"), key=lambda k: kern_us[k])
    achieved = alg[dom] / (kern_us[dom] * 1e-6) / 1e9
    traffic = None
    pmc_path = os.path.join(ROOT, "profiles", f"pmc_{dom}_{args.workload}_N{N}_{args.dtype}.json")
    if os.path.exists(pmc_path):
        with open(pmc_path) as f:
            pmc = json.load(f)
        # counters taken on another build of these kernels or another tuning are stale
        if pmc.get("src_hash") == src_hash():
            traffic = pmc.get("hbm_bytes_per_launch")
    # the product kernel each op ran, from the plan's tuning (group_rows)
    kname = {0: "k_spmm", 1: "k_spmm_grp", 2: "k_spmm_flat", 3: "k_spmm_win"}
    kf = kname[shiro.get_tuning(plan, "spmm", N, tdt)["group_rows"]]
    tb = shiro.get_tuning(plan, "spmm_t", N, tdt)
    kb = kname[tb["group_rows"]]
    # the fused FP32 transposed walk with one nonzero per step and lane groups
    # of 16 or more runs as the 8-wavefronts-per-SIMD build of that walk
    vec = 4 if N % 4 == 0 else 1
    lanes = 64
    while lanes > 8 and lanes // 2 >= -(-N // vec):
        lanes //= 2
    if tb["group_rows"] == 3 and tb["unroll"] == 1 and tdt == torch.float32 and lanes >= 16:
        kb = "k_spmm_win_w8"
    kernels_of = {"pack_B": "k_pack", "spmm": f"{kf} + k_fixup",
                  "backward": f"k_gather_vals + {kb}<dot> + k_fixup + k_scatter_vals"}
    roofline = {"bound": "hbm", "kernel": f"{dom} ({kernels_of[dom]})", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": int(alg[dom]), "duration_us": round(kern_us[dom], 2)}
    if traffic:
        # the rate at which the op moves the bytes the counters saw, beside the
        # device-copy rate measured in the same run (copy_GBs)
        roofline["traffic_rate_GBs"] = round(traffic / (kern_us[dom] * 1e-6) / 1e9, 1)

    out = {
        "metric": "local SpMM GFLOP/s & % HBM peak; BF16/batched/fwd+bwd vs plain FP32",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": A.n_rows, "P": A.P, "p": A.p, "rows": M, "nnz": nnz,
                   "U": U, "N": N, "step": "select+pack_B+spmm+spmm_backward(dB rows, dvals)"},
        "roofline": roofline,
        "step_hbm_frac": round(alg_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        # the flop side of the roofline: the whole step's 2*nnz*N per product
        # against the FP32 vector peak (the large workloads reach 5-12 flop/B)
        "step_fp32_vector_frac": round(gflops / FP32_VECTOR_PEAK_GFLOPS, 4),
        "step_us_stats": {"mean": round(ms_step * 1e3, 2), "median": round(float(np.median(per_step)) * 1e3, 2),
                          "min": round(float(np.min(per_step)) * 1e3, 2)},
        "kernels_us": {k: round(v, 2) for k, v in kern_us.items()},
        "kernels_us_stats": kern_stats,
        "kernels_hbm_frac": {k: round(alg[k] / (kern_us[k] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) for k in kern_us},
        "algorithmic_bytes": {k: int(v) for k, v in alg.items()},
        "setup_ms": {"partition": round(t_part * 1e3, 2), "select_rows": round(t_sel * 1e3, 2)},
        # per-block sizes: |Cols(A^(p,q))| and nonzeros of each column block
        "blocks": {"P": A.P, "U_q": spread(np, Uq), "nnz_q": spread(np, bnz),
                   "nnz_q_lt_1k": int((bnz < 1000).sum()), "nnz_q_gt_200k": int((bnz > 200000).sum())},
    }

    # achievable bandwidth of a plain device copy (1 GiB read + 1 GiB written)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(1 if args.calib_copy else 5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    if kern_flushed:
        out["kernels_us_flushed"] = kern_flushed
    out["copy_GBs"] = round(2 * src.numel() * 4 / (a.elapsed_time(b) / (1 if args.calib_copy else 5) * 1e-3) / 1e9, 1)
    del src, dst

    if not args.no_extras:
        # batched (one launch, row-merged) vs one launch per column block
        def timed(fn, n=5):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(n):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / n * 1e3

        t_pb = timed(lambda: shiro.spmm(plan, vals, Bp, out=Y, mode="per_block"))
        out["per_block_spmm_us"] = round(t_pb, 2)
        out["batched_speedup"] = round(t_pb / kern_us["spmm"], 3)
        fwd_us = kern_us["select"] + kern_us["pack_B"] + kern_us["spmm"]
        out["fwd_gflops"] = round(2.0 * nnz * N / (fwd_us * 1e-6) / 1e9, 2)
        out["fwd_bwd_over_fwd"] = round(ms_step * 1e3 / fwd_us, 3)
        if tdt == torch.float32:
            # same step with bfloat16 storage (B, Y, dY, dBpacked, dB), float32 arithmetic
            Bh = B.to(torch.bfloat16)
            Gh = G.to(torch.bfloat16)
            shiro.prepare(plan, N, torch.bfloat16, ops=("spmm", "backward"))
            Bph = torch.empty(U, N, dtype=torch.bfloat16, device=dev)
            Yh = torch.empty(M, N, dtype=torch.bfloat16, device=dev)
            dBh = torch.zeros(A.n_cols, N, dtype=torch.bfloat16, device=dev)

            def step_bf16():
                shiro.refresh_selection(plan)
                shiro.pack_B(plan, Bh, out=Bph)
                shiro.spmm(plan, vals, Bph, out=Yh)
                shiro.spmm_backward(plan, vals, Gh, Bph, dB=dBh, dvals=dvals, dB_overwrite=True)

            if not args.no_autotune:
                shiro.autotune(plan, N, torch.bfloat16, ops=("spmm", "backward"))
            t_bf = timed(step_bf16)
            step_out[torch.bfloat16] = take_samples(samples, Yh, dBh, dvals)
            out["bf16_step_us"] = round(t_bf, 2)
            out["bf16_speedup"] = round(ms_step * 1e3 / t_bf, 3)
            out["bf16_kernels_us"] = {
                "pack_B": round(timed(lambda: shiro.pack_B(plan, Bh, out=Bph)), 2),
                "spmm": round(timed(lambda: shiro.spmm(plan, vals, Bph, out=Yh)), 2),
                "backward": round(timed(lambda: shiro.spmm_backward(plan, vals, Gh, Bph, dB=dBh, dvals=dvals, dB_overwrite=True)), 2),
            }
            del Bh, Gh, Bph, Yh, dBh
        # the row-based scheme on the same panel: Rows(A^(p,q)) per block, the
        # owner's partial C rows and their sum into the panel (volumes of
        # Sec. 3.1 Eq. V_row against Eq. V_col; off-diagonal blocks apart,
        # since the paper uses local rows for the diagonal block)
        t = time.perf_counter()
        R, Rq = shiro.select_c_rows(plan)
        t_rsel = time.perf_counter() - t
        if not args.no_autotune:
            shiro.autotune(plan, N, tdt, ops=("row_based",))
        shiro.prepare(plan, N, tdt, ops=("row_based",))
        Cp = torch.empty(R, N, dtype=tdt, device=dev)
        t_pc = timed(lambda: shiro.partial_c(plan, vals, B, R, out=Cp))
        t_ag = timed(lambda: shiro.aggregate_c(plan, Cp, out=Y))
        out["row_based"] = {"R": R, "U": U, "R_offdiag": R - Rq[A.p], "U_offdiag": U - Uq[A.p],
                            "v_row_bytes": R * N * sz, "v_col_bytes": U * N * sz,
                            "setup_ms": round(t_rsel * 1e3, 2), "partial_c_us": round(t_pc, 2),
                            "aggregate_c_us": round(t_ag, 2), "forward_us": round(t_pc + t_ag, 2)}
        log(f"row-based: {out['row_based']}")
        del Cp
        # the joint row-column strategy (Sec. 5): per-block minimum covers
        # planned on the host, then the column-based part through select /
        # pack / spmm and the row-based part through partial / sum (volumes
        # of Sec. 5.4 Eq. V_joint against V_col and V_row, off-diagonal)
        out["joint"] = None  # one block: nothing off the diagonal to plan
        if A.P > 1:
            t = time.perf_counter()
            js = shiro.JointSpMM(A.row_ptr, A.col, A.n_rows, A.n_cols, A.P, A.p)
            t_plan = time.perf_counter() - t
            st = js.stats.numpy()
            off = np.arange(A.P) != A.p
            mu = int(st[off, 0].sum())
            if not args.no_autotune:
                shiro.autotune(js.col_plan, N, tdt, ops=("spmm",))
                shiro.autotune(js.row_plan, N, tdt, ops=("row_based",))
            js.prepare(N, tdt)
            Yj = torch.empty(M, N, dtype=tdt, device=dev)
            Bpj = torch.empty(js.U, N, dtype=tdt, device=dev)
            Cpj = torch.empty(js.R, N, dtype=tdt, device=dev)
            t_joint = timed(lambda: js.forward(vals, B, out=Yj, Bp=Bpj, Cp=Cpj))
            rows_off, cols_off = int(st[off, 1].sum()), int(st[off, 2].sum())
            out["joint"] = {"mu_offdiag": mu, "rows_offdiag": rows_off, "cols_offdiag": cols_off,
                            "red_col": round(1 - mu / cols_off, 4) if cols_off else None,
                            "red_row": round(1 - mu / rows_off, 4) if rows_off else None,
                            "v_joint_bytes": mu * N * sz, "plan_s": round(t_plan, 2),
                            "col_part_nnz": int(js.col_plan.info()["nnz"]),
                            "row_part_nnz": int(js.row_plan.info()["nnz"]), "forward_us": round(t_joint, 2)}
            log(f"joint: {out['joint']}")
            del js, Yj, Bpj, Cpj
        if tdt == torch.bfloat16:
            # BF16 storage in, FP32 output
            Y32 = torch.empty(M, N, dtype=torch.float32, device=dev)
            out["spmm_bf16_to_f32_us"] = round(timed(lambda: shiro.spmm(plan, vals, Bp, out=Y32)), 2)
            del Y32
        if args.workload in ("rmat24_p128_panel0", "er24_p128_panel0") and args.N is None:
            out["n_sweep"] = n_sweep(shiro, synth, plan, A, vals, U, M, tdt, dev, timed, args)
        if args.workload == "rmat24_p128_panel0" and args.N is None:
            # the batched form's contrast case: the Erdos-Renyi panel, whose
            # blocks are all about the same size
            Ae = synth.config3_er(device=dev)
            pe = shiro.partition(Ae.row_ptr, Ae.col, Ae.n_rows, Ae.n_cols, Ae.P, Ae.p)
            Ue, _ = shiro.select_rows(pe)
            out["n_sweep_er24_p128_panel0"] = n_sweep(shiro, synth, pe, Ae, Ae.vals, Ue, pe.info()["rows"], tdt, dev,
                                                      timed, args)
            del pe, Ae
            torch.cuda.empty_cache()
        # the same layer through the autograd Function (allocates and zero-fills
        # dB and dvals on every backward, as autograd does)
        vp = vals.detach().clone().requires_grad_(True)
        Bg = B.detach().clone().requires_grad_(True)

        def autograd_step():
            Yg = shiro.shiro_spmm(plan, vp, Bg)
            Yg.backward(G)
            vp.grad = None
            Bg.grad = None

        out["autograd_step_us"] = round(timed(autograd_step, n=3), 2)
        del vp, Bg
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, G, N, args, out)
        # error of each output against the FP64 oracle, beside the BF16 speedup
        out["precision"] = precision_report(A, B, G, samples, step_out)
        if not args.no_extras and args.workload == "rmat24_p128_panel0" and tdt == torch.float32:
            del B, G
            torch.cuda.empty_cache()
            out["precision_form"] = precision_form(shiro, synth, args, dev)
            out["differentiation_form"] = differentiation_form(shiro, synth, args, dev)
            out["plain_form"] = plain_form(shiro, synth, args, dev)

    print(json.dumps(out), flush=True)


def precision_form(shiro, synth, args, dev):
    """The precision form on its own matrix: the 2^22 R-MAT (250M nonzeros, one
    block) at N = 256, the step (select, pack, spmm, backward with dB rows and
    dvals) with float32 and with bfloat16 storage, the BF16 speedup, and the
    error of each output against the FP64 oracle on the float32 inputs."""
    import numpy as np
    import torch

    A = synth.config4(device=dev)
    N = 256
    plan = shiro.partition(A.row_ptr, A.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    info = plan.info()
    M = info["rows"]
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev)
    G = synth.dense(M, N, 0, synth.STREAM_DY, device=dev)
    smp = sample_outputs(A, info, np, torch)
    res = {"workload": "rmat22_ef64", "N": N, "nnz": int(A.nnz), "U": int(U)}
    outs = {}
    for dt in (torch.float32, torch.bfloat16):
        if not args.no_autotune:
            shiro.autotune(plan, N, dt, ops=("spmm", "backward"))
        shiro.prepare(plan, N, dt, ops=("spmm", "backward"))
        Bd, Gd = B.to(dt), G.to(dt)
        Bp = torch.empty(U, N, dtype=dt, device=dev)
        Y = torch.empty(M, N, dtype=dt, device=dev)
        dB = torch.zeros(A.n_cols, N, dtype=dt, device=dev)
        dv = torch.zeros(A.nnz, device=dev)

        def stp():
            shiro.refresh_selection(plan)
            shiro.pack_B(plan, Bd, out=Bp)
            shiro.spmm(plan, A.vals, Bp, out=Y)
            shiro.spmm_backward(plan, A.vals, Gd, Bp, dB=dB, dvals=dv, dB_overwrite=True)

        stp()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            stp()
        b.record()
        torch.cuda.synchronize()
        res["bf16_step_us" if dt == torch.bfloat16 else "f32_step_us"] = round(a.elapsed_time(b) / 3 * 1e3, 1)
        outs[dt] = take_samples(smp, Y, dB, dv)
        del Bd, Gd, Bp, Y, dB, dv
        torch.cuda.empty_cache()
    res["bf16_speedup"] = round(res["f32_step_us"] / res["bf16_step_us"], 3)
    res["precision"] = precision_report(A, B, G, smp, outs)
    log(f"precision form: {res}")
    return res


def plain_form(shiro, synth, args, dev):
    """The plain single-block case: the 4096-vertex R-MAT (one block) at
    N = 32, the step's time, its selection against the oracle's unique-column
    set (bit for bit) and the error of each output against the FP64 oracle."""
    import numpy as np
    import torch

    import oracle

    A = synth.config1(device=dev)
    N = 32
    plan = shiro.partition(A.row_ptr, A.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    info = plan.info()
    M = info["rows"]
    if not args.no_autotune:
        shiro.autotune(plan, N, torch.float32, ops=("spmm", "backward"))
    shiro.prepare(plan, N, torch.float32, ops=("spmm", "backward"))
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev)
    G = synth.dense(M, N, 0, synth.STREAM_DY, device=dev)
    Bp = torch.empty(U, N, device=dev)
    Y = torch.empty(M, N, device=dev)
    dB = torch.zeros(A.n_cols, N, device=dev)
    dv = torch.zeros(A.nnz, device=dev)

    def stp():
        shiro.refresh_selection(plan)
        shiro.pack_B(plan, B, out=Bp)
        shiro.spmm(plan, A.vals, Bp, out=Y)
        shiro.spmm_backward(plan, A.vals, G, Bp, dB=dB, dvals=dv, dB_overwrite=True)

    stp()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(20):
        stp()
    b.record()
    torch.cuda.synchronize()
    uc = shiro.selection(plan)[0].cpu().numpy()
    Ac = oracle.Csr.from_synth(A.to(torch.device("cpu")))
    smp = sample_outputs(A, info, np, torch)
    res = {"workload": "rmat12_ef16", "N": N, "nnz": int(A.nnz), "U": int(U),
           "step_us": round(a.elapsed_time(b) / 20 * 1e3, 1),
           "unique_cols_match_oracle": bool(np.array_equal(uc, oracle.select(Ac)[0])),
           "precision": precision_report(A, B, G, smp, {torch.float32: take_samples(smp, Y, dB, dv)})}
    log(f"plain form: {res}")
    return res


def differentiation_form(shiro, synth, args, dev):
    """The differentiation form on its own matrix: the GCN layer (symmetrised,
    normalised 2^21 R-MAT, N = 128) through the autograd Function, forward and
    backward (dB and dvals), timed as autograd runs it (it allocates and
    zero-fills the gradients) and as library calls, with the error of Y, dB
    and dvals against the FP64 oracle on sampled outputs."""
    import numpy as np
    import torch

    A = synth.config5(device=dev)
    N = 128
    plan = shiro.partition(A.row_ptr, A.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    info = plan.info()
    M = info["rows"]
    if not args.no_autotune:
        shiro.autotune(plan, N, torch.float32, ops=("spmm", "backward"))
    shiro.prepare(plan, N, torch.float32, ops=("spmm", "backward"))
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev)
    G = synth.dense(M, N, 0, synth.STREAM_DY, device=dev)
    smp = sample_outputs(A, info, np, torch)
    vp = A.vals.clone().requires_grad_(True)
    Bg = B.clone().requires_grad_(True)
    res = {"workload": "gcn_rmat21_ef25", "N": N, "nnz": int(A.nnz), "U": int(U)}

    def autograd_step():
        vp.grad = None
        Bg.grad = None
        Y = shiro.shiro_spmm(plan, vp, Bg)
        Y.backward(G)
        return Y

    def timed(fn, n=3):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return round(a.elapsed_time(b) / n * 1e3, 1)

    res["autograd_step_us"] = timed(autograd_step)
    Y = autograd_step()
    torch.cuda.synchronize()
    samples = take_samples(smp, Y.detach(), Bg.grad, vp.grad)
    del Y
    Bp = torch.empty(U, N, device=dev)
    Yl = torch.empty(M, N, device=dev)
    dB = torch.zeros(A.n_cols, N, device=dev)
    dv = torch.zeros(A.nnz, device=dev)

    def library_step():
        shiro.refresh_selection(plan)
        shiro.pack_B(plan, B, out=Bp)
        shiro.spmm(plan, A.vals, Bp, out=Yl)
        shiro.spmm_backward(plan, A.vals, G, Bp, dB=dB, dvals=dv, dB_overwrite=True)

    res["library_step_us"] = timed(library_step)
    del Bp, Yl, dB, dv, vp, Bg
    torch.cuda.empty_cache()
    res["precision"] = precision_report(A, B, G, smp, {torch.float32: samples})
    log(f"differentiation form: {res}")
    return res


def n_sweep(shiro, synth, plan, A, vals, U, M, tdt, dev, timed, args):
    """Dense widths N = 32 .. 256 on the same panel: pack, batched spmm and
    the per-block baseline, and the whole step (library calls, no graph)."""
    import torch

    res = {}
    for n in (32, 64, 128, 256):
        Bn = synth.dense(A.n_cols, n, 0, synth.STREAM_B, device=dev).to(tdt)
        Gn = synth.dense(M, n, 0, synth.STREAM_DY, device=dev).to(tdt)
        if not args.no_autotune:
            shiro.autotune(plan, n, tdt, ops=("spmm", "backward"))
        shiro.prepare(plan, n, tdt, ops=("spmm", "backward", "per_block"))
        Bpn = torch.empty(U, n, dtype=tdt, device=dev)
        Yn = torch.empty(M, n, dtype=tdt, device=dev)
        dBn = torch.zeros(A.n_cols, n, dtype=tdt, device=dev)
        dvn = torch.zeros(A.nnz, dtype=torch.float32, device=dev)

        def stp():
            shiro.refresh_selection(plan)
            shiro.pack_B(plan, Bn, out=Bpn)
            shiro.spmm(plan, vals, Bpn, out=Yn)
            shiro.spmm_backward(plan, vals, Gn, Bpn, dB=dBn, dvals=dvn, dB_overwrite=True)

        t_step = timed(stp)
        t_b = timed(lambda: shiro.spmm(plan, vals, Bpn, out=Yn))
        t_pb = timed(lambda: shiro.spmm(plan, vals, Bpn, out=Yn, mode="per_block"))
        res[str(n)] = {"step_us": round(t_step, 2),
                       "gflops": round(3 * 2.0 * int(plan.info()["nnz"]) * n / (t_step * 1e-6) / 1e9, 1),
                       "pack_B_us": round(timed(lambda: shiro.pack_B(plan, Bn, out=Bpn)), 2),
                       "spmm_batched_us": round(t_b, 2), "spmm_per_block_us": round(t_pb, 2),
                       "batched_speedup": round(t_pb / t_b, 2)}
        log(f"N={n}: {res[str(n)]}")
        del Bn, Gn, Bpn, Yn, dBn, dvn
        torch.cuda.empty_cache()
    return res


def spread(np, x):
    x = np.asarray(x, np.int64)
    return {"min": int(x.min()), "median": int(np.median(x)), "max": int(x.max())} if x.size else {}


def sample_outputs(A, info, np, torch):
    """Host indices of the outputs the precision report checks: 64 rows of
    the panel (evenly spaced and the longest), 64 columns (those of random
    nonzeros of the panel and the busiest one) and the panel nonzeros of the
    sampled rows."""
    rp = A.row_ptr.cpu().numpy()
    col = A.col.cpu().numpy()
    rb, M = info["row_begin"], info["rows"]
    prp = rp[rb:rb + M + 1]
    lens = np.diff(prp)
    rows = np.unique(np.concatenate([np.linspace(0, M - 1, 56).astype(np.int64), np.argsort(lens)[-8:]]))
    nz0, nz1 = prp[0], prp[-1]
    rng = np.random.default_rng(11)
    pcol = col[nz0:nz1]
    busiest = np.argmax(np.bincount(pcol, minlength=A.n_cols)) if pcol.size else 0
    cols = np.unique(np.concatenate([pcol[rng.integers(0, max(pcol.size, 1), 63)] if pcol.size else [], [busiest]]))
    ks = np.concatenate([np.arange(prp[r], prp[r + 1]) for r in rows]) if rows.size else np.zeros(0, np.int64)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).long().to(A.col.device)
    return {"rows": rows, "cols": cols.astype(np.int64), "ks": ks.astype(np.int64), "rp": rp, "col": col,
            "rows_t": t(rows), "cols_t": t(cols), "ks_t": t(ks)}


def take_samples(smp, Y, dB, dvals):
    return (Y.index_select(0, smp["rows_t"]).float().cpu().numpy(),
            dB.index_select(0, smp["cols_t"]).float().cpu().numpy(),
            dvals.index_select(0, smp["ks_t"]).cpu().numpy())


def precision_report(A, B, G, smp, step_out):
    """Max relative error (componentwise, |A||B|-normalised) of the sampled
    outputs of each timed step against the FP64 oracle on the original
    float32 inputs: Y rows, dB columns (A^T dY) and the dvals of the
    sampled rows."""
    import numpy as np
    import torch

    import oracle

    rp, col, rows, cols, ks = smp["rp"], smp["col"], smp["rows"], smp["cols"], smp["ks"]
    vals = A.vals.cpu().numpy()
    M = G.shape[0]
    rb = A.p * (-(-A.n_rows // A.P))
    # the sampled rows as a CSR of their own over the columns they touch
    scols = np.unique(col[ks]) if ks.size else np.zeros(0, np.int64)
    remap = np.zeros(A.n_cols, np.int32)
    remap[scols] = np.arange(scols.size, dtype=np.int32)
    srp = np.concatenate([[0], np.cumsum([rp[rb + r + 1] - rp[rb + r] for r in rows])]).astype(np.int64)
    sub = oracle.Csr(len(rows), max(scols.size, 1), srp, remap[col[ks]], vals[ks], 1, 0)
    Bs = B.index_select(0, torch.from_numpy(scols).long().to(B.device)).float().cpu().numpy()
    Gs = G.index_select(0, torch.from_numpy(rows).long().to(G.device)).float().cpu().numpy()
    srows = np.arange(len(rows))
    y_ref, y_den = oracle.spmm_rows(sub, srows, Bs, None), oracle.spmm_rows(sub, srows, Bs, None, abs_mode=True)
    dv_ref, dv_den = oracle.sddmm(sub, Gs, Bs, None), oracle.sddmm(sub, Gs, Bs, None, abs_mode=True)
    # columns of A^T dY: the panel's nonzeros in the sampled columns
    nz0, nz1 = rp[rb], rp[rb + M]
    slot = np.full(A.n_cols, -1, np.int32)
    slot[cols] = np.arange(cols.size, dtype=np.int32)
    keep = slot[col[nz0:nz1]] >= 0
    kept_before = np.concatenate([[0], np.cumsum(keep, dtype=np.int64)])
    trp = kept_before[rp[rb:rb + M + 1] - nz0]
    tsub = oracle.Csr(M, cols.size, trp, slot[col[nz0:nz1]][keep], vals[nz0:nz1][keep], 1, 0)
    Gh = G.float().cpu().numpy()
    db_ref, db_den = oracle.spmm_t(tsub, Gh, None), oracle.spmm_t(tsub, Gh, None, abs_mode=True)
    rep = {"metric": "max |out - oracle| / (|A||B|, |A|^T|dY|, sum |dY||B|), sampled outputs, FP64 oracle "
                     "on the float32 inputs",
           "samples": {"Y_rows": int(len(rows)), "dB_cols": int(cols.size), "dvals": int(ks.size)}}
    for dt, (y, db, dv) in step_out.items():
        rep["bf16" if dt == torch.bfloat16 else "f32"] = {
            "Y": oracle.rel_err(y, y_ref, y_den), "dB": oracle.rel_err(db, db_ref, db_den),
            "dvals": oracle.rel_err(dv, dv_ref, dv_den)}
    rep["bounds"] = {"f32": 1e-5, "bf16": 1e-2}
    return rep


def cpu_baseline(A, B, G, N, args, out):
    """The FP64 oracle on the host cores: select, pack, spmm, A^T dY and
    dvals.  The sample is the whole panel when it has at most 6M nonzeros,
    else the leading rows of the panel up to 6M nonzeros (only for one-block
    workloads, P = 1); it is run repeatedly until about 10 s of host time
    have passed, and the rate is the mean over those runs."""
    import numpy as np

    import oracle

    Ac = oracle.Csr(A.n_rows, A.n_cols, A.row_ptr.cpu().numpy(), A.col.cpu().numpy(), A.vals.cpu().numpy(),
                    A.P, A.p)
    if Ac.nnz_panel > 6_000_000:
        assert A.P == 1, "row samples are taken of one-block workloads only"
        rp = Ac.row_ptr
        r1 = int(np.searchsorted(rp, rp[Ac.row_begin] + 6_000_000))
        Ac = oracle.Csr(r1, A.n_cols, rp[: r1 + 1], Ac.col[: rp[r1]], Ac.vals[: rp[r1]], 1, 0)
    Bh = B.float().cpu().numpy()
    Gh = G[: Ac.M].float().cpu().numpy()
    runs, dt = 0, 0.0
    while dt < 10.0 and runs < 1000:
        t = time.perf_counter()
        uc, off, cm = oracle.select(Ac)
        Bp = oracle.pack(Bh, uc)
        oracle.spmm(Ac, Bp, cm)
        oracle.spmm_t(Ac, Gh, cm, n_out=len(uc))
        oracle.sddmm(Ac, Gh, Bp, cm)
        dt += time.perf_counter() - t
        runs += 1
    flops = 3 * 2.0 * Ac.nnz_panel * N * runs
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"rows [{Ac.row_begin},{Ac.row_end}) of {args.workload} ({Ac.nnz_panel} nonzeros, "
                      f"P={Ac.P}, N={N}): select+pack+spmm+A^T dY+dvals in FP64, {runs} runs, {dt:.2f} s",
            "seconds": round(dt, 3)}


if __name__ == "__main__":
    main()
