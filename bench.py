"""Benchmark of the p2o hot path on one MI355X.

Workload: the paper's sensor count and time steps (Nd = 600, Nt = 420, so
L = 840 and 421 frequency blocks) on one GPU's share of the spatial
parameters, Nm = 40000; synthetic seeded blocks F_k[s, p] = z exp(-k/80) /
sqrt(Nm) generated on the device, m and d standard normal.

One step = one F apply plus one F* apply on a single right-hand side (the
pair a Hessian matvec needs), inputs resident in HBM.  Every precision
path in --precs runs in its own plan lifetime (the float64 and 16-bit
frequency blocks do not fit together); the first one listed is the
headline `value`.  The mixed paths' relative error is measured against
the float64 path on the same inputs.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
ENTRY_BYTES = {"fp64": 16, "mixed_fp16": 8, "mixed_bf16": 8, "fast_bf16": 4}
VEC_BYTES = {"fp64": 16, "mixed_fp16": 8, "mixed_bf16": 8, "fast_bf16": 8}
SCALE_TILE = 256
DEFAULT_PRECS = "mixed_bf16,fp64,mixed_fp16,fast_bf16"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--Nd", type=int, default=600)
    ap.add_argument("--Nm", type=int, default=40000)
    ap.add_argument("--Nt", type=int, default=420)
    ap.add_argument("--tau", type=float, default=80.0)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--precs", default=DEFAULT_PRECS)
    ap.add_argument("--cpu-cols", type=int, default=40000,
                    help="columns of the workload the CPU oracle baseline runs on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-gb", type=float, default=4.0,
                    help="size of the plain device copy (the byte counters' calibration kernel)")
    ap.add_argument("--read-gb", type=float, default=8.0,
                    help="size of the streaming read timed as the measured HBM read ceiling")
    ap.add_argument("--mrhs", type=int, default=64,
                    help="single workload: also time this many right-hand sides per apply on "
                         "the float64 and bfloat16 hi+lo plans (matrix cores); 0 skips")
    ap.add_argument("--mrhs-steps", type=int, default=3)
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the float64 100x5000x200 single-RHS leg")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "mrhs"],
                    help="single: the 600x40000x420 F+F* step (default); batch: 64 uneven "
                         "instances with 1..256 right-hand sides each; mrhs: one plan, "
                         "--nrhs right-hand sides per apply (matrix-core products)")
    ap.add_argument("--nrhs", type=int, default=64,
                    help="mrhs workload: right-hand sides per apply")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="batch workload: device memory per wave of resident instances")
    ap.add_argument("--no-inversion", action="store_true",
                    help="skip the K-assembly / posterior-solve timing (100x5000x200)")
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="batch workload: keep the persistent kernel's default configuration")
    ap.add_argument("--no-fp64-loop", action="store_true",
                    help="batch workload: skip the instance-by-instance float64 comparison")
    return ap.parse_args()


def measured_copy(torch, gb, reps=5):
    """Plain device-to-device copy of `gb` GB: the streaming ceiling actually
    reachable (read + write bytes / time), and the calibration kernel for
    the hardware byte counters."""
    n = int(gb * 1e9) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": n * 8, "bytes_written": n * 8, "ms": ms,
            "gbs": 2 * n * 8 / (ms * 1e-3) / 1e9}


def product_bytes(prec, op, Nd, Nm, nf, n_pc):
    """Algorithmic HBM bytes of one block-product launch (single RHS)."""
    blocks = nf * Nd * Nm * ENTRY_BYTES[prec]
    vb = VEC_BYTES[prec]
    scales = 0 if prec == "fp64" else nf * ((Nm + SCALE_TILE - 1) // SCALE_TILE) * 4
    if op == "F":   # read xhat [nf][Nm], write partial spectra [n_pc][nf][Nd] (fp64)
        return blocks + scales + nf * Nm * vb + n_pc * nf * Nd * 16
    return blocks + scales + nf * Nd * vb + nf * Nm * vb   # F*: read dhat, write xhat


def step_bytes(prec, Nd, Nm, Nt, nf, n_pc):
    """Algorithmic HBM bytes of one step (F + F*), transforms included."""
    vb = VEC_BYTES[prec]
    fF = Nt * Nm * 8 + nf * Nm * vb                               # read m, write mhat
    iF = n_pc * nf * Nd * 16 + Nt * Nd * 8                        # read partials, write d
    fA = Nt * Nd * 8 + nf * Nd * vb
    iA = nf * Nm * vb + Nt * Nm * 8
    return (product_bytes(prec, "F", Nd, Nm, nf, n_pc) + product_bytes(prec, "FADJ", Nd, Nm, nf, 1)
            + fF + iF + fA + iA)


def n_chunks(Nd, Nm, nf, prec="fp64"):
    """Column chunking of the F product (mirrors the library's choice: the
    16-bit tiers also cap a chunk at 4096 columns)."""
    base = nf * ((Nd + 3) // 4)
    n = max(1, (16384 + base - 1) // base)
    n = min(n, max(1, Nm // 256))
    if prec != "fp64":
        n = max(n, (Nm + 4095) // 4096)
    ln = (Nm + n - 1) // n
    ln = (ln + 63) // 64 * 64
    return (Nm + ln - 1) // ln


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic_600x40000x420.json")


def load_traffic():
    """Calibrated counter bytes per launch of the product kernels, if they were
    measured on the current kernel source (else None: traffic is then null)."""
    from paper_2504_16344_amd.rocprof_summary import source_digest
    try:
        t = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    return t if t.get("source_sha256") == source_digest() else None


def make_plan(P, S, torch, prec, Nd, Nm, Nt, env_dev, seed, stream):
    """Chunked setup from blocks generated on the device, 2048 columns at a time."""
    plan = P.Plan.begin(Nd, Nm, Nt, prec)
    chunk = 2048
    buf = torch.empty((Nt, Nd, chunk), dtype=torch.float64, device="cuda")
    for p0 in range(0, Nm, chunk):
        p1 = min(Nm, p0 + chunk)
        view = buf[:, :, : p1 - p0] if p1 - p0 == chunk else \
            torch.empty((Nt, Nd, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(view.data_ptr(), Nt, Nd, Nm, p0, p1, seed, env_dev.data_ptr(),
                        stream.cuda_stream)
        plan.setup_columns(view, p0, p1)
    plan.setup_end()
    del buf
    return plan


def cpu_baseline(torch, S, args, nf, headline_step_bytes, env):
    """Time the FP64 oracle (as it stands) on a column sample of the workload.

    F and F* are separable over parameter columns (F sums over them, F*
    produces them), so the sample is processed in column chunks of 4096 whose
    blocks are drawn on the device and copied to the host outside the timed
    region; only the oracle calls are timed, then scaled to all Nm columns.
    """
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    Nd, Nm, Nt = args.Nd, args.Nm, args.Nt
    cols = min(args.cpu_cols, Nm)
    stream = torch.cuda.current_stream()
    env_dev = torch.from_numpy(env).cuda()
    m_all = S.vector(args.seed, S.ARRAY_M, Nt * Nm).reshape(Nt, Nm)
    d = S.vector(args.seed, S.ARRAY_D, Nt * Nd).reshape(Nt, Nd)
    dt = 0.0
    step = 4096
    buf = torch.empty((Nt, Nd, step), dtype=torch.float64, device="cuda")
    for p0 in range(0, cols, step):
        p1 = min(cols, p0 + step)
        view = buf[:, :, : p1 - p0] if p1 - p0 == step else \
            torch.empty((Nt, Nd, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(view.data_ptr(), Nt, Nd, Nm, p0, p1, args.seed, env_dev.data_ptr(),
                        stream.cuda_stream)
        blocks = view.cpu().numpy()
        m = np.ascontiguousarray(m_all[:, p0:p1])
        t0 = time.perf_counter()
        oracle.apply_F(blocks, m)
        oracle.apply_Fadj(blocks, d)
        dt += time.perf_counter() - t0
    del buf
    full = dt * Nm / cols
    return {"value": headline_step_bytes / full / 1e9, "unit": "GB/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"time-domain FP64 oracle F + F* on parameter columns 0..{cols - 1} "
                      f"of {Nm} ({dt:.2f} s of oracle time), scaled by {Nm / cols:.2f} to "
                      f"the full step ({full:.1f} s); value = the headline step's "
                      f"algorithmic bytes / that time"}


# ----------------------------------------------------------------------------
# Batched uneven instances
# ----------------------------------------------------------------------------
def instance_bytes(prec, Nd, Nm, Nt, R, nf, n_pc):
    """Device bytes one resident instance needs: frequency blocks, apply
    workspace (largest of F and F*) and its input/output vectors."""
    n8 = lambda n: (n + 7) // 8 * 8
    if prec == "fp64":
        fhat = 16 * nf * Nd * Nm
        ws = max(R * nf * Nm * 16 + R * n_pc * nf * Nd * 16, R * nf * (Nd + Nm) * 16)
    else:
        fhat = 8 * nf * Nd * Nm + 4 * nf * ((Nm + 255) // 256)
        ws = max(R * nf * Nm * 8 + R * n_pc * nf * Nd * 16 + R * nf * 8 * n8(Nm),
                 R * nf * (Nd + Nm) * 8 + R * nf * 8 * n8(Nd))
    vec = 2 * R * Nt * (Nm + Nd) * 8
    return fhat + ws + vec


def batch_apply_bytes(prec, Nd, Nm, Nt, R, nf, n_pc):
    """Algorithmic HBM bytes of one F apply plus one F* apply of an instance:
    blocks streamed once per op, vectors and spectra read and written once."""
    eb, vb = ENTRY_BYTES[prec], VEC_BYTES[prec]
    blocks = nf * Nd * Nm * eb
    vecF = R * (Nt * Nm * 8 + 2 * nf * Nm * vb + 2 * n_pc * nf * Nd * 16 + Nt * Nd * 8)
    vecA = R * (Nt * Nd * 8 + 2 * nf * Nd * vb + 2 * nf * Nm * vb + Nt * Nm * 8)
    return 2 * blocks + vecF + vecA


def bench_batch(args):
    import torch
    import p2o_synth as S
    import paper_2504_16344_amd as P

    n, seed, Nt = args.instances, 4, args.Nt
    Nd = S.uniform_ints(seed, S.ARRAY_SHAPES, n, 50, 600)
    Nm = S.uniform_ints(seed, S.ARRAY_SHAPES, n, 1000, 20000, offset=n)
    R = S.uniform_ints(seed, S.ARRAY_SHAPES, n, 1, 256, offset=2 * n)
    L = P.smooth_length(Nt)
    nf = L // 2 + 1
    stream = torch.cuda.current_stream()
    prec = "mixed_bf16"
    npc = [n_chunks(int(Nd[i]), int(Nm[i]), nf, prec) for i in range(n)]
    need = [instance_bytes(prec, int(Nd[i]), int(Nm[i]), Nt, int(R[i]), nf, npc[i]) for i in range(n)]
    budget = args.budget_gb * 1e9
    waves, cur, used = [], [], 0
    for i in range(n):
        if cur and used + need[i] > budget:
            waves.append(cur)
            cur, used = [], 0
        cur.append(i)
        used += need[i]
    waves.append(cur)

    def inputs(i):
        inst_seed = 1000 * seed + i
        m = torch.empty((int(R[i]), Nt, int(Nm[i])), dtype=torch.float64, device="cuda")
        d = torch.empty((int(R[i]), Nt, int(Nd[i])), dtype=torch.float64, device="cuda")
        S.device_normals(m.data_ptr(), m.numel(), 0, inst_seed, S.ARRAY_M, 1.0, stream.cuda_stream)
        S.device_normals(d.data_ptr(), d.numel(), 0, inst_seed, S.ARRAY_D, 1.0, stream.cuda_stream)
        return m, d

    def plan_for(i, p):
        env = torch.from_numpy(S.envelope(Nt, 80.0, 1.0 / np.sqrt(int(Nm[i])))).cuda()
        return make_plan(P, S, torch, p, int(Nd[i]), int(Nm[i]), Nt, env, 1000 * seed + i, stream)

    reps = max(1, args.steps)
    total_ms = {"F": 0.0, "FADJ": 0.0}
    wave_info, samples = [], {}
    for w, ids in enumerate(waves):
        t0 = time.perf_counter()
        plans = [plan_for(i, prec) for i in ids]
        vecs = [inputs(i) for i in ids]
        yF = [torch.empty((int(R[i]), Nt, int(Nd[i])), dtype=torch.float64, device="cuda") for i in ids]
        yA = [torch.empty((int(R[i]), Nt, int(Nm[i])), dtype=torch.float64, device="cuda") for i in ids]
        batch = P.Batch(plans)
        tuned = {}
        if not args.no_batch_tune:  # the persistent kernel's tiles, timed on this wave
            for op, name, xs, ys in ((P.OP_F, "F", [v[0] for v in vecs], yF),
                                     (P.OP_FADJ, "FADJ", [v[1] for v in vecs], yA)):
                c, t = batch.autotune(op, xs, ys, reps=1)
                tuned[name] = {"chosen": c, "candidate_ms": [round(x, 3) for x in t]}
        gF = batch.capture(P.OP_F, [v[0] for v in vecs], yF)
        gA = batch.capture(P.OP_FADJ, [v[1] for v in vecs], yA)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        for _ in range(args.warmup):
            gF.launch()
            gA.launch()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(reps):
            gF.launch()
        ev[1].record()
        for _ in range(reps):
            gA.launch()
        ev[2].record()
        torch.cuda.synchronize()
        msF, msA = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
        total_ms["F"] += msF
        total_ms["FADJ"] += msA
        for j, i in enumerate(ids):
            samples[i] = (yF[j][0].cpu(), yA[j][0].cpu())
        wave_info.append({"instances": len(ids), "resident_gb": round(sum(need[i] for i in ids) / 1e9, 1),
                          "ms_F": round(msF, 3), "ms_FADJ": round(msA, 3), "setup_s": round(setup_s, 1),
                          "tuned": tuned})
        print(f"[batch] wave {w}: {len(ids)} instances, F {msF:.2f} ms, F* {msA:.2f} ms, "
              f"setup {setup_s:.1f} s", file=sys.stderr, flush=True)
        gF.close()
        gA.close()
        batch.close()
        for p in plans:
            p.close()
        del plans, vecs, yF, yA, batch
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    fp64 = None
    errs = []
    if not args.no_fp64_loop:
        fp64_ms = 0.0
        for i in range(n):
            p = plan_for(i, "fp64")
            m, d = inputs(i)
            yf = p.F(m)
            ya = p.FT(d)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(reps):
                p.F(m, out=yf)
                p.FT(d, out=ya)
            ev[1].record()
            torch.cuda.synchronize()
            fp64_ms += ev[0].elapsed_time(ev[1]) / reps
            sF, sA = samples[i]
            errs.append(max((torch.linalg.norm(sF - yf[0].cpu()) / torch.linalg.norm(yf[0].cpu())).item(),
                            (torch.linalg.norm(sA - ya[0].cpu()) / torch.linalg.norm(ya[0].cpu())).item()))
            p.close()
            del p, m, d, yf, ya
            torch.cuda.empty_cache()
        fp64 = fp64_ms
        print(f"[batch] fp64 instance loop: {fp64_ms:.1f} ms per F+F* over all instances",
              file=sys.stderr, flush=True)

    step_ms = total_ms["F"] + total_ms["FADJ"]
    bytes_total = sum(batch_apply_bytes(prec, int(Nd[i]), int(Nm[i]), Nt, int(R[i]), nf, npc[i])
                      for i in range(n))
    flops = sum(2 * 8 * nf * int(Nd[i]) * int(Nm[i]) * int(R[i]) for i in range(n))
    out = {
        "metric": "batched F/F* apply time, uneven instances; mixed (bf16 hi+lo, matrix cores) vs FP64 instance loop",
        "value": round(bytes_total / (step_ms * 1e-3) / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x2/f32", "data": "synthetic (seeded counter-based normals, generated on device)",
        "config": {"workload": f"{n} independent p2o instances, Nt={Nt}, Nd U{{50..600}}, "
                               f"Nm U{{1000..20000}}, 1..256 RHS each; F and F* as captured HIP "
                               f"graphs (per op and memory wave: one warp-specialised product launch "
                               f"per matrix-core instance, one persistent launch for the others)",
                   "instances": n, "Nt": Nt, "waves": len(waves),
                   "rhs_total": int(R.sum()), "budget_gb": args.budget_gb},
        "complex_tflops": round(flops / (step_ms * 1e-3) / 1e12, 2),
        "waves": wave_info,
        "op_ms": {k: round(v, 3) for k, v in total_ms.items()},
    }
    if fp64 is not None:
        out["fp64_loop_ms"] = round(fp64, 3)
        out["speedup_vs_fp64_loop"] = round(fp64 / step_ms, 3)
        out["rel_err_vs_fp64_max"] = max(errs)
    print(json.dumps(out), flush=True)

PEAK_TFLOPS = {"fp64": 78.6, "mixed_bf16": 2500.0, "fast_bf16": 2500.0}
# matrix-core flops per useful flop: bfloat16 hi+lo splits form H xh + H xl + Lo xh
SPLIT_FACTOR = {"fp64": 1, "mixed_bf16": 3, "fast_bf16": 2}


def mrhs_product_bytes(prec, op, Nd, Nm, nf, n_pc, B):
    """Algorithmic HBM bytes of one matrix-core product launch sequence for B
    right-hand sides: the blocks once per pass of 64, plus the vector operand
    read and the product written, per right-hand side."""
    passes = (B + 63) // 64
    blocks = nf * Nd * Nm * ENTRY_BYTES[prec] * passes
    scales = 0 if prec == "fp64" else nf * ((Nm + SCALE_TILE - 1) // SCALE_TILE) * 4 * passes
    r8 = lambda n: (n + 7) // 8 * 8
    if prec == "fp64":
        vin = nf * (Nm if op == "F" else Nd) * 16
        vout = n_pc * nf * Nd * 16 if op == "F" else nf * Nm * 16
    else:  # four bfloat16 planes in; F partial spectra float64, F* float32 out
        vin = nf * r8(Nm if op == "F" else Nd) * 8
        vout = n_pc * nf * Nd * 16 if op == "F" else nf * Nm * 8
    return blocks + scales + B * (vin + vout)


def bench_mrhs(args):
    """One plan at the 600 x 40000 x 420 shape, applies on --nrhs right-hand
    sides: the per-frequency products run as complex GEMMs on the matrix
    cores.  Reports per-op product-kernel times against the MFMA and HBM
    rooflines, and the mixed paths' error against float64 on the same inputs."""
    import torch
    import p2o_synth as S
    import paper_2504_16344_amd as P

    Nd, Nm, Nt, B = args.Nd, args.Nm, args.Nt, args.nrhs
    L = P.smooth_length(Nt)
    nf = L // 2 + 1
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    if args.precs == DEFAULT_PRECS:
        precs = ["mixed_bf16", "fp64"]
    precs = [p for p in precs if p in PEAK_TFLOPS]
    stream = torch.cuda.current_stream()
    env_dev = torch.from_numpy(S.envelope(Nt, args.tau, 1.0 / np.sqrt(Nm))).cuda()
    m = torch.empty((B, Nt, Nm), dtype=torch.float64, device="cuda")
    d = torch.empty((B, Nt, Nd), dtype=torch.float64, device="cuda")
    S.device_normals(m.data_ptr(), m.numel(), 0, args.seed, S.ARRAY_M, 1.0, stream.cuda_stream)
    S.device_normals(d.data_ptr(), d.numel(), 0, args.seed, S.ARRAY_D, 1.0, stream.cuda_stream)
    flops = 8 * nf * Nd * Nm * B
    copy = measured_copy(torch, args.copy_gb) if args.copy_gb > 0 else None
    results, ref = {}, None
    order = (["fp64"] if "fp64" in precs else []) + [p for p in precs if p != "fp64"]
    for prec in order:
        plan = make_plan(P, S, torch, prec, Nd, Nm, Nt, env_dev, args.seed, stream)
        plan.reserve(B)
        yF = torch.empty((B, Nt, Nd), dtype=torch.float64, device="cuda")
        yA = torch.empty((B, Nt, Nm), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            plan.F(m, out=yF)
            plan.FT(d, out=yA)
        torch.cuda.synchronize()
        plan.set_kernel_timing(True)
        plan.kernel_time(P.OP_F)
        plan.kernel_time(P.OP_FADJ)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(args.steps):
            plan.F(m, out=yF)
        ev[1].record()
        for _ in range(args.steps):
            plan.FT(d, out=yA)
        ev[2].record()
        torch.cuda.synchronize()
        kF, nF = plan.kernel_time(P.OP_F)
        kA, nA = plan.kernel_time(P.OP_FADJ)
        plan.set_kernel_timing(False)
        r = {"apply_ms": {"F": ev[0].elapsed_time(ev[1]) / args.steps,
                          "FADJ": ev[1].elapsed_time(ev[2]) / args.steps},
             "product_kernel_ms": {"F": kF / max(nF, 1), "FADJ": kA / max(nA, 1)},
             "roofline": {}}
        for op in ("F", "FADJ"):
            ms = r["product_kernel_ms"][op]
            nbytes = mrhs_product_bytes(prec, op, Nd, Nm, nf, n_chunks(Nd, Nm, nf, prec), B)
            hw = flops * SPLIT_FACTOR[prec]
            t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
            t_mfma = hw / (PEAK_TFLOPS[prec] * 1e12)
            gbs = nbytes / (ms * 1e-3) / 1e9
            tfs = hw / (ms * 1e-3) / 1e12
            if t_mfma >= t_hbm:
                rf = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK_TFLOPS[prec],
                      "unit": "TFLOP/s", "frac": round(tfs / PEAK_TFLOPS[prec], 4)}
            else:
                rf = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                      "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}
            rf.update({"traffic": None, "avg_ms": round(ms, 4), "bytes_per_launch": nbytes,
                       "mfma_flops_per_launch": hw, "hbm_gbs": round(gbs, 1),
                       "mfma_tflops": round(tfs, 2),
                       "mfma_frac": round(tfs / PEAK_TFLOPS[prec], 4)})
            r["roofline"][op] = rf
        r["ms_per_step"] = r["apply_ms"]["F"] + r["apply_ms"]["FADJ"]
        n_pc = n_chunks(Nd, Nm, nf, prec)
        r["step_bytes"] = (mrhs_product_bytes(prec, "F", Nd, Nm, nf, n_pc, B)
                           + mrhs_product_bytes(prec, "FADJ", Nd, Nm, nf, 1, B)
                           + B * (Nt * Nm * 8 * 2 + Nt * Nd * 8 * 2))
        if prec == "fp64":
            ref = (yF, yA)  # kept as the reference (no copy: the counter calibration
            #                 takes the largest device copy in the run to be the 4 GB one)
        elif ref is not None:
            r["rel_err_vs_fp64"] = {
                "F": (torch.linalg.norm(yF - ref[0]) / torch.linalg.norm(ref[0])).item(),
                "FADJ": (torch.linalg.norm(yA - ref[1]) / torch.linalg.norm(ref[1])).item()}
        results[prec] = r
        print(f"[mrhs] {prec}: F {r['apply_ms']['F']:.2f} ms (product {r['product_kernel_ms']['F']:.2f}),"
              f" F* {r['apply_ms']['FADJ']:.2f} ms (product {r['product_kernel_ms']['FADJ']:.2f})",
              file=sys.stderr, flush=True)
        plan.close()
        del plan, yF, yA
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    head = precs[0]
    h = results[head]
    dom = max(("F", "FADJ"), key=lambda o: h["product_kernel_ms"][o])
    out = {
        "metric": "multi-RHS F/F* apply time and product-kernel roofline (matrix cores) "
                  f"@Nd={Nd},Nt={Nt}; mixed vs FP64",
        "value": round(h["step_bytes"] / (h["ms_per_step"] * 1e-3) / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed_bf16": "bf16x2/f32", "fast_bf16": "bf16/f32"}[head],
        "data": "synthetic (seeded counter-based normals, generated on device)",
        "config": {"workload": f"p2o F+F* on {B} right-hand sides, Nd={Nd} Nm={Nm} Nt={Nt} "
                               f"(L={L}, {nf} frequency blocks), precision {head}",
                   "Nd": Nd, "Nm": Nm, "Nt": Nt, "nrhs": B, "precision": head},
        "roofline": h["roofline"][dom],
        "roofline_other": h["roofline"]["FADJ" if dom == "F" else "F"],
        "paths": results,
        "measured_copy": copy,
    }
    if "fp64" in results and head != "fp64":
        out["speedup_vs_fp64"] = round(results["fp64"]["ms_per_step"] / h["ms_per_step"], 3)
    print(json.dumps(out), flush=True)


def inversion_cpu_baseline(torch, S, K_dev, env_dev, Nd, Nm, Nt, seed, s2, t_chol, t_gram):
    """The oracle beside the inversion workload on the host cores: LAPACK
    Cholesky (scipy cho_factor, as the oracle's posterior mean uses it) of
    the same K, and the oracle's Gram-recurrence K from the same blocks
    (drawn on the device, copied to the host outside the timed region)."""
    import scipy.linalg
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    n = Nt * Nd
    Kh = K_dev.cpu().numpy()
    t0 = time.perf_counter()
    scipy.linalg.cho_factor(Kh, lower=True, overwrite_a=True, check_finite=False)
    t_potrf = time.perf_counter() - t0
    del Kh
    blk = torch.empty((Nt, Nd, Nm), dtype=torch.float64, device="cuda")
    S.device_blocks(blk.data_ptr(), Nt, Nd, Nm, 0, Nm, seed, env_dev.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    blocks = blk.cpu().numpy()
    del blk
    t0 = time.perf_counter()
    oracle.hessian_gram(blocks, 0.25, s2)
    t_k = time.perf_counter() - t0
    del blocks
    return {"kind": "oracle", "cores": int(cores),
            "cholesky_s": round(t_potrf, 3), "cholesky_gflops": round(n ** 3 / 3 / t_potrf / 1e9, 1),
            "hessian_gram_s": round(t_k, 3),
            "gpu_over_cpu": {"cholesky": round(t_potrf / t_chol, 1),
                             "hessian_gram": round(t_k / t_gram, 1)},
            "sample": f"the whole {n}x{n} K: scipy.linalg.cho_factor (LAPACK dpotrf) and the "
                      f"oracle's hessian_gram (one {n}x{Nm}x{n} GEMM plus the block-diagonal "
                      f"recurrence)"}


def bench_inversion(torch, S, P, cpu=True):
    """K = Gn + F Gp F* (20000 x 20000; by the paper's unit-vector matvecs
    and in Gram form), the posterior mean, and the QoI posterior
    (Q, Gamma_post(q); both assembly methods) with its online prediction
    q = Q d at the 100 x 5000 x 200 inversion workload with 21 QoI
    locations: wall time of each call (the prediction by events)."""
    Nd, Nm, Nt, seed = 100, 5000, 200, 5
    stream = torch.cuda.current_stream()
    env = torch.from_numpy(S.envelope(Nt, 40.0, 1.0 / np.sqrt(Nm))).cuda()
    plan = make_plan(P, S, torch, "fp64", Nd, Nm, Nt, env, seed, stream)
    n = Nt * Nd
    m_true = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
    S.device_normals(m_true.data_ptr(), m_true.numel(), 0, seed, S.ARRAY_M, 1.0, stream.cuda_stream)
    d_clean = plan.F(m_true)
    s2 = 1e-2 * float((d_clean ** 2).mean())
    eps = torch.empty_like(d_clean)
    S.device_normals(eps.data_ptr(), eps.numel(), 0, seed, S.ARRAY_NOISE, 1.0, stream.cuda_stream)
    d_obs = d_clean + (s2 ** 0.5) * eps
    nv = torch.full((n,), s2, dtype=torch.float64, device="cuda")
    K = torch.empty((n, n), dtype=torch.float64, device="cuda")
    plan.hessian(0.25, nv, out=K)  # warm-up (also allocates)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.hessian(0.25, nv, out=K)
    torch.cuda.synchronize()
    t_k = time.perf_counter() - t0
    # the same K in Gram form (time-domain blocks, one GEMM, block-diagonal sums)
    K2 = torch.empty_like(K)
    plan.hessian(0.25, nv, out=K2, method="gram")  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.hessian(0.25, nv, out=K2, method="gram")
    torch.cuda.synchronize()
    t_kg = time.perf_counter() - t0
    e_kg = ((K2 - K).abs().max() / K.abs().max()).item()
    del K2
    plan.set_assembly("matvec")
    K_keep = K.clone()
    t0 = time.perf_counter()
    m = plan.posterior(K, d_obs, 0.25, refine_steps=1)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    # without refinement: factorisation + two sweeps + F*, for the Cholesky estimate
    Kc = K_keep.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.posterior(Kc, d_obs, 0.25, refine_steps=0)
    torch.cuda.synchronize()
    t_m0 = time.perf_counter() - t0
    del Kc
    # Phase 4 online: m from the factor alone (two triangular sweeps + F*)
    m_on = plan.posterior_mean(K, d_obs, 0.25)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(5):
        plan.posterior_mean(K, d_obs, 0.25, out=m_on)
    ev[1].record()
    torch.cuda.synchronize()
    t_on = ev[0].elapsed_time(ev[1]) / 5 * 1e-3
    e_on = (torch.linalg.norm(m_on - m) / torch.linalg.norm(m)).item()
    # Phase 4 online from K^{-1} (formed offline from the factor): one pass
    # over K^{-1} and one F*
    Kinv = torch.empty_like(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.posterior_invert(K, out=Kinv)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    m_ki = plan.posterior_mean_kinv(Kinv, d_obs, 0.25)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(20):
        plan.posterior_mean_kinv(Kinv, d_obs, 0.25, out=m_ki)
    ev[1].record()
    torch.cuda.synchronize()
    t_ki = ev[0].elapsed_time(ev[1]) / 20 * 1e-3
    e_ki = (torch.linalg.norm(m_ki - m) / torch.linalg.norm(m)).item()
    del Kinv
    # MAP optimality residual F* Gn^-1 (F m - d) + m / Gp, relative to m / Gp
    g = plan.FT((plan.F(m) - d_obs) / s2) + m / 0.25
    res = (torch.linalg.norm(g) / torch.linalg.norm(m / 0.25)).item()
    # Phases 3-4 with the paper's 21 QoI locations: Q and Gamma_post(q) from K's
    # factor, then the online prediction q = Q d (HBM-bound: Q streamed once)
    Nq = 21
    planq = make_plan(P, S, torch, "fp64", Nq, Nm, Nt, env, seed + S.QOI_SEED_OFFSET, stream)
    plan.qoi_precompute(planq, K, 0.25)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q, Gq = plan.qoi_precompute(planq, K, 0.25)
    torch.cuda.synchronize()
    t_q = time.perf_counter() - t0
    del Gq
    plan.qoi_precompute(planq, K, 0.25, method="gram")  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q2, Gq = plan.qoi_precompute(planq, K, 0.25, method="gram")
    torch.cuda.synchronize()
    t_qg = time.perf_counter() - t0
    e_qg = ((Q2 - Q).abs().max() / Q.abs().max()).item()
    del Q2
    q = P.qoi_predict(Q, d_obs)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 20
    ev[0].record()
    for _ in range(reps):
        P.qoi_predict(Q, d_obs)
    ev[1].record()
    torch.cuda.synchronize()
    t_p = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    q_map = planq.F(m).reshape(-1)
    e_q = (torch.linalg.norm(q - q_map) / torch.linalg.norm(q_map)).item()
    q_bytes = Q.numel() * 8 + n * 8 + Nq * Nt * 8
    planq.close()
    plan.close()
    del K, Q, Gq
    torch.cuda.empty_cache()
    units = n
    nf = P.smooth_length(Nt) // 2 + 1
    # roofline fractions: float64 matrix-core peak for the assembly and the
    # factorisation, HBM for the online steps (one pass over the factor per
    # sweep, or over K^{-1}, plus one F* product's bytes)
    fadj_bytes = product_bytes("fp64", "FADJ", Nd, Nm, nf, 1)
    t_chol = max(t_m0 - t_on, 1e-9)
    flops = {"hessian_unit_vectors": 8 * nf * Nd * Nm * n, "hessian_gram": n * n * Nm,
             "cholesky": n ** 3 / 3}
    secs = {"hessian_unit_vectors": t_k, "hessian_gram": t_kg, "cholesky": t_chol}
    roof = {}
    for k in flops:
        tf = flops[k] / secs[k] / 1e12
        roof[k] = {"bound": "mfma", "achieved": round(tf, 2), "peak": 78.6, "unit": "TFLOP/s",
                   "frac": round(tf / 78.6, 4), "flops": flops[k], "s": round(secs[k], 4)}
    hbm = {"posterior_online_factor": (n * n * 8 + fadj_bytes, t_on),
           "posterior_online_kinv": (n * n * 8 + fadj_bytes, t_ki),
           "qoi_predict": (q_bytes, t_p)}
    for k, (b, t) in hbm.items():
        gbs = b / t / 1e9
        roof[k] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes": b, "ms": round(t * 1e3, 4)}
    cpu_out = None
    if cpu:
        cpu_out = inversion_cpu_baseline(torch, S, K_keep, env, Nd, Nm, Nt, seed, s2, t_chol, t_kg)
    del K_keep
    torch.cuda.empty_cache()
    return {"workload": f"Nd={Nd} Nm={Nm} Nt={Nt}, K {n}x{n} float64; Nq={Nq} QoI locations",
            "roofline": roof, "cholesky_s_est": round(t_chol, 4),
            "posterior_solve_norefine_s": round(t_m0, 4), "cpu_baseline": cpu_out,
            "hessian_assemble_s": round(t_k, 3), "unit_vectors_per_s": round(units / t_k, 1),
            "hessian_gram_s": round(t_kg, 4), "hessian_gram_vs_matvec_rel": e_kg,
            "posterior_solve_s": round(t_m, 3), "map_gradient_rel": res,
            "posterior_online_ms": round(t_on * 1e3, 3), "posterior_online_vs_refined_rel": e_on,
            "posterior_invert_s": round(t_inv, 3),
            "posterior_online_kinv_ms": round(t_ki * 1e3, 3),
            "posterior_online_kinv_vs_refined_rel": e_ki,
            "qoi_precompute_s": round(t_q, 3), "qoi_precompute_gram_s": round(t_qg, 3),
            "qoi_gram_vs_matvec_rel": e_qg,
            "qoi_predict_ms": round(t_p * 1e3, 4),
            "qoi_predict_hbm_gbs": round(q_bytes / t_p / 1e9, 1),
            "qoi_predict_vs_fq_mmap_rel": e_q}


def read_ceiling(torch, P, gb, reps=5):
    """The device's streaming-read ceiling: the library's plain read kernel
    (the product kernels' non-temporal 16-byte loads, nothing else) over
    `gb` GB, timed by events on the current stream."""
    n = int(gb * 1e9) // 16 * 2
    buf = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.read_bandwidth(buf, sink)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        P.read_bandwidth(buf, sink)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del buf
    torch.cuda.empty_cache()
    return {"bytes": n * 8, "ms": ms, "gbs": n * 8 / (ms * 1e-3) / 1e9,
            "frac_of_peak": round(n * 8 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def time_ops(torch, P, plan, xF, xA, yF, yA, warmup, steps):
    """Apply time (events on the current stream) and product-kernel time
    (the library's events around each product launch) of F and F*."""
    for _ in range(warmup):
        plan.F(xF, out=yF)
        plan.FT(xA, out=yA)
    torch.cuda.synchronize()
    plan.set_kernel_timing(True)
    plan.kernel_time(P.OP_F)
    plan.kernel_time(P.OP_FADJ)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(steps):
        plan.F(xF, out=yF)
    ev[1].record()
    for _ in range(steps):
        plan.FT(xA, out=yA)
    ev[2].record()
    torch.cuda.synchronize()
    kF, nF = plan.kernel_time(P.OP_F)
    kA, nA = plan.kernel_time(P.OP_FADJ)
    plan.set_kernel_timing(False)
    return ({"F": ev[0].elapsed_time(ev[1]) / steps, "FADJ": ev[1].elapsed_time(ev[2]) / steps},
            {"F": kF / max(nF, 1), "FADJ": kA / max(nA, 1)})


def mrhs_roofline(prec, op, Nd, Nm, nf, B, ms):
    """Roofline of one many-RHS product launch sequence (matrix cores):
    algorithmic bytes and matrix-core flops against HBM and the dtype's
    dense matrix-core peak; `bound` is whichever the algorithm hits first."""
    nbytes = mrhs_product_bytes(prec, op, Nd, Nm, nf, n_chunks(Nd, Nm, nf, prec), B)
    hw = 8 * nf * Nd * Nm * B * SPLIT_FACTOR[prec]
    gbs = nbytes / (ms * 1e-3) / 1e9
    tfs = hw / (ms * 1e-3) / 1e12
    if hw / (PEAK_TFLOPS[prec] * 1e12) >= nbytes / (PEAK_HBM_GBS * 1e9):
        rf = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK_TFLOPS[prec],
              "unit": "TFLOP/s", "frac": round(tfs / PEAK_TFLOPS[prec], 4)}
    else:
        rf = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
              "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}
    rf.update({"traffic": None, "avg_ms": round(ms, 4), "bytes_per_launch": nbytes,
               "mfma_flops_per_launch": hw, "hbm_gbs": round(gbs, 1),
               "mfma_tflops": round(tfs, 2), "mfma_frac": round(tfs / PEAK_TFLOPS[prec], 4)})
    return rf


def c2_fp64_leg(torch, S, P, reps=200, rotate=4):
    """FP64 single-RHS F and F* at 100 x 5000 x 200 (201 frequency blocks,
    1.6 GB per plan).  The blocks are only ~6x the 256 MB last-level cache,
    so `rotate` plans with different seeds take turns (each launch streams
    blocks the previous launches did not touch); product-kernel time from
    the library's events, apply time from events around all launches."""
    Nd, Nm, Nt = 100, 5000, 200
    nf = P.smooth_length(Nt) // 2 + 1
    stream = torch.cuda.current_stream()
    env = torch.from_numpy(S.envelope(Nt, 40.0, 1.0 / np.sqrt(Nm))).cuda()
    plans = [make_plan(P, S, torch, "fp64", Nd, Nm, Nt, env, 2 + j, stream) for j in range(rotate)]
    m = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
    d = torch.empty((Nt, Nd), dtype=torch.float64, device="cuda")
    S.device_normals(m.data_ptr(), m.numel(), 0, 2, S.ARRAY_M, 1.0, stream.cuda_stream)
    S.device_normals(d.data_ptr(), d.numel(), 0, 2, S.ARRAY_D, 1.0, stream.cuda_stream)
    yF = torch.empty((Nt, Nd), dtype=torch.float64, device="cuda")
    yA = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
    for p in plans:
        p.reserve(1)
        for op in (P.OP_F, P.OP_FADJ):
            p.autotune(op, reps=3)
        p.F(m, out=yF)
        p.FT(d, out=yA)
    torch.cuda.synchronize()
    for p in plans:
        p.set_kernel_timing(True)
        p.kernel_time(P.OP_F)
        p.kernel_time(P.OP_FADJ)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for i in range(reps):
        plans[i % rotate].F(m, out=yF)
    ev[1].record()
    for i in range(reps):
        plans[i % rotate].FT(d, out=yA)
    ev[2].record()
    torch.cuda.synchronize()
    k = {"F": [0.0, 0], "FADJ": [0.0, 0]}
    for p in plans:
        for op, name in ((P.OP_F, "F"), (P.OP_FADJ, "FADJ")):
            ms, n = p.kernel_time(op)
            k[name][0] += ms
            k[name][1] += n
        p.set_kernel_timing(False)
    out = {"workload": f"p2o F and F* single RHS, Nd={Nd} Nm={Nm} Nt={Nt} ({nf} frequency "
                       f"blocks), float64, {rotate} plans in rotation, {reps} launches per op",
           "apply_ms": {"F": ev[0].elapsed_time(ev[1]) / reps, "FADJ": ev[1].elapsed_time(ev[2]) / reps}}
    for name in ("F", "FADJ"):
        ms = k[name][0] / max(k[name][1], 1)
        nbytes = product_bytes("fp64", name, Nd, Nm, nf, n_chunks(Nd, Nm, nf, "fp64") if name == "F" else 1)
        ach = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(ach / PEAK_HBM_GBS, 4), "avg_ms": round(ms, 5),
                     "bytes_per_launch": nbytes}
    for p in plans:
        p.close()
    del plans
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not a measured path)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "mrhs":
        return bench_mrhs(args)
    import torch
    import p2o_synth as S
    import paper_2504_16344_amd as P

    Nd, Nm, Nt, B = args.Nd, args.Nm, args.Nt, args.mrhs
    L = P.smooth_length(Nt)
    nf = L // 2 + 1
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    stream = torch.cuda.current_stream()
    env = S.envelope(Nt, args.tau, 1.0 / np.sqrt(Nm))
    env_dev = torch.from_numpy(env).cuda()
    m = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
    d = torch.empty((Nt, Nd), dtype=torch.float64, device="cuda")
    S.device_normals(m.data_ptr(), m.numel(), 0, args.seed, S.ARRAY_M, 1.0, stream.cuda_stream)
    S.device_normals(d.data_ptr(), d.numel(), 0, args.seed, S.ARRAY_D, 1.0, stream.cuda_stream)
    mB = dB = None
    if B > 0:  # right-hand side 0 of the B is the single one above
        mB = torch.empty((B, Nt, Nm), dtype=torch.float64, device="cuda")
        dB = torch.empty((B, Nt, Nd), dtype=torch.float64, device="cuda")
        S.device_normals(mB.data_ptr(), mB.numel(), 0, args.seed, S.ARRAY_M, 1.0, stream.cuda_stream)
        S.device_normals(dB.data_ptr(), dB.numel(), 0, args.seed, S.ARRAY_D, 1.0, stream.cuda_stream)
    torch.cuda.synchronize()

    read = read_ceiling(torch, P, args.read_gb) if args.read_gb > 0 else None
    copy = measured_copy(torch, args.copy_gb) if args.copy_gb > 0 else None
    results = {}
    ref = refB = None
    order = (["fp64"] if "fp64" in precs else []) + [p for p in precs if p != "fp64"]
    for prec in order:
        t_setup = time.perf_counter()
        plan = make_plan(P, S, torch, prec, Nd, Nm, Nt, env_dev, args.seed, stream)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        plan.reserve(1)
        tuned = {}
        for op, name in ((P.OP_F, "F"), (P.OP_FADJ, "FADJ")):
            c, times = plan.autotune(op, reps=3)
            tuned[name] = {"chosen": c, "candidate_ms": [round(t, 4) for t in times]}
        yF = torch.empty((Nt, Nd), dtype=torch.float64, device="cuda")
        yA = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            plan.F(m, out=yF)
            plan.FT(d, out=yA)
        torch.cuda.synchronize()
        plan.set_kernel_timing(True)
        plan.kernel_time(P.OP_F)
        plan.kernel_time(P.OP_FADJ)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.F(m, out=yF)
            plan.FT(d, out=yA)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        msF, nF = plan.kernel_time(P.OP_F)
        msA, nA = plan.kernel_time(P.OP_FADJ)
        plan.set_kernel_timing(False)
        apply_ms, _ = time_ops(torch, P, plan, m, d, yF, yA, 0, args.steps)
        r = {
            "setup_s": round(t_setup, 3),
            "ms_per_step": wall * 1e3 / args.steps,
            "apply_ms": apply_ms,
            "product_kernel_ms": {"F": msF / max(nF, 1), "FADJ": msA / max(nA, 1)},
            "product_bytes": {"F": product_bytes(prec, "F", Nd, Nm, nf, n_chunks(Nd, Nm, nf, prec)),
                              "FADJ": product_bytes(prec, "FADJ", Nd, Nm, nf, 1)},
            "step_bytes": step_bytes(prec, Nd, Nm, Nt, nf, n_chunks(Nd, Nm, nf, prec)),
            "autotune": tuned,
        }
        r["gbs"] = r["step_bytes"] / (r["ms_per_step"] * 1e-3) / 1e9
        for op in ("F", "FADJ"):
            r.setdefault("product_frac_of_peak", {})[op] = round(
                r["product_bytes"][op] / (r["product_kernel_ms"][op] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        if prec == "fp64":
            ref = (yF.clone(), yA.clone())
        elif ref is not None:
            eF = (torch.linalg.norm(yF - ref[0]) / torch.linalg.norm(ref[0])).item()
            eA = (torch.linalg.norm(yA - ref[1]) / torch.linalg.norm(ref[1])).item()
            r["rel_err_vs_fp64"] = {"F": eF, "FADJ": eA}
        if B > 0 and prec in PEAK_TFLOPS and prec != "fast_bf16":
            # B right-hand sides on the same plan: the matrix-core products
            plan.reserve(B)
            yFB = torch.empty((B, Nt, Nd), dtype=torch.float64, device="cuda")
            yAB = torch.empty((B, Nt, Nm), dtype=torch.float64, device="cuda")
            appB, kB = time_ops(torch, P, plan, mB, dB, yFB, yAB, 1, args.mrhs_steps)
            rb = {"nrhs": B, "apply_ms": appB, "product_kernel_ms": kB,
                  "ms_per_step": appB["F"] + appB["FADJ"],
                  "roofline": {op: mrhs_roofline(prec, op, Nd, Nm, nf, B, kB[op])
                               for op in ("F", "FADJ")}}
            if prec == "fp64":
                refB = (yFB, yAB)
            elif refB is not None:
                rb["rel_err_vs_fp64"] = {
                    "F": (torch.linalg.norm(yFB - refB[0]) / torch.linalg.norm(refB[0])).item(),
                    "FADJ": (torch.linalg.norm(yAB - refB[1]) / torch.linalg.norm(refB[1])).item()}
            r["mrhs"] = rb
            del yFB, yAB
            print(f"[bench] {prec} {B} RHS: F {appB['F']:.2f} ms (product {kB['F']:.2f}), "
                  f"F* {appB['FADJ']:.2f} ms (product {kB['FADJ']:.2f})", file=sys.stderr, flush=True)
        results[prec] = r
        plan.close()
        del plan
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step, {r['gbs']:.0f} GB/s, "
              f"kernels F {r['product_kernel_ms']['F']:.3f} ms F* "
              f"{r['product_kernel_ms']['FADJ']:.3f} ms, setup {t_setup:.1f} s",
              file=sys.stderr, flush=True)
    del mB, dB, refB
    torch.cuda.empty_cache()

    head = precs[0]
    h = results[head]
    rooflines = {}
    for op, kname in (("F", "gemv_rows"), ("FADJ", "gemv_cols")):
        ach = h["product_bytes"][op] / (h["product_kernel_ms"][op] * 1e-3) / 1e9
        rooflines[op] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                         "kernel": kname, "avg_ms": h["product_kernel_ms"][op],
                         "bytes_per_launch": h["product_bytes"][op]}
    if read:
        for r in rooflines.values():
            r["frac_of_measured_read"] = round(r["achieved"] / read["gbs"], 4)
    traffic = load_traffic()
    if traffic is not None:
        for op, r in rooflines.items():
            kname = traffic["by_family"].get(f"{head}/{op}")
            if kname:
                kv = traffic["kernels"][kname]
                r["traffic"] = round(kv["read_bytes"] + kv["write_bytes"])
                r["traffic_kernel"] = kname
    dom = max(("F", "FADJ"), key=lambda o: h["product_kernel_ms"][o])
    out = {
        "metric": "F/F* apply time & HBM GB/s @Nd=600,Nt=420; mixed vs FP64 at stated rel err",
        "value": round(h["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed_bf16": "bf16x2/f32", "mixed_fp16": "f16x2/f32",
                  "fast_bf16": "bf16/f32"}[head],
        "data": "synthetic (seeded counter-based normals, generated on device)",
        "config": {"workload": f"p2o F+F* single RHS, Nd={Nd} Nm={Nm} Nt={Nt} "
                               f"(L={L}, {nf} frequency blocks), precision {head}",
                   "Nd": Nd, "Nm": Nm, "Nt": Nt, "L": L, "nrhs": 1, "precision": head},
        "roofline": rooflines[dom],
        "roofline_other": rooflines["FADJ" if dom == "F" else "F"],
        "paths": {p: {k: v for k, v in r.items()} for p, r in results.items()},
        "measured_read": read,
        "measured_copy": copy,
    }
    if "fp64" in results and head != "fp64":
        out["speedup_vs_fp64"] = round(results["fp64"]["ms_per_step"] / h["ms_per_step"], 3)
    if head in results and "mrhs" in results[head]:
        hb = results[head]["mrhs"]
        domB = max(("F", "FADJ"), key=lambda o: hb["product_kernel_ms"][o])
        out["mrhs"] = {"nrhs": B, "precision": head, "roofline": hb["roofline"][domB],
                       "roofline_other": hb["roofline"]["FADJ" if domB == "F" else "F"]}
        if "fp64" in results and "mrhs" in results["fp64"]:
            out["mrhs"]["speedup_vs_fp64"] = round(
                results["fp64"]["mrhs"]["ms_per_step"] / hb["ms_per_step"], 3)
    if not args.no_c2:
        out["c2_fp64"] = c2_fp64_leg(torch, S, P)
        print(f"[bench] 100x5000x200 fp64: {out['c2_fp64']}", file=sys.stderr, flush=True)
    if not args.no_inversion:
        out["inversion"] = bench_inversion(torch, S, P, cpu=not args.no_cpu_baseline)
        print(f"[bench] inversion: {out['inversion']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(torch, S, args, nf, h["step_bytes"], env)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
