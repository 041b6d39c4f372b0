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
    ap.add_argument("--precs", default="mixed_bf16,fp64,mixed_fp16")
    ap.add_argument("--cpu-cols", type=int, default=40000,
                    help="columns of the workload the CPU oracle baseline runs on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-gb", type=float, default=4.0,
                    help="size of the plain device copy timed as the measured HBM ceiling")
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


def n_chunks(Nd, Nm, nf):
    """Column chunking of the F product (mirrors the library's choice)."""
    base = nf * ((Nd + 3) // 4)
    n = max(1, (16384 + base - 1) // base)
    n = min(n, max(1, Nm // 256))
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not a measured path)", file=sys.stderr)
        sys.exit(2)
    import torch
    import p2o_synth as S
    import paper_2504_16344_amd as P

    Nd, Nm, Nt = args.Nd, args.Nm, args.Nt
    L = P.smooth_length(Nt)
    nf = L // 2 + 1
    n_pc = n_chunks(Nd, Nm, nf)
    precs = [p.strip() for p in args.precs.split(",") if p.strip()]
    stream = torch.cuda.current_stream()
    env = S.envelope(Nt, args.tau, 1.0 / np.sqrt(Nm))
    env_dev = torch.from_numpy(env).cuda()
    m = torch.empty((Nt, Nm), dtype=torch.float64, device="cuda")
    d = torch.empty((Nt, Nd), dtype=torch.float64, device="cuda")
    S.device_normals(m.data_ptr(), m.numel(), 0, args.seed, S.ARRAY_M, 1.0, stream.cuda_stream)
    S.device_normals(d.data_ptr(), d.numel(), 0, args.seed, S.ARRAY_D, 1.0, stream.cuda_stream)
    torch.cuda.synchronize()

    copy = measured_copy(torch, args.copy_gb) if args.copy_gb > 0 else None
    results = {}
    ref = None
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
        # per-op apply times (not overlapped with each other)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(args.steps):
            plan.F(m, out=yF)
        ev[1].record()
        for _ in range(args.steps):
            plan.FT(d, out=yA)
        ev[2].record()
        torch.cuda.synchronize()
        r = {
            "setup_s": round(t_setup, 3),
            "ms_per_step": wall * 1e3 / args.steps,
            "apply_ms": {"F": ev[0].elapsed_time(ev[1]) / args.steps,
                         "FADJ": ev[1].elapsed_time(ev[2]) / args.steps},
            "product_kernel_ms": {"F": msF / max(nF, 1), "FADJ": msA / max(nA, 1)},
            "product_bytes": {"F": product_bytes(prec, "F", Nd, Nm, nf, n_pc),
                              "FADJ": product_bytes(prec, "FADJ", Nd, Nm, nf, 1)},
            "step_bytes": step_bytes(prec, Nd, Nm, Nt, nf, n_pc),
            "autotune": tuned,
        }
        r["gbs"] = r["step_bytes"] / (r["ms_per_step"] * 1e-3) / 1e9
        if prec == "fp64":
            ref = (yF.clone(), yA.clone())
        elif ref is not None:
            eF = (torch.linalg.norm(yF - ref[0]) / torch.linalg.norm(ref[0])).item()
            eA = (torch.linalg.norm(yA - ref[1]) / torch.linalg.norm(ref[1])).item()
            r["rel_err_vs_fp64"] = {"F": eF, "FADJ": eA}
        results[prec] = r
        plan.close()
        del plan
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step, {r['gbs']:.0f} GB/s, "
              f"kernels F {r['product_kernel_ms']['F']:.3f} ms F* "
              f"{r['product_kernel_ms']['FADJ']:.3f} ms, setup {t_setup:.1f} s",
              file=sys.stderr, flush=True)

    head = precs[0]
    h = results[head]
    rooflines = {}
    for op, kname in (("F", "gemv_rows"), ("FADJ", "gemv_cols")):
        ach = h["product_bytes"][op] / (h["product_kernel_ms"][op] * 1e-3) / 1e9
        rooflines[op] = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                         "kernel": kname, "avg_ms": h["product_kernel_ms"][op],
                         "bytes_per_launch": h["product_bytes"][op]}
    if copy:
        for r in rooflines.values():
            r["frac_of_measured_copy"] = round(r["achieved"] / copy["gbs"], 4)
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
        "measured_copy": copy,
    }
    if "fp64" in results and head != "fp64":
        out["speedup_vs_fp64"] = round(results["fp64"]["ms_per_step"] / h["ms_per_step"], 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(torch, S, args, nf, h["step_bytes"], env)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
