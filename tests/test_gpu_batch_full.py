"""The batched uneven-instance workload at its real sizes: all 64 instances of
the seeded draw (Nt = 420, Nd in 50..600, Nm in 1000..20000, 1..256
right-hand sides each), set up from blocks generated on the device and
applied in memory-resident waves, one batch per wave (bfloat16 hi+lo,
matrix cores where the right-hand-side count calls for it), as the
benchmark runs them.  Every instance is checked on sampled outputs of its
first and last right-hand side (first, last and random steps; random
sensors and columns), each computed by the oracle's one-output forms from
block rows / columns drawn by the same counter-based generator.

Error measure: |y - y*| over the output's full-history scale (the root of
the summed squared sizes of all terms any output of that row / column can
hold), the element-wise counterpart of the normwise relative error.  The
mixed path's rounding error is spread evenly over time by the inverse
transform, so a single element's error is a random variable with standard
deviation about the normwise error (~3.5e-6 on the matrix-core path, ~2e-6
on the vector units); the tolerance 2e-5 sits about six standard
deviations out.
"""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P

pytestmark = pytest.mark.gpu

SEED, NT, N_ALL = 4, 420, 64
BUDGET = 200e9
TOL = 2e-5


def _env(Nm):
    return S.envelope(NT, 80.0, 1.0 / np.sqrt(Nm))


def _plan(i, Nd, Nm, prec):
    env = torch.from_numpy(_env(Nm)).cuda()
    plan = P.Plan.begin(Nd, Nm, NT, prec)
    stream = torch.cuda.current_stream()
    for p0 in range(0, Nm, 2048):
        p1 = min(Nm, p0 + 2048)
        chunk = torch.empty((NT, Nd, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(chunk.data_ptr(), NT, Nd, Nm, p0, p1, 1000 * SEED + i, env.data_ptr(),
                        stream.cuda_stream)
        plan.setup_columns(chunk, p0, p1)
        del chunk
    plan.setup_end()
    return plan


def _rows_cols(i, Nd, Nm, ss, ps):
    """Block rows F_k[s, :] for s in ss and columns F_k[:, p] for p in ps
    (all k), drawn on the device chunk by chunk and copied to the host."""
    env = torch.from_numpy(_env(Nm)).cuda()
    stream = torch.cuda.current_stream()
    rows = np.empty((len(ss), NT, Nm))
    cols = np.empty((len(ps), NT, Nd))
    sidx = torch.tensor(ss, device="cuda")
    for p0 in range(0, Nm, 2048):
        p1 = min(Nm, p0 + 2048)
        chunk = torch.empty((NT, Nd, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(chunk.data_ptr(), NT, Nd, Nm, p0, p1, 1000 * SEED + i, env.data_ptr(),
                        stream.cuda_stream)
        rows[:, :, p0:p1] = chunk.index_select(1, sidx).permute(1, 0, 2).cpu().numpy()
        for j, p in enumerate(ps):
            if p0 <= p < p1:
                cols[j] = chunk[:, :, p - p0].cpu().numpy()
        del chunk
    return rows, cols


def _need(Nd, Nm, R, nf):
    """Device bytes of a resident instance, with room to spare: blocks,
    transform and product workspaces, inputs and outputs."""
    return 8 * nf * Nd * Nm + 3 * 8 * R * nf * (Nm + Nd) + 2 * 8 * R * NT * (Nm + Nd)


def test_batched_instances_full_size_all_64_sampled():
    Nd = S.uniform_ints(SEED, S.ARRAY_SHAPES, N_ALL, 50, 600)
    Nm = S.uniform_ints(SEED, S.ARRAY_SHAPES, N_ALL, 1000, 20000, offset=N_ALL)
    R = S.uniform_ints(SEED, S.ARRAY_SHAPES, N_ALL, 1, 256, offset=2 * N_ALL)
    nf = P.smooth_length(NT) // 2 + 1
    waves, cur, used = [], [], 0
    for i in range(N_ALL):
        need = _need(int(Nd[i]), int(Nm[i]), int(R[i]), nf)
        if cur and used + need > BUDGET:
            waves.append(cur)
            cur, used = [], 0
        cur.append(i)
        used += need
    waves.append(cur)
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(0)
    worst, checked = 0.0, 0
    for w, ids in enumerate(waves):
        print(f"\n[batch full] wave {w}: instances {ids}", flush=True)
        plans, ms, ds = [], [], []
        for i in ids:
            nd, nm, r = int(Nd[i]), int(Nm[i]), int(R[i])
            plans.append(_plan(i, nd, nm, "mixed_bf16"))
            m = torch.empty((r, NT, nm), dtype=torch.float64, device="cuda")
            d = torch.empty((r, NT, nd), dtype=torch.float64, device="cuda")
            S.device_normals(m.data_ptr(), m.numel(), 0, 1000 * SEED + i, S.ARRAY_M, 1.0,
                             stream.cuda_stream)
            S.device_normals(d.data_ptr(), d.numel(), 0, 1000 * SEED + i, S.ARRAY_D, 1.0,
                             stream.cuda_stream)
            ms.append(m)
            ds.append(d)
        batch = P.Batch(plans)
        yF = batch.apply(P.OP_F, ms)
        yA = batch.apply(P.OP_FADJ, ds)
        torch.cuda.synchronize()
        batch.close()
        for p in plans:
            p.close()
        del plans, batch
        torch.cuda.empty_cache()
        for j, i in enumerate(ids):
            nd, nm, r = int(Nd[i]), int(Nm[i]), int(R[i])
            ss = [0, int(rng.integers(nd)), nd - 1]
            ps = [0, int(rng.integers(nm)), nm - 1]
            rows, cols = _rows_cols(i, nd, nm, ss, ps)
            for b in sorted({0, r - 1}):
                m_b = ms[j][b].cpu().numpy()
                d_b = ds[j][b].cpu().numpy()
                msq = float(np.mean(np.sum(m_b * m_b, axis=1)))
                dsq = float(np.mean(np.sum(d_b * d_b, axis=1)))
                yFb = yF[j][b].cpu().numpy()
                yAb = yA[j][b].cpu().numpy()
                for (t, q) in ((0, 0), (NT - 1, 2), (int(rng.integers(NT)), 1)):
                    s, p = ss[q], ps[q]
                    ref = oracle.F_entry(rows[q], m_b, t)
                    scale = np.sqrt(np.sum(rows[q] * rows[q]) * msq / nm)
                    eF = abs(float(yFb[t, s]) - ref) / scale
                    refa = oracle.Fadj_entry(cols[q], d_b, t)
                    scalea = np.sqrt(np.sum(cols[q] * cols[q]) * dsq / nd)
                    eA = abs(float(yAb[t, p]) - refa) / scalea
                    worst = max(worst, eF, eA)
                    checked += 2
                print(f"  inst {i} ({nd}x{nm}, {r} RHS) rhs {b}: worst so far {worst:.2e}",
                      flush=True)
        del ms, ds, yF, yA
        torch.cuda.empty_cache()
    print(f"  {checked} sampled outputs over {N_ALL} instances in {len(waves)} waves: "
          f"worst {worst:.2e}", flush=True)
    assert worst <= TOL
