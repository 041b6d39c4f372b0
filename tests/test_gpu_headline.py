"""The headline workload at its full size, in the launch configuration the
benchmark times: Nd = 600, Nm = 40000, Nt = 420 (L = 840, 421 frequency
blocks), blocks generated on the device and set up in 2048-column chunks,
both product kernels autotuned on the plan, one right-hand side (the
vector-unit kernels) and 64 (the matrix-core kernels of the many-RHS
benchmark); FP64 and bfloat16 hi+lo plans, each in its own lifetime (161.7
GB and 80.8 GB of frequency blocks).  Sampled outputs of F m and F* d are checked one by one
against the oracle, with the block rows / columns and the input vectors
redrawn on the host from the same counter-based generator.

Error measure: |y - y*| over the output's full-history scale (as in the
batched full-size test).  FP64: 1e-11; bf16 hi+lo: 5e-5 (the normwise error
of this path is ~2e-6 and an element's error is spread like it)."""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P

pytestmark = pytest.mark.gpu

ND, NM, NT, SEED, TAU = 600, 40000, 420, 3, 80.0
TOL = {"fp64": 1e-11, "mixed_bf16": 5e-5}


def _plan(prec, env_dev, stream):
    plan = P.Plan.begin(ND, NM, NT, prec)
    chunk = 2048
    buf = torch.empty((NT, ND, chunk), dtype=torch.float64, device="cuda")
    for p0 in range(0, NM, chunk):
        p1 = min(NM, p0 + chunk)
        view = buf[:, :, : p1 - p0]
        if p1 - p0 != chunk:
            view = torch.empty((NT, ND, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(view.data_ptr(), NT, ND, NM, p0, p1, SEED, env_dev.data_ptr(),
                        stream.cuda_stream)
        plan.setup_columns(view, p0, p1)
    plan.setup_end()
    del buf
    return plan


@pytest.mark.parametrize("prec", ["mixed_bf16", "fp64"])
def test_headline_600x40000x420_sampled(prec):
    print(f"\n[headline] 600x40000x420 {prec}", flush=True)
    stream = torch.cuda.current_stream()
    env = S.envelope(NT, TAU, 1.0 / np.sqrt(NM))
    env_dev = torch.from_numpy(env).cuda()
    outs = {}
    plan = _plan(prec, env_dev, stream)
    try:
        for op in (P.OP_F, P.OP_FADJ):
            plan.autotune(op, reps=1)
        for nrhs in (1, 64):
            shape_m = (NT, NM) if nrhs == 1 else (nrhs, NT, NM)
            shape_d = (NT, ND) if nrhs == 1 else (nrhs, NT, ND)
            m = torch.empty(shape_m, dtype=torch.float64, device="cuda")
            d = torch.empty(shape_d, dtype=torch.float64, device="cuda")
            S.device_normals(m.data_ptr(), m.numel(), 0, SEED, S.ARRAY_M, 1.0, stream.cuda_stream)
            S.device_normals(d.data_ptr(), d.numel(), 0, SEED, S.ARRAY_D, 1.0, stream.cuda_stream)
            y = plan.F(m).reshape(nrhs, NT, ND)
            x = plan.FT(d).reshape(nrhs, NT, NM)
            del m, d
            outs[nrhs] = (y, x)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rng = np.random.default_rng(7)
    worst = 0.0
    for nrhs, (y, x) in outs.items():
        for t, s, b in ((NT - 1, 0, nrhs - 1), (0, ND - 1, 0),
                        (int(rng.integers(NT)), int(rng.integers(ND)), int(rng.integers(nrhs)))):
            rows = S.blocks(SEED, ND, NM, NT, env, s=[s])[:, 0, :]
            m_b = S.vector(SEED, S.ARRAY_M, NT * NM, offset=b * NT * NM).reshape(NT, NM)
            ref = oracle.F_entry(rows, m_b, t)
            msq = float(np.mean(np.sum(m_b * m_b, axis=1)))
            scale = np.sqrt(sum(float(rows[k] @ rows[k]) for k in range(NT)) * msq / NM)
            err = abs(float(y[b, t, s]) - ref) / scale
            worst = max(worst, err)
            print(f"  nrhs {nrhs}: F[{b},{t},{s}] err {err:.2e}", flush=True)
        for t, p, b in ((0, 0, 0), (NT - 1, NM - 1, nrhs - 1),
                        (int(rng.integers(NT)), int(rng.integers(NM)), int(rng.integers(nrhs)))):
            cols = S.blocks(SEED, ND, NM, NT, env, p=[p])[:, :, 0]
            d_b = S.vector(SEED, S.ARRAY_D, NT * ND, offset=b * NT * ND).reshape(NT, ND)
            ref = oracle.Fadj_entry(cols, d_b, t)
            dsq = float(np.mean(np.sum(d_b * d_b, axis=1)))
            scale = np.sqrt(sum(float(cols[k] @ cols[k]) for k in range(NT)) * dsq / ND)
            err = abs(float(x[b, t, p]) - ref) / scale
            worst = max(worst, err)
            print(f"  nrhs {nrhs}: F*[{b},{t},{p}] err {err:.2e}", flush=True)
    del outs
    torch.cuda.empty_cache()
    assert worst <= TOL[prec]


def host(t):
    return t.detach().cpu().numpy()
