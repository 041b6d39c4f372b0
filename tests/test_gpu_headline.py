"""The headline workload at its full size, in the launch configuration the
benchmark times: Nd = 600, Nm = 40000, Nt = 420 (L = 840, 421 frequency
blocks), blocks generated on the device and set up in 2048-column chunks,
both product kernels autotuned on the plan, one right-hand side (the
vector-unit kernels) and 64 (the matrix-core kernels of the many-RHS
benchmark); FP64 and bfloat16 hi+lo plans, each in its own lifetime (161.7
GB and 80.8 GB of frequency blocks).

Every output of F m and F* d is compared with the FP64 oracle for the
single right-hand side and for right-hand sides 0 and 63 of the 64-RHS
applies (right-hand side 0 of the 64 is the single one).  The oracle runs on
the host in 4096-column chunks: F and F* are separable over parameter
columns (F m sums the chunks' contributions, F* d produces each chunk's
columns), and each chunk's blocks are drawn on the device by the same
counter-based generator and copied to the host.  Further right-hand sides
of the 64 are checked on sampled outputs with the oracle's one-output forms.

Tolerances (normwise per right-hand side, and element-wise against the
largest output):
  * FP64: 1e-12.  Rounding of O(u64 log2 L) in the transforms; measured
    ~2e-15.
  * bfloat16 hi+lo, the stated bound 1e-5, and an expected-size bound
    derived from the encoding: random rounding of lo gives ~0.15 u16^2
    ~ 2.2e-6 normwise (u16 = 2^-8) plus float32 transforms (a few 1e-7):
    4e-6 for the vector-unit kernels; the matrix-core kernels also split the
    float32 vector into bfloat16 hi + lo (~2.5e-6 more, independent): 6e-6.
"""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P
from gpu_helpers import check_close

pytestmark = pytest.mark.gpu

ND, NM, NT, SEED, TAU, B = 600, 40000, 420, 3, 80.0, 64
FULL_RHS = (0, B - 1)
TOL = {"fp64": (1e-12, 1e-12), "mixed_bf16": (4e-6, 6e-6)}  # (vector units, matrix cores)
CHUNK = 4096


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


def _inputs(b):
    """Right-hand side b of the 64 (b = 0 is the single one), drawn on the
    device exactly as the applies draw them, copied to the host."""
    stream = torch.cuda.current_stream()
    m = torch.empty((NT, NM), dtype=torch.float64, device="cuda")
    d = torch.empty((NT, ND), dtype=torch.float64, device="cuda")
    S.device_normals(m.data_ptr(), m.numel(), b * NT * NM, SEED, S.ARRAY_M, 1.0, stream.cuda_stream)
    S.device_normals(d.data_ptr(), d.numel(), b * NT * ND, SEED, S.ARRAY_D, 1.0, stream.cuda_stream)
    return m.cpu().numpy(), d.cpu().numpy()


@pytest.fixture(scope="module")
def full_oracle():
    """F m_b and F* d_b for b in FULL_RHS over all 40000 columns (host, FP64)."""
    print("\n[headline] oracle over 4096-column chunks", flush=True)
    stream = torch.cuda.current_stream()
    env_dev = torch.from_numpy(S.envelope(NT, TAU, 1.0 / np.sqrt(NM))).cuda()
    ms, ds = zip(*(_inputs(b) for b in FULL_RHS))
    m, d = np.stack(ms), np.stack(ds)
    yF = np.zeros((len(FULL_RHS), NT, ND))
    yA = np.zeros((len(FULL_RHS), NT, NM))
    buf = torch.empty((NT, ND, CHUNK), dtype=torch.float64, device="cuda")
    for p0 in range(0, NM, CHUNK):
        p1 = min(NM, p0 + CHUNK)
        view = buf[:, :, : p1 - p0] if p1 - p0 == CHUNK else \
            torch.empty((NT, ND, p1 - p0), dtype=torch.float64, device="cuda")
        S.device_blocks(view.data_ptr(), NT, ND, NM, p0, p1, SEED, env_dev.data_ptr(),
                        stream.cuda_stream)
        blk = view.cpu().numpy()
        yF += oracle.apply_F(blk, np.ascontiguousarray(m[:, :, p0:p1]))
        yA[:, :, p0:p1] = oracle.apply_Fadj(blk, d)
        del blk
        print(f"  oracle columns {p0}..{p1 - 1} done", flush=True)
    del buf
    torch.cuda.empty_cache()
    return m, d, yF, yA


@pytest.mark.parametrize("prec", ["mixed_bf16", "fp64"])
def test_headline_600x40000x420_full(prec, full_oracle):
    m_ref, d_ref, yF_ref, yA_ref = full_oracle
    print(f"\n[headline] 600x40000x420 {prec}", flush=True)
    stream = torch.cuda.current_stream()
    env = S.envelope(NT, TAU, 1.0 / np.sqrt(NM))
    env_dev = torch.from_numpy(env).cuda()
    outs = {}
    plan = _plan(prec, env_dev, stream)
    try:
        for op in (P.OP_F, P.OP_FADJ):
            plan.autotune(op, reps=1)
        for nrhs in (1, B):
            shape_m = (NT, NM) if nrhs == 1 else (nrhs, NT, NM)
            shape_d = (NT, ND) if nrhs == 1 else (nrhs, NT, ND)
            m = torch.empty(shape_m, dtype=torch.float64, device="cuda")
            d = torch.empty(shape_d, dtype=torch.float64, device="cuda")
            S.device_normals(m.data_ptr(), m.numel(), 0, SEED, S.ARRAY_M, 1.0, stream.cuda_stream)
            S.device_normals(d.data_ptr(), d.numel(), 0, SEED, S.ARRAY_D, 1.0, stream.cuda_stream)
            for j, b in enumerate(FULL_RHS if nrhs == B else (0,)):  # the oracle's inputs
                assert np.array_equal(m.reshape(nrhs, NT, NM)[b].cpu().numpy(), m_ref[j])
                assert np.array_equal(d.reshape(nrhs, NT, ND)[b].cpu().numpy(), d_ref[j])
            y = plan.F(m).reshape(nrhs, NT, ND)
            x = plan.FT(d).reshape(nrhs, NT, NM)
            del m, d
            outs[nrhs] = (y.cpu().numpy(), x.cpu().numpy())
            del y, x
        torch.cuda.synchronize()
    finally:
        plan.close()
        torch.cuda.empty_cache()
    tv, tm = TOL[prec]
    # every output: the single right-hand side (vector units), and right-hand
    # sides 0 and 63 of the 64-RHS applies (matrix cores)
    check_close(outs[1][0], yF_ref[0], tv, "F   1 RHS, all outputs")
    check_close(outs[1][1], yA_ref[0], tv, "F*  1 RHS, all outputs")
    idx = list(FULL_RHS)
    check_close(outs[B][0][idx], yF_ref, tm, f"F   {B} RHS, rhs {idx}, all outputs")
    check_close(outs[B][1][idx], yA_ref, tm, f"F*  {B} RHS, rhs {idx}, all outputs")
    # sampled outputs of other right-hand sides of the 64
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(3):
        b = int(rng.integers(1, B - 1))
        t, s, p = int(rng.integers(NT)), int(rng.integers(ND)), int(rng.integers(NM))
        m_b, d_b = _inputs(b)
        rows = S.blocks(SEED, ND, NM, NT, env, s=[s])[:, 0, :]
        cols = S.blocks(SEED, ND, NM, NT, env, p=[p])[:, :, 0]
        ref = oracle.F_entry(rows, m_b, t)
        refa = oracle.Fadj_entry(cols, d_b, t)
        eF = abs(float(outs[B][0][b, t, s]) - ref) / np.abs(yF_ref).max()
        eA = abs(float(outs[B][1][b, t, p]) - refa) / np.abs(yA_ref).max()
        worst = max(worst, eF, eA)
        print(f"  rhs {b}: F[{t},{s}] err {eF:.2e}  F*[{t},{p}] err {eA:.2e}", flush=True)
    assert worst <= tm
