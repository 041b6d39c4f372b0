"""Many right-hand sides: the float64 matrix-core (MFMA) product kernels and
the vector-unit kernels both match the oracle, for ragged sensor counts
(not a multiple of 16), ragged column chunks, right-hand-side counts that
are not a multiple of 16 and that need two passes of 64."""
import numpy as np
import pytest
import torch

import oracle
import paper_2504_16344_amd as P
from gpu_helpers import check_close, dev, host, rel_err, workload

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1, 1), (37, 300, 13, 5), (17, 1000, 97, 20), (130, 1028, 33, 70),
          (600, 96, 420, 3), (100, 777, 40, 33)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_mfma_and_vector_paths_match_oracle(shape):
    Nd, Nm, Nt, nrhs = shape
    print(f"\n[multi-rhs] shape={shape}", flush=True)
    blocks, m, d = workload(11, Nd, Nm, Nt, tau=Nt / 3, nrhs=nrhs)
    ref_F = oracle.apply_F(blocks, m)
    ref_A = oracle.apply_Fadj(blocks, d)
    out = {}
    with P.Plan(dev(blocks), "fp64") as plan:
        for name, thr in (("mfma", 1), ("vector", 0)):
            plan.set_mfma_threshold(P.OP_F, thr)
            plan.set_mfma_threshold(P.OP_FADJ, thr)
            yF = host(plan.F(dev(m)))
            yA = host(plan.FT(dev(d)))
            check_close(yF, ref_F, 1e-10, f"{name} F")
            check_close(yA, ref_A, 1e-10, f"{name} F*")
            out[name] = (yF, yA)
    assert rel_err(out["mfma"][0], out["vector"][0]) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("mixed_bf16", 1e-5), ("fast_bf16", 2e-2)])
@pytest.mark.parametrize("shape", [(37, 300, 13, 5), (17, 1001, 97, 20), (130, 1028, 33, 70),
                                   (100, 777, 40, 33), (5, 4100, 8, 17), (20, 33, 9, 40),
                                   (12, 34, 7, 18), (140, 1030, 21, 36)],
                         ids=lambda s: "x".join(map(str, s)))
def test_bf16_matrix_core_path_matches_oracle(shape, prec, tol):
    """bfloat16 matrix-core products (hi+lo vector split, float32 accumulation)
    against the oracle and against the vector-unit products of the same tier
    (same operand precision: they differ by float32 rounding only, so a
    misplaced block entry shows far above it); Nm of every residue modulo 4
    exercises block rows at 16-, 8- and 4-byte alignment and every length of
    the last 32-entry chunk's ragged tail, Nm > 4096 several scale tiles per
    column chunk."""
    Nd, Nm, Nt, nrhs = shape
    print(f"\n[multi-rhs {prec}] shape={shape}", flush=True)
    blocks, m, d = workload(12, Nd, Nm, Nt, tau=Nt / 3, nrhs=nrhs)
    ref_F = oracle.apply_F(blocks, m)
    ref_A = oracle.apply_Fadj(blocks, d)
    out = {}
    with P.Plan(dev(blocks), prec) as plan:
        for name, thr in (("mfma", 1), ("vector", 0)):
            plan.set_mfma_threshold(P.OP_F, thr)
            plan.set_mfma_threshold(P.OP_FADJ, thr)
            out[name] = (host(plan.F(dev(m))), host(plan.FT(dev(d))))
            check_close(out[name][0], ref_F, tol, f"{name} F")
            check_close(out[name][1], ref_A, tol, f"{name} F*")
    for i, op in enumerate(("F", "F*")):
        assert rel_err(out["mfma"][i], out["vector"][i]) <= 1e-3, op


@pytest.mark.parametrize("op", ["F", "FADJ"])
def test_bf16_matrix_core_error_not_coherent_in_time(op):
    """Regression: the bfloat16 matrix-core F path once carried an error that
    added up coherently over the frequencies into the first output steps (a
    rounding bias of small addends in a large float32 accumulator).  Its
    error at t = 0, 1, 3, measured against the FP64 plan (itself checked
    against the oracle), must look like the error elsewhere: mean signed
    error over all outputs and right-hand sides small against its RMS.
    F: 200 x 20000 x 420, 16 right-hand sides (contraction over 4096-column
    chunks).  F*: 2048 sensors, so the contraction over sensors is as long as
    an F chunk's (64 steps of 32), at 2048 x 2000 x 420."""
    import p2o_synth as S
    Nd, Nm = (200, 20000) if op == "F" else (2048, 2000)
    Nt, B, seed = 420, 16, 8
    code = P.OP_F if op == "F" else P.OP_FADJ
    stream = torch.cuda.current_stream()
    env = torch.from_numpy(S.envelope(Nt, 80.0, 1.0 / np.sqrt(Nm))).cuda()
    n_in = Nm if op == "F" else Nd
    x = torch.empty((B, Nt, n_in), dtype=torch.float64, device="cuda")
    S.device_normals(x.data_ptr(), x.numel(), 0, seed, S.ARRAY_M if op == "F" else S.ARRAY_D,
                     1.0, stream.cuda_stream)
    ys = {}
    for prec in ("fp64", "mixed_bf16"):
        plan = P.Plan.begin(Nd, Nm, Nt, prec)
        for p0 in range(0, Nm, 2048):
            p1 = min(Nm, p0 + 2048)
            chunk = torch.empty((Nt, Nd, p1 - p0), dtype=torch.float64, device="cuda")
            S.device_blocks(chunk.data_ptr(), Nt, Nd, Nm, p0, p1, seed, env.data_ptr(),
                            stream.cuda_stream)
            plan.setup_columns(chunk, p0, p1)
            del chunk
        plan.setup_end()
        if prec != "fp64":
            plan.set_mfma_threshold(code, 1)
        ys[prec] = host(plan.apply(code, x))
        plan.close()
        torch.cuda.empty_cache()
    ref = ys["fp64"]
    sc = np.sqrt((ref ** 2).mean(axis=1, keepdims=True))
    en = (ys["mixed_bf16"] - ref) / sc
    for t in (0, 1, 3):
        mean, rms = float(en[:, t, :].mean()), float(np.sqrt((en[:, t, :] ** 2).mean()))
        print(f"\n  {op} t={t}: mean signed {mean:.2e}  rms {rms:.2e}", flush=True)
        assert abs(mean) <= 0.2 * rms
    assert rel_err(ys["mixed_bf16"], ref) <= 1e-5
