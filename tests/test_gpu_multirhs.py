"""Many right-hand sides: the float64 matrix-core (MFMA) product kernels and
the vector-unit kernels both match the oracle, for ragged sensor counts
(not a multiple of 16), ragged column chunks, right-hand-side counts that
are not a multiple of 16 and that need two passes of 64."""
import numpy as np
import pytest
import torch

import oracle
import paper_2504_16344_amd as P
from gpu_helpers import dev, host, rel_err, workload

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
            eF, eA = rel_err(yF, ref_F), rel_err(yA, ref_A)
            print(f"  {name}: F {eF:.2e}  F* {eA:.2e}", flush=True)
            assert eF <= 1e-10 and eA <= 1e-10
            out[name] = (yF, yA)
    assert rel_err(out["mfma"][0], out["vector"][0]) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("mixed_bf16", 1e-5), ("fast_bf16", 2e-2)])
@pytest.mark.parametrize("shape", [(37, 300, 13, 5), (17, 1001, 97, 20), (130, 1028, 33, 70),
                                   (100, 777, 40, 33), (5, 4100, 8, 17)],
                         ids=lambda s: "x".join(map(str, s)))
def test_bf16_matrix_core_path_matches_oracle(shape, prec, tol):
    """bfloat16 matrix-core products (hi+lo vector split, float32 accumulation)
    against the oracle; odd Nm exercises the unaligned block loads and
    Nm > 4096 several scale tiles per column chunk."""
    Nd, Nm, Nt, nrhs = shape
    print(f"\n[multi-rhs {prec}] shape={shape}", flush=True)
    blocks, m, d = workload(12, Nd, Nm, Nt, tau=Nt / 3, nrhs=nrhs)
    ref_F = oracle.apply_F(blocks, m)
    ref_A = oracle.apply_Fadj(blocks, d)
    with P.Plan(dev(blocks), prec) as plan:
        for name, thr in (("mfma", 1), ("vector", 0)):
            plan.set_mfma_threshold(P.OP_F, thr)
            plan.set_mfma_threshold(P.OP_FADJ, thr)
            eF = rel_err(host(plan.F(dev(m))), ref_F)
            eA = rel_err(host(plan.FT(dev(d))), ref_A)
            print(f"  {name}: F {eF:.2e}  F* {eA:.2e}", flush=True)
            assert eF <= tol and eA <= tol
