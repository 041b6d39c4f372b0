"""The mixed tiers against the quantised-spectrum oracle (oracle/quantised.py):
the same encoded frequency blocks applied exactly in float64.  What remains
is the GPU's own arithmetic, so the tolerance is derived from float32, not
from the tiers' stated bound 1e-5.

Vector-unit kernels (one right-hand side and small counts): the blocks are
decoded exactly in float32 (hi has 8 or 11 significant bits, lo sits below
it, so hi + c lo fits float32's 24); the remaining errors are the float32
transforms, O(u32 log2 L) normwise with u32 = 2^-24 (Higham, "Accuracy and
Stability of Numerical Algorithms", section 24.1; ~6e-7 at L = 840 for the
worst case, a few 1e-7 for random rounding), and float32 accumulation of
at most 64 products per lane before a tree reduction (F chunk partials are
then added in float64).  Tolerance 2e-6: several times the random-rounding
size, five times below the stated bound, and below the bfloat16 encoding
error itself (~2e-6), so a kernel error as large as the encoding's fails.

Matrix-core kernels (bfloat16 tiers, many right-hand sides): the float32
vector spectra are also split into bfloat16 hi + lo, whose rounding error
is bounded like the blocks' (2^-16 per entry; ~2e-6 normwise for random
data), so the tolerance is 8e-6.
"""
import numpy as np
import pytest
import torch

import paper_2504_16344_amd as P
from gpu_helpers import check_close, dev, host, rel_err, workload
from oracle import quantised as Q

pytestmark = pytest.mark.gpu

ENC = {"mixed_bf16": ("bf16", True), "mixed_fp16": ("fp16", True), "fast_bf16": ("bf16", False)}
TOL_VECTOR = 2e-6
TOL_MATRIX = 8e-6

# (Nd, Nm, Nt, nrhs): tiles and ragged tails, several scale tiles (Nm > 256,
# Nm not a multiple of 256), prime Nt (L = 196), the paper's Nd and Nt.
SHAPES = [(8, 64, 32, 1), (3, 5, 7, 2), (5, 300, 13, 3), (17, 1000, 97, 1),
          (130, 257, 33, 6), (600, 96, 420, 1), (7, 2100, 50, 1), (64, 4100, 40, 2)]


def _refs(plan, blocks, m, d, prec):
    fmt, lo = ENC[prec]
    fq = Q.quantised_spectra(Q.spectra(blocks, plan.L), fmt, lo)
    return Q.apply_F_spectral(fq, m, plan.L), Q.apply_Fadj_spectral(fq, d, plan.L)


@pytest.mark.parametrize("prec", list(ENC))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_vector_units_match_quantised_oracle(shape, prec):
    Nd, Nm, Nt, nrhs = shape
    print(f"\n[quantised] shape={shape} prec={prec}", flush=True)
    blocks, m, d = workload(17, Nd, Nm, Nt, tau=max(Nt / 4, 1.0),
                            nrhs=None if nrhs == 1 else nrhs)
    with P.Plan(dev(blocks), prec) as plan:
        plan.set_mfma_threshold(P.OP_F, 0)
        plan.set_mfma_threshold(P.OP_FADJ, 0)
        refF, refA = _refs(plan, blocks, m, d, prec)
        yF = host(plan.F(dev(m)))
        yA = host(plan.FT(dev(d)))
        torch.cuda.synchronize()
    check_close(yF, refF, TOL_VECTOR, "F vs quantised oracle")
    check_close(yA, refA, TOL_VECTOR, "F* vs quantised oracle")


@pytest.mark.parametrize("prec", ["mixed_bf16", "fast_bf16"])
@pytest.mark.parametrize("shape", [(37, 300, 13, 5), (17, 1001, 97, 20), (130, 1028, 33, 70),
                                   (5, 4100, 8, 17)], ids=lambda s: "x".join(map(str, s)))
def test_matrix_cores_match_quantised_oracle(shape, prec):
    Nd, Nm, Nt, nrhs = shape
    print(f"\n[quantised, matrix cores] shape={shape} prec={prec}", flush=True)
    blocks, m, d = workload(18, Nd, Nm, Nt, tau=Nt / 3, nrhs=nrhs)
    with P.Plan(dev(blocks), prec) as plan:
        plan.set_mfma_threshold(P.OP_F, 1)
        plan.set_mfma_threshold(P.OP_FADJ, 1)
        refF, refA = _refs(plan, blocks, m, d, prec)
        yF = host(plan.F(dev(m)))
        yA = host(plan.FT(dev(d)))
        torch.cuda.synchronize()
    check_close(yF, refF, TOL_MATRIX, "F vs quantised oracle")
    check_close(yA, refA, TOL_MATRIX, "F* vs quantised oracle")


def test_quantised_oracle_explains_the_bf16_error():
    """At 100 x 5000 x 200 the bfloat16 hi+lo tier's error against the exact
    FP64 oracle (~2e-6) is the encoding's: against the quantised oracle it
    drops below the float32 tolerance."""
    import oracle
    Nd, Nm, Nt = 100, 5000, 200
    blocks, m, d = workload(2, Nd, Nm, Nt, tau=40.0)
    with P.Plan(dev(blocks), "mixed_bf16") as plan:
        refF, refA = _refs(plan, blocks, m, d, "mixed_bf16")
        yF = host(plan.F(dev(m)))
        yA = host(plan.FT(dev(d)))
        torch.cuda.synchronize()
    exF, exA = rel_err(yF, oracle.apply_F(blocks, m)), rel_err(yA, oracle.apply_Fadj(blocks, d))
    print(f"\n  vs exact oracle: F {exF:.2e} F* {exA:.2e}", flush=True)
    eF, _ = check_close(yF, refF, TOL_VECTOR, "F vs quantised oracle")
    eA, _ = check_close(yA, refA, TOL_VECTOR, "F* vs quantised oracle")
    assert exF > 2 * eF and exA > 2 * eA
