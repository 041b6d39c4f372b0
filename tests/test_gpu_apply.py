"""Parity of the HIP path (through the C ABI) with the FP64 oracle for F and
F*, at small shapes spanning several tiles and ragged tails, and at the
100 x 5000 x 200 workload in full.  Tolerances: 1e-10 relative for the
float64 path (the target the method is held to); 1e-5 for the 16-bit hi+lo
paths (stated bound); 2e-2 for the bfloat16 hi-only tier.  Each is asserted
both normwise (per right-hand side) and element-wise (every output against
the largest output of its right-hand side; 2e-5 for bfloat16 hi+lo, whose
per-entry encoding error is up to 2^-16, gpu_helpers.TOL_VS_FP64)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2504_16344_amd as P
from gpu_helpers import TOL_VS_FP64, check_close, check_tier, dev, host, rel_err, workload

pytestmark = pytest.mark.gpu

TOL = TOL_VS_FP64

# (Nd, Nm, Nt, nrhs): the 8 x 64 x 32 workload, degenerate sizes, ragged
# column tails, odd and prime Nt (L = 196 for Nt = 97), Nt = 1, right-hand
# side counts that exercise every batching pass, the paper's Nd/Nt.
SHAPES = [
    (8, 64, 32, 1),
    (1, 1, 1, 1),
    (3, 5, 7, 2),
    (5, 300, 13, 3),
    (17, 1000, 97, 1),
    (2, 70, 1, 5),
    (130, 257, 33, 6),
    (600, 96, 420, 1),
    (7, 2100, 50, 1),
]


def _case(shape, seed=1):
    Nd, Nm, Nt, nrhs = shape
    return workload(seed, Nd, Nm, Nt, tau=max(Nt / 4, 1.0), nrhs=None if nrhs == 1 else nrhs)


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp16", "mixed_bf16", "fast_bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_apply_matches_oracle(shape, prec):
    print(f"\n[apply] shape={shape} prec={prec}", flush=True)
    blocks, m, d = _case(shape)
    ref_F = oracle.apply_F(blocks, m)
    ref_A = oracle.apply_Fadj(blocks, d)
    with P.Plan(dev(blocks), prec) as plan:
        yF = host(plan.F(dev(m)))
        yA = host(plan.FT(dev(d)))
        torch.cuda.synchronize()
    check_tier(yF, ref_F, prec, "F")
    check_tier(yA, ref_A, prec, "F*")


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp16", "mixed_bf16"])
def test_full_100x5000x200(prec):
    """The full 100 x 5000 x 200 workload (201 frequency blocks), F and F*."""
    print(f"\n[c2] prec={prec}", flush=True)
    Nd, Nm, Nt = 100, 5000, 200
    blocks, m, d = workload(2, Nd, Nm, Nt, tau=40.0)
    ref_F = oracle.apply_F(blocks, m)
    ref_A = oracle.apply_Fadj(blocks, ref_F)
    with P.Plan(dev(blocks), prec) as plan:
        assert plan.L == 400
        yF = plan.F(dev(m))
        yA = plan.FT(dev(ref_F))
        torch.cuda.synchronize()
    check_tier(host(yF), ref_F, prec, "F")
    check_tier(host(yA), ref_A, prec, "F*")


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16"])
def test_chunked_setup_equals_one_shot(prec):
    Nd, Nm, Nt = 9, 1300, 21
    blocks, m, d = workload(3, Nd, Nm, Nt, tau=6.0)
    bd = dev(blocks)
    with P.Plan(bd, prec) as one:
        y1 = one.F(dev(m))
        z1 = one.FT(dev(d))
        plan = P.Plan.begin(Nd, Nm, Nt, prec)
        for p0, p1 in ((512, 1300), (0, 256), (256, 512)):
            plan.setup_columns(bd[:, :, p0:p1].contiguous(), p0, p1)
        plan.setup_end()
        y2 = plan.F(dev(m))
        z2 = plan.FT(dev(d))
        torch.cuda.synchronize()
        plan.close()
    assert torch.equal(y1, y2) and torch.equal(z1, z2)


def test_repeat_applies_are_bitwise_identical():
    blocks, m, d = _case((130, 257, 33, 6))
    with P.Plan(dev(blocks), "fp64") as plan:
        a = [plan.F(dev(m)) for _ in range(3)]
        b = [plan.FT(dev(d)) for _ in range(3)]
        torch.cuda.synchronize()
    assert all(torch.equal(a[0], x) for x in a) and all(torch.equal(b[0], x) for x in b)


def test_error_codes():
    blocks, m, d = _case((3, 300, 5, 1))
    plan = P.Plan.begin(3, 300, 5, "mixed_fp16")
    bd = dev(blocks)
    with pytest.raises(P.P2OError) as e:       # misaligned column range (mixed)
        plan.setup_columns(bd[:, :, 10:300].contiguous(), 10, 300)
    assert e.value.status == 1
    with pytest.raises(P.P2OError) as e:       # apply before setup_end
        plan.F(dev(m))
    assert e.value.status == 5
    with pytest.raises(P.P2OError) as e:       # columns not all provided
        plan.setup_end()
    assert e.value.status == 5
    plan.setup_columns(bd[:, :, 0:256].contiguous(), 0, 256)
    plan.setup_columns(bd[:, :, 256:300].contiguous(), 256, 300)
    plan.setup_end()
    with pytest.raises(P.P2OError) as e:       # second setup_end
        plan.setup_end()
    assert e.value.status == 5
    lib = P.load_library()
    x = dev(m)
    assert lib.p2o_apply(plan.handle, 2, x.data_ptr(), x.data_ptr(), 1, None) == 1
    assert lib.p2o_apply(plan.handle, 0, x.data_ptr(), x.data_ptr(), 0, None) == 1
    assert lib.p2o_apply(plan.handle, 0, None, x.data_ptr(), 1, None) == 1
    y = plan.F(x)  # handle still usable after errors
    torch.cuda.synchronize()
    assert rel_err(host(y), oracle.apply_F(blocks, m)) < 1e-5
    plan.close()
    # a size whose frequency blocks cannot be allocated
    with pytest.raises(P.P2OError) as e:
        P.Plan.begin(60000, 10**9, 420, "fp64")
    assert e.value.status == 2
