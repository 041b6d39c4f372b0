"""F forward and F* backward behind torch.autograd.Function: gradcheck at a
tiny size, and the gradient of 0.5 ||F m - d||^2 at the 100 x 5000 x 200
workload against the oracle's F*(F m - d) and against central differences
(exact for a quadratic up to rounding)."""
import numpy as np
import pytest
import torch

import oracle
import p2o_synth as S
import paper_2504_16344_amd as P
from gpu_helpers import dev, host, workload

pytestmark = pytest.mark.gpu


def test_gradcheck_tiny():
    blocks, m, d = workload(9, 3, 10, 6, tau=3.0)
    with P.Plan(dev(blocks), "fp64") as plan:
        x = dev(m).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda t: P.P2OApply.apply(plan, t), (x,),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)
        y = dev(d).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda t: P.P2OAdjoint.apply(plan, t), (y,),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)


def test_misfit_gradient_100x5000x200():
    Nd, Nm, Nt = 100, 5000, 200
    blocks, m, _ = workload(5, Nd, Nm, Nt, tau=40.0)
    d = S.vector(5, S.ARRAY_D, Nt * Nd).reshape(Nt, Nd)
    v = S.vector(5, S.ARRAY_DIRECTION, Nt * Nm).reshape(Nt, Nm)
    ref = oracle.misfit_gradient(blocks, m, d)
    with P.Plan(dev(blocks), "fp64") as plan:
        x = dev(m).requires_grad_(True)
        dd = dev(d)
        loss = 0.5 * ((P.P2OApply.apply(plan, x) - dd) ** 2).sum()
        loss.backward()
        g = host(x.grad)
        f = lambda t: 0.5 * float(((plan.F(t) - dd) ** 2).sum())
        h = 1e-3 * np.linalg.norm(m) / np.linalg.norm(v)
        vd = dev(v)
        fd = (f(dev(m) + h * vd) - f(dev(m) - h * vd)) / (2 * h)
    e = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    gv = float(np.vdot(g, v))
    print(f"\n  grad err vs oracle {e:.2e}; <g,v>={gv:.6e} fd={fd:.6e}", flush=True)
    assert e <= 1e-10
    assert abs(fd - gv) <= 1e-8 * abs(gv)
