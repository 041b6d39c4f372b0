"""Every candidate configuration of the block-product kernels gives the
oracle's result (to each precision's tolerance), the autotuner only picks
valid candidates, and its on-disk cache is applied to new plans."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2504_16344_amd as P
from gpu_helpers import TOL_VS_FP64, check_close, check_tier, dev, host, rel_err, workload

pytestmark = pytest.mark.gpu

TOL = TOL_VS_FP64
# Nm divisible by 4, by 2 only, and odd: vector widths 4, 2, 1 become (in)valid
SHAPES = [(130, 1028, 33), (9, 1026, 21), (5, 301, 13)]


@pytest.mark.parametrize("prec", list(TOL))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_every_candidate_matches_oracle(shape, prec):
    Nd, Nm, Nt = shape
    print(f"\n[candidates] shape={shape} prec={prec}", flush=True)
    blocks, m, d = workload(4, Nd, Nm, Nt, tau=Nt / 3)
    ref = {P.OP_F: oracle.apply_F(blocks, m), P.OP_FADJ: oracle.apply_Fadj(blocks, d)}
    x = {P.OP_F: dev(m), P.OP_FADJ: dev(d)}
    with P.Plan(dev(blocks), prec) as plan:
        for op in (P.OP_F, P.OP_FADJ):
            n = plan.config(op)[1]
            ran = 0
            for c in range(n):
                try:
                    plan.set_config(op, c)
                except P.P2OError as e:
                    assert e.status == 6  # vector width does not divide Nm
                    continue
                y = host(plan.apply(op, x[op]))
                check_tier(y, ref[op], prec, f"op={op} cfg={c}")
                ran += 1
            assert ran >= 1


def test_autotune_and_cache(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("P2O_TUNE_CACHE", str(cache))
    Nd, Nm, Nt = 64, 4096, 40
    blocks, m, d = workload(5, Nd, Nm, Nt, tau=10.0)
    bd = dev(blocks)
    chosen = {}
    with P.Plan(bd, "mixed_bf16") as plan:
        for op in (P.OP_F, P.OP_FADJ):
            c, times = plan.autotune(op, reps=2)
            print(f"\n  op={op} chosen={c} times={times}", flush=True)
            assert 0 <= c < len(times) and times[c] > 0
            assert times[c] == min(t for t in times if t >= 0)
            assert plan.config(op)[0] == c
            chosen[op] = c
        y = host(plan.F(dev(m)))
        assert rel_err(y, oracle.apply_F(blocks, m)) <= 1e-5
    stored = json.loads(cache.read_text())
    assert len(stored) == 2 and sorted(stored.values()) == sorted(chosen.values())
    with P.Plan(bd, "mixed_bf16") as plan2:       # a new plan picks the cached choice
        assert plan2.config(P.OP_F)[0] == chosen[P.OP_F]
        assert plan2.config(P.OP_FADJ)[0] == chosen[P.OP_FADJ]
