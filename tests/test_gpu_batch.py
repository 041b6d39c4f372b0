"""Batched uneven instances through the C ABI: one persistent product launch
over all instances, each on its own path (vector units for few right-hand
sides, matrix cores for many), bitwise equal to the single-plan applies and
within tolerance of the oracle; a captured HIP graph replayed several
times, with eager work and synchronisations between replays and a changed
input, matches the eager results bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import paper_2504_16344_amd as P
from gpu_helpers import TOL_VS_FP64, check_close, check_tier, dev, host, workload

pytestmark = pytest.mark.gpu

TOL = TOL_VS_FP64
# (Nd, Nm, Nt, nrhs): uneven shapes, odd and even Nm, 1..70 right-hand sides
# (Nd = 100 with 40: two 64-sensor tiles, one of them ragged, on the FP64
# matrix cores)
INSTANCES = [(1, 1, 5, 1), (37, 300, 13, 5), (130, 1028, 33, 70), (17, 1001, 21, 20),
             (64, 777, 40, 3), (5, 4100, 8, 17), (9, 512, 1, 9), (100, 300, 11, 40)]


def _setup(prec, seed=21):
    cases, plans = [], []
    for i, (Nd, Nm, Nt, r) in enumerate(INSTANCES):
        blocks, m, d = workload(seed + i, Nd, Nm, Nt, tau=max(Nt / 3, 1.0), nrhs=r)
        cases.append((blocks, m, d))
        plans.append(P.Plan(dev(blocks), prec))
    return cases, plans


@pytest.mark.parametrize("prec", list(TOL))
def test_batch_matches_single_plans_and_oracle(prec):
    print(f"\n[batch] prec={prec}", flush=True)
    cases, plans = _setup(prec)
    batch = P.Batch(plans)
    for op in (P.OP_F, P.OP_FADJ):
        xs = [dev(c[1] if op == P.OP_F else c[2]) for c in cases]
        ys = batch.apply(op, xs)
        torch.cuda.synchronize()
        for (blocks, m, d), p, x, y in zip(cases, plans, xs, ys):
            single = p.apply(op, x)
            ref = oracle.apply_F(blocks, m) if op == P.OP_F else oracle.apply_Fadj(blocks, d)
            assert torch.equal(y, single), (p.Nd, p.Nm, p.Nt)
            check_tier(host(y), ref, prec, f"op={op} {p.Nd}x{p.Nm}x{p.Nt}")
        print(f"  op={op}: {len(plans)} instances equal to single applies", flush=True)
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_bf16"])
def test_graph_replays_match_eager(prec):
    cases, plans = _setup(prec, seed=40)
    batch = P.Batch(plans)
    for op in (P.OP_F, P.OP_FADJ):
        xs = [dev(c[1] if op == P.OP_F else c[2]) for c in cases]
        ys = [torch.full_like(p.apply(op, x), float("nan")) for p, x in zip(plans, xs)]
        graph = batch.capture(op, xs, ys)
        eager = batch.apply(op, xs)
        torch.cuda.synchronize()
        for rep in range(3):
            for y in ys:
                y.fill_(float("nan"))
            graph.launch()
            torch.cuda.synchronize()
            for y, e in zip(ys, eager):
                assert torch.equal(y, e), (op, rep)
            _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
        for x in xs:  # new input in the same buffers
            x.mul_(-0.5).add_(0.25)
        graph.launch()
        eager2 = batch.apply(op, xs)
        torch.cuda.synchronize()
        for y, e in zip(ys, eager2):
            assert torch.equal(y, e)
        graph.close()
    batch.close()


def test_batch_argument_errors():
    cases, plans = _setup("fp64", seed=60)
    with pytest.raises(P.P2OError) as e:
        P.Batch([plans[0], plans[0]])
    assert e.value.status == 1
    other = P.Plan(dev(cases[1][0]), "mixed_bf16")
    with pytest.raises(P.P2OError) as e:
        P.Batch([plans[0], other])
    assert e.value.status == 1
    other.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("prec", list(TOL))
def test_every_batch_configuration_is_bitwise_equal(prec):
    """Each configuration of the persistent kernel (vector-unit tiles) gives
    the same bits as configuration 0 and as the single-plan applies, for
    both ops (matrix-core instances of the bfloat16 tiers take their own
    launches of the single-plan kernels)."""
    print(f"\n[batch cfg] prec={prec}", flush=True)
    cases, plans = _setup(prec, seed=70)
    batch = P.Batch(plans)
    n = batch.config(P.OP_F)[1]
    assert n >= 2
    for op in (P.OP_F, P.OP_FADJ):
        xs = [dev(c[1] if op == P.OP_F else c[2]) for c in cases]
        singles = [p.apply(op, x) for p, x in zip(plans, xs)]
        for cfg in range(n):
            batch.set_config(op, cfg)
            assert batch.config(op)[0] == cfg
            ys = batch.apply(op, xs)
            torch.cuda.synchronize()
            for y, s1 in zip(ys, singles):
                assert torch.equal(y, s1), (op, cfg)
        print(f"  op={op}: {n} configurations equal", flush=True)
    with pytest.raises(P.P2OError) as e:
        batch.set_config(P.OP_F, n)
    assert e.value.status == 1
    batch.close()
    for p in plans:
        p.close()


def test_batch_autotune_and_cache(tmp_path, monkeypatch):
    """The autotuner times every configuration, keeps a valid one, stores it
    in the tune cache, and a new batch of the same shapes picks it up from
    there (its results unchanged)."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("P2O_TUNE_CACHE", str(cache))
    cases, plans = _setup("mixed_bf16", seed=80)
    batch = P.Batch(plans)
    for op in (P.OP_F, P.OP_FADJ):
        xs = [dev(c[1] if op == P.OP_F else c[2]) for c in cases]
        chosen, times = batch.autotune(op, xs, reps=1)
        print(f"\n  op={op} chosen {chosen} times {times}", flush=True)
        assert 0 <= chosen < len(times) and all(t > 0 for t in times)
        assert batch.config(op)[0] == chosen
        ref = batch.apply(op, xs)
        fresh = P.Batch(plans)
        assert fresh.config(op)[0] == -1  # nothing set: the cache decides at apply time
        ys = fresh.apply(op, xs)
        torch.cuda.synchronize()
        for y, r in zip(ys, ref):
            assert torch.equal(y, r)
        fresh.close()
    text = cache.read_text()
    assert "|batch|" in text
    batch.close()
    for p in plans:
        p.close()
