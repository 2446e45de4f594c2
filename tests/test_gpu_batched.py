"""Batched step (many independent 2-D periodic grids of uneven size in one
launch per step, optionally replayed from a HIP graph) against the oracle and
against single-grid runs of the same grids."""
import numpy as np
import pytest
import torch

import oracle
from paper_1407_1309_amd import mpdata, synth
from tests.gpu_util import TOL, as_dtype, dev, rel_l2

pytestmark = pytest.mark.gpu
FCT = 1


def _grids(shapes, seed, courant=0.4):
    children = np.random.SeedSequence(seed).spawn(len(shapes))
    out = []
    for shp, ch in zip(shapes, children):
        gen = np.random.Generator(np.random.PCG64(ch))
        c0, c1 = synth.stream_advector_2d(shp, courant, gen, n_modes=4, kmax=2)
        m = min(shp)
        psi = synth.blob_field(shp, 6, (max(m / 32, 1.0), max(m / 8, 2.0)), "uniform", gen)
        out.append((psi, c0, c1))
    return out


SHAPES = [(3, 3), (64, 64), (768, 64), (7, 300), (131, 97), (64, 768), (200, 5), (97, 131),
          (257, 255), (41, 43), (128, 128), (5, 700)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("n_iters,opts", [(2, FCT), (3, FCT), (2, FCT | mpdata.OPT_KAHAN)])
def test_batched_matches_oracle_and_single(dtype, n_iters, opts):
    grids = _grids(SHAPES, seed=11)
    bp = mpdata.BatchedPlan(SHAPES, dtype=dtype, n_iters=n_iters, opts=opts)
    psi = bp.pack([as_dtype(g[0], dtype) for g in grids], "psi")
    c0 = bp.pack([g[1] for g in grids], "c0")
    c1 = bp.pack([g[2] for g in grids], "c1")
    n_steps = 6
    bp.step(psi, c0, c1, n_steps=n_steps, use_graph=False)
    torch.cuda.synchronize()
    outs = bp.unpack(psi, "psi")
    for (p0, a, b), shp, got in zip(grids, SHAPES, outs):
        ref = oracle.step(as_dtype(p0, dtype), [as_dtype(a, dtype), as_dtype(b, dtype)],
                          n_iters=n_iters, opts=opts, n_steps=n_steps)
        assert rel_l2(got.double().cpu().numpy(), ref) <= TOL[dtype], shp
        single = dev(as_dtype(p0, dtype), dtype)
        plan = mpdata.Plan(shp, dtype=dtype, n_iters=n_iters, opts=opts)
        plan.step(single, [dev(a, dtype), dev(b, dtype)], n_steps=n_steps)
        torch.cuda.synchronize()
        assert torch.equal(single, got), shp        # tile-size independent, bit for bit


def test_batched_graph_replays_match_eager():
    grids = _grids(SHAPES, seed=12)
    dtype = torch.float32
    bp = mpdata.BatchedPlan(SHAPES, dtype=dtype, n_iters=2, opts=FCT)
    psi0 = bp.pack([g[0] for g in grids], "psi")
    c0 = bp.pack([g[1] for g in grids], "c0")
    c1 = bp.pack([g[2] for g in grids], "c1")
    eager = psi0.clone()
    graph = psi0.clone()
    for rep in range(3):
        bp.step(eager, c0, c1, n_steps=5, use_graph=False)
        bp.step(graph, c0, c1, n_steps=5, use_graph=True)
        torch.cuda.synchronize()
        _ = (eager * 2).sum().item()          # eager work between replays
        assert torch.equal(eager, graph), rep
    pg = psi0.clone()
    bp.step_per_grid(pg, c0, c1, n_steps=15)
    torch.cuda.synchronize()
    assert torch.equal(pg, graph)


def test_batched_tiling_and_autotune_bitwise():
    """Chunk length and tile order change only the speed: every tiling, and
    the autotuner's choice (also replayed from a graph), gives the same bits."""
    grids = _grids(SHAPES, seed=13)
    dtype = torch.float32
    bp = mpdata.BatchedPlan(SHAPES, dtype=dtype, n_iters=2, opts=FCT)
    psi0 = bp.pack([g[0] for g in grids], "psi")
    c0 = bp.pack([g[1] for g in grids], "c0")
    c1 = bp.pack([g[2] for g in grids], "c1")
    ref = None
    for rows, xcd in [(0, False), (1, True), (7, False), (16, True), (100, True), (1000, False)]:
        bp.set_tiling(rows, xcd)
        p = psi0.clone()
        bp.step(p, c0, c1, n_steps=4, use_graph=False)
        torch.cuda.synchronize()
        if ref is None:
            ref = p
        assert torch.equal(p, ref), (rows, xcd)
    rows, xcd = bp.autotune(psi0, c0, c1)
    assert rows > 0
    for use_graph in (False, True, True):
        p = psi0.clone()
        bp.step(p, c0, c1, n_steps=4, use_graph=use_graph)
        torch.cuda.synchronize()
        assert torch.equal(p, ref), (rows, xcd, use_graph)


def test_batched_workload_sampled():
    """1024 grids, sides uniform in [64, 768], FP32, n_iters=2 with the
    limiter, 100 steps, graph-captured: the smallest grids against the oracle
    over all 100 steps; every grid against its per-grid launch, bit for bit."""
    shapes = synth.batch_shapes()
    order = np.argsort([a * b for a, b in shapes])
    sample = [int(i) for i in order[:3]]
    cases = synth.case_batch()
    bp = mpdata.BatchedPlan(shapes, dtype=torch.float32, n_iters=2, opts=FCT)
    psi = bp.pack([c.psi for c in cases], "psi")
    c0 = bp.pack([c.c[0] for c in cases], "c0")
    c1 = bp.pack([c.c[1] for c in cases], "c1")
    ref_pg = psi.clone()
    bp.step(psi, c0, c1, n_steps=100, use_graph=True)
    bp.step_per_grid(ref_pg, c0, c1, n_steps=100)
    torch.cuda.synchronize()
    assert torch.equal(psi, ref_pg)
    outs = bp.unpack(psi, "psi")
    for i in sample:
        cs = cases[i]
        ref = oracle.step(as_dtype(cs.psi, torch.float32),
                          [as_dtype(x, torch.float32) for x in cs.c], n_iters=2, opts=FCT,
                          n_steps=100)
        assert rel_l2(outs[i].double().cpu().numpy(), ref) <= 1e-5, shapes[i]


def test_batched_rejects_bad_shapes():
    with pytest.raises(ValueError):
        mpdata.BatchedPlan([(64, 64), (2, 64)])


def test_autotune_cache_roundtrip(tmp_path):
    """The autotune cache stores a choice on a miss and restores it on a hit
    without timing, for a single grid and for a batch; each plan kind and
    shape has its own key, and a restored choice gives the same bits."""
    import json
    cache = str(tmp_path / "tune.json")
    case = synth.case_2d(n=192, n_iters=2, n_steps=1)
    plan = mpdata.Plan(case.psi.shape, n_iters=2, opts=FCT)
    psi = torch.from_numpy(case.psi).cuda()
    c = [torch.from_numpy(x).cuda() for x in case.c]
    th = plan.autotune(psi, c, cache=cache)
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0] == {"tile_rows": th}
    plan2 = mpdata.Plan(case.psi.shape, n_iters=2, opts=FCT)
    assert plan2.autotune(psi, c, cache=cache) == th
    a, b = psi.clone(), psi.clone()
    plan.step(a, c, n_steps=3)
    plan2.step(b, c, n_steps=3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)

    shapes = SHAPES[:6]
    grids = _grids(shapes, seed=21)
    bp = mpdata.BatchedPlan(shapes, n_iters=2, opts=FCT)
    psi0 = bp.pack([g[0] for g in grids], "psi")
    c0 = bp.pack([g[1] for g in grids], "c0")
    c1 = bp.pack([g[2] for g in grids], "c1")
    rows, xcd = bp.autotune(psi0, c0, c1, cache=cache)
    assert len(json.load(open(cache))) == 2
    bp2 = mpdata.BatchedPlan(shapes, n_iters=2, opts=FCT)
    assert bp2.autotune(psi0, c0, c1, cache=cache) == (rows, xcd)
    p, q = psi0.clone(), psi0.clone()
    bp.step(p, c0, c1, n_steps=2, use_graph=False)
    bp2.step(q, c0, c1, n_steps=2, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(p, q)
