"""Uneven batches: persistent longest-first scheduling, graph capture, autotuner.

Bar: the same instance gives bit-identical results under every launch shape (each instance is
computed by one workgroup in a fixed order); solutions match the oracle as in the uniform
tests (rel_res <= 1e-10 by the library and by the oracle's residual; forward error <= 1e-7 for
this workload, whose KKT condition numbers reach ~5e5)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import kkt, riccati

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import api, tune  # noqa: E402
from gpu_util import forward_error, instance_solution, run  # noqa: E402


def _solve(plan, data, mode_max_it=0, tol=1e-10):
    ws = plan.workspace()
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
    its = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    x, u, lam = plan.empty_outputs()
    L.factor(plan, data, ws, info)
    L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=tol, max_it=mode_max_it)
    torch.cuda.synchronize()
    return x, u, lam, rel.cpu().numpy(), info.cpu().numpy(), its.cpu().numpy()


def _ragged_sample(n=48):
    # a spread of the uneven workload's instances, reduced horizons for speed
    insts = synth.make_ragged(n)
    for p in insts:
        if p.N > 40:
            p.A, p.B, p.R, p.r = p.A[:40], p.B[:40], p.R[:40], p.r[:40]
            p.Q, p.q = p.Q[:41], p.q[:41]
    return insts


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8)])
def test_launch_shapes_give_identical_results(mode, max_it):
    """Every launch shape of a variant gives bit-identical results (the work of an instance does
    not depend on where it runs); the tile and generic variants agree to rounding."""
    insts = _ragged_sample()
    print(f"case: ragged launch shapes {mode}", flush=True)
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode=mode)
    assert plan.variant == "tile" and plan.get_launch()["persistent"] == 1
    data = L.pack(insts)
    refs = {}
    for c in tune.candidates(plan):
        plan.set_variant(c["variant"])
        plan.set_launch(**c["launch"])
        out = _solve(plan, data, max_it)
        assert np.all(out[4] == 0), (c, out[4])
        assert out[3].max() <= 1e-10, (c, out[3].max())
        ref = refs.setdefault(c["variant"], out)
        for a, b in zip(out[:3], ref[:3]):
            assert torch.equal(a, b), c
    assert set(refs) == {"tile", "generic"}
    for i in range(len(insts)):
        sols = [(L.unpack(plan, "x", r[0], i), L.unpack(plan, "u", r[1], i), L.unpack(plan, "lam", r[2], i))
                for r in refs.values()]
        assert forward_error(sols[0], sols[1]) <= (1e-11 if mode == "f64" else 1e-8), i


def test_ragged_matches_oracle_f64_and_mixed():
    insts = _ragged_sample(24)
    print("case: ragged vs oracle", flush=True)
    for mode, max_it in (("f64", 0), ("mixed_f32", 8)):
        res = run(insts, mode, max_it=max_it)
        assert np.all(res["info"] == 0)
        assert res["rel"].max() <= 1e-10
        for i, p in enumerate(insts):
            sol = instance_solution(res, i)
            assert kkt.residual(p, *sol)[1] <= 1e-10
            assert forward_error(sol, riccati.solve(p)) <= 1e-7, (mode, i)


def test_full_uneven_workload_sampled():
    """All 2048 instances of the uneven workload in one persistent launch (f64 and mixed), the
    library's residual for every instance, the oracle on a sample."""
    print("case: full uneven workload (2048 instances)", flush=True)
    insts = synth.make_ragged(2048)
    plan64 = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="f64")
    data = L.pack(insts)
    for mode, max_it in (("f64", 0), ("mixed_f32", 8)):
        plan = plan64 if mode == "f64" else L.Plan(plan64.N, plan64.nx, plan64.nu, mode=mode)
        x, u, lam, rel, info, its = _solve(plan, data, max_it)
        print(f"  {mode}: max rel_res {rel.max():.2e}, iterations max {its.max()}", flush=True)
        assert np.all(info == 0)
        assert rel.max() <= 1e-10
        for i in (0, 1, 500, 1023, 2047):
            sol = (L.unpack(plan, "x", x, i), L.unpack(plan, "u", u, i), L.unpack(plan, "lam", lam, i))
            assert kkt.residual(insts[i], *sol)[1] <= 1e-10


@pytest.mark.parametrize("kind", ["ragged", "uniform_small"])
def test_graph_capture_replays_match_eager(kind):
    print(f"case: graph capture {kind}", flush=True)
    if kind == "ragged":
        insts = _ragged_sample(20)
        plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="mixed_f32")
        data = L.pack(insts)
    else:
        b = synth.make_batch(2, batch=64)
        plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode="mixed_f32")
        data = L.pack(b)
    ex, eu, el, erel, einfo, _ = _solve(plan, data, 8)
    ws = plan.workspace()
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
    x, u, lam = plan.empty_outputs()
    g = api.capture(plan, data, ws, x, u, lam, rel, None, info, tol=1e-10, max_it=8)
    for rep in range(4):
        # eager work of the program between replays
        x.fill_(float("nan"))
        u.zero_()
        junk = (data["A"][:1000] * 2.0).sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, ex) and torch.equal(u, eu) and torch.equal(lam, el), rep
        assert np.array_equal(rel.cpu().numpy(), erel), rep
        assert float(junk) == float(junk)


def test_autotuner_records_and_reapplies(tmp_path):
    print("case: autotuner", flush=True)
    insts = _ragged_sample(32)
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="f64")
    data = L.pack(insts)
    path = str(tmp_path / "tune.json")
    choice = tune.tune(plan, data, path=path, reps=1)
    assert choice["launch"] == plan.get_launch() and choice["variant"] == plan.variant
    db = json.load(open(path))
    assert len(db) == 1 and len(next(iter(db.values()))["tried"]) == len(tune.candidates(plan))
    other = L.Plan(plan.N, plan.nx, plan.nu, mode="f64")
    assert tune.apply_cached(other, path) is not None
    assert other.get_launch() == choice["launch"] and other.variant == choice["variant"]


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8)])
def test_ragged_tile_plan_launches_per_kernel_shape(mode, max_it):
    """A ragged tile plan groups its instances by kernel shape (one launch per group per call): the
    groups together cover every instance exactly once (each solved, residual certified, oracle
    checked on a sample), with and without the persistent grid, and agree with the generic
    variant to rounding.  Uniform and checkpointed plans keep one group."""
    insts = _ragged_sample(48)
    shapes = {((p.nx + 15) // 16 + (p.nu + 15) // 16 <= 3, p.nx <= 32, p.nu <= 16) for p in insts}
    print(f"case: per-shape launches {mode}, {len(shapes)} shape classes", flush=True)
    data = L.pack(insts)
    Ns, nxs, nus = [p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts]
    plan = L.Plan(Ns, nxs, nus, mode=mode)
    assert plan.variant == "tile" and plan.launch_groups >= 2, plan.launch_groups
    ref = None
    for persistent in (1, 0):
        plan.set_launch(threads=128, persistent=persistent, blocks_per_cu=0)
        x, u, lam, rel, info, its = _solve(plan, data, max_it)
        assert np.all(info == 0) and rel.max() <= 1e-10, (info, rel.max())
        sols = [(L.unpack(plan, "x", x, i), L.unpack(plan, "u", u, i), L.unpack(plan, "lam", lam, i))
                for i in range(len(insts))]
        if ref is None:
            ref = sols
        else:
            for a_, b_ in zip(sols, ref):
                assert all(np.array_equal(p_, q_) for p_, q_ in zip(a_, b_))
    for i in (0, 7, 23, 47):
        assert kkt.residual(insts[i], *ref[i])[1] <= 1e-10, i
    gplan = L.Plan(Ns, nxs, nus, mode=mode)
    gplan.set_variant("generic")
    assert gplan.launch_groups == 1
    gx, gu, glam, grel, ginfo, _ = _solve(gplan, data, max_it)
    for i in range(len(insts)):
        g = (L.unpack(gplan, "x", gx, i), L.unpack(gplan, "u", gu, i), L.unpack(gplan, "lam", glam, i))
        assert forward_error(ref[i], g) <= 1e-8, i
    assert L.Plan(20, 30, 8, batch=5, mode=mode).launch_groups == 1
    assert L.Plan(Ns, nxs, nus, mode=mode, ckpt_stride=5).launch_groups == 1
