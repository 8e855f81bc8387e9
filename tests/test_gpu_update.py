"""Factorisation updates on the GPU (include/lqupdate.h) against the oracle's refactorisation of the
modified problem (oracle/update.py).

* lq_update_data: R, S, Q after the penalty changes of eq. low-rank-update-Hj, entry by entry
  against ``update.modified_problem`` (<= 1e-14 of the largest entry of each stage block).
* lq_factor_update: the updated factors of every stage against the Cholesky factors of the
  modified problem's recursion (unique for positive diagonals): <= 1e-11 of the stage block's
  largest entry (a hyperbolic transformation per pivot and change, float64); the solution that
  lq_solve then returns against the oracle's solve of the modified problem (forward error
  <= 1e-9) with the library's float64 KKT residual of the modified system <= 1e-10.  Factors made by
  the size-specialised, tile and general kernels, uniform and ragged batches, box rows and dense
  rows, updates followed by downdates.
* without rows: a new right-hand side (q, r, f, x0) for the stored factors, which stay bit-identical.
* status: more nonzero rows than the kernel holds (info = LQ_INFO_UPDATE_RANK, instance untouched),
  an indefinite downdate (info = first failing stage + 1), refused plans and arguments.
* the full batch-4096 workload (N = 50, nx = 12, nu = 4) in the configuration the benchmark times,
  sampled instances against the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import kkt, update

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import update as U  # noqa: E402
from gpu_util import (forward_error, instance_solution, oracle_solution, stage_elems, unpack_factor_block,  # noqa: E402
                      workspace_views)


def _insts(b):
    return [b.instance(i) for i in range(b.batch)] if hasattr(b, "batched") and b.batched else list(b)


def _setup(insts, variant=None, packed=None):
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="f64")
    if variant:
        plan.set_variant(variant)
        assert plan.variant == variant
    data = L.pack(insts) if packed is None else L.pack(packed)
    if "S" not in data:
        data["S"] = torch.zeros(plan.totals["S"], dtype=torch.float64, device="cuda")
    ws = plan.workspace()
    info = torch.full((plan.batch,), 99, dtype=torch.int32, device="cuda")
    L.factor(plan, data, ws, info)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    return plan, data, ws, info


def _solve(plan, data, ws, info):
    x, u, lam = plan.empty_outputs()
    rel = torch.full((plan.batch,), -1.0, dtype=torch.float64, device="cuda")
    L.solve(plan, data, ws, x, u, lam, rel, None, info, tol=1e-10, max_it=0, check_res=True)
    torch.cuda.synchronize()
    return {"plan": plan, "ws": ws, "x": x, "u": u, "lam": lam, "rel": rel.cpu().numpy(),
            "info": info.cpu().numpy()}


def _block_err(blocks, ref, nx, nu, N):
    LQ, LR, LS = ref
    worst = 0.0
    for k in range(N + 1):
        Lr, dR, Ls, Lq, dQ = unpack_factor_block(blocks[k], nx, nu)
        pairs = []
        if k < N:
            pairs += [(Lr, LR[k]), (Ls, LS[k]), (dR, 1.0 / np.diag(LR[k]))]
        if k >= 1:
            pairs += [(Lq, LQ[k]), (dQ, 1.0 / np.diag(LQ[k]))]
        for a, b in pairs:
            worst = max(worst, np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    return worst


def _rows(insts, seed, m, density=0.5, box=True, sigma=(0.5, 2.0)):
    Cs, Ds, ss = [], [], []
    for i, p in enumerate(insts):
        C, D, s = synth.random_update_rows(seed * 1000 + i, 1, p.N, p.nx, p.nu, m, density=density, box=box,
                                           sigma=sigma)
        Cs.append(C[0]); Ds.append(D[0]); ss.append(s[0])
    return Cs, Ds, ss


def _check_update(plan, data, ws, info, insts, Cs, Ds, ss, label, sample=None):
    rows = U.pack_rows(Cs, Ds, ss)
    U.update_data(plan, rows, data)
    U.factor_update(plan, data, rows, ws, info, U.workspace(plan))
    res = _solve(plan, data, ws, info)
    assert np.all(res["info"] == 0), (label, res["info"])
    assert np.all(res["rel"] <= 1e-10), (label, res["rel"].max())
    mods = []
    idx = range(len(insts)) if sample is None else sample
    views = workspace_views(res)
    for i in idx:
        p = insts[i]
        mod = update.modified_problem(p, Cs[i], Ds[i], ss[i])
        mods.append(mod)
        for name in ("R", "S", "Q"):
            got = L.unpack(plan, name, data[name], i)
            want = getattr(mod, name)
            assert np.abs(got - want).max() <= 1e-14 * max(np.abs(want).max(), 1.0), (label, i, name)
        err = _block_err(views[i][0], update.updated_factors(p, Cs[i], Ds[i], ss[i]), p.nx, p.nu, p.N)
        assert err <= 1e-11, (label, i, err)
        fe = forward_error(instance_solution(res, i), oracle_solution(mod))
        assert fe <= 1e-9, (label, i, fe)
        _, rel_o = kkt.residual(mod, *instance_solution(res, i))
        assert rel_o <= 1e-10, (label, i, rel_o)
    return mods


CASES = [("small", 12, 4, 20, 2, True), ("small", 6, 2, 15, 3, False), ("tile", 12, 4, 17, 2, True),
         ("tile", 20, 5, 12, 1, False), ("tile", 60, 15, 6, 2, True), ("generic", 12, 4, 9, 2, True),
         ("generic", 33, 7, 8, 2, False)]


@pytest.mark.parametrize("variant,nx,nu,N,m,box", CASES)
def test_update_matches_refactorisation(variant, nx, nu, N, m, box):
    print(f"case: update {variant} nx={nx} nu={nu} N={N} m={m} box={box}", flush=True)
    b = synth.random_problem(900 + nx + N, N, nx, nu, batch=6)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, variant)
    cols = U.max_columns(plan)
    Cs, Ds, ss = _rows(insts, nx + N, m, density=min(0.5, 0.9 * cols / ((N + 1) * m)), box=box)
    assert max(int(np.count_nonzero(s)) for s in ss) <= cols
    _check_update(plan, data, ws, info, insts, Cs, Ds, ss, "update")


def test_update_then_downdate_and_new_rows():
    print("case: update then downdate (small kernel factors)", flush=True)
    b = synth.random_problem(77, 14, 12, 4, batch=5)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, "small")
    Cs, Ds, ss = _rows(insts, 3, 2, density=0.4)
    mods = _check_update(plan, data, ws, info, insts, Cs, Ds, ss, "first")
    # remove the first row of every stage again (a downdate) and add other rows
    C2, D2, s2 = _rows(insts, 4, 2, density=0.3)
    for i in range(len(insts)):
        C2[i][:, 0], D2[i][:, 0], s2[i][:, 0] = Cs[i][:, 0], Ds[i][:, 0], -ss[i][:, 0]
    _check_update(plan, data, ws, info, mods, C2, D2, s2, "second")


def test_ragged_batch_update():
    print("case: ragged batch update (general kernels)", flush=True)
    sizes = [(7, 5, 2), (12, 9, 3), (5, 12, 4), (9, 3, 1), (15, 16, 6)]
    insts = [synth.random_problem(40 + j, N, nx, nu) for j, (N, nx, nu) in enumerate(sizes)]
    plan, data, ws, info = _setup(insts)
    Cs, Ds, ss = _rows(insts, 8, 2, density=0.3, box=False, sigma=(0.1, 0.5))
    _check_update(plan, data, ws, info, insts, Cs, Ds, ss, "ragged")


def test_new_right_hand_side_for_stored_factors():
    print("case: new right-hand side without rows", flush=True)
    b = synth.random_problem(5, 11, 12, 4, batch=4)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, "small")
    before = ws.clone()
    b2 = synth.random_problem(6, 11, 12, 4, batch=4)
    for name in ("q", "r", "f", "x0"):
        data[name] = L.pack(b2)[name]
    U.factor_update(plan, data, None, ws, info)
    res = _solve(plan, data, ws, info)
    assert np.all(res["info"] == 0) and np.all(res["rel"] <= 1e-10)
    fb = int(np.sum((plan.N + 1) * np.array([stage_elems(x, u) for x, u in zip(plan.nx, plan.nu)]))) * 8
    assert torch.equal(before[:fb], ws[:fb])  # factors untouched
    for i, p in enumerate(insts):
        p2 = b2.instance(i)
        p2.A, p2.B, p2.Q, p2.R, p2.S = p.A, p.B, p.Q, p.R, p.S
        fe = forward_error(instance_solution(res, i), oracle_solution(p2))
        assert fe <= 1e-9, (i, fe)


def test_rank_limit_leaves_instance_untouched():
    print("case: rank limit", flush=True)
    b = synth.random_problem(8, 30, 12, 4, batch=3)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, "small")
    cols = U.max_columns(plan)
    assert cols >= 8
    Cs, Ds, ss = _rows(insts, 9, 4, density=0.0)
    ss[1][:] = 1.0                      # instance 1: 31 * 4 rows > cols
    ss[2][3, 0] = 1.0                   # instance 2: one row
    assert np.count_nonzero(ss[1]) > cols
    before = ws.clone()
    rows = U.pack_rows(Cs, Ds, ss)
    U.factor_update(plan, data, rows, ws, info, U.workspace(plan))
    got = info.cpu().numpy()
    assert got[0] == 0 and got[1] == U.LQ_INFO_UPDATE_RANK and got[2] == 0, got
    views_b = workspace_views({"plan": plan, "ws": before})
    views_a = workspace_views({"plan": plan, "ws": ws})
    # bytes, not values: parts no kernel writes (stage N's L^R block) hold whatever the workspace
    # held, NaN included, and must stay as they were
    assert views_a[1][0].tobytes() == views_b[1][0].tobytes()
    assert views_a[0][0].tobytes() == views_b[0][0].tobytes()   # no rows: factors kept


def test_indefinite_downdate_reports_stage():
    print("case: indefinite downdate", flush=True)
    N, nx, nu = 10, 6, 2
    b = synth.random_problem(12, N, nx, nu, batch=2)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, "small")
    Cs, Ds, ss = _rows(insts, 13, 1, density=0.0)
    j = 6
    for i in range(2):
        Ds[i][j, 0] = np.eye(nu)[0]
        Cs[i][j, 0] = 0.0
    ss[0][j, 0] = -1e6          # removes far more than the stage's input curvature
    ss[1][j, 0] = 0.25          # an ordinary update
    mod = update.modified_problem(insts[0], Cs[0], Ds[0], ss[0])
    assert np.linalg.eigvalsh(kkt.sym(mod.R[j]))[0] < 0
    rows = U.pack_rows(Cs, Ds, ss)
    U.update_data(plan, rows, data)
    U.factor_update(plan, data, rows, ws, info, U.workspace(plan))
    torch.cuda.synchronize()
    got = info.cpu().numpy()
    assert got[0] == j + 1 and got[1] == 0, got


def test_refusals():
    b = synth.random_problem(1, 5, 4, 2, batch=2)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts)
    Cs, Ds, ss = _rows(insts, 1, 1)
    rows = U.pack_rows(Cs, Ds, ss)
    bad = dict(rows, m=U.LQ_UPDATE_MAX_ROWS + 1)
    with pytest.raises(RuntimeError, match="outside"):
        U.factor_update(plan, data, bad, ws, info, U.workspace(plan))
    mixed = L.Plan(5, 4, 2, batch=2, mode="mixed_f32")
    with pytest.raises(RuntimeError, match="float64 plan"):
        U.factor_update(mixed, data, rows, mixed.workspace(), info, U.workspace(plan))
    ck = L.Plan(5, 4, 2, batch=2, mode="f64", ckpt_stride=2)
    with pytest.raises(RuntimeError, match="float64 plan"):
        U.factor_update(ck, data, rows, ck.workspace(), info, U.workspace(plan))
    with pytest.raises(RuntimeError, match="update workspace"):
        U.factor_update(plan, data, rows, ws, info, None)
    nos = {k: v for k, v in data.items() if k != "S"}
    with pytest.raises((RuntimeError, KeyError)):
        U.update_data(plan, rows, nos)


def test_batch4096_update_full_size_sampled():
    print("case: batch 4096 N=50 nx=12 nu=4 update, sampled", flush=True)
    batch, N, nx, nu, m = 4096, 50, 12, 4, 2
    b = synth.make_batch(2, batch)
    insts = _insts(b)
    plan, data, ws, info = _setup(insts, packed=b)
    C, D, s = synth.random_update_rows(21, batch, N, nx, nu, m, density=0.1)
    Cs, Ds, ss = list(C), list(D), list(s)
    assert max(int(np.count_nonzero(x)) for x in ss) <= U.max_columns(plan)
    sample = [0, 1, 777, 2048, 4095]
    _check_update(plan, data, ws, info, insts, Cs, Ds, ss, "batch4096", sample=sample)
