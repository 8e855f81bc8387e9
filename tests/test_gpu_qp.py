"""Box-constrained QPs on the GPU (include/lqqp.h) against the QP oracle (oracle/qp.py).

The QP's solution (x, u) and its multipliers (y of the bounds, lam of the dynamics) are unique for
these problems (strictly convex cost, linearly independent active rows), so the GPU result is
compared with the oracle's solve on every instance: primal entries within 1e-7 of the largest,
multipliers within 1e-6 (the outer loop stops at violations of 1e-9), and the QP's optimality
certificate evaluated by the oracle on the GPU's result: stationarity <= 1e-8, dynamics <= 1e-11,
complementarity <= 1e-8.  Workloads: the mass-spring benchmark (box rows on positions and inputs,
many active), random QPs with dense rows, S and f and one-sided bounds, a warm start from the
solution, and argument refusals.
"""
import numpy as np
import pytest

import synth
from oracle import qp as oqp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import qp as Q  # noqa: E402


def _run(insts, Cs, Ds, bls, bus, opts=None, warm=None):
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="f64")
    data = L.pack(insts)
    for k in ("S", "f"):
        if k not in data:
            data[k] = torch.zeros(plan.totals[k], dtype=torch.float64, device="cuda")
    cons = Q.pack_constraints(Cs, Ds, bls, bus)
    ws = plan.workspace()
    qws = Q.workspace(plan, cons["m"], (opts or {}).get("intervals", 0))
    x, u, lam = plan.empty_outputs()
    m = cons["m"]
    y = torch.zeros(sum((p.N + 1) * m for p in insts), dtype=torch.float64, device="cuda")
    status = torch.full((plan.batch,), 9, dtype=torch.int32, device="cuda")
    iters = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    if warm is not None:
        u.copy_(warm[0])
        y.copy_(warm[1])
    Q.solve(plan, data, cons, ws, qws, x, u, lam, y, status, iters, opts=opts)
    torch.cuda.synchronize()
    return plan, x, u, lam, y, status.cpu().numpy(), iters.cpu().numpy()


def _inst_y(y, insts, m, i):
    o = sum((p.N + 1) * m for p in insts[:i])
    return y[o:o + (insts[i].N + 1) * m].cpu().numpy().reshape(insts[i].N + 1, m)


def _check(insts, Cs, Ds, bls, bus, res, label):
    plan, x, u, lam, y, status, iters = res
    assert np.all(status == 0), (label, status)
    m = Cs[0].shape[1]
    for i, p in enumerate(insts):
        xs, us, ls = (L.unpack(plan, n, t, i) for n, t in (("x", x), ("u", u), ("lam", lam)))
        ys = _inst_y(y, insts, m, i)
        st, dy, co = oqp.certificate(p, Cs[i], Ds[i], bls[i], bus[i], xs, us, ls, ys)
        assert st <= 1e-8 and dy <= 1e-11 and co <= 1e-8, (label, i, st, dy, co)
        xr, ur, lr, yr, _ = oqp.solve(p, Cs[i], Ds[i], bls[i], bus[i])
        zs = max(np.abs(xr).max(), np.abs(ur).max(), 1.0)
        assert max(np.abs(xs - xr).max(), np.abs(us - ur).max()) <= 1e-7 * zs, (label, i)
        ms = max(np.abs(yr).max(), np.abs(lr).max(), 1.0)
        assert max(np.abs(ys - yr).max(), np.abs(ls - lr).max()) <= 1e-6 * ms, (label, i)
    return iters


@pytest.mark.parametrize("M,N,P", [(6, 8, 0), (6, 16, 0), (12, 8, 0), (6, 16, 4), (12, 12, 3)])
def test_mass_spring_matches_oracle(M, N, P):
    print(f"case: mass-spring M={M} N={N} intervals={P}", flush=True)
    prob, C, D, bl, bu = synth.mass_spring(M, N, 3, seed=5)
    insts = [prob.instance(i) for i in range(3)]
    res = _run(insts, [C] * 3, [D] * 3, [bl] * 3, [bu] * 3, opts={"intervals": P})
    iters = _check(insts, [C] * 3, [D] * 3, [bl] * 3, [bu] * 3, res, "mass-spring")
    print(f"  inner steps {iters.tolist()}", flush=True)


def test_random_qps_with_S_f_and_one_sided_rows():
    print("case: random QPs", flush=True)
    insts, Cs, Ds, bls, bus = [], [], [], [], []
    for s in range(4):
        p = synth.random_problem(300 + s, 6, 3, 2)
        rng = np.random.default_rng(300 + s)
        C = rng.standard_normal((7, 2, 3))
        D = rng.standard_normal((6, 2, 2))
        uf = rng.standard_normal((6, 2))
        wf = oqp.constraint_values(p, C, D, oqp.rollout(p, uf), uf)
        bl = wf - rng.uniform(0.05, 0.5, wf.shape)
        bu = wf + rng.uniform(0.05, 0.5, wf.shape)
        bl[rng.uniform(size=bl.shape) < 0.3] = -np.inf
        insts.append(p); Cs.append(C); Ds.append(D); bls.append(bl); bus.append(bu)
    _check(insts, Cs, Ds, bls, bus, _run(insts, Cs, Ds, bls, bus), "random")


def test_wide_qps_with_stage_matrices_read_from_global_memory():
    """nx = 60, nu = 10: a stage's matrices would take the stage-parallel kernels' workgroup past
    64 KiB of LDS, so the Newton-system and direction kernels read them from global memory (the
    other cases here run the instances that stage them in LDS)."""
    print("case: wide QPs", flush=True)
    insts, Cs, Ds, bls, bus = [], [], [], [], []
    for s in range(2):
        p = synth.random_problem(700 + s, 5, 60, 10)
        rng = np.random.default_rng(700 + s)
        p.A = 0.9 * np.linalg.qr(rng.standard_normal((5, 60, 60)))[0]
        p.B = p.B / np.sqrt(60)
        C = rng.standard_normal((6, 4, 60)) / np.sqrt(60)
        D = rng.standard_normal((5, 4, 10)) / np.sqrt(10)
        uf = rng.standard_normal((5, 10))
        wf = oqp.constraint_values(p, C, D, oqp.rollout(p, uf), uf)
        bl = wf - rng.uniform(0.05, 0.5, wf.shape)
        bu = wf + rng.uniform(0.05, 0.5, wf.shape)
        insts.append(p); Cs.append(C); Ds.append(D); bls.append(bl); bus.append(bu)
    _check(insts, Cs, Ds, bls, bus, _run(insts, Cs, Ds, bls, bus), "wide")


def test_warm_start_from_the_solution():
    print("case: warm start", flush=True)
    prob, C, D, bl, bu = synth.mass_spring(6, 12, 2, seed=9)
    insts = [prob.instance(i) for i in range(2)]
    r1 = _run(insts, [C] * 2, [D] * 2, [bl] * 2, [bu] * 2)
    r2 = _run(insts, [C] * 2, [D] * 2, [bl] * 2, [bu] * 2, warm=(r1[2], r1[4]))
    _check(insts, [C] * 2, [D] * 2, [bl] * 2, [bu] * 2, r2, "warm")
    assert np.all(r2[6] <= r1[6]), (r1[6], r2[6])


def test_refusals():
    prob, C, D, bl, bu = synth.mass_spring(6, 4, 1, seed=1)
    insts = [prob.instance(0)]
    mixed = L.Plan(4, 12, 3, batch=1, mode="mixed_f32")
    data = L.pack(insts)
    cons = Q.pack_constraints([C], [D], [bl], [bu])
    x, u, lam = mixed.empty_outputs()
    y = torch.zeros(5 * cons["m"], dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    it = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="float64"):
        Q.solve(mixed, data, cons, mixed.workspace(), Q.workspace(mixed, cons["m"]), x, u, lam, y, st, it)
    plan = L.Plan(4, 12, 3, batch=1, mode="f64")
    with pytest.raises(RuntimeError, match="positive"):
        Q.solve(plan, data, cons, plan.workspace(), Q.workspace(plan, cons["m"]), x, u, lam, y, st, it,
                opts={"max_outer": 0})
    with pytest.raises(RuntimeError, match="intervals"):
        Q.solve(plan, data, cons, plan.workspace(), Q.workspace(plan, cons["m"], 4), x, u, lam, y, st, it,
                opts={"intervals": 5})
