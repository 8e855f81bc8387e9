"""Float64 fallback of the mixed path: an instance whose stage matrix is positive definite but so
ill-conditioned that float32 stage products lose that (info = k + 1 from the mixed factor) is
factored and solved again in float64 through a subset plan, in place in the batch's arrays.

The crafted instance (N = 3, nx = 2, nu = 1, entries of order one): at the last stage Q_N = I,
B = [b, 0]^T with b = sqrt(2 + 1e-8), R = -2 and S = -B^T Q_N A, so that Rhat = R + B^T P_N B = 1e-8
and Shat = 0: the stage matrix diag(1e-8, Q + A^T A) is positive definite.  In float32, b rounds
down to 1.41421353 and b^2 to 1.99999988, so Rhat = -1.2e-7 and the mixed factor reports info = 3
(stage 2).  r at that stage cancels the right-hand side along the weak direction up to 1e-8, so the
solution is of order one.  The float64 solution is checked against the oracle's dense solve within
what the conditioning allows (forward error <= 10 eps cond(K); cond(K) ~ 2e9, the oracle's own two
routes agree to 1.2e-8) and its KKT residual (library and oracle) <= 1e-10.  The other instances
keep their mixed-precision solution (not re-solved) at <= 1e-10 relative residual.
"""
import numpy as np
import pytest

import synth
from oracle import kkt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import api  # noqa: E402
from gpu_util import instance_solution  # noqa: E402

EPS = np.finfo(np.float64).eps


def _crafted(seed):
    p = synth.random_problem(seed, 3, 2, 1, with_S=True)
    b = np.sqrt(2.0 + 1e-8)
    k = 2
    p.B = p.B.copy(); p.R = p.R.copy(); p.S = p.S.copy(); p.Q = p.Q.copy(); p.r = p.r.copy()
    p.Q[3] = np.eye(2)
    p.B[k] = np.array([[b], [0.0]])
    p.R[k] = np.array([[-2.0]])
    p.S[k] = -(p.B[k].T @ p.Q[3] @ p.A[k])
    p.r[k] = -(p.B[k].T @ (p.q[3] + p.f[k])) + 1e-8
    return p


def _batch():
    insts = [synth.random_problem(60 + i, 3, 2, 1) for i in range(6)]
    insts[2] = _crafted(7)
    return insts


def _run(insts, fallback):
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="mixed_f32")
    data = L.pack(insts)
    ws = plan.workspace()
    x, u, lam = plan.empty_outputs()
    rel = torch.full((plan.batch,), -1.0, dtype=torch.float64, device="cuda")
    its = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    if fallback:
        redone = api.solve_with_fallback(plan, data, ws, x, u, lam, rel, its, info, tol=1e-10, max_it=10)
    else:
        L.factor(plan, data, ws, info)
        L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=1e-10, max_it=10, check_res=True)
        redone = None
    torch.cuda.synchronize()
    return {"plan": plan, "x": x, "u": u, "lam": lam, "rel": rel.cpu().numpy(), "info": info.cpu().numpy(),
            "redone": redone}


def test_crafted_instance_fails_in_mixed_precision():
    print("case: mixed solve of the crafted batch, no fallback", flush=True)
    insts = _batch()
    # the stage matrix is positive definite in exact arithmetic (and in the oracle)
    r = _run(insts, fallback=False)
    assert r["plan"].variant == "small_padded"
    assert r["info"][2] == 3, r["info"]
    assert all(r["info"][i] == 0 for i in range(6) if i != 2), r["info"]


def test_fallback_recovers_the_instance():
    print("case: mixed solve with float64 fallback", flush=True)
    insts = _batch()
    r = _run(insts, fallback=True)
    # (2, 1) has no size-specialised kernel of its own: the mixed plan runs padded to (4, 2), and the
    # float64 subset plan addresses the parent's unpadded arrays
    assert r["plan"].variant == "small_padded"
    assert list(r["redone"]) == [2]
    assert np.all(r["info"] == 0), r["info"]
    for i, p in enumerate(insts):
        K, bvec, lay = kkt.assemble(p)
        Kd = K.toarray()
        ref = kkt.solve_dense(p)
        sol = instance_solution(r, i)
        z = kkt.join(*sol, lay)
        zr = kkt.join(*ref, lay)
        _, rel_o = kkt.residual(p, *sol)
        if i == 2:
            cond = np.linalg.cond(Kd)
            fe = np.abs(z - zr).max() / np.abs(zr).max()
            print(f"  recovered instance: forward error {fe:.2e}, cond {cond:.2e}, residual {rel_o:.2e}", flush=True)
            assert fe <= 10 * EPS * cond, (fe, cond)
        assert rel_o <= 1e-10 and r["rel"][i] <= 1e-10, (i, rel_o, r["rel"][i])


def test_subset_plan_refuses_bad_indices():
    insts = _batch()
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="mixed_f32")
    with pytest.raises(RuntimeError, match="twice"):
        plan.subset([1, 1])
    with pytest.raises(RuntimeError, match="outside"):
        plan.subset([7])
    sub = plan.subset([4, 0])
    assert sub.batch == 2 and sub.variant in ("tile", "generic")
    assert np.array_equal(sub.offsets["x"], plan.offsets["x"][[4, 0]])
