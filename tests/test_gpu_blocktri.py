"""Batched block-tridiagonal solvers (CR, PCR, PCG) on the GPU against the pinned CPU oracle.

Bar: the CR factor blocks L_k, U_k, Y_k against the oracle's Cholesky factor of the
valuation-ordered matrix, entry-wise within 1e-12 of the block's largest entry; CR and PCR
solutions against the dense LAPACK solve within 1e-12 (relative, inf-norm; these systems have
condition numbers below 10); PCG: the library's relative residual <= tol and the solution within
10 tol of the dense one.  Sizes include Nb not a power of two, Nb = 1 and 2, and blocks wider than
one 64-column panel."""
import numpy as np
import pytest

import synth
from oracle import blocktri as obt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2512_09058_amd import blocktri as bt  # noqa: E402

SIZES = [(1, 3), (2, 4), (3, 1), (5, 3), (8, 8), (13, 5), (16, 16), (7, 70), (33, 2), (4, 130)]


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrs]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("Nb,n", SIZES)
def test_cr_factor_blocks_and_solution(Nb, n):
    print(f"case: cr Nb={Nb} n={n}", flush=True)
    M, K, b = synth.random_blocktri(10 + Nb + n, 3, Nb, n)
    Md, Kd, bd = _dev(M, K, b)
    ws, info = bt.cr_factor(Md, Kd)
    x = bt.cr_solve(3, Nb, n, ws, bd)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    L, U, Y = (t.cpu().numpy() for t in bt.cr_views(ws, 3, Nb, n))
    xh = x.cpu().numpy()
    for s in range(3):
        Lo, Uo, Yo, _ = obt.cr_factors(M[s], K[s])
        for k in range(Nb):
            assert np.abs(np.tril(L[s, k]) - Lo[k]).max() <= 1e-12 * np.abs(Lo[k]).max(), (s, k, "L")
            if Uo[k] is not None:
                assert np.abs(U[s, k] - Uo[k]).max() <= 1e-12 * max(np.abs(Uo[k]).max(), 1e-300), (s, k, "U")
            if Yo[k] is not None:
                assert np.abs(Y[s, k] - Yo[k]).max() <= 1e-12 * max(np.abs(Yo[k]).max(), 1e-300), (s, k, "Y")
        assert _rel(xh[s], obt.solve(M[s], K[s], b[s])) <= 1e-12, s


@pytest.mark.parametrize("Nb,n", SIZES)
def test_pcr_solution(Nb, n):
    print(f"case: pcr Nb={Nb} n={n}", flush=True)
    M, K, b = synth.random_blocktri(40 + Nb + n, 3, Nb, n)
    Md, Kd, bd = _dev(M, K, b)
    x, info = bt.pcr_solve(Md, Kd, bd)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    xh = x.cpu().numpy()
    for s in range(3):
        ref = obt.solve(M[s], K[s], b[s])
        assert _rel(xh[s], ref) <= 1e-12, s
        assert _rel(xh[s], obt.pcr(M[s], K[s], b[s])) <= 1e-12, s


@pytest.mark.parametrize("precond", ["jacobi", "stair"])
@pytest.mark.parametrize("Nb,n", [(1, 3), (6, 4), (13, 5), (64, 8), (9, 70)])
def test_pcg(precond, Nb, n):
    print(f"case: pcg {precond} Nb={Nb} n={n}", flush=True)
    M, K, b = synth.random_blocktri(80 + Nb + n, 3, Nb, n, dominance=1.0)
    Md, Kd, bd = _dev(M, K, b)
    tol = 1e-11
    x, iters, rel, info = bt.pcg(Md, Kd, bd, precond=precond, tol=tol, max_it=500)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert np.all(rel.cpu().numpy() <= tol)
    xh = x.cpu().numpy()
    its = iters.cpu().numpy()
    for s in range(3):
        ref = obt.solve(M[s], K[s], b[s])
        assert _rel(xh[s], ref) <= 10 * tol, s
        _, it_o, _ = obt.pcg(M[s], K[s], b[s], precond=precond, tol=tol)
        assert abs(int(its[s]) - it_o) <= 2, (s, its[s], it_o)


def test_stair_takes_fewer_iterations_than_jacobi():
    M, K, b = synth.random_blocktri(5, 4, 64, 8, dominance=0.5)
    Md, Kd, bd = _dev(M, K, b)
    _, it_j, _, _ = bt.pcg(Md, Kd, bd, precond="jacobi", tol=1e-12)
    _, it_s, _, _ = bt.pcg(Md, Kd, bd, precond="stair", tol=1e-12)
    torch.cuda.synchronize()
    assert np.all(it_s.cpu().numpy() <= it_j.cpu().numpy())


def test_nonpositive_block_reports_info():
    M, K, b = synth.random_blocktri(3, 3, 8, 4)
    M[1, 3] = -np.eye(4)  # block row 3 is eliminated first (level 0): info = 4
    Md, Kd, bd = _dev(M, K, b)
    _, info = bt.cr_factor(Md, Kd)
    _, info2 = bt.pcr_solve(Md, Kd, bd)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 4, 0]
    assert info2.cpu().tolist()[0] == 0 and info2.cpu().tolist()[1] != 0 and info2.cpu().tolist()[2] == 0


def test_schur_shaped_batch_sampled():
    """The Schur complement shapes of the parallel-in-time solve: 64 systems of 16 blocks of 128;
    CR and PCR on every system, the oracle's written-out CR recursion on a sample."""
    M, K, b = synth.random_blocktri(99, 64, 16, 128)
    Md, Kd, bd = _dev(M, K, b)
    ws, info = bt.cr_factor(Md, Kd)
    x = bt.cr_solve(64, 16, 128, ws, bd)
    xp, info2 = bt.pcr_solve(Md, Kd, bd)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and np.all(info2.cpu().numpy() == 0)
    xh, xph = x.cpu().numpy(), xp.cpu().numpy()
    for s in (0, 31, 63):
        ref = obt.cr_recursive(M[s], K[s], b[s])
        assert _rel(xh[s], ref) <= 1e-12 and _rel(xph[s], ref) <= 1e-12, s
