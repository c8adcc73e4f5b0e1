"""Solve and grid solution in one call (ibdl_solve_grid / ibdl_batch_solve_grid).

For MIXED plans the grid solution comes out of the FP64 residual pass of the
final iterate: u = L^-1 (g~ - S~ x [- S V_b]) on the grid and the residual from
the same spectrum at the points.  Bars: u is bit-identical to ibdl_eval_grid of
the returned solution (the same FP64 spread, transforms and grid store); the
solution and u are within 1e-6 of the oracle; the solution agrees with
ibdl_solve's to 1e-7 (its first FP32 solve starts from an FP32 right-hand side
and its FP64 residuals are formed from the boundary data instead of the stored
right-hand side; both meet the FP64 residual tolerance); FP64 plans are
unchanged (bit-identical to ibdl_solve + ibdl_eval_grid); a batch equals its
instances solved alone.
"""
import ctypes

import numpy as np
import pytest

from oracle import ibdl_oracle as O
from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402

SOLVE_MIXED_TOL = 1e-6


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def relerr(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("bc,alpha", [(W.DIRICHLET, 1.0), (W.NEUMANN, 1.0), (W.NEUMANN, 100.0)])
def test_star1024_solve_grid_mixed(bc, alpha):
    p = W.config_star1024(m=4096, alpha=alpha, bc=bc)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, bc=bc, tol=1e-13)
    uref = O.eval_grid(st, tight.x, vb=p.data if bc == W.NEUMANN else None, g_tilde=p.g_tilde, bc=bc)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    data = T(np.stack([p.data, p.data]))
    g = T(np.stack([p.g_tilde, p.g_tilde]))
    sol, u, info = pl.solve_grid(data, g, tol=1e-8)
    assert all(i["rel_resid_true"] <= 1e-8 for i in info)
    ue = pl.eval_grid(sol, vb=data if bc == W.NEUMANN else None, g=g)
    assert torch.equal(u, ue)
    for r in range(2):
        assert relerr(sol[r].cpu().numpy(), tight.x) < SOLVE_MIXED_TOL
        assert relerr(u[r].cpu().numpy(), uref) < SOLVE_MIXED_TOL
    # the reported residual is the system's FP64 residual: b - A x with an FP64 plan
    p64 = ibdl.Plan.from_problem(p, prec=ibdl.FP64)
    b64 = p64.rhs(data, g)
    res = (b64 - p64.apply(sol)).norm(dim=1) / b64.norm(dim=1)
    for r in range(2):
        assert abs(float(res[r]) - info[r]["rel_resid_true"]) <= 1e-10
    p64.close()
    # ibdl_solve forms b in FP64 and its residuals from b: a different rounding
    # path to the same system, both meeting tol = 1e-8 in the FP64 residual
    s1, i1 = pl.solve(data, g, tol=1e-8)
    assert all(i["rel_resid_true"] <= 1e-8 for i in i1)
    assert relerr(sol.cpu().numpy(), s1.cpu().numpy()) < 1e-7
    pl.close()


def test_solve_grid_3d_mixed():
    p = W.table2_problem(32, 2000)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, bc=p.bc, tol=1e-13)
    uref = O.eval_grid(st, tight.x, g_tilde=p.g_tilde, bc=p.bc)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    data, g = T(p.data[None]), T(p.g_tilde[None])
    sol, u, info = pl.solve_grid(data, g, tol=1e-9)
    assert torch.equal(u, pl.eval_grid(sol, g=g))
    assert relerr(sol[0].cpu().numpy(), tight.x) < SOLVE_MIXED_TOL
    assert relerr(u[0].cpu().numpy(), uref) < SOLVE_MIXED_TOL
    pl.close()


@pytest.mark.parametrize("bc", [W.DIRICHLET, W.NEUMANN])
def test_solve_grid_fp64_unchanged(bc):
    p = W.config_star1024(m=1200, n=192, alpha=2.0, bc=bc, seed=8)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.FP64)
    data, g = T(p.data[None]), T(p.g_tilde[None])
    sol, u, info = pl.solve_grid(data, g, tol=1e-10)
    s1, i1 = pl.solve(data, g, tol=1e-10)
    assert torch.equal(sol, s1)
    assert torch.equal(u, pl.eval_grid(s1, vb=data if bc == W.NEUMANN else None, g=g))
    pl.close()


def test_batch_solve_grid_equals_alone():
    items = []
    for sp in W.config_batch(count=5, seed=41, sizes=(64, 96, 128)):
        sp["nrhs"] = 1 + sp["nrhs"] % 3
        _, _, probs = W.batch_instance(sp)
        items.append(probs)
    batch = ibdl.Batch.from_problems([(probs[0], len(probs)) for probs in items], prec=ibdl.MIXED)
    data = [T(np.stack([q.data for q in probs])) for probs in items]
    g = [T(np.stack([q.g_tilde for q in probs])) for probs in items]
    sol, u, info = batch.solve_grid(data, g, tol=1e-9)
    for i, probs in enumerate(items):
        pl = ibdl.Plan.from_problem(probs[0], prec=ibdl.MIXED)
        s1, u1, _ = pl.solve_grid(data[i], g[i], tol=1e-9)
        assert torch.equal(sol[i], s1), f"instance {i}"
        assert torch.equal(u[i], u1), f"instance {i}"
        pl.close()
    batch.close()


def test_solve_grid_argument_errors():
    p = W.config_star1024(m=1200, n=128, seed=3)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    data, g = T(p.data[None]), T(p.g_tilde[None])
    sol = torch.empty_like(data)
    info = (ibdl.SolveInfo * 1)()
    st = ibdl.lib().ibdl_solve_grid(pl._h, 1, data.data_ptr(), g.data_ptr(), None, sol.data_ptr(), None,
                                    info, None)
    assert st == ibdl.ERR_ARG and "u" in ibdl.last_error()
    pl.close()


@pytest.mark.parametrize("bc", [W.DIRICHLET, W.NEUMANN])
def test_solve_grid_mixed_tol_near_first_stage(bc):
    """With tol just below where the first FP32-operator solve stops, the FP64
    residual after it writes no grid solution; whether that residual turns out
    final (the grid solution then comes from a pass of its own) or refinement
    goes on, u equals ibdl_eval_grid of the returned solution."""
    p = W.config_star1024(m=1500, n=256, alpha=1.0, bc=bc, seed=21)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    data = T(np.stack([p.data] * 3))
    g = T(np.stack([p.g_tilde] * 3))
    rounds = set()
    for tol in (9.9e-7, 5e-7, 2e-7, 1e-9):
        sol, u, info = pl.solve_grid(data, g, tol=tol)
        assert all(i["status"] == ibdl.OK and i["rel_resid_true"] <= tol for i in info), (tol, list(info))
        ue = pl.eval_grid(sol, vb=data if bc == W.NEUMANN else None, g=g)
        assert torch.equal(u, ue), tol
        rounds |= {i["fp64_applies"] for i in info}
    print("FP64 residual passes seen:", sorted(rounds))
    pl.close()


@pytest.mark.parametrize("prec", [ibdl.MIXED, ibdl.FP64])
def test_packed_strengths_change_nothing(prec):
    """A mixed solve of 16 right-hand sides on the star 1024^2 plan takes the
    Arnoldi step's spread through strengths packed as FP32 in groups of four; the
    same right-hand sides solved two at a time read them directly (FP64 solves of
    this size read them directly either way: the FP64 threshold is 2^24 entries x
    right-hand sides).  Solutions, grid solutions and iteration counts are
    bit-identical."""
    p = W.config_star1024(m=4096, alpha=1.0, seed=31)
    rng = np.random.default_rng(5)
    R = 16
    data = np.stack([p.data * (1.0 + 0.1 * r) + 0.01 * rng.standard_normal(p.geom.m) for r in range(R)])
    g = np.stack([p.g_tilde * (1.0 - 0.05 * r) for r in range(R)])
    pl = ibdl.Plan.from_problem(p, prec=prec)
    sol, u, info = pl.solve_grid(T(data), T(g), tol=1e-8)
    for r0 in range(0, R, 2):
        s2, u2, i2 = pl.solve_grid(T(data[r0:r0 + 2]), T(g[r0:r0 + 2]), tol=1e-8)
        assert torch.equal(s2, sol[r0:r0 + 2]), r0
        assert torch.equal(u2, u[r0:r0 + 2]), r0
        assert [x["iters"] for x in i2] == [x["iters"] for x in info[r0:r0 + 2]], r0
    pl.close()


def test_packed_fp64_solves_change_nothing():
    """FP64 solves past the FP64 pack threshold (a 64^3 sphere with 20000 points,
    eight right-hand sides: 2.6e7 entries x right-hand sides >= 2^24) read the
    Arnoldi step's strengths packed as FP64 four to a segment; solved two at a time
    they read them directly.  Solutions, grid solutions and iteration counts are
    bit-identical."""
    p = W.table2_problem(64, 20000)
    rng = np.random.default_rng(9)
    R = 8
    data = np.stack([p.data * (1.0 + 0.1 * r) + 0.01 * rng.standard_normal(p.geom.m) for r in range(R)])
    g = np.stack([p.g_tilde * (1.0 - 0.05 * r) for r in range(R)])
    pl = ibdl.Plan.from_problem(p, prec=ibdl.FP64)
    sol, u, info = pl.solve_grid(T(data), T(g), tol=1e-8)
    for r0 in range(0, R, 2):
        s2, u2, i2 = pl.solve_grid(T(data[r0:r0 + 2]), T(g[r0:r0 + 2]), tol=1e-8)
        assert torch.equal(s2, sol[r0:r0 + 2]), r0
        assert torch.equal(u2, u[r0:r0 + 2]), r0
        assert [x["iters"] for x in i2] == [x["iters"] for x in info[r0:r0 + 2]], r0
    pl.close()
