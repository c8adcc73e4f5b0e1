"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: binning keys and order bit-exact; FP64 operator/rhs/grid within 1e-12
relative; mixed (FP32 grid pipeline, FP64 Krylov) operator within the
rounding-error model of error_model.py; solves against the oracle's solution of
the same system (mixed solves to 1e-6).
"""
import math

import numpy as np
import pytest

from error_model import MODEL_FACTOR, mixed_model
from oracle import ibdl_oracle as O
from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402

DEV = "cuda"
FP64_TOL = 1e-12
# Mixed solves refine with the FP64 operator until its residual meets tol, so
# they must match the oracle's solution within 1e-6 relative.
SOLVE_MIXED_TOL = 1e-6


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def plan_for(prob, delta=O.PESKIN4, prec=ibdl.FP64):
    d = ibdl.PESKIN4 if delta == O.PESKIN4 else ibdl.COSINE4
    return ibdl.Plan.from_problem(prob, delta=d, prec=prec)


def random_problem(dim, n, m, seed, bc=W.DIRICHLET, alpha=1.0, lo=None, length=1.0, spread=(-0.2, 1.2)):
    rng = np.random.default_rng(seed)
    X = rng.uniform(spread[0], spread[1], size=(m, dim)) * length
    nr = rng.standard_normal((m, dim))
    nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, size=m) / m
    lo = tuple([0.0] * dim) if lo is None else lo
    grid = W.Grid(dim, n, lo, length)
    geom = W.Geometry(dim, X, nr, w, lambda p: np.zeros(p.shape[0], bool), 1.0)
    sol = W.sol_random_fourier(dim, seed, kmax=2, length=length)
    return W.make_problem(grid, geom, alpha, bc, sol, forcing=False)


# ------------------------------------------------------------------ binning
# the last three sit at and above the point count where ranking gives way to the bitonic sort
@pytest.mark.parametrize("dim,n,m,seed", [(2, 64, 1000, 1), (2, 12, 333, 2), (3, 16, 2000, 3), (2, 1024, 4096, 4),
                                          (2, 256, 16384, 5), (2, 256, 16385, 6), (3, 32, 30000, 7)])
def test_binning_bit_exact(dim, n, m, seed):
    p = random_problem(dim, n, m, seed)
    # force ties and points on cell faces
    p.geom.X[::5] = p.geom.X[0]
    p.geom.X[1::7, 0] = (np.arange(p.geom.X[1::7].shape[0]) % n) / n
    pl = plan_for(p)
    key, perm = pl.binning()
    st = O.setup_from_problem(p)
    okey, operm = O.binning(st)
    assert np.array_equal(key, okey)
    assert np.array_equal(perm, operm)


# ------------------------------------------------------------------ operator
CASES = [
    # dim, n, m, bc, alpha, delta
    (2, 64, 128, W.DIRICHLET, 1.0, O.COSINE4),
    (2, 64, 300, W.NEUMANN, 1.0, O.PESKIN4),
    (2, 12, 17, W.DIRICHLET, 3.0, O.PESKIN4),
    (2, 8, 1, W.DIRICHLET, 1.0, O.PESKIN4),
    (2, 96, 500, W.NEUMANN, 100.0, O.PESKIN4),
    (2, 192, 700, W.DIRICHLET, 0.0, O.PESKIN4),
    (2, 384, 2000, W.DIRICHLET, 10.0, O.PESKIN4),
    (3, 16, 200, W.DIRICHLET, 1.0, O.PESKIN4),
    (3, 24, 500, W.NEUMANN, 5.0, O.COSINE4),
    (3, 32, 900, W.DIRICHLET, 0.0, O.PESKIN4),
]


@pytest.mark.parametrize("dim,n,m,bc,alpha,delta", CASES)
def test_apply_fp64_matches_oracle(dim, n, m, bc, alpha, delta):
    p = random_problem(dim, n, m, seed=n + m, bc=bc, alpha=alpha)
    st = O.setup_from_problem(p, delta=delta)
    pl = plan_for(p, delta=delta)
    q = W.random_density(m, seed=7, nrhs=3)
    out = N(pl.apply(T(q)))
    for r in range(3):
        ref = O.apply_A(st, q[r], bc)
        assert relerr(out[r], ref) < FP64_TOL, (r, relerr(out[r], ref))
        assert maxrel(out[r], ref) < 10 * FP64_TOL


@pytest.mark.parametrize("dim,n,m,bc,alpha,delta", CASES)
def test_apply_mixed_matches_oracle(dim, n, m, bc, alpha, delta):
    p = random_problem(dim, n, m, seed=n + m, bc=bc, alpha=alpha)
    st = O.setup_from_problem(p, delta=delta)
    pl = plan_for(p, delta=delta, prec=ibdl.MIXED)
    q = W.random_density(m, seed=8, nrhs=2)
    out = N(pl.apply(T(q)))
    for r in range(2):
        ref = O.apply_A(st, q[r], bc)
        e, model = relerr(out[r], ref), mixed_model(st, q[r], ref)
        print(f"  mixed apply {dim}-D n={n}: rel err {e:.3e} model {model:.3e}", flush=True)
        assert e < MODEL_FACTOR * model, (e, model)


@pytest.mark.parametrize("dim,n,m,bc,alpha", [(2, 64, 200, W.DIRICHLET, 1.0), (2, 96, 300, W.NEUMANN, 2.0),
                                              (3, 16, 300, W.NEUMANN, 1.0), (3, 24, 400, W.DIRICHLET, 0.0)])
def test_rhs_and_eval_grid_fp64(dim, n, m, bc, alpha):
    p = random_problem(dim, n, m, seed=3 * n + m, bc=bc, alpha=alpha)
    st = O.setup_from_problem(p)
    pl = plan_for(p)
    rng = np.random.default_rng(11)
    data = rng.standard_normal((2, m))
    g = rng.standard_normal((2,) + (n,) * dim)
    if alpha == 0.0:
        g -= g.reshape(2, -1).mean(1).reshape((2,) + (1,) * dim)
    b = N(pl.rhs(T(data), T(g)))
    for r in range(2):
        ref = O.rhs(st, data[r], g[r], bc)
        assert relerr(b[r], ref) < FP64_TOL
    b0 = N(pl.rhs(T(data)))
    for r in range(2):
        assert relerr(b0[r], O.rhs(st, data[r], None, bc)) < FP64_TOL
    sol = rng.standard_normal((2, m))
    vb = rng.standard_normal((2, m)) if bc == W.NEUMANN else None
    u = N(pl.eval_grid(T(sol), T(vb) if vb is not None else None, T(g)))
    u0 = N(pl.eval_grid(T(sol), T(vb) if vb is not None else None))
    for r in range(2):
        ref = O.eval_grid(st, sol[r], None if vb is None else vb[r], g[r], bc)
        assert relerr(u[r], ref) < FP64_TOL
        ref0 = O.eval_grid(st, sol[r], None if vb is None else vb[r], None, bc)
        assert relerr(u0[r], ref0) < FP64_TOL


def test_apply_is_deterministic():
    p = random_problem(2, 256, 3000, seed=5)
    for prec in (ibdl.FP64, ibdl.MIXED):
        pl = plan_for(p, prec=prec)
        q = T(W.random_density(3000, seed=1, nrhs=2))
        a = pl.apply(q).clone()
        for _ in range(5):
            assert torch.equal(pl.apply(q), a)


def test_multi_rhs_equals_single_rhs():
    p = random_problem(2, 128, 700, seed=6, bc=W.NEUMANN)
    pl = plan_for(p, prec=ibdl.MIXED)
    q = T(W.random_density(700, seed=2, nrhs=4))
    allr = pl.apply(q)
    for r in range(4):
        assert torch.equal(pl.apply(q[r:r + 1].contiguous())[0], allr[r])


@pytest.mark.parametrize("prec,m", [(ibdl.MIXED, 2000), (ibdl.FP64, 20000)])
def test_packed_apply_equals_single_rhs(prec, m):
    """An apply of eight right-hand sides over a large spread reads its strengths
    packed four to a segment in the pass's precision (timed as its own stage); the
    values are the ones the sum rounds q to, so every right-hand side equals its
    apply alone (one right-hand side: no packing).  The spreads here pass the pack
    thresholds: 2^21 entries x right-hand sides in FP32, 2^24 in FP64."""
    p = random_problem(3, 64, m, seed=8)
    pl = plan_for(p, prec=prec)
    q = T(W.random_density(m, seed=5, nrhs=8))
    pl.set_timing(True)
    allr = pl.apply(q)
    names = [nm for nm, _, _ in pl.stage_times()]
    pl.set_timing(False)
    assert "pack" in names, names
    for r in range(8):
        assert torch.equal(pl.apply(q[r:r + 1].contiguous())[0], allr[r])


# ------------------------------------------------------------------ full-size workloads
@pytest.mark.parametrize("bc,alpha", [(W.DIRICHLET, 1.0), (W.NEUMANN, 100.0)])
def test_star1024_apply(bc, alpha):
    """The 1024^2 star workload (M=4096) in both precisions."""
    p = W.config_star1024(m=4096, alpha=alpha, bc=bc)
    st = O.setup_from_problem(p)
    q = W.random_density(4096, seed=3, nrhs=1)
    ref = O.apply_A(st, q[0], bc)
    out64 = N(plan_for(p).apply(T(q)))[0]
    assert relerr(out64, ref) < FP64_TOL
    out32 = N(plan_for(p, prec=ibdl.MIXED).apply(T(q)))[0]
    assert relerr(out32, ref) < MODEL_FACTOR * mixed_model(st, q[0], ref)


def test_largest_2d_grid():
    p = random_problem(2, 2048, 5000, seed=9, alpha=3.0)
    st = O.setup_from_problem(p)
    q = W.random_density(5000, seed=5, nrhs=1)
    ref = O.apply_A(st, q[0], W.DIRICHLET)
    assert relerr(N(plan_for(p).apply(T(q)))[0], ref) < FP64_TOL
    assert relerr(N(plan_for(p, prec=ibdl.MIXED).apply(T(q)))[0], ref) < MODEL_FACTOR * mixed_model(st, q[0], ref)


def test_largest_3d_grid():
    """The largest 3-D grid the library takes (512^3, its own radix plan and tile
    shapes): a 4000-point sphere, FP64 within 1e-12 of the oracle and mixed within
    its rounding-error model (the oracle's apply takes about 20 s and 10 GB here)."""
    g = W.Grid(3, 512, (0.0, 0.0, 0.0), 1.0)
    geom = W.fibonacci_sphere((0.5, 0.5, 0.5), 0.3, 4000)
    p = W.make_problem(g, geom, 10.0, W.DIRICHLET, W.sol_harmonic3d(1), forcing=False)
    st = O.setup_from_problem(p)
    q = W.random_density(4000, seed=3, nrhs=1)
    ref = O.apply_A(st, q[0], W.DIRICHLET)
    e64 = relerr(N(plan_for(p).apply(T(q)))[0], ref)
    e32 = relerr(N(plan_for(p, prec=ibdl.MIXED).apply(T(q)))[0], ref)
    model = mixed_model(st, q[0], ref)
    print(f"  512^3: FP64 rel err {e64:.2e}, mixed {e32:.2e} (model {model:.2e})", flush=True)
    assert e64 < FP64_TOL
    assert e32 < MODEL_FACTOR * model


@pytest.mark.parametrize("case", ["3d_one_point", "2d_one_cell", "2d_on_nodes", "3d_on_nodes", "3d_wrapped"])
def test_degenerate_geometries(case):
    """Degenerate point sets: a single 3-D point; 64 points inside one cell (one
    x-line carries every entry, and every node's entries come from one cell);
    points exactly on grid nodes (fractional offset 0, taps at the kernel's
    support edge); coordinates far outside the box, which wrap periodically.  FP64
    operator within 1e-12 of the oracle."""
    rng = np.random.default_rng(17)
    if case == "3d_one_point":
        p = random_problem(3, 16, 1, seed=3)
    elif case == "2d_one_cell":
        p = random_problem(2, 64, 64, seed=4)
        p.geom.X[:] = (np.array([17.0, 40.0]) + rng.uniform(0.0, 1.0, size=(64, 2))) / 64.0
    elif case == "2d_on_nodes":
        p = random_problem(2, 64, 300, seed=5)
        p.geom.X[:] = rng.integers(0, 64, size=(300, 2)) / 64.0
    elif case == "3d_on_nodes":
        p = random_problem(3, 24, 400, seed=6)
        p.geom.X[:] = rng.integers(0, 24, size=(400, 3)) / 24.0
    else:
        p = random_problem(3, 24, 400, seed=7)
        p.geom.X[:] = p.geom.X + rng.integers(-5, 6, size=(400, 3))
    m = p.geom.m
    st = O.setup_from_problem(p)
    q = W.random_density(m, seed=8, nrhs=2)
    out = N(plan_for(p).apply(T(q)))
    for r in range(2):
        ref = O.apply_A(st, q[r], W.DIRICHLET)
        assert relerr(out[r], ref) < FP64_TOL, (case, r)


# ------------------------------------------------------------------ solves
def test_circle64_solve_fp64():
    p = W.config_circle64()
    st = O.setup_from_problem(p, delta=O.COSINE4)
    res, _ = O.solve(st, p.data, p.g_tilde, tol=1e-10)
    pl = plan_for(p, delta=O.COSINE4)
    sol, info = pl.solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-10, true_residual=True)
    assert abs(info[0]["iters"] - res.iters) <= 1
    assert info[0]["rel_resid_true"] < 2e-10
    tight, _ = O.solve(st, p.data, p.g_tilde, tol=1e-14)
    assert relerr(N(sol)[0], tight.x) < 1e-9
    u = N(pl.eval_grid(sol, g=T(p.g_tilde[None])))[0]
    uref = O.eval_grid(st, tight.x, g_tilde=p.g_tilde)
    assert relerr(u, uref) < 1e-9


@pytest.mark.parametrize("n", [64, 128])
def test_neumann_solve_fp64_and_mixed(n):
    p = W.neumann_circle_problem(n)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, bc=O.NEUMANN, tol=1e-14)
    res8, _ = O.solve(st, p.data, p.g_tilde, bc=O.NEUMANN, tol=1e-8)
    sol, info = plan_for(p).solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-8)
    assert abs(info[0]["iters"] - res8.iters) <= 1
    assert relerr(N(sol)[0], tight.x) < 1e-6
    sol, info = plan_for(p).solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-13)
    assert relerr(N(sol)[0], tight.x) < 1e-11
    solm, infom = plan_for(p, prec=ibdl.MIXED).solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-8)
    assert relerr(N(solm)[0], tight.x) < SOLVE_MIXED_TOL
    assert infom[0]["rel_resid_true"] <= 1e-8 and infom[0]["fp64_applies"] >= 1


def test_table1_iterations_on_gpu():
    for n in (64, 128, 256):
        for c in (2.0, 0.75):
            p = W.table1_problem(n, c)
            st = O.setup_from_problem(p)
            res, _ = O.solve(st, p.data, p.g_tilde, tol=1e-8)
            _, info = plan_for(p).solve(T(p.data[None]), None, tol=1e-8)
            assert abs(info[0]["iters"] - res.iters) <= 1, (n, c)


def test_3d_solve():
    p = W.table2_problem(32, 900)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, tol=1e-13)
    sol, info = plan_for(p).solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-12)
    assert relerr(N(sol)[0], tight.x) < 1e-10
    assert 4 <= info[0]["iters"] <= 12


def test_batched_rhs_solve_equals_single():
    p = W.config_star1024(m=1116, n=256, alpha=100.0)
    pl = plan_for(p)
    rng = np.random.default_rng(1)
    data = np.stack([p.data, rng.standard_normal(p.geom.m), 0.5 * p.data])
    g = np.stack([p.g_tilde, np.zeros_like(p.g_tilde), p.g_tilde])
    sols, infos = pl.solve(T(data), T(g), tol=1e-10)
    for r in range(3):
        s1, i1 = pl.solve(T(data[r:r + 1]), T(g[r:r + 1]), tol=1e-10)
        assert i1[0]["iters"] == infos[r]["iters"]
        assert torch.equal(s1[0], sols[r])


def test_restart_and_noconv():
    p = W.table1_problem(64, 1.0)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, tol=1e-14)
    pl = plan_for(p)
    sol, info = pl.solve(T(p.data[None]), None, tol=1e-11, restart=2, maxit=200)
    assert relerr(N(sol)[0], tight.x) < 1e-9
    with pytest.raises(ibdl.IbdlError) as e:
        pl.solve(T(p.data[None]), None, tol=1e-12, maxit=1)
    assert e.value.status == ibdl.ERR_NOCONV
    sol, info = pl.solve(T(p.data[None]), None, tol=1e-12, maxit=1, raise_on_noconv=False)
    assert info[0]["iters"] == 1 and info[0]["status"] == ibdl.ERR_NOCONV


def test_nonfinite_geometry_rejected():
    p = random_problem(2, 32, 10, seed=1)
    X = p.geom.X.copy()
    X[3, 1] = np.nan
    with pytest.raises(ibdl.IbdlError) as e:
        ibdl.Plan(2, 32, (0.0, 0.0), 1.0, 1.0, T(X), T(p.geom.normal), T(p.geom.weight))
    assert e.value.status == ibdl.ERR_NUMERIC


@pytest.mark.parametrize("bc,alpha", [(W.DIRICHLET, 1.0), (W.DIRICHLET, 100.0), (W.NEUMANN, 1.0),
                                      (W.NEUMANN, 100.0)])
def test_star1024_solve_mixed_within_1e6(bc, alpha):
    """The 1024^2 star workload: mixed solve and grid solution within 1e-6 of the oracle."""
    p = W.config_star1024(m=4096, alpha=alpha, bc=bc)
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, bc=bc, tol=1e-13)
    pl = plan_for(p, prec=ibdl.MIXED)
    sol, info = pl.solve(T(p.data[None]), T(p.g_tilde[None]), tol=1e-8)
    assert info[0]["rel_resid_true"] <= 1e-8
    assert relerr(N(sol)[0], tight.x) < SOLVE_MIXED_TOL
    vb = T(p.data[None]) if bc == W.NEUMANN else None
    u = N(pl.eval_grid(sol, vb, T(p.g_tilde[None])))[0]
    uref = O.eval_grid(st, tight.x, vb=p.data if bc == W.NEUMANN else None, g_tilde=p.g_tilde, bc=bc)
    assert relerr(u, uref) < SOLVE_MIXED_TOL
