"""The Poisson equation (alpha = 0) on the GPU against the oracle: the original
IBDL method on the starfish exterior (Sec. 6.4; balanced forcing, mean-zero
inverse) and the completed IBDL method on the large exterior box (Sec. 5.4.1,
Sec. 6.3, App. C): bordered operator and right-hand side within 1e-12, the
solution [Q; ubar] and the grid solution against the oracle's tight GMRES solve
of the bordered system."""
import numpy as np
import pytest

from oracle import ibdl_oracle as O
from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n", [128, 256])
def test_starfish_original_ibdl(n):
    p = W.starfish_problem(n)
    st = O.setup_from_problem(p)
    res, _ = O.solve(st, p.data, p.g_tilde, tol=1e-8)
    tight, _ = O.solve(st, p.data, p.g_tilde, tol=1e-13)
    for prec in (ibdl.FP64, ibdl.MIXED):
        pl = ibdl.Plan.from_problem(p, prec=prec)
        sol, u, info = pl.solve_grid(T(p.data[None]), T(p.g_tilde[None]), tol=1e-8)
        if prec == ibdl.FP64:
            assert abs(info[0]["iters"] - res.iters) <= 1
        uref = O.eval_grid(st, tight.x, g_tilde=p.g_tilde)
        assert relerr(N(sol)[0], tight.x) < 1e-6 and relerr(N(u)[0], uref) < 1e-6
        pl.close()


@pytest.mark.parametrize("n,prec", [(128, ibdl.FP64), (256, ibdl.FP64), (256, ibdl.MIXED)])
def test_completed_exterior_box(n, prec):
    eta = 10.0
    p = W.poisson_exterior_problem(n, 8.0, balanced=False)
    st = O.setup_from_problem(p)
    M = p.geom.m
    pl = ibdl.Plan.from_problem(p, prec=prec, form=ibdl.FORM_COMPLETED, eta=eta)
    # the bordered operator and right-hand side
    z = W.random_density(M + 1, seed=3, nrhs=2)
    az = N(pl.apply(T(z)))
    b = N(pl.rhs(T(np.stack([p.data, 0.3 * p.data])), T(np.stack([p.g_tilde, -p.g_tilde]))))
    if prec == ibdl.FP64:
        for r in range(2):
            assert relerr(az[r], O.apply_completed(st, z[r], eta)) < 1e-12
        assert relerr(b[0], O.rhs_completed(st, p.data, p.g_tilde)) < 1e-12
        assert relerr(b[1], O.rhs_completed(st, 0.3 * p.data, -p.g_tilde)) < 1e-12
    # the solve: [Q; ubar] and u against the oracle's GMRES on the bordered system
    tight, _ = O.solve_completed(st, p.data, p.g_tilde, eta=eta, tol=1e-13)
    uref = O.eval_grid_completed(st, tight.x, p.g_tilde, eta)
    data = T(np.stack([p.data, 2.0 * p.data]))
    g = T(np.stack([p.g_tilde, 2.0 * p.g_tilde]))
    sol, u, info = pl.solve_grid(data, g, tol=1e-10 if prec == ibdl.FP64 else 1e-8)
    sol, u = N(sol), N(u)
    bar = 1e-8 if prec == ibdl.FP64 else 1e-6
    for r, s in enumerate((1.0, 2.0)):
        assert info[r]["status"] == ibdl.OK
        assert relerr(sol[r], s * tight.x) < bar, (r, relerr(sol[r], s * tight.x))
        assert relerr(u[r], s * uref) < bar
    # the grid solution of eval_grid equals that of solve_grid
    ue = N(pl.eval_grid(T(sol), g=g))
    assert np.max(np.abs(ue - u)) < 1e-12 * np.max(np.abs(u))
    pl.close()


def test_completed_rejects_wrong_problems():
    p = W.poisson_exterior_problem(64, 8.0, balanced=False)
    t = lambda a: T(a)
    g = p.grid
    with pytest.raises(ibdl.IbdlError) as e:
        ibdl.Plan(2, 64, tuple(g.lo), g.length, 1.0, t(p.geom.X), t(p.geom.normal), t(p.geom.weight),
                  form=ibdl.FORM_COMPLETED, eta=10.0)
    assert e.value.status == ibdl.ERR_ARG
    with pytest.raises(ibdl.IbdlError):
        ibdl.Plan(2, 64, tuple(g.lo), g.length, 0.0, t(p.geom.X), t(p.geom.normal), t(p.geom.weight),
                  form=ibdl.FORM_COMPLETED, eta=0.0)
