"""Oracle parity of every kernel instantiation the workloads use.

Each grid size compiles its own radix plan, tile width, lines per block and
thread count, so every size of the 2-D and 3-D workloads is checked against the
FP64 oracle on geometry of the workloads' shapes (ellipse, star, circle,
sphere, ellipsoid) with both boundary conditions:

* FP64 operator (Sec. 5.3, the equation for Q; Sec. 4.4, the equation for
  U_b), right-hand side and grid solution within 1e-12 relative;
* the mixed (FP32 grid) operator within its rounding-error model (below),
  with the measured error printed;
* the 256^3 sphere solves in both precisions against the oracle's tight solve.

The mixed operator is held to the rounding-error model of error_model.py
(measured errors printed beside the model).
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

FP64_TOL = 1e-12
SOLVE_MIXED_TOL = 1e-6


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def N(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def geometry_problem(dim, n, shape, bc, alpha, c=1.0, seed=17):
    """A problem of the workloads' recipe at grid size n: 2-D ellipse (batch recipe),
    circle or star (served recipe); 3-D sphere or ellipsoid (served recipe)."""
    if dim == 2 and shape == "ellipse":
        a, b, rot = 0.27, 0.14, 0.6
        m = max(16, int(round(W.ellipse_perimeter(a, b) / (c / n))))
        spec = dict(n=n, a=a, b=b, rot=rot, nrhs=1, bc=bc, alpha=alpha, m=m, seed=seed)
        _, _, probs = W.batch_instance(spec)
        return probs[0]
    if dim == 2:
        radius = 0.31
        per = 2 * math.pi * radius if shape == "circle" else W.star_perimeter(W.STAR_R0, W.STAR_AMP, W.STAR_LOBES)
        m = int(min(max(round(per / (c / n)), 1000), 16000))
        spec = dict(dim=2, n=n, shape=shape, radius=radius, bc=bc, alpha=alpha, m=m, c=c, seed=seed)
        return W.serve_instance(spec)
    axes = (0.3, 0.3, 0.3) if shape == "sphere" else (0.33, 0.24, 0.21)
    m = int(min(max(round(W.ellipsoid_area(axes) / (c / n) ** 2), 5000), 40000))
    spec = dict(dim=3, n=n, shape=shape, axes=axes, bc=bc, alpha=alpha, m=m, c=c, seed=seed)
    return W.serve_instance(spec)


D, NEU = W.DIRICHLET, W.NEUMANN
CASES = [
    # dim, n, shape, bc, alpha, spacing c
    (2, 256, "ellipse", D, 10.0, 0.75),
    (2, 256, "circle", NEU, 300.0, 1.5),
    (2, 512, "star", NEU, 1.0, 1.0),
    (2, 512, "ellipse", D, 1000.0, 0.75),
    (2, 768, "circle", D, 100.0, 1.0),
    (2, 768, "star", NEU, 3.0, 2.0),
    (2, 1536, "star", NEU, 1000.0, 0.6),
    (2, 1536, "circle", D, 1.0, 1.0),
    (3, 64, "sphere", D, 10.0, 1.0),
    (3, 64, "ellipsoid", NEU, 5.0, 1.5),
    (3, 96, "ellipsoid", D, 300.0, 1.0),
    (3, 128, "sphere", NEU, 1.0, 1.5),
    (3, 128, "ellipsoid", D, 30.0, 1.0),
    (3, 192, "ellipsoid", D, 3.0, 1.2),
    (3, 256, "sphere", D, 10.0, 0.0),  # the 256^3 sphere workload itself (M = 40000)
]


def case_problem(dim, n, shape, bc, alpha, c):
    if dim == 3 and n == 256:
        return W.config_sphere256()
    return geometry_problem(dim, n, shape, bc, alpha, c)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dim,n,shape,bc,alpha,c", CASES)
def test_operator_rhs_grid_at_size(dim, n, shape, bc, alpha, c):
    p = case_problem(dim, n, shape, bc, alpha, c)
    st = O.setup_from_problem(p)
    m = p.geom.m
    nrhs = 2
    q = W.random_density(m, seed=n + m, nrhs=nrhs)
    print(f"\n[{dim}-D n={n} {shape} bc={bc} alpha={alpha} M={m}]", flush=True)
    refs = [O.apply_A(st, q[r], bc) for r in range(nrhs)]
    # FP64 operator
    pl = ibdl.Plan.from_problem(p)
    out = N(pl.apply(T(q)))
    for r in range(nrhs):
        e = relerr(out[r], refs[r])
        assert e < FP64_TOL, (r, e)
    # right-hand side and grid solution (FP64 passes), with the forcing of the problem
    data = np.stack([p.data, 0.5 * p.data + q[0]])
    g = np.stack([p.g_tilde, -p.g_tilde])
    b = N(pl.rhs(T(data), T(g)))
    sol = q
    vb = data if bc == NEU else None
    u = N(pl.eval_grid(T(sol), T(vb) if vb is not None else None, T(g)))
    for r in range(nrhs):
        rb = O.rhs(st, data[r], g[r], bc)
        assert relerr(b[r], rb) < FP64_TOL, ("rhs", r, relerr(b[r], rb))
        ru = O.eval_grid(st, sol[r], None if vb is None else vb[r], g[r], bc)
        assert relerr(u[r], ru) < FP64_TOL, ("grid", r, relerr(u[r], ru))
    pl.close()
    # mixed operator against the rounding-error model
    plm = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    outm = N(plm.apply(T(q)))
    plm.close()
    for r in range(nrhs):
        e = relerr(outm[r], refs[r])
        model = mixed_model(st, q[r], refs[r])
        print(f"  mixed apply rel err {e:.3e}  model {model:.3e}  ratio {e / model:.2f}", flush=True)
        assert e < MODEL_FACTOR * model, (r, e, model)


@pytest.fixture(scope="module")
def sphere256_tight():
    p = W.config_sphere256()
    st = O.setup_from_problem(p)
    tight, _ = O.solve(st, p.data, p.g_tilde, tol=1e-11)
    u = O.eval_grid(st, tight.x, g_tilde=p.g_tilde)
    return p, tight, u


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [(ibdl.FP64, 1e-10), (ibdl.MIXED, 1e-8)])
def test_sphere256_solve_matches_oracle(sphere256_tight, prec, tol):
    """The 256^3 sphere (M = 40000): solve and grid solution against the oracle's
    solve to 1e-11, in both precisions."""
    p, tight, uref = sphere256_tight
    pl = ibdl.Plan.from_problem(p, prec=prec)
    sol, u, info = pl.solve_grid(T(p.data[None]), T(p.g_tilde[None]), tol=tol)
    pl.close()
    es = relerr(N(sol)[0], tight.x)
    eu = relerr(N(u)[0], uref)
    print(f"\n[sphere256 prec={prec}] iters {info[0]['iters']} Q err {es:.3e} u err {eu:.3e}", flush=True)
    assert info[0]["status"] == ibdl.OK
    assert 4 <= info[0]["iters"] <= 14
    bar = 1e-8 if prec == ibdl.FP64 else SOLVE_MIXED_TOL
    assert es < bar and eu < bar


@pytest.mark.timeout(600)
def test_batch_at_c4_sizes_matches_oracle():
    """Batched mixed solves with grid solutions over instances of every size of the
    512-instance batch (n = 128 .. 512, both boundary conditions) against the oracle."""
    specs = W.config_batch(count=64, seed=12126)
    chosen = []
    for n in (128, 192, 256, 384, 512):
        for want_bc in (D, NEU):
            sp = next(s for s in specs if s["n"] == n and s["bc"] == want_bc)
            sp = dict(sp)
            sp["nrhs"] = 2
            chosen.append(sp)
    items = [W.batch_instance(sp)[2] for sp in chosen]
    batch = ibdl.Batch.from_problems([(probs[0], len(probs)) for probs in items], prec=ibdl.MIXED)
    data = [T(np.stack([q.data for q in probs])) for probs in items]
    g = [T(np.stack([q.g_tilde for q in probs])) for probs in items]
    sol, u, info = batch.solve_grid(data, g, tol=1e-8)
    r0 = 0
    for i, probs in enumerate(items):
        st = O.setup_from_problem(probs[0])
        for r, pr in enumerate(probs):
            tight, _ = O.solve(st, pr.data, pr.g_tilde, bc=pr.bc, tol=1e-13)
            uref = O.eval_grid(st, tight.x, vb=pr.data if pr.bc == NEU else None, g_tilde=pr.g_tilde, bc=pr.bc)
            es = relerr(N(sol[i][r]), tight.x)
            eu = relerr(N(u[i][r]), uref)
            assert info[r0 + r]["status"] == ibdl.OK
            assert es < SOLVE_MIXED_TOL and eu < SOLVE_MIXED_TOL, (chosen[i]["n"], pr.bc, r, es, eu)
        r0 += len(probs)
    batch.close()
