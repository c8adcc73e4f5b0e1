"""Step 3 of the method on the GPU against the oracle: the domain flags of the
App. D indicator and the near-boundary re-interpolation of App. A (Sec. 5.5).

Bars: chi within 1e-12 (absolute, chi is O(1)); flags identical except at
nodes whose chi lies within 1e-9 of the threshold (the decision is taken in
FP64 on both sides from sums in different orders); re-interpolated values
within 1e-12 relative to max |u|, the set of replaced nodes identical except
where the nearest-point distance lies within 1e-12 of m1 h."""
import math

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


def flip(geom):
    """The same boundary with normals pointing into the enclosed region (the PDE
    domain is then the rest of the box)."""
    return W.Geometry(geom.dim, geom.X, -geom.normal, geom.weight, lambda p: ~geom.inside(p), geom.measure)


def problems():
    out = []
    p = W.table1_problem(128, 0.75)
    out.append(("circle128", p, 6.0, 8.0, ibdl.LAP_FD))
    # exterior of a star on a 256^2 grid, Dirichlet data of the random-Fourier field
    g = W.Grid(2, 256, (0.0, 0.0), 1.0)
    st_geom = flip(W.star((0.5, 0.5), 0.3, 0.05, 5, 1500))
    out.append(("star256-exterior", W.make_problem(g, st_geom, 4.0, W.DIRICHLET, W.sol_random_fourier(2, 3)),
                6.0, 8.0, ibdl.LAP_FD))
    # spectral widths m1 = 2(log2 n - 4), m2 = m1 + 2 (Sec. 6.2.1)
    p2 = W.table1_problem(256, 1.0)
    m1 = 2.0 * (math.log2(256) - 4)
    out.append(("circle256-spectral", p2, m1, m1 + 2.0, ibdl.LAP_SPECTRAL))
    g3 = W.Grid(3, 48, (0.0, 0.0, 0.0), 1.0)
    out.append(("sphere48", W.make_problem(g3, W.fibonacci_sphere((0.5, 0.5, 0.5), 0.3, 6000), 2.0, W.DIRICHLET,
                                            W.sol_exp_cos3d()), 4.0, 6.0, ibdl.LAP_FD))
    return out


@pytest.mark.parametrize("name,prob,m1,m2,lap", problems(), ids=lambda v: v if isinstance(v, str) else "")
def test_indicator_and_fixup_match_oracle(name, prob, m1, m2, lap):
    st = O.setup_from_problem(prob, lap=O.LAP_SPECTRAL if lap == ibdl.LAP_SPECTRAL else O.LAP_FD)
    pl = ibdl.Plan.from_problem(prob, lap=lap)
    chi, flags = pl.indicator()
    chi_o, flags_o = O.omega_flags(st)
    chi, flags = N(chi), N(flags)
    assert np.max(np.abs(chi - chi_o)) < 1e-12
    thr = 0.5 * O.orientation(st)
    decided = np.abs(chi_o - thr) > 1e-9
    assert np.array_equal(flags[decided], flags_o[decided].astype(np.uint8))
    # a grid solution to re-interpolate: the solve of the problem (two right-hand sides)
    data = np.stack([prob.data, 0.5 * prob.data + 1.0])
    g = np.stack([prob.g_tilde, 0.5 * prob.g_tilde])
    sol, u, info = pl.solve_grid(T(data), T(g), tol=1e-10)
    fl = torch.as_tensor(flags, dtype=torch.uint8, device="cuda").contiguous()
    fixed = N(pl.fixup(u, T(data), fl, m1=m1, m2=m2))
    un = N(u)
    nodes = np.stack([c.ravel() for c in prob.grid.nodes()], axis=1)
    d1 = O.distance_to_points(st, nodes, prob.geom.X).reshape(flags.shape)
    edge = np.abs(d1 - m1 * st.h) < 1e-12
    nrep = 0
    for r in range(2):
        ref, done = O.near_boundary_fixup(st, un[r], data[r], flags, m1, m2)
        changed = fixed[r] != un[r]
        assert np.array_equal(changed[~edge], (done & (ref != un[r]))[~edge])
        scale = np.max(np.abs(un[r]))
        assert np.max(np.abs(fixed[r] - ref)[~edge]) < 1e-12 * scale, name
        nrep = int(done.sum())
    print(f"  {name}: {nrep} nodes re-interpolated", flush=True)
    assert nrep > 100
    pl.close()


def test_fixup_after_a_neumann_solve():
    """Neumann data: the boundary values of the re-interpolation are the solved U_b
    (the unknown of the Neumann system, Sec. 4.4), the grid solution that of the
    same solve; against the oracle's fix-up of the same arrays."""
    prob = W.neumann_circle_problem(128)
    st = O.setup_from_problem(prob)
    pl = ibdl.Plan.from_problem(prob)
    _, flags = pl.indicator()
    flags = N(flags)
    sol, u, info = pl.solve_grid(T(prob.data[None]), T(prob.g_tilde[None]), tol=1e-10)
    fl = torch.as_tensor(flags, dtype=torch.uint8, device="cuda").contiguous()
    fixed = N(pl.fixup(u, sol, fl, m1=6.0, m2=8.0))[0]
    un, ub = N(u)[0], N(sol)[0]
    ref, done = O.near_boundary_fixup(st, un, ub, flags, 6.0, 8.0)
    nodes = np.stack([c.ravel() for c in prob.grid.nodes()], axis=1)
    d1 = O.distance_to_points(st, nodes, prob.geom.X).reshape(flags.shape)
    edge = np.abs(d1 - 6.0 * st.h) < 1e-12
    assert np.max(np.abs(fixed - ref)[~edge]) < 1e-12 * np.max(np.abs(un))
    assert int(done.sum()) > 100
    pl.close()


def test_fixup_argument_errors():
    p = W.table1_problem(64, 1.0)
    pl = ibdl.Plan.from_problem(p)
    u = torch.zeros(1, 64, 64, dtype=torch.float64, device="cuda")
    ub = torch.zeros(1, p.geom.m, dtype=torch.float64, device="cuda")
    fl = torch.ones(64, 64, dtype=torch.uint8, device="cuda")
    for m1, m2 in ((0.0, 8.0), (6.0, 6.0), (6.0, 40.0)):
        with pytest.raises(ibdl.IbdlError) as e:
            pl.fixup(u, ub, fl, m1=m1, m2=m2)
        assert e.value.status == ibdl.ERR_ARG
    pl.close()
