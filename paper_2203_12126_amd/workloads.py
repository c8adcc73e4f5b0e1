"""Seeded synthetic inputs for the IBDL hot path.

This module is shared by the oracle and the HIP path and therefore holds none of
the method's arithmetic: it only builds boundary geometries (points, unit
normals pointing out of the PDE domain, quadrature weights), periodic grids and
manufactured solutions with their forcing and boundary data.

Conventions (Sec. 5.1 of the paper): the computational domain is a periodic box
of side ``length`` with ``n`` nodes per axis, node ``i`` at ``lo + i*h`` with
``h = length/n``.  Grid arrays are C-ordered ``[iz][iy][ix]`` (x fastest);
point coordinates are ``X[:, 0] = x``, ``X[:, 1] = y``, ``X[:, 2] = z``.
The PDE is ``Lap(u) - alpha*u = g`` (the model problem of Sec. 2 with ``alpha = k^2``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

DIRICHLET = 0
NEUMANN = 1


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
@dataclass
class Grid:
    dim: int
    n: int
    lo: tuple
    length: float

    @property
    def h(self) -> float:
        return self.length / self.n

    def axis_coords(self, d: int) -> np.ndarray:
        return self.lo[d] + self.h * np.arange(self.n)

    def nodes(self):
        """Coordinate arrays (x, y[, z]) shaped like a grid field."""
        ax = [self.axis_coords(d) for d in range(self.dim)]
        # C-order [iz][iy][ix]: meshgrid with reversed axes
        mesh = np.meshgrid(*ax[::-1], indexing="ij")
        return tuple(mesh[::-1])


# ----------------------------------------------------------------------------
# closed curves, points equispaced in arclength (Sec. 5.2: Delta s = L_IB/N_IB)
# ----------------------------------------------------------------------------
def _arclength_points(pos: Callable, vel: Callable, m: int, nfine: int = 4096):
    """Place m points equispaced in arclength along a smooth closed curve.

    ``pos(theta)`` and ``vel(theta)`` give the position and d/dtheta of a
    counter-clockwise 2-pi-periodic parametrisation.  The speed is expanded in
    a Fourier series, integrated term by term, and s(theta) = s_k is inverted
    by Newton's method.  Returns (theta_k, perimeter).
    """
    th = 2 * np.pi * np.arange(nfine) / nfine
    sp = np.hypot(*vel(th))
    c = np.fft.rfft(sp) / nfine
    perim = 2 * np.pi * c[0].real
    k = np.arange(1, c.size)

    def s_of(t):
        t = np.atleast_1d(t)
        # s(t) = c0 t + sum_k 2 Re( c_k (e^{ikt}-1)/(ik) )
        e = np.exp(1j * np.outer(t, k)) - 1.0
        return c[0].real * t + 2.0 * np.real(e @ (c[1:] / (1j * k)))

    target = perim * np.arange(m) / m
    t = target / perim * 2 * np.pi
    for _ in range(30):
        f = s_of(t) - target
        t = t - f / np.hypot(*vel(t))
        if np.max(np.abs(f)) < 1e-15 * perim:
            break
    return t, perim


def _curve_geometry(pos, vel, m, level, interior=True):
    """``level(p) < 0`` strictly inside the curve, ``> 0`` strictly outside."""
    t, perim = _arclength_points(pos, vel, m)
    x, y = pos(t)
    vx, vy = vel(t)
    sp = np.hypot(vx, vy)
    # outward normal of a counter-clockwise curve
    nrm = np.stack([vy / sp, -vx / sp], axis=1)
    if not interior:
        nrm = -nrm
    X = np.stack([x, y], axis=1)
    w = np.full(m, perim / m)
    body = lambda p: level(p) < 0
    dom = body if interior else (lambda p: level(p) > 0)
    return Geometry(2, X, nrm, w, dom, perim, body_inside=body)


@dataclass
class Geometry:
    dim: int
    X: np.ndarray        # (M, dim) boundary points
    normal: np.ndarray   # (M, dim) unit normals pointing out of Omega
    weight: np.ndarray   # (M,) arclength Delta s_i (2-D) or area dA_i (3-D)
    inside: Callable     # strict membership test of the PDE domain Omega
    measure: float       # perimeter (2-D) or area (3-D) of Gamma
    body_inside: Optional[Callable] = None

    @property
    def m(self) -> int:
        return self.X.shape[0]


def circle(center, radius, m, interior=True, equispaced_theta=True) -> Geometry:
    c = np.asarray(center, dtype=np.float64)
    th = 2 * np.pi * np.arange(m) / m
    X = c + radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    nrm = np.stack([np.cos(th), np.sin(th)], axis=1)

    def body(p):
        return np.sum((p - c) ** 2, axis=1) < radius ** 2

    if not interior:
        nrm = -nrm
        dom = lambda p: np.sum((p - c) ** 2, axis=1) > radius ** 2
    else:
        dom = body
    return Geometry(2, X, nrm, np.full(m, 2 * np.pi * radius / m), dom,
                    2 * np.pi * radius, body_inside=body)


def star(center, r0, amp, lobes, m, interior=True, phase=0.0) -> Geometry:
    """r(theta) = r0 + amp*cos(lobes*theta + phase) about ``center``."""
    c = np.asarray(center, dtype=np.float64)

    def pos(t):
        r = r0 + amp * np.cos(lobes * t + phase)
        return c[0] + r * np.cos(t), c[1] + r * np.sin(t)

    def vel(t):
        r = r0 + amp * np.cos(lobes * t + phase)
        dr = -amp * lobes * np.sin(lobes * t + phase)
        return dr * np.cos(t) - r * np.sin(t), dr * np.sin(t) + r * np.cos(t)

    def level(p):
        d = p - c
        rr = np.hypot(d[:, 0], d[:, 1])
        th = np.arctan2(d[:, 1], d[:, 0])
        return rr - (r0 + amp * np.cos(lobes * th + phase))

    return _curve_geometry(pos, vel, m, level, interior)


def star_perimeter(r0, amp, lobes) -> float:
    def vel(t):
        r = r0 + amp * np.cos(lobes * t)
        dr = -amp * lobes * np.sin(lobes * t)
        return dr * np.cos(t) - r * np.sin(t), dr * np.sin(t) + r * np.cos(t)
    th = 2 * np.pi * np.arange(8192) / 8192
    return float(np.mean(np.hypot(*vel(th))) * 2 * np.pi)


def ellipse(center, a, b, rot, m, interior=True) -> Geometry:
    c = np.asarray(center, dtype=np.float64)
    cr, sr = math.cos(rot), math.sin(rot)

    def pos(t):
        u, v = a * np.cos(t), b * np.sin(t)
        return c[0] + cr * u - sr * v, c[1] + sr * u + cr * v

    def vel(t):
        u, v = -a * np.sin(t), b * np.cos(t)
        return cr * u - sr * v, sr * u + cr * v

    def level(p):
        d = p - c
        u = cr * d[:, 0] + sr * d[:, 1]
        v = -sr * d[:, 0] + cr * d[:, 1]
        return (u / a) ** 2 + (v / b) ** 2 - 1.0

    return _curve_geometry(pos, vel, m, level, interior)


def ellipse_perimeter(a, b) -> float:
    th = 2 * np.pi * np.arange(8192) / 8192
    return float(np.mean(np.hypot(a * np.sin(th), b * np.cos(th))) * 2 * np.pi)


def fibonacci_sphere(center, radius, m) -> Geometry:
    """Fibonacci lattice on a sphere, equal weights 4 pi R^2 / M, radial normals."""
    c = np.asarray(center, dtype=np.float64)
    k = np.arange(m)
    z = 1.0 - (2 * k + 1) / m
    rho = np.sqrt(np.maximum(0.0, 1 - z * z))
    az = k * math.pi * (3.0 - math.sqrt(5.0))
    u = np.stack([rho * np.cos(az), rho * np.sin(az), z], axis=1)
    X = c + radius * u
    body = lambda p: np.sum((p - c) ** 2, axis=1) < radius ** 2
    return Geometry(3, X, u.copy(), np.full(m, 4 * math.pi * radius ** 2 / m), body,
                    4 * math.pi * radius ** 2, body_inside=body)


def fibonacci_ellipsoid(center, axes, m) -> Geometry:
    """Image of the Fibonacci lattice under diag(a, b, c) with matching area weights."""
    cen = np.asarray(center, dtype=np.float64)
    a, b, cc = axes
    k = np.arange(m)
    z = 1.0 - (2 * k + 1) / m
    rho = np.sqrt(np.maximum(0.0, 1 - z * z))
    az = k * math.pi * (3.0 - math.sqrt(5.0))
    u = np.stack([rho * np.cos(az), rho * np.sin(az), z], axis=1)
    X = cen + u * np.array([a, b, cc])
    g = u / np.array([a, b, cc])
    gn = np.linalg.norm(g, axis=1)
    nrm = g / gn[:, None]
    w = (4 * math.pi / m) * a * b * cc * gn
    body = lambda p: np.sum(((p - cen) / np.array([a, b, cc])) ** 2, axis=1) < 1.0
    return Geometry(3, X, nrm, w, body, float(np.sum(w)), body_inside=body)


# ----------------------------------------------------------------------------
# manufactured solutions: u, grad u, Lap u
# ----------------------------------------------------------------------------
@dataclass
class Solution:
    u: Callable          # (P, dim) -> (P,)
    grad: Callable       # (P, dim) -> (P, dim)
    lap: Callable        # (P, dim) -> (P,)


def sol_exp_sin() -> Solution:
    """u = exp(x) sin(y) (harmonic)."""
    return Solution(
        lambda p: np.exp(p[:, 0]) * np.sin(p[:, 1]),
        lambda p: np.stack([np.exp(p[:, 0]) * np.sin(p[:, 1]),
                            np.exp(p[:, 0]) * np.cos(p[:, 1])], axis=1),
        lambda p: np.zeros(p.shape[0]))


def sol_x2_minus_y2() -> Solution:
    return Solution(
        lambda p: p[:, 0] ** 2 - p[:, 1] ** 2,
        lambda p: np.stack([2 * p[:, 0], -2 * p[:, 1]], axis=1),
        lambda p: np.zeros(p.shape[0]))


def sol_exp_cos3d() -> Solution:
    """u = exp(x+y) cos(sqrt(2) z - 0.3) (harmonic)."""
    s2 = math.sqrt(2.0)

    def u(p):
        return np.exp(p[:, 0] + p[:, 1]) * np.cos(s2 * p[:, 2] - 0.3)

    def grad(p):
        e = np.exp(p[:, 0] + p[:, 1])
        c = np.cos(s2 * p[:, 2] - 0.3)
        s = np.sin(s2 * p[:, 2] - 0.3)
        return np.stack([e * c, e * c, -s2 * e * s], axis=1)

    return Solution(u, grad, lambda p: np.zeros(p.shape[0]))


def harmonic3d_params(seed: int):
    """(k, l, phase) of u = exp(k.x) cos(l.x + phase) with |k| = |l|, k . l = 0, so
    that u is harmonic.  seed 0 is exp(x+y) cos(sqrt(2) z - 0.3); other seeds
    draw an orthonormal pair of directions, a common length in U(0.8, 1.6) and a
    phase in U(0, 2 pi)."""
    if seed == 0:
        return np.array([1.0, 1.0, 0.0]), np.array([0.0, 0.0, math.sqrt(2.0)]), -0.3
    rng = np.random.default_rng(seed)
    e1 = rng.standard_normal(3)
    e1 /= np.linalg.norm(e1)
    e2 = rng.standard_normal(3)
    e2 -= np.dot(e2, e1) * e1
    e2 /= np.linalg.norm(e2)
    s = rng.uniform(0.8, 1.6)
    return s * e1, s * e2, float(rng.uniform(0.0, 2 * math.pi))


def sol_harmonic3d(seed: int) -> Solution:
    """u = exp(k.x) cos(l.x + phase) with the parameters of harmonic3d_params (harmonic)."""
    k, l, ph = harmonic3d_params(seed)

    def u(p):
        return np.exp(p @ k) * np.cos(p @ l + ph)

    def grad(p):
        e = np.exp(p @ k)
        c = np.cos(p @ l + ph)
        s = np.sin(p @ l + ph)
        return e[:, None] * (c[:, None] * k[None, :] - s[:, None] * l[None, :])

    return Solution(u, grad, lambda p: np.zeros(p.shape[0]))


def harmonic3d_grid(seed: int, grid: "Grid") -> np.ndarray:
    """sol_harmonic3d(seed) at the grid nodes by separable evaluation:
    u = Re(e^{i phase} prod_d exp((k_d + i l_d) x_d))."""
    k, l, ph = harmonic3d_params(seed)
    f = [np.exp((k[d] + 1j * l[d]) * grid.axis_coords(d)) for d in range(3)]
    return np.real(np.exp(1j * ph) * f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :])


def sol_bessel_sin2(center=(0.0, 0.0), radius=0.25, k=1.0) -> Solution:
    """u = I_2(k r) sin(2 theta) / I_2(k R): solves Lap u - k^2 u = 0 (Sec. 6.1)."""
    from scipy.special import iv, ivp
    c = np.asarray(center, dtype=np.float64)
    i2r = iv(2, k * radius)

    def u(p):
        d = p - c
        r = np.hypot(d[:, 0], d[:, 1])
        th = np.arctan2(d[:, 1], d[:, 0])
        return iv(2, k * r) * np.sin(2 * th) / i2r

    def grad(p):
        d = p - c
        r = np.maximum(np.hypot(d[:, 0], d[:, 1]), 1e-300)
        th = np.arctan2(d[:, 1], d[:, 0])
        ur = k * ivp(2, k * r) * np.sin(2 * th) / i2r
        ut = iv(2, k * r) * 2 * np.cos(2 * th) / i2r / r
        return np.stack([ur * np.cos(th) - ut * np.sin(th),
                         ur * np.sin(th) + ut * np.cos(th)], axis=1)

    return Solution(u, grad, lambda p: k * k * u(p))


def sol_random_fourier(dim: int, seed: int, kmax: int = 4, length: float = 1.0) -> Solution:
    """u = sum_{m in [-kmax,kmax]^dim} a_m cos(2 pi m.x/L) + b_m sin(2 pi m.x/L), a,b ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    rng_m = np.arange(-kmax, kmax + 1)
    ms = np.stack(np.meshgrid(*([rng_m] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    a = rng.standard_normal(ms.shape[0])
    b = rng.standard_normal(ms.shape[0])
    kv = 2 * np.pi * ms / length          # (K, dim)
    k2 = np.sum(kv * kv, axis=1)

    def u(p):
        ph = p @ kv.T
        return np.cos(ph) @ a + np.sin(ph) @ b

    def grad(p):
        ph = p @ kv.T
        coef = -np.sin(ph) * a + np.cos(ph) * b       # (P, K)
        return coef @ kv

    def lap(p):
        ph = p @ kv.T
        return -(np.cos(ph) @ (a * k2) + np.sin(ph) @ (b * k2))

    return Solution(u, grad, lap)


def random_fourier_grid_2d(seed: int, grid: "Grid", kmax: int = 4):
    """u and Lap u of sol_random_fourier(2, seed, kmax, grid.length) at the grid
    nodes, by separable evaluation: u[iy, ix] = Re sum_ab C_ab e^{i kx_a x} e^{i ky_b y}
    with C = a - i b (same draws as sol_random_fourier)."""
    rng = np.random.default_rng(seed)
    K = 2 * kmax + 1
    a = rng.standard_normal(K * K).reshape(K, K)
    b = rng.standard_normal(K * K).reshape(K, K)
    kk = 2 * np.pi * np.arange(-kmax, kmax + 1) / grid.length
    C = a - 1j * b
    Ex = np.exp(1j * np.outer(grid.axis_coords(0), kk))     # (n, K): [ix, mx]
    Ey = np.exp(1j * np.outer(grid.axis_coords(1), kk))     # (n, K): [iy, my]
    k2 = kk[:, None] ** 2 + kk[None, :] ** 2
    u = np.real(Ey @ C.T @ Ex.T)
    lap = np.real(Ey @ (-(k2 * C)).T @ Ex.T)
    return u, lap


# ----------------------------------------------------------------------------
# problems
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    grid: Grid
    geom: Geometry
    alpha: float
    bc: int
    data: np.ndarray            # U_b (Dirichlet) or V_b (Neumann), (M,)
    g_tilde: np.ndarray         # forcing inside Omega, g_e = 0 outside; grid shaped
    sol: Optional[Solution] = None
    name: str = ""
    extra: dict = field(default_factory=dict)

    def exact_grid(self) -> np.ndarray:
        pts = np.stack([c.ravel() for c in self.grid.nodes()], axis=1)
        return self.sol.u(pts).reshape((self.grid.n,) * self.grid.dim)

    def inside_mask(self) -> np.ndarray:
        pts = np.stack([c.ravel() for c in self.grid.nodes()], axis=1)
        return self.geom.inside(pts).reshape((self.grid.n,) * self.grid.dim)


def make_problem(grid: Grid, geom: Geometry, alpha: float, bc: int, sol: Solution,
                 name: str = "", forcing: bool = True) -> Problem:
    """Manufactured data: g = Lap u - alpha u inside Omega (g_e = 0 outside),
    U_b = u(X) for Dirichlet, V_b = grad u . n for Neumann."""
    pts = np.stack([c.ravel() for c in grid.nodes()], axis=1)
    if forcing:
        g = sol.lap(pts) - alpha * sol.u(pts)
        g = np.where(geom.inside(pts), g, 0.0)
    else:
        g = np.zeros(pts.shape[0])
    g = g.reshape((grid.n,) * grid.dim)
    if bc == DIRICHLET:
        data = sol.u(geom.X)
    else:
        data = np.sum(sol.grad(geom.X) * geom.normal, axis=1)
    return Problem(grid, geom, alpha, bc, np.ascontiguousarray(data), np.ascontiguousarray(g),
                   sol, name)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------
def config_circle64(delta: str = "cosine") -> Problem:
    """2-D Dirichlet, FP64: unit periodic square, 64^2 grid, circle R=0.25 at
    (0.5,0.5) with 128 equispaced points, alpha=1, u = exp(x) sin(y)."""
    grid = Grid(2, 64, (0.0, 0.0), 1.0)
    geom = circle((0.5, 0.5), 0.25, 128)
    p = make_problem(grid, geom, 1.0, DIRICHLET, sol_exp_sin(), name="circle64")
    p.extra["delta"] = delta
    p.extra["tol"] = 1e-10
    return p


STAR_R0, STAR_AMP, STAR_LOBES = 0.3, 0.05, 5


def star_point_counts(n: int = 1024) -> list:
    """M for the star workload: 4096 and round(L/(c h)) for c in {1, 1.5, 2}."""
    per = star_perimeter(STAR_R0, STAR_AMP, STAR_LOBES)
    h = 1.0 / n
    return [4096] + [int(round(per / (c * h))) for c in (1.0, 1.5, 2.0)]


def config_star1024(m: int = 4096, alpha: float = 1.0, bc: int = DIRICHLET,
                    n: int = 1024, seed: int = 2203) -> Problem:
    """2-D star r = 0.3 + 0.05 cos(5 theta) at (0.5,0.5) on a periodic unit
    square, random-Fourier manufactured solution (modes |m_i| <= 4, N(0,1))."""
    grid = Grid(2, n, (0.0, 0.0), 1.0)
    geom = _star_geometry(m)
    sol = sol_random_fourier(2, seed)
    # forcing by separable evaluation (same values as make_problem up to rounding)
    key = (m, n)
    if key not in _STAR_INSIDE:
        pts = np.stack([c.ravel() for c in grid.nodes()], axis=1)
        _STAR_INSIDE[key] = geom.inside(pts).reshape(n, n)
    inside = _STAR_INSIDE[key]
    u, lap = random_fourier_grid_2d(seed, grid)
    g = np.where(inside, lap - alpha * u, 0.0)
    data = sol.u(geom.X) if bc == DIRICHLET else np.sum(sol.grad(geom.X) * geom.normal, axis=1)
    return Problem(grid, geom, alpha, bc, np.ascontiguousarray(data), np.ascontiguousarray(g), sol,
                   f"star{n}_m{m}")


_STAR_CACHE: dict = {}
_STAR_INSIDE: dict = {}


def _star_geometry(m: int) -> Geometry:
    """The star's points (cached: every right-hand side of a workload shares them)."""
    if m not in _STAR_CACHE:
        _STAR_CACHE[m] = star((0.5, 0.5), STAR_R0, STAR_AMP, STAR_LOBES, m)
    return _STAR_CACHE[m]


def config_sphere256(n: int = 256, m: int = 40000, alpha: float = 10.0, seed: int = 0) -> Problem:
    """3-D Dirichlet: sphere R=0.3 at the box centre, Fibonacci lattice, alpha = 10,
    manufactured harmonic u = exp(k.x) cos(l.x + phase) (seed 0: exp(x+y)
    cos(sqrt(2) z - 0.3)); forcing g = -alpha u inside the sphere (separable
    evaluation, the same values as make_problem up to rounding)."""
    grid = Grid(3, n, (0.0, 0.0, 0.0), 1.0)
    if m not in _SPHERE_CACHE:
        _SPHERE_CACHE.clear()
        _SPHERE_CACHE[m] = fibonacci_sphere((0.5, 0.5, 0.5), 0.3, m)
    geom = _SPHERE_CACHE[m]
    x = grid.axis_coords(0) - 0.5
    inside = (x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2) < 0.3 ** 2
    u = harmonic3d_grid(seed, grid)
    g = np.where(inside, -alpha * u, 0.0)
    data = sol_harmonic3d(seed).u(geom.X)
    return Problem(grid, geom, alpha, DIRICHLET, np.ascontiguousarray(data), np.ascontiguousarray(g),
                   sol_harmonic3d(seed), f"sphere{n}_m{m}_s{seed}")


_SPHERE_CACHE: dict = {}


def config_batch(count: int = 512, seed: int = 12126, sizes=(128, 192, 256, 384, 512),
                 spacing: float = 0.75):
    """Independent 2-D ellipse instances: N ~ U(sizes), semi-axes ~ U(0.1,0.3),
    rotation ~ U(0,pi), 2..8 right-hand sides, Dirichlet/Neumann 50/50,
    alpha log-uniform in [1,1000].  Returns a list of dicts (lazy data)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        a, b = rng.uniform(0.1, 0.3, size=2)
        rot = rng.uniform(0.0, math.pi)
        nrhs = int(rng.integers(2, 9))
        bc = int(rng.integers(0, 2))
        alpha = float(math.exp(rng.uniform(math.log(1.0), math.log(1000.0))))
        per = ellipse_perimeter(a, b)
        m = max(16, int(round(per / (spacing / n))))
        out.append(dict(n=n, a=float(a), b=float(b), rot=float(rot), nrhs=nrhs, bc=bc,
                        alpha=alpha, m=m, seed=int(rng.integers(0, 2**31 - 1))))
    return out


def batch_instance(spec: dict, fast: bool = True):
    """Materialise one batch instance: (grid, geom, alpha, bc, [Problem per rhs]).
    fast: grid forcing by separable evaluation (same values as make_problem up
    to rounding)."""
    grid = Grid(2, spec["n"], (0.0, 0.0), 1.0)
    geom = ellipse((0.5, 0.5), spec["a"], spec["b"], spec["rot"], spec["m"])
    probs = []
    inside = None
    for r in range(spec["nrhs"]):
        sol = sol_random_fourier(2, spec["seed"] + r)
        if not fast:
            probs.append(make_problem(grid, geom, spec["alpha"], spec["bc"], sol))
            continue
        if inside is None:
            pts = np.stack([c.ravel() for c in grid.nodes()], axis=1)
            inside = geom.inside(pts).reshape(grid.n, grid.n)
        u, lap = random_fourier_grid_2d(spec["seed"] + r, grid)
        g = np.where(inside, lap - spec["alpha"] * u, 0.0)
        if spec["bc"] == DIRICHLET:
            data = sol.u(geom.X)
        else:
            data = np.sum(sol.grad(geom.X) * geom.normal, axis=1)
        probs.append(Problem(grid, geom, spec["alpha"], spec["bc"], np.ascontiguousarray(data),
                             np.ascontiguousarray(g), sol, f"batch_n{grid.n}"))
    return grid, geom, probs


SERVE_SIZES_2D = (256, 384, 512, 768, 1024, 1536, 2048)
SERVE_SIZES_3D = (64, 96, 128, 192, 256)


def config_serve(count: int = 2000, seed: int = 355, sizes2=SERVE_SIZES_2D, sizes3=SERVE_SIZES_3D,
                 frac3d: float = 0.2):
    """A stream of solve requests: 80% 2-D (circle or star 50/50, Dirichlet or
    Neumann 50/50, M = clip(round(L / (c h)), 1000, 16000) with c ~ U(0.5, 2)),
    20% 3-D (sphere or ellipsoid, Dirichlet, M = clip(round(A / (c h)^2), 5000,
    40000)); alpha log-uniform in [1, 1000]; unit-rate exponential gaps between
    arrivals (scale by 1/QPS).  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(1.0))
        alpha = float(math.exp(rng.uniform(0.0, math.log(1000.0))))
        c = float(rng.uniform(0.5, 2.0))
        sd = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() >= frac3d:
            n = int(rng.choice(sizes2))
            shape = "circle" if rng.uniform() < 0.5 else "star"
            bc = int(rng.integers(0, 2))
            radius = float(rng.uniform(0.15, 0.35))
            per = 2 * math.pi * radius if shape == "circle" else star_perimeter(STAR_R0, STAR_AMP, STAR_LOBES)
            m = int(min(max(round(per / (c / n)), 1000), 16000))
            out.append(dict(dim=2, n=n, shape=shape, radius=radius, bc=bc, alpha=alpha, m=m, c=c,
                            seed=sd, arrival=t))
        else:
            n = int(rng.choice(sizes3))
            shape = "sphere" if rng.uniform() < 0.5 else "ellipsoid"
            axes = tuple(float(v) for v in rng.uniform(0.2, 0.35, size=3))
            if shape == "sphere":
                axes = (axes[0],) * 3
            area = ellipsoid_area(axes)
            m = int(min(max(round(area / (c / n) ** 2), 5000), 40000))
            out.append(dict(dim=3, n=n, shape=shape, axes=axes, bc=DIRICHLET, alpha=alpha, m=m, c=c,
                            seed=sd, arrival=t))
    return out


def ellipsoid_area(axes) -> float:
    """Surface area of an ellipsoid (Knud Thomsen's formula, p = 1.6075; exact for spheres)."""
    a, b, c = axes
    p = 1.6075
    return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1.0 / p)


def serve_instance(spec: dict) -> Problem:
    """Materialise one request of config_serve: 2-D data from sol_random_fourier
    (separable grid evaluation), 3-D data from exp(x+y) cos(sqrt2 z - 0.3)."""
    n, dim = spec["n"], spec["dim"]
    grid = Grid(dim, n, (0.0,) * dim, 1.0)
    alpha = spec["alpha"]
    if dim == 2:
        if spec["shape"] == "circle":
            geom = circle((0.5, 0.5), spec["radius"], spec["m"])
        else:
            geom = star((0.5, 0.5), STAR_R0, STAR_AMP, STAR_LOBES, spec["m"])
        sol = sol_random_fourier(2, spec["seed"])
        pts = np.stack([c.ravel() for c in grid.nodes()], axis=1)
        inside = geom.inside(pts).reshape(n, n)
        u, lap = random_fourier_grid_2d(spec["seed"], grid)
        g = np.where(inside, lap - alpha * u, 0.0)
    else:
        if spec["shape"] == "sphere":
            geom = fibonacci_sphere((0.5, 0.5, 0.5), spec["axes"][0], spec["m"])
        else:
            geom = fibonacci_ellipsoid((0.5, 0.5, 0.5), spec["axes"], spec["m"])
        sol = sol_exp_cos3d()
        x = grid.axis_coords(0)
        # u = e^x e^y cos(sqrt2 z - 0.3) is harmonic: g = -alpha u inside
        u = (np.cos(math.sqrt(2.0) * x - 0.3)[:, None, None] * np.exp(x)[None, :, None] *
             np.exp(x)[None, None, :])
        a, b, c = spec["axes"]
        dz = (x - 0.5)[:, None, None] / c
        dy = (x - 0.5)[None, :, None] / b
        dx = (x - 0.5)[None, None, :] / a
        inside = dx * dx + dy * dy + dz * dz < 1.0
        g = np.where(inside, -alpha * u, 0.0)
    if spec["bc"] == DIRICHLET:
        data = sol.u(geom.X)
    else:
        data = np.sum(sol.grad(geom.X) * geom.normal, axis=1)
    return Problem(grid, geom, alpha, spec["bc"], np.ascontiguousarray(data), np.ascontiguousarray(g), sol,
                   f"serve{dim}d_n{n}")


def table1_problem(n: int, c: float, k: float = 1.0) -> Problem:
    """Sec. 6.1: Lap u - u = 0 in the disc R=0.25 at the origin, U_b = sin(2 theta),
    periodic box [-1/2,1/2]^2, points equispaced with Delta s ~ c Delta x."""
    grid = Grid(2, n, (-0.5, -0.5), 1.0)
    m = int(round(2 * math.pi * 0.25 / (c / n)))
    geom = circle((0.0, 0.0), 0.25, m)
    sol = sol_bessel_sin2((0.0, 0.0), 0.25, k)
    return make_problem(grid, geom, k * k, DIRICHLET, sol, name=f"table1_n{n}_c{c}",
                        forcing=False)


def neumann_circle_problem(n: int, c: float = 0.75) -> Problem:
    """Sec. 6.6: Lap u - u = -(x^2 - y^2) in the disc R=0.25, du/dn = 8(x^2-y^2)."""
    grid = Grid(2, n, (-0.5, -0.5), 1.0)
    m = int(round(2 * math.pi * 0.25 / (c / n)))
    geom = circle((0.0, 0.0), 0.25, m)
    return make_problem(grid, geom, 1.0, NEUMANN, sol_x2_minus_y2(), name=f"neumann_n{n}")


def table2_problem(n: int, m: int) -> Problem:
    """Sec. 6.7 geometry: sphere R=0.25 at the origin in [-1/2,1/2]^3, alpha=1.
    Data from the harmonic u = exp(x+y) cos(sqrt(2) z - 0.3)."""
    grid = Grid(3, n, (-0.5, -0.5, -0.5), 1.0)
    geom = fibonacci_sphere((0.0, 0.0, 0.0), 0.25, m)
    return make_problem(grid, geom, 1.0, DIRICHLET, sol_exp_cos3d(), name=f"table2_n{n}_m{m}")


def _balance_forcing(p: "Problem") -> "Problem":
    """g_e = -(sum of g over the domain's nodes) / (number of other nodes): the
    discrete form of the solvability choice g_e = -int_Omega g / |C \\ Omega| for
    the periodic Laplacian (App. C), so that the grid sum of g~ vanishes."""
    inside = p.inside_mask()
    ge = -float(np.sum(p.g_tilde[inside])) / float(np.count_nonzero(~inside))
    p.g_tilde = np.ascontiguousarray(np.where(inside, p.g_tilde, ge))
    return p


def sol_exp_sin2pix() -> Solution:
    """u = exp(sin(2 pi x)), Lap u = 4 pi^2 exp(sin 2 pi x) (cos^2 2 pi x - sin 2 pi x) (Sec. 6.3)."""
    tp = 2 * math.pi

    def u(p):
        return np.exp(np.sin(tp * p[:, 0]))

    def grad(p):
        g = np.zeros_like(p)
        g[:, 0] = tp * np.cos(tp * p[:, 0]) * u(p)
        return g

    def lap(p):
        x = p[:, 0]
        return tp * tp * np.exp(np.sin(tp * x)) * (np.cos(tp * x) ** 2 - np.sin(tp * x))

    return Solution(u, grad, lap)


def poisson_exterior_problem(n: int, length: float, c: float = 0.75, balanced: bool = True) -> Problem:
    """Sec. 6.3: Lap u = g exterior to the circle R = 0.25 at the origin in the
    periodic box [-L/2, L/2]^2, u = exp(sin 2 pi x), alpha = 0, Dirichlet data,
    points with Delta s ~ c Delta x.  balanced: g inside the circle set so the
    grid sum of g~ vanishes (App. C, the original formulation); else g_e = 0 (the
    completed formulation needs no condition on g_e)."""
    grid = Grid(2, n, (-length / 2, -length / 2), length)
    m = int(round(2 * math.pi * 0.25 / (c * length / n)))
    geom = circle((0.0, 0.0), 0.25, m, interior=False)
    p = make_problem(grid, geom, 0.0, DIRICHLET, sol_exp_sin2pix(), name=f"poisson_ext_n{n}_L{length:g}")
    return _balance_forcing(p) if balanced else p


def starfish_problem(n: int, c: float = 0.75) -> Problem:
    """Sec. 6.4: Lap u = g exterior to the starfish r = 1 + sin(10 pi theta)/4 in the
    periodic box [-2, 2]^2, u = sin(pi x/2) - cos(pi y/2), alpha = 0, Dirichlet,
    points with Delta s ~ c Delta x, forcing balanced for solvability (App. C)."""
    grid = Grid(2, n, (-2.0, -2.0), 4.0)
    per = star_perimeter(1.0, 0.25, 5)
    m = int(round(per / (c * 4.0 / n)))
    geom = star((0.0, 0.0), 1.0, 0.25, 5, m, interior=False, phase=-math.pi / 2)
    hp = math.pi / 2
    sol = Solution(lambda p: np.sin(hp * p[:, 0]) - np.cos(hp * p[:, 1]),
                   lambda p: np.stack([hp * np.cos(hp * p[:, 0]), hp * np.sin(hp * p[:, 1])], axis=1),
                   lambda p: hp * hp * (np.cos(hp * p[:, 1]) - np.sin(hp * p[:, 0])))
    return _balance_forcing(make_problem(grid, geom, 0.0, DIRICHLET, sol, name=f"starfish_n{n}"))


def random_density(m: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """A seeded boundary density (nrhs, M) ~ N(0,1)."""
    return np.random.default_rng(seed).standard_normal((nrhs, m))
