"""Plain FP64 CPU oracle of the IBDL hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  The product path (the HIP library and its
binding) never imports, links or calls it, and it shares no code with it: the
only common module is the seeded input generator, which holds none of the
method's arithmetic.

Everything is written to be checked by eye against the paper (Leathers & Guy,
"Immersed Boundary Double Layer method: an introduction of methodology on the
Helmholtz equation"):

* the Peskin four-point kernel phi and delta_h             (Sec. 5.2, delta_h as a product of phi)
* the spread S and interpolation S*                        (Sec. 5.2, their discrete sums)
* the dipole spread  S~Q = div(S Q n), centred divergence  (Sec. 5.2; Sec. 4.1, the IBDL system)
* L = Lap_h - alpha with the 5-/7-point Laplacian on a periodic box,
  inverted by diagonalisation with the DFT                 (Sec. 5.1; Sec. 5.3)
* the Dirichlet operator  -S* L^-1 S~ + 1/2 I  and RHS     (Sec. 5.3, the equation for Q)
* the Neumann operator    -S* L^-1 S~ - 1/2 I  and RHS     (Sec. 4.4, the equation for U_b)
* the grid solution  L u = g~ - S~Q  (- S V_b for Neumann) (Sec. 4.2 step 2; Sec. 4.4, the Neumann grid equation)
* unpreconditioned GMRES on the boundary density           (Sec. 5.3)
* the mean-zero inverse for alpha = 0                      (Sec. 5.4.2; App. C)
* the completed IBDL system for the Poisson equation       (Sec. 5.4.1; App. C)
* the IB constraint (single-layer) system and MINRES, the
  comparison method of the paper's tables                  (Sec. 2.1; Table 1, Table 2)
* the Fourier-spectral Laplacian as an alternative to the
  finite-difference one                                    (Sec. 5.1; Sec. 6.2.1)
* the indicator-function construction and the flags of the
  PDE domain                                               (App. D)
* the near-boundary re-interpolation of the grid solution  (Sec. 5.5; App. A)
* the discrete L1/L2 norms rescaled by |Omega|             (Sec. 5.1)

Library primitives used as single steps: numpy's FFT (the DFT that diagonalises
the periodic Laplacian) and numpy/scipy dense linear algebra in tests.

Readings taken where the paper is silent (also listed in the design notes):
node-centred grid with node i at lo + i h; the stencil wraps periodically;
cell index c = floor((X - lo)/h) mod n computed in IEEE FP64; alpha = k^2;
for alpha = 0 the zero Fourier mode of the solution is set to 0 (mean-zero
inverse); GMRES starts from x0 = 0 and stops on the relative residual
||b - A x|| / ||b|| <= tol, counting one iteration per operator application.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DIRICHLET = 0
NEUMANN = 1
PESKIN4 = "peskin4"
COSINE4 = "cosine"
LAP_FD = "fd"              # the 5-point (2-D) / 7-point (3-D) Laplacian (Sec. 5.1)
LAP_SPECTRAL = "spectral"  # the Fourier-spectral Laplacian (Sec. 6.2.1)


# ----------------------------------------------------------------------------
# the discrete delta (Sec. 5.2)
# ----------------------------------------------------------------------------
def phi_peskin4(r):
    """Peskin's four-point kernel phi(r) (Sec. 5.2)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    a1 = a[m1]
    a2 = a[m2]
    out[m1] = (3.0 - 2.0 * a1 + np.sqrt(1.0 + 4.0 * a1 - 4.0 * a1 * a1)) / 8.0
    out[m2] = (5.0 - 2.0 * a2 - np.sqrt(np.maximum(0.0, -7.0 + 12.0 * a2 - 4.0 * a2 * a2))) / 8.0
    return out


def phi_cosine4(r):
    """The four-point cosine kernel phi(r) = (1 + cos(pi r / 2)) / 4 for |r| < 2."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    return np.where(a < 2.0, 0.25 * (1.0 + np.cos(0.5 * np.pi * a)), 0.0)


def phi(r, kind=PESKIN4):
    return phi_peskin4(r) if kind == PESKIN4 else phi_cosine4(r)


# ----------------------------------------------------------------------------
# grid and boundary description
# ----------------------------------------------------------------------------
@dataclass
class Setup:
    dim: int
    n: int
    lo: np.ndarray        # (dim,)
    length: float
    alpha: float
    X: np.ndarray         # (M, dim)
    normal: np.ndarray    # (M, dim), pointing out of Omega
    weight: np.ndarray    # (M,) Delta s_i or dA_i
    delta: str = PESKIN4
    lap: str = LAP_FD     # discretisation of the Laplacian in L = Lap_h - alpha

    @property
    def h(self):
        return self.length / self.n

    @property
    def m(self):
        return self.X.shape[0]

    @property
    def shape(self):
        return (self.n,) * self.dim


def setup_from_problem(prob, delta=PESKIN4, lap=LAP_FD) -> Setup:
    g = prob.grid
    return Setup(g.dim, g.n, np.asarray(g.lo, dtype=np.float64), float(g.length), float(prob.alpha),
                 np.asarray(prob.geom.X, dtype=np.float64), np.asarray(prob.geom.normal, dtype=np.float64),
                 np.asarray(prob.geom.weight, dtype=np.float64), delta, lap)


def _axis(st: Setup, d: int) -> int:
    """Array axis of coordinate direction d (x is the last axis)."""
    return st.dim - 1 - d


def cell_and_offsets(st: Setup):
    """Per point and direction: the unwrapped floor index and t - floor(t), t = (X - lo)/h."""
    t = (st.X - st.lo[None, :]) / st.h
    fl = np.floor(t)
    return fl.astype(np.int64), t - fl


def stencil(st: Setup):
    """The 4^d nodes of each point's delta stencil and their weights Prod_d phi(p_d - t_d).

    Returns (flat node index (M, 4^d), weight (M, 4^d)); nodes wrap periodically.
    phi vanishes for |p - t| >= 2, so the nodes floor(t)-1 .. floor(t)+2 carry all of it.
    """
    fl, fr = cell_and_offsets(st)
    m, d = st.m, st.dim
    idx = np.zeros((m, 4 ** d), dtype=np.int64)
    wts = np.ones((m, 4 ** d))
    for combo in range(4 ** d):
        flat = np.zeros(m, dtype=np.int64)
        w = np.ones(m)
        stride = 1
        for dd in range(d):
            i = (combo // (4 ** dd)) % 4          # offset -1..2 along direction dd
            p = fl[:, dd] - 1 + i
            w = w * phi(p - (fl[:, dd] + fr[:, dd]), st.delta)
            flat = flat + np.mod(p, st.n) * stride
            stride *= st.n
        idx[:, combo] = flat
        wts[:, combo] = w
    return idx, wts


# ----------------------------------------------------------------------------
# spread and interpolation (Sec. 5.2)
# ----------------------------------------------------------------------------
def spread(st: Setup, F):
    """(S F)(x) = sum_k F_k delta_h(x - X_k) Delta s_k  (Sec. 5.2, the discrete spread)."""
    idx, wts = stencil(st)
    vals = (np.asarray(F, dtype=np.float64) * st.weight)[:, None] * wts / st.h ** st.dim
    out = np.bincount(idx.ravel(), weights=vals.ravel(), minlength=st.n ** st.dim)
    return out.reshape(st.shape)


def interp(st: Setup, u):
    """(S* u)_k = sum_x u(x) delta_h(x - X_k) h^d  (Sec. 5.2, the discrete interpolation)."""
    idx, wts = stencil(st)
    return np.sum(np.asarray(u, dtype=np.float64).ravel()[idx] * wts, axis=1)


def divergence(st: Setup, v):
    """Centred second-order divergence of a vector grid field v[d] (Sec. 5.2)."""
    out = np.zeros(st.shape)
    for d in range(st.dim):
        ax = _axis(st, d)
        out += (np.roll(v[d], -1, axis=ax) - np.roll(v[d], 1, axis=ax)) / (2.0 * st.h)
    return out


def gradient(st: Setup, u):
    """Centred second-order gradient (the adjoint partner of ``divergence``)."""
    return [(np.roll(u, -1, axis=_axis(st, d)) - np.roll(u, 1, axis=_axis(st, d))) / (2.0 * st.h)
            for d in range(st.dim)]


def spread_dipole(st: Setup, Q):
    """S~ Q = div(S (Q n))  (Sec. 5.2): spread the vector Q n, then the centred divergence."""
    Q = np.asarray(Q, dtype=np.float64)
    v = [spread(st, Q * st.normal[:, d]) for d in range(st.dim)]
    return divergence(st, v)


# ----------------------------------------------------------------------------
# L = Lap_h - alpha on the periodic box (Sec. 5.1, Sec. 5.3, App. C)
# ----------------------------------------------------------------------------
def symbol(st: Setup):
    """Eigenvalues of the periodic Laplacian minus alpha on the DFT modes m:
    5-point (2-D) / 7-point (3-D) stencil, -(4/h^2) sin^2(pi m_d/n) per axis
    (Sec. 5.1); Fourier-spectral, -(2 pi k_d/L)^2 per axis with k_d the signed
    frequency of m_d (Sec. 6.2.1)."""
    lam = np.zeros(st.shape)
    for d in range(st.dim):
        m = np.arange(st.n)
        if st.lap == LAP_SPECTRAL:
            k = np.where(m <= st.n // 2, m, m - st.n)
            ev = -(2.0 * np.pi * k / st.length) ** 2
        else:
            ev = -(4.0 / st.h ** 2) * np.sin(np.pi * m / st.n) ** 2
        sh = [1] * st.dim
        sh[_axis(st, d)] = st.n
        lam = lam + ev.reshape(sh)
    return lam - st.alpha


def apply_L(st: Setup, u):
    """L u with the explicit stencil (used to check the inverse; finite differences only)."""
    assert st.lap == LAP_FD
    out = -st.alpha * u
    for d in range(st.dim):
        ax = _axis(st, d)
        out = out + (np.roll(u, -1, axis=ax) - 2.0 * u + np.roll(u, 1, axis=ax)) / st.h ** 2
    return out


def solve_L(st: Setup, f):
    """u = L^-1 f by the DFT; for alpha = 0 the mean-zero solution (Delta_0^-1, App. C)."""
    fh = np.fft.fftn(np.asarray(f, dtype=np.float64))
    lam = symbol(st)
    if st.alpha == 0.0:
        lam = lam.copy()
        lam.flat[0] = 1.0
        uh = fh / lam
        uh.flat[0] = 0.0
    else:
        uh = fh / lam
    return np.real(np.fft.ifftn(uh))


# ----------------------------------------------------------------------------
# the IBDL boundary operator and its right-hand sides
# ----------------------------------------------------------------------------
def apply_A(st: Setup, q, bc=DIRICHLET):
    """Dirichlet: -S* L^-1 S~ q + q/2 (Sec. 5.3, the equation for Q);
    Neumann:   -S* L^-1 S~ q - q/2 (Sec. 4.4, the equation for U_b)."""
    q = np.asarray(q, dtype=np.float64)
    w = -interp(st, solve_L(st, spread_dipole(st, q)))
    return w + 0.5 * q if bc == DIRICHLET else w - 0.5 * q


def rhs(st: Setup, data, g_tilde=None, bc=DIRICHLET):
    """Dirichlet: U_b - S* L^-1 g~;  Neumann: S* L^-1 S V_b - S* L^-1 g~."""
    data = np.asarray(data, dtype=np.float64)
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    if bc == DIRICHLET:
        return data - interp(st, solve_L(st, g))
    return interp(st, solve_L(st, spread(st, data))) - interp(st, solve_L(st, g))


def eval_grid(st: Setup, sol, vb=None, g_tilde=None, bc=DIRICHLET):
    """Grid solution: L u = g~ - S~ Q (Dirichlet, step 2 of Sec. 4.2), or
    L u = g~ - S~ U_b - S V_b (Neumann, the grid equation of Sec. 4.4)."""
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    f = g - spread_dipole(st, sol)
    if bc == NEUMANN:
        f = f - spread(st, vb)
    return solve_L(st, f)


# ----------------------------------------------------------------------------
# the completed IBDL system for the Poisson equation (Sec. 5.4.1; App. C)
# ----------------------------------------------------------------------------
def apply_completed(st: Setup, z, eta):
    """App. C on z = [Q; ubar] (alpha = 0, Delta_0^-1 the mean-zero inverse):
    rows 1..M:  -S* Delta_0^-1 S~ Q - eta S* Delta_0^-1 S Q + ubar + Q/2,
    row M+1:    eta sum_k Delta s_k Q_k  (the solvability condition; Delta s_k the
    point weights, the paper's uniform Delta s)."""
    assert st.alpha == 0.0
    z = np.asarray(z, dtype=np.float64)
    Q, ubar = z[:-1], z[-1]
    top = -interp(st, solve_L(st, spread_dipole(st, Q))) - eta * interp(st, solve_L(st, spread(st, Q)))
    top = top + ubar + 0.5 * Q
    return np.append(top, eta * np.sum(st.weight * Q))


def rhs_completed(st: Setup, data, g_tilde=None):
    """App. C right-hand side: [U_b - S* Delta_0^-1 g~;  h^d sum_x g~(x)]."""
    assert st.alpha == 0.0
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    return np.append(np.asarray(data, dtype=np.float64) - interp(st, solve_L(st, g)), st.h ** st.dim * np.sum(g))


def eval_grid_completed(st: Setup, z, g_tilde=None, eta=0.0):
    """App. C: u = -Delta_0^-1 (S~ + eta S) Q + Delta_0^-1 g~ + ubar."""
    z = np.asarray(z, dtype=np.float64)
    Q, ubar = z[:-1], z[-1]
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    return solve_L(st, g - spread_dipole(st, Q) - eta * spread(st, Q)) + ubar


def solve_completed(st: Setup, data, g_tilde=None, eta=10.0, tol=1e-8, restart=50, maxit=500):
    """GMRES on the completed system for [Q; ubar] (App. C)."""
    b = rhs_completed(st, data, g_tilde)
    return gmres(lambda v: apply_completed(st, v, eta), b, tol=tol, restart=restart, maxit=maxit), b


# ----------------------------------------------------------------------------
# the IB constraint (single-layer) system compared with the IBDL method (Sec. 2.1)
# ----------------------------------------------------------------------------
def apply_ibsl(st: Setup, F):
    """-(S* L^-1 S) F: the Schur complement of the IB constraint system (Sec. 2.1)."""
    return -interp(st, solve_L(st, spread(st, np.asarray(F, dtype=np.float64))))


def rhs_ibsl(st: Setup, data, g_tilde=None):
    """U_b - S* L^-1 g~ (Sec. 2.1)."""
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    return np.asarray(data, dtype=np.float64) - interp(st, solve_L(st, g))


def eval_grid_ibsl(st: Setup, F, g_tilde=None):
    """u = L^-1 (g~ - S F) (Sec. 2.1, the first row of the constraint system)."""
    g = np.zeros(st.shape) if g_tilde is None else np.asarray(g_tilde, dtype=np.float64)
    return solve_L(st, g - spread(st, F))


@dataclass
class MinresResult:
    x: np.ndarray
    iters: int
    rel_resid: float
    converged: bool


def minres(apply, b, weight, tol=1e-8, maxit=20000):
    """MINRES (Paige and Saunders) for an operator self-adjoint in the inner product
    <x, y>_W = sum_k w_k x_k y_k (the IBSL operator -S* L^-1 S is, since S spreads
    with the weights w); with equal weights it is the plain MINRES the paper runs.
    x0 = 0; stops when the W-norm residual estimate falls to tol ||b||_W; one
    iteration per operator application."""
    b = np.asarray(b, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    dot = lambda a, c: float(np.sum(w * a * c))
    x = np.zeros_like(b)
    beta1 = math.sqrt(dot(b, b))
    if beta1 == 0.0:
        return MinresResult(x, 0, 0.0, True)
    r1 = b.copy()
    r2 = b.copy()
    beta, oldb = beta1, 0.0
    dbar = epsln = 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    wv = np.zeros_like(b)
    w2 = np.zeros_like(b)
    itn = 0
    while itn < maxit:
        itn += 1
        v = r2 / beta
        y = apply(v)
        if itn >= 2:
            y = y - (beta / oldb) * r1
        alfa = dot(v, y)
        y = y - (alfa / beta) * r2
        r1, r2 = r2, y
        oldb, beta = beta, math.sqrt(dot(r2, r2))
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = math.hypot(gbar, beta)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, wv
        wv = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * wv
        if phibar / beta1 <= tol or beta == 0.0:
            return MinresResult(x, itn, phibar / beta1, True)
    return MinresResult(x, itn, phibar / beta1, False)


def solve_ibsl(st: Setup, data, g_tilde=None, tol=1e-8, maxit=20000):
    """The IBSL comparison: MINRES on -(S* L^-1 S) F = U_b - S* L^-1 g~ (Sec. 2.1, Table 1)."""
    b = rhs_ibsl(st, data, g_tilde)
    return minres(lambda v: apply_ibsl(st, v), b, st.weight, tol=tol, maxit=maxit), b


# ----------------------------------------------------------------------------
# GMRES (Sec. 5.3): Arnoldi with modified Gram-Schmidt, Givens rotations
# ----------------------------------------------------------------------------
@dataclass
class GmresResult:
    x: np.ndarray
    iters: int            # number of operator applications
    rel_resid: float      # the Arnoldi residual estimate / ||b||
    converged: bool
    history: list


def gmres(apply, b, tol=1e-8, restart=50, maxit=500, x0=None):
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    if nb == 0.0:
        return GmresResult(np.zeros_like(b), 0, 0.0, True, hist)
    iters = 0
    first = True
    while True:
        # residual of the current iterate (no operator application for x0 = 0);
        # only Arnoldi steps count as iterations
        r = b.copy() if (first and x0 is None) else b - apply(x)
        first = False
        beta = float(np.linalg.norm(r))
        if beta / nb <= tol:
            return GmresResult(x, iters, beta / nb, True, hist)
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        conv = False
        for j in range(m):
            w = apply(V[j])
            iters += 1
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            res = abs(g[j + 1]) / nb
            hist.append(res)
            j_done = j + 1
            if res <= tol or iters >= maxit:
                conv = res <= tol
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:j_done], y[i + 1:j_done])) / H[i, i]
        x = x + V[:j_done].T @ y
        if conv or iters >= maxit:
            return GmresResult(x, iters, hist[-1], conv, hist)


def solve(st: Setup, data, g_tilde=None, bc=DIRICHLET, tol=1e-8, restart=50, maxit=500):
    """Step 1 of the method: the boundary density Q (Dirichlet) or U_b (Neumann)."""
    b = rhs(st, data, g_tilde, bc)
    return gmres(lambda v: apply_A(st, v, bc), b, tol=tol, restart=restart, maxit=maxit), b


# ----------------------------------------------------------------------------
# cell binning (the ordering the GPU path builds): key and stable order
# ----------------------------------------------------------------------------
def cell_keys(st: Setup):
    """Row-major cell index of floor((X - lo)/h) mod n, x fastest."""
    fl, _ = cell_and_offsets(st)
    key = np.zeros(st.m, dtype=np.int64)
    stride = 1
    for d in range(st.dim):
        key += np.mod(fl[:, d], st.n) * stride
        stride *= st.n
    return key.astype(np.uint32)


def binning(st: Setup):
    """Keys and the stable sort permutation (equal keys keep the input order)."""
    key = cell_keys(st)
    perm = sorted(range(st.m), key=lambda k: int(key[k]))
    return key, np.asarray(perm, dtype=np.uint32)


# ----------------------------------------------------------------------------
# indicator function (App. D) and error norms (Sec. 5.1)
# ----------------------------------------------------------------------------
def indicator(st: Setup, corner_index=0):
    """chi_h = -Delta_0^-1 S~ 1 shifted so the chosen corner node is 0; and its 1/2 threshold."""
    st0 = Setup(st.dim, st.n, st.lo, st.length, 0.0, st.X, st.normal, st.weight, st.delta, st.lap)
    u = -solve_L(st0, spread_dipole(st0, np.ones(st.m)))
    chi_h = u - u.flat[corner_index]
    return chi_h, (chi_h > 0.5).astype(np.int8)


def orientation(st: Setup):
    """+1 when the normals point away from the region the boundary encloses (the PDE
    domain is that region), -1 when they point into it (the PDE domain is the rest of
    the box): the sign of sum_k w_k (X_k - X_0) . n_k, the discrete form of the
    divergence theorem's  int_Gamma x . n ds = d |enclosed region|  for outward n."""
    v = float(np.sum(st.weight * np.sum((st.X - st.X[0]) * st.normal, axis=1)))
    return 1 if v > 0.0 else -1


def omega_flags(st: Setup):
    """App. D with the corner as the far-field reference: chi_h is ~1 inside the
    enclosed region for outward normals, so the PDE domain is chi_h > 1/2; with
    normals pointing into the enclosed region chi_h is ~-1 there and 0 in the
    domain, which is then chi_h > -1/2.  Returns (chi_h, flags of the domain)."""
    chi_h, _ = indicator(st)
    thr = 0.5 if orientation(st) > 0 else -0.5
    return chi_h, (chi_h > thr).astype(np.int8)


def _min_image(st: Setup, v):
    """Periodic minimum-image form of displacement vectors."""
    L = st.length
    return v - L * np.round(v / L)


def near_boundary_fixup(st: Setup, u, ub, in_omega, m1=6.0, m2=8.0):
    """App. A: every node of the PDE domain whose nearest boundary point lies within
    m1 meshwidths gets u(x_p) = u(x_A) |x_B - x_p|/|x_B - x_A| + u(x_B) |x_A - x_p|/|x_B - x_A|.

    2-D: x_A is the point of the segment between the two nearest boundary points x1,
    x2 closest to x_p (orthogonal projection; when it falls outside the segment the
    third nearest point is taken and the two of the three farthest apart span the
    segment), with u(x_A) interpolated linearly from U_b(x1), U_b(x2).
    3-D: x_A is the nearest boundary point and u(x_A) its U_b.
    x_B = x_A + (x_p - x_A)/|x_p - x_A| m2 h, with u(x_B) the bi-/trilinear
    interpolation of the grid solution.  Values are read from u before any
    replacement.  Returns the new grid and the mask of replaced nodes."""
    from scipy.spatial import cKDTree
    u = np.asarray(u, dtype=np.float64)
    ub = np.asarray(ub, dtype=np.float64)
    h, L, d = st.h, st.length, st.dim
    out = u.copy()
    done = np.zeros(st.shape, dtype=bool)
    tree = cKDTree(np.mod(st.X - st.lo, L), boxsize=L)
    nodes = np.stack([c.ravel() for c in _grid_nodes(st)], axis=1)
    dist, idx = tree.query(np.mod(nodes - st.lo, L), k=3 if d == 2 else 1)
    d1 = dist[:, 0] if d == 2 else dist
    cand = np.nonzero((np.asarray(in_omega).ravel() != 0) & (d1 <= m1 * h))[0]
    for p in cand:
        xp = nodes[p]
        if d == 2:
            i1, i2, i3 = idx[p]
            x1 = xp + _min_image(st, st.X[i1] - xp)
            x2 = xp + _min_image(st, st.X[i2] - xp)
            e = x1 - x2
            t = float(np.dot(xp - x2, e) / np.dot(e, e))
            if t < 0.0 or t > 1.0:
                x3 = xp + _min_image(st, st.X[i3] - xp)
                pairs = [((i1, x1), (i2, x2)), ((i1, x1), (i3, x3)), ((i2, x2), (i3, x3))]
                (i1, x1), (i2, x2) = max(pairs, key=lambda ab: float(np.sum((ab[0][1] - ab[1][1]) ** 2)))
                e = x1 - x2
                t = min(1.0, max(0.0, float(np.dot(xp - x2, e) / np.dot(e, e))))
            xa = x2 + t * e
            le = math.sqrt(float(np.dot(e, e)))
            ua = (ub[i1] * math.sqrt(float(np.sum((xa - x2) ** 2))) +
                  ub[i2] * math.sqrt(float(np.sum((xa - x1) ** 2)))) / le
        else:
            i1 = idx[p]
            xa = xp + _min_image(st, st.X[i1] - xp)
            ua = ub[i1]
        dp = math.sqrt(float(np.sum((xp - xa) ** 2)))
        if dp == 0.0:
            val = ua
        else:
            xb = xa + (xp - xa) / dp * (m2 * h)
            ubv = _multilinear(st, u, xb)
            dab = math.sqrt(float(np.sum((xb - xa) ** 2)))
            dbp = math.sqrt(float(np.sum((xb - xp) ** 2)))
            val = ua * dbp / dab + ubv * dp / dab
        out.flat[p] = val
        done.flat[p] = True
    return out, done


def _grid_nodes(st: Setup):
    ax = [st.lo[dd] + st.h * np.arange(st.n) for dd in range(st.dim)]
    mesh = np.meshgrid(*ax[::-1], indexing="ij")
    return tuple(mesh[::-1])


def _multilinear(st: Setup, u, x):
    """Bi-/trilinear interpolation of the grid field u at the point x (periodic)."""
    t = (np.asarray(x) - st.lo) / st.h
    fl = np.floor(t)
    fr = t - fl
    val = 0.0
    for corner in range(2 ** st.dim):
        w = 1.0
        ix = []
        for dd in range(st.dim):
            bit = (corner >> dd) & 1
            w *= fr[dd] if bit else 1.0 - fr[dd]
            ix.append(int(fl[dd] + bit) % st.n)
        val += w * u[tuple(ix[::-1])]
    return val


def norms(st: Setup, err, mask, area):
    """Discrete L1, L2 (rescaled by |Omega|) and max norms over the masked nodes."""
    e = np.abs(np.asarray(err))[mask]
    hd = st.h ** st.dim
    return (hd / area * float(np.sum(e)), math.sqrt(hd / area * float(np.sum(e * e))),
            float(np.max(e)) if e.size else 0.0)


def distance_to_points(st: Setup, nodes, X):
    """Distance from grid nodes to the nearest boundary point (periodic minimum image)."""
    from scipy.spatial import cKDTree
    L = st.length
    tree = cKDTree(np.mod(X - st.lo, L), boxsize=L)
    d, _ = tree.query(np.mod(nodes - st.lo, L))
    return d
