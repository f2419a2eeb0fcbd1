"""Closed forms and independent reference solvers that pin the oracle.

TEST INFRASTRUCTURE.  Nothing here calls the oracle or the HIP library.

Lattice units throughout (dx = dt = 1); nu = (tau_f - 1/2)/3 and
eta = D = (tau - 1/2)/4 (Section 2 relations with c_s^2 = 1/3, c^2 = 1/4).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize, sparse
from scipy.sparse import linalg as spla


# ---------------------------------------------------------------------------
# Plane Poiseuille flow, BGK + Guo forcing, walls half-way (d = 0.5)
# ---------------------------------------------------------------------------
def poiseuille_discrete(N: int, tau: float, g: float) -> np.ndarray:
    """Exact steady velocity of the discrete D2Q9 BGK channel with half-way
    bounce-back walls and Guo forcing (derived from the x-odd parts of the
    populations, which obey a linear recurrence across the channel):

        u_j = g/(2 nu) (y_j + 1/2)(N - 1/2 - y_j) + u_s,
        u_s = g/(2 nu) (16 Lambda - 3)/12,  Lambda = (tau - 1/2)^2.

    The parabola is exact (u_s = 0) at Lambda = 3/16.
    """
    nu = (tau - 0.5) / 3.0
    y = np.arange(N, dtype=float)
    lam = (tau - 0.5) ** 2
    return g / (2 * nu) * (y + 0.5) * (N - 0.5 - y) + g / (2 * nu) * (16 * lam - 3) / 12.0


def poiseuille_continuum(y: np.ndarray, y_lo: float, y_hi: float, g: float, nu: float) -> np.ndarray:
    return g / (2 * nu) * (y - y_lo) * (y_hi - y)


def couette(y: np.ndarray, y_lo: float, y_hi: float, u_lo: float, u_hi: float) -> np.ndarray:
    return u_lo + (u_hi - u_lo) * (y - y_lo) / (y_hi - y_lo)


# ---------------------------------------------------------------------------
# Hartmann(-Couette) flow between flat walls at y = -H and y = +H
# ---------------------------------------------------------------------------
def hartmann_couette(y: np.ndarray, H: float, B0: float, nu: float, eta: float, rho: float = 1.0,
                     mu: float = 1.0, U_top: float = 0.0, U_bot: float = 0.0, c_bot: float = 0.0,
                     c_top: float = 0.0, g: float = 0.0):
    """Steady u1(y), B1(y) of the unidirectional MHD channel.

    rho nu u'' + (B0/mu) B1' + rho g = 0,   eta B1'' + B0 u' = 0,
    u(-H) = U_bot, u(H) = U_top; wall conductance ratios c (Shercliff):
    bottom  c_bot H B1' - B1 = 0,  top  c_top H B1' + B1 = 0
    (c = 0: B1 = 0 insulating; c = inf: B1' = 0 perfectly conducting).

    Integrating the induction equation once, eta B1' + B0 u = K, gives
    u = K/B0 + rho g mu eta/B0^2 + a1 cosh(k y) + a2 sinh(k y), k = Ha/H,
    B1 = -(rho g mu/B0) y - (B0/(eta k)) (a1 sinh + a2 cosh) + K2,
    with Ha^2 = B0^2 H^2/(rho nu mu eta); K, a1, a2, K2 from a 4x4 solve.
    """
    k = B0 / math.sqrt(rho * nu * mu * eta)
    up = rho * g * mu * eta / B0 ** 2

    def rows(yy):
        ch, sh = math.cosh(k * yy), math.sinh(k * yy)
        # unknown vector x = (K, a1, a2, K2)
        u_row = np.array([1.0 / B0, ch, sh, 0.0])
        u_c = up
        b_row = np.array([0.0, -(B0 / (eta * k)) * sh, -(B0 / (eta * k)) * ch, 1.0])
        b_c = -(rho * g * mu / B0) * yy
        db_row = np.array([0.0, -(B0 / eta) * ch, -(B0 / eta) * sh, 0.0])
        db_c = -(rho * g * mu / B0)
        return u_row, u_c, b_row, b_c, db_row, db_c

    M = np.zeros((4, 4))
    r = np.zeros(4)
    ub, ubc, bb, bbc, dbb, dbbc = rows(-H)
    ut, utc, bt, btc, dbt, dbtc = rows(H)
    M[0], r[0] = ub, U_bot - ubc
    M[1], r[1] = ut, U_top - utc

    # bottom: c H B1' - B1 = 0; top: c H B1' + B1 = 0
    if c_bot == 0.0:
        M[2], r[2] = bb, -bbc
    elif math.isinf(c_bot):
        M[2], r[2] = dbb, -dbbc
    else:
        M[2], r[2] = c_bot * H * dbb - bb, -(c_bot * H * dbbc - bbc)
    if c_top == 0.0:
        M[3], r[3] = bt, -btc
    elif math.isinf(c_top):
        M[3], r[3] = dbt, -dbtc
    else:
        M[3], r[3] = c_top * H * dbt + bt, -(c_top * H * dbtc + btc)
    x = np.linalg.solve(M, r)
    K, a1, a2, K2 = x
    y = np.asarray(y, float)
    u = K / B0 + up + a1 * np.cosh(k * y) + a2 * np.sinh(k * y)
    B1 = -(rho * g * mu / B0) * y - (B0 / (eta * k)) * (a1 * np.sinh(k * y) + a2 * np.cosh(k * y)) + K2
    return u, B1


def hartmann_channel_fd(y: np.ndarray, H: float, B0: float, nu: float, eta: float,
                        rho: float = 1.0, mu: float = 1.0, U_top: float = 0.0,
                        U_bot: float = 0.0, c_bot: float = 0.0, c_top: float = 0.0,
                        g: float = 0.0, v0: float = 0.0, m: int = 4000):
    """Same channel with uniform transpiration v0 (fluid enters at y = -H and
    leaves at y = +H), solved by second-order finite differences on m cells
    with one Richardson extrapolation (m and 2m):

    rho nu u'' - rho v0 u' + (B0/mu) B1' + rho g = 0
    eta B1'' - v0 B1' + B0 u' = 0.
    """

    def solve(mm):
        hh = 2 * H / mm
        yy = np.linspace(-H, H, mm + 1)
        n = mm + 1
        A = sparse.lil_matrix((2 * n, 2 * n))
        rhs = np.zeros(2 * n)
        for i in range(1, n - 1):
            # u equation
            A[i, i - 1] += rho * nu / hh ** 2 + rho * v0 / (2 * hh)
            A[i, i] += -2 * rho * nu / hh ** 2
            A[i, i + 1] += rho * nu / hh ** 2 - rho * v0 / (2 * hh)
            A[i, n + i + 1] += B0 / mu / (2 * hh)
            A[i, n + i - 1] += -B0 / mu / (2 * hh)
            rhs[i] = -rho * g
            # B equation
            j = n + i
            A[j, n + i - 1] += eta / hh ** 2 + v0 / (2 * hh)
            A[j, n + i] += -2 * eta / hh ** 2
            A[j, n + i + 1] += eta / hh ** 2 - v0 / (2 * hh)
            A[j, i + 1] += B0 / (2 * hh)
            A[j, i - 1] += -B0 / (2 * hh)
        A[0, 0] = 1.0
        rhs[0] = U_bot
        A[n - 1, n - 1] = 1.0
        rhs[n - 1] = U_top
        # B1 walls with second-order one-sided derivatives
        d0 = {n: -1.5 / hh, n + 1: 2.0 / hh, n + 2: -0.5 / hh}
        dN = {2 * n - 1: 1.5 / hh, 2 * n - 2: -2.0 / hh, 2 * n - 3: 0.5 / hh}
        for (row, c, dd, node, sgn) in ((n, c_bot, d0, n, -1.0), (2 * n - 1, c_top, dN, 2 * n - 1, 1.0)):
            if c == 0.0:
                A[row, node] = 1.0
            elif math.isinf(c):
                for col, v in dd.items():
                    A[row, col] = v
            else:
                for col, v in dd.items():
                    A[row, col] = c * H * v
                A[row, node] += sgn
        sol = spla.spsolve(A.tocsr(), rhs)
        return yy, sol[:n], sol[n:]

    y1, u1, b1 = solve(m)
    y2, u2, b2 = solve(2 * m)
    ue = (4 * u2[::2] - u1) / 3.0
    be = (4 * b2[::2] - b1) / 3.0
    return np.interp(y, y1, ue), np.interp(y, y1, be)


# ---------------------------------------------------------------------------
# Diffusion with a surface reaction (Section 5.3 set-up)
# ---------------------------------------------------------------------------
def reaction_eigenvalues(Da: float, n: int) -> np.ndarray:
    """First n positive roots z of z tan z = Da (z = beta W)."""
    roots = []
    for k in range(n):
        lo = k * math.pi + 1e-12
        hi = k * math.pi + math.pi / 2 - 1e-12
        roots.append(optimize.brentq(lambda z: z * math.tan(z) - Da, lo, hi, xtol=1e-15))
    return np.array(roots)


def diffusion_reaction(x: np.ndarray, y: np.ndarray, W: float, L: float, Da: float,
                       C_BC: float = 10.0, C_eq: float = 1.0, nterms: int = 200) -> np.ndarray:
    """Steady C(x, y) on [0, L] x [0, W]: C = C_BC at x = 0, zero normal
    gradient at y = 0 and x = L, and -D dC/dn = -k_r (C - C_eq) at y = W
    (n into the fluid), Da = k_r W / D.  Separation of variables:

    C - C_eq = sum_n A_n cos(beta_n y) cosh(beta_n (L - x))/cosh(beta_n L),
    beta_n W tan(beta_n W) = Da,
    A_n = (C_BC - C_eq) (sin(beta_n W)/beta_n) / (W/2 + sin(2 beta_n W)/(4 beta_n)).
    """
    z = reaction_eigenvalues(Da, nterms)
    beta = z / W
    x = np.asarray(x, float)[..., None]
    y = np.asarray(y, float)[..., None]
    A = (C_BC - C_eq) * (np.sin(beta * W) / beta) / (W / 2 + np.sin(2 * beta * W) / (4 * beta))
    # cosh ratio written with exponentials to avoid overflow
    ratio = (np.exp(-beta * x) + np.exp(-beta * (2 * L - x))) / (1.0 + np.exp(-2 * beta * L))
    return C_eq + np.sum(A * np.cos(beta * y) * ratio, axis=-1)


# ---------------------------------------------------------------------------
# Pipes
# ---------------------------------------------------------------------------
def hagen_poiseuille(r: np.ndarray, R: float, g: float, nu: float) -> np.ndarray:
    return g * (R * R - np.asarray(r) ** 2) / (4 * nu)


def pipe_mhd_polar(R: float, B0: float, nu: float, eta: float, g: float, wall: str,
                   c_w: float = 0.0, rho: float = 1.0, mu: float = 1.0, nr: int = 64,
                   nt: int = 128):
    """Fully developed MHD pipe flow (axis x1, applied field B0 along x2),
    second-order finite differences on a cell-centred polar grid
    r_i = (i + 1/2) dr, t_j = j dt (x2 = r cos t, x3 = r sin t):

        nu lap(u) + (B0/(rho mu)) d2 B1 + g = 0,   eta lap(B1) + B0 d2 u = 0,
        d2 = cos(t) d_r - (sin(t)/r) d_t.

    Walls (r = R): u = 0; B1 = 0 (insulating), d_r B1 = 0 (perfectly
    conducting) or c_w R d_r B1 + B1 = 0 (Shercliff thin wall), each imposed
    through a ghost value at r = R + dr/2.  Returns (r, t, U, B1) grids.
    """
    dr = R / nr
    dt = 2 * math.pi / nt
    r = (np.arange(nr) + 0.5) * dr
    t = np.arange(nt) * dt
    n = nr * nt

    def ghost_coef(field):
        # ghost = coef * (value at the last cell)
        if field == 0 or wall == "insulating":
            return -1.0
        if wall == "conducting":
            return 1.0
        a = c_w * R / dr
        return (a - 0.5) / (a + 0.5)

    rows, cols, vals = [], [], []
    rhs = np.zeros(2 * n)

    def add(rw, cl, v):
        rows.append(rw)
        cols.append(cl)
        vals.append(v)

    idx = lambda f, i, j: f * n + i * nt + (j % nt)
    coefs = ((nu, B0 / (rho * mu), g), (eta, B0, 0.0))   # (diffusivity, coupling, source)
    for f in (0, 1):
        lam, cpl, src = coefs[f]
        o = 1 - f
        for i in range(nr):
            rp, rm = r[i] + dr / 2, r[i] - dr / 2
            for j in range(nt):
                row = idx(f, i, j)
                ct, st = math.cos(t[j]), math.sin(t[j])
                # (1/r) d_r (r d_r)
                if i > 0:
                    add(row, idx(f, i - 1, j), lam * rm / (r[i] * dr * dr))
                    add(row, row, -lam * rm / (r[i] * dr * dr))
                if i < nr - 1:
                    add(row, idx(f, i + 1, j), lam * rp / (r[i] * dr * dr))
                    add(row, row, -lam * rp / (r[i] * dr * dr))
                else:
                    add(row, row, lam * rp / (r[i] * dr * dr) * (ghost_coef(f) - 1.0))
                # (1/r^2) d_tt
                ctt = lam / (r[i] ** 2 * dt * dt)
                add(row, idx(f, i, j + 1), ctt)
                add(row, idx(f, i, j - 1), ctt)
                add(row, row, -2 * ctt)
                # coupling cpl * (cos t d_r - sin t / r d_t) of the other field
                cr = cpl * ct / (2 * dr)
                if i < nr - 1:
                    add(row, idx(o, i + 1, j), cr)
                else:
                    add(row, idx(o, i, j), cr * ghost_coef(o))
                if i > 0:
                    add(row, idx(o, i - 1, j), -cr)
                else:
                    add(row, idx(o, 0, j + nt // 2), -cr)
                cth = -cpl * st / (r[i] * 2 * dt)
                add(row, idx(o, i, j + 1), cth)
                add(row, idx(o, i, j - 1), -cth)
                rhs[row] = -src
    A = sparse.csr_matrix((vals, (rows, cols)), shape=(2 * n, 2 * n))
    sol = spla.spsolve(A, rhs)
    return r, t, sol[:n].reshape(nr, nt), sol[n:].reshape(nr, nt)


def polar_sample(r, t, F, x2, x3):
    """Bilinear interpolation of a polar-grid field at Cartesian points."""
    nr, nt = F.shape
    dr = r[1] - r[0]
    dt = t[1] - t[0]
    x2 = np.asarray(x2, float)
    x3 = np.asarray(x3, float)
    rr = np.hypot(x2, x3)
    tt = np.mod(np.arctan2(x3, x2), 2 * math.pi)
    fi = np.clip(rr / dr - 0.5, 0.0, nr - 1 - 1e-12)
    fj = tt / dt
    i0 = np.floor(fi).astype(int)
    j0 = np.floor(fj).astype(int)
    wi = fi - i0
    wj = fj - j0
    i1 = np.minimum(i0 + 1, nr - 1)
    j1 = (j0 + 1) % nt
    j0 = j0 % nt
    return ((1 - wi) * (1 - wj) * F[i0, j0] + wi * (1 - wj) * F[i1, j0]
            + (1 - wi) * wj * F[i0, j1] + wi * wj * F[i1, j1])


def stokes_second(y: np.ndarray, t: float, U: float, omega: float, nu: float, H: float) -> np.ndarray:
    """Stokes' second problem between a static wall at y = 0 and a wall at
    y = H moving tangentially at U cos(omega t) (Eq. 45): the periodic state
    u(y, t) = Re[U exp(i omega t) sinh(k y) / sinh(k H)], k = (1 + i) sqrt(omega / (2 nu)),
    the solution of u_t = nu u_yy with those wall values once the start has
    decayed."""
    k = (1.0 + 1.0j) * np.sqrt(omega / (2.0 * nu))
    return np.real(U * np.exp(1j * omega * t) * np.sinh(k * np.asarray(y)) / np.sinh(k * H))


def duct_poiseuille(x: np.ndarray, y: np.ndarray, a: float, b: float, G: float, mu: float,
                    nterms: int = 200) -> np.ndarray:
    """Fully developed flow along a rectangular duct -a < x < a, -b < y < b
    driven by G = -dp/dz: the solution of mu (u_xx + u_yy) = -G with u = 0 on
    the walls, as the cosine series in x (odd n) whose y-dependence meets the
    walls at y = +-b:
        u = (16 a^2 G / (mu pi^3)) sum_n (-1)^((n-1)/2) / n^3
            [1 - cosh(n pi y / 2a) / cosh(n pi b / 2a)] cos(n pi x / 2a).
    The far field of the channel of Section 5.1."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    u = np.zeros(np.broadcast(x, y).shape)
    for j in range(nterms):
        n = 2 * j + 1
        k = n * math.pi / (2.0 * a)
        # cosh ratio written with exponentials that cannot overflow
        ratio = (np.exp(k * (np.abs(y) - b)) + np.exp(-k * (np.abs(y) + b))) / (1.0 + math.exp(-2.0 * k * b))
        u += (-1.0) ** j / n ** 3 * (1.0 - ratio) * np.cos(k * x)
    return 16.0 * a * a * G / (mu * math.pi ** 3) * u
