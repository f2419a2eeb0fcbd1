"""Seeded synthetic scene descriptions for the coupled-LBM hot path.

This module is pure input data: lattice choices, domain extents, relaxation
times, forcing, and the boundary objects (flat walls, open planes, cylinders)
with the boundary-condition kind and the wall data each lattice uses there.  It
holds none of the method's arithmetic: no equilibria, no link geometry, no
collision.  Both the FP64 oracle and the HIP library build their node masks
and boundary-link tables from a ``Scene`` independently.

Random draws (wall offsets q, Hartmann numbers, conductance ratios, per-position
reaction rates, item sizes) come from SplitMix64 (Steele, Lea & Flood, 2014),
implemented here from its published definition.

Units are lattice units (dx = dt = 1).  The paper's parameter sets are stated in
SI units with c = dx/dt (Section 2.1); ``paper_case_to_lattice`` converts.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# SplitMix64
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1
BASE_SEED = 2506009070


class SplitMix64:
    """64-bit SplitMix generator: add the golden-ratio increment, then mix."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))

    def log_uniform(self, lo: float, hi: float) -> float:
        return math.exp(self.uniform(math.log(lo), math.log(hi)))

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on [lo, hi] inclusive."""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo

    def _block(self, n: int) -> np.ndarray:
        """the next n raw outputs at once (the state advances by n increments)."""
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * 0x9E3779B97F4A7C15) & _M64
        return z

    def uniform_array(self, n: int) -> np.ndarray:
        """n uniforms on [0, 1), the same values as n calls of uniform()."""
        return (self._block(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def normal_array(self, n: int) -> np.ndarray:
        """Box-Muller normals from consecutive pairs of uniforms (used to draw
        perturbed initial states and network parameters)."""
        m = (n + 1) // 2
        u = self.uniform_array(2 * m)
        r = np.sqrt(-2.0 * np.log(np.maximum(u[0::2], 1e-300)))
        out = np.empty(2 * m)
        out[0::2] = r * np.cos(2 * math.pi * u[1::2])
        out[1::2] = r * np.sin(2 * math.pi * u[1::2])
        return out[:n]


# ---------------------------------------------------------------------------
# Scene description
# ---------------------------------------------------------------------------
# lattice names
D2Q9, D3Q19, D2Q5, D3Q7 = "D2Q9", "D3Q19", "D2Q5", "D3Q7"
# boundary-condition kinds (per lattice, per boundary)
VEL, PRES, CONC, FLUX, BB0, MAG_DIR, MAG_FLUX, MAG_THETA = (
    "VEL", "PRES", "CONC", "FLUX", "BB0", "MAG_DIR", "MAG_FLUX", "MAG_THETA")
KIND_CODES = {VEL: 1, PRES: 2, CONC: 3, FLUX: 4, BB0: 5, MAG_DIR: 6, MAG_FLUX: 7, MAG_THETA: 8}
LATTICE_CODES = {D2Q9: 1, D3Q19: 2, D2Q5: 3, D3Q7: 4}
STORAGE_CODES = {"f64": 1, "f32": 2, "f16": 3, "bf16": 4}


@dataclass
class BC:
    """Boundary condition of one lattice (or one magnetic component) on a boundary.

    kind   : one of VEL, PRES, CONC, FLUX, BB0, MAG_DIR, MAG_FLUX, MAG_THETA
    value  : given rho (PRES), C (CONC) or B_k (MAG_DIR)
    u_given: the wall velocity is used in the moving-wall terms; False means the
             velocity at the boundary point is extrapolated from the fluid
    law    : how a FLUX, MAG_FLUX or MAG_THETA wall states its physics.  This
             module only describes it; the oracle and the library each form
             the link coefficients from it:
               "coef"      the flux law F(phi) = a1 phi + quad phi^2 - a3 with
                           the coefficients given (lattice units)
               "robin"     d phi/dn = k phi, n pointing into the fluid
               "reaction"  a first-order surface reaction F = -k (phi - phi_eq)
               "shercliff" a thin wall of conductance ratio c_w over the length
                           scale H (c_w = inf: perfectly conducting)
    a1, a3, quad: coefficients of the "coef" law
    k, phi_eq: rate and equilibrium value of the "robin" and "reaction" laws
    c_w, H : conductance ratio and length scale of the "shercliff" law
    profile: optional per-position k ("robin", "reaction") or a1 ("coef") along
             ``profile_axis`` (indexed by the first fluid node's coordinate on
             that axis)
    alt    : the comparison form of Section 5 instead of the method's: VEL
             and PRES extrapolated at every d (Eqs. 15-16), FLUX and MAG_FLUX
             with the flux added at the wall (Eq. 33)
    cross_comps, cross: a scalar FLUX wall of component i under the "coef"
             law whose flux also depends on components (j, l) = cross_comps:
             F_i = a1 C_i + quad C_i^2 + cross C_j C_l - a3 (Section 4.2.2, a
             surface reaction between components, e.g. A + B -> P); (-1, -1):
             none
    """
    kind: str
    value: float = 0.0
    a1: float = 0.0
    a3: float = 0.0
    u_given: bool = True
    profile: Optional[np.ndarray] = None
    profile_axis: int = 0
    alt: bool = False
    quad: float = 0.0
    law: str = "coef"
    k: float = 0.0
    phi_eq: float = 0.0
    c_w: float = 0.0
    H: float = 0.0
    cross_comps: Tuple[int, int] = (-1, -1)
    cross: float = 0.0


@dataclass
class Boundary:
    """A flat plane (wall or open inlet/outlet) or a cylinder.

    plane   : ``axis`` is the wall normal axis, ``side`` 0 = below node 0,
              1 = above node n-1; the wall sits ``q`` lattice units outside the
              first/last node row (q in (0, 1]).
    cylinder: ``axis`` is the cylinder axis; nodes are fluid strictly inside
              radius ``radius`` about ``center`` (the axis coordinate of
              ``center`` is ignored).
    """
    type: str                    # "plane" | "cylinder" | "box"
    axis: int
    side: int = 0
    q: float = 0.5
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    is_open: bool = False
    u_w: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    u_osc: bool = False          # the velocity is u_w cos(wall_omega t') (Scene.wall_omega)
    d_scheme: float = 0.0        # > 0: the links use this d, not the measured one (Section 5.2 mismatch)
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # box: closed solid block lo <= x <= hi
    hi: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    f: Optional[BC] = None
    h: object = None             # a BC, or one per scalar component (list)
    g: List[Optional[BC]] = field(default_factory=list)   # one per evolved component

    def h_of(self, k: int) -> Optional[BC]:
        """the condition of scalar component k (a single BC serves all)"""
        if isinstance(self.h, (list, tuple)):
            return self.h[k] if k < len(self.h) else None
        return self.h


@dataclass
class Scene:
    name: str
    dim: int
    n: Tuple[int, int, int]               # node counts (nx, ny, nz); nz = 1 in 2D
    periodic: Tuple[bool, bool, bool]
    fluid_lattice: str
    scalar_lattice: Optional[str] = None
    mag_lattice: Optional[str] = None
    mag_comps: Tuple[int, ...] = ()       # evolved Cartesian components of B
    tau_f: float = 0.8
    tau_c: float = 1.0
    tau_m: float = 1.0
    rho0: float = 1.0
    C0: float = 0.0                       # rest (reference) concentration
    mu: float = 1.0                       # magnetic permeability
    B_ext: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    accel: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # body force per unit mass
    boundaries: List[Boundary] = field(default_factory=list)
    storage: str = "f64"
    store_scale: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    steps: int = 1000
    wall_omega: float = 0.0               # rad per step of the boundaries with u_osc
    init_C: float = 0.0                   # initial uniform concentration (every scalar component)
    scalar_ncomp: int = 1                 # scalar components C_0 .. (1..3), one D2Q5/D3Q7 lattice each
    tau_cs: Tuple[float, ...] = ()        # relaxation times of components 1, 2 (component 0: tau_c)
    # optional initial fields (fluid-domain arrays, shape (nz, ny, nx[, 3]);
    # init_Cf of several scalar components: (scalar_ncomp, nz, ny, nx))
    init_rho: Optional[np.ndarray] = None
    init_u: Optional[np.ndarray] = None
    init_Cf: Optional[np.ndarray] = None
    init_B: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def tau_scalar(self, k: int) -> float:
        """relaxation time of scalar component k"""
        return self.tau_c if k == 0 else self.tau_cs[k - 1]

    def with_(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Helpers for the configurations
# ---------------------------------------------------------------------------
def _nu(tau: float) -> float:
    return (tau - 0.5) / 3.0


def _diff(tau: float) -> float:
    """Diffusivity of the 5/7-velocity lattices (c^2 = 1/4 in lattice units)."""
    return (tau - 0.5) / 4.0


def hartmann_B0(Ha: float, H: float, rho: float, nu: float, eta: float, mu: float) -> float:
    """B0 from Ha^2 = B0^2 H^2 sigma/(rho nu), sigma = 1/(mu eta)."""
    return Ha * math.sqrt(rho * nu * eta * mu) / H


def poiseuille(nx: int = 64, ny: int = 32, tau: float = 0.8, g: float = 1e-6,
               q: float = 0.5, storage: str = "f64", steps: int = 20000,
               u_top: float = 0.0) -> Scene:
    """Plane channel between static (or sliding) walls, body-force driven."""
    wall = lambda side, u: Boundary("plane", axis=1, side=side, q=q, u_w=(u, 0.0, 0.0),
                                    f=BC(VEL))
    return Scene(name=f"poiseuille_{nx}x{ny}", dim=2, n=(nx, ny, 1),
                 periodic=(True, False, True), fluid_lattice=D2Q9, tau_f=tau,
                 accel=(g, 0.0, 0.0), boundaries=[wall(0, 0.0), wall(1, u_top)],
                 storage=storage, steps=steps)


def stokes_second(nx: int = 4, ny: int = 40, tau: float = 0.8, U: float = 0.01, period: int = 2000,
                  q: float = 0.5, storage: str = "f64", steps: int = 6000, dim: int = 2,
                  d_scheme: float = 0.0) -> Scene:
    """Stokes' second problem (the oscillating-wall validation of Section 5,
    Eq. 45): fluid at rest between a static wall below and a wall above that
    moves tangentially at U cos(omega t), omega = 2 pi / period, with walls
    at distance q outside the first and last node rows.  2D: D2Q9, walls
    normal to y, nx nodes periodic in x.  3D: D3Q19, walls normal to z,
    nx x nx nodes periodic in x and y, ny rows between the walls.
    d_scheme > 0 makes both walls use the scheme for that d whatever q is
    (the paper runs the d = 0.5 scheme on walls at q = 1 to show the error
    a layout/scheme mismatch brings)."""
    ax = 1 if dim == 2 else 2
    bottom = Boundary("plane", axis=ax, side=0, q=q, d_scheme=d_scheme, f=BC(VEL))
    top = Boundary("plane", axis=ax, side=1, q=q, u_w=(U, 0.0, 0.0), u_osc=True, d_scheme=d_scheme,
                   f=BC(VEL))
    if dim == 2:
        n, per, lat = (nx, ny, 1), (True, False, True), D2Q9
    else:
        n, per, lat = (nx, nx, ny), (True, True, False), D3Q19
    return Scene(name=f"stokes_{dim}d_{nx}x{ny}", dim=dim, n=n, periodic=per, fluid_lattice=lat, tau_f=tau,
                 boundaries=[bottom, top], storage=storage, steps=steps, wall_omega=2.0 * math.pi / period)


def channel_reservoirs(layout: str = "half", width: int = 20, res_len: int = 20, ch_len: int = 60,
                       tau: float = 0.7, u_in: float = 0.01, storage: str = "f64",
                       steps: int = 20000, q_io: Optional[float] = None, alt_io: bool = False) -> Scene:
    """The 3D channel of Section 5.1: a square channel between two reservoirs,
    D3Q19, driven by a uniform normal velocity u_in at the inlet (z = 0 end)
    and held at rho = 1 at the outlet (z = end).  The reservoirs' lateral
    sides are periodic; the channel's four walls are solid blocks (static,
    the velocity scheme with u = 0, i.e. Bouzidi's bounceback).

    layout "half": walls half a spacing outside the fluid nodes (d = 0.5),
    width + 2 nodes across; "full": walls on the outer grid layers (d = 1),
    width + 1 nodes across.  Lengths in lattice spacings (the paper: width
    20, reservoirs 20, channel 60, tau 0.7, u_in = 0.01).  ``q_io`` moves the
    inlet and outlet planes to that distance from the end nodes (default: the
    layout's); ``alt_io`` gives them the extrapolated forms at every d (the
    comparison of Section 5.1, unstable at large d)."""
    q = {"half": 0.5, "full": 1.0}[layout]
    n_lat = width + (2 if layout == "half" else 1)
    nz = 2 * res_len + ch_len + (0 if layout == "half" else -1)
    w_lo, w_hi = 1.0 - q, 1.0 - q + width
    z0 = -q + res_len
    z1 = z0 + ch_len
    inf = math.inf
    walls = []
    for ax in (0, 1):
        for lo_c, hi_c in ((-inf, w_lo), (w_hi, inf)):
            lo, hi = [-inf, -inf, z0], [inf, inf, z1]
            lo[ax], hi[ax] = lo_c, hi_c
            walls.append(Boundary("box", axis=2, lo=tuple(lo), hi=tuple(hi), f=BC(VEL)))
    qi = q if q_io is None else q_io
    inlet = Boundary("plane", axis=2, side=0, q=qi, is_open=True, u_w=(0.0, 0.0, u_in), f=BC(VEL, alt=alt_io))
    outlet = Boundary("plane", axis=2, side=1, q=qi, is_open=True, f=BC(PRES, value=1.0, alt=alt_io))
    return Scene(name=f"channel_{layout}_{n_lat}x{n_lat}x{nz}", dim=3, n=(n_lat, n_lat, nz),
                 periodic=(True, True, False), fluid_lattice=D3Q19, tau_f=tau, rho0=1.0,
                 boundaries=walls + [inlet, outlet], storage=storage, steps=steps)


def open_box(nx: int = 24, ny: int = 5, q_in: float = 0.5, q_out: float = 0.5, alt_in: bool = False,
             alt_out: bool = False, u_in: float = 0.01, tau: float = 0.7, storage: str = "f64") -> Scene:
    """Uniform D2Q9 flow through a box periodic in y: velocity inlet at
    x = -q_in, pressure outlet (rho = 1) at nx - 1 + q_out.  With alt_in /
    alt_out the inlet / outlet take the extrapolated forms at every d (the
    comparison of Section 5.1, which loses stability at large d)."""
    inlet = Boundary("plane", axis=0, side=0, q=q_in, is_open=True, u_w=(u_in, 0.0, 0.0), f=BC(VEL, alt=alt_in))
    outlet = Boundary("plane", axis=0, side=1, q=q_out, is_open=True, f=BC(PRES, value=1.0, alt=alt_out))
    return Scene(name=f"open_box_{nx}x{ny}", dim=2, n=(nx, ny, 1), periodic=(False, True, True),
                 fluid_lattice=D2Q9, tau_f=tau, rho0=1.0, boundaries=[inlet, outlet], storage=storage)


def reactive_channel(nx: int = 512, ny: int = 256, k: float = 1e-2, q: float = 0.3,
                     rho_in: float = 1.001, rho_out: float = 1.0, tau_f: float = 0.8,
                     tau_c: float = 0.6, storage: str = "f32", steps: int = 2000,
                     k_range: Optional[Tuple[float, float]] = None, seed: int = BASE_SEED + 2,
                     q_io: float = 0.5) -> Scene:
    """Pressure-driven D2Q9 channel with a D2Q5 solute and Robin walls dC/dn = k C
    (n pointing into the fluid: consumption at the walls).  When ``k_range``
    is given, k is drawn per wall position, log-uniform in that range.
    """
    rng = SplitMix64(seed)
    walls = []
    for side in (0, 1):
        prof = None
        if k_range is not None:
            prof = np.array([rng.log_uniform(*k_range) for _ in range(nx)])
        walls.append(Boundary("plane", axis=1, side=side, q=q, f=BC(VEL),
                              h=BC(FLUX, law="robin", k=k, profile=prof, profile_axis=0)))
    inlet = Boundary("plane", axis=0, side=0, q=q_io, is_open=True,
                     f=BC(PRES, value=rho_in), h=BC(CONC, value=1.0, u_given=False))
    outlet = Boundary("plane", axis=0, side=1, q=q_io, is_open=True,
                      f=BC(PRES, value=rho_out), h=BC(FLUX, a1=0.0, a3=0.0, u_given=False))
    return Scene(name=f"reactive_{nx}x{ny}", dim=2, n=(nx, ny, 1), periodic=(False, False, True),
                 fluid_lattice=D2Q9, scalar_lattice=D2Q5, tau_f=tau_f, tau_c=tau_c,
                 rho0=1.0, C0=0.0, init_C=0.0, boundaries=walls + [inlet, outlet],
                 storage=storage, store_scale=(1024.0, 1024.0, 1.0), steps=steps)


def reactive_species(nx: int = 512, ny: int = 256, k: float = 2e-2, q: float = 0.3, ncomp: int = 3,
                     C_in: Tuple[float, ...] = (1.0, 0.8, 0.0), taus: Tuple[float, ...] = (0.6, 0.7, 0.65),
                     rho_in: float = 1.001, rho_out: float = 1.0, tau_f: float = 0.8, storage: str = "f32",
                     steps: int = 2000, q_io: float = 0.5) -> Scene:
    """The pressure-driven reactive channel with several scalar components
    (Section 4.2.2): A (0) and B (1) enter at the inlet and react at both
    walls, A + B -> P at the rate k C_A C_B, so F_A = F_B = -k C_A C_B; with
    three components the product P (2) leaves the walls at F_P = +k C_A C_B.
    Zero flux at the outlet for every component."""
    if ncomp not in (2, 3):
        raise ValueError("ncomp must be 2 or 3")
    walls = [Boundary("plane", axis=1, side=side, q=q, f=BC(VEL),
                      h=[BC(FLUX, cross_comps=(0, 1), cross=-k if i < 2 else k) for i in range(ncomp)])
             for side in (0, 1)]
    inlet = Boundary("plane", axis=0, side=0, q=q_io, is_open=True, f=BC(PRES, value=rho_in),
                     h=[BC(CONC, value=C_in[i], u_given=False) for i in range(ncomp)])
    outlet = Boundary("plane", axis=0, side=1, q=q_io, is_open=True, f=BC(PRES, value=rho_out),
                      h=[BC(FLUX, a1=0.0, a3=0.0, u_given=False) for _ in range(ncomp)])
    return Scene(name=f"reactive_species{ncomp}_{nx}x{ny}", dim=2, n=(nx, ny, 1), periodic=(False, False, True),
                 fluid_lattice=D2Q9, scalar_lattice=D2Q5, scalar_ncomp=ncomp, tau_f=tau_f, tau_c=taus[0],
                 tau_cs=tuple(taus[1:ncomp]), rho0=1.0, C0=0.0, init_C=0.0, boundaries=walls + [inlet, outlet],
                 storage=storage, store_scale=(1024.0, 1024.0, 1.0), steps=steps)


def hartmann_couette(nx: int = 1024, ny: int = 512, Ha: float = 5.0, c_top: float = 0.1,
                     u_top: float = 0.01, v0: float = 0.002, qb: Optional[float] = None,
                     qt: Optional[float] = None, tau_f: float = 0.8, tau_m: float = 0.9,
                     storage: str = "f32", steps: int = 2000, seed: int = BASE_SEED + 3,
                     accel: float = 0.0, top_scheme: str = "M") -> Scene:
    """Sheared MHD channel with transverse field B_ext = (0, B0).

    Bottom wall: insulating (B1 = 0), velocity (0, v0).  Top wall: velocity
    (u_top, v0), conductance ratio ``c_top``: 0 -> given B1 = 0,
    inf -> perfectly conducting (zero flux), otherwise a thin wall of that
    ratio over the half-width H (Eq. 30).  B2 = B0 is given on both walls.  With v0 != 0 both
    walls transpire uniformly, which keeps the flow x-invariant.
    ``top_scheme`` for a finite c_top: "M" (the method, flux at the point M),
    "X" (the simplified Eq. 33, flux at the wall) or "theta" (the link-based
    form of Eqs. 39-40).
    """
    rng = SplitMix64(seed)
    qb = rng.uniform(0.1, 0.9) if qb is None else qb
    qt = rng.uniform(0.1, 0.9) if qt is None else qt
    H = (ny - 1 + qb + qt) / 2.0
    nu, eta, rho, mu = _nu(tau_f), _diff(tau_m), 1.0, 1.0
    B0 = hartmann_B0(Ha, H, rho, nu, eta, mu)
    if c_top == 0.0:
        top_b1 = BC(MAG_DIR, value=0.0)
    elif math.isinf(c_top):
        top_b1 = BC(MAG_FLUX, law="shercliff", c_w=math.inf, H=H)
    elif top_scheme == "theta":
        top_b1 = BC(MAG_THETA, law="shercliff", c_w=c_top, H=H)
    else:
        top_b1 = BC(MAG_FLUX, law="shercliff", c_w=c_top, H=H, alt=top_scheme == "X")
    bottom = Boundary("plane", axis=1, side=0, q=qb, u_w=(0.0, v0, 0.0), f=BC(VEL),
                      g=[BC(MAG_DIR, value=0.0), BC(MAG_DIR, value=B0)])
    top = Boundary("plane", axis=1, side=1, q=qt, u_w=(u_top, v0, 0.0), f=BC(VEL),
                   g=[top_b1, BC(MAG_DIR, value=B0)])
    sc = Scene(name=f"hartmann_{nx}x{ny}", dim=2, n=(nx, ny, 1), periodic=(True, False, True),
               fluid_lattice=D2Q9, mag_lattice=D2Q5, mag_comps=(0, 1), tau_f=tau_f, tau_m=tau_m,
               rho0=rho, mu=mu, B_ext=(0.0, B0, 0.0), accel=(accel, 0.0, 0.0),
               boundaries=[bottom, top], storage=storage, store_scale=(1024.0, 1.0, 1024.0),
               steps=steps)
    sc.meta = dict(H=H, qb=qb, qt=qt, B0=B0, Ha=Ha, c_top=c_top, nu=nu, eta=eta)
    return sc


def mhd_pipe(nx: int = 64, side: int = 128, R: float = 60.0, wall: str = "insulating",
             c_w: float = 0.05, Ha: float = 10.0, g: float = 1e-6, tau_f: float = 0.8,
             tau_m: float = 0.9, storage: str = "f32", steps: int = 2000,
             ncomp: int = 1, mag_lattice: str = D3Q7) -> Scene:
    """Pipe along x (periodic), circular cross-section in (y, z), B_ext along y.

    ``wall``: "insulating" (given B1 = 0), "conducting" (zero flux) or
    "shercliff" (a thin wall of conductance ratio c_w, Eq. 30 with H = R).  With ``ncomp`` = 3 the transverse
    components are also evolved with given-B walls (B2 = B0, B3 = 0).
    ``mag_lattice`` D3Q19 solves B1 on the 19-velocity lattice (c_g^2 = 1/3,
    eta = (tau_m - 1/2)/3), the option Section 6.1 suggests for conducting
    walls.
    """
    nu, rho, mu = _nu(tau_f), 1.0, 1.0
    eta = _nu(tau_m) if mag_lattice == D3Q19 else _diff(tau_m)
    B0 = hartmann_B0(Ha, R, rho, nu, eta, mu)
    c = (side - 1) / 2.0
    if wall == "insulating":
        b1 = BC(MAG_DIR, value=0.0)
    elif wall == "conducting":
        b1 = BC(MAG_FLUX, law="shercliff", c_w=math.inf, H=R)
    elif wall == "shercliff":
        b1 = BC(MAG_FLUX, law="shercliff", c_w=c_w, H=R)
    else:
        raise ValueError(wall)
    gbc = [b1] + ([BC(MAG_DIR, value=B0), BC(MAG_DIR, value=0.0)] if ncomp == 3 else [])
    cyl = Boundary("cylinder", axis=0, center=(0.0, c, c), radius=R, f=BC(VEL), g=gbc)
    comps = (0,) if ncomp == 1 else (0, 1, 2)
    sc = Scene(name=f"pipe_{nx}x{side}x{side}_{wall}", dim=3, n=(nx, side, side),
               periodic=(True, False, False), fluid_lattice=D3Q19, mag_lattice=mag_lattice,
               mag_comps=comps, tau_f=tau_f, tau_m=tau_m, rho0=rho, mu=mu,
               B_ext=(0.0, B0, 0.0), accel=(g, 0.0, 0.0), boundaries=[cyl], storage=storage,
               store_scale=(1024.0, 1.0, 1024.0), steps=steps)
    sc.meta = dict(R=R, B0=B0, Ha=Ha, wall=wall, c_w=c_w, nu=nu, eta=eta, center=c)
    return sc


def diffusion_reaction(layout: str = "half", Da: float = 4.8, tau_D: float = 0.9,
                       W_nodes: Optional[int] = None, steps: int = 20000) -> Scene:
    """Pure diffusion (u = 0) with C given on the left, zero normal gradient on
    the bottom and right, and a first-order surface reaction on the top.

    Half-grid layout: walls half-way between nodes (d = 0.5).  Full-grid
    layout: first and last node rows on the walls (d = 1).  Lattice sizes
    follow the paper's 102 x 82 / 101 x 81 node case (W = 0.01, L = 0.0125,
    dx = 1.25e-4, outer layers included) unless ``W_nodes`` rescales it.  C_BC = 10, C_eq = 1.
    Reaction F(C) = -k_r (C - C_eq) with k_r = Da D / W.
    """
    D = _diff(tau_D)
    if W_nodes is None:
        W_cells = 80             # W / dx
    else:
        W_cells = W_nodes
    L_cells = W_cells * 1.25   # L / W = 1.25
    # half-grid: walls half-way between the outer node layers and the first
    # fluid layers; full-grid: the outer node layers lie on the walls, so the
    # fluid nodes start one spacing inside (d = 1).  Node j sits at j + q from
    # the lower wall in both layouts.
    if layout == "half":
        nx, ny, q = int(round(L_cells)), int(W_cells), 0.5
    else:
        nx, ny, q = int(round(L_cells)) - 1, int(W_cells) - 1, 1.0
    kr = Da * D / W_cells
    left = Boundary("plane", axis=0, side=0, q=q, h=BC(CONC, value=10.0), f=BC(VEL))
    right = Boundary("plane", axis=0, side=1, q=q, h=BC(BB0), f=BC(VEL))
    bottom = Boundary("plane", axis=1, side=0, q=q, h=BC(BB0), f=BC(VEL))
    top = Boundary("plane", axis=1, side=1, q=q, h=BC(FLUX, law="reaction", k=kr, phi_eq=1.0), f=BC(VEL))
    # the bottom/right walls use the d >= 0.5 bounce-back (Eq. 22 form); with
    # q = 0.5 both forms coincide.  Walls win ties against each other by order.
    sc = Scene(name=f"diffreact_{layout}_Da{Da}", dim=2, n=(nx, ny, 1),
               periodic=(False, False, True), fluid_lattice=D2Q9, scalar_lattice=D2Q5,
               tau_f=1.0, tau_c=tau_D, C0=0.0, init_C=1.0,
               boundaries=[bottom, top, left, right], storage="f64", steps=steps)
    sc.meta = dict(W=float(W_cells), L=float(L_cells), D=D, kr=kr, Da=Da, layout=layout)
    return sc


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def config(index: int, **kw) -> Scene:
    """Workload ``index`` (1..4) at its full size; keyword overrides apply."""
    if index == 1:
        return poiseuille(**kw)
    if index == 2:
        return reactive_channel(**kw)
    if index == 3:
        return hartmann_couette(**kw)
    if index == 4:
        return mhd_pipe(**kw)
    raise ValueError(index)


@dataclass
class BatchItem:
    shape: str            # "duct" | "pipe"
    ny: int
    nz: int
    q: Tuple[float, ...]  # duct: (y-lo, y-hi, z-lo, z-hi); pipe: (q,)
    Ha: float
    c_w: float                # drawn wall conductance ratio
    c_eff: Tuple[float, ...]  # ratio each wall runs with (c_w, or the stable floor above it), order of q
    scene: Scene

    @property
    def raised(self) -> bool:
        """True when some wall runs with a conductance ratio above the drawn one."""
        return any(c > self.c_w for c in self.c_eff)


# The thin-wall flux is explicit: every step adds F(B_X) times the link weight
# to one bounced population per link, and F changes by eta / (c_w H) per unit
# of B.  FP64 oracle runs of 3000 steps (widths 16-64, d in [0.1, 0.9]) diverge
# once that slope passes 0.4-0.5 at duct corners with d near 0.1, and 0.5-0.7
# on pipe walls.  The batched items therefore narrow the drawn range
# c_w ~ logU[1e-3, 10] from below: a wall runs with c_eff = max(c_w, c_min),
# c_min = eta / (FLUX_SLOPE_MAX H), the smallest ratio whose slope stays at
# FLUX_SLOPE_MAX.  Each item records c_w and c_eff; results are reported
# separately for the items with a raised wall (BatchItem.raised).
FLUX_SLOPE_MAX = 0.3


def batch_items(n_items: int = 256, seed: int = BASE_SEED + 5, side_lo: int = 64,
                side_hi: int = 256, Ha_hi: float = 50.0, c_lo: float = 1e-3, c_hi: float = 10.0,
                tau_f: float = 0.8, tau_m: float = 0.9, u_target: float = 0.01,
                storage: str = "f16", ducts_only: bool = False,
                q_duct: Optional[float] = None) -> List[BatchItem]:
    """Uneven duct / pipe cross-sections (axial extent 1, periodic) for the
    batched solver: D3Q19 fluid + D3Q7 magnetic lattice evolving B1 only,
    B_ext along y, thin walls of conductance ratio c_w everywhere (raised to
    the stable floor where needed, see FLUX_SLOPE_MAX).  ducts_only makes
    every item a duct and q_duct puts every duct wall at that distance (the
    draws are made as usual, so the other parameters do not change)."""
    rng = SplitMix64(seed)
    nu, eta = _nu(tau_f), _diff(tau_m)
    c_min = lambda H: eta / (FLUX_SLOPE_MAX * H)
    items = []
    for i in range(n_items):
        shape = "duct" if rng.uniform() < 0.5 else "pipe"
        shape = "duct" if ducts_only else shape
        Ha = rng.uniform(0.0, Ha_hi)
        c_w = rng.log_uniform(c_lo, c_hi)
        if shape == "duct":
            a = rng.randint(side_lo, side_hi)
            b = rng.randint(side_lo, side_hi)
            qs = tuple(rng.uniform(0.1, 0.9) for _ in range(4))
            if q_duct is not None:
                qs = (q_duct,) * 4
            Hy = (a - 1 + qs[0] + qs[1]) / 2.0
            Hz = (b - 1 + qs[2] + qs[3]) / 2.0
            Hmin = min(Hy, Hz)
            B0 = hartmann_B0(Ha, Hy, 1.0, nu, eta, 1.0)
            # Poiseuille-duct centre speed ~ g h^2/(2 nu) * 0.59 (h = short half side)
            g = u_target * 2.0 * nu / (0.59 * Hmin * Hmin)
            bnds, c_eff = [], []
            for ax, (side, qq) in [(1, (0, qs[0])), (1, (1, qs[1])), (2, (0, qs[2])), (2, (1, qs[3]))]:
                H = Hy if ax == 1 else Hz
                c = max(c_w, c_min(H))
                c_eff.append(c)
                bnds.append(Boundary("plane", axis=ax, side=side, q=qq, f=BC(VEL),
                                     g=[BC(MAG_FLUX, law="shercliff", c_w=c, H=H)]))
            ny, nz = a, b
        else:
            s = rng.randint(side_lo, side_hi)
            qq = rng.uniform(0.1, 0.9)
            R = s / 2.0 - 2.0 + qq
            B0 = hartmann_B0(Ha, R, 1.0, nu, eta, 1.0)
            g = u_target * 4.0 * nu / (R * R)
            c = (s - 1) / 2.0
            cw = max(c_w, c_min(R))
            c_eff = [cw]
            bnds = [Boundary("cylinder", axis=0, center=(0.0, c, c), radius=R, f=BC(VEL),
                             g=[BC(MAG_FLUX, law="shercliff", c_w=cw, H=R)])]
            ny = nz = s
            qs = (qq,)
        sc = Scene(name=f"item{i}_{shape}", dim=3, n=(1, ny, nz), periodic=(True, False, False),
                   fluid_lattice=D3Q19, mag_lattice=D3Q7, mag_comps=(0,), tau_f=tau_f,
                   tau_m=tau_m, B_ext=(0.0, B0, 0.0), accel=(g, 0.0, 0.0), boundaries=bnds,
                   storage=storage, store_scale=(1024.0, 1.0, 1024.0))
        items.append(BatchItem(shape, ny, nz, qs, Ha, c_w, tuple(c_eff), sc))
    return items


def paper_case_to_lattice(dx: float, c: float, nu: float = None, D: float = None,
                          eta: float = None) -> dict:
    """Convert an SI parameter set (dx, c = dx/dt) into relaxation times.

    nu = dt c^2/3 (tau_nu - 1/2); D, eta = dt c^2/4 (tau - 1/2).
    """
    dt = dx / c
    out = {"dt": dt}
    if nu is not None:
        out["tau_f"] = 0.5 + nu / (dt * c * c / 3.0)
    if D is not None:
        out["tau_c"] = 0.5 + D / (dt * c * c / 4.0)
    if eta is not None:
        out["tau_m"] = 0.5 + eta / (dt * c * c / 4.0)
    return out


def developed(sc: Scene, seed: int = BASE_SEED + 7, u_amp: float = 0.02, b_amp: float = None,
              rho_amp: float = 1e-3, C_amp: float = 0.5) -> Scene:
    """The scene with smooth, seeded initial fields of realistic size: a few
    low-order Fourier modes per component with SplitMix64 amplitudes (velocity
    ~u_amp, density deviation ~rho_amp, induced field ~b_amp, concentration
    ~C_amp around its initial value).  Used to start parity runs from a
    developed state rather than from rest."""
    rng = SplitMix64(seed)
    nx, ny, nz = sc.n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def smooth():
        f = np.zeros((nz, ny, nx))
        for _ in range(3):
            kx, ky, kz = (rng.randint(0, 2) for _ in range(3))
            ph = [rng.uniform(0, 2 * math.pi) for _ in range(3)]
            amp = rng.uniform(-1.0, 1.0)
            f += amp * (np.cos(2 * math.pi * kx * x / max(nx, 1) + ph[0])
                        * np.cos(math.pi * ky * y / max(ny, 1) + ph[1])
                        * np.cos(math.pi * kz * z / max(nz, 1) + ph[2]))
        return f / 3.0

    B0 = max(abs(b) for b in sc.B_ext) if any(sc.B_ext) else 1e-2
    b_amp = 0.3 * B0 if b_amp is None else b_amp
    u = np.stack([smooth(), smooth(), smooth() if sc.dim == 3 else np.zeros((nz, ny, nx))], -1) * u_amp
    rho = sc.rho0 + rho_amp * smooth()
    B = np.broadcast_to(np.asarray(sc.B_ext, float), (nz, ny, nx, 3)).copy()
    for c in sc.mag_comps:
        B[..., c] += b_amp * smooth()
    Cf = sc.init_C + C_amp * smooth() if sc.scalar_lattice else None
    if Cf is not None and sc.scalar_ncomp > 1:
        Cf = np.stack([Cf] + [sc.init_C + C_amp * smooth() for _ in range(sc.scalar_ncomp - 1)])
    return sc.with_(init_rho=rho, init_u=u, init_B=B if sc.mag_lattice else None, init_Cf=Cf)


def axial_start(sc: Scene, seed: int = BASE_SEED + 9, u_amp: float = 0.01, b_rel: float = 0.3) -> Scene:
    """A duct / pipe item (axial extent 1) started from smooth axial fields
    only, the form a warm start takes: u = (u_x, 0, 0), B = B_ext + (b_x, 0, 0),
    rho = rho0.  u_x is a seeded multiple of a sine bump over the box (~u_amp),
    b_x a seeded multiple of b_rel |B_ext| times the bump, odd in y.  In-plane
    velocities and density changes are left out: started from those, the BGK
    update keeps a row-alternating in-plane velocity that never decays."""
    rng = SplitMix64(seed)
    nx, ny, nz = sc.n
    z, y = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    bump = np.sin(math.pi * (y + 0.5) / ny) * np.sin(math.pi * (z + 0.5) / nz)
    a, c = rng.uniform(0.5, 1.5), rng.uniform(-1.0, 1.0)
    u = np.zeros((nz, ny, nx, 3))
    u[..., 0] = (u_amp * a * bump * (1.0 + 0.3 * np.cos(math.pi * y / ny)))[..., None]
    B = np.broadcast_to(np.asarray(sc.B_ext, float), (nz, ny, nx, 3)).copy()
    B0 = max(abs(b) for b in sc.B_ext)
    B[..., 0] += (b_rel * c * B0 * bump * np.sin(2.0 * math.pi * y / ny))[..., None]
    return sc.with_(init_u=u, init_B=B if sc.mag_lattice else None)
