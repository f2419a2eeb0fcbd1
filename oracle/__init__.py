"""FP64 CPU oracle for the coupled lattice Boltzmann sweep — TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py`` use
this package.  It wraps ``oracle.c`` (plain C, double precision) through
ctypes and shares nothing with the HIP library.  ``analytic`` holds the closed
forms and independent reference solvers the oracle is pinned to.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

import scenes as S

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source in extended precision (x87 long double): a tighter
# reference for FP64 parity, whose error is below double rounding
_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, IEEE arithmetic, OpenMP loops),
    once in double precision and once in long double."""
    for out, extra in ((_LIB, []), (_LIB_LD, ["-DOR_REAL=long double"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
                                   "-shared", "-Wall", "-Wno-unused-function", *extra, _SRC, "-o", tmp,
                                   "-lm"])
            os.replace(tmp, out)
    return _LIB


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("u_given", C.c_int32), ("profile_axis", C.c_int32),
                ("profile_len", C.c_int32), ("alt", C.c_int32), ("law", C.c_int32), ("value", C.c_double),
                ("a1", C.c_double), ("a3", C.c_double), ("quad", C.c_double),
                ("profile", C.POINTER(C.c_double)), ("k", C.c_double), ("phi_eq", C.c_double),
                ("c_w", C.c_double), ("H", C.c_double), ("cj", C.c_int32), ("cl", C.c_int32),
                ("cross", C.c_double)]


_LAWS = {"coef": 0, "robin": 1, "reaction": 2, "shercliff": 3}


class _Boundary(C.Structure):
    _fields_ = [("type", C.c_int32), ("axis", C.c_int32), ("side", C.c_int32),
                ("is_open", C.c_int32), ("q", C.c_double), ("center", C.c_double * 3),
                ("radius", C.c_double), ("u_w", C.c_double * 3), ("f", _BC), ("h", _BC * 3),
                ("g", _BC * 3), ("omega", C.c_double), ("d_used", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class _Scene(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("fl", C.c_int32), ("sl", C.c_int32), ("ml", C.c_int32), ("ncomp", C.c_int32),
                ("comps", C.c_int32 * 3), ("tau_f", C.c_double), ("tau_c", C.c_double),
                ("tau_m", C.c_double), ("rho0", C.c_double), ("C0", C.c_double),
                ("mu", C.c_double), ("B_ext", C.c_double * 3), ("accel", C.c_double * 3),
                ("init_C", C.c_double), ("nb", C.c_int32), ("b", C.POINTER(_Boundary)),
                ("ns", C.c_int32), ("pad", C.c_int32), ("tau_s", C.c_double * 3)]


class Link(C.Structure):
    _fields_ = [("A", C.c_int32), ("E", C.c_int32), ("field", C.c_int32), ("comp", C.c_int32),
                ("dir", C.c_int32), ("kind", C.c_int32), ("bnd", C.c_int32),
                ("u_given", C.c_int32), ("d", C.c_double), ("value", C.c_double),
                ("a1", C.c_double), ("a3", C.c_double), ("weight", C.c_double),
                ("u_w", C.c_double * 3), ("omega", C.c_double), ("compare", C.c_int32), ("pad", C.c_int32),
                ("quad", C.c_double), ("cj", C.c_int32), ("cl", C.c_int32), ("cross", C.c_double)]


class LinkIn(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("kind", C.c_int32), ("dir", C.c_int32),
                ("comp_axis", C.c_int32), ("u_given", C.c_int32), ("d", C.c_double),
                ("value", C.c_double), ("a1", C.c_double), ("a3", C.c_double),
                ("weight", C.c_double), ("u_w", C.c_double * 3), ("x_ap_E", C.c_double),
                ("x_ap_A", C.c_double), ("x_a_A", C.c_double), ("mA", C.c_double * 10),
                ("mE", C.c_double * 10), ("compare", C.c_int32), ("quad", C.c_double),
                ("cslot", C.c_int32), ("jslot", C.c_int32), ("lslot", C.c_int32),
                ("cross", C.c_double)]


_libs = {}


def lib(precision: str = "f64"):
    """The oracle library: precision "f64" (default) or "ld" (long double)."""
    if precision not in _libs:
        build()
        L = C.CDLL(_LIB if precision == "f64" else _LIB_LD)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Scene)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_step.argtypes = [C.c_void_p, C.c_long]
        L.or_moments.argtypes = [C.c_void_p, C.c_void_p]
        L.or_moment_width.argtypes = [C.c_void_p]
        L.or_populations.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_set_populations.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_num_links.argtypes = [C.c_void_p]
        L.or_get_links.argtypes = [C.c_void_p, C.c_void_p]
        L.or_get_mask.argtypes = [C.c_void_p, C.c_void_p]
        L.or_time.argtypes = [C.c_void_p]
        L.or_time.restype = C.c_long
        L.or_init_fields.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.or_link_eval.argtypes = [C.POINTER(LinkIn)]
        L.or_link_eval.restype = C.c_double
        L.or_segment_sum.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.or_segment_sum.restype = C.c_double
        L.or_lattice_table.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_double), C.c_void_p]
        L.or_equilibria.argtypes = [C.c_int, C.c_double, C.c_void_p, C.c_double, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        assert L.or_sizeof_link() == C.sizeof(Link)
        assert L.or_sizeof_link_in() == C.sizeof(LinkIn)
        assert L.or_sizeof_scene() == C.sizeof(_Scene)
        assert L.or_sizeof_boundary() == C.sizeof(_Boundary)
        assert L.or_real_bytes() == (8 if precision == "f64" else 16)
        _libs[precision] = L
    return _libs[precision]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def lattice_table(name: str):
    """(e [Q,3] int, w [Q], c2, opp [Q]) of the oracle's lattice ``name``."""
    code = S.LATTICE_CODES[name]
    Q = C.c_int()
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    c2 = C.c_double()
    lib().or_lattice_table(code, C.byref(Q), _ptr(e), _ptr(w), C.byref(c2), _ptr(opp))
    q = Q.value
    return e[:q].copy(), w[:q].copy(), c2.value, opp[:q].copy()


def equilibria(name: str, rho: float, u, C_: float = 0.0, B=(0.0, 0.0, 0.0)):
    """(f_eq, h_eq, g_eq[Q,3]) of the oracle on lattice ``name``."""
    e, w, c2, opp = lattice_table(name)
    Q = len(w)
    u = np.asarray(u, float).reshape(3)
    B = np.asarray(B, float).reshape(3)
    f = np.zeros(Q)
    h = np.zeros(Q)
    g = np.zeros((Q, 3))
    lib().or_equilibria(S.LATTICE_CODES[name], rho, _ptr(u), C_, _ptr(B), _ptr(f), _ptr(h), _ptr(g))
    return f, h, g


def link_eval(**kw) -> float:
    """Evaluates the oracle's boundary-link formula on explicit inputs.

    Keywords: lattice (name), kind (name), dir, d, x_ap_E, x_ap_A, x_a_A,
    mA, mE (vectors rho, u, C_0, B, C_1, C_2), value, a1, quad, a3, weight,
    u_w, u_given, comp_axis; FLUX of several components: cslot (moment slot
    of the link's component, 4 by default), jslot, lslot (of the bilinear
    term's components, -1 none) and cross.
    """
    li = LinkIn()
    li.lattice = S.LATTICE_CODES[kw.get("lattice", "D2Q9")]
    li.kind = S.KIND_CODES[kw["kind"]]
    li.dir = kw["dir"]
    li.comp_axis = kw.get("comp_axis", 0)
    li.u_given = int(kw.get("u_given", True))
    li.compare = int(kw.get("compare", False))
    li.d = kw["d"]
    for k in ("value", "a1", "quad", "a3", "x_ap_E", "x_ap_A", "x_a_A"):
        setattr(li, k, float(kw.get(k, 0.0)))
    li.weight = float(kw.get("weight", 1.0))
    li.cslot = int(kw.get("cslot", 4))
    li.jslot = int(kw.get("jslot", -1))
    li.lslot = int(kw.get("lslot", -1))
    li.cross = float(kw.get("cross", 0.0))
    for i, v in enumerate(kw.get("u_w", (0.0, 0.0, 0.0))):
        li.u_w[i] = v
    for i, v in enumerate(kw.get("mA", [1.0] + [0.0] * 7)):
        li.mA[i] = v
    for i, v in enumerate(kw.get("mE", [1.0] + [0.0] * 7)):
        li.mE[i] = v
    return lib().or_link_eval(C.byref(li))


class _SceneHolder:
    """Keeps the ctypes structures (and profile arrays) of a scene alive."""

    def __init__(self, sc: S.Scene):
        self.keep = []
        cs = _Scene()
        cs.dim = sc.dim
        for k in range(3):
            cs.n[k] = sc.n[k]
            cs.periodic[k] = int(sc.periodic[k])
            cs.B_ext[k] = sc.B_ext[k]
            cs.accel[k] = sc.accel[k]
        cs.fl = S.LATTICE_CODES[sc.fluid_lattice]
        cs.sl = S.LATTICE_CODES[sc.scalar_lattice] if sc.scalar_lattice else 0
        cs.ml = S.LATTICE_CODES[sc.mag_lattice] if sc.mag_lattice else 0
        cs.ncomp = len(sc.mag_comps)
        for i, c in enumerate(sc.mag_comps):
            cs.comps[i] = c
        cs.tau_f, cs.tau_c, cs.tau_m = sc.tau_f, sc.tau_c, sc.tau_m
        cs.ns = sc.scalar_ncomp if sc.scalar_lattice else 0
        for k in range(max(cs.ns, 1)):
            cs.tau_s[k] = sc.tau_scalar(k)
        cs.rho0, cs.C0, cs.mu, cs.init_C = sc.rho0, sc.C0, sc.mu, sc.init_C
        arr = (_Boundary * max(1, len(sc.boundaries)))()
        for i, b in enumerate(sc.boundaries):
            cb = arr[i]
            cb.type = {"plane": 0, "cylinder": 1, "box": 2}[b.type]
            cb.axis, cb.side, cb.is_open, cb.q, cb.radius = b.axis, b.side, int(b.is_open), b.q, b.radius
            for k in range(3):
                cb.center[k] = b.center[k]
                cb.u_w[k] = b.u_w[k]
            cb.omega = sc.wall_omega if b.u_osc else 0.0
            cb.d_used = b.d_scheme
            for k in range(3):
                cb.lo[k], cb.hi[k] = b.lo[k], b.hi[k]
            self._bc(cb.f, b.f)
            for k in range(3):
                self._bc(cb.h[k], b.h_of(k) if k < max(sc.scalar_ncomp, 1) else None)
            for k in range(3):
                self._bc(cb.g[k], b.g[k] if k < len(b.g) else None)
        cs.nb = len(sc.boundaries)
        cs.b = C.cast(arr, C.POINTER(_Boundary))
        self.keep.append(arr)
        self.cs = cs

    def _bc(self, dst: _BC, bc: Optional[S.BC]):
        if bc is None:
            dst.kind = 0
            return
        dst.kind = S.KIND_CODES[bc.kind]
        dst.u_given = int(bc.u_given)
        dst.alt = int(bc.alt)
        dst.law = _LAWS[bc.law]
        dst.value, dst.a1, dst.a3, dst.quad = bc.value, bc.a1, bc.a3, bc.quad
        dst.k, dst.phi_eq, dst.c_w, dst.H = bc.k, bc.phi_eq, bc.c_w, bc.H
        dst.profile_axis = bc.profile_axis
        dst.cj, dst.cl = bc.cross_comps
        dst.cross = bc.cross
        if bc.profile is not None:
            p = np.ascontiguousarray(bc.profile, dtype=np.float64)
            self.keep.append(p)
            dst.profile = p.ctypes.data_as(C.POINTER(C.c_double))
            dst.profile_len = len(p)
        else:
            dst.profile_len = 0


class OracleSim:
    """Plain FP64 simulation of a scene (one node at a time, paper order)."""

    FIELDS = ("rho", "ux", "uy", "uz", "C", "Bx", "By", "Bz")

    def __init__(self, sc: S.Scene, precision: str = "f64"):
        self.scene = sc
        self.precision = precision
        self._L = lib(precision)
        self._h = _SceneHolder(sc)
        p = self._L.or_create(C.byref(self._h.cs))
        if not p:
            raise ValueError("oracle: scene has a boundary link with no boundary condition")
        self._p = C.c_void_p(p)
        self.shape = (sc.n[2], sc.n[1], sc.n[0])
        self.N = sc.nodes
        if any(x is not None for x in (sc.init_rho, sc.init_u, sc.init_Cf, sc.init_B)):
            self.init_fields(sc.init_rho, sc.init_u, sc.init_Cf, sc.init_B)

    def __del__(self):
        try:
            self._L.or_destroy(self._p)
        except Exception:
            pass

    def init_fields(self, rho=None, u=None, C_=None, B=None):
        conv = lambda a, k: None if a is None else np.ascontiguousarray(
            np.asarray(a, np.float64).reshape(self.N * k))
        ns = self.scene.scalar_ncomp if self.scene.scalar_lattice else 1
        arrs = [conv(rho, 1), conv(u, 3), conv(C_, ns), conv(B, 3)]
        ptrs = [None if a is None else _ptr(a) for a in arrs]
        self._L.or_init_fields(self._p, *ptrs)

    def step(self, n: int = 1):
        self._L.or_step(self._p, int(n))

    @property
    def t(self) -> int:
        return self._L.or_time(self._p)

    def moments(self) -> np.ndarray:
        """[nz, ny, nx, W] array of rho, u(3), C_0, B(3), then C_1, C_2 of
        several scalar components (W = 8 + components - 1); zeros at solid
        nodes."""
        W = self._L.or_moment_width(self._p)
        out = np.zeros((self.N, W))
        self._L.or_moments(self._p, _ptr(out))
        return out.reshape(self.shape + (W,))

    def populations(self, field: int) -> np.ndarray:
        sc = self.scene
        Q = {0: sc.fluid_lattice, 1: sc.scalar_lattice, 2: sc.mag_lattice}[field]
        q = len(lattice_table(Q)[1])
        nc = len(sc.mag_comps) if field == 2 else (sc.scalar_ncomp if field == 1 else 1)
        out = np.zeros(nc * q * self.N)
        if self._L.or_populations(self._p, field, _ptr(out)) != 0:
            raise ValueError(field)
        if field == 2 or (field == 1 and nc > 1):
            return out.reshape((nc, q) + self.shape)
        return out.reshape((q,) + self.shape)

    def set_populations(self, field: int, arr: np.ndarray):
        a = np.ascontiguousarray(arr, np.float64)
        self._L.or_set_populations(self._p, field, _ptr(a))

    def links(self) -> np.ndarray:
        n = self._L.or_num_links(self._p)
        out = (Link * max(n, 1))()
        self._L.or_get_links(self._p, out)
        dt = np.dtype([("A", "i4"), ("E", "i4"), ("field", "i4"), ("comp", "i4"), ("dir", "i4"),
                       ("kind", "i4"), ("bnd", "i4"), ("u_given", "i4"), ("d", "f8"),
                       ("value", "f8"), ("a1", "f8"), ("a3", "f8"), ("weight", "f8"),
                       ("u_w", "f8", 3), ("omega", "f8"), ("compare", "i4"), ("pad", "i4"),
                       ("quad", "f8"), ("cj", "i4"), ("cl", "i4"), ("cross", "f8")])
        assert dt.itemsize == C.sizeof(Link)
        return np.frombuffer(bytes(out), dtype=dt, count=n).copy()

    def mask(self) -> np.ndarray:
        out = np.zeros(self.N, np.uint8)
        self._L.or_get_mask(self._p, _ptr(out))
        return out.reshape(self.shape)

    def segment_sum(self):
        n = C.c_int()
        s = self._L.or_segment_sum(self._p, C.byref(n))
        return s, n.value
