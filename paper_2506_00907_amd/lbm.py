"""Python face of liblbm: the C-ABI calls with PyTorch device buffers.

Argument marshalling only.  PyTorch allocates the device buffers the library
asks for and supplies the HIP stream; all arithmetic runs in liblbm's kernels.
Names follow include/lbm.h: ``build_links``, ``Lattice.step``,
``Lattice.read_moments``, ``Lattice.reduce`` ...
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np

from . import _lib as L

LATTICES = {"D2Q9": 1, "D3Q19": 2, "D2Q5": 3, "D3Q7": 4}
KINDS = {"VEL": 1, "PRES": 2, "CONC": 3, "FLUX": 4, "BB0": 5, "MAG_DIR": 6, "MAG_FLUX": 7, "MAG_THETA": 8}
BOUNDARY_TYPES = {"plane": 0, "cylinder": 1, "box": 2}
STORAGES = {"f64": L.LBM_F64, "f32": L.LBM_F32, "f16": L.LBM_F16, "bf16": L.LBM_BF16}

LINK_DTYPE = np.dtype([("node", "<u4"), ("enode", "<u4"), ("field", "u1"), ("dir", "u1"), ("kind", "u1"),
                       ("comp", "u1"), ("flags", "u1"), ("cross_comp", "u1", 2), ("pad", "u1"), ("d", "<f8"),
                       ("value", "<f8"), ("a1", "<f8"), ("a3", "<f8"), ("weight", "<f8"), ("u_w", "<f8", 3),
                       ("quad", "<f8"), ("cross", "<f8")])
assert LINK_DTYPE.itemsize == C.sizeof(L.lbm_link)


def params_from_scene(sc) -> L.lbm_params:
    p = L.lbm_params()
    p.dim = sc.dim
    for k in range(3):
        p.n[k] = sc.n[k]
        p.periodic[k] = int(sc.periodic[k])
        p.B_ext[k] = sc.B_ext[k]
        p.accel[k] = sc.accel[k]
        p.store_scale[k] = sc.store_scale[k]
    p.fluid = LATTICES[sc.fluid_lattice]
    p.scalar = LATTICES[sc.scalar_lattice] if sc.scalar_lattice else 0
    p.magnetic = LATTICES[sc.mag_lattice] if sc.mag_lattice else 0
    p.mag_ncomp = len(sc.mag_comps) if sc.mag_lattice else 0
    for i, c in enumerate(sc.mag_comps):
        p.mag_comp[i] = c
    p.storage = STORAGES[sc.storage]
    p.tau_f, p.tau_c, p.tau_m = sc.tau_f, sc.tau_c, sc.tau_m
    p.scalar_ncomp = sc.scalar_ncomp if sc.scalar_lattice else 0
    for k in range(1, p.scalar_ncomp):
        p.tau_cs[k - 1] = sc.tau_scalar(k)
    p.rho0, p.C0, p.mu = sc.rho0, sc.C0, sc.mu
    p.wall_omega = sc.wall_omega
    return p


def boundaries_from_scene(sc):
    keep = []
    arr = (L.lbm_boundary * max(1, len(sc.boundaries)))()

    def put(dst, bc):
        if bc is None:
            dst.kind = 0
            return
        dst.kind = KINDS[bc.kind]
        dst.u_given = int(bc.u_given)
        dst.alt = int(bc.alt)
        dst.law = L.LAWS[bc.law]
        dst.value, dst.a1, dst.a3, dst.quad = bc.value, bc.a1, bc.a3, bc.quad
        dst.k, dst.phi_eq, dst.c_w, dst.H = bc.k, bc.phi_eq, bc.c_w, bc.H
        dst.profile_axis = bc.profile_axis
        dst.cross_comp[0], dst.cross_comp[1] = bc.cross_comps
        dst.cross = bc.cross
        if bc.profile is not None:
            prof = np.ascontiguousarray(bc.profile, dtype=np.float64)
            keep.append(prof)
            dst.profile = prof.ctypes.data_as(C.POINTER(C.c_double))
            dst.profile_len = len(prof)

    for i, b in enumerate(sc.boundaries):
        d = arr[i]
        d.type = BOUNDARY_TYPES[b.type]
        d.axis, d.side, d.is_open, d.q, d.radius = b.axis, b.side, int(b.is_open), b.q, b.radius
        d.u_osc = int(b.u_osc)
        d.d_scheme = b.d_scheme
        for k in range(3):
            d.lo[k], d.hi[k] = b.lo[k], b.hi[k]
        for k in range(3):
            d.center[k] = b.center[k]
            d.u_w[k] = b.u_w[k]
        put(d.f, b.f)
        put(d.h, b.h_of(0))
        for k in range(1, max(sc.scalar_ncomp, 1)):
            put(d.h_more[k - 1], b.h_of(k))
        for k in range(3):
            put(d.g[k], b.g[k] if k < len(b.g) else None)
    return arr, len(sc.boundaries), keep


def build_links(sc) -> Tuple[np.ndarray, np.ndarray]:
    """lbm_build_links: (fluid mask [nz, ny, nx] uint8, link table)."""
    p = params_from_scene(sc)
    arr, nb, keep = boundaries_from_scene(sc)
    n = C.c_size_t()
    mask = np.zeros(sc.nodes, np.uint8)
    L.check(L.lib().lbm_build_links(C.byref(p), arr, nb, mask.ctypes.data_as(C.c_void_p), None, 0,
                                    C.byref(n)), what="lbm_build_links (count)")
    links = np.zeros(max(n.value, 1), LINK_DTYPE)
    L.check(L.lib().lbm_build_links(C.byref(p), arr, nb, mask.ctypes.data_as(C.c_void_p),
                                    links.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
            what="lbm_build_links")
    del keep
    return mask.reshape(sc.n[2], sc.n[1], sc.n[0]), links[:n.value]


def lattice_table(code: int):
    Q = C.c_int32()
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    c2 = C.c_double()
    L.check(L.lib().lbm_lattice_table(code, C.byref(Q), e.ctypes.data_as(C.c_void_p),
                                      w.ctypes.data_as(C.c_void_p), C.byref(c2),
                                      opp.ctypes.data_as(C.c_void_p)), what="lbm_lattice_table")
    q = Q.value
    return e[:q].copy(), w[:q].copy(), c2.value, opp[:q].copy()


def required_bytes(p: L.lbm_params, n_links: int):
    sizes = (C.c_size_t * L.LBM_NBUF)()
    tot = L.lib().lbm_required_bytes(C.byref(p), n_links, sizes)
    if tot == 0:
        raise L.LbmError(-1, "invalid parameters")
    return list(sizes)


def stream_bandwidth(kind: str, nbytes: int, per_thread: int = 4, reps: int = 10, device="cuda:0"):
    """lbm_stream_bandwidth: mean ms per launch of a plain 16-byte-access
    read, write or copy kernel over nbytes (torch-allocated buffers)."""
    import torch
    k = {"read": 0, "write": 1, "copy": 2}[kind]
    dev = torch.device(device)
    src = torch.ones(nbytes // 4 if k != 1 else 1, dtype=torch.int32, device=dev)
    dst = torch.zeros(nbytes // 4 if k != 0 else 4, dtype=torch.int32, device=dev)
    out = C.c_float()
    stream = torch.cuda.current_stream(dev)
    code = L.lib().lbm_stream_bandwidth(k, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), int(nbytes),
                                        int(per_thread), int(reps), C.c_void_p(stream.cuda_stream), C.byref(out))
    L.check(code)
    return float(out.value)


def _torch_device(torch, device):
    if not torch.cuda.is_available():
        raise RuntimeError("liblbm needs a HIP device")
    return torch.device(device)


def _pool(torch, device, sizes):
    bufs = [torch.empty(max(s, 1), dtype=torch.uint8, device=device) for s in sizes]
    ptrs = (C.c_void_p * L.LBM_NBUF)(*[b.data_ptr() if s > 0 else None for b, s in zip(bufs, sizes)])
    return bufs, ptrs


class Lattice:
    """One context of the fused coupled sweep on a torch device and stream."""

    def __init__(self, sc, device: str = "cuda", stream=None, links: Optional[np.ndarray] = None,
                 mask: Optional[np.ndarray] = None, init: bool = True, _ctx=None, _owner=None):
        import torch
        self.torch = torch
        self.device = _torch_device(torch, device)
        self.scene = sc
        self.params = params_from_scene(sc)
        if links is None or mask is None:
            mask, links = build_links(sc)
        self.mask = np.ascontiguousarray(mask, np.uint8).reshape(-1)
        self.links = np.ascontiguousarray(links)
        self.n_links = len(self.links)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._owner = _owner
        if _ctx is None:
            self.sizes = required_bytes(self.params, self.n_links)
            self.bufs, ptrs = _pool(torch, self.device, self.sizes)
            ctx = C.c_void_p()
            L.check(L.lib().lbm_create(C.byref(self.params), self.n_links, ptrs,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), what="lbm_create")
            self.ctx = ctx
        else:
            self.ctx = _ctx  # an item of a Batch (owned by it)
        self._call("lbm_set_geometry", self.mask.ctypes.data_as(C.c_void_p))
        self._call("lbm_set_links", self.links.ctypes.data_as(C.c_void_p), self.n_links)
        self.N = sc.nodes
        self.shape = (sc.n[2], sc.n[1], sc.n[0])
        self.n_scalar = max(int(self.params.scalar_ncomp), 1)
        self.moment_width = 8 + self.n_scalar - 1
        if init:
            self.init(sc.init_rho, sc.init_u, sc.init_Cf, sc.init_B, C_uniform=sc.init_C)

    def _call(self, name, *args):
        L.check(getattr(L.lib(), name)(self.ctx, *args), self.ctx)

    def __del__(self):
        try:
            if getattr(self, "ctx", None) and self._owner is None:
                L.lib().lbm_destroy(self.ctx)
            self.ctx = None
        except Exception:
            pass

    # -- ABI calls ----------------------------------------------------------
    def init(self, rho=None, u=None, C_=None, B=None, C_uniform: Optional[float] = None):
        """lbm_init from fields (arrays of the domain shape; u, B with a last
        axis of 3; C of several scalar components with a first axis of
        components) or the uniform rest state; C_uniform fills C when given."""
        torch = self.torch
        N = self.N

        def dev(a, comps):
            if a is None:
                return None
            t = torch.as_tensor(np.asarray(a, np.float64))
            if comps == 1:
                t = t.reshape(N)
            else:
                t = t.reshape(N, 3).t().contiguous()
            return t.to(self.device)

        ns = self.n_scalar
        tr, tu, tB = dev(rho, 1), dev(u, 3), dev(B, 3)
        tC = None if C_ is None else torch.as_tensor(np.asarray(C_, np.float64)).reshape(ns * N).to(self.device)
        if tC is None and C_uniform is not None and C_uniform != self.params.C0:
            tC = torch.full((ns * N,), float(C_uniform), dtype=torch.float64, device=self.device)
        self._keep_init = (tr, tu, tC, tB)
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        self._call("lbm_init", ptr(tr), ptr(tu), ptr(tC), ptr(tB))

    def step(self, n: int = 1):
        self._call("lbm_step", int(n))

    def step_prepare(self, n: int):
        """lbm_step_prepare: capture the graphs a later step(n) replays."""
        self._call("lbm_step_prepare", int(n))

    def set_step_overlap(self, mode: int):
        """lbm_set_step_overlap: 0 links then the whole sweep (default), 1 the
        next step's link kernel beside the sweep of the waves without links."""
        self._call("lbm_set_step_overlap", int(mode))

    def step_stats(self):
        """lbm_step_stats: (graph replays, steps inside them, single steps)."""
        out = (C.c_int64 * 3)()
        self._call("lbm_step_stats", out)
        return int(out[0]), int(out[1]), int(out[2])

    def step_timed(self, n: int):
        """lbm_step_timed: mean (link kernel, sweep kernel) durations in ms.
        The state is saved into a torch-allocated scratch buffer of
        lbm_timing_scratch_bytes and restored from it."""
        nbytes = L.lib().lbm_timing_scratch_bytes(self.ctx)
        scratch = self.torch.empty(max(nbytes, 1), dtype=self.torch.uint8, device=self.device)
        out = (C.c_float * 2)()
        self._call("lbm_step_timed", int(n), C.c_void_p(scratch.data_ptr()), nbytes, out)
        del scratch
        return float(out[0]), float(out[1])

    @property
    def time(self) -> int:
        return L.lib().lbm_time(self.ctx)

    def read_moments(self, dtype: str = "f64", out=None):
        """[W, nz, ny, nx] tensor of rho, u, C_0, B, then C_1, C_2 of several
        scalar components (W = 8 + components - 1), at the current time."""
        torch = self.torch
        td = torch.float64 if dtype == "f64" else torch.float32
        if out is None:
            out = torch.empty((self.moment_width,) + self.shape, dtype=td, device=self.device)
        self._call("lbm_read_moments", C.c_void_p(out.data_ptr()), L.LBM_F64 if dtype == "f64" else L.LBM_F32)
        return out

    def read_populations(self, field: int):
        """[slots, nz, ny, nx] FP64 tensor of one field's populations."""
        torch = self.torch
        sc = self.scene
        lat = {0: sc.fluid_lattice, 1: sc.scalar_lattice, 2: sc.mag_lattice}[field]
        q = len(lattice_table(LATTICES[lat])[1])
        nc = len(sc.mag_comps) if field == 2 else (self.n_scalar if field == 1 else 1)
        out = torch.empty((nc * q,) + self.shape, dtype=torch.float64, device=self.device)
        self._call("lbm_read_populations", field, C.c_void_p(out.data_ptr()))
        return out

    def reduce(self, static_scratch: bool = False) -> np.ndarray:
        """lbm_reduce (static_scratch: lbm_reduce_static, the variant whose
        scratch is the library's own device array)."""
        out = (C.c_double * 8)()
        fn = L.lib().lbm_reduce_static if static_scratch else L.lib().lbm_reduce
        code = fn(self.ctx, out)
        vals = np.array(out[:])
        if code == -4:
            raise L.LbmError(code, "non-finite values")
        L.check(code, self.ctx)
        return vals

    def read_normalised(self, axis: int = 0, U: float = 0.0):
        """lbm_read_normalised: [2, nz, ny, nx] FP64 tensor of u* and B* along
        `axis` (U = 0: scaled by the mean velocity over the fluid nodes)."""
        torch = self.torch
        out = torch.empty((2,) + self.shape, dtype=torch.float64, device=self.device)
        self._call("lbm_read_normalised", int(axis), float(U), C.c_void_p(out.data_ptr()))
        return out

    def boundary_flux(self) -> np.ndarray:
        """lbm_boundary_flux: net inflow through the boundary links over the
        last step: mass, solute, B_x, B_y, B_z."""
        out = (C.c_double * 5)()
        self._call("lbm_boundary_flux", out)
        return np.array(out[:])

    def scalar_flux(self) -> np.ndarray:
        """lbm_boundary_flux_scalar: net inflow of each scalar component
        through the boundary links over the last step."""
        out = (C.c_double * 3)()
        self._call("lbm_boundary_flux_scalar", out)
        return np.array(out[:self.n_scalar])

    def save(self) -> bytes:
        nb = L.lib().lbm_state_bytes(self.ctx)
        buf = (C.c_char * nb)()
        self._call("lbm_save", buf)
        return bytes(buf)

    def load(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        self._call("lbm_load", buf)


class Batch:
    """lbm_batch_*: many independent scenes (one lattice combination and
    storage) advanced by shared launches.  ``items[i]`` is a Lattice view of
    item i (geometry, links, init and readback go through the single-context
    calls)."""

    def __init__(self, scs, device: str = "cuda", stream=None, init: bool = True, tables=None):
        import torch
        self.torch = torch
        self.device = _torch_device(torch, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.scenes = list(scs)
        n = len(self.scenes)
        if tables is None:
            tables = [build_links(sc) for sc in self.scenes]
        self.params = (L.lbm_params * n)(*[params_from_scene(sc) for sc in self.scenes])
        self.cap = (C.c_size_t * n)(*[len(t[1]) for t in tables])
        sizes = (C.c_size_t * L.LBM_NBUF)()
        if L.lib().lbm_batch_required_bytes(n, self.params, self.cap, sizes) == 0:
            raise L.LbmError(-1, "invalid batch (parameters, or items differ in lattices or storage)")
        self.sizes = list(sizes)
        self.bufs, ptrs = _pool(torch, self.device, self.sizes)
        b = C.c_void_p()
        L.check(L.lib().lbm_batch_create(n, self.params, self.cap, ptrs, C.c_void_p(self.stream.cuda_stream),
                                         C.byref(b)), what="lbm_batch_create")
        self.b = b
        self.items = []
        for i, (sc, (mask, links)) in enumerate(zip(self.scenes, tables)):
            ctx = C.c_void_p(L.lib().lbm_batch_item(self.b, i))
            self.items.append(Lattice(sc, device=device, stream=self.stream, links=links, mask=mask,
                                      init=init, _ctx=ctx, _owner=self))

    def _call(self, name, *args):
        code = getattr(L.lib(), name)(self.b, *args)
        if code != 0:
            raise L.LbmError(code, L.lib().lbm_batch_last_error(self.b).decode())

    def __len__(self):
        return len(self.items)

    def __del__(self):
        try:
            if getattr(self, "b", None):
                for it in self.items:
                    it.ctx = None
                L.lib().lbm_batch_destroy(self.b)
                self.b = None
        except Exception:
            pass

    @property
    def config(self) -> dict:
        c = L.lbm_batch_config()
        self._call("lbm_batch_get_config", C.byref(c))
        return dict(mode={1: "tiled", 2: "resident"}[c.mode], block=c.block,
                    steps_per_launch=c.steps_per_launch, graph_steps=c.graph_steps)

    def configure(self, mode: str = "tiled", block: int = 256, steps_per_launch: int = 1, graph_steps: int = 64):
        c = L.lbm_batch_config({"tiled": 1, "resident": 2}[mode], block, steps_per_launch, graph_steps)
        self._call("lbm_batch_configure", C.byref(c))

    def set_active(self, flags):
        """lbm_batch_set_active: which items take part in step / run / tune."""
        f = np.ascontiguousarray(np.asarray(flags, dtype=bool).astype(np.uint8))
        assert f.size == len(self.items)
        self._call("lbm_batch_set_active", f.ctypes.data_as(C.c_void_p))

    def step(self, n: int = 1):
        self._call("lbm_batch_step", int(n))

    def run(self, tol: float = 1e-8, interval: int = 100, max_steps: int = 10 ** 7):
        """lbm_batch_run: per item (steps, residual, status name)."""
        n = len(self.items)
        steps = (C.c_int64 * n)()
        res = (C.c_double * n)()
        st = (C.c_int32 * n)()
        self._call("lbm_batch_run", float(tol), int(interval), int(max_steps), steps, res, st)
        return np.array(steps[:]), np.array(res[:]), [L.ITEM_STATUS[s] for s in st[:]]

    def tune(self, trial_steps: int = 128):
        """lbm_batch_tune: (best config dict, [(config dict, ms per step)])."""
        cap = 32
        cands = (L.lbm_batch_config * cap)()
        ms = (C.c_double * cap)()
        nout = C.c_int32()
        best = L.lbm_batch_config()
        self._call("lbm_batch_tune", int(trial_steps), C.byref(best), cands, ms, cap, C.byref(nout))
        conv = lambda c: dict(mode={1: "tiled", 2: "resident"}[c.mode], block=c.block,
                              steps_per_launch=c.steps_per_launch, graph_steps=c.graph_steps)
        return conv(best), [(conv(cands[k]), ms[k]) for k in range(nout.value)]


class Network:
    """lbm_nn_*: the warm-start encoder-decoder on torch device buffers.
    Images are NHWC float32 device tensors."""

    def __init__(self, batch: int, size: int, in_ch: int = 4, out_ch: int = 2, width: int = 32,
                 precision: str = "bf16", device: str = "cuda", stream=None):
        import torch
        self.torch = torch
        self.device = _torch_device(torch, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.desc = L.lbm_nn_desc(batch, size, in_ch, out_ch, width,
                                  {"bf16": L.LBM_BF16, "f32": L.LBM_F32}[precision])
        sizes = (C.c_size_t * 4)()
        if L.lib().lbm_nn_required_bytes(C.byref(self.desc), sizes) == 0:
            raise L.LbmError(-1, "invalid network description")
        self.sizes = list(sizes)
        self.bufs = [torch.empty(s, dtype=torch.uint8, device=self.device) for s in self.sizes]
        ptrs = (C.c_void_p * 4)(*[b.data_ptr() for b in self.bufs])
        n = C.c_void_p()
        L.check(L.lib().lbm_nn_create(C.byref(self.desc), ptrs, C.c_void_p(self.stream.cuda_stream), C.byref(n)),
                what="lbm_nn_create")
        self.n = n
        self.size, self.in_ch, self.out_ch, self.batch = size, in_ch, out_ch, batch

    def _call(self, name, *args):
        code = getattr(L.lib(), name)(self.n, *args)
        if code != 0:
            raise L.LbmError(code, L.lib().lbm_nn_last_error(self.n).decode())

    def __del__(self):
        try:
            if getattr(self, "n", None):
                L.lib().lbm_nn_destroy(self.n)
                self.n = None
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(L.lib().lbm_nn_num_params(self.n))

    def _dev(self, a, shape=None):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
        if shape is not None:
            assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
        return t

    def set_params(self, theta):
        t = self._dev(theta).reshape(-1)
        assert t.numel() == self.num_params
        self._call("lbm_nn_set_params", C.c_void_p(t.data_ptr()))
        self.torch.cuda.current_stream(self.device).synchronize()

    def params(self):
        out = self.torch.empty(self.num_params, dtype=self.torch.float32, device=self.device)
        self._call("lbm_nn_get_params", C.c_void_p(out.data_ptr()))
        return out

    def grads(self):
        out = self.torch.empty(self.num_params, dtype=self.torch.float32, device=self.device)
        self._call("lbm_nn_get_grads", C.c_void_p(out.data_ptr()))
        return out

    def forward(self, x, out=None):
        """x [n, S, S, in_ch] -> y [n, S, S, out_ch]."""
        x = self._dev(x)
        n = x.shape[0]
        assert tuple(x.shape[1:]) == (self.size, self.size, self.in_ch)
        if out is None:
            out = self.torch.empty((n, self.size, self.size, self.out_ch), dtype=self.torch.float32,
                                   device=self.device)
        self._x = x  # kept alive while the launches run
        self._call("lbm_nn_forward", int(n), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
        return out

    def backward(self, target, weight, want_loss: bool = True):
        n = self._x.shape[0]
        t = self._dev(target, (n, self.size, self.size, self.out_ch))
        w = self._dev(weight, (n, self.size, self.size))
        self._tw = (t, w)
        loss = C.c_double()
        self._call("lbm_nn_backward", C.c_void_p(t.data_ptr()), C.c_void_p(w.data_ptr()),
                   C.byref(loss) if want_loss else None)
        return loss.value if want_loss else None

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._call("lbm_nn_adam_step", float(lr), float(beta1), float(beta2), float(eps))
