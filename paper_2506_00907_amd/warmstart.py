"""Learned warm start for batches of duct / pipe cross-sections.

The network of lbm_nn_* sees six maps of a cross-section on a fixed S x S
canvas (the section at the top-left corner, rows = z, columns = y): the fluid
mask, the distance to the nearest solid node over the half-width L, the
Hartmann number / 50, log10 of the wall conductance ratio / 3, and the
position relative to the section's centre over L along y (the applied field's
direction, across which the induced field changes sign) and along z, all on
fluid nodes.  It predicts the axial velocity and the induced axial field
scaled in the manner of Eq. 47, with a reference velocity known from the
inputs in place of the mean velocity (not known before solving),
U_ref = g L^2 / (nu (2 + Ha)), which follows the centre speed from the
Poiseuille limit (Ha = 0) to the Hartmann limit (u ~ g L^2 / (nu Ha)):

    u* = u_x / U_ref,      B* = b_x / (U_ref sqrt(rho0 nu mu / eta)).

A prediction becomes an initial state through lbm_init (equilibria of
rho0, u = (u_x, 0, 0), B = B_ext + (b_x, 0, 0)); the lattice update then runs
to convergence from there, so the network changes only where the iteration
starts.  Host-side work here is input preparation (distance transform) and
argument marshalling; every lattice step, network layer and optimiser update
runs in the HIP library.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np

IN_CH, OUT_CH = 6, 2


def _nu_eta(sc):
    return (sc.tau_f - 0.5) / 3.0, (sc.tau_m - 0.5) / 4.0


def half_width(item) -> float:
    """L: the pipe radius, or the smaller half-side of a duct (Section 5's H)."""
    sc = item.scene
    if item.shape == "pipe":
        return float(sc.boundaries[0].radius)
    qy0, qy1, qz0, qz1 = item.q
    return min((item.ny - 1 + qy0 + qy1) / 2.0, (item.nz - 1 + qz0 + qz1) / 2.0)


def scales(item):
    """(U_ref, B_ref) of an item."""
    sc = item.scene
    nu, eta = _nu_eta(sc)
    L = half_width(item)
    U = sc.accel[0] * L * L / (nu * (2.0 + item.Ha))
    return U, U * math.sqrt(sc.rho0 * nu * sc.mu / eta)


def section(a: np.ndarray) -> np.ndarray:
    """[nz, ny, 1, ...] domain array -> [nz, ny, ...] cross-section."""
    return a[:, :, 0]


def features(item, mask: np.ndarray, size: int = 256) -> np.ndarray:
    """input maps [size, size, 4] (float32) of one item; mask is the domain
    fluid mask [nz, ny, 1] (or flat)."""
    from scipy import ndimage
    m = section(np.asarray(mask, bool).reshape(item.nz, item.ny, 1))
    nz, ny = m.shape
    if nz > size or ny > size:
        raise ValueError("cross-section larger than the canvas")
    x = np.zeros((size, size, IN_CH), np.float32)
    L = half_width(item)
    dist = ndimage.distance_transform_edt(np.pad(m, 1))[1:-1, 1:-1]
    c = float(np.exp(np.mean(np.log(item.c_eff))))
    zz, yy = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    x[:nz, :ny, 0] = m
    x[:nz, :ny, 1] = np.where(m, dist / L, 0.0)
    x[:nz, :ny, 2] = np.where(m, item.Ha / 50.0, 0.0)
    x[:nz, :ny, 3] = np.where(m, math.log10(c) / 3.0, 0.0)
    x[:nz, :ny, 4] = np.where(m, (yy - (ny - 1) / 2.0) / L, 0.0)
    x[:nz, :ny, 5] = np.where(m, (zz - (nz - 1) / 2.0) / L, 0.0)
    return x


def targets(item, mask: np.ndarray, moments: np.ndarray, size: int = 256):
    """(target [size, size, 2], weight [size, size]) from converged moments
    [nz, ny, nx, 8] (rho, u, C, B); the weight is the fluid mask over the
    number of fluid nodes."""
    m = section(np.asarray(mask, bool).reshape(item.nz, item.ny, 1))
    U, Bs = scales(item)
    mom = section(moments)
    t = np.zeros((size, size, OUT_CH), np.float32)
    w = np.zeros((size, size), np.float32)
    nz, ny = m.shape
    t[:nz, :ny, 0] = np.where(m, mom[..., 1] / U, 0.0)
    t[:nz, :ny, 1] = np.where(m, (mom[..., 5] - item.scene.B_ext[0]) / Bs, 0.0)
    w[:nz, :ny] = m / max(int(m.sum()), 1)
    return t, w


def init_fields(item, mask: np.ndarray, pred: np.ndarray):
    """(u [nz, ny, 1, 3], B [nz, ny, 1, 3]) for lbm_init from a prediction
    [size, size, 2]; zero velocity and the applied field on solid nodes."""
    m = np.asarray(mask, bool).reshape(item.nz, item.ny, 1)
    U, Bs = scales(item)
    nz, ny = item.nz, item.ny
    u = np.zeros((nz, ny, 1, 3))
    B = np.zeros((nz, ny, 1, 3)) + np.asarray(item.scene.B_ext, float)
    u[..., 0] = np.where(m, pred[:nz, :ny, 0:1] * U, 0.0)
    B[..., 0] = np.where(m, item.scene.B_ext[0] + pred[:nz, :ny, 1:2] * Bs, item.scene.B_ext[0])
    return u, B


def thin_wall_shift(item, links, B):
    """B [nz, ny, nx, 3] with the constant added to its induced axial field
    b_x that makes the start satisfy the steady balance of the thin walls.

    Collision and streaming conserve sum(b_x); only the wall links change it,
    each by its flux weight times a1 (b_X - a3/a1) (Eq. 30 with the Eq. 48
    split, a1 = -eta / (c_w H)).  At the steady state these fluxes cancel, so
    sum_links weight b_X = 0, b_X being the Eq. 13 extrapolation of b to the
    wall.  A uniform offset of b_x relaxes only through these fluxes, at a
    rate of about eta / (c_w H^2) per step (2e-6 for c_w = 10 and H = 64), far
    slower than any other mode, so a start that misses the balance keeps its
    offset long after the residual is small.  Adding c to b_x adds c to every
    b_X; c = -sum w b_X / sum w restores the balance.  Other fields and the
    rest of b_x are unchanged."""
    sel = (links["field"] == 2) & (links["kind"] == 7)
    if not sel.any():
        return B
    L = links[sel]
    w = L["weight"]
    if not np.any(w != 0.0):
        return B
    b = (np.asarray(B)[..., 0] - item.scene.B_ext[0]).reshape(-1)
    A = L["node"].astype(np.int64)
    E = np.where((L["flags"] & 2) != 0, A, L["enode"].astype(np.int64))
    d = L["d"]
    bX = -d * b[E] + (1.0 + d) * b[A]
    c = -float(np.sum(w * bX) / np.sum(w))
    out = np.array(B, dtype=float, copy=True)
    out[..., 0] += c
    return out


# ---------------------------------------------------------------------------
# solving many items with the batch
# ---------------------------------------------------------------------------
def solve(items, storage: str = "f16", tol: float = 1e-8, interval: int = 1000, max_steps: int = 2_000_000,
          chunk: int = 20_000, inits: Optional[list] = None, tune: bool = True, log=print,
          max_seconds: float = float("inf"), stall: Optional[float] = None, retune: bool = True):
    """Runs every item to its steady state with lbm_batch_run in chunks of
    `chunk` steps (items that finish are disabled between chunks).
    inits[i] = (u, B) initial fields or None for rest; the solve also stops
    after max_seconds (checked between chunks).  With stall = s, an item whose
    residual fell by less than the factor s over a chunk (the noise floor of
    its storage format, or the mass drift of interpolated walls) stops with
    status "stalled".  With tune and retune, the launch configuration is
    tuned at the start and tuned again whenever the active items have halved
    (a few large items left run best with other tiles than the full batch).
    Returns a dict with per-item steps, residuals and statuses, the batch
    (for readback), the wall time of the solve (synchronised, excluding
    set-up) and the configurations tuned."""
    import torch
    from . import lbm
    scs = [it.scene.with_(storage=storage) for it in items]
    B = lbm.Batch(scs, init=False)
    for i, lat in enumerate(B.items):
        if inits is not None and inits[i] is not None:
            u, Bf = inits[i]
            lat.init(None, u, None, Bf)
        else:
            lat.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = []
    if tune:
        tuned.append(dict(active=len(items), config=B.tune(trial_steps=64)[0]))
    n = len(items)
    n_tuned = n
    steps = np.zeros(n, np.int64)
    res = np.full(n, -1.0)
    status = ["active"] * n
    start_t = np.array([it.time for it in B.items])
    done = 0
    while done < max_steps and time.perf_counter() - t0 < max_seconds:
        active = [s == "active" for s in status]
        if not any(active):
            break
        B.set_active(active)
        k = min(chunk, max_steps - done)
        st, rs, ss = B.run(tol=tol, interval=interval, max_steps=k)
        for i in range(n):
            if active[i]:
                prev = res[i]
                res[i] = rs[i]
                status[i] = ss[i]
                if stall is not None and ss[i] == "active" and prev > 0 and rs[i] > stall * prev:
                    status[i] = "stalled"
        done += k
        n_act = sum(s == "active" for s in status)
        if tune and retune and 0 < n_act <= n_tuned // 2 and done < max_steps:
            B.set_active([s == "active" for s in status])
            tuned.append(dict(active=n_act, config=B.tune(trial_steps=64)[0]))
            n_tuned = n_act
        log(f"  [{storage}] {done} steps: {n - n_act}/{n} items finished, "
            f"max residual of the rest {max([r for r, s in zip(res, status) if s == 'active'] or [0]):.2e}, "
            f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = np.array([it.time for it in B.items]) - start_t
    return dict(batch=B, steps=steps, residual=res, status=status, seconds=wall, tuned=tuned)


def moments_of(B) -> List[np.ndarray]:
    return [lat.read_moments("f64").cpu().numpy().transpose(1, 2, 3, 0) for lat in B.items]


# ---------------------------------------------------------------------------
# network training and inference
# ---------------------------------------------------------------------------
def he_init(seed: int, width: int = 32):
    """He-normal weights and small biases from SplitMix64 (layer shapes as in
    lbm.h: W[c_out][c_in][ky][kx] then b per layer)."""
    from scenes import SplitMix64
    rng = SplitMix64(seed)
    w = width
    shapes = [(IN_CH, w, 3), (w, w, 3), (w, 2 * w, 3), (2 * w, 2 * w, 3), (2 * w, 4 * w, 3), (4 * w, 4 * w, 3),
              (6 * w, 2 * w, 3), (2 * w, 2 * w, 3), (3 * w, w, 3), (w, w, 3), (w, OUT_CH, 1)]
    parts = []
    for ci, co, k in shapes:
        parts.append(rng.normal_array(co * ci * k * k) * math.sqrt(2.0 / (ci * k * k)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def train(X, T, Wt, epochs: int = 20, batch: int = 16, lr: float = 1e-3, seed: int = 7, size: int = 256,
          log=print, net=None):
    """Trains on device tensors X [n, S, S, 4], T [n, S, S, 2], Wt [n, S, S]
    (weights: mask / fluid count); returns (network, loss history)."""
    import torch
    from . import lbm
    from scenes import SplitMix64
    n = X.shape[0]
    if net is None:
        net = lbm.Network(batch, size, in_ch=IN_CH, out_ch=OUT_CH)
        net.set_params(he_init(seed))
    rng = SplitMix64(seed + 1)
    hist = []
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    it = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.as_tensor(np.argsort(rng.uniform_array(n)), device=X.device)
        ep_loss = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            net.forward(X[idx])
            # the loss weights are per image; a mean over the minibatch
            ep_loss += net.backward(T[idx], Wt[idx] / batch)
            # cosine decay of the learning rate
            net.adam_step(lr * 0.5 * (1.0 + math.cos(math.pi * it / total)))
            it += 1
        hist.append(ep_loss / steps_per_epoch)
        log(f"  epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return net, hist


def predict(net, X, batch: int = 16):
    import torch
    out = []
    for s in range(0, X.shape[0], batch):
        out.append(net.forward(X[s:s + batch]).clone())
    return torch.cat(out)
