"""Stokes' second problem at the paper's size (Section 5.2, Eq. 45).

    python -m paper_2506_00907_amd.stokes_study [--storage f64] [--out DIR]

Three-dimensional D3Q19 runs, 5 x 5 nodes periodic in x and y, a static wall
below and a wall above that moves in x at U cos(omega t), period T = 1e5
steps, H = 100 lattice spacings between the walls, both relaxation times of
the paper (tau = 0.53 and 0.8 for the same physical viscosity, so U = 1e-4
and 1e-3 in lattice units) and three layouts:

  half      walls half a spacing outside the outer nodes (d = 0.5, 100 rows)
  full      walls on the outer grid layers (d = 1, 99 fluid rows)
  mismatch  the full layout run with the d = 0.5 scheme

All six cases advance together as one batch from rest.  The profile u_x(z)
after 2T and 3T shows that the periodic state is reached; eight phases of the
fourth period are compared with the closed form.  The mismatch case is also
compared with the closed form for walls half a spacing from the outer nodes,
where the d = 0.5 scheme puts them.  Writes stokes.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenes  # noqa: E402
from paper_2506_00907_amd import lbm  # noqa: E402

PERIOD = 100_000
H = 100
LAYOUTS = {"half": (0.5, 0.0), "full": (1.0, 0.0), "mismatch": (1.0, 0.5)}  # q, d_scheme
TAUS = {0.53: 1e-4, 0.8: 1e-3}  # tau -> U in lattice units (c = dx/dt of each case)


def closed_form(y, t, U, omega, nu, h):
    """u_x between a wall at rest at y = 0 and one at y = h moving at
    U cos(omega t), periodic state: Re[U e^{i omega t} sinh(k y)/sinh(k h)]
    with k = (1 + i) sqrt(omega / (2 nu))."""
    k = (1.0 + 1.0j) * math.sqrt(omega / (2.0 * nu))
    return np.real(U * np.exp(1j * omega * t) * np.sinh(k * y) / np.sinh(k * h))


def cases(storage):
    out = []
    for tau, U in TAUS.items():
        for name, (q, ds) in LAYOUTS.items():
            rows = int(round(H + 1 - 2 * q))
            sc = scenes.stokes_second(nx=5, ny=rows, tau=tau, U=U, period=PERIOD, q=q, storage=storage,
                                      dim=3, d_scheme=ds)
            out.append(dict(name=name, tau=tau, U=U, q=q, rows=rows, scene=sc))
    return out


def profile(item):
    m = item.read_moments("f64").cpu().numpy()
    return m[1].mean(axis=(1, 2))  # u_x(z), the same on every (x, y)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--phases", type=int, default=8)
    ap.add_argument("--out", default="stokes_out")
    a = ap.parse_args(argv)
    import torch

    cs = cases(a.storage)
    B = lbm.Batch([c["scene"] for c in cs])
    best, _ = B.tune(128)
    B.configure(**best)
    print(f"{len(cs)} items, config {best}", flush=True)
    # back to the rest state at t = 0 after tuning
    B = lbm.Batch([c["scene"] for c in cs])
    B.configure(**best)
    omega = 2.0 * math.pi / PERIOD
    nodes = sum(c["scene"].nodes for c in cs)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(2 * PERIOD)
    p2 = [profile(it) for it in B.items]
    B.step(PERIOD)
    p3 = [profile(it) for it in B.items]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    print(f"3T = {3 * PERIOD} steps in {secs:.2f} s ({nodes * 3 * PERIOD / secs / 1e6:.0f} MLUPS)", flush=True)

    res = []
    errs = [[] for _ in cs]
    moved = [[] for _ in cs]
    for k in range(a.phases):
        if k:
            B.step(PERIOD // a.phases)
        t = 3 * PERIOD + k * (PERIOD // a.phases)
        for i, (c, it) in enumerate(zip(cs, B.items)):
            nu = (c["tau"] - 0.5) / 3.0
            u = profile(it)
            z = np.arange(c["rows"]) + c["q"]
            errs[i].append(rel(u, closed_form(z, t, c["U"], omega, nu, H)))
            if c["name"] == "mismatch":
                moved[i].append(rel(u, closed_form(z - 0.5, t, c["U"], omega, nu, H - 1)))
    for i, c in enumerate(cs):
        nu = (c["tau"] - 0.5) / 3.0
        r = dict(layout=c["name"], tau=c["tau"], U=c["U"], rows=c["rows"], q=c["q"],
                 womersley=H * math.sqrt(omega / nu), err_max=max(errs[i]), err_mean=float(np.mean(errs[i])),
                 periodic_2T_3T=rel(p3[i], p2[i]))
        if moved[i]:
            r["err_wall_moved"] = max(moved[i])
        res.append(r)
        print(json.dumps(r), flush=True)
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, "stokes.json"), "w") as f:
        json.dump(dict(storage=a.storage, period=PERIOD, H=H, config=best, seconds_3T=secs,
                       mlups=nodes * 3 * PERIOD / secs / 1e6, cases=res), f, indent=1)


if __name__ == "__main__":
    main()
