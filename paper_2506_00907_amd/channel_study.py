"""The 3D channel between reservoirs at the paper's size (Section 5.1).

    python -m paper_2506_00907_amd.channel_study [--storage f64] [--out DIR]

A square channel (width 20 spacings, length 60) between two reservoirs (20
spacings each, periodic sides), D3Q19, tau = 0.7, uniform normal velocity
u_in = 0.01 at the inlet and rho = 1 at the outlet, in the half-grid (d =
0.5, 22 x 22 nodes across) and full-grid (d = 1, 21 x 21) layouts.  Each runs
from rest until u_z changes by less than tol (relative) over a chunk of
steps.  Reported per layout: the flux of the first plane against u_in times
the inlet's sum of rho(X) (Eq. 13), the channel's mean velocity (flux over
the channel's area), the largest u_z, and the middle plane against the
fully developed duct flow at the pressure gradient measured there.  The
ratio of the two layouts' channel velocities follows their inlet node counts
(22^2 / 21^2), the effect Section 5.1 points out.  Writes channel.json.
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

W, RES, CH, TAU, U_IN = 20, 20, 60, 0.7, 0.01


def duct(x, y, a, G, mu, nterms=200):
    """fully developed flow in the square duct |x|, |y| < a at pressure
    gradient -G: the cosine series solving mu (u_xx + u_yy) = -G, u = 0 on
    the walls"""
    u = np.zeros(np.broadcast(x, y).shape)
    for j in range(nterms):
        n = 2 * j + 1
        k = n * math.pi / (2.0 * a)
        ratio = (np.exp(k * (np.abs(y) - a)) + np.exp(-k * (np.abs(y) + a))) / (1.0 + math.exp(-2.0 * k * a))
        u += (-1.0) ** j / n ** 3 * (1.0 - ratio) * np.cos(k * x)
    return 16.0 * a * a * G / (mu * math.pi ** 3) * u


def run(layout, storage, tol, chunk, max_steps):
    import torch
    sc = scenes.channel_reservoirs(layout, width=W, res_len=RES, ch_len=CH, tau=TAU, u_in=U_IN, storage=storage)
    lat = lbm.Lattice(sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prev = None
    steps = 0
    change = math.inf
    while steps < max_steps:
        lat.step(chunk)
        steps += chunk
        uz = lat.read_moments("f64")[3]
        if prev is not None:
            change = float((uz - prev).abs().max() / uz.abs().max())
            if change < tol:
                break
        prev = uz
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    m = lat.read_moments("f64").cpu().numpy()
    rho, uz = m[0], m[3]
    q = 0.5 if layout == "half" else 1.0
    flux = (rho * uz).sum(axis=(1, 2))
    inflow = U_IN * (rho[0] + q * (rho[0] - rho[1])).sum()
    zc = m.shape[1] // 2
    xs = np.arange(sc.n[0]) - (1.0 - q) - W / 2
    Y, X = np.meshgrid(xs, xs, indexing="ij")  # [y][x] like the moments
    fl = (np.abs(X) < W / 2) & (np.abs(Y) < W / 2)
    G = -(rho[zc + 1][fl] - rho[zc - 1][fl]).mean() / 2.0 / 3.0
    nu = (TAU - 0.5) / 3.0
    us = duct(X, Y, W / 2, G, rho[zc][fl].mean() * nu)
    return dict(layout=layout, nodes=list(sc.n), fluid_nodes=int(lat.mask.sum()), steps=steps,
                last_change=change, seconds=secs, mlups=lat.mask.sum() * steps / secs / 1e6,
                inlet_flux_ratio=float(flux[0] / inflow), outlet_flux_ratio=float(flux[-1] / inflow),
                channel_mean_u=float(flux[zc] / rho[zc][fl].mean() / W ** 2),
                max_uz=float(uz[RES:-RES].max()),
                far_field_err=float(np.linalg.norm((uz[zc] - us)[fl]) / np.linalg.norm(us[fl])))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--max-steps", type=int, default=400_000)
    ap.add_argument("--out", default="channel_out")
    a = ap.parse_args(argv)
    res = {}
    for layout in ("half", "full"):
        res[layout] = run(layout, a.storage, a.tol, a.chunk, a.max_steps)
        print(json.dumps(res[layout]), flush=True)
    ratio = res["half"]["channel_mean_u"] / res["full"]["channel_mean_u"]
    summary = dict(storage=a.storage, mean_u_ratio_half_over_full=ratio, inlet_node_ratio=22 ** 2 / 21 ** 2,
                   cases=res)
    print(json.dumps({k: v for k, v in summary.items() if k != "cases"}), flush=True)
    os.makedirs(a.out, exist_ok=True)
    with open(os.path.join(a.out, "channel.json"), "w") as f:
        json.dump(summary, f, indent=1)


if __name__ == "__main__":
    main()
