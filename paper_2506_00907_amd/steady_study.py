"""Time to steady state of many duct / pipe cross-sections.

    python -m paper_2506_00907_amd.steady_study train --items 4096 --out DIR
    python -m paper_2506_00907_amd.steady_study eval --weights DIR/net.npy --items 256 --out DIR

train: solves the training items (seeded, disjoint from the evaluation
items) with the FP16 batch, builds the network inputs and targets from the
converged fields and trains the warm-start network; writes net.npy and
train.json.

eval: on the evaluation items, three ways to the same steady state:
  plain  FP32 storage, one item at a time (single-context kernels, graph
         replays), rest initial state, residual checked every `interval` steps;
  cold   FP16 storage, all items in the batch (autotuned), rest initial state,
         then an FP32 batch from the FP16 fields (polish);
  warm   as cold, from the network's prediction (inference included);
and an FP64 batch run to a tighter tolerance as the reference of every
field error.  Writes eval.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenes  # noqa: E402
from paper_2506_00907_amd import warmstart as ws  # noqa: E402

TRAIN_SEED = scenes.BASE_SEED + 50
EVAL_SEED = scenes.BASE_SEED + 5


def log(msg):
    print(msg, flush=True)


def dataset(items, batch, moments, size):
    import torch
    n = len(items)
    X = torch.empty((n, size, size, ws.IN_CH), dtype=torch.float32, device="cuda")
    T = torch.empty((n, size, size, ws.OUT_CH), dtype=torch.float32, device="cuda")
    W = torch.empty((n, size, size), dtype=torch.float32, device="cuda")
    for i, it in enumerate(items):
        m = batch.items[i].mask
        X[i] = torch.from_numpy(ws.features(it, m, size))
        t, w = ws.targets(it, m, moments[i], size)
        T[i] = torch.from_numpy(t)
        W[i] = torch.from_numpy(w)
    return X, T, W


def cmd_train(a):
    import torch
    items = scenes.batch_items(a.items, seed=TRAIN_SEED)
    log(f"[train] solving {len(items)} training items (FP16 batch, tol {a.tol:g})")
    sol = ws.solve(items, "f16", tol=a.tol, interval=a.interval, max_steps=a.max_steps, chunk=a.chunk, log=log)
    log(f"[train] solved in {sol['seconds']:.1f} s; statuses {dict(zip(*np.unique(sol['status'], return_counts=True)))}")
    mom = ws.moments_of(sol["batch"])
    X, T, W = dataset(items, sol["batch"], mom, a.size)
    del sol
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    net, hist = ws.train(X, T, W, epochs=a.epochs, batch=a.batch, lr=a.lr, size=a.size, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    os.makedirs(a.out, exist_ok=True)
    np.save(os.path.join(a.out, "net.npy"), net.params().cpu().numpy())
    json.dump(dict(items=a.items, seed=TRAIN_SEED, tol=a.tol, epochs=a.epochs, batch=a.batch, lr=a.lr,
                   loss=hist, train_seconds=t_train), open(os.path.join(a.out, "train.json"), "w"), indent=1)
    log(f"[train] {a.epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")


def field_error(items, batch_moms, ref_moms, masks):
    """per item: relative L2 over fluid nodes of (u_x, b_x) against the reference."""
    out = []
    for it, m, r, mk in zip(items, batch_moms, ref_moms, masks):
        sel = np.asarray(mk, bool).reshape(m.shape[:3])
        Bx = it.scene.B_ext[0]
        a = np.concatenate([m[..., 1][sel], m[..., 5][sel] - Bx])
        b = np.concatenate([r[..., 1][sel], r[..., 5][sel] - Bx])
        out.append(float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
    return np.array(out)


def plain(items, tol, interval, max_steps):
    """FP32, one item at a time, rest start."""
    import torch
    from paper_2506_00907_amd import lbm
    steps, moms, secs = [], [], 0.0
    for i, it in enumerate(items):
        lat = lbm.Lattice(it.scene.with_(storage="f32"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(2)
        lat.reduce()
        while lat.time < max_steps:
            lat.step(interval)
            if lat.reduce()[0] < tol:
                break
        secs += time.perf_counter() - t0
        steps.append(lat.time)
        moms.append(lat.read_moments("f64").cpu().numpy().transpose(1, 2, 3, 0))
        if i % 16 == 15 or i == len(items) - 1:
            log(f"  [plain] {i + 1}/{len(items)} items, {secs:.1f} s")
    return dict(steps=np.array(steps), seconds=secs, moments=moms)


def cmd_eval(a):
    import torch
    from paper_2506_00907_amd import lbm
    items = scenes.batch_items(a.items, seed=EVAL_SEED)
    res = dict(items=a.items, seed=EVAL_SEED, tol=a.tol, interval=a.interval)
    # reference: FP64 batch to a tighter tolerance
    log(f"[eval] FP64 reference, tol {a.ref_tol:g}")
    ref = ws.solve(items, "f64", tol=a.ref_tol, interval=a.interval, max_steps=a.max_steps, chunk=a.chunk, log=log)
    ref_m = ws.moments_of(ref["batch"])
    masks = [lat.mask for lat in ref["batch"].items]
    res["reference"] = dict(seconds=ref["seconds"], steps=ref["steps"].tolist(), status=ref["status"])
    del ref
    torch.cuda.empty_cache()

    def polish(sol, label):
        """FP32 batch from the fields of an FP16 run."""
        m16 = ws.moments_of(sol["batch"])
        inits = []
        for i, it in enumerate(items):
            m = m16[i]
            inits.append((m[..., 1:4], m[..., 5:8]))
        p = ws.solve(items, "f32", tol=a.tol, interval=a.interval, max_steps=a.max_steps, chunk=a.chunk,
                     inits=inits, log=log)
        mp = ws.moments_of(p["batch"])
        return p, m16, mp

    out = {}
    for label in ("cold", "warm"):
        inits, t_inf = None, 0.0
        if label == "warm":
            params = np.load(a.weights)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net = lbm.Network(16, a.size)
            net.set_params(params)
            X = torch.empty((len(items), a.size, a.size, ws.IN_CH), dtype=torch.float32, device="cuda")
            for i, it in enumerate(items):
                X[i] = torch.from_numpy(ws.features(it, masks[i], a.size))
            pred = ws.predict(net, X).cpu().numpy()
            inits = [ws.init_fields(it, masks[i], pred[i]) for i, it in enumerate(items)]
            t_inf = time.perf_counter() - t0
            # prediction error against the reference (before any lattice step)
            pe = []
            for i, it in enumerate(items):
                t_ref, w = ws.targets(it, masks[i], ref_m[i], a.size)
                sel = w > 0
                pe.append(float(np.linalg.norm((pred[i] - t_ref)[sel]) / max(np.linalg.norm(t_ref[sel]), 1e-30)))
            out["prediction_error"] = dict(median=float(np.median(pe)), max=float(np.max(pe)))
        log(f"[eval] {label}: FP16 batch")
        s16 = ws.solve(items, "f16", tol=a.tol, interval=a.interval, max_steps=a.max_steps, chunk=a.chunk,
                       inits=inits, log=log)
        log(f"[eval] {label}: FP32 polish")
        p, m16, mp = polish(s16, label)
        e16 = field_error(items, m16, ref_m, masks)
        ep = field_error(items, mp, ref_m, masks)
        out[label] = dict(inference_seconds=t_inf, fp16_seconds=s16["seconds"], fp16_steps=s16["steps"].tolist(),
                          fp16_status=s16["status"], fp16_error_median=float(np.median(e16)),
                          fp16_error_max=float(np.max(e16)), polish_seconds=p["seconds"],
                          polish_steps=p["steps"].tolist(), polish_status=p["status"],
                          error_median=float(np.median(ep)), error_max=float(np.max(ep)),
                          total_seconds=t_inf + s16["seconds"] + p["seconds"], tuned=s16["tuned"])
        del s16, p
        torch.cuda.empty_cache()
        log(f"[eval] {label}: {out[label]['total_seconds']:.1f} s, error median {out[label]['error_median']:.2e}")
    if a.plain:
        log("[eval] plain FP32, one item at a time")
        pl = plain(items, a.tol, a.interval, a.max_steps)
        e = field_error(items, pl["moments"], ref_m, masks)
        out["plain"] = dict(seconds=pl["seconds"], steps=pl["steps"].tolist(), error_median=float(np.median(e)),
                            error_max=float(np.max(e)))
        for label in ("cold", "warm"):
            out[label]["speedup_vs_plain"] = pl["seconds"] / out[label]["total_seconds"]
    res.update(out)
    os.makedirs(a.out, exist_ok=True)
    json.dump(res, open(os.path.join(a.out, "eval.json"), "w"), indent=1)
    log(json.dumps({k: v for k, v in res.items() if k not in ("reference",)}, default=str)[:3000])


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("train", "eval"):
        p = sub.add_parser(name)
        p.add_argument("--items", type=int, default=4096 if name == "train" else 256)
        p.add_argument("--size", type=int, default=256)
        p.add_argument("--tol", type=float, default=1e-6 if name == "train" else 1e-8)
        p.add_argument("--interval", type=int, default=100)
        p.add_argument("--max-steps", type=int, default=2_000_000)
        p.add_argument("--chunk", type=int, default=20_000)
        p.add_argument("--out", default="gpurun_out/steady")
        if name == "train":
            p.add_argument("--epochs", type=int, default=20)
            p.add_argument("--batch", type=int, default=16)
            p.add_argument("--lr", type=float, default=1e-3)
        else:
            p.add_argument("--weights", required=True)
            p.add_argument("--ref-tol", type=float, default=1e-10)
            p.add_argument("--plain", action="store_true")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cmd_train(a) if a.cmd == "train" else cmd_eval(a)


if __name__ == "__main__":
    main()
