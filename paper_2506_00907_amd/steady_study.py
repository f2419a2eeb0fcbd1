"""Time to steady state of many duct / pipe cross-sections.

    python -m paper_2506_00907_amd.steady_study train --items 4096 --out DIR
    python -m paper_2506_00907_amd.steady_study eval --weights DIR/net.npy --items 256 --out DIR

train: solves the training items (seeded, disjoint from the evaluation
items) with the FP16 batch, builds the network inputs and targets from the
converged fields and trains the warm-start network; writes net.npy and
train.json.

eval: on the evaluation items, four ways to a steady state (residual of
lbm_reduce over a window of `interval` steps below tol):
  plain  FP32 storage, one item at a time (single-context kernels, graph
         replays), rest initial state;
  batch  FP32 storage, all items in one batch (autotuned), rest initial state;
  cold   FP16 storage in the batch to the FP16 tolerance (above the noise floor
         of stochastically rounded storage), then an FP32 batch from its
         fields (polish) to tol;
  warm   as cold, from the network's prediction (inference included);
and the batch's final state continued in FP64 to a tighter tolerance as the
reference of every field error.  Writes eval.json.
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
    sol = ws.solve(items, "f16", tol=a.tol, interval=a.interval, max_steps=a.max_steps, chunk=a.chunk, log=log,
                   max_seconds=a.max_seconds)
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


def inits_from(moms):
    """(u, B) initial fields from moment arrays [nz, ny, nx, 8]."""
    return [(m[..., 1:4], m[..., 5:8]) for m in moms]


def summary(sol, moms, ref_m, items, masks, ref_ok=None):
    """timing, statuses and field errors; with ref_ok (items whose reference
    reached its tolerance) also the error statistics over those items."""
    e = field_error(items, moms, ref_m, masks)
    out = dict(seconds=sol["seconds"], steps=sol["steps"].tolist(), status=sol["status"],
               n_not_steady=int(sum(s != "steady" for s in sol["status"])),
               n_stalled=int(sum(s == "stalled" for s in sol["status"])),
               error_median=float(np.median(e)), error_max=float(np.max(e)), errors=e.tolist(),
               tuned=sol.get("tuned"))
    if ref_ok is not None and ref_ok.any():
        out["error_median_ref_steady"] = float(np.median(e[ref_ok]))
        out["error_max_ref_steady"] = float(np.max(e[ref_ok]))
    return out


def cmd_eval(a):
    import torch
    from paper_2506_00907_amd import lbm
    items = scenes.batch_items(a.items, seed=EVAL_SEED)
    res = dict(items=a.items, seed=EVAL_SEED, tol=a.tol, tol_fp16=a.tol16, interval=a.interval,
               ref_tol=a.ref_tol)
    kw = dict(interval=a.interval, max_steps=a.max_steps, chunk=a.chunk, log=log)

    log(f"[eval] batch: FP32, rest start, tol {a.tol:g}")
    bsol = ws.solve(items, "f32", tol=a.tol, **kw)
    b_m = ws.moments_of(bsol["batch"])
    masks = [lat.mask for lat in bsol["batch"].items]
    del bsol["batch"]
    torch.cuda.empty_cache()

    log(f"[eval] reference: FP64 from the batch's final state, tol {a.ref_tol:g}")
    rsol = ws.solve(items, "f64", tol=a.ref_tol, inits=inits_from(b_m), **kw)
    ref_m = ws.moments_of(rsol["batch"])
    res["reference"] = dict(seconds=rsol["seconds"], steps=rsol["steps"].tolist(), status=rsol["status"])
    ref_ok = np.array([st == "steady" for st in rsol["status"]])
    del rsol
    torch.cuda.empty_cache()
    res["batch"] = summary(bsol, b_m, ref_m, items, masks, ref_ok)

    for label in ("cold", "warm"):
        inits, t_inf = None, 0.0
        if label == "warm":
            params = np.load(a.weights)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net = lbm.Network(16, a.size, in_ch=ws.IN_CH, out_ch=ws.OUT_CH)
            net.set_params(params)
            X = torch.empty((len(items), a.size, a.size, ws.IN_CH), dtype=torch.float32, device="cuda")
            for i, it in enumerate(items):
                X[i] = torch.from_numpy(ws.features(it, masks[i], a.size))
            pred = ws.predict(net, X).cpu().numpy()
            inits = [ws.init_fields(it, masks[i], pred[i]) for i, it in enumerate(items)]
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            pe = []
            for i, it in enumerate(items):
                t_ref, w = ws.targets(it, masks[i], ref_m[i], a.size)
                sel = w > 0
                pe.append(float(np.linalg.norm((pred[i] - t_ref)[sel]) / max(np.linalg.norm(t_ref[sel]), 1e-30)))
            res["prediction_error"] = dict(median=float(np.median(pe)), max=float(np.max(pe)))
            log(f"[eval] warm: inference {t_inf:.2f} s, prediction error median {np.median(pe):.3f}")
        log(f"[eval] {label}: FP16 batch, tol {a.tol16:g}")
        s16 = ws.solve(items, "f16", tol=a.tol16, inits=inits, stall=0.5, **kw)
        m16 = ws.moments_of(s16["batch"])
        del s16["batch"]
        torch.cuda.empty_cache()
        log(f"[eval] {label}: FP32 polish, tol {a.tol:g}")
        p = ws.solve(items, "f32", tol=a.tol, inits=inits_from(m16), **kw)
        mp = ws.moments_of(p["batch"])
        del p["batch"]
        torch.cuda.empty_cache()
        r = summary(p, mp, ref_m, items, masks, ref_ok)
        r16 = summary(s16, m16, ref_m, items, masks, ref_ok)
        res[label] = dict(inference_seconds=t_inf, fp16=r16, polish=r,
                          total_seconds=t_inf + s16["seconds"] + p["seconds"],
                          error_median=r["error_median"], error_max=r["error_max"],
                          error_median_ref_steady=r.get("error_median_ref_steady"))
        log(f"[eval] {label}: {res[label]['total_seconds']:.1f} s, error median {r['error_median']:.2e}")
    if a.plain:
        log("[eval] plain FP32, one item at a time")
        pl = plain(items, a.tol, a.interval, a.max_steps)
        e = field_error(items, pl["moments"], ref_m, masks)
        res["plain"] = dict(seconds=pl["seconds"], steps=pl["steps"].tolist(), error_median=float(np.median(e)),
                            error_max=float(np.max(e)), errors=e.tolist(),
                            error_median_ref_steady=float(np.median(e[ref_ok])) if ref_ok.any() else None)
        for label in ("batch", "cold", "warm"):
            tot = res[label]["seconds"] if label == "batch" else res[label]["total_seconds"]
            res[label]["speedup_vs_plain"] = pl["seconds"] / tot
    os.makedirs(a.out, exist_ok=True)
    json.dump(res, open(os.path.join(a.out, "eval.json"), "w"), indent=1)
    brief = {k: v for k, v in res.items() if k != "reference"}
    for k in ("batch", "cold", "warm", "plain"):
        if k in brief:
            brief[k] = {kk: vv for kk, vv in brief[k].items() if kk not in ("steps", "status", "errors")}
            for sub in ("fp16", "polish"):
                if sub in brief[k]:
                    brief[k][sub] = {kk: vv for kk, vv in brief[k][sub].items()
                                     if kk not in ("steps", "status", "errors")}
    log(json.dumps(brief, default=str))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("train", "eval"):
        p = sub.add_parser(name)
        p.add_argument("--items", type=int, default=4096 if name == "train" else 256)
        p.add_argument("--size", type=int, default=256)
        p.add_argument("--tol", type=float, default=1e-6 if name == "train" else 1e-8)
        p.add_argument("--interval", type=int, default=1000)
        p.add_argument("--max-steps", type=int, default=2_000_000)
        p.add_argument("--chunk", type=int, default=50_000)
        p.add_argument("--out", default="steady_out")
        if name == "train":
            p.add_argument("--max-seconds", type=float, default=float("inf"))
            p.add_argument("--epochs", type=int, default=20)
            p.add_argument("--batch", type=int, default=16)
            p.add_argument("--lr", type=float, default=1e-3)
        else:
            p.add_argument("--weights", required=True)
            p.add_argument("--ref-tol", type=float, default=1e-10)
            p.add_argument("--tol16", type=float, default=1e-6)
            p.add_argument("--plain", action="store_true")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cmd_train(a) if a.cmd == "train" else cmd_eval(a)


if __name__ == "__main__":
    main()
