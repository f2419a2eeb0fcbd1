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
reference of every field error.

Equal error.  Every variant stops on the same residual, which bounds the
rate of change, not the distance to the fixed point: a slowly decaying mode
(for example the mean of the induced field behind nearly conducting walls)
can keep a large error under a small residual.  So after its residual rule,
each item of the cold and warm variants whose reference converged runs on,
in chunks, until its field error is within 1.1 times the plain variant's
error for that item (or a cap on the extra steps); these steps are timed
with the rest.  The table counts the items that meet the rule
|e - e_plain| <= 0.1 e_plain (or are closer than plain).  Items whose wall
conductance was raised to the stable floor (scenes.FLUX_SLOPE_MAX) are
reported apart.  Writes eval.json.
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
                   max_seconds=a.max_seconds, stall=0.5)
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


def field_error_split(items, batch_moms, ref_moms, masks):
    """per item: relative L2 over fluid nodes of u_x and of b_x separately."""
    eu, eb = [], []
    for it, m, r, mk in zip(items, batch_moms, ref_moms, masks):
        sel = np.asarray(mk, bool).reshape(m.shape[:3])
        Bx = it.scene.B_ext[0]
        eu.append(float(np.linalg.norm(m[..., 1][sel] - r[..., 1][sel]) / max(np.linalg.norm(r[..., 1][sel]), 1e-300)))
        bb = r[..., 5][sel] - Bx
        eb.append(float(np.linalg.norm(m[..., 5][sel] - r[..., 5][sel]) / max(np.linalg.norm(bb), 1e-300)))
    return np.array(eu), np.array(eb)


def equalise(batch, items, masks, ref_m, target, eligible, chunk, max_extra):
    """Runs on the eligible items whose error exceeds target[i], `chunk`
    steps at a time, until it does not or max_extra[i] extra steps ran.
    Returns (extra steps per item, seconds spent stepping, moments)."""
    import torch
    n = len(items)
    extra = np.zeros(n, np.int64)
    secs = 0.0
    moms = ws.moments_of(batch)
    e = field_error(items, moms, ref_m, masks)
    todo = eligible & (e > target)
    rounds = 0
    while todo.any():
        batch.set_active(todo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(chunk)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        extra[todo] += chunk
        for i in np.where(todo)[0]:
            moms[i] = batch.items[i].read_moments("f64").cpu().numpy().transpose(1, 2, 3, 0)
        e = field_error(items, moms, ref_m, masks)
        todo = eligible & (e > target) & (extra < max_extra)
        rounds += 1
        if rounds % 20 == 0:
            log(f"    [equal error] {int(todo.sum())} items still above, {secs:.1f} s")
    return extra, secs, moms


def target_verdict(v, label):
    """3x plain's time to steady at equal error: the speed-up after the
    equal-error continuation and the share of reference-converged items
    within the rule; met when the speed-up is at least 3 with at least 90 %
    of the items within the rule.  (Results written before the batch had a
    continuation compare it at the residual rule.)"""
    eq = v.get("equal_error")
    if eq:
        sp, st = eq.get("speedup_vs_plain"), eq.get("all", {})
    else:
        sp, st = v.get("speedup_vs_plain_at_residual"), v.get("at_residual", {}).get("all", {})
    share = st.get("equal")
    met = sp is not None and share is not None and sp >= 3.0 and share >= 0.9
    return dict(speedup=sp, share_within_rule=share, met=bool(met))


def rule_stats(e, e_plain, sel):
    """share of the selected items within the equal-error rule
    |e - e_plain| <= 0.1 e_plain, and within or below it (e <= 1.1 e_plain)."""
    if not sel.any():
        return dict(n=0)
    d = e[sel] - e_plain[sel]
    return dict(n=int(sel.sum()), equal=float(np.mean(np.abs(d) <= 0.1 * e_plain[sel])),
                not_worse=float(np.mean(d <= 0.1 * e_plain[sel])),
                median_ratio=float(np.median(e[sel] / e_plain[sel])))


def plain(items, tol, interval, max_steps, stall=None, chunk=50_000):
    """FP32, one item at a time, rest start; with stall = s an item stops
    when its residual fell by less than the factor s over `chunk` steps
    (the batched variants' rule)."""
    import torch
    from paper_2506_00907_amd import lbm
    steps, moms, secs, status = [], [], 0.0, []
    for i, it in enumerate(items):
        lat = lbm.Lattice(it.scene.with_(storage="f32"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(2)
        lat.reduce()
        st, prev, mark = "max_steps", None, 2 + chunk
        while lat.time < max_steps:
            lat.step(interval)
            r = lat.reduce()[0]
            if r < tol:
                st = "steady"
                break
            if stall is not None and lat.time >= mark:
                if prev is not None and r > stall * prev:
                    st = "stalled"
                    break
                prev, mark = r, mark + chunk
        secs += time.perf_counter() - t0
        status.append(st)
        steps.append(lat.time)
        moms.append(lat.read_moments("f64").cpu().numpy().transpose(1, 2, 3, 0))
        if i % 16 == 15 or i == len(items) - 1:
            log(f"  [plain] {i + 1}/{len(items)} items, {secs:.1f} s")
    return dict(steps=np.array(steps), seconds=secs, moments=moms, status=status)


def axial(u):
    """the axial velocity only: the steady flow of a straight section has no
    in-plane velocity, and equilibria of in-plane velocities excite a
    row-alternating mode the update keeps"""
    v = np.zeros_like(u)
    v[..., 0] = u[..., 0]
    return v


def inits_from(moms, items=None, links=None, shift=True):
    """(u, B) initial fields from moment arrays [nz, ny, nx, 8]; with items
    and links (a handover between phases), the axial velocity only and, with
    shift, b_x shifted to the thin walls' steady balance
    (warmstart.thin_wall_shift)."""
    if items is None:
        return [(m[..., 1:4], m[..., 5:8]) for m in moms]
    return [(axial(m[..., 1:4]), ws.thin_wall_shift(it, lk, m[..., 5:8]) if shift else m[..., 5:8])
            for m, it, lk in zip(moms, items, links)]


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


def item_table(items, masks):
    return [dict(shape=it.shape, ny=it.ny, nz=it.nz, Ha=it.Ha, c_w=it.c_w, c_eff=list(it.c_eff),
                 raised=bool(it.raised), fluid=int(np.asarray(mk).sum())) for it, mk in zip(items, masks)]


# the variants after the plain run and the FP32 batch: FP16 batch from rest
# then FP32 polish; the same from the network's start; the network's start
# straight into the FP32 batch; its velocity only (the induced field from
# rest, as in the plain run) straight into the FP32 batch
VARIANTS = ("cold", "warm", "warm32", "warm32u")


def second_reference(a, items, masks, ref_m, ref_ok, e_plain, finals, kw32, res):
    """How far the reference itself is determined.  The reference continues
    the rest-start trajectory of the FP32 batch; a second FP64 reference run
    to the same tolerance from the warm variant's final state shows how much
    of that start it still carries (slow modes decay over many more steps
    than the residual rule waits).  Reported: the spread between the two
    references, the equal-error statistics over the items whose references
    agree to within a tenth of plain's error (the only items on which a
    difference of that size can be judged), and every variant's errors
    against the second reference."""
    import torch
    log("[eval] second reference: FP64 from the warm variant's final state")
    r2 = ws.solve(items, "f64", tol=a.ref_tol, inits=inits_from(finals["warm_eq"]), **kw32)
    ref2_m = ws.moments_of(r2["batch"])
    ref2_ok = np.array([st == "steady" for st in r2["status"]])
    seconds = r2["seconds"]
    del r2
    torch.cuda.empty_cache()
    both = ref_ok & ref2_ok
    spread = field_error(items, ref2_m, ref_m, masks)
    resolved = both & (spread <= 0.1 * e_plain)
    e2 = {k: field_error(items, m, ref2_m, masks) for k, m in finals.items()}
    out = dict(seconds=seconds, status=ref2_ok.tolist(), spread=spread.tolist(),
               n_both=int(both.sum()), n_resolved=int(resolved.sum()),
               spread_median=float(np.median(spread[both])) if both.any() else None,
               spread_over_plain_median=float(np.median(spread[both] / e_plain[both])) if both.any() else None)
    e1 = {k: field_error(items, m, ref_m, masks) for k, m in finals.items()}
    out["resolved"] = {k: rule_stats(e1[k], e_plain, resolved) for k in finals if k != "plain"}
    out["against_second"] = {k: rule_stats(e2[k], e2["plain"], both) for k in finals if k != "plain"}
    res["reference2"] = out
    log(f"[eval] second reference: {seconds:.1f} s, {int(both.sum())} items with both references, "
        f"{int(resolved.sum())} resolved, spread median {out['spread_median']}")


def cmd_eval(a):
    import torch
    from paper_2506_00907_amd import lbm
    items = scenes.batch_items(a.items, seed=EVAL_SEED)
    res = dict(items=a.items, seed=EVAL_SEED, tol=a.tol, tol_fp16=a.tol16, interval=a.interval,
               ref_tol=a.ref_tol, equal_chunk=a.equal_chunk, wall_shift=a.wall_shift, stall=a.stall)
    kw = dict(interval=a.interval, max_steps=a.max_steps, chunk=a.chunk, log=log)
    kw32 = dict(kw, stall=a.stall)
    raised = np.array([it.raised for it in items])

    log(f"[eval] batch: FP32, rest start, tol {a.tol:g}")
    bsol = ws.solve(items, "f32", tol=a.tol, **kw32)
    b_m = ws.moments_of(bsol["batch"])
    masks = [lat.mask for lat in bsol["batch"].items]
    links = [lat.links for lat in bsol["batch"].items]
    res["item_table"] = item_table(items, masks)

    log(f"[eval] reference: FP64 from the batch's final state, tol {a.ref_tol:g}")
    rsol = ws.solve(items, "f64", tol=a.ref_tol, inits=inits_from(b_m), **kw32)
    ref_m = ws.moments_of(rsol["batch"])
    res["reference"] = dict(seconds=rsol["seconds"], steps=rsol["steps"].tolist(), status=rsol["status"])
    ref_ok = np.array([st == "steady" for st in rsol["status"]])
    del rsol
    torch.cuda.empty_cache()
    res["batch"] = summary(bsol, b_m, ref_m, items, masks, ref_ok)

    e_plain = None
    if a.plain:
        log("[eval] plain FP32, one item at a time")
        pl = plain(items, a.tol, a.interval, a.max_steps, stall=a.stall, chunk=a.chunk)
        e_plain = field_error(items, pl["moments"], ref_m, masks)
        eu, eb = field_error_split(items, pl["moments"], ref_m, masks)
        res["plain"] = dict(seconds=pl["seconds"], steps=pl["steps"].tolist(), status=pl["status"],
                            error_median=float(np.median(e_plain)),
                            error_max=float(np.max(e_plain)), errors=e_plain.tolist(), errors_u=eu.tolist(),
                            errors_b=eb.tolist(),
                            error_median_ref_steady=float(np.median(e_plain[ref_ok])) if ref_ok.any() else None)
        plain_steps = pl["steps"]
        finals = {"plain": pl["moments"], "batch": b_m}
        del pl
        # the batch's items follow plain's trajectories step for step; where
        # the residual rule stopped them elsewhere, they run on as the other
        # variants do
        log("[eval] batch: equal error with plain (reference-converged items)")
        extra, secs, me = equalise(bsol["batch"], items, masks, ref_m, 1.1 * e_plain, ref_ok, a.equal_chunk,
                                   np.maximum(plain_steps, a.equal_chunk))
        e_eq = field_error(items, me, ref_m, masks)
        res["batch"]["equal_error"] = dict(extra_steps=extra.tolist(), extra_seconds=secs,
                                           total_seconds=bsol["seconds"] + secs, errors=e_eq.tolist(),
                                           all=rule_stats(e_eq, e_plain, ref_ok),
                                           unraised=rule_stats(e_eq, e_plain, ref_ok & ~raised),
                                           raised=rule_stats(e_eq, e_plain, ref_ok & raised),
                                           n_extended=int((extra > 0).sum()))
        log(f"[eval] batch: {int((extra > 0).sum())} items ran on, {secs:.1f} s more")
        finals["batch_eq"] = me
    del bsol["batch"]
    torch.cuda.empty_cache()

    net_inits, net_t = None, 0.0
    for label in VARIANTS:
        inits, t_inf = None, 0.0
        if label == "warm32":
            inits, t_inf = net_inits, net_t
        if label == "warm32u":
            inits = [(u, np.zeros_like(B) + np.asarray(it.scene.B_ext, float))
                     for it, (u, B) in zip(items, net_inits)]
            t_inf = net_t
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
            if a.wall_shift:
                inits = [(u, ws.thin_wall_shift(it, links[i], B)) for i, (it, (u, B)) in enumerate(zip(items, inits))]
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            pe = []
            for i, it in enumerate(items):
                t_ref, w = ws.targets(it, masks[i], ref_m[i], a.size)
                sel = w > 0
                pe.append(float(np.linalg.norm((pred[i] - t_ref)[sel]) / max(np.linalg.norm(t_ref[sel]), 1e-30)))
            res["prediction_error"] = dict(median=float(np.median(pe)), max=float(np.max(pe)))
            log(f"[eval] warm: inference {t_inf:.2f} s, prediction error median {np.median(pe):.3f}")
            net_inits, net_t = inits, t_inf
        s16 = None
        if label not in ("warm32", "warm32u"):
            log(f"[eval] {label}: FP16 batch, tol {a.tol16:g}")
            s16 = ws.solve(items, "f16", tol=a.tol16, inits=inits, stall=0.5, **kw)
            m16 = ws.moments_of(s16["batch"])
            del s16["batch"]
            torch.cuda.empty_cache()
            log(f"[eval] {label}: FP32 polish, tol {a.tol:g}")
            t0 = time.perf_counter()
            hand = inits_from(m16, items, links, shift=a.wall_shift)
            t_hand = time.perf_counter() - t0
        else:
            log(f"[eval] {label}: FP32 batch from the network's start, tol {a.tol:g}")
            hand, t_hand = inits, 0.0
        p = ws.solve(items, "f32", tol=a.tol, inits=hand, **kw32)
        p["seconds"] += t_hand
        mp = ws.moments_of(p["batch"])
        if e_plain is not None:
            finals[label] = mp
        r = summary(p, mp, ref_m, items, masks, ref_ok)
        r16 = summary(s16, m16, ref_m, items, masks, ref_ok) if s16 is not None else None
        out = dict(inference_seconds=t_inf, fp16=r16, polish=r,
                   total_seconds=t_inf + (s16["seconds"] if s16 is not None else 0.0) + p["seconds"],
                   error_median=r["error_median"], error_max=r["error_max"],
                   error_median_ref_steady=r.get("error_median_ref_steady"))
        if e_plain is not None:
            e_res = np.array(r["errors"])
            out["at_residual"] = dict(total_seconds=out["total_seconds"],
                                      all=rule_stats(e_res, e_plain, ref_ok),
                                      unraised=rule_stats(e_res, e_plain, ref_ok & ~raised),
                                      raised=rule_stats(e_res, e_plain, ref_ok & raised))
            log(f"[eval] {label}: equal error with plain (reference-converged items)")
            extra, secs, me = equalise(p["batch"], items, masks, ref_m, 1.1 * e_plain, ref_ok, a.equal_chunk,
                                       np.maximum(plain_steps, a.equal_chunk))
            e_eq = field_error(items, me, ref_m, masks)
            eu, eb = field_error_split(items, me, ref_m, masks)
            out["equal_error"] = dict(extra_steps=extra.tolist(), extra_seconds=secs,
                                      total_seconds=out["total_seconds"] + secs, errors=e_eq.tolist(),
                                      errors_u=eu.tolist(), errors_b=eb.tolist(),
                                      all=rule_stats(e_eq, e_plain, ref_ok),
                                      unraised=rule_stats(e_eq, e_plain, ref_ok & ~raised),
                                      raised=rule_stats(e_eq, e_plain, ref_ok & raised),
                                      n_extended=int((extra > 0).sum()))
            log(f"[eval] {label}: {int((extra > 0).sum())} items ran on, {secs:.1f} s more")
            finals[label + "_eq"] = me
        del p["batch"]
        torch.cuda.empty_cache()
        res[label] = out
        log(f"[eval] {label}: {res[label]['total_seconds']:.1f} s, error median {r['error_median']:.2e}")
    if a.plain and a.second_reference:
        second_reference(a, items, masks, ref_m, ref_ok, e_plain, finals, kw32, res)
    if a.plain:
        res["batch"]["at_residual"] = dict(all=rule_stats(np.array(res["batch"]["errors"]), e_plain, ref_ok))
        for label in ("batch",) + VARIANTS:
            tot = res[label]["seconds"] if label == "batch" else res[label]["total_seconds"]
            res[label]["speedup_vs_plain_at_residual"] = res["plain"]["seconds"] / tot
            eq = res[label]["equal_error"]
            eq["speedup_vs_plain"] = res["plain"]["seconds"] / eq["total_seconds"]
        for label in ("batch",) + VARIANTS:
            res[label]["target_3x_at_equal_error"] = target_verdict(res[label], label)
    os.makedirs(a.out, exist_ok=True)
    json.dump(res, open(os.path.join(a.out, "eval.json"), "w"), indent=1)
    brief = {k: v for k, v in res.items() if k not in ("reference", "item_table")}
    drop = ("steps", "status", "errors", "errors_u", "errors_b", "extra_steps")
    for k in ("batch", "plain") + VARIANTS:
        if k in brief:
            brief[k] = {kk: vv for kk, vv in brief[k].items() if kk not in drop}
            for sub in ("fp16", "polish", "equal_error"):
                if brief[k].get(sub):
                    brief[k][sub] = {kk: vv for kk, vv in brief[k][sub].items() if kk not in drop}
    log(json.dumps(brief, default=str))


def cmd_report(a):
    """Markdown summary of eval.json (and train.json)."""
    ev = json.load(open(a.eval))
    tr = json.load(open(a.train)) if a.train else None
    ref_ok = np.array([st == "steady" for st in ev["reference"]["status"]])
    raised = np.array([row["raised"] for row in ev["item_table"]])
    out = []
    w = out.append
    w(f"# Time to steady state: {ev['items']} duct / pipe cross-sections (seed {ev['seed']})")
    w("")
    w(f"Residual rule: R16 over {ev['interval']} steps below {ev['tol']:g} (FP16 phase: {ev['tol_fp16']:g}). "
      f"Reference: FP64 from the FP32 batch's state to {ev['ref_tol']:g}; "
      f"{int(ref_ok.sum())} of {len(ref_ok)} references reach it "
      f"({int((ref_ok & raised).sum())} of them with a raised wall conductance).")
    w("")
    pl = ev.get("plain")
    w("| Variant | seconds at the residual rule | speed-up | seconds at equal error | speed-up | "
      "items within the rule (reference-converged, at equal error) | of them not raised | raised | "
      "median error / plain |")
    w("|---|---|---|---|---|---|---|---|---|")
    if pl:
        w(f"| plain: FP32, one item at a time, rest start | {pl['seconds']:.1f} | 1.00 | {pl['seconds']:.1f} | 1.00 "
          f"| — | — | — | 1 |")
    b = ev["batch"]
    st = b.get("at_residual", {}).get("all", {})
    if not b.get("equal_error"):
        w(f"| batch: FP32, all items, rest start | {b['seconds']:.1f} | "
          f"{b.get('speedup_vs_plain_at_residual', 0):.2f} | — | — | {st.get('equal', float('nan')):.2f} "
          f"(at the residual rule) | — | — | {st.get('median_ratio', float('nan')):.2f} |")
    for label, name in (("batch", "batch: FP32, all items, rest start"),
                        ("cold", "cold: FP16 batch, then FP32 polish"),
                        ("warm", "warm: network, FP16 batch, then FP32 polish"),
                        ("warm32", "warm32: network, then FP32 batch"),
                        ("warm32u", "warm32u: network velocity, induced field from rest, then FP32 batch")):
        if label not in ev:
            continue
        v = ev[label]
        eq = v.get("equal_error", {})
        if not eq:
            continue
        w(f"| {name} | {v.get('total_seconds', v.get('seconds', 0)):.1f} | {v.get('speedup_vs_plain_at_residual', 0):.2f} | "
          f"{eq['total_seconds']:.1f} | {eq.get('speedup_vs_plain', 0):.2f} | {eq['all']['equal']:.2f} "
          f"({eq['all']['not_worse']:.2f} not worse) | {eq['unraised'].get('not_worse', float('nan')):.2f} | "
          f"{eq['raised'].get('not_worse', float('nan')):.2f} | {eq['all']['median_ratio']:.2f} |")
    w("")
    if pl:
        for label in ("batch",) + VARIANTS:
            if label not in ev:
                continue
            tv = ev[label].get("target_3x_at_equal_error") or target_verdict(ev[label], label)
            if tv["speedup"] is None:
                continue
            w(f"- target (3x plain at equal error, >= 90 % of the items within the rule), {label}: "
              f"{'met' if tv['met'] else 'not met'} (speed-up {tv['speedup']:.2f}, "
              f"{tv['share_within_rule']:.2f} within the rule).")
    bq = ev["batch"].get("equal_error")
    if bq and "at_residual" in ev["batch"]:
        ar = ev["batch"]["at_residual"]["all"]
        w(f"- batch: at the residual rule {ar['equal']:.2f} of the reference-converged items are within "
          f"|e - e_plain| <= 0.1 e_plain and {ar['not_worse']:.2f} not worse (median ratio "
          f"{ar['median_ratio']:.2f}): its items follow plain's trajectories step for step but stop where the "
          f"residual rule, checked on other windows, lets them; {bq['n_extended']} items ran on for "
          f"{bq['extra_seconds']:.1f} s.")
    for label in VARIANTS:
        v = ev.get(label, {})
        if "equal_error" not in v:
            continue
        ar = v["at_residual"]
        fp16 = f"FP16 {v['fp16']['seconds']:.1f} s, " if v.get("fp16") else ""
        w(f"- {label}: at the residual rule {ar['all']['equal']:.2f} of the reference-converged items are within "
          f"|e - e_plain| <= 0.1 e_plain and {ar['all']['not_worse']:.2f} not worse (median ratio "
          f"{ar['all']['median_ratio']:.2f}); {v['equal_error']['n_extended']} items ran on for "
          f"{v['equal_error']['extra_seconds']:.1f} s. Phases: inference {v['inference_seconds']:.1f} s, {fp16}"
          f"FP32 {v['polish']['seconds']:.1f} s.")
    if "prediction_error" in ev:
        w(f"- network prediction error (relative L2 of the scaled fields): median {ev['prediction_error']['median']:.3f}, "
          f"max {ev['prediction_error']['max']:.3f}.")
    w(f"- reference: {ev['reference']['seconds']:.1f} s.")
    r2 = ev.get("reference2")
    if r2:
        w("")
        w(f"Second reference (FP64 from the warm variant's final state, same tolerance, {r2['seconds']:.1f} s): "
          f"{r2['n_both']} items have both references; their spread (relative L2 between the two) has median "
          f"{r2['spread_median']:.2e}, {r2['spread_over_plain_median']:.2f} times plain's error. "
          f"{r2['n_resolved']} items have references that agree to within a tenth of plain's error.")
        w("")
        w("| Variant | resolved items within the rule | not worse | median error / plain | "
          "against the second reference: within | not worse | median ratio |")
        w("|---|---|---|---|---|---|---|")
        names = dict(batch="batch (at the residual rule)", batch_eq="batch (at equal error)",
                     cold="cold (at the residual rule)",
                     cold_eq="cold (at equal error)", warm="warm (at the residual rule)",
                     warm_eq="warm (at equal error)", warm32="warm32 (at the residual rule)",
                     warm32_eq="warm32 (at equal error)", warm32u="warm32u (at the residual rule)",
                     warm32u_eq="warm32u (at equal error)")
        for k, name in names.items():
            rs, ag = r2["resolved"].get(k, {}), r2["against_second"].get(k, {})
            if not rs:
                continue
            f = lambda d, key: f"{d[key]:.2f}" if key in d else "—"
            w(f"| {name} | {f(rs, 'equal')} (n = {rs.get('n', 0)}) | {f(rs, 'not_worse')} | {f(rs, 'median_ratio')} "
              f"| {f(ag, 'equal')} (n = {ag.get('n', 0)}) | {f(ag, 'not_worse')} | {f(ag, 'median_ratio')} |")
    if tr:
        w(f"- training: {tr['items']} items (seed {tr['seed']}), {tr['epochs']} epochs in {tr['train_seconds']:.1f} s, "
          f"loss {tr['loss'][0]:.3e} -> {tr['loss'][-1]:.3e}.")
    text = "\n".join(out) + "\n"
    if a.out:
        open(a.out, "w").write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    rp = sub.add_parser("report")
    rp.add_argument("--eval", required=True)
    rp.add_argument("--train", default=None)
    rp.add_argument("--out", default=None)
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
            p.add_argument("--no-wall-shift", dest="wall_shift", action="store_false",
                           help="start the warm and polish phases without the thin-wall offset correction")
            p.add_argument("--stall", type=float, default=0.95,
                           help="FP32/FP64 runs: an item stops when its residual fell by less than this "
                                "factor over a chunk (mass-drift floors of interpolated walls)")
            p.add_argument("--equal-chunk", type=int, default=2000,
                           help="steps per round of the equal-error continuation")
            p.add_argument("--second-reference", action="store_true",
                           help="also run an FP64 reference from the warm variant's final state and report "
                                "how far the reference is determined")
    a = ap.parse_args(argv)
    if a.cmd == "report":
        cmd_report(a)
        return
    import torch
    torch.cuda.set_device(0)
    cmd_train(a) if a.cmd == "train" else cmd_eval(a)


if __name__ == "__main__":
    main()
