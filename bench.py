#!/usr/bin/env python3
"""Benchmark of the fused coupled lattice Boltzmann sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--storage f32]

Default workload: the 3D MHD pipe, D3Q19 flow + D3Q7 magnetic lattice, a
128 x 128 cross-section with a circular wall of radius 60 (per-link distances
from the exact geometry), 64 nodes along the periodic axis, transverse field
at Ha = 10, thin Shercliff walls of conductance ratio 0.05, FP32 storage.
One step = the boundary-link kernel plus one fused sweep over every fluid
node of both lattices.  Prints ONE JSON line:
  value      MLUPS (fluid nodes x steps / s / 1e6), inputs resident in HBM;
  roofline   the fused sweep of the same pipe 1024 nodes long (a 1.8 GB state
             that streams from HBM): algorithmic bytes per launch / mean
             launch duration (HIP events on the launch stream) against 8 TB/s,
             beside the rate plain 16-byte streaming kernels attain;
  roofline_config  the same for the benchmark pipe itself (its 0.19 GB state
             fits the 256 MB Infinity Cache);
  roofline_hbm_2d  the sweep of the Hartmann-Couette channel 32768 x 512;
  cpu_baseline     the FP64 oracle on the host cores, on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X

# HBM bytes per launch of the fused sweep (mean of the two parities) from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE passes of the commands listed in
# profiles/, scaled by the same counters of a 1 GiB device copy (FETCH_SIZE
# reports half of the bytes read, WRITE_SIZE all bytes written): 2 x FETCH +
# WRITE.  Valid only for the kernel sources and build flags they were taken
# with (the digest follows a source change only when the sweep kernels'
# gfx950 instructions are unchanged by it).
KERNEL_SOURCES = ("paper_2506_00907_amd/csrc/lbm_device.hpp", "paper_2506_00907_amd/csrc/lbm_internal.hpp",
                  "paper_2506_00907_amd/build.py")
MEASURED_TRAFFIC = {
    # (workload, storage): (kernel source digest, bytes per launch)
    ("pipe_long", "f32"): ("ce1e15573a42445e", 2463098929.0),
    ("pipe", "f32"): ("ce1e15573a42445e", 153594184.0),
    ("hartmann_wide", "f32"): ("ce1e15573a42445e", 2585135750.0),
}


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str):
    rec = MEASURED_TRAFFIC.get((workload, storage))
    if rec is None or rec[0] != kernel_digest():
        return None
    return rec[1]


def make_scene(name: str, storage: str):
    import scenes
    if name == "reactive":
        return scenes.config(2, storage=storage, k_range=(1e-3, 1e-1)), "reactive channel 512x256 (D2Q9 + D2Q5)"
    if name == "hartmann":
        return scenes.config(3, storage=storage), "Hartmann-Couette 1024x512 (D2Q9 + D2Q5 x2)"
    if name == "pipe":
        return (scenes.config(4, storage=storage, wall="shercliff"),
                "MHD pipe 128x128 cross-section x 64 periodic, R = 60, Ha = 10, Shercliff c_w = 0.05 "
                "(D3Q19 + D3Q7)")
    if name == "species":
        return (scenes.reactive_species(ncomp=3, storage=storage),
                "reactive channel 512x256, A + B -> P at both walls (D2Q9 + 3 x D2Q5)")
    if name == "poiseuille":
        return scenes.config(1, storage=storage), "plane Poiseuille 64x32 (D2Q9)"
    if name == "hartmann_wide":
        return scenes.config(3, storage=storage, nx=32768), "Hartmann-Couette 32768x512 (D2Q9 + D2Q5 x2)"
    if name == "pipe_long":
        return (scenes.config(4, storage=storage, nx=1024, wall="shercliff"),
                "MHD pipe 128x128 cross-section x 1024 periodic, R = 60, Ha = 10, Shercliff c_w = 0.05 "
                "(D3Q19 + D3Q7)")
    raise SystemExit(f"unknown workload {name}")


# the lattice of the same workload whose state streams from HBM (periodic
# axis lengthened; the flow is invariant along it)
ROOFLINE_VARIANT = {"pipe": "pipe_long", "hartmann": "hartmann_wide"}


def links_moment_reads(links, sc) -> np.ndarray:
    """Moments per node (at A, and again at E) each link's formula reads:
    u at X when extrapolated (3), rho_X for a velocity link moving along
    e_alpha (1), C_X (1, and 2 more for a bilinear term in two components)
    or B_X (1, or 3 with a moving wall)."""
    from paper_2506_00907_amd import lbm
    kind, flags, comp = links["kind"], links["flags"], links["comp"]
    u_given = (flags & 1) != 0
    uw = links["u_w"]
    lat = {0: sc.fluid_lattice, 1: sc.scalar_lattice, 2: sc.mag_lattice}
    eu = np.zeros(len(links))
    for f in (0, 1, 2):
        if not lat[f]:
            continue
        e = lbm.lattice_table(lbm.LATTICES[lat[f]])[0]
        sel = links["field"] == f
        eu[sel] = (e[links["dir"][sel]] * uw[sel]).sum(axis=1)
    uw_zero = u_given & (np.abs(uw).sum(axis=1) == 0)
    u3 = np.where(u_given, 0, 3)
    n = np.zeros(len(links), int)
    n = np.where(kind == 1, np.where(u_given & (eu == 0), 0, 1) + u3, n)
    n = np.where(kind == 2, 3, n)
    n = np.where(kind == 4, 1 + u3 + np.where(links["cross"] != 0, 2, 0), n)
    n = np.where(kind == 7, np.where(uw_zero, 1, 3 + u3), n)
    return n


def algorithmic_bytes(lat) -> dict:
    """Bytes each kernel of a step must move at least once, by its design.

    sweep (the fused stream-collide kernel): every population of every fluid
    node read once and written once, one flag byte per padded node, and the
    moments (eight, one more per extra scalar component) stored for each
    node a link extrapolates from.
    links: per link its record, three population reads and one write, and
    the moments of A and of E its formula uses."""
    sc = lat.scene
    s = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[sc.storage]
    cb = 8 if sc.storage == "f64" else 4
    rec = 96 if sc.storage == "f64" else 64
    q = {"D2Q9": 9, "D3Q19": 19, "D2Q5": 5, "D3Q7": 7}
    QT = q[sc.fluid_lattice] + (lat.n_scalar * q[sc.scalar_lattice] if sc.scalar_lattice else 0) + \
        (len(sc.mag_comps) * q[sc.mag_lattice] if sc.mag_lattice else 0)
    n_fluid = int(lat.mask.sum())
    padded = 1
    for k in range(3):
        padded *= sc.n[k] + (0 if sc.periodic[k] else 2)
    links = lat.links
    e_valid = (links["flags"] & 2) == 0
    mom_nodes = np.unique(np.concatenate([links["node"], links["enode"][e_valid]])).size
    sweep = n_fluid * 2 * QT * s + padded + mom_nodes * lat.moment_width * cb
    link = len(links) * (rec + 4 * s) + 2 * cb * int(links_moment_reads(links, sc).sum())
    return dict(sweep=int(sweep), links=int(link), per_fluid_node_populations=2 * QT * s,
                fluid_nodes=n_fluid, n_links=int(len(links)), moment_nodes=int(mom_nodes), planes=QT)


def time_gpu(lat, steps: int, warmup: int):
    """Runs `warmup` steps, captures the graphs a run of `steps` replays from
    there (set-up, not a step), then times exactly `steps` steps with HIP
    events on the lattice's stream.  Returns (ms, launch description)."""
    import torch
    stream = lat.stream
    lat.step(warmup)
    lat.step_prepare(steps)
    torch.cuda.synchronize()
    before = lat.step_stats()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    g, gs, plain = (a - b for a, b in zip(lat.step_stats(), before))
    launch = (f"{gs} steps in {g} hipGraph replays (up to 64 steps each; link kernel + fused sweep "
              f"per step), {plain} steps launched singly; 256 threads/block")
    return t0.elapsed_time(t1), launch  # ms


def time_launches(lat, n: int = 200):
    """Mean durations (ms) of the boundary-link kernel and of the fused sweep
    kernel (lbm_step_timed): n launches of each kernel back to back in a HIP
    graph, timed with HIP events on the stream the kernels run on; the state
    is restored afterwards."""
    return lat.step_timed(n)


def sweep_roofline(name: str, storage: str, steps: int, warmup: int, launches: int = 50):
    """MLUPS of a workload and the roofline of its fused sweep."""
    import torch
    from paper_2506_00907_amd import lbm
    sc, desc = make_scene(name, storage)
    lat = lbm.Lattice(sc)
    ab = algorithmic_bytes(lat)
    ms, _ = time_gpu(lat, steps, warmup)
    lk, sw = time_launches(lat, launches)
    ach = ab["sweep"] / (sw / 1e3)
    out = {"workload": desc, "storage": storage, "bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9,
           "unit": "GB/s", "frac": ach / HBM_PEAK, "traffic": measured_traffic(name, storage),
           "kernel": "k_step (fused stream-collide sweep), both parities", "bytes_per_launch": ab["sweep"],
           "bytes_per_fluid_node": ab["per_fluid_node_populations"], "fluid_nodes": ab["fluid_nodes"],
           "mean_launch_ms": sw, "state_bytes": int(sum(lat.sizes[:5])),
           "mlups": round(ab["fluid_nodes"] * steps / (ms / 1e3) / 1e6, 1),
           "link_kernel": {"bytes_per_launch": ab["links"], "mean_launch_ms": lk, "links": ab["n_links"]}}
    del lat
    torch.cuda.empty_cache()
    return out


def attainable_bandwidth(nbytes: int = 1 << 31):
    """Best rate (GB/s) of plain 16-byte-access read, write and copy kernels
    (lbm_stream_bandwidth) over nbytes, each at 1, 4 and 16 words per
    thread; copy counts the bytes read plus written."""
    import torch
    from paper_2506_00907_amd import lbm
    out = {}
    for kind, mult in (("read", 1), ("write", 1), ("copy", 2)):
        best = None
        for per in (1, 4, 16):
            ms = lbm.stream_bandwidth(kind, nbytes, per_thread=per, reps=10)
            rate = mult * nbytes / (ms / 1e3) / 1e9
            if best is None or rate > best[0]:
                best = (rate, per, ms)
        out[kind] = {"GB/s": round(best[0], 1), "words_per_thread": best[1], "ms": best[2]}
        torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


def bench_batch(n_items: int, steps: int, storage: str = "f16", tune: bool = True):
    """The duct/pipe cross-section batch (D3Q19 + D3Q7, 64-256 wide, FP16
    storage): autotuned configuration, then `steps` steps of every item timed
    with HIP events on the batch's stream."""
    import torch
    import scenes
    from paper_2506_00907_amd import lbm
    its = scenes.batch_items(n_items, storage=storage)
    B = lbm.Batch([it.scene for it in its])
    tuned = None
    if tune:
        best, cands = B.tune(trial_steps=64)
        tuned = {"best": best, "candidates": [dict(c, ms_per_step=round(ms, 5)) for c, ms in cands]}
    ab = [algorithmic_bytes(it) for it in B.items]
    n_fluid = sum(a["fluid_nodes"] for a in ab)
    step_bytes = sum(a["sweep"] + a["links"] for a in ab)
    B.step(64)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(B.stream)
    B.step(steps)
    t1.record(B.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return dict(items=n_items, storage=storage, fluid_nodes=n_fluid, links=sum(a["n_links"] for a in ab),
                steps=steps, ms_per_step=ms / steps, mlups=n_fluid * steps / (ms / 1e3) / 1e6,
                bytes_per_step=step_bytes, hbm_frac=step_bytes / (ms / steps / 1e3) / HBM_PEAK,
                config=B.config, tuning=tuned)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n: int) -> bool:
    """Sets the OpenMP thread count of the process (the oracle's runtime)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except (OSError, AttributeError):
        return False


def cpu_baseline(sc, budget_s: float = 12.0, single_budget_s: float = 4.0):
    """The FP64 oracle on the host cores (OpenMP over nodes), then on one
    thread, each on a bounded number of steps of the same workload."""
    import oracle
    o = oracle.OracleSim(sc)
    n_fluid = int(o.mask().sum())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rate(budget):
        o.step(1)
        t = time.perf_counter()
        o.step(2)
        per = (time.perf_counter() - t) / 2
        k = max(2, int(budget / max(per, 1e-6)))
        t = time.perf_counter()
        o.step(k)
        return n_fluid * k / (time.perf_counter() - t) / 1e6, k

    value, k = rate(budget_s)
    out = dict(value=value, unit="MLUPS", cores=cores, kind="oracle",
               sample=f"{k} steps of the full {sc.n[0]}x{sc.n[1]}x{sc.n[2]} workload, FP64, OpenMP over nodes",
               cpu_model=_cpu_model(), nproc=os.cpu_count())
    if _omp_threads(1):
        v1, k1 = rate(single_budget_s)
        _omp_threads(cores)
        out["single_thread"] = dict(value=v1, steps=k1)
    return out


def cfg1_time_to_steady(steps: int = 20000):
    """The plane Poiseuille channel (64 x 32, FP64) from rest for `steps`
    steps, after which its slowest mode has decayed to ~4e-9: wall time on
    the GPU (graph replays, capture excluded) and of the FP64 oracle on the
    host cores and on one thread, the steady residual the GPU reaches, and
    the largest difference of u between the two at the end."""
    import torch
    import oracle
    from paper_2506_00907_amd import lbm
    sc, desc = make_scene("poiseuille", "f64")
    lat = lbm.Lattice(sc)
    lat.step(1)
    lat.step_prepare(steps - 1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    lat.step(steps - 1)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t
    lat.reduce()
    lat.step(1000)
    resid = float(lat.reduce()[0])
    u_gpu = lat.read_moments("f64").cpu().numpy()[1]
    out = dict(workload=desc, steps=steps, gpu_seconds=gpu_s, residual_after=resid)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    for label, threads in (("oracle_seconds", cores), ("oracle_seconds_one_thread", 1)):
        if not _omp_threads(threads):
            continue
        o = oracle.OracleSim(sc)
        t = time.perf_counter()
        o.step(steps)
        out[label] = time.perf_counter() - t
        if threads == cores:
            o.step(1000)
            out["max_u_difference"] = float(np.abs(o.moments()[..., 1] - u_gpu).max())
    _omp_threads(cores)
    out["cores"] = cores
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="pipe")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true", help="add throughput of the other workloads")
    ap.add_argument("--no-hbm", action="store_true",
                    help="leave out the sweeps of the large lattices that stream from HBM")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--batch", type=int, default=0, metavar="N",
                    help="add the batch of N duct/pipe cross-sections (autotuned)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the sweep would shard "
              "by slab or by batch item). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_00907_amd import lbm

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # 1 GiB read + 1 GiB written per launch of the plain 16-byte copy
        # kernel (k_copy of lbm_stream_bandwidth): the byte counters of this
        # copy calibrate those of the sweep
        ms = lbm.stream_bandwidth("copy", 1 << 30, per_thread=4, reps=3)
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "ms": ms,
                          "GB/s": 2 * (1 << 30) / (ms / 1e3) / 1e9}))
        return
    sc, desc = make_scene(args.workload, args.storage)
    lat = lbm.Lattice(sc)
    ab = algorithmic_bytes(lat)
    ms, launch = time_gpu(lat, args.steps, args.warmup)
    mlups = ab["fluid_nodes"] * args.steps / (ms / 1e3) / 1e6
    link_ms, sweep_ms = time_launches(lat)
    achieved = ab["sweep"] / (sweep_ms / 1e3)
    res = lat.reduce()
    if not np.isfinite(res[1:6]).all():
        raise SystemExit("non-finite state")
    state_bytes = int(sum(lat.sizes[:5]))
    del lat
    torch.cuda.empty_cache()
    own = {"workload": desc, "storage": args.storage, "bound": "hbm", "achieved": achieved / 1e9,
           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
           "traffic": measured_traffic(args.workload, args.storage),
           "kernel": "k_step (fused stream-collide sweep), both parities",
           "bytes_per_launch": ab["sweep"], "bytes_per_fluid_node": ab["per_fluid_node_populations"],
           "fluid_nodes": ab["fluid_nodes"], "mean_launch_ms": sweep_ms, "state_bytes": state_bytes,
           "regime": ("Infinity-Cache resident (state below 256 MB)" if state_bytes < (256 << 20)
                      else "streams from HBM"),
           "link_kernel": {"bytes_per_launch": ab["links"], "mean_launch_ms": link_ms, "links": ab["n_links"]}}
    out = {
        "metric": "MLUPS + HBM GB/s fraction; time-to-steady (fp16-store+warm-start vs plain)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-store/f32", "bf16": "bf16-store/f32"}[args.storage],
        "data": "synthetic (seeded scene, SplitMix64)",
        "config": {"workload": desc, "storage": args.storage, "fluid_nodes": ab["fluid_nodes"],
                   "links": ab["n_links"], "launch": launch},
    }
    big = ROOFLINE_VARIANT.get(args.workload)
    if big and not args.no_hbm:
        # the same sweep over a state that does not fit the Infinity Cache
        out["roofline"] = sweep_roofline(big, args.storage, 200, 20)
        out["roofline"]["attainable"] = attainable_bandwidth()
        out["roofline"]["frac_of_attainable_copy"] = \
            out["roofline"]["achieved"] / out["roofline"]["attainable"]["copy"]["GB/s"]
        out["roofline_config"] = own
    else:
        out["roofline"] = own
    if not args.no_hbm and args.workload != "hartmann_wide":
        out["roofline_hbm_2d"] = sweep_roofline("hartmann_wide", "f32", 200, 20)
    if args.extra:
        extra = {}
        for w, st in (("reactive", "f32"), ("reactive", "f16"), ("reactive", "bf16"), ("hartmann", "f32"),
                      ("hartmann", "f16"),
                      ("pipe", "f32"), ("pipe", "bf16"), ("hartmann_wide", "f32"), ("hartmann_wide", "f16"),
                      ("pipe_long", "f32"), ("pipe_long", "f16"), ("pipe_long", "bf16"), ("pipe_long", "f64"),
                      ("species", "f32")):
            s2, d2 = make_scene(w, st)
            l2 = lbm.Lattice(s2)
            a2 = algorithmic_bytes(l2)
            m2, _ = time_gpu(l2, 1000, 100)
            lk2, sw2 = time_launches(l2, 50)
            extra[f"{w}_{st}"] = dict(mlups=round(a2["fluid_nodes"] * 1000 / (m2 / 1e3) / 1e6, 1),
                                      sweep_frac=a2["sweep"] / (sw2 / 1e3) / HBM_PEAK,
                                      sweep_bytes=a2["sweep"], sweep_ms=sw2, link_ms=lk2)
            del l2
            torch.cuda.empty_cache()
        out["extra"] = extra
        out["cfg1_time_to_steady"] = cfg1_time_to_steady()
    if args.batch:
        out["batch"] = bench_batch(args.batch, 1000)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
