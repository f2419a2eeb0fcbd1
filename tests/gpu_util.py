"""Helpers shared by the GPU parity tests: run a scene on the HIP library and on
the FP64 oracle and compare them element by element."""
import numpy as np

import oracle
from paper_2506_00907_amd import lbm

FIELDS = ("rho", "ux", "uy", "uz", "C", "Bx", "By", "Bz")


def direction_map(name):
    """library direction index -> oracle direction index (matched by e)."""
    el, _, _, _ = lbm.lattice_table(lbm.LATTICES[name])
    eo, _, _, _ = oracle.lattice_table(name)
    return np.array([[b for b in range(len(eo)) if np.array_equal(eo[b], el[a])][0] for a in range(len(el))])


def gpu_moments(lat):
    """[nz, ny, nx, W] numpy array from the library (W = 8, plus one column
    per scalar component beyond the first)."""
    return lat.read_moments("f64").cpu().numpy().transpose(1, 2, 3, 0)


def gpu_populations(lat, field):
    """populations of one field in the oracle's direction order."""
    sc = lat.scene
    name = {0: sc.fluid_lattice, 1: sc.scalar_lattice, 2: sc.mag_lattice}[field]
    m = direction_map(name)
    P = lat.read_populations(field).cpu().numpy()
    q = len(m)
    nc = P.shape[0] // q
    out = np.zeros_like(P)
    for c in range(nc):
        for a in range(q):
            out[c * q + m[a]] = P[c * q + a]
    return out.reshape((nc, q) + P.shape[1:]) if field == 2 or (field == 1 and nc > 1) else out


def rel_l2(a, b, floor=1e-300):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), floor))


def field_errors(mg, mo, mask, B_ext=(0.0, 0.0, 0.0)):
    """relative L2 over fluid nodes of rho, the velocity vector u, C and the
    induced field b = B - B_ext (vector); a field whose reference is
    identically zero is reported in absolute terms."""
    sel = mask.astype(bool)
    Be = np.asarray(B_ext, float)
    groups = {
        "rho": (mg[..., 0][sel], mo[..., 0][sel]),
        "u": (mg[..., 1:4][sel], mo[..., 1:4][sel]),
        "C": (mg[..., 4][sel], mo[..., 4][sel]),
        "b": (mg[..., 5:8][sel] - Be, mo[..., 5:8][sel] - Be),
    }
    out = {}
    for k, (a, b) in groups.items():
        nb = np.linalg.norm(b)
        rms_ref = nb / np.sqrt(max(b.size, 1))
        # a field that is zero by construction (up to round-off) is compared
        # by its absolute rms difference
        if rms_ref > 1e-12:
            out[k] = float(np.linalg.norm(a - b) / nb)
        else:
            out[k] = float(np.linalg.norm(a - b) / np.sqrt(max(b.size, 1)))
    return out


def run_pair(sc, steps, chunks=1, precision=None):
    """Runs the scene on both sides; returns (lattice, oracle sim).  FP64
    storage is compared with the long-double build of the oracle, whose own
    rounding is far below the 1e-12 bar; other storages with the FP64 build."""
    lat = lbm.Lattice(sc)
    if precision is None:
        precision = "ld" if sc.storage == "f64" else "f64"
    o = oracle.OracleSim(sc, precision)
    per = max(1, steps // chunks)
    done = 0
    while done < steps:
        k = min(per, steps - done)
        lat.step(k)
        o.step(k)
        done += k
    return lat, o
