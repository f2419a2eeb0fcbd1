"""Host-side checks of liblbm (no GPU): the C ABI is complete, the library's
own geometry / link builder agrees with the oracle's independent builder, and
invalid inputs are rejected before any device work."""
import ctypes as C
import dataclasses
import math
import os
import re

import numpy as np
import pytest

import oracle
import scenes
from paper_2506_00907_amd import _lib as L
from paper_2506_00907_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 18
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, n
    assert set(L.SIGNATURES) == set(names)
    assert b"gfx950" in lib.lbm_version()
    # constants of the header that the binding mirrors
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    m = re.search(r"#define LBM_REDUCE_STATIC_MAX_BLOCKS (\d+)", src)
    assert m and int(m.group(1)) == L.LBM_REDUCE_STATIC_MAX_BLOCKS


def _lat_map(name):
    """library direction index -> oracle direction index, matched by e."""
    code = lbm.LATTICES[name]
    el, wl, c2l, oppl = lbm.lattice_table(code)
    eo, wo, c2o, oppo = oracle.lattice_table(name)
    m = np.zeros(len(wl), int)
    for a in range(len(wl)):
        hits = [b for b in range(len(wo)) if np.array_equal(eo[b], el[a])]
        assert len(hits) == 1
        m[a] = hits[0]
    return m


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D2Q5", "D3Q7"])
def test_lattice_tables_agree(name):
    code = lbm.LATTICES[name]
    el, wl, c2l, oppl = lbm.lattice_table(code)
    eo, wo, c2o, oppo = oracle.lattice_table(name)
    m = _lat_map(name)
    assert c2l == c2o
    assert np.allclose(wl, wo[m], rtol=0, atol=1e-17)
    for a in range(len(wl)):
        assert np.array_equal(el[oppl[a]], -el[a])


SCENES = {
    "poiseuille": lambda: scenes.poiseuille(nx=8, ny=6),
    "reactive": lambda: scenes.reactive_channel(nx=14, ny=9, q=0.3, k_range=(1e-3, 1e-1)),
    "reactive_q08": lambda: scenes.reactive_channel(nx=9, ny=6, q=0.8),
    "hartmann": lambda: scenes.hartmann_couette(nx=5, ny=11, c_top=0.1),
    "hartmann_cinf": lambda: scenes.hartmann_couette(nx=3, ny=7, c_top=math.inf, qb=1.0, qt=0.2),
    "pipe_shercliff": lambda: scenes.mhd_pipe(nx=2, side=27, R=11.37, wall="shercliff"),
    "pipe_ins3": lambda: scenes.mhd_pipe(nx=1, side=17, R=6.3, wall="insulating", ncomp=3),
    "diffreact_full": lambda: scenes.diffusion_reaction(layout="full", W_nodes=8),
    "duct_item": lambda: scenes.batch_items(3, side_lo=20, side_hi=30)[0].scene,
    "pipe_item": lambda: scenes.batch_items(3, side_lo=20, side_hi=30)[1].scene,
    "stokes_d03": lambda: scenes.stokes_second(nx=3, ny=9, q=0.3),
    "stokes_mismatch": lambda: scenes.stokes_second(nx=3, ny=9, q=1.0, d_scheme=0.5),
    "stokes_3d": lambda: scenes.stokes_second(nx=3, ny=8, q=0.5, dim=3),
    "channel_half": lambda: scenes.channel_reservoirs("half", width=4, res_len=3, ch_len=6),
    "channel_full": lambda: scenes.channel_reservoirs("full", width=4, res_len=3, ch_len=6),
    "box_offgrid": lambda: _offgrid_box(),
    "hartmann_X": lambda: scenes.hartmann_couette(nx=3, ny=7, c_top=0.1, qb=1.0, qt=1.0, top_scheme="X"),
    "hartmann_theta": lambda: scenes.hartmann_couette(nx=3, ny=7, c_top=0.1, qb=1.0, qt=1.0, top_scheme="theta"),
    "open_box_alt": lambda: scenes.open_box(nx=6, ny=3, q_in=0.52, q_out=0.7, alt_in=True, alt_out=True),
    "pipe_conducting_q19": lambda: scenes.mhd_pipe(nx=2, side=17, R=6.3, wall="conducting", mag_lattice="D3Q19"),
    "reactive_quadratic": lambda: _quadratic_walls(scenes.reactive_channel(nx=9, ny=6, q=0.3)),
    "species2": lambda: scenes.reactive_species(nx=11, ny=7, q=0.7, ncomp=2),
    "species3": lambda: scenes.reactive_species(nx=9, ny=6, q=0.3, ncomp=3),
    "species3_3d": lambda: _species_3d(),
}


def _species_3d():
    """three components in a D3Q7 pipe: A + B -> P on the curved wall"""
    sc = scenes.mhd_pipe(nx=2, side=13, R=5.3, wall="insulating")
    wall = dataclasses.replace(sc.boundaries[0], g=[], h=[scenes.BC(scenes.FLUX, cross_comps=(0, 1), cross=c)
                                                          for c in (-0.02, -0.02, 0.02)])
    return sc.with_(boundaries=[wall], mag_lattice=None, mag_comps=(), scalar_lattice="D3Q7", scalar_ncomp=3,
                    tau_c=0.6, tau_cs=(0.7, 0.65), B_ext=(0.0, 0.0, 0.0))


def _quadratic_walls(sc, k=0.02):
    """the channel's walls with a second-order surface reaction F = -k C^2"""
    for b in sc.boundaries[:2]:
        b.h = scenes.BC(scenes.FLUX, a1=0.0, quad=-k)
    return sc


def _offgrid_box():
    """a finite block at off-grid faces inside a periodic box: every link
    distance differs (diagonal entries through faces, edges and corners)"""
    sc = scenes.channel_reservoirs("half", width=4, res_len=3, ch_len=6)
    blk = scenes.Boundary("box", axis=2, lo=(2.3, 1.6, 4.2), hi=(3.7, 2.45, 6.9), f=scenes.BC(scenes.VEL))
    return sc.with_(boundaries=sc.boundaries + [blk])


def compare_link_tables(sc):
    mask, ll = lbm.build_links(sc)
    o = oracle.OracleSim(sc)
    ol = o.links()
    assert np.array_equal(mask, o.mask())
    assert len(ll) == len(ol)
    names = {0: sc.fluid_lattice, 1: sc.scalar_lattice, 2: sc.mag_lattice}
    maps = {f: _lat_map(n) for f, n in names.items() if n}
    okey = {}
    for r in ol:
        okey[(int(r["A"]), int(r["field"]), int(r["comp"]), int(r["dir"]))] = r
    for r in ll:
        f = int(r["field"])
        k = (int(r["node"]), f, int(r["comp"]), int(maps[f][r["dir"]]))
        o_ = okey[k]
        assert int(r["kind"]) == int(o_["kind"])
        assert abs(r["d"] - o_["d"]) < 1e-12
        e_invalid = bool(r["flags"] & 2)
        assert e_invalid == (o_["E"] < 0)
        if not e_invalid:
            assert int(r["enode"]) == int(o_["E"])
        assert bool(r["flags"] & 1) == bool(o_["u_given"])
        assert bool(r["flags"] & 4) == (o_["omega"] != 0.0)
        assert bool(r["flags"] & 8) == bool(o_["compare"])
        for fld in ("value", "a1", "quad", "a3", "cross"):
            assert r[fld] == o_[fld], (fld, r[fld], o_[fld])
        if r["cross"] != 0.0:
            assert (int(r["cross_comp"][0]), int(r["cross_comp"][1])) == (int(o_["cj"]), int(o_["cl"]))
        assert abs(r["weight"] - o_["weight"]) < 1e-12 * max(1.0, abs(o_["weight"]))
        assert np.array_equal(r["u_w"], o_["u_w"])
    return ll


@pytest.mark.parametrize("key", sorted(SCENES))
def test_link_builder_matches_oracle(key):
    ll = compare_link_tables(SCENES[key]())
    assert len(ll) > 0


def test_link_builder_ordering_and_counts():
    sc = scenes.hartmann_couette(nx=6, ny=9)
    mask, ll = lbm.build_links(sc)
    keys = [(int(r["node"]), int(r["field"]), int(r["comp"]), int(r["dir"])) for r in ll]
    assert keys == sorted(keys)
    # flat walls: 3 f links and (1 per component) g links per wall node
    assert len(ll) == 6 * 2 * (3 + 2 * 1)


# ---------------------------------------------------------------------------
# validation (no device work happens before it)
# ---------------------------------------------------------------------------
class _FakeCtx:
    """A context over fake, aligned device addresses: lbm_create and the
    validation paths of lbm_set_geometry / lbm_set_links never touch them."""

    def __init__(self, sc, n_links):
        self.p = lbm.params_from_scene(sc)
        sizes = lbm.required_bytes(self.p, n_links)
        ptrs = (C.c_void_p * L.LBM_NBUF)(*[(0x100000 * (i + 1)) if s else None for i, s in enumerate(sizes)])
        self.ctx = C.c_void_p()
        assert L.lib().lbm_create(C.byref(self.p), n_links, ptrs, None, C.byref(self.ctx)) == 0

    def set_links(self, links):
        a = np.ascontiguousarray(links)
        return L.lib().lbm_set_links(self.ctx, a.ctypes.data_as(C.c_void_p), len(a))

    def err(self):
        return L.lib().lbm_last_error(self.ctx).decode()

    def __del__(self):
        L.lib().lbm_destroy(self.ctx)


@pytest.fixture
def small():
    sc = scenes.reactive_channel(nx=10, ny=6, q=0.3)
    mask, links = lbm.build_links(sc)
    fc = _FakeCtx(sc, len(links) + 4)
    assert L.lib().lbm_set_geometry(fc.ctx, mask.ctypes.data_as(C.c_void_p)) == 0
    return sc, mask, links, fc


def test_rejects_missing_link(small):
    sc, mask, links, fc = small
    assert fc.set_links(links[1:]) == -1
    assert "no boundary link" in fc.err()


def test_rejects_duplicate_link(small):
    sc, mask, links, fc = small
    assert fc.set_links(np.concatenate([links, links[:1]])) == -1
    assert "duplicate" in fc.err()


@pytest.mark.parametrize("field,value", [("d", 0.0), ("d", 1.5), ("d", float("nan")), ("kind", 3),
                                         ("dir", 0), ("node", 10 ** 6), ("a1", float("inf"))])
def test_rejects_bad_link_fields(small, field, value):
    sc, mask, links, fc = small
    bad = links.copy()
    bad[0][field] = value
    assert fc.set_links(bad) == -1


def test_rejects_wrong_second_node(small):
    sc, mask, links, fc = small
    bad = links.copy()
    i = int(np.nonzero((bad["flags"] & 2) == 0)[0][0])
    bad[i]["enode"] = bad[i]["node"]
    assert fc.set_links(bad) == -1
    assert "enode" in fc.err()


def test_rejects_known_population(small):
    sc, mask, links, fc = small
    bad = links.copy()
    i = int(np.nonzero(bad["field"] == 0)[0][0])
    bad[i]["dir"] = 0 if bad[i]["dir"] != 1 else 3
    assert fc.set_links(bad) == -1


def test_too_many_links_and_order(small):
    sc, mask, links, fc = small
    assert fc.set_links(np.concatenate([links] * 2)) == -2
    fc2 = _FakeCtx(sc, len(links))
    assert fc2.set_links(links) == -5        # geometry first
    assert L.lib().lbm_step(fc2.ctx, 1) == -5  # init first


@pytest.mark.parametrize("mut", [
    dict(dim=4), dict(tau_f=0.5), dict(fluid=2), dict(storage=9), dict(mag_ncomp=2),
    dict(n=(0, 4, 1)), dict(store_scale=(0.0, 1.0, 1.0)),
    # padded node indices must fit 32 bits (2e9 padded nodes at most)
    dict(dim=3, fluid=2, n=(2000, 2000, 600), periodic=(0, 0, 0)),
])
def test_rejects_bad_params(mut):
    sc = scenes.poiseuille(nx=4, ny=4)
    p = lbm.params_from_scene(sc)
    for k, v in mut.items():
        if isinstance(v, tuple):
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        else:
            setattr(p, k, v)
    sizes = (C.c_size_t * L.LBM_NBUF)()
    assert L.lib().lbm_required_bytes(C.byref(p), 10, sizes) == 0
    ctx = C.c_void_p()
    ptrs = (C.c_void_p * L.LBM_NBUF)(*[0x100000] * L.LBM_NBUF)
    assert L.lib().lbm_create(C.byref(p), 10, ptrs, None, C.byref(ctx)) == -1


def test_buffer_layout():
    sc = scenes.hartmann_couette(nx=64, ny=30, storage="f16")
    p = lbm.params_from_scene(sc)
    sizes = lbm.required_bytes(p, 100)
    plane = ((64 * 32 + 63) // 64) * 64
    assert sizes[0] == ((19 * plane * 2 + 255) // 256) * 256      # populations, 2 bytes
    assert sizes[3] == ((2 * 8 * plane * 4 + 255) // 256) * 256 + 256   # moment planes (FP32), time base
    assert sizes[5] == sizes[6] == sizes[7] == 0
    assert all(s % 256 == 0 for s in sizes)


def test_scheme_distance_override():
    """d_scheme replaces the measured d of every link of its boundary; values
    outside (0, 1] are rejected"""
    _, ll = lbm.build_links(scenes.stokes_second(nx=3, ny=9, q=1.0, d_scheme=0.5))
    assert np.all(ll["d"] == 0.5)
    _, ll = lbm.build_links(scenes.stokes_second(nx=3, ny=9, q=1.0))
    assert np.all(ll["d"] == 1.0)
    for bad in (-0.5, 1.5, math.nan):
        with pytest.raises(L.LbmError):
            lbm.build_links(scenes.stokes_second(nx=3, ny=9, q=1.0, d_scheme=bad))


def test_box_distances_and_validation():
    """a block's links enter it where the segment crosses its first face;
    inverted bounds are rejected"""
    _, ll = lbm.build_links(_offgrid_box())
    d = np.round(ll["d"], 6)
    assert {0.5}.issubset(set(d)) and len(set(d)) > 4, sorted(set(d))
    assert np.all((ll["d"] > 0) & (ll["d"] <= 1))
    sc = scenes.channel_reservoirs("half", width=4, res_len=3, ch_len=6)
    bad = scenes.Boundary("box", axis=2, lo=(1.0, 0.0, 0.0), hi=(0.0, 1.0, 1.0), f=scenes.BC(scenes.VEL))
    with pytest.raises(L.LbmError):
        lbm.build_links(sc.with_(boundaries=sc.boundaries + [bad]))


def test_comparison_forms_validation():
    """the comparison flag only exists for VEL, PRES, FLUX and MAG_FLUX;
    theta must not be negative"""
    sc = scenes.hartmann_couette(nx=3, ny=7, c_top=0.0)
    sc.boundaries[1].g[0] = scenes.BC(scenes.MAG_DIR, value=0.0, alt=True)
    with pytest.raises(L.LbmError):
        lbm.build_links(sc)
    _, ll = lbm.build_links(scenes.hartmann_couette(nx=3, ny=7, c_top=0.1, top_scheme="X"))
    assert np.any(ll["flags"] & 8)
    sc = scenes.hartmann_couette(nx=3, ny=7, c_top=0.1, top_scheme="theta")
    mask, ll = lbm.build_links(sc)
    fc = _FakeCtx(sc, len(ll))
    assert L.lib().lbm_set_geometry(fc.ctx, mask.ctypes.data_as(C.c_void_p)) == 0
    assert fc.set_links(ll) != -1  # passes validation (no device here to upload to)
    th = ll.copy()
    th["a1"][th["kind"] == lbm.KINDS["MAG_THETA"]] = -1.0
    assert fc.set_links(th) == -1 and "theta" in fc.err()
    bad = ll.copy()
    i = int(np.nonzero(bad["kind"] == lbm.KINDS["MAG_DIR"])[0][0])
    bad["flags"][i] |= 8
    assert fc.set_links(bad) == -1 and "flag bit 3" in fc.err()
    bad = ll.copy()
    bad["flags"][0] |= 16
    assert fc.set_links(bad) == -1 and "unknown flag" in fc.err()


def test_d3q19_magnetic_lattice_walls():
    """every wall kind but the theta form on a D3Q19 magnetic lattice; a flat
    face's flux is split over its five crossing links, a curved wall's share
    S_i over all links of B_i (Eq. 48), so the shares of a cross-section still
    add up to the perimeter"""
    for wall in ("conducting", "insulating", "shercliff"):
        sc = scenes.mhd_pipe(nx=1, side=17, R=6.3, wall=wall, mag_lattice="D3Q19")
        mask, ll = lbm.build_links(sc)
        fc = _FakeCtx(sc, len(ll))
        assert L.lib().lbm_set_geometry(fc.ctx, mask.ctypes.data_as(C.c_void_p)) == 0
        assert fc.set_links(ll) != -1, (wall, fc.err())
        if wall == "shercliff":
            g = ll[ll["field"] == 2]
            assert abs(g["weight"].sum() - 2 * math.pi * 6.3) < 1e-9
            th = ll.copy()
            th["kind"][th["field"] == 2] = lbm.KINDS["MAG_THETA"]
            th["a1"][th["field"] == 2] = 1.0
            assert fc.set_links(th) == -1 and "theta" in fc.err()
    p = lbm.params_from_scene(scenes.mhd_pipe(nx=1, side=17, R=6.3, mag_lattice="D3Q19"))
    p.mag_ncomp = 3
    with pytest.raises(L.LbmError):
        lbm.required_bytes(p, 10)


def test_quadratic_flux_term_validation(small):
    """quad is copied to the links of flux walls and rejected elsewhere"""
    sc, mask, links, fc = small
    bad = links.copy()
    i = int(np.nonzero(bad["kind"] == lbm.KINDS["VEL"])[0][0])
    bad["quad"][i] = 0.1
    assert fc.set_links(bad) == -1 and "quad" in fc.err()
    ok = links.copy()
    ok["quad"][ok["kind"] == lbm.KINDS["FLUX"]] = -0.01
    assert fc.set_links(ok) != -1
    bad = links.copy()
    bad["quad"][0] = float("nan")
    assert fc.set_links(bad) == -1


def _law_links(sc):
    mask, ll = lbm.build_links(sc)
    return ll[(ll["kind"] == lbm.KINDS["FLUX"]) | (ll["kind"] >= lbm.KINDS["MAG_FLUX"])]


def test_flux_laws_form_their_coefficients():
    """The builder forms a1, a3 from a wall's physical law with the field's own
    transport coefficient c^2 (tau - 1/2): a Robin wall d phi/dn = k phi gives
    F = -k D phi (Eq. 17 with a2 = D), a reaction F = -k (phi - phi_eq), a thin
    wall F = -eta (B_k - B_ext,k) / (c_w H) (Eq. 30), and the theta form
    theta = c_w H / (tau_m - 1/2) (Eqs. 39-40).  Stated values: tau_c = 0.6 on
    D2Q5 has D = 0.025; tau_m = 0.9 on D3Q7 has eta = 0.1, on D3Q19 eta = 0.4/3."""
    e5 = lbm.lattice_table(lbm.LATTICES["D2Q5"])[0]
    up = int(np.nonzero((e5[:, 0] == 0) & (e5[:, 1] == 1))[0][0])  # links entering from the bottom wall

    def bottom(sc):
        fl = _law_links(sc)
        return fl[fl["dir"] == up]

    sc = scenes.reactive_channel(nx=9, ny=6, q=0.3, k=0.04)
    wall = bottom(sc)
    assert len(wall) == 9 and np.allclose(wall["a1"], -0.04 * 0.025, rtol=1e-15) and np.all(wall["a3"] == 0.0)
    prof = np.linspace(0.01, 0.09, 9)
    sc.boundaries[0].h = scenes.BC(scenes.FLUX, law="robin", profile=prof, profile_axis=0)
    wall = bottom(sc)
    assert np.allclose(wall["a1"], -prof[wall["node"] % 9] * 0.025, rtol=1e-15)
    sc.boundaries[0].h = scenes.BC(scenes.FLUX, law="reaction", k=0.3, phi_eq=2.0)
    wall = bottom(sc)
    assert np.allclose(wall["a1"], -0.3) and np.allclose(wall["a3"], -0.6)
    pipe = scenes.mhd_pipe(nx=1, side=17, R=6.3, wall="shercliff", c_w=0.05)
    ml = _law_links(pipe)
    assert len(ml) and np.allclose(ml["a1"], -0.1 / (0.05 * 6.3), rtol=1e-14) and np.all(ml["a3"] == 0.0)
    q19 = scenes.mhd_pipe(nx=1, side=17, R=6.3, wall="shercliff", c_w=0.05, mag_lattice="D3Q19")
    assert np.allclose(_law_links(q19)["a1"], -(0.4 / 3) / (0.05 * 6.3), rtol=1e-14)
    cond = scenes.mhd_pipe(nx=1, side=17, R=6.3, wall="conducting")
    assert np.all(_law_links(cond)["a1"] == 0.0)
    # a thin wall on a component with an applied field: a3 = a1 B_ext,k
    hc = scenes.hartmann_couette(nx=3, ny=7, c_top=0.2)
    hc.boundaries[1].g[1] = scenes.BC(scenes.MAG_FLUX, law="shercliff", c_w=0.5, H=hc.meta["H"])
    hl = _law_links(hc)
    by = hl[hl["comp"] == 1]
    a1 = -0.1 / (0.5 * hc.meta["H"])
    assert len(by) and np.allclose(by["a1"], a1, rtol=1e-14) and np.allclose(by["a3"], a1 * hc.B_ext[1], rtol=1e-14)
    th = scenes.hartmann_couette(nx=3, ny=7, c_top=0.2, top_scheme="theta")
    tl = _law_links(th)
    assert len(tl) and np.allclose(tl["a1"], 0.2 * th.meta["H"] / 0.4, rtol=1e-14)


@pytest.mark.parametrize("bad", [
    dict(kind="MAG_FLUX", law="robin", k=0.1),
    dict(kind="FLUX", law="shercliff", c_w=0.1, H=3.0),
    dict(kind="FLUX", law="robin", k=-0.1),
    dict(kind="FLUX", law="robin", k=float("nan")),
    dict(kind="VEL", law="robin", k=0.1),
])
def test_flux_law_validation(bad):
    """a law that does not fit its kind, or invalid law data, is rejected"""
    sc = scenes.reactive_channel(nx=9, ny=6, q=0.3)
    if bad["kind"] == "MAG_FLUX":
        sc = scenes.hartmann_couette(nx=3, ny=7, c_top=0.2)
        sc.boundaries[1].g[0] = scenes.BC(**bad)
    elif bad["kind"] == "VEL":
        sc.boundaries[0].f = scenes.BC(**bad)
    else:
        sc.boundaries[0].h = scenes.BC(**bad)
    with pytest.raises(L.LbmError):
        lbm.build_links(sc)
    for c_w, H in ((0.0, 3.0), (0.1, 0.0), (math.inf, 3.0)):
        th = scenes.hartmann_couette(nx=3, ny=7, c_top=0.2, top_scheme="theta")
        th.boundaries[1].g[0] = scenes.BC(scenes.MAG_THETA, law="shercliff", c_w=c_w, H=H)
        with pytest.raises(L.LbmError):
            lbm.build_links(th)


def test_builder_rejects_uncovered_boundary():
    sc = scenes.poiseuille(nx=4, ny=4)
    sc.boundaries[1].f = None
    with pytest.raises(L.LbmError):
        lbm.build_links(sc)


# ---------------------------------------------------------------------------
# several scalar components (Section 4.2.2)
# ---------------------------------------------------------------------------
def test_several_components_buffer_layout():
    """m components: m scalar lattices of populations, 7 + m moment planes
    per parity, 6 + m snapshot planes"""
    sc = scenes.reactive_species(nx=64, ny=30, ncomp=3)
    p = lbm.params_from_scene(sc)
    sizes = lbm.required_bytes(p, 100)
    plane = ((66 * 32 + 63) // 64) * 64   # one halo layer on each side of both axes
    up = lambda x: ((x + 255) // 256) * 256
    assert sizes[0] == up((9 + 3 * 5) * plane * 4)
    assert sizes[3] == up(2 * 10 * plane * 4) + 256
    assert sizes[4] == up(9 * plane * 4) + up(16 * 8)


@pytest.mark.parametrize("mut", [
    dict(scalar_ncomp=4), dict(scalar_ncomp=-1), dict(tau_cs=(0.5, 0.7)), dict(scalar_ncomp=3, tau_cs=(0.7, 0.4)),
])
def test_several_components_rejects_bad_params(mut):
    sc = scenes.reactive_species(nx=6, ny=5, ncomp=2)
    p = lbm.params_from_scene(sc)
    for k, v in mut.items():
        if isinstance(v, tuple):
            for i, x in enumerate(v):
                getattr(p, k)[i] = x
        else:
            setattr(p, k, v)
    assert L.lib().lbm_required_bytes(C.byref(p), 10, (C.c_size_t * L.LBM_NBUF)()) == 0


def test_several_components_need_a_scalar_lattice_and_no_magnetic_one():
    for sc in (scenes.poiseuille(nx=4, ny=4), scenes.hartmann_couette(nx=3, ny=7)):
        p = lbm.params_from_scene(sc)
        p.scalar_ncomp = 2
        p.tau_cs[0] = 0.7
        assert L.lib().lbm_required_bytes(C.byref(p), 10, (C.c_size_t * L.LBM_NBUF)()) == 0


def _species_walls(sc, **kw):
    for b in sc.boundaries[:2]:
        b.h = [dataclasses.replace(bc, **kw) for bc in b.h]
    return sc


@pytest.mark.parametrize("bad", [
    dict(cross_comps=(0, 2)),              # a component beyond scalar_ncomp
    dict(cross_comps=(-1, 1)),
    dict(law="robin", k=0.1),              # the bilinear term belongs to the given-coefficient law
    dict(cross=float("nan")),
])
def test_several_components_builder_validation(bad):
    sc = _species_walls(scenes.reactive_species(nx=6, ny=5, ncomp=2), **bad)
    with pytest.raises(L.LbmError):
        lbm.build_links(sc)


def test_several_components_need_a_condition_for_each():
    sc = scenes.reactive_species(nx=6, ny=5, ncomp=3)
    sc.boundaries[0].h = sc.boundaries[0].h[:2]
    with pytest.raises(L.LbmError):
        lbm.build_links(sc)
    # a bilinear term with one component only
    one = scenes.reactive_channel(nx=6, ny=5)
    one.boundaries[0].h = scenes.BC(scenes.FLUX, cross_comps=(0, 0), cross=-0.01)
    with pytest.raises(L.LbmError):
        lbm.build_links(one)


def test_several_components_link_validation():
    sc = scenes.reactive_species(nx=6, ny=5, ncomp=2)
    mask, links = lbm.build_links(sc)
    fc = _FakeCtx(sc, len(links) + 4)
    assert L.lib().lbm_set_geometry(fc.ctx, mask.ctypes.data_as(C.c_void_p)) == 0
    flux = np.nonzero(links["cross"] != 0)[0]
    conc = np.nonzero((links["field"] == 1) & (links["kind"] == lbm.KINDS["CONC"]))[0]
    assert len(flux) and len(conc)
    bad = links.copy()
    bad["cross_comp"][flux[0]] = (0, 2)
    assert fc.set_links(bad) == -1 and "bilinear" in fc.err()
    bad = links.copy()
    bad["cross"][conc[0]] = 0.1
    assert fc.set_links(bad) == -1 and "bilinear" in fc.err()
    bad = links.copy()
    bad["comp"][conc[0]] = 2
    assert fc.set_links(bad) == -1 and "component" in fc.err()
    # one component's links missing
    keep = ~((links["field"] == 1) & (links["comp"] == 1))
    assert fc.set_links(links[keep]) == -1 and "no boundary link" in fc.err()
    assert fc.set_links(links) != -1   # valid: only the upload (no device here) fails


def test_batch_rejects_several_components():
    scs = [scenes.reactive_species(nx=6, ny=5, ncomp=2)] * 2
    params = _batch_params(scs)
    caps = (C.c_size_t * 2)(*[len(lbm.build_links(sc)[1]) for sc in scs])
    assert L.lib().lbm_batch_required_bytes(2, params, caps, (C.c_size_t * L.LBM_NBUF)()) == 0


# ---------------------------------------------------------------------------
# batches (host-side checks only)
# ---------------------------------------------------------------------------
def _batch_params(scs):
    n = len(scs)
    return (L.lbm_params * n)(*[lbm.params_from_scene(s) for s in scs])


def test_batch_layout_is_items_back_to_back():
    items = [it.scene for it in scenes.batch_items(4, side_lo=20, side_hi=40)]
    tables = [lbm.build_links(sc) for sc in items]
    params = _batch_params(items)
    caps = (C.c_size_t * 4)(*[len(t[1]) for t in tables])
    sizes = (C.c_size_t * L.LBM_NBUF)()
    tot = L.lib().lbm_batch_required_bytes(4, params, caps, sizes)
    assert tot == sum(sizes)
    for k in range(5):
        per = [lbm.required_bytes(params[i], caps[i])[k] for i in range(4)]
        assert sizes[k] == sum(((s + 255) // 256) * 256 for s in per)
    assert all(sizes[k] > 0 for k in range(5, 8))
    assert all(s % 256 == 0 for s in sizes)


def test_batch_rejects_mixed_items():
    a = scenes.batch_items(2, side_lo=20, side_hi=30)[0].scene
    b = a.with_(storage="f32")
    c = scenes.hartmann_couette(nx=4, ny=9)
    sizes = (C.c_size_t * L.LBM_NBUF)()
    for pair in ([a, b], [a, c]):
        caps = (C.c_size_t * 2)(10, 10)
        assert L.lib().lbm_batch_required_bytes(2, _batch_params(pair), caps, sizes) == 0
    assert L.lib().lbm_batch_required_bytes(0, _batch_params([a]), (C.c_size_t * 1)(10), sizes) == 0
    bad = a.with_(tau_f=0.4)
    assert L.lib().lbm_batch_required_bytes(1, _batch_params([bad]), (C.c_size_t * 1)(10), sizes) == 0


class _FakeBatch:
    """A batch over fake aligned device addresses: creation, item contexts,
    configuration and the state checks never touch device memory."""

    def __init__(self, scs):
        n = len(scs)
        self.tables = [lbm.build_links(sc) for sc in scs]
        self.params = _batch_params(scs)
        self.caps = (C.c_size_t * n)(*[len(t[1]) for t in self.tables])
        sizes = (C.c_size_t * L.LBM_NBUF)()
        assert L.lib().lbm_batch_required_bytes(n, self.params, self.caps, sizes) > 0
        base, ptrs = 1 << 40, []
        for s in sizes:
            ptrs.append(base if s else None)
            base += ((s + (1 << 20)) >> 20) << 20
        self.b = C.c_void_p()
        assert L.lib().lbm_batch_create(n, self.params, self.caps, (C.c_void_p * L.LBM_NBUF)(*ptrs), None,
                                        C.byref(self.b)) == 0

    def err(self):
        return L.lib().lbm_batch_last_error(self.b).decode()

    def __del__(self):
        L.lib().lbm_batch_destroy(self.b)


def test_batch_items_and_configuration():
    scs = [it.scene for it in scenes.batch_items(3, side_lo=20, side_hi=30)]
    fb = _FakeBatch(scs)
    lib = L.lib()
    items = [lib.lbm_batch_item(fb.b, i) for i in range(3)]
    assert all(items) and len(set(items)) == 3
    assert lib.lbm_batch_item(fb.b, 3) is None and lib.lbm_batch_item(fb.b, -1) is None
    # an item belongs to the batch: destroy is a no-op, its stream is fixed
    lib.lbm_destroy(items[0])
    assert lib.lbm_set_stream(items[0], None) == -1
    # the geometry of an item goes through the single-context call
    mask = fb.tables[0][0]
    assert lib.lbm_set_geometry(items[0], mask.ctypes.data_as(C.c_void_p)) == 0
    cfg = L.lbm_batch_config()
    assert lib.lbm_batch_get_config(fb.b, C.byref(cfg)) == 0
    assert (cfg.mode, cfg.block, cfg.steps_per_launch, cfg.graph_steps) == (1, 256, 1, 64)
    good = [(1, 64, 1, 64), (1, 128, 1, 2), (2, 512, 2, 64), (2, 256, 32, 64), (2, 64, 8, 8)]
    bad = [(1, 96, 1, 64), (1, 256, 2, 64), (2, 1024, 2, 64), (2, 256, 3, 64), (2, 256, 8, 12),
           (2, 100, 2, 64), (3, 256, 1, 64), (1, 256, 1, 63)]
    for g in good:
        assert lib.lbm_batch_configure(fb.b, C.byref(L.lbm_batch_config(*g))) == 0, g
    for bcfg in bad:
        assert lib.lbm_batch_configure(fb.b, C.byref(L.lbm_batch_config(*bcfg))) == -1, bcfg
    # stepping needs every item initialised
    assert lib.lbm_batch_step(fb.b, 4) == -5
    assert "not initialised" in fb.err()
    assert lib.lbm_batch_run(fb.b, 1e-8, 3, 100, None, None, None) == -1   # odd interval
    assert lib.lbm_batch_tune(fb.b, 1, None, None, None, 0, None) == -1


# ---------------------------------------------------------------------------
# warm-start network (host-side checks only)
# ---------------------------------------------------------------------------
def test_network_layout_and_parameter_count():
    from oracle import surrogate
    d = L.lbm_nn_desc(16, 256, 4, 2, 32, L.LBM_BF16)
    sizes = (C.c_size_t * 4)()
    assert L.lib().lbm_nn_required_bytes(C.byref(d), sizes) == sum(sizes) > 0
    assert sizes[0] == 4 * ((surrogate.num_params(4, 2, 32) * 4 + 255) // 256) * 256
    ptrs = (C.c_void_p * 4)(*[(1 << 40) + (k << 36) for k in range(4)])
    n = C.c_void_p()
    assert L.lib().lbm_nn_create(C.byref(d), ptrs, None, C.byref(n)) == 0
    assert L.lib().lbm_nn_num_params(n) == surrogate.num_params(4, 2, 32) == 471874
    assert L.lib().lbm_nn_forward(n, 1, C.c_void_p(1 << 40), None) == -5   # parameters first
    assert L.lib().lbm_nn_forward(n, 17, C.c_void_p(1 << 40), None) == -1  # more than the batch
    assert L.lib().lbm_nn_backward(n, C.c_void_p(1 << 40), C.c_void_p(1 << 40), None) == -5
    L.lib().lbm_nn_destroy(n)
    for bad in [(0, 256, 4, 2, 32, 4), (1, 250, 4, 2, 32, 4), (1, 256, 17, 2, 32, 4), (1, 256, 4, 33, 32, 4),
                (1, 256, 4, 2, 48, 4), (1, 256, 4, 2, 32, 3)]:
        assert L.lib().lbm_nn_required_bytes(C.byref(L.lbm_nn_desc(*bad)), sizes) == 0, bad
