"""Batched items (lbm_batch_*): every item of a batch evolves exactly as the
same scene run alone, in every execution mode (batch invariance); the
device-side steady-state detection stops each item where the single-context
residual says it is steady; the autotuner's trial steps are real steps."""
import numpy as np
import pytest

import oracle
import scenes
from .gpu_util import field_errors, gpu_moments
from paper_2506_00907_amd import lbm

pytestmark = pytest.mark.gpu

MODES = [("tiled", 256, 1, 64), ("tiled", 64, 1, 64), ("resident", 256, 2, 64), ("resident", 128, 8, 64),
         ("resident", 512, 32, 64)]


def duct_pipe_items(storage, n=5, lo=20, hi=44, seed=None, developed=True, Ha_hi=8.0):
    """Small duct / pipe items; Ha is capped so that B0 stays well below the
    lattice speeds at these widths (the full-size items are 64-256 wide)."""
    kw = {} if seed is None else {"seed": seed}
    its = scenes.batch_items(n, side_lo=lo, side_hi=hi, storage=storage, Ha_hi=Ha_hi, **kw)
    scs = [it.scene for it in its]
    if developed:
        scs = [scenes.developed(sc, seed=1000 + i, u_amp=0.005) for i, sc in enumerate(scs)]
    return scs


def reactive_items(storage):
    shapes = [(40, 20, 0.3), (57, 26, 0.7), (33, 31, 0.5)]
    return [scenes.developed(scenes.reactive_channel(nx=nx, ny=ny, q=q, k_range=(1e-3, 1e-1), storage=storage),
                             seed=2000 + i, u_amp=0.005)
            for i, (nx, ny, q) in enumerate(shapes)]


def assert_items_equal_alone(B, scs, steps):
    for i, sc in enumerate(scs):
        alone = lbm.Lattice(sc)
        alone.step(steps)
        assert B.items[i].time == alone.time == steps
        a, b = gpu_moments(B.items[i]), gpu_moments(alone)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), (i, np.abs(a - b).max())


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("mode", MODES, ids=lambda m: f"{m[0]}{m[1]}x{m[2]}")
def test_batch_item_equals_item_alone(storage, mode):
    scs = duct_pipe_items(storage)
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(130)  # two single steps from time 0, two captured runs of 64 steps
    assert_items_equal_alone(B, scs, 130)


@pytest.mark.parametrize("mode", [MODES[0], MODES[3]], ids=["tiled", "resident"])
def test_bf16_batch_item_equals_item_alone(mode):
    scs = duct_pipe_items("bf16", n=3)
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(130)
    assert_items_equal_alone(B, scs, 130)


@pytest.mark.parametrize("mode", [MODES[0], MODES[3]], ids=["tiled", "resident"])
def test_oscillating_walls_in_a_batch(mode):
    """Time-dependent wall data take each item's own time in the batch."""
    scs = [scenes.stokes_second(nx=5, ny=17, period=150, q=0.3, storage="f32"),
           scenes.stokes_second(nx=4, ny=23, period=90, q=0.7, U=0.02, storage="f32")]
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(130)
    assert_items_equal_alone(B, scs, 130)


@pytest.mark.parametrize("mode", [MODES[0], MODES[3]], ids=["tiled", "resident"])
def test_d3q19_magnetic_items_in_a_batch(mode):
    """pipes whose B1 lives on the D3Q19 lattice (conducting and Shercliff
    walls), batched: each equals the same pipe alone"""
    scs = [scenes.developed(scenes.mhd_pipe(nx=2, side=side, R=R, wall=w, tau_m=0.8, mag_lattice="D3Q19",
                                            storage="f32"), seed=3000 + i, u_amp=0.005)
           for i, (side, R, w) in enumerate([(21, 8.1, "conducting"), (25, 10.6, "shercliff")])]
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(66)
    assert_items_equal_alone(B, scs, 66)


@pytest.mark.parametrize("mode", [MODES[0], MODES[3]], ids=["tiled", "resident"])
def test_comparison_and_quadratic_forms_in_a_batch(mode):
    """items with the comparison link forms, the theta form and a quadratic
    surface reaction, batched: each equals the same item alone"""
    def quad(sc):
        for b in sc.boundaries[:2]:
            b.h = scenes.BC(scenes.FLUX, a1=-0.001, quad=-0.02)
        return sc
    scs = [scenes.hartmann_couette(nx=4, ny=19, c_top=0.1, qb=1.0, qt=1.0, top_scheme="X", storage="f32"),
           scenes.hartmann_couette(nx=4, ny=23, c_top=0.5, qb=0.6, qt=1.0, top_scheme="theta", storage="f32")]
    B = lbm.Batch([scenes.developed(sc, seed=4000 + i, u_amp=0.005) for i, sc in enumerate(scs)])
    B.configure(*mode)
    B.step(66)
    assert_items_equal_alone(B, B.scenes, 66)
    rc = [scenes.developed(quad(scenes.reactive_channel(nx=nx, ny=ny, q=q, storage="f32")), seed=5000 + i,
                           u_amp=0.005) for i, (nx, ny, q) in enumerate([(33, 12, 0.3), (41, 15, 0.8)])]
    B = lbm.Batch(rc)
    B.configure(*mode)
    B.step(66)
    assert_items_equal_alone(B, rc, 66)


@pytest.mark.parametrize("mode", [MODES[0], MODES[3]], ids=["tiled", "resident"])
def test_batch_of_2d_channels_equals_alone(mode):
    scs = reactive_items("f32")
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(71)  # odd count: a single step after the captured run
    assert_items_equal_alone(B, scs, 71)


@pytest.mark.parametrize("mode", [("resident", 256, 8, 64), ("tiled", 128, 1, 64)])
def test_batch_fp64_item_matches_oracle(mode):
    scs = duct_pipe_items("f64", n=3, lo=16, hi=24)
    B = lbm.Batch(scs)
    B.configure(*mode)
    B.step(66)
    for i, sc in enumerate(scs):
        o = oracle.OracleSim(sc, "ld")
        o.step(66)
        err = field_errors(gpu_moments(B.items[i]), o.moments(), o.mask(), sc.B_ext)
        assert max(err.values()) < 1e-12, (i, err)


def test_batch_run_stops_each_item_where_its_residual_is_below_tol():
    scs = duct_pipe_items("f32", n=4, lo=14, hi=22, seed=77, developed=False, Ha_hi=5.0)
    B = lbm.Batch(scs)
    B.configure("resident", 256, 8, 64)
    tol, I = 1e-6, 100
    steps, res, status = B.run(tol=tol, interval=I, max_steps=40000)
    assert status == ["steady"] * len(scs), (status, steps, res)
    assert (res < tol).all() and (res > 0).all()
    assert len(set(steps.tolist())) > 1  # items converge at their own pace
    for i, sc in enumerate(scs):
        # the same residual with the single-context reduction, evaluated at
        # the same times: snapshot after the two start steps and one interval
        alone = lbm.Lattice(sc)
        alone.step(2 + I)
        alone.reduce()
        t_steady = None
        while alone.time < 40000:
            alone.step(I)
            r = alone.reduce()[0]
            if r < tol:
                t_steady = alone.time
                break
        assert t_steady == steps[i], (i, t_steady, steps[i])
        assert B.items[i].time == steps[i]
        assert np.array_equal(gpu_moments(B.items[i]), gpu_moments(alone))


def test_batch_run_respects_max_steps():
    scs = duct_pipe_items("f32", n=3, lo=30, hi=40, developed=False)
    B = lbm.Batch(scs)
    steps, res, status = B.run(tol=1e-12, interval=50, max_steps=302)
    assert status == ["active"] * 3
    assert (steps == 302).all()  # 2 start steps + 6 intervals of 50
    assert (res > 0).all()


def test_batch_run_flags_a_nonfinite_item_and_keeps_the_others():
    scs = duct_pipe_items("f32", n=3, lo=20, hi=24, developed=False)
    scs[1] = scs[1].with_(accel=(0.5, 0.0, 0.0), tau_f=0.5001)
    B = lbm.Batch(scs)
    steps, res, status = B.run(tol=1e-12, interval=20, max_steps=2002)
    assert status[1] == "nonfinite"
    assert status[0] == status[2] == "active"
    assert steps[1] < 2002 and steps[0] == steps[2] == 2002
    for i in (0, 2):
        assert np.isfinite(gpu_moments(B.items[i])).all()


def test_tuner_candidates_and_real_steps():
    scs = duct_pipe_items("f16", n=6, lo=24, hi=48)
    B = lbm.Batch(scs)
    best, cands = B.tune(trial_steps=64)
    assert len(cands) == 12
    assert all(ms > 0 for _, ms in cands)
    assert best in [c for c, _ in cands]
    assert min(cands, key=lambda c: c[1])[0] == best
    assert B.config == best
    t = B.items[0].time
    assert t == 2 + 12 * 128
    assert_items_equal_alone(B, scs, t)


def test_full_size_fp16_items_against_the_oracle():
    """Eight full-size CFG5 items (sides 64-256) in one FP16 batch, 258 steps
    from a developed state, each against the FP64 oracle run of the same
    item (FP16 storage has no parity bound; the error is reported and held to
    loose bounds)."""
    its = scenes.batch_items(8)
    s16 = [scenes.developed(it.scene, seed=3000 + i, u_amp=0.005) for i, it in enumerate(its)]
    B16 = lbm.Batch(s16)
    B16.configure("resident", 512, 32, 64)
    B16.step(258)
    for i in range(len(its)):
        o = oracle.OracleSim(s16[i].with_(storage="f64"), "f64")
        o.step(258)
        m16 = gpu_moments(B16.items[i])
        err = field_errors(m16, o.moments(), o.mask(), s16[i].B_ext)
        print(i, its[i].shape, its[i].ny, its[i].nz, {k: f"{v:.1e}" for k, v in err.items()}, flush=True)
        assert np.isfinite(m16).all()
        assert err["rho"] < 1e-3 and err["u"] < 2e-2 and err["b"] < 2e-2, (i, err)
    # one item of the FP16 batch against the same item alone
    alone = lbm.Lattice(s16[0])
    alone.step(258)
    assert np.array_equal(gpu_moments(B16.items[0]), gpu_moments(alone))


def test_disabled_items_keep_their_state():
    scs = duct_pipe_items("f32", n=4, lo=20, hi=30)
    B = lbm.Batch(scs)
    B.step(40)
    before = [gpu_moments(it) for it in B.items]
    B.set_active([True, False, True, False])
    B.configure("resident", 256, 8, 64)
    B.step(66)
    assert [it.time for it in B.items] == [106, 40, 106, 40]
    for i in (1, 3):
        assert np.array_equal(gpu_moments(B.items[i]), before[i])
    for i in (0, 2):
        alone = lbm.Lattice(scs[i])
        alone.step(106)
        assert np.array_equal(gpu_moments(B.items[i]), gpu_moments(alone))
    steps, res, status = B.run(tol=1e-12, interval=20, max_steps=100)
    assert status == ["active", "disabled", "active", "disabled"]
    assert steps.tolist() == [100, 0, 100, 0]
    assert [it.time for it in B.items] == [206, 40, 206, 40]


def test_converged_fields_do_not_depend_on_the_start():
    """P13: the same items run to steady state from rest and from a warm start
    of the network's form (smooth axial u_x and b_x) agree to within what their
    residual allows (FP64 storage).  The ducts have half-way walls (d = 0.5),
    where the link updates conserve mass exactly; at other d the mass drifts
    slowly and no steady state exists below the residual of that drift."""
    import dataclasses
    ducts = [it.scene for it in scenes.batch_items(12, side_lo=14, side_hi=20, storage="f64", seed=91, Ha_hi=4.0)
             if it.shape == "duct"][:3]
    scs = [sc.with_(boundaries=[dataclasses.replace(b, q=0.5) for b in sc.boundaries]) for sc in ducts]
    warm = [scenes.axial_start(sc, seed=700 + i) for i, sc in enumerate(scs)]
    out = []
    for group in (scs, warm):
        B = lbm.Batch(group)
        steps, res, status = B.run(tol=3e-12, interval=100, max_steps=200000)
        assert status == ["steady"] * 3, (status, res, steps)
        out.append([gpu_moments(it) for it in B.items])
    for i, sc in enumerate(scs):
        a, b = out[0][i], out[1][i]
        # the slowest mode decays at about nu pi^2 (1/a^2 + 1/b^2) per step, so a
        # residual of 3e-12 leaves at most ~3e-12 / lambda ~ 1e-8 of the field
        # (the FP64 oracle: 2e-8 at most on these items)
        for q in (1, 5):
            d = np.abs(a[..., q] - b[..., q]).max() / max(np.abs(a[..., q] - sc.B_ext[0] * (q == 5)).max(), 1e-30)
            assert d < 1e-7, (i, q, d)


def test_fp64_batch_steady_state_is_a_fixed_point_of_the_oracle():
    """The time-to-steady study takes its reference from FP64 batch runs
    converged to a residual of 1e-11.  Handed to the CPU oracle, such a state
    must stay put: over 2000 oracle steps u and b change by less than
    2000 x the residual bound (relative), far below the field errors the
    study compares."""
    from .gpu_util import gpu_populations
    its = scenes.batch_items(3, seed=scenes.BASE_SEED + 62, side_lo=20, side_hi=28, c_lo=0.05, c_hi=1.0,
                             Ha_hi=20.0, storage="f64", ducts_only=True, q_duct=0.5)
    scs = [it.scene for it in its]
    B = lbm.Batch(scs)
    steps, res, status = B.run(tol=1e-11, interval=1000, max_steps=2_000_000)
    assert status == ["steady"] * len(scs), (status, res)
    for i, sc in enumerate(scs):
        lat = B.items[i]
        o = oracle.OracleSim(sc, "ld")
        o.set_populations(0, gpu_populations(lat, 0))
        o.set_populations(2, gpu_populations(lat, 2))
        m0 = o.moments()
        mg = gpu_moments(lat)
        sel = o.mask().astype(bool)
        # the handed-over state is the GPU's
        assert np.abs(m0 - mg)[sel].max() < 1e-13
        o.step(2000)
        m1 = o.moments()
        for q, name in ((1, "u"), (5, "b")):
            ref = m0[..., q][sel] - (sc.B_ext[0] if q == 5 else 0.0)
            d = np.linalg.norm((m1 - m0)[..., q][sel]) / np.linalg.norm(ref)
            print(i, name, f"{d:.1e}", flush=True)
            assert d < 2000 * 1e-11 * 10, (i, name, d)
