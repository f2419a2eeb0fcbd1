"""lbm_reduce_static (the reductions with the library's own device scratch)
against lbm_reduce, through the C ABI: two contexts with the same seeded
state, one reduced by each entry point, compared on two calls in a row; then
the same on a smaller lattice, whose call finds the larger lattice's records
still in the shared array.  FP64 sums of up to ~10^4 terms in another order:
relative 1e-13 (each sum's rounding is ~n eps |terms| / |sum| with terms of
one sign); the non-finite count and the step window exactly."""
import numpy as np
import pytest

import scenes
from paper_2506_00907_amd import _lib as L
from paper_2506_00907_amd import lbm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(sc):
    return lbm.Lattice(sc), lbm.Lattice(sc)


def _check(a, b):
    assert a[7] == b[7] == 0.0
    assert a[6] == b[6]
    np.testing.assert_allclose(b[1:6], a[1:6], rtol=1e-13, atol=1e-300)
    if a[0] < 0:
        assert b[0] == a[0]
    else:
        assert abs(b[0] - a[0]) <= 1e-12 * a[0], (a[0], b[0])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_reduce_static_matches_reduce_on_two_sizes(storage):
    big = scenes.developed(scenes.hartmann_couette(nx=96, ny=61, c_top=0.1, storage=storage))
    small = scenes.developed(scenes.hartmann_couette(nx=12, ny=9, c_top=0.1, storage=storage))
    for sc in (big, small):
        print(f"\n[case] lbm_reduce_static {sc.name} {sc.n} {storage}", flush=True)
        l_ref, l_st = _pair(sc)
        for k in range(2):
            l_ref.step(30)
            l_st.step(30)
            a = l_ref.reduce()
            b = l_st.reduce(static_scratch=True)
            _check(a, b)
            if k == 1:
                assert a[0] > 0.0


def test_reduce_static_rejects_lattices_beyond_its_scratch():
    nmax = 256 * L.LBM_REDUCE_STATIC_MAX_BLOCKS
    # a D2Q9 channel of 8192 x 4096 fluid rows: 8192 x 4098 padded nodes
    sc = scenes.poiseuille(nx=8192, ny=4096, storage="f32")
    assert 8192 * 4098 > nmax
    print(f"\n[case] lbm_reduce_static too large {sc.n}", flush=True)
    lat = lbm.Lattice(sc)
    out = (L.C.c_double * 8)()
    code = L.lib().lbm_reduce_static(lat.ctx, out)
    assert code == -2  # LBM_ESIZE
    assert b"static reduction scratch" in L.lib().lbm_last_error(lat.ctx)
    # the ordinary reduction still works on it
    r = lat.reduce()
    assert r[7] == 0.0
