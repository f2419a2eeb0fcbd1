"""Host-side checks of the study scripts: their closed forms agree with the
independently written ones of oracle/analytic.py, and their case lists are
the paper's configurations (no device work)."""
import math

import numpy as np

import scenes
from oracle import analytic as an
from paper_2506_00907_amd import channel_study, lbm, stokes_study


def test_stokes_study_closed_form_and_cases():
    y = np.linspace(0.0, 100.0, 21)
    for t in (0.0, 123.0, 7.5e4):
        a = stokes_study.closed_form(y, t, 1e-3, 2 * math.pi / 1e5, 0.1, 100.0)
        b = an.stokes_second(y, t, 1e-3, 2 * math.pi / 1e5, 0.1, 100.0)
        assert np.allclose(a, b, rtol=1e-13, atol=1e-18)
    cs = stokes_study.cases("f64")
    assert len(cs) == 6
    for c in cs:
        sc = c["scene"]
        # H = 100 spacings between the walls in every layout (Section 5.2)
        assert sc.n[2] - 1 + 2 * c["q"] == stokes_study.H
        assert sc.n[:2] == (5, 5) and abs(sc.wall_omega - 2 * math.pi / 1e5) < 1e-18
        _, ll = lbm.build_links(sc)
        d = 0.5 if c["name"] != "full" else 1.0
        assert np.all(ll["d"] == d)


def test_channel_study_duct_series_and_layouts():
    x = np.linspace(-9.5, 9.5, 7)
    X, Y = np.meshgrid(x, x, indexing="ij")
    assert np.allclose(channel_study.duct(X, Y, 10.0, 1e-4, 0.07), an.duct_poiseuille(X, Y, 10.0, 10.0, 1e-4, 0.07),
                       rtol=1e-13, atol=1e-20)
    half = scenes.channel_reservoirs("half")
    full = scenes.channel_reservoirs("full")
    # 22 x 22 and 21 x 21 inlet nodes (Section 5.1), 100 spacings between inlet and outlet
    assert half.n == (22, 22, 100) and full.n == (21, 21, 99)
    assert half.n[2] - 1 + 2 * 0.5 == 100 and full.n[2] - 1 + 2 * 1.0 == 100
