"""The library's host resampler (lbs_resample_curve_host: FFT, fine tables,
Newton on interpolants) against the oracle's plain arclength resampling
(trigonometric interpolant, adaptive quadrature, root bracketing) and the
reparametrized circle's closed form.  No GPU needed."""
import os

import numpy as np
import pytest

import synth
from oracle.geometry import curve_on_sphere
from oracle.resample import resample


@pytest.fixture(scope="module")
def lbs():
    from paper_1306_0612_amd import lbs as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1306_0612_amd import build
        build.build()
    mod.load()
    return mod


def test_circle_closed_form(lbs):
    c = np.array([0.3, -0.5, 0.8])
    c /= np.linalg.norm(c)
    f1 = np.cross(c, [1.0, 0.0, 0.0])
    f1 /= np.linalg.norm(f1)
    f2 = np.cross(c, f1)
    rho = 0.35
    for n_in in (64, 75):            # power of two and Bluestein lengths
        tau = 2 * np.pi * np.arange(n_in) / n_in
        th_in = tau + 0.3 * np.sin(tau)
        x_in = (np.cos(rho) * c + np.sin(rho) * (np.cos(th_in)[:, None] * f1
                                                 + np.sin(th_in)[:, None] * f2))
        x, xt, xtt, L = lbs.resample_curve(x_in, c, 48)
        th = 2 * np.pi * np.arange(48) / 48
        u = np.cos(th)[:, None] * f1 + np.sin(th)[:, None] * f2
        v = -np.sin(th)[:, None] * f1 + np.cos(th)[:, None] * f2
        assert abs(L - 2 * np.pi * np.sin(rho)) < 1e-13
        assert np.abs(x - (np.cos(rho) * c + np.sin(rho) * u)).max() < 1e-13
        assert np.abs(xt - np.sin(rho) * v).max() < 1e-12
        assert np.abs(xtt + np.sin(rho) * u).max() < 1e-10


@pytest.mark.parametrize("n_in,n_out,modes", [(256, 120, 0), (301, 97, 0),
                                              (256, 90, 40)])
def test_matches_oracle(lbs, n_in, n_out, modes):
    isl = synth.star_islands(31, 1, (0.15, 0.15), k_range=(3, 3), nodes=n_in)
    x_in, _, _ = curve_on_sphere(isl.center[0], isl.e1[0], isl.r0[0],
                                 isl.coef[0], n_in)
    ref = resample(x_in, isl.center[0], n_out, modes or None)
    got = lbs.resample_curve(x_in, isl.center[0], n_out, modes)
    assert abs(got[3] - ref[3]) < 1e-13 * ref[3]
    # the two transforms' rounding noise in the top modes (~1e-16 each)
    # differs, and x_t, x_tt weigh mode k by k and k^2
    for a, b, tol in zip(got[:3], ref[:3], (1e-13, 1e-11, 1e-9)):
        assert np.abs(a - b).max() < tol * np.abs(b).max()


def test_rejects_bad_input(lbs):
    c = np.array([0.0, 0.0, -1.0])
    x = np.tile(c, (16, 1))
    x[3] = -c                               # opposite the centre
    with pytest.raises(lbs.LBSError) as e:
        lbs.resample_curve(x, c, 16)
    assert e.value.status == "LBS_ERR_GEOMETRY"
    with pytest.raises(lbs.LBSError) as e:
        lbs.resample_curve(np.tile(c, (16, 1)), c, 16, n_modes=8)
    assert e.value.status == "LBS_ERR_INVALID_ARG"
