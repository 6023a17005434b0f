"""Pins of the oracle's weighted absolute sensitivities (grad_abs), the bound
used for end-to-end gradient parity: sum_p w_p |dI_p/dtheta| for w >= 0.

* one selected pixel: exactly |dI_p/dtheta| times its weight, i.e. the absolute
  value of the signed gradient with dL/dI = 1 at that pixel;
* several pixels: the sum of those single-pixel absolute gradients (brute force
  over separate one-pixel calls);
* never below the absolute value of the signed gradient (triangle inequality),
  and equal to it where every pixel's derivative has the same sign (emission
  with a constant absorption and emission per leaf: dI/deps >= 0);
* negative weights are refused.
"""

import numpy as np
import pytest

import synth


def _scene():
    return synth.small_scene(7, lmin=1, lmax=4, ngauss=3, w=20, h=16, background=0.5)


def test_single_pixel_is_absolute_signed_gradient(oracle_mod):
    s = _scene()
    cam = s.cameras[0]
    ref = oracle_mod.render(s.forest, s.fields, cam, "rk4", 4)
    p = int(np.argmax(ref["nseg"]))
    pix = np.array([p], np.int64)
    gk, ge = oracle_mod.grad(s.forest, s.fields, cam, np.array([1.0]), "rk4", 4, pixels=pix)
    ak, ae = oracle_mod.grad_abs(s.forest, s.fields, cam, np.array([1.0]), "rk4", 4, pixels=pix)
    assert np.abs(gk).max() > 0
    assert np.array_equal(ak, np.abs(gk)) and np.array_equal(ae, np.abs(ge))
    hk, he = oracle_mod.grad_abs(s.forest, s.fields, cam, np.array([0.25]), "rk4", 4, pixels=pix)
    assert np.array_equal(hk, 0.25 * ak) and np.array_equal(he, 0.25 * ae)


def test_sum_over_pixels_is_brute_force_sum(oracle_mod):
    s = _scene()
    cam = s.cameras[0]
    rng = np.random.default_rng(71)
    pix = np.sort(rng.choice(cam.npix, 40, replace=False)).astype(np.int64)
    w = rng.uniform(0.0, 2.0, pix.shape[0])
    ak, ae = oracle_mod.grad_abs(s.forest, s.fields, cam, w, "rk4", 4, pixels=pix)
    bk, be = np.zeros_like(ak), np.zeros_like(ae)
    for q, p in enumerate(pix):
        gk, ge = oracle_mod.grad(s.forest, s.fields, cam, np.array([w[q]]), "rk4", 4,
                                 pixels=np.array([p], np.int64))
        bk += np.abs(gk)
        be += np.abs(ge)
    assert np.abs(bk).max() > 0
    np.testing.assert_allclose(ak, bk, rtol=1e-12, atol=1e-15 * np.abs(bk).max())
    np.testing.assert_allclose(ae, be, rtol=1e-12, atol=1e-15 * np.abs(be).max())


def test_bounds_signed_gradient_and_equals_it_for_sign_definite_emission(oracle_mod):
    s = synth.small_scene(8, lmin=1, lmax=3, ngauss=2, w=24, h=20, method="analytic")
    cam = s.cameras[0]
    rng = np.random.default_rng(72)
    w = rng.uniform(0.0, 1.0, cam.npix)
    gk, ge = oracle_mod.grad(s.forest, s.fields, cam, w, "analytic", 1)
    ak, ae = oracle_mod.grad_abs(s.forest, s.fields, cam, w, "analytic", 1)
    assert np.all(ak >= np.abs(gk) * (1 - 1e-12)) and np.all(ae >= np.abs(ge) * (1 - 1e-12))
    # closed form, constant coefficients: dI/deps = T (1 - A) / kappa >= 0, and dI/dkappa <= 0
    np.testing.assert_allclose(ae, ge, rtol=1e-12, atol=0)
    np.testing.assert_allclose(ak, -gk, rtol=1e-12, atol=0)


def test_negative_weight_refused(oracle_mod):
    s = _scene()
    w = np.zeros(s.cameras[0].npix)
    w[3] = -1e-9
    with pytest.raises(ValueError):
        oracle_mod.grad_abs(s.forest, s.fields, s.cameras[0], w, "rk4", 4)
