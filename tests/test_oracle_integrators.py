"""Pins of the oracle's integrator variants (Sec. 2.7): implicit Gauss with two
stages (eq. gaussAB), Simpson quadrature of the closed form (eq. simpson), the
recursion of Alg. adaptiverk, and the equilibrium-intensity field (eq. BIrelation).

Checked against what the mathematics fixes independently: the (2,2) Pade
approximant of exp(-x), exactness of Simpson for a cubic emission without
absorption (3-point Gauss-Legendre in numpy), fourth-order convergence to a
scipy quadrature of the exact solution, and the reduction of the recursion to
uniform substeps for constant coefficients.
"""

import math

import numpy as np

import synth
from test_oracle_pins import _exact_linear

GAUSS, SIMPSON, RK4 = 2, 3, 1


def _linear_leaf():
    # unit cube at level 0, ray along +x; kappa 0.4 -> 2.6 and eps 1.0 -> 0.2 along x
    kc = np.array([0.4, 2.6] * 4)
    ec = np.array([1.0, 0.2] * 4)
    return kc, ec, np.array([0.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])


def test_gauss2_constant_coefficients_is_the_pade_approximant(oracle_mod):
    O = oracle_mod
    rho, r = np.array([0.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])
    for beta, gamma, L in [(0.3, 0.7, 1.0), (2.0, 0.4, 1.0), (5.0, 1.0, 0.6)]:
        ab, _ = O.segment(0, [beta], [gamma], 0, 0, 0, 0, rho, r, 0.0, L, GAUSS, 1)
        x = beta * L
        pade = (1 - x / 2 + x * x / 12) / (1 + x / 2 + x * x / 12)
        assert math.isclose(ab[0], pade, rel_tol=1e-14)
        assert math.isclose(ab[1], gamma / beta * (1 - pade), rel_tol=1e-13)  # B = I (1 - A)


def _orders(O, method, kc, ec, ex):
    rho, r = np.array([0.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])
    errs = []
    for sub in (2, 4, 8, 16, 32):
        ab, _ = O.segment(1, kc, ec, 0, 0, 0, 0, rho, r, 0.0, 1.0, method, sub)
        errs.append(abs(ab[0] - ex[0]) + abs(ab[1] - ex[1]))
    return [errs[i] / errs[i + 1] for i in range(4)]


def test_gauss2_converges_at_order_four(oracle_mod):
    kc, ec, _, _ = _linear_leaf()
    ratios = _orders(oracle_mod, GAUSS, kc, ec, _exact_linear(2.6, 0.4, 0.2, 1.0, 1.0))
    # the first doublings are pre-asymptotic; the last ratio is close to 2^4
    assert all(12.0 < q < 24.0 for q in ratios) and 15.0 < ratios[-1] < 17.0, ratios


def test_simpson_orders(oracle_mod):
    """With constant kappa the midpoint attenuation sqrt(A) is exact and Simpson is
    fourth order; with kappa varying along the ray it is off by O(dx^2) in the
    midpoint weight, and B converges at second order."""
    O = oracle_mod
    kc, ec, _, _ = _linear_leaf()
    flat = np.full(8, 1.3)
    ratios = _orders(O, SIMPSON, flat, ec, _exact_linear(1.3, 1.3, 0.2, 1.0, 1.0))
    assert 15.0 < ratios[-1] < 17.0, ratios
    ratios = _orders(O, SIMPSON, kc, ec, _exact_linear(2.6, 0.4, 0.2, 1.0, 1.0))
    assert 3.8 < ratios[-1] < 4.2, ratios


def test_simpson_is_exact_for_emission_without_absorption(oracle_mod):
    """kappa = 0: B is the integral of the trilinear eps along the ray, a cubic."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    ec = rng.uniform(0.0, 1.0, 8)
    rho, r = np.array([-0.2, 0.05, 0.1]), np.array([1.0, 0.6, 0.45])
    s0, s1 = 0.25, 0.55  # inside the level-1 leaf at the origin
    lo, h = np.zeros(3), 0.5
    xg, wg = np.polynomial.legendre.leggauss(3)
    exact = 0.0
    for xq, wq in zip(xg, wg):
        s = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * xq
        xi = (rho + s * r - lo) / h
        val = 0.0
        for c in range(8):
            w = 1.0
            for k in range(3):
                w *= xi[k] if (c >> k) & 1 else 1 - xi[k]
            val += ec[c] * w
        exact += 0.5 * (s1 - s0) * wq * val
    exact *= np.linalg.norm(r)
    for sub in (1, 2, 4):
        ab, _ = O.segment(1, np.zeros(8), ec, 1, 0, 0, 0, rho, r, s0, s1, SIMPSON, sub)
        assert ab[0] == 1.0
        assert math.isclose(ab[1], exact, rel_tol=1e-13), (sub, ab[1], exact)


def test_recursion_reduces_to_uniform_substeps_for_constant_coefficients(oracle_mod):
    O = oracle_mod
    rho, r = np.array([0.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])
    beta, gamma, L = 1.7, 0.6, 1.0
    for m in range(0, 5):
        c_rk = beta * L / 2 ** m * 1.0001  # pieces of length L / 2^m are the first to pass
        for method in (RK4, GAUSS, SIMPSON):
            ad, _ = O.segment(0, [beta], [gamma], 0, 0, 0, 0, rho, r, 0.0, L, method, 1, c_rk)
            un, _ = O.segment(0, [beta], [gamma], 0, 0, 0, 0, rho, r, 0.0, L, method, 2 ** m)
            np.testing.assert_allclose(ad, un, rtol=1e-13, atol=0)


def test_recursion_accuracy_improves_with_the_stability_parameter(oracle_mod):
    """Smaller c_RK, smaller pieces where kappa is large, smaller error (Sec. 2.7)."""
    O = oracle_mod
    kc, ec, rho, r = _linear_leaf()
    Aex, Bex = _exact_linear(2.6, 0.4, 0.2, 1.0, 1.0)
    for method in (RK4, GAUSS, SIMPSON):
        errs = []
        for c_rk in (0.4, 0.2, 0.1, 0.05, 0.025):
            ab, _ = O.segment(1, kc, ec, 0, 0, 0, 0, rho, r, 0.0, 1.0, method, 1, c_rk)
            errs.append(abs(ab[0] - Aex) + abs(ab[1] - Bex))
        assert all(errs[i + 1] < errs[i] for i in range(4)), (method, errs)
        # RK4 and Gauss: fourth order in the piece length; Simpson: second order
        # while kappa varies along the ray (see test_simpson_orders)
        assert errs[0] / errs[-1] > (8.0 ** 4 if method != SIMPSON else 3.0 ** 4), (method, errs)
    # no split when c_RK exceeds every dx beta: the single-step value
    for method in (GAUSS, SIMPSON):
        a, _ = O.segment(1, kc, ec, 0, 0, 0, 0, rho, r, 0.0, 1.0, method, 1, 100.0)
        b, _ = O.segment(1, kc, ec, 0, 0, 0, 0, rho, r, 0.0, 1.0, method, 1)
        assert np.array_equal(a, b)


def test_equilibrium_intensity_fields_match_emission_fields(oracle_mod):
    """eq. BIrelation: constant (kappa, I) renders as (kappa, eps = kappa I)."""
    O = oracle_mod
    sc = synth.small_scene(12, w=40, h=32)
    N = sc.forest.nleaves
    rng = np.random.default_rng(12)
    kap = rng.uniform(0.1, 2.0, N).astype(np.float32)
    inten = rng.uniform(0.0, 1.5, N).astype(np.float32)
    eq = synth.equilibrium_fields(kap, inten)
    em = synth.Fields("const", kap[None].astype(np.float64), (kap.astype(np.float64) * inten)[None])
    for method in ("analytic", "rk4", "gauss2", "simpson"):
        a = O.render(sc.forest, eq, sc.cameras[0], method, 2)
        b = O.render(sc.forest, em, sc.cameras[0], method, 2)
        for k in ("A", "B", "I"):
            np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-14)
        assert a["segments"] > 0


def test_integrator_gradients_match_finite_differences(oracle_mod):
    """The oracle's coefficient gradients (dual numbers through eq. gaussAB and eq. simpson over equal pieces,
    and through Alg. adaptiverk's pieces, whose split decisions a step of 1e-6 leaves unchanged) against central
    finite differences of its own loss L = sum (I - I*)^2, trilinear fields, background 0.4."""
    O = oracle_mod
    s = synth.small_scene(12, lmin=1, lmax=3, ngauss=3, w=24, h=18, background=0.4)
    cam = s.cameras[0]
    f = s.fields
    kap0, eps0 = f.kappa.astype(np.float64), f.eps.astype(np.float64)
    rng = np.random.default_rng(13)
    for method, sub, c_rk in (("gauss2", 4, 0.0), ("simpson", 2, 0.0), ("gauss2", 1, 0.0), ("rk4", 1, 0.05),
                              ("gauss2", 2, 0.05), ("simpson", 1, 0.05)):
        r = O.render(s.forest, f, cam, method, sub, c_rk=c_rk)
        target = r["I"] + rng.normal(0, 0.05, r["I"].shape)

        def loss(kap, eps):
            return ((O.render(s.forest, f, cam, method, sub, kappa=kap, eps=eps, c_rk=c_rk)["I"] - target) ** 2).sum()

        gk, ge = O.grad(s.forest, f, cam, 2 * (r["I"] - target), method, sub, c_rk=c_rk)
        leaves = np.flatnonzero(np.abs(gk).sum(0) > 0)
        assert len(leaves) >= 5
        for l in rng.choice(leaves, 5, replace=False):
            c = int(rng.integers(8))
            for which in ("k", "e"):
                kp, km, ep, em = kap0.copy(), kap0.copy(), eps0.copy(), eps0.copy()
                base = kap0 if which == "k" else eps0
                h = 1e-6 * max(1.0, abs(base[c, l]))
                if which == "k":
                    kp[c, l] += h
                    km[c, l] -= h
                else:
                    ep[c, l] += h
                    em[c, l] -= h
                fd = (loss(kp, ep) - loss(km, em)) / (2 * h)
                an = gk[c, l] if which == "k" else ge[c, l]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (method, sub, c_rk, which, l, c, fd, an)


def test_equilibrium_field_gradient_matches_finite_differences(oracle_mod):
    """eq. BIrelation fields (constant kappa, equilibrium intensity I in place of eps), closed form: the oracle's
    gradients with respect to kappa and I against central finite differences of L = sum (I_pix - I*)^2."""
    O = oracle_mod
    s = synth.small_scene(14, lmin=1, lmax=3, ngauss=3, w=24, h=18, background=0.3)
    rng = np.random.default_rng(14)
    N = s.forest.nleaves
    f = synth.equilibrium_fields(rng.uniform(0.1, 3.0, N), rng.uniform(0.0, 1.5, N))
    cam = s.cameras[0]
    r = O.render(s.forest, f, cam, "analytic", 1)
    target = r["I"] + rng.normal(0, 0.05, r["I"].shape)
    kap0, int0 = f.kappa.astype(np.float64), f.eps.astype(np.float64)

    def loss(kap, inten):
        return ((O.render(s.forest, f, cam, "analytic", 1, kappa=kap, eps=inten)["I"] - target) ** 2).sum()

    gk, gi = O.grad(s.forest, f, cam, 2 * (r["I"] - target), "analytic", 1)
    leaves = np.flatnonzero(np.abs(gk).sum(0) > 0)
    for l in rng.choice(leaves, 8, replace=False):
        for which in ("k", "i"):
            kp, km, ip, im = kap0.copy(), kap0.copy(), int0.copy(), int0.copy()
            base = kap0 if which == "k" else int0
            h = 1e-6 * max(1.0, abs(base[0, l]))
            if which == "k":
                kp[0, l] += h
                km[0, l] -= h
            else:
                ip[0, l] += h
                im[0, l] -= h
            fd = (loss(kp, ip) - loss(km, im)) / (2 * h)
            an = gk[0, l] if which == "k" else gi[0, l]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, l, fd, an)
