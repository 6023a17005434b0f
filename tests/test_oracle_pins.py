"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, group identities, Taylor expansions, independent quadrature, an
independent ray/cube intersection, a hand-written column formula for the
axis-aligned workload, brute-force marching and finite differences.
"""

import math

import numpy as np
import pytest

import synth


def _rng(k=0):
    return np.random.default_rng([7, 7, k])


# ---------------------------------------------------------------- group (Sec. 2.4-2.6)


def test_group_identity_inverse_associative(oracle_mod):
    O = oracle_mod
    rng = _rng(1)
    for _ in range(200):
        s1, s2, s3 = (np.array([rng.uniform(0.01, 1.5), rng.normal()]) for _ in range(3))
        # identity (1, 0) on both sides (eq. identityinverse)
        np.testing.assert_allclose(O.combine([1.0, 0.0], s1), s1, rtol=0, atol=0)
        np.testing.assert_allclose(O.combine(s1, [1.0, 0.0]), s1, rtol=0, atol=0)
        # inverse on both sides
        np.testing.assert_allclose(O.combine(s1, O.inverse(s1)), [1.0, 0.0], atol=1e-12)
        np.testing.assert_allclose(O.combine(O.inverse(s1), s1), [1.0, 0.0], atol=1e-12)
        # associativity (theorem in Sec. 2.4)
        a = O.combine(O.combine(s1, s2), s3)
        b = O.combine(s1, O.combine(s2, s3))
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


def test_group_is_not_abelian(oracle_mod):
    O = oracle_mod
    s1, s2 = np.array([0.5, 0.3]), np.array([0.8, 0.1])
    assert abs(O.combine(s1, s2)[1] - O.combine(s2, s1)[1]) > 1e-3
    # the nearer operand is the left one: applying to I goes far segment first
    I1 = 0.7
    near_then_far = s1[0] * (s2[0] * I1 + s2[1]) + s1[1]
    c = O.combine(s1, s2)
    assert math.isclose(c[0] * I1 + c[1], near_then_far, rel_tol=1e-15)


def test_split_then_combine_reproduces(oracle_mod):
    O = oracle_mod
    rng = _rng(2)
    for _ in range(100):
        beta, gamma, dx = rng.uniform(0.01, 3), rng.uniform(-1, 1), rng.uniform(0.01, 2)
        A = math.exp(-beta * dx)
        s = np.array([A, gamma / beta * (1 - A)])
        f = rng.uniform(0.05, 0.95)
        p1, p2 = O.split(s, f)
        # each piece is the constant-coefficient segment of its own length (eq. segsplit)
        A1 = math.exp(-beta * dx * f)
        assert math.isclose(p1[0], A1, rel_tol=1e-12)
        assert math.isclose(p1[1], gamma / beta * (1 - A1), rel_tol=1e-9, abs_tol=1e-14)
        # in either order, the pieces combine back to the segment
        np.testing.assert_allclose(O.combine(p1, p2), s, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(O.combine(p2, p1), s, rtol=1e-12, atol=1e-14)
    # transparent special case A = 1: B splits proportionally
    p1, p2 = O.split([1.0, 0.6], 0.25)
    np.testing.assert_allclose(p1, [1.0, 0.15])
    np.testing.assert_allclose(p2, [1.0, 0.45])


def test_average_and_physical_inverse(oracle_mod):
    O = oracle_mod
    s = np.array([0.4, 0.25])
    np.testing.assert_allclose(O.average(s, s), s, rtol=1e-15)
    np.testing.assert_allclose(O.average([0.25, 0.2], [0.64, 0.6]), [0.4, 0.4], rtol=1e-15)
    rng = _rng(3)
    for _ in range(50):
        beta, gamma, dx = rng.uniform(0.01, 3), rng.uniform(0, 2), rng.uniform(0.01, 2)
        A = math.exp(-beta * dx)
        bg = O.physical([A, gamma / beta * (1 - A)], dx)  # eq. betagammafromAB
        np.testing.assert_allclose(bg, [beta, gamma], rtol=1e-10)


def test_reversal_is_negated_coefficients(oracle_mod):
    """(-)(A,B) = f(-beta, -gamma) for constant coefficients (eq. substbetagamma)."""
    O = oracle_mod
    rho, r = np.zeros(3), np.array([1.0, 0.0, 0.0])
    for beta, gamma in [(0.7, 0.4), (2.0, -0.3), (0.05, 1.2)]:
        ab, _ = O.segment(0, [beta], [gamma], 0, 0, 0, 0, rho, r, 0.0, 0.6, 0)
        ab_neg, _ = O.segment(0, [-beta], [-gamma], 0, 0, 0, 0, rho, r, 0.0, 0.6, 0)
        np.testing.assert_allclose(ab_neg, O.inverse(ab), rtol=1e-13)


# ---------------------------------------------------------------- segment values (Sec. 2.3, 2.7)


def test_constant_segment_closed_form(oracle_mod):
    O = oracle_mod
    rho, r = np.zeros(3), np.array([0.0, 1.0, 0.0])
    for kap, eps, L in [(0.7, 0.3, 0.5), (2.0, 1.0, 1.0), (1e-9, 0.5, 0.25), (0.0, 0.8, 0.3)]:
        ab, dab = O.segment(0, [kap], [eps], 0, 0, 0, 0, rho, r, 0.25, 0.25 + L, 0)
        A = math.exp(-kap * L)
        B = eps * L if kap == 0 else eps / kap * (1 - A) if kap > 1e-6 else eps * L * (1 - kap * L / 2)
        assert math.isclose(ab[0], A, rel_tol=1e-14)
        assert math.isclose(ab[1], B, rel_tol=1e-12)
        # derivatives: dA/dkap = -L A, dB/deps = B/eps
        assert math.isclose(dab[0, 0], -L * A, rel_tol=1e-12)
        assert math.isclose(dab[1, 1], B / eps, rel_tol=1e-12)
    # kappa = 0 exactly: A = 1, B = eps L
    ab, _ = O.segment(0, [0.0], [0.8], 0, 0, 0, 0, rho, r, 0.0, 0.3, 0)
    assert ab[0] == 1.0 and math.isclose(ab[1], 0.8 * 0.3, rel_tol=1e-15)


def test_rk4_step_taylor_forms(oracle_mod):
    O = oracle_mod
    for beta, gamma, h in [(0.3, 0.7, 0.5), (1.9, 0.2, 0.4), (0.05, 1.0, 2.0)]:
        x = beta * h
        A, B = O.rk4_step([beta] * 4, [gamma] * 4, h)
        assert math.isclose(A, 1 - x + x ** 2 / 2 - x ** 3 / 6 + x ** 4 / 24, rel_tol=1e-14)
        assert math.isclose(B, gamma * h * (1 - x / 2 + x ** 2 / 6 - x ** 3 / 24), rel_tol=1e-14)
    # the amplification polynomial stays positive; its minimum is about 0.2704
    xs = np.linspace(0, 4, 40001)
    amp = np.array([O.rk4_step([1.0] * 4, [0.0] * 4, x)[0] for x in xs[::100]])
    assert amp.min() > 0.27
    poly = 1 - xs + xs ** 2 / 2 - xs ** 3 / 6 + xs ** 4 / 24
    assert abs(poly.min() - 0.27039) < 1e-4


def _exact_linear(b0, b1, g0, g1, L):
    """Exact (A, B) for beta, gamma varying linearly from the far end (x=0) to the near end (x=L)."""
    from scipy.integrate import quad

    beta = lambda x: b0 + (b1 - b0) * x / L  # noqa: E731
    gamma = lambda x: g0 + (g1 - g0) * x / L  # noqa: E731
    Bint = lambda x: b0 * x + (b1 - b0) * x * x / (2 * L)  # noqa: E731  integral of beta from 0
    A = math.exp(-Bint(L))
    B = quad(lambda x: gamma(x) * math.exp(-(Bint(L) - Bint(x))), 0, L, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    return A, B


def test_rk4_substeps_converge_at_order_four(oracle_mod):
    """A trilinear field varying along the ray: RK4 error drops ~16x per substep doubling."""
    O = oracle_mod
    # leaf = unit cube at level 0; ray along +x through its middle; field linear in x
    kc = np.array([0.4, 2.6] * 4)  # corner c: bx = c & 1 -> kappa 0.4 at x=0, 2.6 at x=1
    ec = np.array([1.0, 0.2] * 4)
    rho, r = np.array([0.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])
    # far end s_out = 1 (x=1), near end s_in = 0: beta goes 2.6 -> 0.4 from far to near
    Aex, Bex = _exact_linear(2.6, 0.4, 0.2, 1.0, 1.0)
    errs = []
    for sub in (2, 4, 8, 16):
        ab, _ = O.segment(1, kc, ec, 0, 0, 0, 0, rho, r, 0.0, 1.0, 1, sub)
        errs.append(abs(ab[0] - Aex) + abs(ab[1] - Bex))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(12.0 < q < 20.0 for q in ratios), ratios


def test_trilinear_gradient_matches_finite_differences(oracle_mod):
    O = oracle_mod
    rng = _rng(5)
    kc, ec = rng.uniform(0.2, 2.0, 8), rng.uniform(0.0, 1.0, 8)
    rho = np.array([-0.3, 0.1, 0.2])
    r = np.array([1.0, 0.35, 0.5])
    ab, dab = O.segment(1, kc, ec, 1, 0, 0, 0, rho, r, 0.4, 0.9, 1, 4)
    h = 1e-6
    for p in range(16):
        kp, ep = kc.copy(), ec.copy()
        km, em = kc.copy(), ec.copy()
        if p < 8:
            kp[p] += h
            km[p] -= h
        else:
            ep[p - 8] += h
            em[p - 8] -= h
        fp, _ = O.segment(1, kp, ep, 1, 0, 0, 0, rho, r, 0.4, 0.9, 1, 4)
        fm, _ = O.segment(1, km, em, 1, 0, 0, 0, rho, r, 0.4, 0.9, 1, 4)
        np.testing.assert_allclose(dab[:, p], (fp - fm) / (2 * h), rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------- visibility / pairing (Sec. 2.2, 3.1)


def test_config1_rectangles_and_segment_count(oracle_mod):
    O = oracle_mod
    s = synth.config_scene(1)
    rect, nvis = O.prune(s.forest, s.cameras[0].raw())
    assert nvis == 512
    assert np.all(rect[0, :, 1] - rect[0, :, 0] == 7) and np.all(rect[0, :, 3] - rect[0, :, 2] == 7)
    r = O.render(s.forest, s.fields, s.cameras[0], method="analytic")
    assert r["segments"] == 32768 and np.all(r["nseg"] == 8) and r["overlaps"] == 0


def test_camera_looking_away_sees_nothing(oracle_mod):
    O = oracle_mod
    s = synth.small_scene(0)
    c = synth.perspective_camera([0.5, 0.5, 3.0], [0.5, 0.5, 9.0], [0, 1, 0], 1.0, 42, 64, 48, 5.0)
    rect, nvis = O.prune(s.forest, c.raw())
    assert nvis == 0
    r = O.render(s.forest, s.fields, c)
    assert r["segments"] == 0 and np.all(r["A"] == 1.0) and np.all(r["B"] == 0.0)


def _project(cam, pts):
    """Independent pinhole projection of world points to continuous pixel coordinates."""
    v = np.asarray(cam.v)
    n = np.linalg.norm(v)
    d = pts - cam.o
    X, Y, Z = d @ cam.t, d @ cam.u, d @ (v / n)
    return X / Z * n / cam.ell + (cam.w - 1) / 2, Y / Z * n / cam.ell + (cam.h - 1) / 2, Z


def test_rectangles_are_conservative_and_nested(oracle_mod):
    O = oracle_mod
    rng = _rng(6)
    s = synth.small_scene(1, w=80, h=60)
    cam = s.cameras[0]
    rect, _ = O.prune(s.forest, cam.raw())
    f = s.forest
    scale = 2.0 ** -synth.QMAX
    for l in rng.choice(f.nleaves, 300, replace=False):
        lo = np.array([f.x[l], f.y[l], f.z[l]], np.float64) * scale
        h = 2.0 ** -int(f.level[l])
        pts = lo + h * rng.uniform(0, 1, (500, 3))
        px, py, _ = _project(cam, pts)
        i0, i1, j0, j1 = rect[0, l]
        inside = (px >= 0) & (px <= cam.w - 1) & (py >= 0) & (py <= cam.h - 1)
        ii, jj = np.round(px[inside]).astype(int), np.round(py[inside]).astype(int)
        near = (np.abs(px[inside] - ii) < 1e-3) & (np.abs(py[inside] - jj) < 1e-3)
        # a sample point projecting onto a pixel centre must lie in the leaf's rectangle
        assert np.all((ii[near] >= i0) & (ii[near] <= i1) & (jj[near] >= j0) & (jj[near] <= j1))
        # every continuous projection lies within one pixel of the rectangle
        if i0 <= i1:
            assert np.all(px[inside] > i0 - 1) and np.all(px[inside] < i1 + 1)
        # nesting: the rectangle lies inside the parent's rectangle
        lv = int(f.level[l])
        if lv > 0:
            m = np.uint32(~((1 << (synth.QMAX - lv + 1)) - 1) & 0xFFFFFFFF)
            pr, pvis = O.node_rect(lv - 1, f.x[l] & m, f.y[l] & m, f.z[l] & m, cam.raw())
            if i0 <= i1:
                assert pvis and pr[0] <= i0 and i1 <= pr[1] and pr[2] <= j0 and j1 <= pr[3]


def _cube_chord(rho, r, smin, smax):
    """Ray/unit-cube chord via the six face planes (independent of the slab test)."""
    hits = []
    for k in range(3):
        if r[k] == 0:
            continue
        for face in (0.0, 1.0):
            s = (face - rho[k]) / r[k]
            p = rho + s * r
            others = [q for q in range(3) if q != k]
            if all(-1e-12 <= p[q] <= 1 + 1e-12 for q in others):
                hits.append(s)
    if len(hits) < 2:
        return 0.0
    a, b = max(min(hits), smin), min(max(hits), smax)
    return max(b - a, 0.0)


def _camera_rays(cam):
    v = np.asarray(cam.v)
    n = np.linalg.norm(v)
    for j in range(cam.h):
        for i in range(cam.w):
            a, b = cam.ell * (i - (cam.w - 1) / 2), cam.ell * (j - (cam.h - 1) / 2)
            if cam.ortho:
                yield j * cam.w + i, cam.o + a * cam.t + b * cam.u, v / n, n, cam.zfar
            else:
                yield j * cam.w + i, cam.o, v + a * cam.t + b * cam.u, 1.0, cam.zfar / n


def test_constant_medium_whole_forest_closed_form(oracle_mod):
    """Constant kappa, eps over an adaptive forest: I = (eps/kap)(1 - e^{-kap L}) + e^{-kap L} I_b."""
    O = oracle_mod
    s = synth.small_scene(2, w=48, h=40)
    N = s.forest.nleaves
    kap, eps, bg = 1.3, 0.45, 0.25
    for method, fields in (("analytic", synth.constant_fields(np.full(N, kap), np.full(N, eps))),
                           ("rk4", synth.Fields("trilinear", np.full((8, N), kap, np.float32),
                                                np.full((8, N), eps, np.float32)))):
        cam = s.cameras[0]
        r = O.render(s.forest, fields, cam, method=method, background=bg)
        kf, ef = float(np.float32(kap)), float(np.float32(eps))
        for p, rho, rr, smin, smax in _camera_rays(cam):
            L = _cube_chord(rho, rr, smin, smax) * np.linalg.norm(rr)
            A = math.exp(-kf * L)
            I = ef / kf * (1 - A) + A * bg
            tol = 1e-12 if method == "analytic" else 2e-5  # RK4 x 4 truncation per leaf
            assert abs(r["I"][p] - I) <= tol * max(1.0, abs(I)), (method, p, r["I"][p], I)


def test_config1_column_formula(oracle_mod):
    """Axis-aligned orthographic workload: each pixel crosses 8 cells of one column."""
    O = oracle_mod
    s = synth.config_scene(1)
    cam = s.cameras[0]
    f = s.forest
    idx = {}
    sh = synth.QMAX - 3
    for l in range(f.nleaves):
        idx[(int(f.x[l]) >> sh, int(f.y[l]) >> sh, int(f.z[l]) >> sh)] = l
    kap = s.fields.kappa[0].astype(np.float64)
    eps = s.fields.eps[0].astype(np.float64)
    r = O.render(f, s.fields, cam, method="analytic")
    axis, sign = s.extra["axis"], s.extra["sign"]
    for p, rho, _, _, _ in _camera_rays(cam):
        cell = [int(math.floor(rho[k] * 8)) for k in range(3)]
        order = range(8) if sign > 0 else range(7, -1, -1)  # front (camera side) first
        A, B = 1.0, 0.0
        for c in order:
            cell[axis] = c
            l = idx[tuple(cell)]
            a = math.exp(-kap[l] / 8)
            b = eps[l] / kap[l] * (1 - a)
            A, B = A * a, B + A * b
        assert math.isclose(r["A"][p], A, rel_tol=1e-13) and math.isclose(r["B"][p], B, rel_tol=1e-12)


def test_watertight_segments_tile_the_chord(oracle_mod):
    O = oracle_mod
    s = synth.small_scene(3, w=40, h=30)
    N = s.forest.nleaves
    # kappa = 0, eps = 1: B equals the real length of the ray inside the forest
    fields = synth.constant_fields(np.zeros(N), np.ones(N))
    cam = s.cameras[0]
    r = O.render(s.forest, fields, cam, method="analytic")
    assert r["overlaps"] == 0
    for p, rho, rr, smin, smax in _camera_rays(cam):
        L = _cube_chord(rho, rr, smin, smax) * np.linalg.norm(rr)
        assert abs(r["B"][p] - L) < 1e-12


def test_brute_force_marching_converges_to_oracle(oracle_mod):
    O = oracle_mod
    s = synth.small_scene(4, lmin=1, lmax=3, ngauss=2, w=24, h=20)
    ref = O.render(s.forest, s.fields, s.cameras[0])
    errs = []
    for M in (64, 256, 1024):
        m = O.march(s.forest, s.fields, s.cameras[0], M=M)
        errs.append(np.abs(m["I"] - ref["I"]).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-4


def test_fold_order_matters(oracle_mod):
    """Guard against an accidental abelian fold: the reversed order changes pixels."""
    O = oracle_mod
    s = synth.small_scene(5, w=32, h=24)
    r = O.render(s.forest, s.fields, s.cameras[0])
    nseg = r["nseg"]
    assert nseg.max() >= 3
    # a pixel with several segments: B differs from what the reversed fold would give unless
    # all segments were identical; check directly on the oracle's combine
    a, b = np.array([0.3, 0.2]), np.array([0.9, 0.5])
    assert not np.allclose(O.combine(a, b), O.combine(b, a))


# ---------------------------------------------------------------- gradients


def test_gradient_eps_linearity_and_fd(oracle_mod):
    O = oracle_mod
    s = synth.small_scene(6, lmin=1, lmax=4, ngauss=3, w=28, h=22)
    cam = s.cameras[0]
    f = s.fields
    r = O.render(s.forest, f, cam)
    # B is linear in eps: sum_c eps_c dB_p/deps_c = B_p (one-hot loss gradient on pixel p)
    for p in np.flatnonzero(r["nseg"] > 0)[:5]:
        g = np.zeros(cam.npix)
        g[p] = 1.0
        gk, ge = O.grad(s.forest, f, cam, g)
        assert math.isclose((ge * f.eps.astype(np.float64)).sum(), r["B"][p], rel_tol=1e-12)
    # L = sum (I - I*)^2: central finite differences on sampled parameters
    rng = _rng(9)
    target = r["I"] + rng.normal(0, 0.05, r["I"].shape)
    kap0, eps0 = f.kappa.astype(np.float64), f.eps.astype(np.float64)

    def loss(kap, eps):
        return ((O.render(s.forest, f, cam, kappa=kap, eps=eps)["I"] - target) ** 2).sum()

    gk, ge = O.grad(s.forest, f, cam, 2 * (r["I"] - target))
    leaves = np.flatnonzero(np.abs(gk).sum(0) > 0)
    for l in rng.choice(leaves, 6, replace=False):
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
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (which, l, c, fd, an)


def test_gradient_constant_medium_closed_form(oracle_mod):
    """One leaf, constant coefficients: dI/dkap = -L A I_b + eps d/dkap[(1-A)/kap]."""
    O = oracle_mod
    f = synth.uniform_forest(0)
    fields = synth.constant_fields([0.8], [0.6])
    cam = synth.orthographic_axis_camera(2, 1, w=4, h=4, ell=0.2, background=0.3)
    r = O.render(f, fields, cam, method="analytic")
    g = np.ones(cam.npix)
    gk, ge = O.grad(f, fields, cam, g, method="analytic")
    k, e, L, Ib = float(np.float32(0.8)), float(np.float32(0.6)), 1.0, 0.3
    A = math.exp(-k * L)
    dIdk = -L * A * Ib + e * (L * A / k - (1 - A) / k ** 2)
    dIde = (1 - A) / k
    assert np.all(r["nseg"] == 1)
    assert math.isclose(gk[0, 0], cam.npix * dIdk, rel_tol=1e-12)
    assert math.isclose(ge[0, 0], cam.npix * dIde, rel_tol=1e-12)
