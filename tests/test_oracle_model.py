"""Pins of the FP64 oracle's shading model against what the paper and the
mathematics fix: SplitMix64 reference outputs, the concentric map's area
preservation, the SGGX projected-area identity behind Eq. (2), reciprocity and
albedo bounds of Eq. (1), the Lambertian closed forms, the geometry's
invariants (unit, orthogonal, flat for beta = 0, periodic, pattern
symmetries, warp/weft transposition), coverage fractions, the flat-fabric
closed form of the footprint filter Eq. (3)-(5), its r -> 0 and r -> infinity
limits and its Monte-Carlo convergence."""
import math

import numpy as np
import pytest

import fabric_inputs as fi


def unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


def sph(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi),
                     math.cos(theta)])


def hemisphere_grid(n_theta, n_phi):
    th = (np.arange(n_theta) + 0.5) * (0.5 * np.pi / n_theta)
    ph = (np.arange(n_phi) + 0.5) * (2 * np.pi / n_phi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    w = np.sin(T) * (0.5 * np.pi / n_theta) * (2 * np.pi / n_phi)
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1)
    return d.reshape(-1, 3), w.reshape(-1)


# ---------------------------------------------------------------------------
# Random numbers and footprint sampling
# ---------------------------------------------------------------------------

def test_splitmix64_reference_outputs(orc):
    # First three outputs of the published SplitMix64 generator started at state 0.
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert orc.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert orc.splitmix64(0, 2) == 0x06C45D188009454F


def test_splitmix64_bits_balanced(orc):
    vals = np.array([orc.splitmix64(12345, k) for k in range(4096)], dtype=np.uint64)
    bits = ((vals[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(float)
    p = bits.mean(axis=0)
    # 4096 fair bits: sd 0.0078 per position; allow 5 sd.
    assert np.all(np.abs(p - 0.5) < 0.04)


def test_concentric_map_fixed_points(orc):
    assert np.allclose(orc.concentric(0.5, 0.5), [0.0, 0.0])
    assert np.allclose(orc.concentric(1.0, 0.5), [1.0, 0.0])
    assert np.allclose(orc.concentric(0.5, 1.0), [0.0, 1.0])
    assert np.allclose(orc.concentric(0.0, 0.5), [-1.0, 0.0], atol=1e-15)
    c = orc.concentric(1.0, 1.0)
    assert np.allclose(c, [math.sqrt(0.5), math.sqrt(0.5)])


def test_concentric_map_preserves_area(orc):
    m = 200
    xs = (np.arange(m) + 0.5) / m
    pts = np.array([orc.concentric(x, y) for x in xs for y in xs])
    r2 = (pts ** 2).sum(axis=1)
    assert r2.max() <= 1.0 + 1e-12
    # Uniform on the unit disk: E[r^2] = 1/2, P(r < 1/2) = 1/4, zero mean.
    assert abs(r2.mean() - 0.5) < 1e-4
    assert abs((r2 < 0.25).mean() - 0.25) < 2e-3
    assert np.allclose(pts.mean(axis=0), 0.0, atol=1e-12)


# ---------------------------------------------------------------------------
# SGGX fiber microflake, Eq. (2)
# ---------------------------------------------------------------------------

def test_sggx_isotropic_case(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        t = unit(rng.normal(size=3))
        h = unit(rng.normal(size=3))
        assert orc.sggx_D(1.0, t, h) == pytest.approx(1.0 / math.pi, rel=1e-14)
        assert orc.sggx_sigma(1.0, t, h) == pytest.approx(1.0, rel=1e-14)


def test_sggx_axisymmetric_and_even(orc):
    t = unit([0.3, -0.5, 0.8])
    e1 = unit(np.cross(t, [1.0, 0, 0]))
    e2 = np.cross(t, e1)
    for mu in (-0.9, -0.2, 0.0, 0.4, 0.95):
        ref = None
        for phi in np.linspace(0, 2 * np.pi, 7):
            h = mu * t + math.sqrt(1 - mu * mu) * (math.cos(phi) * e1 + math.sin(phi) * e2)
            d = orc.sggx_D(0.3, t, h)
            assert orc.sggx_D(0.3, t, -h) == pytest.approx(d, rel=1e-13)
            if ref is None:
                ref = d
            assert d == pytest.approx(ref, rel=1e-12)
    # The fiber-like lobe peaks where h is perpendicular to t.
    assert orc.sggx_D(0.3, t, e1) > orc.sggx_D(0.3, t, t) * 100


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.1])
def test_sggx_projected_area_identity(orc, alpha):
    """int <w.m>+ D(m) dm = sigma(w): D is the projected-area-normalised SGGX
    distribution whose projected area is sigma (Heitz et al. 2015)."""
    t = unit([0.2, 0.7, -0.4])
    e1 = unit(np.cross(t, [0.0, 0.0, 1.0]))
    n_mu = 40001
    mu = np.linspace(-1, 1, n_mu)
    wmu = np.full(n_mu, 2.0 / (n_mu - 1))
    wmu[0] *= 0.5
    wmu[-1] *= 0.5
    f = np.array([orc.sggx_D(alpha, t, m * t + math.sqrt(max(0.0, 1 - m * m)) * e1) for m in mu])
    for gamma in (0.0, 0.4, 1.1, math.pi / 2):
        w = math.cos(gamma) * t + math.sin(gamma) * e1
        a = math.sin(gamma) * np.sqrt(np.clip(1 - mu * mu, 0, None))
        b = math.cos(gamma) * mu
        # int_0^2pi max(a cos(phi) + b, 0) dphi in closed form
        inner = np.where(b >= a, 2 * np.pi * b, 0.0)
        mid = (b < a) & (b > -a)
        phi0 = np.arccos(np.clip(-b[mid] / a[mid], -1, 1))
        inner[mid] = 2 * (a[mid] * np.sin(phi0) + b[mid] * phi0)
        integral = float((inner * f * wmu).sum())
        assert integral == pytest.approx(orc.sggx_sigma(alpha, t, w), rel=1e-3)


# ---------------------------------------------------------------------------
# Point BRDF, Eq. (1)
# ---------------------------------------------------------------------------

def test_specular_reciprocity(orc):
    rng = np.random.default_rng(2)
    checked = 0
    for _ in range(200):
        n = unit(rng.normal(size=3) * [0.3, 0.3, 1] + [0, 0, 1.5])
        t = unit(np.cross(n, rng.normal(size=3)))
        wi = unit(rng.normal(size=3) + [0, 0, 1.2])
        wo = unit(rng.normal(size=3) + [0, 0, 1.2])
        if wi[2] <= 0 or wo[2] <= 0:
            continue
        alpha = rng.uniform(0.05, 1.0)
        a = orc.point_brdf(alpha, 0.5, n, t, wi, wo)
        b = orc.point_brdf(alpha, 0.5, n, t, wo, wi)
        assert a[0] == pytest.approx(b[0], rel=1e-13, abs=1e-300)
        checked += a[0] > 0
    assert checked > 50


def test_lobes_vanish_below_the_ply(orc):
    n = unit([0.6, 0.0, 0.8])
    t = [0.0, 1.0, 0.0]
    wi = unit([-0.9, 0.0, 0.3])    # above the macro surface, below the ply
    wo = unit([0.2, 0.1, 0.9])
    assert np.all(orc.point_brdf(0.4, 0.5, n, t, wi, wo) == 0.0)
    assert np.all(orc.point_brdf(0.4, 0.5, n, t, wo, wi) == 0.0)


@pytest.mark.parametrize("alpha", [1.0, 0.3, 0.1])
@pytest.mark.parametrize("theta_o", [0.2, 1.0, 1.5])
def test_specular_albedo_below_one(orc, alpha, theta_o):
    d, w = hemisphere_grid(600, 1200)
    n = np.array([0.0, 0.0, 1.0])
    t = np.array([1.0, 0.0, 0.0])
    wo = sph(theta_o, 0.7)
    f = orc.point_brdf_batch(alpha, 0.5, n, t, d, np.broadcast_to(wo, d.shape))
    albedo = float((f[:, 0] * d[:, 2] * w).sum())
    assert 0.02 < albedo < 1.0


def test_lambertian_part_albedo(orc):
    d, w = hemisphere_grid(800, 64)
    n = np.array([0.0, 0.0, 1.0])
    t = np.array([1.0, 0.0, 0.0])
    wo = sph(0.5, 0.2)
    for wb in (0.0, 0.3):
        f = orc.point_brdf_batch(0.5, wb, n, t, d, np.broadcast_to(wo, d.shape))
        # With n_p = n_s the blended terms sum to k_d/pi: albedo exactly 1.
        assert float((f[:, 1] * d[:, 2] * w).sum()) == pytest.approx(1.0, rel=1e-5)
    # (1 - w) alone integrates to 1 - w.
    f0 = orc.point_brdf_batch(0.5, 0.0, n, t, d, np.broadcast_to(wo, d.shape))
    assert float((0.7 * f0[:, 1] * d[:, 2] * w).sum()) == pytest.approx(0.7, rel=1e-5)


@pytest.mark.parametrize("theta_n", [0.0, 0.4, 0.9])
def test_blended_lambert_term_closed_form(orc, theta_n):
    """w <wi.n_p> / (pi <wi.n_s>) under the macro cosine integrates to
    w (1 + cos theta_n) / 2: the tilted-plane sky view pi (1 + cos)/2."""
    d, w = hemisphere_grid(1500, 3000)
    n = sph(theta_n, 0.3)
    t = unit(np.cross(n, [0.0, 1.0, 0.0]))
    f = orc.point_brdf_batch(0.5, 1.0, n, t, d, np.broadcast_to(n, d.shape))
    val = float((f[:, 1] * d[:, 2] * w).sum())
    assert val == pytest.approx((1 + math.cos(theta_n)) / 2, rel=2e-4)


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------

DIR_I = unit([0.3, 0.2, 0.9])
DIR_O = unit([-0.1, 0.4, 0.8])


def test_geometry_unit_and_orthogonal(orc):
    rng = np.random.default_rng(3)
    mats = fi.materials_for(8, 11)
    for m in mats:
        us = rng.uniform(-5, 20, 2000)
        vs = rng.uniform(-5, 20, 2000)
        e = orc.point_eval_batch(m, us, vs, DIR_I, DIR_O)
        yarn = e["yarn"] != 2
        assert yarn.mean() > 0.9
        n, t = e["n"][yarn], e["t"][yarn]
        assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
        assert np.allclose(np.linalg.norm(t, axis=1), 1.0, atol=1e-12)
        assert np.allclose((n * t).sum(axis=1), 0.0, atol=1e-12)
        assert np.all(n[:, 2] > 0)


def test_flat_yarn_when_beta_zero(orc):
    psi = 0.37
    m = fi.uniform_material(fi.pattern_twill(3, 2), beta=0.0, twist=psi)
    rng = np.random.default_rng(4)
    us, vs = rng.uniform(0, 3, 500), rng.uniform(0, 3, 500)
    e = orc.point_eval_batch(m, us, vs, DIR_I, DIR_O)
    for k in range(500):
        if e["yarn"][k] == 2:
            continue
        assert np.allclose(e["n"][k], [0, 0, 1], atol=1e-15)
        if e["yarn"][k] == 0:   # warp axis +y rotated about +z by psi
            assert np.allclose(e["t"][k], [-math.sin(psi), math.cos(psi), 0], atol=1e-15)
        else:                   # weft axis +x rotated about +z by psi
            assert np.allclose(e["t"][k], [math.cos(psi), math.sin(psi), 0], atol=1e-15)


def test_cross_section_and_float_slopes(orc):
    beta, incl, gap = 0.8, 0.5, 0.2
    m = fi.uniform_material(fi.pattern_twill(4, 3), beta=beta, incl=incl, gap=gap)
    beta, incl = float(m.beta[0]), float(m.incl[0])     # the float32 values the model sees
    half = 0.5 * (1 - float(m.gap[0]))
    # Twill 3/1: column 0 reads rows [1, 0, 1, 1]; the warp run through row 3
    # is rows 2, 3, 0 (length 3) and row 3 sits one cell into it.
    s, t = 0.5 + 0.5 * half, 0.25
    e = orc.point_eval(m, 0 + s, 3 + t, DIR_I, DIR_O)
    assert e["yarn"] == 0 and e["on_top"] == 1
    along = 2 * (1 + t) / 3 - 1
    ma = beta * math.tan(incl * along)
    mb = beta * math.tan(math.pi / 3 * 0.5)
    assert e["n"] == pytest.approx(unit([mb, ma, 1.0]), abs=1e-14)
    # Row 0 has the weft on top only in column 3: a float of length 1 whose
    # middle (s = 1/2) is level along the yarn.
    e2 = orc.point_eval(m, 3 + 0.5, 0 + 0.5 + 0.25 * half, DIR_I, DIR_O)
    assert e2["yarn"] == 1 and e2["on_top"] == 1
    mb2 = beta * math.tan(math.pi / 3 * 0.25)
    assert e2["n"] == pytest.approx(unit([0.0, mb2, 1.0]), abs=1e-14)


def test_hole_and_lower_yarn(orc):
    m = fi.uniform_material(fi.pattern_plain(), beta=1.2, gap=0.2)
    # Cell (0, 0) has warp on top.  Both gaps: hole.
    e = orc.point_eval(m, 0.05, 0.05, DIR_I, DIR_O)
    assert e["yarn"] == 2 and e["rho_s"] == 0 and e["rho_c"] == 0
    assert e["area"] == pytest.approx(DIR_O[2], rel=1e-15)
    # Warp gap, weft band: the lower weft shows, without tilt along its axis.
    e = orc.point_eval(m, 0.05, 0.5, DIR_I, DIR_O)
    assert e["yarn"] == 1 and e["on_top"] == 0
    assert e["n"] == pytest.approx([0, 0, 1], abs=1e-15)
    # Coverage bounds are inclusive: s = g/2 lies exactly on the warp's edge.
    e = orc.point_eval(m, float(m.gap[0]) / 2, 0.0, DIR_I, DIR_O)
    assert e["yarn"] == 0
    e = orc.point_eval(m, float(m.gap[0]) / 2 * (1 - 1e-12), 0.0, DIR_I, DIR_O)
    assert e["yarn"] == 2


def fraction_grid(m, k=400):
    xs = (np.arange(k * m.wx) + 0.5) / k
    ys = (np.arange(k * m.wy) + 0.5) / k
    U, V = np.meshgrid(xs, ys, indexing="xy")
    e = orc_mod().point_eval_batch(m, U.reshape(-1), V.reshape(-1), DIR_I, DIR_O)
    return np.bincount(e["yarn"], minlength=3) / e["yarn"].size


def orc_mod():
    import oracle
    return oracle


@pytest.mark.parametrize("gap", [0.2, 0.3])
def test_plain_coverage_fractions(orc, gap):
    m = fi.uniform_material(fi.pattern_plain(), gap=gap)
    frac = fraction_grid(m)
    assert frac[0] == pytest.approx((1 - gap * gap) / 2, abs=2e-3)
    assert frac[1] == pytest.approx((1 - gap * gap) / 2, abs=2e-3)
    assert frac[2] == pytest.approx(gap * gap, abs=2e-3)


def test_satin_coverage_fractions(orc):
    gap = 0.2
    m = fi.uniform_material(fi.pattern_satin5(), gap=gap)
    frac = fraction_grid(m, k=200)
    warp_top = fi.pattern_satin5().mean()           # 4/5 of cells
    expect_warp = warp_top * (1 - gap) + (1 - warp_top) * gap * (1 - gap)
    assert frac[0] == pytest.approx(expect_warp, abs=3e-3)
    assert frac[2] == pytest.approx(gap * gap, abs=3e-3)


def test_periodicity_bitwise(orc):
    for m in fi.materials_for(8, 5):
        rng = np.random.default_rng(6)
        us = rng.uniform(0, 8, 300).astype(np.float32).astype(float)
        vs = rng.uniform(0, 8, 300).astype(np.float32).astype(float)
        a = orc.point_eval_batch(m, us, vs, DIR_I, DIR_O)
        b = orc.point_eval_batch(m, us + m.wx, vs, DIR_I, DIR_O)
        c = orc.point_eval_batch(m, us, vs - 2 * m.wy, DIR_I, DIR_O)
        for key in ("yarn", "rho_s", "rho_c", "area", "n", "t"):
            assert np.array_equal(a[key], b[key])
            assert np.array_equal(a[key], c[key])


@pytest.mark.parametrize("name,shift", [("plain", (1, 1)), ("twill21", (1, 1)),
                                        ("twill31", (1, 1)), ("satin5", (2, 1))])
def test_pattern_diagonal_symmetry(orc, name, shift):
    m = fi.uniform_material(fi.NAMED_PATTERNS[name](), beta=1.1, twist=0.2)
    rng = np.random.default_rng(7)
    us = rng.uniform(0, 5, 500).astype(np.float32).astype(float)
    vs = rng.uniform(0, 5, 500).astype(np.float32).astype(float)
    a = orc.point_eval_batch(m, us, vs, DIR_I, DIR_O)
    b = orc.point_eval_batch(m, us + shift[0], vs + shift[1], DIR_I, DIR_O)
    for key in ("yarn", "rho_s", "rho_c", "area"):
        assert np.array_equal(a[key], b[key])


def test_warp_weft_transposition(orc):
    """Reflecting the fabric across u = v swaps warp and weft: transpose and
    invert the pattern, swap the yarn parameters (the reflection reverses the
    twist), swap u <-> v and x <-> y of both directions."""
    rng = np.random.default_rng(8)
    for base in fi.materials_for(8, 9):
        P = base.pattern
        T = fi.Material(
            pattern=np.ascontiguousarray((1 - P.T).astype(np.uint8)),
            alpha=base.alpha[::-1].copy(), beta=base.beta[::-1].copy(),
            twist=-base.twist[::-1].copy(), incl=base.incl[::-1].copy(),
            gap=base.gap[::-1].copy(), wblend=base.wblend[::-1].copy(),
            kd=base.kd[::-1].copy(), ks=base.ks[::-1].copy())
        us = rng.uniform(0, 8, 400)
        vs = rng.uniform(0, 8, 400)
        wi, wo = unit([0.35, -0.2, 0.9]), unit([-0.3, 0.5, 0.7])
        a = orc.point_eval_batch(base, us, vs, wi, wo)
        b = orc.point_eval_batch(T, vs, us, wi[[1, 0, 2]], wo[[1, 0, 2]])
        ya, yb = a["yarn"], b["yarn"]
        swapped = np.where(ya == 2, 2, 1 - ya)
        assert np.array_equal(swapped, yb)
        assert np.allclose(a["rho_s"], b["rho_s"], rtol=1e-12, atol=1e-300)
        assert np.allclose(a["rho_c"], b["rho_c"], rtol=1e-12, atol=1e-300)
        assert np.allclose(a["area"], b["area"], rtol=1e-12)
        assert np.allclose(a["n"][:, [1, 0, 2]], b["n"], atol=1e-13)


# ---------------------------------------------------------------------------
# Footprint filter, Eq. (3)-(5) and (7)-(8)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("wi_theta,wo_theta", [(0.3, 0.6), (1.1, 0.2)])
def test_flat_fabric_closed_form(orc, wi_theta, wo_theta):
    """beta = 0 and alpha = 1: every yarn point is flat and isotropic, every
    sample (holes included) has projected area wo.z, so C_y = (n_y / N) wi.z / pi
    exactly, S_y / C_y = pi D G / (4 wo.z wi.z) with D = 1/pi and Lambda =
    1/cos, and over a wide footprint n_y / N -> (1 - g^2) / 2 for plain."""
    gap = 0.2
    m = fi.uniform_material(fi.pattern_plain(), alpha=1.0, beta=0.0, gap=gap, wblend=0.3)
    wi, wo = sph(wi_theta, 0.4), sph(wo_theta, 2.0)
    N = 128 * 128
    comp, area, _ = orc.filter_pixel(m, 0.3, 0.7, 20.0, wi, wo, N, 99)
    L = 1 / wi[2] + 1 / wo[2]
    G = (1 - math.exp(-2 * L)) / L
    rho_s = (1 / math.pi) * G / (4 * wo[2])
    assert area == pytest.approx(N * wo[2], rel=1e-12)
    for y in (0, 1):
        count = comp[y] * math.pi / wi[2] * N
        assert abs(count - round(count)) < 1e-6
        assert comp[2 + y] / comp[y] == pytest.approx(rho_s * math.pi / wi[2], rel=1e-12)
        assert comp[y] == pytest.approx((1 - gap * gap) / 2 * wi[2] / math.pi, rel=1e-2)


def test_radius_to_zero_limit(orc):
    m = fi.uniform_material(fi.pattern_twill(3, 2), alpha=0.4, beta=1.0, twist=0.3)
    u, v = 0.47, 0.52                    # well inside a warp band, away from edges
    wi, wo = sph(0.5, 0.3), sph(0.4, 2.5)
    e = orc.point_eval(m, u, v, wi, wo)
    assert e["yarn"] == 0 and e["edge"] > 0.2
    point = np.array([e["rho_c"], 0.0, e["rho_s"], 0.0])
    errs = []
    radii = [0.04, 0.02, 0.01]
    for r in radii:
        comp, _, _ = orc.filter_pixel(m, u, v, r, wi, wo, 64 * 64, 3)
        assert comp[1] == 0.0 and comp[3] == 0.0
        errs.append(np.abs(comp - point).max())
    slope = np.polyfit(np.log(radii), np.log(errs), 1)[0]
    assert 1.6 < slope < 2.4
    assert errs[-1] < 1e-3 * np.abs(point).max()


def test_radius_to_infinity_limit(orc):
    """A footprint covering many pattern periods averages over the period, so
    the components stop depending on where it is centred (edge effects fall
    off at least like W / r)."""
    m = fi.uniform_material(fi.pattern_twill(3, 2), alpha=0.4, beta=1.0, twist=0.3)
    wi, wo = sph(0.5, 0.3), sph(0.4, 2.5)
    centres = [(0.3, 0.7), (1.1, 0.2), (2.45, 1.6), (0.9, 2.2)]

    def spread(r):
        cs = np.array([orc.filter_pixel(m, u, v, r, wi, wo, 512 * 512, 5)[0] for u, v in centres])
        return (cs.max(axis=0) - cs.min(axis=0)).max() / np.abs(cs).max()

    near, far = spread(3.0), spread(12.0)
    assert near > 1e-2            # a 2-period footprint still sees where it sits
    assert far < 0.25 * near and far < 1e-2


def test_monte_carlo_convergence(orc):
    rng = np.random.default_rng(10)
    m = fi.materials_for(8, 12)[1]
    cases = []
    for _ in range(6):
        cases.append((rng.uniform(0, 3), rng.uniform(0, 3), rng.uniform(0.3, 0.8),
                      unit(rng.normal(size=3) * [0.4, 0.4, 0.2] + [0, 0, 1]),
                      unit(rng.normal(size=3) * [0.4, 0.4, 0.2] + [0, 0, 1])))
    ref = [orc.filter_pixel(m, u, v, r, wi, wo, 384 * 384, 77)[0] for u, v, r, wi, wo in cases]
    Ns = [4 ** 2, 8 ** 2, 16 ** 2, 32 ** 2]
    rms = []
    for N in Ns:
        e2 = []
        for (u, v, r, wi, wo), rf in zip(cases, ref):
            for seed in range(4):
                c = orc.filter_pixel(m, u, v, r, wi, wo, N, 1000 + seed)[0]
                e2.append(((c - rf) ** 2).sum() / ((rf ** 2).sum() + 1e-30))
        rms.append(math.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(Ns), np.log(rms), 1)[0]
    assert slope < -0.5


def test_filter_periodic_and_deterministic(orc):
    m = fi.materials_for(8, 13)[3]
    wi, wo = unit([0.2, 0.1, 0.9]), unit([-0.3, 0.2, 0.8])
    a = orc.filter_pixel(m, 1.25, 2.5, 0.3, wi, wo, 256, 5, pixel=17)
    b = orc.filter_pixel(m, 1.25, 2.5, 0.3, wi, wo, 256, 5, pixel=17)
    assert np.array_equal(a[0], b[0])
    c = orc.filter_pixel(m, 1.25 + m.wx, 2.5 - m.wy, 0.3, wi, wo, 256, 5, pixel=17)
    assert np.allclose(a[0], c[0], rtol=1e-12)
    d = orc.filter_pixel(m, 1.25, 2.5, 0.3, wi, wo, 256, 6, pixel=17)
    assert not np.array_equal(a[0], d[0])


def test_compose_and_faults(orc):
    m = fi.uniform_material(fi.pattern_plain())
    m.kd = np.array([[1, 0, 0], [0, 1, 0]], dtype=np.float32)
    m.ks = np.array([[0, 0, 1], [0, 0, 0]], dtype=np.float32)
    g = fi.make_gbuffer(8, 4, 1, seed=3)
    g.wo_z[3] = -0.1          # below the surface
    g.radius[5] = 0.0         # empty footprint
    g.u[7] = np.nan
    g.fabric_id[9] = 1        # only one fabric
    comp, rgb, flagged, fault = orc.filter_gbuffer([m], g, 64, 4)
    assert list(np.nonzero(fault)[0]) == [3, 5, 7, 9]
    assert np.all(comp[:, fault == 1] == 0) and np.all(rgb[:, fault == 1] == 0)
    ok = fault == 0
    # Eq. (8) with unit albedo vectors reads the components back.
    assert np.allclose(rgb[0, ok], comp[0, ok])
    assert np.allclose(rgb[1, ok], comp[1, ok])
    assert np.allclose(rgb[2, ok], comp[2, ok])
