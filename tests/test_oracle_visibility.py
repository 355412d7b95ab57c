"""Pins of the oracle's inter-yarn visibility V of Eq. (3)-(4) (stand-in
height field and march): the height field's gradient reproduces the ply
normals (the same slopes define both), a flat fabric occludes nothing and
filters exactly as with V = 1, the zenith and the highest texel see
everything, visibility only grows with elevation, a hole looking along the
surface at a grazing angle is shadowed, periodicity, V only removes
projected area, and an axis-aligned march against a direct scan of the
table row."""
import math

import numpy as np

import fabric_inputs as fi
import oracle as orc


def direction(elev, azim):
    c = math.cos(elev)
    return np.array([c * math.cos(azim), c * math.sin(azim), math.sin(elev)])


def some_materials(seed=3):
    rng = np.random.default_rng(seed)
    mats = fi.materials_for(8, seed)
    for m in mats:
        m.beta[:] = rng.uniform(0.5, 2.0, 2).astype(np.float32)
    return mats


def test_height_gradient_matches_normals():
    """dH/du = -n.x / n.z and dH/dv = -n.y / n.z at points away from yarn
    edges and float ends (central differences, step 1e-6 cells)."""
    rng = np.random.default_rng(11)
    checked = 0
    for m in some_materials():
        for _ in range(200):
            u, v = rng.uniform(0, m.wx), rng.uniform(0, m.wy)
            p = orc.point_eval(m, u, v, [0, 0, 1], [0, 0, 1])
            if p["yarn"] == 2 or p["edge"] < 1e-3:
                continue
            h = 1e-6
            du = (orc.surface_height(m, u + h, v) - orc.surface_height(m, u - h, v)) / (2 * h)
            dv = (orc.surface_height(m, u, v + h) - orc.surface_height(m, u, v - h)) / (2 * h)
            n = p["n"]
            assert abs(du + n[0] / n[2]) < 1e-6 * (1 + abs(du)), (u, v, du, n)
            assert abs(dv + n[1] / n[2]) < 1e-6 * (1 + abs(dv)), (u, v, dv, n)
            checked += 1
    assert checked > 500


def test_flat_fabric_sees_everything():
    mats = fi.materials_for(8, 12)
    rng = np.random.default_rng(12)
    for m in mats:
        m.beta[:] = 0.0
        t, hmax = orc.height_table(m)
        assert not t.any() and hmax == 0.0
        for _ in range(50):
            w = direction(rng.uniform(0.01, 1.5), rng.uniform(0, 2 * math.pi))
            assert orc.visible(m, rng.uniform(0, 8), rng.uniform(0, 8), w) == 1
    # The filter with V is the filter with V = 1, bit for bit.
    g = fi.make_gbuffer(16, 8, 8, seed=13)
    a = orc.filter_gbuffer(mats, g, 64, 14, visibility=False)[0]
    b = orc.filter_gbuffer(mats, g, 64, 14, visibility=True)[0]
    assert np.array_equal(a, b)


def test_zenith_and_highest_texel_see_everything():
    rng = np.random.default_rng(15)
    for m in some_materials(16):
        for _ in range(30):
            assert orc.visible(m, rng.uniform(0, 8), rng.uniform(0, 8), [0.0, 0.0, 1.0]) == 1
        t, hmax = orc.height_table(m)
        b, a = np.unravel_index(int(np.argmax(t)), t.shape)
        uc, vc = (a + 0.5) / 16, (b + 0.5) / 16
        for _ in range(100):
            w = direction(rng.uniform(0.005, 1.5), rng.uniform(0, 2 * math.pi))
            assert orc.visible(m, uc, vc, w) == 1


def test_visibility_grows_with_elevation():
    rng = np.random.default_rng(17)
    elevs = np.radians([1, 3, 6, 10, 20, 35, 60, 85])
    blocked_low = 0
    for m in some_materials(18):
        for _ in range(60):
            u, v, az = rng.uniform(0, 8), rng.uniform(0, 8), rng.uniform(0, 2 * math.pi)
            vis = [orc.visible(m, u, v, direction(e, az)) for e in elevs]
            assert all(a <= b for a, b in zip(vis, vis[1:])), vis
            blocked_low += 1 - vis[0]
    assert blocked_low > 0      # grazing rays are blocked somewhere


def test_hole_shadowed_at_grazing_angle():
    """Plain weave, wide gaps, tall yarns: from the hole at a cell corner a ray
    along +u at 2 degrees runs into the next yarn; steeply up it is free."""
    m = fi.uniform_material(fi.pattern_plain(), beta=2.0, gap=0.3)
    p = orc.point_eval(m, 0.02, 0.02, [0, 0, 1], [0, 0, 1])
    assert p["yarn"] == 2
    assert orc.visible(m, 0.02, 0.02, direction(math.radians(2), 0.0)) == 0
    assert orc.visible(m, 0.02, 0.02, direction(math.radians(80), 0.0)) == 1


def test_periodic():
    rng = np.random.default_rng(19)
    for m in some_materials(20):
        for _ in range(40):
            u, v = rng.uniform(0, m.wx), rng.uniform(0, m.wy)
            w = direction(rng.uniform(0.02, 0.6), rng.uniform(0, 2 * math.pi))
            assert orc.visible(m, u, v, w) == orc.visible(m, u + 3 * m.wx, v - 2 * m.wy, w)


def test_visibility_only_removes_area():
    """Same samples with and without V: the visible projected area sum never
    grows (V <= 1 multiplies each sample's A(p, wo))."""
    mats = some_materials(21)
    rng = np.random.default_rng(22)
    for k in range(40):
        m = mats[k % len(mats)]
        wi = direction(rng.uniform(0.05, 1.5), rng.uniform(0, 6.3))
        wo = direction(rng.uniform(0.05, 1.5), rng.uniform(0, 6.3))
        args = (m, rng.uniform(0, 8), rng.uniform(0, 8), rng.uniform(0.05, 1.0), wi, wo, 64, 23, k)
        _, a0, _ = orc.filter_pixel(*args, visibility=False)
        c1, a1, _ = orc.filter_pixel(*args, visibility=True)
        assert a1 <= a0 + 1e-12
        assert np.all(np.isfinite(c1)) and np.all(c1 >= 0)


def test_axis_aligned_march_scans_the_row():
    """For w in the x-z plane the march visits the texels of the point's row
    one by one: compare with a scan of that row of the table."""
    rng = np.random.default_rng(24)
    f32 = np.float32
    for m in some_materials(25):
        t, hmax = orc.height_table(m)
        th, tw = t.shape
        for _ in range(40):
            u, v = rng.uniform(0, m.wx), rng.uniform(0, m.wy)
            e = rng.uniform(0.01, 0.5)
            w = np.array([math.cos(e), 0.0, math.sin(e)])
            a0, b0 = int(math.floor(f32(u) * 16)) % tw, int(math.floor(f32(v) * 16)) % th
            rise = f32(f32(f32(w[2]) / f32(w[0])) * f32(1 / 16))
            want = 1
            for k in range(1, 33):
                h = f32(t[b0, a0] + f32(f32(k) * rise))
                if h >= hmax:
                    break
                if t[b0, (a0 + k) % tw] > h:
                    want = 0
                    break
            assert orc.visible(m, u, v, w) == want


def test_zero_inclination_and_single_cell_period():
    """Zero inclination: floats are flat, the height is the cross-section
    profile alone (finite everywhere).  A 1 x 1 period (one yarn on top
    everywhere): rays wrap over the period several times."""
    m = fi.uniform_material(fi.pattern_twill(3, 2), beta=1.5, incl=0.0)
    t, hmax = orc.height_table(m)
    assert np.all(np.isfinite(t))
    p = orc.point_eval(m, 1.5, 1.5, [0, 0, 1], [0, 0, 1])
    assert p["n"][1] == 0.0 and p["n"][0] == 0.0           # centre of a flat top float
    assert orc.surface_height(m, 1.5, 1.5) == 0.0
    one = fi.uniform_material(np.ones((1, 1), dtype=np.uint8), beta=1.0, gap=0.3)
    rng = np.random.default_rng(26)
    for _ in range(50):
        w = direction(rng.uniform(0.01, 0.3), rng.uniform(0, 2 * math.pi))
        u, v = rng.uniform(0, 1), rng.uniform(0, 1)
        assert orc.visible(one, u, v, w) == orc.visible(one, u + 5, v + 7, w)


# ---------------------------------------------------------------------------
# The march over hand-built height tables, against elementary geometry: a
# ray leaving a texel's centre at elevation e clears a wall of height H whose
# centre lies d cells away along the ray's horizontal direction iff
# tan e > H / d (taken at the texel centres the march visits).
# ---------------------------------------------------------------------------

RES = 16


def flat_table(wx, wy):
    return np.zeros((wy * RES, wx * RES), dtype=np.float32)


def test_hand_built_wall_critical_elevation():
    """A wall of height 0.25 cells filling texel column 8 of a 3x1-cell
    period; rays along +u from texel column 0 (its centre is 8 texels =
    0.5 cells from the wall's): blocked iff tan e < 0.25 / 0.5."""
    t = flat_table(3, 1)
    t[:, 8] = 0.25
    crit = math.atan(0.25 / 0.5)
    for b in (0, 7, 15):
        vp = (b + 0.5) / RES
        for up in (0.001, 0.5 / RES, 0.999 / RES):      # anywhere inside texel 0
            assert orc.visible_in_table(t, 0.25, up, vp, direction(crit - 0.01, 0.0)) == 0
            assert orc.visible_in_table(t, 0.25, up, vp, direction(crit + 0.01, 0.0)) == 1
            # Looking away from the wall (-u) the ray wraps round the period
            # and meets the wall after 48 - 8 = 40 texels: beyond the
            # 32-step patch, so free at any elevation.
            assert orc.visible_in_table(t, 0.25, up, vp, direction(0.01, math.pi)) == 1


def test_hand_built_wall_through_the_period():
    """A wall in texel column 29 of a 2-cell-wide period, seen from column 2
    looking along -u: the ray wraps from column 0 to 31 and reaches the wall
    after 5 texels (5/16 cells)."""
    t = flat_table(2, 2)
    t[:, 29] = 0.1
    crit = math.atan(0.1 / (5 / RES))
    up, vp = (2 + 0.5) / RES, 0.3
    assert orc.visible_in_table(t, 0.1, up, vp, direction(crit - 0.01, math.pi)) == 0
    assert orc.visible_in_table(t, 0.1, up, vp, direction(crit + 0.01, math.pi)) == 1
    # The same wall looked at along +u is 27 texels away.
    crit_far = math.atan(0.1 / (27 / RES))
    assert orc.visible_in_table(t, 0.1, up, vp, direction(crit_far - 0.005, 0.0)) == 0
    assert orc.visible_in_table(t, 0.1, up, vp, direction(crit_far + 0.005, 0.0)) == 1


def test_hand_built_pillar_on_the_diagonal():
    """A single tall texel 4 texels up the diagonal: along azimuth 45 deg the
    march visits texels (a0 + k, b0 + k), so it meets the pillar at a
    horizontal distance of 4 sqrt(2)/16 cells; a pillar one texel off the
    diagonal is never visited."""
    t = flat_table(2, 2)
    a0, b0 = 5, 9
    t[b0 + 4, a0 + 4] = 0.3
    up, vp = (a0 + 0.5) / RES, (b0 + 0.5) / RES
    crit = math.atan(0.3 / (4 * math.sqrt(2) / RES))
    assert orc.visible_in_table(t, 0.3, up, vp, direction(crit - 0.01, math.pi / 4)) == 0
    assert orc.visible_in_table(t, 0.3, up, vp, direction(crit + 0.01, math.pi / 4)) == 1
    t2 = flat_table(2, 2)
    t2[b0 + 3, a0 + 4] = 0.3
    assert orc.visible_in_table(t2, 0.3, up, vp, direction(0.02, math.pi / 4)) == 1


def test_hand_built_minor_axis_steps():
    """Azimuth atan(1/2): one texel along u per step and half a texel along
    v, so from the centre of texel (0, 0) the march visits v-texels 0, 1, 1,
    2, 2, ... (centre 0.5 + k/2): a pillar at (4, 2) is met at step 4, a
    pillar at (4, 3) is not."""
    az = math.atan2(1.0, 2.0)
    hdist = 4 * math.hypot(1.0, 0.5) / RES
    crit = math.atan(0.2 / hdist)
    t = flat_table(2, 2)
    t[2, 4] = 0.2
    assert orc.visible_in_table(t, 0.2, 0.5 / RES, 0.5 / RES, direction(crit - 0.01, az)) == 0
    assert orc.visible_in_table(t, 0.2, 0.5 / RES, 0.5 / RES, direction(crit + 0.01, az)) == 1
    t2 = flat_table(2, 2)
    t2[3, 4] = 0.2
    assert orc.visible_in_table(t2, 0.2, 0.5 / RES, 0.5 / RES, direction(0.02, az)) == 1


def test_hand_built_pit():
    """A point at the bottom of a one-texel pit of depth 0.05 cells with a
    flat surround: the rim's texel centre is 1/16 cell away, so the point
    sees out iff tan e > 0.05 / (1/16), in every axis direction."""
    t = flat_table(2, 2)
    t[6, 6] = -0.05
    crit = math.atan(0.05 * RES)
    up = vp = 6.5 / RES
    for az in (0.0, math.pi / 2, math.pi, 1.5 * math.pi):
        assert orc.visible_in_table(t, 0.0, up, vp, direction(crit - 0.01, az)) == 0
        assert orc.visible_in_table(t, 0.0, up, vp, direction(crit + 0.01, az)) == 1
