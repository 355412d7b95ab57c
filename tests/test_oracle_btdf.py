"""Pins of the oracle's transmission lobe (light below the fabric): the
isotropic case against a direct numerical integral over the slab's depth
(the single-scattering definition, written without its closed form), the
same for reflection, the reciprocal-and-mirrored symmetry of the slab,
positivity, continuity where Lambda_i = Lambda_o, the single-scattering
energy bound R + T <= 1 - e^{-T Lambda_i} by quadrature, the Lambertian
share, no delta transmission, the flat-fabric closed form of the filter,
the k = 1000 mapping of the loss for transmission queries, and the batch
recipe's share of samples lit from below."""
import math

import numpy as np
import pytest

import fabric_inputs as fi

Z = np.array([0.0, 0.0, 1.0])
T_RHO = 2.0


def sph(theta, phi, below=False):
    v = np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
    if below:
        v[2] = -v[2]
    return v


def depth_integral(mu_i, mu_o, transmit):
    """Single scattering in a slab of optical depth T with an isotropic phase
    1/(4 pi), unit extinction: light enters (from the top for reflection,
    from the bottom for transmission), first scatters at depth t with density
    e^{-path}/|mu_i|, leaves through the top with e^{-t/mu_o}; divided by
    mu_o to give a BSDF.  Gauss-Legendre over t."""
    x, wts = np.polynomial.legendre.leggauss(200)
    t = 0.5 * T_RHO * (x + 1.0)
    path_in = (T_RHO - t) if transmit else t
    vals = np.exp(-path_in / abs(mu_i)) / abs(mu_i) / (4 * math.pi) * np.exp(-t / mu_o)
    return 0.5 * T_RHO * float(np.dot(wts, vals)) / mu_o


@pytest.mark.parametrize("ti,to", [(0.2, 0.3), (0.9, 0.4), (1.3, 1.2), (0.5, 0.5)])
def test_isotropic_slab_against_depth_integral(orc, ti, to):
    """alpha = 1 makes the fiber SGGX isotropic (D = 1/pi, sigma = 1): f_t
    and f_s must be the depth integrals of the single-scattering slab."""
    t = np.array([1.0, 0.0, 0.0])
    wi_b, wo = sph(ti, 0.7, below=True), sph(to, 2.9)
    f_t = orc.point_brdf(1.0, 0.4, Z, t, wi_b, wo)[0]
    assert f_t == pytest.approx(depth_integral(wi_b[2], wo[2], True), rel=1e-10)
    wi_a = sph(ti, 0.7)
    f_r = orc.point_brdf(1.0, 0.4, Z, t, wi_a, wo)[0]
    assert f_r == pytest.approx(depth_integral(wi_a[2], wo[2], False), rel=1e-10)


def test_slab_symmetry_and_positivity(orc):
    """Reciprocity with the slab turned over: light from below along a seen
    from above along b equals light from below along Mb seen along Ma
    (M mirrors z; the ply normal is z and the fiber axis in the plane)."""
    rng = np.random.default_rng(5)
    M = np.array([1.0, 1.0, -1.0])
    for _ in range(200):
        ang = rng.uniform(0, 2 * math.pi)
        t = np.array([math.cos(ang), math.sin(ang), 0.0])
        a = sph(rng.uniform(0.05, 1.5), rng.uniform(0, 6.3), below=True)
        b = sph(rng.uniform(0.05, 1.5), rng.uniform(0, 6.3))
        alpha = rng.uniform(0.1, 1.0)
        f1 = orc.point_brdf(alpha, 0.5, Z, t, a, b)
        f2 = orc.point_brdf(alpha, 0.5, Z, t, M * b, M * a)
        assert f1[0] > 0
        assert f1[0] == pytest.approx(f2[0], rel=1e-12)


def test_continuous_where_lambdas_meet(orc):
    """wi = M wo gives Lambda_i = Lambda_o (the limit branch); a tiny tilt
    of wo leaves the value nearly unchanged."""
    t = np.array([0.0, 1.0, 0.0])
    wo = sph(0.6, 1.0)
    wi = wo * np.array([1.0, 1.0, -1.0])
    f0 = orc.point_brdf(0.5, 0.5, Z, t, wi, wo)[0]
    f1 = orc.point_brdf(0.5, 0.5, Z, t, wi, sph(0.6 + 1e-7, 1.0))[0]
    assert f0 > 0 and f1 == pytest.approx(f0, rel=1e-5)


@pytest.mark.parametrize("alpha", [0.3, 0.6, 1.0])
@pytest.mark.parametrize("theta_i", [0.2, 0.8, 1.3])
def test_single_scattering_energy_bound(orc, alpha, theta_i):
    """Light from below: what leaves upward (T) plus what the mirrored slab
    reflects (R, the same slab seen from its other face) is at most the
    share scattered once, 1 - e^{-T rho Lambda_i}; both are positive."""
    t = np.array([math.cos(0.3), math.sin(0.3), 0.0])
    wi_b = sph(theta_i, 0.5, below=True)
    nt, nph = 400, 800
    th = (np.arange(nt) + 0.5) * (math.pi / 2) / nt
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    wo = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    dw = (math.pi / 2 / nt) * (2 * math.pi / nph) * np.sin(TH).reshape(-1)
    ft = orc.point_brdf_batch(alpha, 0.5, Z, t, np.tile(wi_b, (wo.shape[0], 1)), wo)[:, 0]
    fr = orc.point_brdf_batch(alpha, 0.5, Z, t, np.tile(wi_b * [1, 1, -1], (wo.shape[0], 1)), wo)[:, 0]
    T = float(np.sum(ft * wo[:, 2] * dw))
    R = float(np.sum(fr * wo[:, 2] * dw))
    sig = orc.sggx_sigma(alpha, t, wi_b)
    bound = 1 - math.exp(-T_RHO * sig / abs(wi_b[2]))
    assert T > 0 and R > 0
    assert R + T <= bound * (1 + 1e-3), (R, T, bound)


def test_lambertian_share_and_no_delta(orc):
    t = np.array([1.0, 0.0, 0.0])
    wo = sph(0.4, 0.2)
    f = orc.point_brdf(0.5, 0.3, Z, t, sph(0.7, 1.9, below=True), wo)
    assert f[1] == pytest.approx(0.7 / math.pi, rel=1e-15)
    f = orc.point_brdf(0.5, 0.3, Z, t, -wo, wo)
    assert f[0] == 0.0 and f[1] == pytest.approx(0.7 / math.pi, rel=1e-15)
    # Light above the macro surface but behind a tilted ply: no transmission.
    n = np.array([0.6, 0.0, 0.8])
    assert np.all(orc.point_brdf(0.5, 0.3, n, [0, 1, 0], [-0.9, 0.0, 0.3], wo) == 0.0)


def test_flat_fabric_transmission_closed_form(orc):
    """beta = 0: every yarn point has n = z and every sample projects wo.z,
    so C_y = (n_y / N) (1 - w) |wi.z| / pi exactly (holes transmit nothing)."""
    w = 0.3
    m = fi.uniform_material(fi.pattern_plain(), alpha=0.5, beta=0.0, gap=0.2, wblend=w)
    wi, wo = sph(0.8, 0.4, below=True), sph(0.5, 2.0)
    N = 64 * 64
    comp, area, _ = orc.filter_pixel(m, 0.3, 0.7, 3.0, wi, wo, N, 98)
    assert area == pytest.approx(N * wo[2], rel=1e-12)
    for y in (0, 1):
        count = comp[y] * math.pi / ((1 - float(np.float32(w))) * abs(wi[2])) * N
        assert abs(count - round(count)) < 1e-6 and count > 0
        assert comp[2 + y] > 0


def test_loss_maps_transmission_with_k_1000(orc):
    """One sample lit from below, hand-built decoder output y: the S terms of
    the loss use ln(1000 x + 1); flipping the light to above uses k = 100."""
    mats = fi.materials_for(2, 6)
    g = fi.make_gbuffer(1, 1, 2, seed=7)
    g.wi_z[:] = -np.abs(g.wi_z)
    params = fi.init_params(8, bias_scale=0.05).astype(np.float64)
    tg = np.array([[0.1], [0.2], [0.5], [0.01]], dtype=np.float32)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:], mats)
    y, _ = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    t64 = tg[:, 0].astype(np.float64)

    def expect(k):
        return (0.1 * ((y[0, 0] - t64[0]) ** 2 + (y[1, 0] - t64[1]) ** 2)
                + 0.4 * ((y[2, 0] - math.log(k * t64[2] + 1)) ** 2
                         + (y[3, 0] - math.log(k * t64[3] + 1)) ** 2))
    loss, _, _ = orc.loss_grad(params, mats, g, tg)
    assert loss == pytest.approx(expect(1000.0), rel=1e-12)
    g.wi_z[:] = np.abs(g.wi_z)
    y, _ = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    loss, _, _ = orc.loss_grad(params, mats, g, tg)
    assert loss == pytest.approx(expect(100.0), rel=1e-12)


def test_batch_recipe_transmission_share(orc):
    b0 = orc.batch_gen(11, 200_000, 8)
    b1 = orc.batch_gen(11, 200_000, 8, btdf_frac=0.25)
    assert np.all(b0.wi_z > 0)
    below = b1.wi_z < 0
    assert abs(below.mean() - 0.25) < 0.005
    assert np.array_equal(np.abs(b1.wi_z), b0.wi_z)
    for f in ("u", "v", "radius", "wi_x", "wi_y", "wo_x", "wo_y", "wo_z"):
        assert np.array_equal(getattr(b0, f), getattr(b1, f))
