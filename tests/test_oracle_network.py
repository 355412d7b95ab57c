"""Pins of the oracle's network side (Sec. 4.2, Eq. (9)-(11)): spatial
encoding values at points where sin/cos and the one-blob bins are known,
layer wiring through hand-built weights, the layer chain against numpy's
float64 matmul, central finite differences of the loss against backprop, the
loss and its gradient at a hand-computed point, Adam's constant-gradient
closed form, and the training-batch recipe's distributions."""
import math

import numpy as np
import pytest

import fabric_inputs as fi

NDEC = fi.N_DECODER_PARAMS


def dec_slices():
    out, off = {}, 0
    for k, (o, i) in enumerate(fi.DECODER_SHAPES):
        out[f"W{k + 1}"] = slice(off, off + o * i)
        off += o * i
        out[f"b{k + 1}"] = slice(off, off + o)
        off += o
    return out


def enc_slices():
    out, off = {}, NDEC
    for k, (o, i) in enumerate(fi.ENCODER_SHAPES):
        out[f"E{k + 1}"] = slice(off, off + o * i)
        off += o * i
        out[f"c{k + 1}"] = slice(off, off + o)
        off += o
    return out


def one_pixel(u, v, r, wi, wo, fid=0):
    f = lambda x: np.array([x], dtype=np.float32)
    return fi.GBuffer(np.array([fid], dtype=np.uint16), f(u), f(v), f(r), f(wi[0]), f(wi[1]),
                      f(wi[2]), f(wo[0]), f(wo[1]), f(wo[2]))


def test_param_counts(orc):
    assert orc.param_counts() == (13572, 104352)
    assert fi.N_DECODER_PARAMS == 13572 and fi.N_ENCODER_PARAMS == 104352


def test_spatial_features_known_values(orc):
    # wx = wy = 2; u = 0.5 -> px = 1/4; v = 1.5 -> py = 3/4.
    b = 1
    r = 2.0 ** (-14 + 16 * (b + 0.5) / 8)
    s = orc.spatial_features(0.5, 1.5, r, 2, 2)
    sin_x, cos_x, sin_y, cos_y, blob = s[0:8], s[8:16], s[16:24], s[24:32], s[32:40]
    assert np.allclose(sin_x, [1, 0, 0, 0, 0, 0, 0, 0], atol=1e-15)
    assert np.allclose(cos_x, [0, -1, 1, 1, 1, 1, 1, 1], atol=1e-15)
    assert np.allclose(sin_y, [-1, 0, 0, 0, 0, 0, 0, 0], atol=1e-15)
    assert np.allclose(cos_y, [0, -1, 1, 1, 1, 1, 1, 1], atol=1e-15)
    expect = [math.exp(-0.5 * (b - k) ** 2) for k in range(8)]
    assert np.allclose(blob, expect, rtol=1e-12)
    # Below the encoded range the size clamps to tau = 0.
    s0 = orc.spatial_features(0.5, 1.5, 1e-9, 2, 2)
    assert s0[32] == pytest.approx(math.exp(-0.125), rel=1e-14)
    # Period of the pattern in u and v.
    s1 = orc.spatial_features(0.5 + 2 * 3, 1.5 - 2, r, 2, 2)
    assert np.allclose(s, s1, atol=1e-13)


def test_spatial_features_uses_the_fabric_period(orc):
    a = orc.spatial_features(1.2, 0.7, 0.01, 3, 5)
    b = orc.spatial_features(1.2 + 3, 0.7 + 5, 0.01, 3, 5)
    c = orc.spatial_features(1.2 + 2, 0.7, 0.01, 3, 5)
    assert np.allclose(a, b, atol=1e-13)
    assert not np.allclose(a[:16], c[:16])
    assert a[0] == pytest.approx(math.sin(2 * math.pi * 1.2 / 3), rel=1e-13)


def test_decoder_wiring_with_hand_built_weights(orc):
    sl = dec_slices()
    P = np.zeros(NDEC)
    W1 = np.zeros((64, 72)); W1[0, 32 + 0] = 1.0; W1[1, 5] = 1.0      # s[0] and z[5]
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    W3 = np.zeros((64, 69)); W3[0, 0] = 1.0; W3[1, 64 + 2] = 1.0; W3[2, 64 + 4] = 1.0
    W3[3, 1] = 1.0
    W4 = np.zeros((4, 64)); W4[[0, 1, 2, 3], [0, 1, 2, 3]] = 1.0
    P[sl["W1"]] = W1.ravel(); P[sl["W2"]] = W2.ravel(); P[sl["W3"]] = W3.ravel()
    P[sl["W4"]] = W4.ravel()
    z = np.zeros((1, 32)); z[0, 5] = 0.75
    wi, wo = [0.1, 0.2, 0.97467943], [-0.3, 0.4, 0.8660254]
    m = fi.uniform_material(fi.pattern_plain())
    y, _ = orc.decoder_gbuffer(P, z, [m], one_pixel(0.5, 1.5, 0.01, wi, wo))
    # y = (relu(sin 2 pi px) = 1, wi.z, wo.y, relu(z5)); wi.z enters through a
    # ReLU, which passes it since wi.z > 0.
    assert y[:, 0] == pytest.approx([1.0, np.float32(wi[2]), np.float32(wo[1]), 0.75], rel=1e-7)
    # wo.y negative is clipped by h3's ReLU.
    y2, _ = orc.decoder_gbuffer(P, z, [m], one_pixel(0.5, 1.5, 0.01, wi, [0.3, -0.4, 0.8660254]))
    assert y2[2, 0] == 0.0


def numpy_decoder(P, z, s, ang):
    sl = dec_slices()
    W = {k: P[v] for k, v in sl.items()}
    x1 = np.concatenate([z, s])
    h1 = np.maximum(W["W1"].reshape(64, 72) @ x1 + W["b1"], 0)
    h2 = np.maximum(W["W2"].reshape(64, 64) @ h1 + W["b2"], 0)
    h3 = np.maximum(W["W3"].reshape(64, 69) @ np.concatenate([h2, ang]) + W["b3"], 0)
    return W["W4"].reshape(4, 64) @ h3 + W["b4"]


def test_decoder_matches_numpy_chain(orc):
    P = fi.init_params(21, bias_scale=0.1)[:NDEC].astype(np.float64)
    mats = fi.materials_for(8, 22)
    Z = fi.random_latents(8, 23)
    g = fi.make_gbuffer(16, 8, 8, seed=24)
    g.fabric_id[:] = np.arange(g.n) % 8
    y, rgb = orc.decoder_gbuffer(P, Z, mats, g)
    for p in range(g.n):
        m = mats[g.fabric_id[p]]
        s = orc.spatial_features(float(g.u[p]), float(g.v[p]), float(g.radius[p]), m.wx, m.wy)
        ang = np.array([g.wi_x[p], g.wi_y[p], g.wi_z[p], g.wo_x[p], g.wo_y[p]], dtype=float)
        ref = numpy_decoder(P, Z[g.fabric_id[p]].astype(float), s, ang)
        assert np.allclose(y[:, p], ref, rtol=1e-12, atol=1e-12)


def test_decoded_components_and_rgb(orc):
    sl = dec_slices()
    P = np.zeros(NDEC)
    P[sl["b4"]] = [0.2, 0.3, math.log(1 + 100 * 0.05), math.log(1 + 100 * 0.02)]
    m = fi.uniform_material(fi.pattern_plain())
    m.kd = np.array([[1, 0, 0], [0, 1, 0]], dtype=np.float32)
    m.ks = np.array([[0, 0, 1], [0, 0, 2]], dtype=np.float32)
    _, rgb = orc.decoder_gbuffer(P, np.zeros((1, 32)), [m],
                                 one_pixel(0.1, 0.2, 0.01, [0, 0, 1.0], [0, 0, 1.0]))
    assert rgb[:, 0] == pytest.approx([0.2, 0.3, 0.05 + 2 * 0.02], rel=1e-12)
    # Negative predictions clamp to 0 (C linear, S through g^-1).
    P[sl["b4"]] = [-0.2, -0.3, -1.0, -2.0]
    _, rgb = orc.decoder_gbuffer(P, np.zeros((1, 32)), [m],
                                 one_pixel(0.1, 0.2, 0.01, [0, 0, 1.0], [0, 0, 1.0]))
    assert np.all(rgb == 0.0)


def test_encoder_input_layout(orc):
    m = fi.uniform_material(fi.pattern_plain(), alpha=0.55, beta=0.5, twist=0.0,
                            incl=math.pi / 6, gap=0.25, wblend=0.2)
    x = orc.encoder_input(m)
    assert x[:512].sum() == 4
    assert list(x[[0, 1, 2, 3, 32, 33, 34, 35]]) == [1, 0, 0, 1, 0, 1, 1, 0]
    expect = [0.5, 0.5, 0.25, 0.25, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.2, 0.2]
    assert x[512:] == pytest.approx(expect, abs=1e-7)
    big = fi.uniform_material(fi.random_pattern(np.random.default_rng(1), 16, 16))
    xb = orc.encoder_input(big)
    assert xb[:512].sum() == 256
    assert np.all(xb[0:512:2] + xb[1:512:2] == 1)


def test_encoder_wiring_with_hand_built_weights(orc):
    """The encoder's wiring traced through hand-built weights: e1 picks a
    one-hot cell and a scaled yarn scalar; the residual block adds its
    branch to e1 before the last ReLU (a negative c3 lowers a positive skip,
    which a skip added after the ReLU would not); the branch's inner ReLU
    shuts a negative pre-activation; z is linear."""
    sl = enc_slices()
    Q = np.zeros(fi.N_PARAMS)
    E1 = np.zeros((128, 524)); c1 = np.zeros(128)
    E1[0, 0] = 1.0             # cell (0, 0) of the plain weave has the warp on top
    E1[1, 512] = 1.0           # warp roughness, min-max scaled
    E1[2, 512] = -1.0          # shut by e1's ReLU
    c1[3] = 0.75
    E2 = np.zeros((128, 128)); c2 = np.zeros(128)
    E3 = np.zeros((128, 128)); c3 = np.zeros(128)
    c3[3] = -0.5               # skip before the last ReLU: relu(0.75 - 0.5)
    E2[4, 0] = -1.0; E3[4, 4] = 1.0                 # relu(-1) = 0 in the branch
    E2[5, 0] = 2.0; E3[5, 5] = 3.0                  # 3 relu(2 e1[0]) = 6
    E2[6, 0] = 0.5; c2[6] = -1.0; E3[6, 6] = 1.0; c3[6] = 1.0   # relu(1 + relu(-0.5))
    E4 = np.zeros((32, 128)); c4 = np.zeros(32)
    for k in range(7):
        E4[k, k] = 1.0
    E4[7, 1] = -2.0            # z is linear: a negative output passes
    c4[31] = 0.125
    for name, arr in (("E1", E1), ("c1", c1), ("E2", E2), ("c2", c2), ("E3", E3), ("c3", c3),
                      ("E4", E4), ("c4", c4)):
        Q[sl[name]] = arr.ravel()
    m = fi.uniform_material(fi.pattern_plain(), alpha=0.55)
    z = orc.encoder(Q[NDEC:], [m])[0]
    expect = np.zeros(32)
    expect[:8] = [1.0, 0.5, 0.0, 0.25, 0.0, 6.0, 1.0, -1.0]
    expect[31] = 0.125
    assert z == pytest.approx(expect, abs=1e-7)


def test_encoder_matches_numpy_chain(orc):
    params = fi.init_params(31, bias_scale=0.1).astype(np.float64)
    Q = params[NDEC:]
    mats = fi.materials_for(8, 32)
    z = orc.encoder(Q, mats)
    sl = enc_slices()
    W = {k: params[v] for k, v in sl.items()}
    for f, m in enumerate(mats):
        x = orc.encoder_input(m)
        e1 = np.maximum(W["E1"].reshape(128, 524) @ x + W["c1"], 0)
        r2 = np.maximum(W["E2"].reshape(128, 128) @ e1 + W["c2"], 0)
        e2 = np.maximum(e1 + W["E3"].reshape(128, 128) @ r2 + W["c3"], 0)
        ref = W["E4"].reshape(32, 128) @ e2 + W["c4"]
        assert np.allclose(z[f], ref, rtol=1e-12, atol=1e-12)


def test_loss_and_gradient_at_a_hand_computed_point(orc):
    sl = dec_slices()
    params = np.zeros(fi.N_PARAMS)
    params[sl["b4"]] = [0.5, 0.0, math.log(2.0), 1.0]
    m = fi.uniform_material(fi.pattern_plain())
    g = fi.make_gbuffer(4, 1, 1, seed=5)
    # C targets (0.5, 0.25); S targets (0.01, 0): g(0.01) = ln 2, g(0) = 0.
    tg = np.tile(np.array([[0.5], [0.25], [0.01], [0.0]], dtype=np.float32), (1, 4))
    loss, grad, _ = orc.loss_grad(params, [m], g, tg)
    # 0.1 (0^2 + 0.25^2) + 0.4 (0^2 + 1^2)
    assert loss == pytest.approx(0.40625, rel=1e-6)
    assert grad[sl["b4"]] == pytest.approx([0.0, -0.05, 0.0, 0.8], abs=1e-6)
    mask = np.ones(fi.N_PARAMS, bool)
    mask[sl["b4"]] = False
    assert np.all(grad[mask] == 0.0)   # all-zero weights: every ReLU is shut


@pytest.mark.slow
def test_gradients_match_central_differences(orc):
    rng = np.random.default_rng(41)
    params = fi.init_params(42, bias_scale=0.05).astype(np.float64)
    mats = fi.materials_for(8, 43)[:3]
    g = fi.make_gbuffer(12, 4, 3, seed=44)
    g.fabric_id[:] = np.arange(g.n) % 3
    tg = fi.random_targets(g.n, 45)
    loss, grad, _ = orc.loss_grad(params, mats, g, tg)
    picks = []
    for sl in list(dec_slices().values()) + list(enc_slices().values()):
        idx = np.arange(sl.start, sl.stop)
        big = idx[np.argsort(-np.abs(grad[idx]))[:3]]
        picks += list(big) + list(rng.choice(idx, 3, replace=False))
    h = 1e-6
    scale = np.abs(grad).max()
    for k in picks:
        p1 = params.copy(); p1[k] += h
        p2 = params.copy(); p2[k] -= h
        fd = (orc.loss_grad(p1, mats, g, tg)[0] - orc.loss_grad(p2, mats, g, tg)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * scale + 1e-6 * abs(grad[k]), (k, fd, grad[k])


def test_decoder_backward_matches_differences(orc):
    P = fi.init_params(51, bias_scale=0.05)[:NDEC].astype(np.float64)
    mats = fi.materials_for(8, 52)[:2]
    Z = fi.random_latents(2, 53).astype(np.float64)
    g = fi.make_gbuffer(6, 3, 2, seed=54)
    g.fabric_id[:] = np.arange(g.n) % 2
    dy = np.random.default_rng(55).normal(size=(4, g.n))
    gd, gl = orc.decoder_backward(P, Z, mats, g, dy)

    def obj(Pp, Zp):
        return float((orc.decoder_gbuffer(Pp, Zp, mats, g)[0] * dy).sum())

    h = 1e-6
    rng = np.random.default_rng(56)
    for k in rng.choice(NDEC, 40, replace=False):
        p1 = P.copy(); p1[k] += h
        p2 = P.copy(); p2[k] -= h
        fd = (obj(p1, Z) - obj(p2, Z)) / (2 * h)
        assert abs(fd - gd[k]) <= 1e-7 * np.abs(gd).max() + 1e-6 * abs(gd[k])
    for f in range(2):
        for k in (0, 7, 31):
            z1 = Z.copy(); z1[f, k] += h
            z2 = Z.copy(); z2[f, k] -= h
            fd = (obj(P, z1) - obj(P, z2)) / (2 * h)
            assert abs(fd - gl[f, k]) <= 1e-7 * np.abs(gl).max() + 1e-6 * abs(gl[f, k])


def test_adam_constant_gradient_closed_form(orc):
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by -lr g / (|g| + eps) (Kingma and Ba)."""
    g = np.array([0.3, -2e-3, 5.0, 0.0, -1e-9])
    theta = np.array([1.0, -0.5, 0.25, 0.7, 0.1], dtype=np.float32)
    start = theta.astype(np.float64).copy()
    m = np.zeros(5)
    v = np.zeros(5)
    lr = 1e-3
    for t in range(1, 11):
        orc.adam_step(theta, g, m, v, t, lr)
        expect = start - t * lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(theta, expect, rtol=0, atol=3e-7 * t)
    assert theta[3] == np.float32(0.7)


def test_batch_recipe_distributions(orc):
    n = 200_000
    g = orc.batch_gen(77, n, 8, 1e-3, 0.5)
    counts = np.bincount(g.fabric_id, minlength=8) / n
    assert np.all(np.abs(counts - 0.125) < 0.004)
    for a in (g.u, g.v):
        assert a.min() >= 0 and a.max() < 8
        assert np.all(a.astype(np.float64) * 2 ** 21 == np.round(a.astype(np.float64) * 2 ** 21))
        assert abs(a.mean() - 4.0) < 0.03
    lr = np.log(g.radius.astype(np.float64))
    assert lr.min() >= math.log(1e-3) - 1e-6 and lr.max() <= math.log(0.5) + 1e-6
    assert abs(lr.mean() - 0.5 * (math.log(1e-3) + math.log(0.5))) < 0.02
    for x, y, z in ((g.wi_x, g.wi_y, g.wi_z), (g.wo_x, g.wo_y, g.wo_z)):
        norm = np.sqrt(x.astype(float) ** 2 + y.astype(float) ** 2 + z.astype(float) ** 2)
        assert np.allclose(norm, 1.0, atol=1e-6)
        assert z.min() > 0
        # Cosine-weighted hemisphere: E[z] = 2/3, E[z^2] = 1/2.
        assert abs(z.mean() - 2 / 3) < 3e-3
        assert abs((z.astype(float) ** 2).mean() - 0.5) < 3e-3
    g2 = orc.batch_gen(77, 16, 8, 1e-3, 0.5)
    assert np.array_equal(g2.u, g.u[:16]) and np.array_equal(g2.fabric_id, g.fabric_id[:16])
