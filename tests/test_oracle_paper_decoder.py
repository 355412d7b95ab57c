"""Pins of the oracle's paper-size decoder (Sec. 4.2 "Decoder"): the
one-blob position bins are periodic and circular, and eight Gaussian bins
one bin apart sum to sqrt(2 pi) at any position (Poisson summation); the
size bins equal the config decoder's; hand-built weights trace the leaky
slope through all six activations, the residual skip and the angular
inputs; random weights against a numpy float64 chain."""
import math

import numpy as np
import pytest

import fabric_inputs as fi
import oracle as orc

SH = fi.PAPER_DECODER_SHAPES


def slices():
    out, off = [], 0
    for o, i in SH:
        out.append((slice(off, off + o * i), slice(off + o * i, off + o * i + o), o, i))
        off += o * i + o
    return out


def one_pixel(u, v, r, wi, wo, fid=0):
    f = lambda x: np.array([x], dtype=np.float32)
    return fi.GBuffer(np.array([fid], dtype=np.uint16), f(u), f(v), f(r), f(wi[0]), f(wi[1]),
                      f(wi[2]), f(wo[0]), f(wo[1]), f(wo[2]))


def test_blob_bins():
    rng = np.random.default_rng(1)
    for _ in range(200):
        wx, wy = rng.integers(1, 17, 2)
        u, v, r = rng.uniform(-20, 20), rng.uniform(-20, 20), math.exp(rng.uniform(-9, 1))
        f = orc.paper_features(u, v, r, wx, wy)
        g = orc.paper_features(u + 3 * wx, v - 2 * wy, r, wx, wy)
        np.testing.assert_allclose(f, g, rtol=0, atol=1e-9)
        # Gaussian bins one apart on a circle of 8: sum = sqrt(2 pi) up to
        # the terms beyond +-4 bins (< 4e-4).
        for a in (0, 1):
            assert abs(f[8 * a: 8 * a + 8].sum() - math.sqrt(2 * math.pi)) < 4e-4
        # size bins: those of the config decoder's spatial features
        s = orc.spatial_features(u, v, r, wx, wy)
        np.testing.assert_allclose(f[16:], s[32:], rtol=0, atol=1e-15)
    # a bin centre gives 1; the wrap makes bins 0 and 7 neighbours
    f = orc.paper_features(2.5 / 8 * 4, 0.0, 0.1, 4, 4)
    assert f[2] == pytest.approx(1.0, abs=1e-15) and f[1] == pytest.approx(f[3], abs=1e-15)
    f = orc.paper_features(0.0, 0.0, 0.1, 4, 4)           # 8p = 0: between bins 7 and 0
    assert f[0] == pytest.approx(f[7], abs=1e-15) and f[0] == pytest.approx(math.exp(-0.125))


def build(c1, wa2_id=False, wa3_id=False, ang_col=None):
    p = np.zeros(fi.N_PAPER_DECODER_PARAMS)
    sl = slices()
    eye = np.eye(64)
    p[sl[0][1]] = c1                                   # bF1; WF1 = 0
    p[sl[1][0]] = eye.ravel()                          # WF2 = I
    wa1 = np.zeros((64, 69))
    wa1[:, :64] = eye
    if ang_col is not None:
        wa1[:, :64] = 0
        wa1[0, 64 + ang_col] = 1.0
    p[sl[2][0]] = wa1.ravel()
    if wa2_id:
        p[sl[3][0]] = eye.ravel()
    if wa3_id:
        p[sl[4][0]] = eye.ravel()
    p[sl[5][0]] = eye.ravel()                          # WA4 = I
    wa5 = np.zeros((4, 64))
    wa5[np.arange(4), np.arange(4)] = 1.0
    p[sl[6][0]] = wa5.ravel()
    return p


def run(p, wi=(0.1, 0.2, 0.9), wo=(0.3, -0.1, 0.8)):
    mats = fi.materials_for(1, 2)
    g = one_pixel(0.3, 0.4, 0.1, wi, wo)
    y, _ = orc.paper_decoder_gbuffer(p, np.zeros((1, 64)), mats, g)
    return y[:, 0]


def test_leaky_slope_and_residual_skip():
    c1 = np.zeros(64)
    c1[:4] = [2.0, -3.0, 0.5, -1.0]
    # WA2 = WA3 = 0: F1, F2, A1, the block's sum, A4: five activations of
    # the negative inputs -> x 0.01^5 (A2's output is zero).
    y = run(build(c1))
    np.testing.assert_allclose(y, [2.0, -3e-10, 0.5, -1e-10], rtol=1e-12, atol=0)
    # WA2 = WA3 = I: h = lrelu(x), block = lrelu(h + x): the skip adds x.
    y = run(build(c1, wa2_id=True, wa3_id=True))
    x = np.array([2.0, -3e-6, 0.5, -1e-6])
    h = np.where(x > 0, x, 0.01 * x)
    blk = h + x
    blk = np.where(blk > 0, blk, 0.01 * blk)
    np.testing.assert_allclose(y, np.where(blk > 0, blk, 0.01 * blk), rtol=1e-12, atol=0)


@pytest.mark.parametrize("col,val", [(0, 0.1), (1, 0.2), (2, 0.9), (3, 0.3), (4, -0.1)])
def test_angular_inputs(col, val):
    y = run(build(np.zeros(64), ang_col=col))
    expect = np.float32(val) if val > 0 else 0.01 ** 3 * np.float32(val)
    # x = lrelu(angle); the block gives lrelu(x); A4 another lrelu
    assert y[0] == pytest.approx(float(expect), rel=1e-6)


def test_against_numpy_chain():
    rng = np.random.default_rng(3)
    mats = fi.materials_for(4, 4)
    g = fi.make_gbuffer(9, 7, 4, seed=5)
    g.fabric_id[:] = rng.integers(0, 4, g.n).astype(np.uint16)
    p = fi.init_paper_params(6, bias_scale=0.1).astype(np.float64)
    z = fi.random_latents(4, 7, dim=64).astype(np.float64)
    y, _ = orc.paper_decoder_gbuffer(p, z, mats, g)
    lr = lambda a: np.where(a > 0, a, 0.01 * a)
    W = [(p[a].reshape(o, i), p[b]) for a, b, o, i in slices()]
    for k in range(g.n):
        m = mats[g.fabric_id[k]]
        f = orc.paper_features(g.u[k], g.v[k], g.radius[k], m.wx, m.wy)
        t = lr(W[0][0] @ np.concatenate([z[g.fabric_id[k]], f]) + W[0][1])
        s = lr(W[1][0] @ t + W[1][1])
        ang = np.array([g.wi_x[k], g.wi_y[k], g.wi_z[k], g.wo_x[k], g.wo_y[k]], dtype=float)
        x = lr(W[2][0] @ np.concatenate([s, ang]) + W[2][1])
        h = lr(W[3][0] @ x + W[3][1])
        r = lr(W[4][0] @ h + W[4][1] + x)
        q = lr(W[5][0] @ r + W[5][1])
        out = W[6][0] @ q + W[6][1]
        np.testing.assert_allclose(y[:, k], out, rtol=1e-12, atol=1e-12)
