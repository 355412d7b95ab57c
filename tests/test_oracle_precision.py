"""Pins of the oracle's reduced-precision decoders (operand rounding of the
BF16 / FP16 shading paths: round to nearest, ties to even): the rounding
itself against numpy's IEEE binary16 conversion and an independent
bfloat16 rounding of float32 bit patterns, including ties, binary16
subnormals and overflow; the decoders with rounded operands against numpy
chains that round the same operands with those independent routines (the
latent's product and every bias, activation and sum exact)."""
import math

import numpy as np
import pytest

import fabric_inputs as fi
import oracle as orc

NDEC = fi.N_DECODER_PARAMS


def bf16_of_f32(x):
    """bfloat16 round-to-nearest-even of float32 values by their bit patterns."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def test_round_operand_fp16_matches_numpy():
    rng = np.random.default_rng(1)
    mags = np.exp(rng.uniform(math.log(1e-9), math.log(6e4), 4000))
    x = mags * rng.choice([-1.0, 1.0], mags.size)
    # Ties: halfway between two binary16 neighbours (normal and subnormal).
    ties = [1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2.0 ** -20 + 2.0 ** -25, 65504.0 + 16.0,
            3 * 2.0 ** -25, -(1.0 + 2.0 ** -11)]
    for v in list(x) + ties + [0.0, 65519.0, 65520.0, 1e6, 2.0 ** -26]:
        with np.errstate(over="ignore"):
            want = float(np.float16(v))
        got = orc.round_operand(v, orc.FP16_BITS)
        assert got == want or (math.isinf(want) and got == want), (v, got, want)


def test_round_operand_bf16_matches_bit_rounding():
    rng = np.random.default_rng(2)
    x = (np.exp(rng.uniform(-30, 30, 4000)) * rng.choice([-1.0, 1.0], 4000)).astype(np.float32)
    # Exact ties: low 16 bits 0x8000 (even and odd upper halves).
    ties = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40490000 | 0x8000],
                     dtype=np.uint32)).view(np.float32)
    x = np.concatenate([x, ties])
    want = bf16_of_f32(x)
    got = np.array([orc.round_operand(float(v), orc.BF16_BITS) for v in x])
    np.testing.assert_array_equal(got, want)
    assert orc.round_operand(1.0 + 2.0 ** -8, orc.BF16_BITS) == 1.0          # tie to even
    assert orc.round_operand(1.0 + 3 * 2.0 ** -8, orc.BF16_BITS) == 1.0 + 2.0 ** -6
    assert orc.round_operand(0.3, 0) == 0.3


def dec_mats(P):
    out, off = [], 0
    for o, i in fi.DECODER_SHAPES:
        out.append((P[off:off + o * i].reshape(o, i), P[off + o * i:off + o * i + o]))
        off += o * i + o
    return out


@pytest.mark.parametrize("bits", [orc.FP16_BITS, orc.BF16_BITS])
def test_decoder_rounds_the_product_operands(bits):
    rnd = (lambda a: np.asarray(a, np.float64).astype(np.float16).astype(np.float64)) \
        if bits == orc.FP16_BITS else (lambda a: bf16_of_f32(np.asarray(a, np.float64)))
    P = fi.init_params(51, bias_scale=0.1)[:NDEC].astype(np.float64)
    if bits == orc.BF16_BITS:
        P = P.astype(np.float32).astype(np.float64)   # the bit rounding takes float32 inputs
    mats = fi.materials_for(4, 52)
    Z = fi.random_latents(4, 53).astype(np.float64)
    g = fi.make_gbuffer(8, 6, 4, seed=54)
    g.fabric_id[:] = np.arange(g.n) % 4
    y, _ = orc.decoder_gbuffer(P, Z, mats, g, operand_bits=bits)
    y0, _ = orc.decoder_gbuffer(P, Z, mats, g)
    assert not np.allclose(y, y0, rtol=1e-6, atol=0)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = dec_mats(P)
    for p in range(g.n):
        m = mats[g.fabric_id[p]]
        s = orc.spatial_features(float(g.u[p]), float(g.v[p]), float(g.radius[p]), m.wx, m.wy)
        if bits == orc.BF16_BITS:
            s = s.astype(np.float32).astype(np.float64)
        ang = np.array([g.wi_x[p], g.wi_y[p], g.wi_z[p], g.wo_x[p], g.wo_y[p]], dtype=float)
        z = Z[g.fabric_id[p]]
        a1 = W1[:, :32] @ z + rnd(W1[:, 32:]) @ rnd(s) + b1
        h1 = np.maximum(a1, 0)
        h2 = np.maximum(rnd(W2) @ rnd(h1.astype(np.float32) if bits == orc.BF16_BITS else h1) + b2, 0)
        x3 = np.concatenate([h2, ang])
        h3 = np.maximum(rnd(W3) @ rnd(x3.astype(np.float32) if bits == orc.BF16_BITS else x3) + b3, 0)
        out = rnd(W4) @ rnd(h3.astype(np.float32) if bits == orc.BF16_BITS else h3) + b4
        # The oracle rounds the FP64 activations themselves; the chain above
        # rounds their float32 values for bfloat16 (the same result unless a
        # value lies within float32's spacing of a bfloat16 tie).
        np.testing.assert_allclose(y[:, p], out, rtol=1e-9, atol=1e-12)


def test_paper_decoder_rounds_the_product_operands():
    """The paper-size decoder in binary16 operands against a numpy chain
    (leaky ReLU, residual add and biases exact)."""
    r16 = lambda a: np.asarray(a, np.float64).astype(np.float16).astype(np.float64)
    mats = fi.materials_for(3, 61)
    g = fi.make_gbuffer(7, 5, 3, seed=62)
    g.fabric_id[:] = np.arange(g.n) % 3
    P = fi.init_paper_params(63, bias_scale=0.1).astype(np.float64)
    Z = fi.random_latents(3, 64, dim=64).astype(np.float64)
    y, _ = orc.paper_decoder_gbuffer(P, Z, mats, g, operand_bits=orc.FP16_BITS)
    W, off = [], 0
    for o, i in fi.PAPER_DECODER_SHAPES:
        W.append((P[off:off + o * i].reshape(o, i), P[off + o * i:off + o * i + o]))
        off += o * i + o
    lr = lambda a: np.where(a > 0, a, 0.01 * a)
    q = lambda k, x: r16(W[k][0]) @ r16(x) + W[k][1]
    for k in range(g.n):
        m = mats[g.fabric_id[k]]
        f = orc.paper_features(g.u[k], g.v[k], g.radius[k], m.wx, m.wy)
        z = Z[g.fabric_id[k]]
        t = lr(W[0][0][:, :64] @ z + r16(W[0][0][:, 64:]) @ r16(f) + W[0][1])
        sp = lr(q(1, t))
        ang = np.array([g.wi_x[k], g.wi_y[k], g.wi_z[k], g.wo_x[k], g.wo_y[k]], dtype=float)
        x = lr(q(2, np.concatenate([sp, ang])))
        h = lr(q(3, x))
        rr = lr(q(4, h) + x)
        gg = lr(q(5, rr))
        out = q(6, gg)
        np.testing.assert_allclose(y[:, k], out, rtol=1e-10, atol=1e-12)
