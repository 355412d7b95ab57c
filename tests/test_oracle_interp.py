"""Pins of the oracle's latent interpolation (Sec. 5 "Interpolation"): the
paper's parameter points (tests/golden/latent_interpolation_points.txt) and
their interpolation / extrapolation split, exact recovery of a latent that
is affine in the parameter, the endpoints, translation equivariance of an
affine blend, and read-before-write over a table."""
import os

import numpy as np
import pytest

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "latent_interpolation_points.txt")


def golden_points():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append((line[0], float(line[1])))
    return rows


def test_paper_points_split():
    rows = golden_points()
    p_a, p_b = [p for k, p in rows if k == "encoded"]
    weights = {p: orc.parameter_weight(p, p_a, p_b) for k, p in rows if k != "encoded"}
    # Hand-computed: (0.3 - 0.2) / 0.6, (0.6 - 0.2) / 0.6, (0.9 - 0.2) / 0.6.
    assert weights[0.3] == pytest.approx(1 / 6, abs=1e-12)
    assert weights[0.6] == pytest.approx(2 / 3, abs=1e-12)
    assert weights[0.9] == pytest.approx(7 / 6, abs=1e-12)
    for k, p in rows:
        if k == "interpolated":
            assert 0.0 < weights[p] < 1.0
        elif k == "extrapolated":
            assert weights[p] > 1.0
    assert orc.parameter_weight(p_a, p_a, p_b) == 0.0
    assert orc.parameter_weight(p_b, p_a, p_b) == 1.0


def test_affine_latent_recovered():
    """If the encoder's latent were affine in the parameter, z(p) = u + p w,
    blending z(0.2) and z(0.8) must give z(p) at every other point exactly."""
    rng = np.random.default_rng(7)
    u, w = rng.normal(size=32), rng.normal(size=32)
    pts = [p for _, p in golden_points()]
    table = np.stack([u + p * w for p in pts])
    garbage = table.copy()
    garbage[2:] = rng.normal(size=(len(pts) - 2, 32))
    dst = list(range(2, len(pts)))
    t = [orc.parameter_weight(pts[d], pts[0], pts[1]) for d in dst]
    out = orc.interpolate_latents(garbage, dst, [0] * len(dst), [1] * len(dst), t)
    np.testing.assert_allclose(out, table, rtol=0, atol=1e-12)


def test_endpoints_and_midpoint():
    rng = np.random.default_rng(8)
    z = rng.normal(size=(3, 32))
    out = orc.interpolate_latents(z, [2], [0], [1], [0.0])
    assert np.array_equal(out[2], z[0])
    out = orc.interpolate_latents(z, [2], [0], [1], [1.0])
    assert np.array_equal(out[2], z[1])
    out = orc.interpolate_latents(z, [2], [0], [1], [0.5])
    np.testing.assert_allclose(out[2], (z[0] + z[1]) / 2, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(out[:2], z[:2])


def test_translation_equivariant():
    """Blend weights sum to one: shifting every latent by c shifts every
    blend by c, for interpolation and extrapolation alike."""
    rng = np.random.default_rng(9)
    z = rng.normal(size=(4, 32))
    c = rng.normal(size=32)
    args = ([2, 3], [0, 1], [1, 0], [7 / 6, -0.5])
    a = orc.interpolate_latents(z, *args)
    b = orc.interpolate_latents(z + c, *args)
    np.testing.assert_allclose(b - c, a, rtol=0, atol=1e-12)


def test_reads_precede_writes():
    """Slot 0 is overwritten by one blend and read by another: the reader
    sees the table as it was before the call."""
    z = np.arange(3 * 32, dtype=np.float64).reshape(3, 32)
    out = orc.interpolate_latents(z, [0, 2], [1, 0], [2, 1], [0.25, 0.5])
    np.testing.assert_allclose(out[0], 0.75 * z[1] + 0.25 * z[2], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[2], 0.5 * z[0] + 0.5 * z[1], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(out[1], z[1])
