"""Seeded synthetic inputs for the woven-fabric shading path.

This module only draws inputs: weave patterns, per-yarn material parameters,
albedos, G-buffers (fabric id, pattern-tiled uv, footprint radius, light and
view directions) and initial network weights.  It holds none of the shading
model's or the network's arithmetic, so both the FP64 oracle and the HIP
library can be driven from it without sharing any computation.

Parameter ranges follow the paper's Table 2 (sampling distributions) where the
workload descriptions below are silent:
  * inclination u ~ U(15 deg, 45 deg), height-field scale beta ~ U(0, 2),
    gap = 0.2 of the yarn (Sec. 5.1);
  * twist psi ~ U(0, 0.5) rad and roughness alpha ~ U(0.1, 0.6) as the
    workloads fix them (Table 2's discrete +-30 deg twist and U(0.1, 1)
    roughness are the paper's training ranges);
  * diffuse blend weight w ~ U(0.2, 0.8) (the paper gives no value, Eq. (1));
  * RGB albedos k_d, k_s ~ U(0.2, 0.9).
Directions are cosine-weighted on the upper hemisphere; the paper's
rejection of (x, y) ~ U(-1, 1)^2 outside the unit disk with z computed from
x, y (Table 2, Sec. 5.1) draws exactly this distribution.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Weave patterns.  P[j][i] = 1 means the warp yarn (running along +y / v) is
# on top at column i, row j; 0 means the weft yarn (along +x / u) is on top.
# ---------------------------------------------------------------------------


def pattern_plain() -> np.ndarray:
    return np.array([[1, 0], [0, 1]], dtype=np.uint8)


def pattern_twill(n: int, up: int) -> np.ndarray:
    """n x n twill whose warp floats over `up` consecutive rows."""
    p = np.zeros((n, n), dtype=np.uint8)
    for j in range(n):
        for i in range(n):
            p[j, i] = 1 if (i - j) % n < up else 0
    return p


def pattern_satin5() -> np.ndarray:
    """Warp-faced 5-harness satin with move 2: weft on top once per row."""
    p = np.zeros((5, 5), dtype=np.uint8)
    for j in range(5):
        for i in range(5):
            p[j, i] = 0 if (i - 2 * j) % 5 == 0 else 1
    return p


def pattern_basket22() -> np.ndarray:
    base = pattern_plain()
    p = np.zeros((4, 4), dtype=np.uint8)
    for j in range(4):
        for i in range(4):
            p[j, i] = base[(j // 2) % 2, (i // 2) % 2]
    return p


def _interlaced(p: np.ndarray) -> bool:
    rows_ok = all(0 < p[j].sum() < p.shape[1] for j in range(p.shape[0]))
    cols_ok = all(0 < p[:, i].sum() < p.shape[0] for i in range(p.shape[1]))
    return rows_ok and cols_ok


def random_pattern(rng: np.random.Generator, min_side: int, max_side: int) -> np.ndarray:
    """Bernoulli(1/2) cells, redrawn until every row and column interlaces."""
    wx = int(rng.integers(min_side, max_side + 1))
    wy = int(rng.integers(min_side, max_side + 1))
    while True:
        p = (rng.random((wy, wx)) < 0.5).astype(np.uint8)
        if _interlaced(p):
            return p


NAMED_PATTERNS = {
    "plain": pattern_plain,
    "twill21": lambda: pattern_twill(3, 2),
    "twill31": lambda: pattern_twill(4, 3),
    "satin5": pattern_satin5,
    "basket22": pattern_basket22,
}


# ---------------------------------------------------------------------------
# Materials (Table 1 parameters per yarn type; index 0 = warp, 1 = weft)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Material:
    pattern: np.ndarray          # uint8 [wy, wx]
    alpha: np.ndarray            # float32 [2] roughness
    beta: np.ndarray             # float32 [2] height-field scaling
    twist: np.ndarray            # float32 [2] twist angle psi (rad)
    incl: np.ndarray             # float32 [2] inclination angle u (rad)
    gap: np.ndarray              # float32 [2] gap fraction of the yarn
    wblend: np.ndarray           # float32 [2] diffuse blend weight w
    kd: np.ndarray               # float32 [2, 3] diffuse albedo RGB
    ks: np.ndarray               # float32 [2, 3] specular albedo RGB

    @property
    def wx(self) -> int:
        return int(self.pattern.shape[1])

    @property
    def wy(self) -> int:
        return int(self.pattern.shape[0])


def _f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32)


def random_material(rng: np.random.Generator, pattern: np.ndarray,
                    alpha_range=(0.1, 0.6), twist_range=(0.0, 0.5)) -> Material:
    deg = math.pi / 180.0
    return Material(
        pattern=np.ascontiguousarray(pattern, dtype=np.uint8),
        alpha=_f32(rng.uniform(*alpha_range, size=2)),
        beta=_f32(rng.uniform(0.0, 2.0, size=2)),
        twist=_f32(rng.uniform(*twist_range, size=2)),
        incl=_f32(rng.uniform(15 * deg, 45 * deg, size=2)),
        gap=_f32([0.2, 0.2]),
        wblend=_f32(rng.uniform(0.2, 0.8, size=2)),
        kd=_f32(rng.uniform(0.2, 0.9, size=(2, 3))),
        ks=_f32(rng.uniform(0.2, 0.9, size=(2, 3))),
    )


def uniform_material(pattern: np.ndarray, alpha=0.5, beta=1.0, twist=0.0,
                     incl=math.pi / 6, gap=0.2, wblend=0.5, kd=0.5, ks=0.5) -> Material:
    """Identical warp and weft parameters (handy for closed-form checks)."""
    return Material(
        pattern=np.ascontiguousarray(pattern, dtype=np.uint8),
        alpha=_f32([alpha, alpha]), beta=_f32([beta, beta]),
        twist=_f32([twist, twist]), incl=_f32([incl, incl]),
        gap=_f32([gap, gap]), wblend=_f32([wblend, wblend]),
        kd=_f32(np.full((2, 3), kd)), ks=_f32(np.full((2, 3), ks)),
    )


# The parameter points of the latent interpolation study (Sec. 5
# "Interpolation"): latents encoded at 0.2 and 0.8, blended at 0.3 and 0.6,
# extrapolated to 0.9.
INTERP_ENDPOINTS = (0.2, 0.8)
INTERP_POINTS = (0.3, 0.6, 0.9)


def parameter_sweep(field: str, values: Sequence[float], seed: int,
                    pattern: Optional[np.ndarray] = None,
                    other: Optional[float] = None) -> List[Material]:
    """One seeded material (twill 2/1 unless `pattern` is given) repeated with
    its `field` ("alpha": roughness, or "beta": height-field scaling) set to
    each of `values` on both yarns; every other field is shared, the other
    of the two set to `other` on both yarns when given.  The same seed gives
    the same material as `sweep_training_set`'s variants start from."""
    if field not in ("alpha", "beta"):
        raise ValueError("field is alpha or beta")
    rng = np.random.default_rng(seed)
    base = random_material(rng, NAMED_PATTERNS["twill21"]() if pattern is None else pattern)
    if other is not None:
        base = dataclasses.replace(base, **{("beta" if field == "alpha" else "alpha"): _f32([other, other])})
    out = []
    for val in values:
        m = dataclasses.replace(base, **{field: _f32([val, val])})
        out.append(m)
    return out


def sweep_training_set(n: int, seed: int, lo: float = 0.15, hi: float = 0.95,
                       pattern: Optional[np.ndarray] = None,
                       variant_seed: Optional[int] = None) -> List[Material]:
    """n variants of one seeded material whose roughness and height-field
    scale are drawn uniformly from [lo, hi] (per yarn): a training table that
    spans the parameter range of the interpolation study.  With
    `variant_seed` the draws come from a generator of their own: variants of
    the same material that a table made without it does not hold."""
    rng = np.random.default_rng(seed)
    base = random_material(rng, NAMED_PATTERNS["twill21"]() if pattern is None else pattern)
    if variant_seed is not None:
        rng = np.random.default_rng(variant_seed)
    return [dataclasses.replace(base, alpha=_f32(rng.uniform(lo, hi, 2)),
                                beta=_f32(rng.uniform(lo, hi, 2))) for _ in range(n)]


def materials_for(n_fabrics: int, seed: int, max_random_side: int = 8) -> List[Material]:
    """The fabric set of a workload.

    1 fabric: the plain weave.  8 fabrics: plain, twill 2/1, twill 3/1,
    satin 5, basket 2x2 and 3 seeded random cells of side 2..8.  More fabrics:
    those 8 followed by seeded random cells of side 2..max_random_side.
    Random patterns are deduplicated.
    """
    rng = np.random.default_rng(seed)
    pats: List[np.ndarray] = []
    named = list(NAMED_PATTERNS.values())
    if n_fabrics == 1:
        pats = [pattern_plain()]
    else:
        pats = [f() for f in named][:n_fabrics]
        seen = {(p.shape, p.tobytes()) for p in pats}
        first_random = 3 if n_fabrics >= 8 else 0
        while len(pats) < n_fabrics:
            side = 8 if len(pats) < 5 + first_random else max_random_side
            p = random_pattern(rng, 2, side)
            key = (p.shape, p.tobytes())
            if key in seen:
                continue
            seen.add(key)
            pats.append(p)
    return [random_material(rng, p) for p in pats]


# ---------------------------------------------------------------------------
# G-buffers: structure-of-arrays, float32 fields plus a uint16 fabric id.
# ---------------------------------------------------------------------------

GBUF_FIELDS = ("u", "v", "radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z")


@dataclasses.dataclass
class GBuffer:
    fabric_id: np.ndarray        # uint16 [n]
    u: np.ndarray                # float32 [n] (cells)
    v: np.ndarray
    radius: np.ndarray           # footprint radius (cells)
    wi_x: np.ndarray
    wi_y: np.ndarray
    wi_z: np.ndarray
    wo_x: np.ndarray
    wo_y: np.ndarray
    wo_z: np.ndarray

    @property
    def n(self) -> int:
        return int(self.u.shape[0])

    def subset(self, idx: np.ndarray) -> "GBuffer":
        return GBuffer(**{f.name: np.ascontiguousarray(getattr(self, f.name)[idx])
                          for f in dataclasses.fields(self)})

    def nbytes(self) -> int:
        return sum(getattr(self, f.name).nbytes for f in dataclasses.fields(self))


def cosine_directions(rng: np.random.Generator, n: int):
    """Cosine-weighted hemisphere directions (Malley's method)."""
    xi1 = rng.random(n)
    xi2 = rng.random(n)
    s = np.sqrt(xi1)
    x = s * np.cos(2 * np.pi * xi2)
    y = s * np.sin(2 * np.pi * xi2)
    z = np.sqrt(1.0 - xi1)
    return _f32(x), _f32(y), _f32(z)


def log_uniform(rng: np.random.Generator, lo: float, hi: float, n: int) -> np.ndarray:
    return _f32(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n)))


def tile_fabric_ids(rng: np.random.Generator, width: int, height: int,
                    n_fabrics: int, tile: int = 64) -> np.ndarray:
    """One fabric per tile x tile block of pixels, row-major pixel order."""
    ty = (height + tile - 1) // tile
    tx = (width + tile - 1) // tile
    ids = rng.integers(0, n_fabrics, size=(ty, tx))
    full = np.repeat(np.repeat(ids, tile, axis=0), tile, axis=1)[:height, :width]
    return np.ascontiguousarray(full.reshape(-1).astype(np.uint16))


def make_gbuffer(width: int, height: int, n_fabrics: int, seed: int,
                 r_range=(1e-3, 0.5), uv_max: float = 8.0,
                 out_of_range_frac: float = 0.0, btdf_frac: float = 0.0) -> GBuffer:
    """A seeded width x height G-buffer (row-major pixels).

    Per pixel, iid: uv ~ U[0, uv_max)^2, radius log-uniform over r_range,
    wi and wo cosine-weighted.  With out_of_range_frac > 0 that fraction of
    pixels (iid) is moved outside the network's training range: half get
    radius ~ log-U[1, 2] cells, half a grazing view wo.z ~ U(0, 0.05).
    With btdf_frac > 0 that fraction (iid, from a stream of its own) is lit
    from below the fabric (wi.z negated): transmission queries.
    """
    rng = np.random.default_rng(seed)
    n = width * height
    fid = tile_fabric_ids(rng, width, height, n_fabrics)
    u = _f32(rng.uniform(0.0, uv_max, size=n))
    v = _f32(rng.uniform(0.0, uv_max, size=n))
    r = log_uniform(rng, r_range[0], r_range[1], n)
    wix, wiy, wiz = cosine_directions(rng, n)
    wox, woy, woz = cosine_directions(rng, n)
    if out_of_range_frac > 0.0:
        sel = rng.random(n) < out_of_range_frac
        half = rng.random(n) < 0.5
        big = sel & half
        graze = sel & ~half
        r[big] = log_uniform(rng, 1.0, 2.0, int(big.sum()))
        m = int(graze.sum())
        z = 0.05 * (0.001 + 0.998 * rng.random(m))
        phi = 2 * np.pi * rng.random(m)
        sxy = np.sqrt(1.0 - z * z)
        wox[graze] = _f32(sxy * np.cos(phi))
        woy[graze] = _f32(sxy * np.sin(phi))
        woz[graze] = _f32(z)
    if btdf_frac > 0.0:
        below = np.random.default_rng(seed + 7919).random(n) < btdf_frac
        wiz[below] = -wiz[below]
    return GBuffer(fid, u, v, r, wix, wiy, wiz, wox, woy, woz)


def jitter_gbuffer(g: GBuffer, frame_seed: int) -> GBuffer:
    """Camera jitter for a frame sequence: uv += delta * radius, delta ~ U[-1,1)^2."""
    rng = np.random.default_rng(frame_seed)
    d = rng.uniform(-1.0, 1.0, size=(2, g.n))
    out = dataclasses.replace(g)
    out.u = _f32(g.u + d[0] * g.radius)
    out.v = _f32(g.v + d[1] * g.radius)
    return out


def subset_indices(n: int, frac: float, seed: int) -> np.ndarray:
    """A seeded, sorted subset of pixel indices (e.g. 1 % of a frame)."""
    rng = np.random.default_rng(seed)
    k = max(1, int(round(n * frac)))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# Network parameter vector: seeded Kaiming-uniform weights, zero biases.
# Layout (row-major, rows = output units):
#   decoder  W1[64][72] b1[64] W2[64][64] b2[64] W3[64][69] b3[64] W4[4][64] b4[4]
#   encoder  E1[128][524] c1[128] E2[128][128] c2[128] E3[128][128] c3[128]
#            E4[32][128] c4[32]
# ---------------------------------------------------------------------------

DECODER_SHAPES = [(64, 72), (64, 64), (64, 69), (4, 64)]
ENCODER_SHAPES = [(128, 524), (128, 128), (128, 128), (32, 128)]


def _layer_sizes(shapes: Sequence[tuple]) -> int:
    return sum(o * i + o for o, i in shapes)


N_DECODER_PARAMS = _layer_sizes(DECODER_SHAPES)   # 13,572
N_ENCODER_PARAMS = _layer_sizes(ENCODER_SHAPES)   # 104,352
N_PARAMS = N_DECODER_PARAMS + N_ENCODER_PARAMS


def init_params(seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """Kaiming-uniform U(+-sqrt(6 / fan_in)) weights; biases U(+-bias_scale)."""
    rng = np.random.default_rng(seed)
    out = []
    for shapes in (DECODER_SHAPES, ENCODER_SHAPES):
        for o, i in shapes:
            bound = math.sqrt(6.0 / i)
            out.append(rng.uniform(-bound, bound, size=o * i))
            out.append(rng.uniform(-bias_scale, bias_scale, size=o) if bias_scale > 0
                       else np.zeros(o))
    return _f32(np.concatenate(out))


def random_latents(n_fabrics: int, seed: int, scale: float = 1.0, dim: int = 32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _f32(rng.normal(0.0, scale, size=(n_fabrics, dim)))


# The decoder at the paper's own form (latent 64, 24 one-blob channels, two
# fusion and five angular layers of width 64): rows x columns per layer
# [F1 (z, blob), F2, A1 (s, wi.xyz, wo.xy), A2, A3, A4, A5].
PAPER_DECODER_SHAPES = [(64, 88), (64, 64), (64, 69), (64, 64), (64, 64), (64, 64), (4, 64)]
N_PAPER_DECODER_PARAMS = _layer_sizes(PAPER_DECODER_SHAPES)   # 27,076


def init_paper_params(seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """Paper-size decoder parameters, Kaiming-uniform like init_params."""
    rng = np.random.default_rng(seed)
    out = []
    for o, i in PAPER_DECODER_SHAPES:
        bound = math.sqrt(6.0 / i)
        out.append(rng.uniform(-bound, bound, size=o * i))
        out.append(rng.uniform(-bias_scale, bias_scale, size=o) if bias_scale > 0 else np.zeros(o))
    return _f32(np.concatenate(out))


# The paper-size network's encoder: the config encoder's layers with a
# latent of 64 (E1 [128][524] .. E4 [64][128], c4 [64]).
PAPER_ENCODER_SHAPES = [(128, 524), (128, 128), (128, 128), (64, 128)]
N_PAPER_ENCODER_PARAMS = _layer_sizes(PAPER_ENCODER_SHAPES)   # 108,480


def init_paper_encoder_params(seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """Paper-size encoder parameters, Kaiming-uniform like init_params."""
    rng = np.random.default_rng(seed)
    out = []
    for o, i in PAPER_ENCODER_SHAPES:
        bound = math.sqrt(6.0 / i)
        out.append(rng.uniform(-bound, bound, size=o * i))
        out.append(rng.uniform(-bias_scale, bias_scale, size=o) if bias_scale > 0 else np.zeros(o))
    return _f32(np.concatenate(out))


def random_targets(n: int, seed: int) -> np.ndarray:
    """Plausible component targets [4][n]: C in [0, 0.4], S log-spread."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 0.4, size=(2, n))
    s = np.exp(rng.uniform(math.log(1e-4), math.log(5.0), size=(2, n)))
    return _f32(np.concatenate([c, s], axis=0))


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    width: int
    height: int
    n_fabrics: int
    n_samples: int
    r_range: tuple
    out_of_range_frac: float = 0.0
    max_random_side: int = 8
    subset_frac: float = 1.0
    btdf_frac: float = 0.0

    def seed(self, run: int = 0) -> int:
        return 1000 * WORKLOAD_INDEX[self.name] + run

    def materials(self, run: int = 0) -> List[Material]:
        return materials_for(self.n_fabrics, self.seed(run), self.max_random_side)

    def gbuffer(self, run: int = 0) -> GBuffer:
        return make_gbuffer(self.width, self.height, self.n_fabrics, self.seed(run) + 17,
                            r_range=self.r_range, out_of_range_frac=self.out_of_range_frac,
                            btdf_frac=self.btdf_frac)


WORKLOADS = {
    "plain128": Workload("plain128", 128, 128, 1, 64, (1e-3, 0.5)),
    "fabric8_1080p": Workload("fabric8_1080p", 1920, 1080, 8, 256, (1e-3, 0.5), subset_frac=0.01),
    "train_2p20": Workload("train_2p20", 1024, 1024, 8, 256, (1e-3, 0.5)),
    "fabric64_4k": Workload("fabric64_4k", 3840, 2160, 64, 256, (1e-4, 2.0),
                            max_random_side=16, subset_frac=0.0025),
    "hybrid_1080p": Workload("hybrid_1080p", 1920, 1080, 8, 256, (1e-3, 0.5),
                             out_of_range_frac=0.2, subset_frac=0.01),
    # The 1080p frame with half its pixels lit from below (transmission).
    "btdf_1080p": Workload("btdf_1080p", 1920, 1080, 8, 256, (1e-3, 0.5), subset_frac=0.01,
                           btdf_frac=0.5),
}
WORKLOAD_INDEX = {"plain128": 1, "fabric8_1080p": 2, "train_2p20": 3,
                  "fabric64_4k": 4, "hybrid_1080p": 5, "btdf_1080p": 6}
