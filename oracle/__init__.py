"""ctypes front end of the FP64 CPU oracle (``oracle/fabric_oracle.c``).

TEST INFRASTRUCTURE: imported only by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  It never imports the HIP
library's package and the HIP library never imports it; the two meet only in
the seeded inputs of ``fabric_inputs``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fabric_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64; no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        # No contraction of a*b+c: the visibility march's float32 steps must
        # round once per operation.
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-ffp-contract=off",
               "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Material(ctypes.Structure):
    _fields_ = [
        ("wx", ctypes.c_int32), ("wy", ctypes.c_int32),
        ("pattern", ctypes.c_uint8 * 256),
        ("alpha", ctypes.c_double * 2), ("beta", ctypes.c_double * 2),
        ("twist", ctypes.c_double * 2), ("incl", ctypes.c_double * 2),
        ("gap", ctypes.c_double * 2), ("wblend", ctypes.c_double * 2),
        ("kd", (ctypes.c_double * 3) * 2), ("ks", (ctypes.c_double * 3) * 2),
    ]


class GBuf(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("fabric_id", ctypes.c_void_p)] + [
        (f, ctypes.c_void_p) for f in
        ("u", "v", "radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z")]


_P = ctypes.c_void_p
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_concentric.argtypes = [ctypes.c_double, ctypes.c_double, _P]
        L.orc_sggx_D.restype = ctypes.c_double
        L.orc_sggx_D.argtypes = [ctypes.c_double, _P, _P]
        L.orc_sggx_sigma.restype = ctypes.c_double
        L.orc_sggx_sigma.argtypes = [ctypes.c_double, _P, _P]
        L.orc_point_brdf.argtypes = [ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P]
        L.orc_point_brdf_batch.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                           _P, _P, _P, _P, _P]
        L.orc_point_eval.argtypes = [_P, ctypes.c_double, ctypes.c_double, _P, _P, _P]
        L.orc_point_eval_batch.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P, _P]
        L.orc_filter_pixel.restype = ctypes.c_int
        L.orc_filter_pixel.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       _P, _P, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_int, _P, _P]
        L.orc_filter_batch.restype = ctypes.c_int64
        L.orc_filter_batch.argtypes = [_P, ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]
        L.orc_surface_height.restype = ctypes.c_double
        L.orc_surface_height.argtypes = [_P, ctypes.c_double, ctypes.c_double]
        L.orc_height_table.restype = ctypes.c_float
        L.orc_height_table.argtypes = [_P, _P]
        L.orc_visible.restype = ctypes.c_int
        L.orc_visible.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, _P]
        L.orc_visible_at.restype = ctypes.c_int
        L.orc_visible_at.argtypes = [_P, ctypes.c_double, ctypes.c_double, _P]
        L.orc_param_counts.restype = ctypes.c_int
        L.orc_param_counts.argtypes = [_P]
        L.orc_spatial_features.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, _P]
        L.orc_decoder_batch.restype = ctypes.c_int64
        L.orc_decoder_batch.argtypes = [_P, _P, _P, ctypes.c_int, _P, _P, _P]
        L.orc_decoder_batch_q.restype = ctypes.c_int64
        L.orc_decoder_batch_q.argtypes = [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, _P, _P]
        L.orc_round_operand.restype = ctypes.c_double
        L.orc_round_operand.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_encoder_input.argtypes = [_P, _P]
        L.orc_paper_param_count.restype = ctypes.c_int
        L.orc_paper_features.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, _P]
        L.orc_paper_decoder_batch.restype = ctypes.c_int64
        L.orc_paper_decoder_batch.argtypes = [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int,
                                              _P, _P]
        L.orc_paper_decoder_batch_q.restype = ctypes.c_int64
        L.orc_paper_decoder_batch_q.argtypes = [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, _P, _P]
        L.orc_paper_features_raw.argtypes = L.orc_paper_features.argtypes
        L.orc_encoder_batch.argtypes = [_P, _P, ctypes.c_int, _P]
        L.orc_encoder_batch_n.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, _P]
        L.orc_encoder_param_count.restype = ctypes.c_int
        L.orc_encoder_param_count.argtypes = [ctypes.c_int]
        L.orc_encoder_backward_batch.argtypes = [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P]
        L.orc_paper_loss_grad.restype = ctypes.c_double
        L.orc_paper_loss_grad.argtypes = [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int,
                                          _P, _P, _P]
        L.orc_loss_grad.restype = ctypes.c_double
        L.orc_loss_grad.argtypes = [_P, _P, ctypes.c_int, _P, _P, _P, _P]
        L.orc_decoder_backward_batch.argtypes = [_P, _P, _P, ctypes.c_int, _P, _P, _P, _P]
        L.orc_adam_step.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double]
        L.orc_batch_gen.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double] + [_P] * 10
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _d(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# Conversions from fabric_inputs objects
# ---------------------------------------------------------------------------

def materials(mats: Sequence) -> ctypes.Array:
    arr = (Material * max(1, len(mats)))()
    for k, m in enumerate(mats):
        o = arr[k]
        o.wx, o.wy = m.wx, m.wy
        flat = np.ascontiguousarray(m.pattern, dtype=np.uint8).reshape(-1)
        for q in range(flat.size):
            o.pattern[q] = int(flat[q])
        for name in ("alpha", "beta", "twist", "incl", "gap", "wblend"):
            vals = getattr(m, name)
            getattr(o, name)[0] = float(vals[0])
            getattr(o, name)[1] = float(vals[1])
        for y in range(2):
            for c in range(3):
                o.kd[y][c] = float(m.kd[y][c])
                o.ks[y][c] = float(m.ks[y][c])
    return arr


class _GBufHolder:
    """Keeps the numpy arrays alive while the C side holds pointers."""

    def __init__(self, g):
        self.arrays = [np.ascontiguousarray(g.fabric_id, dtype=np.uint16)] + [
            np.ascontiguousarray(getattr(g, f), dtype=np.float32) for f in
            ("u", "v", "radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z")]
        self.s = GBuf(int(self.arrays[1].shape[0]), *[_ptr(a) for a in self.arrays])

    @property
    def ref(self):
        return ctypes.byref(self.s)


# ---------------------------------------------------------------------------
# Python-facing functions
# ---------------------------------------------------------------------------

def splitmix64(seed: int, index: int) -> int:
    return int(lib().orc_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(index)))


def concentric(x: float, y: float) -> np.ndarray:
    out = np.zeros(2)
    lib().orc_concentric(x, y, _ptr(out))
    return out


def sggx_D(alpha: float, t, h) -> float:
    return float(lib().orc_sggx_D(alpha, _ptr(_d(t)), _ptr(_d(h))))


def sggx_sigma(alpha: float, t, w) -> float:
    return float(lib().orc_sggx_sigma(alpha, _ptr(_d(t)), _ptr(_d(w))))


def point_brdf(alpha: float, w: float, n, t, wi, wo) -> np.ndarray:
    """(f_s / k_s, f_d / k_d) of Eq. (1)."""
    out = np.zeros(2)
    lib().orc_point_brdf(alpha, w, _ptr(_d(n)), _ptr(_d(t)), _ptr(_d(wi)), _ptr(_d(wo)), _ptr(out))
    return out


def point_brdf_batch(alpha: float, w: float, n, t, wi, wo) -> np.ndarray:
    """point_brdf over arrays of direction pairs wi, wo [k, 3]; returns [k, 2]."""
    WI = _d(wi).reshape(-1, 3)
    WO = _d(wo).reshape(-1, 3)
    out = np.zeros((WI.shape[0], 2))
    lib().orc_point_brdf_batch(WI.shape[0], alpha, w, _ptr(_d(n)), _ptr(_d(t)), _ptr(WI),
                               _ptr(WO), _ptr(out))
    return out


def point_eval(mat, us: float, vs: float, wi, wo) -> dict:
    m = materials([mat])
    out = np.zeros(16)
    lib().orc_point_eval(ctypes.byref(m[0]), us, vs, _ptr(_d(wi)), _ptr(_d(wo)), _ptr(out))
    return {"yarn": int(out[0]), "on_top": int(out[1]), "edge": out[2], "rho_s": out[3],
            "rho_c": out[4], "area": out[5], "n": out[6:9].copy(), "t": out[9:12].copy()}


def point_eval_batch(mat, us, vs, wi, wo) -> dict:
    """point_eval at arrays of points; returns arrays keyed like point_eval."""
    m = materials([mat])
    U = _d(us).reshape(-1)
    V = _d(vs).reshape(-1)
    out = np.zeros((U.shape[0], 16))
    lib().orc_point_eval_batch(ctypes.byref(m[0]), U.shape[0], _ptr(U), _ptr(V), _ptr(_d(wi)),
                               _ptr(_d(wo)), _ptr(out))
    return {"yarn": out[:, 0].astype(int), "on_top": out[:, 1].astype(int), "edge": out[:, 2],
            "rho_s": out[:, 3], "rho_c": out[:, 4], "area": out[:, 5], "n": out[:, 6:9],
            "t": out[:, 9:12]}


def filter_pixel(mat, u: float, v: float, r: float, wi, wo, n_samples: int, seed: int,
                 pixel: int = 0, same_sample: bool = False, visibility: bool = False):
    m = materials([mat])
    comp = np.zeros(4)
    area = np.zeros(1)
    fl = lib().orc_filter_pixel(ctypes.byref(m[0]), u, v, r, _ptr(_d(wi)), _ptr(_d(wo)),
                                int(n_samples), ctypes.c_uint64(seed), ctypes.c_uint64(pixel),
                                int(same_sample), int(visibility), _ptr(comp), _ptr(area))
    return comp, float(area[0]), int(fl)


def surface_height(mat, us: float, vs: float) -> float:
    """Height (cells) of the stand-in fabric surface at (us, vs)."""
    return float(lib().orc_surface_height(ctypes.byref(materials([mat])[0]), us, vs))


def height_table(mat):
    """The float32 height texels [wy*16, wx*16] and their maximum."""
    t = np.zeros((mat.wy * 16, mat.wx * 16), dtype=np.float32)
    hmax = lib().orc_height_table(ctypes.byref(materials([mat])[0]), _ptr(t))
    return t, float(hmax)


def visible(mat, us: float, vs: float, w) -> int:
    """V(x_p, w) of the sample point (us, vs) toward w."""
    return int(lib().orc_visible_at(ctypes.byref(materials([mat])[0]), us, vs, _ptr(_d(w))))


def visible_in_table(table, hmax: float, up: float, vp: float, w) -> int:
    """V of the march over a caller-given float32 height table [th, tw]
    (16 texels per cell) from the point (up, vp) of the period toward w."""
    t = np.ascontiguousarray(table, dtype=np.float32)
    th, tw = t.shape
    return int(lib().orc_visible(_ptr(t), tw, th, float(hmax), float(up), float(vp), _ptr(_d(w))))


def filter_gbuffer(mats: Sequence, g, n_samples: int, seed: int, same_sample: bool = True,
                   pixel_index: Optional[np.ndarray] = None, visibility: bool = False):
    """Footprint filter over a G-buffer: returns comp [4,n], rgb [3,n], flagged [n], fault [n].
    visibility=True includes the inter-yarn visibility V of Eq. (3)-(4)."""
    h = _GBufHolder(g)
    n = h.s.n
    comp = np.zeros((4, n))
    rgb = np.zeros((3, n))
    flagged = np.zeros(n, dtype=np.int32)
    fault = np.zeros(n, dtype=np.int32)
    pidx = None if pixel_index is None else np.ascontiguousarray(pixel_index, dtype=np.int64)
    m = materials(mats)
    lib().orc_filter_batch(m, len(mats), h.ref, None if pidx is None else _ptr(pidx),
                           int(n_samples), ctypes.c_uint64(seed), int(same_sample),
                           int(visibility), _ptr(comp), _ptr(rgb), _ptr(flagged), _ptr(fault))
    return comp, rgb, flagged, fault


def param_counts():
    out = np.zeros(2, dtype=np.int32)
    lib().orc_param_counts(_ptr(out))
    return int(out[0]), int(out[1])


def spatial_features(u: float, v: float, r: float, wx: int, wy: int) -> np.ndarray:
    s = np.zeros(40)
    lib().orc_spatial_features(u, v, r, wx, wy, _ptr(s))
    return s


# Significant bits of the reduced operand precisions (operand_bits below).
BF16_BITS = 8
FP16_BITS = 11


def round_operand(x: float, bits: int) -> float:
    """x rounded to a reduced operand precision (8: bfloat16, 11: binary16)."""
    return float(lib().orc_round_operand(float(x), int(bits)))


def decoder_gbuffer(params, latents, mats: Sequence, g, operand_bits: int = 0):
    """Decoder forward: raw outputs y [4,n] and composed rgb [3,n].
    operand_bits > 0: every matrix product's operands (weights and per-pixel
    inputs, not the latent term) rounded to that precision, sums exact."""
    h = _GBufHolder(g)
    n = h.s.n
    P = _d(params)
    Z = _d(latents).reshape(-1)
    y = np.zeros((4, n))
    rgb = np.zeros((3, n))
    lib().orc_decoder_batch_q(_ptr(P), _ptr(Z), materials(mats), len(mats), h.ref,
                              int(operand_bits), _ptr(y), _ptr(rgb))
    return y, rgb


def paper_param_count() -> int:
    return int(lib().orc_paper_param_count())


def paper_features(u: float, v: float, r: float, wx: int, wy: int, raw: bool = False) -> np.ndarray:
    """One-blob footprint encoding of the paper-size decoder (24 channels);
    raw: the unencoded inputs p_u, p_v, tau in channels 0, 8, 16."""
    f = np.zeros(24)
    (lib().orc_paper_features_raw if raw else lib().orc_paper_features)(u, v, r, wx, wy, _ptr(f))
    return f


def paper_decoder_gbuffer(params, latents, mats: Sequence, g, raw: bool = False,
                          fused: bool = True, operand_bits: int = 0):
    """Paper-size decoder forward: raw outputs y [4,n] and composed rgb [3,n]
    (raw: footprint inputs without the one-blob encoding; fused = False: the
    angular inputs enter the first layer, no spatial fusion stage;
    operand_bits as in decoder_gbuffer)."""
    h = _GBufHolder(g)
    n = h.s.n
    P = _d(params)
    Z = _d(latents).reshape(-1)
    y = np.zeros((4, n))
    rgb = np.zeros((3, n))
    lib().orc_paper_decoder_batch_q(_ptr(P), _ptr(Z), materials(mats), len(mats), h.ref,
                                    int(raw), int(fused), int(operand_bits), _ptr(y), _ptr(rgb))
    return y, rgb


def paper_loss_grad(params, latents, mats: Sequence, g, targets, raw: bool = False,
                    fused: bool = True):
    """Loss of Eq. (11) of the paper-size decoder with per-fabric latents
    [F, 64] and its gradient: (loss, grad [27076], dlatent [F, 64])."""
    h = _GBufHolder(g)
    P = _d(params)
    Z = _d(latents).reshape(-1)
    T = np.ascontiguousarray(targets, dtype=np.float32)
    grad = np.zeros_like(P)
    dlat = np.zeros((len(mats), 64))
    loss = lib().orc_paper_loss_grad(_ptr(P), _ptr(Z), materials(mats), len(mats), h.ref, int(raw),
                                     int(fused), _ptr(T),
                                     _ptr(grad), _ptr(dlat))
    return float(loss), grad, dlat


def encoder_input(mat) -> np.ndarray:
    x = np.zeros(524)
    lib().orc_encoder_input(ctypes.byref(materials([mat])[0]), _ptr(x))
    return x


def encoder_param_count(lat: int = 32) -> int:
    return int(lib().orc_encoder_param_count(int(lat)))


def encoder(params_enc, mats: Sequence, lat: int = 32) -> np.ndarray:
    """Latents [n_mats][lat] of the encoder (lat 32: the config-size network,
    64: the paper-size network's encoder)."""
    Q = _d(params_enc)
    assert Q.size == encoder_param_count(lat)
    z = np.zeros((len(mats), lat))
    lib().orc_encoder_batch_n(_ptr(Q), materials(mats), len(mats), int(lat), _ptr(z))
    return z


def encoder_backward(params_enc, mats: Sequence, dz, lat: int = 32) -> np.ndarray:
    """Gradient of the encoder parameters from the latents' gradients dz [n_mats][lat]."""
    Q = _d(params_enc)
    D = _d(dz).reshape(-1)
    grad = np.zeros(encoder_param_count(lat))
    lib().orc_encoder_backward_batch(_ptr(Q), materials(mats), len(mats), int(lat), _ptr(D), _ptr(grad))
    return grad


def parameter_weight(p: float, p_a: float, p_b: float) -> float:
    """Blend weight of a material whose varied parameter (roughness or
    height-field scale) is p, between latents encoded at p_a and p_b
    (Sec. 5 "Interpolation"): the parameter's relative position, so that
    p = p_a gives 0, p = p_b gives 1, and p beyond p_b extrapolates."""
    return (float(p) - float(p_a)) / (float(p_b) - float(p_a))


def interpolate_latents(latents, dst: Sequence[int], a: Sequence[int], b: Sequence[int],
                        t: Sequence[float]) -> np.ndarray:
    """Latent table after the blends z[dst_k] = (1 - t_k) z[a_k] + t_k z[b_k]
    of Sec. 5 "Interpolation", in FP64.  Every blend reads the table as it
    was before any of them, then all are written."""
    before = np.array(latents, dtype=np.float64)
    after = before.copy()
    for d, i, j, w in zip(dst, a, b, t):
        w = float(w)
        after[d] = (1.0 - w) * before[i] + w * before[j]
    return after


def loss_grad(params, mats: Sequence, g, targets):
    """Loss of Eq. (11) and its gradient w.r.t. [decoder | encoder] parameters."""
    h = _GBufHolder(g)
    P = _d(params)
    T = np.ascontiguousarray(targets, dtype=np.float32)
    grad = np.zeros_like(P)
    dlat = np.zeros((len(mats), 32))
    loss = lib().orc_loss_grad(_ptr(P), materials(mats), len(mats), h.ref, _ptr(T), _ptr(grad),
                               _ptr(dlat))
    return float(loss), grad, dlat


def decoder_backward(params_dec, latents, mats: Sequence, g, dy):
    h = _GBufHolder(g)
    P = _d(params_dec)
    Z = _d(latents).reshape(-1)
    DY = _d(dy)
    gd = np.zeros(P.shape[0])
    gl = np.zeros((len(mats), 32))
    lib().orc_decoder_backward_batch(_ptr(P), _ptr(Z), materials(mats), len(mats), h.ref,
                                     _ptr(DY), _ptr(gd), _ptr(gl))
    return gd, gl


def adam_step(theta: np.ndarray, grad, m: np.ndarray, v: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    assert theta.dtype == np.float32 and m.dtype == np.float64 and v.dtype == np.float64
    G = _d(grad)
    lib().orc_adam_step(_ptr(theta), _ptr(G), _ptr(m), _ptr(v), int(theta.size), int(t),
                        lr, beta1, beta2, eps)


def batch_gen(seed: int, n: int, n_fabrics: int, r_lo: float = 1e-3, r_hi: float = 0.5,
              btdf_frac: float = 0.0):
    """Training batch recipe; btdf_frac (a float32 value) of the samples are
    lit from below (transmission)."""
    import fabric_inputs as fi
    fid = np.zeros(n, dtype=np.uint16)
    arrs = [np.zeros(n, dtype=np.float32) for _ in range(9)]
    lib().orc_batch_gen(ctypes.c_uint64(seed), n, n_fabrics, r_lo, r_hi,
                        float(np.float32(btdf_frac)), _ptr(fid), *[_ptr(a) for a in arrs])
    return fi.GBuffer(fid, *arrs)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
