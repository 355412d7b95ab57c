"""Derives the polynomial coefficients of model.hpp's sincospi_quarter and
tan_small, and reports their float32 error.

Each function is written as a polynomial in s = x^2 over the interval the
model evaluates it on:

  sin(pi x) = x S(s),          |x| <= 1/4  (the concentric disk map's angle)
  cos(pi x) = 1 + s C(s),      |x| <= 1/4
  tan(x)    = x + x s Q(s) / ((pi/2)^2 - s),   |x| <= 1.5  (yarn slopes)

The fits are least squares on Chebyshev nodes, reweighted by the current
error at each node (Lawson's algorithm), which converges towards the
minimax polynomial; S and C are fitted in absolute error of the function,
Q in relative error.  The coefficients are then rounded to float32, and the
float32 evaluation of model.hpp (fused multiply-adds in the same order) is
emulated on a dense sample of arguments to bound the error in ulp.

    python fit_model_polys.py
"""
import numpy as np

HALF_PI_SQ = (np.pi / 2) ** 2


def lawson(f, lo, hi, deg, scale, iters=60, npts=4000):
    t = np.cos(np.pi * (np.arange(npts) + 0.5) / npts)
    s = lo + (hi - lo) * (t + 1) / 2
    y = f(s)
    V = np.vander(s, deg + 1, increasing=True)
    w = np.full(npts, 1.0 / npts)
    for _ in range(iters):
        W = np.sqrt(w) / scale(s)
        c, *_ = np.linalg.lstsq(V * W[:, None], y * W, rcond=None)
        e = np.abs(V @ c - y) / scale(s)
        w = w * e
        w /= w.sum()
    return c


def sin_ratio(s):
    x = np.sqrt(s)
    return np.where(s > 0, np.sin(np.pi * x) / np.maximum(x, 1e-300), np.pi)


def cos_ratio(s):
    # (cos(pi x) - 1) / s = -2 sin^2(pi x / 2) / s, free of cancellation
    x = np.sqrt(s)
    return np.where(s > 0, -2 * np.sin(np.pi * x / 2) ** 2 / np.maximum(s, 1e-300),
                    -np.pi ** 2 / 2)


def tan_ratio(s):
    x = np.sqrt(s)
    series = s / 3 + 2 * s ** 2 / 15 + 17 * s ** 3 / 315 + 62 * s ** 4 / 2835
    t1 = np.where(s < 1e-4, series, np.tan(x) / np.maximum(x, 1e-300) - 1)
    return np.where(s > 0, (HALF_PI_SQ - s) * t1 / np.maximum(s, 1e-300), HALF_PI_SQ / 3)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def fit():
    """Coefficients (lowest order first), rounded to float32."""
    S = f32(lawson(sin_ratio, 0.0, 1 / 16, 3, lambda s: np.full_like(s, np.pi)))
    C = f32(lawson(cos_ratio, 0.0, 1 / 16, 3, lambda s: np.ones_like(s)))
    Q = f32(lawson(tan_ratio, 0.0, 2.25, 4, tan_ratio))
    hi = f32(HALF_PI_SQ)
    return S, C, Q, hi, f32(HALF_PI_SQ - hi)


# float32 operations emulated in float64 (a product of two float32 values is
# exact in float64, so fma rounds once there and once to float32)
def _fma(a, b, c):
    return f32(np.asarray(a) * np.asarray(b) + np.asarray(c))


def _mul(a, b):
    return f32(np.asarray(a) * np.asarray(b))


def _add(a, b):
    return f32(np.asarray(a) + np.asarray(b))


def eval_sincospi(x, S, C):
    s = _mul(x, x)
    p = _fma(s, S[3], S[2])
    p = _fma(p, s, S[1])
    p = _fma(p, s, S[0])
    c = _fma(s, C[3], C[2])
    c = _fma(c, s, C[1])
    c = _fma(c, s, C[0])
    return _mul(x, p), _fma(c, s, 1.0)


def eval_tan(x, Q, hi, lo):
    s = _mul(x, x)
    p = _fma(s, Q[4], Q[3])
    p = _fma(p, s, Q[2])
    p = _fma(p, s, Q[1])
    p = _fma(p, s, Q[0])
    d = _add(_fma(-x, x, hi), lo)
    num = _mul(_mul(x, s), p)
    r = f32(1.0 / d)                 # the hardware reciprocal, within 1 ulp
    q = _mul(num, r)
    q = _fma(_fma(-d, q, num), r, q)
    return _add(q, x)


def ulp_error(got, exact):
    u = np.spacing(np.abs(f32(exact)).astype(np.float32)).astype(np.float64)
    return np.abs(got - exact) / u


def max_errors(S, C, Q, hi, lo, n=2_000_000, seed=1):
    rng = np.random.default_rng(seed)
    x = f32(np.concatenate([rng.uniform(-0.25, 0.25, n), rng.uniform(-1e-3, 1e-3, n // 8),
                            np.linspace(-0.25, 0.25, 100001)]))
    sn, cs = eval_sincospi(x, S, C)
    e_sin = ulp_error(sn, np.sin(np.pi * x)).max()
    e_cos = ulp_error(cs, np.cos(np.pi * x)).max()
    x = f32(np.concatenate([rng.uniform(-1.5, 1.5, n), rng.uniform(1.4, 1.5, n // 4),
                            rng.uniform(-1e-3, 1e-3, n // 8), np.linspace(-1.5, 1.5, 100001)]))
    e_tan = ulp_error(eval_tan(x, Q, hi, lo), np.tan(x)).max()
    return e_sin, e_cos, e_tan


if __name__ == "__main__":
    S, C, Q, hi, lo = fit()
    for name, cs in (("S", S), ("C", C), ("Q", Q)):
        print(name, ", ".join(repr(float(np.float32(c))) + "f" for c in cs))
    print("(pi/2)^2 hi, lo", repr(float(np.float32(hi))), repr(float(np.float32(lo))))
    print("max ulp: sin %.2f cos %.2f tan %.2f" % max_errors(S, C, Q, hi, lo))
