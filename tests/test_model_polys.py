"""The analytic model's float32 sin(pi x), cos(pi x) and tan(x) polynomials
(csrc/model.hpp sincospi_quarter, tan_small): the header's coefficients are
the ones the committed fitting script derives, and their float32 evaluation
(emulated, fused multiply-adds in the header's order) stays within 2 ulp of
sin and cos on |x| <= 1/4 and within 4 ulp of tan on |x| <= 1.5, against
numpy's float64 functions.  Host-side only."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_17782_amd", "csrc")


def load_fit():
    spec = importlib.util.spec_from_file_location("fit_model_polys",
                                                  os.path.join(CSRC, "fit_model_polys.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def header_function(name):
    src = open(os.path.join(CSRC, "model.hpp")).read()
    start = src.index("inline " + ("void " if name == "sincospi_quarter" else "float ") + name)
    return src[start:src.index("\n}\n", start)]


def floats(text):
    return [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", text)]


def test_header_coefficients_are_the_fit():
    fit = load_fit()
    S, C, Q, hi, lo = fit.fit()
    sc = floats(header_function("sincospi_quarter"))
    # p = fma(s, S3, S2), p = fma(p, s, S1), fma(p, s, S0); the same for C
    assert sc[:4] == [S[3], S[2], S[1], S[0]]
    assert sc[4:8] == [C[3], C[2], C[1], C[0]]
    tn = floats(header_function("tan_small"))
    assert tn[:2] == [hi, lo]
    assert tn[2:7] == [Q[4], Q[3], Q[2], Q[1], Q[0]]


def test_float32_error_bounds():
    fit = load_fit()
    e_sin, e_cos, e_tan = fit.max_errors(*fit.fit(), n=1_000_000, seed=7)
    print("max ulp: sin %.2f cos %.2f tan %.2f" % (e_sin, e_cos, e_tan))
    assert e_sin <= 2.0 and e_cos <= 2.0
    assert e_tan <= 4.0


def test_special_values():
    fit = load_fit()
    S, C, Q, hi, lo = fit.fit()
    sn, cs = fit.eval_sincospi(np.array([0.0, 0.25, -0.25]), S, C)
    assert sn[0] == 0.0 and cs[0] == 1.0
    # sin(pi/4) = cos(pi/4) = 1/sqrt(2), correctly rounded here
    r = np.float32(np.sqrt(0.5))
    assert abs(sn[1] - r) <= np.spacing(r) and abs(cs[1] - r) <= np.spacing(r)
    assert sn[2] == -sn[1] and cs[2] == cs[1]
    t = fit.eval_tan(np.array([0.0, 1.5, -1.5, np.pi / 4]), Q, hi, lo)
    assert t[0] == 0.0 and t[2] == -t[1]
    assert abs(t[1] - np.tan(np.float32(1.5))) <= 4 * np.spacing(np.float32(t[1]))
    assert abs(t[3] - 1.0) <= 2 * np.spacing(np.float32(1.0))
