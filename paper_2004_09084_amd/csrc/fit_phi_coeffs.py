"""Derives the float32 polynomial constants of the kernels' Phi(x) = -ln tanh(x/2).

Two regions (x already clipped to [Phi(30), 30]):
  x >= 1:  Phi = 2 atanh(u), u = e^-x <= 1/e, written as u * P(u^2) with
           P(w) ~ 2 atanh(sqrt w)/sqrt w  (degree 3, fitted on w in [0, e^-2]);
  x <  1:  Phi = ln 2 - ln x - ln(tanh(h)/h), h = x/2, written as
           -ln2 * log2(x) + R(x^2) with R(y) ~ ln 2 - ln(tanh(h)/h)
           (degree 3 in y = x^2, fitted on y in [0, 1]).
Fits are linear least squares on Chebyshev nodes against the analytic
functions (numpy FP64).  Prints the constants and the worst relative error
of a float32 emulation over the clip interval.
"""
import numpy as np


def cheb_nodes(lo, hi, N=4000):
    t = np.cos(np.pi * (np.arange(N) + 0.5) / N)
    return lo + (hi - lo) * (t + 1) / 2


def lsq(y, f, powers):
    A = np.stack([y ** p for p in powers], 1)
    c, *_ = np.linalg.lstsq(A, f, rcond=None)
    return c


def fit():
    # region B: P(w) = 2 atanh(u)/u, u = sqrt(w)
    w = cheb_nodes(0.0, np.exp(-2.0))
    u = np.sqrt(w)
    fB = np.where(u > 1e-8, 2.0 * np.arctanh(u) / np.where(u > 0, u, 1), 2.0)
    P = lsq(w, fB, range(4))
    # region A: R(y) = ln 2 - ln(tanh(h)/h), h = sqrt(y)/2
    y = cheb_nodes(0.0, 1.0)
    h = np.sqrt(y) / 2
    g = np.where(h > 1e-6, np.log(np.tanh(h) / np.where(h > 0, h, 1)), -h * h / 3)
    R = lsq(y, np.log(2.0) - g, range(4))
    return P, R


def phi32(x, P, R):
    f32 = np.float32
    x = x.astype(f32)
    Pf = [f32(c) for c in P]
    Rf = [f32(c) for c in R]
    u = np.exp2((x * f32(-np.log2(np.e))).astype(np.float64)).astype(f32)
    w = u * u
    p = Pf[-1]
    for c in Pf[-2::-1]:
        p = (p * w + c).astype(f32)
    big = u * p
    y = x * x
    r = Rf[-1]
    for c in Rf[-2::-1]:
        r = (r * y + c).astype(f32)
    lg = np.log2(x.astype(np.float64)).astype(f32)
    small = (f32(-np.log(2.0)) * lg + r).astype(f32)
    return np.where(x < 1, small, big)


if __name__ == "__main__":
    P, R = fit()
    print("P (u-region):", [repr(float(np.float32(c))) for c in P])
    print("R (log-region):", [repr(float(np.float32(c))) for c in R])
    xs = np.geomspace(1.8715245937680347e-13, 30.0, 1_000_000).astype(np.float32)
    ref = np.log1p(2.0 / np.expm1(xs.astype(np.float64)))
    rel = np.abs(phi32(xs, P, R) - ref) / ref
    print("max relative error of the float32 form:", rel.max())
