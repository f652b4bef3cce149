"""Generates the coefficients of the FP32 complementary error function used
by the real-space pair kernel.

Form: erfc(x) = exp(-x^2) * t * P(t),  t = 1 / (1 + p x),  P of degree 7.
P and p are fitted here, in FP64, to the scaled function erfc(x) exp(x^2)
(scipy.special.erfcx) on x in [0, 6] by iteratively reweighted least squares
on the relative error, with p chosen by a scan. The relative error of the
fitted form is about 4e-8 over [0, 6], below FP32 resolution.

Run: python gen_erfc_fit.py  (prints the C constants pasted into pair.hip)
"""
import numpy as np
from scipy.special import erfcx

X = 6.0
DEG = 7


def fit(p, iters=40):
    tmin = 1.0 / (1.0 + p * X)
    th = np.cos(np.linspace(0, np.pi, 6000)) * 0.5 * (1 - tmin) + 0.5 * (1 + tmin)
    x = (1.0 / th - 1.0) / p
    f = erfcx(x) / th
    w = np.ones_like(th)
    V = np.vander(th, DEG + 1, increasing=True)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(V * (w / f)[:, None], w, rcond=None)
        rel = (V @ c) / f - 1.0
        w = w * (np.abs(rel) / np.abs(rel).max() + 1e-3) ** 0.5
    xs = np.linspace(0.0, X, 400001)
    ts = 1.0 / (1.0 + p * xs)
    err = np.abs((np.vander(ts, DEG + 1, increasing=True) @ c) * ts / erfcx(xs) - 1.0).max()
    return c, err


def main():
    ps = np.linspace(0.28, 0.38, 41)
    res = [fit(p, 20)[1] for p in ps]
    p = float(ps[int(np.argmin(res))])
    c, err = fit(p)
    print(f"// p = {p!r}, max relative error over [0, {X}] = {err:.3e}")
    c32 = c.astype(np.float32)
    xs = np.linspace(0.0, X, 400001)
    ts = 1.0 / (1.0 + np.float32(p) * xs)
    e32 = np.abs((np.vander(ts, DEG + 1, increasing=True) @ c32.astype(np.float64)) * ts / erfcx(xs) - 1).max()
    print(f"// with the coefficients rounded to FP32: {e32:.3e}")
    print(f"#define ERFC_P {float(np.float32(p))!r}f")
    for k, ck in enumerate(c32):
        print(f"#define ERFC_C{k} {float(ck)!r}f")


if __name__ == "__main__":
    main()
