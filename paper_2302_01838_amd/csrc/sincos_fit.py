"""Derivation of the polynomial coefficients of vmap_sincosf (vmap_math.h).

On |r| <= pi/4 (with a 0.05 % margin for the rounding of the range reduction) it fits
  sin r = r + r^3 (a0 + a1 r^2 + a2 r^4),   cos r = 1 + r^2 (b0 + b1 r^2 + b2 r^4)
by iteratively reweighted least squares on Chebyshev nodes, which converges toward the minimax
fit of the absolute error, and prints the coefficients rounded to FP32 with the fit error.

    python paper_2302_01838_amd/csrc/sincos_fit.py
"""
import numpy as np


def fit(kind, ncoef=3, iters=60):
    R = np.pi / 4 * 1.0005
    x = np.cos(np.linspace(0.0, np.pi, 4001)) * R
    r2 = x * x
    if kind == "sin":
        target = (np.sin(x) - x) / np.where(x == 0, 1.0, x ** 3)
        scale = np.abs(x) ** 3
    else:
        target = (np.cos(x) - 1.0) / np.where(x == 0, 1.0, r2)
        scale = r2
    A = np.stack([r2 ** i for i in range(ncoef)], 1)
    w = np.ones_like(x)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * (w * scale)[:, None], target * w * scale, rcond=None)
        err = np.abs(A @ c - target) * scale
        w = w * np.sqrt(err / err.max() + 1e-3)
        w /= w.max()
    return [float(np.float32(v)) for v in c], float(err.max())


if __name__ == "__main__":
    for kind in ("sin", "cos"):
        coef, err = fit(kind)
        print(kind, " ".join(float(v).hex() for v in coef), [f"{v:.9g}" for v in coef],
              f"fit error {err:.2e}")
