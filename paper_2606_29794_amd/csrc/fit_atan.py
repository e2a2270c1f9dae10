"""Fit of the polynomial behind hp_atan2_pos (hp_offset.h).

atan(t) = t * P(t^2) on [0, 1], P of degree 8, chosen to minimise the largest
relative error |t P(t^2) / atan(t) - 1| by Lawson's algorithm: weighted least
squares whose weights are multiplied by the current error after every pass,
which converges to the minimax (equioscillating) fit.  Run it to print the
coefficients (highest power first, as hp_atan2_pos evaluates them) and the
relative error of the fit before and after rounding to float32.

The coefficients in hp_offset.h come from this method on a different sample
grid, so they agree with the printed ones to about 1e-6 relative; their own
error bound is checked by tests/test_hip_host.py.
"""
import numpy as np


def lawson_fit(degree: int = 8, passes: int = 400):
    t = np.sort(np.concatenate([np.cos(np.linspace(0.0, np.pi / 2, 20001)), np.linspace(0.0, 1.0, 20001)]))
    t = t[t > 0]
    f = np.arctan(t) / t
    V = np.stack([t ** (2 * k) for k in range(degree + 1)], 1)
    w = np.full(t.size, 1.0 / t.size)
    for _ in range(passes):
        sw = np.sqrt(w) / f
        c, *_ = np.linalg.lstsq(V * sw[:, None], f * sw, rcond=None)
        err = np.abs(V @ c / f - 1.0)
        w = w * err
        w /= w.sum()
    return c[::-1], float(err.max())


def rel_error(coef_high_first, n: int = 2_000_001) -> float:
    t = np.linspace(1e-6, 1.0, n)
    r = np.zeros_like(t)
    for k in coef_high_first:
        r = r * t * t + k
    return float(np.abs(r / (np.arctan(t) / t) - 1.0).max())


if __name__ == "__main__":
    c, e = lawson_fit()
    print("coefficients (t^16 ... t^0):", ", ".join(f"{x:.8g}" for x in c))
    print(f"fit error {e:.3g}; rounded to float32 {rel_error(np.float32(c).astype(np.float64)):.3g}")
