"""Comparison of a GPU result with the oracle's, per residual and per block.

Two measures, both required: the relative 2-norm error ||z - z_o|| / ||z_o||
(the per-precision tolerance of the method) and the element-wise relative
error max_i |z_i - z_o,i| / max_i |z_o,i|, which a few wrong entries (one
wrong pencil or tile) cannot hide behind the norm of a large block.
"""
import numpy as np

# per-precision tolerance on ||z - z_o||_2 / ||z_o||_2
# (FP8 split: a rounding emulation of the mode products puts it at 2.5-3e-3)
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2, "bf16_split": 1e-4, "f16": 5e-3, "f16_split": 1e-4,
       "fp8_split": 1e-2}
# per-precision tolerance on max_i |z_i - z_o,i| / max_i |z_o,i|
TOL_MAX = dict(TOL)


def errors(z, zo):
    """(relative 2-norm error, relative max-norm error) of z against zo."""
    z = np.asarray(z, dtype=np.float64)
    zo = np.asarray(zo, dtype=np.float64)
    d = z - zo
    return float(np.linalg.norm(d) / np.linalg.norm(zo)), float(np.max(np.abs(d)) / np.max(np.abs(zo)))


def check_close(z, zo, prec, what=""):
    """Assert z matches the oracle's zo to the precision's tolerances; returns both errors."""
    assert np.all(np.isfinite(z)), f"{what}: non-finite entries"
    e2, emax = errors(z, zo)
    assert e2 < TOL[prec] and emax < TOL_MAX[prec], (
        f"{what}: rel 2-norm err {e2:.3e} (tol {TOL[prec]:.0e}), rel max err {emax:.3e} (tol {TOL_MAX[prec]:.0e})")
    return e2, emax


def check_blocks(z, zo, offsets, prec, what=""):
    """check_close on every block [offsets[k], offsets[k+1]) of a block vector; returns the worst errors."""
    worst = (0.0, 0.0)
    for k, (a, b) in enumerate(zip(offsets[:-1], offsets[1:])):
        e = check_close(z[a:b], zo[a:b], prec, f"{what} block {k}")
        worst = (max(worst[0], e[0]), max(worst[1], e[1]))
    return worst
