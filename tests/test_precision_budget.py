"""Which reduced-precision formats meet the error budget of the apply (CPU).

The mode products of Algorithm 1 are emulated with operands rounded to a
storage format (round to nearest even on the significand, written from the
format definitions: BF16 8 significant bits; FP16 11 bits, exponents down to
-14 below which the quantum is fixed; FP8 E4M3 4 bits, exponents down to -6,
largest finite value 448, each tensor scaled by a power of two so that its
largest entry sits in the upper half of the range), accumulated exactly, and
compared with the oracle's FP64 apply. A hi/lo split rounds the remainder
x - hi again and forms hi*hi + lo*hi + hi*lo.

Pin of the emulation itself: its BF16, FP16 and split errors agree with the
errors the GPU kernels show on the same kind of block (BF16 ~6e-3, FP16
~7e-4, BF16 split ~1e-5, FP16 split ~3e-7). The result fixes the reading of
"FP8 where within budget": single FP8 products exceed the 2e-2 budget of the
16-bit classes; an FP8 hi/lo split meets it.
"""
import numpy as np
import pytest

from oracle.assemble import taylor_hood_velocity_1d
from oracle.fd import FDFactors, fd_apply, mode_product, unvec, vec, velocity_weights
from paper_1712_00403_amd import workloads

BUDGET_16BIT = 2e-2

FORMATS = {"bf16": dict(mbits=7), "fp16": dict(mbits=10, emin=-14, maxval=65504.0),
           "e4m3": dict(mbits=3, emin=-6, maxval=448.0)}


def round_to(x, mbits, emin=None, maxval=None):
    """Round to a binary format with `mbits` fraction bits (nearest, ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    scale = 1.0
    if maxval is not None:
        amax = float(np.max(np.abs(x)))
        if amax > 0:
            scale = 2.0 ** np.floor(np.log2(maxval / 2 / amax))
    y = x * scale
    _, E = np.frexp(y)
    e = E - 1
    if emin is not None:
        e = np.maximum(e, emin)
    q = np.ldexp(1.0, e - mbits)
    return np.rint(y / q) * q / scale


def test_rounding_matches_format_definitions():
    # BF16: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1)
    assert round_to(1 + 2.0 ** -8, 7) == 1.0
    assert round_to(1 + 3 * 2.0 ** -8, 7) == 1 + 2.0 ** -6
    # E4M3 (unscaled): 1.0625 -> 1.0 (tie to even), 1.1875 -> 1.25, subnormal quantum 2^-9
    assert round_to(1.0625, 3, emin=-6) == 1.0
    assert round_to(1.1875, 3, emin=-6) == 1.25
    assert round_to(3 * 2.0 ** -10, 3, emin=-6) == 2.0 ** -8
    # FP16 subnormals: quantum 2^-24
    assert round_to(2.0 ** -25 * 3, 10, emin=-14) == 2.0 ** -23


def emulated_apply(f, r, fmt, split=False):
    rnd = lambda x: round_to(x, **FORMATS[fmt])

    def prod(T, A, i):
        Th, Ah = rnd(T), rnd(A)
        out = mode_product(Th, Ah, i)
        if split:
            out = out + mode_product(rnd(T - Th), Ah, i) + mode_product(Th, rnd(A - Ah), i)
        return out

    T = unvec(r, f.n)
    for i in range(f.ndim):
        T = prod(T, f.U[i].T, i)
    T = T / f.eigenvalue_tensor()
    for i in range(f.ndim):
        T = prod(T, f.U[i], i)
    return vec(T)


@pytest.fixture(scope="module")
def block():
    n_el, p = (8, 9, 10), 3
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    f = FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(3, 0))
    r = workloads.residuals(5, 1, int(np.prod(f.n)))[0]
    return f, r, fd_apply(f, r)


def _err(block, fmt, split):
    f, r, z = block
    return np.linalg.norm(emulated_apply(f, r, fmt, split) - z) / np.linalg.norm(z)


@pytest.mark.parametrize("fmt,split,lo,hi", [("bf16", False, 2e-3, 1.5e-2), ("fp16", False, 2e-4, 2e-3),
                                             ("bf16", True, 3e-6, 3e-5), ("fp16", True, 5e-8, 1e-6)])
def test_emulation_reproduces_measured_kernel_errors(block, fmt, split, lo, hi):
    assert lo < _err(block, fmt, split) < hi


def test_fp8_single_exceeds_budget_split_meets_it(block):
    assert _err(block, "e4m3", False) > BUDGET_16BIT
    assert _err(block, "e4m3", True) < BUDGET_16BIT / 4
