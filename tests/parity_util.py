"""Comparison helpers of the parity tests (no shading arithmetic here).

Tolerances, derived from the arithmetic:
* HDR radiance and IBL tables: relative 1e-3 (the stated bar for linear HDR of
  the float32 path) plus an absolute floor of 1e-6 times the image's largest
  value, for values that are themselves zero up to rounding.
* AO: absolute 1e-4.  AO = 1 - (sum of N smoothstep terms) / N, each term a
  handful of float32 operations on O(1) values (<= 1e-6 each).
* 8-bit output: +-1 code (the stated bar), on at least 99.9 % of pixels.
Where the oracle reports an interval [lo, hi] (float decisions within their
float32 rounding band), every GPU value must lie in [lo - tol(lo), hi + tol(hi)];
each check logs its worst excursion and the share of intervals wider than the
tolerance.
"""
from __future__ import annotations

import sys

import numpy as np

HDR_RTOL = 1e-3
HDR_ATOL_REL_MAX = 1e-6
AO_ATOL = 1e-4


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def within_interval(g, lo, hi, rtol=HDR_RTOL, atol=None):
    """Boolean mask of values of ``g`` inside the tolerance band of [lo, hi]."""
    g = np.asarray(g, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    if atol is None:
        atol = HDR_ATOL_REL_MAX * max(1e-30, float(np.abs(hi).max()))
    return (g >= lo - (rtol * np.abs(lo) + atol)) & (g <= hi + (rtol * np.abs(hi) + atol))


def interval_report(g, lo, hi, rtol=HDR_RTOL, atol=None):
    """(worst, wide): the largest distance of ``g`` outside [lo, hi] in units of
    the tolerance (< 1 passes; 0 inside the interval) and the share of values
    whose interval is itself wider than the tolerance."""
    g = np.asarray(g, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    if atol is None:
        atol = HDR_ATOL_REL_MAX * max(1e-30, float(np.abs(hi).max()))
    tol_lo = rtol * np.abs(lo) + atol
    tol_hi = rtol * np.abs(hi) + atol
    out = np.maximum(np.maximum(lo - g, 0.0) / tol_lo, np.maximum(g - hi, 0.0) / tol_hi)
    wide = (hi - lo) > tol_lo
    return float(out.max()) if out.size else 0.0, float(wide.mean()) if wide.size else 0.0


def assert_interval(name, g, lo, hi, rtol=HDR_RTOL, atol=None, min_frac=1.0):
    """Every value of ``g`` within the tolerance band of [lo, hi] (``min_frac``
    of them when given); logs the worst excursion (in tolerances) and the
    share of over-wide oracle intervals.  Returns the fraction within."""
    ok = within_interval(g, lo, hi, rtol, atol)
    frac = ok.mean()
    worst, wide = interval_report(g, lo, hi, rtol, atol)
    log(f"  {name}: worst {worst:.3f} of the tolerance outside the interval; "
        f"intervals wider than the tolerance {100 * wide:.4f}%")
    if frac < min_frac:
        bad = np.argwhere(~ok)[:5]
        g64 = np.asarray(g, np.float64)
        detail = [(tuple(int(v) for v in b), float(g64[tuple(b)]), float(np.asarray(lo)[tuple(b)]),
                   float(np.asarray(hi)[tuple(b)])) for b in bad]
        raise AssertionError(f"{name}: {100 * (1 - frac):.4f}% outside tolerance; first: {detail}")
    return frac


def assert_ldr(name, g, lo, hi, min_frac=0.999):
    """8-bit parity: within [lo - 1, hi + 1] on at least ``min_frac`` of the
    pixels; returns (fraction within, fraction exactly inside [lo, hi])."""
    g = np.asarray(g, np.int32)[..., :3]
    lo = np.asarray(lo, np.int32)[..., :3]
    hi = np.asarray(hi, np.int32)[..., :3]
    ok = ((g >= lo - 1) & (g <= hi + 1)).all(-1)
    exact = ((g >= lo) & (g <= hi)).all(-1)
    frac = ok.mean()
    if frac < min_frac:
        raise AssertionError(f"{name}: only {100 * frac:.3f}% of pixels within +-1 LSB")
    return frac, exact.mean()
