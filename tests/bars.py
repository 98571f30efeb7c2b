"""Parity bars of the GPU tests, each derived from the arithmetic it bounds.

u = 2^-24 is the unit roundoff of FP32 (round to nearest even). The GPU and
the oracle read the same stored exitance (the oracle emulates the FP32
storage), so their fields L_b differ only by the rounding of L = E + eps in
FP32 (one u) and, where a leaf side received several splats, by the order
of the FP32 atomic additions ((C - 1) u for C splats; the inner-node means
are taken in the same octant order on both sides and keep the relative
difference of their children).

* PDF_RTOL -- the stated bar for an FP32 pdf (1e-5 relative). The worst case
  of the arithmetic is well inside it: a row scan and the marginal scan are
  Hillis-Steele trees of depth log2 N each, so every term of the total
  passes through 2 log2 N roundings; with the rounding of L_b, the division,
  the product with the FP32 constant N^2 / (4 pi) and that constant's own
  rounding, |pdf - pdf_oracle| / pdf <= (2 log2 N + 4 + (C - 1)) u to first
  order ((2 log2 N + 4) u = 7.2e-7 at N = 16). pdf_bound(N, C) returns it,
  and the tests record the measured maxima against it.
* scan_band(N, C) -- the relative CDF margin inside which the FP32 scan may
  select the neighbouring row or column (Sec. 3.5 inverse-CDF sampling; the
  oracle's margin is the distance of its FP64 target u * total to the nearer
  boundary of the selected interval, over the total). The GPU's boundary
  value carries at most (2 log2 N + 1 + (C - 1)) u of the total, its target
  u * total as much plus one rounding: a selection can differ only when the
  margin is below (4 log2 N + 3 + 2 (C - 1)) u, about 8 FP32 ulps of the
  total at N = 16 (1.1e-6).
* DIR_TOL -- sampled directions within 2e-6 (chord, i.e. radians) of the
  oracle's FP64 decode of the same bin and in-bin offsets: the FP32 decode
  takes a few ulps in sqrt, sin and cos of angles below pi/2.
* scan_band_seq(N) -- the same for the samplers with sequential prefix sums
  (binned fields, product guiding).
* edge_band(N) -- 8 ulps of x * N in bin units (x * N < N, so one ulp is at
  most N u): a direction whose FP64 encode lies that close to a bin edge may
  be encoded into the neighbouring bin by the FP32 encode of pdf_eval.
"""
import json
import math
import os

U = 2.0 ** -24
PDF_RTOL = 1e-5
DIR_TOL = 2e-6


def pdf_bound(N, C=1):
    return (2 * math.log2(N) + 4 + (C - 1)) * U


def scan_band(N, C=1):
    return (4 * math.log2(N) + 3 + 2 * (C - 1)) * U


def scan_band_seq(N):
    """Band of the binned and product samplers, whose CDFs are sequential
    FP32 prefix sums: each pdf value carries at most (log2 N^2 + 4) u (the
    field total is a pairwise block reduction), a row prefix adds (N - 1) u
    and the marginal over the row totals another (N - 1) u, and the target
    u * total one more rounding; this also covers the product sampler's cell
    level ((N/8)^2 - 1 roundings of the cell sum, one of the product, scans of
    depth 3) and its fine level."""
    return (2 * (2 * (N - 1) + 2 * math.log2(N) + 4) + 1) * U


def edge_band(N):
    return 8 * N * U


# measured maxima, written at the end of the session when WFPG_MEASURED names a file
MEASURED = {}


def record(name, value, bar=None):
    v = float(value)
    old = MEASURED.get(name)
    if old is None or v > old["max"]:
        MEASURED[name] = {"max": v, "bar": None if bar is None else float(bar)}


def dump():
    path = os.environ.get("WFPG_MEASURED")
    if path and MEASURED:
        with open(path, "w") as f:
            json.dump(MEASURED, f, indent=1, sort_keys=True)
