"""CPU oracle of cell-averaging CFAR detection on the AMF power map.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this module; the GPU library never does.  It
shares no code, table or constant with the HIP kernels.

Detection is not part of the paper's STAP kernel (Sec. 4.2); it is the step
that consumes its output.  This is the textbook cell-averaging constant
false-alarm-rate detector (Finn and Johnson 1968; e.g. Richards,
Fundamentals of Radar Signal Processing, ch. 7) applied along range to every
(Doppler bin, steering vector) row of the power map ``power[P][S][R]``:

* reference window of cell r: n_ref cells on each side, beyond n_guard guard
  cells, i.e. offsets -(n_guard + n_ref) .. -(n_guard + 1) and
  n_guard + 1 .. n_guard + n_ref; cells outside [0, R) are left out and the
  estimate averages the n_used cells that exist;
* noise estimate  z = (1 / n_used) * sum of the reference cells;
* detection       power[r] > alpha * z.

For exponentially distributed noise power (the AMF output of noise alone)
and n_used = N reference cells, alpha = N (Pfa^(-1/N) - 1) gives the false-
alarm probability Pfa (``alpha_for_pfa``).

The detection is an integer decision taken from floating-point values, so it
is defined here exactly as the kernel takes it: the reference cells are
summed in FP64 one at a time in increasing offset order (left window, then
right window; a missing cell adds 0), and the test is
    (double) power[r] * n_used  >  alpha * sum
with alpha a double.  Both sides therefore take the same decision bit for
bit.
"""
from __future__ import annotations

import numpy as np


def alpha_for_pfa(n_ref_total: int, pfa: float) -> float:
    """CA-CFAR threshold factor for N reference cells of exponential noise."""
    N = n_ref_total
    return N * (pfa ** (-1.0 / N) - 1.0)


def offsets(n_ref: int, n_guard: int) -> np.ndarray:
    """Reference-cell offsets in summation order: left window, then right."""
    left = np.arange(-(n_guard + n_ref), -n_guard)
    right = np.arange(n_guard + 1, n_guard + n_ref + 1)
    return np.concatenate([left, right])


def ca_cfar(power: np.ndarray, n_ref: int, n_guard: int, alpha: float):
    """Detection mask and noise estimate of every cell of ``power[..][R]``.

    Returns (detect bool [..][R], noise float64 [..][R], n_used int [R])."""
    p = np.asarray(power).astype(np.float64)
    R = p.shape[-1]
    r = np.arange(R)
    acc = np.zeros(p.shape, np.float64)
    n_used = np.zeros(R, np.int64)
    for o in offsets(n_ref, n_guard):
        idx = r + o
        ok = (idx >= 0) & (idx < R)
        acc = acc + np.where(ok, p[..., np.clip(idx, 0, R - 1)], 0.0)
        n_used += ok
    detect = p * n_used.astype(np.float64) > float(alpha) * acc
    with np.errstate(invalid="ignore", divide="ignore"):
        noise = acc / n_used
    return detect, noise, n_used
