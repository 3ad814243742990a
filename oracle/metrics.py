"""Error metrics against the FP64 oracle (test infrastructure only).

* normwise relative error  ||A - A_o||_F / ||A_o||_F over a whole array;
* SINR loss per (bin, block, steering vector): 10 log10(SINR(w_o) / SINR(w))
  with SINR(w) = |w^H v|^2 / (w^H R_L,o w) and R_L,o the oracle's FP64 loaded
  covariance.  w_o maximises SINR for R_L,o, so the loss is >= 0 up to
  rounding.
"""
from __future__ import annotations

import numpy as np


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((a - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def per_system_rel_err(W: np.ndarray, W_o: np.ndarray) -> np.ndarray:
    """Normwise error of each system's weight block ``[..][S][D]``."""
    W = np.asarray(W, np.complex128)
    W_o = np.asarray(W_o, np.complex128)
    num = np.sqrt(np.sum(np.abs(W - W_o) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(W_o) ** 2, axis=(-2, -1)))
    return num / np.where(den > 0, den, 1.0)


def sinr(W: np.ndarray, V: np.ndarray, R_L: np.ndarray) -> np.ndarray:
    """SINR of weights ``[..][S][D]`` for steering ``[S][D]`` under ``[..][D][D]``."""
    W = np.asarray(W, np.complex128)
    V = np.asarray(V, np.complex128)
    gain = np.abs(np.sum(np.conj(W) * V, axis=-1)) ** 2
    RW = np.einsum("...ij,...sj->...si", R_L, W)
    den = np.real(np.sum(np.conj(W) * RW, axis=-1))
    return gain / den


def sinr_loss_db(W: np.ndarray, W_o: np.ndarray, V: np.ndarray, R_L_o: np.ndarray) -> np.ndarray:
    return 10.0 * np.log10(sinr(W_o, V, R_L_o) / sinr(W, V, R_L_o))
