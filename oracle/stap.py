"""CPU FP64 oracle of the post-Doppler STAP hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this module; the GPU library never does.  It shares
no code, table or constant with the HIP kernels.

It is written to be checked by eye: complex128 NumPy/SciPy, one processing
step per function, in the order the steps are defined, with no blocking,
fusion or reordering.  Library primitives (``numpy.fft.fft``, ``@``,
``numpy.linalg.solve``, ``numpy.linalg.cholesky``) serve as single steps.

Source.  Shirako et al., "Automatic Parallelization of Python Programs for
Distributed Heterogeneous Computing" (arXiv 2203.06233), Sec. 4.2 and the
figure "Kernel from the STAP Signal Processing Application": the STAP kernel is
an explicit loop (statement S), an ``fft`` along one axis (statement T; Table 2
row fft_{2D,axis=1}: every row of the operand is transformed) and a
2-D x 2-D array multiply (statement U; Table 2 row dot_{2D,2D}), all fused into
one parallel loop over independent units.  Sec. 5.3 states the problem as
datacubes of pulses x channels x samples per pulse and cites Melvin (2014) for
STAP.  The figure's code is not reproduced in the paper's text, so the steps
below follow textbook post-Doppler STAP with time-staggered DOF.  Readings the
paper leaves open, each chosen once and used on both sides:

* Subarrays (optional): the C elements are summed in contiguous groups of
  n_sub into C / n_sub channels before the Doppler step (the reading used
  for the paper's 1000-channel cube, Sec. 5.3).
* Doppler: T taps; tap t applies a symmetric Hann window of length
  L = P - T + 1 placed at pulses t .. t+L-1, then a length-P DFT with kernel
  exp(-j 2 pi k p / P), unnormalised, bins in natural order; DOF index
  d = t*C + c.
* Tap phase reference: absolute pulse index in the DFT kernel (default), or
  each tap referenced to its own first pulse (relative), in which case an
  on-bin target at bin k carries the temporal phase exp(j 2 pi k t / P) in tap
  t and the steering set is given per bin.
* Training: B contiguous blocks of N = R/B range cells; block b's covariance
  is the mean outer product of its own snapshots (cell under test included),
  or, as in standard STAP practice, of the N nearest cells outside the block
  and G guard cells on each side (cell under test excluded).
* Loading: delta = eps * Re tr(R_hat) / D added to the diagonal.
* Weights: adaptive matched filter, w = R_L^-1 v / sqrt(v^H R_L^-1 v).
* Output: y = w^H x per cell, power |y|^2.

Every function below is pinned by tests against brute force, closed forms,
invariants and library routines (see tests/test_oracle_pins.py).
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np


def hann(L: int) -> np.ndarray:
    """Symmetric Hann window h[n] = 1/2 - 1/2 cos(2 pi n / (L-1)), n = 0..L-1."""
    n = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / (L - 1))


def subarray(cube: np.ndarray, n_sub: int) -> np.ndarray:
    """Subarray channels: x'[c'][p][r] = sum_{e < n_sub} x[c' n_sub + e][p][r].

    The paper's datacube has 1000 channels (Sec. 5.3); full element-space
    DOF at that size is far beyond a per-(bin, block) solve, so the elements
    are first summed in contiguous groups of n_sub (uniform subarrays, the
    usual reduced-dimension front end), giving C / n_sub channels that the
    Doppler step then treats as its channels.  n_sub = 1 is the identity.
    """
    C, P, R = cube.shape
    if C % n_sub:
        raise ValueError("channels must be a multiple of the subarray size")
    x = cube.astype(np.complex128)
    out = np.zeros((C // n_sub, P, R), np.complex128)
    for e in range(n_sub):
        out += x[e::n_sub]
    return out


def tap_windows(P: int, T: int) -> np.ndarray:
    """Windows of the T time-staggered taps, ``[T][P]``: h_t[p] = h[p - t]."""
    L = P - T + 1
    h = hann(L)
    W = np.zeros((T, P), np.float64)
    for t in range(T):
        W[t, t:t + L] = h
    return W


def doppler(cube: np.ndarray, T: int, relative: bool = False) -> np.ndarray:
    """Doppler filtering (statements S and T): snapshots ``X[k][t*C + c][r]``.

    Absolute phase reference (default):
        X[k][t*C+c][r] = sum_p h_t[p] x[c][p][r] exp(-j 2 pi k p / P).
    Relative phase reference (``relative``): every tap's DFT is referenced to
    its own first pulse, i.e. the length-P DFT of the windowed sub-CPI
    h[n] x[c][t+n][r], n = 0..L-1, zero-padded:
        X[k][t*C+c][r] = sum_p h_t[p] x[c][p][r] exp(-j 2 pi k (p - t) / P).
    """
    C, P, R = cube.shape
    x = cube.astype(np.complex128)
    X = np.empty((P, T * C, R), np.complex128)
    if relative:
        L = P - T + 1
        h = hann(L)
        for t in range(T):
            sub = np.zeros((C, P, R), np.complex128)
            sub[:, :L, :] = x[:, t:t + L, :] * h[None, :, None]
            X[:, t * C:(t + 1) * C, :] = np.fft.fft(sub, axis=1).transpose(1, 0, 2)
        return X
    W = tap_windows(P, T)
    for t in range(T):
        Xt = np.fft.fft(x * W[t][None, :, None], axis=1)  # [C][k][R]
        X[:, t * C:(t + 1) * C, :] = Xt.transpose(1, 0, 2)
    return X


def training_cells(n_range: int, n_block: int, b: int, guard: int) -> np.ndarray:
    """Range cells that train block b when the cells under test are excluded.

    Block b holds cells [bN, bN + N).  Those cells and ``guard`` cells on each
    side are excluded; the N training cells are the nearest remaining ones,
    half (rounded down) on the left and the rest on the right, moved to the
    other side where a side runs out of cells at the edge of the cube.  Needs
    R >= 2N + 2G so that every block has N cells to train on.
    """
    R, N, G = n_range, n_range // n_block, guard
    lo, hi = b * N - G, b * N + N + G          # excluded cells [lo, hi)
    left_avail, right_avail = max(0, lo), max(0, R - hi)
    if left_avail + right_avail < N:
        raise ValueError("not enough range cells outside the guard region")
    n_right = min(N - min(N // 2, left_avail), right_avail)
    n_left = N - n_right
    return np.concatenate([np.arange(lo - n_left, lo), np.arange(hi, hi + n_right)])


def covariance(X: np.ndarray, n_block: int, guard: Optional[int] = None) -> np.ndarray:
    """Sample covariance per (Doppler bin, training block) (statement U).

    R_hat[k][b] = (1/N) sum_{r in Omega_b} X[k][:, r] X[k][:, r]^H, with
    Omega_b the block's own N cells (``guard`` None: the cell under test is
    part of its training set) or, with ``guard`` = G >= 0, the N cells of
    ``training_cells`` (the block and G guard cells on each side excluded).
    """
    P, D, R = X.shape
    N = R // n_block
    if guard is None:
        Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)  # [k][b][d][n]
    else:
        Xb = np.stack([X[:, :, training_cells(R, n_block, b, guard)] for b in range(n_block)], axis=1)
    return (Xb @ np.conj(Xb).swapaxes(-1, -2)) / N


def loading(R_hat: np.ndarray, eps: float):
    """Diagonal loading: delta = eps * Re tr(R_hat) / D; R_L = R_hat + delta I."""
    D = R_hat.shape[-1]
    tr = np.real(np.trace(R_hat, axis1=-2, axis2=-1))
    delta = eps * tr / D
    R_L = R_hat + delta[..., None, None] * np.eye(D)
    return delta, R_L


def cholesky_info(A: np.ndarray):
    """Lower Cholesky factor of one Hermitian matrix, LAPACK-style status.

    Returns (L, info): info = 0 on success, else j >= 1, the 1-based index of
    the first pivot that is not positive (L is then undefined).  Textbook
    column-by-column (left-looking) factorisation: L[j][j] = sqrt(A[j][j] -
    sum_k |L[j][k]|^2); L[i][j] = (A[i][j] - sum_k L[i][k] conj(L[j][k])) /
    L[j][j].  Only used where a status is needed; the batched path below uses
    numpy.linalg.cholesky for speed and falls back here on failure.
    """
    D = A.shape[0]
    L = np.zeros_like(A, dtype=np.complex128)
    for j in range(D):
        piv = np.real(A[j, j]) - np.sum(np.abs(L[j, :j]) ** 2)
        if not (piv > 0.0) or not np.isfinite(piv):
            return L, j + 1
        L[j, j] = np.sqrt(piv)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ np.conj(L[j, :j])) / L[j, j]
    return L, 0


def solve_weights(R_L: np.ndarray, V: np.ndarray):
    """Adaptive matched-filter weights for every system and steering vector.

    R_L ``[..][D][D]`` loaded covariances, V ``[S][D]`` steering set shared
    by every system, or ``[P][S][D]`` with one set per Doppler bin (then R_L is
    ``[P][B][D][D]`` and bin k's systems use V[k]).
    u_s = R_L^-1 v_s; gamma_s = Re(v_s^H u_s); w_s = u_s / sqrt(gamma_s).
    The weights are defined by the solve, so a general dense solve
    (``numpy.linalg.solve``) computes them; the Cholesky factorisation is used
    only for the status: info = 0 where R_L = L L^H exists, else the 1-based
    index of the first pivot that is not positive, and those systems get zero
    weights.  Returns (W ``[..][S][D]``, gamma ``[..][S]``, info ``[..]``).
    """
    if V.ndim == 3:
        parts = [solve_weights(R_L[k], V[k]) for k in range(V.shape[0])]
        return tuple(np.stack([p[i] for p in parts]) for i in range(3))
    batch = R_L.shape[:-2]
    D = R_L.shape[-1]
    S = V.shape[0]
    flat = R_L.reshape(-1, D, D)
    info = np.zeros(flat.shape[0], np.int32)
    try:
        np.linalg.cholesky(flat)
    except np.linalg.LinAlgError:
        for i in range(flat.shape[0]):
            info[i] = cholesky_info(flat[i])[1]
    ok = info == 0
    W = np.zeros((flat.shape[0], S, D), np.complex128)
    G = np.zeros((flat.shape[0], S), np.float64)
    if np.any(ok):
        Vt = V.astype(np.complex128).T                       # [D][S]
        u = np.linalg.solve(flat[ok], Vt[None])              # [..][D][S]
        gamma = np.real(np.sum(np.conj(Vt)[None] * u, axis=1))  # [..][S]
        W[ok] = (u / np.sqrt(gamma)[:, None, :]).swapaxes(1, 2)
        G[ok] = gamma
    return W.reshape(*batch, S, D), G.reshape(*batch, S), info.reshape(batch)


def inner_products(W: np.ndarray, X: np.ndarray, n_block: int):
    """Output y[k][s][r] = w_{k, b(r), s}^H X[k][:, r]; power |y|^2.

    W ``[P][B][S][D]``, X ``[P][D][R]``.  Returns (y, power) ``[P][S][R]``.
    """
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)  # [k][b][d][n]
    Yb = np.conj(W) @ Xb                                     # [k][b][s][n]
    y = Yb.transpose(0, 2, 1, 3).reshape(P, W.shape[2], R)
    return y, np.abs(y) ** 2


def run(cube: np.ndarray, V: np.ndarray, T: int, n_block: int, eps: float,
        keep: bool = True, relative: bool = False, guard: Optional[int] = None,
        n_sub: int = 1) -> Dict[str, np.ndarray]:
    """The whole chain on one cube ``[C][P][R]`` with steering set ``[S][D]``
    (or ``[P][S][D]`` per bin); with ``n_sub`` > 1 the elements are first
    summed into C / n_sub subarray channels."""
    X = doppler(cube if n_sub == 1 else subarray(cube, n_sub), T, relative)
    R_hat = covariance(X, n_block, guard)
    delta, R_L = loading(R_hat, eps)
    W, gamma, info = solve_weights(R_L, V)
    y, power = inner_products(W, X, n_block)
    out = dict(W=W, gamma=gamma, info=info, delta=delta, y=y, power=power)
    if keep:
        out.update(X=X, R_hat=R_hat, R_L=R_L)
    return out


def run_block(cube_block: np.ndarray, V: np.ndarray, T: int, eps: float,
              bins: Optional[np.ndarray] = None, relative: bool = False,
              train_block: Optional[np.ndarray] = None, n_sub: int = 1) -> Dict[str, np.ndarray]:
    """The chain for ONE training block: ``cube_block`` is ``[C][P][N]``.

    Doppler filtering acts on each (channel, range cell) column alone, so the
    block's snapshots need only its own cells; ``bins`` selects Doppler bins.
    ``train_block`` (``[C][P][N]``, the cube at the block's training cells,
    e.g. ``training_cells``) trains the covariance instead of the block
    itself.  V is ``[S][D]`` or ``[P][S][D]``.  Returns arrays indexed [k][...]
    over the selected bins with B = 1.  ``n_sub`` > 1 sums the elements into
    subarray channels first.
    """
    if n_sub > 1:
        cube_block = subarray(cube_block, n_sub)
        train_block = None if train_block is None else subarray(train_block, n_sub)
    X = doppler(cube_block, T, relative)
    Xt = None if train_block is None else doppler(train_block, T, relative)
    if bins is not None:
        X = X[np.asarray(bins)]
        Xt = None if Xt is None else Xt[np.asarray(bins)]
        if V.ndim == 3:
            V = V[np.asarray(bins)]
    return run_from_snapshots(X, V, 1, eps, X_train=Xt)


def run_from_snapshots(X: np.ndarray, V: np.ndarray, n_block: int, eps: float,
                       X_train: Optional[np.ndarray] = None):
    R_hat = covariance(X if X_train is None else X_train, n_block)
    delta, R_L = loading(R_hat, eps)
    W, gamma, info = solve_weights(R_L, V)
    y, power = inner_products(W, X, n_block)
    return dict(X=X, R_hat=R_hat, R_L=R_L, delta=delta, W=W, gamma=gamma,
                info=info, y=y, power=power)
