"""Planted mistakes: each plausible slip in the oracle must fail some pin.

A broken copy of the oracle module is built on the CPU (the shipped module is
never touched), one mistake at a time, and the pins of test_oracle_pins are run
against it.
"""
import types

import numpy as np
import pytest

import oracle.metrics as metrics_mod
import oracle.stap as stap_mod
import synth
from tests import test_oracle_pins as pins


def _mutant(name, fn_src, base=stap_mod):
    src = open(base.__file__).read()
    mod = types.ModuleType("oracle_mutant_" + name)
    mod.__dict__["__name__"] = mod.__name__
    exec(compile(src, base.__file__, "exec"), mod.__dict__)
    exec(fn_src, mod.__dict__)
    return mod


MUTANTS = {
    "periodic_hann": """
def hann(L):
    n = np.arange(L, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * n / L)
""",
    "window_shift_reversed": """
def tap_windows(P, T):
    L = P - T + 1
    h = hann(L)
    W = np.zeros((T, P))
    for t in range(T):
        W[t, T - 1 - t:T - 1 - t + L] = h
    return W
""",
    "dof_order_c_major": """
def doppler(cube, T, relative=False):
    C, P, R = cube.shape
    x = cube.astype(np.complex128)
    W = tap_windows(P, T)
    X = np.empty((P, T * C, R), np.complex128)
    for t in range(T):
        Xt = np.fft.fft(x * W[t][None, :, None], axis=1)
        if relative:
            Xt = Xt * np.exp(2j * np.pi * np.arange(P) * t / P)[None, :, None]
        X[:, t::T, :] = Xt.transpose(1, 0, 2)
    return X
""",
    "fft_sign": """
def doppler(cube, T, relative=False):
    C, P, R = cube.shape
    x = cube.astype(np.complex128)
    W = tap_windows(P, T)
    X = np.empty((P, T * C, R), np.complex128)
    for t in range(T):
        Xt = P * np.fft.ifft(x * W[t][None, :, None], axis=1)
        if relative:
            Xt = Xt * np.exp(-2j * np.pi * np.arange(P) * t / P)[None, :, None]
        X[:, t * C:(t + 1) * C, :] = Xt.transpose(1, 0, 2)
    return X
""",
    "covariance_conj_side": """
def covariance(X, n_block, guard=None):
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)
    if guard is not None:
        Xb = np.stack([X[:, :, training_cells(R, n_block, b, guard)] for b in range(n_block)], axis=1)
    return (np.conj(Xb) @ Xb.swapaxes(-1, -2)) / N
""",
    "covariance_no_scale": """
def covariance(X, n_block, guard=None):
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)
    if guard is not None:
        Xb = np.stack([X[:, :, training_cells(R, n_block, b, guard)] for b in range(n_block)], axis=1)
    return Xb @ np.conj(Xb).swapaxes(-1, -2)
""",
    "loading_no_div_D": """
def loading(R_hat, eps):
    D = R_hat.shape[-1]
    delta = eps * np.real(np.trace(R_hat, axis1=-2, axis2=-1))
    return delta, R_hat + delta[..., None, None] * np.eye(D)
""",
    "weights_norm_gamma": """
_orig_solve = solve_weights
def solve_weights(R_L, V):
    W, G, info = _orig_solve(R_L, V)
    return W / np.sqrt(np.where(G > 0, G, 1.0))[..., None], G, info
""",
    "inner_no_conj": """
def inner_products(W, X, n_block):
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)
    Yb = W @ Xb
    y = Yb.transpose(0, 2, 1, 3).reshape(P, W.shape[2], R)
    return y, np.abs(y) ** 2
""",
    "info_zero_based": """
_orig_ci = cholesky_info
def cholesky_info(A):
    L, info = _orig_ci(A)
    return L, max(info - 1, 0) if info else 0
""",
    "relative_phase_wrong_shift": """
_orig_dop = doppler
def doppler(cube, T, relative=False):
    X = _orig_dop(cube, T, False)
    if relative:
        P = X.shape[0]
        C = X.shape[1] // T
        t = np.repeat(np.arange(T), C)
        X = X * np.exp(-2j * np.pi * np.outer(np.arange(P), t) / P)[:, :, None]
    return X
""",
    "training_ignores_guard": """
_orig_tc = training_cells
def training_cells(n_range, n_block, b, guard):
    return _orig_tc(n_range, n_block, b, 0)
""",
    "training_keeps_cell_under_test": """
def training_cells(n_range, n_block, b, guard):
    N = n_range // n_block
    return np.arange(b * N, b * N + N)
""",
    "per_bin_steering_first_bin_only": """
_orig_sw = solve_weights
def solve_weights(R_L, V):
    if V.ndim == 3:
        V = V[0]
    return _orig_sw(R_L, V)
""",
    "subarray_interleaved": """
def subarray(cube, n_sub):
    C, P, R = cube.shape
    if C % n_sub:
        raise ValueError("channels must be a multiple of the subarray size")
    x = cube.astype(np.complex128)
    m = C // n_sub
    return np.stack([x[c::m].sum(axis=0) for c in range(m)])
""",
    "subarray_mean": """
def subarray(cube, n_sub):
    C, P, R = cube.shape
    if C % n_sub:
        raise ValueError("channels must be a multiple of the subarray size")
    x = cube.astype(np.complex128)
    return x.reshape(C // n_sub, n_sub, P, R).mean(axis=1)
""",
    "pivot_test_in_fp32": """
def cholesky_info(A):
    D = A.shape[0]
    L = np.zeros_like(A, dtype=np.complex128)
    for j in range(D):
        piv = np.float32(np.real(A[j, j]))
        for k in range(j):
            piv = np.float32(float(piv) - float(np.abs(L[j, k]) ** 2))
        if not (piv > 0.0) or not np.isfinite(piv):
            return L, j + 1
        L[j, j] = np.sqrt(float(piv))
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ np.conj(L[j, :j])) / L[j, j]
    return L, 0
""",
}


@pytest.fixture(scope="module")
def cube_v():
    wl = synth.SMALL
    return wl, synth.make_cube(wl), synth.steering(wl)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mistake_is_caught(name, cube_v):
    mod = _mutant(name, MUTANTS[name])
    wl, cube, V = cube_v
    failures = []
    for chk in pins.CHECKS:
        try:
            chk(mod)
        except AssertionError:
            failures.append(chk.__name__)
    res = (wl, cube, V, mod.run(cube, V, wl.tdof, wl.n_block, wl.load_eps))
    for chk in pins.CHAIN_CHECKS:
        try:
            chk(mod, res=res)
        except (AssertionError, np.linalg.LinAlgError):
            failures.append(chk.__name__)
    assert failures, f"mutant {name} passed every pin"


# Mistakes in the error metrics (oracle/metrics.py), each caught by the
# hand-computed metric pins.
METRIC_MUTANTS = {
    "rel_err_divides_by_result": """
def rel_err(a, ref):
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.linalg.norm(a.ravel())
    num = np.linalg.norm((a - ref).ravel())
    return float(num / den) if den > 0 else float(num)
""",
    "rel_err_no_sqrt": """
def rel_err(a, ref):
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.sum(np.abs(ref) ** 2)
    num = np.sum(np.abs(a - ref) ** 2)
    return float(num / den) if den > 0 else float(num)
""",
    "per_system_pools_systems": """
def per_system_rel_err(W, W_o):
    W = np.asarray(W, np.complex128)
    W_o = np.asarray(W_o, np.complex128)
    num = np.sqrt(np.sum(np.abs(W - W_o) ** 2, axis=(-2, -1)))
    den = np.sqrt(np.sum(np.abs(W_o) ** 2))
    return num / den
""",
    "sinr_gain_not_squared": """
def sinr(W, V, R_L):
    W = np.asarray(W, np.complex128)
    V = np.asarray(V, np.complex128)
    gain = np.abs(np.sum(np.conj(W) * V, axis=-1))
    RW = np.einsum("...ij,...sj->...si", R_L, W)
    den = np.real(np.sum(np.conj(W) * RW, axis=-1))
    return gain / den
""",
    "sinr_transposed_covariance": """
def sinr(W, V, R_L):
    W = np.asarray(W, np.complex128)
    V = np.asarray(V, np.complex128)
    gain = np.abs(np.sum(np.conj(W) * V, axis=-1)) ** 2
    RW = np.einsum("...ji,...sj->...si", R_L, W)
    den = np.real(np.sum(W * RW, axis=-1))
    return gain / den
""",
    "sinr_loss_inverted": """
def sinr_loss_db(W, W_o, V, R_L_o):
    return 10.0 * np.log10(sinr(W, V, R_L_o) / sinr(W_o, V, R_L_o))
""",
    "sinr_loss_natural_log": """
def sinr_loss_db(W, W_o, V, R_L_o):
    return 10.0 * np.log(sinr(W_o, V, R_L_o) / sinr(W, V, R_L_o))
""",
}


@pytest.mark.parametrize("name", sorted(METRIC_MUTANTS))
def test_metric_mistake_is_caught(name):
    mod = _mutant(name, METRIC_MUTANTS[name], base=metrics_mod)
    failures = []
    for chk in pins.METRIC_CHECKS:
        try:
            chk(mod)
        except AssertionError:
            failures.append(chk.__name__)
    assert failures, f"metric mutant {name} passed every pin"
