"""Planted mistakes: each plausible slip in the oracle must fail some pin.

A broken copy of the oracle module is built on the CPU (the shipped module is
never touched), one mistake at a time, and the pins of test_oracle_pins are run
against it.
"""
import types

import numpy as np
import pytest

import oracle.stap as stap_mod
import synth
from tests import test_oracle_pins as pins


def _mutant(name, fn_src):
    src = open(stap_mod.__file__).read()
    mod = types.ModuleType("oracle_mutant_" + name)
    mod.__dict__["__name__"] = mod.__name__
    exec(compile(src, stap_mod.__file__, "exec"), mod.__dict__)
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
def doppler(cube, T):
    C, P, R = cube.shape
    x = cube.astype(np.complex128)
    W = tap_windows(P, T)
    X = np.empty((P, T * C, R), np.complex128)
    for t in range(T):
        Xt = np.fft.fft(x * W[t][None, :, None], axis=1)
        X[:, t::T, :] = Xt.transpose(1, 0, 2)
    return X
""",
    "fft_sign": """
def doppler(cube, T):
    C, P, R = cube.shape
    x = cube.astype(np.complex128)
    W = tap_windows(P, T)
    X = np.empty((P, T * C, R), np.complex128)
    for t in range(T):
        Xt = P * np.fft.ifft(x * W[t][None, :, None], axis=1)
        X[:, t * C:(t + 1) * C, :] = Xt.transpose(1, 0, 2)
    return X
""",
    "covariance_conj_side": """
def covariance(X, n_block):
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)
    return (np.conj(Xb) @ Xb.swapaxes(-1, -2)) / N
""",
    "covariance_no_scale": """
def covariance(X, n_block):
    P, D, R = X.shape
    N = R // n_block
    Xb = X.reshape(P, D, n_block, N).transpose(0, 2, 1, 3)
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
