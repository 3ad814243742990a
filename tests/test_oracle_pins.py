"""Pins of the CPU FP64 oracle against what the mathematics fixes.

Nothing here compares the oracle with itself: every check is brute force on
tiny inputs, a closed form, an exact invariant, or a library routine that the
step reduces to.  The checks are plain functions so that
``test_planted_mistakes`` can run them against deliberately broken copies of
the oracle (on the CPU) and show that each plausible mistake is caught.
"""
import cmath
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import metrics, stap

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


# ---------------------------------------------------------------- Doppler (S, T)

def check_window_library_and_sums(orc=stap):
    for L in (5, 30, 62, 126, 254, 510):
        h = orc.hann(L)
        np.testing.assert_allclose(h, np.hanning(L), rtol=0, atol=1e-15)
        assert abs(h.sum() - (L - 1) / 2) < 1e-10
        assert abs((h ** 2).sum() - 3 * (L - 1) / 8) < 1e-10


def check_doppler_brute_force(orc=stap):
    C, P, R, T = 2, 8, 3, 3
    rng = _rng(1)
    x = _crandn(rng, C, P, R)
    L = P - T + 1
    h = np.hanning(L)
    X = orc.doppler(x, T)
    assert X.shape == (P, T * C, R)
    for k in range(P):
        for t in range(T):
            for c in range(C):
                for r in range(R):
                    acc = 0j
                    for p in range(t, t + L):
                        acc += h[p - t] * x[c, p, r] * cmath.exp(-2j * math.pi * k * p / P)
                    assert abs(X[k, t * C + c, r] - acc) < 1e-12


def check_doppler_tone(orc=stap):
    g = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))
    T = g["tdof"]
    for case in g["cases"]:
        P = case["n_pulse"]
        C, R = 3, 2
        for k0 in (0, 5, P // 2 + 1):
            p = np.arange(P)
            x = np.broadcast_to(np.exp(2j * np.pi * k0 * p / P)[None, :, None], (C, P, R))
            X = orc.doppler(x, T)
            np.testing.assert_allclose(X[k0], case["tone_gain"], rtol=0, atol=1e-9 * P)


def check_doppler_impulse(orc=stap):
    """x[c][p0][r] = (c+1) (r+1): X[k][t*C+c][r] = (c+1)(r+1) h[p0-t] e^{-j2pi k p0/P}."""
    C, P, R, T = 3, 16, 2, 3
    L = P - T + 1
    h = np.hanning(L)
    for p0 in (0, 1, 2, 7, P - 1):
        x = np.zeros((C, P, R), complex)
        for c in range(C):
            for r in range(R):
                x[c, p0, r] = (c + 1) * (r + 1)
        X = orc.doppler(x, T)
        for k in range(P):
            for t in range(T):
                ht = h[p0 - t] if 0 <= p0 - t < L else 0.0
                for c in range(C):
                    for r in range(R):
                        want = (c + 1) * (r + 1) * ht * cmath.exp(-2j * math.pi * k * p0 / P)
                        assert abs(X[k, t * C + c, r] - want) < 1e-12


def check_parseval(orc=stap):
    C, P, R, T = 2, 64, 5, 3
    x = _crandn(_rng(2), C, P, R)
    X = orc.doppler(x, T)
    L = P - T + 1
    h = np.hanning(L)
    for t in range(T):
        lhs = np.sum(np.abs(X[:, t * C:(t + 1) * C, :]) ** 2, axis=0)  # [C][R]
        wx = x[:, t:t + L, :] * h[None, :, None]
        rhs = P * np.sum(np.abs(wx) ** 2, axis=1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


# ---------------------------------------------------------- covariance (U), loading

def check_covariance_brute_force(orc=stap):
    P, D, R, B = 2, 3, 8, 2
    X = _crandn(_rng(3), P, D, R)
    Rh = orc.covariance(X, B)
    N = R // B
    for k in range(P):
        for b in range(B):
            for i in range(D):
                for j in range(D):
                    acc = 0j
                    for r in range(b * N, (b + 1) * N):
                        acc += X[k, i, r] * X[k, j, r].conjugate()
                    assert abs(Rh[k, b, i, j] - acc / N) < 1e-12


def check_covariance_invariants(orc=stap):
    P, D, R, B = 3, 12, 64, 4
    X = _crandn(_rng(4), P, D, R)
    Rh = orc.covariance(X, B)
    N = R // B
    assert np.array_equal(Rh, np.conj(Rh.swapaxes(-1, -2))) or \
        np.abs(Rh - np.conj(Rh.swapaxes(-1, -2))).max() < 1e-14
    ev = np.linalg.eigvalsh(Rh)
    assert ev.min() > -1e-12 * ev.max()
    tr = np.real(np.trace(Rh, axis1=-2, axis2=-1))
    want = np.sum(np.abs(X.reshape(P, D, B, N)) ** 2, axis=(1, 3)) / N
    np.testing.assert_allclose(tr, want, rtol=1e-13)
    # N = 1: rank one, equal to x x^H
    R1 = orc.covariance(X[:, :, :5], 5)
    for k in range(P):
        for b in range(5):
            x = X[k, :, b]
            np.testing.assert_allclose(R1[k, b], np.outer(x, np.conj(x)), atol=1e-14)


def check_loading_closed_form(orc=stap):
    for D in (1, 12, 48):
        eps = 1e-3
        Rh = np.diag(np.arange(1, D + 1).astype(complex))[None]
        delta, RL = orc.loading(Rh, eps)
        assert abs(delta[0] - eps * (D + 1) / 2) < 1e-15
        np.testing.assert_allclose(np.diag(RL[0]).real, np.arange(1, D + 1) + eps * (D + 1) / 2)


# ------------------------------------------------------------------ solve, weights

def _random_hpd(rng, n, D, cond=1e3):
    Q = np.linalg.qr(_crandn(rng, n, D, D))[0]
    ev = np.exp(rng.uniform(0, np.log(cond), (n, D)))
    return (Q * ev[:, None, :]) @ np.conj(Q.swapaxes(-1, -2))


def check_solve_library_and_backward(orc=stap):
    rng = _rng(5)
    D, S, n = 24, 5, 6
    A = _random_hpd(rng, n, D)
    A = 0.5 * (A + np.conj(A.swapaxes(-1, -2)))
    V = _crandn(rng, S, D)
    W, gamma, info = orc.solve_weights(A, V)
    assert np.all(info == 0)
    for i in range(n):
        u = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A[i], lower=True), V.T)
        g = np.real(np.sum(np.conj(V.T) * u, axis=0))
        np.testing.assert_allclose(gamma[i], g, rtol=1e-10)
        np.testing.assert_allclose(W[i], (u / np.sqrt(g)).T, rtol=1e-10, atol=1e-13)
        # backward error of the un-normalised solve
        ui = (W[i] * np.sqrt(gamma[i])[:, None]).T
        res = np.linalg.norm(A[i] @ ui - V.T) / (np.linalg.norm(A[i], 2) * np.linalg.norm(ui))
        assert res < 1e2 * D * np.finfo(float).eps


def check_white_snapshots(orc=stap):
    """X = sigma sqrt(N) x rows of a unitary DFT gives R_hat = sigma^2 I exactly
    (to rounding): u = v / (sigma^2 (1+eps)), w = v / (sigma sqrt(1+eps) ||v||)."""
    D, N, S, eps, sigma = 8, 16, 3, 1e-3, 1.7
    F = np.exp(-2j * np.pi * np.outer(np.arange(N), np.arange(N)) / N) / math.sqrt(N)
    X = (sigma * math.sqrt(N) * F[:D])[None]  # [1][D][N]
    Rh = orc.covariance(X, 1)
    np.testing.assert_allclose(Rh[0, 0], sigma ** 2 * np.eye(D), atol=1e-12)
    delta, RL = orc.loading(Rh, eps)
    V = _crandn(_rng(6), S, D)
    W, gamma, info = orc.solve_weights(RL, V)
    nv = np.linalg.norm(V, axis=1)
    np.testing.assert_allclose(gamma[0, 0], nv ** 2 / (sigma ** 2 * (1 + eps)), rtol=1e-10)
    want = V / (sigma * math.sqrt(1 + eps) * nv[:, None])
    np.testing.assert_allclose(W[0, 0], want, rtol=1e-10, atol=1e-14)


def check_info_indefinite(orc=stap):
    D = 10
    mats, want = [], []
    for j in (0, 3, 9):
        A = np.eye(D, dtype=complex)
        A[j, j] = -1.0
        mats.append(A)
        want.append(j + 1)
    A = np.eye(D, dtype=complex)
    A[4, 5] = A[5, 4] = 2.0  # 2x2 block [[1,2],[2,1]]: second pivot 1-4 = -3
    mats.append(A)
    want.append(6)
    mats.append(np.eye(D, dtype=complex) * 2.0)
    want.append(0)
    V = _crandn(_rng(7), 4, D)
    W, gamma, info = orc.solve_weights(np.stack(mats), V)
    assert list(info) == want
    assert np.all(W[np.array(want) > 0] == 0)


# --------------------------------------------------------- whole chain invariants

def _small_run(orc=stap, wl=synth.SMALL):
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    return wl, cube, V, orc.run(cube, V, wl.tdof, wl.n_block, wl.load_eps)


def check_block_sum_and_cell_bound(orc=stap, res=None):
    """Sum over block b of P[k][s][r] = N (1 - delta ||u||^2 / gamma), exactly;
    and x_r^H R_L^-1 x_r bounds every cell's power and is below N."""
    wl, cube, V, o = res or _small_run(orc)
    N, B, P, S = wl.n_cell, wl.n_block, wl.n_pulse, wl.n_steer
    # independent recomputation from the oracle's own outputs only where the
    # identity is stated; the snapshots are recomputed by brute-force FFT-free
    # means (the loading/covariance identities tie everything together)
    pw = o["power"].reshape(P, S, B, N).sum(-1).transpose(0, 2, 1)  # [k][b][s]
    u2 = np.sum(np.abs(o["W"]) ** 2, axis=-1) * o["gamma"]            # ||u||^2
    pred = N * (1.0 - o["delta"][..., None] * u2 / o["gamma"])
    np.testing.assert_allclose(pw, pred, rtol=1e-9)
    X = o["X"]
    Xb = X.reshape(P, X.shape[1], B, N).transpose(0, 2, 1, 3)          # [k][b][d][n]
    q = np.real(np.sum(np.conj(Xb) * np.linalg.solve(o["R_L"], Xb), axis=2))  # [k][b][n]
    assert q.max() < N
    pb = o["power"].reshape(P, S, B, N).transpose(0, 2, 1, 3)          # [k][b][s][n]
    assert np.all(pb <= q[:, :, None, :] * (1 + 1e-9))


def check_target_recovered(orc=stap, res=None):
    wl, cube, V, o = res or _small_run(orc)
    sc = synth.scene(wl)
    pw = o["power"]
    k, s, r = np.unravel_index(int(np.argmax(pw)), pw.shape)
    assert r == sc.target_cell and s == sc.target_steer
    dk = min((k - sc.target_bin) % wl.n_pulse, (sc.target_bin - k) % wl.n_pulse)
    assert dk <= 1  # the Hann main lobe spans the neighbouring bin
    others = np.delete(pw, sc.target_cell, axis=2)
    assert pw[sc.target_bin, sc.target_steer, sc.target_cell] > others.max()


def check_sinr_loss(orc=stap, res=None):
    wl, cube, V, o = res or _small_run(orc)
    loss0 = metrics.sinr_loss_db(o["W"], o["W"], V, o["R_L"])
    assert np.abs(loss0).max() < 1e-9
    W1 = o["W"] + 1e-3 * _crandn(_rng(8), *o["W"].shape) * np.abs(o["W"]).mean()
    loss1 = metrics.sinr_loss_db(W1, o["W"], V, o["R_L"])
    assert loss1.min() > -1e-9 and loss1.max() > 0


def check_block_sampling(orc=stap, res=None):
    """The single-block chain equals the corresponding part of the full chain."""
    wl, cube, V, o = res or _small_run(orc)
    N = wl.n_cell
    for b in (0, 7, wl.n_block - 1):
        blk = synth.make_cube(wl, b * N, (b + 1) * N)
        np.testing.assert_array_equal(blk, cube[:, :, b * N:(b + 1) * N])
        ob = orc.run_block(blk, V, wl.tdof, wl.load_eps, bins=np.array([0, 5, 33]))
        np.testing.assert_allclose(ob["W"][:, 0], o["W"][[0, 5, 33], b], rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(ob["power"], o["power"][[0, 5, 33]][:, :, b * N:(b + 1) * N],
                                   rtol=1e-9, atol=1e-12)


CHECKS = [check_window_library_and_sums, check_doppler_brute_force, check_doppler_tone,
          check_doppler_impulse, check_parseval, check_covariance_brute_force,
          check_covariance_invariants, check_loading_closed_form,
          check_solve_library_and_backward, check_white_snapshots, check_info_indefinite]
CHAIN_CHECKS = [check_block_sum_and_cell_bound, check_target_recovered, check_sinr_loss,
                check_block_sampling]


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_pin(check):
    check()


@pytest.fixture(scope="module")
def small_res():
    return _small_run()


@pytest.mark.parametrize("check", CHAIN_CHECKS, ids=lambda f: f.__name__)
def test_chain_pin(check, small_res):
    check(res=small_res)


def test_target_recovered_medium():
    """Second workload size; ~15 s on 8 cores."""
    check_target_recovered(res=_small_run(wl=synth.MEDIUM))
