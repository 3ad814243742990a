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


# ------------------------------------------------------------------ error metrics
#
# The metrics decide every parity verdict, so they are pinned by hand-computed
# values: vectors of known norm, a block-diagonal batch, and the SINR of a
# diagonal covariance in closed form.

def check_rel_err_known_norms(met=metrics):
    ref = np.array([3.0, 4.0j])                 # ||ref|| = 5
    a = ref + np.array([0.0, 1.0])              # ||a - ref|| = 1
    assert abs(met.rel_err(a, ref) - 0.2) < 1e-15
    # a second error of norm 13 on a reference of norm 13 (5-12-13 triangle)
    ref2 = np.array([[5.0, 0.0], [0.0, 12.0j]])
    a2 = ref2 + np.array([[0.0, 12.0], [5.0j, 0.0]])
    assert abs(met.rel_err(a2, ref2) - 1.0) < 1e-15
    # a zero reference returns the absolute norm of the difference
    assert abs(met.rel_err(np.array([3.0, 4.0]), np.zeros(2)) - 5.0) < 1e-15


def check_per_system_rel_err_block_diagonal(met=metrics):
    S, D = 2, 3
    W_o = np.ones((3, S, D), complex)           # every system: norm sqrt(6)
    W = W_o.copy()
    W[0, 0, 0] += 0.6                           # system 0: 0.6 / sqrt(6)
    W[1] *= 2.0                                 # system 1: 1
    # system 2 exact
    got = met.per_system_rel_err(W, W_o)
    np.testing.assert_allclose(got, [0.6 / math.sqrt(6.0), 1.0, 0.0], rtol=0, atol=1e-15)
    # a system with zero reference reports its absolute norm
    Wz = np.zeros((1, S, D), complex)
    Wz2 = Wz.copy()
    Wz2[0, 1, 2] = 3.0 + 4.0j
    np.testing.assert_allclose(met.per_system_rel_err(Wz2, Wz), [5.0], rtol=0, atol=1e-15)


def check_sinr_closed_form(met=metrics):
    """R = sigma^2 I: SINR(w) = |w^H v|^2 / (sigma^2 ||w||^2), = ||v||^2 / sigma^2
    for w proportional to v.  Diagonal R = diag(r): SINR(R^-1 v) = sum |v_i|^2 / r_i,
    SINR(v) = ||v||^4 / sum r_i |v_i|^2."""
    v = np.array([[1.0, 2.0j, -2.0]])           # ||v||^2 = 9
    sig2 = 2.5
    R = sig2 * np.eye(3)[None]
    np.testing.assert_allclose(met.sinr((0.7 - 0.2j) * v[None], v, R), [[9.0 / 2.5]], rtol=1e-14)
    w = np.array([[[1.0, 0.0, 0.0]]])           # |w^H v|^2 = 1, ||w|| = 1
    np.testing.assert_allclose(met.sinr(w, v, R), [[1.0 / 2.5]], rtol=1e-14)
    r = np.array([1.0, 4.0, 0.5])
    Rd = np.diag(r)[None]
    w_opt = (v / r)[None]
    np.testing.assert_allclose(met.sinr(w_opt, v, Rd), [[1.0 + 4.0 / 4.0 + 4.0 / 0.5]], rtol=1e-14)
    np.testing.assert_allclose(met.sinr(v[None], v, Rd), [[81.0 / (1.0 + 16.0 + 2.0)]], rtol=1e-14)


def check_sinr_loss_closed_form(met=metrics):
    """w = v against w_o = R^-1 v under R = diag(1, 4) and v = (1, 1):
    SINR(w_o) = 1 + 1/4 = 1.25, SINR(v) = 4 / 5, loss = 10 log10(1.5625)."""
    v = np.array([[1.0, 1.0]])
    R = np.diag([1.0, 4.0])[None]
    w_o = np.array([[[1.0, 0.25]]])
    loss = met.sinr_loss_db(v[None], w_o, v, R)
    np.testing.assert_allclose(loss, [[1.9382002601611283]], rtol=1e-13)
    # the loss is invariant to a complex scale of either weight vector
    loss2 = met.sinr_loss_db((2.0 - 1.0j) * v[None], 0.5j * w_o, v, R)
    np.testing.assert_allclose(loss2, loss, rtol=1e-13)
    np.testing.assert_allclose(met.sinr_loss_db(w_o, w_o, v, R), [[0.0]], atol=1e-14)


# ----------------------------------- relative tap phase, per-bin steering (f4)

def check_doppler_relative_brute_force(orc=stap):
    """Each tap referenced to its own first pulse:
    X[k][t*C+c][r] = sum_{p=t}^{t+L-1} h[p-t] x[c][p][r] e^{-j 2 pi k (p-t)/P}."""
    C, P, R, T = 2, 8, 3, 3
    x = _crandn(_rng(11), C, P, R)
    L = P - T + 1
    h = np.hanning(L)
    X = orc.doppler(x, T, relative=True)
    for k in range(P):
        for t in range(T):
            for c in range(C):
                for r in range(R):
                    acc = 0j
                    for p in range(t, t + L):
                        acc += h[p - t] * x[c, p, r] * cmath.exp(-2j * math.pi * k * (p - t) / P)
                    assert abs(X[k, t * C + c, r] - acc) < 1e-12


def check_relative_chain_equivalence(orc=stap):
    """Relative taps are the absolute ones times exp(j 2 pi k t / P), so the
    covariance becomes Phi R Phi^H with Phi = diag(exp(j 2 pi k t / P)); with
    the steering set carried through the same phases (per bin) the weights
    are Phi w and the output power is unchanged."""
    wl = synth.with_(synth.SMALL, n_range=128, n_block=8)
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    Vk = synth.steering_per_bin(wl).astype(np.complex128)
    P, C, T = wl.n_pulse, wl.n_chan, wl.tdof
    phi = np.exp(2j * np.pi * np.outer(np.arange(P), np.repeat(np.arange(T), C)) / P)  # [P][D]
    np.testing.assert_allclose(Vk, phi[:, None, :] * V[None].astype(np.complex128), atol=2e-7)
    a = orc.run(cube, V, T, wl.n_block, wl.load_eps)
    b = orc.run(cube, phi[:, None, :] * V[None].astype(np.complex128), T, wl.n_block, wl.load_eps,
                relative=True)
    np.testing.assert_allclose(b["X"], phi[:, :, None] * a["X"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(b["W"], phi[:, None, None, :] * a["W"], rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(b["power"], a["power"], rtol=1e-8, atol=1e-10)


def check_offbin_target_per_bin(orc=stap):
    """A target a quarter bin off its Doppler bin, relative taps and per-bin
    steering: the largest output is at the target's cell and steering vector,
    within one bin of its Doppler."""
    wl = synth.with_(synth.SMALL, target_offset=0.25)
    cube = synth.make_cube(wl)
    o = orc.run(cube, synth.steering_per_bin(wl), wl.tdof, wl.n_block, wl.load_eps, relative=True)
    sc = synth.scene(wl)
    k, s, r = np.unravel_index(int(np.argmax(o["power"])), o["power"].shape)
    assert (r, s) == (sc.target_cell, sc.target_steer)
    assert min((k - sc.target_bin) % wl.n_pulse, (sc.target_bin - k) % wl.n_pulse) <= 1


# ------------------------------------- training without the cell under test (f1)

def check_training_cells(orc=stap):
    """Hand-worked cases (R = 64, B = 8, N = 8, G = 2) and the definition's
    invariants: N distinct cells, none of the block or its guard cells, the
    nearest ones on each side, half (rounded down) on the left away from the
    edges."""
    want = {0: list(range(10, 18)), 3: list(range(18, 22)) + list(range(34, 38)),
            7: list(range(46, 54)), 1: [2, 3, 4, 5, 18, 19, 20, 21]}
    for b, cells in want.items():
        assert list(orc.training_cells(64, 8, b, 2)) == cells, b
    for R, B, G in ((64, 8, 0), (96, 12, 3), (512, 32, 4), (40, 5, 1), (30, 3, 5)):
        N = R // B
        for b in range(B):
            cells = orc.training_cells(R, B, b, G)
            assert len(cells) == N and len(set(cells.tolist())) == N
            assert cells.min() >= 0 and cells.max() < R
            assert not np.any((cells >= b * N - G) & (cells < b * N + N + G))
            left, right = cells[cells < b * N], cells[cells >= b * N]
            if len(left):
                assert left.max() == b * N - G - 1 and np.all(np.diff(left) == 1)
            if len(right):
                assert right.min() == b * N + N + G and np.all(np.diff(right) == 1)
            if b * N - G >= N // 2 and R - (b * N + N + G) >= N - N // 2:
                assert len(left) == N // 2
    with pytest.raises(ValueError):
        orc.training_cells(30, 3, 1, 6)


def check_covariance_excluded_brute_force(orc=stap):
    P, D, R, B, G = 2, 3, 24, 4, 2
    X = _crandn(_rng(12), P, D, R)
    Rh = orc.covariance(X, B, guard=G)
    N = R // B
    for b in range(B):
        cells = [r for r in range(R) if not (b * N - G <= r < b * N + N + G)]
        cells.sort(key=lambda r: (abs(r - (b * N + N / 2 - 0.5)), r))
        train = orc.training_cells(R, B, b, G)
        for k in range(P):
            acc = np.zeros((D, D), complex)
            for r in train:
                acc += np.outer(X[k, :, r], np.conj(X[k, :, r]))
            np.testing.assert_allclose(Rh[k, b], acc / N, atol=1e-13)


def check_excluded_cut_no_self_nulling(orc=stap):
    """With its own cells in the training set a target nulls itself: its AMF
    power is bounded by x^H R_L^-1 x < N.  Excluding the block and its guard
    cells, the covariance no longer depends on the target's snapshot, so its
    power is the closed form |v^H R^-1 x_t|^2 / (v^H R^-1 v) with R built from
    the training cells alone, it grows as |alpha|^2 when the target's cube
    column is scaled by alpha (2 here, exact in complex64), and it exceeds N."""
    wl = synth.SMALL
    G = 2
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    sc = synth.scene(wl)
    k, s, r = sc.target_bin, sc.target_steer, sc.target_cell
    N = wl.n_cell
    b = r // N
    inc = orc.run(cube, V, wl.tdof, wl.n_block, wl.load_eps)
    exc = orc.run(cube, V, wl.tdof, wl.n_block, wl.load_eps, guard=G)
    assert inc["power"][k, s, r] < N < exc["power"][k, s, r]
    # closed form from the training cells alone (snapshots by the pinned DFT)
    X = exc["X"]
    train = orc.training_cells(wl.n_range, wl.n_block, b, G)
    Rh = sum(np.outer(X[k, :, c], np.conj(X[k, :, c])) for c in train) / N
    Rl = Rh + wl.load_eps * np.real(np.trace(Rh)) / wl.dof * np.eye(wl.dof)
    v = V[s].astype(np.complex128)
    ri_x = np.linalg.solve(Rl, X[k, :, r])
    ri_v = np.linalg.solve(Rl, v)
    want = abs(np.vdot(v, ri_x)) ** 2 / np.real(np.vdot(v, ri_v))
    assert abs(exc["power"][k, s, r] - want) < 1e-9 * want
    cube2 = cube.copy()
    cube2[:, :, r] *= 2.0  # exact in complex64
    exc2 = orc.run(cube2, V, wl.tdof, wl.n_block, wl.load_eps, guard=G)
    assert abs(exc2["power"][k, s, r] - 4.0 * exc["power"][k, s, r]) < 1e-9 * exc2["power"][k, s, r]


def check_run_block_matches_excluded(orc=stap):
    """The sampled single-block chain with explicit training cells equals the
    full excluded-training chain."""
    wl = synth.with_(synth.SMALL, n_range=256, n_block=16)
    G = 3
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    o = orc.run(cube, V, wl.tdof, wl.n_block, wl.load_eps, guard=G)
    N = wl.n_cell
    for b in (0, 5, wl.n_block - 1):
        cells = orc.training_cells(wl.n_range, wl.n_block, b, G)
        ob = orc.run_block(cube[:, :, b * N:(b + 1) * N], V, wl.tdof, wl.load_eps, bins=np.array([1, 9]),
                           train_block=cube[:, :, cells])
        np.testing.assert_allclose(ob["W"][:, 0], o["W"][[1, 9], b], rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(ob["power"], o["power"][[1, 9]][:, :, b * N:(b + 1) * N], rtol=1e-9,
                                   atol=1e-12)


def check_subarray_brute_force(orc=stap):
    """Subarray channels by explicit loops: channel c' sums elements
    c' n .. c' n + n - 1; n = 1 is the identity."""
    rng = _rng(21)
    x = _crandn(rng, 12, 5, 3)
    for n in (1, 2, 3, 4, 6, 12):
        y = orc.subarray(x, n)
        assert y.shape == (12 // n, 5, 3)
        for c in range(12 // n):
            for p in range(5):
                for r in range(3):
                    acc = 0j
                    for e in range(n):
                        acc += x[c * n + e, p, r]
                    assert abs(y[c, p, r] - acc) < 1e-12
    with pytest.raises(ValueError):
        orc.subarray(x, 5)


def check_subarray_plane_wave(orc=stap):
    """A plane wave exp(j 2 pi theta c) over the elements gives subarray c'
    the closed form exp(j 2 pi theta c' n) (1 - exp(j 2 pi theta n)) /
    (1 - exp(j 2 pi theta)): the phase centre steps by n elements and the
    magnitude is the array factor of n elements."""
    C, n = 40, 8
    for theta in (0.013, -0.21, 0.37):
        x = np.exp(2j * np.pi * theta * np.arange(C))[:, None, None] * np.ones((1, 2, 2))
        y = orc.subarray(x, n)
        geo = (1 - cmath.exp(2j * math.pi * theta * n)) / (1 - cmath.exp(2j * math.pi * theta))
        for c in range(C // n):
            want = cmath.exp(2j * math.pi * theta * c * n) * geo
            assert np.all(np.abs(y[c] - want) < 1e-12)


def check_doppler_p100(orc=stap):
    """The paper's pulse count P = 100 (not a power of two): brute-force DFT
    of every tap, and the on-bin tone giving sum h = (L - 1) / 2 = 48.5 in
    every tap (L = 98)."""
    C, P, R, T = 1, 100, 2, 3
    rng = _rng(3)
    x = _crandn(rng, C, P, R)
    L = P - T + 1
    h = np.hanning(L)
    X = orc.doppler(x, T)
    for k in (0, 1, 37, 50, 99):
        for t in range(T):
            for r in range(R):
                acc = 0j
                for p in range(t, t + L):
                    acc += h[p - t] * x[0, p, r] * cmath.exp(-2j * math.pi * k * p / P)
                assert abs(X[k, t, r] - acc) < 1e-11
    for k0 in (3, 50, 71):
        tone = np.exp(2j * np.pi * k0 * np.arange(P) / P)[None, :, None] * np.ones((2, 1, 1))
        Xt = orc.doppler(tone, T)
        assert np.all(np.abs(Xt[k0] - 48.5) < 1e-10)


def near_singular_cases():
    """The two matrices of golden/near_singular_pivots.json as complex64
    arrays, with the sign of their last pivot from exact rational
    arithmetic."""
    from fractions import Fraction
    g = json.load(open(os.path.join(GOLDEN, "near_singular_pivots.json")))
    out = []
    for case in g["cases"]:
        a = [np.float32(1.0 + k * 2.0 ** -23) for k in case["k"]]
        n = len(a)
        R = np.eye(n + 1, dtype=np.complex64)
        R[n, :n] = a
        R[:n, n] = a
        R[n, n] = np.float32(case["r_last"])
        exact = Fraction(float(R[n, n].real)) - sum(Fraction(float(x)) ** 2 for x in a)
        out.append((R, exact))
    return out


def check_info_near_singular(orc=stap):
    """Pivots that FP32 accumulation gets wrong: the exact last pivot (rational
    arithmetic) is positive for one matrix and negative for the other, and
    the oracle's status follows it (0, and 20 = the 1-based index of the last
    pivot).  A running FP32 update of the last diagonal (each fused
    multiply-add rounded to FP32) ends with the opposite sign in both cases,
    which is why the pivot test is taken in FP64."""
    for R, exact in near_singular_cases():
        n = R.shape[0] - 1
        want = 0 if exact > 0 else n + 1
        assert exact != 0
        _, info = orc.cholesky_info(R.astype(np.complex128))
        assert info == want, (info, want)
        A = np.float32(R[n, n].real)
        for k in range(n):
            A = np.float32(float(A) - float(R[n, k].real) ** 2)
        assert (float(A) > 0) != (exact > 0)


METRIC_CHECKS = [check_rel_err_known_norms, check_per_system_rel_err_block_diagonal,
                 check_sinr_closed_form, check_sinr_loss_closed_form]


CHECKS = [check_window_library_and_sums, check_doppler_brute_force, check_doppler_tone,
          check_doppler_impulse, check_parseval, check_covariance_brute_force,
          check_covariance_invariants, check_loading_closed_form,
          check_solve_library_and_backward, check_white_snapshots, check_info_indefinite,
          check_doppler_relative_brute_force, check_relative_chain_equivalence,
          check_offbin_target_per_bin, check_training_cells, check_covariance_excluded_brute_force,
          check_excluded_cut_no_self_nulling, check_run_block_matches_excluded,
          check_subarray_brute_force, check_subarray_plane_wave, check_doppler_p100,
          check_info_near_singular]
CHAIN_CHECKS = [check_block_sum_and_cell_bound, check_target_recovered, check_sinr_loss,
                check_block_sampling]


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_pin(check):
    check()


@pytest.mark.parametrize("check", METRIC_CHECKS, ids=lambda f: f.__name__)
def test_metric_pin(check):
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
