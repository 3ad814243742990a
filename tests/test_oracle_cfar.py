"""Pins of the CA-CFAR oracle: brute force on small inputs, closed forms of
constant and single-spike maps, edge windows, and the textbook false-alarm
rate of CA-CFAR on exponential noise; planted mistakes in a copy of the
oracle must each fail one of them."""
import math
import types

import numpy as np
import pytest

import oracle.cfar as cfar_mod


def check_brute_force(orc=cfar_mod):
    """Pure-Python loops over every cell and window position."""
    rng = np.random.default_rng(5)
    for (R, n_ref, n_guard) in [(40, 4, 2), (17, 3, 0), (9, 5, 1), (64, 8, 3)]:
        p = rng.exponential(1.0, (3, R)).astype(np.float32)
        p[1, R // 2] = 40.0
        alpha = 3.7
        det, noise, n_used = orc.ca_cfar(p, n_ref, n_guard, alpha)
        for row in range(3):
            for r in range(R):
                acc, n = 0.0, 0
                for o in list(range(-(n_guard + n_ref), -n_guard)) + list(range(n_guard + 1, n_guard + n_ref + 1)):
                    if 0 <= r + o < R:
                        acc += float(p[row, r + o])
                        n += 1
                assert n_used[r] == n
                assert det[row, r] == (float(p[row, r]) * n > alpha * acc)
                if n:
                    assert noise[row, r] == acc / n


def check_constant_map(orc=cfar_mod):
    """A constant map: the estimate is the constant wherever a cell has
    references, and nothing crosses a threshold alpha >= 1."""
    p = np.full((2, 50), 2.5, np.float32)
    for alpha in (1.0, 1.5, 10.0):
        det, noise, n_used = orc.ca_cfar(p, 6, 2, alpha)
        assert not det.any()
        assert np.all(noise == 2.5)
    det, _, _ = orc.ca_cfar(p, 6, 2, 0.5)
    assert det.all()
    _, _, n_used = orc.ca_cfar(p, 6, 2, 1.0)
    # offsets -8..-3 and 3..8: cell 3 has one left reference (cell 0), cell 8
    # the full window, the last cell only its left window
    assert n_used[25] == 12 and n_used[0] == 6 and n_used[49] == 6 and n_used[3] == 7 and n_used[8] == 12


def check_single_spike(orc=cfar_mod):
    """Spike h on a background of ones (interior, n references per side, g
    guards): the spike is detected iff h > alpha; a cell with the spike in its
    window sees (2n - 1 + h) / 2n; a cell with the spike in its guard zone
    is unaffected."""
    n, g, R, r0 = 5, 2, 60, 30
    for h, alpha in ((8.0, 7.9), (8.0, 8.0), (8.0, 3.0)):
        p = np.ones((1, R), np.float32)
        p[0, r0] = h
        det, noise, _ = orc.ca_cfar(p, n, g, alpha)
        assert det[0, r0] == (h > alpha)
        for d in range(1, g + 1):
            assert noise[0, r0 + d] == 1.0 and noise[0, r0 - d] == 1.0
        for d in range(g + 1, g + n + 1):
            assert noise[0, r0 + d] == (2 * n - 1 + h) / (2 * n)
            assert noise[0, r0 - d] == (2 * n - 1 + h) / (2 * n)
        assert noise[0, r0 + g + n + 1] == 1.0


def check_false_alarm_rate(orc=cfar_mod):
    """CA-CFAR on i.i.d. exponential noise with alpha = N (Pfa^(-1/N) - 1)
    has false-alarm probability Pfa (interior cells): binomial tolerance of
    5 standard deviations over 4e6 cells."""
    rng = np.random.default_rng(9)
    n, g, pfa = 8, 2, 1e-3
    alpha = orc.alpha_for_pfa(2 * n, pfa)
    p = rng.exponential(1.0, (400, 10000))
    det, _, n_used = orc.ca_cfar(p, n, g, alpha)
    inner = n_used == 2 * n
    cells = det[:, inner].size
    rate = det[:, inner].mean()
    sd = math.sqrt(pfa * (1 - pfa) / cells)
    assert abs(rate - pfa) < 5 * sd, (rate, pfa, sd)
    # the closed form itself: N (Pfa^(-1/N) - 1) at N = 16, Pfa = 1e-3
    assert abs(orc.alpha_for_pfa(16, 1e-3) - 16 * (10 ** (3 / 16) - 1)) < 1e-12


CHECKS = [check_brute_force, check_constant_map, check_single_spike, check_false_alarm_rate]


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_cfar_pin(check):
    check()


MUTANTS = {
    "cut_in_window": """
def offsets(n_ref, n_guard):
    left = np.arange(-(n_guard + n_ref), -n_guard)
    right = np.arange(n_guard, n_guard + n_ref)
    return np.concatenate([left, right])
""",
    "guard_off_by_one": """
def offsets(n_ref, n_guard):
    left = np.arange(-(n_guard + n_ref) + 1, -n_guard + 1)
    right = np.arange(n_guard + 1, n_guard + n_ref + 1)
    return np.concatenate([left, right])
""",
    "sum_not_mean": """
def ca_cfar(power, n_ref, n_guard, alpha):
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
    detect = p > float(alpha) * acc
    with np.errstate(invalid="ignore", divide="ignore"):
        noise = acc / n_used
    return detect, noise, n_used
""",
    "edges_wrap": """
def ca_cfar(power, n_ref, n_guard, alpha):
    p = np.asarray(power).astype(np.float64)
    R = p.shape[-1]
    r = np.arange(R)
    acc = np.zeros(p.shape, np.float64)
    n_used = np.zeros(R, np.int64)
    for o in offsets(n_ref, n_guard):
        acc = acc + p[..., (r + o) % R]
        n_used += 1
    detect = p * n_used.astype(np.float64) > float(alpha) * acc
    noise = acc / n_used
    return detect, noise, n_used
""",
    "pfa_formula_exponent": """
def alpha_for_pfa(n_ref_total, pfa):
    N = n_ref_total
    return N * (pfa ** (-1.0 / (N + 1)) - 1.0)
""",
    "greater_equal": """
def ca_cfar(power, n_ref, n_guard, alpha):
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
    detect = p * n_used.astype(np.float64) >= float(alpha) * acc
    with np.errstate(invalid="ignore", divide="ignore"):
        noise = acc / n_used
    return detect, noise, n_used
""",
}


def _mutant(name, src):
    mod = types.ModuleType("cfar_mutant_" + name)
    exec(compile(open(cfar_mod.__file__).read(), cfar_mod.__file__, "exec"), mod.__dict__)
    exec(src, mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_cfar_planted_mistake_is_caught(name):
    mod = _mutant(name, MUTANTS[name])
    failed = []
    for check in CHECKS:
        try:
            check(orc=mod)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"planted mistake {name} passes every pin"
