"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/stap.h, and rejects invalid requests on the host before
any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stap.h")
LIB = os.path.join(ROOT, "paper_2203_06233_amd", "libstap.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stap_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def binding():
    if not os.path.exists(LIB):
        from paper_2203_06233_amd import build
        build.build()
    from paper_2203_06233_amd import stap
    return stap


def test_header_declares_the_five_entry_points():
    names = _declared()
    for n in ("stap_doppler", "stap_covariance", "stap_solve_weights", "stap_inner_products", "stap_run"):
        assert n in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version(binding):
    assert binding.version().count(".") == 2
    for code in range(-6, 1):
        assert binding._string(code) != "unknown status"
    assert binding._string(-99) == "unknown status"


GOOD = dict(n_chan=4, n_pulse=64, n_range=512, tdof=3, n_block=32, n_steer=8)


@pytest.mark.parametrize("change,code", [
    (dict(n_pulse=48), -2), (dict(n_pulse=1024), -2), (dict(n_pulse=16), -2),
    (dict(n_range=500), -2), (dict(n_range=0), -2), (dict(n_block=0), -2), (dict(n_pulse=100, tdof=3), 0),
    (dict(tdof=0), -2), (dict(tdof=5), -2), (dict(n_chan=65), -2),
    (dict(n_steer=0), -2), (dict(n_steer=65), -2),
    (dict(load_eps=-1.0), -1), (dict(load_eps=float("nan")), -1),
    (dict(precision="fp32", refine_steps=5), -1),
    (dict(cube_stride_pulse=100), -2),
])
def test_problem_validation(binding, change, code):
    kw = dict(GOOD)
    kw.update(change)
    p = binding.problem(**kw)
    assert binding._lib.stap_check_problem(ctypes.byref(p)) == code


def test_valid_problems(binding):
    for kw in (GOOD, dict(n_chan=32, n_pulse=256, n_range=16384, tdof=3, n_block=128, n_steer=32),
               dict(n_chan=64, n_pulse=512, n_range=32768, tdof=3, n_block=256, n_steer=64),
               dict(n_chan=5, n_pulse=32, n_range=7, tdof=1, n_block=7, n_steer=1)):
        binding.check_problem(binding.problem(**kw))


def test_bad_precision_code(binding):
    p = binding.problem(**GOOD)
    p.precision = 7
    assert binding._lib.stap_check_problem(ctypes.byref(p)) == -1
    p.precision = 0
    p.subarray = -1
    assert binding._lib.stap_check_problem(ctypes.byref(p)) == -1


def test_paper_cube_shape_and_subarrays(binding):
    """The paper's cube (100 pulses, 1000 elements, 30000 samples) is valid
    with subarrays that keep D within the limit, in either nesting of the
    cube's channel and pulse axes; full element-space DOF is not."""
    lib = binding._lib

    def code(**kw):
        p = binding.problem(**kw)
        return lib.stap_check_problem(ctypes.byref(p))

    paper = dict(n_chan=1000, n_pulse=100, n_range=30000, tdof=3, n_block=250, n_steer=32)
    assert code(**paper, n_sub=50) == 0
    assert code(**paper) == -2                      # D = 3000
    assert code(**paper, n_sub=3) == -2             # 1000 elements are not a multiple of 3
    assert code(**paper, n_sub=10) == -2            # D = 300
    # the paper's pulses x channels x samples order: pulse stride C R, channel stride R
    assert code(**paper, n_sub=50, cube_stride_chan=30000, cube_stride_pulse=1000 * 30000) == 0
    assert code(**paper, n_sub=50, cube_stride_chan=30000, cube_stride_pulse=999 * 30000) == -2
    assert code(**dict(GOOD, n_pulse=100)) == 0
    for P in (96, 200, 1000):
        assert code(**dict(GOOD, n_pulse=P)) == -2
    p = binding.problem(**paper, n_sub=50)
    assert p.dof == 60 and p.channels == 20


def test_training_phase_and_steering_fields(binding):
    """Cell-under-test exclusion, tap phase and per-bin steering are checked
    on the host: codes out of range, guard cells without exclusion, and
    blocks that cannot find N training cells outside themselves and their
    guard cells."""
    lib = binding._lib

    def code(**kw):
        p = binding.problem(**dict(GOOD, **kw))
        return lib.stap_check_problem(ctypes.byref(p))

    assert code(guard=0) == 0 and code(guard=3) == 0
    assert code(tap_phase="relative") == 0 and code(steer_per_bin=True) == 0
    # N = 16, R = 512: interior blocks need R - N - 2G >= N
    assert code(guard=(512 - 32) // 2) == 0
    assert code(guard=(512 - 32) // 2 + 1) == -2
    # a single block has no cells outside itself
    assert code(n_block=1, n_range=64, guard=0) == -2
    # two blocks of N: each trains on the other (G = 0 only)
    assert code(n_block=2, n_range=64, guard=0) == 0
    assert code(n_block=2, n_range=64, guard=1) == -2
    for field, value in (("training", 2), ("training", -1), ("tap_phase", 2), ("steer_per_bin", 2),
                         ("guard_cells", -1)):
        p = binding.problem(**GOOD)
        setattr(p, field, value)
        if field == "guard_cells":
            p.training = 1
        assert lib.stap_check_problem(ctypes.byref(p)) == -1, field
    p = binding.problem(**GOOD)
    p.guard_cells = 2  # guard cells without exclusion
    assert lib.stap_check_problem(ctypes.byref(p)) == -1


def test_entry_points_reject_before_touching_the_device(binding):
    """Null or misaligned pointers and bad shapes return without a HIP call,
    so these work on a machine with no GPU."""
    lib = binding._lib
    p = binding.problem(**GOOD)
    bp = ctypes.byref(p)
    fake = ctypes.c_void_p(0x10000)
    odd = ctypes.c_void_p(0x10004)
    assert lib.stap_doppler(bp, None, fake, None) == -1
    assert lib.stap_doppler(bp, fake, None, None) == -1
    assert lib.stap_doppler(bp, odd, fake, None) == -3
    assert lib.stap_covariance(bp, fake, None, None, None) == -1
    assert lib.stap_covariance(bp, fake, fake, ctypes.c_void_p(0x10002), None) == -3
    assert lib.stap_solve_weights(bp, fake, fake, fake, None, None) == -1
    assert lib.stap_inner_products(bp, fake, fake, None, None, None) == -1
    bad = binding.problem(**dict(GOOD, n_range=500))
    assert lib.stap_doppler(ctypes.byref(bad), fake, fake, None) == -2
    # null info is rejected for the solve
    big = binding.problem(n_chan=64, n_pulse=512, n_range=32768, tdof=3, n_block=256, n_steer=64)
    assert lib.stap_solve_weights(ctypes.byref(big), fake, fake, fake, None, None) == -1


def test_run_rejects_before_touching_the_device(binding):
    lib = binding._lib
    probs = (binding.Problem * 2)(binding.problem(**GOOD), binding.problem(**GOOD))
    VP = ctypes.c_void_p * 2
    fake = VP(0x10000, 0x20000)
    need = lib.stap_workspace_size(probs, 2)
    assert need > 0
    # workspace too small
    assert lib.stap_run(probs, 2, fake, fake, fake, None, None, ctypes.c_void_p(0x100000), need - 1, None) == -4
    assert lib.stap_run(probs, 2, fake, fake, fake, None, None, None, need, None) == -4
    # workspace misaligned
    assert lib.stap_run(probs, 2, fake, fake, fake, None, None, ctypes.c_void_p(0x100010), need, None) == -3
    # mixed precision across the batch
    probs[1].precision = 1
    assert lib.stap_run(probs, 2, fake, fake, fake, None, None, ctypes.c_void_p(0x100000), need, None) == -1
    assert lib.stap_run(probs, 0, fake, fake, fake, None, None, ctypes.c_void_p(0x100000), need, None) == -1


def test_noalloc_rejects_on_the_host(binding):
    """stap_run_noalloc checks its arguments and the fixed scratch size before
    any HIP call: a cube whose workspace exceeds STAP_NOALLOC_MAX_BYTES gets
    STAP_ERR_WORKSPACE, bad pointers their usual codes."""
    lib = binding._lib
    one = ctypes.c_void_p * 1
    fake = one(0x10000)
    big = (binding.Problem * 1)(binding.problem(n_chan=32, n_pulse=256, n_range=16384, tdof=3, n_block=128,
                                                n_steer=32))
    assert binding.workspace_size(list(big)) > binding.NOALLOC_MAX_BYTES
    assert lib.stap_run_noalloc(big, 1, fake, fake, fake, None, None, None) == -4
    small = (binding.Problem * 1)(binding.problem(**GOOD))
    assert lib.stap_run_noalloc(small, 1, one(0x10004), fake, fake, None, None, None) == -3
    assert lib.stap_run_noalloc(small, 0, fake, fake, fake, None, None, None) == -1
    assert lib.stap_run_noalloc(small, 1, None, fake, fake, None, None, None) == -1


def test_tuning_table(binding):
    lib = binding._lib
    saved = binding.tune_get(96, 32, "bf16", 1)
    try:
        binding.tune_set(96, 32, "bf16", 1, 0)
        assert binding.tune_get(96, 32, "bf16", 1) == 0
        binding.tune_set(96, 32, "bf16", 1, 32)
        assert binding.tune_get(96, 32, "bf16", 1) == 32
        assert binding.tune_get(90, 20, "bf16", 2) == 32  # same class
        binding.tune_set(96, 32, "bf16", 1, 16)
        assert binding.tune_get(96, 32, "bf16", 1) == 16
    finally:
        binding.tune_set(96, 32, "bf16", 1, saved)
    assert lib.stap_tune_set(0, 96, 32, 1, 1, 24) == -1
    assert lib.stap_tune_set(1, 96, 32, 1, 0, 8) == 0 and lib.stap_tune_get(1, 96, 32, 1, 0) == 8
    assert lib.stap_tune_set(1, 96, 32, 1, 0, 0) == 0
    assert lib.stap_tune_set(0, 200, 32, 1, 1, 16) == -1
    assert lib.stap_tune_get(0, 96, 65, 1, 1) == -1
    # variant 1 (one wave per system) is a valid entry for both kinds
    for kind in (0, 1):
        old = lib.stap_tune_get(kind, 96, 32, 1, 0)
        assert lib.stap_tune_set(kind, 96, 32, 1, 0, 1) == 0 and lib.stap_tune_get(kind, 96, 32, 1, 0) == 1
        assert lib.stap_tune_set(kind, 96, 32, 1, 0, old) == 0
    assert lib.stap_tune_set(0, 96, 32, 1, 0, 2) == -1
    # kind 2: waves per system of the stage covariance; kind 3: range tiles
    # per wave step of the inner products
    for kind, good, bad in ((2, (0, 4, 8, 16), (1, 2, 32)), (3, (0, 1, 2, 4), (8, 16, 3))):
        old = lib.stap_tune_get(kind, 96, 32, 1, 1)
        for v in good:
            assert lib.stap_tune_set(kind, 96, 32, 1, 1, v) == 0 and lib.stap_tune_get(kind, 96, 32, 1, 1) == v
        for v in bad:
            assert lib.stap_tune_set(kind, 96, 32, 1, 1, v) == -1
        assert lib.stap_tune_set(kind, 96, 32, 1, 1, old) == 0
    assert lib.stap_tune_set(4, 96, 32, 1, 1, 0) == -1


def test_tuner_candidates():
    """The autotuner times the one-wave solve only where it applies."""
    from paper_2203_06233_amd import tune
    assert 1 in tune.candidates(96, 0, 0, 32) and 1 in tune.candidates(12, 1, 1, 8)
    assert 1 not in tune.candidates(112, 0, 0, 32)  # D > 96
    assert 1 not in tune.candidates(96, 0, 0, 33)  # S > 32
    assert tune.candidates(192, 1, 1, 64) == [0, 8]
    assert 32 not in tune.candidates(32, 0)  # the 32-row grid needs D > 32


def test_kernel_tuning_candidates():
    """Covariance wave counts and inner-product tile counts the tuner tries
    per DOF class (0 = the default)."""
    from paper_2203_06233_amd import tune
    assert tune.kernel_candidates(2, 96, "bf16") == [0, 4, 16]
    assert tune.kernel_candidates(2, 48, "fp32") == [0, 4, 8]
    assert tune.kernel_candidates(2, 128, "fp32") == [0, 16]
    assert tune.kernel_candidates(2, 24, "fp32") == [0] and tune.kernel_candidates(2, 192, "fp8") == [0]
    assert tune.kernel_candidates(3, 96, "bf16") == [0, 1, 2]
    assert tune.kernel_candidates(3, 96, "fp32") == [0, 1, 2, 4]
    assert tune.kernel_candidates(3, 192, "fp8") == [0, 1, 2, 4]  # D > 128 takes the FP32 form


def test_workspace_size_formula(binding):
    p = binding.problem(**GOOD)
    P, D, R, B, S = 64, 12, 512, 32, 8

    def up(x):
        return (x + 255) // 256 * 256
    table = 136  # one problem descriptor (the kernels' copy of the shapes and pointers)
    queues = 24 * 8  # a work-queue counter per shape class (8 DOF classes x 3 steering classes)
    per = up(P * D * R * 8) + up(P * B * S * D * 8) + up(P * B * 4)
    cov = up(P * B * D * D * 8) + up(P * B * 4)
    # D <= 96 and S <= 32: the one-wave stage route may run, covariance and delta included
    assert binding.workspace_size([p]) == up(table + queues) + per + cov
    assert binding.workspace_size([p, p]) == up(2 * table + queues) + 2 * (per + cov)
    # D in (96, 128] takes the fused kernel: no covariance
    f = binding.problem(n_chan=40, n_pulse=32, n_range=256, tdof=3, n_block=2, n_steer=20)
    P, D, R, B, S = 32, 120, 256, 2, 20
    per_f = up(P * D * R * 8) + up(P * B * S * D * 8) + up(P * B * 4)
    assert binding.workspace_size([f]) == up(table + queues) + per_f
    # D > 128 keeps the covariance and delta in the workspace
    q = binding.problem(n_chan=48, n_pulse=32, n_range=256, tdof=3, n_block=2, n_steer=20)
    P, D, R, B, S = 32, 144, 256, 2, 20
    per_q = (up(P * D * R * 8) + up(P * B * D * D * 8) + up(P * B * 4) + up(P * B * S * D * 8)
             + up(P * B * 4))
    assert binding.workspace_size([q]) == up(table + queues) + per_q
    # FP8 does not use the fused kernel either
    p8 = binding.problem(**dict(GOOD, precision="fp8"))
    P, D, R, B, S = 64, 12, 512, 32, 8
    assert binding.workspace_size([p8]) == up(table + queues) + per + cov
