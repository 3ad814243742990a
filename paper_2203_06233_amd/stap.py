"""Python binding of libstap.so (the gfx950 STAP hot path).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/stap.h``.  PyTorch supplies
device memory (complex64 / float32 / int32 CUDA tensors) and the stream.  If
the shared library is missing the import of this module raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import List, Optional, Sequence

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstap.so")

PREC = {"fp32": 0, "bf16": 1, "fp8": 2}

STATUS = {
    0: "STAP_OK", -1: "STAP_ERR_ARG", -2: "STAP_ERR_SHAPE", -3: "STAP_ERR_ALIGN",
    -4: "STAP_ERR_WORKSPACE", -5: "STAP_ERR_HIP", -6: "STAP_ERR_UNSUPPORTED",
}


class StapError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({_string(code)})")


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_chan", ctypes.c_int32), ("n_pulse", ctypes.c_int32), ("n_range", ctypes.c_int32),
        ("tdof", ctypes.c_int32), ("n_block", ctypes.c_int32), ("n_steer", ctypes.c_int32),
        ("load_eps", ctypes.c_float), ("precision", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32), ("training", ctypes.c_int32),
        ("cube_stride_chan", ctypes.c_int64), ("cube_stride_pulse", ctypes.c_int64),
        ("guard_cells", ctypes.c_int32), ("tap_phase", ctypes.c_int32),
        ("steer_per_bin", ctypes.c_int32), ("subarray", ctypes.c_int32),
    ]

    @property
    def channels(self) -> int:
        return self.n_chan // max(self.subarray, 1)

    @property
    def dof(self) -> int:
        return self.tdof * self.channels

    @property
    def n_cell(self) -> int:
        return self.n_range // self.n_block

    def __repr__(self):
        return (f"Problem(C={self.n_chan}, P={self.n_pulse}, R={self.n_range}, T={self.tdof}, "
                f"B={self.n_block}, S={self.n_steer}, eps={self.load_eps}, prec={self.precision}, "
                f"refine={self.refine_steps}, training={self.training}, guard={self.guard_cells}, "
                f"tap_phase={self.tap_phase}, steer_per_bin={self.steer_per_bin})")


class CfarParams(ctypes.Structure):
    _fields_ = [("n_ref", ctypes.c_int32), ("n_guard", ctypes.c_int32), ("alpha", ctypes.c_double)]


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"libstap.so not built at {path}; run `python -m paper_2203_06233_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "stap_doppler": [P(Problem), vp, vp, vp],
        "stap_covariance": [P(Problem), vp, vp, vp, vp],
        "stap_solve_weights": [P(Problem), vp, vp, vp, vp, vp],
        "stap_covariance_solve": [P(Problem), vp, vp, vp, vp, vp],
        "stap_inner_products": [P(Problem), vp, vp, vp, vp, vp],
        "stap_run": [P(Problem), ctypes.c_int32, P(vp), P(vp), P(vp), P(vp), P(vp), vp, ctypes.c_size_t, vp],
        "stap_check_problem": [P(Problem)],
        "stap_cfar": [P(Problem), P(CfarParams), vp, vp, vp],
        "stap_run_noalloc": [P(Problem), ctypes.c_int32, P(vp), P(vp), P(vp), P(vp), P(vp), vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.stap_workspace_size.argtypes = [P(Problem), ctypes.c_int32]
    lib.stap_workspace_size.restype = ctypes.c_size_t
    lib.stap_status_string.argtypes = [ctypes.c_int]
    lib.stap_status_string.restype = ctypes.c_char_p
    lib.stap_version.argtypes = []
    lib.stap_version.restype = ctypes.c_char_p
    i32 = ctypes.c_int32
    lib.stap_tune_set.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.stap_tune_set.restype = ctypes.c_int
    lib.stap_tune_get.argtypes = [i32, i32, i32, i32, i32]
    lib.stap_tune_get.restype = i32
    lib.stap_use_graphs.argtypes = [i32]
    lib.stap_use_graphs.restype = None
    return lib


_lib = load_library()


def _string(code: int) -> str:
    return _lib.stap_status_string(code).decode()


def version() -> str:
    return _lib.stap_version().decode()


def tune_set(dof: int, n_steer: int, precision: str, refine: int, variant: int, kind: int = 0) -> None:
    """Select the kernel variant for a shape class (see stap_tune_set)."""
    _check(_lib.stap_tune_set(kind, dof, n_steer, PREC[precision], refine, variant), "stap_tune_set")


def use_graphs(enable: bool) -> None:
    """Replay batched stap_run launch chains from cached hipGraphs (default on)."""
    _lib.stap_use_graphs(1 if enable else 0)


def tune_get(dof: int, n_steer: int, precision: str, refine: int, kind: int = 0) -> int:
    return int(_lib.stap_tune_get(kind, dof, n_steer, PREC[precision], refine))


TAP_PHASE = {"absolute": 0, "relative": 1}


def problem(n_chan: int, n_pulse: int, n_range: int, tdof: int, n_block: int, n_steer: int,
            load_eps: float = 1e-3, precision: str = "fp32", refine_steps: int = 0,
            cube_stride_chan: int = 0, cube_stride_pulse: int = 0, guard: Optional[int] = None,
            tap_phase: str = "absolute", steer_per_bin: bool = False, n_sub: int = 1) -> Problem:
    """``guard`` None: each block trains on its own cells; an integer G >= 0:
    the block and G guard cells per side are excluded from its training.
    ``n_sub`` > 1: n_chan counts array elements, summed n_sub at a time into
    the channels the processing sees."""
    training, guard_cells = (0, 0) if guard is None else (1, int(guard))
    return Problem(n_chan, n_pulse, n_range, tdof, n_block, n_steer, load_eps, PREC[precision],
                   refine_steps, training, cube_stride_chan, cube_stride_pulse, guard_cells,
                   TAP_PHASE[tap_phase], 1 if steer_per_bin else 0, n_sub if n_sub > 1 else 0)


def check_problem(prob: Problem) -> None:
    rc = _lib.stap_check_problem(ctypes.byref(prob))
    if rc != 0:
        raise StapError(rc, "stap_check_problem")


def _ptr(t: Optional[torch.Tensor], dtype, name: str, numel: Optional[int] = None) -> Optional[int]:
    """Device address of ``t`` after checking dtype, device, layout and size.

    The C ABI takes raw pointers, so this is where a buffer that is smaller
    than the problem says is caught, before any kernel is launched."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _cube_numel(prob: Problem) -> int:
    sp = prob.cube_stride_pulse or prob.n_range
    sc = prob.cube_stride_chan or prob.n_pulse * sp
    return (prob.n_chan - 1) * sc + (prob.n_pulse - 1) * sp + prob.n_range


def _cube_ptr(prob: Problem, cube: torch.Tensor) -> int:
    if not isinstance(cube, torch.Tensor) or cube.dtype != torch.complex64 or not cube.is_cuda:
        raise TypeError("cube: expected a complex64 GPU tensor")
    if not cube.is_contiguous():
        raise ValueError("cube: must be contiguous (use the problem's strides for padding)")
    if cube.numel() < _cube_numel(prob):
        raise ValueError(f"cube: needs at least {_cube_numel(prob)} elements, got {cube.numel()}")
    return cube.data_ptr()


def _sizes(prob: Problem):
    P, D, R, B, S = prob.n_pulse, prob.dof, prob.n_range, prob.n_block, prob.n_steer
    return dict(snap=P * D * R, cov=P * B * D * D, delta=P * B,
                steer=(P if prob.steer_per_bin else 1) * S * D, w=P * B * S * D,
                info=P * B, power=P * S * R, y=P * S * R)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _check(rc: int, what: str):
    if rc != 0:
        raise StapError(rc, what)


def _empty(shape, dtype, like: torch.Tensor):
    return torch.empty(shape, dtype=dtype, device=like.device)


def doppler(prob: Problem, cube: torch.Tensor, snap: Optional[torch.Tensor] = None, stream=None):
    """Snapshots X[P][D][R] complex64 from the cube x[C][P][R]."""
    if snap is None:
        snap = _empty((prob.n_pulse, prob.dof, prob.n_range), torch.complex64, cube)
    n = _sizes(prob)
    _check(_lib.stap_doppler(ctypes.byref(prob), _cube_ptr(prob, cube), _ptr(snap, torch.complex64, "snap", n["snap"]),
                             _stream(stream)), "stap_doppler")
    return snap


def covariance(prob: Problem, snap: torch.Tensor, cov: Optional[torch.Tensor] = None,
               delta: Optional[torch.Tensor] = None, stream=None):
    """Loaded covariances cov[P][B][D][D] complex64 and delta[P][B] float32."""
    D = prob.dof
    if cov is None:
        cov = _empty((prob.n_pulse, prob.n_block, D, D), torch.complex64, snap)
    if delta is None:
        delta = _empty((prob.n_pulse, prob.n_block), torch.float32, snap)
    n = _sizes(prob)
    _check(_lib.stap_covariance(ctypes.byref(prob), _ptr(snap, torch.complex64, "snap", n["snap"]),
                                _ptr(cov, torch.complex64, "cov", n["cov"]),
                                _ptr(delta, torch.float32, "delta", n["delta"]),
                                _stream(stream)), "stap_covariance")
    return cov, delta


def solve_weights(prob: Problem, cov: torch.Tensor, steer: torch.Tensor, w: Optional[torch.Tensor] = None,
                  info: Optional[torch.Tensor] = None, stream=None):
    """Weights w[P][B][S][D] complex64 and info[P][B] int32."""
    if w is None:
        w = _empty((prob.n_pulse, prob.n_block, prob.n_steer, prob.dof), torch.complex64, cov)
    if info is None:
        info = _empty((prob.n_pulse, prob.n_block), torch.int32, cov)
    n = _sizes(prob)
    _check(_lib.stap_solve_weights(ctypes.byref(prob), _ptr(cov, torch.complex64, "cov", n["cov"]),
                                   _ptr(steer, torch.complex64, "steer", n["steer"]),
                                   _ptr(w, torch.complex64, "w", n["w"]),
                                   _ptr(info, torch.int32, "info", n["info"]), _stream(stream)),
           "stap_solve_weights")
    return w, info


def covariance_solve(prob: Problem, snap: torch.Tensor, steer: torch.Tensor, w: Optional[torch.Tensor] = None,
                     info: Optional[torch.Tensor] = None, stream=None):
    """Fused covariance -> solve: weights w[P][B][S][D] and info[P][B]."""
    if w is None:
        w = _empty((prob.n_pulse, prob.n_block, prob.n_steer, prob.dof), torch.complex64, snap)
    if info is None:
        info = _empty((prob.n_pulse, prob.n_block), torch.int32, snap)
    n = _sizes(prob)
    _check(_lib.stap_covariance_solve(ctypes.byref(prob), _ptr(snap, torch.complex64, "snap", n["snap"]),
                                      _ptr(steer, torch.complex64, "steer", n["steer"]),
                                      _ptr(w, torch.complex64, "w", n["w"]),
                                      _ptr(info, torch.int32, "info", n["info"]), _stream(stream)),
           "stap_covariance_solve")
    return w, info


def inner_products(prob: Problem, w: torch.Tensor, snap: torch.Tensor, power: Optional[torch.Tensor] = None,
                   y: Optional[torch.Tensor] = None, want_y: bool = False, stream=None):
    """Output power[P][S][R] float32 (and y complex64 if requested)."""
    if power is None:
        power = _empty((prob.n_pulse, prob.n_steer, prob.n_range), torch.float32, snap)
    if y is None and want_y:
        y = _empty((prob.n_pulse, prob.n_steer, prob.n_range), torch.complex64, snap)
    n = _sizes(prob)
    _check(_lib.stap_inner_products(ctypes.byref(prob), _ptr(w, torch.complex64, "w", n["w"]),
                                    _ptr(snap, torch.complex64, "snap", n["snap"]),
                                    _ptr(power, torch.float32, "power", n["power"]),
                                    _ptr(y, torch.complex64, "y", n["y"]), _stream(stream)),
           "stap_inner_products")
    return (power, y) if want_y else power


def cfar(prob: Problem, power: torch.Tensor, n_ref: int, n_guard: int, alpha: float,
         detect: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """CA-CFAR detection mask detect[P][S][R] uint8 from power[P][S][R]."""
    if detect is None:
        detect = _empty((prob.n_pulse, prob.n_steer, prob.n_range), torch.uint8, power)
    n = _sizes(prob)
    par = CfarParams(n_ref, n_guard, alpha)
    _check(_lib.stap_cfar(ctypes.byref(prob), ctypes.byref(par), _ptr(power, torch.float32, "power", n["power"]),
                          _ptr(detect, torch.uint8, "detect", n["power"]), _stream(stream)), "stap_cfar")
    return detect


def workspace_size(probs: Sequence[Problem]) -> int:
    arr = (Problem * len(probs))(*probs)
    return int(_lib.stap_workspace_size(arr, len(probs)))


class Runner:
    """Holds the workspace for repeated ``stap_run`` calls on fixed shapes."""

    def __init__(self, probs: Sequence[Problem], device="cuda"):
        self.probs = list(probs)
        self._arr = (Problem * len(self.probs))(*self.probs)
        nbytes = workspace_size(self.probs)
        if nbytes == 0:
            raise StapError(-1, "stap_workspace_size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)

    def run(self, cubes: Sequence[torch.Tensor], steers: Sequence[torch.Tensor],
            powers: Optional[Sequence[torch.Tensor]] = None,
            weights: Optional[Sequence[Optional[torch.Tensor]]] = None,
            info: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None):
        n = len(self.probs)
        if len(cubes) != n or len(steers) != n:
            raise ValueError("one cube and one steering set per problem")
        if powers is None:
            powers = [_empty((p.n_pulse, p.n_steer, p.n_range), torch.float32, c) for p, c in zip(self.probs, cubes)]
        for name, lst in (("powers", powers), ("weights", weights), ("info", info)):
            if lst is not None and len(lst) != n:
                raise ValueError(f"{name}: one entry per problem")
        sz = [_sizes(p) for p in self.probs]
        VP = ctypes.c_void_p * n
        cp = VP(*[_cube_ptr(p, c) for p, c in zip(self.probs, cubes)])
        sp = VP(*[_ptr(s, torch.complex64, "steer", z["steer"]) for s, z in zip(steers, sz)])
        pp = VP(*[_ptr(p, torch.float32, "power", z["power"]) for p, z in zip(powers, sz)])
        wp = (VP(*[_ptr(x, torch.complex64, "weights", z["w"]) for x, z in zip(weights, sz)])
              if weights is not None else None)
        ip = (VP(*[_ptr(x, torch.int32, "info", z["info"]) for x, z in zip(info, sz)])
              if info is not None else None)
        _check(_lib.stap_run(self._arr, n, cp, sp, pp, wp, ip, self.workspace.data_ptr(),
                             self.workspace.numel(), _stream(stream)), "stap_run")
        return powers


NOALLOC_MAX_BYTES = 256 << 20


def run_noalloc(probs: Sequence[Problem], cubes: Sequence[torch.Tensor], steers: Sequence[torch.Tensor],
                powers: Sequence[torch.Tensor], weights: Optional[Sequence[Optional[torch.Tensor]]] = None,
                info: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None) -> None:
    """stap_run_noalloc: the chain on the library's fixed scratch array, with
    caller-allocated outputs (``powers`` is required; nothing is allocated)."""
    n = len(probs)
    if len(cubes) != n or len(steers) != n or len(powers) != n:
        raise ValueError("one cube, steering set and power array per problem")
    for name, lst in (("weights", weights), ("info", info)):
        if lst is not None and len(lst) != n:
            raise ValueError(f"{name}: one entry per problem")
    arr = (Problem * n)(*probs)
    sz = [_sizes(p) for p in probs]
    VP = ctypes.c_void_p * n
    cp = VP(*[_cube_ptr(p, c) for p, c in zip(probs, cubes)])
    sp = VP(*[_ptr(s, torch.complex64, "steer", z["steer"]) for s, z in zip(steers, sz)])
    pp = VP(*[_ptr(p, torch.float32, "power", z["power"]) for p, z in zip(powers, sz)])
    wp = VP(*[_ptr(x, torch.complex64, "weights", z["w"]) for x, z in zip(weights, sz)]) if weights is not None else None
    ip = VP(*[_ptr(x, torch.int32, "info", z["info"]) for x, z in zip(info, sz)]) if info is not None else None
    _check(_lib.stap_run_noalloc(arr, n, cp, sp, pp, wp, ip, _stream(stream)), "stap_run_noalloc")


def run(probs: Sequence[Problem], cubes, steers, **kw) -> List[torch.Tensor]:
    return Runner(probs, device=cubes[0].device).run(cubes, steers, **kw)


def _apply_tuning() -> None:
    """Load the autotuner's cache (tune.py) into the library's variant table."""
    if os.environ.get("STAP_NO_TUNE"):
        return
    from . import tune
    try:
        tune.apply_cache(sys.modules[__name__])
    except (OSError, ValueError, KeyError):
        pass


_apply_tuning()
