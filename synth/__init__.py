"""Seeded synthetic STAP datacubes and steering sets.

Both the CPU oracle and the GPU library consume these inputs; this module holds
no step of the processing chain itself (no window, FFT, covariance, solve or
inner product), only the scene that a radar would observe:

* receiver noise, circular complex Gaussian CN(0, 1) per channel, pulse and
  range cell;
* ground clutter from ``n_scat`` point scatterers on the angle-Doppler ridge
  (normalised Doppler equal to the spatial frequency, i.e. slope 1), with
  complex amplitudes drawn independently per range cell, total power CNR per
  element per pulse;
* one target at a steering direction of the steering set, an on-bin Doppler
  at least three bins away from the ridge at that direction, and a single
  range cell, power SNR per element per pulse.

The paper states the problem as datacubes of pulses x channels x samples per
pulse (Sec. 5.3); the cube here is stored channel-major, ``x[c][p][r]`` with
the range cell fastest, as complex64.

Every range chunk of ``CHUNK`` cells is generated from its own
``SeedSequence([seed, cube_index, chunk])``, so any part of a cube can be
regenerated on its own (the parity tests sample single training blocks of the
largest workloads that way).  The scatterer geometry and the target come from
``SeedSequence([seed, cube_index])``.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional

import numpy as np

CHUNK = 256  # range cells per independently seeded chunk


@dataclass(frozen=True)
class Workload:
    """Shape and scene parameters of one datacube.

    n_chan C, n_pulse P, n_range R, tdof T (time-staggered taps), n_block B
    (training blocks along range, N = R/B cells each), n_steer S, load_eps
    (diagonal loading factor), cnr_db / snr_db per element per pulse.
    """

    name: str
    n_chan: int
    n_pulse: int
    n_range: int
    tdof: int
    n_block: int
    n_steer: int
    load_eps: float = 1e-3
    cnr_db: float = 30.0
    snr_db: float = 10.0
    n_scat: int = 32
    seed: int = 1000
    cube_index: int = 0
    target_offset: float = 0.0   # target Doppler off its bin, in bins (0 = on-bin)
    n_sub: int = 1               # array elements per subarray channel (1 = none)

    @property
    def channels(self) -> int:
        """Channels the processing sees: subarrays of n_sub elements."""
        return self.n_chan // self.n_sub

    @property
    def dof(self) -> int:
        return self.tdof * self.channels

    @property
    def n_cell(self) -> int:
        return self.n_range // self.n_block

    @property
    def sub_cpi(self) -> int:
        return self.n_pulse - self.tdof + 1

    @property
    def n_systems(self) -> int:
        return self.n_pulse * self.n_block

    @property
    def cells_dof(self) -> int:
        """Range cells x DOF of one cube (the throughput unit)."""
        return self.n_range * self.dof


# The five workloads: sizes, clutter level, seeds.
SMALL = Workload("c4-p64-r512-d12", 4, 64, 512, 3, 32, 8, cnr_db=30.0, seed=1000)
MEDIUM = Workload("c16-p128-r4096-d48", 16, 128, 4096, 3, 64, 16, cnr_db=30.0, seed=1001)
LARGE = Workload("c32-p256-r16384-d96", 32, 256, 16384, 3, 128, 32, cnr_db=40.0, seed=1002)
XLARGE = Workload("c64-p512-r32768-d192", 64, 512, 32768, 3, 256, 64, cnr_db=40.0, seed=1004)

# The paper's STAP cube (Sec. 5.3): 100 pulses x 1000 channels x 30000
# samples per pulse, the 1000 elements summed into 20 subarrays of 50; T = 3
# gives D = 60, and 250 training blocks of 120 cells = 2 D each.
PAPER = Workload("c1000s50-p100-r30000-d60", 1000, 100, 30000, 3, 250, 32, cnr_db=40.0, seed=1005, n_sub=50)

WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, LARGE, XLARGE, PAPER)}


def uneven_batch(count: int = 64, seed: int = 1003) -> List[Workload]:
    """Independent cubes of uneven size for one batched launch.

    Channels in {4, 8, 16, 32}, pulses in {32, 64, 128, 256}, range cells a
    multiple of 128 in [1024, 8192], 8..32 steering vectors, training blocks
    of 128 cells, T = 3, CNR 40 dB, SNR 10 dB.
    """
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        c = int(rng.choice([4, 8, 16, 32]))
        p = int(rng.choice([32, 64, 128, 256]))
        r = 128 * int(rng.integers(8, 65))
        s = int(rng.integers(8, 33))
        out.append(Workload(f"uneven{i}-c{c}-p{p}-r{r}", c, p, r, 3, r // 128, s,
                            cnr_db=40.0, seed=seed, cube_index=i))
    return out


@dataclass(frozen=True)
class Scene:
    scat_theta: np.ndarray   # [n_scat] spatial frequency, cycles per element
    scat_doppler: np.ndarray  # [n_scat] normalised Doppler, cycles per pulse
    target_steer: int        # index s_t into the steering set
    target_bin: int          # Doppler bin k_t (doppler = (k_t + target_offset) / P)
    target_cell: int         # range cell r_t
    target_amp: complex      # complex amplitude a, |a|^2 = SNR


def steer_theta(n_steer: int) -> np.ndarray:
    """Spatial frequencies of the steering set, evenly spaced in [-1/2, 1/2)."""
    return -0.5 + (np.arange(n_steer) + 0.5) / n_steer


def scene(wl: Workload) -> Scene:
    rng = np.random.default_rng(np.random.SeedSequence([wl.seed, wl.cube_index]))
    theta = rng.uniform(-0.5, 0.5, wl.n_scat)
    doppler = 1.0 * theta  # the clutter ridge
    s_t = int(rng.integers(wl.n_steer))
    th_t = steer_theta(wl.n_steer)[s_t]
    P = wl.n_pulse
    ridge_bin = (th_t * P) % P
    dist = np.abs(np.arange(P) - ridge_bin)
    dist = np.minimum(dist, P - dist)
    candidates = np.nonzero(dist >= 3.0)[0]
    k_t = int(rng.choice(candidates))
    r_t = int(rng.integers(wl.n_range))
    phase = rng.uniform(0.0, 2.0 * np.pi)
    amp = np.sqrt(10.0 ** (wl.snr_db / 10.0)) * np.exp(1j * phase)
    return Scene(theta, doppler, s_t, k_t, r_t, complex(amp))


def _chunk(wl: Workload, sc: Scene, chunk: int) -> np.ndarray:
    C, P = wl.n_chan, wl.n_pulse
    r0 = chunk * CHUNK
    n = min(CHUNK, wl.n_range - r0)
    rng = np.random.default_rng(np.random.SeedSequence([wl.seed, wl.cube_index, chunk]))
    noise = (rng.standard_normal((C, P, n)) + 1j * rng.standard_normal((C, P, n))) / np.sqrt(2.0)
    cnr = 10.0 ** (wl.cnr_db / 10.0)
    sig = np.sqrt(cnr / wl.n_scat / 2.0)
    alpha = sig * (rng.standard_normal((wl.n_scat, n)) + 1j * rng.standard_normal((wl.n_scat, n)))
    c = np.arange(C)[:, None, None]
    p = np.arange(P)[None, :, None]
    phase = sc.scat_theta[None, None, :] * c + sc.scat_doppler[None, None, :] * p
    basis = np.exp(2j * np.pi * phase).reshape(C * P, wl.n_scat)
    x = noise + (basis @ alpha).reshape(C, P, n)
    if r0 <= sc.target_cell < r0 + n:
        th_t = steer_theta(wl.n_steer)[sc.target_steer]
        f_t = (sc.target_bin + wl.target_offset) / P
        tgt = sc.target_amp * np.exp(2j * np.pi * (th_t * np.arange(C)[:, None] + f_t * np.arange(P)[None, :]))
        x[:, :, sc.target_cell - r0] += tgt
    return x.astype(np.complex64)


def make_cube(wl: Workload, r0: int = 0, r1: Optional[int] = None) -> np.ndarray:
    """Cube cells [r0, r1) as complex64 ``[C][P][r1 - r0]``."""
    r1 = wl.n_range if r1 is None else r1
    if not (0 <= r0 <= r1 <= wl.n_range):
        raise ValueError("range slice out of bounds")
    sc = scene(wl)
    out = np.empty((wl.n_chan, wl.n_pulse, r1 - r0), np.complex64)
    for ch in range(r0 // CHUNK, (r1 + CHUNK - 1) // CHUNK):
        a, b = ch * CHUNK, min((ch + 1) * CHUNK, wl.n_range)
        lo, hi = max(a, r0), min(b, r1)
        if lo >= hi:
            continue
        out[:, :, lo - r0:hi - r0] = _chunk(wl, sc, ch)[:, :, lo - a:hi - a]
    return out


def steering(wl: Workload) -> np.ndarray:
    """Steering set ``[S][D]`` complex64: v_s[t*C + c] = exp(j 2 pi theta_s c).

    A uniform linear array at half-wavelength spacing; the temporal part is one
    for every tap, matching on-bin targets with the window of tap t placed at
    pulses t .. t+L-1.  With subarrays of n elements the channel response is
    that of its elements, v_s[t*C' + c'] = sum_{e < n} exp(j 2 pi theta_s
    (c' n + e)), the array's own response to a plane wave from theta_s.
    """
    th = steer_theta(wl.n_steer)
    n = wl.n_sub
    spatial = np.exp(2j * np.pi * th[:, None] * n * np.arange(wl.channels)[None, :])   # [S][C/n]
    if n > 1:
        # array factor of n elements: exp(j pi theta (n-1)) sin(pi theta n) / sin(pi theta)
        s = np.sin(np.pi * th)
        af = np.where(np.abs(s) > 1e-12, np.sin(np.pi * th * n) / np.where(s == 0, 1.0, s), float(n))
        spatial = spatial * (np.exp(1j * np.pi * th * (n - 1)) * af)[:, None]
    return np.tile(spatial, (1, wl.tdof)).astype(np.complex64)


def steering_per_bin(wl: Workload) -> np.ndarray:
    """Steering set per Doppler bin ``[P][S][D]`` complex64 for taps that are
    each referenced to their own first pulse: v_{k,s}[t*C + c] =
    exp(j 2 pi k t / P) exp(j 2 pi theta_s c).  A target on bin k then carries
    the temporal phase exp(j 2 pi k t / P) across the taps.
    """
    P, T = wl.n_pulse, wl.tdof
    spatial = steering(wl)[:, :wl.channels].astype(np.complex128)        # [S][C]
    ramp = np.exp(2j * np.pi * np.outer(np.arange(P), np.arange(T)) / P)  # [P][T]
    V = ramp[:, None, :, None] * spatial[None, :, None, :]               # [P][S][T][C]
    return V.reshape(P, wl.n_steer, T * wl.channels).astype(np.complex64)


def with_(wl: Workload, **kw) -> Workload:
    return replace(wl, **kw)
