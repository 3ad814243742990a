"""Helpers shared by the GPU tests: tensors in and out of the device, the
binding, and error bounds derived from FP32 arithmetic."""
import numpy as np
import torch

U32 = 2.0 ** -24  # unit roundoff of FP32


def binding():
    from paper_2203_06233_amd import stap
    return stap


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def prob_of(wl, precision="fp32", refine=0, **kw):
    stap = binding()
    if wl.n_sub > 1:
        kw.setdefault("n_sub", wl.n_sub)
    return stap.problem(wl.n_chan, wl.n_pulse, wl.n_range, wl.tdof, wl.n_block, wl.n_steer,
                        load_eps=wl.load_eps, precision=precision, refine_steps=refine, **kw)


def fft_bound(cube, T, c=8.0):
    """Elementwise bound on the FP32 Doppler error: c * u * log2(P) * sum_p |h_t x|,
    arranged as X[k][t*C+c][r] (the same for every k)."""
    from oracle import stap as orc
    C, P, R = cube.shape
    W = orc.tap_windows(P, T)
    l1 = np.einsum("tp,cpr->tcr", W, np.abs(cube.astype(np.complex128)))  # [T][C][R]
    bnd = c * U32 * np.log2(P) * l1.reshape(T * C, R)
    return np.broadcast_to(bnd[None], (P, T * C, R))
