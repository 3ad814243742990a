"""The paper's own STAP cube (Sec. 5.3: 100 pulses x 1000 channels x 30000
samples per pulse) through the C ABI: the 100-pulse Doppler step, subarray
channels formed from the 1000 elements, the paper's pulses x channels x
samples memory order, and the whole chain at full size with sampled blocks
checked against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import metrics
from oracle import stap as orc
from tests.gpu_common import U32, binding, dev, fft_bound, host, prob_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stap():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding()


def _report(tag, **vals):
    print(tag, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in vals.items()),
          flush=True)


def _sub_bound(cube, n_sub, T):
    """FFT bound of the subarray cube plus the FP32 error of summing n_sub
    elements before the transform (n_sub u sum_e |x_e| per sample, windowed)."""
    xs = orc.subarray(cube, n_sub)
    b = fft_bound(xs.astype(np.complex64), T)
    C, P, R = cube.shape
    W = orc.tap_windows(P, T)
    absum = np.abs(cube.astype(np.complex128)).reshape(C // n_sub, n_sub, P, R).sum(axis=1)
    extra = 2.0 * n_sub * U32 * np.einsum("tp,cpr->tcr", W, absum).reshape(T * (C // n_sub), R)
    return b + extra[None]


@pytest.mark.parametrize("C,R,T,rel", [(3, 75, 3, False), (8, 40, 1, False), (2, 130, 4, True), (5, 25, 3, True)])
def test_doppler_p100_parity(stap, C, R, T, rel):
    wl = synth.Workload("p100", C, 100, R, T, 1, 4, cnr_db=30.0, seed=23)
    cube = synth.make_cube(wl)
    prob = prob_of(wl, tap_phase="relative" if rel else "absolute")
    X = host(stap.doppler(prob, dev(cube)))
    Xo = orc.doppler(cube, T, relative=rel)
    bnd = fft_bound(cube, T, c=16.0)
    err = np.abs(X - Xo)
    _report("doppler-p100", C=C, R=R, T=T, rel=rel, max_ratio=float((err / bnd).max()))
    assert np.all(err <= bnd)


@pytest.mark.parametrize("P", [64, 100])
def test_doppler_subarrays(stap, P):
    """40 elements in subarrays of 8: the Doppler step of the summed
    channels, element by element."""
    wl = synth.Workload("sub", 40, P, 70, 3, 1, 4, cnr_db=30.0, seed=29, n_sub=8)
    cube = synth.make_cube(wl)
    X = host(stap.doppler(prob_of(wl), dev(cube)))
    Xo = orc.doppler(orc.subarray(cube, 8), 3)
    bnd = _sub_bound(cube, 8, 3)
    err = np.abs(X - Xo)
    _report("doppler-sub", P=P, max_ratio=float((err / bnd).max()))
    assert X.shape == (P, 15, 70)
    assert np.all(err <= bnd)


def test_pulses_outermost_layout_is_bitwise_the_same(stap):
    """The cube in the paper's pulses x channels x samples order, described
    by its strides, gives bitwise the snapshots of the channel-major cube."""
    wl = synth.Workload("layout", 30, 100, 96, 3, 1, 4, cnr_db=30.0, seed=31, n_sub=5)
    cube = synth.make_cube(wl)                       # [C][P][R]
    pcr = np.ascontiguousarray(cube.transpose(1, 0, 2))  # [P][C][R]
    X0 = host(stap.doppler(prob_of(wl), dev(cube)))
    X1 = host(stap.doppler(prob_of(wl, cube_stride_chan=96, cube_stride_pulse=30 * 96), dev(pcr)))
    assert np.array_equal(X0, X1)


@pytest.mark.parametrize("precision,refine", [("fp32", 0), ("bf16", 1)])
def test_chain_paper_cube_slice(stap, precision, refine):
    """Five training blocks (600 cells) of the paper's cube, all 1000
    elements: subarrays of 50 (D = 60), 100 pulses, 32 steering vectors,
    against the oracle."""
    wl = synth.with_(synth.PAPER, n_range=600, n_block=5)
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    prob = prob_of(wl, precision, refine)
    W = torch.empty((wl.n_pulse, wl.n_block, wl.n_steer, wl.dof), dtype=torch.complex64, device="cuda")
    info = torch.full((wl.n_pulse, wl.n_block), -7777, dtype=torch.int32, device="cuda")
    power = host(stap.run([prob], [dev(cube)], [dev(V)], weights=[W], info=[info])[0])
    W, info = host(W), host(info)
    o = orc.run(cube, V, wl.tdof, wl.n_block, wl.load_eps, n_sub=wl.n_sub)
    assert np.array_equal(info, o["info"])
    pe, we = metrics.rel_err(power, o["power"]), metrics.rel_err(W, o["W"])
    sl = metrics.sinr_loss_db(W, o["W"], V, o["R_L"])
    _report("paper-slice", prec=precision, power=pe, weights=we, sinr_max=float(sl.max()))
    if precision == "fp32":
        assert pe <= 1e-4
    assert we <= 1e-3 and sl.max() <= 0.1


def test_chain_paper_cube_full_size_sampled(stap):
    """One stap_run over the whole 100 x 1000 x 30000 cube (24 GB) in the
    paper's pulses x channels x samples order.  Three sampled training
    blocks hold the seeded scene and are checked against the oracle; the
    other cells hold device-generated complex Gaussian noise (blocks are
    independent under block training, so they do not reach the samples)."""
    wl = synth.PAPER
    C, P, R, N = wl.n_chan, wl.n_pulse, wl.n_range, wl.n_cell
    print("paper cube full size: generating", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(1005)
    cube = torch.randn((P, C, R), dtype=torch.complex64, device="cuda", generator=g)
    blocks = [0, 137, wl.n_block - 1]
    ref = {}
    for b in blocks:
        blk = synth.make_cube(wl, b * N, (b + 1) * N)           # [C][P][N]
        cube[:, :, b * N:(b + 1) * N] = dev(np.ascontiguousarray(blk.transpose(1, 0, 2)))
        ref[b] = blk
    V = synth.steering(wl)
    prob = prob_of(wl, "bf16", 1, cube_stride_chan=R, cube_stride_pulse=C * R)
    W = torch.empty((P, wl.n_block, wl.n_steer, wl.dof), dtype=torch.complex64, device="cuda")
    info = torch.full((P, wl.n_block), -7777, dtype=torch.int32, device="cuda")
    print("paper cube full size: running", flush=True)
    power = stap.run([prob], [cube], [dev(V)], weights=[W], info=[info])[0]
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    assert bool(torch.isfinite(power).all())
    worst_w, worst_sl = 0.0, 0.0
    for b in blocks:
        ob = orc.run_block(ref[b], V, wl.tdof, wl.load_eps, n_sub=wl.n_sub)
        Wb = host(W[:, b])
        we = metrics.rel_err(Wb, ob["W"][:, 0])
        sl = float(metrics.sinr_loss_db(Wb, ob["W"][:, 0], V, ob["R_L"][:, 0]).max())
        pe = metrics.rel_err(host(power[:, :, b * N:(b + 1) * N]), ob["power"])
        _report("paper-full", block=b, weights=we, sinr_max=sl, power=pe)
        worst_w, worst_sl = max(worst_w, we), max(worst_sl, sl)
        assert pe <= 1e-3
    assert worst_w <= 1e-3 and worst_sl <= 0.1
    del cube, power, W
    torch.cuda.empty_cache()
