"""CA-CFAR kernel against the CFAR oracle: the detection mask must match bit
for bit (both sides sum the reference cells in FP64 in the same order and
take the same FP64 test)."""
import numpy as np
import pytest
import torch

import synth
from oracle import cfar as ocfar
from oracle import stap as orc
from tests.gpu_common import binding, dev, host, prob_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stap():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding()


def _prob(P, S, R):
    return binding().problem(4, P, R, 3, 1, S)


def _map(rng, P, S, R, spikes=20):
    p = rng.exponential(1.0, (P, S, R)).astype(np.float32)
    idx = rng.integers(0, p.size, spikes)
    p.reshape(-1)[idx] = rng.uniform(5.0, 200.0, spikes).astype(np.float32)
    return p


@pytest.mark.parametrize("P,S,R,n_ref,n_guard", [
    (32, 3, 2048, 8, 2),     # one full tile per row
    (32, 5, 2049, 16, 3),    # ragged tail of one cell
    (64, 2, 5000, 1, 0),     # smallest window
    (32, 4, 4099, 64, 64),   # largest halo
    (32, 2, 7, 4, 1),        # row shorter than a window: partial windows only
    (32, 1, 131, 50, 60),    # windows wider than the row
])
def test_cfar_mask_bitwise(stap, P, S, R, n_ref, n_guard):
    rng = np.random.default_rng(P * 1000 + R)
    p = _map(rng, P, S, R)
    for pfa in (1e-2, 1e-4):
        alpha = ocfar.alpha_for_pfa(2 * n_ref, pfa)
        want, _, _ = ocfar.ca_cfar(p, n_ref, n_guard, alpha)
        got = host(stap.cfar(_prob(P, S, R), dev(p), n_ref, n_guard, alpha))
        assert got.dtype == np.uint8 and set(np.unique(got)) <= {0, 1}
        bad = np.argwhere(got.astype(bool) != want)
        assert bad.size == 0, f"{len(bad)} cells differ, first {bad[:4].tolist()}"
        print("cfar", P, S, R, n_ref, n_guard, pfa, "detections", int(want.sum()), flush=True)


def test_cfar_ties_and_constant_rows(stap):
    """Exact ties (constant rows, alpha = 1) are not detections; a spike of
    exactly alpha times the background is not, one ulp above is."""
    P, S, R = 32, 2, 300
    p = np.ones((P, S, R), np.float32)
    p[0, 0, 150] = 3.0
    p[0, 1, 150] = np.nextafter(np.float32(3.0), np.float32(4.0))
    for alpha in (1.0, 3.0):
        want, _, _ = ocfar.ca_cfar(p, 6, 2, alpha)
        got = host(stap.cfar(_prob(P, S, R), dev(p), 6, 2, alpha)).astype(bool)
        assert np.array_equal(got, want)
    got = host(stap.cfar(_prob(P, S, R), dev(p), 6, 2, 3.0)).astype(bool)
    assert not got[0, 0, 150] and got[0, 1, 150]


def test_cfar_on_stap_output(stap):
    """Detection on the chain's own output power of the 4-channel cube with
    the cells under test excluded from training: the mask equals the
    oracle's CFAR of the same power map, and the injected target is
    detected at its cell."""
    wl = synth.with_(synth.SMALL, snr_db=20.0)
    cube = synth.make_cube(wl)
    V = synth.steering(wl)
    prob = prob_of(wl, guard=2)
    power = stap.run([prob], [dev(cube)], [dev(V)])[0]
    n_ref, n_guard = 8, 2
    alpha = ocfar.alpha_for_pfa(2 * n_ref, 1e-4)
    got = host(stap.cfar(prob, power, n_ref, n_guard, alpha)).astype(bool)
    want, _, _ = ocfar.ca_cfar(host(power), n_ref, n_guard, alpha)
    assert np.array_equal(got, want)
    sc = synth.scene(wl)
    assert got[sc.target_bin, sc.target_steer, sc.target_cell]


def test_cfar_full_size_sampled_rows(stap):
    """The 256-bin x 32-steering x 16384-cell map of the largest mixed
    workload in one launch; the oracle recomputes 48 sampled rows."""
    P, S, R = 256, 32, 16384
    rng = np.random.default_rng(77)
    p = _map(rng, P, S, R, spikes=5000)
    n_ref, n_guard = 16, 2
    alpha = ocfar.alpha_for_pfa(2 * n_ref, 1e-3)
    got = host(stap.cfar(_prob(P, S, R), dev(p), n_ref, n_guard, alpha))
    rows = rng.choice(P * S, 48, replace=False)
    pr = p.reshape(P * S, R)[rows]
    want, _, _ = ocfar.ca_cfar(pr, n_ref, n_guard, alpha)
    assert np.array_equal(got.reshape(P * S, R)[rows].astype(bool), want)


def test_cfar_rejects_bad_parameters(stap):
    p = torch.zeros((32, 1, 64), dtype=torch.float32, device="cuda")
    pr = _prob(32, 1, 64)
    for n_ref, n_guard, alpha in ((0, 1, 2.0), (65, 1, 2.0), (4, -1, 2.0), (4, 65, 2.0), (4, 1, 0.0),
                                  (4, 1, float("inf")), (4, 1, float("nan"))):
        with pytest.raises(binding().StapError):
            stap.cfar(pr, p, n_ref, n_guard, alpha)
