"""stap_run_noalloc (the entry point for callers that cannot allocate)
against stap_run through the C ABI: two calls in a row on the library's one
scratch array, the second with a smaller input, each bitwise equal to
stap_run on the same cubes."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import binding, dev, host, prob_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stap():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return binding()


def _outputs(wls):
    P = [torch.full((w.n_pulse, w.n_steer, w.n_range), -1.0, dtype=torch.float32, device="cuda") for w in wls]
    W = [torch.full((w.n_pulse, w.n_block, w.n_steer, w.dof), complex(np.nan, np.nan), dtype=torch.complex64,
                    device="cuda") for w in wls]
    I = [torch.full((w.n_pulse, w.n_block), -7777, dtype=torch.int32, device="cuda") for w in wls]
    return P, W, I


@pytest.mark.parametrize("precision,refine", [("fp32", 0), ("bf16", 1)])
def test_noalloc_equals_run_on_two_calls(stap, precision, refine):
    """First call: a batch of five cubes (the batched launch chain); second
    call: one smaller cube (the single-cube route)."""
    uneven = synth.uneven_batch(10)
    first = [synth.SMALL, uneven[0], uneven[1], uneven[5], uneven[8]]
    second = [synth.with_(synth.SMALL, n_range=256, n_block=16, seed=1010)]
    for wls in (first, second):
        print("noalloc call", [w.name for w in wls], precision, refine, flush=True)
        probs = [prob_of(w, precision, refine) for w in wls]
        assert stap.workspace_size(probs) <= stap.NOALLOC_MAX_BYTES
        cubes = [dev(synth.make_cube(w)) for w in wls]
        Vs = [dev(synth.steering(w)) for w in wls]
        P0, W0, I0 = _outputs(wls)
        stap.Runner(probs).run(cubes, Vs, powers=P0, weights=W0, info=I0)
        P1, W1, I1 = _outputs(wls)
        stap.run_noalloc(probs, cubes, Vs, P1, weights=W1, info=I1)
        for i in range(len(wls)):
            assert np.array_equal(host(P1[i]), host(P0[i])), i
            assert np.array_equal(host(W1[i]), host(W0[i])), i
            assert np.array_equal(host(I1[i]), host(I0[i])), i
            assert np.all(host(I1[i]) == 0)


def test_noalloc_rejects_oversized_requests(stap):
    """A cube whose scratch exceeds the fixed array is refused before any
    launch."""
    big = prob_of(synth.LARGE, "bf16", 1)
    assert stap.workspace_size([big]) > stap.NOALLOC_MAX_BYTES
    x = torch.empty(8, dtype=torch.complex64, device="cuda")
    pw = torch.empty(8, dtype=torch.float32, device="cuda")
    one = ctypes.c_void_p * 1
    rc = stap._lib.stap_run_noalloc((stap.Problem * 1)(big), 1, one(x.data_ptr()), one(x.data_ptr()),
                                    one(pw.data_ptr()), None, None, None)
    assert rc == -4
