"""The allocation-free entry point (spk_reconstruct_noalloc), called through
the C ABI, against spk_reconstruct: identical outputs, bit for bit, on two
calls in a row (the second on a smaller input, so the fixed scratch array
holds the first call's tables and records when the second one starts).
Also a stream long enough to be split into time chunks whose records live
in the array, and unsorted output times with duplicates (plane map in the
array)."""
import ctypes

import numpy as np
import pytest
import torch

import spkgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2412_11639_amd as m
    assert torch.cuda.is_available(), "no GPU"
    return m


def _noalloc(spk, ds, H, W, T, t_out, order, out):
    lib = spk._lib.load()
    tp = (ctypes.c_int32 * len(t_out))(*t_out)
    rc = lib.spk_reconstruct_noalloc(ds.data_ptr(), H, W, T, 1.0, tp, len(t_out),
                                     out.data_ptr(), order,
                                     torch.cuda.current_stream().cuda_stream)
    assert rc == 0, rc


@pytest.mark.parametrize("order_name", ["FSR", "SSR", "TFI", "TSR"])
def test_noalloc_equals_reconstruct_twice(spk, order_name):
    order = getattr(spk, order_name)
    rng = np.random.default_rng(21)
    cases = [(120, 200, 6000, 31), (37, 91, 1500, 32)]   # the second call is smaller
    for H, W, T, seed in cases:
        print("noalloc %s H=%d W=%d T=%d" % (order_name, H, W, T), flush=True)
        s = spkgen.gratings(H, W, T, seed=seed)
        ds = torch.from_numpy(s).cuda()
        t_out = [int(t) for t in rng.integers(0, T, 300)] + [0, T - 1, T - 1]
        ref = spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order)
        out = torch.full((len(t_out), H, W), -1.0, dtype=torch.float32, device="cuda")
        _noalloc(spk, ds, H, W, T, t_out, order, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
