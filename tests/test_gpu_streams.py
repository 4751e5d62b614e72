"""Calls on several HIP streams share the library's cached output-time
tables.  A call that finds tables another stream is still uploading must
wait for that upload: its results must equal the oracle's even when the
uploading stream is held back by long (finite) work queued before it."""
import numpy as np
import pytest
import torch

import oracle
import spkgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2412_11639_amd as m
    assert torch.cuda.is_available(), "no GPU"
    return m


@pytest.mark.parametrize("order_name", ["FSR", "SSR"])
def test_tables_uploaded_on_another_stream(spk, order_name):
    order = getattr(spk, order_name)
    H, W, T = 64, 96, 1500
    s = spkgen.gratings(H, W, T, seed=71)
    ds = torch.from_numpy(s).cuda()
    rng = np.random.default_rng(4)
    t_out = [int(t) for t in rng.permutation(np.arange(3, T, 13))]
    ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order).astype(np.float32)
    # fill every cache slot with other output lists of the same length T, so
    # the slot the new list takes holds other tables until its upload lands
    for j in range(12):
        spk.reconstruct(ds, H, W, T, 1.0, [j, j + 5 * j + 1], order=spk.FSR)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    big = torch.randn(4096, 4096, device="cuda")
    prod = torch.empty_like(big)
    out_a = torch.empty((len(t_out), H, W), dtype=torch.float32, device="cuda")
    out_b = torch.full((len(t_out), H, W), -1.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    print("stream A: long matmuls, then the call that uploads the tables", flush=True)
    with torch.cuda.stream(a):
        for _ in range(40):
            torch.matmul(big, big, out=prod)
        spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order, out=out_a, stream=a)
    # stream B reuses the cached tables while A is still busy
    with torch.cuda.stream(b):
        spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order, out=out_b, stream=b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out_a.cpu().numpy(), ref)
    np.testing.assert_array_equal(out_b.cpu().numpy(), ref)
