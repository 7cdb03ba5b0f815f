"""The allocation-free batched entry point against the batched entry point
with a caller workspace: identical barcodes on two calls in a row, the second
with a smaller input (the fixed scratch array keeps the first call's contents,
so this also checks that each call clears what must start at zero)."""
import numpy as np
import pytest

import oracle
from paper_2203_02527_amd import ph0, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a HIP device"
    ph0.lib()
    return t


def _both(torch, pts, offsets):
    x = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    ref = ph0.ph0_barcodes_batched_device(x, offsets)
    out = torch.full((x.shape[0], 2), -7, dtype=torch.int32, device="cuda")
    ph0.ph0_barcodes_batched_device_noalloc(x, offsets, out=out)
    torch.cuda.synchronize()
    return ref.cpu().numpy().view(np.uint32), out.cpu().numpy().view(np.uint32)


def test_noalloc_matches_workspace_call_twice_second_smaller(torch):
    pts, offsets = synth.batch_clouds(count=400, seed=31)
    print("noalloc call 1: 400 clouds, %d rows" % offsets[-1], flush=True)
    ref, got = _both(torch, pts, offsets)
    np.testing.assert_array_equal(got, ref)
    for c in range(0, 400, 37):  # and the oracle on a sample
        lo, hi = int(offsets[c]), int(offsets[c + 1])
        np.testing.assert_array_equal(got[lo:hi, 1], oracle.barcode(pts[lo:hi]).canonical)
    pts2, offsets2 = synth.batch_clouds(count=25, seed=32)
    print("noalloc call 2: 25 clouds, %d rows" % offsets2[-1], flush=True)
    ref2, got2 = _both(torch, pts2, offsets2)
    np.testing.assert_array_equal(got2, ref2)


def test_noalloc_int8_high_dimension_and_stream(torch):
    clouds = [synth.mixture_cloud(n, 16, 3, 10.0, seed=s) for s, n in enumerate([40, 300, 511, 2])]
    offsets = np.zeros(len(clouds) + 1, np.int64)
    offsets[1:] = np.cumsum([c.shape[0] for c in clouds])
    pts = np.concatenate(clouds)
    x = torch.from_numpy(pts).to("cuda")
    ref = ph0.ph0_barcodes_batched_device(x, offsets)
    stream = torch.cuda.Stream()
    out = torch.zeros((x.shape[0], 2), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ph0.ph0_barcodes_batched_device_noalloc(x, offsets, out=out, stream=stream)
    assert stream.query()  # returns after the work is complete
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_rejects_clouds_beyond_its_limits(torch):
    pts = np.zeros((600, 3), np.int16)
    x = torch.from_numpy(pts).to("cuda")
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_barcodes_batched_device_noalloc(x, np.array([0, 40, 600], np.int64))
    assert ei.value.code == -1 and "allocation-free" in str(ei.value)
