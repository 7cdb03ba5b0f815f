"""GPU tests of the continuous-batching server."""
import numpy as np
import pytest

import oracle
from paper_2203_02527_amd import ph0, serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a HIP device"
    ph0.lib()
    return t


def _requests(count, seed, n_hi=2048):
    return synth.serving_requests(count, seed=seed, n_lo=64, n_hi=n_hi)


def test_each_result_is_the_same_alone_and_in_the_mix(torch):
    reqs = _requests(24, seed=2)
    alone = [ph0.ph0_barcodes(r) for r in reqs]
    mixed = serve.serve(reqs, rate=None, mem_budget=2 << 30, slots=4, keep_results=True)
    assert mixed["requests"] == 24
    for k, r in enumerate(reqs):
        np.testing.assert_array_equal(mixed["results"][k], alone[k], err_msg="request %d" % k)
    for k in (0, 5, 11):
        np.testing.assert_array_equal(alone[k][:, 1], oracle.barcode(reqs[k]).canonical)


def test_poisson_stream_and_latency_report(torch):
    reqs = _requests(40, seed=4, n_hi=1024)
    out = serve.serve(reqs, rate=400.0, mem_budget=1 << 30, slots=4, keep_results=True)
    assert out["requests"] == 40 and out["p99_ms"] >= out["p50_ms"] > 0
    for k in (0, 17, 39):
        np.testing.assert_array_equal(out["results"][k][:, 1], oracle.barcode(reqs[k]).canonical)


def test_admission_is_by_memory(torch):
    big = synth.mixture_cloud(4096, 16, 8, 10.0, seed=1)
    need = ph0.ph0_server_request_bytes(4096, 16, np.int8)
    with ph0.Server(need + need // 2, max_slots=4) as srv:
        # a request larger than the whole pool is refused outright
        huge = synth.mixture_cloud(8192, 16, 8, 10.0, seed=2)
        with pytest.raises(ph0.Ph0Error) as ei:
            srv.submit(huge, 99)
        assert ei.value.code == -3
        assert srv.submit(big, 1)
        # the pool has room for one such request: the next waits for memory
        assert not srv.submit(big, 2)
        got = None
        while got is None:
            got = srv.poll()
        assert got[0] == 1 and got[1] == 0
        assert srv.submit(big, 2)
        got = None
        while got is None:
            got = srv.poll()
        assert got[0] == 2
        np.testing.assert_array_equal(got[2][:, 1], oracle.barcode(big).canonical)
