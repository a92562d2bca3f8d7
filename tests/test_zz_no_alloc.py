"""hqa_classify_noalloc (the read-out for callers that cannot allocate device memory)
against hqa_classify on the same handles: bit-identical outputs for the MD-alone
read-out and the exact solve, on two calls in a row (the second with a smaller
instance, so the fixed scratch array holds the first call's contents), host and device
outputs, and the refusal of a read-out larger than the fixed array."""
import numpy as np
import pytest

from paper_2004_03972_amd import instances as inst

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    from paper_2004_03972_amd import hqa
    hqa.lib()
    return hqa


FIELDS = ("spins", "amb_idx", "energy", "cut", "h_eff", "code", "e_reduced")


def _outs(H, R, N, n):
    res = dict(spins=np.zeros((R, N), np.int8), amb_idx=np.zeros((R, max(n, 1)), np.int32),
               energy=np.zeros(R), cut=np.zeros(R), h_eff=np.zeros((R, max(n, 1))),
               code=np.full(R, -1, np.int64), e_reduced=np.full(R, np.nan))
    o = H.hqa_classify_out(*(res[f].ctypes.data for f in FIELDS))
    return res, o


def _compare(H, md, R, N, n, solve):
    a, oa = _outs(H, R, N, n)
    b, ob = _outs(H, R, N, n)
    H.hqa_classify(md.h, 0, n, solve, oa, H.HQA_HOST)
    H.hqa_classify_noalloc(md.h, 0, n, solve, ob, H.HQA_HOST)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f], equal_nan=True), f


def test_noalloc_readout_matches_classify(H):
    # first call: SK with real couplings (binary64 walk + exact rescoring), n = 20;
    # second: a smaller ER instance (integer walk), n = 12
    cases = [(inst.sk(600, 71), 64, 20, "bf16"), (inst.er_maxcut(300, 0.05, 72), 16, 12, "fp8")]
    for J, R, n, prec in cases:
        N = J.shape[0]
        print("noalloc read-out N", N, "R", R, "n", n, flush=True)
        md = H.MD(H.Problem(J), H.make_schedule(300, 50), R, prec, seed=5)
        md.run()
        md.sync()
        for solve in (1, 0):
            _compare(H, md, R, N, n, solve)
        md.close()


def test_noalloc_device_outputs(H):
    import torch
    J = inst.er_maxcut(200, 0.08, 73)
    N, R, n = 200, 32, 10
    md = H.MD(H.Problem(J), H.make_schedule(200, 50), R, "fp8", seed=6)
    md.run()
    md.sync()
    a, oa = _outs(H, R, N, n)
    H.hqa_classify(md.h, 0, n, 1, oa, H.HQA_HOST)
    dev = {"spins": torch.zeros((R, N), dtype=torch.int8, device="cuda"),
           "amb_idx": torch.zeros((R, n), dtype=torch.int32, device="cuda"),
           "energy": torch.zeros(R, dtype=torch.float64, device="cuda"),
           "cut": torch.zeros(R, dtype=torch.float64, device="cuda"),
           "h_eff": torch.zeros((R, n), dtype=torch.float64, device="cuda"),
           "code": torch.zeros(R, dtype=torch.int64, device="cuda"),
           "e_reduced": torch.zeros(R, dtype=torch.float64, device="cuda")}
    od = H.hqa_classify_out(*(dev[f].data_ptr() for f in FIELDS))
    H.hqa_classify_noalloc(md.h, 0, n, 1, od, H.HQA_DEVICE)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert np.array_equal(dev[f].cpu().numpy(), a[f]), f
    md.close()


def test_noalloc_refuses_oversized_readout(H):
    # spins alone, R * N bytes, exceed the fixed array: refused before any device work
    N, R = 4500, 4096
    J = inst.er_maxcut(N, 0.001, 74)
    md = H.MD(H.Problem(J), H.make_schedule(4, 2), R, "fp8", seed=7)
    md.run()
    md.sync()
    assert R * N > H.HQA_NOALLOC_SCRATCH_BYTES
    res, o = _outs(H, R, N, 0)
    with pytest.raises(H.HQAError) as e:
        H.hqa_classify_noalloc(md.h, 0, 0, 0, o, H.HQA_HOST)
    assert e.value.status == H.HQA_EUNSUPPORTED
    for bad in (2, -1):
        with pytest.raises(H.HQAError) as e:
            H.hqa_classify_noalloc(md.h, 0, 0, bad, o, H.HQA_HOST)
        assert e.value.status == H.HQA_EINVAL
    md.close()
