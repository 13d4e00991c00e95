"""acom_match_noalloc: acom_match without a workspace, its scratch memory a
static device array of the library.  Called through the C ABI (ctypes) twice in
a row, the second time with a smaller input, on the scan plan; each result must
equal acom_match's on the same input (the same kernels in chunks of
acom_match_noalloc_chunk patterns; results do not depend on the chunk) bit for
bit.  A plan whose 64-pattern chunk exceeds the scratch is refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests import helpers

pytestmark = pytest.mark.gpu


def _call_noalloc(acom, gpl, pk, top_k, precision):
    n = pk.n_patterns
    out = gpl.empty_matches(n, top_k, True, "cuda")
    m = acom._Matches(*(None if out.get(k) is None else out[k].data_ptr()
                        for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated")))
    c = pk.c()
    st = acom.lib().acom_match_noalloc(gpl._h, ctypes.byref(c), int(top_k), acom.PRECISIONS[precision],
                                       ctypes.byref(m), acom._stream(None))
    return st, out


def test_match_noalloc_equals_match_twice():
    from paper_2111_00171_amd import acom
    gpl = helpers.gpu_plan(["fcc"], precisions=("fp32", "bf16"), **helpers.SCAN)
    # the chunk is the largest multiple of 64 (at most 16384) whose workspace,
    # as acom_match_workspace_size reports it, fits the 128 MiB scratch
    for prec in ("bf16", "fp32"):
        chunk = ctypes.c_int32()
        assert acom.lib().acom_match_noalloc_chunk(gpl._h, acom.PRECISIONS[prec], ctypes.byref(chunk)) == 0
        fits = [c for c in range(64, 16385, 64) if gpl.match_workspace_bytes(prec, c) <= 128 << 20]
        assert fits and chunk.value == max(fits), (prec, chunk.value)
    d = synth.make("scan")
    for precision, n in (("bf16", 3000), ("bf16", 700), ("fp32", 1000), ("fp32", 130)):
        sub = synth.subset(d, np.arange(n) * 7 % 65536)
        pk = acom.Peaks.from_host(sub)
        st, got = _call_noalloc(acom, gpl, pk, 4, precision)
        assert st == 0, acom.lib().acom_last_error()
        ref = gpl.match(pk, top_k=4, precision=precision)
        torch.cuda.synchronize()
        for k in ("zone", "phase", "bin", "mirror", "score", "phi3", "orient", "n_evaluated"):
            assert torch.equal(got[k], ref[k]), (precision, n, k)
        assert (got["zone"][:, 0] >= 0).all()


def test_match_noalloc_refuses_oversized_plan():
    from paper_2111_00171_amd import acom
    gpl = acom.Plan([acom.fcc(zones=[[0, 0, 1.0], [0, 1.0, 1.0]])],
                    acom.PlanParams(k_max=2.0, n_radial=1024, n_angular=1024, precisions=["fp32"]))
    chunk = ctypes.c_int32()
    assert acom.lib().acom_match_noalloc_chunk(gpl._h, 0, ctypes.byref(chunk)) == 0
    assert chunk.value == 0
    d = synth.subset(synth.make("small"), np.arange(8))
    st, _ = _call_noalloc(acom, gpl, acom.Peaks.from_host(d), 1, "fp32")
    assert st == 4
    assert b"128 MiB" in acom.lib().acom_last_error()
