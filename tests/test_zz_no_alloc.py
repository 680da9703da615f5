"""The allocation-free entry point (ff_match_pair_noalloc) against the
ordinary one (ff_match_pair), through the C ABI, bit for bit: two calls in a
row on one handle, the second with a smaller pair, and a fresh handle whose
calls leave the device's free memory unchanged.  The first pair is also
checked against the CPU oracle.  Each GPU step prints its case first."""
import numpy as np
import pytest

from paper_1805_03517_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU test run without a visible GPU"
    return _t


@pytest.fixture(scope="module")
def ffm():
    from paper_1805_03517_amd import ff
    return ff


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _equal(a, b, tag):
    for k in a:
        assert a[k].shape == b[k].shape and bool((a[k] == b[k]).all()), (tag, k)


@pytest.mark.parametrize("opts", [{}, dict(sparse_min=7, seed2=0xBEEF)], ids=["plain", "sparse_second_check"])
def test_noalloc_equals_match_pair(torch, ffm, orc, opts):
    big = synth.config1(seed=5)[:2]                       # 1242 x 375 RGB, 4 levels
    small = synth.config0()[:2]                           # 128 x 96 gray
    m = ffm.Matcher(levels=4, **opts)
    ref = ffm.Matcher(levels=4, **opts)
    for tag, (a, b) in (("1242x375 RGB", big), ("128x96 gray", small)):
        say("noalloc vs match_pair,", tag, opts)
        da, db = _dev(torch, a), _dev(torch, b)
        got = m.match_noalloc(da, db)
        want = ref.match(da, db)
        torch.cuda.synchronize()
        _equal(got, want, tag)
        if tag.startswith("1242") and not opts:
            r = orc.match(a, b, orc.params(levels=4))
            for k in ("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b"):
                assert np.array_equal(got[k].cpu().numpy(), r[k]), k
    m.close()
    ref.close()


def test_noalloc_allocates_nothing_and_rejects_oversize(torch, ffm):
    a, b = (_dev(torch, v) for v in synth.config1(seed=6)[:2])
    warm = ffm.Matcher(levels=4)
    warm.match_noalloc(a, b)                              # runtime pools warmed up
    torch.cuda.synchronize()
    m = ffm.Matcher(levels=4)
    out = m._outputs(375, 1242)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("noalloc on a fresh handle, free bytes before", free0)
    for _ in range(3):
        m.match_noalloc(a, b, out=out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("free bytes after", free1)
    assert free0 - free1 < (1 << 20), (free0, free1)      # an arena for this pair would be ~60 MB
    want = warm.match(a, b)
    torch.cuda.synchronize()
    _equal(out, want, "fresh handle")
    say("noalloc rejects a pair beyond the scratch")
    huge = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    with pytest.raises(ffm.FFError) as e:
        m.match_noalloc(huge, huge)
    assert e.value.status == ffm.FF_ERR_BUDGET
    assert "allocation-free" in str(e.value)
    m.close()
    warm.close()
