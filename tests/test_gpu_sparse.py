"""3x3-block sparsification (Sec. 3.1, s from Table 3) and the consistency
error output, through the C ABI, against the oracle: bit-exact, like every
other output.  Each GPU step prints the case it runs first."""
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


def _expected(orc, i1, i2, p, s):
    r = orc.match(i1, i2, p)
    r["fberr_f"] = orc.fb_error(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"])
    r["fberr_b"] = orc.fb_error(r["flow_b"], r["cost_b"], r["flow_f"], r["cost_f"])
    r["sparse_f"] = orc.sparsify(r["mask_f"], r["fberr_f"], s)
    r["sparse_b"] = orc.sparsify(r["mask_b"], r["fberr_b"], s)
    return r


def _check(ref, got, tag):
    for k in ("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b",
              "fberr_f", "fberr_b", "sparse_f", "sparse_b"):
        g = got[k].cpu().numpy()
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(g != ref[k])
            raise AssertionError(f"{tag}: {k} differs at {len(bad)} places, first {bad[:3].tolist()}")


def _run(torch, ffm, orc, i1, i2, levels, eps, s, tag):
    say(tag, "shape", i1.shape, "levels", levels, "eps", eps, "s", s)
    p = orc.params(levels=levels, fb_eps=eps)
    m = ffm.Matcher(levels=levels, fb_eps=eps, sparse_min=s)
    got = m.match(torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda())
    torch.cuda.synchronize()
    ref = _expected(orc, i1, i2, p, s)
    _check(ref, got, tag)
    m.close()
    return ref


@pytest.mark.parametrize("cfg,eps,s", [("c0", 1, 7), ("c1", 1, 7), ("c2", 7, 4)])
def test_sparsify_configs(torch, ffm, orc, cfg, eps, s):
    if cfg == "c0":
        i1, i2, _ = synth.config0()
        L = 3
    elif cfg == "c1":
        i1, i2, _ = synth.config1(seed=12)
        L = 4
    else:
        i1, i2, _ = synth.config2(seed=13)
        L = 4
    ref = _run(torch, ffm, orc, i1, i2, L, eps, s, f"sparsify {cfg}")
    assert ref["sparse_f"].any()                   # the case selects something


@pytest.mark.parametrize("W,H", [(131, 67), (1, 1), (2, 5), (65, 9), (300, 301)])
@pytest.mark.parametrize("s", [1, 5, 9])
def test_sparsify_ragged_blocks(torch, ffm, orc, W, H, s):
    rng = np.random.default_rng(W * 31 + H)
    i1, i2, _ = synth.translated_pair(rng, W, H, d=(2, -1), rect=(min(8, W // 2), min(6, H // 2)), rect_d=(3, 2))
    L = 1 if min(W, H) < 4 else 2
    _run(torch, ffm, orc, i1, i2, L, 1, s, f"ragged {W}x{H}")


def test_sparsify_batch_equals_single(torch, ffm, orc):
    rng = np.random.default_rng(41)
    pairs = []
    for k, (w, h) in enumerate([(97, 61), (160, 120), (64, 48), (131, 67)]):
        a, b, _ = synth.translated_pair(np.random.default_rng([41, k]), w, h, d=(int(rng.integers(-5, 6)), 2))
        pairs.append((a, b))
    m = ffm.Matcher(levels=3, sparse_min=4)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    say("sparsify batch of", len(dev))
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        _check(_expected(orc, a, b, orc.params(levels=3), 4), o, f"batch member {k}")
    m.close()


def test_fberr_without_sparsify(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    m = ffm.Matcher(levels=3)
    out = m._outputs(i1.shape[0], i1.shape[1])
    out["fberr_f"] = torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda")
    say("fberr only, config0")
    m.match(torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda(), out=out)
    torch.cuda.synchronize()
    r = orc.match(i1, i2, orc.params(levels=3))
    assert np.array_equal(out["fberr_f"].cpu().numpy(),
                          orc.fb_error(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"]))
    m.close()


def test_sparsify_rejections(torch, ffm):
    say("sparsify parameter checks")
    with pytest.raises(ffm.FFError) as e:
        ffm.Matcher(levels=2, sparse_min=10)
    assert e.value.status == ffm.FF_ERR_INVALID
    m = ffm.Matcher(levels=2)
    img = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    out = m._outputs(32, 32)
    out["sparse_f"] = torch.empty((32, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(ffm.FFError) as e:
        m.match(img, img, out=out)                 # sparse output without FF_SPARSIFY
    assert e.value.status == ffm.FF_ERR_INVALID
    m.close()
    ms = ffm.Matcher(levels=2, sparse_min=3)
    out = ms._outputs(32, 32)
    del out["sparse_f"]
    with pytest.raises(ffm.FFError) as e:
        ms.match(img, img, out=out)                # sparse_fwd missing
    assert e.value.status == ffm.FF_ERR_INVALID
    ms.close()


def test_sparsify_served(torch, ffm, orc):
    import time
    rng = np.random.default_rng(43)
    pairs = [synth.translated_pair(np.random.default_rng([43, k]), 96 + 16 * k, 80, d=(3, -2))[:2] for k in range(6)]
    m = ffm.Matcher(levels=3, sparse_min=5)
    m.serve_config(lanes=2, lane_bytes=128 << 20)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    say("sparsify served, 6 requests")
    outs = [m.submit(a, b, tag=k) for k, (a, b) in enumerate(dev)]
    done, t0 = [], time.time()
    while len(done) < len(outs):
        done += m.poll()
        assert time.time() - t0 < 60
        time.sleep(0.001)
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        _check(_expected(orc, a, b, orc.params(levels=3), 5), o, f"served {k}")
    m.close()
