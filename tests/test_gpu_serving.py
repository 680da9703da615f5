"""Serving engine (continuous batching over concurrent lanes) through the C
ABI: every result is bit-identical to the same pair run alone, whatever
cohort it landed in; admission respects the lane workspace; misuse is
rejected."""
import time

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


def _pairs(n, seed=31):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        w, h = [(96, 80), (160, 120), (320, 240), (250, 97), (131, 211)][k % 5]
        d = (int(rng.integers(-12, 13)), int(rng.integers(-12, 13)))
        i1, i2, _ = synth.translated_pair(np.random.default_rng([seed, k]), w, h, d=d)
        if k % 3 == 0:
            i1 = np.stack([i1, np.roll(i1, 1, 0), np.roll(i1, 2, 1)], -1)
            i2 = np.stack([i2, np.roll(i2, 1, 0), np.roll(i2, 2, 1)], -1)
        out.append((i1, i2))
    return out


def _wait_all(m, tags, timeout_s=60.0):
    done = []
    t0 = time.time()
    while len(done) < len(tags):
        done += m.poll()
        if time.time() - t0 > timeout_s:
            raise AssertionError(f"serving did not finish: {len(done)}/{len(tags)}")
        time.sleep(0.0005)
    return done


def test_served_results_equal_results_alone(torch, ffm, orc):
    pairs = _pairs(24)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    alone = ffm.Matcher(levels=3)
    ref = []
    for k, (a, b) in enumerate(dev):
        say("alone", k, tuple(a.shape))
        ref.append(alone.match(a, b))
    torch.cuda.synchronize()
    served = ffm.Matcher(levels=3)
    served.serve_config(lanes=3, lane_bytes=256 << 20)
    outs = {}
    say("submit burst of 16, then 8 staggered")
    for k in range(16):
        outs[k] = served.submit(dev[k][0], dev[k][1], tag=1000 + k)
    for k in range(16, 24):
        time.sleep(0.002)
        outs[k] = served.submit(dev[k][0], dev[k][1], tag=1000 + k)
    done = _wait_all(served, list(range(24)))
    assert sorted(done) == [1000 + k for k in range(24)]
    assert served.inflight() == 0
    for k in range(24):
        for key in ref[k]:
            assert torch.equal(ref[k][key], outs[k][key]), (k, key)
    # two members against the oracle as well
    for k in (0, 7):
        r = orc.match(pairs[k][0], pairs[k][1], orc.params(levels=3))
        assert np.array_equal(outs[k]["flow_f"].cpu().numpy(), r["flow_f"])
        assert np.array_equal(outs[k]["mask_b"].cpu().numpy(), r["mask_b"])
    alone.close()
    served.close()


@pytest.mark.parametrize("opts", [dict(sub_iters=1, sub_radius=2, sparse_min=4),
                                  dict(cost="census", seed2=0xBEEF, fb_eps=7)],
                         ids=["subpixel_sparse", "census_second_check"])
def test_served_options_equal_results_alone(torch, ffm, orc, opts):
    """Served with the options on (sub-pixel refinement and sparsification;
    Census cost and the second check): every result equals the same pair
    run alone, the first one also the oracle."""
    pairs = _pairs(10, seed=41)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    alone = ffm.Matcher(levels=3, **opts)
    ref = []
    for k, (a, b) in enumerate(dev):
        say("alone", opts, k, tuple(a.shape))
        ref.append(alone.match(a, b))
    torch.cuda.synchronize()
    served = ffm.Matcher(levels=3, **opts)
    served.serve_config(lanes=2, lane_bytes=256 << 20)
    outs = {}
    say("served burst of 10", opts)
    for k in range(10):
        outs[k] = served.submit(dev[k][0], dev[k][1], tag=2000 + k)
    done = _wait_all(served, list(range(10)))
    assert sorted(done) == [2000 + k for k in range(10)]
    for k in range(10):
        for key in ref[k]:
            assert torch.equal(ref[k][key], outs[k][key]), (k, key)
    kw = dict(levels=3, fb_eps=opts.get("fb_eps", 1), sub_iters=opts.get("sub_iters", 0),
              sub_radius=opts.get("sub_radius", 2))
    if opts.get("cost") == "census":
        kw.update(cost_kind=orc.COST_CENSUS, two_checks=1, seed2=opts["seed2"])
    r = orc.match(pairs[0][0], pairs[0][1], orc.params(**kw))
    for key in ("flow_f", "cost_f", "mask_f", "flow_b", "mask_b"):
        assert np.array_equal(outs[0][key].cpu().numpy(), r[key]), key
    alone.close()
    served.close()


def test_tiny_lane_workspace_queues_fifo(torch, ffm):
    pairs = _pairs(10, seed=32)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    m = ffm.Matcher(levels=3)
    need = max(m.workspace_bytes([(a.shape[0], a.shape[1], 1 if a.dim() == 2 else 3)]) for a, _ in dev)
    m.serve_config(lanes=1, lane_bytes=need)          # one pair at a time
    say("tiny lane workspace, 10 requests")
    outs = [m.submit(a, b, tag=k) for k, (a, b) in enumerate(dev)]
    done = _wait_all(m, list(range(10)))
    assert done == list(range(10))                    # one lane, cohorts of one: FIFO order
    ref = ffm.Matcher(levels=3)
    for k, (a, b) in enumerate(dev):
        r = ref.match(a, b)
        assert torch.equal(r["flow_f"], outs[k]["flow_f"]) and torch.equal(r["mask_f"], outs[k]["mask_f"])
    m.close()
    ref.close()


def test_serving_rejections(torch, ffm):
    m = ffm.Matcher(levels=2)
    m.serve_config(lanes=2, lane_bytes=1 << 20)
    big = torch.zeros((480, 640), dtype=torch.uint8, device="cuda")
    say("oversized pair rejected")
    with pytest.raises(ffm.FFError) as e:
        m.submit(big, big, tag=1)
    assert e.value.status == ffm.FF_ERR_BUDGET
    budget = ffm.Matcher(levels=2, hbm_budget=8 << 20)
    with pytest.raises(ffm.FFError) as e:
        budget.serve_config(lanes=4, lane_bytes=4 << 20)
    assert e.value.status == ffm.FF_ERR_BUDGET
    say("reconfigure while busy")
    m.serve_config(lanes=1, lane_bytes=64 << 20)
    small = torch.zeros((240, 320), dtype=torch.uint8, device="cuda")
    for t in range(6):
        m.submit(small, small, tag=t)
    if m.inflight() > 0:
        with pytest.raises(ffm.FFError) as e:
            m.serve_config(lanes=2, lane_bytes=64 << 20)
        assert e.value.status == ffm.FF_ERR_BUSY
    _wait_all(m, list(range(6)))
    m.serve_config(lanes=2, lane_bytes=64 << 20)      # idle again: allowed
    m.close()
    budget.close()
