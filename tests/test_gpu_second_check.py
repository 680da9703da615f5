"""Second consistency check (Sec. 3.1: a match is also checked against an
inverse field matched with other parameters -- here the same search keyed
by seed2) through the C ABI, bit-exact against the oracle, alone and with
the Census cost and sparsification.  Each GPU step prints its case first."""
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


def _expected(orc, i1, i2, levels, eps, seed2, cost_kind, s=0):
    p = orc.params(levels=levels, fb_eps=eps, cost_kind=cost_kind, two_checks=1, seed2=seed2)
    r = orc.match(i1, i2, p)
    alt = orc.match(i1, i2, orc.params(levels=levels, fb_eps=eps, cost_kind=cost_kind, seed=seed2))
    r["fberr_f"] = orc.fb_error2(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"], alt["flow_b"], alt["cost_b"])
    r["fberr_b"] = orc.fb_error2(r["flow_b"], r["cost_b"], r["flow_f"], r["cost_f"], alt["flow_f"], alt["cost_f"])
    assert np.array_equal(r["mask_f"], (r["fberr_f"] <= eps * eps).astype(np.uint8))
    if s:
        r["sparse_f"] = orc.sparsify(r["mask_f"], r["fberr_f"], s)
        r["sparse_b"] = orc.sparsify(r["mask_b"], r["fberr_b"], s)
    return r


def _check(ref, got, tag):
    for k in ref:
        if k not in got:
            continue
        g = got[k].cpu().numpy()
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(g != ref[k])
            raise AssertionError(f"{tag}: {k} differs at {len(bad)} places, first {bad[:3].tolist()}")


@pytest.mark.parametrize("cfg,cost,eps,s", [("c0", "wh", 1, 0), ("c1", "wh", 1, 7), ("c2", "census", 7, 4)])
def test_second_check_configs(torch, ffm, orc, cfg, cost, eps, s):
    if cfg == "c0":
        i1, i2, _ = synth.config0()
        L = 3
    elif cfg == "c1":
        i1, i2, _ = synth.config1(seed=61)
        L = 4
    else:
        i1, i2, _ = synth.config2(seed=62)
        L = 4
    seed2 = 0xBEEF
    say("second check", cfg, "cost", cost, "eps", eps, "s", s, "shape", i1.shape)
    m = ffm.Matcher(levels=L, fb_eps=eps, cost=cost, seed2=seed2, sparse_min=s)
    out = m._outputs(i1.shape[0], i1.shape[1])
    if not s:
        out["fberr_f"] = torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda")
        out["fberr_b"] = torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda")
    got = m.match(torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda(), out=out)
    torch.cuda.synchronize()
    ck = 1 if cost == "census" else 0
    _check(_expected(orc, i1, i2, L, eps, seed2, ck, s), got, f"second check {cfg}")
    m.close()


def test_second_check_batch_and_same_key(torch, ffm, orc):
    pairs = [synth.translated_pair(np.random.default_rng([63, k]), w, h, d=(2 + k, -1))[:2]
             for k, (w, h) in enumerate([(97, 61), (160, 120), (131, 67)])]
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    m = ffm.Matcher(levels=3, seed2=0x1234)
    say("second check batch of 3")
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        _check(_expected(orc, a, b, 3, 1, 0x1234, 0), o, f"batch member {k}")
    m.close()
    # a second search with the first search's key changes nothing
    one = ffm.Matcher(levels=3)
    same = ffm.Matcher(levels=3, seed2=0x5EED)
    say("second check with the same key")
    r1 = one.match(*dev[1])
    r2 = same.match(*dev[1])
    torch.cuda.synchronize()
    for k in r1:
        assert torch.equal(r1[k], r2[k]), k
    one.close()
    same.close()


@pytest.mark.parametrize("cfg,iters2,radius2", [("c0", 1, 4), ("c0", 3, 40), ("c1", 0, 16), ("c1", 3, 8)])
def test_second_check_with_its_own_parameters(torch, ffm, orc, cfg, iters2, radius2):
    """FF_SECOND_PARAMS: the second search runs iters2 iterations per level
    at random-search radius rs_radius2 (Sec. 3.1: the inverse fields of the
    two checks come from differently parameterised searches); flows, costs,
    errors and masks bit-exact against the oracle."""
    if cfg == "c0":
        i1, i2, _ = synth.config0()
        L = 3
    else:
        i1, i2, _ = synth.config1(seed=64)
        L = 4
    seed2 = 0xBEEF
    say("second check with its own parameters", cfg, "iters2", iters2, "radius2", radius2)
    m = ffm.Matcher(levels=L, seed2=seed2, iters2=iters2, rs_radius2=radius2)
    out = m._outputs(i1.shape[0], i1.shape[1])
    out["fberr_f"] = torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda")
    out["fberr_b"] = torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda")
    got = m.match(torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda(), out=out)
    torch.cuda.synchronize()
    p = orc.params(levels=L, two_checks=1, seed2=seed2, iters2=iters2, rs_radius2=radius2)
    r = orc.match(i1, i2, p)
    alt = orc.match(i1, i2, orc.params(levels=L, seed=seed2, iters=iters2, rs_radius=radius2))
    r["fberr_f"] = orc.fb_error2(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"], alt["flow_b"], alt["cost_b"])
    r["fberr_b"] = orc.fb_error2(r["flow_b"], r["cost_b"], r["flow_f"], r["cost_f"], alt["flow_f"], alt["cost_f"])
    _check(r, got, f"second check with own parameters {cfg}")
    m.close()
    with pytest.raises(ffm.FFError):
        ffm.Matcher(levels=L, iters2=2)                # needs the second check
