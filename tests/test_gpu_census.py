"""Census matching cost (Sec. 3.1, the paper's Sintel cost) through the C
ABI against the oracle: Census strings of every level and image, the search
state after every step, and end-to-end outputs, bit for bit.  Each GPU step
prints the case it runs first."""
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


def _prm(orc, **kw):
    base = dict(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, cost_kind=orc.COST_CENSUS)
    base.update(kw)
    return orc.params(**base)


def _matcher(ffm, p, **kw):
    return ffm.Matcher(levels=p.levels, seed_stride=p.seed_stride, iters=p.iters, rs_radius=p.rs_radius,
                       fb_eps=p.fb_eps, seed=p.seed, cost="census", **kw)


def _compare(ref, got, tag, keys=("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b")):
    for k in keys:
        g = got[k].cpu().numpy()
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(g != ref[k])
            raise AssertionError(f"{tag}: {k} differs at {len(bad)} places, first {bad[:3].tolist()}")


def _run(torch, ffm, orc, i1, i2, p, tag, schedule=None):
    say(tag, "shape", i1.shape, "levels", p.levels, "R", p.rs_radius, "eps", p.fb_eps, "schedule", schedule)
    m = _matcher(ffm, p)
    if schedule is not None:
        m.set_tuning(schedule)
    got = m.match(torch.from_numpy(np.ascontiguousarray(i1)).cuda(), torch.from_numpy(np.ascontiguousarray(i2)).cuda())
    torch.cuda.synchronize()
    _compare(orc.match(i1, i2, p), got, tag)
    m.close()


def test_census_stage_parity_config0(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    p = _prm(orc)
    trace = {}

    def tr(d, l, t, s, f, c):
        trace[(d, l, t, s)] = (f, c)
    orc.match(i1, i2, p, trace=tr)
    m = _matcher(ffm, p)
    a, b = torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda()
    pyrs = [orc.pyramid(orc.gray(x), 3) for x in (i1, i2)]
    for img in (0, 1):
        for l in range(3):
            say("census strings image", img, "level", l)
            c = m.debug_stage(a, b, ffm.STAGE_CENSUS, image=img, level=l).cpu().numpy().view(np.uint64)
            assert np.array_equal(c, orc.census(pyrs[img][l])), (img, l)
    for d in (0, 1):
        for l in (2, 1, 0):
            steps = [(-1, 0)] + [(t, s) for t in range(2) for s in range(1, 8)]
            for t, s in steps:
                say("census state dir", d, "level", l, "iter", t, "step", s)
                st = m.debug_stage(a, b, ffm.STAGE_STATE, dir=d, level=l, iter=max(t, 0), step=s)
                flow, cost = ffm.state_split(st)
                rf, rc = trace[(d, l, t, s)]
                if not (np.array_equal(flow, rf) and np.array_equal(cost, rc)):
                    bad = np.argwhere((flow != rf).any(-1) | (cost != rc))
                    raise AssertionError(f"state dir {d} level {l} iter {t} step {s}: "
                                         f"{len(bad)} px differ, first {bad[:4].tolist()}")
    m.close()


@pytest.mark.parametrize("cfg", ["c0", "c1", "c2"])
def test_census_configs(torch, ffm, orc, cfg):
    if cfg == "c0":
        i1, i2, _ = synth.config0()
        p = _prm(orc)
    elif cfg == "c1":
        i1, i2, _ = synth.config1(seed=21)
        p = _prm(orc, levels=4)
    else:
        i1, i2, _ = synth.config2(seed=22)
        p = _prm(orc, levels=4, fb_eps=7)                 # Sintel settings of Table 3
    _run(torch, ffm, orc, i1, i2, p, f"census {cfg}")


EDGE = [
    # (W, H, C, levels, stride, radius, eps, iters)
    (63, 47, 3, 3, 3, 16, 1, 2),
    (1, 1, 1, 1, 1, 16, 1, 2),
    (5, 300, 1, 3, 2, 5, 0, 1),
    (300, 5, 3, 2, 1, 1, 3, 3),
    (129, 130, 1, 1, 5, 0, 1, 2),
    (6, 8192, 1, 2, 3, 3, 1, 1),
]


@pytest.mark.parametrize("sched", ["default", "pipelined", "wide", "lockstep", "lockstep_mixed"])
@pytest.mark.parametrize("case", EDGE, ids=[f"{c[0]}x{c[1]}c{c[2]}L{c[3]}" for c in EDGE])
def test_census_edge_shapes(torch, ffm, orc, case, sched):
    W, H, C, L, st, R, eps, T = case
    rng = np.random.default_rng(W * 7 + H * 13)
    d = (int(rng.integers(-6, 7)), int(rng.integers(-6, 7)))
    if C == 1:
        i1, i2, _ = synth.translated_pair(rng, W, H, d=d, rect=(min(16, W // 2), min(12, H // 2)), rect_d=(3, -2))
    else:
        ch = [synth.translated_pair(np.random.default_rng(k), W, H, d=d, rect=(0, 0)) for k in range(3)]
        i1 = np.stack([c[0] for c in ch], -1)
        i2 = np.stack([c[1] for c in ch], -1)
    p = _prm(orc, levels=L, seed_stride=st, iters=T, rs_radius=R, fb_eps=eps)
    # lockstep: a block's lines take their windows together (mode 2), alone or
    # mixed with free-running levels
    schedule = {"default": None, "pipelined": [1, 8, 0] * L + [2, 4, 0] * L, "wide": [8, 2, 0] * L + [4, 8, 0] * L,
                "lockstep": [1, 4, 2] * L + [1, 8, 2] * L, "lockstep_mixed": [2, 2, 2, 1, 8, 0] * L}[sched]
    _run(torch, ffm, orc, i1, i2, p, f"census edge {case}", schedule=schedule)


def test_census_batch_and_sparsify(torch, ffm, orc):
    """A batch of uneven pairs with the Census cost and the Sintel filter
    settings (eps 7, s 4): every member equals the oracle, sparse output
    included."""
    pairs = []
    for k, (w, h) in enumerate([(97, 61), (160, 120), (64, 48), (131, 67)]):
        a, b, _ = synth.translated_pair(np.random.default_rng([51, k]), w, h, d=(3 - k, 2))
        pairs.append((a, b))
    p = _prm(orc, fb_eps=7)
    m = _matcher(ffm, p, sparse_min=4)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    say("census batch + sparsify, 4 pairs")
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        r = orc.match(a, b, p)
        r["fberr_f"] = orc.fb_error(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"])
        r["sparse_f"] = orc.sparsify(r["mask_f"], r["fberr_f"], 4)
        _compare(r, o, f"census batch member {k}",
                 keys=("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b", "fberr_f", "sparse_f"))
    m.close()


def test_census_schedules_and_rejections(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    p = _prm(orc)
    m = _matcher(ffm, p)
    say("census: staged schedule rejected, autotune keeps outputs")
    with pytest.raises(ffm.FFError) as e:
        m.set_tuning([1, 8, 1] * 3 + [2, 8, 1] * 3)
    assert e.value.status == ffm.FF_ERR_INVALID
    a, b = torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda()
    m.autotune([(a, b)] * 4)
    assert all(v in (0, 2) for v in m.tuning()[2::3])        # free-running or lockstep, never staged
    got = m.match(a, b)
    torch.cuda.synchronize()
    _compare(orc.match(i1, i2, p), got, "census after autotune")
    m.close()
    w = ffm.Matcher(levels=3)
    with pytest.raises(ffm.FFError):
        w.debug_stage(a, b, ffm.STAGE_CENSUS)             # no Census strings without the flag
    w.close()
