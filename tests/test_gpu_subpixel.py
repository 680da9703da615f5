"""Sub-pixel refinement (Sec. 3.1: the last level searched again on
bilinearly interpolated descriptors, flows in quarter pixels) through the C
ABI against the oracle: the refinement state after every step, end-to-end
outputs with one and two consistency checks and sparsification, uneven
batches, edge shapes and the rejections, bit for bit.  Each GPU step prints
the case it runs first."""
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
    base = dict(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, sub_iters=2, sub_radius=2)
    base.update(kw)
    return orc.params(**base)


def _matcher(ffm, p, **kw):
    return ffm.Matcher(levels=p.levels, seed_stride=p.seed_stride, iters=p.iters, rs_radius=p.rs_radius,
                       fb_eps=p.fb_eps, seed=p.seed, sub_iters=p.sub_iters, sub_radius=p.sub_radius, **kw)


def _compare(ref, got, tag):
    for k in ref:
        if k not in got:
            continue
        g = got[k].cpu().numpy()
        if not np.array_equal(g, ref[k]):
            bad = np.argwhere(g != ref[k])
            raise AssertionError(f"{tag}: {k} differs at {len(bad)} places, first {bad[:3].tolist()}")


def _expected(orc, i1, i2, p, s=0, seed2=None):
    """Oracle outputs plus the consistency errors in 1/16 px^2."""
    if seed2 is not None:
        p = orc.params(levels=p.levels, seed_stride=p.seed_stride, iters=p.iters, rs_radius=p.rs_radius,
                       fb_eps=p.fb_eps, seed=p.seed, two_checks=1, seed2=seed2, sub_iters=p.sub_iters,
                       sub_radius=p.sub_radius)
    r = orc.match(i1, i2, p)
    if seed2 is None:
        r["fberr_f"] = orc.fb_error(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"], unit=4)
        r["fberr_b"] = orc.fb_error(r["flow_b"], r["cost_b"], r["flow_f"], r["cost_f"], unit=4)
    else:
        q = orc.params(levels=p.levels, seed_stride=p.seed_stride, iters=p.iters, rs_radius=p.rs_radius,
                       fb_eps=p.fb_eps, seed=seed2, sub_iters=p.sub_iters, sub_radius=p.sub_radius)
        alt = orc.match(i1, i2, q)
        r["fberr_f"] = orc.fb_error2(r["flow_f"], r["cost_f"], r["flow_b"], r["cost_b"], alt["flow_b"], alt["cost_b"],
                                     unit=4)
        r["fberr_b"] = orc.fb_error2(r["flow_b"], r["cost_b"], r["flow_f"], r["cost_f"], alt["flow_f"], alt["cost_f"],
                                     unit=4)
    eps2 = 16 * p.fb_eps * p.fb_eps
    assert np.array_equal(r["mask_f"], (r["fberr_f"] <= eps2).astype(np.uint8))
    if s:
        r["sparse_f"] = orc.sparsify(r["mask_f"], r["fberr_f"], s)
        r["sparse_b"] = orc.sparsify(r["mask_b"], r["fberr_b"], s)
    return r


def _run(torch, ffm, orc, i1, i2, p, tag, s=0, seed2=None, schedule=None):
    say(tag, "shape", i1.shape, "levels", p.levels, "sub_iters", p.sub_iters, "sub_radius", p.sub_radius,
        "s", s, "seed2", seed2, "schedule", schedule)
    m = _matcher(ffm, p, sparse_min=s, seed2=seed2)
    if schedule is not None:
        m.set_tuning(schedule)
    out = m._outputs(i1.shape[0], i1.shape[1])
    out.setdefault("fberr_f", torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda"))
    out.setdefault("fberr_b", torch.empty(i1.shape[:2], dtype=torch.int32, device="cuda"))
    got = m.match(torch.from_numpy(np.ascontiguousarray(i1)).cuda(), torch.from_numpy(np.ascontiguousarray(i2)).cuda(),
                  out=out)
    torch.cuda.synchronize()
    _compare(_expected(orc, i1, i2, p, s, seed2), got, tag)
    m.close()


def test_subpixel_stage_parity_config0(torch, ffm, orc):
    """Every step of both refinement iterations, both directions, equals the
    oracle's trace at the refinement level (level index = levels)."""
    i1, i2, _ = synth.config0()
    p = _prm(orc)
    L = p.levels
    trace = {}

    def tr(d, l, t, s, f, c):
        if l == L:
            trace[(d, t, s)] = (f, c)
    orc.match(i1, i2, p, trace=tr)
    m = _matcher(ffm, p)
    a, b = torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda()
    for d in (0, 1):
        steps = [(-1, 0)] + [(t, s) for t in range(p.sub_iters) for s in range(1, 8)]
        for t, s in steps:
            say("sub-pixel state dir", d, "iter", t, "step", s)
            st = m.debug_stage(a, b, ffm.STAGE_STATE, dir=d, level=L, iter=max(t, 0), step=s)
            flow, cost = ffm.state_split(st)
            rf, rc = trace[(d, t, s)]
            if not (np.array_equal(flow, rf) and np.array_equal(cost, rc)):
                bad = np.argwhere((flow != rf).any(-1) | (cost != rc))
                raise AssertionError(f"sub-pixel state dir {d} iter {t} step {s}: "
                                     f"{len(bad)} px differ, first {bad[:4].tolist()}")
    m.close()


@pytest.mark.parametrize("cfg", ["c0", "c1", "c2"])
def test_subpixel_configs(torch, ffm, orc, cfg):
    if cfg == "c0":
        i1, i2, _ = synth.config0()
        p = _prm(orc, sub_iters=1)
        _run(torch, ffm, orc, i1, i2, p, "sub-pixel c0")
    elif cfg == "c1":
        i1, i2, _ = synth.config1(seed=81)
        p = _prm(orc, levels=4, sub_radius=4)
        _run(torch, ffm, orc, i1, i2, p, "sub-pixel c1", s=7)
    else:
        i1, i2, _ = synth.config2(seed=82)
        p = _prm(orc, levels=4, fb_eps=7)
        _run(torch, ffm, orc, i1, i2, p, "sub-pixel c2 + second check + sparsify", s=4, seed2=0xBEEF)


EDGE = [
    # (W, H, C, levels, stride, radius, eps, iters, sub_iters, sub_radius)
    (63, 47, 3, 3, 3, 16, 1, 2, 2, 2),
    (1, 1, 1, 1, 1, 16, 1, 2, 1, 2),
    (2, 2, 1, 1, 1, 1, 0, 1, 3, 5),
    (5, 300, 1, 3, 2, 5, 0, 1, 1, 3),
    (300, 5, 3, 2, 1, 1, 3, 3, 2, 1),
    (129, 130, 1, 1, 5, 0, 1, 2, 1, 0),
    (97, 61, 1, 2, 3, 16, 2, 0, 2, 64),
    (2048, 6, 1, 2, 3, 3, 1, 1, 1, 2),
    (6, 2048, 1, 2, 3, 3, 1, 1, 1, 2),
]


@pytest.mark.parametrize("case", EDGE, ids=[f"{c[0]}x{c[1]}c{c[2]}L{c[3]}s{c[8]}r{c[9]}" for c in EDGE])
def test_subpixel_edge_shapes(torch, ffm, orc, case):
    W, H, C, L, st, R, eps, T, S, SR = case
    rng = np.random.default_rng(W * 11 + H * 17)
    d = (int(rng.integers(-6, 7)), int(rng.integers(-6, 7)))
    if C == 1:
        i1, i2, _ = synth.translated_pair(rng, W, H, d=d, rect=(min(16, W // 2), min(12, H // 2)), rect_d=(3, -2))
    else:
        ch = [synth.translated_pair(np.random.default_rng(k), W, H, d=d, rect=(0, 0)) for k in range(3)]
        i1 = np.stack([c[0] for c in ch], -1)
        i2 = np.stack([c[1] for c in ch], -1)
    p = _prm(orc, levels=L, seed_stride=st, iters=T, rs_radius=R, fb_eps=eps, sub_iters=S, sub_radius=SR)
    _run(torch, ffm, orc, i1, i2, p, f"sub-pixel edge {case}")


@pytest.mark.parametrize("sched", ["pipelined", "wide"])
def test_subpixel_under_other_integer_schedules(torch, ffm, orc, sched):
    """The refinement's own fixed schedule does not depend on the tuning of
    the integer levels: outputs stay the oracle's under other schedules."""
    i1, i2, _ = synth.config0()
    p = _prm(orc)
    L = p.levels
    schedule = {"pipelined": [1, 8, 0] * L + [2, 4, 0] * L, "wide": [8, 2, 0] * L + [4, 8, 0] * L}[sched]
    _run(torch, ffm, orc, i1, i2, p, f"sub-pixel schedule {sched}", schedule=schedule)


def test_subpixel_batch(torch, ffm, orc):
    """Uneven pairs in one batch: every member equals the oracle."""
    pairs = []
    for k, (w, h) in enumerate([(97, 61), (160, 120), (64, 48), (131, 67)]):
        a, b, _ = synth.translated_pair(np.random.default_rng([83, k]), w, h, d=(3 - k, 2))
        pairs.append((a, b))
    p = _prm(orc)
    m = _matcher(ffm, p, sparse_min=3)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    say("sub-pixel batch + sparsify, 4 pairs")
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        _compare(_expected(orc, a, b, p, s=3), o, f"sub-pixel batch member {k}")
    m.close()


def test_subpixel_half_pixel_shift(torch, ffm, orc):
    """A half-pixel horizontal shift (even vs odd columns of a blurred
    texture twice as wide): the device result is the oracle's, and inside
    the border it lands within half a quarter pixel of -2 on average."""
    rng = np.random.default_rng(73)
    S = synth._to_u8(synth.noise_texture(rng, 96, 2 * 128, sigma=3.0))
    j1, j2 = np.ascontiguousarray(S[:, 0::2]), np.ascontiguousarray(S[:, 1::2])
    p = _prm(orc)
    say("sub-pixel half-pixel shift", j1.shape)
    m = _matcher(ffm, p)
    got = m.match(torch.from_numpy(j1).cuda(), torch.from_numpy(j2).cuda())
    torch.cuda.synchronize()
    _compare(orc.match(j1, j2, p), got, "half-pixel shift")
    fx = got["flow_f"].cpu().numpy()[12:84, 12:116, 0].astype(np.int32)
    assert np.abs(fx + 2).mean() < 0.5
    m.close()


def test_subpixel_rejections(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    a, b = torch.from_numpy(i1).cuda(), torch.from_numpy(i2).cuda()
    say("sub-pixel rejections")
    for kw in (dict(cost="census", sub_iters=1), dict(sub_iters=17), dict(sub_iters=1, sub_radius=65),
               dict(sub_iters=1, sub_radius=-1)):
        with pytest.raises(ffm.FFError) as e:
            ffm.Matcher(levels=3, **kw)
        assert e.value.status == ffm.FF_ERR_INVALID, kw
    m = ffm.Matcher(levels=2, sub_iters=1)
    wide = torch.zeros((4, 2049), dtype=torch.uint8, device="cuda")
    with pytest.raises(ffm.FFError) as e:
        m.match(wide, wide)
    assert e.value.status == ffm.FF_ERR_INVALID
    with pytest.raises(ffm.FFError):
        m.debug_stage(a, b, ffm.STAGE_STATE, level=2, iter=1, step=1)      # iter beyond sub_iters
    m.close()
    w = ffm.Matcher(levels=3)
    with pytest.raises(ffm.FFError):
        w.debug_stage(a, b, ffm.STAGE_STATE, level=3)                      # no refinement level without the flag
    w.close()
