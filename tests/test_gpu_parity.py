"""GPU <-> oracle parity through the C ABI.  All outputs are integer, so the
bar is bit-exactness: flows, costs and masks, and every intermediate the
debug export exposes (luma, pyramid, descriptors, seed indices, search state
after every step of every level and iteration).

Each GPU step prints the case it runs (test, shape, parameters) first."""
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


def _prm(orc, levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED):
    return orc.params(levels=levels, seed_stride=seed_stride, iters=iters, rs_radius=rs_radius,
                      fb_eps=fb_eps, seed=seed)


def _matcher(ffm, p):
    return ffm.Matcher(levels=p.levels, seed_stride=p.seed_stride, iters=p.iters,
                       rs_radius=p.rs_radius, fb_eps=p.fb_eps, seed=p.seed)


def _compare_outputs(ref, got, tag):
    for k in ("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b"):
        g = got[k].cpu().numpy()
        r = ref[k]
        if not np.array_equal(g, r):
            bad = np.argwhere(g != r)
            raise AssertionError(f"{tag}: {k} differs at {len(bad)} places, first {bad[:3].tolist()}")


def _run_pair(torch, ffm, orc, i1, i2, p, tag, schedule=None):
    say(tag, "shape", i1.shape, "levels", p.levels, "stride", p.seed_stride, "R", p.rs_radius,
        "eps", p.fb_eps, "entry ff_match_pair", "schedule", schedule)
    m = _matcher(ffm, p)
    if schedule is not None:
        m.set_tuning(schedule)
    got = m.match(_dev(torch, i1), _dev(torch, i2))
    torch.cuda.synchronize()
    ref = orc.match(i1, i2, p)
    _compare_outputs(ref, got, tag)
    m.close()
    return ref


# ------------------------------------------------------ stage parity ----
@pytest.mark.parametrize("W,H,L", [(131, 67, 4), (1242, 375, 4), (64, 32, 4), (65, 33, 2), (200, 130, 6),
                                   (300, 257, 8), (97, 45, 3)])
def test_pyramid_levels(torch, ffm, orc, W, H, L):
    """Every pyramid level against the oracle, up to 8 levels: odd sizes
    whose floor dimensions drop a source row or column, sizes that are
    multiples of the block and a full 1242 x 375 frame."""
    rng = np.random.default_rng(W * 7 + H)
    i1, i2, _ = synth.translated_pair(rng, W, H, d=(3, -2), rect=(min(16, W // 2), min(12, H // 2)), rect_d=(2, 1))
    m = _matcher(ffm, _prm(orc, levels=L))
    a, b = _dev(torch, i1), _dev(torch, i2)
    for img, x in ((0, i1), (1, i2)):
        pyr = orc.pyramid(orc.gray(x), L)
        for l in range(L):
            say("pyramid", W, H, "levels", L, "image", img, "level", l)
            g = m.debug_stage(a, b, ffm.STAGE_PYRAMID, image=img, level=l).cpu().numpy()
            assert np.array_equal(g, pyr[l]), (W, H, L, img, l)
    m.close()


@pytest.mark.parametrize("schedule", ["default", "generic"])
def test_stage_parity_config0(torch, ffm, orc, schedule):
    """Every intermediate against the oracle: with the default schedule
    (software-pipelined pass; the row phase takes over the level init) and
    with the generic windowed pass (separate init kernel)."""
    i1, i2, _ = synth.config0()
    p = _prm(orc, levels=3)
    trace = {}

    def tr(d, l, t, s, f, c):
        trace[(d, l, t, s)] = (f, c)
    orc.match(i1, i2, p, trace=tr)
    m = _matcher(ffm, p)
    if schedule == "generic":
        m.set_tuning([4, 4, 0] * 6)
    a, b = _dev(torch, i1), _dev(torch, i2)
    grays = [orc.gray(i1), orc.gray(i2)]
    pyrs = [orc.pyramid(g, 3) for g in grays]
    for img in (0, 1):
        say("stage gray image", img)
        g = m.debug_stage(a, b, ffm.STAGE_GRAY, image=img).cpu().numpy()
        assert np.array_equal(g, grays[img])
        for l in range(3):
            say("stage pyramid image", img, "level", l)
            g = m.debug_stage(a, b, ffm.STAGE_PYRAMID, image=img, level=l).cpu().numpy()
            assert np.array_equal(g, pyrs[img][l]), (img, l)
            say("stage desc image", img, "level", l)
            d = m.debug_stage(a, b, ffm.STAGE_DESC, image=img, level=l).cpu().numpy()
            assert np.array_equal(d, orc.descriptors(pyrs[img][l])), (img, l)
    D = [orc.descriptors(pyrs[i][2]) for i in (0, 1)]
    for d in (0, 1):
        say("stage seeds dir", d)
        s = m.debug_stage(a, b, ffm.STAGE_SEEDS, dir=d).cpu().numpy()
        assert np.array_equal(s, orc.seed_nn(D[d], D[1 - d], 3)), d
    for d in (0, 1):
        for l in (2, 1, 0):
            steps = [(-1, 0)] + [(t, s) for t in range(2) for s in range(1, 8)]
            for t, s in steps:
                say("stage state dir", d, "level", l, "iter", t, "step", s)
                st = m.debug_stage(a, b, ffm.STAGE_STATE, dir=d, level=l, iter=max(t, 0), step=s)
                flow, cost = ffm.state_split(st)
                rf, rc = trace[(d, l, t, s)]
                if not (np.array_equal(flow, rf) and np.array_equal(cost, rc)):
                    bad = np.argwhere((flow != rf).any(-1) | (cost != rc))
                    raise AssertionError(f"state dir {d} level {l} iter {t} step {s}: "
                                         f"{len(bad)} px differ, first {bad[:4].tolist()}")
    m.close()


# -------------------------------------------------- end-to-end parity ----
def test_config0_end_to_end(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    _run_pair(torch, ffm, orc, i1, i2, _prm(orc, levels=3), "config0 128x96 gray")


def test_config1_end_to_end(torch, ffm, orc):
    i1, i2, _ = synth.config1()
    ref = _run_pair(torch, ffm, orc, i1, i2, _prm(orc, levels=4), "config1 1242x375 rgb")
    assert ref["mask_f"].mean() > 0.3


def test_config2_end_to_end(torch, ffm, orc):
    i1, i2, _ = synth.config2()
    _run_pair(torch, ffm, orc, i1, i2, _prm(orc, levels=4), "config2 1024x436 rgb")


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_staged_schedule_end_to_end(torch, ffm, orc, cfg):
    i1, i2, _ = getattr(synth, cfg)()
    _run_pair(torch, ffm, orc, i1, i2, _prm(orc, levels=4), f"{cfg} staged", schedule=_staged_schedule(4))


@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_pipelined_schedule_end_to_end(torch, ffm, orc, cfg):
    i1, i2, _ = getattr(synth, cfg)()
    _run_pair(torch, ffm, orc, i1, i2, _prm(orc, levels=4), f"{cfg} pipelined",
              schedule=[1, 4, 0] * 4 + [2, 8, 0] * 4)


EDGE_CASES = [
    # (W, H, C, levels, stride, radius, eps, iters)
    (64, 48, 1, 3, 3, 16, 1, 2),
    (63, 47, 3, 3, 3, 16, 1, 2),       # odd sizes, ragged chunks
    (65, 9, 1, 2, 3, 16, 1, 2),        # one pixel past a 64-wide chunk, few rows
    (1, 1, 1, 1, 1, 16, 1, 2),         # single pixel
    (5, 300, 1, 3, 2, 5, 0, 1),        # narrow and tall, runtime radius, eps 0
    (300, 5, 3, 2, 1, 1, 3, 3),        # wide and flat, stride 1
    (129, 130, 1, 1, 5, 0, 1, 2),      # one level, no random search
    (200, 17, 1, 5, 3, 16, 2, 1),      # coarsest level 12x1
    (8192, 8, 1, 4, 3, 16, 1, 1),      # maximum width
    (6, 8192, 1, 2, 3, 3, 1, 1),       # maximum height, runtime radius
    (97, 71, 3, 3, 4, 2, 1, 0),        # zero iterations: init only
    (512, 384, 1, 8, 3, 16, 1, 1),     # maximum levels: coarsest 4x3
    (100, 80, 3, 2, 64, 1024, 1024, 1),  # maximum stride, radius (11 trials) and eps
    (40, 30, 1, 2, 3, 4, 1, 64),       # maximum iterations
    (2000, 40, 1, 3, 3, 16, 1, 2),     # rows longer than the LDS-held part: first windows via global memory
]


STAGED = {"row": (1, 8, 1), "col": (2, 8, 1)}


def _staged_schedule(levels):
    return list(STAGED["row"]) * levels + list(STAGED["col"]) * levels


@pytest.mark.parametrize("staged", [False, True, "pipelined"], ids=["generic", "staged", "pipelined"])
@pytest.mark.parametrize("case", EDGE_CASES, ids=[f"{c[0]}x{c[1]}c{c[2]}L{c[3]}s{c[4]}R{c[5]}e{c[6]}T{c[7]}"
                                                  for c in EDGE_CASES])
def test_edge_shapes(torch, ffm, orc, case, staged):
    W, H, C, L, st, R, eps, T = case
    rng = np.random.default_rng(W * 7919 + H)
    d = (int(rng.integers(-6, 7)), int(rng.integers(-6, 7)))
    if C == 1:
        i1, i2, _ = synth.translated_pair(rng, W, H, d=d, rect=(min(16, W // 2), min(12, H // 2)), rect_d=(3, -2))
    else:
        chans = [synth.translated_pair(np.random.default_rng(k), W, H, d=d, rect=(0, 0)) for k in range(3)]
        i1 = np.stack([c[0] for c in chans], -1)
        i2 = np.stack([c[1] for c in chans], -1)
    p = _prm(orc, levels=L, seed_stride=st, iters=T, rs_radius=R, fb_eps=eps)
    sched = [4, 4, 0] * L + [4, 4, 0] * L                  # generic windowed pass
    if staged == "pipelined":
        sched = [1, 8, 0] * L + [2, 4, 0] * L
    elif staged:
        sched = _staged_schedule(L)
    _run_pair(torch, ffm, orc, i1, i2, p, f"edge {case} schedule={staged}", schedule=sched)


def test_periodic_texture_seed_ties(torch, ffm, orc):
    """A texture that repeats every 8 px makes many coarsest descriptors
    identical: seed search ties must go to the lowest linear index."""
    rng = np.random.default_rng(21)
    tile = rng.integers(0, 256, size=(8, 8), dtype=np.uint8)
    i1 = np.tile(tile, (12, 16))
    i2 = np.roll(i1, (1, 2), axis=(0, 1)).copy()
    p = _prm(orc, levels=2)
    m = _matcher(ffm, p)
    say("seed ties periodic 128x96")
    a, b = _dev(torch, i1), _dev(torch, i2)
    g = [orc.pyramid(orc.gray(x), 2)[-1] for x in (i1, i2)]
    D = [orc.descriptors(x) for x in g]
    for d in (0, 1):
        s = m.debug_stage(a, b, ffm.STAGE_SEEDS, dir=d).cpu().numpy()
        assert np.array_equal(s, orc.seed_nn(D[d], D[1 - d], 3))
    m.close()
    _run_pair(torch, ffm, orc, i1, i2, p, "periodic texture")


@pytest.mark.parametrize("kind", ["flat", "stripes", "two_level"])
def test_seed_ties_within_and_across_chunks(torch, ffm, orc, kind):
    """Whole-plane ties at one level (levels = 1, 300x200: N = 60000 pixels,
    30 database splits of 8 LDS chunks): a flat image makes every score
    equal, vertical stripes repeat every column's descriptor down the plane,
    a two-level noise image leaves few distinct descriptors.  Every seed
    must take the lowest tied linear index, exactly as the oracle."""
    rng = np.random.default_rng(31)
    if kind == "flat":
        i1 = np.full((200, 300), 77, np.uint8)
        i2 = np.full((200, 300), 77, np.uint8)
    elif kind == "stripes":
        row = rng.integers(0, 256, size=300, dtype=np.uint8)
        i1 = np.tile(row, (200, 1))
        i2 = np.roll(i1, 3, axis=1).copy()
    else:
        i1 = (rng.integers(0, 2, size=(200, 300)) * 200 + 20).astype(np.uint8)
        i2 = np.roll(i1, (2, -1), axis=(0, 1)).copy()
    p = _prm(orc, levels=1)
    m = _matcher(ffm, p)
    a, b = _dev(torch, i1), _dev(torch, i2)
    D = [orc.descriptors(orc.gray(x)) for x in (i1, i2)]
    for d in (0, 1):
        say("seed ties", kind, "dir", d)
        s = m.debug_stage(a, b, ffm.STAGE_SEEDS, dir=d).cpu().numpy()
        assert np.array_equal(s, orc.seed_nn(D[d], D[1 - d], 3)), (kind, d)
    m.close()


@pytest.mark.parametrize("kind", ["kitti", "periodic"])
def test_seed_search_full_resolution_sampled(torch, ffm, orc, kind):
    """Seed search over a whole 1242x375 level (levels = 1: Q = 51750 seeds
    against N = 465750 pixels, hundreds of database splits and LDS chunks),
    in the launch configuration the benchmark times; sampled seeds, the
    first and last ones included, against the oracle's one-query search.
    The periodic image makes most coarsest descriptors repeat, so ties
    cross split boundaries."""
    if kind == "kitti":
        i1, i2, _ = synth.config1(seed=11)
    else:
        rng = np.random.default_rng(23)
        tile = rng.integers(0, 256, size=(8, 8), dtype=np.uint8)
        i1 = np.tile(tile, (47, 156))[:375, :1242].copy()
        i2 = np.roll(i1, (3, 5), axis=(0, 1)).copy()
    p = _prm(orc, levels=1)
    m = _matcher(ffm, p)
    a, b = _dev(torch, i1), _dev(torch, i2)
    D = [orc.descriptors(orc.gray(x)) for x in (i1, i2)]
    rng = np.random.default_rng(24)
    for d in (0, 1):
        say("seed search full resolution", kind, "dir", d, "shape", i1.shape)
        s = m.debug_stage(a, b, ffm.STAGE_SEEDS, dir=d).cpu().numpy()
        nsy, nsx = s.shape
        Q = nsy * nsx
        qs = np.unique(np.concatenate([np.arange(70), np.arange(Q - 70, Q),
                                       rng.integers(0, Q, size=120)]))
        for q in qs:
            y, x = (q // nsx) * 3, (q % nsx) * 3
            assert s.reshape(-1)[q] == orc.nearest(D[d][y, x], D[1 - d]), (kind, d, int(q))
    m.close()


@pytest.mark.parametrize("kind", ["noise", "periodic"])
def test_seed_search_over_a_million_pixels(torch, ffm, orc, kind):
    """Seed search over a single 1280x900 level (levels = 1: N = 1,152,000
    pixels, 72,000 tiles of 16): past 65,536 tiles the merged key names the
    winning chunk by its first tile alone and the resolve pass scans every
    column of it.  Sampled seeds, the first and last ones included, against
    the oracle's one-query search; the periodic image makes equal scores
    cross split boundaries."""
    W, H = 1280, 900
    if kind == "noise":
        i1, i2, _ = synth.translated_pair(np.random.default_rng(41), W, H, d=(7, -5))
    else:
        rng = np.random.default_rng(42)
        tile = rng.integers(0, 256, size=(8, 8), dtype=np.uint8)
        i1 = np.tile(tile, (H // 8 + 1, W // 8 + 1))[:H, :W].copy()
        i2 = np.roll(i1, (3, 5), axis=(0, 1)).copy()
    p = _prm(orc, levels=1)
    m = _matcher(ffm, p)
    a, b = _dev(torch, i1), _dev(torch, i2)
    D = [orc.descriptors(orc.gray(x)) for x in (i1, i2)]
    assert (W * H + 15) // 16 > 65536
    rng = np.random.default_rng(43)
    for d in (0, 1):
        say("seed search over a million pixels", kind, "dir", d, "shape", i1.shape)
        s = m.debug_stage(a, b, ffm.STAGE_SEEDS, dir=d).cpu().numpy()
        nsy, nsx = s.shape
        Q = nsy * nsx
        qs = np.unique(np.concatenate([np.arange(40), np.arange(Q - 40, Q), rng.integers(0, Q, size=80)]))
        for q in qs:
            y, x = (q // nsx) * 3, (q % nsx) * 3
            assert s.reshape(-1)[q] == orc.nearest(D[d][y, x], D[1 - d]), (kind, d, int(q))
    m.close()


@pytest.mark.parametrize("C", [1, 3])
def test_unaligned_buffers(torch, ffm, orc, C):
    """Images starting at odd addresses and outputs that are only 4-byte
    (flow, cost) or 1-byte (mask) aligned take the element-wise paths of the
    ingest and output kernels; results are those of aligned buffers."""
    W, H = 131, 67
    rng = np.random.default_rng(25 + C)
    i1, i2, _ = synth.translated_pair(rng, W, H, d=(3, -2))
    if C == 3:
        i1 = np.stack([i1, np.roll(i1, 1, 0), np.roll(i1, 2, 1)], -1)
        i2 = np.stack([i2, np.roll(i2, 1, 0), np.roll(i2, 2, 1)], -1)
    p = _prm(orc, levels=3)
    m = _matcher(ffm, p)
    n = i1.size
    def odd_view(a):
        buf = torch.zeros(n + 1, dtype=torch.uint8, device="cuda")
        v = buf[1:].view(*a.shape)
        v.copy_(torch.from_numpy(np.ascontiguousarray(a)))
        return v
    a, b = odd_view(i1), odd_view(i2)
    assert a.data_ptr() % 2 == 1
    out = {}
    for k, dt, shape, off in [("flow_f", torch.int16, (H, W, 2), 2), ("flow_b", torch.int16, (H, W, 2), 2),
                              ("cost_f", torch.int32, (H, W), 1), ("cost_b", torch.int32, (H, W), 1),
                              ("mask_f", torch.uint8, (H, W), 1), ("mask_b", torch.uint8, (H, W), 1)]:
        cnt = int(np.prod(shape))
        out[k] = torch.zeros(cnt + off, dtype=dt, device="cuda")[off:].view(*shape)
    say("unaligned buffers C", C, "shape", i1.shape)
    got = m.match(a, b, out=out)
    torch.cuda.synchronize()
    _compare_outputs(orc.match(i1, i2, p), got, f"unaligned C={C}")
    m.close()


def test_identical_frames_zero_flow(torch, ffm, orc):
    rng = np.random.default_rng(22)
    img = synth._to_u8(synth.noise_texture(rng, 96, 160))
    p = _prm(orc, levels=3)
    say("identical frames 160x96")
    m = _matcher(ffm, p)
    o = m.match(_dev(torch, img), _dev(torch, img))
    torch.cuda.synchronize()
    assert int(o["flow_f"].abs().max()) == 0 and int(o["cost_f"].max()) == 0
    assert int(o["mask_f"].min()) == 1
    m.close()


# ------------------------------------------------- batch and determinism ----
def test_batch_equals_single_pairs(torch, ffm, orc):
    rng = np.random.default_rng(23)
    pairs = []
    for k in range(7):
        W, H = int(rng.integers(40, 260)), int(rng.integers(40, 200))
        d = (int(rng.integers(-20, 21)), int(rng.integers(-20, 21)))
        i1, i2, _ = synth.translated_pair(np.random.default_rng(k), W, H, d=d)
        pairs.append((i1, i2))
    p = _prm(orc, levels=3)
    m = _matcher(ffm, p)
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b in pairs]
    say("batch of 7 uneven gray pairs, entry ff_match_batch")
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k, ((a, b), o) in enumerate(zip(pairs, outs)):
        say("batch member", k, a.shape)
        ref = orc.match(a, b, p)
        _compare_outputs(ref, o, f"batch member {k}")
    # the same batch again, in a different order, reuses the workspace
    say("batch reordered")
    outs2 = m.match_batch(dev[::-1])
    torch.cuda.synchronize()
    for o1, o2 in zip(outs, outs2[::-1]):
        for key in o1:
            assert torch.equal(o1[key], o2[key])
    m.close()


def test_batch_of_config1_pairs_full_size(torch, ffm, orc):
    """The launch configuration the benchmark times: a batch of 1242x375 RGB
    pairs through ff_match_batch; two members are checked in full."""
    pairs = [synth.config1(seed=100 + k)[:2] for k in range(8)]
    p = _prm(orc, levels=4)
    m = _matcher(ffm, p)
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b in pairs]
    say("batch of 8 config1 pairs, entry ff_match_batch")
    outs = m.match_batch(dev)
    torch.cuda.synchronize()
    for k in (0, 5):
        say("check member", k)
        _compare_outputs(orc.match(pairs[k][0], pairs[k][1], p), outs[k], f"config1 batch member {k}")
    m.close()


def test_repeat_runs_are_bitwise_identical(torch, ffm, orc):
    i1, i2, _ = synth.config1(seed=7)
    p = _prm(orc, levels=4)
    m = _matcher(ffm, p)
    a, b = _dev(torch, i1), _dev(torch, i2)
    say("determinism config1 x5")
    first = m.match(a, b)
    for _ in range(4):
        o = m.match(a, b)
        for key in first:
            assert torch.equal(first[key], o[key]), key
    torch.cuda.synchronize()
    m.close()


def test_swap_invariant_on_gpu(torch, ffm, orc):
    i1, i2, _ = synth.config0()
    p = _prm(orc, levels=3)
    m = _matcher(ffm, p)
    say("swap invariant config0")
    a = m.match(_dev(torch, i1), _dev(torch, i2))
    b = m.match(_dev(torch, i2), _dev(torch, i1))
    torch.cuda.synchronize()
    assert torch.equal(a["flow_b"], b["flow_f"]) and torch.equal(a["cost_b"], b["cost_f"])
    assert torch.equal(a["mask_b"], b["mask_f"])
    m.close()


def test_invalid_arguments_are_rejected(torch, ffm):
    m = ffm.Matcher(levels=4)
    small = torch.zeros((4, 4), dtype=torch.uint8, device="cuda")
    say("invalid: too small for levels")
    with pytest.raises(ffm.FFError) as e:
        m.match(small, small)
    assert e.value.status == ffm.FF_ERR_INVALID
    say("invalid: budget")
    tight = ffm.Matcher(levels=2, hbm_budget=1024)
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(ffm.FFError) as e:
        tight.match(img, img)
    assert e.value.status == ffm.FF_ERR_BUDGET
    m.close()
    tight.close()


@pytest.mark.parametrize("opts", [{}, dict(sub_iters=2, sub_radius=3, sparse_min=5),
                                  dict(cost="census", seed2=0xBEEF, fb_eps=3, sparse_min=4)],
                         ids=["plain", "subpixel_sparse", "census_second_check_sparse"])
def test_graph_replays_match_direct_launches(torch, ffm, orc, monkeypatch, opts):
    """The second call with a geometry is captured into a hipGraph and later
    calls replay it with a freshly uploaded pair table.  Every replay, with
    eager work and synchronisation in between, must equal direct launches,
    with every option flag as well."""
    monkeypatch.setenv("FF_GRAPHS", "0")
    direct = ffm.Matcher(levels=3, **opts)
    monkeypatch.setenv("FF_GRAPHS", "1")
    graphed = ffm.Matcher(levels=3, **opts)
    sets = []
    for s in range(3):
        pairs = [synth.translated_pair(np.random.default_rng([40, s, k]), 150 + 7 * k, 90 + 5 * k,
                                       d=(k - 2, 3 - k))[:2] for k in range(4)]
        sets.append([(_dev(torch, a), _dev(torch, b)) for a, b in pairs])
    for rep in range(6):
        dev = sets[rep % 3]
        say("graph replay", opts, rep)
        g = graphed.match_batch(dev)
        scratch = torch.randn(1 << 20, device="cuda").sum()       # eager work between replays
        torch.cuda.synchronize()
        r = direct.match_batch(dev)
        torch.cuda.synchronize()
        assert float(scratch) == float(scratch)
        for o1, o2 in zip(g, r):
            for key in o1:
                assert torch.equal(o1[key], o2[key]), (rep, key)
    # single pairs through ff_match_pair as well
    a, b = sets[0][0]
    for rep in range(4):
        say("graph replay single pair", rep)
        g = graphed.match(a, b)
        r = direct.match(a, b)
        torch.cuda.synchronize()
        for key in g:
            assert torch.equal(g[key], r[key])
    direct.close()
    graphed.close()


def test_schedule_tuning_never_changes_output(torch, ffm, orc):
    pairs = [synth.config1(seed=200)[:2], synth.config0()[:2], synth.config2(seed=201)[:2]]
    pairs = [pairs[0], (np.stack([pairs[1][0]] * 3, -1), np.stack([pairs[1][1]] * 3, -1)), pairs[2]]
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b in pairs]
    m = ffm.Matcher(levels=4)
    say("default schedule")
    ref = m.match_batch(dev)
    torch.cuda.synchronize()
    r0 = orc.match(pairs[1][0], pairs[1][1], orc.params(levels=4))
    _compare_outputs(r0, ref[1], "default schedule vs oracle")
    say("autotune")
    cfg = m.autotune(dev)
    assert len(cfg) == 24 and all(cfg[i + 2] in (0, 1, 2) for i in range(0, 24, 3))
    trials = [cfg, [2, 2, 0] * 8, [8, 8, 0] * 8, [2, 8, 0, 8, 2, 0] * 4, [1, 8, 1] * 8, [1, 16, 1] * 8,
              [1, 4, 1] * 8, [2, 8, 1] * 8, [1, 8, 1, 4, 4, 0] * 4, [1, 2, 0] * 8, [1, 8, 0, 2, 4, 0] * 4,
              [1, 8, 2] * 8, [2, 2, 2] * 8, [1, 4, 2, 1, 8, 1] * 4, [2, 8, 2, 4, 4, 0] * 4]
    for trial in trials:
        say("schedule", trial)
        m.set_tuning(trial)
        got = m.match_batch(dev)
        torch.cuda.synchronize()
        for o1, o2 in zip(ref, got):
            for key in o1:
                assert torch.equal(o1[key], o2[key]), (trial, key)
    with pytest.raises(ffm.FFError):
        m.set_tuning([3, 3, 0] * 8)
    with pytest.raises(ffm.FFError):
        m.set_tuning([4, 4, 1] * 8)          # staging is not built for 256-px windows
    with pytest.raises(ffm.FFError):
        m.set_tuning([4, 4, 2] * 8)          # lockstep is a mode of the pipelined pass (1-2 chunks)
    m.close()


def test_config4_style_batch_equals_per_pair(torch, ffm, orc):
    """Uneven gray pairs (sides 96..256, translations up to 24 px) as one
    batch equal per-pair calls bit for bit; three members against the oracle."""
    pairs = synth.config4_batch(seed=4, n=96)
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b, _ in pairs]
    mb = ffm.Matcher(levels=3)
    mp = ffm.Matcher(levels=3)
    say("config4-style batch of 96")
    ob = mb.match_batch(dev)
    ob = mb.match_batch(dev)          # graph capture on the repeated geometry
    op = [mp.match(a, b) for a, b in dev]
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(ob, op)):
        for key in x:
            assert torch.equal(x[key], y[key]), (k, key)
    for k in (0, 41, 95):
        a, b, _ = pairs[k]
        _compare_outputs(orc.match(a, b, orc.params(levels=3)), ob[k], f"config4 member {k}")
    mb.close()
    mp.close()


@pytest.mark.parametrize("sched", ["default", "generic", "pipelined", "narrow"])
def test_uneven_batch_work_lists_at_edge_shapes(torch, ffm, orc, sched):
    """A batch of 36 uneven pairs -- enough for the line phases' device work
    lists -- mixing extreme shapes (2 px sides, 300 px lines, one pixel past
    a 64-px window) under several schedules: every member equals its own
    ff_match_pair call bit for bit, and four equal the oracle."""
    rng = np.random.default_rng(77)
    shapes = [(2, 2), (2, 300), (300, 2), (65, 9), (9, 65), (129, 3), (64, 64), (3, 129)]
    while len(shapes) < 36:
        shapes.append((int(rng.integers(2, 301)), int(rng.integers(2, 241))))
    pairs = []
    for k, (W, H) in enumerate(shapes):
        d = (int(rng.integers(-5, 6)), int(rng.integers(-5, 6)))
        pairs.append(synth.translated_pair(np.random.default_rng(500 + k), W, H, d=d,
                                           rect=(min(8, W // 2), min(6, H // 2)), rect_d=(2, -1))[:2])
    L = 2
    tuning = {"default": None, "generic": [4, 4, 0] * (2 * L), "pipelined": [1, 8, 0] * L + [2, 4, 0] * L,
              "narrow": [1, 2, 0] * L + [2, 2, 0] * L}[sched]
    mb, mp = ffm.Matcher(levels=L), ffm.Matcher(levels=L)
    if tuning:
        mb.set_tuning(tuning)
        mp.set_tuning(tuning)
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b in pairs]
    say("36 uneven pairs with edge shapes, schedule", sched)
    ob = mb.match_batch(dev)
    op = [mp.match(a, b) for a, b in dev]
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(ob, op)):
        for key in x:
            assert torch.equal(x[key], y[key]), (k, shapes[k], key)
    for k in (0, 2, 3, 20):
        _compare_outputs(orc.match(pairs[k][0], pairs[k][1], orc.params(levels=L)), ob[k], f"edge batch member {k}")
    mb.close()
    mp.close()
