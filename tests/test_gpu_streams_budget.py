"""Calls on one handle from two streams, and one HBM budget per handle.

Both are properties of the C ABI's runtime (include/ff.h: stream ordering,
budget), checked through the HIP path against the CPU oracle bit for bit.
Each GPU step prints the case it runs first."""
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


def _same(ref, got, tag):
    for k in ("flow_f", "cost_f", "mask_f", "flow_b", "cost_b", "mask_b"):
        g = got[k].cpu().numpy()
        if not np.array_equal(g, ref[k]):
            raise AssertionError(f"{tag}: {k} differs at {int((g != ref[k]).sum())} places")


def test_two_streams_on_one_handle(torch, ffm, orc):
    """A large batch on one stream and, right after it with no host sync, a
    batch of other pairs on a second stream: the second call reuses the
    handle's workspace and device table, so it must start after the first.
    Both batches are compared with the oracle."""
    big = [synth.config1(seed=300 + k)[:2] for k in range(4)]
    rng = np.random.default_rng(301)
    small = []
    for k in range(6):
        W, H = int(rng.integers(96, 200)), int(rng.integers(96, 160))
        d = (int(rng.integers(-12, 13)), int(rng.integers(-12, 13)))
        small.append(synth.translated_pair(np.random.default_rng(310 + k), W, H, d=d)[:2])
    m = ffm.Matcher(levels=3)
    dbig = [(_dev(torch, a), _dev(torch, b)) for a, b in big]
    dsmall = [(_dev(torch, a), _dev(torch, b)) for a, b in small]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    for rep in range(2):                        # the second round replays captured graphs
        say("two streams, round", rep, ": 4 x 1242x375 RGB on s1, then 6 small gray pairs on s2")
        with torch.cuda.stream(s1):
            ob = m.match_batch(dbig)
        with torch.cuda.stream(s2):
            osm = m.match_batch(dsmall)
        torch.cuda.synchronize()
        p = orc.params(levels=3)
        for k, (a, b) in enumerate(small):
            _same(orc.match(a, b, p), osm[k], f"round {rep} small member {k}")
        for k in (0, 3):
            _same(orc.match(big[k][0], big[k][1], p), ob[k], f"round {rep} big member {k}")
    m.close()


def test_budget_covers_arena_and_serving_lanes(torch, ffm):
    """params.hbm_budget caps the handle's own workspace and its serving
    lanes together: with a budget that holds one of the two, configuring the
    lanes releases the arena, and matching then fails with FF_ERR_BUDGET."""
    i1, i2, _ = synth.config0()                       # 128 x 96 gray
    img, img2 = _dev(torch, i1), _dev(torch, i2)
    probe = ffm.Matcher(levels=3)
    need = probe.workspace_bytes([(96, 128, 1)])
    probe.close()
    say("budget: arena then lanes, pair needs", need)
    m = ffm.Matcher(levels=3, hbm_budget=2 * need)
    m.match(img, img2)                                  # the arena fits the budget alone
    torch.cuda.synchronize()
    m.serve_config(lanes=1, lane_bytes=(3 * need) // 2)  # fits alone; the arena is released
    with pytest.raises(ffm.FFError) as e:
        m.match(img, img2)                              # arena + lanes > budget
    assert e.value.status == ffm.FF_ERR_BUDGET
    o = m.submit(img, img2, tag=7)                     # the lanes still serve
    import time
    t0 = time.time()
    got = []
    while not got and time.time() - t0 < 60:
        got = m.poll()
    assert got == [7]
    ref = probe_ref = ffm.Matcher(levels=3)
    want = ref.match(img, img2)
    torch.cuda.synchronize()
    for k in want:
        assert torch.equal(want[k], o[k]), k
    probe_ref.close()
    m.close()
    say("budget: lanes then arena")
    m = ffm.Matcher(levels=3, hbm_budget=3 * need)
    m.serve_config(lanes=2, lane_bytes=need)
    m.match(img, img2)                                  # 2 need + need fits
    torch.cuda.synchronize()
    with pytest.raises(ffm.FFError) as e:
        m.serve_config(lanes=3, lane_bytes=need + 1)   # the lanes alone exceed the budget
    assert e.value.status == ffm.FF_ERR_BUDGET
    m.close()


def test_repeated_pair_array_after_other_calls(torch, ffm, orc):
    """A batch whose ff_pair array is passed again unchanged reuses the
    validated plan and the device table; calls that replace the table in
    between (another batch, a single pair, a debug stage, a new schedule)
    must not leave it stale.  Every repeat equals the first result, and the
    first equals the oracle."""
    # 40 uneven pairs: enough for the line phases' device work lists, which
    # are part of the table and depend on the schedule
    rng = np.random.default_rng(401)
    pairs = []
    for k in range(40):
        W, H = int(rng.integers(64, 220)), int(rng.integers(64, 180))
        d = (int(rng.integers(-16, 17)), int(rng.integers(-16, 17)))
        pairs.append(synth.translated_pair(np.random.default_rng(410 + k), W, H, d=d)[:2])
    m = ffm.Matcher(levels=3)
    dev = [(_dev(torch, a), _dev(torch, b)) for a, b in pairs]
    prep = m.prepare_batch(dev)
    say("repeated pair array: first call")
    m.match_prepared(prep)
    torch.cuda.synchronize()
    first = [{k: v.clone() for k, v in o.items()} for o in prep.outs]
    p = orc.params(levels=3)
    for k in (0, 17, 39):
        _same(orc.match(pairs[k][0], pairs[k][1], p), first[k], f"member {k}")

    def again(tag):
        say("repeated pair array after", tag)
        for o in prep.outs:
            for v in o.values():
                v.fill_(-1 if v.dtype != torch.uint8 else 255)
        m.match_prepared(prep)
        torch.cuda.synchronize()
        for k, o in enumerate(prep.outs):
            for key in o:
                assert torch.equal(o[key], first[k][key]), (tag, k, key)

    again("itself (graph capture)")
    again("itself (graph replay)")
    m.match_batch(dev[::-1][:35])
    again("another batch")
    m.match(*dev[2])
    again("a single pair")
    m.debug_stage(dev[0][0], dev[0][1], ffm.STAGE_STATE, dir=1, level=1, iter=0, step=4)
    again("a debug stage")
    m.set_tuning([2, 8, 0] * 3 + [1, 4, 0] * 3)
    again("a schedule change")
    big = [(_dev(torch, a), _dev(torch, b)) for a, b in (synth.config1(seed=402)[:2],)]
    m.match_batch(big)                                   # grows the arena
    again("an arena regrowth")
    m.close()


def test_allocation_faults_return_oom_without_leaks(torch, ffm, orc, monkeypatch):
    """Injected allocation failures (ff_debug_fault_alloc, and
    FF_FAULT_ALLOC_AFTER at creation) give FF_ERR_OOM at every allocation
    site -- handle creation, workspace arena, pair table, serving lanes --
    the handle stays usable and bit-exact afterwards, and once every handle
    is destroyed the device's free memory is back where it started."""
    i1, i2, _ = synth.config0()
    a, b = _dev(torch, i1), _dev(torch, i2)
    ref = ffm.Matcher(levels=3)
    out = ref._outputs(96, 128)
    want = {k: v.clone() for k, v in ref.match(a, b, out=out).items()}
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("fault injection at creation (four pinned staging buffers)")
    for k in range(4):
        monkeypatch.setenv("FF_FAULT_ALLOC_AFTER", str(k))
        with pytest.raises(ffm.FFError) as e:
            ffm.Matcher(levels=3)
        assert e.value.status == ffm.FF_ERR_OOM, k
    monkeypatch.delenv("FF_FAULT_ALLOC_AFTER")
    say("fault injection in a call (arena, then pair table)")
    for k in range(2):
        m = ffm.Matcher(levels=3)
        m.fault_alloc(k)
        with pytest.raises(ffm.FFError) as e:
            m.match(a, b, out=out)
        assert e.value.status == ffm.FF_ERR_OOM, k
        m.fault_alloc(-1)
        got = m.match(a, b, out=out)
        torch.cuda.synchronize()
        for key in want:
            assert torch.equal(got[key], want[key]), (k, key)
        m.close()
    m = ffm.Matcher(levels=3)
    m.fault_alloc(2)
    m.match(a, b, out=out)                                # arena + table: exactly two
    torch.cuda.synchronize()
    m.close()
    say("fault injection while configuring two serving lanes")
    need = ref.workspace_bytes([(96, 128, 1)])
    for k in (0, 3, 4, 7, 9):
        m = ffm.Matcher(levels=3)
        m.fault_alloc(k)
        with pytest.raises(ffm.FFError) as e:
            m.serve_config(lanes=2, lane_bytes=need)
        assert e.value.status == ffm.FF_ERR_OOM, k
        assert m.inflight() == 0
        m.fault_alloc(-1)
        m.serve_config(lanes=2, lane_bytes=need)
        o = m.submit(a, b, tag=k)
        import time
        t0, got = time.time(), []
        while not got and time.time() - t0 < 60:
            got = m.poll()
        assert got == [k]
        for key in want:
            assert torch.equal(o[key], want[key]), (k, key)
        m.close()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("free device bytes before / after", free0, free1)
    assert abs(free0 - free1) < (2 << 20), (free0, free1)
    ref.close()


def test_failed_table_upload_never_leaves_a_stale_table(torch, ffm):
    """A batch of 17 pairs outgrows the device pair table (16 entries from
    its first allocation).  With the table regrown but the pinned staging
    buffer that the upload needs next refused, the call fails with
    FF_ERR_OOM.  The next call, with the single pair whose table the handle
    uploaded before, must upload it again into the new allocation (which
    holds nothing yet) and give the same bits as a fresh handle."""
    i1, i2, _ = synth.config0()
    a, b = _dev(torch, i1), _dev(torch, i2)
    ref = ffm.Matcher(levels=3)
    want = {k: v.clone() for k, v in ref.match(a, b).items()}
    torch.cuda.synchronize()
    m = ffm.Matcher(levels=3)
    say("two 480x360 pairs (arena room for 17 config-0 pairs, table of 16 entries)")
    big = [synth.translated_pair(np.random.default_rng(410 + k), 480, 360, d=(5, -3))[:2] for k in range(2)]
    m.match_batch([(_dev(torch, x), _dev(torch, y)) for x, y in big])
    need17 = m.workspace_bytes([(96, 128, 1)] * 17)
    need2 = m.workspace_bytes([(360, 480, 1)] * 2)
    assert need17 < need2, (need17, need2)             # no arena regrowth below
    say("one config-0 pair (the table the handle then holds)")
    out = m._outputs(96, 128)
    m.match(a, b, out=out)
    torch.cuda.synchronize()
    say("17 pairs: table regrown, staging buffer refused")
    m.fault_alloc(1)
    with pytest.raises(ffm.FFError) as e:
        m.match_batch([(a, b)] * 17, outs=[m._outputs(96, 128) for _ in range(17)])
    assert e.value.status == ffm.FF_ERR_OOM
    assert "staging" in str(e.value), str(e.value)
    m.fault_alloc(-1)
    say("the single pair again")
    for t in out.values():
        t.zero_()
    got = m.match(a, b, out=out)
    torch.cuda.synchronize()
    for key in want:
        assert torch.equal(got[key], want[key]), key
    say("and the 17-pair batch once allocations succeed")
    outs = m.match_batch([(a, b)] * 17)
    torch.cuda.synchronize()
    for o in outs:
        for key in want:
            assert torch.equal(o[key], want[key]), key
    m.close()
    ref.close()


def test_serving_cohort_that_cannot_start_stays_queued(torch, ffm):
    """A served pair whose cohort cannot start (its lane's first pair-table
    allocation refused) stays queued: ff_submit succeeds, ff_poll reports
    the error while it persists, and once allocations succeed the pair runs
    and matches a fresh handle bit for bit."""
    import time
    i1, i2, _ = synth.config0()
    a, b = _dev(torch, i1), _dev(torch, i2)
    ref = ffm.Matcher(levels=3)
    want = {k: v.clone() for k, v in ref.match(a, b).items()}
    torch.cuda.synchronize()
    m = ffm.Matcher(levels=3)
    m.serve_config(lanes=1, lane_bytes=4 * ref.workspace_bytes([(96, 128, 1)]))
    say("submit with every allocation refused")
    m.fault_alloc(0)
    o = m.submit(a, b, tag=7)
    assert m.inflight() == 1
    with pytest.raises(ffm.FFError) as e:
        m.poll()
    assert "cohort launch" in str(e.value), str(e.value)
    assert m.inflight() == 1
    m.fault_alloc(-1)
    say("poll once allocations succeed")
    t0, got = time.time(), []
    while not got and time.time() - t0 < 60:
        got = m.poll()
    assert got == [7]
    assert m.inflight() == 0
    for key in want:
        assert torch.equal(o[key], want[key]), key
    m.close()
    ref.close()


def test_failed_autotune_keeps_the_schedule(torch, ffm):
    """An autotune whose first timed run cannot allocate its workspace fails
    with FF_ERR_OOM and leaves the handle on the schedule it had; the
    handle then still matches bit for bit."""
    i1, i2, _ = synth.config0()
    a, b = _dev(torch, i1), _dev(torch, i2)
    ref = ffm.Matcher(levels=3)
    want = {k: v.clone() for k, v in ref.match(a, b).items()}
    torch.cuda.synchronize()
    m = ffm.Matcher(levels=3)
    sched = [1, 2, 0] * 3 + [2, 4, 0] * 3
    m.set_tuning(sched)
    say("autotune with every allocation refused")
    m.fault_alloc(0)
    with pytest.raises(ffm.FFError) as e:
        m.autotune([(a, b)])
    assert e.value.status == ffm.FF_ERR_OOM
    m.fault_alloc(-1)
    assert list(m.tuning()) == sched
    got = m.match(a, b)
    torch.cuda.synchronize()
    for key in want:
        assert torch.equal(got[key], want[key]), key
    m.close()
    ref.close()


def test_output_tensors_are_checked_before_any_launch(torch, ffm):
    """The binding refuses outputs whose shape, dtype, layout or device
    differ from what the library writes (the library would write past
    them); the handle then still matches bit for bit."""
    i1, i2, _ = synth.config0()
    a, b = _dev(torch, i1), _dev(torch, i2)
    m = ffm.Matcher(levels=3)
    want = {k: v.clone() for k, v in m.match(a, b).items()}
    torch.cuda.synchronize()
    say("rejected outputs")
    bad = [("flow_f", torch.empty((96, 127, 2), dtype=torch.int16, device="cuda")),
           ("cost_f", torch.empty((96, 128), dtype=torch.int16, device="cuda")),
           ("mask_b", torch.empty((128, 96), dtype=torch.uint8, device="cuda").t()),
           ("flow_b", torch.empty((96, 128, 2), dtype=torch.int16))]
    for k, t in bad:
        out = m._outputs(96, 128)
        out[k] = t
        with pytest.raises(ffm.FFError) as e:
            m.match(a, b, out=out)
        assert e.value.status == ffm.FF_ERR_INVALID and k in str(e.value), (k, str(e.value))
    got = m.match(a, b)
    torch.cuda.synchronize()
    for key in want:
        assert torch.equal(got[key], want[key]), key
    m.close()
