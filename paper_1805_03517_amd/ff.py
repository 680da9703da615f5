"""ctypes binding of libff (include/ff.h): argument marshalling only.

Every step of the search runs in the HIP library; torch supplies device
memory and the current HIP stream.  Importing this module never falls back
to anything: if libff.so is missing or the device is not gfx950, the calls
raise FFError.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libff.so")

FF_OK, FF_ERR_INVALID, FF_ERR_OOM, FF_ERR_BUDGET, FF_ERR_HIP, FF_ERR_UNSUPPORTED, FF_ERR_BUSY = range(7)
FF_SPARSIFY = 1                                  # params.flags: 3x3-block sparsification
FF_COST_CENSUS = 2                               # params.flags: 7x7 Census (Hamming) matching cost
FF_SECOND_CHECK = 4                              # params.flags: second consistency check (search keyed by seed2)
FF_SUBPIXEL = 8                                  # params.flags: quarter-pixel refinement at level 0
FF_SECOND_PARAMS = 16                            # params.flags: the second search's own iters / radius
STAGE_GRAY, STAGE_PYRAMID, STAGE_DESC, STAGE_SEEDS, STAGE_STATE, STAGE_CENSUS = range(6)
INF = 2**31 - 1

# Every symbol include/ff.h declares, in declaration order.
EXPORTS = ("ff_create", "ff_match_pair", "ff_match_batch", "ff_match_pair_noalloc", "ff_destroy", "ff_last_error",
           "ff_workspace_bytes", "ff_serve_config", "ff_submit", "ff_poll", "ff_serve_inflight",
           "ff_autotune", "ff_tune_get", "ff_tune_set", "ff_profile_enable", "ff_profile_read",
           "ff_debug_stage", "ff_debug_fault_alloc")


class FFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ff status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("seed_stride", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("rs_radius", ctypes.c_int32),
                ("fb_eps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("sparse_min", ctypes.c_int32), ("seed2", ctypes.c_uint64),
                ("sub_iters", ctypes.c_int32), ("sub_radius", ctypes.c_int32),
                ("iters2", ctypes.c_int32), ("rs_radius2", ctypes.c_int32)]


class Pair(ctypes.Structure):
    _fields_ = [("img1", ctypes.c_void_p), ("img2", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("flow_fwd", ctypes.c_void_p), ("cost_fwd", ctypes.c_void_p),
                ("mask_fwd", ctypes.c_void_p), ("flow_bwd", ctypes.c_void_p),
                ("cost_bwd", ctypes.c_void_p), ("mask_bwd", ctypes.c_void_p),
                ("fberr_fwd", ctypes.c_void_p), ("sparse_fwd", ctypes.c_void_p),
                ("fberr_bwd", ctypes.c_void_p), ("sparse_bwd", ctypes.c_void_p)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


class Stage(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("image", ctypes.c_int32), ("dir", ctypes.c_int32),
                ("level", ctypes.c_int32), ("iter", ctypes.c_int32), ("step", ctypes.c_int32)]


class PreparedBatch:
    """An ff_pair array built once (Matcher.prepare_batch) and the tensors
    it points to."""

    def __init__(self, arr, n, pairs, outs):
        self.arr, self.n, self.pairs, self.outs = arr, n, pairs, outs


_lib = None


def lib():
    """Load libff.so (raises FFError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FFError(FF_ERR_UNSUPPORTED,
                          f"{LIB_PATH} is missing: build it with python -m paper_1805_03517_amd.build")
        l = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        l.ff_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(vp)]
        l.ff_create.restype = ctypes.c_int
        l.ff_match_pair.argtypes = [vp, ctypes.POINTER(Pair), vp]
        l.ff_match_pair.restype = ctypes.c_int
        l.ff_match_batch.argtypes = [vp, ctypes.POINTER(Pair), i32, vp]
        l.ff_match_batch.restype = ctypes.c_int
        l.ff_match_pair_noalloc.argtypes = [vp, ctypes.POINTER(Pair), vp]
        l.ff_match_pair_noalloc.restype = ctypes.c_int
        l.ff_destroy.argtypes = [vp]
        l.ff_destroy.restype = None
        l.ff_last_error.argtypes = [vp]
        l.ff_last_error.restype = ctypes.c_char_p
        l.ff_workspace_bytes.argtypes = [vp, ctypes.POINTER(Pair), i32]
        l.ff_workspace_bytes.restype = ctypes.c_uint64
        l.ff_serve_config.argtypes = [vp, i32, ctypes.c_uint64]
        l.ff_serve_config.restype = ctypes.c_int
        l.ff_submit.argtypes = [vp, ctypes.POINTER(Pair), ctypes.c_uint64, vp]
        l.ff_submit.restype = ctypes.c_int
        l.ff_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32]
        l.ff_poll.restype = i32
        l.ff_serve_inflight.argtypes = [vp]
        l.ff_serve_inflight.restype = i32
        l.ff_autotune.argtypes = [vp, ctypes.POINTER(Pair), i32, vp]
        l.ff_autotune.restype = ctypes.c_int
        l.ff_tune_get.argtypes = [vp, ctypes.POINTER(i32), i32]
        l.ff_tune_get.restype = i32
        l.ff_tune_set.argtypes = [vp, ctypes.POINTER(i32), i32]
        l.ff_tune_set.restype = ctypes.c_int
        l.ff_profile_enable.argtypes = [vp, i32]
        l.ff_profile_enable.restype = ctypes.c_int
        l.ff_profile_read.argtypes = [vp, ctypes.POINTER(ProfileEntry), i32]
        l.ff_profile_read.restype = i32
        l.ff_debug_stage.argtypes = [vp, ctypes.POINTER(Pair), ctypes.POINTER(Stage), vp, vp]
        l.ff_debug_stage.restype = ctypes.c_int
        l.ff_debug_fault_alloc.argtypes = [vp, ctypes.c_int64]
        l.ff_debug_fault_alloc.restype = ctypes.c_int
        _lib = l
    return _lib


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Matcher:
    """One libff handle.  Images are torch uint8 tensors on the device,
    [H, W] (gray) or [H, W, 3] (RGB), contiguous."""

    def __init__(self, levels=4, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED,
                 hbm_budget=0, device=0, sparse_min=0, cost="wh", seed2=None, sub_iters=0, sub_radius=2,
                 iters2=None, rs_radius2=None):
        """sparse_min > 0 turns on the 3x3-block sparsification (FF_SPARSIFY)
        with that minimum number of matches s; outputs then include
        sparse_f / sparse_b and the consistency errors fberr_f / fberr_b.
        cost: "wh" (descriptor SAD) or "census" (7x7 Census Hamming distance,
        FF_COST_CENSUS).  seed2 (not None) adds the second consistency check
        against the inverse fields of a search keyed by seed2 (FF_SECOND_CHECK).
        sub_iters > 0 adds that many quarter-pixel refinement iterations at
        level 0 (FF_SUBPIXEL, random-search radius sub_radius quarter pixels);
        flows are then in quarter pixels and fberr in 1/16 px^2.  iters2 /
        rs_radius2 (with seed2) give the second search its own iterations and
        random-search radius (FF_SECOND_PARAMS); None = the first search's."""
        if cost not in ("wh", "census"):
            raise FFError(FF_ERR_INVALID, "cost must be 'wh' or 'census'")
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        self.sparse = sparse_min > 0
        second = iters2 is not None or rs_radius2 is not None
        flags = ((FF_SPARSIFY if self.sparse else 0) | (FF_COST_CENSUS if cost == "census" else 0) |
                 (FF_SECOND_CHECK if seed2 is not None else 0) | (FF_SUBPIXEL if sub_iters > 0 else 0) |
                 (FF_SECOND_PARAMS if second else 0))
        self.params = Params(levels, seed_stride, iters, rs_radius, fb_eps, seed, hbm_budget, flags, sparse_min,
                             seed2 if seed2 is not None else 0, sub_iters, sub_radius,
                             iters if iters2 is None else iters2, rs_radius if rs_radius2 is None else rs_radius2)
        h = ctypes.c_void_p()
        st = lib().ff_create(ctypes.byref(self.params), device, ctypes.byref(h))
        if st != FF_OK:
            why = {FF_ERR_INVALID: "invalid parameters or device index", FF_ERR_UNSUPPORTED: "the device is not gfx950",
                   FF_ERR_OOM: "pinned staging memory could not be allocated"}.get(st, "HIP error")
            raise FFError(st, "ff_create failed: " + why)
        self._h = h

    # -- helpers --------------------------------------------------------
    def _check(self, st):
        if st != FF_OK:
            msg = lib().ff_last_error(self._h)
            raise FFError(st, msg.decode() if msg else "")

    def _outputs(self, H, W, bwd=True, cost=True):
        t = self._torch
        d = self.device
        o = {"flow_f": t.empty((H, W, 2), dtype=t.int16, device=d),
             "mask_f": t.empty((H, W), dtype=t.uint8, device=d)}
        if cost:
            o["cost_f"] = t.empty((H, W), dtype=t.int32, device=d)
        if bwd:
            o["flow_b"] = t.empty((H, W, 2), dtype=t.int16, device=d)
            o["mask_b"] = t.empty((H, W), dtype=t.uint8, device=d)
            if cost:
                o["cost_b"] = t.empty((H, W), dtype=t.int32, device=d)
        if self.sparse:
            for sfx in ("f", "b") if bwd else ("f",):
                o["sparse_" + sfx] = t.empty((H, W), dtype=t.uint8, device=d)
                o["fberr_" + sfx] = t.empty((H, W), dtype=t.int32, device=d)
        return o

    @staticmethod
    def _ptr(o, k):
        v = o.get(k)
        return ctypes.c_void_p(v.data_ptr()) if v is not None else None

    # output name -> (dtype name, trailing shape after [H, W])
    _OUT_SPEC = {"flow_f": ("int16", (2,)), "flow_b": ("int16", (2,)), "cost_f": ("int32", ()),
                 "cost_b": ("int32", ()), "mask_f": ("uint8", ()), "mask_b": ("uint8", ()),
                 "fberr_f": ("int32", ()), "fberr_b": ("int32", ()), "sparse_f": ("uint8", ()),
                 "sparse_b": ("uint8", ())}

    def _pair(self, img1, img2, out):
        for im in (img1, img2):
            if im.dtype != self._torch.uint8 or not im.is_contiguous() or im.device != self.device:
                raise FFError(FF_ERR_INVALID, "images must be contiguous uint8 tensors on the handle's device")
        if img1.shape != img2.shape or img1.dim() not in (2, 3):
            raise FFError(FF_ERR_INVALID, "images must share a [H, W] or [H, W, C] shape")
        H, W = int(img1.shape[0]), int(img1.shape[1])
        # the library writes every given output in full: check each against
        # the layout it writes before handing its pointer over
        for k, v in out.items():
            spec = self._OUT_SPEC.get(k)
            if spec is None or v is None:
                continue
            dt, tail = spec
            if (v.dtype != getattr(self._torch, dt) or tuple(v.shape) != (H, W) + tail or not v.is_contiguous()
                    or v.device != self.device):
                raise FFError(FF_ERR_INVALID, f"output {k} must be a contiguous {dt} tensor of shape "
                                              f"{(H, W) + tail} on the handle's device")
        C = 1 if img1.dim() == 2 else int(img1.shape[2])
        p = Pair(img1.data_ptr(), img2.data_ptr(), W, H, C,
                 self._ptr(out, "flow_f"), self._ptr(out, "cost_f"), self._ptr(out, "mask_f"),
                 self._ptr(out, "flow_b"), self._ptr(out, "cost_b"), self._ptr(out, "mask_b"),
                 self._ptr(out, "fberr_f"), self._ptr(out, "sparse_f"),
                 self._ptr(out, "fberr_b"), self._ptr(out, "sparse_b"))
        return p

    # -- API --------------------------------------------------------------
    def match(self, img1, img2, bwd=True, cost=True, out=None):
        H, W = int(img1.shape[0]), int(img1.shape[1])
        o = out if out is not None else self._outputs(H, W, bwd, cost)
        p = self._pair(img1, img2, o)
        self._check(lib().ff_match_pair(self._h, ctypes.byref(p), _stream_ptr(self._torch, self.device)))
        return o

    def match_noalloc(self, img1, img2, bwd=True, cost=True, out=None):
        """ff_match_pair_noalloc: the same search in the library's fixed
        per-device scratch (no device allocation by the library)."""
        H, W = int(img1.shape[0]), int(img1.shape[1])
        o = out if out is not None else self._outputs(H, W, bwd, cost)
        p = self._pair(img1, img2, o)
        self._check(lib().ff_match_pair_noalloc(self._h, ctypes.byref(p), _stream_ptr(self._torch, self.device)))
        return o

    def prepare_batch(self, pairs, bwd=True, cost=True, outs=None):
        """Marshal a batch once: the ff_pair array of these inputs and
        outputs, for repeated ff_match_batch calls (match_prepared) without
        rebuilding it in Python each time.  Keeps the tensors alive."""
        outs = outs if outs is not None else [
            self._outputs(int(a.shape[0]), int(a.shape[1]), bwd, cost) for a, _ in pairs]
        arr = (Pair * len(pairs))(*[self._pair(a, b, o) for (a, b), o in zip(pairs, outs)])
        return PreparedBatch(arr, len(pairs), pairs, outs)

    def match_prepared(self, prep):
        """ff_match_batch on a prepared batch; returns its outputs."""
        self._check(lib().ff_match_batch(self._h, prep.arr, prep.n, _stream_ptr(self._torch, self.device)))
        return prep.outs

    def match_batch(self, pairs, bwd=True, cost=True, outs=None):
        return self.match_prepared(self.prepare_batch(pairs, bwd, cost, outs))

    def workspace_bytes(self, shapes):
        arr = (Pair * len(shapes))(*[Pair(None, None, w, h, c) for (h, w, c) in shapes])
        return int(lib().ff_workspace_bytes(self._h, arr, len(shapes)))

    def debug_stage(self, img1, img2, kind, image=0, dir=0, level=0, iter=0, step=0):
        """Intermediate of one pair (see ff_debug_stage); returns a tensor."""
        t = self._torch
        H, W = int(img1.shape[0]), int(img1.shape[1])
        Wl, Hl = W, H
        # the sub-pixel refinement's state (level == levels) is level 0's
        for _ in range(0 if kind == STAGE_STATE and level == self.params.levels else level):
            Wl, Hl = Wl >> 1, Hl >> 1
        if kind == STAGE_GRAY:
            dst = t.empty((H, W), dtype=t.uint8, device=self.device)
        elif kind == STAGE_PYRAMID:
            dst = t.empty((Hl, Wl), dtype=t.uint8, device=self.device)
        elif kind == STAGE_DESC:
            dst = t.empty((Hl, Wl, 16), dtype=t.int8, device=self.device)
        elif kind == STAGE_SEEDS:
            Wc, Hc = W, H
            for _ in range(self.params.levels - 1):
                Wc, Hc = Wc >> 1, Hc >> 1
            s = self.params.seed_stride
            dst = t.empty((-(-Hc // s), -(-Wc // s)), dtype=t.int32, device=self.device)
        elif kind == STAGE_STATE:
            dst = t.empty((Hl, Wl, 2), dtype=t.int32, device=self.device)
        elif kind == STAGE_CENSUS:
            dst = t.empty((Hl, Wl), dtype=t.int64, device=self.device)
        else:
            raise FFError(FF_ERR_INVALID, "unknown stage kind")
        o = self._outputs(H, W, True, True)
        p = self._pair(img1, img2, o)
        st = Stage(kind, image, dir, level, iter, step)
        self._check(lib().ff_debug_stage(self._h, ctypes.byref(p), ctypes.byref(st),
                                         ctypes.c_void_p(dst.data_ptr()),
                                         _stream_ptr(self._torch, self.device)))
        return dst

    def fault_alloc(self, after):
        """ff_debug_fault_alloc: the first `after` allocations from now on
        succeed, later ones fail as out of memory (after < 0: off)."""
        self._check(lib().ff_debug_fault_alloc(self._h, int(after)))

    # -- serving ----------------------------------------------------------
    def serve_config(self, lanes=4, lane_bytes=4 << 30):
        self._check(lib().ff_serve_config(self._h, lanes, lane_bytes))

    def submit(self, img1, img2, tag, bwd=True, cost=True, out=None):
        """Queue one pair; returns its output dict (complete once poll() has
        returned ``tag``).  The tensors are kept alive until then."""
        H, W = int(img1.shape[0]), int(img1.shape[1])
        o = out if out is not None else self._outputs(H, W, bwd, cost)
        p = self._pair(img1, img2, o)
        if not hasattr(self, "_inflight"):
            self._inflight = {}
        self._inflight[int(tag)] = (img1, img2, o)
        st = lib().ff_submit(self._h, ctypes.byref(p), int(tag), _stream_ptr(self._torch, self.device))
        if st != FF_OK:
            self._inflight.pop(int(tag), None)
            self._check(st)
        return o

    def poll(self, max_tags=1024):
        """Tags finished since the last poll (non-blocking)."""
        buf = (ctypes.c_uint64 * max_tags)()
        n = lib().ff_poll(self._h, buf, max_tags)
        if n < 0:
            self._check(FF_ERR_HIP)
        tags = [int(buf[i]) for i in range(n)]
        for t in tags:
            getattr(self, "_inflight", {}).pop(t, None)
        return tags

    def inflight(self):
        return int(lib().ff_serve_inflight(self._h))

    # -- schedule tuning ----------------------------------------------------
    def autotune(self, pairs, outs=None):
        """Pick the line-kernel schedule per phase and level on this batch."""
        outs = outs if outs is not None else [
            self._outputs(int(a.shape[0]), int(a.shape[1])) for a, _ in pairs]
        arr = (Pair * len(pairs))(*[self._pair(a, b, o) for (a, b), o in zip(pairs, outs)])
        self._check(lib().ff_autotune(self._h, arr, len(pairs), _stream_ptr(self._torch, self.device)))
        return self.tuning()

    def tuning(self):
        n = 6 * self.params.levels
        buf = (ctypes.c_int32 * n)()
        if lib().ff_tune_get(self._h, buf, n) != n:
            self._check(FF_ERR_INVALID)
        return [int(v) for v in buf]

    def set_tuning(self, cfg):
        buf = (ctypes.c_int32 * len(cfg))(*cfg)
        self._check(lib().ff_tune_set(self._h, buf, len(cfg)))

    def profile(self, on: bool):
        """Bracket every launch with HIP events (per-kernel device time)."""
        self._check(lib().ff_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms)} since the last read; synchronises."""
        arr = (ProfileEntry * 32)()
        n = lib().ff_profile_read(self._h, arr, 32)
        if n < 0:
            self._check(FF_ERR_HIP)
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}

    def close(self):
        if getattr(self, "_h", None):
            lib().ff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def state_split(state):
    """Split a STATE intermediate ([H, W, 2] int32) into flow [H, W, 2]
    int16 and cost [H, W] int32 (numpy)."""
    import numpy as np
    s = state.cpu().numpy() if hasattr(state, "cpu") else state
    flow = s[..., 0].copy().view(np.int16).reshape(s.shape[0], s.shape[1], 2)
    return flow, s[..., 1].copy()
