"""CPU oracle of the Flow Fields search (FlowFields++, Sec. 3.1).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

``build()`` compiles ``ff_oracle.c`` into ``libff_oracle.so`` beside it; the
functions below are thin ctypes/numpy wrappers with no arithmetic of their
own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ff_oracle.c")
_LIB = os.path.join(_HERE, "libff_oracle.so")

INF = 2**31 - 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, -O2, single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("seed_stride", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("rs_radius", ctypes.c_int32),
                ("fb_eps", ctypes.c_int32), ("seed", ctypes.c_uint64), ("cost_kind", ctypes.c_int32),
                ("two_checks", ctypes.c_int32), ("seed2", ctypes.c_uint64),
                ("sub_iters", ctypes.c_int32), ("sub_radius", ctypes.c_int32),
                ("second_params", ctypes.c_int32), ("iters2", ctypes.c_int32), ("rs_radius2", ctypes.c_int32)]


COST_WH, COST_CENSUS = 0, 1


TRACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_int16), ctypes.POINTER(ctypes.c_int32))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        l = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i = ctypes.c_int
        l.ffo_gray.argtypes = [P, i, i, i, P]
        l.ffo_down2.argtypes = [P, i, i, P]
        l.ffo_descriptors.argtypes = [P, i, i, P]
        l.ffo_seed_nn.argtypes = [P, P, i, i, i, P]
        l.ffo_nearest.argtypes = [P, P, i]
        l.ffo_fb_error.argtypes = [i, i, P, P, P, P, P]
        l.ffo_sparsify.argtypes = [i, i, P, P, i, P]
        l.ffo_fb_error2.argtypes = [i, i, P, P, P, P, P, P, P]
        l.ffo_fb_error_u.argtypes = [i, i, i, P, P, P, P, P]
        l.ffo_fb_error2_u.argtypes = [i, i, i, P, P, P, P, P, P, P]
        l.ffo_cost_subpix.argtypes = [P, P, i, i, i, i, i, i]
        l.ffo_cost_subpix.restype = ctypes.c_int32
        l.ffo_sweep_subpix.argtypes = [P, P, i, i, i, P, P]
        l.ffo_random_search_subpix.argtypes = [P, P, i, i, i, i, i, i, ctypes.c_uint64, P, P]
        l.ffo_census.argtypes = [P, i, i, P]
        l.ffo_cost_census.argtypes = [P, P, i, i, i, i, i, i]
        l.ffo_cost_census.restype = ctypes.c_int32
        l.ffo_sweep_census.argtypes = [P, P, i, i, i, P, P]
        l.ffo_random_search_census.argtypes = [P, P, i, i, i, i, i, i, ctypes.c_uint64, P, P]
        l.ffo_nearest.restype = ctypes.c_int32
        l.ffo_philox4x32_10.argtypes = [P, P, P]
        l.ffo_cost.argtypes = [P, P, i, i, i, i, i, i]
        l.ffo_cost.restype = ctypes.c_int32
        l.ffo_sweep.argtypes = [P, P, i, i, i, P, P]
        l.ffo_random_search.argtypes = [P, P, i, i, i, i, i, i, ctypes.c_uint64, P, P]
        l.ffo_match.argtypes = [ctypes.POINTER(Params), P, P, i, i, i, P, P, P, P, P, P,
                                TRACE_FN, P]
        l.ffo_match.restype = ctypes.c_int
        _lib = l
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def params(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, cost_kind=COST_WH,
           two_checks=0, seed2=0, sub_iters=0, sub_radius=2, iters2=None, rs_radius2=None) -> Params:
    """iters2 / rs_radius2 (with two_checks): the second search's own
    iterations and random-search radius (None: the first search's)."""
    second = iters2 is not None or rs_radius2 is not None
    return Params(levels, seed_stride, iters, rs_radius, fb_eps, seed, cost_kind, two_checks, seed2,
                  sub_iters, sub_radius, 1 if second else 0, iters if iters2 is None else iters2,
                  rs_radius if rs_radius2 is None else rs_radius2)


def gray(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape[:2]
    C = 1 if img.ndim == 2 else img.shape[2]
    out = np.empty((H, W), np.uint8)
    lib().ffo_gray(_p(img), W, H, C, _p(out))
    return out


def down2(plane: np.ndarray) -> np.ndarray:
    plane = np.ascontiguousarray(plane, dtype=np.uint8)
    H, W = plane.shape
    out = np.empty((H >> 1, W >> 1), np.uint8)
    lib().ffo_down2(_p(plane), W, H, _p(out))
    return out


def pyramid(gray_plane: np.ndarray, levels: int) -> list:
    out = [np.ascontiguousarray(gray_plane, dtype=np.uint8)]
    for _ in range(1, levels):
        out.append(down2(out[-1]))
    return out


def descriptors(plane: np.ndarray) -> np.ndarray:
    plane = np.ascontiguousarray(plane, dtype=np.uint8)
    H, W = plane.shape
    out = np.empty((H, W, 16), np.int8)
    lib().ffo_descriptors(_p(plane), W, H, _p(out))
    return out


def seed_nn(DA: np.ndarray, DB: np.ndarray, stride: int) -> np.ndarray:
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    nsx, nsy = -(-W // stride), -(-H // stride)
    out = np.empty((nsy, nsx), np.int32)
    lib().ffo_seed_nn(_p(DA), _p(DB), W, H, stride, _p(out))
    return out


def nearest(a: np.ndarray, DB: np.ndarray) -> int:
    """Sec. 3.1 seed search for one query descriptor: lowest index of the
    minimum squared L2 distance over all descriptors of DB."""
    a = np.ascontiguousarray(a, dtype=np.int8).reshape(16)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    return int(lib().ffo_nearest(_p(a), _p(DB), DB.size // 16))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().ffo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def cost(DA, DB, x, y, fx, fy) -> int:
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    return int(lib().ffo_cost(_p(DA), _p(DB), W, H, x, y, fx, fy))


def sweep(DA, DB, flow, cst, dir_code: int):
    """In-place copy semantics: returns new (flow, cost) after one sweep."""
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_sweep(_p(DA), _p(DB), W, H, dir_code, _p(f), _p(c))
    return f, c


def random_search(DA, DB, flow, cst, level, it, pss, radius, seed):
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_random_search(_p(DA), _p(DB), W, H, level, it, pss, radius,
                            ctypes.c_uint64(seed), _p(f), _p(c))
    return f, c


def census(plane: np.ndarray) -> np.ndarray:
    """Sec. 3.1 7x7 Census strings of a luma plane, [H, W] uint64."""
    plane = np.ascontiguousarray(plane, dtype=np.uint8)
    H, W = plane.shape
    out = np.empty((H, W), np.uint64)
    lib().ffo_census(_p(plane), W, H, _p(out))
    return out


def cost_census(CA, CB, x, y, fx, fy) -> int:
    CA = np.ascontiguousarray(CA, dtype=np.uint64)
    CB = np.ascontiguousarray(CB, dtype=np.uint64)
    H, W = CA.shape
    return int(lib().ffo_cost_census(_p(CA), _p(CB), W, H, x, y, fx, fy))


def sweep_census(CA, CB, flow, cst, dir_code: int):
    CA = np.ascontiguousarray(CA, dtype=np.uint64)
    CB = np.ascontiguousarray(CB, dtype=np.uint64)
    H, W = CA.shape
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_sweep_census(_p(CA), _p(CB), W, H, dir_code, _p(f), _p(c))
    return f, c


def random_search_census(CA, CB, flow, cst, level, it, pss, radius, seed):
    CA = np.ascontiguousarray(CA, dtype=np.uint64)
    CB = np.ascontiguousarray(CB, dtype=np.uint64)
    H, W = CA.shape
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_random_search_census(_p(CA), _p(CB), W, H, level, it, pss, radius,
                                   ctypes.c_uint64(seed), _p(f), _p(c))
    return f, c


def fb_error(F, cF, B, cB, unit: int = 1) -> np.ndarray:
    """Sec. 3.1 consistency error per pixel: |F(p) + B(p + F(p))|^2, INF
    where either match is invalid; flows in 1/unit pixels (q rounded)."""
    F = np.ascontiguousarray(F, dtype=np.int16)
    B = np.ascontiguousarray(B, dtype=np.int16)
    cF = np.ascontiguousarray(cF, dtype=np.int32)
    cB = np.ascontiguousarray(cB, dtype=np.int32)
    H, W = cF.shape
    out = np.empty((H, W), np.int32)
    if unit == 1:
        lib().ffo_fb_error(W, H, _p(F), _p(cF), _p(B), _p(cB), _p(out))
    else:
        lib().ffo_fb_error_u(W, H, unit, _p(F), _p(cF), _p(B), _p(cB), _p(out))
    return out


def cost_subpix(DA, DB, x, y, u, v) -> int:
    """Sec. 3.1 sub-pixel cost, (u, v) in quarter pixels."""
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    return int(lib().ffo_cost_subpix(_p(DA), _p(DB), W, H, x, y, u, v))


def sweep_subpix(DA, DB, flow, cst, dir_code: int):
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_sweep_subpix(_p(DA), _p(DB), W, H, dir_code, _p(f), _p(c))
    return f, c


def random_search_subpix(DA, DB, flow, cst, level, it, pss, radius, seed):
    DA = np.ascontiguousarray(DA, dtype=np.int8)
    DB = np.ascontiguousarray(DB, dtype=np.int8)
    H, W = DA.shape[:2]
    f = np.array(flow, dtype=np.int16, copy=True, order="C")
    c = np.array(cst, dtype=np.int32, copy=True, order="C")
    lib().ffo_random_search_subpix(_p(DA), _p(DB), W, H, level, it, pss, radius,
                                   ctypes.c_uint64(seed), _p(f), _p(c))
    return f, c


def fb_error2(F, cF, B1, cB1, B2, cB2, unit: int = 1) -> np.ndarray:
    """Sec. 3.1 two consistency checks: the larger of the errors against the
    inverse fields B1 and B2 (INF when either is)."""
    a = [np.ascontiguousarray(v, dtype=np.int16) for v in (F, B1, B2)]
    c = [np.ascontiguousarray(v, dtype=np.int32) for v in (cF, cB1, cB2)]
    H, W = c[0].shape
    out = np.empty((H, W), np.int32)
    if unit == 1:
        lib().ffo_fb_error2(W, H, _p(a[0]), _p(c[0]), _p(a[1]), _p(c[1]), _p(a[2]), _p(c[2]), _p(out))
    else:
        lib().ffo_fb_error2_u(W, H, unit, _p(a[0]), _p(c[0]), _p(a[1]), _p(c[1]), _p(a[2]), _p(c[2]), _p(out))
    return out


def sparsify(mask, err, s: int) -> np.ndarray:
    """Sec. 3.1 sparsification: per 3x3 block with >= s consistent matches,
    keep the lowest-error one (lowest index on ties)."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    err = np.ascontiguousarray(err, dtype=np.int32)
    H, W = mask.shape
    out = np.empty((H, W), np.uint8)
    lib().ffo_sparsify(W, H, _p(mask), _p(err), int(s), _p(out))
    return out


def match(img1: np.ndarray, img2: np.ndarray, prm: Params | None = None, trace=None):
    """Run the whole search.  Returns dict with flow_f/cost_f/mask_f and the
    backward outputs.  ``trace(dir, level, iter, stage, flow, cost)`` is
    called with copies of the state after every stage when given."""
    prm = prm or params()
    img1 = np.ascontiguousarray(img1, dtype=np.uint8)
    img2 = np.ascontiguousarray(img2, dtype=np.uint8)
    assert img1.shape == img2.shape
    H, W = img1.shape[:2]
    C = 1 if img1.ndim == 2 else img1.shape[2]
    out = {
        "flow_f": np.empty((H, W, 2), np.int16), "cost_f": np.empty((H, W), np.int32),
        "mask_f": np.empty((H, W), np.uint8), "flow_b": np.empty((H, W, 2), np.int16),
        "cost_b": np.empty((H, W), np.int32), "mask_b": np.empty((H, W), np.uint8),
    }
    if trace is not None:
        def _cb(user, d, l, t, s, w, h, fp, cp):
            f = np.ctypeslib.as_array(fp, shape=(h, w, 2)).copy()
            c = np.ctypeslib.as_array(cp, shape=(h, w)).copy()
            trace(d, l, t, s, f, c)
        cb = TRACE_FN(_cb)
    else:
        cb = TRACE_FN()
    rc = lib().ffo_match(ctypes.byref(prm), _p(img1), _p(img2), W, H, C,
                         _p(out["flow_f"]), _p(out["cost_f"]), _p(out["mask_f"]),
                         _p(out["flow_b"]), _p(out["cost_b"]), _p(out["mask_b"]), cb, None)
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return out
