"""Sequential CPU oracle for the filter-partition path (numpy front end).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library: the arithmetic lives in ``ixoracle.c`` (plain C, one
thread), this module only marshals numpy arrays through ctypes.

The C file writes out the plain definition of every result:
  * combinators map / scatter .............. Section 2.1
  * partition2, sgmSum, mkSgmDescr, mkII ... Section 2.1
  * partition2L (segmented partition) ...... Section 6, "Segmented operations"
  * Range / Monotonic / Inj / Bij / FiltPart  Section 2.3, figure "Array Properties"

Every function is pinned by ``tests/test_oracle_pins.py`` against values
the paper prints, closed forms, library routines and brute force.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libixoracle.so")

I32, I64, F32 = 0, 1, 2
PRED_MOD_EQ, PRED_LT, PRED_FLAGS = 0, 1, 2
MODE_PARTITION, MODE_FILTER = 0, 1
MONO_LE, MONO_LT, MONO_GE, MONO_GT = 0, 1, 2, 3

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIBPATH)
        P, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float
        sig = {
            "ixo_map_pred": [P, i32, i64, i32, i64, i64, f32, P, P],
            "ixo_scatter": [P, i64, P, P, i64, i64],
            "ixo_gather": [P, P, i64, P, i64, i64],
            "ixo_hist_min": [P, i64, i64, P, P, i64],
            "ixo_scatter_checked": [P, i64, P, P, i64, i64, P],
            "ixo_get_smallest_pairs": [i64, i64, P, P, i64, P, P, P],
            "ixo_partition_v": [P, i64, i32, i32, P, P, P, P, P],
            "ixo_partition2L_rows": [P, i32, i64, P, i64, i32, i64, P, i32, P, P, P, P],
            "ixo_partition2": [P, i32, i64, i32, i64, i64, f32, P, i32, P, P, P],
            "ixo_sgm_sum": [P, P, i64, P],
            "ixo_mk_sgm_descr": [P, i64, P, P, i64],
            "ixo_mk_ii": [P, i64, P, i64],
            "ixo_partition2L": [P, i32, i64, P, i64, i32, i64, i64, f32, P, i32,
                                P, P, P, P],
            "ixo_check_range": [P, i64, i64, i64, P],
            "ixo_check_mono": [P, i64, i32, P],
            "ixo_check_inj": [P, i64, i64, i64, P],
            "ixo_check_bij": [P, i64, i64, i64, i64, i64, P],
            "ixo_check_filtpart": [P, i32, i64, i32, i64, i64, f32, P, i32, P, P,
                                   i64, P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


@dataclass
class Pred:
    """Predicate p of partition2: MOD_EQ (floor-mod key by d equals r), LT
    (f32 key < s) or FLAGS (a caller boolean array, partition2L's csL)."""
    kind: int
    d: int = 1
    r: int = 0
    s: float = 0.0
    flags: Optional[np.ndarray] = None

    @staticmethod
    def mod_eq(d, r):
        return Pred(PRED_MOD_EQ, d=int(d), r=int(r))

    @staticmethod
    def lt(s):
        return Pred(PRED_LT, s=float(np.float32(s)))

    @staticmethod
    def from_flags(flags):
        return Pred(PRED_FLAGS, flags=np.ascontiguousarray(flags, dtype=np.uint8))


def _key_t(keys: np.ndarray) -> int:
    if keys.dtype == np.int32:
        return I32
    if keys.dtype == np.int64:
        return I64
    if keys.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported key dtype {keys.dtype}")


def _pred_args(p: Pred):
    return (p.kind, p.d, p.r, p.s, _ptr(p.flags))


def map_pred(keys: np.ndarray, p: Pred) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    cs = np.zeros(len(keys), dtype=np.uint8)
    _check(_load().ixo_map_pred(_ptr(keys), _key_t(keys), len(keys),
                                *_pred_args(p), _ptr(cs)), "map_pred")
    return cs.astype(bool)


def partition2(keys: np.ndarray, p: Pred, mode: int = MODE_PARTITION):
    """Returns (ys, indices[int64], num_true) of partition2 (or filter)."""
    keys = np.ascontiguousarray(keys)
    n = len(keys)
    ys = np.zeros(n, dtype=keys.dtype)
    idx = np.zeros(n, dtype=np.int64)
    nt = ctypes.c_int64(0)
    _check(_load().ixo_partition2(_ptr(keys), _key_t(keys), n, *_pred_args(p),
                                  mode, _ptr(ys), _ptr(idx), ctypes.addressof(nt)),
           "partition2")
    t = nt.value
    if mode == MODE_FILTER:
        ys = ys[:t].copy()
    return ys, idx, t


def partition2L(keys: np.ndarray, shape: np.ndarray, p: Pred,
                mode: int = MODE_PARTITION):
    """Returns (ys, indices[int64], seg_split[int64 m], flags[uint8 n])."""
    keys = np.ascontiguousarray(keys)
    shape = np.ascontiguousarray(shape, dtype=np.int64)
    n, m = len(keys), len(shape)
    ys = np.zeros(n, dtype=keys.dtype)
    idx = np.zeros(n, dtype=np.int64)
    seg = np.zeros(m, dtype=np.int64)
    flags = np.zeros(n, dtype=np.uint8)
    _check(_load().ixo_partition2L(_ptr(keys), _key_t(keys), n, _ptr(shape), m,
                                   *_pred_args(p), mode, _ptr(ys), _ptr(idx),
                                   _ptr(seg), _ptr(flags)), "partition2L")
    if mode == MODE_FILTER:
        ys = ys[: int(seg.sum())].copy()
    return ys, idx, seg, flags


ROW_LT, ROW_MOD = 0, 1


def partition2L_rows(keys: np.ndarray, shape: np.ndarray, row_kind: int, d: int = 1,
                     s_rows: Optional[np.ndarray] = None, mode: int = MODE_PARTITION):
    """partition2L with a predicate of the row number: ROW_LT (x < s_rows[k])
    or ROW_MOD (floor-mod(x, d) == floor-mod(k, d)).  Returns as partition2L."""
    keys = np.ascontiguousarray(keys)
    shape = np.ascontiguousarray(shape, dtype=np.int64)
    n, m = len(keys), len(shape)
    sr = None if s_rows is None else np.ascontiguousarray(s_rows, dtype=np.float32)
    ys = np.zeros(n, dtype=keys.dtype)
    idx = np.zeros(n, dtype=np.int64)
    seg = np.zeros(m, dtype=np.int64)
    flags = np.zeros(n, dtype=np.uint8)
    _check(_load().ixo_partition2L_rows(_ptr(keys), _key_t(keys), n, _ptr(shape), m, row_kind, d,
                                        _ptr(sr), mode, _ptr(ys), _ptr(idx), _ptr(seg), _ptr(flags)),
           "partition2L_rows")
    if mode == MODE_FILTER:
        ys = ys[: int(seg.sum())].copy()
    return ys, idx, seg, flags


def sgm_sum(flags: np.ndarray, xs: np.ndarray) -> np.ndarray:
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    out = np.zeros(len(xs), dtype=np.int64)
    _check(_load().ixo_sgm_sum(_ptr(flags), _ptr(xs), len(xs), _ptr(out)), "sgm_sum")
    return out


def mk_sgm_descr(shape: np.ndarray, xs: np.ndarray) -> np.ndarray:
    shape = np.ascontiguousarray(shape, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    total = int(shape.sum()) if len(shape) else 0
    out = np.zeros(max(total, 0), dtype=np.int64)
    _check(_load().ixo_mk_sgm_descr(_ptr(shape), len(shape), _ptr(xs), _ptr(out),
                                    total), "mk_sgm_descr")
    return out


def mk_ii(shape: np.ndarray) -> np.ndarray:
    shape = np.ascontiguousarray(shape, dtype=np.int64)
    total = int(shape.sum()) if len(shape) else 0
    out = np.zeros(max(total, 0), dtype=np.int64)
    _check(_load().ixo_mk_ii(_ptr(shape), len(shape), _ptr(out), total), "mk_ii")
    return out


def scatter(dst: np.ndarray, idx: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """scatter dst idx vals on rows (first axis); returns the updated copy."""
    dst = np.ascontiguousarray(dst).copy()
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=dst.dtype)
    row = dst.itemsize * (int(np.prod(dst.shape[1:])) if dst.ndim > 1 else 1)
    _check(_load().ixo_scatter(_ptr(dst), dst.shape[0], _ptr(idx), _ptr(vals),
                               len(idx), row), "scatter")
    return dst


def gather(src: np.ndarray, idx: np.ndarray) -> np.ndarray:
    src = np.ascontiguousarray(src)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((len(idx),) + src.shape[1:], dtype=src.dtype)
    row = src.itemsize * (int(np.prod(src.shape[1:])) if src.ndim > 1 else 1)
    _check(_load().ixo_gather(_ptr(out), _ptr(src), src.shape[0], _ptr(idx),
                              len(idx), row), "gather")
    return out


def hist_min(n_dst: int, neutral: int, idx: np.ndarray, vals: Optional[np.ndarray] = None) -> np.ndarray:
    """Reduce-by-index with min into replicate n_dst neutral (vals None = iota)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.int64)
    out = np.zeros(n_dst, dtype=np.int64)
    _check(_load().ixo_hist_min(_ptr(out), n_dst, int(neutral), _ptr(idx), _ptr(v), len(idx)),
           "hist_min")
    return out


def scatter_checked(n_dst: int, idx: np.ndarray, vals: np.ndarray):
    """Dynamically verified scatter into replicate n_dst 0: (dst, verdict)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    vals = np.ascontiguousarray(vals)
    dst = np.zeros((n_dst,) + vals.shape[1:], dtype=vals.dtype)
    row = vals.itemsize * (int(np.prod(vals.shape[1:])) if vals.ndim > 1 else 1)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_scatter_checked(_ptr(dst), n_dst, _ptr(idx), _ptr(vals), len(idx), row,
                                       _ptr(v)), "scatter_checked")
    return dst, _verdict(v)


def get_smallest_pairs(n_verts: int, n_es: int, es: np.ndarray, is_: np.ndarray):
    """(es', is'): the entries holding the least id at their endpoint."""
    es = np.ascontiguousarray(es, dtype=np.int64)
    is_ = np.ascontiguousarray(is_, dtype=np.int64)
    eo = np.zeros(len(es), dtype=np.int64)
    io = np.zeros(len(es), dtype=np.int64)
    c = np.zeros(1, dtype=np.int64)
    _check(_load().ixo_get_smallest_pairs(n_verts, n_es, _ptr(es), _ptr(is_), len(es), _ptr(eo),
                                          _ptr(io), _ptr(c)), "get_smallest_pairs")
    return eo[: int(c[0])], io[: int(c[0])]


CLASS_MOD, CLASS_THRESH, CLASS_BYTES = 0, 1, 2


def partition_v(xs: Optional[np.ndarray], v: int, kind: int, s=(0.0, 0.0, 0.0),
                cls: Optional[np.ndarray] = None, n: Optional[int] = None):
    """v-way stable partition: (ys, idx, counts)."""
    if xs is not None:
        xs = np.ascontiguousarray(xs)
        n = len(xs)
    sv = np.ascontiguousarray(np.array(list(s) + [0.0] * (3 - len(s)), dtype=np.float32))
    c = None if cls is None else np.ascontiguousarray(cls, dtype=np.uint8)
    ys = np.zeros(n, dtype=xs.dtype if xs is not None else np.int32)
    idx = np.zeros(n, dtype=np.int64)
    counts = np.zeros(4, dtype=np.int64)
    _check(_load().ixo_partition_v(_ptr(xs), n, kind, v, _ptr(sv), _ptr(c), _ptr(ys), _ptr(idx),
                                   _ptr(counts)), "partition_v")
    return ys, idx, counts[:v]


def _verdict(v):
    return (int(v[0]), int(v[1]), int(v[2]))


def check_range(X, lo, hi):
    X = np.ascontiguousarray(X, dtype=np.int64)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_check_range(_ptr(X), len(X), lo, hi, _ptr(v)), "check_range")
    return _verdict(v)


def check_mono(X, op):
    X = np.ascontiguousarray(X, dtype=np.int64)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_check_mono(_ptr(X), len(X), op, _ptr(v)), "check_mono")
    return _verdict(v)


def check_inj(X, lo, hi):
    X = np.ascontiguousarray(X, dtype=np.int64)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_check_inj(_ptr(X), len(X), lo, hi, _ptr(v)), "check_inj")
    return _verdict(v)


def check_bij(X, lo, hi, ilo, ihi):
    X = np.ascontiguousarray(X, dtype=np.int64)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_check_bij(_ptr(X), len(X), lo, hi, ilo, ihi, _ptr(v)),
           "check_bij")
    return _verdict(v)


def check_filtpart(X, p: Pred, mode, Y, Z, split):
    X = np.ascontiguousarray(X)
    Yn = np.zeros(len(X), dtype=X.dtype)       # Y is read at positions < n only
    Yn[: min(len(Y), len(X))] = np.asarray(Y, dtype=X.dtype)[: len(X)]
    Y = Yn
    Z = np.ascontiguousarray(Z, dtype=np.int64)
    v = np.zeros(3, dtype=np.int64)
    _check(_load().ixo_check_filtpart(_ptr(X), _key_t(X), len(X), *_pred_args(p),
                                      mode, _ptr(Y), _ptr(Z), int(split), _ptr(v)),
           "check_filtpart")
    return _verdict(v)
