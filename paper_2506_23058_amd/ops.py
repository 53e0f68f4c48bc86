"""Python front end of the MI355X filter-partition library.

Thin wrappers over the C ABI (include/ixpart.h): they allocate outputs and
workspaces with torch on the input's device, pass raw device pointers and the
current HIP stream, and check the returned status.  All computation happens in
the library's HIP kernels.
"""
import ctypes
import functools
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L

_KEY_T = {torch.int32: L.I32, torch.float32: L.F32, torch.int64: L.I64}
_IDX_T = {torch.int32: L.I32, torch.int64: L.I64}


@dataclass(frozen=True)
class Pred:
    """Predicate p of partition2 (Section 2.1): MOD_EQ (floor-mod of an int32
    key by d equals r), LT (f32 key < s) or FLAGS (a u8 tensor, nonzero = true);
    for segmented calls also predicates of the row number k: LT_ROW (x <
    row_s[k], an f32 tensor of m thresholds) and MOD_ROW (x mod d == k mod d)."""
    kind: int
    d: int = 1
    r: int = 0
    s: float = 0.0
    flags: Optional[torch.Tensor] = None
    row_s: Optional[torch.Tensor] = None

    @staticmethod
    def mod_eq(d: int, r: int) -> "Pred":
        return Pred(L.PRED_MOD_EQ, d=int(d), r=int(r))

    @staticmethod
    def lt(s: float) -> "Pred":
        return Pred(L.PRED_LT, s=float(s))

    @staticmethod
    def from_flags(flags: torch.Tensor) -> "Pred":
        if flags.dtype == torch.bool:
            flags = flags.view(torch.uint8)
        return Pred(L.PRED_FLAGS, flags=flags.contiguous())

    @staticmethod
    def lt_rows(row_s: torch.Tensor) -> "Pred":
        return Pred(L.PRED_LT_ROW, row_s=row_s.to(torch.float32).contiguous())

    @staticmethod
    def mod_rows(d: int) -> "Pred":
        return Pred(L.PRED_MOD_ROW, d=int(d))

    def c(self) -> L.ixp_pred:
        """The C struct, built once per predicate and device pointers (the
        library copies it during the call)."""
        ptrs = (self.flags.data_ptr() if self.flags is not None else None,
                self.row_s.data_ptr() if self.row_s is not None else None)
        cached = self.__dict__.get("_c")
        if cached is not None and cached[0] == ptrs:
            return cached[1]
        p = L.ixp_pred()
        p.kind = self.kind
        p.d = self.d
        p.r = self.r
        p.s = self.s
        p.flags, p.row_s = ptrs
        object.__setattr__(self, "_c", (ptrs, p))   # a cache, not a field
        return p


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(device) -> int:
    """The current HIP stream of `device`, as a raw pointer."""
    if _raw_stream is not None:
        idx = device.index if isinstance(device, torch.device) else device
        return _raw_stream(torch.cuda.current_device() if idx is None else idx)
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


_ws_cache = {}


def _ws_key(device, tag: str):
    if not isinstance(device, torch.device):
        device = torch.device(device)
    return (device.type, device.index, tag)


def workspace(nbytes: int, device, tag: str = "default") -> torch.Tensor:
    """A cached device workspace of at least ``nbytes`` bytes (one per tag and
    device; calls that share a tag must not overlap on different streams)."""
    key = _ws_key(device, tag)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on a GPU")


@functools.lru_cache(maxsize=256)
def _partition_ws_bytes(n: int) -> int:
    return L.lib().ixp_partition_workspace(n)


def partition(keys: torch.Tensor, pred: Pred, mode: int = L.MODE_PARTITION,
              idx_dtype=torch.int64, want_keys: bool = True, want_idx: bool = True,
              out_keys: Optional[torch.Tensor] = None, out_idx: Optional[torch.Tensor] = None,
              split: Optional[torch.Tensor] = None):
    """Stable partition (partition2) or filter of a 1-D int32/f32 tensor.

    Returns (out_keys, out_idx, split) with split a 1-element int64 device
    tensor holding T.  In FILTER mode out_keys has length n and only its first
    T entries are written.
    """
    _check_dev(keys)
    keys = keys.contiguous()
    n = keys.numel()
    dev = keys.device
    if want_keys and out_keys is None:
        out_keys = torch.empty_like(keys)
    if want_idx and out_idx is None:
        out_idx = torch.empty(n, dtype=idx_dtype, device=dev)
    if split is None:
        split = torch.empty(1, dtype=torch.int64, device=dev)
    ws = workspace(_partition_ws_bytes(n), dev, "partition")
    pc = pred.c()
    rc = L.lib().ixp_partition(
        _ptr(keys), _KEY_T[keys.dtype], n, ctypes.byref(pc), mode,
        _ptr(out_keys) if want_keys else None, _ptr(out_idx) if want_idx else None,
        _IDX_T[idx_dtype if out_idx is None else out_idx.dtype], _ptr(split),
        _ptr(ws), ws.numel(), _stream_ptr(dev))
    L.check(rc, "ixp_partition")
    return (out_keys if want_keys else None), (out_idx if want_idx else None), split


class Classes:
    """Classes of the v-way partition (2 <= v <= 4): floor-mod of an int32
    key, f32 thresholds s[0] <= s[1] <= ..., or a uint8 class per element."""

    def __init__(self, kind: int, v: int, s=(), classes: Optional[torch.Tensor] = None):
        self.kind, self.v = int(kind), int(v)
        self.s = tuple(float(x) for x in s) + (0.0,) * (3 - len(s))
        self.classes = classes.contiguous() if classes is not None else None

    @staticmethod
    def mod(v: int) -> "Classes":
        return Classes(L.CLASS_MOD, v)

    @staticmethod
    def thresholds(*s: float) -> "Classes":
        return Classes(L.CLASS_THRESH, len(s) + 1, s)

    @staticmethod
    def from_bytes(classes: torch.Tensor, v: int) -> "Classes":
        return Classes(L.CLASS_BYTES, v, classes=classes.to(torch.uint8))

    def c(self) -> L.ixp_classes:
        c = L.ixp_classes()
        c.kind, c.v = self.kind, self.v
        for i in range(3):
            c.s[i] = self.s[i]
        c.classes = self.classes.data_ptr() if self.classes is not None else None
        return c


def partition_v(keys: torch.Tensor, classes: Classes, idx_dtype=torch.int64, want_keys: bool = True,
                want_idx: bool = True, out_keys: Optional[torch.Tensor] = None,
                out_idx: Optional[torch.Tensor] = None, counts: Optional[torch.Tensor] = None):
    """Stable v-way partition of a 1-D int32/f32 tensor: (out_keys, out_idx,
    counts) with counts the int64 class sizes on the device."""
    _check_dev(keys)
    keys = keys.contiguous()
    n = keys.numel()
    dev = keys.device
    if want_keys and out_keys is None:
        out_keys = torch.empty_like(keys)
    if want_idx and out_idx is None:
        out_idx = torch.empty(n, dtype=idx_dtype, device=dev)
    if counts is None:
        counts = torch.empty(classes.v, dtype=torch.int64, device=dev)
    ws = workspace(L.lib().ixp_partition_v_workspace(n), dev, "partition_v")
    cc = classes.c()
    rc = L.lib().ixp_partition_v(
        _ptr(keys), _KEY_T[keys.dtype], n, ctypes.byref(cc), _ptr(out_keys) if want_keys else None,
        _ptr(out_idx) if want_idx else None, _IDX_T[idx_dtype if out_idx is None else out_idx.dtype],
        _ptr(counts), _ptr(ws), ws.numel(), _stream_ptr(dev))
    L.check(rc, "ixp_partition_v")
    return (out_keys if want_keys else None), (out_idx if want_idx else None), counts


def read_error(ws: torch.Tensor) -> int:
    """Blocking: the device error recorded in a workspace (0 if none)."""
    return L.lib().ixp_read_error(_ptr(ws), _stream_ptr(ws.device))


def profile_enable(on: bool = True):
    """Bracket every library kernel with HIP events on its own stream."""
    L.check(L.lib().ixp_profile_enable(1 if on else 0), "ixp_profile_enable")


def profile_read():
    """Blocking: {kernel name: (launches, total ms)} since the last read."""
    buf = (L.ixp_kernel_stat * 64)()
    cnt = ctypes.c_int(0)
    L.check(L.lib().ixp_profile_read(ctypes.cast(buf, ctypes.c_void_p), 64, ctypes.byref(cnt)),
            "ixp_profile_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(min(cnt.value, 64))}


# ---------------------------------------------------------------- segmented --

def _tuning(tune):
    if tune is None:
        return None
    t = L.ixp_tuning()
    t.block, t.rows = int(tune[0]), int(tune[1])
    t.wgs_per_cu = int(tune[2]) if len(tune) > 2 else 0
    t.row_sync = int(tune[3]) if len(tune) > 3 else L.ROW_SYNC_AUTO
    return t


def _seg_outputs(keys, shape, idx_dtype, want_flags, out_keys, out_idx, seg_split, flags):
    n, m, dev = keys.numel(), shape.numel(), keys.device
    if out_keys is None:
        out_keys = torch.empty_like(keys)
    if out_idx is None:
        out_idx = torch.empty(n, dtype=idx_dtype, device=dev)
    if seg_split is None:
        seg_split = torch.empty(m, dtype=torch.int64, device=dev)
    if want_flags and flags is None:
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
    return out_keys, out_idx, seg_split, (flags if want_flags else None)


def segmented_partition(keys: torch.Tensor, shape: torch.Tensor, pred: Pred,
                        mode: int = L.MODE_PARTITION, idx_dtype=torch.int32,
                        want_flags: bool = True, tune=None, out_keys=None, out_idx=None,
                        seg_split=None, flags=None, ws_tag: str = "segmented"):
    """partition2L / filter_seg: stable partition (or filter) of every row of
    the jagged array whose row sizes are ``shape`` (int64, on the device).

    Returns (out_keys, out_idx, seg_split, flags).  ``tune`` is a
    (block, rows[, wgs_per_cu[, row_sync]]) tuple, or None for the library
    default.
    """
    _check_dev(keys, shape)
    keys = keys.contiguous()
    shape = shape.contiguous()
    if shape.dtype != torch.int64:
        raise ValueError("shape must be int64")
    out_keys, out_idx, seg_split, flags = _seg_outputs(keys, shape, idx_dtype, want_flags,
                                                       out_keys, out_idx, seg_split, flags)
    t = _tuning(tune)
    tp = ctypes.byref(t) if t is not None else None
    n, m = keys.numel(), shape.numel()
    ws = workspace(L.lib().ixp_segmented_workspace(n, m, tp), keys.device, ws_tag)
    pc = pred.c()
    rc = L.lib().ixp_segmented_partition(
        _ptr(keys), _KEY_T[keys.dtype], n, _ptr(shape), m, ctypes.byref(pc), mode,
        _ptr(out_keys), _ptr(out_idx), _IDX_T[out_idx.dtype], _ptr(seg_split), _ptr(flags),
        tp, _ptr(ws), ws.numel(), _stream_ptr(keys.device))
    L.check(rc, "ixp_segmented_partition")
    return out_keys, out_idx, seg_split, flags


def _tool_out(out, n, dtype, device):
    if out is None:
        return torch.empty(n, dtype=dtype, device=device)
    if out.dtype != dtype or out.numel() != n or not out.is_contiguous() or out.device != device:
        raise ValueError(f"out must be a contiguous {dtype} tensor of {n} elements on {device}")
    return out


def mk_ii(shape: torch.Tensor, n: int, out_dtype=torch.int64, ws_tag: str = "shape_tools",
          out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """mkII: the row number of every element of rows of the given sizes."""
    _check_dev(shape)
    shape = shape.contiguous()
    m = shape.numel()
    out = _tool_out(out, n, out_dtype, shape.device)
    ws = workspace(L.lib().ixp_mk_ii_workspace(n, m), shape.device, ws_tag)
    rc = L.lib().ixp_mk_ii(_ptr(shape), m, n, _ptr(out), _IDX_T[out_dtype], _ptr(ws), ws.numel(),
                           _stream_ptr(shape.device))
    L.check(rc, "ixp_mk_ii")
    return out


def mk_sgm_descr(shape: torch.Tensor, xs: torch.Tensor, n: int, ws_tag: str = "shape_tools",
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """mkSgmDescr: xs[k] at the first position of every non-empty row k, 0 elsewhere."""
    _check_dev(shape, xs)
    shape = shape.contiguous()
    xs = xs.contiguous().to(torch.int64)
    m = shape.numel()
    out = _tool_out(out, n, torch.int64, shape.device)
    ws = workspace(L.lib().ixp_mk_ii_workspace(n, m), shape.device, ws_tag)
    rc = L.lib().ixp_mk_sgm_descr(_ptr(shape), m, n, _ptr(xs), _ptr(out), _ptr(ws), ws.numel(),
                                  _stream_ptr(shape.device))
    L.check(rc, "ixp_mk_sgm_descr")
    return out


def sgm_sum(flags: torch.Tensor, xs: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sgmSum: running int64 sums of xs that restart at every nonzero flag."""
    _check_dev(flags, xs)
    flags = flags.contiguous().view(torch.uint8) if flags.dtype == torch.bool else flags.contiguous()
    xs = xs.contiguous()
    if xs.dtype != torch.int64 or flags.dtype != torch.uint8 or flags.numel() != xs.numel():
        raise ValueError("sgm_sum needs uint8/bool flags and int64 values of one length")
    n = xs.numel()
    if out is None:
        out = torch.empty_like(xs)
    ws = workspace(L.lib().ixp_sgm_sum_workspace(n), xs.device, "sgm_sum")
    rc = L.lib().ixp_sgm_sum(_ptr(flags), _ptr(xs), n, _ptr(out), _ptr(ws), ws.numel(), _stream_ptr(xs.device))
    L.check(rc, "ixp_sgm_sum")
    return out


def shape_tools_error(ws_tag: str = "shape_tools", device="cuda:0") -> int:
    """Blocking: the error recorded by the last mk_ii / mk_sgm_descr call."""
    ws = _ws_cache.get(_ws_key(device, ws_tag))
    return 0 if ws is None else L.lib().ixp_read_error(_ptr(ws), _stream_ptr(ws.device))


def segmented_error(ws_tag: str = "segmented", device="cuda:0") -> int:
    """Blocking: status recorded by the last segmented call on this workspace
    (IXP_EINVAL for an invalid shape array), then cleared."""
    ws = _ws_cache.get(_ws_key(device, ws_tag))
    if ws is None:
        return L.IXP_OK
    return L.lib().ixp_read_error(_ptr(ws), _stream_ptr(ws.device))


def tune_segmented(keys, shape, pred, mode=L.MODE_PARTITION, idx_dtype=torch.int32,
                   want_flags=True, reps: int = 5):
    """Blocking autotuner: times every supported tiling on these arguments and
    returns ((block, rows, wgs_per_cu, row_sync), milliseconds)."""
    keys = keys.contiguous()
    shape = shape.contiguous()
    out_keys, out_idx, seg_split, flags = _seg_outputs(keys, shape, idx_dtype, want_flags,
                                                       None, None, None, None)
    n, m = keys.numel(), shape.numel()
    big = L.ixp_tuning()
    big.block, big.rows = 256, 2     # smallest tile: largest workspace
    ws = workspace(L.lib().ixp_segmented_workspace(n, m, ctypes.byref(big)), keys.device,
                   "segmented_tune")
    best = L.ixp_tuning()
    ms = ctypes.c_float(0)
    pc = pred.c()
    rc = L.lib().ixp_tune_segmented(
        _ptr(keys), _KEY_T[keys.dtype], n, _ptr(shape), m, ctypes.byref(pc), mode,
        _ptr(out_keys), _ptr(out_idx), _IDX_T[idx_dtype], _ptr(seg_split), _ptr(flags),
        _ptr(ws), ws.numel(), reps, ctypes.byref(best), ctypes.byref(ms),
        _stream_ptr(keys.device))
    L.check(rc, "ixp_tune_segmented")
    return (best.block, best.rows, best.wgs_per_cu, best.row_sync), ms.value


class SegmentedGraph:
    """One segmented partition captured into a HIP graph by the library
    (ixp_segmented_graph_create); launch() replays it on the current stream with
    the same buffers.  The input tensors may be refilled between launches."""

    def __init__(self, keys, shape, pred, mode=L.MODE_PARTITION, idx_dtype=torch.int32,
                 want_flags=True, tune=None):
        _check_dev(keys, shape)
        self.keys = keys.contiguous()
        self.shape = shape.contiguous()
        self.pred = pred          # keeps a flag tensor alive
        (self.out_keys, self.out_idx, self.seg_split,
         self.flags) = _seg_outputs(self.keys, self.shape, idx_dtype, want_flags,
                                    None, None, None, None)
        t = _tuning(tune)
        tp = ctypes.byref(t) if t is not None else None
        n, m = self.keys.numel(), self.shape.numel()
        self.ws = torch.empty(max(L.lib().ixp_segmented_workspace(n, m, tp), 256),
                              dtype=torch.uint8, device=self.keys.device)
        pc = pred.c()
        h = ctypes.c_void_p()
        rc = L.lib().ixp_segmented_graph_create(
            ctypes.byref(h), _ptr(self.keys), _KEY_T[self.keys.dtype], n, _ptr(self.shape), m,
            ctypes.byref(pc), mode, _ptr(self.out_keys), _ptr(self.out_idx),
            _IDX_T[idx_dtype], _ptr(self.seg_split), _ptr(self.flags), tp, _ptr(self.ws),
            self.ws.numel())
        L.check(rc, "ixp_segmented_graph_create")
        self._h = h

    def launch(self):
        L.check(L.lib().ixp_graph_launch(self._h, _stream_ptr(self.keys.device)),
                "ixp_graph_launch")
        return self.out_keys, self.out_idx, self.seg_split, self.flags

    def error(self) -> int:
        return L.lib().ixp_read_error(_ptr(self.ws), _stream_ptr(self.ws.device))

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.keys.device)
            L.lib().ixp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- properties --

@dataclass
class FiltPartArgs:
    """Outputs of a flat partition to check with FILTPART: the partitioned keys
    ``src``, the output keys ``dst``, the predicate, the mode and the split
    point (a 1-element int64 device tensor)."""
    src: torch.Tensor
    dst: torch.Tensor
    pred: Pred
    split: torch.Tensor
    mode: int = L.MODE_PARTITION


def check_props(x: torch.Tensor, mask: int, lo: int = 0, hi: int = 0, img_lo: int = 0,
                img_hi: int = 0, mono_op: int = L.MONO_LE, fp: Optional[FiltPartArgs] = None):
    """Run-time property checks (Range, Monotonic, Inj, Bij, FiltPart) of an
    int32/int64 device array.  Returns a [5, 3] int64 device tensor of
    (holds, first_violation, aux) per property, in the order of the IXP_*
    bits; unselected properties read (1, -1, 0)."""
    _check_dev(x)
    x = x.contiguous()
    n = x.numel()
    a = L.ixp_prop_args()
    a.lo, a.hi, a.img_lo, a.img_hi, a.mono_op = int(lo), int(hi), int(img_lo), int(img_hi), int(mono_op)
    if fp is not None:
        a.fp_mode = fp.mode
        a.fp_src = fp.src.data_ptr()
        a.fp_dst = fp.dst.data_ptr()
        a.fp_key_t = _KEY_T[fp.src.dtype]
        a.fp_pred = fp.pred.c()
        a.fp_split = fp.split.data_ptr()
    out = torch.empty(5 * 3, dtype=torch.int64, device=x.device)
    ws = workspace(L.lib().ixp_check_props_workspace(n, mask, ctypes.byref(a)), x.device, "props")
    rc = L.lib().ixp_check_props(_ptr(x), _IDX_T[x.dtype], n, mask, ctypes.byref(a), _ptr(out),
                                 _ptr(ws), ws.numel(), _stream_ptr(x.device))
    L.check(rc, "ixp_check_props")
    v = out.view(5, 3).clone()
    v[:, 0] = v[:, 0] & 0xFFFFFFFF   # holds is the low 32 bits of the first word
    return v


def verdicts(v: torch.Tensor):
    """[(holds, first_violation, aux)] * 5 on the host (synchronises)."""
    return [tuple(int(t) for t in row) for row in v.cpu().tolist()]


# ---------------------------------------------------------- rows / autograd --

def scatter_inj(dst: torch.Tensor, idx: torch.Tensor, vals: torch.Tensor) -> torch.Tensor:
    """dst[idx[i]] = vals[i] on rows (first axis), in place; out-of-range
    indices are ignored.  ``idx`` must be injective on [0, len(dst))."""
    _check_dev(dst, idx, vals)
    vals = vals.contiguous()
    idx = idx.contiguous()
    if not dst.is_contiguous() or dst.dtype != vals.dtype or dst.shape[1:] != vals.shape[1:]:
        raise ValueError("dst must be contiguous with the row shape and dtype of vals")
    rb = vals.element_size()
    for d in vals.shape[1:]:
        rb *= d
    rc = L.lib().ixp_scatter_inj(_ptr(dst), dst.shape[0], _ptr(idx), _IDX_T[idx.dtype], _ptr(vals),
                                 vals.shape[0], rb, _stream_ptr(dst.device))
    L.check(rc, "ixp_scatter_inj")
    return dst


def gather(src: torch.Tensor, idx: torch.Tensor, err: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[i] = src[idx[i]] on rows; an index outside [0, len(src)) gives a zero
    row (and sets err[0] = 1 when an int32 error tensor is given)."""
    _check_dev(src, idx)
    src = src.contiguous()
    idx = idx.contiguous()
    out = torch.empty((idx.shape[0],) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device)
    rb = src.element_size()
    for d in src.shape[1:]:
        rb *= d
    rc = L.lib().ixp_gather(_ptr(out), _ptr(src), src.shape[0], _ptr(idx), _IDX_T[idx.dtype],
                            idx.shape[0], rb, _ptr(err), _stream_ptr(src.device))
    L.check(rc, "ixp_gather")
    return out


def hist_min(n_dst: int, neutral: int, idx: torch.Tensor, vals: Optional[torch.Tensor] = None,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Reduce-by-index with min: replicate n_dst neutral, then
    out[idx[i]] = min(out[idx[i]], vals[i]) (vals None: i); out-of-range
    indices are ignored.  int64 result."""
    _check_dev(idx)
    idx = idx.contiguous()
    if vals is not None:
        _check_dev(vals)
        vals = vals.contiguous()
        if vals.dtype != torch.int64 or vals.shape[0] != idx.shape[0]:
            raise ValueError("vals must be int64 with one entry per index")
    if out is None:
        out = torch.empty(n_dst, dtype=torch.int64, device=idx.device)
    rc = L.lib().ixp_hist_min(_ptr(out), n_dst, int(neutral), _ptr(idx), _IDX_T[idx.dtype], _ptr(vals),
                              idx.shape[0], _stream_ptr(idx.device))
    L.check(rc, "ixp_hist_min")
    return out


def scatter_checked(n_dst: int, idx: torch.Tensor, vals: torch.Tensor,
                    out: Optional[torch.Tensor] = None, verdict: Optional[torch.Tensor] = None):
    """Dynamically verified scatter into a zeroed array of n_dst elements:
    returns (dst, verdict) with verdict = int64 [holds, first_violation, aux]
    of Inj over [0, n_dst); where a location is written twice the least
    index wins."""
    _check_dev(idx, vals)
    idx = idx.contiguous()
    vals = vals.contiguous()
    if vals.dim() != 1 or vals.element_size() not in (4, 8):
        raise ValueError("vals must be 1-D with 4- or 8-byte elements")
    if out is None:
        out = torch.empty(n_dst, dtype=vals.dtype, device=vals.device)
    if verdict is None:
        verdict = torch.empty(3, dtype=torch.int64, device=vals.device)
    ws = workspace(L.lib().ixp_scatter_checked_workspace(n_dst), vals.device, "checked")
    rc = L.lib().ixp_scatter_checked(_ptr(out), n_dst, _ptr(idx), _IDX_T[idx.dtype], _ptr(vals),
                                     idx.shape[0], vals.element_size(), _ptr(verdict), _ptr(ws),
                                     ws.numel(), _stream_ptr(vals.device))
    L.check(rc, "ixp_scatter_checked")
    return out, verdict


def zero_(t: torch.Tensor) -> torch.Tensor:
    """Zeroes a contiguous tensor with the library's fill kernel."""
    _check_dev(t)
    if not t.is_contiguous():
        raise ValueError("zero_ needs a contiguous tensor")
    rc = L.lib().ixp_zero(_ptr(t), t.numel() * t.element_size(), _stream_ptr(t.device))
    L.check(rc, "ixp_zero")
    return t


def match_min(hist: torch.Tensor, idx: torch.Tensor, vals: torch.Tensor,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """uint8 flags: hist[idx[k]] == vals[k] for in-range idx[k]."""
    _check_dev(hist, idx, vals)
    idx = idx.contiguous()
    vals = vals.contiguous()
    m = idx.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.uint8, device=idx.device)
    rc = L.lib().ixp_match_min(_ptr(out), _ptr(hist), hist.shape[0], _ptr(idx), _IDX_T[idx.dtype],
                               _ptr(vals), m, _stream_ptr(idx.device))
    L.check(rc, "ixp_match_min")
    return out


class SmallestPairs:
    """get_smallest_pairs (Sections 5.4 and 6, maximal matching) on the device, with
    buffers kept across calls: H = hist min over es with values is, keep
    entry k iff H[es[k]] == is[k], and filter es and is by the kept flags
    (positions from a filter over the flags, then two 8-byte scatters).
    ``run`` enqueues everything without a host synchronisation and leaves the
    number of kept pairs in ``split``; ``__call__`` returns the trimmed
    outputs (synchronising)."""

    def __init__(self, n_verts: int, n_es: int, es: torch.Tensor, is_: torch.Tensor):
        _check_dev(es, is_)
        if es.dtype != torch.int64 or is_.dtype != torch.int64 or es.shape != is_.shape:
            raise ValueError("es and is must be int64 arrays of one length")
        self.n_verts, self.n_es = int(n_verts), int(n_es)
        self.es, self.is_ = es.contiguous(), is_.contiguous()
        m = es.shape[0]
        dev = es.device
        self.hist = torch.empty(max(self.n_verts, 1), dtype=torch.int64, device=dev)
        self.flags = torch.empty(m, dtype=torch.uint8, device=dev)
        self.pos = torch.empty(m, dtype=torch.int64, device=dev)
        self.es_out = torch.empty(m, dtype=torch.int64, device=dev)
        self.is_out = torch.empty(m, dtype=torch.int64, device=dev)
        self.split = torch.empty(1, dtype=torch.int64, device=dev)
        self.ws = torch.empty(max(L.lib().ixp_partition_workspace(m), 256), dtype=torch.uint8, device=dev)
        self._pred = Pred.from_flags(self.flags).c()

    def run(self):
        lib, m, st = L.lib(), self.es.shape[0], _stream_ptr(self.es.device)
        L.check(lib.ixp_hist_min(_ptr(self.hist), self.n_verts, self.n_es, _ptr(self.es), L.I64,
                                 _ptr(self.is_), m, st), "ixp_hist_min")
        L.check(lib.ixp_match_min(_ptr(self.flags), _ptr(self.hist), self.n_verts, _ptr(self.es), L.I64,
                                  _ptr(self.is_), m, st), "ixp_match_min")
        L.check(lib.ixp_partition(None, L.I32, m, ctypes.byref(self._pred), L.MODE_FILTER, None,
                                  _ptr(self.pos), L.I64, _ptr(self.split), _ptr(self.ws), self.ws.numel(), st),
                "ixp_partition")
        for src, dst in ((self.es, self.es_out), (self.is_, self.is_out)):
            L.check(lib.ixp_scatter_inj(_ptr(dst), m, _ptr(self.pos), L.I64, _ptr(src), m, 8, st),
                    "ixp_scatter_inj")
        return self.es_out, self.is_out, self.split

    def __call__(self):
        self.run()
        c = int(self.split.item())
        return self.es_out[:c], self.is_out[:c]


def get_smallest_pairs(n_verts: int, n_es: int, es: torch.Tensor, is_: torch.Tensor):
    """(es', is'): the entries whose id is the least id at their endpoint."""
    return SmallestPairs(n_verts, n_es, es, is_)()


class PartitionScatter(torch.autograd.Function):
    """Differentiable partition of a payload carried by its keys.

    forward(keys, payload, pred, mode): the partition2 indices of ``keys``
    (from the HIP partition; int32 when n < 2^31, else int64) move every
    payload row to its partitioned position with the atomic-free row scatter;
    returns (y, partitioned keys, indices, split).  In FILTER mode y holds the kept rows
    first (its remaining rows are zero).
    backward: the indices are a bijection onto [0, n) (PARTITION) or an
    injection into [0, split) (FILTER), so the gradient of a row is the
    upstream gradient at its destination -- one row gather; dropped rows (index
    -1) get zero.
    """

    @staticmethod
    def forward(ctx, keys, payload, pred, mode=L.MODE_PARTITION):
        # narrower indices move fewer bytes in both directions
        idx_dtype = torch.int32 if keys.numel() < (1 << 31) else torch.int64
        ok, idx, split = partition(keys, pred, mode, idx_dtype)
        y = torch.zeros_like(payload) if mode == L.MODE_FILTER else torch.empty_like(payload)
        scatter_inj(y, idx, payload)
        ctx.save_for_backward(idx)
        ctx.mark_non_differentiable(ok, idx, split)
        return y, ok, idx, split

    @staticmethod
    def backward(ctx, gy, *unused):
        (idx,) = ctx.saved_tensors
        return None, gather(gy, idx), None, None


def partition_scatter(keys, payload, pred, mode=L.MODE_PARTITION):
    return PartitionScatter.apply(keys, payload, pred, mode)


def _tune_cache_path():
    import os
    return os.environ.get("IXP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ixpart", "tune.json"))


def autotuned_tiling(keys, shape, pred, mode=L.MODE_PARTITION, idx_dtype=torch.int32,
                     want_flags=True, reps: int = 5):
    """Tiling for a segmented call from the autotuner cache (a JSON file keyed
    by GPU architecture, key dtype, mode, index dtype and the power-of-two bins
    of n and m; path in $IXP_TUNE_CACHE), running the tuner on a miss."""
    import json
    import math
    import os
    arch = torch.cuda.get_device_properties(keys.device).gcnArchName.split(":")[0]
    n, m = keys.numel(), shape.numel()
    key = "|".join(["tiling+rowsync", arch, str(keys.dtype), str(mode), str(idx_dtype), pred.kind.__str__(),
                    f"n2^{int(math.log2(max(n, 1)))}", f"m2^{int(math.log2(max(m, 1)))}"])
    path = _tune_cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return tuple(cache[key]["tiling"]), cache[key]["ms"], True
    tiling, ms = tune_segmented(keys, shape, pred, mode, idx_dtype, want_flags, reps)
    cache[key] = {"tiling": list(tiling), "ms": ms}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return tiling, ms, False
