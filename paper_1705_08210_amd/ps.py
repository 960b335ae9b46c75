"""ctypes binding of libps (include/ps.h).

Argument marshalling only: tensors are checked and their device pointers,
sizes and the current HIP stream are passed to the C ABI, where every step of
the computation runs in HIP kernels.  PyTorch provides device memory and
streams.  There is no fallback: if libps.so is missing, importing this module
fails.
"""

from __future__ import annotations

import contextlib
import ctypes
import os
import re

import torch  # load torch's HIP runtime first; libps binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libps.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ps.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                      "(or python paper_1705_08210_amd/csrc/build.py)")

lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
SZ = ctypes.c_size_t

PS_F32, PS_F16, PS_U8, PS_F64 = 0, 1, 2, 3
ACC = {"plain": 0, "blocked": 1, "auto": 2}
PATH = {"auto": 0, "valu": 1, "mfma": 2, "mfma_fp4": 3, "bits": 4}
DTYPES = {torch.float32: PS_F32, torch.float16: PS_F16, torch.uint8: PS_U8,
          torch.float64: PS_F64}


class Opts(ctypes.Structure):
    _fields_ = [("acc", I32), ("path", I32), ("levels", I32), ("tile", I32)]


class Problem(ctypes.Structure):
    _fields_ = [("V", P), ("n_f", I64), ("n_v", I64), ("ld", I64), ("s", P),
                ("c2", P), ("n2", P)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ps_status_string", ctypes.c_char_p, [ctypes.c_int])
_sig("ps_last_error", ctypes.c_char_p, [])
_sig("ps_version", I32, [])
_sig("ps_vector_sums", ctypes.c_int, [P, I32, I64, I64, I64, P, P, P])
_sig("ps2_workspace_size", SZ, [I32, I64, I64, I32, ctypes.POINTER(Opts)])
_sig("ps2_compute", ctypes.c_int,
     [P, I32, I64, I64, I64, P, P, P, P, SZ, ctypes.POINTER(Opts), P])
_sig("ps2_compute_shard", ctypes.c_int,
     [P, I32, I64, I64, I64, P, P, P, I64, I64, P, SZ, ctypes.POINTER(Opts), P])
_sig("ps3_workspace_size", SZ, [I32, I64, I64, I32, I32, I64, I64, ctypes.POINTER(Opts)])
_sig("ps3_compute", ctypes.c_int,
     [P, I32, I64, I64, I64, P, P, I64, I64, P, P, SZ, ctypes.POINTER(Opts), P])
_sig("ps3_compute_noalloc", ctypes.c_int,
     [P, I32, I64, I64, I64, P, P, I64, I64, P, ctypes.POINTER(Opts), P])
_sig("ps3_stage_size", I64, [I64, I64, I64])
_sig("ps2_batched_workspace_size", SZ, [ctypes.POINTER(Problem), I32, I32,
                                        ctypes.POINTER(Opts)])
_sig("ps2_compute_batched", ctypes.c_int,
     [ctypes.POINTER(Problem), I32, I32, P, SZ, ctypes.POINTER(Opts), P])
_sig("ps_plan_create_batched", ctypes.c_int,
     [ctypes.POINTER(P), ctypes.POINTER(Problem), I32, I32, ctypes.POINTER(Opts), P, SZ, P])
_sig("ps_plan_create_3way", ctypes.c_int,
     [ctypes.POINTER(P), P, I32, I64, I64, I64, P, P, I64, I64, P, P, SZ, ctypes.POINTER(Opts)])
_sig("ps_plan_execute", ctypes.c_int, [P, P])
_sig("ps_plan_destroy", None, [P])
_sig("ps_tile_config", I32, [I32, I32, I32, I32, ctypes.POINTER(I32),
                             ctypes.POINTER(I32), ctypes.POINTER(I32)])
_sig("ps_tune_register", ctypes.c_int, [I32, I32, I32, I64, I64, I64, I64, I32])
_sig("ps_tune_clear", None, [])
_sig("ps_path_choice", I32, [I32, I32, I64, I64, I64, ctypes.POINTER(Opts)])
_sig("ps_quantize_u8", ctypes.c_int, [P, I64, P, P])
_sig("ps_threshold_workspace_size", SZ, [I64])
_sig("ps_threshold", ctypes.c_int, [P, I64, ctypes.c_float, I64, P, P, I64, P, P, SZ, P])
_sig("ps_clock_probe_workspace_size", SZ, [])
_sig("ps_clock_probe", ctypes.c_int, [I64, P, SZ, P])


def header_functions() -> list[str]:
    """Names of the functions declared in include/ps.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(ps\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


class PSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{lib.ps_status_string(status).decode()}: {msg}")
        self.status = status


def _check(st: int) -> None:
    if st != 0:
        raise PSError(st, lib.ps_last_error().decode())


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _on(stream):
    """Allocation context of a call: with an explicit stream, the binding's
    allocations (workspace, outputs) are made on that stream, so the caching
    allocator never hands their blocks to other work while the library's
    kernels on `stream` may still use them."""
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


def _opts(acc="auto", path="auto", levels=0, tile=0) -> Opts:
    return Opts(ACC[acc] if isinstance(acc, str) else int(acc),
                PATH[path] if isinstance(path, str) else int(path), int(levels), int(tile))


def _matrix(V: torch.Tensor):
    if not isinstance(V, torch.Tensor) or V.dim() != 2:
        raise ValueError("V must be a 2-D tensor of shape (n_v, n_f)")
    if not V.is_cuda:
        raise ValueError("V must be on a GPU (device memory)")
    if V.dtype not in DTYPES:
        raise TypeError(f"unsupported dtype {V.dtype}; use float32, float16, uint8 or float64")
    if V.shape[1] > 1 and V.stride(1) != 1:
        raise ValueError("the fields of a vector must be contiguous (V.stride(1) == 1)")
    n_v, n_f = V.shape
    ld = V.stride(0) if n_v > 1 else max(n_f, 1)
    return DTYPES[V.dtype], n_f, n_v, max(ld, n_f, 1)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _workspace(nbytes: int, device) -> torch.Tensor:
    # 256-byte alignment: torch's caching allocator returns 512-byte aligned
    # blocks
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def n2_dtype(V_dtype) -> torch.dtype:
    if V_dtype == torch.uint8:
        return torch.int32
    return torch.float64 if V_dtype == torch.float64 else torch.float32


def vector_sums(V: torch.Tensor, out: torch.Tensor | None = None, want_bad: bool = True,
                stream=None):
    """s_i = sum_q V[i, q] (FP64) and, if want_bad, the count of negative,
    NaN or infinite entries (as a 1-element int32 tensor)."""
    dt, n_f, n_v, ld = _matrix(V)
    with _on(stream):
        s = out if out is not None else torch.empty(n_v, dtype=torch.float64, device=V.device)
        bad = torch.empty(1, dtype=torch.int32, device=V.device) if want_bad else None
        _check(lib.ps_vector_sums(V.data_ptr(), dt, n_f, n_v, ld, s.data_ptr(), _ptr(bad),
                                  _stream(stream)))
    return s, bad


def ps2(V: torch.Tensor, s: torch.Tensor | None = None, want_c2: bool = True,
        want_n2: bool = False, acc="auto", path="auto", levels=0, tile=0,
        c2: torch.Tensor | None = None, n2: torch.Tensor | None = None, stream=None):
    """2-way metric of all pairs i<j, colex packed.  Returns (c2, n2); either
    may be None when not requested."""
    dt, n_f, n_v, ld = _matrix(V)
    m = n_v * (n_v - 1) // 2
    with _on(stream):
        if want_c2 and c2 is None:
            c2 = torch.empty(m, dtype=torch.float32, device=V.device)
        if want_n2 and n2 is None:
            n2 = torch.empty(m, dtype=n2_dtype(V.dtype), device=V.device)
        o = _opts(acc, path, levels, tile)
        ws_n = lib.ps2_workspace_size(dt, n_f, n_v, int(s is not None), ctypes.byref(o))
        ws = _workspace(ws_n, V.device)
        _check(lib.ps2_compute(V.data_ptr(), dt, n_f, n_v, ld, _ptr(s), _ptr(c2), _ptr(n2),
                               ws.data_ptr(), ws.numel(), ctypes.byref(o), _stream(stream)))
    return c2, n2


def ps2_shard(V: torch.Tensor, shard: int, nshards: int, s: torch.Tensor | None = None,
              want_c2: bool = True, want_n2: bool = False, acc="auto", path="auto", levels=0,
              tile=0, c2: torch.Tensor | None = None, n2: torch.Tensor | None = None,
              stream=None):
    """One GPU's share of ps2 when the pairs are spread over nshards GPUs by
    tiles (ps2_compute_shard): writes the full-size colex c2 / n2 at the pairs
    of the upper-triangle tiles t with t % nshards == shard only, with the
    same tile configuration and accumulation plan as ps2.  Returns (c2, n2)."""
    dt, n_f, n_v, ld = _matrix(V)
    m = n_v * (n_v - 1) // 2
    with _on(stream):
        if want_c2 and c2 is None:
            c2 = torch.empty(m, dtype=torch.float32, device=V.device)
        if want_n2 and n2 is None:
            n2 = torch.empty(m, dtype=n2_dtype(V.dtype), device=V.device)
        o = _opts(acc, path, levels, tile)
        ws_n = lib.ps2_workspace_size(dt, n_f, n_v, int(s is not None), ctypes.byref(o))
        ws = _workspace(ws_n, V.device)
        _check(lib.ps2_compute_shard(V.data_ptr(), dt, n_f, n_v, ld, _ptr(s), _ptr(c2),
                                     _ptr(n2), shard, nshards, ws.data_ptr(), ws.numel(),
                                     ctypes.byref(o), _stream(stream)))
    return c2, n2


def stage_size(n_v: int, j_begin: int, j_end: int) -> int:
    return int(lib.ps3_stage_size(n_v, j_begin, j_end))


def ps3(V: torch.Tensor, s: torch.Tensor | None = None, n2: torch.Tensor | None = None,
        j_begin: int = 1, j_end: int | None = None, acc="auto", tile=0,
        c3: torch.Tensor | None = None, stream=None, path="auto",
        levels=0) -> torch.Tensor:
    """3-way metric of the triples i<j<k with j in [j_begin, j_end), j-slab
    packed from offset 0.  path "bits" (with levels=1) for binary uint8 data;
    "mfma" / "mfma_fp4" (with levels >= max(V)) for uint8 levels."""
    dt, n_f, n_v, ld = _matrix(V)
    if j_end is None:
        j_end = max(n_v - 1, j_begin)
    m = stage_size(n_v, j_begin, j_end)
    with _on(stream):
        if c3 is None:
            c3 = torch.empty(m, dtype=torch.float32, device=V.device)
        o = _opts(acc, path, levels, tile)
        ws_n = lib.ps3_workspace_size(dt, n_f, n_v, int(s is not None), int(n2 is not None),
                                      j_begin, j_end, ctypes.byref(o))
        ws = _workspace(ws_n, V.device)
        _check(lib.ps3_compute(V.data_ptr(), dt, n_f, n_v, ld, _ptr(s), _ptr(n2), j_begin,
                               j_end, c3.data_ptr() if m > 0 else None, ws.data_ptr(),
                               ws.numel(), ctypes.byref(o), _stream(stream)))
    return c3


def noalloc_scratch_bytes() -> int:
    """PS_NOALLOC_SCRATCH_BYTES of include/ps.h: the static scratch per GPU
    behind ps3_compute_noalloc."""
    m = re.search(r"#define\s+PS_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)",
                  open(HEADER).read())
    return int(m.group(1)) << int(m.group(2))


def ps3_noalloc(V: torch.Tensor, c3: torch.Tensor, s: torch.Tensor | None = None,
                n2: torch.Tensor | None = None, j_begin: int = 1, j_end: int | None = None,
                acc="auto", tile=0, path="auto", levels=0, stream=None) -> torch.Tensor:
    """ps3 through ps3_compute_noalloc: the library takes its scratch from a
    static per-GPU array instead of a workspace, and this wrapper allocates
    nothing either (c3, and s / n2 if given, are the caller's).  Calls that
    overlap on one GPU race on that array."""
    dt, n_f, n_v, ld = _matrix(V)
    if j_end is None:
        j_end = max(n_v - 1, j_begin)
    m = stage_size(n_v, j_begin, j_end)
    if c3.dtype != torch.float32 or not c3.is_cuda or not c3.is_contiguous() or c3.numel() < m:
        raise ValueError(f"c3 must be a contiguous float32 GPU tensor of >= {m} values")
    o = _opts(acc, path, levels, tile)
    _check(lib.ps3_compute_noalloc(V.data_ptr(), dt, n_f, n_v, ld, _ptr(s), _ptr(n2), j_begin,
                                   j_end, c3.data_ptr() if m > 0 else None, ctypes.byref(o),
                                   _stream(stream)))
    return c3


def _problems(Vs, outs):
    arr = (Problem * len(Vs))()
    dt = None
    for t, (V, (c2, n2, s)) in enumerate(zip(Vs, outs)):
        d, n_f, n_v, ld = _matrix(V)
        if dt is None:
            dt = d
        elif d != dt:
            raise TypeError("all problems of a batch must share one dtype")
        arr[t] = Problem(V.data_ptr(), n_f, n_v, ld, _ptr(s), _ptr(c2), _ptr(n2))
    return arr, (dt if dt is not None else PS_F32)


def _batch_outputs(Vs, want_n2=False):
    outs = []
    for V in Vs:
        m = V.shape[0] * (V.shape[0] - 1) // 2
        c2 = torch.empty(m, dtype=torch.float32, device=V.device)
        n2 = torch.empty(m, dtype=n2_dtype(V.dtype), device=V.device) if want_n2 else None
        outs.append((c2, n2, None))
    return outs


def ps2_batched(Vs, outs=None, acc="auto", tile=0, want_n2=False, stream=None):
    """Many independent 2-way problems in one launch.  Returns the
    list of (c2, n2, s) tuples (s is None: sums computed inside)."""
    with _on(stream):
        if outs is None:
            outs = _batch_outputs(Vs, want_n2)
        arr, dt = _problems(Vs, outs)
        o = _opts(acc, "valu", 0, tile)
        ws_n = lib.ps2_batched_workspace_size(arr, len(Vs), dt, ctypes.byref(o))
        dev = Vs[0].device if Vs else torch.device("cuda")
        ws = _workspace(ws_n, dev)
        _check(lib.ps2_compute_batched(arr, len(Vs), dt, ws.data_ptr(), ws.numel(),
                                       ctypes.byref(o), _stream(stream)))
    return outs


class BatchedPlan:
    """A batch captured into a HIP graph (table writes included); run()
    replays it."""

    def __init__(self, Vs, outs=None, acc="auto", tile=0, want_n2=False, stream=None):
        self.Vs = list(Vs)
        with _on(stream):
            self.outs = outs if outs is not None else _batch_outputs(self.Vs, want_n2)
            arr, dt = _problems(self.Vs, self.outs)
            self._arr = arr
            o = _opts(acc, "valu", 0, tile)
            ws_n = lib.ps2_batched_workspace_size(arr, len(self.Vs), dt, ctypes.byref(o))
            dev = self.Vs[0].device if self.Vs else torch.device("cuda")
            self.ws = _workspace(ws_n, dev)
            self._home = torch.cuda.current_stream(dev)
        h = P()
        _check(lib.ps_plan_create_batched(ctypes.byref(h), arr, len(self.Vs), dt,
                                          ctypes.byref(o), self.ws.data_ptr(),
                                          self.ws.numel(), _stream(stream)))
        self._h = h

    def run(self, stream=None):
        s = torch.cuda.current_stream() if stream is None else stream
        if s != self._home:   # keep the workspace from reuse while this replay runs
            self.ws.record_stream(s)
        _check(lib.ps_plan_execute(self._h, s.cuda_stream))
        return self.outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.ps_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan3:
    """A 3-way stage captured into a HIP graph (ps_plan_create_3way); run()
    replays it.  V, s, n2 and c3 are kept alive by the plan; their contents
    may change between replays."""

    def __init__(self, V, s=None, n2=None, j_begin: int = 1, j_end: int | None = None,
                 acc="auto", tile=0, path="auto", levels=0, c3=None):
        dt, n_f, n_v, ld = _matrix(V)
        if j_end is None:
            j_end = max(n_v - 1, j_begin)
        m = stage_size(n_v, j_begin, j_end)
        self.V, self.s, self.n2 = V, s, n2
        self.c3 = c3 if c3 is not None else torch.empty(m, dtype=torch.float32, device=V.device)
        o = _opts(acc, path, levels, tile)
        ws_n = lib.ps3_workspace_size(dt, n_f, n_v, int(s is not None), int(n2 is not None),
                                      j_begin, j_end, ctypes.byref(o))
        self.ws = _workspace(ws_n, V.device)
        self._home = torch.cuda.current_stream(V.device)
        h = P()
        _check(lib.ps_plan_create_3way(ctypes.byref(h), V.data_ptr(), dt, n_f, n_v, ld, _ptr(s),
                                       _ptr(n2), j_begin, j_end,
                                       self.c3.data_ptr() if m > 0 else None,
                                       self.ws.data_ptr(), self.ws.numel(), ctypes.byref(o)))
        self._h = h

    def run(self, stream=None):
        s = torch.cuda.current_stream() if stream is None else stream
        if s != self._home:
            self.ws.record_stream(s)
        _check(lib.ps_plan_execute(self._h, s.cuda_stream))
        return self.c3

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.ps_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_configs(dtype=torch.float32, way: int = 2, path: str = "valu"):
    """List of (bm, bn, bk) of the compiled tile configurations."""
    dt = DTYPES[dtype]
    bm, bn, bk = I32(), I32(), I32()
    n = lib.ps_tile_config(dt, way, PATH[path], 0, None, None, None)
    out = []
    for i in range(n):
        lib.ps_tile_config(dt, way, PATH[path], i, ctypes.byref(bm), ctypes.byref(bn),
                           ctypes.byref(bk))
        out.append((bm.value, bn.value, bk.value))
    return out


def tune_register(dtype, way, path, nf_range, nv_range, idx) -> None:
    _check(lib.ps_tune_register(DTYPES[dtype], way, PATH[path], nf_range[0], nf_range[1],
                                nv_range[0], nv_range[1], idx))


def tune_clear() -> None:
    lib.ps_tune_clear()


def path_choice(dtype, way: int, n_f: int, n_v: int, ld: int | None = None, path="auto",
                levels=0, tile=0, acc="auto") -> int:
    """The ps_path code that ps2 (way 2) / ps3 (way 3) run for these
    arguments (AUTO resolved by the library's policy and tuning table).
    dtype: a torch or numpy dtype."""
    import numpy as np
    dt = DTYPES[dtype] if dtype in DTYPES else {np.dtype(np.float32): PS_F32,
                                                 np.dtype(np.float16): PS_F16,
                                                 np.dtype(np.uint8): PS_U8,
                                                 np.dtype(np.float64): PS_F64}[np.dtype(dtype)]
    o = _opts(acc, path, levels, tile)
    return int(lib.ps_path_choice(dt, way, n_f, n_v, n_f if ld is None else ld, ctypes.byref(o)))


def quantize_u8(c: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """One byte per metric: round-half-even(255 * clamp(c, 0, 1))."""
    if c.dtype != torch.float32 or not c.is_cuda or not c.is_contiguous():
        raise ValueError("c must be a contiguous float32 GPU tensor")
    n = c.numel()
    with _on(stream):
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=c.device)
        _check(lib.ps_quantize_u8(c.data_ptr() if n else None, n,
                                  out.data_ptr() if n else None, _stream(stream)))
    return out


def threshold(c: torch.Tensor, thr: float, base: int = 0, cap: int | None = None,
              stream=None):
    """Entries with c >= thr in index order: (idx int64, val float32, count)
    device tensors; idx = base + position; only the first cap are written."""
    if c.dtype != torch.float32 or not c.is_cuda or not c.is_contiguous():
        raise ValueError("c must be a contiguous float32 GPU tensor")
    n = c.numel()
    cap = n if cap is None else int(cap)
    with _on(stream):
        idx = torch.empty(max(cap, 1), dtype=torch.int64, device=c.device)
        val = torch.empty(max(cap, 1), dtype=torch.float32, device=c.device)
        count = torch.empty(1, dtype=torch.int64, device=c.device)
        ws = _workspace(lib.ps_threshold_workspace_size(n), c.device)
        _check(lib.ps_threshold(c.data_ptr() if n else None, n, float(thr), int(base),
                                idx.data_ptr(), val.data_ptr(), cap, count.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream)))
    return idx, val, count


def clock_probe(iters: int = 200000, stream=None) -> float:
    """Mean shader clock in GHz under a full vector-ALU load (a measurement
    aid; synchronises)."""
    with _on(stream):
        ws = _workspace(lib.ps_clock_probe_workspace_size(), torch.device("cuda"))
        _check(lib.ps_clock_probe(int(iters), ws.data_ptr(), ws.numel(), _stream(stream)))
        torch.cuda.synchronize()
        v = ws.view(torch.int64).reshape(-1, 3).cpu()
    return float(v[:, 0].sum()) / float(v[:, 1].sum()) / 10.0


# The C ABI's names (include/ps.h) for the same calls.
ps_vector_sums = vector_sums
ps2_compute = ps2
ps2_compute_shard = ps2_shard
ps3_compute = ps3
ps3_compute_noalloc = ps3_noalloc
ps2_compute_batched = ps2_batched
ps3_stage_size = stage_size
