"""Per-rank, column-based (sparsity-aware) SpMM of SHIRO on MI355X (gfx950).

Thin Python binding over libshiro.so (C ABI in include/shiro.h).  The
functions keep the C names without the prefix: partition, select_rows,
pack_B, spmm, spmm_backward (plus prepare, autotune, tuning and graph
capture).  PyTorch provides device memory and the stream; every step of
the path runs in the library's HIP kernels.  There is no CPU fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
from typing import Optional, Tuple

import torch

from . import _lib
from ._lib import ShiroError, Tuning  # noqa: F401

__all__ = [
    "Plan",
    "ShiroError",
    "partition",
    "select_rows",
    "selection",
    "refresh_selection",
    "block_nnz",
    "pack_B",
    "spmm",
    "spmm_backward",
    "spmm_noalloc",
    "select_c_rows",
    "c_row_selection",
    "partial_c",
    "aggregate_c",
    "partition_subset",
    "JointSpMM",
    "JointSpMMFunction",
    "mvc_bipartite",
    "joint_plan",
    "prepare",
    "autotune",
    "get_tuning",
    "set_tuning",
    "ShiroSpMM",
    "shiro_spmm",
    "use_torch_allocator",
    "version",
]

_DT = {torch.float32: _lib.F32, torch.bfloat16: _lib.BF16}
_KERNELS = {"spmm": _lib.KERNEL_SPMM, "spmm_t": _lib.KERNEL_SPMM_T, "sddmm": _lib.KERNEL_SDDMM,
            "partial_c": _lib.KERNEL_PARTIAL_C, "aggregate_c": _lib.KERNEL_AGGREGATE_C}


def _L():
    return _lib.load()


# ---------------------------------------------------------------------------
# allocator hook: the library's device memory from torch's caching allocator
# ---------------------------------------------------------------------------
_alloc_hooks = None  # keeps the ctypes callbacks alive while installed


def use_torch_allocator(enable: bool = True) -> None:
    """Route the library's own device allocations through torch's caching
    allocator (so torch.cuda.memory_allocated() accounts for plans), or back
    to hipMalloc with enable=False.  Affects allocations made afterwards."""
    global _alloc_hooks
    if not enable:
        _lib.check(_L().shiro_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None))
        _alloc_hooks = None
        return

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def _free(ptr, nbytes, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    _lib.check(_L().shiro_set_allocator(hooks[0], hooks[1], None))
    _alloc_hooks = hooks


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dt(t: torch.dtype) -> int:
    if t not in _DT:
        raise TypeError(f"unsupported dtype {t}: float32 or bfloat16")
    return _DT[t]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        raise ValueError("dense operands must be 2-D")
    if t.numel() == 0:  # an empty operand has no meaningful strides
        return max(t.shape[1], 1)
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError("dense operands must be row-major with unit column stride")
    return t.stride(0)


def _dev(t: torch.Tensor):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("operands must be tensors on the GPU")


def _mat(t: Optional[torch.Tensor], name: str, min_rows: int, N: int, dtypes=None):
    """Check a dense operand before its pointer reaches the library: on the
    GPU, 2-D, at least min_rows rows of exactly N columns, row-major with unit
    column stride, of an allowed dtype."""
    if t is None:
        return
    _dev(t)
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.shape[0] < min_rows or t.shape[1] != N:
        raise ValueError(f"{name} must have at least {min_rows} rows and {N} columns, got {tuple(t.shape)}")
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError(f"{name} must be one of {dtypes}, got {t.dtype}")
    _ld(t)


def _vec(t: Optional[torch.Tensor], name: str, min_numel: int):
    """Check a float32 vector indexed like the CSR's nonzeros (vals, dvals)."""
    if t is None:
        return
    _dev(t)
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name} must have at least {min_numel} entries (indexed like the CSR's nonzeros), "
                         f"got {t.numel()}")


def version() -> int:
    return int(_L().shiro_version())


class Plan:
    """Library-owned plan of rank p's panel (freed when garbage collected)."""

    def __init__(self, handle: int, device: torch.device, value_extent: Optional[int] = None):
        self._h = ctypes.c_void_p(handle)
        self.device = device
        self._graphs = []
        inf = self.info()
        # entries of the CSR's value array the plan reads (vals, dvals)
        self.value_extent = value_extent if value_extent is not None else inf["nz_begin"] + inf["nnz"]
        self.R = None  # sum of |Rows(A^(p,q))| once select_c_rows ran

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _lib.PlanInfo()
        _lib.check(_L().shiro_plan_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def __getattr__(self, name):
        if name in ("n_rows", "n_cols", "P", "p", "M", "K", "row_begin", "rows", "nz_begin", "nnz", "U"):
            return self.info()[name]
        raise AttributeError(name)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L().shiro_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # HIP graph capture of pack_B / spmm / spmm_backward calls
    @contextlib.contextmanager
    def capture(self, stream: torch.cuda.Stream):
        """Record the library calls issued on `stream` inside the block.

        Yields a list that receives the graph id once capture ends."""
        holder = []
        _lib.check(_L().shiro_graph_begin(self._h, ctypes.c_void_p(stream.cuda_stream)))
        try:
            with torch.cuda.stream(stream):
                yield holder
        finally:
            gid = ctypes.c_int32(-1)
            _lib.check(_L().shiro_graph_end(self._h, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(gid)))
            holder.append(gid.value)

    def replay(self, graph_id: int, stream=None):
        _lib.check(_L().shiro_graph_launch(self._h, int(graph_id), ctypes.c_void_p(_stream(stream))))


def partition(row_ptr: torch.Tensor, col: torch.Tensor, n_rows: int, n_cols: int, P: int, p: int,
              check: bool = False, stream=None) -> Plan:
    """Plan of panel p of P for the CSR (row_ptr int64[n_rows+1], col int32[nnz])."""
    _dev(row_ptr)
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col int32")
    if row_ptr.numel() != n_rows + 1:
        raise ValueError("row_ptr must have n_rows + 1 entries")
    _dev(col)
    h = ctypes.c_void_p()
    nnz = col.numel()
    _lib.check(_L().shiro_partition(int(n_rows), int(n_cols), int(nnz), _ptr(row_ptr.contiguous()),
                                    _ptr(col.contiguous()) if nnz else None, int(P), int(p),
                                    _lib.CHECK_CSR if check else 0, ctypes.c_void_p(_stream(stream)),
                                    ctypes.byref(h)))
    return Plan(h.value, row_ptr.device)


def partition_subset(row_ptr: torch.Tensor, col: torch.Tensor, n_rows: int, n_cols: int, P: int, p: int,
                     keep: torch.Tensor, keep_value: int, check: bool = False, stream=None) -> Plan:
    """Plan over the panel's nonzeros k with keep[k] == keep_value (keep: uint8
    on the device, one entry per nonzero of panel p)."""
    _dev(row_ptr)
    _dev(col)
    _dev(keep)
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or keep.dtype != torch.uint8:
        raise TypeError("row_ptr int64, col int32, keep uint8")
    if row_ptr.numel() != n_rows + 1:
        raise ValueError("row_ptr must have n_rows + 1 entries")
    if P < 1 or not 0 <= p < P:
        raise ValueError("need P >= 1 and 0 <= p < P")
    M = -(-n_rows // P)
    r0, r1 = min(p * M, n_rows), min(p * M + M, n_rows)
    nz0, nz1 = int(row_ptr[r0].item()), int(row_ptr[r1].item())
    if keep.numel() < nz1 - nz0:
        raise ValueError(f"keep must have one entry per panel nonzero ({nz1 - nz0}), got {keep.numel()}")
    h = ctypes.c_void_p()
    nnz = col.numel()
    _lib.check(_L().shiro_partition_subset(int(n_rows), int(n_cols), int(nnz), _ptr(row_ptr.contiguous()),
                                           _ptr(col.contiguous()) if nnz else None, _ptr(keep.contiguous()),
                                           int(keep_value), int(P), int(p), _lib.CHECK_CSR if check else 0,
                                           ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    return Plan(h.value, row_ptr.device, value_extent=nz1)


def select_rows(plan: Plan, stream=None) -> Tuple[int, list]:
    """Run the selection; returns (U, [|Cols_q| for q in range(P)])."""
    P = plan.info()["P"]
    U = ctypes.c_int64()
    per = (ctypes.c_int64 * P)()
    _lib.check(_L().shiro_select_rows(plan.handle, ctypes.c_void_p(_stream(stream)), ctypes.byref(U), per))
    return U.value, list(per)


def refresh_selection(plan: Plan, stream=None):
    """Re-run the selection kernels (stream-ordered, no sync; capturable)."""
    _lib.check(_L().shiro_refresh_selection(plan.handle, ctypes.c_void_p(_stream(stream))))


def selection(plan: Plan, stream=None):
    """Copies of (unique_cols int32[U], block_off int64[P+1], colmap int32[nnz])."""
    inf = plan.info()
    if inf["U"] < 0:
        raise ShiroError(-6, "select_rows has not run")
    dev = plan.device
    uc = torch.empty(inf["U"], dtype=torch.int32, device=dev)
    off = torch.empty(inf["P"] + 1, dtype=torch.int64, device=dev)
    cm = torch.empty(inf["nnz"], dtype=torch.int32, device=dev)
    _lib.check(_L().shiro_copy_selection(plan.handle, _ptr(uc), _ptr(off), _ptr(cm), ctypes.c_void_p(_stream(stream))))
    return uc, off, cm


def block_nnz(plan: Plan, stream=None) -> torch.Tensor:
    out = torch.empty(plan.info()["P"], dtype=torch.int64, device=plan.device)
    _lib.check(_L().shiro_block_nnz(plan.handle, _ptr(out), ctypes.c_void_p(_stream(stream))))
    return out


def pack_B(plan: Plan, B: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Bpacked[u] = B[unique_cols[u]] (bit-exact), shape U x N."""
    inf = plan.info()
    U = inf["U"]
    if U < 0:
        raise ShiroError(-6, "pack_B: call select_rows first")
    _dev(B)
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    N = B.shape[1]
    _mat(B, "B", inf["n_cols"], N, tuple(_DT))
    if out is None:
        out = torch.empty(U, N, dtype=B.dtype, device=B.device)
    _mat(out, "out", U, N, (B.dtype,))
    _lib.check(_L().shiro_pack_B(plan.handle, _ptr(B), _ld(B), N, _dt(B.dtype), _ptr(out), _ld(out),
                                 ctypes.c_void_p(_stream(stream))))
    return out


def spmm(plan: Plan, vals: torch.Tensor, Bpacked: torch.Tensor, out: Optional[torch.Tensor] = None,
         out_dtype: Optional[torch.dtype] = None, mode: str = "batched", stream=None) -> torch.Tensor:
    """Y = A^(p,:) Bpacked (rows x N); vals is the CSR's float32 value array."""
    inf = plan.info()
    rows = inf["rows"]
    _dev(Bpacked)
    if Bpacked.dim() != 2:
        raise ValueError("Bpacked must be 2-D")
    N = Bpacked.shape[1]
    _mat(Bpacked, "Bpacked", max(inf["U"], 0), N, tuple(_DT))
    _vec(vals, "vals", plan.value_extent)
    out_dtype = out_dtype or Bpacked.dtype
    if out is None:
        out = torch.empty(rows, N, dtype=out_dtype, device=Bpacked.device)
    _mat(out, "out", rows, N, tuple(_DT))
    if mode not in ("batched", "per_block"):
        raise ValueError("mode must be 'batched' or 'per_block'")
    m = {"batched": _lib.MODE_BATCHED, "per_block": _lib.MODE_PER_BLOCK}[mode]
    _lib.check(_L().shiro_spmm(plan.handle, _ptr(vals), _ptr(Bpacked), _ld(Bpacked), N, _dt(Bpacked.dtype),
                               _ptr(out), _ld(out), _dt(out.dtype), m, ctypes.c_void_p(_stream(stream))))
    return out


def spmm_noalloc(plan: Plan, vals: torch.Tensor, Bpacked: torch.Tensor, out: torch.Tensor,
                 stream=None) -> torch.Tensor:
    """The batched spmm into a caller-given `out` through the library's
    allocation-free entry point (fixed device work area; the plan must be
    prepared for (N, dtype) first).  Same result as spmm, bit for bit."""
    inf = plan.info()
    _dev(Bpacked)
    if Bpacked.dim() != 2:
        raise ValueError("Bpacked must be 2-D")
    N = Bpacked.shape[1]
    _mat(Bpacked, "Bpacked", max(inf["U"], 0), N, tuple(_DT))
    _vec(vals, "vals", plan.value_extent)
    _mat(out, "out", inf["rows"], N, tuple(_DT))
    _lib.check(_L().shiro_spmm_noalloc(plan.handle, _ptr(vals), _ptr(Bpacked), _ld(Bpacked), N,
                                       _dt(Bpacked.dtype), _ptr(out), _ld(out), _dt(out.dtype),
                                       ctypes.c_void_p(_stream(stream))))
    return out


def spmm_backward(plan: Plan, vals: torch.Tensor, dY: torch.Tensor, Bpacked: Optional[torch.Tensor],
                  dBpacked: Optional[torch.Tensor] = None, dB: Optional[torch.Tensor] = None,
                  dvals: Optional[torch.Tensor] = None, stream=None, dB_overwrite: bool = False):
    """dBpacked = A^T dY (overwrite), dB[unique_cols] += dBpacked, dvals = SDDMM(dY, Bpacked).

    Pass the output tensors to compute; None skips an output.  With
    dB_overwrite the rows dB[unique_cols] are overwritten instead of added to
    (the other rows are left as they are)."""
    inf = plan.info()
    _dev(dY)
    if dY.dim() != 2:
        raise ValueError("dY must be 2-D")
    N = dY.shape[1]
    dt = _dt(dY.dtype)
    U = max(inf["U"], 0)
    _mat(dY, "dY", inf["rows"], N)
    _mat(Bpacked, "Bpacked", U, N, (dY.dtype,))
    _mat(dBpacked, "dBpacked", U, N, (dY.dtype,))
    _mat(dB, "dB", inf["n_cols"], N, (dY.dtype,))
    if dBpacked is not None or dB is not None:
        _vec(vals, "vals", plan.value_extent)
    _vec(dvals, "dvals", plan.value_extent)
    if dvals is not None and Bpacked is None:
        raise ValueError("dvals needs Bpacked")
    _lib.check(_L().shiro_spmm_backward(
        plan.handle, _ptr(vals), _ptr(dY), _ld(dY), _ptr(Bpacked), _ld(Bpacked) if Bpacked is not None else N,
        N, dt, _ptr(dBpacked), _ld(dBpacked) if dBpacked is not None else N, _ptr(dB),
        _ld(dB) if dB is not None else N, _ptr(dvals), _lib.DB_OVERWRITE if dB_overwrite else 0,
        ctypes.c_void_p(_stream(stream))))
    return dBpacked, dB, dvals


# ---------------------------------------------------------------------------
# row-based scheme: owner-side partial C rows and their sum into the panel
# ---------------------------------------------------------------------------
def select_c_rows(plan: Plan, stream=None) -> Tuple[int, list]:
    """Build Rows(A^(p,q)) for every block; returns (R, [|Rows_q|])."""
    R = ctypes.c_int64()
    per = (ctypes.c_int64 * max(plan.P, 1))()
    _lib.check(_L().shiro_select_c_rows(plan.handle, ctypes.c_void_p(_stream(stream)), ctypes.byref(R), per))
    plan.R = R.value
    return R.value, list(per[:plan.P])


def c_row_selection(plan: Plan, R: int, stream=None):
    """(rows int32[R], rblock_off int64[P+1]) on the plan's device."""
    rows = torch.empty(max(R, 1), dtype=torch.int32, device=plan.device)
    off = torch.empty(plan.P + 1, dtype=torch.int64, device=plan.device)
    _lib.check(_L().shiro_copy_c_row_selection(plan.handle, _ptr(rows), _ptr(off), ctypes.c_void_p(_stream(stream))))
    return rows[:R], off


def partial_c(plan: Plan, vals: torch.Tensor, B: torch.Tensor, R: int, out: Optional[torch.Tensor] = None,
              out_dtype=None, stream=None) -> torch.Tensor:
    """Cp[e] = sum over block q's nonzeros of row Rows_q[t] of vals[k] * B[col[k]] (R x N)."""
    _dev(B)
    if B.dim() != 2:
        raise ValueError("B must be 2-D")
    N = B.shape[1]
    _mat(B, "B", plan.info()["n_cols"], N, tuple(_DT))
    _vec(vals, "vals", plan.value_extent)
    if getattr(plan, "R", None) is not None and R != plan.R:
        raise ValueError(f"R must be the plan's |Rows| total {plan.R}, got {R}")
    if out is None:
        out = torch.empty(R, N, dtype=out_dtype or B.dtype, device=B.device)
    _mat(out, "out", R, N, tuple(_DT))
    _lib.check(_L().shiro_partial_c(plan.handle, _ptr(vals), _ptr(B), _ld(B), N, _dt(B.dtype), _ptr(out), _ld(out),
                                    _dt(out.dtype), ctypes.c_void_p(_stream(stream))))
    return out


def aggregate_c(plan: Plan, Cp: torch.Tensor, out: Optional[torch.Tensor] = None, out_dtype=None,
                accumulate: bool = False, stream=None) -> torch.Tensor:
    """Y[i] = sum over blocks (ascending) of row i's partial rows (rows x N);
    with accumulate the sums are added to `out`."""
    _dev(Cp)
    if Cp.dim() != 2:
        raise ValueError("Cp must be 2-D")
    N = Cp.shape[1]
    _mat(Cp, "Cp", getattr(plan, "R", None) or 0, N, tuple(_DT))
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty(plan.rows, N, dtype=out_dtype or Cp.dtype, device=Cp.device)
    _mat(out, "out", plan.rows, N, tuple(_DT))
    _lib.check(_L().shiro_aggregate_c(plan.handle, _ptr(Cp), _ld(Cp), N, _dt(Cp.dtype), _ptr(out), _ld(out),
                                      _dt(out.dtype), _lib.AGG_ACCUMULATE if accumulate else 0,
                                      ctypes.c_void_p(_stream(stream))))
    return out


class JointSpMM:
    """The joint row-column strategy on panel p (Sec. 5.1 steps 1-5): plan the
    per-block covers on the host, split the panel into a column-based and a
    row-based subset plan, then Y = A_col B (select / pack / spmm) plus the
    row-based partial rows of A_row B summed into Y."""

    def __init__(self, row_ptr, col, n_rows, n_cols, P, p, w_row=None, w_col=None, n_threads=0):
        base = partition(row_ptr, col, n_rows, n_cols, P, p)
        self.assign, self.stats = joint_plan(base, w_row, w_col, n_threads)
        base.close()
        keep = self.assign.to(row_ptr.device)
        if keep.numel() == 0:
            keep = torch.zeros(1, dtype=torch.uint8, device=row_ptr.device)
        self.col_plan = partition_subset(row_ptr, col, n_rows, n_cols, P, p, keep, 0)
        self.row_plan = partition_subset(row_ptr, col, n_rows, n_cols, P, p, keep, 1)
        self.U, self.Uq = select_rows(self.col_plan)
        self.R, self.Rq = select_c_rows(self.row_plan)
        # the row-based part's own column selection serves its backward
        self.U_row, _ = select_rows(self.row_plan)

    def prepare(self, N: int, dtype=torch.float32, backward: bool = False):
        prepare(self.col_plan, N, dtype, ops=("spmm", "backward") if backward else ("spmm",))
        prepare(self.row_plan, N, dtype, ops=("row_based", "backward") if backward else ("row_based",))

    def forward(self, vals: torch.Tensor, B: torch.Tensor, out: Optional[torch.Tensor] = None,
                Bp: Optional[torch.Tensor] = None, Cp: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        Bp = pack_B(self.col_plan, B, out=Bp, stream=stream)
        Y = spmm(self.col_plan, vals, Bp, out=out, stream=stream)
        Cp = partial_c(self.row_plan, vals, B, self.R, out=Cp, stream=stream)
        return aggregate_c(self.row_plan, Cp, out=Y, accumulate=True, stream=stream)

    def backward(self, vals: torch.Tensor, B: torch.Tensor, dY: torch.Tensor, dB: Optional[torch.Tensor] = None,
                 dvals: Optional[torch.Tensor] = None, stream=None):
        """Gradients of <dY, Y> with Y = forward(vals, B): dB (zero-filled, the
        shape of B) and dvals (float32 like vals, the panel's entries).  The
        column-based part writes its columns' rows of dB, the row-based part
        adds its own; each part gives the value gradients of its nonzeros."""
        if dB is None:
            dB = torch.zeros_like(B)
        if dvals is None:
            dvals = torch.zeros_like(vals)
        Bp = pack_B(self.col_plan, B, stream=stream)
        spmm_backward(self.col_plan, vals, dY, Bp, None, dB, dvals, stream=stream, dB_overwrite=True)
        if self.R > 0:
            Bpr = pack_B(self.row_plan, B, stream=stream)
            spmm_backward(self.row_plan, vals, dY, Bpr, None, dB, dvals, stream=stream)
        return dB, dvals


class JointSpMMFunction(torch.autograd.Function):
    """Y = A^(p,:) B through the joint strategy, with gradients for the values
    and for B (the backward of JointSpMM)."""

    @staticmethod
    def forward(ctx, vals, B, js):
        ctx.js = js
        ctx.save_for_backward(vals, B)
        return js.forward(vals, B)

    @staticmethod
    def backward(ctx, dY):
        vals, B = ctx.saved_tensors
        dB, dvals = ctx.js.backward(vals, B, dY.to(B.dtype).contiguous())
        return (dvals if ctx.needs_input_grad[0] else None), (dB if ctx.needs_input_grad[1] else None), None


# ---------------------------------------------------------------------------
# joint row-column strategy (host planner)
# ---------------------------------------------------------------------------
def _host_i64(a, n):
    if a is None:
        return None, None
    t = torch.as_tensor(a, dtype=torch.int64).contiguous().cpu()
    if t.numel() != n:
        raise ValueError(f"expected {n} costs, got {t.numel()}")
    return t, ctypes.c_void_p(t.data_ptr())


def mvc_bipartite(n_left: int, n_right: int, left, right, w_left=None, w_right=None):
    """Minimum weighted vertex cover of a bipartite graph (host):
    returns (cost, cover_left bool tensor, cover_right bool tensor)."""
    le = torch.as_tensor(left, dtype=torch.int32).contiguous().cpu()
    ri = torch.as_tensor(right, dtype=torch.int32).contiguous().cpu()
    if le.numel() != ri.numel():
        raise ValueError("left and right must have one entry per edge")
    wl, pwl = _host_i64(w_left, n_left)
    wr, pwr = _host_i64(w_right, n_right)
    cl = torch.zeros(max(n_left, 1), dtype=torch.uint8)
    cr = torch.zeros(max(n_right, 1), dtype=torch.uint8)
    w = ctypes.c_int64()
    _lib.check(_L().shiro_mvc_bipartite(int(n_left), int(n_right), le.numel(), ctypes.c_void_p(le.data_ptr()),
                                        ctypes.c_void_p(ri.data_ptr()), pwl, pwr, ctypes.c_void_p(cl.data_ptr()),
                                        ctypes.c_void_p(cr.data_ptr()), ctypes.byref(w)))
    return w.value, cl[:n_left].bool(), cr[:n_right].bool()


def joint_plan(plan: Plan, w_row=None, w_col=None, n_threads: int = 0, stream=None):
    """Per-block minimum covers of the panel (host).  Returns (assign uint8
    tensor over the panel's nonzeros: 1 = row-based, stats int64 (P, 5): cover
    cost, |Rows_q|, |Cols_q|, rows in the cover, columns in the cover)."""
    inf = plan.info()
    wr_, pwr = _host_i64(w_row, inf["rows"])
    wc_, pwc = _host_i64(w_col, inf["n_cols"])
    assign = torch.zeros(max(inf["nnz"], 1), dtype=torch.uint8)
    stats = torch.zeros(inf["P"], 5, dtype=torch.int64)
    _lib.check(_L().shiro_joint_plan(plan.handle, pwr, pwc, ctypes.c_void_p(assign.data_ptr()),
                                     ctypes.c_void_p(stats.data_ptr()), int(n_threads),
                                     ctypes.c_void_p(_stream(stream))))
    return assign[:inf["nnz"]], stats


_OPS = {"spmm": _lib.OP_SPMM, "backward": _lib.OP_BACKWARD, "per_block": _lib.OP_PER_BLOCK,
        "row_based": _lib.OP_ROW_BASED}


def _ops(ops) -> int:
    if isinstance(ops, int):
        return ops
    v = 0
    for o in ops:
        v |= _OPS[o]
    return v


def prepare(plan: Plan, N: int, dtype=torch.float32, ops=("spmm", "backward"), stream=None):
    _lib.check(_L().shiro_prepare(plan.handle, int(N), _dt(dtype), _ops(ops), ctypes.c_void_p(_stream(stream))))


def autotune(plan: Plan, N: int, dtype=torch.float32, ops=("spmm", "backward"), stream=None):
    _lib.check(_L().shiro_autotune(plan.handle, int(N), _dt(dtype), _ops(ops), ctypes.c_void_p(_stream(stream))))


def get_tuning(plan: Plan, kernel: str, N: int, dtype=torch.float32) -> dict:
    t = Tuning()
    _lib.check(_L().shiro_get_tuning(plan.handle, _KERNELS[kernel], int(N), _dt(dtype), ctypes.byref(t)))
    return t.as_dict()


def set_tuning(plan: Plan, kernel: str, N: int, dtype=torch.float32, **knobs):
    cur = get_tuning(plan, kernel, N, dtype)
    cur.update(knobs)
    t = Tuning(**cur)
    _lib.check(_L().shiro_set_tuning(plan.handle, _KERNELS[kernel], int(N), _dt(dtype), ctypes.byref(t)))


# ---------------------------------------------------------------------------
# autograd: Y = A B with gradients for the values and for B
# ---------------------------------------------------------------------------
class ShiroSpMM(torch.autograd.Function):
    """Y = A^(p,:) B through select/pack/spmm; backward through spmm_backward.

    Inputs: vals (float32, the CSR's value array), B (n_cols x N, float32 or
    bfloat16).  The plan must have run select_rows.  Gradients: dvals (float32,
    nonzero entries of the panel only) and dB (B's dtype, rows outside
    Cols(panel) are zero).
    """

    @staticmethod
    def forward(ctx, vals, B, plan, out_dtype=None):
        Bp = pack_B(plan, B)
        Y = spmm(plan, vals, Bp, out_dtype=out_dtype)
        ctx.plan = plan
        ctx.save_for_backward(vals, Bp)
        ctx.B_shape = B.shape
        ctx.B_dtype = B.dtype
        return Y

    @staticmethod
    def backward(ctx, dY):
        vals, Bp = ctx.saved_tensors
        plan = ctx.plan
        dY = dY.to(ctx.B_dtype).contiguous()
        dvals = dB = None
        if ctx.needs_input_grad[0]:
            dvals = torch.zeros_like(vals)
        if ctx.needs_input_grad[1]:
            dB = torch.zeros(ctx.B_shape, dtype=ctx.B_dtype, device=dY.device)
        # dB is zero-filled here, so its selected rows are simply written
        spmm_backward(plan, vals, dY, Bp, None, dB, dvals, dB_overwrite=True)
        return dvals, dB, None, None


def shiro_spmm(plan: Plan, vals: torch.Tensor, B: torch.Tensor, out_dtype=None) -> torch.Tensor:
    return ShiroSpMM.apply(vals, B, plan, out_dtype)
