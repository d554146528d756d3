"""FP64 CPU oracle of the per-rank column-based SpMM path (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the GPU library.  The arithmetic lives in
``oracle.c`` (plain loops, double precision); this module only marshals
numpy arrays through ctypes.

Every function here is pinned by the ``-m "not gpu"`` tests against results
the paper or the mathematics fixes (worked example of Fig. 1, brute-force
column sets, dense products, closed-form byte counts, adjoint identities).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (host-only, OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            L.oracle_threads.restype = ctypes.c_int
            L.oracle_partition.argtypes = [_i64, _i64, _i32, _i32, _p, _p, _p]
            L.oracle_block_nnz.argtypes = [_p, _p, _i64, _i64, _i64, _i32, _p]
            L.oracle_select.argtypes = [_p, _p, _i64, _i64, _i64, _i32, _p, _p, _p]
            L.oracle_select.restype = _i64
            L.oracle_pack.argtypes = [_p, _i64, _i64, _i64, _p, _i64, _p, _i64]
            L.oracle_spmm.argtypes = [_p, _p, _p, _i64, _i64, _p, _p, _i64, _i64, _p, _i64, ctypes.c_int]
            L.oracle_spmm_rows.argtypes = [_p, _p, _p, _i64, _p, _i64, _p, _p, _i64, _i64, _p, _i64, ctypes.c_int]
            L.oracle_spmm_t.argtypes = [_p, _p, _p, _i64, _i64, _p, _p, _i64, _i64, _p, _i64, ctypes.c_int]
            L.oracle_spmm_t_sampled.argtypes = [_p, _p, _i64, _i64, _p, _p, _p, _i64, _i64, _p, _i64, ctypes.c_int]
            L.oracle_sddmm.argtypes = [_p, _p, _i64, _i64, _p, _p, _i64, _p, _i64, _i64, _p, ctypes.c_int]
            L.oracle_select_c_rows.argtypes = [_p, _p, _i64, _i64, _i64, _i32, _p, _p]
            L.oracle_select_c_rows.restype = _i64
            L.oracle_partial_c.argtypes = [_p, _p, _p, _i64, _i64, _i32, _p, _p, _p, _i64, _i64, _p, _i64,
                                           ctypes.c_int]
            L.oracle_aggregate_c.argtypes = [_i64, _i32, _p, _p, _p, _p, _i64, _i64, _p, _i64]
            _lib = L
    return _lib


def threads() -> int:
    return int(lib().oracle_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


class Csr:
    """Host CSR in numpy: global row_ptr (int64), col (int32), vals (float32)."""

    def __init__(self, n_rows, n_cols, row_ptr, col, vals, P=1, p=0):
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.row_ptr = _c(row_ptr, np.int64)
        self.col = _c(col, np.int32)
        self.vals = _c(vals, np.float32)
        self.P, self.p = int(P), int(p)
        self.row_begin, self.row_end, self.K = partition(self.n_rows, self.n_cols, self.P, self.p)

    @classmethod
    def from_synth(cls, A) -> "Csr":
        return cls(A.n_rows, A.n_cols, A.row_ptr.cpu().numpy(), A.col.cpu().numpy(), A.vals.cpu().numpy(), A.P, A.p)

    @property
    def M(self) -> int:
        return self.row_end - self.row_begin

    @property
    def nz_begin(self) -> int:
        return int(self.row_ptr[self.row_begin])

    @property
    def nnz_panel(self) -> int:
        return int(self.row_ptr[self.row_end] - self.row_ptr[self.row_begin])


def partition(n_rows: int, n_cols: int, P: int, p: int):
    """(row_begin, row_end, K) of panel p of P (Sec. 2.2; Table 1)."""
    b, e, k = _i64(), _i64(), _i64()
    lib().oracle_partition(n_rows, n_cols, P, p, ctypes.byref(b), ctypes.byref(e), ctypes.byref(k))
    return b.value, e.value, k.value


def block_nnz(A: Csr) -> np.ndarray:
    out = np.zeros(A.P, np.int64)
    lib().oracle_block_nnz(_ptr(A.row_ptr), _ptr(A.col), A.row_begin, A.row_end, A.K, A.P, _ptr(out))
    return out


def select(A: Csr):
    """(unique_cols int32[U], block_off int64[P+1], colmap int32[nnz_panel])."""
    nnz = A.nnz_panel
    uc = np.empty(max(nnz, 1), np.int32)
    off = np.empty(A.P + 1, np.int64)
    cm = np.empty(max(nnz, 1), np.int32)
    U = lib().oracle_select(_ptr(A.row_ptr), _ptr(A.col), A.row_begin, A.row_end, A.K, A.P, _ptr(uc), _ptr(off), _ptr(cm))
    return uc[:U].copy(), off, cm[:nnz].copy()


def pack(B: np.ndarray, unique_cols: np.ndarray) -> np.ndarray:
    """Bpacked[u] = B[unique_cols[u]] for 2-D B of 4- or 2-byte elements."""
    B = np.ascontiguousarray(B)
    assert B.ndim == 2 and B.dtype.itemsize in (2, 4)
    uc = _c(unique_cols, np.int32)
    out = np.empty((uc.size, B.shape[1]), B.dtype)
    lib().oracle_pack(_ptr(B), B.shape[1], B.shape[1], B.dtype.itemsize, _ptr(uc), uc.size, _ptr(out), B.shape[1])
    return out


def spmm(A: Csr, Bsrc: np.ndarray, colmap=None, abs_mode=False) -> np.ndarray:
    """Y (M x N, float64) = A^(p,:) Bsrc over packed rows (colmap) or B rows."""
    Bsrc = _c(Bsrc, np.float32)
    N = Bsrc.shape[1]
    Y = np.empty((A.M, N), np.float64)
    cm = None if colmap is None else _c(colmap, np.int32)
    lib().oracle_spmm(_ptr(A.row_ptr), _ptr(A.col), _ptr(A.vals), A.row_begin, A.row_end, _ptr(cm), _ptr(Bsrc), N, N, _ptr(Y), N, int(abs_mode))
    return Y


def spmm_rows(A: Csr, rows, Bsrc: np.ndarray, colmap=None, abs_mode=False) -> np.ndarray:
    """Rows ``rows`` (panel-local) of the product, float64."""
    Bsrc = _c(Bsrc, np.float32)
    rows = _c(rows, np.int64)
    N = Bsrc.shape[1]
    Y = np.empty((rows.size, N), np.float64)
    cm = None if colmap is None else _c(colmap, np.int32)
    lib().oracle_spmm_rows(_ptr(A.row_ptr), _ptr(A.col), _ptr(A.vals), A.row_begin, _ptr(rows), rows.size, _ptr(cm), _ptr(Bsrc), N, N, _ptr(Y), N, int(abs_mode))
    return Y


def spmm_t(A: Csr, G: np.ndarray, colmap=None, n_out=None, abs_mode=False) -> np.ndarray:
    """A^(p,:)^T G (float64) onto packed rows (colmap, n_out = U) or B rows."""
    G = _c(G, np.float32)
    N = G.shape[1]
    if n_out is None:
        n_out = A.n_cols if colmap is None else int(np.max(colmap)) + 1 if len(colmap) else 0
    dX = np.zeros((n_out, N), np.float64)
    cm = None if colmap is None else _c(colmap, np.int32)
    lib().oracle_spmm_t(_ptr(A.row_ptr), _ptr(A.col), _ptr(A.vals), A.row_begin, A.row_end, _ptr(cm), _ptr(G), N, N, _ptr(dX), N, int(abs_mode))
    return dX


def spmm_t_sampled(A: Csr, G: np.ndarray, colmap: np.ndarray, U: int, targets, abs_mode=False) -> np.ndarray:
    """Rows ``targets`` of A^T G over packed rows, float64."""
    G = _c(G, np.float32)
    N = G.shape[1]
    targets = _c(targets, np.int64)
    slot = np.full(U, -1, np.int64)
    slot[targets] = np.arange(targets.size)
    out = np.zeros((targets.size, N), np.float64)
    cm = _c(colmap, np.int32)
    lib().oracle_spmm_t_sampled(_ptr(A.row_ptr), _ptr(A.vals), A.row_begin, A.row_end, _ptr(cm), _ptr(slot), _ptr(G), N, N, _ptr(out), N, int(abs_mode))
    return out


def sddmm(A: Csr, G: np.ndarray, Bsrc: np.ndarray, colmap=None, abs_mode=False) -> np.ndarray:
    """dvals[k] = G[i(k)] . Bsrc[r(k)] for every panel nonzero, float64."""
    G = _c(G, np.float32)
    Bsrc = _c(Bsrc, np.float32)
    N = G.shape[1]
    out = np.empty(A.nnz_panel, np.float64)
    cm = None if colmap is None else _c(colmap, np.int32)
    lib().oracle_sddmm(_ptr(A.row_ptr), _ptr(A.col), A.row_begin, A.row_end, _ptr(cm), _ptr(G), N, _ptr(Bsrc), N, N, _ptr(out), int(abs_mode))
    return out


def v_col_bytes(block_off: np.ndarray, N: int, sz: int) -> np.ndarray:
    """Per-block column-based payload V_col = |Cols(A^(p,q))| * N * sz (Sec. 3.1)."""
    return np.diff(np.asarray(block_off, np.int64)) * N * sz


def rel_err(Y, Yref, den) -> float:
    """max |Y - Yref| / den, elementwise; entries with den == 0 must match exactly.

    den is |A||B| (or the analogous absolute product) computed by the oracle.
    Returns +inf if an entry with a zero denominator is not exactly equal.
    """
    Y = np.asarray(Y, np.float64)
    Yref = np.asarray(Yref, np.float64)
    den = np.asarray(den, np.float64)
    diff = np.abs(Y - Yref)
    zero = den == 0
    if np.any(diff[zero] != 0):
        return float("inf")
    if not np.any(~zero):
        return 0.0
    return float(np.max(diff[~zero] / den[~zero]))


def row_rel_err(Y, Yref, den) -> float:
    """max over rows of max_j |dY| / max_j den (looser per-row form)."""
    Y = np.asarray(Y, np.float64)
    num = np.max(np.abs(Y - np.asarray(Yref, np.float64)), axis=1) if Y.size else np.zeros(0)
    d = np.max(np.asarray(den, np.float64), axis=1) if Y.size else np.zeros(0)
    ok = d > 0
    if np.any(num[~ok] != 0):
        return float("inf")
    return float(np.max(num[ok] / d[ok])) if np.any(ok) else 0.0


# ----------------------------------------------------------------------------
# row-based scheme (Sec. 3.1; Sec. 5.1 stages 3 and 5)
# ----------------------------------------------------------------------------
def select_c_rows(A: Csr):
    """(row_sel int32[R], rblock_off int64[P+1]): Rows(A^(p,q)) for every block
    q, panel-local row ids, ascending within each block, blocks back to back."""
    nnz = A.nnz_panel
    row_sel = np.zeros(max(nnz, 1), np.int32)
    off = np.zeros(A.P + 1, np.int64)
    R = lib().oracle_select_c_rows(_ptr(A.row_ptr), _ptr(A.col), A.row_begin, A.row_end, A.K, A.P,
                                   _ptr(row_sel), _ptr(off))
    return row_sel[:R].copy(), off


def v_row_bytes(A: Csr, N: int, sz: int) -> np.ndarray:
    """Sec. 3.1 Eq. V_row per block: |Rows(A^(p,q))| * N * sz."""
    _, off = select_c_rows(A)
    return np.diff(off) * N * sz


def partial_c(A: Csr, B: np.ndarray, row_sel, rblock_off, abs_mode: bool = False) -> np.ndarray:
    """Owner-side partial rows of C (R x N, float64) over B's global rows."""
    B = _c(B, np.float32)
    N = B.shape[1]
    R = len(row_sel)
    out = np.zeros((max(R, 1), N), np.float64)
    rs = _c(row_sel if R else np.zeros(1, np.int32), np.int32)
    lib().oracle_partial_c(_ptr(A.row_ptr), _ptr(A.col), _ptr(A.vals), A.row_begin, A.K, A.P, _ptr(rs),
                           _ptr(_c(rblock_off, np.int64)), _ptr(B), N, N, _ptr(out), N, int(abs_mode))
    return out[:R]


def aggregate_c(A: Csr, Cp: np.ndarray, row_sel, rblock_off) -> np.ndarray:
    """Receiver-side sum of partial rows into the panel's rows (M x N, float64),
    blocks in ascending order.  Cp may be float64 or float32."""
    N = Cp.shape[1] if Cp.ndim == 2 else 0
    Y = np.zeros((max(A.M, 1), N), np.float64)
    R = len(row_sel)
    rs = _c(row_sel if R else np.zeros(1, np.int32), np.int32)
    if Cp.dtype == np.float64:
        cd, cf = _c(Cp if R else np.zeros((1, N)), np.float64), None
    else:
        cd, cf = None, _c(Cp if R else np.zeros((1, N)), np.float32)
    lib().oracle_aggregate_c(A.M, A.P, _ptr(rs), _ptr(_c(rblock_off, np.int64)), _ptr(cd), _ptr(cf), N, N,
                             _ptr(Y), N)
    return Y[:A.M]


# ----------------------------------------------------------------------------
# joint row-column strategy (Sec. 5.2 problem; Sec. 5.3 minimum weighted
# vertex cover of the bipartite graph, solved as a minimum s-t cut)
# ----------------------------------------------------------------------------
def mvc_bipartite(n_left: int, n_right: int, edges, w_left=None, w_right=None):
    """Minimum weighted vertex cover of a bipartite graph (left = rows of C,
    right = rows of B; edges = nonzeros) by the flow network of Sec. 5.3:
    s -> left i with capacity w_left[i], left -> right with capacity larger
    than any cut, right j -> t with capacity w_right[j]; the cover is the
    left vertices cut off from s plus the right vertices still reachable from
    s in the residual graph.  Max flow by scipy (a library step).
    Returns (weight, cover_left bool[n_left], cover_right bool[n_right])."""
    import scipy.sparse as sps
    from scipy.sparse.csgraph import maximum_flow

    edges = np.asarray(edges, np.int64).reshape(-1, 2)
    wl = np.ones(n_left, np.int64) if w_left is None else np.asarray(w_left, np.int64)
    wr = np.ones(n_right, np.int64) if w_right is None else np.asarray(w_right, np.int64)
    if len(edges) == 0:
        return 0, np.zeros(n_left, bool), np.zeros(n_right, bool)
    big = int(wl.sum() + wr.sum() + 1)
    s, t = n_left + n_right, n_left + n_right + 1
    V = n_left + n_right + 2
    src = np.concatenate([np.full(n_left, s), edges[:, 0], n_left + np.arange(n_right)])
    dst = np.concatenate([np.arange(n_left), n_left + edges[:, 1], np.full(n_right, t)])
    cap = np.concatenate([wl, np.full(len(edges), big), wr])
    G = sps.csr_array((cap.astype(np.int64), (src, dst)), shape=(V, V))
    G.sum_duplicates()
    res = maximum_flow(G, s, t)
    F = res.flow.tocsr()
    # residual graph: forward capacity left, and reverse capacity = flow
    Gc = G.tocoo()
    fwd = sps.csr_array((Gc.data - F[Gc.row, Gc.col], (Gc.row, Gc.col)), shape=(V, V))
    Fc = F.tocoo()
    pos = Fc.data > 0
    back = sps.csr_array((Fc.data[pos], (Fc.col[pos], Fc.row[pos])), shape=(V, V))
    Rg = (fwd + back).tocsr()
    seen = np.zeros(V, bool)
    seen[s] = True
    stack = [s]
    while stack:
        u = stack.pop()
        for k in range(Rg.indptr[u], Rg.indptr[u + 1]):
            v = Rg.indices[k]
            if Rg.data[k] > 0 and not seen[v]:
                seen[v] = True
                stack.append(v)
    cover_left = ~seen[:n_left]
    cover_right = seen[n_left:n_left + n_right]
    weight = int(wl[cover_left].sum() + wr[cover_right].sum())
    assert weight == int(res.flow_value)  # max-flow min-cut
    return weight, cover_left, cover_right


def joint_cover(A: Csr, w_row=None, w_col=None):
    """Per column block q: (mu_q, Rows_q, Cols_q, rows in the cover, cols in
    the cover) for the off-diagonal blocks (q != p); None for the diagonal
    block, whose B rows are local.  w_row: cost per panel row (panel-local
    index), w_col: cost per global column; None means unit costs."""
    out = []
    nz0 = A.nz_begin
    rows_of = np.repeat(np.arange(A.M), np.diff(A.row_ptr[A.row_begin:A.row_end + 1]))
    cols = A.col[nz0:nz0 + A.nnz_panel].astype(np.int64)
    for q in range(A.P):
        if q == A.p:
            out.append(None)
            continue
        m = (cols // A.K) == q
        r, c = rows_of[m], cols[m]
        ur, ri = np.unique(r, return_inverse=True)
        uc, ci = np.unique(c, return_inverse=True)
        wl = None if w_row is None else np.asarray(w_row)[ur]
        wr = None if w_col is None else np.asarray(w_col)[uc]
        mu, cl, cr = mvc_bipartite(len(ur), len(uc), np.stack([ri, ci], 1), wl, wr)
        out.append((mu, ur, uc, ur[cl], uc[cr]))
    return out
