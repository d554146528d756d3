"""Seeded synthetic inputs for the per-rank sparsity-aware SpMM path.

This module is shared by the oracle's tests, the GPU tests and the benchmark.
It generates sparsity patterns, values and dense operands and holds none of
the SpMM method's arithmetic (no column selection, packing or products).

Every random draw is counter based (splitmix64 over an int64 counter), so a
pattern or value array depends only on (seed, stream, index) and is identical
whether it is produced on the CPU or on a GPU.  Dense N(0,1) operands are the
one exception: they come from ``torch.randn`` with a seeded generator on the
device that will hold them; tests that need them on both sides generate them
once and copy.

Workload shapes follow the paper's evaluation (Table 2 matrices are power-law
graphs; dense widths N in {32, 64, 128}, Sec. 7.1 and 7.5): R-MAT graphs with
a/b/c/d = 0.57/0.19/0.19/0.05 stand in for the social/web matrices and an
Erdos-Renyi G(n, m) panel for the uniform pattern the joint-strategy analysis
contrasts (Sec. 5.4, Fig. 5 pattern 3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

# ----------------------------------------------------------------------------
# splitmix64 in int64 tensor arithmetic (wrapping multiply, logical shifts)
# ----------------------------------------------------------------------------
_M64 = 1 << 64


def _s64(c: int) -> int:
    c %= _M64
    return c - _M64 if c >= (1 << 63) else c


GAMMA = _s64(0x9E3779B97F4A7C15)
_C1 = _s64(0xBF58476D1CE4E5B9)
_C2 = _s64(0x94D049BB133111EB)

STREAM_PATTERN = 0
STREAM_VALS = 1
STREAM_B = 2
STREAM_DY = 3


def _srl(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """splitmix64 output function (Steele, Lea, Flood 2014) on int64 tensors."""
    z = (z ^ _srl(z, 30)) * _C1
    z = (z ^ _srl(z, 27)) * _C2
    return z ^ _srl(z, 31)


def mix64_py(z: int) -> int:
    """Pure-Python splitmix64 output function (unsigned), used to pin mix64."""
    z %= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % _M64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """64-bit key of one random stream (as a signed int64 value)."""
    return _s64(mix64_py(seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019 * (stream + 1)))


def draw_u64(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Counter-based 64-bit draws: mix64(key + (idx + 1) * GAMMA), int64 tensor."""
    return mix64((idx + 1) * GAMMA + key)


def draw_uniform_f64(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform [0, 1) doubles with 53 random bits (exact on any device)."""
    return _srl(draw_u64(key, idx), 11).to(torch.float64) * (2.0 ** -53)


def draw_uniform_f32(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform [0, 1) floats with 24 random bits (exact on any device)."""
    return _srl(draw_u64(key, idx), 40).to(torch.float32) * (2.0 ** -24)


# ----------------------------------------------------------------------------
# Sparse inputs
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class SparseInput:
    """A CSR matrix (global ids) plus the 1D row-partition the rank works on."""

    name: str
    n_rows: int
    n_cols: int
    row_ptr: torch.Tensor  # int64 [n_rows + 1]
    col: torch.Tensor  # int32 [nnz], ascending within each row, no duplicates
    vals: torch.Tensor  # float32 [nnz]
    P: int = 1
    p: int = 0

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def device(self) -> torch.device:
        return self.col.device

    def to(self, device) -> "SparseInput":
        return dataclasses.replace(
            self,
            row_ptr=self.row_ptr.to(device),
            col=self.col.to(device),
            vals=self.vals.to(device),
        )


def coo_to_csr(rows: torch.Tensor, cols: torch.Tensor, n_rows: int, n_cols: int):
    """Merge duplicate (row, col) pairs and return (row_ptr int64, col int32).

    Columns come out ascending inside every row (canonical CSR).
    """
    key = rows.to(torch.int64) * n_cols + cols.to(torch.int64)
    key = torch.unique(key, sorted=True)
    r = torch.div(key, n_cols, rounding_mode="floor")
    c = key - r * n_cols
    counts = torch.bincount(r, minlength=n_rows)
    row_ptr = torch.zeros(n_rows + 1, dtype=torch.int64, device=key.device)
    torch.cumsum(counts, 0, out=row_ptr[1:])
    return row_ptr, c.to(torch.int32)


def rmat_coo(
    row_bits: int,
    col_bits: int,
    nsamples: int,
    abcd=(0.57, 0.19, 0.19, 0.05),
    seed: int = 0,
    fixed_zero_row_bits: int = 0,
    device="cpu",
    chunk: int = 1 << 24,
):
    """R-MAT edge samples (Chakrabarti, Zhan, Faloutsos 2004).

    Each sample walks max(row_bits, col_bits) levels, most significant bit
    first; at every level it picks quadrant a=(0,0), b=(0,1), c=(1,0) or
    d=(1,1).  No noise and no vertex permutation, so hubs sit at low ids.
    The top ``fixed_zero_row_bits`` row bits are forced to 0 by drawing those
    levels from the a/b half only (probabilities a/(a+b), b/(a+b)): this
    samples exactly the rows of panel 0 of a 2^fixed-way row partition.
    Levels beyond a short side's bit count leave that side unchanged.
    """
    a, b, c, _d = abcd
    levels = max(row_bits, col_bits)
    key = stream_key(seed, STREAM_PATTERN)
    rows_out = []
    cols_out = []
    t_ab = a + b
    t_abc = a + b + c
    t_cond = a / (a + b)
    for s0 in range(0, nsamples, chunk):
        s = torch.arange(s0, min(nsamples, s0 + chunk), dtype=torch.int64, device=device)
        r = torch.zeros_like(s)
        cc = torch.zeros_like(s)
        base = s * levels
        for lvl in range(levels):
            u = draw_uniform_f64(key, base + lvl)
            if lvl < fixed_zero_row_bits:
                rbit = torch.zeros_like(s)
                cbit = (u >= t_cond).to(torch.int64)
            else:
                rbit = (u >= t_ab).to(torch.int64)
                cbit = ((u >= a) & (u < t_ab)).to(torch.int64) | (u >= t_abc).to(torch.int64)
            if lvl < row_bits:
                r = (r << 1) | rbit
            if lvl < col_bits:
                cc = (cc << 1) | cbit
        rows_out.append(r)
        cols_out.append(cc)
    return torch.cat(rows_out), torch.cat(cols_out)


def uniform_vals(nnz: int, seed: int, lo: float = 0.0, device="cpu") -> torch.Tensor:
    """Per-nonzero float32 values in CSR order: U(0,1), or U(-1,1) if lo == -1."""
    key = stream_key(seed, STREAM_VALS)
    u = draw_uniform_f32(key, torch.arange(nnz, dtype=torch.int64, device=device))
    if lo == -1.0:
        return u * 2.0 - 1.0  # exact: 24-bit grid maps onto a 23-bit grid
    assert lo == 0.0
    return u


def rmat_matrix(
    name: str,
    scale: int,
    nsamples: int,
    seed: int = 0,
    vals_lo: float = 0.0,
    P: int = 1,
    p: int = 0,
    panel0_only: bool = False,
    device="cpu",
) -> SparseInput:
    """Square 2^scale R-MAT CSR with merged duplicates and uniform values."""
    n = 1 << scale
    fixed = int(round(math.log2(P))) if panel0_only else 0
    if panel0_only:
        assert P == 1 << fixed and p == 0
    r, c = rmat_coo(scale, scale, nsamples, seed=seed, fixed_zero_row_bits=fixed, device=device)
    row_ptr, col = coo_to_csr(r, c, n, n)
    del r, c
    vals = uniform_vals(col.numel(), seed, vals_lo, device=device)
    return SparseInput(name, n, n, row_ptr, col, vals, P, p)


def er_panel(
    name: str,
    scale: int,
    P: int,
    avg_degree: int,
    seed: int = 0,
    device="cpu",
) -> SparseInput:
    """Panel 0 of an n x n Erdos-Renyi G(n, m) matrix, n = 2^scale.

    m = avg_degree * M samples with uniform rows in [0, M) and uniform columns
    in [0, n), duplicates merged (expected loss ~ m^2 / (2 M n), negligible).
    """
    n = 1 << scale
    M = n // P
    m = avg_degree * M
    key = stream_key(seed, STREAM_PATTERN)
    idx = torch.arange(m, dtype=torch.int64, device=device)
    rows = torch.floor(draw_uniform_f64(key, 2 * idx) * M).to(torch.int64)
    cols = torch.floor(draw_uniform_f64(key, 2 * idx + 1) * n).to(torch.int64)
    row_ptr, col = coo_to_csr(rows, cols, n, n)
    vals = uniform_vals(col.numel(), seed, 0.0, device=device)
    return SparseInput(name, n, n, row_ptr, col, vals, P, 0)


def gcn_normalised_rmat(name: str, scale: int, edge_factor: int, seed: int = 0, device="cpu") -> SparseInput:
    """Symmetrised R-MAT pattern with values 1/sqrt(d_i d_j) (no self-loop added).

    d_i is the number of nonzeros of row i of the symmetrised pattern.  The
    value is formed in float64 and rounded to float32 (round to nearest even).
    """
    n = 1 << scale
    r, c = rmat_coo(scale, scale, edge_factor * n, seed=seed, device=device)
    rr = torch.cat([r, c])
    cc = torch.cat([c, r])
    del r, c
    row_ptr, col = coo_to_csr(rr, cc, n, n)
    del rr, cc
    deg = (row_ptr[1:] - row_ptr[:-1]).to(torch.float64)
    rows = torch.repeat_interleave(torch.arange(n, device=device), row_ptr[1:] - row_ptr[:-1])
    vals = (1.0 / torch.sqrt(deg[rows] * deg[col.to(torch.int64)])).to(torch.float32)
    return SparseInput(name, n, n, row_ptr, col, vals, 1, 0)


def induced_subgraph(A: SparseInput, nv: int) -> SparseInput:
    """Rows and columns 0..nv-1 of A, values inherited (not renormalised)."""
    row_ptr = A.row_ptr[: nv + 1]
    col = A.col[: int(row_ptr[-1])]
    vals = A.vals[: int(row_ptr[-1])]
    rows = torch.repeat_interleave(torch.arange(nv, device=col.device), row_ptr[1:] - row_ptr[:-1])
    keep = col < nv
    rows, col, vals = rows[keep], col[keep], vals[keep]
    counts = torch.bincount(rows, minlength=nv)
    rp = torch.zeros(nv + 1, dtype=torch.int64, device=col.device)
    torch.cumsum(counts, 0, out=rp[1:])
    return SparseInput(A.name + f"_induced{nv}", nv, nv, rp, col.contiguous(), vals.contiguous(), 1, 0)


def dense(n: int, N: int, seed: int, stream: int, device="cpu", dtype=torch.float32) -> torch.Tensor:
    """Row-major n x N N(0,1) matrix from a seeded torch generator on ``device``."""
    g = torch.Generator(device=device)
    g.manual_seed(stream_key(seed, stream) & 0x7FFFFFFFFFFFFFFF)
    return torch.randn(n, N, generator=g, device=device, dtype=torch.float32).to(dtype)


# ----------------------------------------------------------------------------
# The five workloads (seed 0).  Readings of unspecified details:
#  * avg degree d -> d * n edge samples before duplicates are merged;
#  * the 2^24 graph's panel 0 is sampled directly (top 7 row bits fixed to 0)
#    with M * 32 samples, giving ~4.2M nonzeros in the panel;
#  * the GCN graph takes edge factor 25 (avg degree 50 counted over both
#    directions) and is symmetrised.
# ----------------------------------------------------------------------------
def config1(device="cpu") -> SparseInput:
    """4096^2 R-MAT, 16 samples per row, U(0,1) values, one block (P = 1)."""
    return rmat_matrix("rmat12_ef16", 12, 16 * 4096, device=device)


def config2(device="cpu") -> SparseInput:
    """Panel 0 of a 2^24 R-MAT at P = 128 (131072 rows, ~4.2M nonzeros)."""
    M = (1 << 24) // 128
    return rmat_matrix("rmat24_p128_panel0", 24, 32 * M, P=128, p=0, panel0_only=True, device=device)


def config3_er(device="cpu") -> SparseInput:
    """Panel 0 of a 2^24 Erdos-Renyi matrix at P = 128, average degree 32."""
    return er_panel("er24_p128_panel0", 24, 128, 32, device=device)


def config4(device="cpu") -> SparseInput:
    """2^22 R-MAT, 64 samples per row, U(-1,1) values, one block (P = 1)."""
    return rmat_matrix("rmat22_ef64", 22, 64 << 22, vals_lo=-1.0, device=device)


def config5(device="cpu") -> SparseInput:
    """GCN layer matrix: symmetrised, normalised 2^21 R-MAT (edge factor 25)."""
    return gcn_normalised_rmat("gcn_rmat21_ef25", 21, 25, device=device)


def small_rmat(scale: int, edge_factor: int, P: int = 1, p: int = 0, seed: int = 0, vals_lo=0.0, device="cpu") -> SparseInput:
    """Small R-MAT test case of the same family (any P; ragged panels allowed)."""
    n = 1 << scale
    return rmat_matrix(f"rmat{scale}_ef{edge_factor}_P{P}_p{p}", scale, edge_factor * n, seed=seed, vals_lo=vals_lo, P=P, p=p, device=device)


def from_dense_pattern(mask, vals=None, P: int = 1, p: int = 0, name="dense_pattern") -> SparseInput:
    """CSR of a small dense 0/1 (or value) matrix given as nested lists or a tensor."""
    m = torch.as_tensor(mask, dtype=torch.float64)
    n_rows, n_cols = m.shape
    nz = m != 0
    rows, cols = torch.nonzero(nz, as_tuple=True)
    counts = torch.bincount(rows, minlength=n_rows)
    row_ptr = torch.zeros(n_rows + 1, dtype=torch.int64)
    torch.cumsum(counts, 0, out=row_ptr[1:])
    v = m[nz].to(torch.float32) if vals is None else torch.as_tensor(vals, dtype=torch.float32)
    return SparseInput(name, n_rows, n_cols, row_ptr, cols.to(torch.int32), v, P, p)
