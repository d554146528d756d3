"""Property-based pins of the FP64 oracle (hypothesis): random CSR panels with
empty rows, empty and dense column blocks, single-column blocks and sizes
that P does not divide, checked against routes that share nothing with the
oracle's loops: a brute-force column scan for Cols(A^(p,q)) (Table 1), dense
numpy products for the SpMM, its transpose and the sampled product, the
adjoint identity of L = <G, A B> for the gradients, a (row, block) scan and
dense block products for the row-based scheme, and exhaustive search for
the minimum weighted vertex cover of the joint strategy."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle


@st.composite
def panels(draw):
    n_rows = draw(st.integers(1, 40))
    n_cols = draw(st.integers(1, 40))
    P = draw(st.integers(1, min(8, max(n_rows, n_cols))))
    p = draw(st.integers(0, P - 1))
    density = draw(st.sampled_from([0.0, 0.05, 0.2, 0.6, 1.0]))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    mask = rng.random((n_rows, n_cols)) < density
    if draw(st.booleans()):  # some empty rows
        mask[rng.random(n_rows) < 0.3, :] = False
    K = -(-n_cols // P)
    if draw(st.booleans()):  # one empty column block
        q = int(rng.integers(0, P))
        mask[:, q * K:(q + 1) * K] = False
    if draw(st.booleans()):  # one dense block in the panel
        q = int(rng.integers(0, P))
        M = -(-n_rows // P)
        mask[p * M:(p + 1) * M, q * K:(q + 1) * K] = True
    rows, cols = np.nonzero(mask)
    vals = rng.uniform(-1, 1, size=len(rows)).astype(np.float32)
    row_ptr = np.zeros(n_rows + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n_rows), out=row_ptr[1:])
    A = oracle.Csr(n_rows, n_cols, row_ptr, cols.astype(np.int32), vals, P, p)
    N = draw(st.integers(1, 6))
    return A, N, rng


def panel_dense(A):
    D = np.zeros((A.M, A.n_cols))
    for i in range(A.row_begin, A.row_end):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i - A.row_begin, A.col[k]] = A.vals[k]
    return D


SETTINGS = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(panels())
def test_select_against_column_scan(case):
    A, N, rng = case
    uc, off, cm = oracle.select(A)
    present = np.zeros(A.n_cols, bool)
    present[A.col[A.nz_begin:A.nz_begin + A.nnz_panel]] = True
    expect = []
    counts = []
    for q in range(A.P):
        ids = [c for c in range(q * A.K, min(A.n_cols, (q + 1) * A.K)) if present[c]]
        expect += ids
        counts.append(len(ids))
    assert uc.tolist() == expect
    assert off.tolist() == np.concatenate([[0], np.cumsum(counts)]).tolist()
    # colmap round-trips to the column ids, ascending inside each row
    assert np.array_equal(uc[cm], A.col[A.nz_begin:A.nz_begin + A.nnz_panel])
    for i in range(A.row_begin, A.row_end):
        seg = cm[A.row_ptr[i] - A.nz_begin:A.row_ptr[i + 1] - A.nz_begin]
        assert np.all(np.diff(seg) > 0)
    # payload bytes of the column-based scheme (Sec. 3.1, V_col)
    assert int(oracle.v_col_bytes(off, N, 4).sum()) == len(uc) * N * 4


@SETTINGS
@given(panels())
def test_products_against_dense(case):
    A, N, rng = case
    uc, off, cm = oracle.select(A)
    B = rng.standard_normal((A.n_cols, N)).astype(np.float32)
    G = rng.standard_normal((A.M, N)).astype(np.float32)
    D = panel_dense(A)
    Bp = oracle.pack(B, uc)
    assert np.array_equal(Bp, B[uc])
    Y = oracle.spmm(A, Bp, cm)
    assert np.allclose(Y, D @ B.astype(np.float64), rtol=1e-12, atol=1e-12)
    assert np.array_equal(Y, oracle.spmm(A, B, None))  # packed and direct agree exactly
    dBp = oracle.spmm_t(A, G, cm, n_out=len(uc))
    dB = D.T @ G.astype(np.float64)
    assert np.allclose(dBp, dB[uc], rtol=1e-12, atol=1e-12)
    dv = oracle.sddmm(A, G, Bp, cm)
    full = G.astype(np.float64) @ B.astype(np.float64).T
    rr, cc = np.nonzero(D)
    # nonzeros of the panel in CSR order are exactly np.nonzero's row-major order
    assert np.allclose(dv, full[rr, cc], rtol=1e-12, atol=1e-12)
    # adjoint identity <G, A B> = <dB, B> = <vals, dvals>
    L = float(np.sum(G * Y))
    assert np.isclose(L, float(np.sum(dBp * Bp.astype(np.float64))), rtol=1e-10, atol=1e-10)
    vals = A.vals[A.nz_begin:A.nz_begin + A.nnz_panel].astype(np.float64)
    assert np.isclose(L, float(np.dot(vals, dv)), rtol=1e-10, atol=1e-10)


@SETTINGS
@given(panels())
def test_abs_denominators_against_dense(case):
    """The error denominators |A||B|, |A|^T|G| and sum_j |G||B| (whole,
    row-sampled and column-sampled forms) against dense products of
    absolute values."""
    A, N, rng = case
    uc, off, cm = oracle.select(A)
    U = len(uc)
    B = rng.standard_normal((A.n_cols, N)).astype(np.float32)
    G = rng.standard_normal((A.M, N)).astype(np.float32)
    D = np.abs(panel_dense(A))
    aB, aG = np.abs(B.astype(np.float64)), np.abs(G.astype(np.float64))
    Bp = oracle.pack(B, uc)
    den = D @ aB
    assert np.allclose(oracle.spmm(A, Bp, cm, abs_mode=True), den, rtol=1e-12, atol=1e-12)
    if A.M:
        rows = rng.integers(0, A.M, size=min(A.M, 5))
        assert np.allclose(oracle.spmm_rows(A, rows, Bp, cm, abs_mode=True), den[rows], rtol=1e-12, atol=1e-12)
    den_t = D.T @ aG
    assert np.allclose(oracle.spmm_t(A, G, cm, n_out=U, abs_mode=True), den_t[uc], rtol=1e-12, atol=1e-12)
    if U:
        t = rng.permutation(U)[: min(U, 5)]
        assert np.allclose(oracle.spmm_t_sampled(A, G, cm, U, t, abs_mode=True), den_t[uc[t]],
                           rtol=1e-12, atol=1e-12)
    rr, cc = np.nonzero(D)
    assert np.allclose(oracle.sddmm(A, G, Bp, cm, abs_mode=True), (aG @ aB.T)[rr, cc], rtol=1e-12, atol=1e-12)


@SETTINGS
@given(panels())
def test_row_based_against_scan_and_dense(case):
    """Rows(A^(p,q)) by a (row, block) scan; the owner's partial rows are each
    block's dense slice times B; their sum over blocks is the panel product."""
    A, N, rng = case
    rs, off = oracle.select_c_rows(A)
    expect, counts = [], []
    for q in range(A.P):
        lo, hi = q * A.K, min(A.n_cols, (q + 1) * A.K)
        rows_q = [i - A.row_begin for i in range(A.row_begin, A.row_end)
                  if any(lo <= c < hi for c in A.col[A.row_ptr[i]:A.row_ptr[i + 1]])]
        expect += rows_q
        counts.append(len(rows_q))
    assert rs.tolist() == expect
    assert off.tolist() == np.concatenate([[0], np.cumsum(counts)]).tolist()
    B = rng.standard_normal((A.n_cols, N)).astype(np.float32)
    Cp = oracle.partial_c(A, B, rs, off)
    D = panel_dense(A)
    for q in range(A.P):
        lo, hi = q * A.K, min(A.n_cols, (q + 1) * A.K)
        sl = D[:, lo:hi] @ B[lo:hi].astype(np.float64)
        assert np.allclose(Cp[off[q]:off[q + 1]], sl[rs[off[q]:off[q + 1]]], rtol=1e-12, atol=1e-12)
    Y = oracle.aggregate_c(A, Cp, rs, off)
    assert np.allclose(Y[:A.M], D @ B.astype(np.float64), rtol=1e-12, atol=1e-12)


@settings(max_examples=80, deadline=None)
@given(st.integers(1, 7), st.integers(1, 7), st.integers(0, 2**31 - 1), st.booleans())
def test_cover_against_brute_force(n_left, n_right, seed, weighted):
    """The max-flow cover of Sec. 5.3 is a vertex cover of minimum weight:
    every edge is covered, and no subset of the vertices covers the edges
    with less weight (exhaustive over all 2^(n_left + n_right) subsets)."""
    rng = np.random.default_rng(seed)
    m = rng.random((n_left, n_right)) < 0.4
    edges = np.argwhere(m)
    wl = rng.integers(1, 6, n_left) if weighted else np.ones(n_left, np.int64)
    wr = rng.integers(1, 6, n_right) if weighted else np.ones(n_right, np.int64)
    w, cl, cr = oracle.mvc_bipartite(n_left, n_right, edges, wl, wr)
    assert all(cl[a] or cr[b] for a, b in edges)
    assert w == int(wl[cl].sum() + wr[cr].sum())
    best = None
    V = n_left + n_right
    for mask in range(1 << V):
        sel = [(mask >> v) & 1 for v in range(V)]
        if all(sel[a] or sel[n_left + b] for a, b in edges):
            cost = sum(int(wl[v]) for v in range(n_left) if sel[v]) + sum(int(wr[v]) for v in range(n_right) if sel[n_left + v])
            best = cost if best is None else min(best, cost)
    assert w == (best if best is not None else 0)
