"""Pins of the FP64 oracle against results fixed by the paper or by mathematics.

Each check uses an independent route to the answer: a brute-force scan of
columns instead of sort-and-dedup, dense numpy/scipy products instead of the
CSR loops, the worked example of Fig. 1, closed-form byte counts (Sec. 3.1
Eq. V_col), identity/permutation/linearity invariants and the adjoint
identity of the bilinear form L = <G, A B>.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from conftest import load_golden


# ----------------------------------------------------------------------------
# helpers (test-local; no oracle arithmetic)
# ----------------------------------------------------------------------------
def random_csr(rng, n_rows, n_cols, density, P=1, p=0, empty_rows=0.0, empty_block=None, dense_block=None):
    mask = rng.random((n_rows, n_cols)) < density
    if empty_rows:
        mask[rng.random(n_rows) < empty_rows, :] = False
    K = -(-n_cols // P)
    if empty_block is not None:
        mask[:, empty_block * K:(empty_block + 1) * K] = False
    if dense_block is not None:
        M = -(-n_rows // P)
        mask[p * M:(p + 1) * M, dense_block * K:(dense_block + 1) * K] = True
    vals = rng.uniform(-1, 1, size=mask.sum()).astype(np.float32)
    vals[vals == 0] = 0.5
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n_rows + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n_rows), out=row_ptr[1:])
    return oracle.Csr(n_rows, n_cols, row_ptr, cols.astype(np.int32), vals, P, p)


def dense_of(A: oracle.Csr) -> np.ndarray:
    D = np.zeros((A.n_rows, A.n_cols), np.float64)
    for i in range(A.n_rows):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col[k]] = A.vals[k]
    return D


def brute_cols(A: oracle.Csr):
    """Cols(A^(p,q)) by scanning every column id of every block (no sorting)."""
    panel = set()
    for i in range(A.row_begin, A.row_end):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            panel.add(int(A.col[k]))
    out = []
    for q in range(A.P):
        lo, hi = q * A.K, min(A.n_cols, (q + 1) * A.K)
        out.append([c for c in range(lo, hi) if c in panel])
    return out


CASES = [
    # (n_rows, n_cols, density, P, p, kwargs)
    (37, 41, 0.15, 1, 0, {}),
    (64, 64, 0.05, 4, 1, {"empty_rows": 0.3}),
    (50, 53, 0.10, 7, 6, {}),  # ragged last panel and last block
    (40, 40, 0.20, 5, 2, {"empty_block": 3, "dense_block": 1}),
    (16, 96, 0.30, 3, 0, {}),  # rectangular
    (9, 9, 0.0, 2, 1, {}),  # empty panel
    (12, 1, 0.5, 1, 0, {}),  # single column
    (30, 30, 0.08, 30, 29, {}),  # one row per panel, one column per block
]


@pytest.fixture(params=range(len(CASES)))
def case(request):
    n_rows, n_cols, dens, P, p, kw = CASES[request.param]
    rng = np.random.default_rng(1000 + request.param)
    return random_csr(rng, n_rows, n_cols, dens, P, p, **kw)


# ----------------------------------------------------------------------------
# partition (Sec. 2.2; Table 1)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n,P", [(8, 2), (10, 3), (4096, 1), (1 << 24, 128), (5, 8), (7, 7)])
def test_partition_closed_form(n, P):
    covered = []
    for p in range(P):
        b, e, K = oracle.partition(n, n, P, p)
        M = -(-n // P)
        assert K == M
        assert b == min(n, p * M) and e == min(n, (p + 1) * M)
        covered.extend(range(b, e)) if n < 10000 else None
    if n < 10000:
        assert covered == list(range(n))


def test_block_nnz_counts(case):
    bn = oracle.block_nnz(case)
    ref = np.zeros(case.P, np.int64)
    for i in range(case.row_begin, case.row_end):
        for k in range(case.row_ptr[i], case.row_ptr[i + 1]):
            ref[int(case.col[k]) // case.K] += 1
    assert np.array_equal(bn, ref)
    assert bn.sum() == case.nnz_panel


# ----------------------------------------------------------------------------
# select (Table 1 Cols; Sec. 3.1 column-based scheme)
# ----------------------------------------------------------------------------
def test_select_matches_brute_force(case):
    uc, off, cm = oracle.select(case)
    ref = brute_cols(case)
    assert list(np.diff(off)) == [len(c) for c in ref]
    for q in range(case.P):
        assert list(uc[off[q]:off[q + 1]]) == ref[q]
    nz0 = case.nz_begin
    for k in range(nz0, nz0 + case.nnz_panel):
        q = int(case.col[k]) // case.K
        assert cm[k - nz0] == off[q] + ref[q].index(int(case.col[k]))


def test_select_fig1_worked_example():
    g = load_golden("fig1_block01.txt")
    n, P, p = g["n"][0][0], g["P"][0][0], g["p"][0][0]
    mask = np.zeros((n, n))
    for r, c, v in g["nz"]:
        mask[r, c] = v
    A = synth.from_dense_pattern(mask, P=P, p=p)
    Ac = oracle.Csr.from_synth(A)
    uc, off, cm = oracle.select(Ac)
    (q, *cols), = g["expect_cols_block"]
    assert list(uc[off[q]:off[q + 1]]) == cols
    (q2, vol), = g["expect_volume_rows"]
    assert off[q2 + 1] - off[q2] == vol
    # the V_col formula of Sec. 3.1 for N = 32 float32 columns
    assert oracle.v_col_bytes(off, 32, 4)[q2] == vol * 32 * 4
    # Rows(A^(0,1)) of the fixture (the row-based volume), by its definition
    (qr, *rows), = g["expect_rows_block"]
    blk_rows = sorted({int(r) for r, c, _ in g["nz"] if c // Ac.K == qr})
    assert blk_rows == rows


def test_select_invariants_rmat():
    A = oracle.Csr.from_synth(synth.small_rmat(11, 8, P=8, p=3))
    uc, off, cm = oracle.select(A)
    col = A.col[A.nz_begin:A.nz_begin + A.nnz_panel]
    assert np.array_equal(uc[cm], col)  # round trip
    for q in range(A.P):
        s = uc[off[q]:off[q + 1]]
        assert np.all(np.diff(s) > 0)
        assert np.all((s >= q * A.K) & (s < (q + 1) * A.K))
    assert off[-1] == np.unique(col).size  # blocks are disjoint, together Cols(panel)
    rp = A.row_ptr[A.row_begin:A.row_end + 1] - A.nz_begin
    for i in range(A.M):
        assert np.all(np.diff(cm[rp[i]:rp[i + 1]]) > 0)  # monotone inside rows
    assert np.array_equal(np.unique(cm), np.arange(off[-1]))  # every packed row used


def test_select_identity():
    n = 33
    A = synth.from_dense_pattern(np.eye(n), P=3, p=0)
    Ac = oracle.Csr.from_synth(A)
    uc, off, cm = oracle.select(Ac)
    assert list(uc) == list(range(Ac.row_begin, Ac.row_end))


# ----------------------------------------------------------------------------
# pack (Sec. 3.1 Eq. V_col; Sec. 5.1 stage 3)
# ----------------------------------------------------------------------------
def test_pack_rows_and_bytes(case):
    rng = np.random.default_rng(7)
    N = 5
    B = rng.standard_normal((case.n_cols, N)).astype(np.float32)
    uc, off, _ = oracle.select(case)
    Bp = oracle.pack(B, uc)
    assert Bp.shape == (off[-1], N)
    for u in range(off[-1]):
        assert Bp[u].tobytes() == B[uc[u]].tobytes()
    assert Bp.nbytes == oracle.v_col_bytes(off, N, 4).sum()
    # bfloat16 payload handled as raw 2-byte elements
    Bh = rng.integers(0, 1 << 16, size=(case.n_cols, 3), dtype=np.uint16)
    assert np.array_equal(oracle.pack(Bh, uc), Bh[uc])


def test_pack_identity_is_copy():
    A = oracle.Csr.from_synth(synth.from_dense_pattern(np.eye(20), P=1, p=0))
    B = np.arange(20 * 4, dtype=np.float32).reshape(20, 4)
    uc, _, _ = oracle.select(A)
    assert oracle.pack(B, uc).tobytes() == B.tobytes()


# ----------------------------------------------------------------------------
# spmm (Sec. 2.1 C = A B; Sec. 2.2 stages 3-4 aggregation)
# ----------------------------------------------------------------------------
def test_spmm_matches_dense_and_scipy(case):
    rng = np.random.default_rng(11)
    N = 6
    B = rng.standard_normal((case.n_cols, N)).astype(np.float32)
    uc, off, cm = oracle.select(case)
    Y = oracle.spmm(case, oracle.pack(B, uc), cm)
    D = dense_of(case)[case.row_begin:case.row_end]
    ref = D @ B.astype(np.float64)
    assert np.allclose(Y, ref, rtol=1e-12, atol=1e-12)
    S = sp.csr_matrix((case.vals.astype(np.float64), case.col, case.row_ptr), shape=(case.n_rows, case.n_cols))
    ref2 = (S @ B.astype(np.float64))[case.row_begin:case.row_end]
    assert np.allclose(Y, ref2, rtol=1e-12, atol=1e-12)
    # packed and unpacked forms are the same sums in the same order: identical
    assert np.array_equal(Y, oracle.spmm(case, B, None))


def test_spmm_identity_exact():
    n, N = 40, 7
    A = oracle.Csr.from_synth(synth.from_dense_pattern(np.eye(n), P=1, p=0))
    B = np.random.default_rng(3).standard_normal((n, N)).astype(np.float32)
    assert np.array_equal(oracle.spmm(A, B, None), B.astype(np.float64))


def test_spmm_empty_rows_zero_and_rows_subset():
    A = oracle.Csr.from_synth(synth.small_rmat(10, 4, P=4, p=1))
    B = np.random.default_rng(5).standard_normal((A.n_cols, 8)).astype(np.float32)
    uc, off, cm = oracle.select(A)
    Bp = oracle.pack(B, uc)
    Y = oracle.spmm(A, Bp, cm)
    rp = A.row_ptr[A.row_begin:A.row_end + 1]
    empty = np.nonzero(np.diff(rp) == 0)[0]
    assert empty.size > 0 and np.all(Y[empty] == 0.0)
    rows = np.array([0, 5, A.M - 1, int(np.argmax(np.diff(rp)))])
    assert np.array_equal(oracle.spmm_rows(A, rows, Bp, cm), Y[rows])
    assert np.array_equal(oracle.spmm_rows(A, rows, B, None), Y[rows])


def test_spmm_permutation_invariance():
    rng = np.random.default_rng(21)
    A = random_csr(rng, 30, 30, 0.2)
    D = dense_of(A)
    B = rng.standard_normal((30, 4)).astype(np.float32)
    pr = rng.permutation(30)
    pc = rng.permutation(30)
    Dp = D[pr][:, pc]  # P_r A P_c^T
    rows, cols = np.nonzero(Dp)
    rp = np.zeros(31, np.int64)
    np.cumsum(np.bincount(rows, minlength=30), out=rp[1:])
    Ap = oracle.Csr(30, 30, rp, cols.astype(np.int32), Dp[rows, cols].astype(np.float32))
    Y = oracle.spmm(A, B, None)
    Yp = oracle.spmm(Ap, B[pc], None)  # (P_r A P_c^T)(P_c B) = P_r A B
    assert np.allclose(Yp, Y[pr], rtol=1e-13, atol=1e-13)


def test_spmm_linearity():
    rng = np.random.default_rng(8)
    A = random_csr(rng, 25, 31, 0.2, P=2, p=1)
    B1 = rng.standard_normal((31, 3)).astype(np.float32)
    B2 = rng.standard_normal((31, 3)).astype(np.float32)
    Y1, Y2 = oracle.spmm(A, B1), oracle.spmm(A, B2)
    Y12 = oracle.spmm(A, (B1.astype(np.float64) + B2).astype(np.float32))
    # B1 + B2 rounds in float32; compare against the rounded sum's exact product
    assert np.allclose(Y12, Y1 + Y2, rtol=1e-6, atol=1e-6)
    A2 = oracle.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, A.vals * 2, A.P, A.p)  # exact scaling
    assert np.array_equal(oracle.spmm(A2, B1), 2 * Y1)


def test_spmm_abs_denominator():
    rng = np.random.default_rng(9)
    A = random_csr(rng, 20, 20, 0.3)
    B = rng.standard_normal((20, 5)).astype(np.float32)
    den = oracle.spmm(A, B, None, abs_mode=True)
    assert np.allclose(den, np.abs(dense_of(A)) @ np.abs(B.astype(np.float64)), rtol=1e-13)


# The absolute-value forms are the denominators of every floating-point parity
# check (componentwise |Y - Y*| / (|A||B|)): each is pinned against a dense
# product of absolute values, on signed values and signed dense rows so that
# dropping either absolute value, transposing the operands or reading the
# wrong row changes the result.
def test_abs_denominators_against_dense(case):
    rng = np.random.default_rng(61)
    N = 5
    B = rng.standard_normal((case.n_cols, N)).astype(np.float32)
    G = rng.standard_normal((case.M, N)).astype(np.float32)
    uc, off, cm = oracle.select(case)
    U = int(off[-1])
    Bp = oracle.pack(B, uc)
    D = np.abs(dense_of(case)[case.row_begin:case.row_end])
    aB, aG = np.abs(B.astype(np.float64)), np.abs(G.astype(np.float64))
    # |A|^T |G| onto B rows and onto packed rows
    den_t = D.T @ aG
    assert np.allclose(oracle.spmm_t(case, G, None, abs_mode=True), den_t, rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle.spmm_t(case, G, cm, n_out=U, abs_mode=True), den_t[uc], rtol=1e-12, atol=1e-12)
    # the sampled form: rows of the packed result, in any order
    if U:
        t = rng.permutation(U)[: max(1, U // 2)]
        assert np.allclose(oracle.spmm_t_sampled(case, G, cm, U, t, abs_mode=True), den_t[uc[t]],
                           rtol=1e-12, atol=1e-12)
    # sum_j |G[i(k), j]| |B[c(k), j]| at every nonzero, packed and direct
    full = aG @ aB.T
    rr, cc = np.nonzero(D)
    assert np.allclose(oracle.sddmm(case, G, Bp, cm, abs_mode=True), full[rr, cc], rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle.sddmm(case, G, B, None, abs_mode=True), full[rr, cc], rtol=1e-12, atol=1e-12)
    # rows of |A| |B|, in any order, packed and direct
    den = D @ aB
    rows = rng.permutation(case.M)[: max(1, case.M // 2)] if case.M else np.zeros(0, np.int64)
    assert np.allclose(oracle.spmm_rows(case, rows, Bp, cm, abs_mode=True), den[rows], rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle.spmm_rows(case, rows, B, None, abs_mode=True), den[rows], rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle.spmm(case, Bp, cm, abs_mode=True), den, rtol=1e-12, atol=1e-12)


def test_abs_denominators_bound_the_signed_forms():
    """|sum a_k b_k| <= sum |a_k| |b_k| for every output, with equality when
    every term is non-negative: each denominator is at least the magnitude of
    its signed result, and equals it on non-negative data."""
    A = oracle.Csr.from_synth(synth.small_rmat(9, 6, P=2, p=1, vals_lo=-1.0))
    rng = np.random.default_rng(62)
    N = 6
    B = rng.standard_normal((A.n_cols, N)).astype(np.float32)
    G = rng.standard_normal((A.M, N)).astype(np.float32)
    uc, off, cm = oracle.select(A)
    U = int(off[-1])
    Bp = oracle.pack(B, uc)
    pairs = [
        (oracle.spmm(A, Bp, cm), oracle.spmm(A, Bp, cm, abs_mode=True)),
        (oracle.spmm_t(A, G, cm, n_out=U), oracle.spmm_t(A, G, cm, n_out=U, abs_mode=True)),
        (oracle.sddmm(A, G, Bp, cm), oracle.sddmm(A, G, Bp, cm, abs_mode=True)),
    ]
    for signed, den in pairs:
        assert np.all(np.abs(signed) <= den * (1 + 1e-12) + 1e-300)
        assert np.any(den > np.abs(signed) * (1 + 1e-6))  # signed data cancels somewhere
    # non-negative data: the absolute forms are the signed forms
    Ap = oracle.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(A.vals), A.P, A.p)
    aBp, aG = np.abs(Bp), np.abs(G)
    assert np.array_equal(oracle.spmm(Ap, aBp, cm), oracle.spmm(A, Bp, cm, abs_mode=True))
    assert np.array_equal(oracle.spmm_t(Ap, aG, cm, n_out=U), oracle.spmm_t(A, G, cm, n_out=U, abs_mode=True))
    assert np.array_equal(oracle.sddmm(Ap, aG, aBp, cm), oracle.sddmm(A, G, Bp, cm, abs_mode=True))
    t = np.arange(0, U, 7)
    assert np.array_equal(oracle.spmm_t_sampled(Ap, aG, cm, U, t), oracle.spmm_t_sampled(A, G, cm, U, t, abs_mode=True))
    rows = np.arange(0, A.M, 5)
    assert np.array_equal(oracle.spmm_rows(Ap, rows, aBp, cm), oracle.spmm_rows(A, rows, Bp, cm, abs_mode=True))


# ----------------------------------------------------------------------------
# backward: dB = A^T G, dvals = (G B^T) sampled at the nonzeros
# ----------------------------------------------------------------------------
def test_backward_dense_and_adjoint(case):
    rng = np.random.default_rng(31)
    N = 4
    B = rng.standard_normal((case.n_cols, N)).astype(np.float32)
    G = rng.standard_normal((case.M, N)).astype(np.float32)
    uc, off, cm = oracle.select(case)
    Bp = oracle.pack(B, uc)
    dBp = oracle.spmm_t(case, G, cm, n_out=int(off[-1]))
    dB = oracle.spmm_t(case, G, None)
    D = dense_of(case)[case.row_begin:case.row_end]
    assert np.allclose(dB, D.T @ G.astype(np.float64), rtol=1e-12, atol=1e-12)
    assert np.array_equal(dB[uc], dBp)  # packed rows = the selected rows of dB
    mask = np.ones(case.n_cols, bool)
    mask[uc] = False
    assert np.all(dB[mask] == 0)  # unselected rows get no gradient
    dv = oracle.sddmm(case, G, Bp, cm)
    assert np.array_equal(dv, oracle.sddmm(case, G, B, None))
    GB = G.astype(np.float64) @ B.astype(np.float64).T
    for i in range(case.M):
        for k in range(case.row_ptr[case.row_begin + i], case.row_ptr[case.row_begin + i + 1]):
            assert abs(dv[k - case.nz_begin] - GB[i, case.col[k]]) <= 1e-12 * (1 + abs(GB[i, case.col[k]]))
    # adjoint identity <G, A B> = <A^T G, B> = <vals, dvals>
    Y = oracle.spmm(case, Bp, cm)
    L1 = float(np.sum(G.astype(np.float64) * Y))
    L2 = float(np.sum(dB * B.astype(np.float64)))
    vp = case.vals[case.nz_begin:case.nz_begin + case.nnz_panel].astype(np.float64)
    L3 = float(np.dot(vp, dv))
    scale = 1.0 + float(np.sum(np.abs(G) @ np.ones(N))) * float(np.max(np.abs(B)) + 1) * float(np.max(np.abs(vp), initial=0) + 1) * 10
    assert abs(L1 - L2) <= 1e-12 * scale and abs(L1 - L3) <= 1e-12 * scale


def test_backward_finite_difference_exact_for_bilinear():
    """L(B) = <G, A B> is linear in B and in vals, so a central difference
    with any step equals the directional derivative up to rounding."""
    A = oracle.Csr.from_synth(synth.small_rmat(9, 6, P=2, p=0, vals_lo=-1.0))
    rng = np.random.default_rng(41)
    N = 8
    # B on a 2^-10 grid inside (-8, 8) so that B +- 1 is exact in float32
    B = (np.round(np.clip(rng.standard_normal((A.n_cols, N)), -7, 7) * 1024) / 1024).astype(np.float32)
    G = rng.standard_normal((A.M, N)).astype(np.float32)
    dB = oracle.spmm_t(A, G, None)
    uc, off, cm = oracle.select(A)
    dv = oracle.sddmm(A, G, B, None)

    def L(Bm, vals=None):
        Am = A if vals is None else oracle.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, vals, A.P, A.p)
        return float(np.sum(G.astype(np.float64) * oracle.spmm(Am, Bm, None)))

    for trial in range(3):
        E = rng.choice([-1.0, 0.0, 1.0], size=B.shape).astype(np.float32)  # exact B +- E
        fd = (L(B + E) - L(B - E)) / 2.0
        assert abs(fd - float(np.sum(dB * E))) <= 1e-10 * (1 + abs(fd))
        e = np.zeros_like(A.vals)
        idx = rng.integers(A.nz_begin, A.nz_begin + A.nnz_panel, size=16)
        e[idx] = 1.0
        fdv = (L(B, A.vals + e) - L(B, A.vals - e)) / 2.0
        # vals +- 1 is exact in float32 for |vals| < 1
        assert abs(fdv - float(np.sum(dv[np.unique(idx) - A.nz_begin]))) <= 1e-10 * (1 + abs(fdv))


def test_backward_sampled_matches_full():
    A = oracle.Csr.from_synth(synth.small_rmat(10, 8, P=4, p=2))
    rng = np.random.default_rng(43)
    N = 5
    G = rng.standard_normal((A.M, N)).astype(np.float32)
    uc, off, cm = oracle.select(A)
    U = int(off[-1])
    full = oracle.spmm_t(A, G, cm, n_out=U)
    t = np.array([0, U // 3, U - 1, 7])
    assert np.array_equal(oracle.spmm_t_sampled(A, G, cm, U, t), full[t])


def test_backward_transpose_on_nonsymmetric():
    """A^T G differs from A G on a non-symmetric matrix (a dropped transpose fails)."""
    rng = np.random.default_rng(2)
    A = random_csr(rng, 12, 12, 0.3)
    D = dense_of(A)
    assert not np.allclose(D, D.T)
    G = rng.standard_normal((12, 3)).astype(np.float32)
    dB = oracle.spmm_t(A, G, None)
    assert np.allclose(dB, D.T @ G.astype(np.float64), rtol=1e-13, atol=1e-13)
    assert not np.allclose(dB, D @ G.astype(np.float64))


# ----------------------------------------------------------------------------
# error metric
# ----------------------------------------------------------------------------
def test_rel_err_metric():
    Yref = np.array([[1.0, 0.0], [2.0, -1.0]])
    den = np.array([[2.0, 0.0], [4.0, 1.0]])
    assert oracle.rel_err(Yref, Yref, den) == 0.0
    Y = Yref + np.array([[0.5, 0.0], [0.0, 0.25]])
    assert oracle.rel_err(Y, Yref, den) == 0.25
    Y2 = Yref.copy()
    Y2[0, 1] = 1e-30  # denominator 0 demands an exact zero
    assert oracle.rel_err(Y2, Yref, den) == float("inf")
    assert oracle.row_rel_err(Y, Yref, den) == 0.25


def test_generator_counter_hash_pinned():
    """The splitmix64 tensor implementation equals the pure-Python one."""
    import torch

    key = synth.stream_key(0, synth.STREAM_PATTERN)
    idx = torch.arange(0, 2000, dtype=torch.int64) * 7919
    got = synth.draw_u64(key, idx)
    ref = [synth._s64(synth.mix64_py(key + (int(i) + 1) * 0x9E3779B97F4A7C15)) for i in idx]
    assert torch.equal(got, torch.tensor(ref, dtype=torch.int64))


# ----------------------------------------------------------------------------
# row-based scheme (Table 1 Rows; Sec. 3.1 Eq. V_row; Sec. 5.1 stages 3, 5)
# ----------------------------------------------------------------------------
def brute_rows(A: oracle.Csr):
    """Rows(A^(p,q)) by testing every (panel row, block) pair for a nonzero."""
    out = []
    for q in range(A.P):
        lo, hi = q * A.K, min(A.n_cols, (q + 1) * A.K)
        rows = []
        for i in range(A.M):
            g = A.row_begin + i
            cols = A.col[A.row_ptr[g]:A.row_ptr[g + 1]]
            if np.any((cols >= lo) & (cols < hi)):
                rows.append(i)
        out.append(rows)
    return out


def test_c_rows_brute_force(case):
    rs, off = oracle.select_c_rows(case)
    ref = brute_rows(case)
    assert off[0] == 0 and len(off) == case.P + 1
    for q in range(case.P):
        assert list(rs[off[q]:off[q + 1]]) == ref[q]
    # R counts (row, block) pairs with a nonzero: distinct blocks per row
    nz0, n = case.nz_begin, case.nnz_panel
    rows = np.repeat(np.arange(case.M), np.diff(case.row_ptr[case.row_begin:case.row_end + 1]))
    pairs = set(zip(rows.tolist(), (case.col[nz0:nz0 + n] // case.K).tolist()))
    assert off[-1] == len(pairs)


def test_c_rows_fig1_worked_example():
    g = load_golden("fig1_block01.txt")
    n, P, p = g["n"][0][0], g["P"][0][0], g["p"][0][0]
    mask = np.zeros((n, n))
    for r, c, v in g["nz"]:
        mask[r, c] = v
    Ac = oracle.Csr.from_synth(synth.from_dense_pattern(mask, P=P, p=p))
    rs, off = oracle.select_c_rows(Ac)
    (q, *rows), = g["expect_rows_block"]
    assert list(rs[off[q]:off[q + 1]]) == rows
    # Eq. V_row of Sec. 3.1: |Rows(A^(0,1))| N sz, here 3 rows (Fig. 1c)
    assert oracle.v_row_bytes(Ac, 32, 4)[q] == 3 * 32 * 4


def test_c_rows_one_block_is_nonempty_rows():
    A = oracle.Csr.from_synth(synth.small_rmat(10, 8, P=1, p=0))
    rs, off = oracle.select_c_rows(A)
    nonempty = np.flatnonzero(np.diff(A.row_ptr[A.row_begin:A.row_end + 1]) > 0)
    assert np.array_equal(rs, nonempty)


def test_partial_then_aggregate_is_the_product(case):
    rng = np.random.default_rng(11)
    N = 6
    B = rng.standard_normal((case.n_cols, N)).astype(np.float32)
    rs, off = oracle.select_c_rows(case)
    Cp = oracle.partial_c(case, B, rs, off)
    assert Cp.shape == (off[-1], N)
    Y = oracle.aggregate_c(case, Cp, rs, off)
    D = dense_of(case)[case.row_begin:case.row_end]
    assert np.allclose(Y, D @ B.astype(np.float64), rtol=1e-12, atol=1e-12)
    # each partial row is the block's own slice of the product
    for q in range(case.P):
        lo, hi = q * case.K, min(case.n_cols, (q + 1) * case.K)
        ref = D[:, lo:hi] @ B[lo:hi].astype(np.float64)
        assert np.allclose(Cp[off[q]:off[q + 1]], ref[rs[off[q]:off[q + 1]]], rtol=1e-12, atol=1e-12)
    # the absolute-value form gives |A| |B|
    Ya = oracle.aggregate_c(case, oracle.partial_c(case, B, rs, off, abs_mode=True), rs, off)
    assert np.allclose(Ya, np.abs(D) @ np.abs(B.astype(np.float64)), rtol=1e-12, atol=1e-12)


def test_aggregate_is_indexed_add():
    A = oracle.Csr.from_synth(synth.small_rmat(9, 8, P=4, p=1))
    rs, off = oracle.select_c_rows(A)
    rng = np.random.default_rng(5)
    Cp = rng.integers(-8, 9, size=(len(rs), 3)).astype(np.float32)  # exact in any order
    Y = oracle.aggregate_c(A, Cp, rs, off)
    ref = np.zeros((A.M, 3))
    np.add.at(ref, rs, Cp.astype(np.float64))
    assert np.array_equal(Y, ref)


# ----------------------------------------------------------------------------
# joint strategy: minimum (weighted) vertex cover per block (Sec. 5.2-5.4)
# ----------------------------------------------------------------------------
def brute_mvc(n_left, n_right, edges, wl, wr):
    best = None
    n = n_left + n_right
    w = np.concatenate([wl, wr])
    for mask in range(1 << n):
        sel = [(mask >> v) & 1 for v in range(n)]
        if all(sel[i] or sel[n_left + j] for i, j in edges):
            cost = sum(w[v] for v in range(n) if sel[v])
            best = cost if best is None else min(best, cost)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_mvc_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nl, nr = int(rng.integers(1, 7)), int(rng.integers(1, 7))
    mask = rng.random((nl, nr)) < 0.45
    edges = np.argwhere(mask)
    weighted = seed % 2 == 1
    wl = rng.integers(1, 9, nl) if weighted else np.ones(nl, np.int64)
    wr = rng.integers(1, 9, nr) if weighted else np.ones(nr, np.int64)
    mu, cl, cr = oracle.mvc_bipartite(nl, nr, edges, wl, wr)
    assert mu == brute_mvc(nl, nr, edges, wl, wr)
    assert all(cl[i] or cr[j] for i, j in edges)  # a cover
    assert mu == int(wl[cl].sum() + wr[cr].sum())


def test_mvc_unit_costs_is_max_matching():
    """Koenig: with unit costs the minimum cover has the size of a maximum matching."""
    from scipy.sparse import csr_array
    from scipy.sparse.csgraph import maximum_bipartite_matching

    rng = np.random.default_rng(4)
    for _ in range(6):
        nl, nr = 60, 45
        mask = rng.random((nl, nr)) < 0.05
        edges = np.argwhere(mask)
        mu, cl, cr = oracle.mvc_bipartite(nl, nr, edges)
        match = maximum_bipartite_matching(csr_array(mask.astype(np.int8)), perm_type="column")
        assert mu == int((match >= 0).sum())
        assert all(cl[i] or cr[j] for i, j in edges)


def test_joint_cover_fig1_worked_example():
    g = load_golden("fig1_block01.txt")
    n, P, p = g["n"][0][0], g["P"][0][0], g["p"][0][0]
    mask = np.zeros((n, n))
    for r, c, v in g["nz"]:
        mask[r, c] = v
    Ac = oracle.Csr.from_synth(synth.from_dense_pattern(mask, P=P, p=p))
    res = oracle.joint_cover(Ac)
    (q, mu), = g["expect_joint_cover_block"]
    assert res[p] is None
    assert res[q][0] == mu
    (_, *rows), = g["expect_joint_rows"]
    (_, *cols), = g["expect_joint_cols"]
    assert list(res[q][3]) == rows and list(res[q][4]) == cols


def test_joint_cover_bounds_rmat():
    """mu <= min(|Rows|, |Cols|) per block (the dominance of Sec. 5.4)."""
    A = oracle.Csr.from_synth(synth.small_rmat(10, 8, P=8, p=2))
    uc, off, _ = oracle.select(A)
    rs, roff = oracle.select_c_rows(A)
    for q, r in enumerate(oracle.joint_cover(A)):
        if r is None:
            continue
        mu, rows, cols, crow, ccol = r
        assert len(cols) == off[q + 1] - off[q] and len(rows) == roff[q + 1] - roff[q]
        assert mu <= min(len(rows), len(cols))
        assert mu == len(crow) + len(ccol)
