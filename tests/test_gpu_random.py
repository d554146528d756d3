"""Randomised shapes through every GPU entry point, against the oracle.

Ragged panels and blocks, dense widths that are not multiples of the 16-byte
vector (scalar lanes), several column tiles, padded leading dimensions on
both sides, float32 and bfloat16.  Sizes stay small so the oracle answers
in milliseconds.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

TOL_F32 = 1e-5
TOL_BF16 = 1e-2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shiro():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20178_amd as s

    s._lib.load()
    return s


def random_case(seed):
    rng = np.random.default_rng(500 + seed)
    n_rows = int(rng.integers(40, 2500))
    n_cols = int(rng.integers(40, 2500))
    dens = float(rng.uniform(0.001, 0.03))
    mask = rng.random((n_rows, n_cols)) < dens
    if seed % 3 == 0:  # a hub row and an empty stretch of rows
        mask[n_rows // 3, :] = rng.random(n_cols) < 0.6
        mask[n_rows // 2: n_rows // 2 + 20, :] = False
    vals = rng.uniform(-1, 1, size=(n_rows, n_cols)).astype(np.float32) * mask
    vals[mask & (vals == 0)] = 0.5
    P = int(rng.integers(1, 10))
    p = int(rng.integers(0, P))
    N = int(rng.choice([1, 3, 8, 33, 64, 100, 160, 264]))
    return synth.from_dense_pattern(vals, P=P, p=p, name=f"rand{seed}"), N, rng


def padded(t: torch.Tensor, pad: int) -> torch.Tensor:
    """The same values in a buffer with `pad` extra columns (leading dimension > N)."""
    out = torch.full((t.shape[0], t.shape[1] + pad), float("nan"), dtype=t.dtype, device=t.device)
    out[:, : t.shape[1]] = t
    return out[:, : t.shape[1]]


@pytest.mark.parametrize("seed", range(10))
def test_random_shapes(shiro, seed):
    A, N, rng = random_case(seed)
    dtype = torch.float32 if seed % 2 == 0 else torch.bfloat16
    tol = TOL_F32 if dtype == torch.float32 else TOL_BF16
    dev = torch.device("cuda")
    Ad = A.to(dev)
    Ac = oracle.Csr.from_synth(A)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p, check=True)
    U, _ = shiro.select_rows(plan)
    uc, off, cm = oracle.select(Ac)
    assert U == len(uc)
    B = synth.dense(A.n_cols, N, seed, synth.STREAM_B)
    G = synth.dense(max(Ac.M, 1), N, seed, synth.STREAM_DY)[: Ac.M]
    Bd = padded(B.to(dtype).to(dev), 3 + seed % 5)
    Gd = padded(G.to(dtype).to(dev), 1 + seed % 3)
    Bn, Gn = B.numpy(), G.numpy()
    # pack (bit-exact, strided source)
    Bp = shiro.pack_B(plan, Bd)
    ref_p = oracle.pack(B.to(dtype).float().numpy(), uc)
    assert np.array_equal(Bp.float().cpu().numpy(), ref_p)
    # forward, batched and per block, into a padded output
    Yref = oracle.spmm(Ac, Bn, None)
    den = oracle.spmm(Ac, Bn, None, abs_mode=True)
    for mode in ("batched", "per_block"):
        Y = padded(torch.empty(Ac.M, N, dtype=dtype, device=dev), 2)
        shiro.spmm(plan, Ad.vals, Bp, out=Y, mode=mode)
        assert oracle.rel_err(Y.float().cpu().numpy(), Yref, den) <= tol, mode
    # backward: dBpacked, dB (add onto ones), dvals
    dBp = torch.empty(U, N, dtype=dtype, device=dev)
    dB = padded(torch.ones(A.n_cols, N, dtype=dtype, device=dev), 4)
    dvals = torch.zeros(A.nnz, device=dev)
    shiro.spmm_backward(plan, Ad.vals, Gd, Bp, dBpacked=dBp, dB=dB, dvals=dvals)
    rdBp = oracle.spmm_t(Ac, Gn, cm, n_out=U)
    rden = oracle.spmm_t(Ac, Gn, cm, n_out=U, abs_mode=True)
    assert oracle.rel_err(dBp.float().cpu().numpy(), rdBp, rden) <= tol
    full = np.ones((A.n_cols, N))
    full[uc] += rdBp
    fden = np.ones((A.n_cols, N))
    fden[uc] += rden
    assert oracle.rel_err(dB.float().cpu().numpy(), full, fden) <= tol
    rdv = oracle.sddmm(Ac, Gn, Bn, None)
    rdvd = oracle.sddmm(Ac, Gn, Bn, None, abs_mode=True)
    assert oracle.rel_err(dvals.cpu().numpy()[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel], rdv, rdvd) <= tol
    # row-based scheme and joint strategy (float32 in, float32 out)
    R, _ = shiro.select_c_rows(plan)
    Cp = shiro.partial_c(plan, Ad.vals, Bd, R, out_dtype=torch.float32)
    Yr = shiro.aggregate_c(plan, Cp)
    assert oracle.rel_err(Yr.cpu().numpy(), Yref, den) <= tol
    if A.P > 1:
        js = shiro.JointSpMM(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
        Yj = js.forward(Ad.vals, Bd)
        assert oracle.rel_err(Yj.float().cpu().numpy(), Yref, den) <= tol


def random_tuning(rng, walk=True):
    return dict(chunk=int(rng.choice([16, 48, 100, 128, 512, 2048])),
                lanes=int(rng.choice([8, 16, 32, 64])),
                unroll=int(rng.choice([1, 2, 4])),
                group_rows=int(rng.integers(0, 4 if walk else 2)),
                xcd_remap=int(rng.integers(0, 2)),
                wg_per_cu=int(rng.choice([1, 2, 4, 8, 16])))


@pytest.mark.parametrize("seed", range(10, 22))
def test_random_shapes_random_tunings(shiro, seed):
    """Random shapes with a random launch configuration per kernel family
    (chunk sizes that are not powers of two, every lane width, depth and
    layout, XCD remap, one to sixteen workgroups per CU, rows in LDS)."""
    A, N, rng = random_case(seed)
    dtype = torch.float32 if seed % 2 == 0 else torch.bfloat16
    tol = TOL_F32 if dtype == torch.float32 else TOL_BF16
    dev = torch.device("cuda")
    Ad = A.to(dev)
    Ac = oracle.Csr.from_synth(A)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    uc, off, cm = oracle.select(Ac)
    knobs = {k: random_tuning(rng, walk=k != "sddmm") for k in ("spmm", "spmm_t", "sddmm", "partial_c", "aggregate_c")}
    for k in ("spmm", "spmm_t"):  # rows kept in LDS by the windowed walk
        if knobs[k]["group_rows"] == 3:
            knobs[k]["lds_rows"] = int(rng.choice([0, 1, 7, 64]))
    for k, t in knobs.items():
        shiro.set_tuning(plan, k, N, dtype, **t)
        if k in ("partial_c", "aggregate_c"):
            shiro.set_tuning(plan, k, N, torch.float32, **t)
    B = synth.dense(A.n_cols, N, seed, synth.STREAM_B)
    G = synth.dense(max(Ac.M, 1), N, seed, synth.STREAM_DY)[: Ac.M]
    Bd, Gd = B.to(dtype).to(dev), G.to(dtype).to(dev)
    Bn, Gn = B.numpy(), G.numpy()
    Bp = shiro.pack_B(plan, Bd)
    Yref = oracle.spmm(Ac, Bn, None)
    den = oracle.spmm(Ac, Bn, None, abs_mode=True)
    Y = shiro.spmm(plan, Ad.vals, Bp)
    assert oracle.rel_err(Y.float().cpu().numpy(), Yref, den) <= tol, knobs
    dBp = torch.empty(U, N, dtype=dtype, device=dev)
    dvals = torch.zeros(A.nnz, device=dev)
    shiro.spmm_backward(plan, Ad.vals, Gd, Bp, dBpacked=dBp, dvals=dvals)
    rdBp = oracle.spmm_t(Ac, Gn, cm, n_out=U)
    rden = oracle.spmm_t(Ac, Gn, cm, n_out=U, abs_mode=True)
    assert oracle.rel_err(dBp.float().cpu().numpy(), rdBp, rden) <= tol, knobs
    rdv = oracle.sddmm(Ac, Gn, Bn, None)
    rdvd = oracle.sddmm(Ac, Gn, Bn, None, abs_mode=True)
    assert oracle.rel_err(dvals.cpu().numpy()[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel], rdv, rdvd) <= tol, knobs
    # dvals alone (the sampled product's own kernel)
    dv2 = torch.zeros_like(dvals)
    shiro.spmm_backward(plan, Ad.vals, Gd, Bp, dvals=dv2)
    assert oracle.rel_err(dv2.cpu().numpy()[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel], rdv, rdvd) <= tol, knobs
    R, _ = shiro.select_c_rows(plan)
    Cp = shiro.partial_c(plan, Ad.vals, Bd, R, out_dtype=torch.float32)
    Yr = shiro.aggregate_c(plan, Cp)
    assert oracle.rel_err(Yr.cpu().numpy(), Yref, den) <= tol, knobs
