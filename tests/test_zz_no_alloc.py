"""GPU test of shiro_spmm_noalloc, the allocation-free form of the batched
product (carry slots in the library's fixed device array).

Called through the C ABI (ctypes) and compared bit for bit with shiro_spmm
in SHIRO_MODE_BATCHED on the same plan, tuning and inputs: the two share
their kernels, so the outputs must be identical; the result is also checked
against the FP64 oracle at the float32 tolerance.  Two calls in a row, the
second on a smaller pattern, so the second call runs on an array that still
holds the first call's slots.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20178_amd as s

    s._lib.load()
    return s


def _setup(s, A, N, dtype, tuning=None):
    dev = torch.device("cuda:0")
    Ad = A.to(dev)
    plan = s.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = s.select_rows(plan)
    if tuning:
        s.set_tuning(plan, "spmm", N, dtype, **tuning)
    s.prepare(plan, N, dtype, ops=("spmm",))
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev).to(dtype)
    Bp = s.pack_B(plan, B)
    return plan, Ad, B, Bp


def _call_noalloc(s, plan, vals, Bp, Y):
    L = s._lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    return L.shiro_spmm_noalloc(plan.handle, ctypes.c_void_p(vals.data_ptr()), ctypes.c_void_p(Bp.data_ptr()),
                                Bp.stride(0), Bp.shape[1], s._dt(Bp.dtype), ctypes.c_void_p(Y.data_ptr()),
                                Y.stride(0), s._dt(Y.dtype), ctypes.c_void_p(stream))


def _check_against_spmm_and_oracle(s, A, plan, Ad, B, Bp, dtype):
    rows = plan.info()["rows"]
    N = Bp.shape[1]
    Y_ref = torch.full((rows, N), float("nan"), dtype=dtype, device=Bp.device)
    s.spmm(plan, Ad.vals, Bp, out=Y_ref)
    Y = torch.full((rows, N), float("nan"), dtype=dtype, device=Bp.device)
    rc = _call_noalloc(s, plan, Ad.vals, Bp, Y)
    assert rc == 0, s._lib.load().shiro_last_error()
    torch.cuda.synchronize()
    assert torch.equal(Y.view(torch.int16 if dtype == torch.bfloat16 else torch.int32),
                       Y_ref.view(torch.int16 if dtype == torch.bfloat16 else torch.int32))
    Ac = oracle.Csr.from_synth(A)
    Bh = B.float().cpu().numpy()
    ref = oracle.spmm(Ac, Bh, None)
    den = oracle.spmm(Ac, Bh, None, abs_mode=True)
    err = oracle.rel_err(Y.float().cpu().numpy(), ref, den)
    assert err <= (TOL_F32 if dtype == torch.float32 else 1e-2), err


def test_noalloc_matches_spmm_two_calls(lib):
    s = lib
    # first call: a multi-block panel with a split-heavy tuning (small chunks,
    # many carry slots); second call: a smaller pattern and width
    A1 = synth.small_rmat(13, 16, P=8, p=0)
    p1 = _setup(s, A1, 128, torch.float32, tuning={"chunk": 32, "group_rows": 2, "unroll": 4})
    _check_against_spmm_and_oracle(s, A1, *p1, torch.float32)
    A2 = synth.small_rmat(10, 8, P=3, p=2)
    p2 = _setup(s, A2, 64, torch.float32, tuning={"chunk": 48, "group_rows": 0, "unroll": 2})
    _check_against_spmm_and_oracle(s, A2, *p2, torch.float32)


def test_noalloc_bf16_and_row_kernels(lib):
    s = lib
    A = synth.small_rmat(12, 8, P=4, p=1)
    for grp in (0, 1, 2, 3):
        p = _setup(s, A, 128, torch.bfloat16, tuning={"chunk": 64, "group_rows": grp})
        _check_against_spmm_and_oracle(s, A, *p, torch.bfloat16)


def test_noalloc_windowed_walk_lds_rows(lib):
    s = lib
    A = synth.small_rmat(13, 16, P=4, p=0)
    for H in (0, 16):
        p = _setup(s, A, 128, torch.float32, tuning={"chunk": 64, "group_rows": 3, "lds_rows": H})
        _check_against_spmm_and_oracle(s, A, *p, torch.float32)
    # LDS rows of a size the plan has not prepared: refused before any launch
    plan, Ad, B, Bp = p
    s.set_tuning(plan, "spmm", 128, torch.float32, chunk=64, group_rows=3, lds_rows=32)
    Y = torch.full((plan.info()["rows"], 128), 7.0, device=Bp.device)
    assert _call_noalloc(s, plan, Ad.vals, Bp, Y) == -6
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    s.prepare(plan, 128, torch.float32, ops=("spmm",))
    _check_against_spmm_and_oracle(s, A, plan, Ad, B, Bp, torch.float32)


def test_noalloc_not_prepared_and_too_large(lib):
    s = lib
    dev = torch.device("cuda:0")
    A = synth.small_rmat(13, 16, P=1, p=0)
    Ad = A.to(dev)
    plan = s.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    s.select_rows(plan)
    info = plan.info()
    N = 1024
    Bp = torch.zeros(info["U"], N, device=dev)
    Y = torch.zeros(info["rows"], N, device=dev)
    # no prepare for this width: refused, nothing launched
    assert _call_noalloc(s, plan, Ad.vals, Bp, Y) == -6
    # a tuning whose carry slots exceed the fixed area: 2 * W * N floats with
    # W = (rows + nnz) / 16 chunks of 16 items
    s.set_tuning(plan, "spmm", N, torch.float32, chunk=16)
    s.prepare(plan, N, torch.float32, ops=("spmm",))
    W = -(-(info["rows"] + info["nnz"]) // 16)
    assert 2 * W * N * 4 > 32 << 20
    Y.fill_(7.0)
    assert _call_noalloc(s, plan, Ad.vals, Bp, Y) == -8
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())  # refused before any launch
