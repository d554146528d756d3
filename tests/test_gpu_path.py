"""GPU parity of the HIP path against the FP64 oracle (small and medium sizes).

Every case runs partition -> select_rows -> pack_B -> spmm -> spmm_backward
through the C ABI (via the ctypes binding) and compares element by element:
indices, offsets and packed bytes bit-exactly; float32 outputs within 1e-5
and bfloat16 outputs within 1e-2 of the oracle, relative to the oracle's
absolute product (|A||B|, |A|^T|dY|, sum |dY||B|) entry by entry.
"""
import gc

import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import load_golden

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_BF16 = 1e-2


@pytest.fixture(scope="module")
def shiro():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_20178_amd as s

    s._lib.load()  # fails loudly if the library is missing
    return s


def bf16_to_f32(t: torch.Tensor) -> np.ndarray:
    return t.float().cpu().numpy()


def make_case(name):
    """(SparseInput, N) for a named small case."""
    if name == "config1_rmat12":
        return synth.config1(), 32
    if name == "rmat12_P8_p0":
        return synth.small_rmat(12, 16, P=8, p=0), 128
    if name == "rmat11_P7_p6_ragged":
        return synth.small_rmat(11, 8, P=7, p=6), 64
    if name == "rmat10_P3_N3_scalar":
        return synth.small_rmat(10, 4, P=3, p=1, vals_lo=-1.0), 3
    if name == "rmat12_P16_N256":
        return synth.small_rmat(12, 8, P=16, p=5), 256
    if name == "rmat11_N384_multitile":
        return synth.small_rmat(11, 8, P=2, p=0), 384
    if name == "empty_panel":
        return synth.from_dense_pattern(np.zeros((9, 9)), P=2, p=1), 8
    if name == "hub_row":
        rng = np.random.default_rng(5)
        n = 40000
        m = np.zeros((64, n), np.float32)
        m[0, rng.choice(n, 30000, replace=False)] = rng.uniform(-1, 1, 30000)  # one very long row
        m[5, :] = 0.5  # a full row
        m[7, rng.choice(n, 300, replace=False)] = 1.0
        rows, cols = np.nonzero(m)
        rp = np.zeros(65, np.int64)
        np.cumsum(np.bincount(rows, minlength=64), out=rp[1:])
        A = synth.SparseInput("hub", 64, n, torch.from_numpy(rp), torch.from_numpy(cols.astype(np.int32)),
                              torch.from_numpy(m[rows, cols]), 1, 0)
        return A, 128
    if name == "rect_empty_block":
        rng = np.random.default_rng(9)
        mask = rng.random((300, 1000)) < 0.02
        mask[:, 250:500] = False  # an empty column block
        mask[150:300, 0:250] = True  # a dense block
        vals = rng.uniform(0.1, 1, size=(300, 1000)).astype(np.float32) * mask
        return synth.from_dense_pattern(vals, P=4, p=1, name="rect"), 64
    raise KeyError(name)


CASES = ["config1_rmat12", "rmat12_P8_p0", "rmat11_P7_p6_ragged", "rmat10_P3_N3_scalar",
         "rmat12_P16_N256", "rmat11_N384_multitile", "empty_panel", "hub_row", "rect_empty_block"]


class Run:
    """One case run through the GPU path plus its oracle references."""

    def __init__(self, shiro, name):
        A, N = make_case(name)
        self.A, self.N = A, N
        self.dev = torch.device("cuda")
        self.Ad = A.to(self.dev)
        self.Ac = oracle.Csr.from_synth(A)
        self.plan = shiro.partition(self.Ad.row_ptr, self.Ad.col, A.n_rows, A.n_cols, A.P, A.p, check=True)
        self.U, self.Uq = shiro.select_rows(self.plan)
        self.B = synth.dense(A.n_cols, N, 0, synth.STREAM_B)
        self.G = synth.dense(max(self.Ac.M, 1), N, 0, synth.STREAM_DY)[: self.Ac.M]
        self.uc, self.off, self.cm = oracle.select(self.Ac)


@pytest.fixture(scope="module", params=CASES)
def run(request, shiro):
    return Run(shiro, request.param)


def test_partition_and_block_nnz(shiro, run):
    inf = run.plan.info()
    Ac = run.Ac
    assert (inf["row_begin"], inf["rows"], inf["K"]) == (Ac.row_begin, Ac.M, Ac.K)
    assert (inf["nz_begin"], inf["nnz"]) == (Ac.nz_begin, Ac.nnz_panel)
    assert np.array_equal(shiro.block_nnz(run.plan).cpu().numpy(), oracle.block_nnz(Ac))


def test_select_bit_exact(shiro, run):
    uc, off, cm = (t.cpu().numpy() for t in shiro.selection(run.plan))
    assert run.U == len(run.uc)
    assert run.Uq == list(np.diff(run.off))
    assert np.array_equal(uc, run.uc)
    assert np.array_equal(off, run.off)
    assert np.array_equal(cm, run.cm)


def test_pack_bit_exact(shiro, run):
    Bp = shiro.pack_B(run.plan, run.B.to(run.dev))
    ref = oracle.pack(run.B.numpy(), run.uc)
    assert Bp.cpu().numpy().tobytes() == ref.tobytes()
    Bh = run.B.to(torch.bfloat16)
    Bph = shiro.pack_B(run.plan, Bh.to(run.dev))
    refh = oracle.pack(Bh.view(torch.int16).numpy(), run.uc)
    assert Bph.cpu().view(torch.int16).numpy().tobytes() == refh.tobytes()
    # strided source and destination (leading dimensions > N)
    Bw = torch.zeros(run.A.n_cols, run.N + 5, device=run.dev)
    Bw[:, : run.N] = run.B.to(run.dev)
    out = torch.full((run.U, run.N + 3), -7.0, device=run.dev)
    shiro.pack_B(run.plan, Bw[:, : run.N], out=out[:, : run.N])
    o = out.cpu().numpy()
    assert o[:, : run.N].tobytes() == ref.tobytes() and np.all(o[:, run.N:] == -7.0)


def _fwd_ref(run, B):
    Y = oracle.spmm(run.Ac, B, None)
    den = oracle.spmm(run.Ac, B, None, abs_mode=True)
    return Y, den


@pytest.mark.parametrize("mode", ["batched", "per_block"])
def test_spmm_f32(shiro, run, mode):
    Bp = shiro.pack_B(run.plan, run.B.to(run.dev))
    Y = shiro.spmm(run.plan, run.Ad.vals, Bp, mode=mode)
    Yref, den = _fwd_ref(run, run.B.numpy())
    err = oracle.rel_err(Y.cpu().numpy(), Yref, den)
    assert err <= TOL_F32, err
    # run-to-run determinism
    Y2 = shiro.spmm(run.plan, run.Ad.vals, Bp, mode=mode)
    assert torch.equal(Y, Y2)


def test_spmm_bf16(shiro, run):
    Bh = run.B.to(torch.bfloat16).to(run.dev)
    Bp = shiro.pack_B(run.plan, Bh)
    Yf = shiro.spmm(run.plan, run.Ad.vals, Bp, out_dtype=torch.float32)
    Yh = shiro.spmm(run.plan, run.Ad.vals, Bp, out_dtype=torch.bfloat16)
    Yh2 = shiro.spmm(run.plan, run.Ad.vals, Bp, out_dtype=torch.bfloat16, mode="per_block")
    Yref, den = _fwd_ref(run, run.B.numpy())  # end to end: FP64 on the original FP32 B
    for Y in (Yf, Yh, Yh2):
        assert oracle.rel_err(bf16_to_f32(Y), Yref, den) <= TOL_BF16
    # kernel only: FP64 on the bf16-rounded inputs, float32 accumulation error only
    Bq = Bh.float().cpu().numpy()
    Yq, denq = _fwd_ref(run, Bq)
    assert oracle.rel_err(Yf.cpu().numpy(), Yq, denq) <= TOL_F32
    assert oracle.rel_err(bf16_to_f32(Yh), Yq, denq) <= 2.0 ** -8 + TOL_F32


def _bwd_refs(run, B, G):
    Ac = run.Ac
    dBp = oracle.spmm_t(Ac, G, run.cm, n_out=run.U)
    dBp_den = oracle.spmm_t(Ac, G, run.cm, n_out=run.U, abs_mode=True)
    dv = oracle.sddmm(Ac, G, B, None)
    dv_den = oracle.sddmm(Ac, G, B, None, abs_mode=True)
    return dBp, dBp_den, dv, dv_den


def test_backward_f32(shiro, run):
    dev = run.dev
    Bp = shiro.pack_B(run.plan, run.B.to(dev))
    dY = run.G.to(dev)
    dBp = torch.empty(run.U, run.N, device=dev)
    base = torch.randn(run.A.n_cols, run.N, generator=torch.Generator().manual_seed(3))
    dB = base.to(dev)  # add-scatter on top of existing values
    dvals = torch.zeros(run.A.nnz, device=dev)
    shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dBpacked=dBp, dB=dB, dvals=dvals)
    rdBp, rden, rdv, rdv_den = _bwd_refs(run, run.B.numpy(), run.G.numpy())
    assert oracle.rel_err(dBp.cpu().numpy(), rdBp, rden) <= TOL_F32
    full = base.numpy().astype(np.float64)
    full[run.uc] += rdBp
    fden = np.abs(base.numpy()).astype(np.float64)
    fden[run.uc] += rden
    got = dB.cpu().numpy()
    assert oracle.rel_err(got, full, np.maximum(fden, 1e-300)) <= TOL_F32
    mask = np.ones(run.A.n_cols, bool)
    mask[run.uc] = False
    assert np.array_equal(got[mask], base.numpy()[mask])  # rows outside Cols untouched
    gv = dvals.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
    assert oracle.rel_err(gv, rdv, rdv_den) <= TOL_F32
    # determinism of every output
    dBp2 = torch.empty_like(dBp)
    dvals2 = torch.zeros_like(dvals)
    shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dBpacked=dBp2, dvals=dvals2)
    assert torch.equal(dBp, dBp2) and torch.equal(dvals, dvals2)
    # dvals alone (row-order SDDMM pass, no transposed product)
    dvals3 = torch.zeros_like(dvals)
    shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dvals=dvals3)
    gv3 = dvals3.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
    assert oracle.rel_err(gv3, rdv, rdv_den) <= TOL_F32
    # dB alone (transposed product without dBpacked and without dvals)
    dB4 = torch.zeros(run.A.n_cols, run.N, device=dev)
    shiro.spmm_backward(run.plan, run.Ad.vals, dY, None, dB=dB4)
    assert oracle.rel_err(dB4.cpu().numpy()[run.uc], rdBp, rden) <= TOL_F32
    # overwrite form: selected rows of dB replaced, the others untouched,
    # with and without the fused dvals
    for with_dvals in (True, False):
        dB5 = base.to(dev)
        dvals5 = torch.zeros_like(dvals)
        shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp if with_dvals else None, dB=dB5,
                            dvals=dvals5 if with_dvals else None, dB_overwrite=True)
        got5 = dB5.cpu().numpy()
        assert oracle.rel_err(got5[run.uc], rdBp, rden) <= TOL_F32
        assert np.array_equal(got5[mask], base.numpy()[mask])
        if with_dvals:
            assert torch.equal(dvals5, dvals)


def test_backward_bf16(shiro, run):
    dev = run.dev
    Bh = run.B.to(torch.bfloat16)
    Gh = run.G.to(torch.bfloat16)
    Bp = shiro.pack_B(run.plan, Bh.to(dev))
    dBp = torch.empty(run.U, run.N, dtype=torch.bfloat16, device=dev)
    dB = torch.zeros(run.A.n_cols, run.N, dtype=torch.bfloat16, device=dev)
    dvals = torch.zeros(run.A.nnz, device=dev)
    shiro.spmm_backward(run.plan, run.Ad.vals, Gh.to(dev), Bp, dBpacked=dBp, dB=dB, dvals=dvals)
    rdBp, rden, rdv, rdv_den = _bwd_refs(run, run.B.numpy(), run.G.numpy())
    assert oracle.rel_err(bf16_to_f32(dBp), rdBp, rden) <= TOL_BF16
    assert oracle.rel_err(bf16_to_f32(dB)[run.uc], rdBp, rden) <= TOL_BF16
    gv = dvals.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
    assert oracle.rel_err(gv, rdv, rdv_den) <= TOL_BF16
    # overwrite form on a buffer of ones: selected rows equal the add form's
    # result on zeros (one rounding either way), the others stay one
    dB2 = torch.ones(run.A.n_cols, run.N, dtype=torch.bfloat16, device=dev)
    shiro.spmm_backward(run.plan, run.Ad.vals, Gh.to(dev), Bp, dB=dB2, dvals=dvals, dB_overwrite=True)
    mask = torch.ones(run.A.n_cols, dtype=torch.bool)
    mask[torch.from_numpy(run.uc).long()] = False
    assert torch.equal(dB2.cpu()[~mask], dB.cpu()[~mask])
    assert bool((dB2.cpu()[mask] == 1).all())
    # the group kernel in bfloat16 (lanes below one tile are raised to it)
    for lanes in (8, 16, 32):
        shiro.set_tuning(run.plan, "spmm_t", run.N, torch.bfloat16, lanes=lanes, group_rows=1, chunk=64, unroll=2)
        dB3 = torch.zeros_like(dB)
        dvals3 = torch.zeros_like(dvals)
        shiro.spmm_backward(run.plan, run.Ad.vals, Gh.to(dev), Bp, dB=dB3, dvals=dvals3, dB_overwrite=True)
        assert oracle.rel_err(bf16_to_f32(dB3)[run.uc], rdBp, rden) <= TOL_BF16
        gv3 = dvals3.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
        assert oracle.rel_err(gv3, rdv, rdv_den) <= TOL_BF16
    shiro.set_tuning(run.plan, "spmm_t", run.N, torch.bfloat16, lanes=64, group_rows=0, chunk=128, unroll=2)


@pytest.mark.parametrize("knobs", [
    dict(chunk=16, lanes=8, unroll=1),
    dict(chunk=64, lanes=64, unroll=4),
    dict(chunk=1024, lanes=16, unroll=2, xcd_remap=1, wg_per_cu=2),
    dict(chunk=4096, lanes=32, unroll=4, wg_per_cu=1),
    dict(chunk=16, lanes=32, unroll=1, group_rows=1),
    dict(chunk=64, lanes=16, unroll=2, group_rows=1, xcd_remap=1),
    dict(chunk=512, lanes=8, unroll=4, group_rows=1),
])
def test_tunings_all_correct(shiro, run, knobs):
    """Small chunks split rows over many wavefronts (carry + fix-up path)."""
    for k in ("spmm", "spmm_t", "sddmm"):
        shiro.set_tuning(run.plan, k, run.N, torch.float32, **knobs)
    dev = run.dev
    Bp = shiro.pack_B(run.plan, run.B.to(dev))
    Y = shiro.spmm(run.plan, run.Ad.vals, Bp)
    Yref, den = _fwd_ref(run, run.B.numpy())
    assert oracle.rel_err(Y.cpu().numpy(), Yref, den) <= TOL_F32
    dBp = torch.empty(run.U, run.N, device=dev)
    dvals = torch.zeros(run.A.nnz, device=dev)
    shiro.spmm_backward(run.plan, run.Ad.vals, run.G.to(dev), Bp, dBpacked=dBp, dvals=dvals)
    rdBp, rden, rdv, rdv_den = _bwd_refs(run, run.B.numpy(), run.G.numpy())
    assert oracle.rel_err(dBp.cpu().numpy(), rdBp, rden) <= TOL_F32
    gv = dvals.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
    assert oracle.rel_err(gv, rdv, rdv_den) <= TOL_F32
    # the form autograd uses: dB rows overwritten, dvals fused (carries of cut
    # rows are stored by the fix-up)
    dB = torch.full((run.A.n_cols, run.N), 7.0, device=dev)
    dvals2 = torch.zeros_like(dvals)
    shiro.spmm_backward(run.plan, run.Ad.vals, run.G.to(dev), Bp, dB=dB, dvals=dvals2, dB_overwrite=True)
    got = dB.cpu().numpy()
    assert oracle.rel_err(got[run.uc], rdBp, rden) <= TOL_F32
    mask = np.ones(run.A.n_cols, bool)
    mask[run.uc] = False
    assert bool((got[mask] == 7.0).all())
    assert oracle.rel_err(dvals2.cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel], rdv,
                          rdv_den) <= TOL_F32
    for k in ("spmm", "spmm_t", "sddmm"):  # back to the defaults for other tests
        shiro.set_tuning(run.plan, k, run.N, torch.float32, chunk=256 if k != "sddmm" else 512, lanes=64,
                         unroll=2, xcd_remap=0, wg_per_cu=8, group_rows=0)


@pytest.mark.parametrize("knobs", [
    dict(chunk=16, lanes=32, unroll=1),
    dict(chunk=64, lanes=16, unroll=4, xcd_remap=1),
    dict(chunk=512, lanes=8, unroll=2, wg_per_cu=2),
    dict(chunk=128, lanes=64, unroll=4),
    dict(chunk=2048, lanes=32, unroll=2, wg_per_cu=1),
])
@pytest.mark.parametrize("walk", [2, 3])
def test_nonzero_walk_correct(shiro, run, knobs, walk):
    """The nonzero walk (group_rows 2, and 3 with windowed index streams) of
    every kernel that has it: forward,
    transposed product, partial rows and their sum.  Small chunks cut rows
    into many carried pieces; with few workers each lane group walks a long
    run of chunks (indices loaded one step ahead across chunk ends); rows
    with no nonzeros (the hub, empty and R-MAT cases) are written as zeros,
    or left alone when the sum is added."""
    dev = run.dev
    kinds = (("spmm", torch.float32), ("spmm", torch.bfloat16), ("spmm_t", torch.float32),
             ("spmm_t", torch.bfloat16), ("partial_c", torch.float32), ("aggregate_c", torch.float32))
    saved = {k: shiro.get_tuning(run.plan, k[0], run.N, k[1]) for k in kinds}
    for k in kinds:
        shiro.set_tuning(run.plan, k[0], run.N, k[1], group_rows=walk, **knobs)
    try:
        Bp = shiro.pack_B(run.plan, run.B.to(dev))
        Yref, Yden = _fwd_ref(run, run.B.numpy())
        # forward on a buffer of NaNs: every row, empty ones included, is written
        Y = torch.full((run.Ac.M, run.N), float("nan"), device=dev)
        shiro.spmm(run.plan, run.Ad.vals, Bp, out=Y)
        assert oracle.rel_err(Y.cpu().numpy(), Yref, Yden) <= TOL_F32
        Bph0 = shiro.pack_B(run.plan, run.B.to(torch.bfloat16).to(dev))
        for odt in (torch.bfloat16, torch.float32):
            Yh = shiro.spmm(run.plan, run.Ad.vals, Bph0, out_dtype=odt)
            assert oracle.rel_err(bf16_to_f32(Yh), Yref, Yden) <= TOL_BF16
        dY = run.G.to(dev)
        rdBp, rden, rdv, rdv_den = _bwd_refs(run, run.B.numpy(), run.G.numpy())
        nz = slice(run.Ac.nz_begin, run.Ac.nz_begin + run.Ac.nnz_panel)
        dBp = torch.empty(run.U, run.N, device=dev)
        dvals = torch.zeros(run.A.nnz, device=dev)
        shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dBpacked=dBp, dvals=dvals)
        assert oracle.rel_err(dBp.cpu().numpy(), rdBp, rden) <= TOL_F32
        assert oracle.rel_err(dvals.cpu().numpy()[nz], rdv, rdv_den) <= TOL_F32
        # overwrite form: selected rows replaced, the others untouched
        dB = torch.full((run.A.n_cols, run.N), 7.0, device=dev)
        dv2 = torch.zeros_like(dvals)
        shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dB=dB, dvals=dv2, dB_overwrite=True)
        got = dB.cpu()
        sel = torch.zeros(run.A.n_cols, dtype=torch.bool)
        sel[torch.from_numpy(run.uc).long()] = True
        assert torch.equal(got[sel], dBp.cpu())
        assert bool((got[~sel] == 7.0).all())
        assert torch.equal(dv2, dvals)
        # add form on ones: each selected row is 1 + the same sum, rounded once
        dBa = torch.ones(run.A.n_cols, run.N, device=dev)
        shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dB=dBa)
        assert torch.equal(dBa.cpu()[sel], (1.0 + dBp).cpu())
        assert bool((dBa.cpu()[~sel] == 1.0).all())
        # bfloat16 storage, float32 accumulation
        Bph = shiro.pack_B(run.plan, run.B.to(torch.bfloat16).to(dev))
        dBph = torch.empty(run.U, run.N, dtype=torch.bfloat16, device=dev)
        dvh = torch.zeros_like(dvals)
        shiro.spmm_backward(run.plan, run.Ad.vals, run.G.to(torch.bfloat16).to(dev), Bph, dBpacked=dBph, dvals=dvh)
        assert oracle.rel_err(bf16_to_f32(dBph), rdBp, rden) <= TOL_BF16
        assert oracle.rel_err(dvh.cpu().numpy()[nz], rdv, rdv_den) <= TOL_BF16
        # the row-based scheme's partial rows
        R, _ = shiro.select_c_rows(run.plan)
        rs, off = oracle.select_c_rows(run.Ac)
        Cp = shiro.partial_c(run.plan, run.Ad.vals, run.B.to(dev), R)
        Bn = run.B.numpy()
        ref = oracle.partial_c(run.Ac, Bn, rs, off)
        den = oracle.partial_c(run.Ac, Bn, rs, off, abs_mode=True)
        assert oracle.rel_err(Cp.cpu().numpy(), ref, den) <= TOL_F32
        # their sum, written over NaNs and added onto ones
        Yr = torch.full((run.Ac.M, run.N), float("nan"), device=dev)
        shiro.aggregate_c(run.plan, Cp, out=Yr)
        assert oracle.rel_err(Yr.cpu().numpy(), Yref, Yden) <= TOL_F32
        Ya = torch.ones(run.Ac.M, run.N, device=dev)
        shiro.aggregate_c(run.plan, Cp, out=Ya, accumulate=True)
        assert torch.equal(Ya, 1.0 + Yr)
    finally:
        for k, t in saved.items():
            shiro.set_tuning(run.plan, k[0], run.N, k[1], **t)


def test_allocator_failure_reports_oom(shiro):
    """An allocator callback that hands out no memory makes plan construction
    fail with SHIRO_ERR_OOM and a message (no launch touches a null buffer),
    and the library works again once hipMalloc is restored."""
    from paper_2512_20178_amd import _lib

    A, N = make_case("rmat12_P8_p0")
    Ad = A.to(torch.device("cuda"))
    alloc = _lib.ALLOC_FN(lambda n, c: None)
    free = _lib.FREE_FN(lambda p, n, c: None)
    assert shiro._L().shiro_set_allocator(alloc, free, None) == 0
    try:
        with pytest.raises(_lib.ShiroError) as e:
            plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
            shiro.select_rows(plan)
        assert e.value.name == "OOM"
        assert "allocator returned NULL" in str(e.value)
    finally:
        shiro.use_torch_allocator(False)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    assert U == len(oracle.select(oracle.Csr.from_synth(A))[0])


def test_backward_walk_builds_bit_exact(shiro, run):
    """The fused float32 transposed walk with one nonzero per step runs from
    the build compiled for eight wavefronts per SIMD (lane groups of 16 or
    more); with two per step it runs from the default build.  Both keep each
    packed column's sum in nonzero order over the same chunks, so dBpacked and
    the value gradients are bit-identical, and within tolerance of the oracle."""
    dev = run.dev
    N = run.N
    dt = torch.float32
    saved = shiro.get_tuning(run.plan, "spmm_t", N, dt)
    Bp = shiro.pack_B(run.plan, run.B.to(dev))
    dY = run.G.to(dev)
    outs = []
    try:
        for unroll in (1, 2):
            shiro.set_tuning(run.plan, "spmm_t", N, dt, chunk=64, lanes=32, unroll=unroll, group_rows=3, lds_rows=0)
            dBp = torch.full((run.U, N), float("nan"), device=dev)
            dvals = torch.zeros(run.A.nnz, device=dev)
            shiro.spmm_backward(run.plan, run.Ad.vals, dY, Bp, dBpacked=dBp, dvals=dvals)
            torch.cuda.synchronize()
            outs.append((dBp, dvals))
    finally:
        shiro.set_tuning(run.plan, "spmm_t", N, dt, **saved)
    for a, b in zip(*outs):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    rdBp, rden, rdv, rdv_den = _bwd_refs(run, run.B.numpy(), run.G.numpy())
    assert oracle.rel_err(outs[0][0].cpu().numpy(), rdBp, rden) <= TOL_F32
    gv = outs[0][1].cpu().numpy()[run.Ac.nz_begin:run.Ac.nz_begin + run.Ac.nnz_panel]
    assert oracle.rel_err(gv, rdv, rdv_den) <= TOL_F32


@pytest.mark.parametrize("H", [1, 5, 64])
def test_lds_rows_bit_exact(shiro, run, H):
    """The windowed walk with its H most referenced gathered rows in LDS
    (knob lds_rows): forward, and backward with dB rows and fused dvals, in
    float32 and bfloat16, bit-identical to the same walk reading every row
    from memory, and within tolerance of the oracle."""
    dev = run.dev
    N = run.N
    dY = run.G.to(dev)
    for dt in (torch.float32, torch.bfloat16):
        saved = {k: shiro.get_tuning(run.plan, k, N, dt) for k in ("spmm", "spmm_t")}
        outs = []
        try:
            for lds in (0, H):
                for k in ("spmm", "spmm_t"):
                    shiro.set_tuning(run.plan, k, N, dt, chunk=64, lanes=32, unroll=2, group_rows=3, lds_rows=lds)
                Bp = shiro.pack_B(run.plan, run.B.to(dt).to(dev))
                Y = shiro.spmm(run.plan, run.Ad.vals, Bp)
                dB = torch.zeros(run.A.n_cols, N, dtype=dt, device=dev)
                dvals = torch.zeros(run.A.nnz, device=dev)
                shiro.spmm_backward(run.plan, run.Ad.vals, dY.to(dt), Bp, dB=dB, dvals=dvals, dB_overwrite=True)
                torch.cuda.synchronize()
                outs.append((Y, dB, dvals))
        finally:
            for k, t in saved.items():
                shiro.set_tuning(run.plan, k, N, dt, **t)
        view = torch.int16 if dt == torch.bfloat16 else torch.int32
        for a, b in zip(*outs):
            assert torch.equal(a.view(view) if a.dtype == dt else a, b.view(view) if b.dtype == dt else b)
        if dt == torch.float32:
            Yref, Yden = _fwd_ref(run, run.B.numpy())
            assert oracle.rel_err(outs[1][0].cpu().numpy(), Yref, Yden) <= TOL_F32
    with pytest.raises(shiro.ShiroError) as e:  # only the windowed walk keeps rows in LDS
        shiro.set_tuning(run.plan, "spmm", N, group_rows=2, lds_rows=4)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(shiro.ShiroError) as e:
        shiro.set_tuning(run.plan, "partial_c", N, group_rows=3, lds_rows=4)
    assert e.value.name == "INVALID_ARG"
    # 128 FP32 rows of a 64-lane tile (1 KB each) would need 128 KB of LDS;
    # 64 of them fit the 64 KB a workgroup may take
    with pytest.raises(shiro.ShiroError) as e:
        shiro.set_tuning(run.plan, "spmm", 256, torch.float32, lanes=64, group_rows=3, lds_rows=128)
    assert e.value.name == "INVALID_ARG" and "64 KB" in str(e.value)
    shiro.set_tuning(run.plan, "spmm", 256, torch.float32, lanes=64, group_rows=3, lds_rows=64)


def test_graph_replays_match_eager(shiro):
    """A captured select+pack+spmm+backward graph, replayed several times with
    eager work in between, gives bit-identical results to the eager calls."""
    A, N = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    shiro.prepare(plan, N, torch.float32, ops=("spmm", "backward"))
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B).to(dev)
    G = synth.dense(plan.info()["rows"], N, 0, synth.STREAM_DY).to(dev)
    Bp = torch.empty(U, N, device=dev)
    Y = torch.empty(plan.info()["rows"], N, device=dev)
    dBp = torch.empty(U, N, device=dev)
    dvals = torch.zeros(A.nnz, device=dev)

    def step():
        shiro.refresh_selection(plan)
        shiro.pack_B(plan, B, out=Bp)
        shiro.spmm(plan, Ad.vals, Bp, out=Y)
        shiro.spmm_backward(plan, Ad.vals, G, Bp, dBpacked=dBp, dvals=dvals)

    inf = plan.info()
    dv_panel = dvals[inf["nz_begin"]:inf["nz_begin"] + inf["nnz"]]  # the entries the panel owns
    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (Bp, Y, dBp, dv_panel)]
    cs = torch.cuda.Stream()
    torch.cuda.synchronize()
    with plan.capture(cs) as holder:
        step()
    gid = holder[0]
    for i in range(4):
        for t in (Bp, Y, dBp, dv_panel):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.replay(gid, stream=cs)
        cs.synchronize()
        for a, b in zip((Bp, Y, dBp, dv_panel), ref):
            assert torch.equal(a, b), f"replay {i}"
        _ = (B * 2).sum().item()  # unrelated eager work between replays
    uc, off, cm = shiro.selection(plan)
    Ac = oracle.Csr.from_synth(A)
    ruc, roff, rcm = oracle.select(Ac)
    assert np.array_equal(uc.cpu().numpy(), ruc) and np.array_equal(cm.cpu().numpy(), rcm)


def test_graph_survives_buffer_growth(shiro):
    """A graph captured at N = 32 keeps its carry and scratch buffers when a
    later eager call at N = 256 (and a new tuning with smaller chunks) needs
    larger ones: its replays still match the eager N = 32 result bit for
    bit, and the eager N = 256 call matches the oracle."""
    A, _ = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    rows = plan.info()["rows"]
    shiro.prepare(plan, 32, torch.float32, ops=("spmm", "backward"))
    B32 = synth.dense(A.n_cols, 32, 0, synth.STREAM_B).to(dev)
    G32 = synth.dense(rows, 32, 0, synth.STREAM_DY).to(dev)
    Bp = torch.empty(U, 32, device=dev)
    Y = torch.empty(rows, 32, device=dev)
    dBp = torch.empty(U, 32, device=dev)

    def step():
        shiro.refresh_selection(plan)
        shiro.pack_B(plan, B32, out=Bp)
        shiro.spmm(plan, Ad.vals, Bp, out=Y)
        shiro.spmm_backward(plan, Ad.vals, G32, Bp, dBpacked=dBp)

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (Bp, Y, dBp)]
    cs = torch.cuda.Stream()
    torch.cuda.synchronize()
    with plan.capture(cs) as holder:
        step()
    gid = holder[0]
    # eager calls that grow the carry buffer (wider N, then smaller chunks)
    B256 = synth.dense(A.n_cols, 256, 0, synth.STREAM_B).to(dev)
    Bp256 = shiro.pack_B(plan, B256)
    Y256 = shiro.spmm(plan, Ad.vals, Bp256)
    shiro.set_tuning(plan, "spmm", 256, chunk=16)
    Y256b = shiro.spmm(plan, Ad.vals, Bp256)
    torch.cuda.synchronize()
    Ac = oracle.Csr.from_synth(A)
    Bh = B256.cpu().numpy()
    ref256, den256 = oracle.spmm(Ac, Bh, None), oracle.spmm(Ac, Bh, None, abs_mode=True)
    assert oracle.rel_err(Y256.cpu().numpy(), ref256, den256) <= TOL_F32
    assert oracle.rel_err(Y256b.cpu().numpy(), ref256, den256) <= TOL_F32
    for i in range(3):
        for t in (Bp, Y, dBp):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.replay(gid, stream=cs)
        cs.synchronize()
        for a, b in zip((Bp, Y, dBp), ref):
            assert torch.equal(a, b), f"replay {i}"
        _ = shiro.spmm(plan, Ad.vals, Bp256)  # eager work on the grown buffers between replays
        torch.cuda.synchronize()


def test_autograd_function(shiro):
    A, N = make_case("rmat11_P7_p6_ragged")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    shiro.select_rows(plan)
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B).to(dev).requires_grad_(True)
    vals = Ad.vals.clone().requires_grad_(True)
    Y = shiro.shiro_spmm(plan, vals, B)
    G = synth.dense(Y.shape[0], N, 0, synth.STREAM_DY).to(dev)
    (Y * G).sum().backward()
    Ac = oracle.Csr.from_synth(A)
    Gn, Bn = G.cpu().numpy(), B.detach().cpu().numpy()
    dB = oracle.spmm_t(Ac, Gn, None)
    den = oracle.spmm_t(Ac, Gn, None, abs_mode=True)
    assert oracle.rel_err(B.grad.cpu().numpy(), dB, den) <= TOL_F32
    dv = np.zeros(A.nnz)
    dvd = np.zeros(A.nnz)
    dv[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel] = oracle.sddmm(Ac, Gn, Bn, None)
    dvd[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel] = oracle.sddmm(Ac, Gn, Bn, None, abs_mode=True)
    assert oracle.rel_err(vals.grad.cpu().numpy(), dv, dvd) <= TOL_F32


def test_autotune_then_correct(shiro, monkeypatch, tmp_path):
    monkeypatch.setenv("SHIRO_TUNE_CACHE", str(tmp_path / "tune.txt"))  # time every candidate here
    A, N = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    shiro.select_rows(plan)
    shiro.autotune(plan, N, torch.float32, ops=("spmm", "backward"))
    for k in ("spmm", "spmm_t", "sddmm"):
        t = shiro.get_tuning(plan, k, N)
        assert t["lanes"] in (8, 16, 32, 64) and t["unroll"] in (1, 2, 4)
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B).to(dev)
    Y = shiro.spmm(plan, Ad.vals, shiro.pack_B(plan, B))
    Ac = oracle.Csr.from_synth(A)
    Yref = oracle.spmm(Ac, B.cpu().numpy(), None)
    den = oracle.spmm(Ac, B.cpu().numpy(), None, abs_mode=True)
    assert oracle.rel_err(Y.cpu().numpy(), Yref, den) <= TOL_F32
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(lines) == 3 and all(ln.split()[0].endswith(("|k=0", "|k=1", "|k=2")) for ln in lines)
    # the row-based scheme's two kernels
    shiro.autotune(plan, N, torch.float32, ops=("row_based",))
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(lines) == 5 and lines[3].split()[0].endswith("|k=3") and lines[4].split()[0].endswith("|k=4")
    R, _ = shiro.select_c_rows(plan)
    Yr = shiro.aggregate_c(plan, shiro.partial_c(plan, Ad.vals, B, R))
    assert oracle.rel_err(Yr.cpu().numpy(), Yref, den) <= TOL_F32


# ----------------------------------------------------------------------------
# row-based scheme: Rows(A^(p,q)), partial C rows, their sum into the panel
# ----------------------------------------------------------------------------
def test_c_rows_bit_exact(shiro, run):
    R, per = shiro.select_c_rows(run.plan)
    rs, off = oracle.select_c_rows(run.Ac)
    assert R == len(rs) and per == list(np.diff(off))
    grs, goff = shiro.c_row_selection(run.plan, R)
    assert np.array_equal(grs.cpu().numpy(), rs)
    assert np.array_equal(goff.cpu().numpy(), off)


def test_partial_and_aggregate_f32(shiro, run):
    R, _ = shiro.select_c_rows(run.plan)
    rs, off = oracle.select_c_rows(run.Ac)
    B = run.B.to(run.dev)
    Cp = shiro.partial_c(run.plan, run.Ad.vals, B, R)
    Bn = run.B.numpy()
    ref = oracle.partial_c(run.Ac, Bn, rs, off)
    den = oracle.partial_c(run.Ac, Bn, rs, off, abs_mode=True)
    assert oracle.rel_err(Cp.cpu().numpy(), ref, den) <= TOL_F32
    Y = shiro.aggregate_c(run.plan, Cp)
    Yref, Yden = _fwd_ref(run, Bn)
    assert oracle.rel_err(Y.cpu().numpy(), Yref, Yden) <= TOL_F32
    # the sum on its own, on seeded partial rows (integers: exact in any order)
    rng = np.random.default_rng(3)
    Cx = rng.integers(-4, 5, size=(R, run.N)).astype(np.float32)
    Yx = shiro.aggregate_c(run.plan, torch.from_numpy(Cx).to(run.dev))
    assert np.array_equal(Yx.cpu().numpy(), oracle.aggregate_c(run.Ac, Cx, rs, off))
    # reproducible
    assert torch.equal(shiro.partial_c(run.plan, run.Ad.vals, B, R), Cp)


def test_partial_and_aggregate_bf16(shiro, run):
    R, _ = shiro.select_c_rows(run.plan)
    rs, off = oracle.select_c_rows(run.Ac)
    Bh = run.B.to(torch.bfloat16).to(run.dev)
    Bn = run.B.numpy()
    Yref, Yden = _fwd_ref(run, Bn)
    for mid in (torch.bfloat16, torch.float32):
        Cp = shiro.partial_c(run.plan, run.Ad.vals, Bh, R, out_dtype=mid)
        ref = oracle.partial_c(run.Ac, Bn, rs, off)
        den = oracle.partial_c(run.Ac, Bn, rs, off, abs_mode=True)
        assert oracle.rel_err(bf16_to_f32(Cp), ref, den) <= TOL_BF16
        for out_dtype in ((torch.bfloat16, torch.float32) if mid == torch.bfloat16 else (torch.float32,)):
            Y = shiro.aggregate_c(run.plan, Cp, out_dtype=out_dtype)
            assert oracle.rel_err(bf16_to_f32(Y), Yref, Yden) <= TOL_BF16


def test_row_based_graph_replays(shiro, run):
    R, _ = shiro.select_c_rows(run.plan)
    shiro.prepare(run.plan, run.N, torch.float32, ops=("row_based",))
    B = run.B.to(run.dev)
    Cp = torch.empty(R, run.N, device=run.dev)
    Y = torch.empty(run.Ac.M, run.N, device=run.dev)
    ref = shiro.aggregate_c(run.plan, shiro.partial_c(run.plan, run.Ad.vals, B, R))
    cs = torch.cuda.Stream()
    torch.cuda.synchronize()
    with run.plan.capture(cs) as gid:
        shiro.partial_c(run.plan, run.Ad.vals, B, R, out=Cp, stream=cs)
        shiro.aggregate_c(run.plan, Cp, out=Y, stream=cs)
    for _ in range(3):
        Y.fill_(float("nan"))
        torch.cuda.synchronize()
        run.plan.replay(gid[0], stream=cs)
        cs.synchronize()
        assert torch.equal(Y, ref)


# ----------------------------------------------------------------------------
# joint row-column strategy: per-block minimum covers, subset plans, forward
# ----------------------------------------------------------------------------
def _assign_cover(Ac, assign, q):
    """(rows sent row-based, columns fetched column-based) of block q under an assignment."""
    nz0, n = Ac.nz_begin, Ac.nnz_panel
    rows = np.repeat(np.arange(Ac.M), np.diff(Ac.row_ptr[Ac.row_begin:Ac.row_end + 1]))
    cols = Ac.col[nz0:nz0 + n]
    m = (cols // Ac.K) == q
    a = assign[m]
    return set(rows[m][a == 1].tolist()), set(cols[m][a == 0].tolist())


@pytest.mark.parametrize("weighted", [False, True])
def test_joint_plan_matches_oracle(shiro, run, weighted):
    rng = np.random.default_rng(8)
    w_row = rng.integers(1, 6, run.Ac.M) if weighted else None
    w_col = rng.integers(1, 6, run.A.n_cols) if weighted else None
    assign, stats = shiro.joint_plan(run.plan, w_row, w_col)
    assign, stats = assign.numpy(), stats.numpy()
    ref = oracle.joint_cover(run.Ac, w_row, w_col)
    rs, roff = oracle.select_c_rows(run.Ac)
    for q in range(run.A.P):
        assert stats[q, 1] == roff[q + 1] - roff[q] and stats[q, 2] == run.off[q + 1] - run.off[q]
        rows, cols = _assign_cover(run.Ac, assign, q)
        if ref[q] is None:  # the diagonal block stays column-based
            assert stats[q, 0] == 0 and not rows
            continue
        mu = ref[q][0]
        assert stats[q, 0] == mu
        wr = np.ones(run.Ac.M, np.int64) if w_row is None else w_row
        wc = np.ones(run.A.n_cols, np.int64) if w_col is None else w_col
        # the assignment realises a cover of the optimal cost
        assert sum(int(wr[i]) for i in rows) + sum(int(wc[j]) for j in cols) <= mu
        assert stats[q, 3] == len(rows)


def test_joint_plan_fig1(shiro):
    g = load_golden("fig1_block01.txt")
    n, P, p = g["n"][0][0], g["P"][0][0], g["p"][0][0]
    mask = np.zeros((n, n))
    for r, c, v in g["nz"]:
        mask[r, c] = v
    A = synth.from_dense_pattern(mask, P=P, p=p)
    Ad = A.to(torch.device("cuda"))
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    assign, stats = shiro.joint_plan(plan)
    (q, mu), = g["expect_joint_cover_block"]
    assert int(stats[q, 0]) == mu
    # b, c, d (row 0) go row-based; f, h are covered by fetching b_6
    assert assign.tolist() == [1, 1, 1, 0, 0]


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_joint_forward(shiro, run, dtype):
    A = run.A
    js = shiro.JointSpMM(run.Ad.row_ptr, run.Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    assert js.U + js.R >= int(js.stats[:, 0].sum())  # volumes before and after planning
    js.prepare(run.N, dtype)
    B = run.B.to(dtype).to(run.dev)
    Y = js.forward(run.Ad.vals, B)
    Yref, den = _fwd_ref(run, run.B.numpy())
    tol = TOL_F32 if dtype == torch.float32 else TOL_BF16
    assert oracle.rel_err(bf16_to_f32(Y), Yref, den) <= tol
    if dtype == torch.float32:
        assert torch.equal(js.forward(run.Ad.vals, B), Y)  # reproducible


def test_joint_backward_and_autograd(shiro, run):
    A, Ac = run.A, run.Ac
    js = shiro.JointSpMM(run.Ad.row_ptr, run.Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    B = run.B.to(run.dev)
    dY = run.G.to(run.dev)
    dB, dvals = js.backward(run.Ad.vals, B, dY)
    rdB = oracle.spmm_t(Ac, run.G.numpy(), None)
    rden = oracle.spmm_t(Ac, run.G.numpy(), None, abs_mode=True)
    assert oracle.rel_err(dB.cpu().numpy(), rdB, np.maximum(rden, 0)) <= TOL_F32
    nz0 = Ac.nz_begin
    rdv = oracle.sddmm(Ac, run.G.numpy(), run.B.numpy(), None)
    rdvd = oracle.sddmm(Ac, run.G.numpy(), run.B.numpy(), None, abs_mode=True)
    assert oracle.rel_err(dvals.cpu().numpy()[nz0:nz0 + Ac.nnz_panel], rdv, rdvd) <= TOL_F32
    # through autograd: the same gradients
    vp = run.Ad.vals.clone().requires_grad_(True)
    Bg = B.clone().requires_grad_(True)
    Y = shiro.JointSpMMFunction.apply(vp, Bg, js)
    Y.backward(dY)
    assert torch.equal(Bg.grad, dB) and torch.equal(vp.grad, dvals)


def test_subset_plan_backward(shiro, run):
    """A column-based subset plan: A_col^T dY and dvals through the value map."""
    A, Ac = run.A, run.Ac
    js = shiro.JointSpMM(run.Ad.row_ptr, run.Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    keep = js.assign.numpy() == 0
    nz0 = Ac.nz_begin
    # host CSR of the column-based part: the panel's kept nonzeros, other rows empty
    rows = np.repeat(np.arange(Ac.M), np.diff(Ac.row_ptr[Ac.row_begin:Ac.row_end + 1]))[keep]
    counts = np.zeros(Ac.n_rows, np.int64)
    counts[Ac.row_begin:Ac.row_end] = np.bincount(rows, minlength=Ac.M)
    rp = np.concatenate([[0], np.cumsum(counts)])
    Acol = oracle.Csr(Ac.n_rows, Ac.n_cols, rp, Ac.col[nz0:nz0 + Ac.nnz_panel][keep],
                      Ac.vals[nz0:nz0 + Ac.nnz_panel][keep], Ac.P, Ac.p)
    uc, off, cm = oracle.select(Acol)
    assert js.U == len(uc)
    Bp = shiro.pack_B(js.col_plan, run.B.to(run.dev))
    dY = run.G.to(run.dev)
    dBp = torch.empty(js.U, run.N, device=run.dev)
    dvals = torch.full((A.nnz,), -5.0, device=run.dev)
    shiro.spmm_backward(js.col_plan, run.Ad.vals, dY, Bp, dBpacked=dBp, dvals=dvals)
    ref = oracle.spmm_t(Acol, run.G.numpy(), cm, n_out=len(uc))
    rden = oracle.spmm_t(Acol, run.G.numpy(), cm, n_out=len(uc), abs_mode=True)
    assert oracle.rel_err(dBp.cpu().numpy(), ref, rden) <= TOL_F32
    dv = dvals.cpu().numpy()[nz0:nz0 + Ac.nnz_panel]
    full = oracle.sddmm(Ac, run.G.numpy(), run.B.numpy(), None)
    fden = oracle.sddmm(Ac, run.G.numpy(), run.B.numpy(), None, abs_mode=True)
    assert oracle.rel_err(dv[keep], full[keep], fden[keep]) <= TOL_F32
    assert bool((dv[~keep] == -5.0).all())  # the row-based nonzeros are not touched


def test_lds_rows_setup_failure_frees_its_buffers(shiro):
    """When the LDS-row setup cannot get its second buffer, the call reports
    OOM, hands back the buffer it already had, and a later prepare with a
    working allocator builds the rows (results bit-identical to no LDS rows)."""
    from paper_2512_20178_amd import _lib

    A, N = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    shiro.select_rows(plan)
    base = {"chunk": 64, "lanes": 32, "unroll": 2, "group_rows": 3, "lds_rows": 0}
    shiro.set_tuning(plan, "spmm", N, torch.float32, **base)
    shiro.prepare(plan, N, torch.float32, ops=("spmm",))
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B, device=dev)
    Bp = shiro.pack_B(plan, B)
    Y0 = shiro.spmm(plan, Ad.vals, Bp)
    torch.cuda.synchronize()
    live = {}

    def _alloc(nbytes, ctx):
        if nbytes <= 4096:  # the hot-row slot list (a few bytes) is refused
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(ptr, nbytes, ctx):
        live.pop(ptr)

    hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    shiro.set_tuning(plan, "spmm", N, torch.float32, **dict(base, lds_rows=16))
    assert shiro._L().shiro_set_allocator(hooks[0], hooks[1], None) == 0
    try:
        with pytest.raises(_lib.ShiroError) as e:
            shiro.prepare(plan, N, torch.float32, ops=("spmm",))
        assert e.value.name == "OOM"
        assert not live, "the index copy was not handed back"
    finally:
        shiro.use_torch_allocator(False)
    shiro.prepare(plan, N, torch.float32, ops=("spmm",))
    Y1 = shiro.spmm(plan, Ad.vals, Bp)
    torch.cuda.synchronize()
    assert torch.equal(Y1.view(torch.int32), Y0.view(torch.int32))


def test_torch_allocator(shiro):
    """Plan memory from torch's caching allocator: accounted by torch while the
    plan lives, returned when it is destroyed, results unchanged."""
    A, N = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B).to(dev)
    G = None
    Ac = oracle.Csr.from_synth(A)
    # tensors of earlier tests that are only cyclic garbage would otherwise be
    # freed in the middle of this test and move the baseline
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    shiro.use_torch_allocator(True)
    try:
        plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
        U, _ = shiro.select_rows(plan)
        shiro.prepare(plan, N, torch.float32, ops=("spmm", "backward"))
        held = torch.cuda.memory_allocated() - base
        assert held >= 4 * Ac.nnz_panel  # at least the panel's column copy
        Bp = shiro.pack_B(plan, B)
        Y = shiro.spmm(plan, Ad.vals, Bp)
        Yref = oracle.spmm(Ac, B.cpu().numpy(), None)
        den = oracle.spmm(Ac, B.cpu().numpy(), None, abs_mode=True)
        assert oracle.rel_err(Y.cpu().numpy(), Yref, den) <= TOL_F32
        G = synth.dense(Ac.M, N, 0, synth.STREAM_DY).to(dev)
        dBp = torch.empty(U, N, device=dev)
        dvals = torch.zeros(A.nnz, device=dev)
        shiro.spmm_backward(plan, Ad.vals, G, Bp, dBpacked=dBp, dvals=dvals)
        uc, off, cm = oracle.select(Ac)
        ref = oracle.spmm_t(Ac, G.cpu().numpy(), cm, n_out=len(uc))
        rden = oracle.spmm_t(Ac, G.cpu().numpy(), cm, n_out=len(uc), abs_mode=True)
        assert oracle.rel_err(dBp.cpu().numpy(), ref, rden) <= TOL_F32
        plan.close()
        del Bp, Y, G, dBp, dvals
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        shiro.use_torch_allocator(False)


def test_error_paths_on_device(shiro):
    dev = torch.device("cuda")
    # malformed CSR caught by the check mode
    rp = torch.tensor([0, 2, 1, 3], dtype=torch.int64, device=dev)
    col = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    with pytest.raises(shiro.ShiroError) as e:
        shiro.partition(rp, col, 3, 3, 1, 0, check=True)
    assert e.value.name == "BAD_CSR"
    rp = torch.tensor([0, 2, 3], dtype=torch.int64, device=dev)
    col = torch.tensor([1, 1, 0], dtype=torch.int32, device=dev)  # repeated column in row 0
    with pytest.raises(shiro.ShiroError) as e:
        shiro.partition(rp, col, 2, 3, 1, 0, check=True)
    assert e.value.name == "BAD_CSR"
    col = torch.tensor([0, 1, 7], dtype=torch.int32, device=dev)  # column out of range
    with pytest.raises(shiro.ShiroError) as e:
        shiro.partition(rp, col, 2, 3, 1, 0, check=True)
    assert e.value.name == "BAD_CSR"
    # call order
    col = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    plan = shiro.partition(rp, col, 2, 3, 1, 0, check=True)
    B = torch.zeros(3, 4, device=dev)
    with pytest.raises(shiro.ShiroError) as e:
        shiro.pack_B(plan, B, out=torch.zeros(3, 4, device=dev))
    assert e.value.name == "NOT_READY"
    shiro.select_rows(plan)
    with pytest.raises(shiro.ShiroError) as e:  # float32 input with bfloat16 output
        shiro.spmm(plan, torch.ones(3, device=dev), torch.zeros(3, 4, device=dev), out_dtype=torch.bfloat16)
    assert e.value.name == "UNSUPPORTED"
    with pytest.raises(shiro.ShiroError) as e:
        shiro.set_tuning(plan, "spmm", 4, lanes=12)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(shiro.ShiroError) as e:  # the sampled product has no nonzero walk
        shiro.set_tuning(plan, "sddmm", 4, group_rows=2)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(shiro.ShiroError) as e:
        shiro.set_tuning(plan, "sddmm", 4, group_rows=3)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(shiro.ShiroError) as e:
        shiro.set_tuning(plan, "spmm_t", 4, group_rows=4)
    assert e.value.name == "INVALID_ARG"


def test_binding_rejects_bad_operands(shiro):
    """The binding checks device, dtype and shape of every tensor against the
    plan before a pointer reaches the library: undersized or host tensors
    raise, and the outputs are left untouched (nothing was launched)."""
    A, N = make_case("rmat12_P8_p0")
    dev = torch.device("cuda")
    Ad = A.to(dev)
    plan = shiro.partition(Ad.row_ptr, Ad.col, A.n_rows, A.n_cols, A.P, A.p)
    U, _ = shiro.select_rows(plan)
    inf = plan.info()
    rows, ext = inf["rows"], inf["nz_begin"] + inf["nnz"]
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B).to(dev)
    Bp = shiro.pack_B(plan, B)
    G = synth.dense(rows, N, 0, synth.STREAM_DY).to(dev)
    sentinel = 3.0
    Y = torch.full((rows, N), sentinel, device=dev)
    bad = [
        lambda: shiro.pack_B(plan, B[: A.n_cols - 1]),                      # B short of n_cols rows
        lambda: shiro.pack_B(plan, B, out=torch.empty(U - 1, N, device=dev)),  # Bpacked short of U rows
        lambda: shiro.spmm(plan, Ad.vals[: ext - 1], Bp, out=Y),             # vals short of the panel
        lambda: shiro.spmm(plan, Ad.vals.cpu(), Bp, out=Y),                  # vals on the host
        lambda: shiro.spmm(plan, Ad.vals.double(), Bp, out=Y),               # vals not float32
        lambda: shiro.spmm(plan, Ad.vals, Bp[: U - 1], out=Y),               # Bpacked short of U rows
        lambda: shiro.spmm(plan, Ad.vals, Bp, out=Y[: rows - 1]),            # Y short of the panel rows
        lambda: shiro.spmm(plan, Ad.vals, Bp, out=Y.cpu()),                  # Y on the host
        lambda: shiro.spmm(plan, Ad.vals, Bp, out=torch.empty(rows, N + 1, device=dev)),
        lambda: shiro.spmm_noalloc(plan, Ad.vals, Bp, Y[: rows - 1]),
        lambda: shiro.spmm_backward(plan, Ad.vals, G[: rows - 1], Bp, dB=torch.zeros(A.n_cols, N, device=dev)),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, Bp, dB=torch.zeros(A.n_cols - 1, N, device=dev)),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, Bp, dBpacked=torch.zeros(U - 1, N, device=dev)),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, Bp, dvals=torch.zeros(ext - 1, device=dev)),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, Bp, dvals=torch.zeros(ext, device="cpu")),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, None, dvals=torch.zeros(ext, device=dev)),
        lambda: shiro.spmm_backward(plan, Ad.vals, G, Bp.to(torch.bfloat16), dB=torch.zeros(A.n_cols, N, device=dev)),
    ]
    for i, f in enumerate(bad):
        with pytest.raises((ValueError, TypeError)):
            f()
        torch.cuda.synchronize()
        assert bool((Y == sentinel).all()), f"case {i} wrote Y"
    # the same calls with correct operands still work
    shiro.spmm(plan, Ad.vals, Bp, out=Y)
    Ac = oracle.Csr.from_synth(A)
    Bh = B.cpu().numpy()
    assert oracle.rel_err(Y.cpu().numpy(), oracle.spmm(Ac, Bh, None), oracle.spmm(Ac, Bh, None, abs_mode=True)) <= TOL_F32
