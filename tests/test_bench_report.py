"""CPU tests of the benchmark's per-output error report (the `precision`
fields of its JSON line): fed the oracle's own outputs it reports errors at
rounding level, and a planted error in one output of Y, dB or dvals shows up
in that output's figure at the planted size."""
import numpy as np
import pytest
import torch

import bench
import oracle
import synth


@pytest.fixture(scope="module")
def case():
    A = synth.small_rmat(10, 8, P=4, p=1, vals_lo=-1.0)
    N = 16
    Ac = oracle.Csr.from_synth(A)
    B = synth.dense(A.n_cols, N, 0, synth.STREAM_B)
    G = synth.dense(Ac.M, N, 0, synth.STREAM_DY)
    Y = oracle.spmm(Ac, B.numpy(), None)
    dB = oracle.spmm_t(Ac, G.numpy(), None)
    dv = np.zeros(A.nnz)
    dv[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel] = oracle.sddmm(Ac, G.numpy(), B.numpy(), None)
    smp = bench.sample_outputs(A, {"row_begin": Ac.row_begin, "rows": Ac.M}, np, torch)
    return A, Ac, B, G, Y, dB, dv, smp


def _report(case, Y, dB, dv):
    A, Ac, B, G, _, _, _, smp = case
    out = bench.take_samples(smp, torch.from_numpy(Y).float(), torch.from_numpy(dB).float(),
                             torch.from_numpy(dv).float())
    return bench.precision_report(A, B, G, smp, {torch.float32: out})["f32"]


def test_exact_outputs_report_rounding_error(case):
    _, _, _, _, Y, dB, dv, smp = case
    assert len(smp["rows"]) > 8 and len(smp["cols"]) > 8 and len(smp["ks"]) > 8
    rep = _report(case, Y, dB, dv)
    for k in ("Y", "dB", "dvals"):
        assert rep[k] <= 2 ** -24, (k, rep[k])  # float32 rounding of the oracle's values


def test_planted_errors_are_reported(case):
    A, Ac, B, G, Y, dB, dv, smp = case
    r = int(smp["rows"][3])
    c = int(smp["cols"][2])
    k = int(smp["ks"][5])
    # relative to the metric's denominators: |A||B| for Y, |A|^T|dY| for dB,
    # sum_j |dY||B| for dvals
    yden = oracle.spmm(Ac, B.numpy(), None, abs_mode=True)
    dbden = oracle.spmm_t(Ac, G.numpy(), None, abs_mode=True)
    dvden = np.zeros(A.nnz)
    dvden[Ac.nz_begin:Ac.nz_begin + Ac.nnz_panel] = oracle.sddmm(Ac, G.numpy(), B.numpy(), None, abs_mode=True)
    j = int(np.argmax(yden[r]))
    Yp = Y.copy()
    Yp[r, j] += 1e-3 * yden[r, j]
    rep = _report(case, Yp, dB, dv)
    assert rep["Y"] == pytest.approx(1e-3, rel=1e-3) and rep["dB"] <= 2 ** -24 and rep["dvals"] <= 2 ** -24
    jb = int(np.argmax(dbden[c]))
    dBp = dB.copy()
    dBp[c, jb] -= 3e-4 * dbden[c, jb]
    rep = _report(case, Y, dBp, dv)
    assert rep["dB"] == pytest.approx(3e-4, rel=1e-3) and rep["Y"] <= 2 ** -24
    dvp = dv.copy()
    dvp[k] += 2e-3 * dvden[k]
    rep = _report(case, Y, dB, dvp)
    assert rep["dvals"] == pytest.approx(2e-3, rel=1e-3) and rep["Y"] <= 2 ** -24
