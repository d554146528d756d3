"""Host-side checks of the C-ABI library (no GPU needed, no compute calls).

The library must load, export every function include/shiro.h declares, and
reject bad arguments with the documented status codes before touching HIP.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shiro.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"SHIRO_API\s+[\w\s\*]+?\b(shiro_\w+)\s*\(", text)


@pytest.fixture(scope="module")
def lib():
    from paper_2512_20178_amd import _lib

    return _lib.load()


def test_header_declares_the_path_calls():
    names = set(declared_functions())
    for n in ("shiro_partition", "shiro_select_rows", "shiro_pack_B", "shiro_spmm", "shiro_spmm_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2512_20178_amd import _lib

    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (shiro_\w+)", out))
    assert set(names) == exported  # nothing else is exported


def test_library_is_built_for_gfx950():
    from paper_2512_20178_amd import _lib

    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_library_stamp_matches_the_sources(lib):
    """The library in the tree was built from the sources in the tree."""
    from paper_2512_20178_amd import _lib, build

    assert len(build.source_hash()) == 16
    assert _lib.build_hash() == build.source_hash()
    assert _lib.check_build(strict=False)


def test_version(lib):
    assert lib.shiro_version() == 10000


def _err(lib):
    return lib.shiro_last_error().decode()


def test_partition_argument_errors(lib):
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        ((10, 10, 0, fake, None, 1, 0, 0, None, None), "out_plan"),
        ((0, 10, 0, fake, None, 1, 0, 0, None, ctypes.byref(h)), "n_rows"),
        ((10, 0, 0, fake, None, 1, 0, 0, None, ctypes.byref(h)), "n_cols"),
        ((1 << 31, 10, 0, fake, None, 1, 0, 0, None, ctypes.byref(h)), "n_rows"),
        ((10, 10, -1, fake, None, 1, 0, 0, None, ctypes.byref(h)), "nnz"),
        ((10, 10, 0, None, None, 1, 0, 0, None, ctypes.byref(h)), "d_row_ptr"),
        ((10, 10, 5, fake, None, 1, 0, 0, None, ctypes.byref(h)), "d_col"),
        ((10, 10, 0, fake, None, 0, 0, 0, None, ctypes.byref(h)), "P < 1"),
        ((10, 10, 0, fake, None, 4, 4, 0, None, ctypes.byref(h)), "p outside"),
        ((10, 10, 0, fake, None, 4, -1, 0, None, ctypes.byref(h)), "p outside"),
    ]
    for args, frag in cases:
        assert lib.shiro_partition(*args) == -1
        assert frag in _err(lib)


def test_null_plan_errors(lib):
    P = ctypes.c_void_p(None)
    assert lib.shiro_select_rows(P, None, None, None) == -1
    assert lib.shiro_pack_B(P, None, 0, 0, 0, None, 0, None) == -1
    assert lib.shiro_spmm(P, None, None, 0, 0, 0, None, 0, 0, 0, None) == -1
    assert lib.shiro_spmm_backward(P, None, None, 0, None, 0, 0, 0, None, 0, None, 0, None, 0, None) == -1
    assert lib.shiro_prepare(P, 1, 0, 1, None) == -1
    assert lib.shiro_autotune(P, 1, 0, 1, None) == -1
    assert lib.shiro_plan_info(P, None) == -1
    assert lib.shiro_copy_selection(P, None, None, None, None) == -1
    assert lib.shiro_graph_launch(P, 0, None) == -1
    assert lib.shiro_plan_destroy(P) == 0  # NULL is accepted


def test_tuning_validation(lib):
    from paper_2512_20178_amd import _lib

    t = _lib.Tuning(chunk=256, lanes=64, unroll=2, group_rows=0, xcd_remap=0, wg_per_cu=8)
    assert lib.shiro_set_tuning(ctypes.c_void_p(None), 0, 128, 0, ctypes.byref(t)) == -1


def test_set_allocator_arguments(lib):
    from paper_2512_20178_amd import _lib

    keep = _lib.ALLOC_FN(lambda n, c: None)
    assert lib.shiro_set_allocator(keep, _lib.FREE_FN(), None) == -1
    assert "both" in _err(lib)
    assert lib.shiro_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None) == 0  # back to hipMalloc


@pytest.mark.parametrize("seed", range(10))
def test_mvc_bipartite_matches_oracle(seed):
    """The library's host max-flow cover against the oracle's (same minimum
    cost; the returned set must be a cover of exactly that cost)."""
    import numpy as np

    import oracle
    import paper_2512_20178_amd as shiro

    rng = np.random.default_rng(100 + seed)
    nl, nr = int(rng.integers(1, 300)), int(rng.integers(1, 300))
    mask = rng.random((nl, nr)) < rng.uniform(0.002, 0.05)
    if seed == 0:
        mask[:] = False  # no edges: empty cover
    edges = np.argwhere(mask)
    weighted = seed % 3 == 2
    wl = rng.integers(0, 20, nl) if weighted else None
    wr = rng.integers(0, 20, nr) if weighted else None
    mu, cl, cr = shiro.mvc_bipartite(nl, nr, edges[:, 0], edges[:, 1], wl, wr)
    ref, _, _ = oracle.mvc_bipartite(nl, nr, edges, wl, wr)
    assert mu == ref
    cl, cr = cl.numpy(), cr.numpy()
    assert all(cl[i] or cr[j] for i, j in edges)
    wlv = np.ones(nl, np.int64) if wl is None else wl
    wrv = np.ones(nr, np.int64) if wr is None else wr
    assert mu == int(wlv[cl].sum() + wrv[cr].sum())


def test_mvc_bipartite_argument_errors(lib):
    import ctypes as c

    w = c.c_int64()
    left = (c.c_int32 * 1)(5)
    right = (c.c_int32 * 1)(0)
    cl = (c.c_uint8 * 2)()
    cr = (c.c_uint8 * 2)()
    assert lib.shiro_mvc_bipartite(2, 2, 1, left, right, None, None, cl, cr, c.byref(w)) == -1
    assert "out of range" in _err(lib)
    neg = (c.c_int64 * 2)(1, -1)
    left[0] = 1
    assert lib.shiro_mvc_bipartite(2, 2, 1, left, right, neg, None, cl, cr, c.byref(w)) == -1
    assert "negative" in _err(lib)
    assert lib.shiro_mvc_bipartite(-1, 2, 0, None, None, None, None, cl, cr, c.byref(w)) == -1


class _FakePlan:
    """Stands in for a Plan in binding checks that never reach the library."""

    def __init__(self, **info):
        base = dict(n_rows=8, n_cols=8, P=1, p=0, M=8, K=8, row_begin=0, rows=8, nz_begin=0, nnz=10, U=5)
        base.update(info)
        self._info = base
        self.value_extent = base["nz_begin"] + base["nnz"]
        self.R = None
        self.handle = ctypes.c_void_p(0)
        self.rows = base["rows"]

    def info(self):
        return dict(self._info)


def test_binding_rejects_host_operands_before_any_call():
    """CPU tensors never become device pointers: every compute wrapper
    raises before it calls into the library (the fake plan's NULL handle
    would fail any library call with INVALID_ARG instead)."""
    import torch

    import paper_2512_20178_amd as shiro

    plan = _FakePlan()
    B = torch.zeros(8, 4)
    vals = torch.zeros(10)
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.pack_B(plan, B)
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.spmm(plan, vals, torch.zeros(5, 4))
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.spmm_noalloc(plan, vals, torch.zeros(5, 4), torch.zeros(8, 4))
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.spmm_backward(plan, vals, torch.zeros(8, 4), torch.zeros(5, 4), dB=torch.zeros(8, 4))
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.partial_c(plan, vals, B, 3)
    with pytest.raises(ValueError, match="on the GPU"):
        shiro.aggregate_c(plan, torch.zeros(3, 4))
