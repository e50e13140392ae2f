"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/merbit.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def _declared():
    with open(os.path.join(ROOT, "include", "merbit.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(merbit_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("merbit_plan_create", "merbit_spmv", "merbit_pagerank",
                     "merbit_plan_destroy", "merbit_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2605_07391_amd as pkg
    lib = pkg.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(pkg.EXPORTED)
    assert "gfx950" in pkg.version()


def test_argument_errors_without_gpu():
    import paper_2605_07391_amd.merbit as mb
    lib = mb.load()
    out = ctypes.c_void_p()
    vp = ctypes.c_void_p

    def opts(**kw):
        o = mb.Opts()
        lib.merbit_opts_init(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return ctypes.byref(o)

    d = mb.Opts()
    lib.merbit_opts_init(ctypes.byref(d))
    assert (d.sigma, d.block_lanes, d.commit, d.hot_columns, d.validate,
            d.eager_loops, d.desc_bits, d.stripes) == (0, 0, 0, -1, 1, 0, 0, 0)
    # NULL out pointer
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, None, None, None) == mb.EINVAL
    # unsupported dtype
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 7, None, None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    # sigma 13 does not fit a 32-bit descriptor at omega = 64
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(sigma=13), None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    assert b"sigma" in lib.merbit_last_error()
    # size limit n_rows + nnz < 2^31
    assert lib.merbit_plan_create(1 << 30, 1, 1 << 30, vp(8), vp(8), vp(8), 0, None, None,
                                  ctypes.byref(out)) == mb.EINVAL
    # block size not built
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(block_lanes=192), None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    # commit mode out of range; the wave kernel has no 128-lane build
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(commit=7), None,
                                  ctypes.byref(out)) == mb.EINVAL
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0,
                                  opts(commit=2, block_lanes=128), None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    # descriptor width: only 32 or 64; 64 bits need the wave kernel and a built sigma
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(desc_bits=48), None,
                                  ctypes.byref(out)) == mb.EINVAL
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0,
                                  opts(desc_bits=64, sigma=24, commit=1), None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(desc_bits=64, sigma=41),
                                  None, ctypes.byref(out)) == mb.EUNSUPPORTED
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(desc_bits=64, sigma=18),
                                  None, ctypes.byref(out)) == mb.EUNSUPPORTED
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 1, opts(desc_bits=64, sigma=28),
                                  None, ctypes.byref(out)) == mb.EUNSUPPORTED
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0,
                                  opts(desc_bits=64, sigma=24, block_lanes=1024), None,
                                  ctypes.byref(out)) == mb.EUNSUPPORTED
    # column stripes: a power of two up to 32, wave commit only, nnz < 2^30
    for bad in (3, 6, 64, -1):
        assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(stripes=bad), None,
                                      ctypes.byref(out)) == mb.EINVAL
    assert b"stripes" in lib.merbit_last_error()
    assert lib.merbit_plan_create(1, 1, 0, vp(8), None, None, 0, opts(stripes=8, commit=1),
                                  None, ctypes.byref(out)) == mb.EUNSUPPORTED
    assert lib.merbit_plan_create(1, 1 << 20, 1 << 30, vp(8), vp(8), vp(8), 0,
                                  opts(stripes=8), None, ctypes.byref(out)) == mb.EUNSUPPORTED
    assert not out.value
    # calls on a NULL plan
    assert lib.merbit_spmv(None, None, None, None) == mb.EINVAL
    assert lib.merbit_pagerank(None, 0.85, 0.0, 1, 1, None, None, None, None) == mb.EINVAL
    assert lib.merbit_spmm(None, None, 1, None, 1, 1, None) == mb.EINVAL
    assert lib.merbit_spmm_dual(None, None, 1, None, 1, None, 1, 1, None) == mb.EINVAL
    assert lib.merbit_spmm_zero_boundary(None, None, 1, 1, None) == mb.EINVAL
    assert lib.merbit_pagerank_personalized(None, 0.85, 0.0, 1, 1, None, 1, None, None, None,
                                            None) == mb.EINVAL
    assert lib.merbit_pagerank_multi(None, None, 1, 0.85, 0.0, 1, 1, None, None, None,
                                     None) == mb.EINVAL
    # adjoint pieces
    assert lib.merbit_transpose(None, None, None, None, None) == mb.EINVAL
    assert lib.merbit_sddmm(None, None, None, 1.0, None, None) == mb.EINVAL
    assert lib.merbit_gather_values(7, 1, vp(8), vp(8), None, vp(16), None) == mb.EUNSUPPORTED
    assert lib.merbit_gather_values(0, -1, vp(8), vp(8), None, vp(16), None) == mb.EINVAL
    assert lib.merbit_gather_values(0, 1, vp(8), vp(8), None, vp(8), None) == mb.EINVAL  # alias
    assert lib.merbit_gather_values(0, 0, None, None, None, None, None) == mb.OK  # nothing to do
    assert lib.merbit_column_scale(1, 1, None, vp(8), None, vp(8), vp(8), None) == mb.EINVAL
    assert lib.merbit_pagerank_adjoint(None, None, 0.85, 0.0, 1, 1, None, None, None, None,
                                       None) == mb.EINVAL
    assert lib.merbit_bicgstab(None, None, None, 1e-10, 1, 1, None, None, None) == mb.EINVAL
    # tuner
    assert lib.merbit_tune(1, 1, 0, vp(8), None, None, 0, None, 0, None, 0, 5, None, None,
                           None) == mb.EINVAL
    assert lib.merbit_tune(1, 1, 0, vp(8), None, None, 7, None, 0, None, 0, 5,
                           ctypes.byref(d), None, None) == mb.EUNSUPPORTED
    assert lib.merbit_tune(1, 1, 0, vp(8), None, None, 0, None, 0, None, 0, 0,
                           ctypes.byref(d), None, None) == mb.EINVAL


def test_oracle_is_not_imported_by_the_package():
    pkg_dir = os.path.join(ROOT, "paper_2605_07391_amd")
    for dirpath, _, files in os.walk(pkg_dir):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                with open(os.path.join(dirpath, fn)) as f:
                    src = f.read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "merbit_oracle" not in src, fn
