"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/fld.h, and rejects invalid arguments before touching a
device."""
import os
import re

import pytest

import paper_1403_8105_amd as F

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "fld.h")


def declared_symbols():
    text = open(HEADER).read()
    decl = r"^(?:fld_status|void|const char)\s*\*?\s*(fld_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = F.lib()
    syms = declared_symbols()
    assert len(syms) >= 17
    for name in syms:
        assert hasattr(lib, name), name
    assert set(F.EXPORTS) <= set(syms)


def test_default_options():
    o = F.fld_default_options()
    assert o.struct_size == F.C.sizeof(F.fld_options)
    assert o.limiter == F.LIMITERS["lp"] and o.method == F.METHODS["mg"]
    assert o.eps == 1e-20 and o.sigma_eps < 0 and o.tol == 1e-6
    assert (o.nu1, o.nu2, o.max_coarsest) == (2, 2, 512)


@pytest.mark.parametrize("kw,dims,h", [
    ({}, (0, 4, 4), 0.1),
    ({}, (8, 8, 8), 0.0),
    ({}, (8, 8, 8), float("nan")),
    ({"omega": 2.0}, (8, 8, 8), 0.1),
    ({"omega_s": 0.0}, (8, 8, 8), 0.1),
    ({"limiter": 9}, (8, 8, 8), 0.1),
    ({"method": "rbsor", "precision": "mixed"}, (8, 8, 8), 0.1),
    ({"tol": -1.0}, (8, 8, 8), 0.1),
    ({"max_coarsest": 0}, (8, 8, 8), 0.1),
    ({"nu1": 0, "nu2": 0}, (8, 8, 8), 0.1),
    ({}, (100, 100, 100), 0.01),          # multigrid: coarsest 25^3 > 512
    ({"limiter": "larsen", "larsen_n": 0.0}, (8, 8, 8), 0.1),
    ({"nested_tol": -1.0}, (8, 8, 8), 0.1),
    ({"nested_tol": 1e-3}, (5, 8, 8), 0.1),            # grid sequencing needs even axes
    ({"nested_tol": 1e-3, "method": "rbsor"}, (8, 8, 8), 0.1),
    ({"nested_tol": 1e-3, "anisotropy_g": 0.5}, (8, 8, 8), 0.1),
    ({"fuse_lr": 2}, (8, 8, 8), 0.1),
    ({"fuse_rb": -1}, (8, 8, 8), 0.1),
    ({"aa_m": 17}, (8, 8, 8), 0.1),
    ({"aa_reg": -1.0}, (8, 8, 8), 0.1),
    ({"nu_coarse": 65}, (8, 8, 8), 0.1),
    ({"nu_coarse": -1}, (8, 8, 8), 0.1),
    ({"nu_coarse": 8, "coarse_from": 0}, (8, 8, 8), 0.1),
    ({"nested_inherit": 2}, (8, 8, 8), 0.1),
])
def test_create_rejects_invalid_arguments(kw, dims, h):
    o = F.fld_default_options(**kw)
    with pytest.raises(F.FldError) as ei:
        F.fld_create(o, *dims, h)
    assert ei.value.status == F.FLD_ERR_INVALID_ARGUMENT


def test_struct_size_is_checked():
    o = F.fld_default_options()
    o.struct_size = 8
    with pytest.raises(F.FldError):
        F.fld_create(o, 8, 8, 8, 0.1)


def test_null_handles():
    lib = F.lib()
    assert lib.fld_set_medium(None, None, None, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert lib.fld_solve(None, None, None, None) == F.FLD_ERR_INVALID_ARGUMENT
    lib.fld_destroy(None)
    lib.fld_batch_destroy(None)
    assert F.fld_status_string(F.FLD_ERR_STATE) == "invalid call order"


def test_light_bake_rejects_invalid_arguments():
    import paper_1403_8105_amd as F

    L = F.lib()
    assert L.fld_light_bake(None, None, 1.0, 4, 4, 4, 0.25, None, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert L.fld_light_bake(1, 1, 1.0, 0, 4, 4, 0.25, 1, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert L.fld_light_bake(1, 1, -1.0, 4, 4, 4, 0.25, 1, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert L.fld_light_bake(1, 1, 1.0, 4, 4, 4, float("nan"), 1, None) == F.FLD_ERR_INVALID_ARGUMENT


def test_render_rejects_invalid_arguments():
    import paper_1403_8105_amd as F

    L = F.lib()
    assert L.fld_render(None, 1, 1, 1, 0.0, 4, 4, 4, 0.25, 1, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert L.fld_render(1, 1, 1, 1, -1.0, 4, 4, 4, 0.25, 1, None) == F.FLD_ERR_INVALID_ARGUMENT
    assert L.fld_render(1, 1, 1, 1, 0.0, 4, 4, 0, 0.25, 1, None) == F.FLD_ERR_INVALID_ARGUMENT


def test_batch_grid_sequencing_needs_even_axes():
    o = F.fld_default_options(nested_tol=1e-3, precision="mixed")
    with pytest.raises(F.FldError) as ei:
        F.fld_batch_create(o, [(16, 16, 16), (10, 8, 5)], [1.0 / 16, 0.1], 1)
    assert ei.value.status == F.FLD_ERR_INVALID_ARGUMENT


def test_one_library_copy_per_process():
    # a context belongs to the copy of libfld.so that created it; asking the
    # binding for a second copy (another path) in the same process is refused
    F.lib()
    saved = F.LIB_PATH
    try:
        F.LIB_PATH = saved + ".other"
        with pytest.raises(RuntimeError, match="already loaded"):
            F.lib()
    finally:
        F.LIB_PATH = saved
    assert F.lib() is not None
