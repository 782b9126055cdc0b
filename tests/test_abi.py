"""The C-ABI library loads and exports every entry point include/phurbas.h
declares; the binding knows each of them.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phurbas.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("phb_neighbors_build", "phb_mls_derivs", "phb_mhd_rhs", "phb_mhd_rhs_adjoint",
                 "phb_pc_step", "phb_neighbors_transpose"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1110_0836_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libphurbas.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(P.EXPORTS) == declared()


def test_host_only_calls():
    import paper_1110_0836_amd as P
    lib = P.lib()
    assert lib.phb_strerror(P.PHB_ECAPACITY) == b"output buffer too small"
    # rows of n rounded up to 64, plus 104 (no power-of-two row stride)
    assert lib.phb_tape_bytes(1000) == ((1024 + 104) * 31 + 340 * 1000) * 8
    assert lib.phb_tape_bytes(1 << 20) == (((1 << 20) + 104) * 31 + 340 * (1 << 20)) * 8
    assert lib.phb_tape_bytes(0) == 0
    # null arguments are rejected before any device work
    assert lib.phb_create(None, 0, None) == P.PHB_EINVAL
    assert lib.phb_destroy(None) == P.PHB_EINVAL
    assert lib.phb_neighbors_build(None, None, 10, None, None, None, None, 0, None) == P.PHB_EINVAL


def test_params_layout_matches_header():
    import paper_1110_0836_amd as P
    # double L[3]; int32 periodic[3]; (pad) double gamma; double rf_ratio; int32 x3; (pad)
    # double visc_grid, visc_adapt, divb_diff
    assert ctypes.sizeof(P.Params) == 24 + 12 + 4 + 8 + 8 + 12 + 4 + 3 * 8
    assert P.Params.gamma.offset == 40
    assert P.Params.visc_grid.offset == 72 and P.Params.divb_diff.offset == 88


def test_batch_io_layout_and_null_batch():
    import paper_1110_0836_amd as P
    # sixteen pointers in the order of the header's phb_batch_io
    assert ctypes.sizeof(P.BatchIO) == 16 * 8
    assert [f[0] for f in P.BatchIO._fields_][:4] == ["pos", "lambda_", "offsets", "idx"]
    assert P.BatchIO.pos_bar.offset == 15 * 8
    lib = P.lib()
    assert lib.phb_batch_destroy(None) == P.PHB_EINVAL
    assert lib.phb_batch_launch(None, None) == P.PHB_EINVAL
    assert lib.phb_batch_create(None, None, 1, None, None) == P.PHB_EINVAL
