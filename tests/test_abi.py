"""The C-ABI library loads on the host and exports every function include/md.h declares (no GPU calls)."""
import ctypes
import os

import pytest

from paper_1912_04232_amd import md


def test_header_declares_the_boundary():
    names = md.header_functions()
    for required in ("nl_build", "pair_energy_force", "verlet_step", "fire_init", "fire_step", "md_ctx_create",
                     "md_ctx_reserve", "md_flags_read"):
        assert required in names


def test_library_exports_every_header_symbol():
    if not os.path.exists(md.LIB_PATH):
        pytest.fail("libmdcore.so is not built (python -m paper_1912_04232_amd.build)")
    lib = ctypes.CDLL(md.LIB_PATH)
    for name in md.header_functions():
        assert hasattr(lib, name), name
    assert set(md.header_functions()) <= set(md._SIGNATURES)


def test_struct_layouts_match_header():
    # sizes follow from the field lists in include/md.h (natural alignment, x86-64)
    assert ctypes.sizeof(md.c_box) == 16
    assert ctypes.sizeof(md.c_potential) == 4 * 2 + 8 * 64 * 2 + 4 * 4 + 8 * 64
    assert ctypes.sizeof(md.c_nlist) == 24 + 4 * 8
    assert ctypes.sizeof(md.c_fire_params) == 32
    assert ctypes.sizeof(md.c_fire_state) == 6 * 8 + 8 + 8
    assert ctypes.sizeof(md.c_flock_params) == 10 * 4 + 2 * 4 + 16 * 3 * 4
    assert ctypes.sizeof(md.c_flock_predators) == 6 * 4 + 2 * 8
    assert ctypes.sizeof(md.c_batch_config) == 8


def test_host_side_helpers_without_gpu():
    lib = md.load()
    b = md.Box((10.772174, 10.772174, 10.772174), 3).c()
    assert lib.md_cell_count(ctypes.byref(b), ctypes.c_float(2.8)) == 27
    b = md.Box((67.29563, 67.29563, 67.29563), 3).c()
    assert lib.md_cell_count(ctypes.byref(b), ctypes.c_float(2.8)) == 24 ** 3
    b = md.Box((5.0, 5.0, 5.0), 3).c()
    assert lib.md_cell_count(ctypes.byref(b), ctypes.c_float(2.0)) == 1   # < 3 cells per side: scanned whole
    b = md.Box((290.93402, 290.93402, 0.0), 2).c()
    assert lib.md_cell_count(ctypes.byref(b), ctypes.c_float(1.7)) == 171 ** 2
    assert lib.md_version().startswith(b"md-gfx950")


def test_argument_errors_are_returned_synchronously():
    lib = md.load()
    # NULL context / bad dims are rejected before any device work
    b = md.c_box()
    b.dim = 4
    assert lib.nl_build(None, ctypes.byref(b), None, 0, None, None) == -1
    assert lib.md_ctx_reserve(None, 10, 3, 1, 1, 1, 1) == -1
    assert lib.md_sum(None, None, 0, None, None) == -1
    fp = md.c_flock_params()
    b.dim = 2
    assert lib.flock_step(None, ctypes.byref(b), None, None, 0, None, ctypes.byref(fp), None, None, None) == -1


def test_unrolled_fire_workspace_size_and_argument_errors():
    lib = md.load()
    B, total, K = 3, 300, 10
    rec = (40 * K * B + 255) // 256 * 256
    assert lib.fire_unrolled_workspace_bytes(B, total, K) == rec + 24 * (K + 1) * total
    assert lib.fire_unrolled_workspace_bytes(0, 0, 0) == 0
    assert lib.fire_unrolled_workspace_bytes(-1, 5, 5) == 0
    pot = md.Potential("soft_sphere", ((1.0,),), ((1.0,),), alpha=2.0).c()
    fp = md.FireParams().c()
    b = md.c_batch()
    b.B, b.dim, b.max_n = 1, 2, 10
    args = [ctypes.byref(b), ctypes.byref(pot), None, ctypes.byref(fp), 5, None, 0] + [None] * 7 + [None]
    assert lib.fire_unrolled_grad(None, *args) == -1           # no context
    b.dim = 3
    assert lib.fire_unrolled_grad(None, *args) == -1
