"""Host-side checks of the C ABI that need no GPU: every symbol the header
declares is exported, and argument errors are reported before any device
work is queued."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tuckvsie.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tv_[a-z_0-9]+)\s*\(", txt)))


def test_header_symbols_exported():
    from paper_2103_06393_amd import lib
    names = _declared()
    assert len(names) >= 14
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n
    assert set(lib.EXPORTED) == set(names)


def test_status_strings():
    from paper_2103_06393_amd import lib
    for code, name in lib.STATUS.items():
        assert lib.tv_status_string(code) == name


def _factors(dims, ranks):
    n1, n2, n3 = dims
    r = np.asarray(ranks).reshape(-1, 3)
    G = np.ones(int(np.sum(np.prod(r, axis=1))), complex)
    U1 = np.ones(int(np.sum(n1 * r[:, 0])), complex)
    U2 = np.ones(int(np.sum(n2 * r[:, 1])), complex)
    U3 = np.ones(int(np.sum(n3 * r[:, 2])), complex)
    return G, U1, U2, U3


def test_plan_argument_errors():
    from paper_2103_06393_amd import lib
    dims = (8, 8, 8)
    g = lib.make_grid(*dims, 3, 2)
    ranks = np.full((6, 3), 2, np.int32)
    G, U1, U2, U3 = _factors(dims, ranks)
    bad = ranks.copy()
    bad[4, 1] = 9                       # rank above n2
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_plan_from_factors(g, bad, *_factors(dims, bad))
    assert e.value.status == -3 and "mode 2" in str(e.value)
    bad[4, 1] = 0
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_plan_from_factors(g, bad, *_factors(dims, np.maximum(bad, 1)))
    assert e.value.status == -3
    G2 = G.copy()
    G2[3] = np.nan
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_plan_from_factors(g, ranks, G2, U1, U2, U3)
    assert e.value.status == -7
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_plan_from_factors(lib.make_grid(0, 8, 8, 3, 2), ranks, G, U1, U2, U3)
    assert e.value.status == -2
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_plan_from_factors(g, ranks, G, U1, U2, U3, precision=7)
    assert e.value.status == -1


def test_call_argument_errors_without_device_work():
    from paper_2103_06393_amd import lib
    assert lib._tv_matvec(None, None, 1, 1, None, 1, None, 0, None) == -1
    assert lib._tv_rmatvec(None, None, 1, 1, None, 1, None, 0, None) == -1
    assert lib._tv_workspace_bytes(None, 0, 1, None) == -1
    g = lib.make_grid(4, 4, 4, 3, 2)
    # compression parameters are validated on the host
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_compress_begin(g, -1.0, 1, 0)
    assert e.value.status == -1
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_compress_begin(g, 1e-3, 5, 3)
    assert e.value.status == -3
    h = lib.tv_compress_begin(g, 1e-3, 1, 0)
    with pytest.raises(lib.TuckVsieError):
        lib.tv_plan_finalize(h, None)      # no column appended yet
    lib.tv_plan_destroy(h)
    # a source inside the voxel domain is refused before any launch
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_dipole_columns(4, 4, 4, 0.01, 1.0, 0, np.zeros((1, 3)),
                              np.array([[1.0, 0, 0]]), 1, None)
    assert e.value.status == -1


def test_aca_entry_points_reject_null_plan():
    """The ACA + Tucker entry points validate on the host before queueing
    any device work (no GPU needed for these paths)."""
    from paper_2103_06393_amd import lib
    with pytest.raises(lib.TuckVsieError) as e:
        lib.tv_aca_workspace_bytes(None, 0, 1)
    assert e.value.status == -1
    for f in (lib.tv_aca_matvec, lib.tv_aca_rmatvec):
        with pytest.raises(lib.TuckVsieError) as e:
            f(None, None, 1, 1, None, 1, 1, None, 1, None, 0, None)
        assert e.value.status == -1 and "plan is NULL" in str(e.value)


def test_plan_arena_is_the_callers():
    """Plans are packed on the host; their device memory is an arena the
    caller binds.  A short or misaligned arena is refused before any device
    work, and an unbound plan refuses products."""
    from paper_2103_06393_amd import lib
    dims = (8, 6, 5)
    g = lib.make_grid(*dims, 3, 2)
    ranks = np.full((6, 3), 2, np.int32)
    h = lib.tv_plan_from_factors(g, ranks, *_factors(dims, ranks))
    try:
        need = lib.tv_plan_required_bytes(h)
        assert need > 0 and need % 256 == 0
        assert lib.tv_plan_info(h).device_bytes == need
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_plan_bind_arena(h, 1 << 20, need - 256, None)       # short
        assert e.value.status == -8
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_plan_bind_arena(h, (1 << 20) + 16, need, None)      # misaligned
        assert e.value.status == -1
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_plan_bind_arena(h, None, need, None)
        assert e.value.status == -1
        # products and autotuning need the arena
        assert lib._tv_matvec(h, 8, 2, 1, 4096, 3 * 240, 0, 0, None) == -1
        assert "arena" in lib.tv_last_error()
        with pytest.raises(lib.TuckVsieError):
            lib.tv_autotune(h, 2, None, None)
        with pytest.raises(lib.TuckVsieError):
            lib.tv_batch_create([h], 0, [1])
    finally:
        lib.tv_plan_destroy(h)


def test_compression_workspace_is_the_callers():
    from paper_2103_06393_amd import lib
    g = lib.make_grid(12, 10, 9, 3, 4)
    h = lib.tv_compress_begin(g, 1e-3, 1, 6)
    try:
        need = lib.tv_compress_workspace_bytes(h, 2)
        assert need > 0 and need % 256 == 0
        assert lib.tv_compress_workspace_bytes(h, 4) > need
        # a short workspace is refused before any device work
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_compress_append(h, 1 << 20, 2, 1 << 24, need - 256, None)
        assert e.value.status == -8
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_compress_append(h, 1 << 20, 2, None, need, None)
        assert e.value.status == -8
    finally:
        lib.tv_plan_destroy(h)


def test_aca_assembly_workspace_is_the_callers():
    from paper_2103_06393_amd import lib
    g = lib.make_grid(6, 5, 4, 3, 10)
    ang = np.linspace(0, 2 * np.pi, 10, endpoint=False)
    pos = np.stack([0.2 * np.cos(ang), 0.2 * np.sin(ang), np.zeros(10)], axis=1)
    ori = np.stack([-np.sin(ang), np.cos(ang), np.zeros(10)], axis=1)
    need = lib.tv_aca_assemble_workspace_bytes(g, 4, 1e-3)
    assert need > 0 and need % 256 == 0
    assert lib.tv_aca_assemble_workspace_bytes(g, 4, 1e-3, rank_cap=2) < need
    for ws, nb in ((None, need), (1 << 24, need - 256)):
        with pytest.raises(lib.TuckVsieError) as e:
            lib.tv_aca_assemble(g, 0.01, 6.0, 0, pos, ori, 1e-3, max_terms=4,
                                ws_ptr=ws, ws_bytes=nb)
        assert e.value.status == -8
