"""The C-ABI library loads and exports every function include/soma.h declares;
host-side argument checks (no GPU work) return the documented codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2606_09356_amd import soma as S
from paper_2606_09356_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "soma.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(soma_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return S.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 17, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(S.EXPORTS) == set(names)


def _opts(**kw):
    o = S.soma_options()
    o.seed, o.pos_repr, o.count_width, o.use_graph = 1, S.POS_F32, S.COUNT_U16, 1
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_workspace_size_scales_with_representation(lib):
    sysd = W.plain_small()
    arr, keep = S._desc_array(sysd)
    sizes = {}
    for repr_, cw in [(S.POS_F32, S.COUNT_U16), (S.POS_CELL_F32, S.COUNT_U32)]:
        n = C.c_size_t(0)
        assert lib.soma_workspace_size(arr, 1, C.byref(_opts(pos_repr=repr_, count_width=cw)), C.byref(n)) == 0
        sizes[(repr_, cw)] = n.value
    B, M = sysd[0].n_beads, sysd[0].n_cells
    assert sizes[(S.POS_F32, S.COUNT_U16)] >= 12 * B + 3 * 4 * M + 8 * M
    assert sizes[(S.POS_CELL_F32, S.COUNT_U32)] - sizes[(S.POS_F32, S.COUNT_U16)] >= 12 * B + 3 * 4 * M


@pytest.mark.parametrize("field,value", [("N", 1), ("N", 129), ("n_chains", 0), ("n_chains_a", 300),
                                         ("move_halfwidth", 0.3), ("chiN", float("nan")),
                                         ("ham_form", 2), ("grid", (0, 16, 16))])
def test_invalid_descriptors_are_rejected(lib, field, value):
    s = W.plain_small()[0]
    arr, keep = S._desc_array([s])
    if field == "grid":
        arr[0].grid = (C.c_int32 * 3)(*value)
    else:
        setattr(arr[0], field, value)
    n = C.c_size_t(0)
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts()), C.byref(n)) == S.SOMA_EINVAL
    assert lib.soma_last_error(None)


def test_empty_batches_and_null_arguments_are_rejected(lib):
    """No systems, a null descriptor array or a null size pointer: EINVAL
    with a message, before anything touches a GPU."""
    arr, keep = S._desc_array(W.plain_small())
    n = C.c_size_t(0)
    assert lib.soma_workspace_size(arr, 0, C.byref(_opts()), C.byref(n)) == S.SOMA_EINVAL
    assert lib.soma_last_error(None)
    assert lib.soma_workspace_size(None, 1, C.byref(_opts()), C.byref(n)) == S.SOMA_EINVAL
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts()), None) == S.SOMA_EINVAL


def test_invalid_options_are_rejected(lib):
    arr, keep = S._desc_array(W.plain_small())
    n = C.c_size_t(0)
    for kw in [dict(pos_repr=3), dict(count_width=7), dict(waves_per_block=17), dict(density_mode=4),
               dict(density_mode=-1), dict(sys_id_base=-1), dict(launch_order=2), dict(waves_per_cu=65),
               dict(packed_tiles=3), dict(packed_tiles=1, waves_per_cu=8), dict(packed_tiles=2, waves_per_cu=8)]:
        assert lib.soma_workspace_size(arr, 1, C.byref(_opts(**kw)), C.byref(n)) == S.SOMA_EINVAL, kw


@pytest.mark.parametrize("walls,zones,dm", [((0, 20), (0, 0), 0), ((5, 3), (0, 0), 0), ((-1, 8), (0, 0), 0),
                                            ((0, 0), (2, 0), 0), ((0, 16), (9, 8), 0), ((0, 16), (2, 2), 2),
                                            ((0, 16), (-1, 0), 0)])
def test_invalid_walls_and_zones_are_rejected(lib, walls, zones, dm):
    s = W.plain_small()[0]
    s.walls, s.zones = walls, zones
    arr, keep = S._desc_array([s])
    n = C.c_size_t(0)
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts(density_mode=dm)), C.byref(n)) == S.SOMA_EINVAL


def test_walls_zones_and_packed_tiles_accepted_when_valid(lib):
    s = W.plain_small()[0]
    s.walls, s.zones = (2, 14), (3, 3)
    arr, keep = S._desc_array([s])
    n = C.c_size_t(0)
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts(density_mode=1)), C.byref(n)) == 0
    # zones exclude block tiles; without zones they are accepted
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts(packed_tiles=1)), C.byref(n)) == S.SOMA_EINVAL
    s.zones = (0, 0)
    arr, keep = S._desc_array([s])
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts(packed_tiles=1)), C.byref(n)) == 0
    # the coupling workspace adds target fields (8 B/cell) and placement sums (16 B/cell)
    m = C.c_size_t(0)
    assert lib.soma_workspace_size(arr, 1, C.byref(_opts(coupling=1)), C.byref(m)) == 0
    assert m.value - n.value >= 24 * s.n_cells


def test_create_rejects_short_or_misaligned_workspace(lib):
    arr, keep = S._desc_array(W.plain_small())
    ctx = C.c_void_p()
    buf = (C.c_uint8 * 4096)()
    # misaligned pointer: rejected before any device call
    addr = C.addressof(buf)
    mis = addr + (1 if addr % 256 == 0 else 0)
    assert lib.soma_create(arr, 1, C.byref(_opts()), mis, 4096, C.byref(ctx)) == S.SOMA_EINVAL
    aligned = (addr + 255) & ~255
    assert lib.soma_create(arr, 1, C.byref(_opts()), aligned, 1024, C.byref(ctx)) == S.SOMA_ENOMEM
    assert not ctx.value


def test_autotune_rejects_null_context(lib):
    assert lib.soma_autotune(None, 5, None) == S.SOMA_EINVAL


def test_batch_totals_are_bounded(lib):
    """Count words and chains are indexed with 32-bit values across a batch."""
    big = W.diblock_system(64, 32, 0.5, 10.0, 50.0, (1024.0, 1024.0, 256.0), (4096, 4096, 32), "big")
    n = C.c_size_t(0)
    arr, keep = S._desc_array([big] * 2)
    # 2^29 cells each: one system fits, two reach the 2^30 count-word bound
    one, keep1 = S._desc_array([big])
    assert lib.soma_workspace_size(one, 1, C.byref(_opts()), C.byref(n)) == 0
    assert lib.soma_workspace_size(arr, 2, C.byref(_opts()), C.byref(n)) == S.SOMA_EINVAL
