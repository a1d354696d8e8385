"""soma_observables_noalloc through the C-ABI: the same results as
soma_observables (same kernels, partial sums in the library's static device
array instead of the workspace), on two calls in a row, the second on a
smaller system, and a clear error for a system beyond the array's limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_09356_amd import workloads as W
from paper_2606_09356_amd.soma import Soma, SomaError, SOMA_EINVAL, soma_obs

pytestmark = pytest.mark.gpu
SEED = 20260609
FIELDS = [f for f, _ in soma_obs._fields_]


def both(g, sys):
    a, b = soma_obs(), soma_obs()
    g._c(g.lib.soma_observables(g.ctx, sys, C.byref(a)))
    g._c(g.lib.soma_observables_noalloc(g.ctx, sys, C.byref(b)))
    return {f: getattr(a, f) for f in FIELDS}, {f: getattr(b, f) for f in FIELDS}


@pytest.mark.parametrize("r,dm", [("cell", 1), ("f32", 0)])
def test_noalloc_observables_equal_the_workspace_path(r, dm):
    large = W.diblock_system(131072, 32, 0.5, 20.0, 50.0, (32, 32, 32), (128, 128, 128), "large")
    small = W.batched_mixed(n_systems=1, seed=77, bead_range=(3000, 5000))[0]
    g = Soma([large, small], seed=SEED, pos_repr=r, count_width=16, density_mode=dm)
    g.sweep(3)
    # the large system first (8704 blocks of partial sums), then the small one
    for sys in (0, 1, 0, 1):
        ref, got = both(g, sys)
        print(f"[noalloc] system {sys}: Re2 {got['Re2']:.9f} Enb {got['Enb_per_chain']:.6f}", flush=True)
        assert got == ref, (sys, {k: (ref[k], got[k]) for k in FIELDS if ref[k] != got[k]})
        g.sweep(1)
    g.close()


def test_noalloc_rejects_a_system_beyond_the_limit():
    # 4.2M cells: ceil(1000/256) + 16384 blocks > 10922
    big_grid = W.diblock_system(1000, 8, 0.5, 0.0, 10.0, (64, 64, 16), (256, 256, 64), "big grid")
    g = Soma([big_grid], seed=SEED, pos_repr="f32", count_width=16)
    o = soma_obs()
    rc = g.lib.soma_observables_noalloc(g.ctx, 0, C.byref(o))
    assert rc == SOMA_EINVAL
    assert b"too large" in g.lib.soma_last_error(g.ctx)
    # the context stays usable, and the workspace path still serves it
    g.sweep(1)
    assert g.observables(0)["sweep"] == 1
    g.close()
