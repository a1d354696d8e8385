"""Pins of the oracle's density histogram, fields, energy and observables.

Pinned against hand-set cases whose values follow from the model by hand,
and against exact identities:
  * density: a bead placed in a known cell lands at linear index
    (ix*ny + iy)*nz + iz; faces belong to the upper cell; periodic images and
    negative unwrapped coordinates wrap; the histogram sums to the bead count;
  * fields: phiA = phiB = 1/2 gives omega = 0; a pure-A cell at phiA = 1 and an
    empty cell give the closed values below; omega equals the exact central
    difference of the non-bonded energy (the energy is quadratic in counts);
  * energy: a uniform 50/50 melt has zero Helfand energy; a pure-A melt has
    H/kT = -n_chains chiN / 4;
  * observables: a straight chain has Re^2 = ((N-1) b)^2,
    Rg^2 = b^2 (N^2 - 1) / 12 and bond energy (k/2)(N-1) b^2;
  * the compensated sum agrees with Python's exactly rounded math.fsum.
"""
import math

import numpy as np
import pytest

from paper_2606_09356_amd import workloads as W
from tests.helpers.positions import face_adjacent_fp32


def small_system(n_chains=4, N=4, grid=(4, 5, 6), box=(1.0, 1.25, 1.5), chiN=20.0, kappaN=50.0,
                 ham_form=0, f=0.5):
    s = W.diblock_system(n_chains, N, f, chiN, kappaN, box, grid)
    s.ham_form = ham_form
    return s


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_density_layout_faces_and_wrap(orc, mode):
    s = small_system(n_chains=1, N=4)        # edges 0.25 in every direction
    O = orc.OracleSystem(s, mode=mode)
    nx, ny, nz = s.grid
    xyz = np.array([
        [0.30, 0.25, -0.01, 1.0 + 0.30],     # x: cell 1, face -> 1, wraps to 3, image of cell 1
        [0.60, 0.0, -0.26, 1.25 * 3 + 0.60],  # y: cell 2, face -> 0, -2 -> 3, image of 2
        [1.40, 0.5, 1.5, -1.5 + 1.40],        # z: cell 5, face 2, 6 -> 0, image of 5
    ])
    O.set_positions(xyz)
    c = O.counts
    lin = lambda ix, iy, iz: (ix * ny + iy) * nz + iz
    # pattern f=0.5, N=4: beads 0,1 are A (type 0), beads 2,3 are B (type 1)
    assert c[0, lin(1, 2, 5)] == 1
    assert c[0, lin(1, 0, 2)] == 1
    assert c[1, lin(3, 3, 0)] == 1
    assert c[1, lin(1, 2, 5)] == 1
    assert c.sum() == 4 and c[0].sum() == 2 and c[1].sum() == 2


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_density_sums_and_permutation_invariance(orc, mode):
    s = W.batched_mixed(n_systems=1, seed=3, bead_range=(2000, 4000))[0]
    xyz = W.gaussian_walks(s, seed=5)
    O = orc.OracleSystem(s, mode=mode)
    O.set_positions(xyz)
    t = s.bead_types()
    assert O.counts[0].sum() == (t == 0).sum()
    assert O.counts[1].sum() == (t == 1).sum()
    # Reversing chain order (types follow their chains only when the system is
    # not a blend, so use the pattern-independent total here).
    perm = np.arange(s.n_chains)[::-1]
    xyz2 = xyz.reshape(3, s.n_chains, s.N)[:, perm].reshape(3, -1)
    O2 = orc.OracleSystem(s, mode=mode)
    O2.set_positions(xyz2)
    assert (O2.counts.sum(axis=0) == O.counts.sum(axis=0)).all()


@pytest.mark.parametrize("ham_form", [0, 1])
def test_fields_hand_cases(orc, ham_form):
    s = small_system(n_chains=6, N=4, grid=(2, 2, 2), box=(0.5, 0.5, 0.5), ham_form=ham_form)
    # B = 24 beads, M = 8 cells -> phi = n * M / B = n / 3
    O = orc.OracleSystem(s)
    counts = np.zeros((2, 8), np.uint32)
    counts[:, 0] = (3, 0)       # pure A, phiA = 1
    counts[:, 1] = (0, 0)       # empty
    counts[:, 2] = (0, 3)       # pure B
    counts[:, 3] = (3, 3)       # phiA = phiB = 1
    counts[:, 4] = (0, 6)       # phiB = 2
    O.counts[...] = counts
    w = O.fields()
    chi, kap, N = s.chiN, s.kappaN, s.N
    if ham_form == 0:
        expect = {0: (-chi / 2 / N, chi / 2 / N), 1: (-kap / N, -kap / N), 2: (chi / 2 / N, -chi / 2 / N),
                  3: (kap / N, kap / N), 4: (kap / N + chi / N, kap / N - chi / N)}
    else:
        expect = {0: (0.0, chi / N), 1: (-kap / N, -kap / N), 2: (chi / N, 0.0),
                  3: (kap / N + chi / N, kap / N + chi / N), 4: (kap / N + 2 * chi / N, kap / N)}
    for c, (wa, wb) in expect.items():
        assert w[0, c] == pytest.approx(wa, abs=1e-12), c
        assert w[1, c] == pytest.approx(wb, abs=1e-12), c


def test_fields_half_half_is_zero(orc):
    s = small_system(n_chains=8, N=4, grid=(2, 2, 2), box=(0.5, 0.5, 0.5))
    O = orc.OracleSystem(s)
    O.counts[...] = 2                       # B = 32, M = 8: phiA = phiB = 1/2
    w = O.fields()
    assert np.abs(w).max() < 1e-14
    assert abs(O.energy_nb()) < 1e-12


@pytest.mark.parametrize("ham_form", [0, 1])
def test_fields_are_exact_derivative_of_energy(orc, ham_form):
    s = small_system(n_chains=30, N=8, grid=(3, 2, 4), box=(0.75, 0.5, 1.0), ham_form=ham_form,
                     chiN=17.0, kappaN=33.0)
    O = orc.OracleSystem(s)
    rng = np.random.default_rng(2)
    base = rng.integers(2, 25, size=(2, s.n_cells)).astype(np.uint32)
    O.counts[...] = base
    w = O.fields().copy()
    for t in range(2):
        for c in range(s.n_cells):
            O.counts[...] = base
            O.counts[t, c] += 1
            ep = O.energy_nb()
            O.counts[t, c] -= 2
            em = O.energy_nb()
            assert (ep - em) / 2 == pytest.approx(w[t, c], rel=1e-9, abs=1e-9)


def test_energy_pure_a_melt(orc):
    s = small_system(n_chains=6, N=4, grid=(2, 2, 2), box=(0.5, 0.5, 0.5))
    O = orc.OracleSystem(s)
    O.counts[0] = 3                          # phiA = 1 everywhere (B = 24, M = 8)
    O.counts[1] = 0
    assert O.energy_nb() == pytest.approx(-s.n_chains * s.chiN / 4, rel=1e-12)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_observables_straight_chain(orc, mode):
    N, b = 16, 0.125
    s = small_system(n_chains=3, N=N, grid=(4, 4, 4), box=(4.0, 4.0, 4.0))
    xyz = np.zeros((3, 3 * N))
    for c in range(3):
        xyz[c % 3, c * N:(c + 1) * N] = 1.0 + b * np.arange(N)   # along x, y or z
        xyz[(c + 1) % 3, c * N:(c + 1) * N] = 0.5
    O = orc.OracleSystem(s, mode=mode)
    O.set_positions(xyz)
    o = O.observables()
    k = 3 * (N - 1)
    assert o["Re2"] == pytest.approx(((N - 1) * b) ** 2, rel=1e-12)
    assert o["Rg2"] == pytest.approx(b * b * (N * N - 1) / 12, rel=1e-12)
    assert o["Ebond_per_chain"] == pytest.approx(0.5 * k * (N - 1) * b * b, rel=1e-12)
    assert o["Re2_err"] == pytest.approx(0.0, abs=1e-12)


def test_neumaier_matches_fsum(orc):
    cases = [[1e16, 1.0, -1e16], [1.0, 1e100, 1.0, -1e100], [0.1] * 10]
    rng = np.random.default_rng(0)
    v = rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, size=10000)
    cases.append(list(v))
    for c in cases:
        assert orc.neumaier_sum(c) == pytest.approx(math.fsum(c), rel=1e-15, abs=1e-300)


def test_cell_offset_representation_round_trip(orc):
    s = small_system(n_chains=64, N=16, grid=(8, 8, 8), box=(2.0, 2.0, 2.0))
    xyz = W.gaussian_walks(s, seed=9) * 7.0 - 5.0      # spread over several images
    O = orc.OracleSystem(s, mode=2)
    O.set_positions(xyz, refresh=False)
    assert (O.off >= 0).all() and (O.off < 0.25).all()
    assert (O.cell == np.floor(xyz / 0.25)).mean() > 0.999
    back = O.positions()
    assert np.abs(back - xyz).max() < 2 ** -26    # FP32 offset resolution below 0.25


@pytest.mark.parametrize("mode", [0, 1])
def test_ngp_cell_is_exact_quotient_for_non_dyadic_edge(orc, mode):
    """NGP cell = floor(x / e) of the exact quotient, e = box/grid rounded to
    FP32, checked with rational arithmetic on coordinates within a few ulps of
    the faces of a grid whose edge (1.275 / 25 = 0.051) is not a power of two."""
    from fractions import Fraction
    box, grid = 1.275, 25
    edge32 = np.float32(box / grid)
    rng = np.random.default_rng(11)
    xs = face_adjacent_fp32(edge32, list(range(-30, 60, 7)), rng)
    n = len(xs)
    s = W.diblock_system(n, 2, 0.5, 0.0, 0.0, (box, box, box), (grid, grid, grid))
    O = orc.OracleSystem(s, mode=mode)
    xyz = np.zeros((3, 2 * n))
    xyz[0, 0::2] = xs                       # bead 0 (type A) of every chain on the test coordinate
    xyz[0, 1::2] = 0.5 * float(edge32)      # bead 1 (type B) in the middle of x-cell 0
    xyz[1:, :] = 0.5 * float(edge32)
    O.set_positions(xyz)
    E = Fraction(float(edge32))
    expect = np.zeros(s.n_cells, np.uint32)
    for x in xs:
        k = math.floor(Fraction(x) / E)
        expect[(k % grid) * grid * grid] += 1
    assert (O.counts[0] == expect).all()
    assert O.counts[1][0] == n and O.counts[1].sum() == n


@pytest.mark.parametrize("box", [2.0, 2.04])
def test_cell_offset_window_after_trial_moves(orc, box):
    """Cell + offset state after trial moves: every offset lies in the
    window [-e, 2e) and some lie outside [0, e) (cells step only when an
    offset leaves the window), and the density of the stored pairs is the
    NGP histogram of floor(x / e) of the points x = c e + o, evaluated with
    exact rational arithmetic (edge 0.25, and 2.04 / 8 = 0.255 rounded to
    FP32, which is not a power of two)."""
    from fractions import Fraction
    s = W.diblock_system(64, 16, 0.5, 0.0, 0.0, (box, box, box), (8, 8, 8), move_halfwidth=0.2)
    O = orc.OracleSystem(s, mode=2)
    O.set_positions(W.gaussian_walks(s, seed=13))
    O.run(seed=3, first_sweep=0, n_sweeps=60)
    e32 = np.float32(box / 8)
    assert (O.off >= -e32).all() and (O.off < 2 * e32).all()
    assert ((O.off < 0) | (O.off >= e32)).mean() > 0.2
    e = Fraction(float(e32))
    n = 8
    types = s.bead_types()
    expect = np.zeros((2, n ** 3), np.int64)
    for b in range(s.n_beads):
        idx = []
        for a in range(3):
            x = Fraction(int(O.cell[a, b])) * e + Fraction(float(O.off[a, b]))
            idx.append(math.floor(x / e) % n)
        expect[types[b], (idx[0] * n + idx[1]) * n + idx[2]] += 1
    O.density()
    assert (O.counts == expect).all()
