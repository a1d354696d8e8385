"""Closed forms of the model used as pins (independent of oracle and GPU code).

acceptance_closed_form: chain-mean Metropolis acceptance of ideal chains at
  equilibrium.  For a trial displacement d, dE is Gaussian with mean mu and
  variance 2 mu (mu = k|d|^2 interior, k|d|^2/2 end bead), so
  P(accept | d) = 2 Phi(-sqrt(mu/2)); the mean over the uniform cube is a
  Gauss-Legendre quadrature.
pair_weight_1d: sum over periodic images of the double integral of the bond
  weight exp(-(k/2)(x-y)^2) over two grid cells, by the erf antiderivative.
two_bead_cell_probabilities: exact joint cell occupancy of a two-bead chain
  (A-B) with harmonic bond k in frozen fields omega_A, omega_B.
two_bead_cell_probabilities_walls: the same with hard walls at the z-cell
  faces lo and hi (no periodic images in z, zero weight outside).
"""
import math

import numpy as np
from scipy import special


def acceptance_closed_form(N, delta, Re=1.0, n_nodes=64):
    k = 3.0 * (N - 1) / Re ** 2
    x, w = np.polynomial.legendre.leggauss(n_nodes)
    x = 0.5 * delta * (x + 1.0)
    w = 0.5 * w
    d2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    ww = w[:, None, None] * w[None, :, None] * w[None, None, :]

    def mean_acc(mu):
        return float((ww * 2.0 * special.ndtr(-np.sqrt(mu / 2.0))).sum())
    if N == 1:
        return 1.0
    p_int = mean_acc(k * d2)
    p_end = mean_acc(0.5 * k * d2)
    return (2 * p_end + (N - 2) * p_int) / N


def pair_weight_1d(n, L, k, n_images=6):
    a = 0.5 * k
    F = lambda u: 0.5 * math.sqrt(math.pi / a) * special.erf(math.sqrt(a) * u)
    G2 = lambda u: u * F(u) + (math.exp(-a * u * u) - 1.0) / (2 * a)
    h = L / n
    Wm = np.zeros((n, n))
    for i in range(n):
        lo1, hi1 = i * h, (i + 1) * h
        for j in range(n):
            tot = 0.0
            for m in range(-n_images, n_images + 1):
                lo2, hi2 = j * h + m * L, (j + 1) * h + m * L
                tot += G2(hi1 - lo2) - G2(hi1 - hi2) - G2(lo1 - lo2) + G2(lo1 - hi2)
            Wm[i, j] = tot
    return Wm


def pair_weight_1d_open(n, L, k):
    """Double integral of exp(-(k/2)(x-y)^2) over two cells of an open
    (non-periodic) line: the m = 0 image of pair_weight_1d."""
    return pair_weight_1d(n, L, k, n_images=0)


def two_bead_cell_probabilities_walls(omega, n, L, k, lo, hi):
    """P[c1, c2] for a cubic grid n^3 with periodic x and y and hard walls at
    the z-cell faces lo < hi: both beads confined to z cells [lo, hi)."""
    M = n ** 3
    Wx = pair_weight_1d(n, L, k)
    Wz = pair_weight_1d_open(n, L, k)
    idx = np.array(np.unravel_index(np.arange(M), (n, n, n)))
    inside = (idx[2] >= lo) & (idx[2] < hi)
    Wpair = Wx[idx[0][:, None], idx[0][None, :]] * Wx[idx[1][:, None], idx[1][None, :]] \
        * Wz[idx[2][:, None], idx[2][None, :]]
    Wpair = Wpair * inside[:, None] * inside[None, :]
    P = np.exp(-omega[0])[:, None] * np.exp(-omega[1])[None, :] * Wpair
    return P / P.sum(), idx


def two_bead_cell_probabilities(omega, n, L, k):
    """P[c1, c2] for cubic grid n^3, linear index (ix*n + iy)*n + iz."""
    M = n ** 3
    Wx = pair_weight_1d(n, L, k)
    idx = np.array(np.unravel_index(np.arange(M), (n, n, n)))
    Wpair = Wx[idx[0][:, None], idx[0][None, :]] * Wx[idx[1][:, None], idx[1][None, :]] \
        * Wx[idx[2][:, None], idx[2][None, :]]
    P = np.exp(-omega[0])[:, None] * np.exp(-omega[1])[None, :] * Wpair
    return P / P.sum(), idx


def smart_acceptance_two_beads(A, edge, k=3.0, n=4_000_000, seed=0):
    """E[accept] of one bond-force-biased move of an N = 2 ideal chain in
    equilibrium, by numpy Monte Carlo over the bond b ~ N(0, 1/k) and the
    proposal d = A F + sqrt(2A) xi with F = -k b (F at the trial position
    -k (b + d)); displacements of 0.99 cell edges or more are rejected.
    Returns the estimate and its standard error."""
    import math

    import numpy as np
    rng = np.random.default_rng(seed)
    b = rng.normal(0.0, 1.0 / math.sqrt(k), size=(n, 3))
    xi = rng.normal(size=(n, 3))
    F = -k * b
    d = A * F + math.sqrt(2 * A) * xi
    inside = (np.abs(d) < 0.99 * edge).all(axis=1)
    b2 = b + d
    dE = 0.5 * k * ((b2 ** 2).sum(1) - (b ** 2).sum(1))
    F2 = -k * b2
    lnq = (((d - A * F) ** 2).sum(1) - ((d + A * F2) ** 2).sum(1)) / (4 * A)
    p = np.where(inside, np.minimum(1.0, np.exp(np.minimum(-dE + lnq, 0.0))), 0.0)
    return p.mean(), p.std() / math.sqrt(n)


def ideal_chain_re2_variance(Re=1.0):
    """Per-chain variance of Re^2 = |r_{N-1} - r_0|^2 for an ideal chain: the
    end-to-end vector has three independent N(0, Re^2/3) components, so
    3 Re^2/Re^2 is chi-squared with 3 degrees of freedom and
    Var(Re^2) = (Re^2/3)^2 * 2 * 3 = (2/3) Re^4."""
    return 2.0 / 3.0 * Re ** 4


def ideal_chain_rg2_moments(N, Re=1.0):
    """Exact mean and per-chain variance of Rg^2 = (1/N) sum_i |r_i - r_cm|^2
    for a discrete Gaussian chain of N beads with bond components
    N(0, s2), s2 = Re^2 / (3 (N - 1)).

    Per axis, Rg^2 is the quadratic form b^T Q b of the N-1 bond components
    b, with Q = L^T C L / N (L: bead i = sum of the bonds before it; C: the
    centring projector).  For b ~ N(0, s2 I): mean s2 tr Q, variance
    2 s2^2 tr Q^2; the three axes are independent."""
    s2 = Re ** 2 / (3.0 * (N - 1))
    L = np.tril(np.ones((N, N - 1)), -1)
    C = np.eye(N) - np.full((N, N), 1.0 / N)
    Q = L.T @ C @ L / N
    return 3.0 * s2 * np.trace(Q), 3.0 * 2.0 * s2 ** 2 * np.trace(Q @ Q)
