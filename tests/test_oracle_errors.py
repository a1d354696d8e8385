"""Pins of the oracle's standard errors Re2_err and Rg2_err.

The oracle reports, per snapshot, the mean of a per-chain quantity over the
n chains of a system and its standard error sqrt(Var/n), with Var the
variance over the chains.  Two independent checks:
  * closed forms: for ideal chains (chiN = kappaN = 0) the Gaussian-walk
    start is the exact equilibrium, and the per-chain variances of Re^2 and
    Rg^2 are known exactly (Re^2: chi-squared with three degrees of freedom,
    Var = (2/3) Re^4; Rg^2: a quadratic form of Gaussian bonds), so the
    reported errors must equal sqrt(Var/n) up to the sampling error of a
    standard deviation;
  * definition: the errors equal numpy's population standard deviation of
    the oracle's own per-chain values divided by sqrt(n).
A standard error wrong by a factor sqrt(n) (sqrt(Var)/n) or a variance that
drops the squared mean fails both.
"""
import math

import numpy as np
import pytest

from paper_2606_09356_amd import workloads as W
from tests.helpers.closed_forms import ideal_chain_re2_variance, ideal_chain_rg2_moments


def ideal_system(n_chains, N, box=16.0):
    g = int(round(box * 4))
    return W.diblock_system(n_chains, N, 0.5, 0.0, 0.0, (box, box, box), (g, g, g))


def test_rg2_closed_form_against_continuum_limit():
    # the discrete result tends to the Gaussian-coil values <Rg^2> = Re^2/6 and
    # <Rg^4>/<Rg^2>^2 = 19/15 (Debye) for long chains
    mean, var = ideal_chain_rg2_moments(2000)
    assert mean == pytest.approx((2000 + 1) / (6 * 2000), rel=1e-12)
    assert (var + mean ** 2) / mean ** 2 == pytest.approx(19 / 15, rel=2e-3)


@pytest.mark.parametrize("N", [32, 8])
def test_standard_errors_match_ideal_chain_closed_forms(orc, N):
    n_chains = 8192
    s = ideal_system(n_chains, N)
    O = orc.OracleSystem(s)
    re_err, rg_err = [], []
    for seed in range(6):
        O.set_positions(O.init_walks(seed=100 + seed))
        o = O.observables()
        re_err.append(o["Re2_err"])
        rg_err.append(o["Rg2_err"])
    re_exp = math.sqrt(ideal_chain_re2_variance() / n_chains)
    _, rg_var = ideal_chain_rg2_moments(N)
    rg_exp = math.sqrt(rg_var / n_chains)
    # the sample standard deviation of n = 8192 chi-squared-like values has a
    # relative spread of about sqrt((kurtosis - 1) / (4 n)) < 1.5 %; averaged
    # over six snapshots a 4 % band is more than five of those
    assert np.mean(re_err) == pytest.approx(re_exp, rel=0.04), (np.mean(re_err), re_exp)
    assert np.mean(rg_err) == pytest.approx(rg_exp, rel=0.04), (np.mean(rg_err), rg_exp)


def test_standard_errors_match_definition(orc):
    N, n_chains = 16, 3000
    s = ideal_system(n_chains, N)
    O = orc.OracleSystem(s)
    O.set_positions(O.init_walks(seed=5))
    O.run(seed=9, first_sweep=0, n_sweeps=3)
    o = O.observables(per_chain=True)
    re2, rg2 = o["per_chain"][0], o["per_chain"][1]
    assert o["Re2"] == pytest.approx(re2.mean(), rel=1e-13)
    assert o["Rg2"] == pytest.approx(rg2.mean(), rel=1e-13)
    assert o["Re2_err"] == pytest.approx(re2.std() / math.sqrt(n_chains), rel=1e-10)
    assert o["Rg2_err"] == pytest.approx(rg2.std() / math.sqrt(n_chains), rel=1e-10)
