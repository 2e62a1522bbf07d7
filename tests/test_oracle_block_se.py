"""Pins of the oracle's burst standard error (the 20-batch estimate behind the
agreement bar |delta| <= 3 sqrt(SE1^2 + SE2^2) for burst averages), against
values fixed by construction rather than by the formula itself:

  - a series that is constant within each batch: the batch means are known
    exactly, so the estimate is the textbook standard error of 20 numbers;
  - samples past the last whole batch are ignored;
  - an i.i.d. series: the estimate scatters around sigma / sqrt(n) with the
    spread of a chi distribution with 19 degrees of freedom;
  - an AR(1) series: the estimate approaches the exact long-run standard
    error sigma_e / (1 - phi) / sqrt(n), which the naive i.i.d. formula
    misses by a factor ~ sqrt((1 + phi) / (1 - phi));
  - fewer than 20 samples: undefined (NaN).
"""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def test_batch_constant_series_closed_form(orc):
    # batch b holds 7 copies of b: batch means 0..19, grand mean 9.5,
    # sum of squared deviations 665, SE = sqrt(665 / (20 * 19)) = sqrt(1.75)
    x = np.repeat(np.arange(20.0), 7)
    assert orc.block_se(x) == pytest.approx(math.sqrt(1.75), rel=1e-14)
    # shifting and scaling the series: SE scales with |scale| only
    assert orc.block_se(3.0 - 2.5 * x) == pytest.approx(2.5 * math.sqrt(1.75), rel=1e-13)


def test_samples_beyond_the_last_batch_are_ignored(orc):
    x = np.repeat(np.arange(20.0), 5)
    tail = np.array([1e6, -3e5, 7.0])  # 103 samples: batches of 5, the last 3 unused
    assert orc.block_se(np.concatenate([x, tail])) == pytest.approx(math.sqrt(1.75), rel=1e-14)


def test_two_valued_batches(orc):
    # 19 batches of zeros and one of ones: means (0 x 19, 1), mean 1/20,
    # sum of squares 19/400 + 361/400 = 0.95, SE = sqrt(0.95 / 380) = 0.05
    x = np.zeros(200)
    x[130:140] = 1.0
    assert orc.block_se(x) == pytest.approx(0.05, rel=1e-13)


def test_iid_series_matches_sigma_over_sqrt_n(orc):
    rng = synth.rng(11)
    n, sigma = 20000, 2.0
    ratios = []
    for _ in range(40):
        ratios.append(orc.block_se(rng.normal(0.0, sigma, n)) / (sigma / math.sqrt(n)))
    r = np.array(ratios)
    # each ratio ~ chi_19 / sqrt(19): mean ~0.987, sd ~0.161; the mean of 40
    # has sd ~0.026
    assert abs(r.mean() - 0.987) < 0.1
    assert 0.08 < r.std() < 0.26


def test_ar1_series_long_run_error(orc):
    rng = synth.rng(12)
    phi, se_e, n = 0.9, 1.0, 200000
    exact = se_e / (1.0 - phi) / math.sqrt(n)
    vals = []
    for _ in range(12):
        e = rng.normal(0.0, se_e, n)
        x = np.empty(n)
        x[0] = e[0] / math.sqrt(1 - phi * phi)
        for k in range(1, n):
            x[k] = phi * x[k - 1] + e[k]
        vals.append(orc.block_se(x) / exact)
    v = np.array(vals)
    assert abs(v.mean() - 1.0) < 0.12
    naive = np.std(x) / math.sqrt(n)
    assert orc.block_se(x) > 2.5 * naive  # the batches see the correlation


def test_too_few_samples(orc):
    assert math.isnan(orc.block_se(np.arange(19.0)))


def test_burst_uses_block_se_on_its_series(orc):
    """run_burst's standard errors are this estimate applied to its own
    K, U and sigma_zz columns."""
    x, y, z, g, _ = orc.fcc_cube(4, 4.05, True)
    vx, vy, vz = orc.mb_velocities(g, 300.0, 3)
    st = orc.State(x, y, z, vx, vy, vz, g, 4 ** 3 * 4.05 ** 3, (4 * 4.05) ** 2)
    avg, ser = orc.run_burst(st, orc.sc_params(), orc.md_params(), 60, series=True)
    assert avg["ke_se"] == orc.block_se(ser[:, 0])
    assert avg["pe_se"] == orc.block_se(ser[:, 1])
    assert avg["szz_se"] == orc.block_se(ser[:, 2])
