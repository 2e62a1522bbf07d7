"""Pins of the slow-time oracle (oracle/pta.py) and host parity of the
library's slow-step arithmetic.

Oracle pins (closed forms the paper's definitions reduce to):
  - App. A, Eq. (R_m_conv) on a linear drift m_i = alpha i: R(i) = alpha (i+1)/2,
    so e(i) = k / (i+1) exactly and N_s is the first checkpoint with
    k/(i+1) < tol; on a constant series N_s = 2k; on a step series the
    running average has the closed form (c p + d (i-p)) / i.
  - batch-means standard error against the exact standard error of an AR(1)
    series, sigma_e / (1 - phi) / sqrt(n) (statistical, seeded).
  - Sec. 2.2: for a measure linear in the strain the prediction of
    Eq. (pta_pred) equals the Simpson value of Eq. (simp) (e_v = 0, every jump
    a match); for a quadratic measure A + B e + C e^2 the Simpson value is the
    exact window average, so v_d - v_pred = C d_eps_h^2; a step in the
    measure is flagged by Eq. (jump_err) exactly at the slow step that
    crosses it.
Host parity: ptamd_pta_update (C++, no GPU) against oracle.pta.pta_update on
the same inputs, bit for bit.
"""
import math

import numpy as np
import pytest

from oracle import pta as T


def _cols(m):
    m = np.asarray(m, np.float64)
    return np.stack([m, m, m, m], 1)


@pytest.mark.parametrize("lag,tol", [(10, 0.05), (7, 0.02), (100, 0.03)])
def test_linear_drift_convergence_closed_form(lag, tol):
    alpha = 0.37
    n = 4000
    s = _cols(alpha * np.arange(1, n + 1))
    idx, errs = T.conv_errors(s, lag)
    assert np.allclose(errs[:, 0], lag / (idx + 1.0), rtol=1e-12, atol=0)
    want = next(i for i in range(2 * lag, n + 1, lag) if lag / (i + 1.0) < tol)
    assert T.converged_at(s, lag, (tol, 0, 0, 0)) == want


def test_constant_and_zero_series():
    s = _cols(np.full(100, -3.5))
    assert T.converged_at(s, 10, (0.05, 0.05, 0.05, 0.05)) == 20
    z = _cols(np.zeros(100))
    # 0/0: no relative error can be formed, so the plain test never passes
    assert T.converged_at(z, 10, (0.05, 0, 0, 0)) == 0
    # with an absolute floor the error is 0 and it passes at the first check
    assert T.converged_at(z, 10, (0.05, 0, 0, 0), floor=(1.0, 0, 0, 0)) == 20


def test_step_series_closed_form():
    c, d, p, lag, n = 2.0, 3.0, 150, 25, 2000
    m = np.where(np.arange(1, n + 1) <= p, c, d)
    idx, errs = T.conv_errors(_cols(m), lag)

    def R(i):
        return c if i <= p else (c * p + d * (i - p)) / i

    for q, i in enumerate(idx):
        assert math.isclose(errs[q, 1], abs(R(i) - R(i - lag)) / abs(R(i)), rel_tol=1e-12, abs_tol=1e-15)


def test_tested_functions_only():
    n, lag = 1000, 10
    s = np.zeros((n, 4))
    s[:, 0] = 5.0                                 # converges at once
    s[:, 1] = 0.37 * np.arange(1, n + 1)         # drifts: e = k/(i+1)
    assert T.converged_at(s, lag, (0.05, 0, 0, 0)) == 20
    assert T.converged_at(s, lag, (0.05, 0.05, 0, 0)) == 200


def test_batch_se_ar1():
    """AR(1) x_t = phi x_{t-1} + e_t: the standard error of the mean of n
    samples tends to sigma_e / (1 - phi) / sqrt(n)."""
    phi, n, bs0 = 0.9, 64000, 100
    ratios = []
    for seed in range(8):
        rng = np.random.default_rng(seed)
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0] / math.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        ratios.append(T.batch_se(x, n, bs0) / (1.0 / (1 - phi) / math.sqrt(n)))
    assert abs(np.mean(ratios) - 1.0) < 0.2


def test_batch_se_doubling_rule():
    # n = 20 bs0 keeps bs0 (20 batches); one more sample doubles it (10 complete batches)
    x = np.arange(41, dtype=float)
    se20 = T.batch_se(x, 40, 2)
    se10 = T.batch_se(x, 41, 2)
    means20 = x[:40].reshape(20, 2).mean(1)
    means10 = x[:40].reshape(10, 4).mean(1)
    assert math.isclose(se20, means20.std(ddof=1) / math.sqrt(20), rel_tol=1e-12)
    assert math.isclose(se10, means10.std(ddof=1) / math.sqrt(10), rel_tol=1e-12)
    assert math.isnan(T.batch_se(x, 3, 2))


def _analytic_measure(fn):
    """A measure R(strain) without dynamics: tracks the strain only."""
    state = {"eps": 0.0}

    def measure(d):
        state["eps"] += d
        return state["eps"], np.array(fn(state["eps"]), np.float64), 123

    return measure


def test_linear_measure_always_matches():
    prm = T.PTAParams(d_eps_h=1e-3)
    meas = _analytic_measure(lambda e: [1.0 + 2.0 * e, -5.0 + 40.0 * e, 0.3 - 7.0 * e, 2.0 + e])
    st, rec = T.pta_start(meas, prm)
    d = prm.d_eps_h * prm.delta_over_h
    for _ in range(6):
        r = T.pta_jump(meas, st, prm)
        assert np.all(r.status == T.MATCH)
        assert np.all(r.e_v < 1e-12)
        # v(t) is the window average of a linear R: R at the window's midpoint
        mid = st.strain - 0.5 * d
        assert np.allclose(st.v, [1.0 + 2.0 * mid, -5.0 + 40.0 * mid, 0.3 - 7.0 * mid, 2.0 + mid], rtol=1e-12)


@pytest.mark.parametrize("C", [0.0, 3e3, -8e4])
def test_quadratic_measure_prediction_error(C):
    prm = T.PTAParams(d_eps_h=2e-3, delta_over_h=0.2, tol_v=(0, 0, 0, 0))
    A, B = 1.5, 10.0
    meas = _analytic_measure(lambda e: [A + B * e + C * e * e] * 4)
    st, _ = T.pta_start(meas, prm)
    for _ in range(4):
        v_t = st.v.copy()
        r = T.pta_jump(meas, st, prm)
        # Simpson is exact for quadratics: v_d is the exact window average
        hi = r.strains[2]
        lo = hi - prm.d_eps_h * prm.delta_over_h
        exact = A + B * (hi + lo) / 2 + C * (hi ** 3 - lo ** 3) / (3 * (hi - lo))
        assert np.allclose(r.v_d, exact, rtol=1e-10)
        assert np.allclose(r.v_d - r.v_pred, C * prm.d_eps_h ** 2, atol=1e-10 * (1 + abs(exact)))
        assert np.all(r.status != T.MATCH)  # tol_v = 0 never matches
        # with tol_v = 0 the measured value is kept
        assert np.array_equal(st.v, r.v_d)
        del v_t


def test_step_in_measure_is_flagged_as_jump():
    prm = T.PTAParams(d_eps_h=1e-3, tol_v=(0.01,) * 4, tol_j=(0.05,) * 4)
    e_star = 0.0045  # inside slow step 4 (strains 3.2e-3 .. 4.2e-3 are its runs)
    meas = _analytic_measure(lambda e: [1.0 + 5.0 * e + (0.5 if e >= e_star else 0.0)] * 4)
    st, _ = T.pta_start(meas, prm)
    statuses = []
    for _ in range(7):
        r = T.pta_jump(meas, st, prm)
        statuses.append(int(r.status[0]))
        if r.strains[2] >= e_star > r.strains[2] - prm.d_eps_h:
            hit = len(statuses) - 1
    assert statuses[:hit] == [T.MATCH] * hit
    assert statuses[hit] == T.JUMP


# ---------------------------------------------------------------------------
# host parity: the library's C++ slow step against the oracle's
# ---------------------------------------------------------------------------
def _lib():
    return pytest.importorskip("paper_2603_07321_amd")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_pta_update_matches_oracle(seed):
    P = _lib()
    rng = np.random.default_rng(seed)
    tol_v = tuple(rng.uniform(0.001, 0.05, 4))
    tol_j = tuple(rng.uniform(0.005, 0.1, 4))
    prm_o = T.PTAParams(d_eps_h=1e-3, delta_over_h=0.2, tol_v=tol_v, tol_j=tol_j)
    prm_c = P.pta_params(1e-3, 0.2, tol_v=tol_v, tol_j=tol_j)
    base = np.array([2000.0, -17000.0, 0.5, 0.3])
    R0 = base * (1 + 0.01 * rng.standard_normal((3, 4)))
    st_o = T.PTAState(strain=0.0, R_tmd=R0[0], R_tmh=R0[1], R_t=R0[2], R_prev=None, v=T.simpson(*R0))
    st_c = P.PTAState()
    st_c.R_tmd[:] = list(R0[0]); st_c.R_tmh[:] = list(R0[1]); st_c.R_t[:] = list(R0[2])
    st_c.R_prev[:] = [float("nan")] * 4
    st_c.v[:] = list(T.simpson(*R0))
    eps = 0.0
    for j in range(8):
        # smooth drift, occasionally a large step (a "jump")
        scale = 1 + 0.002 * j + (0.2 if j in (3, 6) else 0.0) * rng.choice([-1, 1], 4)
        R = base * scale * (1 + 0.004 * rng.standard_normal((3, 4)))
        strains = [eps + 8e-4, eps + 9e-4, eps + 1e-3]
        eps += 1e-3
        ns = [100 * (j + 1), 200, 300]
        ro = T.pta_update(st_o, prm_o, strains, R, ns)
        rc = P.pta_update(prm_c, st_c, R, strains, ns)
        for k in ("v_pred", "v_d", "v", "e_v", "e1"):
            assert np.array_equal(getattr(ro, k), rc[k]), (j, k)
        if j > 0:
            assert np.array_equal(ro.e2, rc["e2"])
        assert np.array_equal(ro.status, rc["status"]), j
        assert np.array_equal(st_o.v, np.array(list(st_c.v)))
        assert np.array_equal(st_o.jump_at_t, np.array(list(st_c.jump_at_t), bool))
        assert list(rc["n_steps"]) == ns and st_c.n_jumps == j + 1
        assert st_c.strain == strains[2]


def test_pta_update_rejects_bad_params():
    P = _lib()
    st = P.PTAState()
    for bad in (P.pta_params(0.2), P.pta_params(1e-3, delta_over_h=0.0), P.pta_params(1e-3, delta_over_h=1.5)):
        with pytest.raises(P.PtamdError) as ei:
            P.pta_update(bad, st, np.ones(12), [0, 0, 0], [0, 0, 0])
        assert ei.value.name == "PTAMD_EINVAL"
