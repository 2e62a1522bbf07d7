"""FP64 oracle of the slow-time layer of Practical Time Averaging.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the tests, the smoke
check and the benchmark's CPU-baseline leg use it; the product library never
imports it and it never imports the product library.

What it computes, in the paper's order and notation:

* ``converged_at`` -- App. A, Eq. (R_m_conv): running time averages
  R(i) = (1/i) sum_{r<=i} m_r of each state function, checked at the
  checkpoints i = k, 2k, ... against R(i-k); converged at the first i with
  |R(i) - R(i-k)| / |R(i)| < tol_m for every tested function.
* ``run_until_converged`` -- Sec. 2.2 Step 1 / Eq. (R_m_t): an averaging
  burst of the oracle MD whose length N_t is set by that test (at most
  N_max steps), returning R and the state after sample N_t (x^conv of Step 4).
* ``batch_se`` -- the standard error reported beside each average (not a
  quantity of the paper; the batch-means definition stated at the function).
* ``simpson``, ``rate``, ``predict``, ``rel_err``, ``jump_test`` -- Eqs.
  (simp), (dvdt_algo), (pta_pred), (rel_err), (jump_err) of Sec. 2.2.
* ``pta_start`` / ``pta_jump`` -- Sec. 2.2 Steps 1-4 with the loading
  sequence of Sec. 2.4.2: three converged runs per slow step at
  t+h-Delta, t+h-Delta/2, t+h, each started from the converged state of the
  run before it (Eq. (x_guess_step3)), so one state carries through the
  whole sequence.

Readings where the paper is silent (each restated where it is used):
  R1. Checks happen at multiples of the lag k only, from 2k on (R(i-k) needs
      i-k >= k samples in a check window of k); the paper gives no k.
  R2. The denominator of the convergence error may be bounded below by a
      per-function floor (default 0, the plain relative error).
  R3. Slow time is measured by the applied strain: the first run is at the
      system's current strain (slow time t0 = -Delta), slow time tau is at
      strain eps0 + (tau + Delta) * d_eps_h / h.
  R4. v at the first slow time t = 0 is the Simpson value of the first
      triple (the H-observable over [t-Delta, t]).
  R5. When neither the match (Eq. rel_err) nor a jump (Eq. jump_err) holds,
      the measured value v_d is kept and the step is flagged "neither".
  R6. At the first jump there is no R(t-h); the jump test then takes its
      second form e1 >= tol_j, as after a detected jump.
  R7. Every error is evaluated in IEEE FP64 exactly as written (a division
      by zero gives inf; a NaN comparison is false).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

# state functions carried by every average, in this order
FUNCS = ("K", "U", "szz", "tz")
_SER_COL = {"K": 0, "U": 1, "szz": 2, "tz": 5}  # columns of the oracle MD series

NO_TEST, MATCH, JUMP, NEITHER = -1, 0, 1, 2


# ---------------------------------------------------------------------------
# App. A: convergence of running time averages
# ---------------------------------------------------------------------------
def conv_errors(samples: np.ndarray, lag: int, floor: Sequence[float] = (0.0, 0.0, 0.0, 0.0)):
    """e^m(i) of Eq. (R_m_conv) at the checkpoints i = 2k, 3k, ... <= len.

    samples: (n, 4) array of K, U, sigma_zz, T_z per step.  Returns
    (checkpoints, errors (len(checkpoints), 4)).  Running sums are plain
    sequential FP64 sums."""
    s = np.asarray(samples, np.float64)
    n = s.shape[0]
    csum = np.cumsum(s, axis=0)  # sequential accumulation, row by row
    idx = np.arange(2 * lag, n + 1, lag)
    errs = np.zeros((len(idx), 4))
    for q, i in enumerate(idx):
        ri = csum[i - 1] / i
        rk = csum[i - lag - 1] / (i - lag)
        den = np.maximum(np.abs(ri), np.asarray(floor, np.float64))
        with np.errstate(divide="ignore", invalid="ignore"):
            errs[q] = np.abs(ri - rk) / den
    return idx, errs


def converged_at(samples: np.ndarray, lag: int, tol: Sequence[float],
                 floor: Sequence[float] = (0.0, 0.0, 0.0, 0.0)) -> int:
    """First checkpoint N_s at which every tested function (tol > 0) has
    e < tol (R1, R2); 0 when none does within the samples."""
    idx, errs = conv_errors(samples, lag, floor)
    tested = [f for f in range(4) if tol[f] > 0]
    for q, i in enumerate(idx):
        if all(errs[q, f] < tol[f] for f in tested):
            return int(i)
    return 0


def batch_se(col: np.ndarray, n: int, bs0: int) -> float:
    """Batch-means standard error of the mean of col[:n]: batches of
    bs = bs0 * 2^d samples, d the smallest with n <= 20 bs (a batch length
    that starts at bs0 and doubles whenever 20 batches are full); only the
    complete batches, nb = n // bs of them, enter:
        SE = sqrt( sum_b (mean_b - mean)^2 / (nb (nb - 1)) ),  NaN if nb < 2."""
    bs = bs0
    while n > 20 * bs:
        bs *= 2
    nb = n // bs
    if nb < 2:
        return float("nan")
    means = np.array([np.mean(col[b * bs:(b + 1) * bs]) for b in range(nb)])
    return float(np.sqrt(np.sum((means - means.mean()) ** 2) / (nb * (nb - 1))))


def run_until_converged(st, sc, md, lag: int, n_max: int, tol: Sequence[float],
                        floor: Sequence[float] = (0.0, 0.0, 0.0, 0.0)):
    """Sec. 2.2 Step 1: run the oracle MD from ``st`` (advanced in place)
    until the running averages converge (App. A), at most n_max steps.

    Runs in sub-bursts that end at the checkpoints (the MD oracle recomputes
    forces from the positions at each burst start, so the trajectory is the
    same as one long burst).  Returns (R dict over samples 1..N, N_s or 0,
    series (N, 6))."""
    from . import run_burst
    rows: List[np.ndarray] = []
    done = 0
    ns = 0
    while done < n_max:
        n = min(lag - done % lag, n_max - done)
        _, ser = run_burst(st, sc, md, n, series=True)
        rows.append(ser)
        done += n
        if done % lag == 0 and done >= 2 * lag:
            ser_all = np.concatenate(rows)
            smp = ser_all[:, [_SER_COL[f] for f in FUNCS]]
            idx, errs = conv_errors(smp, lag, floor)
            last = errs[-1]
            if all(last[f] < tol[f] for f in range(4) if tol[f] > 0):
                ns = done
                break
    ser_all = np.concatenate(rows)
    n = ser_all.shape[0]
    R = {f: float(np.sum(ser_all[:, _SER_COL[f]]) / n) for f in FUNCS}
    R["T"] = float(np.sum(ser_all[:, 3]) / n)
    bs0 = max(1, lag // 10)
    R["ke_se"] = batch_se(ser_all[:, 0], n, bs0)
    R["pe_se"] = batch_se(ser_all[:, 1], n, bs0)
    R["szz_se"] = batch_se(ser_all[:, 2], n, bs0)
    R["n_samples"] = n
    return R, ns, ser_all


# ---------------------------------------------------------------------------
# Sec. 2.2: the PTA slow-time step
# ---------------------------------------------------------------------------
def simpson(ra, rb, rc):
    """Eq. (simp): v_d = (R(t+h-Delta) + 4 R(t+h-Delta/2) + R(t+h)) / 6."""
    return (np.asarray(ra) + 4.0 * np.asarray(rb) + np.asarray(rc)) / 6.0


def rate(r_t, r_tmd, delta):
    """Eq. (dvdt_algo): dv/dt(t) = (R_t - R_{t-Delta}) / Delta."""
    return (np.asarray(r_t) - np.asarray(r_tmd)) / delta


def predict(v_t, dvdt, h):
    """Eq. (pta_pred): v(t+h) = v(t) + h dv/dt(t)."""
    return np.asarray(v_t) + h * np.asarray(dvdt)


def rel_err(v_pred, v_d):
    """Eq. (rel_err): |(v(t+h) - v_d(t+h)) / v_d(t+h)| (R7)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs((np.asarray(v_pred) - np.asarray(v_d)) / np.asarray(v_d))


def jump_test(r_th, r_t, r_tmh, tol_j, jump_at_t):
    """Eq. (jump_err), per state function: e1 = |(R_{t+h} - R_t)/R_t|,
    e2 = |(R_t - R_{t-h})/R_{t-h}|; a jump at t+h if |e1/e2 - 1| >= tol_j, or,
    when a jump was detected at t (or there is no R_{t-h}: r_tmh is None, R6),
    if e1 >= tol_j.  Returns (jump flags, e1, e2)."""
    r_th, r_t = np.asarray(r_th, np.float64), np.asarray(r_t, np.float64)
    tol_j = np.asarray(tol_j, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        e1 = np.abs((r_th - r_t) / r_t)
        if r_tmh is None:
            e2 = np.full_like(e1, np.nan)
        else:
            r_tmh = np.asarray(r_tmh, np.float64)
            e2 = np.abs((r_t - r_tmh) / r_tmh)
        ratio = np.abs(e1 / e2 - 1.0)
    second = np.asarray(jump_at_t, bool) | (r_tmh is None)
    jump = np.where(second, e1 >= tol_j, ratio >= tol_j)
    return jump, e1, e2


@dataclass
class PTAParams:
    d_eps_h: float                 # strain advanced per slow jump h (strain rate x h)
    delta_over_h: float = 0.2      # Table 1: Delta = h / 5
    tol_v: Tuple[float, ...] = (0.01, 0.05, 0.01, 0.01)  # Table 1 acceptance: K 1%, U 5%, reaction 1%
    tol_j: Tuple[float, ...] = (0.08, 0.01, 0.05, 0.05)  # Table 1 jump: K 8%, U 1%, reaction 5%


@dataclass
class PTAState:
    strain: float                  # strain at slow time t
    R_tmd: np.ndarray              # R(t - Delta)
    R_tmh: np.ndarray              # R(t - Delta/2)
    R_t: np.ndarray                # R(t)
    R_prev: Optional[np.ndarray]   # R(t - h), None before the first jump
    v: np.ndarray                  # slow variables v(t)
    jump_at_t: np.ndarray = field(default_factory=lambda: np.zeros(4, bool))
    n_jumps: int = 0


@dataclass
class PTARecord:
    strains: Tuple[float, float, float]
    R: np.ndarray                  # (3, 4) converged averages of the three runs
    n_steps: Tuple[int, int, int]
    v_pred: np.ndarray = None
    v_d: np.ndarray = None
    v: np.ndarray = None
    e_v: np.ndarray = None
    e1: np.ndarray = None
    e2: np.ndarray = None
    status: np.ndarray = None


def _triple(measure: Callable, d_first: float, d_half: float):
    """Three converged runs: strain += d_first, run; += d_half, run; += d_half, run.
    ``measure(d_eps)`` applies the increment, runs to convergence from the
    current state and returns (strain, R[4], N_s)."""
    outs = [measure(d_first), measure(d_half), measure(d_half)]
    strains = tuple(o[0] for o in outs)
    R = np.array([o[1] for o in outs], np.float64)
    ns = tuple(int(o[2]) for o in outs)
    return strains, R, ns


def pta_start(measure: Callable, prm: PTAParams) -> Tuple[PTAState, PTARecord]:
    """The runs at t-Delta, t-Delta/2 and t = 0 (Sec. 2.4.2 steps 1-3), the
    first at the current strain (R3); v(0) is their Simpson value (R4)."""
    d_delta = prm.d_eps_h * prm.delta_over_h
    strains, R, ns = _triple(measure, 0.0, 0.5 * d_delta)
    v = simpson(R[0], R[1], R[2])
    st = PTAState(strain=strains[2], R_tmd=R[0], R_tmh=R[1], R_t=R[2], R_prev=None, v=v)
    rec = PTARecord(strains, R, ns, v_d=v, v=v, status=np.full(4, NO_TEST))
    return st, rec


def pta_update(st: PTAState, prm: PTAParams, strains, R: np.ndarray, ns) -> PTARecord:
    """Steps 1-3 of Sec. 2.2 given the three new converged averages R[0..2] at
    t+h-Delta, t+h-Delta/2, t+h; advances ``st`` from t to t+h."""
    h = 1.0
    delta = prm.delta_over_h * h
    dvdt = rate(st.R_t, st.R_tmd, delta)          # Step 1
    v_pred = predict(st.v, dvdt, h)               # Step 2
    v_d = simpson(R[0], R[1], R[2])               # Step 3
    e_v = rel_err(v_pred, v_d)
    jump, e1, e2 = jump_test(R[2], st.R_t, st.R_prev, prm.tol_j, st.jump_at_t)
    match = e_v < np.asarray(prm.tol_v)
    status = np.where(match, MATCH, np.where(jump, JUMP, NEITHER))
    v_new = np.where(match, v_pred, v_d)          # R5: v_d unless matched
    rec = PTARecord(tuple(strains), np.array(R), tuple(ns), v_pred=v_pred, v_d=v_d, v=v_new, e_v=e_v, e1=e1,
                    e2=e2, status=status)
    st.R_prev = st.R_t
    st.R_tmd, st.R_tmh, st.R_t = R[0], R[1], R[2]
    st.v = v_new
    st.jump_at_t = status == JUMP
    st.strain = strains[2]
    st.n_jumps += 1
    return rec


def pta_jump(measure: Callable, st: PTAState, prm: PTAParams) -> PTARecord:
    """One slow step t -> t+h: the runs at t+h-Delta, t+h-Delta/2, t+h, each
    started from the converged state of the run before (Eq. (x_guess_step3)),
    then the prediction, the Simpson measure and the tests."""
    d_delta = prm.d_eps_h * prm.delta_over_h
    strains, R, ns = _triple(measure, prm.d_eps_h - d_delta, 0.5 * d_delta)
    return pta_update(st, prm, strains, R, ns)


def md_measure(state, sc, md, lag: int, n_max: int, tol, floor=(0.0, 0.0, 0.0, 0.0)):
    """A ``measure`` backed by the oracle MD: affine strain increment of the
    carried state, then a run until the averages converge."""
    from . import apply_strain

    def measure(d_eps: float):
        if d_eps != 0.0:
            apply_strain(state, d_eps)
        R, ns, _ = run_until_converged(state, sc, md, lag, n_max, tol, floor)
        return state.strain, np.array([R[f] for f in FUNCS]), ns

    return measure
