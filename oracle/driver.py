"""Adaptive load driver around the staggered increment (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper loads the RVE incrementally with a variable strain increment:
larger steps while the response is smooth, smaller ones once softening sets
in, and a smallest admissible increment of Delta E11 = 1e-5 below which an
analysis is stopped.  It does not spell out the control rule; the reading
used here is:

  * the macro target is proportional to a load factor t in [0, 1]:
    E(t) = t E_end on the strain-controlled components, S(t) = t S_end on the
    stress-controlled ones (mask from the end target);
  * an attempt from t to t' = t + dt (t' = t_end exactly when dt reaches past
    it) runs one staggered increment (staggered.staggered_step) with the
    Newton divergence guard and abort-on-failure switched on;
  * the increment is accepted when the staggered error met its tolerance and
    every inner solve of the last pass (the mechanics and each Helmholtz
    PCG) converged; then t <- t', dt <- min(grow dt, dt_max);
  * otherwise the state is restored, dt <- dt / 2, and the driver stops once
    dt < dt_min (reason 1);
  * it also stops after max_attempts attempts (reason 2) or max_records
    accepted increments (reason 3); reason 0 means t_end was reached.

The driver's position is (state, t, dt): a run split in two calls that carry
them over is the same run (checkpoint / resume).
"""
from __future__ import annotations

import copy

import numpy as np

from . import staggered

REACHED, FLOOR, ATTEMPTS, RECORDS = 0, 1, 2, 3


def target_at(target_end, t):
    """Proportional macro target at load factor t."""
    mask, E, S = target_end
    return (np.asarray(mask), t * np.asarray(E, dtype=np.float64),
            t * np.asarray(S, dtype=np.float64))


def drive(phase, table, nfields, state, target_end, t0=0.0, t_end=1.0, dt=0.1,
          dt_min=1e-5, dt_max=1.0, grow=1.5, max_attempts=1000, max_records=1000,
          newton_div=3, step=None, **tols):
    """Advance `state` (staggered.initial_state layout) from load factor t0
    towards t_end.  `step(state, target)` -> (new_state, homog, stats) may
    replace the staggered increment (tests of the control rule); by default
    it is staggered.staggered_step with **tols.

    Returns dict(state, t, dt, reason, records) with one record per accepted
    increment: dict(t, sigma, eps, cutbacks, stagger_iters, newton_iters,
    cg_iters, pcg_iters, err)."""
    if step is None:
        def step(st, tgt):
            ns, _, hom, stats = staggered.staggered_step(
                phase, table, nfields, st, tgt, newton_div=newton_div,
                abort_on_mech_failure=True, **tols)
            return ns, hom, stats
    t = float(t0)
    records = []
    attempts = 0
    cut = 0
    reason = REACHED
    while t < t_end:
        if len(records) >= max_records:
            reason = RECORDS
            break
        if attempts >= max_attempts:
            reason = ATTEMPTS
            break
        tn = t_end if dt >= t_end - t else t + dt
        attempts += 1
        new_state, hom, stats = step(copy.deepcopy(state), target_at(target_end, tn))
        if stats["converged"] and stats.get("inner_converged", stats["mech_converged"]):
            state = new_state
            t = tn
            records.append(dict(t=t, sigma=np.asarray(hom["sigma"]), eps=np.asarray(hom["eps"]),
                                cutbacks=cut, stagger_iters=stats["stagger_iters"],
                                newton_iters=stats["newton_iters"], cg_iters=stats["cg_iters"],
                                pcg_iters=stats["pcg_iters"], err=stats["err"]))
            cut = 0
            dt = min(dt * grow, dt_max)
        else:
            cut += 1
            dt = dt / 2.0
            if dt < dt_min:
                reason = FLOOR
                break
    return dict(state=state, t=t, dt=dt, reason=reason, records=records)
