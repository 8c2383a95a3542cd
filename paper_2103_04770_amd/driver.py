"""Variable-increment load driver with checkpoint / resume (Sec. 4.2).

The increments themselves run in the library (fftg_drive); this class only
keeps the driver's position -- the packed state on the device, the load
factor t and the next increment dt -- and writes it to / reads it from a
checkpoint file (numpy .npz, plain arrays only).  Because a call to
fftg_drive that starts from a position continues the run it came from, a run
interrupted after any chunk and resumed from its checkpoint accepts the same
increments and reaches the same state.

With keep_states, the driver also keeps the packed state after every accepted
increment on the device, and path_gradient() differentiates the path it took
(the accepted increments, each a converged staggered increment) in the
per-phase lengths, through every increment's history.
"""
from __future__ import annotations

import os

import numpy as np

RECORD_FIELDS = ("t", "err", "cutbacks", "stagger_iters", "newton_iters", "cg_iters",
                 "pcg_iters", "ms")


class LoadDriver:
    """Drives one RVE along the proportional path t -> target(t) = t target_end.

    solver      paper_2103_04770_amd.Solver for the RVE's grid
    phase       device uint8 tensor [N] (numpy axis order)
    table       phase dicts (see microstructure)
    options     fftg_drive keyword options (dt_min, dt_max, grow, newton_div,
                tolerances, max_stagger, ...)
    keep_states keep the packed state after every accepted increment (the
                library is then called one increment at a time) for
                path_gradient(); the states are not written to checkpoints
    """

    def __init__(self, solver, phase, table, nfields, target_end, dt=0.1, keep_states=False,
                 **options):
        import torch
        self.solver, self.phase, self.table, self.nfields = solver, phase, table, nfields
        self.target_end = tuple(np.asarray(a) for a in target_end)
        self.options = options
        shape = solver.spatial
        c = solver.c
        self.state = torch.zeros((c + 7 + 2 * nfields,) + shape, dtype=torch.float64,
                                 device="cuda")
        self.sigma = torch.zeros((c,) + shape, dtype=torch.float64, device="cuda")
        self.t = 0.0
        self.dt = float(dt)
        self.records = []
        self.reason = None
        self.keep_states = keep_states
        self.states = None       # kept packed states: where keeping began, then per increment
        self.state_t = []        # their load factors

    def run(self, t_end=1.0, chunk=None, checkpoint=None, max_attempts=1000, on_records=None):
        """Advance to t_end (or until the driver stops).  With `chunk`, the
        library is called for at most `chunk` accepted increments at a time and
        the checkpoint (if a path is given) is rewritten after every call;
        `on_records(records)` then receives each call's new records."""
        if self.keep_states:
            chunk = 1
            if self.states is None:
                self.states, self.state_t = [self.state.clone()], [self.t]
        while True:
            out = self.solver.fftg_drive(self.phase, self.table, self.nfields, self.state,
                                         self.target_end, self.sigma, t=self.t, t_end=t_end,
                                         dt=self.dt, max_attempts=max_attempts,
                                         max_records=chunk or 100000, **self.options)
            self.t, self.dt, self.reason = out["t"], out["dt"], out["reason"]
            self.records.extend(out["records"])
            if self.keep_states and out["records"]:
                self.states.append(self.state.clone())
                self.state_t.append(out["records"][-1]["t"])
            if checkpoint:
                self.save(checkpoint)
            if on_records is not None:
                on_records(out["records"])
            if out["reason"] != 3:   # not just a full record buffer
                return out["reason"]

    def targets(self):
        """Macro targets of the kept increments: t E_end on the strain-controlled
        components, t S_end on the stress-controlled ones."""
        mask, E, S = self.target_end
        return [(mask, t * E, t * S) for t in self.state_t[1:]]

    def path_gradient(self, g_sig=None, cg_tol=None, pcg_tol=None, tol=1e-8, maxit=200):
        """Gradient of J = g_sig . sigma at the last accepted increment (default
        <sigma_11>) with respect to the squared lengths, through every
        increment kept (the state where keeping began is held fixed).
        Returns (dell2 (nfields, *S) on the device, dJ/dell[j][q] per field j
        and phase q)."""
        import torch

        from . import autograd as ag
        if not self.keep_states or not self.states or len(self.states) < 2:
            raise ValueError("path_gradient needs keep_states and at least one accepted increment")
        S = self.solver.spatial
        if g_sig is None:
            g_sig = torch.zeros((self.solver.c,) + S, dtype=torch.float64, device="cuda")
            g_sig[0] = 1.0 / float(np.prod(S))
        cg_tol = self.options.get("cg_tol", 1e-8) if cg_tol is None else cg_tol
        pcg_tol = self.options.get("pcg_tol", 1e-8) if pcg_tol is None else pcg_tol
        dl, _ = ag.path_gradient(self.solver, self.phase, self.table, self.nfields, self.states,
                                 self.targets(), g_sig, cg_tol=cg_tol, pcg_tol=pcg_tol, tol=tol,
                                 maxit=maxit)
        per = []
        for j in range(self.nfields):
            sums = self.solver.fftg_phase_sums(self.phase, len(self.table), dl[j].contiguous())
            per.append([2.0 * float(t["ell"][j]) * float(v) for t, v in zip(self.table, sums)])
        return dl, per

    # ------------------------------------------------------------ checkpoints
    def save(self, path):
        """Write the position and the records so far (atomic replace)."""
        rec = {k: np.array([r[k] for r in self.records]) for k in RECORD_FIELDS}
        rec["sigma"] = np.array([r["sigma"] for r in self.records]).reshape(len(self.records), -1)
        rec["eps"] = np.array([r["eps"] for r in self.records]).reshape(len(self.records), -1)
        tmp = path + ".tmp.npz"
        np.savez(tmp, state=self.state.cpu().numpy(), sigma=self.sigma.cpu().numpy(),
                 t=np.float64(self.t), dt=np.float64(self.dt),
                 reason=np.int64(-1 if self.reason is None else self.reason),
                 **{"rec_" + k: v for k, v in rec.items()})
        os.replace(tmp, path)

    @classmethod
    def resume(cls, path, solver, phase, table, nfields, target_end, keep_states=False,
               **options):
        """A driver positioned where the checkpoint at `path` left off (kept
        states, if asked for, start from this position)."""
        import torch
        with np.load(path, allow_pickle=False) as z:
            d = cls(solver, phase, table, nfields, target_end, dt=float(z["dt"]),
                    keep_states=keep_states, **options)
            if tuple(z["state"].shape) != tuple(d.state.shape):
                raise ValueError("checkpoint state shape %s does not match the solver's %s"
                                 % (z["state"].shape, tuple(d.state.shape)))
            d.state.copy_(torch.from_numpy(z["state"]))
            d.sigma.copy_(torch.from_numpy(z["sigma"]))
            d.t = float(z["t"])
            r = int(z["reason"])
            d.reason = None if r < 0 else r
            n = len(z["rec_t"])
            d.records = [dict({k: z["rec_" + k][i].item() for k in RECORD_FIELDS},
                              sigma=z["rec_sigma"][i].copy(), eps=z["rec_eps"][i].copy())
                         for i in range(n)]
        return d
