"""Variable-increment load driver with checkpoint / resume (Sec. 4.2).

The increments themselves run in the library (fftg_drive); this class only
keeps the driver's position -- the packed state on the device, the load
factor t and the next increment dt -- and writes it to / reads it from a
checkpoint file (numpy .npz, plain arrays only).  Because a call to
fftg_drive that starts from a position continues the run it came from, a run
interrupted after any chunk and resumed from its checkpoint accepts the same
increments and reaches the same state.
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
    """

    def __init__(self, solver, phase, table, nfields, target_end, dt=0.1, **options):
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

    def run(self, t_end=1.0, chunk=None, checkpoint=None, max_attempts=1000, on_records=None):
        """Advance to t_end (or until the driver stops).  With `chunk`, the
        library is called for at most `chunk` accepted increments at a time and
        the checkpoint (if a path is given) is rewritten after every call;
        `on_records(records)` then receives each call's new records."""
        while True:
            out = self.solver.fftg_drive(self.phase, self.table, self.nfields, self.state,
                                         self.target_end, self.sigma, t=self.t, t_end=t_end,
                                         dt=self.dt, max_attempts=max_attempts,
                                         max_records=chunk or 100000, **self.options)
            self.t, self.dt, self.reason = out["t"], out["dt"], out["reason"]
            self.records.extend(out["records"])
            if checkpoint:
                self.save(checkpoint)
            if on_records is not None:
                on_records(out["records"])
            if out["reason"] != 3:   # not just a full record buffer
                return out["reason"]

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
    def resume(cls, path, solver, phase, table, nfields, target_end, **options):
        """A driver positioned where the checkpoint at `path` left off."""
        import torch
        with np.load(path, allow_pickle=False) as z:
            d = cls(solver, phase, table, nfields, target_end, dt=float(z["dt"]), **options)
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
