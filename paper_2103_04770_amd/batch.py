"""Batches of independent RVEs (fftg_batch_step).

Each RVE gets its own Solver on its own HIP stream (default priority), its
own device state and stress; one call advances every RVE by one staggered
increment.  RVEs of one grid (and precision, field count and macro mask) run
as one lockstep class on the first one's handle, each Krylov iteration one
set of launches over all of them; the library's worker threads drive
several classes at once so that their kernels overlap on the GPU.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from .binding import (BatchItem, FFTGError, KrylovOpts, Solver, _macro, load_library, phase_table,
                      FP64)


class RVEBatch:
    """rves: list of dicts with shape (numpy order), phase (uint8 array),
    table, nfields (see microstructure.batch_workload)."""

    def __init__(self, rves, prec=FP64):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.rves = rves
        self.solvers, self.states, self.sigmas, self.phases, self.tabs = [], [], [], [], []
        for r in rves:
            shape, J = tuple(r["shape"]), r["nfields"]
            st = torch.cuda.Stream()
            s = Solver(tuple(reversed(shape)), prec=prec, stream=st)
            self.solvers.append(s)
            self.states.append(torch.zeros((s.c + 7 + 2 * J,) + shape, dtype=torch.float64,
                                           device="cuda"))
            self.sigmas.append(torch.zeros((s.c,) + shape, dtype=torch.float64, device="cuda"))
            self.phases.append(torch.from_numpy(np.ascontiguousarray(r["phase"])).cuda())
            self.tabs.append(phase_table(r["table"]))
        torch.cuda.synchronize()

    def reset(self):
        for t in self.states:
            t.zero_()
        self.torch.cuda.synchronize()

    def step(self, targets, nworkers=8, cg_tol=1e-8, cg_maxit=5000, pcg_tol=1e-8,
             pcg_maxit=2000, newton_tol=1e-8, newton_maxit=50, stagger_tol=1e-6, max_stagger=20,
             strict=True):
        """One staggered increment of every RVE; targets: one (mask, E, S) per
        RVE, or a single one for all.  Returns per-RVE dicts (stats, converged,
        sigma_mean, eps_mean, status).  strict: raise FFTGError when an RVE
        failed (else its dict holds the status and the error text)."""
        n = len(self.rves)
        if not isinstance(targets, list):
            targets = [targets] * n
        items = (BatchItem * max(n, 1))()
        for i in range(n):
            it = items[i]
            it.h = self.solvers[i].h
            it.phase = self.phases[i].data_ptr()
            it.tab = self.tabs[i]
            it.nphase = len(self.rves[i]["table"])
            it.nfields = self.rves[i]["nfields"]
            it.state = self.states[i].data_ptr()
            it.target = _macro(targets[i])
            it.sigma_out = self.sigmas[i].data_ptr()
        self.torch.cuda.synchronize()   # inputs written on torch's stream
        rc = self.lib.fftg_batch_step(items, n, int(nworkers), ct.byref(KrylovOpts(cg_tol, cg_maxit)),
                                      ct.byref(KrylovOpts(pcg_tol, pcg_maxit)), float(newton_tol),
                                      int(newton_maxit), float(stagger_tol), int(max_stagger))
        out = []
        for i in range(n):
            it = items[i]
            if it.status < 0:
                msg = self.lib.fftg_last_error(self.solvers[i].h).decode()
                if strict:
                    raise FFTGError(it.status, msg)
                out.append(dict(status=it.status, error=msg, converged=False))
                continue
            c = self.solvers[i].c
            d = it.stats.as_dict()
            d["converged"] = it.status == 0
            d["status"] = it.status
            d["sigma_mean"] = np.array(it.homog_out[:c])
            d["eps_mean"] = np.array(it.homog_out[6:6 + c])
            out.append(d)
        if rc < 0 and strict:
            raise FFTGError(rc, "batch step failed")
        return out

    def close(self):
        for s in self.solvers:
            s.close()
