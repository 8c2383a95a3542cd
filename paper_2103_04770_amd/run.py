"""One JSON configuration for a loading run, and a JSON-lines log per accepted
increment.

    python -m paper_2103_04770_amd.run config.json

The configuration (RunConfig) names a workload of the input generator
(microstructure.workload), optional per-phase overrides of its table, the
macroscopic target at the end of the path (uniaxial E11 with the other
stresses zero, or an explicit mask / E / S), the precision and derivative
scheme, the Krylov / Newton / staggered tolerances and the adaptive driver's
options.  The run goes through LoadDriver (the library's fftg_drive), so it
can checkpoint and resume.  Every accepted increment appends one line to the
log: load factor, <sigma>, <eps>, iteration counts, staggered error, cutbacks,
wall time, and the algorithmic bytes one Galerkin CG and one Helmholtz PCG
iteration move on this grid.  With "gradient": true the driver keeps every
increment's state and a last line gives d<sigma_11>/d ell per field and phase
at the end of the path, through every increment of the run.
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
from typing import Optional

import numpy as np


@dataclasses.dataclass
class RunConfig:
    workload: str = "spheres64_20"
    seed: Optional[int] = None
    table_overrides: list = dataclasses.field(default_factory=list)  # per phase: dict of keys
    e11_end: Optional[float] = 0.05          # uniaxial mixed control ...
    target: Optional[dict] = None            # ... or {"mask": [...], "E": [...], "S": [...]}
    precision: str = "fp64"                  # "fp64" | "fp32_refined"
    scheme: str = "rotated"                  # "rotated" | "spectral"
    tolerances: dict = dataclasses.field(default_factory=lambda: dict(
        cg_tol=1e-8, pcg_tol=1e-8, newton_tol=1e-8, stagger_tol=1e-6, max_stagger=20))
    driver: dict = dataclasses.field(default_factory=lambda: dict(
        dt=0.02, dt_min=2e-4, dt_max=1.0, grow=1.5, newton_div=3))
    t_end: float = 1.0
    max_attempts: int = 1000
    log: str = "run.jsonl"
    checkpoint: Optional[str] = None
    chunk: int = 1
    gradient: bool = False                   # d<sigma_11>/d ell through the run at its end

    @classmethod
    def from_json(cls, path_or_text):
        text = path_or_text
        if os.path.exists(path_or_text):
            with open(path_or_text) as f:
                text = f.read()
        d = json.loads(text)
        unknown = set(d) - {f.name for f in dataclasses.fields(cls)}
        if unknown:
            raise ValueError("unknown configuration keys: %s" % sorted(unknown))
        return cls(**d)

    def to_json(self):
        return json.dumps(dataclasses.asdict(self), indent=1, sort_keys=True)

    def target_tuple(self, ndim):
        from . import microstructure as ms
        if self.target is not None:
            c = 6 if ndim == 3 else 3
            return (np.asarray(self.target["mask"], np.uint8)[:c],
                    np.asarray(self.target["E"], np.float64)[:c],
                    np.asarray(self.target["S"], np.float64)[:c])
        if self.e11_end is None:
            raise ValueError("give e11_end or target")
        return ms.uniaxial_mixed(ndim, self.e11_end)


def bytes_per_iteration(shape, prec):
    """Algorithmic bytes of one Galerkin CG iteration (c = 6 or 3 components)
    and one Helmholtz PCG iteration on this grid: every fused pass reads its
    inputs once and writes its outputs once (half-spectrum Krylov vectors)."""
    ndim = len(shape)
    c = 6 if ndim == 3 else 3
    N = int(np.prod(shape))
    Ns = N // shape[-1] * (shape[-1] // 2 + 1)
    z = 16 if prec == "fp64" else 8
    r = z // 2
    inner = ndim == 3                     # y passes exist only in 3D (outer axis: z)
    # x fused (2c z + tangent), y inverse and forward (2c each), outer
    # direction/inverse (6c), outer forward/dot (3c), residual (3c)
    gal = (14 + (4 if inner else 0)) * c * Ns * z + 8 * N * r
    # x fused (2d z + ell2); 3D: y inverse and forward (2 + d each), outer
    # direction/inverse (5 + 2) and divergence/dot (2 + 2), the outer passes
    # transforming two fields; 2D: outer (5 + d) and (d + 2); residual (3)
    if inner:
        helm = (2 * ndim + 2 * (2 + ndim) + 7 + 4 + 3) * Ns * z + N * r
    else:
        helm = (2 * ndim + (5 + ndim) + (ndim + 2) + 3) * Ns * z + N * r
    return gal, helm


def run(cfg: RunConfig):
    """Run the configured path; returns (reason, number of logged increments)."""
    import torch

    from . import FP32_REFINED, FP64, ROTATED, SPECTRAL, Solver, microstructure as ms
    from .driver import LoadDriver
    w = ms.workload(cfg.workload, seed=cfg.seed)
    table = [dict(t) for t in w["table"]]
    for q, o in enumerate(cfg.table_overrides):
        table[q].update(o)
    shape, J = w["shape"], w["nfields"]
    prec = {"fp64": FP64, "fp32_refined": FP32_REFINED}[cfg.precision]
    scheme = {"rotated": ROTATED, "spectral": SPECTRAL}[cfg.scheme]
    solver = Solver(tuple(reversed(shape)), prec=prec, scheme=scheme)
    phase = torch.from_numpy(w["phase"]).cuda()
    tgt = cfg.target_tuple(len(shape))
    opts = dict(cfg.driver)
    dt = opts.pop("dt", 0.02)
    opts.update(cfg.tolerances)
    if cfg.checkpoint and os.path.exists(cfg.checkpoint):
        drv = LoadDriver.resume(cfg.checkpoint, solver, phase, table, J, tgt,
                                keep_states=cfg.gradient, **opts)
    else:
        drv = LoadDriver(solver, phase, table, J, tgt, dt=dt, keep_states=cfg.gradient, **opts)
    gal_b, helm_b = bytes_per_iteration(shape, cfg.precision)
    n0 = len(drv.records)
    with open(cfg.log, "a" if n0 else "w") as log:
        def write(records):
            for rec in records:
                line = dict(workload=cfg.workload, t=rec["t"],
                            sigma=[float(v) for v in rec["sigma"]],
                            eps=[float(v) for v in rec["eps"]],
                            newton_iters=int(rec["newton_iters"]), cg_iters=int(rec["cg_iters"]),
                            pcg_iters=int(rec["pcg_iters"]),
                            stagger_iters=int(rec["stagger_iters"]), err=float(rec["err"]),
                            cutbacks=int(rec["cutbacks"]), ms=float(rec["ms"]),
                            galerkin_bytes_per_iter=gal_b, helmholtz_bytes_per_iter=helm_b)
                log.write(json.dumps(line) + "\n")
            log.flush()

        drv.run(t_end=cfg.t_end, chunk=cfg.chunk, checkpoint=cfg.checkpoint,
                max_attempts=cfg.max_attempts, on_records=write)
        if cfg.gradient and len(drv.records) > n0:
            line = dict(workload=cfg.workload, gradient="d<sigma_11>/d ell",
                        from_t=drv.state_t[0], to_t=drv.state_t[-1])
            try:
                line["dJ_dell_by_field"] = drv.path_gradient()[1]
            except RuntimeError as e:
                # an increment at the edge of stability: its transposed
                # staggered iteration does not contract (no derivative there)
                line.update(dJ_dell_by_field=None, error=str(e))
            log.write(json.dumps(line) + "\n")
    solver.close()
    return drv.reason, len(drv.records) - n0


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 1:
        sys.exit("usage: python -m paper_2103_04770_amd.run config.json")
    reason, n = run(RunConfig.from_json(argv[0]))
    print(json.dumps(dict(reason=reason, increments=n)))


if __name__ == "__main__":
    main()
