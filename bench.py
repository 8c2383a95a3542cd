#!/usr/bin/env python3
"""Throughput of the staggered FFT solver on one MI355X.

A step is one load increment of the iterated staggered scheme (constitutive
update, Newton + Galerkin CG, Helmholtz PCG for every non-local field,
staggered error) on the 128^3 RVE with 25% spheres (radii U(4, 8) voxels),
a J2-damage matrix and cracking particles (two non-local fields), under
uniaxial mixed control with increments of 1e-3 (E11 = 0.001 ... 0.005, the
path restarting from the virgin state every five steps; the default run times
E11 = 0.002 ... 0.005 and then 0.001 ... 0.005, every increment converged to
the staggered tolerance with every inner solve at its own).  Inputs live in
HBM before the timed region starts.

Prints ONE JSON line.  value = voxels x (Galerkin CG + Helmholtz PCG
iterations) / wall time of the timed steps, for the FP64 form; the
FP32-refined form is reported beside it on the same load path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "voxel-Krylov-iters/s and HBM GB/s at 128^3, FP64 vs FP32-refined, at 1e-6"
UNIT = "voxel-Krylov-iters/s"
PEAK_HBM_GBS = 8000.0
TOLS = dict(cg_tol=1e-8, pcg_tol=1e-8, newton_tol=1e-8, stagger_tol=1e-6, max_stagger=100)
PATH_LEN = 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_CLASSES = ["galerkin_x_fused", "galerkin_y_inv", "galerkin_y_fwd", "galerkin_outer_dir_inv",
                  "galerkin_outer_fwd_resid", "galerkin_outer_dot_fwd", "galerkin_resid",
                  "helmholtz_x_fused",
                  "helmholtz_outer_dir_inv", "helmholtz_outer_div_fwd", "helmholtz_resid"]


def kernel_bytes(name, n, c, nd, J, fp32):
    """Algorithmic HBM bytes of one launch of a kernel class (each pass reads
    its inputs once and writes its outputs once)."""
    N = n ** 3
    Ns = (n // 2 + 1) * n * n
    zc = 8 if fp32 else 16       # complex element
    zr = 4 if fp32 else 8        # real element
    table = {
        "galerkin_x_fused": 2 * c * Ns * zc + 8 * N * zr,
        "galerkin_y_inv": 2 * c * Ns * zc,
        "galerkin_y_fwd": 2 * c * Ns * zc,
        "galerkin_outer_dir_inv": 6 * c * Ns * zc,
        # p.Ap is summed in real space by the x pass: the forward pass reads
        # only the transform's input
        "galerkin_outer_dot_fwd": 2 * c * Ns * zc,
        "galerkin_resid": 3 * c * Ns * zc,
        # the forward pass fused with the residual update: reads w and r,
        # writes r (the transform itself is not stored)
        "galerkin_outer_fwd_resid": 3 * c * Ns * zc,
        # the staggered step reads ell^2 through the 1-byte phase index
        "helmholtz_x_fused": 2 * nd * Ns * zc + N,
        # 3D: the outer passes transform two fields; the y passes map two
        # fields to the three gradient components and back
        "helmholtz_y_inv": (2 + nd) * Ns * zc,
        "helmholtz_y_fwd": (nd + 2) * Ns * zc,
        "helmholtz_outer_dir_inv": (5 + 2) * Ns * zc,
        # the forward pass fused with the residual update: the two
        # transformed fields, p and r in, r out (without the fusion: 2 + 2)
        "helmholtz_outer_div_fwd": (2 + 3) * Ns * zc,
        "helmholtz_resid": 3 * Ns * zc,
        "constitutive": N * (1 + 8 * (2 * c + 14 + 2 * J) + 8 * zr),
    }
    return table.get(name)


def step_load(i):
    """Macro target of step i (warmup steps included).  The load path is five
    increments of dE11 = 1e-3 from the virgin state; it restarts every
    PATH_LEN steps.  With increments of 1e-3 the next one (E11 = 0.005 ->
    0.006) does not converge on this RVE: Newton at frozen damage falls into a
    two-cycle (the residual repeats at 1.4e-2 while every CG converges), so
    its cost is not bounded; continuing the path needs smaller increments."""
    from paper_2103_04770_amd import microstructure as ms
    return ms.uniaxial_mixed(3, 1e-3 * ((i % PATH_LEN) + 1))


def run_form(ws, prec, warmup, steps):
    import torch
    from paper_2103_04770_amd import Solver, FP64, FP32_REFINED
    shape, J, c = ws["shape"], ws["nfields"], 6
    s = Solver(tuple(reversed(shape)), prec=FP64 if prec == "fp64" else FP32_REFINED)
    state = torch.zeros((c + 7 + 2 * J,) + shape, dtype=torch.float64, device="cuda")
    sig = torch.empty((c,) + shape, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(ws["phase"]).cuda()
    homog = []

    def step(i):
        if i % PATH_LEN == 0:
            state.zero_()
        return s.staggered_step(ph, ws["table"], J, state, step_load(i), sig, **TOLS)

    for i in range(warmup):
        d = step(i)
        homog.append(d["sigma_mean"])
        log("[%s] warmup step %d (E11 %.3f): cg %d pcg %d newton %d stag %d err %.2e  %.0f ms" % (
            prec, i, step_load(i)[1][0], d["cg_iters"], d["pcg_iters"], d["newton_iters"],
            d["stagger_iters"], d["err"], sum(d["t_ms"])))
    last = warmup + steps - 1
    saved = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # totals over the converged timed increments (staggered error at its
    # tolerance and every inner solve of the last pass at its own)
    tot = dict(cg=0, pcg=0, newton=0, stag=0, t_ms=np.zeros(4), conv_s=0.0)
    records = []
    for i in range(warmup, warmup + steps):
        if i == last:
            # kept for the profiled re-run of this increment after the timed region
            saved = state.clone()
        ti = time.perf_counter()
        d = step(i)
        dt = time.perf_counter() - ti  # the call returns once its outputs are valid
        ok = bool(d["converged"])
        records.append(dict(e11=round(float(step_load(i)[1][0]), 6), converged=ok,
                            inner_converged=bool(d["inner_converged"]),
                            stagger_iters=int(d["stagger_iters"]), err=float(d["err"]),
                            newton=int(d["newton_iters"]), cg=int(d["cg_iters"]),
                            pcg=int(d["pcg_iters"]), ms=round(1e3 * dt, 2),
                            sigma11=round(float(d["sigma_mean"][0]), 6)))
        if ok:
            tot["cg"] += d["cg_iters"]
            tot["pcg"] += d["pcg_iters"]
            tot["newton"] += d["newton_iters"]
            tot["stag"] += d["stagger_iters"]
            tot["t_ms"] += np.array(d["t_ms"])
            tot["conv_s"] += dt
        homog.append(d["sigma_mean"])
        log("[%s] timed step %d (E11 %.3f): cg %d pcg %d newton %d stag %d err %.2e %s "
            "<s11> %.4f MPa  %.0f ms" % (
                prec, i, step_load(i)[1][0], d["cg_iters"], d["pcg_iters"], d["newton_iters"],
                d["stagger_iters"], d["err"], "converged" if ok else "NOT CONVERGED",
                d["sigma_mean"][0], 1e3 * dt))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # after the timed region: the last timed increment again, from the same
    # state, with per-kernel event timers; then back-to-back launches of each
    # kernel class
    state.copy_(saved)
    del saved
    s.profile(True)
    d = s.staggered_step(ph, ws["table"], J, state, step_load(last), sig, **TOLS)
    prof = s.profile(False)
    prof_pcg = d["pcg_iters"]
    log("[%s] profiled re-run of step %d: cg %d pcg %d (per-kernel events)" % (
        prec, last, d["cg_iters"], d["pcg_iters"]))
    b2b = {}
    for nm in KERNEL_CLASSES:
        b2b[nm] = s.time_kernel(nm, reps=30)
    log("[%s] back-to-back kernel timings done" % prec)
    y, o, tms = s.tile_config()
    tiles = dict(y_code=int(y), outer_code=int(o), times_ms=[round(v, 4) for v in tms])
    s.close()
    # state and stress after the last timed increment (the profiled re-run
    # repeats it from the same state; the increment is deterministic)
    return dict(seconds=t1 - t0, tot=tot, homog=np.array(homog), prof=prof, prof_pcg=prof_pcg,
                b2b=b2b, records=records, tiles=tiles, final=dict(state=state, sigma=sig))


def field_errors(ws, a, b):
    """Relative L2 and max-abs differences of the fields of run a against run
    b (same increment): strain, stress, every non-local field and every damage
    field (damage law of the library at the committed fields)."""
    import torch
    from paper_2103_04770_amd import Solver
    shape, J, c = ws["shape"], ws["nfields"], 6
    s = Solver(tuple(reversed(shape)))
    ph = torch.from_numpy(ws["phase"]).cuda()

    def damage(st):
        D = torch.empty((J,) + shape, dtype=torch.float64, device="cuda")
        s.fftg_damage(ph, ws["table"], J, st[c + 7 + J:].contiguous(),
                      st[c + 7:c + 7 + J].contiguous(), D)
        return D

    def err(x, y):
        d = x - y
        ny = float(torch.linalg.vector_norm(y))
        # a field that is zero in the reference (e.g. no damage yet) has no
        # relative error; its absolute difference is still reported
        return dict(rel_l2=float(torch.linalg.vector_norm(d)) / ny if ny > 0 else None,
                    max_abs=float(d.abs().max()))

    sa, sb = a["state"], b["state"]
    out = dict(eps=err(sa[:c], sb[:c]), sigma=err(a["sigma"], b["sigma"]))
    Da, Db = damage(sa), damage(sb)
    for j in range(J):
        out["abar_%d" % j] = err(sa[c + 7 + J + j], sb[c + 7 + J + j])
        out["D_%d" % j] = err(Da[j], Db[j])
    s.close()
    return out


PRECISION_TOLS = dict(cg_tol=1e-12, pcg_tol=1e-12, newton_tol=1e-11, stagger_tol=1e-11,
                      max_stagger=100)


def run_precision(ws, e11=3e-3):
    """The FP32-refined form against the FP64 form on the benchmark RVE at
    tolerances tight enough that both reach the fixed point to ~1e-11 (Krylov
    1e-12, Newton 1e-11, staggered 1e-11): one increment from the virgin state
    to E11 = 0.003 (plastic matrix, cracking particles).  The differences are
    then those of the precision form, not of the stop tests."""
    import torch
    from paper_2103_04770_amd import Solver, FP64, FP32_REFINED
    shape, J, c = ws["shape"], ws["nfields"], 6
    ph = torch.from_numpy(ws["phase"]).cuda()
    runs = {}
    for prec in ("fp64", "fp32"):
        s = Solver(tuple(reversed(shape)), prec=FP64 if prec == "fp64" else FP32_REFINED)
        state = torch.zeros((c + 7 + 2 * J,) + shape, dtype=torch.float64, device="cuda")
        sig = torch.empty((c,) + shape, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = s.staggered_step(ph, ws["table"], J, state, ms_uniaxial(e11), sig, **PRECISION_TOLS)
        torch.cuda.synchronize()
        runs[prec] = dict(d=d, seconds=time.perf_counter() - t0, state=state, sigma=sig)
        s.close()
        log("[precision] %s: E11 %.3f in %.1f s, %d passes, %d Newton, %d CG, %d PCG, %s" % (
            prec, e11, runs[prec]["seconds"], d["stagger_iters"], d["newton_iters"],
            d["cg_iters"], d["pcg_iters"], "converged" if d["converged"] else "NOT CONVERGED"))
    a, b = runs["fp32"], runs["fp64"]
    fe = field_errors(ws, dict(state=a["state"], sigma=a["sigma"]),
                      dict(state=b["state"], sigma=b["sigma"]))
    herr = float(np.abs(a["d"]["sigma_mean"] - b["d"]["sigma_mean"]).max() /
                 np.abs(b["d"]["sigma_mean"]).max())
    log("[precision] FP32-refined vs FP64 at tight tolerances: homogenised stress %.2e; fields "
        "(rel L2 | max abs): " % herr + ", ".join(
            "%s %s|%.1e" % (k, "-" if v["rel_l2"] is None else "%.1e" % v["rel_l2"], v["max_abs"])
            for k, v in fe.items()))
    return dict(e11=e11, tolerances=PRECISION_TOLS,
                converged=dict(fp64=bool(b["d"]["converged"]), fp32=bool(a["d"]["converged"])),
                seconds=dict(fp64=round(b["seconds"], 3), fp32=round(a["seconds"], 3)),
                iters=dict(fp64={k: int(b["d"][k]) for k in ("stagger_iters", "newton_iters",
                                                             "cg_iters", "pcg_iters")},
                           fp32={k: int(a["d"][k]) for k in ("stagger_iters", "newton_iters",
                                                             "cg_iters", "pcg_iters")}),
                homog_stress_rel_err=herr, field_errors=fe)


def ms_uniaxial(e11):
    from paper_2103_04770_amd import microstructure as ms
    return ms.uniaxial_mixed(3, e11)


def run_driver(name="spheres64_20", e11_end=0.05, dt=0.02, max_attempts=60):
    """The adaptive load driver on the 64^3 RVE with 20 spheres: variable
    increments from the virgin state to E11 = 0.05 (FP64, staggered
    tolerance 1e-6, smallest admissible increment Delta E11 = 1e-5)."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload(name)
    S, J = w["shape"], w["nfields"]
    N = int(np.prod(S))
    s = Solver(tuple(reversed(S)))
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(w["phase"]).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.fftg_drive(ph, w["table"], J, state, ms.uniaxial_mixed(3, e11_end), sig, dt=dt,
                       dt_min=1e-5 / e11_end, max_attempts=max_attempts,
                       **dict(TOLS, max_stagger=20))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    rec = out["records"]
    it = sum(r["cg_iters"] + r["pcg_iters"] for r in rec)
    log("[driver] %s: %d accepted / %d attempts, E11 reached %.5f, peak <s11> %.1f MPa, %.1f s" % (
        name, len(rec), out["attempts"], out["t"] * e11_end,
        max((r["sigma"][0] for r in rec), default=0.0), wall))
    return dict(workload=name, e11_end=e11_end, e11_reached=out["t"] * e11_end,
                reason=out["reason"], accepted=len(rec), attempts=out["attempts"],
                cutbacks=sum(r["cutbacks"] for r in rec), wall_s=round(wall, 3),
                peak_sigma11=max((r["sigma"][0] for r in rec), default=0.0),
                final_sigma11=rec[-1]["sigma"][0] if rec else 0.0,
                accepted_voxel_krylov_iters_per_s=round(N * it / wall, 1),
                # the homogenised curve with the Krylov counts of every accepted increment
                curve=[dict(e11=round(r["t"] * e11_end, 6), sigma11=round(r["sigma"][0], 3),
                            cg=int(r["cg_iters"]), pcg=int(r["pcg_iters"]),
                            newton=int(r["newton_iters"]), stagger=int(r["stagger_iters"]),
                            cutbacks=int(r["cutbacks"])) for r in rec])


def run_c3_drive(budget_s=480.0, newton_maxit=12):
    """The benchmark RVE along the whole C3 load path to E11 = 0.01 under the
    adaptive driver (FP64, production tolerances, at most 100 staggered passes
    and `newton_maxit` Newton corrections per pass): increments of 1e-3 while
    they converge, halved after a failed attempt (smallest 1e-5), grown by 1.5
    after an accepted one.  Driven a few attempts per call so that progress
    is printed; stops at E11 = 0.01, at the smallest increment, or after
    `budget_s` seconds."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload("spheres_two_fields_128")
    S, J = w["shape"], w["nfields"]
    s = Solver(tuple(reversed(S)))
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(w["phase"]).cuda()
    t, dt, reason, recs, attempts = 0.0, 0.1, 2, [], 0
    t0 = time.perf_counter()
    while reason == 2 and time.perf_counter() - t0 < budget_s:
        out = s.fftg_drive(ph, w["table"], J, state, ms.uniaxial_mixed(3, 0.01), sig, t=t, dt=dt,
                           dt_min=1e-3, dt_max=0.1, grow=1.5, max_attempts=2, newton_div=3,
                           **dict(TOLS, newton_maxit=newton_maxit))
        t, dt, reason = out["t"], out["dt"], out["reason"]
        attempts += out["attempts"]
        recs += out["records"]
        log("[c3 drive] E11 %.5f, next dE11 %.2e, %d accepted / %d attempts, %.0f s" % (
            t * 0.01, dt * 0.01, len(recs), attempts, time.perf_counter() - t0))
    wall = time.perf_counter() - t0
    s.close()
    return dict(workload="spheres_two_fields_128", e11_end=0.01, e11_reached=round(t * 0.01, 7),
                reason={0: "reached", 1: "increment below 1e-5", 2: "time budget"}.get(reason),
                accepted=len(recs), attempts=attempts, wall_s=round(wall, 1),
                newton_maxit=newton_maxit,
                curve=[dict(e11=round(r["t"] * 0.01, 7), sigma11=round(float(r["sigma"][0]), 3),
                            stagger=int(r["stagger_iters"]), newton=int(r["newton_iters"]),
                            cg=int(r["cg_iters"]), pcg=int(r["pcg_iters"]),
                            cutbacks=int(r["cutbacks"]), ms=round(r["ms"], 1)) for r in recs])


def run_c2_fixed(name="spheres64_20"):
    """The 64^3 RVE with 20 spheres along its fixed path: 50 increments of
    dE11 = 1e-3 to E11 = 0.05 (FP64, staggered tolerance 1e-6, at most 20
    staggered passes per increment); the homogenised curve and the Krylov
    counts of every increment."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload(name)
    S, J = w["shape"], w["nfields"]
    N = int(np.prod(S))
    s = Solver(tuple(reversed(S)))
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(w["phase"]).cuda()
    curve, it = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, tgt in enumerate(w["load"]):
        d = s.staggered_step(ph, w["table"], J, state, tgt, sig, **dict(TOLS, max_stagger=20))
        it += d["cg_iters"] + d["pcg_iters"]
        curve.append(dict(e11=round(float(tgt[1][0]), 6), sigma11=round(float(d["sigma_mean"][0]), 3),
                          cg=int(d["cg_iters"]), pcg=int(d["pcg_iters"]),
                          newton=int(d["newton_iters"]), stagger=int(d["stagger_iters"]),
                          converged=bool(d["converged"])))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    nconv = sum(c["converged"] for c in curve)
    log("[c2] %s: 50 fixed increments to E11 = 0.05 in %.1f s, %d converged, peak <s11> %.1f MPa"
        % (name, wall, nconv, max(c["sigma11"] for c in curve)))
    return dict(workload=name, increments=len(curve), converged=nconv, wall_s=round(wall, 3),
                voxel_krylov_iters_per_s=round(N * it / wall, 1),
                peak_sigma11=max(c["sigma11"] for c in curve), curve=curve)


def run_adjoint():
    """Differentiation at 128^3 on the RVE with 30 spheres of radius 14.94
    (20%): one pass alpha -> abar -> D -> (eps, sigma) of the library's
    autograd chain at E11 = 0.004, then the gradients of <sigma_11> and of the
    mean damage with respect to the per-voxel source and the two per-phase
    lengths (FP64)."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    from paper_2103_04770_amd import autograd as ag
    w = ms.workload("spheres30_128")
    S = w["shape"]
    s = Solver(tuple(reversed(S)))
    rng = np.random.default_rng(11)
    ph = torch.from_numpy(w["phase"]).cuda()
    # local source: an equivalent plastic strain in the matrix crossing the
    # damage onset (eps_C = 0.03)
    alpha = torch.from_numpy(np.where(w["phase"] == 0, rng.uniform(0.0, 0.06, size=S),
                                      0.0)).cuda().requires_grad_(True)
    ell = torch.tensor([float(t["ell"][0]) for t in w["table"]], dtype=torch.float64,
                       device="cuda", requires_grad=True)
    tgt = ms.uniaxial_mixed(3, 4e-3)
    out = {}
    for which in ("sigma11", "mean_damage"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        abar, D, eps, sig = ag.one_pass(s, alpha, ell, ph, w["table"], tgt)
        J = sig[0].mean() if which == "sigma11" else D.mean()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ga, ge = torch.autograd.grad(J, (alpha, ell))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out[which] = dict(J=float(J.detach()), forward_ms=round(1e3 * (t1 - t0), 1),
                          backward_ms=round(1e3 * (t2 - t1), 1),
                          dJ_dell=[float(v) for v in ge.cpu()],
                          dJ_dalpha_l2=float(torch.linalg.vector_norm(ga)))
    # a whole converged increment (damage feeding back into the sources),
    # damage thresholds lowered to dC = 5e-4, dR = 0.02 so that damage is
    # active at E11 = 0.004: forward E11 0.002 -> 0.004, then d<s11>/d ell
    tab = [dict(w["table"][0], dC=5e-4, dR=0.02), dict(w["table"][1])]
    state = torch.zeros((6 + 7 + 2,) + S, dtype=torch.float64, device="cuda")
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    tols = dict(TOLS, max_stagger=100)
    s.staggered_step(ph, tab, 1, state, ms.uniaxial_mixed(3, 2e-3), sig, **tols)
    state_n = state.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = s.staggered_step(ph, tab, 1, state, ms.uniaxial_mixed(3, 4e-3), sig, **tols)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / float(np.prod(S))
    dl = torch.empty((1,) + S, dtype=torch.float64, device="cuda")
    a = s.fftg_staggered_adjoint(ph, tab, 1, state_n, state, ms.uniaxial_mixed(3, 4e-3), dl,
                                 g_sig=g, cg_tol=1e-8, pcg_tol=1e-8, tol=1e-6, maxit=200)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sums = s.fftg_phase_sums(ph, 2, dl[0].contiguous())
    out["staggered_sigma11_lowered_thresholds"] = dict(
        dC=5e-4, dR=0.02, forward_ms=round(1e3 * (t1 - t0), 1),
        forward_converged=bool(d["converged"]),
        forward_stagger_iters=d["stagger_iters"], forward_cg=d["cg_iters"],
        forward_pcg=d["pcg_iters"], adjoint_ms=round(1e3 * (t2 - t1), 1),
        adjoint_passes=a["stagger_iters"], adjoint_cg=a["cg_iters"], adjoint_pcg=a["pcg_iters"],
        adjoint_converged=bool(a["converged"]),
        dJ_dell=[2.0 * float(t["ell"][0]) * float(v) for t, v in zip(tab, sums)])
    s.close()
    log("[adjoint] <s11> fwd %.0f ms / bwd %.0f ms; <D> fwd %.0f ms / bwd %.0f ms; "
        "converged increment %.0f ms (%d passes) / adjoint %.0f ms (%d passes)" % (
            out["sigma11"]["forward_ms"], out["sigma11"]["backward_ms"],
            out["mean_damage"]["forward_ms"], out["mean_damage"]["backward_ms"],
            out["staggered_sigma11_lowered_thresholds"]["forward_ms"], d["stagger_iters"],
            out["staggered_sigma11_lowered_thresholds"]["adjoint_ms"], a["stagger_iters"]))
    out["two_fields"] = run_adjoint_two_fields()
    return dict(workload="spheres30_128", e11=0.004, **out)


def run_c5(forms=("fp64", "fp32")):
    """The differentiation workload of the 30-sphere RVE (128^3, 20%,
    lengths 0.05 L / 0.001 L): 20 staggered increments of dE11 = 2e-3 to
    E11 = 0.04 (through the peak and into softening), then the total derivative
    of <sigma_11> at the last converged increment with respect to the two
    per-phase lengths, at that increment alone and through the whole path
    (plastic history of every increment); FP64 and FP32-refined."""
    import torch
    from paper_2103_04770_amd import FP32_REFINED, FP64, Solver, autograd as ag, microstructure as ms
    w = ms.workload("spheres30_128")
    S, J = w["shape"], w["nfields"]
    tols = dict(TOLS, max_stagger=100)
    out = {}
    for form in forms:
        s = Solver(tuple(reversed(S)), prec=FP64 if form == "fp64" else FP32_REFINED)
        ph = torch.from_numpy(w["phase"]).cuda()
        state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
        sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
        curve = []
        states = [state.clone()]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(20):
            state_n = state.clone()
            d = s.staggered_step(ph, w["table"], J, state, w["load"][k], sig, **tols)
            curve.append(round(float(d["sigma_mean"][0]), 3))
            if not d["converged"]:
                break
            states.append(state.clone())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
        g[0] = 1.0 / float(np.prod(S))
        dl = torch.empty((J,) + S, dtype=torch.float64, device="cuda")
        a = s.fftg_staggered_adjoint(ph, w["table"], J, state_n, state, w["load"][k], dl, g_sig=g,
                                     cg_tol=1e-8, pcg_tol=1e-8, tol=1e-6, maxit=300)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sums = s.fftg_phase_sums(ph, 2, dl[0].contiguous())
        rec = dict(increments=k + 1, e11_reached=float(w["load"][k][1][0]),
                   all_converged=bool(d["converged"]), sigma11_curve=curve,
                   path_s=round(t1 - t0, 3), adjoint_s=round(t2 - t1, 3),
                   adjoint_passes=a["stagger_iters"], adjoint_converged=bool(a["converged"]),
                   dJ_dell=[2.0 * float(t["ell"][0]) * float(v)
                            for t, v in zip(w["table"], sums)])
        if d["converged"]:
            # the same J through the whole path: every increment's plastic
            # history chained backwards (states of all increments kept in HBM)
            t3 = time.perf_counter()
            dlp, alog = ag.path_gradient(s, ph, w["table"], J, states, w["load"][:k + 1], g,
                                         cg_tol=1e-8, pcg_tol=1e-8, tol=1e-6, maxit=300)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            sp = s.fftg_phase_sums(ph, 2, dlp[0].contiguous())
            rec.update(path_gradient_s=round(t4 - t3, 3),
                       path_gradient_passes=[x["stagger_iters"] for x in alog][::-1],
                       dJ_dell_path=[2.0 * float(t["ell"][0]) * float(v)
                                     for t, v in zip(w["table"], sp)],
                       states_gb=round(len(states) * states[0].numel() * 8 / 1e9, 2))
        s.close()
        del states
        out[form] = rec
        log("[c5] %s: %d increments to E11 %.3f in %.1f s, peak <s11> %.1f MPa; gradient %.2f s, "
            "d<s11>/d ell = %s; through the path %s s, %s" % (
                form, k + 1, w["load"][k][1][0], t1 - t0, max(curve), t2 - t1,
                ["%.5f" % v for v in rec["dJ_dell"]], rec.get("path_gradient_s"),
                ["%.5f" % v for v in rec.get("dJ_dell_path", [])]))
    if "fp64" in out and "fp32" in out:
        for key in ("dJ_dell", "dJ_dell_path"):
            if key in out["fp64"] and key in out["fp32"]:
                a64, a32 = np.array(out["fp64"][key]), np.array(out["fp32"][key])
                out["fp32_rel_err_vs_fp64_" + key] = float(np.abs(a32 - a64).max() /
                                                           np.abs(a64).max())
    return dict(workload="spheres30_128", path="20 x dE11 = 2e-3 to 0.04", **out)


def run_two_field_path_gradient(n_inc=4):
    """The benchmark RVE itself (spheres_two_fields_128: J2 damage matrix on
    field 0, particle cracking on field 1), FP64: the first n_inc increments
    of the benchmark path (E11 = 1e-3 ... n_inc 1e-3), then d<sigma_11>/d ell
    of both fields through the whole path (plastic state and damage history
    of every increment chained backwards)."""
    import torch
    from paper_2103_04770_amd import Solver, autograd as ag, microstructure as ms
    w = ms.workload("spheres_two_fields_128")
    S, J = w["shape"], w["nfields"]
    s = Solver(tuple(reversed(S)))
    ph = torch.from_numpy(w["phase"]).cuda()
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    tols = dict(TOLS, max_stagger=100)
    states, targets, conv = [state.clone()], [], True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_inc):
        d = s.staggered_step(ph, w["table"], J, state, step_load(k), sig, **tols)
        conv = conv and bool(d["converged"])
        states.append(state.clone())
        targets.append(step_load(k))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / float(np.prod(S))
    dl, alog = ag.path_gradient(s, ph, w["table"], J, states, targets, g, cg_tol=1e-8,
                                pcg_tol=1e-8, tol=1e-6, maxit=200)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grads = []
    for j in range(J):
        sums = s.fftg_phase_sums(ph, len(w["table"]), dl[j].contiguous())
        grads.append([2.0 * float(t["ell"][j]) * float(v) for t, v in zip(w["table"], sums)])
    s.close()
    log("[c5] benchmark RVE, two fields: %d increments in %.1f s, path gradient %.1f s, "
        "d<s11>/d ell by field %s" % (n_inc, t1 - t0, t2 - t1, grads))
    return dict(workload="spheres_two_fields_128", increments=n_inc,
                e11_end=1e-3 * n_inc, all_converged=conv, path_s=round(t1 - t0, 3),
                path_gradient_s=round(t2 - t1, 3),
                adjoint_passes=[x["stagger_iters"] for x in alog][::-1],
                dJ_dell_by_field=grads)


def run_adjoint_two_fields():
    """The benchmark RVE itself (spheres_two_fields_128: J2 damage matrix on
    field 0, particle cracking on field 1): the converged increment
    E11 0.003 -> 0.004 of the benchmark path and the adjoint of <sigma_11>
    with respect to both fields' per-phase lengths (FP64)."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload("spheres_two_fields_128")
    S, J = w["shape"], w["nfields"]
    s = Solver(tuple(reversed(S)))
    ph = torch.from_numpy(w["phase"]).cuda()
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.empty((6,) + S, dtype=torch.float64, device="cuda")
    tols = dict(TOLS, max_stagger=100)
    for k in range(3):
        s.staggered_step(ph, w["table"], J, state, step_load(k), sig, **tols)
    state_n = state.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = s.staggered_step(ph, w["table"], J, state, step_load(3), sig, **tols)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    g[0] = 1.0 / float(np.prod(S))
    dl = torch.empty((J,) + S, dtype=torch.float64, device="cuda")
    a = s.fftg_staggered_adjoint(ph, w["table"], J, state_n, state, step_load(3), dl, g_sig=g,
                                 cg_tol=1e-8, pcg_tol=1e-8, tol=1e-6, maxit=200)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grads = []
    for j in range(J):
        sums = s.fftg_phase_sums(ph, len(w["table"]), dl[j].contiguous())
        grads.append([2.0 * float(t["ell"][j]) * float(v) for t, v in zip(w["table"], sums)])
    s.close()
    log("[adjoint] benchmark RVE, two fields: increment %.0f ms (%d passes), adjoint %.0f ms "
        "(%d passes)" % (1e3 * (t1 - t0), d["stagger_iters"], 1e3 * (t2 - t1), a["stagger_iters"]))
    return dict(workload="spheres_two_fields_128", e11=[0.003, 0.004],
                forward_ms=round(1e3 * (t1 - t0), 1), forward_converged=bool(d["converged"]),
                forward_stagger_iters=d["stagger_iters"], adjoint_ms=round(1e3 * (t2 - t1), 1),
                adjoint_passes=a["stagger_iters"], adjoint_cg=a["cg_iters"],
                adjoint_pcg=a["pcg_iters"], adjoint_converged=bool(a["converged"]),
                dJ_dell_by_field=grads)


def run_batch(count=64, nworkers=8):
    """One staggered increment (E11 = 1e-3) of 64 RVEs of uneven sizes
    (edges from {32, 48, 64, 96}, particle fractions U(0.05, 0.30)), FP32-refined,
    three ways: every RVE alone on its own stream one at a time, the same with
    `nworkers` host threads overlapping the RVEs, and as lockstep classes
    (one per edge length, each Krylov iteration one set of launches over the
    class; classes overlapping on the worker threads).  Then the lockstep
    loading of every RVE to E11 = 0.01 in 10 increments."""
    import torch
    from paper_2103_04770_amd import FP32_REFINED, microstructure as ms
    from paper_2103_04770_amd.batch import RVEBatch
    rves = ms.batch_workload(count)
    vox = sum(int(np.prod(r["shape"])) for r in rves)
    b = RVEBatch(rves, prec=FP32_REFINED)
    tgt = ms.uniaxial_mixed(3, 1e-3)
    res = {}
    saved = os.environ.get("FFTG_BATCH_LOCKSTEP")
    outs = {}
    for mode, nw, lock in (("one_at_a_time", 1, "0"), ("per_rve_streams", nworkers, "0"),
                           ("lockstep", nworkers, "1")):
        os.environ["FFTG_BATCH_LOCKSTEP"] = lock
        b.reset()
        b.step(tgt, nworkers=nw, **TOLS)  # warm-up: graphs, workspaces
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = b.step(tgt, nworkers=nw, **TOLS)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        outs[mode] = out
        it = sum(o["cg_iters"] + o["pcg_iters"] for o in out)
        res[mode] = dict(seconds=round(dt, 3), workers=nw, krylov_iters=it,
                         voxel_krylov_iters_per_s=round(sum(
                             int(np.prod(r["shape"])) * (o["cg_iters"] + o["pcg_iters"])
                             for r, o in zip(rves, out)) / dt, 1),
                         converged=sum(o["converged"] for o in out))
        log("[batch] %s (%d workers): %.3f s, %.3e voxel-Krylov-iters/s" % (
            mode, nw, dt, res[mode]["voxel_krylov_iters_per_s"]))
    if saved is None:
        os.environ.pop("FFTG_BATCH_LOCKSTEP", None)
    else:
        os.environ["FFTG_BATCH_LOCKSTEP"] = saved
    # lockstep and per-RVE runs agree bitwise (same arithmetic per RVE)
    same = all(a["cg_iters"] == c["cg_iters"] and a["pcg_iters"] == c["pcg_iters"] and
               np.array_equal(a["sigma_mean"], c["sigma_mean"])
               for a, c in zip(outs["lockstep"], outs["per_rve_streams"]))
    # the whole loading of every RVE: 10 increments of 1e-3 to E11 = 0.01
    b.reset()
    vit = 0
    all_conv = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(10):
        out = b.step(ms.uniaxial_mixed(3, 1e-3 * (k + 1)), nworkers=nworkers, **TOLS)
        vit += sum(int(np.prod(r["shape"])) * (o["cg_iters"] + o["pcg_iters"])
                   for r, o in zip(rves, out))
        all_conv = all_conv and all(o["converged"] for o in out)
    torch.cuda.synchronize()
    dpath = time.perf_counter() - t0
    s11 = [float(o["sigma_mean"][0]) for o in out]
    path = dict(increments=10, e11_end=0.01, seconds=round(dpath, 3), all_converged=bool(all_conv),
                voxel_krylov_iters_per_s=round(vit / dpath, 1),
                sigma11_at_end_MPa=[round(min(s11), 1), round(max(s11), 1)])
    tiles = {}
    for r, sv in zip(rves, b.solvers):
        tiles.setdefault(str(r["shape"][0]), list(sv.tile_config()[:2]))
    b.close()
    log("[batch] %d RVEs, %d voxels: one at a time %.2f s, per-RVE streams %.2f s, lockstep "
        "%.2f s (results equal: %s); 10 lockstep increments to E11 = 0.01 in %.2f s "
        "(%.2e voxel-Krylov-iters/s)" % (
            count, vox, res["one_at_a_time"]["seconds"], res["per_rve_streams"]["seconds"],
            res["lockstep"]["seconds"], same, dpath, vit / dpath))
    return dict(rves=count, voxels=vox, sizes=[32, 48, 64, 96], form="fp32_refined",
                increment="E11 = 1e-3 from the virgin state", **res,
                lockstep_equals_per_rve=bool(same),
                speedup_lockstep_vs_one_at_a_time=round(
                    res["one_at_a_time"]["seconds"] / res["lockstep"]["seconds"], 3),
                path_to_e11_0p01=path, tile_shifts_by_edge=tiles)


def run_gtn_drive(name="gtn_spheres30_64", e11_end=0.05, max_records=200):
    """The Gurson RVE (30 spheres, 64^3) under the adaptive driver from the
    virgin state towards E11 = 0.05 (FP64, production tolerances, at most 30
    staggered passes per increment), for at most `max_records` accepted
    increments: porosity growth, increment sizes and the homogenised curve."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload(name)
    S, J = w["shape"], w["nfields"]
    s = Solver(tuple(reversed(S)))
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(w["phase"]).cuda()
    recs, fmax = [], []
    t, dt, reason = 0.0, 0.02, 3
    t0 = time.perf_counter()
    while reason == 3 and len(recs) < max_records:
        out = s.fftg_drive(ph, w["table"], J, state, ms.uniaxial_mixed(3, e11_end), sig, t=t, dt=dt,
                           dt_min=2e-4, max_records=10, max_attempts=400,
                           **dict(TOLS, max_stagger=30))
        t, dt, reason = out["t"], out["dt"], out["reason"]
        recs += out["records"]
        fmax.append((round(t * e11_end, 6), round(state[6 + 7].max().item(), 4)))
        log("[gtn drive] E11 %.5f, %d increments, max porosity %.4f, %.1f s" % (
            t * e11_end, len(recs), fmax[-1][1], time.perf_counter() - t0))
    wall = time.perf_counter() - t0
    s.close()
    return dict(workload=name, e11_reached=t * e11_end, reason=reason, accepted=len(recs),
                wall_s=round(wall, 3), porosity_max_by_e11=fmax,
                curve=[(round(r["t"] * e11_end, 6), round(float(r["sigma"][0]), 2),
                        int(r["stagger_iters"]), int(r["cutbacks"])) for r in recs])


def run_gtn(name="gtn_spheres30_128", steps=6):
    """The Gurson matrix (two non-local fields, Sec. 4.2 parameters) on the
    30-sphere 128^3 RVE: `steps` staggered increments of 1e-3 from the virgin
    state (FP64, production tolerances); Krylov throughput, the share of the
    constitutive update in the wall time and the porosity reached."""
    import torch
    from paper_2103_04770_amd import Solver, microstructure as ms
    w = ms.workload(name)
    S, J = w["shape"], w["nfields"]
    N = int(np.prod(S))
    s = Solver(tuple(reversed(S)))
    state = torch.zeros((6 + 7 + 2 * J,) + S, dtype=torch.float64, device="cuda")
    sig = torch.zeros((6,) + S, dtype=torch.float64, device="cuda")
    ph = torch.from_numpy(w["phase"]).cuda()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ti = time.perf_counter()
        d = s.staggered_step(ph, w["table"], J, state, w["load"][k], sig, **TOLS)
        recs.append(dict(e11=1e-3 * (k + 1), sigma11=float(d["sigma_mean"][0]),
                         cg=d["cg_iters"], pcg=d["pcg_iters"], newton=d["newton_iters"],
                         stagger=d["stagger_iters"], converged=bool(d["converged"]),
                         t_ms=[round(v, 2) for v in d["t_ms"]],
                         wall_ms=round(1e3 * (time.perf_counter() - ti), 1)))
        log("[gtn] E11 %.3f: cg %d pcg %d newton %d stag %d  <s11> %.1f MPa  %.0f ms" % (
            recs[-1]["e11"], d["cg_iters"], d["pcg_iters"], d["newton_iters"],
            d["stagger_iters"], d["sigma_mean"][0], recs[-1]["wall_ms"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fmax = float(state[6 + 7].max())
    s.close()
    it = sum(r["cg"] + r["pcg"] for r in recs)
    tc = sum(r["t_ms"][0] for r in recs)
    return dict(workload=name, increments=steps, form="fp64", wall_s=round(wall, 3),
                voxel_krylov_iters_per_s=round(N * it / wall, 1),
                constitutive_share=round(tc / (1e3 * wall), 4), max_porosity=fmax,
                records=recs)


def copy_ceiling(mib=1024, reps=20):
    """Streaming-copy ceiling of HBM: the library's 16-byte-per-lane copy of a
    `mib` MiB buffer (read + write; 4x the last-level cache), best grid size,
    `reps` copies between one event pair."""
    import torch
    from paper_2103_04770_amd import Solver
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s = Solver((8, 8, 8))
    rate = s.fftg_copy_rate(a, b, reps)
    s.close()
    del a, b
    return round(rate, 1)


def cpu_baseline(ws, tols):
    """The oracle, as it stands, on a bounded sample of the same workload: the
    first increment of the benchmark path (E11 = 0.001 from the virgin state)
    of the 128^3 RVE, run to convergence with the benchmark's tolerances
    (Newton + CG, Helmholtz PCG for both fields, staggered loop).  Its
    transforms are scipy.fft threaded over every core of the process; its
    element-wise numpy work runs on one thread."""
    from oracle import spectral, staggered
    shape, J = ws["shape"], ws["nfields"]
    N = int(np.prod(shape))
    st0 = staggered.initial_state(shape, 3, J)
    t0 = time.perf_counter()
    _, _, hom, stats = staggered.staggered_step(
        ws["phase"], ws["table"], J, st0, step_load(0), cg_tol=tols["cg_tol"],
        pcg_tol=tols["pcg_tol"], newton_tol=tols["newton_tol"], stagger_tol=tols["stagger_tol"],
        max_stagger=tols["max_stagger"])
    wall = time.perf_counter() - t0
    it = stats["cg_iters"] + stats["pcg_iters"]
    return dict(value=N * it / wall, unit=UNIT, cores=spectral.WORKERS, kind="oracle",
                sample="one whole increment of the 128^3 benchmark RVE (E11 = 0.001 from the "
                       "virgin state, converged: %d staggered passes, %d Newton corrections, "
                       "%d Galerkin CG + %d Helmholtz PCG iterations) in %.1f s; scipy.fft on "
                       "%d threads, numpy element-wise work on one" % (
                           stats["stagger_iters"], stats["newton_iters"], stats["cg_iters"],
                           stats["pcg_iters"], wall, spectral.WORKERS),
                converged=bool(stats["converged"] and stats["inner_converged"]),
                sigma11=float(hom["sigma"][0]), seconds=round(wall, 2),
                host_threads_available=len(os.sched_getaffinity(0)), cpu_model=cpu_model())


def cpu_model():
    """The host processor's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_table(r, fp32, n):
    """Per kernel class of the profiled increment: in-flow total and average
    launch time, and the algorithmic rate.  The Helmholtz passes run the
    fields of a staggered pass in lockstep, one launch covering every field
    still iterating, so their algorithmic bytes are those of one field times
    the PCG iterations summed over the fields (pcg_iters), over the class's
    total time."""
    from paper_2103_04770_amd import load_library
    ms_k, n_k = r["prof"]
    lib = load_library()
    out = {}
    for i, (t, cnt) in enumerate(zip(ms_k, n_k)):
        if cnt == 0:
            continue
        nm = lib.fftg_kernel_name(i).decode()
        avg = t / cnt * 1e3
        ent = dict(inflow_total_ms=round(t, 3), launches=int(cnt), inflow_avg_us=round(avg, 2))
        b = kernel_bytes(nm, n, 6, 3, 2, fp32)
        if b is not None and nm.startswith("helmholtz_"):
            ent["field_iterations"] = int(r["prof_pcg"])
            ent["algo_GBps"] = round(b * r["prof_pcg"] / (t * 1e-3) / 1e9, 1)
        elif b is not None:
            ent["algo_GBps"] = round(b / (avg * 1e-6) / 1e9, 1)
        if nm in r["b2b"]:
            ent["b2b_avg_us"] = round(r["b2b"][nm] * 1e3, 2)
        out[nm] = ent
    return out


def stored_traffic(kernel, form):
    """HBM bytes per launch from committed counter runs, valid only while the
    kernel source is unchanged since they were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    src = os.path.join(ROOT, "paper_2103_04770_amd", "csrc")
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_device.hpp"):
        h.update(open(os.path.join(src, f), "rb").read())
    k = rec.get("kernels", {}).get("%s/%s" % (form, kernel))
    if not k or rec.get("source_sha256") != h.hexdigest():
        return None
    return k.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="grid size (128 is the benchmark)")
    ap.add_argument("--forms", default="fp64,fp32", help="comma list of fp64, fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-refined vs FP64 comparison at tight tolerances")
    ap.add_argument("--no-driver", action="store_true",
                    help="skip the adaptive-driver, adjoint-chain and batch runs")
    ap.add_argument("--c5", action="store_true",
                    help="also run the differentiation workload: 20 increments to E11 = 0.04 "
                         "on the 30-sphere RVE, the gradient at the last one and through the "
                         "whole path (FP64, FP32), and the path gradient on the two-field RVE")
    ap.add_argument("--gtn-drive", action="store_true",
                    help="also drive the 64^3 Gurson RVE adaptively towards E11 = 0.05 "
                         "(200 increments, about 1.5 min)")
    ap.add_argument("--c3-drive", action="store_true",
                    help="also drive the benchmark RVE adaptively along the whole path to "
                         "E11 = 0.01 (FP64; at most 8 minutes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run a device copy of MB megabytes (counter calibration)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-RVE batch leg and print its record as the JSON line")
    ap.add_argument("--batch-workers", type=int, default=8,
                    help="host worker threads of the batch leg (1: every call from one thread)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single device, and "
              "splitting an RVE or a batch over several GPUs is not implemented; got --gpus %d"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_04770_amd import microstructure as ms, load_library

    load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        nbytes = args.copy_calibration * (1 << 20)
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb
    if args.batch_only:
        rec = run_batch(nworkers=max(1, args.batch_workers))
        print(json.dumps(dict(batch=rec)), flush=True)
        return
    ws = ms.workload("spheres_two_fields_%d" % args.n)
    N = int(np.prod(ws["shape"]))
    vf = float(ws["phase"].mean())
    log("workload %s: N=%d, particle vf=%.3f" % (ws["name"], N, vf))
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    res = {}
    if args.steps < 1 or args.warmup < 0:
        sys.exit("bench.py: need --steps >= 1 and --warmup >= 0")
    for f in forms:
        res[f] = run_form(ws, f, args.warmup, args.steps)
    main_form = "fp64" if "fp64" in res else forms[0]
    r = res[main_form]
    iters = r["tot"]["cg"] + r["tot"]["pcg"]
    nconv = sum(x["converged"] for x in r["records"])
    # whole-job throughput of the converged timed increments (all of them
    # when every increment converged, which records[] shows)
    value = N * iters / r["tot"]["conv_s"] if nconv else 0.0
    # per-kernel table: in-flow event times of one profiled increment run
    # right after the timed region (every launch a full one), and the
    # back-to-back duration of each class; roofline on the class with the
    # largest in-flow total, priced at its in-flow average launch duration
    kernels = kernel_table(r, main_form == "fp32", args.n)
    dom = max((k for k in kernels if "algo_GBps" in kernels[k]),
              key=lambda k: kernels[k]["inflow_total_ms"])
    bpl = kernel_bytes(dom, args.n, 6, 3, 2, main_form == "fp32")
    avg = kernels[dom]["inflow_avg_us"]
    ach = bpl / (avg * 1e-6) / 1e9
    tr = stored_traffic(dom, main_form)
    cc = copy_ceiling()
    log("streaming copy ceiling %.0f GB/s" % cc)
    roof = dict(bound="hbm", kernel=dom, achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(ach / PEAK_HBM_GBS, 4), traffic=tr, algorithmic_bytes_per_launch=bpl,
                avg_us=avg, launches=kernels[dom]["launches"], copy_ceiling=cc,
                frac_of_copy=round(ach / cc, 4))
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if main_form == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "spheres_two_fields_%d" % args.n,
                   "grid": [args.n] * 3, "voxels": N, "particle_vf": round(vf, 4),
                   "nfields": 2,
                   "load_path": "uniaxial mixed control, dE11 = 1e-3 per step, "
                                "restarting from the virgin state every %d steps "
                                "(E11 = 0.001 ... 0.005)" % PATH_LEN,
                   "timed_steps": [args.warmup, args.warmup + args.steps - 1],
                   "tolerances": TOLS,
                   "tile_codes": r["tiles"]},
        "timed_increments": r["records"],
        "converged_increments": nconv,
        "loops": {
            "galerkin_cg": dict(iters=r["tot"]["cg"],
                                voxel_iters_per_s=round(N * r["tot"]["cg"] / (r["tot"]["t_ms"][1] / 1e3), 1)),
            "helmholtz_pcg": dict(iters=r["tot"]["pcg"],
                                  voxel_iters_per_s=round(N * r["tot"]["pcg"] / max(r["tot"]["t_ms"][2] / 1e3, 1e-9), 1)),
            "newton_iters": r["tot"]["newton"], "stagger_iters": r["tot"]["stag"],
            "t_ms": [round(x, 1) for x in r["tot"]["t_ms"]]},
        "roofline": roof,
        "kernels": kernels,
    }
    if "fp32" in res and main_form != "fp32":
        r32 = res["fp32"]
        it32 = r32["tot"]["cg"] + r32["tot"]["pcg"]
        n32 = sum(x["converged"] for x in r32["records"])
        # homogenised stress of the timed increments both forms converged
        both = [k for k, (a, b) in enumerate(zip(r["records"], r32["records"]))
                if a["converged"] and b["converged"]]
        off = args.warmup
        err = (float(max(np.abs(r32["homog"][off + k] - r["homog"][off + k]).max() /
                         np.abs(r["homog"][off + k]).max() for k in both)) if both else None)
        k32 = kernel_table(r32, True, args.n)
        last_both = bool(r["records"][-1]["converged"] and r32["records"][-1]["converged"])
        out["fp32_refined"] = dict(
            value=round(N * it32 / r32["tot"]["conv_s"], 1) if n32 else 0.0,
            ms_per_step=round(1e3 * r32["seconds"] / args.steps, 2),
            converged_increments=n32, timed_increments=r32["records"],
            cg_iters=r32["tot"]["cg"], pcg_iters=r32["tot"]["pcg"],
            newton_iters=r32["tot"]["newton"],
            # the Helmholtz loop time includes its FP64 refinement sweeps
            loops={
                "galerkin_cg": dict(iters=r32["tot"]["cg"], voxel_iters_per_s=round(
                    N * r32["tot"]["cg"] / max(r32["tot"]["t_ms"][1] / 1e3, 1e-9), 1)),
                "helmholtz_pcg": dict(iters=r32["tot"]["pcg"], voxel_iters_per_s=round(
                    N * r32["tot"]["pcg"] / max(r32["tot"]["t_ms"][2] / 1e3, 1e-9), 1)),
                "t_ms": [round(x, 1) for x in r32["tot"]["t_ms"]]},
            homog_stress_rel_err_vs_fp64=err,
            homog_stress_err_increments=len(both),
            field_errors_vs_fp64=(field_errors(ws, r32["final"], r["final"]) if last_both
                                  else None),
            field_errors_note="after the last timed increment, against the FP64 run of the "
                              "same increment at the same tolerances (staggered 1e-6, Krylov "
                              "and Newton 1e-8), so at the level of those tolerances",
            kernels=k32)
        log("[fp32] FP32-refined %.4g voxel-Krylov-iters/s (%d of %d timed increments "
            "converged); homogenised stress vs FP64 over %d increments: %s" % (
                out["fp32_refined"]["value"], n32, len(r32["records"]), len(both),
                "%.2e" % err if err is not None else "n/a"))
        fe = out["fp32_refined"]["field_errors_vs_fp64"]
        if fe:
            log("[fp32] field errors vs fp64 (rel L2 | max abs): " + ", ".join(
                "%s %s|%.1e" % (k, "-" if v["rel_l2"] is None else "%.1e" % v["rel_l2"],
                                v["max_abs"]) for k, v in fe.items()))
    for f in res.values():
        f.pop("final", None)
    if "fp64" in res and "fp32" in res and not args.no_precision:
        out["precision"] = run_precision(ws)
    if not args.no_driver:
        out["adaptive_driver"] = run_driver()
        out["adjoint"] = run_adjoint()
        out["c2_fixed_path"] = run_c2_fixed()
        out["batch"] = run_batch(nworkers=max(1, args.batch_workers))
        out["gtn"] = run_gtn()
    if args.c5:
        out["c5_path_gradient"] = run_c5()
        out["two_field_path_gradient"] = run_two_field_path_gradient()
    if args.gtn_drive:
        out["gtn_drive"] = run_gtn_drive()
    if args.c3_drive:
        out["c3_drive"] = run_c3_drive()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(ws, TOLS)
    log("[fp64] %.4g voxel-Krylov-iters/s over %d of %d timed increments (converged), "
        "%.1f ms per step; roofline %s %.3f of %.0f GB/s" % (
            value, nconv, len(r["records"]), out["ms_per_step"], roof["kernel"], roof["frac"],
            PEAK_HBM_GBS))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
