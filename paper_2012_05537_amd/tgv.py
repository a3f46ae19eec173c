"""Taylor-Green vortex runs in the paper's own settings (Sec. III C).

``python -m paper_2012_05537_amd.tgv --case re1600_ma125`` runs one of the
paper's TGV cases (``inputs.PAPER_TGV``: Re, Ma, time step in the paper's
convective units, numerator C of the initial density) on 64^3 cells of order
4 (256^3 nodes) and prints one JSON line every ``--every`` steps:

* time in the paper's units (t U / L) and the step count;
* the diagnostics of Sec. III C in the paper's units, per unit volume:
  kinetic energy E_k / U^2 and its ratio to the initial value, solenoidal and
  dilatational dissipation eps / U^3 (the library's domain integrals divided by
  (2 pi)^3);
* the relative drift of the conserved totals (mass, momentum, energy) since
  the start;
* with ``--compare``, the difference in rho, u and T of two companion runs
  against the FP64 run, advanced in lockstep: the FP32-mixed run from the same
  initial fields, and an FP64 run whose initial density is moved by one ulp at
  every node (the rounding floor that any other arithmetic order is judged
  against).

A run stops at the first non-finite result (``sllbm_totals`` /
``sllbm_diagnostics`` report ENONFINITE) and says between which steps it
appeared.  Everything runs in the library; torch holds device memory and
reduces the compared fields.
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import inputs
from .sllbm import CONSTANT, ENONFINITE, FP32_MIXED, FP64, SUTHERLAND, SLLBM, SllbmError


def _fields(ctx, w, perturb=False):
    xs, ys, zs = (c.numpy() for c in ctx.node_coords())
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"], numerator=w["numerator"])
    if perturb:
        rho = np.nextafter(rho, np.inf)
    dev = ctx.device
    return torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev)


def _make(w, precision, perturb=False):
    ctx = SLLBM(w["n_el"], w["p"], w["dt"], w["mu_inf"], gamma=w["gamma"], prandtl=w["Pr"],
                viscosity_law=w.get("law", SUTHERLAND), precision=precision, device=0)
    ctx.init_equilibrium(*_fields(ctx, w, perturb))
    return ctx


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _compare(ref, other):
    r0, u0, T0 = ref.moments()
    r1, u1, T1 = other.moments()
    return {"rho": _rel(r1, r0), "u": _rel(u1, u0), "T": _rel(T1, T0)}


def _totals(ctx):
    try:
        return ctx.totals(), True
    except SllbmError as e:
        if e.code != ENONFINITE:
            raise
        return None, False


def run(case, n_el=None, p=None, precision="fp64", every=20, compare=False, steps=None, log=None,
        prandtl=None, mach_ref="adiabatic", dt_scale=1.0, law=SUTHERLAND):
    """Run one paper TGV case; returns the list of records (also passed to log as they appear).

    Variations of the readings for stability studies: prandtl (Pr = 1 removes
    the quasi-equilibrium term), mach_ref "lattice" (velocity amplitude Ma c_s
    instead of Ma sqrt(gamma T0)), dt_scale (time step times this factor, same
    end time), law (constant viscosity instead of Sutherland's)."""
    over = {}
    if n_el is not None:
        over["n_el"] = n_el
    if p is not None:
        over["p"] = p
    if prandtl is not None:
        over["Pr"] = prandtl
    base = inputs.PAPER_TGV[case]
    if mach_ref == "lattice":
        over["Ma"] = base["Ma"] / math.sqrt(inputs.PAPER_TGV_GRID["gamma"] * inputs.T0)
    if dt_scale != 1.0:
        over["dt_paper"] = base["dt_paper"] * dt_scale
    w = inputs.paper_tgv(case, **over)
    w["law"] = law
    nsteps = w["steps"] if steps is None else int(steps)
    prec = FP64 if precision == "fp64" else FP32_MIXED
    main = _make(w, prec)
    others = {}
    if compare:
        if prec != FP64:
            raise ValueError("--compare needs the FP64 run as its reference")
        others["fp32_mixed"] = _make(w, FP32_MIXED)
        others["fp64_ulp"] = _make(w, FP64, perturb=True)
    U, vol = w["U"], (2 * math.pi) ** 3
    head = {k: w[k] for k in ("name", "Re", "Ma", "dt_paper", "t_end", "n_el", "p", "dt", "mu_inf", "cfl", "Pr", "U")}
    head.update(nodes=main.nodes, steps=nsteps, precision=precision, tau_minus_half=w["mu_inf"] / w["dt"],
                mach_ref=mach_ref, law="constant" if law == CONSTANT else "sutherland")
    records = [dict(kind="setup", **head)]
    if log:
        log(records[-1])
    tot0, _ = _totals(main)
    e0 = None
    step, t_start = 0, time.time()
    while True:
        tot, finite = _totals(main)
        rec = dict(kind="sample", step=step, t=step * w["dt_paper"], wall_s=round(time.time() - t_start, 2))
        if finite:
            try:
                ek, es, ec = main.diagnostics()
            except SllbmError as e:
                if e.code != ENONFINITE:
                    raise
                finite = False
        if not finite:
            rec.update(finite=False, note="first non-finite value after step %d, at or before step %d"
                       % (step - min(every, step), step))
            records.append(rec)
            if log:
                log(rec)
            break
        e0 = ek if e0 is None else e0
        rec.update(finite=True, Ek=ek / (U * U * vol), Ek_ratio=ek / e0, eps_s=es / (U ** 3 * vol),
                   eps_c=ec / (U ** 3 * vol),
                   drift_mass=(tot[0] - tot0[0]) / tot0[0], drift_energy=(tot[4] - tot0[4]) / tot0[4],
                   momentum=[tot[k] / tot0[0] for k in (1, 2, 3)])
        for name, ctx in others.items():
            rec["err_" + name] = _compare(main, ctx)
        records.append(rec)
        if log:
            log(rec)
        if step >= nsteps:
            break
        n = min(every, nsteps - step)
        main.step(n)
        for ctx in others.values():
            ctx.step(n)
        step += n
    torch.cuda.synchronize()
    for ctx in [main, *others.values()]:
        ctx.close()
    return records


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--case", default="re1600_ma125", choices=sorted(inputs.PAPER_TGV))
    ap.add_argument("--n-el", type=int, default=None, help="cells per axis (default 64)")
    ap.add_argument("--p", type=int, default=None, help="order (default 4)")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--steps", type=int, default=None, help="default: t_end / dt_paper")
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--out", default=None, help="also write the records as a JSON list")
    ap.add_argument("--pr", type=float, default=None, help="Prandtl number (default 0.7)")
    ap.add_argument("--mach-ref", choices=("adiabatic", "lattice"), default="adiabatic",
                    help="velocity amplitude Ma sqrt(gamma T0) (default) or Ma c_s")
    ap.add_argument("--dt-scale", type=float, default=1.0, help="time step factor (same end time)")
    ap.add_argument("--law", choices=("sutherland", "constant"), default="sutherland")
    a = ap.parse_args(argv)

    def log(rec):
        print(json.dumps(rec), flush=True)

    recs = run(a.case, a.n_el, a.p, a.precision, a.every, a.compare, a.steps, log, prandtl=a.pr,
               mach_ref=a.mach_ref, dt_scale=a.dt_scale, law=CONSTANT if a.law == "constant" else SUTHERLAND)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(recs, fh)
    return 0 if recs[-1].get("finite", True) else 3


if __name__ == "__main__":
    sys.exit(main())
