"""Per-step run log of an OSCAR context: one JSON line per time step (a
viscous-drag step followed by one capillary relaxation, Section 3).

The paper follows its runs through the share of the capillary sub-steps
that the relaxation performed in each time step, k_f / N (Section 5's
figures).  Each line holds that share, the normalised residual E_k of every
performed sub-step (Section 3.2), the CG iterations and FP64 refinement
steps of the viscous step and of the relaxation, the largest Courant number
and the phase-1 volume of the last transport with the worst conservation
defect so far (FP64 sums), the status codes and the wall time of both calls.

    python -m paper_2105_10576_amd.runlog --case channel --steps 50 --out run.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import cases, oscar


def run(ctx, steps, out, dt_vd=None, n_sub=None, max_iters=None, tol=None):
    """Advance ctx (an oscar.Oscar) by `steps` time steps with its case's
    parameters (or the ones given) and write one JSON line per step to the
    text stream `out`; returns the records."""
    c = ctx.case
    dt_vd = c["dt_vd"] if dt_vd is None else dt_vd
    n_sub = c["n_sub"] if n_sub is None else n_sub
    max_iters = c["max_iters"] if max_iters is None else max_iters
    tol = c["tol"] if tol is None else tol
    recs = []
    for s in range(steps):
        t0 = time.perf_counter()
        rc1 = ctx.viscous_step(dt_vd)
        st1 = ctx.stats()
        t1 = time.perf_counter()
        rc2, kf, E = ctx.capillary_relax(dt_vd, n_sub, max_iters, tol)
        st2 = ctx.stats()
        t2 = time.perf_counter()
        rec = {
            "step": s + 1,
            "k_f": kf,
            "n_sub": int(n_sub),
            "relax_share": kf / float(n_sub),
            "E": [float(x) for x in E],
            "viscous_pcg_iters": st1["pcg_iters_call"],
            "viscous_refine_steps": st1["refine_steps_call"],
            "relax_pcg_iters": st2["pcg_iters_call"],
            "relax_refine_steps": st2["refine_steps_call"],
            "max_courant": st2["max_courant"],
            "mass_phase1": st2["mass_phase1"],
            "mass_defect": st2["mass_defect"],
            "status": [int(rc1), int(rc2)],
            "wall_viscous_s": t1 - t0,
            "wall_relax_s": t2 - t1,
        }
        out.write(json.dumps(rec) + "\n")
        out.flush()
        recs.append(rec)
    return recs


CASES = {
    "channel": cases.channel_bubble,
    "constricted": cases.constricted_channel,
    "micromodel": cases.micromodel,
    "sphere": cases.sphere_pack,
}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--case", choices=sorted(CASES), default="channel")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--precond", choices=("jacobi", "mg"), default="mg")
    ap.add_argument("--out", default="-")
    a = ap.parse_args(argv)
    c = CASES[a.case]()
    c["precond"] = oscar.PC_MG if a.precond == "mg" else oscar.PC_JACOBI
    prec = oscar.MIXED if a.precision == "mixed" else oscar.FP64
    ctx = oscar.Oscar(c, precision=prec)
    out = sys.stdout if a.out == "-" else open(a.out, "w")
    try:
        run(ctx, a.steps, out)
    finally:
        if out is not sys.stdout:
            out.close()
        ctx.close()


if __name__ == "__main__":
    main()
