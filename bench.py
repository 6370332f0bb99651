"""Benchmark of the OSCAR relaxation path on one MI355X.

Workload (the headline): the 3D constricted channel, 128 x 64 x 64 voxels at
5 um with a cosine throat of radius 0.4 R, a CO2 slug in the first 30 % of the
channel, Ca = 1e-4, dt_vd = 0.1 dt_CFL, N = 12 capillary sub-steps below
the Brackbill limit; mixed precision (FP32 fields, stencils, preconditioner
and inner CG; FP64 pressure, refinement residual, dots and mass sums), with
the FP64 path timed beside it.  Pressure solves: conjugate gradient with the
geometric multigrid preconditioner (--precond jacobi for diagonal scaling)
to a 1e-8 relative FP64 residual.

One timed step = one OSCAR global step = one viscous-drag step followed by
the capillary relaxation with max_iters = N and tol = 0, so every sub-step
runs.  value = relaxation Mcell-iter/s: the sub-steps executed times the
voxels, over the device time of the oscar_capillary_relax calls (HIP events
on the stream the library works on), / 1e6; inputs resident on the device.
The whole-step rate, counting the viscous step as one more iteration over
the wall time of the whole steps, is reported beside it.

Kernel timing: inside the timed steps every 8th conjugate-gradient iteration
is sampled by the library's timing hook (its kernels stamp the device wall
clock at the start and end of every workgroup), giving the execution span of
each part of an iteration; rocprofv3's dispatch interval of the same launch
is that span plus the packet dispatch and completion (1.2-1.7 us, the
committed kernel profile), and the roofline entry gives the fraction with
both.  The roofline entry is the fine-grid kernel with the largest share,
its algorithmic bytes (each array it must read or write counted once per
fluid cell, the face-flag byte once per cell) over its average duration.
The 128 x 64 x 64 working set (168 MB mixed) fits the 256 MB last-level
cache, so its GB/s are effective figures; the 256^3 sphere pack (3 GB),
run beside it, streams from HBM.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIMING_PERIOD = 8
# rocprofv3's kernel duration exceeds the timing hook's span by the packet
# dispatch before the first wave and the completion signal after the last
# (the start stamp follows the kernel's argument loads): 1.55-1.91 us for
# every fine kernel and both precisions (profiles/kernels_mg_cg_*.md)
DISPATCH_US = 1.7

# The paper's own speed-up, quoted beside the measurement as context only: it
# compares whole simulations of its CPU solver (hardware not stated) with the
# same solver's plain PISO time stepping, not a throughput of this path.
PAPER_CONTEXT = {
    "oscar_vs_piso_speedup": "2.5x / 25x / 250x at Ca = 1e-5 / 1e-6 / 1e-7",
    "workload": "2D water drainage in an oil-wet micromodel (Benchmark cases, micromodel subsection, Table drainage; "
                "the PISO times at these Ca are extrapolated)",
    "hardware": "CPU, not stated by the paper; precision not stated",
    "comparable": False,
}

# parts of a CG iteration reported by the timing hook (index: kernel name)
MG_PARTS = {1: "k_mgcg_dir", 2: "k_mg_fine_down", 3: "coarse levels (k_mg_smooth, k_mg_tail, k_mg_up)",
            4: "k_mg_fine_up"}


def word(precision):
    return 4 if precision == 1 else 8


def jacobi_cg_bytes(precision, n_fluid, nc):
    """k_cg: reads r, w = A D^-1 r, s_old, D^-1, p_old, rAU and x and writes
    p, s, r, w and x (x: the FP64 pressure in the FP64 path, the FP32
    correction in the mixed path); the face-flag byte of every cell."""
    w = word(precision)
    x = 8 if precision == 0 else 4
    return n_fluid * (6 * w + x + 4 * w + x) + nc


def mg_part_bytes(part, precision, n_fluid, nc, nc1):
    """Algorithmic bytes of the fine-grid kernels of one multigrid-preconditioned
    iteration (nc1: cells of the first coarse level).
      k_mgcg_dir:     reads z, rAU, d_old, q_old (q = A z + beta q_old);
                      writes d, q                                        6 w
      k_mg_fine_down: reads r, q, D^-1, rAU, d and x; writes x, r_new, z0
                      (x: FP64 pressure or FP32 correction, read and written)
                      7 w + 2 |x|, + the level-1 right-hand side (nc1 w)
      k_mg_fine_up:   reads z0, rAU, r, D^-1; writes z                   5 w
                      + the level-1 correction (nc1 w)
    plus the face-flag byte of every cell."""
    w = word(precision)
    if part == 1:
        return n_fluid * 6 * w + nc
    if part == 2:
        x = 16 if precision == 0 else 2 * w
        return n_fluid * (7 * w + x) + nc1 * w + nc
    if part == 4:
        return n_fluid * 5 * w + nc1 * w + nc
    return None


def run_gpu(case, precision, steps, warmup, precond=1, timing_period=TIMING_PERIOD):
    import torch

    from paper_2105_10576_amd import oscar

    g = oscar.Oscar(case, precision=precision, device="cuda:0", precond=precond)
    if case.get("solve_mode", 0) == oscar.SOLVE_PERSISTENT:
        timing_period = 0   # the persistent solve has no per-launch stamps
    n_sub = case["n_sub"]
    for _ in range(warmup):
        g.step(max_iters=n_sub, tol=0.0)
    torch.cuda.synchronize()
    if timing_period:
        g.timing(timing_period)
    stream = torch.cuda.current_stream()
    ev = []
    t0 = time.perf_counter()
    pcg = 0
    refine = 0
    for _ in range(steps):
        g.viscous_step(case["dt_vd"])
        st = g.stats()
        pcg += st["pcg_iters_call"]
        refine += st["refine_steps_call"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc, kf, E = g.capillary_relax(case["dt_vd"], n_sub, n_sub, 0.0)
        e1.record(stream)
        ev.append((e0, e1))
        st = g.stats()
        pcg += st["pcg_iters_call"]
        refine += st["refine_steps_call"]
        assert kf == n_sub
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    relax_s = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    parts = {k: g.timing_read(k) for k in range(5)} if timing_period else None
    if timing_period:
        g.timing(0)
    st = g.stats()
    res = dict(seconds=t, relax_seconds=relax_s, pcg_iters=pcg, refine_steps=refine, parts=parts, stats=st,
               iters=steps * (1 + n_sub), relax_iters=steps * n_sub)
    g.close()
    return res


def step_roofline(precision, precond, dim, n_fluid, nc, nc1, iters_per_step, cg_per_step, refine_per_step, sec_per_step):
    """Whole-step algorithmic bytes and the Mcell-iter/s they allow at the
    HBM peak: per relaxation iteration (and the viscous step) the non-CG
    kernels' (35 d + 54) words per fluid cell (advection, curvature,
    assembly, three correctors' predictor, set-up and correction), per CG
    iteration the fine-grid kernels' bytes (multigrid: search direction,
    fine down, fine up; the coarse levels are not counted) or k_cg's, per
    outer refinement step 48 B per fluid cell (k_refine_x, k_refine_res)."""
    w = word(precision)
    if precond == 1:
        cg = sum(mg_part_bytes(k, precision, n_fluid, nc, nc1) for k in (1, 2, 4))
    else:
        cg = jacobi_cg_bytes(precision, n_fluid, nc)
    b = iters_per_step * n_fluid * (35 * dim + 54) * w + cg_per_step * cg + refine_per_step * 48 * n_fluid
    achieved = b / sec_per_step / 1e9
    return {"alg_bytes_per_step": int(b), "achieved_GBs": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "mcell_iter_s_at_peak": round(nc * iters_per_step / (b / (HBM_PEAK_GBS * 1e9)) / 1e6, 1),
            "counts": "non-CG (35d+54) words per fluid cell per iteration, CG fine-grid kernels, 48 B per "
                      "fluid cell per refinement step"}


def kernel_table(r, precision, precond, n_fluid, nc, nc1):
    """Per-part average durations [us] and, for the fine-grid kernels, GB/s."""
    out = {}
    names = MG_PARTS if precond == 1 else {1: "k_cg"}
    for k, name in names.items():
        ms, n = r["parts"][k]
        if n == 0:
            continue
        avg = ms / 1e3 / n
        e = {"avg_us": round(avg * 1e6, 3), "launches_timed": n}
        b = mg_part_bytes(k, precision, n_fluid, nc, nc1) if precond == 1 else jacobi_cg_bytes(precision, n_fluid, nc)
        if b is not None:
            e["alg_bytes"] = b
            e["GBs"] = round(b / avg / 1e9, 1)
        out[name] = e
    ms, n = r["parts"][0]
    out["iteration"] = {"avg_us": round(ms * 1e3 / max(n, 1), 3), "launches_timed": n}
    return out


def dominant(table):
    """the fine-grid kernel (one with algorithmic bytes) of largest average duration"""
    best = None
    for name, e in table.items():
        if "alg_bytes" in e and (best is None or e["avg_us"] > table[best]["avg_us"]):
            best = name
    return best


def kernel_roofline(ktab, dom, precision, cache_resident, traffic=None):
    """The roofline entry of kernel `dom`: algorithmic bytes over the hook's
    execution span, and over the span plus the dispatch interval rocprofv3
    adds (the figure its kernel trace reports)."""
    d = ktab[dom]
    us_d = d["avg_us"] + DISPATCH_US
    gbs_d = d["alg_bytes"] / (us_d * 1e-6) / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": d["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(d["GBs"] / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_launch_us": d["avg_us"],
           "alg_bytes_per_launch": d["alg_bytes"], "launches_timed": d["launches_timed"],
           "avg_launch_us_with_dispatch": round(us_d, 3), "achieved_with_dispatch": round(gbs_d, 1),
           "frac_with_dispatch": round(gbs_d / HBM_PEAK_GBS, 4),
           "timing": "device wall-clock stamps of every %d-th CG iteration of the timed steps (first wave start "
                     "to last wave end); 'with_dispatch' adds the %.1f us packet dispatch and completion that "
                     "rocprofv3's kernel trace includes" % (TIMING_PERIOD, DISPATCH_US)}
    if cache_resident:
        out["note"] = ("effective GB/s: the working set fits the 256 MB last-level cache, so these bytes are "
                       "not all HBM traffic")
    return out


def k7_roofline(ktab, precision, n_fluid, precond):
    """One CG iteration against the Jacobi-PCG unit of traffic (13 words per
    fluid cell per iteration), and the multigrid iteration's own
    fine-grid bytes, over the whole iteration's time (all its launches and
    the gaps between them, from the timing hook)."""
    it = ktab["iteration"]["avg_us"] * 1e-6
    if it <= 0:
        return None
    b13 = 13 * word(precision) * n_fluid
    out = {"bytes_13_words": b13, "avg_iteration_us": ktab["iteration"]["avg_us"],
           "achieved_GBs": round(b13 / it / 1e9, 1), "frac": round(b13 / it / 1e9 / HBM_PEAK_GBS, 4)}
    if precond == 1:
        fine = sum(ktab[k]["alg_bytes"] for k in ("k_mgcg_dir", "k_mg_fine_down", "k_mg_fine_up") if k in ktab)
        out.update(fine_grid_bytes=fine, fine_grid_GBs=round(fine / it / 1e9, 1),
                   fine_grid_frac=round(fine / it / 1e9 / HBM_PEAK_GBS, 4))
    return out


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter passes (profiles/pmc_traffic.json), or None when the
    kernel's sources changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(workload, {}).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def run_reps(case, precision, reps, warmup, max_iters, precond=1, keep_fields=False):
    """One OSCAR global step with max_iters relaxation sub-steps (tol = 0),
    repeated from a fresh context each time (the checkpoint is the initial
    state): warmup untimed repetitions, then reps timed ones; the median
    time (whole step, and the relaxation alone on HIP events) and the kernel
    timing summed over the timed repetitions."""
    import torch

    from paper_2105_10576_amd import oscar

    times, rtimes, pcg, kfs, refs = [], [], [], [], []
    acc = {k: [0.0, 0] for k in range(5)}
    fields = None
    for r in range(warmup + reps):
        g = oscar.Oscar(case, precision=precision, device="cuda:0", precond=precond)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        timed = r >= warmup
        if timed:
            g.timing(TIMING_PERIOD)
        t0 = time.perf_counter()
        g.viscous_step(case["dt_vd"])
        st = g.stats()
        it, ref = st["pcg_iters_call"], st["refine_steps_call"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc, kf, E = g.capillary_relax(case["dt_vd"], case["n_sub"], max_iters, 0.0)
        e1.record(stream)
        st = g.stats()
        it += st["pcg_iters_call"]
        ref += st["refine_steps_call"]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        tr = e0.elapsed_time(e1) / 1e3
        print("[bench] %s %s repetition %d (%s): %.3f s (relaxation %.3f s), k_f %d"
              % (case["name"], "mixed" if precision else "fp64", r, "timed" if timed else "warm-up", t, tr, kf),
              file=sys.stderr, flush=True)
        if timed:
            for k in range(5):
                ms, n = g.timing_read(k)
                acc[k][0] += ms
                acc[k][1] += n
            g.timing(0)
            times.append(t)
            rtimes.append(tr)
            pcg.append(it)
            kfs.append(kf)
            refs.append(ref)
        if keep_fields and r == warmup + reps - 1:   # every repetition starts from the same state
            fields = {f: g.get(f) for f in ("alpha", "p", "U")}
        g.close()
    order = sorted(range(reps), key=lambda x: times[x])
    m = order[len(order) // 2]
    return dict(seconds=times[m], relax_seconds=rtimes[m], pcg_iters=pcg[m], k_f=kfs[m], refine_steps=refs[m],
                parts={k: tuple(v) for k, v in acc.items()}, times=times, fields=fields)


def rel_linf(x, ref, mask):
    """max |x - ref| / max |ref| over the masked entries"""
    import numpy as np

    den = float(np.abs(ref[mask]).max())
    return float(np.abs(x[mask] - ref[mask]).max()) / (den if den > 0 else 1.0)


CONFIGS = {
    "c3": ("micromodel", "2D micromodel 1024x512 (524288 voxels, %d fluid), Ca=1e-5, 1 viscous + %d relaxation "
                         "iterations (of N=%d), tol=0, pressure rtol 1e-8, %s-preconditioned CG"),
    "c5": ("sphere_pack", "3D sphere pack 256^3 (16777216 voxels, %d fluid), Ca=1e-5, 1 viscous + %d relaxation "
                          "iterations (of N=%d), tol=0, pressure rtol 1e-8, %s-preconditioned CG"),
}


def config_legs(config, pc, reps=3, warmup=1, fp64=True):
    """The c3 / c5 protocol: one viscous step and a relaxation of 20
    sub-steps from the initial state, warmup + reps repetitions, median;
    mixed and FP64.  value: relaxation sub-steps x voxels over the
    relaxation's device time."""
    from paper_2105_10576_amd import cases

    make, fmt = CONFIGS[config]
    case = getattr(cases, make)(tol=0.0)
    case["pcg_rtol"] = 1e-8
    nx, ny, nz, dim = case["nx"], case["ny"], case["nz"], case["dim"]
    nc = nx * ny * nz
    nc1 = ((nx + 1) // 2) * ((ny + 1) // 2) * (((nz + 1) // 2) if dim == 3 else 1)
    n_fluid = int((case["mask"] == 0).sum())
    kmax = min(20, case["n_sub"])
    out = {"workload": fmt % (n_fluid, kmax, case["n_sub"], "multigrid" if pc else "Jacobi"),
           "protocol": "%d warm-up + %d repetitions from the initial state, median" % (warmup, reps)}
    fields = {}
    for prec, key in ((1, "mixed"), (0, "fp64")):
        if prec == 0 and not fp64:
            continue
        r = run_reps(case, prec, reps, warmup, kmax, pc, keep_fields=fp64)
        fields[key] = r["fields"]
        ktab = kernel_table(r, prec, pc, n_fluid, nc, nc1)
        dom = dominant(ktab)
        out[key] = {
            "value": round(nc * r["k_f"] / r["relax_seconds"] / 1e6, 3),
            "whole_step_mcell_iter_s": round(nc * (1 + r["k_f"]) / r["seconds"] / 1e6, 3),
            "ms_per_step": round(1e3 * r["seconds"], 3), "relax_ms": round(1e3 * r["relax_seconds"], 3),
            "k_f": r["k_f"], "pcg_iters_per_step": r["pcg_iters"], "refine_steps_per_step": r["refine_steps"],
            "rep_seconds": [round(t, 4) for t in r["times"]],
            "roofline": kernel_roofline(ktab, dom, prec, cache_resident=nc * 4 * 30 < (256 << 20),
                                        traffic=measured_traffic(dom, case["name"]) if prec == 1 else None),
            "k7_iteration": k7_roofline(ktab, prec, n_fluid, pc),
            "kernels": ktab,
            "step_roofline": step_roofline(prec, pc, dim, n_fluid, nc, nc1, 1 + r["k_f"], r["pcg_iters"],
                                           r["refine_steps"], r["seconds"]),
        }
    if fp64:
        import numpy as np

        fl = case["mask"].reshape(-1) == 0
        a, b = fields["mixed"], fields["fp64"]
        out["mixed"]["error_vs_fp64_gpu"] = {
            "alpha": rel_linf(a["alpha"], b["alpha"], fl), "p": rel_linf(a["p"], b["p"], fl),
            "U": rel_linf(a["U"], b["U"], np.tile(fl, dim)),
            "note": "the same step on the FP64 GPU path (both to pressure rtol 1e-8), relative L-infinity over the "
                    "fluid cells; the FP64 path matches the FP64 oracle on a sample of this medium "
                    "(tests/test_gpu_fullsize.py)"}
    return out


def bench_config(args):
    """--config c3|c5 alone (one JSON line)."""
    pc = 1 if args.precond == "mg" else 0
    legs = config_legs(args.config, pc, fp64=not args.no_fp64)
    m = legs["mixed"]
    out = {"metric": "relaxation Mcell-iter/s (mixed FP32 + FP64 refinement), HBM GB/s of the dominant kernel",
           "value": m["value"], "unit": "Mcell-iter/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic (seeded %s geometry)" % CONFIGS[args.config][0],
           "config": {"workload": legs["workload"], "precision": "mixed", "protocol": legs["protocol"],
                      "whole_step_mcell_iter_s": m["whole_step_mcell_iter_s"],
                      "pcg_iters_per_step": m["pcg_iters_per_step"]},
           "roofline": m["roofline"], "k7_iteration": m["k7_iteration"], "kernels": m["kernels"],
           "step_roofline": m["step_roofline"]}
    if "fp64" in legs:
        out["fp64"] = legs["fp64"]
        out["error_vs_fp64_gpu"] = m["error_vs_fp64_gpu"]
    print(json.dumps(out), flush=True)


def cpu_baseline(case, precond=1):
    """The FP64 oracle on the host, single-threaded: one viscous-drag step of
    the workload (to reach a flowing state), then the first capillary
    sub-step, which is timed: one relaxation iteration over every voxel, the
    unit of the metric.  The same prefix on the GPU (both paths, from the
    same initial state) is compared with it: relative L-infinity error of
    alpha, p and U."""
    import numpy as np

    from oracle.pyoracle import Oracle
    from paper_2105_10576_amd import oscar

    o = Oracle(case)
    t0 = time.perf_counter()
    o.viscous_step(case["dt_vd"])
    t_vd = time.perf_counter() - t0
    it_vd = o.stats()["pcg_iters_step"]
    t0 = time.perf_counter()
    o.capillary_relax(case["dt_vd"], case["n_sub"], 1, 0.0)
    t = time.perf_counter() - t0
    it_cr = o.stats()["pcg_iters_step"]
    nc = case["nx"] * case["ny"] * case["nz"]
    err = {}
    for prec, name in ((1, "mixed"), (0, "fp64")):
        g = oscar.Oscar(case, precision=prec, device="cuda:0", precond=precond)
        g.viscous_step(case["dt_vd"])
        g.capillary_relax(case["dt_vd"], case["n_sub"], 1, 0.0)
        e = {}
        for f in ("alpha", "p", "U"):
            ref = o.get(f)
            den = float(np.abs(ref).max()) or 1.0
            e[f] = float("%.3g" % (float(np.abs(g.get(f) - ref).max()) / den))
        err[name] = e
        g.close()
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=nc / t / 1e6, unit="Mcell-iter/s", cores=1, kind="oracle",
                host=dict(cpu=cpu, threads_available=os.cpu_count()),
                sample="the first capillary sub-step of the same workload (one relaxation iteration over the "
                       "524288 voxels, 3 PISO correctors, %d Jacobi-PCG iterations, %.1f s), after its viscous "
                       "step (%d iterations, %.1f s, not timed); single-threaded FP64 oracle, pressure rtol 1e-8"
                       % (it_cr, t, it_vd, t_vd),
                error_vs_oracle=dict(err, prefix="the same prefix (viscous step + first sub-step) on the GPU, "
                                                 "relative L-infinity; both sides solve to the workload's "
                                                 "pressure rtol"))


def persistent_line(args, case, pc, nc):
    """--solve-mode persistent: the c2 mixed relaxation rate and the serving
    figures with every pressure solve run as one persistent launch."""
    from paper_2105_10576_amd import oscar, serving_bench

    case = dict(case, solve_mode=oscar.SOLVE_PERSISTENT)
    r = run_gpu(case, 1, args.steps, args.warmup, precond=pc)
    out = {"metric": "relaxation Mcell-iter/s (mixed FP32 + FP64 refinement), persistent pressure solves",
           "value": round(r["relax_iters"] * nc / r["relax_seconds"] / 1e6, 3), "unit": "Mcell-iter/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * r["seconds"] / args.steps, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (seeded constricted-channel geometry and CO2 slug)",
           "config": {"workload": "3D constricted channel 128x64x64, N=%d sub-steps, tol=0, pressure rtol 1e-8"
                                  % case["n_sub"], "solve_mode": "persistent",
                      "pcg_iters_per_step": round(r["pcg_iters"] / args.steps, 1)},
           "roofline": None}
    if not args.no_serving:
        out["serving"] = serving_bench.run(n_requests=args.serving_requests, max_iters=args.serving_max_iters,
                                           precond=pc, solve_mode=oscar.SOLVE_PERSISTENT, burst_only=True)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg",
                    help="preconditioner of the pressure conjugate gradient")
    ap.add_argument("--config", choices=["c2", "c3", "c5"], default="c2",
                    help="c2: the default run (the 3D channel, with the 256^3 sphere pack and serving beside it); "
                         "c3 (2D micromodel 1024x512) or c5 (3D sphere pack 256^3) alone")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path beside the mixed path")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving measurement")
    ap.add_argument("--no-sphere", action="store_true", help="skip the 256^3 sphere-pack legs")
    ap.add_argument("--pmc-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--solve-mode", choices=["launches", "persistent"], default="launches",
                    help="persistent: every pressure solve as one launch over a device work queue (bitwise the "
                         "same results); prints the c2 mixed value and the serving figures only")
    ap.add_argument("--serving-max-iters", type=int, default=200,
                    help="cap on relaxation sub-steps per serving request (the mix allows up to 200)")
    args = ap.parse_args()
    if args.pmc_calibration:
        import torch

        a = torch.ones(args.pmc_calibration << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_calibration_copy_bytes": a.numel(), "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2105_10576_amd import cases

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.config != "c2":
        bench_config(args)
        return
    case = cases.constricted_channel(tol=0.0)
    case["pcg_rtol"] = 1e-8   # pressure solves to a 1e-8 relative residual on both paths
    nx, ny, nz = case["nx"], case["ny"], case["nz"]
    nc = nx * ny * nz
    nc1 = ((nx + 1) // 2) * ((ny + 1) // 2) * ((nz + 1) // 2)
    n_fluid = int((case["mask"] == 0).sum())
    n_sub = case["n_sub"]
    pc = 1 if args.precond == "mg" else 0
    if args.solve_mode == "persistent":
        persistent_line(args, case, pc, nc)
        return

    mixed = run_gpu(case, 1, args.steps, args.warmup, precond=pc)
    value = mixed["relax_iters"] * nc / mixed["relax_seconds"] / 1e6
    ms_step = 1e3 * mixed["seconds"] / args.steps
    ktab = kernel_table(mixed, 1, pc, n_fluid, nc, nc1)
    dom = dominant(ktab)

    out = {
        "metric": "relaxation Mcell-iter/s (mixed FP32 + FP64 refinement), HBM GB/s of the dominant kernel",
        "value": round(value, 3),
        "unit": "Mcell-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded constricted-channel geometry and CO2 slug)",
        "config": {
            "workload": "3D constricted channel 128x64x64 (524288 voxels, %d fluid), Ca=1e-4, N=%d sub-steps, "
                        "1 viscous + %d relaxation iterations per step, tol=0, pressure rtol 1e-8, "
                        "%s-preconditioned CG" % (n_fluid, n_sub, n_sub, "multigrid" if pc else "Jacobi"),
            "precision": "mixed",
            "value_counts": "relaxation sub-steps x voxels over the device time of the oscar_capillary_relax "
                            "calls (HIP events on the library's stream)",
            "relax_ms_per_step": round(1e3 * mixed["relax_seconds"] / args.steps, 3),
            "whole_step_mcell_iter_s": round(mixed["iters"] * nc / mixed["seconds"] / 1e6, 3),
            "whole_step_counts": "(1 + N) iterations per voxel and step (the viscous step as one) over the wall "
                                 "time of the whole steps",
            "pcg_iters_per_step": round(mixed["pcg_iters"] / args.steps, 1),
            "refine_steps_per_step": round(mixed["refine_steps"] / args.steps, 1),
        },
        "roofline": kernel_roofline(ktab, dom, 1, cache_resident=True, traffic=measured_traffic(dom, case["name"])),
        "k7_iteration": k7_roofline(ktab, 1, n_fluid, pc),
        "kernels": ktab,
        "step_roofline": step_roofline(1, pc, 3, n_fluid, nc, nc1, mixed["iters"] / args.steps,
                                       mixed["pcg_iters"] / args.steps, mixed["refine_steps"] / args.steps,
                                       mixed["seconds"] / args.steps),
    }
    if not args.no_fp64:
        f = run_gpu(case, 0, args.fp64_steps, 1, precond=pc)
        ftab = kernel_table(f, 0, pc, n_fluid, nc, nc1)
        fdom = dominant(ftab)
        out["fp64"] = {
            "value": round(f["relax_iters"] * nc / f["relax_seconds"] / 1e6, 3),
            "whole_step_mcell_iter_s": round(f["iters"] * nc / f["seconds"] / 1e6, 3),
            "ms_per_step": round(1e3 * f["seconds"] / args.fp64_steps, 3),
            "steps": args.fp64_steps,
            "pcg_iters_per_step": round(f["pcg_iters"] / args.fp64_steps, 1),
            "roofline": kernel_roofline(ftab, fdom, 0, cache_resident=False),
            "k7_iteration": k7_roofline(ftab, 0, n_fluid, pc),
            "kernels": ftab,
            "step_roofline": step_roofline(0, pc, 3, n_fluid, nc, nc1, f["iters"] / args.fp64_steps,
                                           f["pcg_iters"] / args.fp64_steps, 0, f["seconds"] / args.fp64_steps),
        }
        out["fp64"]["roofline"].pop("note", None)
        out["fp64"]["roofline"]["note"] = ("FP64 working set 309 MB, about the size of the 256 MB last-level "
                                          "cache: partly cache-resident")
    if not args.no_sphere:
        out["sphere_pack"] = config_legs("c5", pc, reps=2, warmup=1, fp64=not args.no_fp64)
    if not args.no_serving:
        from paper_2105_10576_amd import serving_bench

        out["serving"] = serving_bench.run(n_requests=args.serving_requests, max_iters=args.serving_max_iters,
                                           precond=1 if args.precond == "mg" else 0,
                                           log=lambda m: print("[serving] " + m, file=sys.stderr, flush=True))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, pc)
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
