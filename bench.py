"""Benchmark of the OSCAR relaxation path on one MI355X.

Workload (default): the 3D constricted channel, 128 x 64 x 64 voxels at
5 um with a cosine throat of radius 0.4 R, a CO2 slug in the first 30 % of the
channel, Ca = 1e-4, dt_vd = 0.1 dt_CFL, N = 12 capillary sub-steps below
the Brackbill limit; mixed precision (FP32 fields and CG, FP64 pressure,
refinement residual, dots and mass sums), with the FP64 path timed beside it.

One timed step = one OSCAR global step = one viscous-drag step followed by
the capillary relaxation with max_iters = N and tol = 0, so every sub-step
runs.  The metric counts (1 + N) cell-iterations per cell and step (the
viscous step counts as one iteration); value = total cell-iterations / wall
time of the K timed steps / 1e6, inputs resident on the device.

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


def cg_bytes_per_fluid_cell(precision):
    """Algorithmic bytes the conjugate-gradient iteration kernel moves per
    fluid cell: it reads r, w = A D^-1 r, s_old, D^-1, p_old, rAU and x and
    writes p, s, r, w and x (x is the FP64 pressure in the FP64 path, the FP32
    correction in the mixed path); every cell also reads its face-flag byte."""
    w = 4 if precision == 1 else 8
    x = 8 if precision == 0 else 4
    return 6 * w + x + 4 * w + x


def run_gpu(case, precision, steps, warmup, timing=True, precond=0):
    import torch

    from paper_2105_10576_amd import oscar

    g = oscar.Oscar(case, precision=precision, device="cuda:0", precond=precond)
    n_sub = case["n_sub"]
    for _ in range(warmup):
        g.step(max_iters=n_sub, tol=0.0)
    torch.cuda.synchronize()
    if timing:
        g.timing(True)
    t0 = time.perf_counter()
    pcg = 0
    for _ in range(steps):
        g.viscous_step(case["dt_vd"])
        pcg += g.stats()["pcg_iters_call"]
        rc, kf, E = g.capillary_relax(case["dt_vd"], n_sub, n_sub, 0.0)
        st = g.stats()
        pcg += st["pcg_iters_call"]
        assert kf == n_sub
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    kt = g.timing_read(0) if timing else None
    if timing:
        g.timing(False)
    st = g.stats()
    res = dict(seconds=t, pcg_iters=pcg, kernel_times=kt, stats=st,
               iters=steps * (1 + n_sub))
    g.close()
    return res


def cpu_baseline(case):
    """The FP64 oracle on the host: the first viscous-drag step of the same
    workload (3 PISO correctors with Jacobi-PCG), one cell-iteration per cell."""
    from oracle.pyoracle import Oracle

    o = Oracle(case)
    t0 = time.perf_counter()
    rc = o.viscous_step(case["dt_vd"])
    t = time.perf_counter() - t0
    nc = case["nx"] * case["ny"] * case["nz"]
    return dict(value=nc / t / 1e6, unit="Mcell-iter/s", cores=1, kind="oracle",
                sample="first viscous-drag step of the same grid (1 cell-iteration per cell, %d PCG iterations), "
                       "single-threaded FP64 oracle, %.1f s" % (o.stats()["pcg_iters_step"], t))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path beside the mixed path")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving measurement")
    ap.add_argument("--pmc-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--precond", choices=["mg", "jacobi"], default="mg",
                    help="preconditioner of the pressure conjugate gradient")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-max-iters", type=int, default=40,
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
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2105_10576_amd import cases

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    case = cases.constricted_channel(tol=0.0)
    case["pcg_rtol"] = 1e-8   # pressure solves to a 1e-8 relative residual on both paths
    nc = case["nx"] * case["ny"] * case["nz"]
    n_fluid = int((case["mask"] == 0).sum())
    n_sub = case["n_sub"]

    pc = 1 if args.precond == "mg" else 0
    mixed = run_gpu(case, 1, args.steps, args.warmup, precond=pc)
    value = mixed["iters"] * nc / mixed["seconds"] / 1e6
    ms_step = 1e3 * mixed["seconds"] / args.steps

    # dominant kernel: the conjugate-gradient iteration kernel
    ms_tot, launches = mixed["kernel_times"]
    avg_s = ms_tot / 1e3 / max(launches, 1)
    alg_bytes = n_fluid * cg_bytes_per_fluid_cell(1) + nc
    achieved = alg_bytes / avg_s / 1e9

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
                        "1 viscous + %d relaxation iterations per step, tol=0, pressure rtol 1e-8" % (n_fluid, n_sub, n_sub),
            "precision": "mixed",
            "pcg_iters_per_step": round(mixed["pcg_iters"] / args.steps, 1),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_cg",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "avg_launch_us": round(avg_s * 1e6, 3),
            "alg_bytes_per_launch": alg_bytes,
            "launches": launches,
        },
    }
    if not args.no_fp64:
        f = run_gpu(case, 0, args.fp64_steps, 1, precond=pc)
        ms64, n64 = f["kernel_times"]
        avg64 = ms64 / 1e3 / max(n64, 1)
        b64 = n_fluid * cg_bytes_per_fluid_cell(0) + nc
        out["fp64"] = {
            "value": round(f["iters"] * nc / f["seconds"] / 1e6, 3),
            "ms_per_step": round(1e3 * f["seconds"] / args.fp64_steps, 3),
            "steps": args.fp64_steps,
            "pcg_iters_per_step": round(f["pcg_iters"] / args.fp64_steps, 1),
            "dominant_kernel": "k_cg",
            "achieved_GBs": round(b64 / avg64 / 1e9, 1),
            "avg_launch_us": round(avg64 * 1e6, 3),
        }
    if not args.no_serving:
        from paper_2105_10576_amd import serving_bench

        out["serving"] = serving_bench.run(n_requests=args.serving_requests, max_iters=args.serving_max_iters,
                                           log=lambda m: print("[serving] " + m, file=sys.stderr, flush=True))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
