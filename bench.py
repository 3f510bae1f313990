"""Benchmark of the MI355X least-squares h-p spectral element hot path.

One step = one PCG iteration on the normal equations: the matrix-free
operator apply (element volume residual and its adjoint, face jumps and
boundary terms, corner reduction), the block-diagonal preconditioner solve
and the CG vector updates and inner products, all on the GPU.

Prints one JSON line.  value = PCG iterations x DOF / s on one GPU with all
inputs resident in HBM.  Also reports the time to solve to the relative
residual 1e-10, the roofline of the dominant kernel (HIP events on the
launch stream), and the FP64 oracle timed on the host cores for a bounded
sample (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector / matrix, FLOP/s
PEAK_HBM = 8.0e12        # bytes/s


def make_workload(name):
    from workloads import mesh as M
    from workloads.problems import SinProduct, RhoPower
    if name == "cube_w4":
        return (M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1), name="unit cube 2x2x2, W=4"),
                SinProduct(), dict(workload="poisson_unit_cube_2x2x2", W=4, N=1))
    if name.startswith("fichera"):
        from workloads.fichera import fichera_mesh
        N = int(name.split("_n")[1])
        mesh = fichera_mesh(N=N, W=N)
        return mesh, RhoPower(2.0 / 3.0), dict(workload="poisson_fichera", N=N, W=N, mu=0.15)
    raise SystemExit("unknown workload %s" % name)


def volume_work(counts, W):
    """Algorithmic FLOPs and HBM bytes of one launch of the element kernel.

    Per element: forward + adjoint sum-factorised contractions (factor 2 x 2
    for multiply-add), 1 / 3 / nf contractions per stage for the diagonal
    Laplacian (2, 3, 3) or the general operator (3, 6, nf), the pointwise
    residual (2 nf) and its adjoint weighting (nf).  Bytes: the coefficient
    fields, u in, q out, traces out.
    """
    n, m = W + 1, 2 * W + 1
    E, Eg, nf = counts["real_elements"], counts["general_elements"], counts["fields"]
    Ed = E - Eg
    fl = 4 * (Ed * (2 * m * n ** 3 + 3 * m * m * n * n) + Eg * (3 * m * n ** 3 + 6 * m * m * n * n)
              + nf * m ** 3 * n) + 3 * nf * m ** 3
    by = 8 * (nf * m ** 3 + 2 * E * n ** 3 + counts["slots"] * 4 * n * n)
    return float(fl), float(by)


def cpu_baseline(name, mesh, problem, budget_s=20.0):
    """FP64 oracle (apply_X + preconditioner = one PCG iteration's work) on the host cores.

    Fichera workloads: a bounded sample, the N = 1 Fichera mesh at the same
    degree W (the same element types: vertex patches, vertex-edge and edge
    boxes, corner elements, curved regular columns), scaled per DOF."""
    from oracle.functional import Discretization
    from oracle.precond import BlockPreconditioner
    sample = "full workload"
    if name.startswith("fichera"):
        from workloads.fichera import fichera_mesh
        mesh = fichera_mesh(N=1, W=mesh.W)
        sample = "Fichera N=1 mesh at the same W (%d real elements)" % int((mesh.kind == 0).sum())
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        pass
    t0 = time.perf_counter()
    disc = Discretization(mesh, problem)
    P = BlockPreconditioner(disc)
    setup = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    u = rng.standard_normal(disc.ndof)
    its = 0
    t0 = time.perf_counter()
    while True:
        q = disc.apply_X(u)
        P.apply(q)
        its += 1
        if time.perf_counter() - t0 > budget_s or its >= 50:
            break
    dt = (time.perf_counter() - t0) / its
    return dict(value=disc.ndof / dt, unit="PCG iterations x DOF / s", cores=int(threads), kind="oracle",
                sample="%s: %d operator+preconditioner applies (one PCG iteration each), %d DOF, "
                       "%.3f s per iteration, oracle setup %.1f s" % (sample, its, disc.ndof, dt, setup))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=os.environ.get("SEM_BENCH_WORKLOAD", "fichera_n6"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the element-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1110_2316_amd import setup_problem

    torch.cuda.set_device(0)
    mesh, problem, cfg = make_workload(args.workload)
    print("bench: workload %s, %d elements" % (cfg["workload"], mesh.E), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = setup_problem(mesh, problem)
    setup_s = time.perf_counter() - t0
    ndof = ctx.ndof
    b = torch.zeros(ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    # warmup: exactly `warmup` iterations (rtol 0 never stops early)
    ctx.pcg_solve(b, u, rtol=0.0, maxit=max(args.warmup, 1), raise_on_fail=False)
    torch.cuda.synchronize()
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.pcg_solve(b, u, rtol=0.0, maxit=args.steps, raise_on_fail=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info["iterations"] == args.steps, info
    value = args.steps * ndof / dt
    print("bench: %d iterations in %.4f s" % (args.steps, dt), file=sys.stderr, flush=True)

    # time to solution (FP64): relative residual 1e-10 from u0 = 0
    uref = torch.zeros_like(b)
    ctx.pcg_solve(b, uref, rtol=1e-13, maxit=20000, raise_on_fail=False)
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info_s = ctx.pcg_solve(b, u, rtol=1e-10, maxit=20000, raise_on_fail=False)
    torch.cuda.synchronize()
    tts = time.perf_counter() - t0
    sol_err = float(torch.linalg.norm(u - uref) / torch.linalg.norm(uref))
    xe = ctx.error_points()
    h1 = ctx.error(uref, problem.u(xe), problem.grad_u(xe))

    # roofline of the dominant kernel: HIP events on the launch stream
    counts = ctx.work_counts()
    ms = ctx.kernel_times(uref, reps=50)
    names = ["volume", "face", "gather", "update"]
    k = int(np.argmax(ms))
    fl, by = volume_work(counts, mesh.W)
    t_vol = ms[0] * 1e-3
    intensity = fl / by
    if intensity >= PEAK_FP64 / PEAK_HBM:
        roof = dict(bound="alu", achieved=fl / t_vol / 1e12, peak=PEAK_FP64 / 1e12, unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=by / t_vol / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = "k_volume (element volume residual + adjoint + traces)"
    roof["algorithmic_flops"] = fl
    roof["algorithmic_bytes"] = by
    roof["avg_ms"] = ms[0]

    out = dict(metric="PCG iterations x DOF / s (FP64 path)", value=value, unit="iterations*DOF/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * dt / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(cfg, elements=int(counts["elements"]), real_elements=int(counts["real_elements"]),
                           dof=int(ndof)),
               time_to_solution_s=tts, tts_iterations=info_s["iterations"], tts_rel_residual=info_s["rel_residual"],
               tts_solution_rel_error=sol_err, h1_rel_error=h1, setup_s=setup_s,
               kernel_ms=dict(zip(names, [float(v) for v in ms])), dominant_kernel=names[k],
               roofline=roof)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, mesh, problem, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
