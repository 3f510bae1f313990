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
PEAK_FP32 = 157.3e12     # MI355X FP32 vector, FLOP/s
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


def kernel_work(counts, W, fp32=False):
    """Algorithmic FLOPs and HBM bytes of one launch of each kernel of an
    iteration: what the method must do per element (the sum-factorised
    contractions, the coefficient fields, vectors and face data, an O(n^4)
    block-diagonal preconditioner), not the dense element matrices a
    particular preconditioner stores.  S = bytes per operator value (8 FP64,
    4 float); vectors are FP64.

    volume: forward + adjoint sum-factorised contractions (x2 multiply-add,
      x2 forward and adjoint) of 1/2/3 stages with 1 / 3 / nf variants for the
      Laplacian-only fields (2, 3 variants) or the general operator (3, 6),
      the pointwise residual and its weighting (3 nf per point); bytes: the
      active coefficient fields, u in, q out, traces out (4 n^2 per slot).
    face: per face term, 4 quantities: the trace interpolation to the m x m
      grid and back (32 (m n^2 + m^2 n)) and the fractional-norm weighting
      (16 m^3 + 12 m^2); bytes: traces in, face results out, coefficients.
    gather: bytes of the face results and q in, q out.
    update: the preconditioner solve of the method, 12 n^4 + n^3 per element
      (three n x n contractions, a diagonal scale, three more); r in, z out.
    """
    n, m = W + 1, 2 * W + 1
    S = 4 if fp32 else 8
    E, Eg, nf = counts["real_elements"], counts["general_elements"], counts["fields"]
    Ed = E - Eg
    slots, ndof, nfaces = counts["slots"], counts["ndof"], counts["faces"]
    fl_v = 4 * (Ed * (2 * m * n ** 3 + 3 * m * m * n * n) + Eg * (3 * m * n ** 3 + 6 * m * m * n * n)
                + nf * m ** 3 * n) + 3 * nf * m ** 3
    by_v = S * nf * m ** 3 + 8 * 2 * E * n ** 3 + S * slots * 4 * n * n
    fl_f = nfaces * (32 * (m * n * n + m * m * n) + 16 * m ** 3 + 12 * m * m)
    by_f = S * (2 * slots * 4 * n * n + counts["face_coef_doubles"])
    by_g = S * slots * 4 * n * n + 8 * 2 * E * n ** 3
    fl_u = E * (12 * n ** 4 + n ** 3)
    by_u = 8 * 2 * ndof
    return dict(volume=(float(fl_v), float(by_v)), face=(float(fl_f), float(by_f)), gather=(0.0, float(by_g)),
                update=(float(fl_u), float(by_u)))


def iteration_work(counts, W, fp32=False):
    """Algorithmic FLOPs and HBM bytes of one whole PCG iteration: the four
    kernels above plus the CG vector work (about 10 FLOPs and 7 FP64 vector
    reads or writes per unknown: u, p, r, q, z updates, two inner products)."""
    work = kernel_work(counts, W, fp32)
    ndof = counts["ndof"]
    fl = sum(v[0] for v in work.values()) + 10 * ndof
    by = sum(v[1] for v in work.values()) + 7 * 8 * ndof
    return fl, by


TRAFFIC_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1110_2316_amd", "csrc", "sem_kernels.hip")


def measured_traffic(workload, path, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a copy of known size), or None
    when there is none or the kernel source changed since it was taken."""
    import hashlib
    f = os.path.join(TRAFFIC_DIR, "traffic_%s.json" % workload)
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        rec = json.load(fh)
    with open(KERNEL_SOURCE, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if rec.get("kernel_source_sha256") != digest:
        return None
    ent = rec.get("paths", {}).get(path, {}).get(kernel)
    return None if ent is None else float(ent["bytes_per_launch"])


def _roof(fl, by, t, fp32):
    peak_fl = PEAK_FP32 if fp32 else PEAK_FP64
    if by > 0 and fl / by < peak_fl / PEAK_HBM:
        r = dict(bound="hbm", achieved=by / t / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s")
    else:
        r = dict(bound="alu", achieved=fl / t / 1e12, peak=peak_fl / 1e12, unit="TFLOP/s")
    r["frac"] = r["achieved"] / r["peak"]
    return r


KERNEL_FAMILIES = ("k_volume", "k_face", "k_gather", "k_update_mfma", "k_update", "k_cg_vec", "k_fin_update")


def _counter_rows(d):
    """(dispatch id, kernel name, counter name, value) rows of the rocprofv3
    counter CSVs under d, in dispatch order."""
    import csv
    import glob
    import gzip
    rows = []
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    files += glob.glob(os.path.join(d, "**", "*counter_collection.csv.gz"), recursive=True)
    for f in files:
        with (gzip.open(f, "rt") if f.endswith(".gz") else open(f)) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return sorted(rows)


def _path_instance(kname, path):
    """The kernel family of a dispatch of the given path (mixed: the float
    element kernels and the float block apply; fp64: the double ones), or None."""
    for k in KERNEL_FAMILIES:
        if ("sem::" + k + "<") in kname or ("sem::" + k + "(") in kname:
            if "<" in kname and k != "k_update":
                targs = kname.split("<", 1)[1].split(">", 1)[0]
                if k == "k_update_mfma":
                    want = ", 3" if path == "mixed" else ", 1"
                    if not targs.endswith(want):
                        return None
                elif ("float" in targs) != (path == "mixed"):
                    return None
            return k
    return None


def summarize_counters(fetch_dir, write_dir, workload, path, calib_bytes=1 << 30, reps=20, copies=5):
    """profiles/traffic_<workload>.json from two rocprofv3 --pmc passes
    (FETCH_SIZE, WRITE_SIZE: KiB per dispatch) of bench.py --profile-kernels
    --copy-calibration.  Per kernel family of the path, the mean over its
    last `reps` dispatches (the timed launches; set-up launches of the same
    kernels come earlier), scaled by what the same counter reads for the
    elementwise 1 GiB copy (the last `copies` elementwise dispatches; bytes
    per launch = KiB / factor x 1024), with the kernel source's hash so that
    a changed kernel drops the figure."""
    import hashlib
    out = {}
    factors = {}
    for cname, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r[2].startswith(cname)]
        copy = [v for _, kname, _, v in rows if "elementwise" in kname][-copies:]
        if len(copy) < copies:
            raise SystemExit("no calibration copy among the %s dispatches" % cname)
        factors[cname] = float(np.mean(copy)) / (calib_bytes / 1024.0)
        fam = {}
        for _, kname, _, v in rows:
            k = _path_instance(kname, path)
            if k is not None:
                fam.setdefault(k, []).append(v)
        for k, vals in fam.items():
            vals = vals[-reps:]
            out.setdefault(k, {})[cname + "_KiB"] = float(np.mean(vals))
            out[k][cname + "_dispatches"] = len(vals)
    for k, ent in out.items():
        by = 0.0
        for cname in ("FETCH_SIZE", "WRITE_SIZE"):
            if cname + "_KiB" in ent:
                by += ent[cname + "_KiB"] / factors[cname] * 1024.0
        ent["bytes_per_launch"] = by
    with open(KERNEL_SOURCE, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    fpath = os.path.join(TRAFFIC_DIR, "traffic_%s.json" % workload)
    rec = {}
    if os.path.exists(fpath):
        with open(fpath) as fh:
            rec = json.load(fh)
    if rec.get("kernel_source_sha256") != digest:
        rec = {"kernel_source_sha256": digest, "paths": {}}
    rec["paths"][path] = out
    rec.setdefault("calibration", {})[path] = dict(copy_bytes=calib_bytes, factors=factors)
    with open(fpath, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    return fpath


def summarize_sq(dirs, workload, path, reps=20):
    """profiles/counters_<workload>_<path>.json from rocprofv3 --pmc passes of
    SQ (shader sequencer) counters over bench.py --profile-kernels: per kernel
    family of the path, each counter's mean over its last `reps` dispatches,
    and ratios of counters of the same scope (per-wave accumulations over
    wave cycles; LDS conflict cycles over LDS-active cycles)."""
    import hashlib
    fam = {}
    for d in dirs:
        for _, kname, cname, v in _counter_rows(d):
            k = _path_instance(kname, path)
            if k is not None:
                fam.setdefault(k, {}).setdefault(cname, []).append(v)
    out = {}
    for k, cs in fam.items():
        ent = {c: float(np.mean(v[-reps:])) for c, v in cs.items()}
        g = ent.get
        r = {}
        if g("SQ_WAVE_CYCLES"):
            for c, name in (("SQ_ACTIVE_INST_LDS", "lds_issue_per_wave_cycle"),
                            ("SQ_WAIT_INST_LDS", "lds_wait_per_wave_cycle"),
                            ("SQ_ACTIVE_INST_VALU", "valu_issue_per_wave_cycle"),
                            ("SQ_ACTIVE_INST_ANY", "any_issue_per_wave_cycle")):
                if g(c) is not None:
                    r[name] = g(c) / g("SQ_WAVE_CYCLES")
        if g("SQ_LDS_IDX_ACTIVE"):
            r["lds_bank_conflict_per_lds_active_cycle"] = g("SQ_LDS_BANK_CONFLICT", 0.0) / g("SQ_LDS_IDX_ACTIVE")
        if g("SQ_BUSY_CYCLES") and g("SQ_VALU_MFMA_BUSY_CYCLES") is not None:
            r["mfma_busy_per_sq_busy_cycle"] = g("SQ_VALU_MFMA_BUSY_CYCLES") / g("SQ_BUSY_CYCLES")
        if g("SQ_INSTS_VALU") and g("SQ_INSTS_LDS") is not None:
            r["lds_insts_per_valu_inst"] = g("SQ_INSTS_LDS") / g("SQ_INSTS_VALU")
        out[k] = dict(counters=ent, ratios=r, dispatches=min(min(len(v), reps) for v in cs.values()))
    with open(KERNEL_SOURCE, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    fpath = os.path.join(TRAFFIC_DIR, "counters_%s_%s.json" % (workload, path))
    with open(fpath, "w") as fh:
        json.dump(dict(kernel_source_sha256=digest, path=path, kernels=out), fh, indent=1, sort_keys=True)
    return fpath


def summarize_trace(trace_dir, workload, path, log, command, reps=20):
    """profiles/kernels_<workload>_<path>.md from a rocprofv3 --kernel-trace
    --stats --output-format csv run of bench.py --profile-kernels: the mean
    duration of each kernel family's last `reps` dispatches of the path (the
    timed launches, the same ones the HIP events of the run time; its
    printed kernel_ms line is read from `log`), and the top of rocprofv3's own
    statistics over every dispatch of the run (set-up included)."""
    import csv
    import glob
    import gzip

    def rows(pattern):
        out = []
        for f in glob.glob(os.path.join(trace_dir, "**", pattern), recursive=True) + \
                glob.glob(os.path.join(trace_dir, "**", pattern + ".gz"), recursive=True):
            with (gzip.open(f, "rt") if f.endswith(".gz") else open(f)) as fh:
                out += list(csv.DictReader(fh))
        return out
    disp = sorted(rows("*kernel_trace.csv"), key=lambda r: int(r["Dispatch_Id"]))
    fam = {}
    for r in disp:
        k = _path_instance(r["Kernel_Name"], path)
        if k is not None:
            fam.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    events = None
    for line in open(log):
        if line.startswith("{") and "kernel_ms" in line:
            events = dict(zip(["k_volume", "k_face", "k_gather", "k_update"], json.loads(line)["kernel_ms"]))
    stats = rows("*kernel_stats.csv")
    lines = ["# Kernel trace: %s, %s path" % (workload, path), "",
             "Command (run from /tmp with TMPDIR=/tmp on an MI355X):", "", "    " + command, "",
             "Timed dispatches (the last %d of each kernel of the path; HIP events of the same run):" % reps, "",
             "| kernel | dispatches | rocprofv3 mean us | HIP events us |", "|---|---|---|---|"]
    for k in ("k_volume", "k_face", "k_gather", "k_update_mfma", "k_update"):
        if k in fam:
            ev = events.get("k_update" if k.startswith("k_update") else k) if events else None
            lines.append("| %s | %d | %.1f | %s |" % (k, min(reps, len(fam[k])), float(np.mean(fam[k][-reps:])),
                                                      "%.1f" % (1e3 * ev) if ev is not None else "-"))
    lines += ["", "rocprofv3 statistics over every dispatch of the run (top 15):", "",
              "| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in stats[:15]:
        name = r["Name"].split("(")[0].replace("void ", "")
        if name.startswith("Cijk_"):
            name = "rocBLAS GEMM " + "_".join(name.split("_")[:4])
        lines.append("| %s | %s | %.1f | %.2f | %.2f |" % (name, r["Calls"], float(r["AverageNs"]) / 1e3,
                                                            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    fpath = os.path.join(TRAFFIC_DIR, "kernels_%s_%s.md" % (workload, path))
    with open(fpath, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return fpath


def roofline(counts, W, ms, fp32, block_precond, ms_per_step):
    """Roofline entry of the kernel with the largest share of the iteration
    time (times measured in iteration order), by the algorithmic work of
    kernel_work; the element-block stream that the preconditioner apply
    reads is reported beside it (stream_gbps), and the whole iteration's
    algorithmic work against the measured time per iteration (iteration)."""
    names = ["volume", "face", "gather", "update"]
    work = kernel_work(counts, W, fp32)
    k = int(np.argmax(ms))
    name = names[k]
    fl, by = work[name]
    t = ms[k] * 1e-3
    roof = _roof(fl, by, t, fp32)
    roof["traffic"] = None
    roof["kernel"] = "k_update_mfma" if (name == "update" and block_precond) else "k_%s" % name
    roof["algorithmic_flops"] = fl
    roof["algorithmic_bytes"] = by
    roof["avg_ms"] = float(ms[k])
    roof["all_kernels"] = {nm: dict(avg_ms=float(ms[i]), gbps=work[nm][1] / (ms[i] * 1e-3) / 1e9,
                                    tflops=work[nm][0] / (ms[i] * 1e-3) / 1e12)
                           for i, nm in enumerate(names)}
    if block_precond:
        sb = counts["block_bytes_mixed" if fp32 else "block_bytes_fp64"]
        roof["block_stream"] = dict(bytes_per_launch=float(sb), stream_gbps=sb / (ms[3] * 1e-3) / 1e9,
                                    note="stored element-block inverses read by the preconditioner apply "
                                         "(not algorithmic work of the method)")
    ifl, iby = iteration_work(counts, W, fp32)
    it = _roof(ifl, iby, ms_per_step * 1e-3, fp32)
    it.update(algorithmic_flops=ifl, algorithmic_bytes=iby, ms=ms_per_step)
    roof["iteration"] = it
    return roof


def _oracle_iteration_seconds(disc, sample, blocks, reps, scale_elem, scale_face):
    """Seconds of the oracle's work of one PCG iteration of the whole mesh,
    from its work on the sampled elements: their volume terms and their
    element-block Cholesky solves (the preconditioner the GPU path applies),
    scaled by scale_elem, and the face terms touching them, scaled by
    scale_face."""
    import scipy.linalg as sla
    rng = np.random.default_rng(0)
    u = rng.standard_normal(disc.ndof)
    n3 = disc.n ** 3
    t_elem = t_face = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        q = disc.apply_volume(u)
        for i, e in enumerate(sample):
            o = disc.offset[e]
            sla.cho_solve(blocks[i % len(blocks)], q[o:o + n3])
        t1 = time.perf_counter()
        disc.apply_faces(u)
        t_elem += t1 - t0
        t_face += time.perf_counter() - t1
    return (t_elem * scale_elem + t_face * scale_face) / reps


def cpu_baseline(name, mesh, problem, budget_s=20.0):
    """The FP64 oracle's PCG iteration (operator apply + element-block solves)
    on the host cores, on a bounded sample of the same workload: the bench's
    own mesh and degree, restricted to a seeded sample of real elements (the
    oracle's rows of those elements are exact: an element couples only
    through its volume term and the face terms on its faces), timed with all
    BLAS threads and with one, and scaled to the whole mesh: the element work
    by E_real / k, the face work by E_real / k times the mean over the
    sampled face terms of 1 / (real elements on the term), since a term
    between two real elements is drawn by either of them.  The block
    solves use Cholesky factors of SPD matrices of the blocks' size (the
    solve's cost does not depend on the values; assembling the true blocks
    is the oracle's setup, not its iteration)."""
    import scipy.linalg as sla
    from oracle.functional import Discretization
    real = mesh.real_elements()
    rng = np.random.default_rng(1)
    k = min(len(real), 24)
    sample = sorted(int(e) for e in rng.choice(real, k, replace=False))
    t0 = time.perf_counter()
    disc = Discretization(mesh, problem, only=sample)
    n3 = disc.n ** 3
    A = rng.standard_normal((n3, n3))
    blocks = [sla.cho_factor(A @ A.T + n3 * np.eye(n3))]
    setup = time.perf_counter() - t0
    real_set = set(int(e) for e in real)
    inv_c = [1.0 / ((T.eA in real_set) + (T.eB is not None and T.eB >= 0 and T.eB in real_set))
             for T in disc.faces]
    scale_elem = len(real) / k
    scale_face = scale_elem * (float(np.mean(inv_c)) if inv_c else 1.0)
    out = {}
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        all_threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threadpool_limits, all_threads = None, os.cpu_count()
    for label, nthreads in (("all", all_threads), ("one", 1)):
        if threadpool_limits is not None:
            with threadpool_limits(limits=nthreads):
                first = _oracle_iteration_seconds(disc, sample, blocks, 1, 1.0, 1.0)
                reps = max(1, min(20, int(budget_s / 2 / max(first, 1e-6))))
                t_iter = _oracle_iteration_seconds(disc, sample, blocks, reps, scale_elem, scale_face)
        else:
            reps = 3
            t_iter = _oracle_iteration_seconds(disc, sample, blocks, reps, scale_elem, scale_face)
        out[label] = dict(threads=int(nthreads), seconds_per_iteration=t_iter, reps=reps)
    ndof = mesh.ndof()
    return dict(value=ndof / out["all"]["seconds_per_iteration"], unit="PCG iterations x DOF / s",
                cores=int(all_threads), kind="oracle",
                value_one_thread=ndof / out["one"]["seconds_per_iteration"],
                sample="the bench's mesh (%d real elements, %d DOF) restricted to %d seeded real elements: "
                       "their volume terms and %d x %d block Cholesky solves (scaled by %d / %d) and the "
                       "%d face terms touching them (scaled by %.2f), %d / %d reps (all threads / one); "
                       "%.2f s (all) and %.2f s (one thread) per iteration of the whole mesh; oracle setup %.1f s"
                       % (len(real), ndof, k, n3, n3, len(real), k, len(inv_c), scale_face,
                          out["all"]["reps"], out["one"]["reps"],
                          out["all"]["seconds_per_iteration"], out["one"]["seconds_per_iteration"], setup))


def time_iterations(ctx, b, precision, steps, warmup):
    import torch
    u = torch.zeros_like(b)
    # warmup: exactly `warmup` iterations (rtol 0 never stops early)
    ctx.pcg_solve(b, u, rtol=0.0, maxit=max(warmup, 1), raise_on_fail=False, precision=precision)
    torch.cuda.synchronize()
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.pcg_solve(b, u, rtol=0.0, maxit=steps, raise_on_fail=False, precision=precision)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info["iterations"] == steps, info
    return dt


def time_to_solution(ctx, b, uref, precision, rtol, maxit):
    """Wall time of one solve from u = 0 to the relative residual rtol, and
    the relative error of its solution against the reference solution."""
    import torch
    u = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.pcg_solve(b, u, rtol=rtol, maxit=maxit, raise_on_fail=False, precision=precision)
    torch.cuda.synchronize()
    tts = time.perf_counter() - t0
    err = float(torch.linalg.norm(u - uref) / torch.linalg.norm(uref))
    return dict(seconds=tts, iterations=info["iterations"], replacements=info["outer"],
                rel_residual=info["rel_residual"], status=info["status"], solution_rel_error=err), u


def run_batch(args):
    """Batched workload: 256 independent Poisson instances (128 on the unit cube
    with 2x2x2 elements, 128 on the Fichera mesh with N = 2 layers), degree W
    drawn from U{4..12} per instance (numpy PCG64, seed 0), 4 right-hand sides
    each (f = sum of 8 seeded Fourier modes, g = 0).  Operator data is shared
    per (mesh, W): one context each, its right-hand sides solved together, all
    contexts in one graph-captured batch.  Sequential single solves of a
    sample (the first right-hand side of every context) give the comparison."""
    import torch
    from paper_1110_2316_amd import Context, pcg_solve_batch
    from workloads import mesh as M
    from workloads.fichera import fichera_mesh
    from workloads.problems import fourier_coef
    rng = np.random.default_rng(0)
    Ws = rng.integers(4, 13, 256)
    kinds = ["cube"] * 128 + ["fichera"] * 128
    groups = {}
    for i, (k, W) in enumerate(zip(kinds, Ws)):
        groups.setdefault((k, int(W)), []).append(i)
    t0 = time.perf_counter()
    ctxs, bs, tiles = [], [], {}
    for (k, W), inst in sorted(groups.items()):
        mesh = M.box_mesh(W, (2, 2, 2), (0, 0, 0), (1, 1, 1)) if k == "cube" else fichera_mesh(N=2, W=W)
        c = Context(mesh)
        # the tile first: the block assembly then runs with the tuned kernel
        tn = c.autotune("fp64", reps=5)
        c.set_preconditioner("block")
        tiles["%s_w%d" % (k, W)] = dict(tile=tn["tile"], slab=tn["slabs"][tn["tile"]])
        rhs = []
        for i in inst:
            for j in range(4):
                c.set_source_fourier(torch.tensor(fourier_coef(1000 * i + j), dtype=torch.float64, device="cuda"))
                b = torch.zeros(c.ndof, dtype=torch.float64, device="cuda")
                c.rhs(b)
                rhs.append(b)
        ctxs.append(c)
        bs.append(torch.stack(rhs))
        print("bench: context %s W=%d: %d instances, %d DOF" % (k, W, len(inst), c.ndof), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    rtol = args.batch_rtol
    print("bench: setup %.1f s; warm-up batch (8 iterations)" % setup_s, file=sys.stderr, flush=True)
    # warm-up: buffers, graph instantiation, 8 iterations; then the timed batches
    us = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, us, rtol=rtol, maxit=8, raise_on_fail=False)
    for c in ctxs:
        c.autotune("mixed", reps=3)
    ndofs = np.concatenate([[c.ndof] * b.shape[0] for c, b in zip(ctxs, bs)])
    res = {}
    for prec in ("mixed", "fp64"):
        u_p = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf = pcg_solve_batch(ctxs, bs, u_p, rtol=rtol, maxit=args.maxit, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its_p = np.array([i["iterations"] for i in inf])
        res[prec] = dict(seconds=dt, infos=inf, its=its_p, u=u_p, work=float((its_p * ndofs).sum()))
        print("bench: %s batch solved in %.2f s" % (prec, dt), file=sys.stderr, flush=True)
    err = max(float(torch.linalg.norm(a[k] - b[k]) / torch.linalg.norm(b[k]))
              for a, b in zip(res["mixed"]["u"], res["fp64"]["u"]) for k in range(b.shape[0]))
    # errors against reference solutions (FP64 batch to the relative residual 1e-13, untimed)
    uref = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, uref, rtol=1e-13, maxit=args.maxit, raise_on_fail=False)
    errs = {p: max(float(torch.linalg.norm(a[k] - r[k]) / torch.linalg.norm(r[k]))
                   for a, r in zip(res[p]["u"], uref) for k in range(r.shape[0])) for p in ("mixed", "fp64")}
    print("bench: max relative error against the 1e-13 reference: %s" % errs, file=sys.stderr, flush=True)
    us = res["fp64"]["u"]
    infos = res["fp64"]["infos"]
    t_batch = res["fp64"]["seconds"]
    its = res["fp64"]["its"]
    work = res["fp64"]["work"]
    t_mixed = res["mixed"]["seconds"]
    # sequential single solves, first right-hand side of every context
    t_seq, t_seq_sample = 0.0, 0
    for c, b in zip(ctxs, bs):
        u1 = torch.zeros_like(b[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.pcg_solve(b[0].contiguous(), u1, rtol=rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_seq += dt * b.shape[0]
        t_seq_sample += 1
        assert torch.equal(u1, us[ctxs.index(c)][0])
    nrhs = int(sum(b.shape[0] for b in bs))
    out = dict(metric="PCG iterations x DOF / s and time to solution (batched, relative residual %g), mixed vs FP64" % rtol,
               value=res["mixed"]["work"] / t_mixed,
               unit="iterations*DOF/s", n_gpus=1, steps=int(res["mixed"]["its"].max()), warmup=1,
               ms_per_step=1e3 * t_mixed / max(1, int(res["mixed"]["its"].max())), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32+f64", data="synthetic",
               config=dict(workload="batched_poisson_256", instances=256, rhs=nrhs, contexts=len(ctxs),
                           degrees="U{4..12}", preconditioner="block", rtol=rtol),
               setup_s=setup_s, mixed_batch_seconds=t_mixed, fp64_batch_seconds=t_batch,
               mixed_vs_fp64_speedup=t_batch / t_mixed, mixed_max_rel_diff_to_fp64=err,
               mixed_max_rel_error=errs["mixed"], fp64_max_rel_error=errs["fp64"],
               error_reference="FP64 batch solved to relative residual 1e-13",
               mixed_outer_steps=int(res["mixed"]["infos"][0]["outer"]),
               mixed_all_converged=all(i["status"] == 0 for i in res["mixed"]["infos"]),
               rhs_per_second=nrhs / t_mixed, fp64_value=work / t_batch,
               iterations_min=int(its.min()), iterations_max=int(its.max()), all_converged=all(i["status"] == 0 for i in infos),
               sequential_seconds_estimate=t_seq,
               sequential_sample="one single solve per context (%d solves), scaled by its right-hand side count" % t_seq_sample,
               batch_speedup=t_seq / t_batch, tiles=tiles)
    print(json.dumps(out), flush=True)


def _roctx():
    """roctx's profiler pause / resume (rocprofv3 --selected-regions), or None."""
    import ctypes
    for name in ("librocprofiler-sdk-roctx.so", "/opt/rocm/lib/librocprofiler-sdk-roctx.so"):
        try:
            L = ctypes.CDLL(name)
        except OSError:
            continue
        for fn in (L.roctxProfilerResume, L.roctxProfilerPause):
            fn.argtypes = [ctypes.c_uint64]
            fn.restype = ctypes.c_int
        return L
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=os.environ.get("SEM_BENCH_WORKLOAD", "fichera_n10"))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="path whose throughput is `value` (default: fp64 for N<10, mixed for N>=10)")
    ap.add_argument("--tts-rtol", type=float, default=1e-10,
                    help="relative residual of the timed solves (their error against the reference is reported)")
    ap.add_argument("--maxit", type=int, default=200000)
    ap.add_argument("--batch-rtol", type=float, default=1e-10,
                    help="relative residual of the batched workload's solves (the largest error against the "
                         "1e-13 reference is reported: 1.8e-8 measured at 1e-10; at 1e-11 the mixed batch "
                         "meets the attainable-accuracy floor of some contexts and stops with SEM_ENOCONV)")
    ap.add_argument("--precond", default="block", choices=["block", "separable"],
                    help="block-diagonal preconditioner: exact element blocks of X, or the thesis's separable forms")
    ap.add_argument("--compare-separable", type=int, default=None,
                    help="also time the FP64 solve with the separable preconditioner (default: for N < 10)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--profile-kernels", default=None, choices=["fp64", "mixed"],
                    help="after setup only time the kernels of that path (for rocprofv3 counter passes) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --profile-kernels: also copy a 1 GiB device buffer 5 times with an "
                         "elementwise kernel (counter scale)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write profiles/traffic_<workload>_n<N>.json from two rocprofv3 --pmc output "
                         "directories of --profile-kernels runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--summarize-sq", nargs="+", metavar="DIR", default=None,
                    help="write profiles/counters_<workload>_n<N>_<path>.json from rocprofv3 --pmc "
                         "output directories of --profile-kernels runs (SQ counters) and exit")
    ap.add_argument("--graded", default=None, metavar="MU1[,MU2]",
                    help="layer-graded degrees (W_l = [mu1 i], V_q = [mu2 k]) on the workload's mesh; "
                         "the throughput then counts the graded space's unknowns")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "LOG", "COMMAND"), default=None,
                    help="write profiles/kernels_<workload>_n<N>_<path>.md from a rocprofv3 --kernel-trace "
                         "--stats csv run of --profile-kernels (its stdout in LOG, the command as run) and exit")
    ap.add_argument("--tile", type=int, default=None,
                    help="element-kernel tile for both paths instead of autotuning (counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (elements would be "
              "sharded by a space-filling curve, with face traces exchanged between neighbours)",
              file=sys.stderr)
        sys.exit(2)

    if args.summarize_trace:
        _, _, cfg = make_workload(args.workload)
        print(summarize_trace(args.summarize_trace[0], "%s_n%d" % (cfg["workload"], cfg.get("N", 0)),
                              args.profile_kernels or "mixed", args.summarize_trace[1], args.summarize_trace[2]))
        return
    if args.summarize_sq:
        _, _, cfg = make_workload(args.workload)
        print(summarize_sq(args.summarize_sq, "%s_n%d" % (cfg["workload"], cfg.get("N", 0)),
                           args.profile_kernels or "mixed"))
        return
    if args.summarize_counters:
        _, _, cfg = make_workload(args.workload)
        path = args.profile_kernels or "mixed"
        print(summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                                 "%s_n%d" % (cfg["workload"], cfg.get("N", 0)), path))
        return

    import torch
    from paper_1110_2316_amd import setup_problem

    torch.cuda.set_device(0)
    if args.workload == "batch256":
        return run_batch(args)
    mesh, problem, cfg = make_workload(args.workload)
    prec = args.precision or ("mixed" if cfg.get("N", 0) >= 10 else "fp64")
    print("bench: workload %s, %d elements, value from the %s path" % (cfg["workload"], mesh.E, prec),
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = setup_problem(mesh, problem)
    setup_s = time.perf_counter() - t0
    ndof = ctx.ndof
    # unknowns the throughput counts: those of the graded space when degrees are graded
    dof_count = ndof
    if args.graded:
        from workloads.grading import layer_degrees
        mu = [float(v) for v in args.graded.split(",")]
        ctx.set_degrees(layer_degrees(mesh, mu[0], mu[-1]))
        dof_count = ctx.graded_ndof
        cfg = dict(cfg, workload=cfg["workload"] + "_graded", mu1=mu[0], mu2=mu[-1], graded_dof=dof_count)
        print("bench: graded degrees mu1 = %g, mu2 = %g: %d of %d unknowns" % (mu[0], mu[-1], dof_count, ndof),
              file=sys.stderr, flush=True)
    # the tile first: the element-block assembly then runs with the tuned kernel
    if args.tile is None:
        tune = {p: ctx.autotune(p, reps=5) for p in ("fp64", "mixed")}
    else:
        for p in ("fp64", "mixed"):
            ctx.set_tile(args.tile, p)
        tune = {p: dict(tile=args.tile, fixed=True) for p in ("fp64", "mixed")}
    print("bench: element-kernel tiles %s" % tune, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx.set_preconditioner(args.precond)
    torch.cuda.synchronize()
    precond_setup_s = time.perf_counter() - t0
    b = torch.zeros(ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    torch.cuda.synchronize()
    print("bench: setup %.1f s + preconditioner %.1f s, %d DOF" % (setup_s, precond_setup_s, ndof),
          file=sys.stderr, flush=True)
    if args.profile_kernels:
        # counters are collected only inside this region (rocprofv3
        # --selected-regions): the timed kernels and the calibration copy
        uk = torch.randn(ndof, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
        if args.copy_calibration:
            n = (1 << 30) // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
        torch.cuda.synchronize()
        rx = _roctx()
        if rx is not None:
            rx.roctxProfilerResume(0)
        ms = ctx.kernel_times(uk, reps=20, precision=args.profile_kernels)
        if args.copy_calibration:
            # an elementwise kernel that reads 1 GiB and writes 1 GiB
            for _ in range(5):
                torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        if rx is not None:
            rx.roctxProfilerPause(0)
        print(json.dumps(dict(profile_kernels=args.profile_kernels, kernel_ms=[float(v) for v in ms],
                              copy_calibration_bytes=(1 << 30) if args.copy_calibration else 0,
                              copies=5 if args.copy_calibration else 0)), flush=True)
        return

    paths = {}
    for p in ("fp64", "mixed"):
        dt = time_iterations(ctx, b, p, args.steps, args.warmup)
        paths[p] = dict(ms_per_step=1e3 * dt / args.steps, value=args.steps * dof_count / dt)
        print("bench: %s %d iterations in %.4f s" % (p, args.steps, dt), file=sys.stderr, flush=True)

    out_extra = {}
    if not args.no_tts:
        # reference solution: FP64 PCG to 1e-13
        uref = torch.zeros_like(b)
        iref = ctx.pcg_solve(b, uref, rtol=1e-13, maxit=args.maxit, raise_on_fail=False)
        print("bench: reference solve %d iterations" % iref["iterations"], file=sys.stderr, flush=True)
        for p in ("fp64", "mixed"):
            res, _ = time_to_solution(ctx, b, uref, p, args.tts_rtol, args.maxit)
            paths[p]["time_to_solution"] = res
            print("bench: %s solve %s" % (p, res), file=sys.stderr, flush=True)
        xe = ctx.error_points()
        out_extra["h1_rel_error"] = ctx.error(uref, problem.u(xe), problem.grad_u(xe))
        out_extra["reference_iterations"] = iref["iterations"]
        t64 = paths["fp64"]["time_to_solution"]["seconds"]
        tmx = paths["mixed"]["time_to_solution"]["seconds"]
        out_extra["tts_speedup_mixed_vs_fp64"] = t64 / tmx if tmx > 0 else None
        out_extra["tts_rtol"] = args.tts_rtol
        cmp_sep = args.compare_separable if args.compare_separable is not None else int(cfg.get("N", 0) < 10)
        if cmp_sep and args.precond != "separable":
            ctx.set_preconditioner("separable")
            res, _ = time_to_solution(ctx, b, uref, "fp64", args.tts_rtol, args.maxit)
            out_extra["fp64_separable_preconditioner_time_to_solution"] = res
            print("bench: fp64 separable-preconditioner solve %s" % res, file=sys.stderr, flush=True)
            ctx.set_preconditioner(args.precond)

    # roofline of the dominant kernel of the reported path: HIP events on the launch stream
    counts = ctx.work_counts()
    uk = torch.randn(ndof, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    for p in ("fp64", "mixed"):
        ms = ctx.kernel_times(uk, reps=50, precision=p)
        paths[p]["kernel_ms"] = dict(zip(["volume", "face", "gather", "update"], [float(v) for v in ms]))
        paths[p]["roofline"] = roofline(counts, mesh.W, ms, p == "mixed", args.precond == "block",
                                        paths[p]["ms_per_step"])
        paths[p]["roofline"]["traffic"] = measured_traffic(
            "%s_n%d" % (cfg["workload"], cfg.get("N", 0)), p, paths[p]["roofline"]["kernel"])

    main_path = paths[prec]
    out = dict(metric="PCG iterations x DOF / s and time to 1e-8 relative error, mixed vs FP64",
               value=main_path["value"], unit="iterations*DOF/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=main_path["ms_per_step"],
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if prec == "fp64" else "f32+f64", data="synthetic",
               config=dict(cfg, path=prec, preconditioner=args.precond, elements=int(counts["elements"]),
                           real_elements=int(counts["real_elements"]), dof=int(ndof)),
               setup_s=setup_s, preconditioner_setup_s=precond_setup_s, element_kernel_tiles=tune, paths=paths, roofline=main_path["roofline"], **out_extra)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, mesh, problem, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
