"""Benchmark: time to relative KKT residual <= 1e-6 of Nys-IP-PMM on one
MI355X, mixed precision (FP32-defined A with FP64-accumulated products, BF16
matrix-core sketch) against the FP64 GPU form, plus the normal-equation
matvec bandwidth against the HBM roofline.

Workload (default): lowrank_20000x100000 -- m = 20000, n = 100000,
A = U diag(i^-1.5) V^T (rank 400) + 1e-3 N(0,1) stored FP32 (8 GB) and BF16
(4 GB), Q = diag(U[0,1]) with 30% exact zeros, planted optimum, sketch 200,
instance seed 0, generated on the GPU.

One JSON line on stdout.  `value` = seconds per mixed-precision solve (one
step = one full solve from the initial point to KKT <= 1e-6), inputs resident
in HBM.  The roofline object is for the dominant kernel (the pass of the
normal-equation operator with the larger total time), timed with HIP events
on the library's stream during the timed steps.  Beside it: the FP64 GPU form
of the same solve (median of three runs), the 50000 x 200000 workload's
forward solve and its adjoint for c and b, and the FP64 oracle on the host's
cores (cpu_baseline).  The oracle runs in a child process on cores of its own
while the GPU works: full solves of the 200 x 500, 2000 x 8000 and
5000 x 20000 configurations, then the initial point and one full iteration on
the bench instance, extrapolated to the GPU run's iteration count.  Optional
legs are dropped, and say so, when the --budget-s budget runs short.

Modes:
  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-fp64] [--no-cpu-baseline]
  python bench.py --compare [--workload NAME]   # Nys-IP-PMM against the paper's
                                    # comparators (Chol-IP-PMM, CG-IP-PMM) on one
                                    # workload: one JSON line per solver
  python bench.py --adaptive [--workload NAME]  # sketch size from the d_eff
                                    # estimate and preconditioner reuse against
                                    # the fixed size: one JSON line per variant
  python bench.py --operator MxN [--ell L] [--nystrom K]
                                    # the normal-equation operator and the BF16
                                    # sketch product alone on an m x n FP32
                                    # matrix (e.g. one column shard of a larger
                                    # A): one JSON line of per-pass rates; with
                                    # K, also K whole Nystrom constructions
  python bench.py --kernel-loop R   # only R normal-equation applies (pass 1 on a
                                    # transposed copy, as in the solver), a plain
                                    # copy and read-stream kernels of known size
                                    # (for counter runs)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOL = 1e-6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# kernel-name prefixes of the two passes (pass 1 over A^T rows, or over
# column stripes of A when there is no transposed copy)
PASS1_TAGS = ("k_gemv_tt<", "k_gemv_t<")
PASS2_TAGS = ("k_gemv_n<",)
PASS_TAGS = PASS1_TAGS + PASS2_TAGS


def gemv_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gemv.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2404_14524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch of the two GEMV passes from the committed counter
    summary, valid only if the kernel source is unchanged since."""
    path = os.path.join(ROOT, "profiles", f"gemv_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("gemv_source_hash") != gemv_source_hash():
        return None
    return rec


def _db(path):
    import glob
    import sqlite3
    dbs = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True)) if os.path.isdir(path) else [path]
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return sqlite3.connect(dbs[0])


def summarize_trace(db_path: str, out_md: str, command: str, workload: str, m: int, n: int, b_A: int):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` database."""
    con = _db(db_path)
    rows = con.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                       "from kernels group by name order by sum(duration) desc limit 20").fetchall()
    bytes_pass = m * n * b_A
    lines = [f"# Kernel trace: {workload}", "", f"Command: `{command}`", "",
             "Launches of the two passes that return at once (a finished PCG solve skips them) are "
             "counted in `calls`; the last two columns cover only the launches that read A "
             "(duration above 10 µs).", "",
             "| kernel | calls | avg µs | min µs | max µs | total ms | reads of A | avg µs (reads of A) "
             "| GB/s (A once) |",
             "|---|---|---|---|---|---|---|---|---|"]
    for name, cnt, avg, mn, mx, tot in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")[:80]
        reads, ravg, gbs = "", "", ""
        if any(t in name for t in PASS_TAGS):
            nr, ra = con.execute("select count(*), avg(duration) from kernels where name = ? and duration > 10000",
                                 (name,)).fetchone()
            reads, ravg = str(nr), f"{ra / 1e3:.1f}"
            gbs = f"{bytes_pass / (ra * 1e-9) / 1e9:.0f}"
        lines.append(f"| `{short}` | {cnt} | {avg / 1e3:.1f} | {mn / 1e3:.1f} | {mx / 1e3:.1f} | "
                     f"{tot / 1e6:.2f} | {reads} | {ravg} | {gbs} |")
    os.makedirs(os.path.dirname(out_md), exist_ok=True)
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_pmc(fetch_db: str, write_db: str, workload: str, m: int, n: int, b_A: int, command: str,
                  out: str = ""):
    """HBM bytes per launch of the two GEMV passes from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for a reference kernel of known size in the same run: FETCH_SIZE by the
    read-stream kernel over A (the same 16-byte non-temporal loads, m*n*b_A
    bytes), WRITE_SIZE by the plain 2 GiB copy."""
    copy_bytes = float(1 << 31)
    read_bytes = float((m * n * b_A) // 16 * 16)
    rec = {"workload": workload, "gemv_source_hash": gemv_source_hash(), "command": command,
           "algorithmic_bytes_per_launch": m * n * b_A, "hbm_bytes_per_launch": {}, "raw_kib": {}}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        con = _db(path)
        rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                           (counter,)).fetchall()
        if counter == "FETCH_SIZE":
            refs = [v for k, v in rows if "k_stream_read" in k]
            known = read_bytes
        else:
            refs = [v for k, v in rows if "copy" in k.lower()]
            known = copy_bytes
        ref = (sum(refs) / len(refs) if counter == "FETCH_SIZE" else max(refs)) if refs else None
        factor = known / (ref * 1024.0) if ref else None
        rec[f"{counter}_reference_kib"] = ref
        rec[f"{counter}_reference_bytes"] = known
        rec[f"{counter}_scale"] = factor
        for key, tags in (("normal_pass1", PASS1_TAGS), ("normal_pass2", PASS2_TAGS)):
            vals = [v for k, v in rows if any(t in k for t in tags)]
            if vals and factor:
                kib = sum(vals) / len(vals)
                rec["raw_kib"][f"{key}_{counter}"] = kib
                per.setdefault(key, 0.0)
                per[key] += kib * 1024.0 * factor
    rec["hbm_bytes_per_launch"] = {k: round(v) for k, v in per.items()}
    out = out or os.path.join(ROOT, "profiles", f"gemv_traffic_{workload}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


# ------------------------------------------------------------------ the oracle on the host cores

# configurations the oracle solves in full beside the GPU work
ORACLE_FULL = ("gauss_200x500", "gauss_2000x8000", "lowrank_5000x20000")


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: the model name string of the
    first processor, with its family, model and stepping numbers (a
    virtualised host may give only a generic model name) and the count of
    logical processors listed."""
    fields, nproc = {}, 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "processor":
                    nproc += 1
                if nproc == 1 and key in ("model name", "cpu family", "model", "stepping", "cpu MHz", "cache size"):
                    fields[key] = val.strip()
    except OSError:
        return "unknown"
    if not fields:
        return "unknown"
    extra = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping", "cpu MHz", "cache size")
                      if k in fields)
    return f"{fields.get('model name', 'unknown')} ({extra}; {nproc} logical processors listed)"


def split_cores(cores):
    """(cores of the oracle child, cores of this process): with four or more,
    the thread that drives the GPU keeps two cores to itself."""
    cores = sorted(cores)
    if len(cores) >= 4:
        return cores[2:], cores[:2]
    return cores, cores


def _write_json(path, rec):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f)
    os.replace(tmp, path)


def oracle_child(workdir: str, seed: int, names=ORACLE_FULL, wait_s: float = 900.0):
    """Child process: the FP64 oracle on this process's cores (BLAS threads =
    the cores of its affinity mask).  First full solves of the small
    configurations (instances drawn on the CPU, same recipes and seed), to
    the GPU's tolerance; then, on the bench instance the parent hands over
    (FP32 A promoted to FP64, b, c, q), the initial point and one full
    IP-PMM iteration (the dense normal matrix of all n columns, its Cholesky
    factor, predictor and corrector).  Results go to workdir/result.json
    after every piece."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from instances import make_instance
    from oracle import ippmm

    cores = len(os.sched_getaffinity(0))
    out = os.path.join(workdir, "result.json")
    res = {"cores": cores, "cpu_model": cpu_model(), "full_solves": {}, "bench_instance": None}
    _write_json(out, res)
    with threadpool_limits(limits=cores):
        for name in names:
            inst = make_instance(name, seed=seed)
            A = inst.A.double().numpy()
            b, c, q = inst.b.numpy(), inst.c.numpy(), inst.q.numpy()
            t0 = time.perf_counter()
            r = ippmm.solve(A, b, c, q, tol=TOL)
            t = time.perf_counter() - t0
            xs = inst.x_star.numpy()
            res["full_solves"][name] = {
                "m": inst.m, "n": inst.n, "seconds": round(t, 3), "ipm_iters": r["iters"], "status": r["status"],
                "kkt_rel": r["kkt"],
                "x_rel_err_vs_planted": float(np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs))}
            _write_json(out, res)
        ready = os.path.join(workdir, "ready")
        t_wait = time.perf_counter()
        while not os.path.exists(ready):
            if time.perf_counter() - t_wait > wait_s:
                return
            time.sleep(0.5)
        A = np.load(os.path.join(workdir, "A.npy"), mmap_mode="r").astype(np.float64)
        b, c, q = (np.load(os.path.join(workdir, f"{v}.npy")) for v in ("b", "c", "q"))
        ts = []
        t0 = time.perf_counter()
        r = ippmm.solve(A, b, c, q, tol=TOL, max_iter=1, timings=ts)
        res["bench_instance"] = {"m": A.shape[0], "n": A.shape[1],
                                 "initial_point_s": ts[0] - t0,
                                 "one_iteration_s": ts[1] - ts[0],
                                 "kkt_rel_after_one_iteration": r["kkt"]}
        _write_json(out, res)


class OracleChild:
    """The oracle leg of the bench, in a child process on host cores of its
    own, started before this process touches the GPU."""

    def __init__(self, seed: int):
        import subprocess
        import tempfile
        base = "/dev/shm" if os.path.isdir("/dev/shm") and os.access("/dev/shm", os.W_OK) else None
        self.dir = tempfile.mkdtemp(prefix="nys_oracle_", dir=base)
        child, own = split_cores(os.sched_getaffinity(0))
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = str(len(child))
        self.log = open(os.path.join(self.dir, "child.log"), "w")
        self.proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-child", self.dir,
                                      "--seed", str(seed)], env=env, stdout=self.log, stderr=subprocess.STDOUT,
                                     preexec_fn=lambda: os.sched_setaffinity(0, child))
        os.sched_setaffinity(0, own)

    def provide(self, inst):
        """Hand the bench instance to the child (FP32 A as stored, b, c, q)."""
        import numpy as np
        np.save(os.path.join(self.dir, "A.npy"), inst.A.cpu().numpy())
        for v in ("b", "c", "q"):
            np.save(os.path.join(self.dir, f"{v}.npy"), getattr(inst, v).cpu().numpy())
        with open(os.path.join(self.dir, "ready"), "w") as f:
            f.write("1")

    def collect(self, gpu_iters: int, wait_s: float):
        """The child's results, waiting at most wait_s for it; the child is
        ended (its own process only) if it is still running then."""
        deadline = time.perf_counter() + max(wait_s, 0.0)
        while True:
            left = deadline - time.perf_counter()
            try:
                self.proc.wait(timeout=max(0.0, min(60.0, left)))
                break
            except subprocess.TimeoutExpired:
                if time.perf_counter() >= deadline:
                    self.proc.kill()
                    self.proc.wait()
                    break
                log("waiting for the oracle child")
        self.log.close()
        path = os.path.join(self.dir, "result.json")
        res = json.load(open(path)) if os.path.exists(path) else {}
        import shutil
        shutil.rmtree(self.dir, ignore_errors=True)
        return oracle_baseline_record(res, gpu_iters)


def oracle_baseline_record(res: dict, gpu_iters: int):
    """cpu_baseline of the JSON line from the child's results: the initial
    point plus gpu_iters times one full iteration of the oracle on the bench
    instance (each measured in full), extrapolated to the GPU run's
    iteration count; the full solves of the small configurations beside it."""
    bi = res.get("bench_instance")
    rec = {"value": None, "unit": "s", "cores": res.get("cores"), "kind": "oracle",
           "cpu_model": res.get("cpu_model"), "full_solves": res.get("full_solves", {})}
    if bi:
        rec["value"] = round(bi["initial_point_s"] + gpu_iters * bi["one_iteration_s"], 1)
        rec["sample"] = (f"the oracle on this instance ({bi['m']} x {bi['n']}, FP64): initial point "
                         f"{bi['initial_point_s']:.1f} s and one full IP-PMM iteration {bi['one_iteration_s']:.1f} s "
                         f"(dense A D A^T + delta I of all n columns, Cholesky, predictor and corrector), both "
                         f"measured; x {gpu_iters} iterations (the GPU run's count): extrapolated")
        rec["bench_instance"] = bi
    else:
        rec["sample"] = "the oracle leg did not finish within the bench's time budget"
    return rec


# SVM-form workloads at the shapes of the paper's dense SVM datasets (Table 3),
# with synthetic features (the datasets are not available): d, n, ell.
SVM_SHAPES = {"svm_sensit": (100, 98528, 50), "svm_cifar10": (3072, 60000, 200),
              "svm_rnaseq": (20531, 801, 200)}


# The portfolio workload (section 5.1): n assets, d correlation constraints,
# s factors, sketch size, tolerance.
PORTFOLIO_SHAPES = {"portfolio_80000x50000": (80000, 50000, 100, 20, 1e-8),
                    "portfolio_20000x12500": (20000, 12500, 50, 20, 1e-8)}


def compare_svm(nys, args):
    """The paper's SVM comparison (section 5.2) on the dual linear SVM in form
    (P~) with synthetic dense features: Nys-IP-PMM, CG-IP-PMM, Chol-IP-PMM."""
    import torch
    from instances import svm_instance
    d, n, ell = SVM_SHAPES[args.workload]
    S = svm_instance(d, n, seed=args.seed, device="cuda", dtype=torch.float32,
                     unit_columns=not args.dense_identity)
    compare_box(nys, args, S, ell, TOL, {"d": d, "n": n})


def compare_portfolio(nys, args):
    """The paper's portfolio comparison (section 5.1): the factor-model
    problem in form (P~) (y = F^T x free, slacks for M x <= u), tolerance
    1e-8, Nys-IP-PMM with ell = 20 against CG-IP-PMM and Chol-IP-PMM."""
    import torch
    from instances import portfolio_instance
    n, d, s_f, ell, tol = PORTFOLIO_SHAPES[args.workload]
    t0 = time.perf_counter()
    S = portfolio_instance(n, d, s_f, seed=args.seed, device="cuda", dtype=torch.float32,
                           unit_columns=not args.dense_identity)
    torch.cuda.synchronize()
    log(f"{args.workload}: A {tuple(S['A'].shape)} FP32 generated in {time.perf_counter() - t0:.1f}s")
    compare_box(nys, args, S, ell, tol, {"n": n, "d": d, "s": s_f})


def compare_box(nys, args, S, ell, tol, shape):
    """Nys-IP-PMM, Chol-IP-PMM and CG-IP-PMM on one (P~) instance (FP32 A,
    BF16 sketch; identity and slack blocks as unit columns unless
    --dense-identity): one warm-up solve (skipped with --no-warmup-solve),
    then one JSON line per solver with its convergence history (seconds,
    rp_rel, rd_rel, mu per IP-PMM iteration).  An iteration limit
    (--max-iter) ends a solve early; its line then carries the KKT reached."""
    import numpy as np
    import torch
    A = S["A"]
    units = S.get("units")
    A_lo = A.to(torch.bfloat16)
    A_t = nys.nys_transpose(A)
    box = (S["vtype"], S["u"])
    extra = dict(verbose=args.verbose, max_iter=args.max_iter, A_t=A_t, units=units)
    if not args.no_warmup_solve:
        try:
            nys.ipm_solve_box(A, S["b"], S["c"], S["q"], *box, ell=ell, tol=tol, seed=args.seed,
                              sketch_dtype="bf16", A_lo=A_lo, **extra)
        except nys.NysError:
            pass
        torch.cuda.synchronize()
    for name, pre in (("Nys-IP-PMM", "nystrom"), ("Chol-IP-PMM", "pchol"), ("CG-IP-PMM", "none")):
        if pre not in args.solvers.split(","):
            continue
        log(f"{args.workload}: {name}")
        tr = np.full((args.max_iter + 1, len(nys.TRACE_FIELDS)), np.nan)
        t0 = time.perf_counter()
        err = None
        try:
            x, y, z, w, s, info = nys.ipm_solve_box(A, S["b"], S["c"], S["q"], *box, ell=ell, tol=tol,
                                                    seed=args.seed, sketch_dtype="bf16", trace=tr,
                                                    A_lo=A_lo if pre == "nystrom" else None, precond=pre, **extra)
        except nys.NysError as e:          # the iteration limit and the like: report what was reached
            err = str(e)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        K = int(np.sum(~np.isnan(tr[:, 0])))
        f = {k: i for i, k in enumerate(nys.TRACE_FIELDS)}
        rec = {"solver": name, "workload": args.workload, **shape, "m": A.shape[0],
               "n_vars": A.shape[1] + (0 if units is None else units[0].numel()),
               "unit_columns": 0 if units is None else units[0].numel(), "ell": ell, "tol": tol,
               "seconds": round(t, 3)}
        if err is None:
            rec.update({"status": info.status, "ipm_iters": info.iters, "pcg_iters": info.pcg_iters_total,
                        "kkt_rel": info.kkt_rel,
                        "time_split_ms": {"precond": round(info.t_sketch_ms, 1), "pcg": round(info.t_pcg_ms, 1),
                                          "other": round(info.t_other_ms, 1)}})
        else:
            rec["error"] = err
        rec["history"] = [[round(tr[k, f["time_ms"]] / 1e3, 2), float(f"{tr[k, f['rp_rel']]:.2e}"),
                           float(f"{tr[k, f['rd_rel']]:.2e}"), float(f"{tr[k, f['mu']]:.2e}"), int(tr[k, f["pcg"]])]
                          for k in range(K)]
        print(json.dumps(rec), flush=True)


def compare(nys, inst, args):
    """The paper's comparison (Nys-IP-PMM against Chol-IP-PMM and CG-IP-PMM,
    section 5): same instance, same tolerance, same sketch/pivot count ell;
    wall time of each solve (one warm-up solve of the method first)."""
    import torch
    A = inst.A
    A_lo = A.to(torch.bfloat16) if A.dtype == torch.float32 else None
    sk = "bf16" if A_lo is not None else "f64"
    nys.ipm_solve(A, inst.b, inst.c, inst.q, ell=inst.ell, tol=TOL, seed=args.seed, sketch_dtype=sk, A_lo=A_lo)
    torch.cuda.synchronize()
    for name, pre in (("Nys-IP-PMM", "nystrom"), ("Chol-IP-PMM", "pchol"), ("CG-IP-PMM", "none")):
        t0 = time.perf_counter()
        x, y, z, info = nys.ipm_solve(A, inst.b, inst.c, inst.q, ell=inst.ell, tol=TOL, seed=args.seed,
                                      sketch_dtype=sk, A_lo=A_lo if pre == "nystrom" else None, precond=pre)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        xs = inst.x_star
        rec = {"solver": name, "workload": args.workload, "seconds": round(t, 3), "status": info.status,
               "ipm_iters": info.iters, "pcg_iters": info.pcg_iters_total, "kkt_rel": info.kkt_rel,
               "x_rel_err_vs_planted": float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)),
               "time_split_ms": {"precond": round(info.t_sketch_ms, 1), "pcg": round(info.t_pcg_ms, 1),
                                 "other": round(info.t_other_ms, 1)}}
        print(json.dumps(rec), flush=True)


def operator_shape(nys, shape: str, ell: int, reps: int, seed: int, nystrom: int = 0):
    """The normal-equation operator (pass 1 on a transposed copy) and the BF16
    matrix-core sketch product (on sketch tiles), as in the solver, alone on a seeded Gaussian
    FP32 m x n matrix: launches and rates per kernel class from the library's
    HIP events, against the read-stream reference over the same matrix.  With
    nystrom > 0, also that many whole Nystrom constructions (Algorithm 1 with
    the BF16 sketch on the same tiles, a fresh Omega each), timed end to end."""
    import torch
    m, n = (int(t) for t in shape.lower().split("x"))
    dev = "cuda"
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A = torch.randn(m, n, dtype=torch.float32, device=dev, generator=g)
    A_t = nys.nys_transpose(A)
    A_lo = A.to(torch.bfloat16)
    # the solver gives the BF16 sketch its operands as sketch tiles of A and of A^T
    tiles = (nys.nys_sketch_tiles(A), nys.nys_sketch_tiles(A, transposed=True))
    d = torch.rand(n, dtype=torch.float64, device=dev, generator=g)
    v = torch.randn(m, dtype=torch.float64, device=dev, generator=g)
    om = torch.randn(m, ell, dtype=torch.float64, device=dev, generator=g)
    out = torch.empty_like(v)
    Y = torch.empty(m, ell, dtype=torch.float64, device=dev)
    for _ in range(3):
        nys.nys_normal_apply(A, d, 1e-3, v, out, A_t=A_t)
    nys.nys_sketch_product(A_lo, d, om, "bf16", out=Y, tiles=tiles)
    torch.cuda.synchronize()
    log(f"operator {m}x{n}: warm")
    nys.nys_profile_enable(True)
    for _ in range(reps):
        nys.nys_normal_apply(A, d, 1e-3, v, out, A_t=A_t)
    sk_reps = max(1, reps // 20)
    for _ in range(sk_reps):
        nys.nys_sketch_product(A_lo, d, om, "bf16", out=Y, tiles=tiles)
    torch.cuda.synchronize()
    prof = nys.nys_profile_read()
    nys.nys_profile_enable(False)
    rs_ms = min(nys.nys_stream_read(A) for _ in range(5))
    bytes_pass = m * n * 4
    rec = {"mode": "operator", "m": m, "n": n, "A_storage": "float32", "applies": reps,
           "read_stream_GBps": round(bytes_pass / (rs_ms * 1e-3) / 1e9, 1)}
    for k in ("normal_pass1", "normal_pass2"):
        nl, ms = prof[k]
        rec[k] = {"launches": nl, "avg_ms": round(ms / nl, 4), "GBps": round(bytes_pass / (ms / nl * 1e-3) / 1e9, 1)}
    rec["normal_apply_ms"] = round(rec["normal_pass1"]["avg_ms"] + rec["normal_pass2"]["avg_ms"], 4)
    flops = 2.0 * m * n * ell
    for k in ("sketch_w", "sketch_y"):
        nl, ms = prof[k]
        rec[k] = {"ell": ell, "launches": nl, "avg_ms": round(ms / nl, 3),
                  "TFLOPs": round(flops / (ms / nl * 1e-3) / 1e12, 1)}
    if nystrom > 0:
        times = []
        for r in range(nystrom + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = nys.nys_sketch(A_lo, d, ell, seed=seed + r, sketch_dtype="bf16", tiles=tiles)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            del P
            log(f"nystrom construction {r}: {t * 1e3:.1f} ms" + (" (warm-up)" if r == 0 else ""))
            if r > 0:
                times.append(t)
        rec["nystrom_construction"] = {"ell": ell, "sketch": "bf16", "runs": nystrom,
                                       "avg_ms": round(1e3 * sum(times) / len(times), 1),
                                       "min_ms": round(1e3 * min(times), 1)}
    print(json.dumps(rec), flush=True)


ADAPTIVE_VARIANTS = (
    ("fixed", dict()),
    ("deff", dict(ell_rule="deff")),
    ("theorem", dict(ell_rule="theorem")),
    ("reuse3", dict(reuse_max_age=3)),
    ("deff+reuse3", dict(ell_rule="deff", reuse_max_age=3)),
)


def adaptive_compare(nys, inst, args):
    """Sketch size from the d_eff estimate and preconditioner reuse against
    the fixed sketch size, on one workload: same instance, tolerance and
    initial size ell (the rules clamp to [min(8, ell), min(m, 4 ell)]); one
    JSON line per variant with the per-iteration sizes and d_hat."""
    import numpy as np
    import torch
    A = inst.A
    A_lo = A.to(torch.bfloat16) if A.dtype == torch.float32 else None
    sk = "bf16" if A_lo is not None else "f64"
    A_t = nys.nys_transpose(A)
    base = dict(ell=inst.ell, tol=TOL, seed=args.seed, sketch_dtype=sk, A_lo=A_lo, A_t=A_t,
                max_iter=args.max_iter, verbose=args.verbose)
    nys.ipm_solve(A, inst.b, inst.c, inst.q, **base)           # warm-up
    torch.cuda.synchronize()
    for name, kw in ADAPTIVE_VARIANTS:
        tr = np.full((args.max_iter + 1, len(nys.TRACE_FIELDS)), np.nan)
        t0 = time.perf_counter()
        x, y, z, info = nys.ipm_solve(A, inst.b, inst.c, inst.q, trace=tr, **base, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        K = info.iters
        xs = inst.x_star
        rec = {"variant": name, "workload": args.workload, "seconds": round(t, 3), "status": info.status,
               "ipm_iters": K, "pcg_iters": info.pcg_iters_total, "builds": info.builds, "kkt_rel": info.kkt_rel,
               "x_rel_err_vs_planted": float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)),
               "time_split_ms": {"precond": round(info.t_sketch_ms, 1), "pcg": round(info.t_pcg_ms, 1),
                                 "other": round(info.t_other_ms, 1)},
               "ell_k": [int(v) for v in tr[:K, 3]], "d_hat_k": [round(float(v), 1) for v in tr[:K, 5]],
               "pcg_k": [int(v) for v in tr[:K, 7]]}
        print(json.dumps(rec), flush=True)


def large_leg(nys, torch, args):
    """lowrank_50000x200000 (FP32 A of 40 GB, BF16 sketch, ell = 400): one
    forward solve to KKT <= 1e-6 from entry to return (first call on this
    shape: the transposed copies are made inside), then the adjoint for
    dL/dc and dL/db with L = 1/2 ||x - x_tgt||^2, x_tgt = x* + 0.01 N(0,1);
    per-pass rates from the library's HIP events."""
    from instances import make_instance
    name = "lowrank_50000x200000"
    t0 = time.perf_counter()
    inst = make_instance(name, seed=args.seed, device="cuda")
    A = inst.A
    A_lo = A.to(torch.bfloat16)
    torch.cuda.synchronize()
    log(f"{name} generated in {time.perf_counter() - t0:.1f}s")
    nys.nys_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, y, z, info = nys.ipm_solve(A, inst.b, inst.c, inst.q, ell=inst.ell, tol=TOL, seed=args.seed,
                                  sketch_dtype="bf16", A_lo=A_lo)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    prof = nys.nys_profile_read()
    nys.nys_profile_enable(False)
    xs = inst.x_star
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed + 1)
    x_tgt = xs + 0.01 * torch.randn(xs.shape, generator=g, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grads, pinfo = nys.ipm_adjoint(A, inst.b, inst.c, inst.q, x, y, z, info.rho, info.delta, x - x_tgt,
                                   ell=inst.ell, A_lo=A_lo, want=("c", "b"), sketch_dtype="bf16")
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    bytes_pass = inst.m * inst.n * A.element_size()
    rates = {}
    for k in ("normal_pass1", "normal_pass2"):
        nl, ms = prof[k]
        rates[k] = round(bytes_pass / (ms / max(nl, 1) * 1e-3) / 1e9, 1)
    sk = {}
    for k in ("sketch_w", "sketch_y"):
        nl, ms = prof[k]
        if nl:
            sk[k] = {"launches": nl, "avg_ms": round(ms / nl, 3),
                     "TFLOPs": round(2.0 * inst.m * inst.n * inst.ell / (ms / nl * 1e-3) / 1e12, 1)}
    rec = {"workload": name, "m": inst.m, "n": inst.n, "ell": inst.ell, "A_storage": "float32",
           "forward_s": round(t_fwd, 3), "ipm_iters": info.iters, "pcg_iters": info.pcg_iters_total,
           "kkt_rel": info.kkt_rel, "x_rel_err_vs_planted": float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)),
           "adjoint_s": round(t_adj, 3), "adjoint_pcg_iters": pinfo.iters, "adjoint_pcg_status": pinfo.status,
           "grad_norms": {k: float(torch.linalg.norm(v)) for k, v in grads.items()},
           "normal_matvec_GBps": rates, "sketch_mfma": sk,
           "time_split_ms": {"sketch": round(info.t_sketch_ms, 1), "pcg": round(info.t_pcg_ms, 1),
                             "other": round(info.t_other_ms, 1)}}
    log(f"{name}: forward {t_fwd:.2f}s ({info.iters} it, {info.pcg_iters_total} PCG, kkt {info.kkt_rel:.1e}), "
        f"adjoint {t_adj:.2f}s ({pinfo.iters} PCG)")
    del A, A_lo, inst, x, y, z, grads
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lowrank_20000x100000")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-loop", type=int, default=0)
    ap.add_argument("--operator", default="", metavar="MxN")
    ap.add_argument("--ell", type=int, default=400)
    ap.add_argument("--nystrom", type=int, default=0)
    ap.add_argument("--reps", type=int, default=200)
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--adaptive", action="store_true")
    ap.add_argument("--dense-identity", action="store_true")
    ap.add_argument("--no-warmup-solve", action="store_true")
    ap.add_argument("--solvers", default="nystrom,pchol,none")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DB", "OUT_MD"))
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
    ap.add_argument("--command", default="")
    ap.add_argument("--out", default="")
    ap.add_argument("--oracle-child", default="", metavar="DIR")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--budget-s", type=float, default=540.0)
    args = ap.parse_args()
    if args.oracle_child:
        oracle_child(args.oracle_child, args.seed)
        return
    if args.compare and args.workload in SVM_SHAPES:
        import paper_2404_14524_amd as nys
        compare_svm(nys, args)
        return
    if args.compare and args.workload in PORTFOLIO_SHAPES:
        import paper_2404_14524_amd as nys
        compare_portfolio(nys, args)
        return
    if args.summarize_trace or args.summarize_pmc:
        from instances import CONFIGS
        cfg = CONFIGS[args.workload]
        b_A = 4 if cfg["a_dtype"] == "f32" else 8
        if args.summarize_trace:
            summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command, args.workload,
                            cfg["m"], cfg["n"], b_A)
        if args.summarize_pmc:
            summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, cfg["m"], cfg["n"], b_A,
                          args.command, args.out)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not supported "
              "(the path would shard A by columns with one all-reduce of the m-vector per operator apply)",
              file=sys.stderr)
        sys.exit(2)

    t_start = time.perf_counter()
    default_run = not (args.operator or args.compare or args.adaptive or args.kernel_loop)
    # the oracle child starts before this process touches the GPU
    oracle = OracleChild(args.seed) if default_run and not args.no_cpu_baseline else None

    import torch

    import paper_2404_14524_amd as nys
    from instances import make_instance

    if args.operator:
        operator_shape(nys, args.operator, args.ell, args.reps, args.seed, args.nystrom)
        return

    dev = "cuda"
    t0 = time.perf_counter()
    inst = make_instance(args.workload, seed=args.seed, device=dev)
    A = inst.A
    A_lo = A.to(torch.bfloat16) if A.dtype == torch.float32 else None
    torch.cuda.synchronize()
    log(f"instance {args.workload} m={inst.m} n={inst.n} ell={inst.ell} A={A.dtype} "
        f"generated in {time.perf_counter() - t0:.1f}s")
    b_A = A.element_size()
    bytes_pass = inst.m * inst.n * b_A
    if oracle is not None:
        oracle.provide(inst)

    if args.compare:
        compare(nys, inst, args)
        return
    if args.adaptive:
        adaptive_compare(nys, inst, args)
        return

    if args.kernel_loop:
        d = torch.rand(inst.n, dtype=torch.float64, device=dev)
        v = torch.randn(inst.m, dtype=torch.float64, device=dev)
        out = torch.empty_like(v)
        A_t = nys.nys_transpose(A)      # the layout ipm_solve gives pass 1
        for _ in range(args.kernel_loop):
            nys.nys_normal_apply(A, d, 1e-3, v, out, A_t=A_t)
        del A_t
        src = torch.ones(1 << 29, dtype=torch.float32, device=dev)    # 2 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        best = min(nys.nys_stream_read(A) for _ in range(5))
        log(f"read-stream reference: {bytes_pass / (best * 1e-3) / 1e9:.0f} GB/s over A")
        torch.cuda.synchronize()
        log(f"kernel loop done: {args.kernel_loop} normal applies ({bytes_pass} B per pass), "
            f"5 copies of {src.numel() * 4} B")
        return

    # measured read-stream reference over A (the achievable streaming rate on this machine)
    rs_ms = min(nys.nys_stream_read(A) for _ in range(5))
    read_stream_gbs = bytes_pass / (rs_ms * 1e-3) / 1e9
    log(f"read-stream reference over A: {read_stream_gbs:.0f} GB/s")

    mixed = dict(ell=inst.ell, tol=TOL, seed=args.seed, sketch_dtype="bf16" if A_lo is not None else "f64",
                 A_lo=A_lo, verbose=args.verbose)
    for w in range(args.warmup):
        x, y, z, info = nys.ipm_solve(A, inst.b, inst.c, inst.q, **mixed)
        torch.cuda.synchronize()
        log(f"warmup {w}: iters={info.iters} pcg={info.pcg_iters_total} kkt={info.kkt_rel:.2e}")

    nys.nys_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        x, y, z, info = nys.ipm_solve(A, inst.b, inst.c, inst.q, **mixed)
        # a progress line per solve (ipm_solve has read its device scalars, so
        # the solve has finished; the print costs microseconds of the ~14 s)
        log(f"step {s}: iters={info.iters} pcg={info.pcg_iters_total}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    prof = nys.nys_profile_read()
    nys.nys_profile_enable(False)
    ms_per_step = 1000.0 * t_total / args.steps
    t_sketch, t_pcg, t_other = info.t_sketch_ms, info.t_pcg_ms, info.t_other_ms
    xs = inst.x_star
    x_err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
    log(f"timed: {ms_per_step:.1f} ms/solve iters={info.iters} pcg={info.pcg_iters_total} "
        f"kkt={info.kkt_rel:.2e} |x-x*|/|x*|={x_err:.2e} sketch={t_sketch:.0f}ms pcg={t_pcg:.0f}ms "
        f"other={t_other:.0f}ms")

    # dominant kernel and its roofline
    passes = {k: prof[k] for k in ("normal_pass1", "normal_pass2")}
    dom = max(passes, key=lambda k: passes[k][1])
    launches, tot_ms = passes[dom]
    avg_ms = tot_ms / max(launches, 1)
    achieved = bytes_pass / (avg_ms * 1e-3) / 1e9
    pair_gbs = 2 * bytes_pass * min(passes["normal_pass1"][0], passes["normal_pass2"][0]) / \
        ((passes["normal_pass1"][1] + passes["normal_pass2"][1]) * 1e-3) / 1e9
    trec = load_traffic(args.workload)
    traffic = None
    if trec is not None:
        traffic = trec["hbm_bytes_per_launch"].get(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"k_gemv_{'tt' if dom == 'normal_pass1' else 'n'} ({dom})",
                "algorithmic_bytes_per_launch": bytes_pass, "launches": launches,
                "avg_launch_ms": round(avg_ms, 4), "read_stream_GBps": round(read_stream_gbs, 1),
                "frac_of_read_stream": round(achieved / read_stream_gbs, 4)}
    sk = {k: prof[k] for k in ("sketch_w", "sketch_y")}
    sketch_flops = 2.0 * inst.m * inst.n * inst.ell
    mfma = {}
    for k, (nl, ms) in sk.items():
        if nl:
            tf = sketch_flops / (ms / nl * 1e-3) / 1e12
            mfma[k] = {"launches": nl, "avg_ms": round(ms / nl, 3), "TFLOPs": round(tf, 1),
                       "mfma_util_bf16": round(tf / 2500.0, 4)}

    def left():
        return args.budget_s - (time.perf_counter() - t_start)

    fp64 = None
    fp64_runs = []
    A64 = None

    def fp64_run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x6, y6, z6, info6 = nys.ipm_solve(A64, inst.b, inst.c, inst.q, ell=inst.ell, tol=TOL, seed=args.seed,
                                          sketch_dtype="f64")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        fp64_runs.append(t64)
        log(f"fp64 run {len(fp64_runs)}: {t64:.2f}s iters={info6.iters} pcg={info6.pcg_iters_total} "
            f"kkt={info6.kkt_rel:.2e}")
        return x6, info6

    if not args.no_fp64:
        A64 = A.double()
        x6, info6 = fp64_run()
        fp64 = {"iters": info6.iters, "pcg_iters": info6.pcg_iters_total, "kkt_rel": info6.kkt_rel,
                "x_rel_err_vs_planted": float(torch.linalg.norm(x6 - xs) / torch.linalg.norm(xs)),
                "x_rel_diff_vs_mixed": float(torch.linalg.norm(x6 - x) / torch.linalg.norm(x6))}
        del x6

    # the large mixed-precision workload: forward solve, then the adjoint for c and b
    large = None
    if not args.no_large and args.workload == "lowrank_20000x100000":
        if left() > 90.0:
            del A64
            A64 = None
            large = large_leg(nys, torch, args)
        else:
            large = {"skipped": f"{left():.0f} s left of the bench's {args.budget_s:.0f} s budget"}

    if fp64 is not None:
        # two more FP64 runs for the median of three, when the budget allows
        while len(fp64_runs) < 3 and left() > 1.3 * fp64_runs[0] + 20.0:
            if A64 is None:
                A64 = A.double()
            fp64_run()
        ts = sorted(fp64_runs)
        fp64.update({"seconds": round(ts[len(ts) // 2], 3), "runs_s": [round(t, 3) for t in fp64_runs],
                     "speedup_mixed_over_fp64": round(ts[len(ts) // 2] / (ms_per_step / 1000.0), 3)})
        if len(fp64_runs) < 3:
            fp64["note"] = "fewer than three runs: the bench's time budget ran short"
        A64 = None

    cpu = None
    if oracle is not None:
        cpu = oracle.collect(info.iters, wait_s=left() - 10.0)
        log(f"cpu baseline: {cpu['value']} s ({cpu['sample']})")

    rec = {
        "metric": "time to 1e-6 KKT residual & normal-eq matvec GB/s: mixed-prec vs FP64, 1 GPU",
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64+f32+bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": inst.m, "n": inst.n, "ell": inst.ell,
                   "A_storage": str(A.dtype).replace("torch.", ""), "sketch": mixed["sketch_dtype"],
                   "pass1_layout": "transposed copy of A made inside the timed solve",
                   "tol": TOL, "instance_seed": args.seed},
        "accuracy": {"kkt_rel": info.kkt_rel, "rp_rel": info.rp_rel, "rd_rel": info.rd_rel, "mu": info.mu,
                     "x_rel_err_vs_planted": x_err, "ipm_iters": info.iters,
                     "pcg_iters": info.pcg_iters_total},
        "time_split_ms": {"sketch": round(t_sketch, 1), "pcg": round(t_pcg, 1), "other": round(t_other, 1)},
        "normal_matvec_GBps": {"pass1": round(bytes_pass / (passes["normal_pass1"][1] /
                                                           max(passes["normal_pass1"][0], 1) * 1e-3) / 1e9, 1),
                               "pass2": round(bytes_pass / (passes["normal_pass2"][1] /
                                                           max(passes["normal_pass2"][0], 1) * 1e-3) / 1e9, 1),
                               "pair": round(pair_gbs, 1)},
        "roofline": roofline,
        "sketch_mfma": mfma,
        "fp64_gpu": fp64,
        "large_mixed_with_adjoint": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
