#!/usr/bin/env python3
"""Benchmark of the canonical DMPT hot path on one MI355X.

Workload (default): the dense random-banded Hamiltonian, N = 8192 (bandwidth
256, entries 0.3 g exp(-|i-j|/32), diagonal U(-2, 2)), Ne = 4096, beta = 40,
n = 30 recursion steps, three diagonal dipole perturbations (x, y, z of a
32 x 16 x 16 grid), orders 0-2 (polarisability and hyperpolarisability), the
canonical Newton loop of Algorithm 1: one order-0 pass with the six int8
digit products of weight <= 2 (three digits) brings mu0 close, then an
order-0 pass and the linear schedule's order-1 and order-2 passes with all
thirteen digit products of weight <= 4 (each operand as one scale per matrix
times four signed int8 digits; products summed exactly in int32).
Per-step solves: the shared inverse of T' by Newton-Schulz (its start fitted
to the step's spectral interval; built once per step in the order-1 pass,
kept for the order-2 pass, applied with one product per right-hand side).
Inputs are synthetic, seeded, already resident in HBM when the timed region
starts.

One step = one complete canonical solve (dmpt_mu_newton): every Newton pass,
every recursion step, every order and direction.  value = response solves
per second = directions / seconds per step.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(the product kernel with the most device time, timed with HIP events on
the library's stream over the timed region), accuracy on the oracle's sampled entries, and
the FP64 CPU oracle timed on a bounded sample on this host.  The roofline's
"traffic" (HBM bytes per launch of that kernel) comes from the hardware
counter summary profiles/traffic_<engine>.json when it was taken on the
current product-kernel source, else null.

The accuracy-matched FP64 form (the same library in DMPT_FP64, same solvers)
is timed on the same workload after the timed region (one solve;
--no-fp64-compare skips it).  roofline.achieved is the algorithmic rate of
the dominant kernel: 2 N^3 flops per logical matrix product (every split
product of the same logical product counts once) over the kernel's device
time; the executed matrix-core rate (every split product counted) is
reported beside it as mfma_executed and mfma_util.

Other modes: --copy-calibration only runs a
plain device copy of known size, the reference that scales the FETCH_SIZE /
WRITE_SIZE counters into bytes; --workload batch64 times the batched
canonical solve of 64 uneven systems (FP32, orders 0-2, 3 directions, one
graph-captured pass per Newton update) and --workload adjoint4096 the
adjoint gradient of Tr(A P0) on the 16^3 cubic lattice (FP32, checkpoints
every 5 steps), each in the same JSON form.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense matrix-core peaks of an MI355X per engine (int8: TOP/s)
PEAKS_TFLOPS = {"bf16x3": 2500.0, "bf16x6": 2500.0, "int8x13": 5000.0, "int8x6": 5000.0, "fp32": 157.3,
                "fp64": 78.6}
DTYPE = {"bf16x3": "bf16", "bf16x6": "bf16", "int8x13": "i8", "int8x6": "i8", "fp32": "f32", "fp64": "f64"}
REFINE_NAME = {1: "bf16x6", 2: "int8x13"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="banded8192",
                    choices=["banded8192", "cubic2048", "chain128", "batch64", "adjoint4096"])
    ap.add_argument("--prec", default="int8x6", choices=list(PEAKS_TFLOPS))
    ap.add_argument("--n", type=int, default=0, help="shrink the banded workload to this N (testing)")
    ap.add_argument("--cpu-sample-n", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol-cg", type=float, default=0.0)
    ap.add_argument("--tol-occ", type=float, default=0.0)
    ap.add_argument("--refine", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="int8x6 / bf16x3: finish with the int8 13-product passes (2, default), the "
                         "6-product split-BF16 passes (1) or not at all (0)")
    ap.add_argument("--acc64", type=int, default=1,
                    help="6-product products: FP32 per 32-wide k slice, FP64 across slices (default 1)")
    ap.add_argument("--solver", default="hybrid", choices=["cg", "ns", "hybrid"],
                    help="per-step solver: conjugate gradients, the Newton-Schulz shared inverse, or the "
                         "shared inverse with FP64 and int8x13 products and CG with the others")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip the FP64 solve of the same workload on the GPU")
    ap.add_argument("--order", type=int, default=-1,
                    help="response order (default: the workload's; batch64 2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def kernel_source_sha():
    """SHA-256 of the product-kernel source the traffic counters must match."""
    path = os.path.join(ROOT, "paper_1503_07037_amd", "csrc", "gemm.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(engine, alg_bytes_per_launch):
    """HBM bytes per launch of the product kernel from the committed counter summary, or None
    when the kernel source changed since the counters were taken or the summary covers another
    launch mix (its algorithmic bytes per launch differ from this run's by more than 1 %)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{engine}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None
    ref = t.get("algorithmic_bytes_per_launch", 0.0)
    if not ref or abs(ref - alg_bytes_per_launch) > 0.01 * ref:
        return None
    return t


def copy_calibration():
    """A plain device-to-device copy of 2 GiB, five times (read 2 GiB + write 2 GiB each)."""
    import torch
    n = 1 << 28
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 5}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample, n_full, dirs):
    """The FP64 oracle on the same recipe at N = n_sample, scaled by (n_full/n_sample)^3."""
    import numpy as np
    import oracle
    import workloads
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max([p.get("num_threads", 1) for p in info] or [1])
        blas = ", ".join(sorted({f"{p.get('internal_api')} {p.get('version')}" for p in info
                                 if p.get("user_api") == "blas"})) or blas
    except Exception:
        threads = len(os.sched_getaffinity(0))
    c = workloads.config("banded8192", n_override=n_sample)
    h1v = [np.diag(h).copy() for h in c["H1"]]
    t0 = time.perf_counter()
    oracle.canonical_response(c["H0"], h1v, None, c["beta"], c["Ne"], c["n"], order=2)
    t = time.perf_counter() - t0
    scale = (n_full / n_sample) ** 3
    return {
        "value": dirs / (t * scale), "unit": "responses/s", "cores": threads, "kind": "oracle",
        "cpu_model": _cpu_model(), "blas": blas,
        "sample": (f"FP64 oracle (eigh + Daleckii-Krein, orders 0-2, {dirs} directions) on the banded "
                   f"recipe at N={n_sample}: {t:.2f} s, scaled by (N/{n_sample})^3 = {scale:.0f} to "
                   f"N={n_full}"),
    }


def accuracy(name, P0, P1, P2, mu, st=None):
    """Max errors on the oracle's stored samples (tests/golden/<name>_samples.npz), and the
    relative errors of the polarisability Tr(H1 P1) and hyperpolarisability Tr(H1 P2)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_samples.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    i = g["i"]
    j = g["j"]
    import torch
    ii = torch.as_tensor(i, device=P0.device)
    jj = torch.as_tensor(j, device=P0.device)
    e0 = float(np.abs(P0[ii, jj].cpu().numpy() - g["P0"]).max())
    e1 = max(float(np.abs(p[ii, jj].cpu().numpy() - g["P1"][z]).max() / g["max_P1"][z])
             for z, p in enumerate(P1))
    e2 = max(float(np.abs(p[ii, jj].cpu().numpy() - g["P2"][z]).max() / g["max_P2"][z])
             for z, p in enumerate(P2))
    res = {"P0_maxabs": e0, "P1_maxabs_rel": e1, "P2_maxabs_rel": e2,
           "mu0_err": abs(mu[0] - float(g["mu0"])), "samples": int(i.size),
           "measure": "max |GPU - oracle| over the sampled entries: P0 absolute, P1 and P2 divided "
                      "by max |P^(k)| of the oracle; traces relative"}
    if st is not None:
        res["tr_h1p1_rel"] = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p1"], g["tr_h1p1"]))
        if len(P2):
            res["tr_h1p2_rel"] = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p2"], g["tr_h1p2"]))
    return res


def fp64_gpu(dm, c, H0, H1, d, order):
    """One FP64 canonical solve of the same workload on the GPU, with the same solvers as the
    timed form (CG in the order-0 passes, the shared inverse in the passes with jets; its fastest
    FP64 form)."""
    import torch
    N = c["N"]
    ctx = dm.Context(N, dirs_max=d, prec="fp64", solver="hybrid")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.mu_newton(H0, H1, None, beta=c["beta"], Ne=c["Ne"], n=c["n"], order=order)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = out[4]
    ctx.close()
    return out, {"seconds": secs, "value": d / secs, "unit": "responses/s", "solver": "hybrid",
                 "newton_iters": st["newton_iters"], "cg_iters_total": st["cg_iters_total"],
                 "mfma_tflops": st["mfma_flops"] / secs / 1e12}


def _timed(fn, steps, warmup, sync):
    """Run fn warmup times untimed, then steps times; returns (last result, seconds per step list)."""
    out = None
    for w in range(warmup):
        t0 = time.perf_counter()
        out = fn()
        sync()
        print(f"warmup {w}: {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    times = []
    sync()
    for s in range(steps):
        t0 = time.perf_counter()
        out = fn()
        sync()
        times.append(time.perf_counter() - t0)
        print(f"step {s}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    return out, times


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return len(os.sched_getaffinity(0))


def run_batch64(args):
    """64 uneven cubic systems, FP32, orders 0-1, 3 directions: one batched canonical solve per step."""
    import numpy as np
    import torch
    import oracle
    import workloads
    import paper_1503_07037_amd as dm
    c = workloads.CONFIGS["batch64"]
    systems = workloads.batched_systems(c["seed"], count=c["count"])
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    H0s, H1s = [], []
    for sy in systems:
        lx, ly, lz = sy["dims"]
        H0s.append(T(workloads.cubic_lattice(lx, ly, lz, sy["seed"])))
        H1s.append([T(np.diag(v)) for v in workloads.lattice_dipoles(lx, ly, lz)])
    nmax = max(sy["N"] for sy in systems)
    d = c["dirs"]
    ctx = dm.Context(nmax, dirs_max=d, prec="fp32")
    betas = [sy["beta"] for sy in systems]
    nes = [sy["Ne"] for sy in systems]
    order = args.order if args.order >= 0 else c["order"]
    step = lambda: ctx.mu_newton_batched(H0s, H1s, betas, nes, n=c["n"], order=order)
    out, times = _timed(step, args.steps, args.warmup, torch.cuda.synchronize)
    P0, P1, P2, mus, st = out
    secs = sum(times)
    value = len(systems) * d * args.steps / secs
    mfma_tf = st["mfma_flops"] / (secs / args.steps) / 1e12
    useful_tf = st["useful_flops"] / (secs / args.steps) / 1e12
    acc = None
    path = os.path.join(ROOT, "tests", "golden", "batch64_samples.npz")
    if os.path.exists(path):
        g = np.load(path)
        e0 = e1 = e2 = 0.0
        for k in range(len(systems)):
            ii = torch.as_tensor(g["i"][k], device=dev)
            jj = torch.as_tensor(g["j"][k], device=dev)
            e0 = max(e0, float(np.abs(P0[k][ii, jj].cpu().numpy() - g["P0"][k]).max()))
            e1 = max(e1, max(float(np.abs(P1[k][z][ii, jj].cpu().numpy() - g["P1"][k][z]).max()
                                   / g["max_P1"][k][z]) for z in range(d)))
            if order >= 2 and "P2" in g.files:
                e2 = max(e2, max(float(np.abs(P2[k][z][ii, jj].cpu().numpy() - g["P2"][k][z]).max()
                                       / g["max_P2"][k][z]) for z in range(d)))
        acc = {"P0_maxabs": e0, "P1_maxabs_rel": e1, "systems": len(systems),
               "samples_per_system": int(g["i"].shape[1]),
               "measure": "max |GPU - oracle| over the sampled entries: P0 absolute, P1 and P2 "
                          "divided by max |P^(k)| of the oracle"}
        if order >= 2:
            acc["P2_maxabs_rel"] = e2
    res = {
        "metric": "batched canonical response solves/sec (P0+P1+P2), 64 uneven systems, FP32 MFMA",
        "value": value, "unit": "responses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64: 64 cubic tight-binding systems, N log-uniform in [256, 3072], "
                               f"beta U(5, 40), Ne = N/2, n = 25, 3 directions, orders 0-{order}",
                   "systems": len(systems), "sum_N": sum(sy["N"] for sy in systems),
                   "precision": "fp32", "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": useful_tf, "peak": PEAKS_TFLOPS["fp32"],
                     "unit": "TFLOP/s", "frac": useful_tf / PEAKS_TFLOPS["fp32"], "traffic": None,
                     "achieved_measure": "algorithmic: 2 N_pad^3 per logical product of the members "
                                         "that run (tallied on the device) over the wall time of one solve",
                     "mfma_executed": mfma_tf, "mfma_util": mfma_tf / PEAKS_TFLOPS["fp32"],
                     "kernel": "every FP32 product of the call"},
        "newton_passes": st["newton_iters"], "cg_iters_total": st["cg_iters_total"],
        "cg_unconverged": st["cg_unconverged"], "flags": st["flags"],
        "step_seconds": times, "accuracy": acc,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        # the oracle on the batch's systems in order until about 15 s, scaled by sum N^3
        t0 = time.perf_counter()
        done = 0
        for sy in systems:
            lx, ly, lz = sy["dims"]
            h0 = workloads.cubic_lattice(lx, ly, lz, sy["seed"])
            oracle.canonical_response(h0, list(workloads.lattice_dipoles(lx, ly, lz)), None, sy["beta"],
                                      sy["Ne"], c["n"], order=order)
            done += 1
            if time.perf_counter() - t0 > 15.0:
                break
        t = time.perf_counter() - t0
        frac = sum(sy["N"] ** 3 for sy in systems[:done]) / sum(sy["N"] ** 3 for sy in systems)
        res["cpu_baseline"] = {
            "value": len(systems) * d / (t / frac), "unit": "responses/s", "cores": _cpu_threads(),
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"FP64 oracle on the first {done} of the 64 systems ({t:.1f} s, "
                      f"{100 * frac:.1f} % of the batch's sum of N^3), scaled to the batch"}
    print(json.dumps(res), flush=True)


def run_adjoint(args):
    """Adjoint gradient of Tr(A P0) w.r.t. H0 (canonical), 16^3 cubic lattice, FP32 forward and backward."""
    import numpy as np
    import torch
    import oracle
    import workloads
    import paper_1503_07037_amd as dm
    c = workloads.config("adjoint4096")
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    N = c["N"]
    H0 = T(c["H0"])
    A = T(c["H1"][0])
    ctx = dm.Context(N, dirs_max=1, prec="fp32", ckpt_every=5)
    step = lambda: ctx.backward(H0, c["beta"], c["Ne"], c["n"], A)
    out, _ = _timed(step, args.warmup, 0, torch.cuda.synchronize)
    ctx.profile(True)
    out, times = _timed(step, args.steps, 0, torch.cuda.synchronize)
    prof = ctx.profile_get()
    ctx.profile(False)
    G, st = out
    secs = sum(times)
    dom = max(prof["engines"], key=lambda e: prof["engines"][e]["ms"])
    pe = prof["engines"][dom]
    achieved = pe["useful_flops"] / max(pe["ms"], 1e-12) / 1e9   # algorithmic
    executed = pe["mfma_flops"] / max(pe["ms"], 1e-12) / 1e9
    acc = None
    path = os.path.join(ROOT, "tests", "golden", "adjoint4096_samples.npz")
    if os.path.exists(path):
        g = np.load(path)
        ii = torch.as_tensor(g["i"], device=dev)
        jj = torch.as_tensor(g["j"], device=dev)
        acc = {"G_maxabs_rel": float(np.abs(G[ii, jj].cpu().numpy() - g["G"]).max() / g["max_G"]),
               "samples": int(g["i"].size)}
    res = {
        "metric": "adjoint gradients/sec of Tr(A P0) w.r.t. H0 (canonical), N=4096, FP32 MFMA",
        "value": args.steps / secs, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "adjoint4096: 16^3 cubic tight-binding, beta 20, n 25, Ne 2048, "
                               "A = diag(x), checkpoints every 5 steps",
                   "N": N, "precision": "fp32", "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAKS_TFLOPS["fp32"],
                     "unit": "TFLOP/s", "frac": achieved / PEAKS_TFLOPS["fp32"], "traffic": None,
                     "achieved_measure": "algorithmic: 2 N^3 per logical product over the kernel's "
                                         "device time",
                     "mfma_executed": executed, "mfma_util": executed / PEAKS_TFLOPS["fp32"],
                     "kernel": f"product kernel, {dom} engine", "launches": pe["launches"],
                     "avg_launch_ms": pe["ms"] / max(pe["launches"], 1),
                     "product_time_share": prof["ms"] / (1e3 * secs)},
        "mfma_tflops_whole_step": st["mfma_flops"] / (secs / args.steps) / 1e12,
        "newton_iters": st["newton_iters"], "cg_iters_total": st["cg_iters_total"],
        "step_seconds": times, "accuracy": acc,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        ns = 2048  # the same recipe on a 16 x 16 x 8 lattice, scaled by (N/2048)^3
        h0 = workloads.cubic_lattice(16, 16, 8, c["seed"])
        x = workloads.lattice_dipoles(16, 16, 8)[0]
        t0 = time.perf_counter()
        oracle.adjoint_grad(h0, c["beta"], ns / 2.0, c["n"], np.diag(x))
        t = time.perf_counter() - t0
        res["cpu_baseline"] = {
            "value": 1.0 / (t * (N / ns) ** 3), "unit": "gradients/s", "cores": _cpu_threads(),
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"FP64 oracle adjoint on the 16 x 16 x 8 lattice: {t:.2f} s, scaled by (N/2048)^3 = 8"}
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded "
              f"path is not built.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch64":
        run_batch64(args)
        return
    if args.workload == "adjoint4096":
        run_adjoint(args)
        return
    import numpy as np
    import torch
    import workloads
    import paper_1503_07037_amd as dm

    dev = torch.device("cuda:0")
    c = workloads.config(args.workload, n_override=args.n or None)
    N, d = c["N"], len(c["H1"])
    order = c["order"]
    H0 = torch.tensor(c["H0"], device=dev)
    H1 = [torch.tensor(h, device=dev) for h in c["H1"]]
    torch.cuda.synchronize()
    refine = (2 if args.prec in ("bf16x3", "int8x6") else 0) if args.refine < 0 else args.refine
    ctx = dm.Context(N, dirs_max=d, prec=args.prec, tol_cg=args.tol_cg, tol_occ=args.tol_occ,
                     refine=refine, acc64=args.acc64, solver=args.solver)

    def step():
        return ctx.mu_newton(H0, H1, None, beta=c["beta"], Ne=c["Ne"], n=c["n"], order=order)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        print(f"warmup {w}: {time.perf_counter() - t0:.2f} s newton={out[4]['newton_iters']} "
              f"cg={out[4]['cg_iters_total']}", file=sys.stderr, flush=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for s in range(args.steps):
        out = step()
        marks.append(time.perf_counter() - t0)
        print(f"step {s}: {marks[-1]:.2f} s cumulative", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    prof = ctx.profile_get()
    ctx.profile(False)
    P0, P1, P2, mu, st = out
    ms_step = 1e3 * secs / args.steps
    value = d * args.steps / secs
    # dominant product kernel: the engine with the most device time
    dom = max(prof["engines"], key=lambda e: prof["engines"][e]["ms"])
    pe = prof["engines"][dom]
    avg_ms = pe["ms"] / max(pe["launches"], 1)
    achieved = pe["useful_flops"] / max(pe["ms"], 1e-12) / 1e9   # algorithmic TFLOP/s
    executed = pe["mfma_flops"] / max(pe["ms"], 1e-12) / 1e9     # every split product counted
    peak = PEAKS_TFLOPS[dom]
    name = args.workload if not args.n else None
    acc = accuracy(name, P0, P1, P2, mu, st) if name else None
    traffic = measured_traffic(dom, pe["bytes"] / max(pe["launches"], 1))
    res = {
        "metric": "response solves/sec (P0+P1+P2) and MFMA TFLOP/s at N=8192, err <=1e-6 vs FP64",
        "value": value, "unit": "responses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[dom], "data": "synthetic",
        "config": {"workload": f"{args.workload}: banded N={N}, d={d}, orders 0-{order}, "
                               f"beta={c['beta']}, n={c['n']}, Ne={c['Ne']}" if args.workload == "banded8192"
                   else args.workload,
                   "N": N, "dirs": d, "order": order, "beta": c["beta"], "n": c["n"],
                   "solver": args.solver,
                   "precision": args.prec + (f"+refine({REFINE_NAME[refine]})" if refine else "")
                   + (", 6-product sums FP64 across 32-wide k slices" if args.acc64 and
                      (refine == 1 or args.prec == "bf16x6") else "")
                   + (", int8 digit products summed exactly in int32" if
                      (refine == 2 or args.prec.startswith("int8")) else ""),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "achieved_measure": "algorithmic: 2 N^3 per logical product and member over "
                                         "the kernel's device time; peak is the dense matrix-core "
                                         f"rate of the kernel's own type ({DTYPE[dom]})",
                     "mfma_executed": executed, "mfma_util": executed / peak,
                     "algorithmic_flops_per_launch": pe["useful_flops"] / max(pe["launches"], 1),
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": pe["bytes"] / max(pe["launches"], 1),
                     "kernel": f"product kernel, {dom} engine", "launches": pe["launches"],
                     "avg_launch_ms": avg_ms,
                     "product_time_share": prof["ms"] / ms_step / args.steps,
                     "engines": {e: {"launches": v["launches"], "ms": v["ms"],
                                     "mfma_tflops": v["mfma_flops"] / max(v["ms"], 1e-12) / 1e9,
                                     "algorithmic_tflops": v["useful_flops"] / max(v["ms"], 1e-12) / 1e9}
                                 for e, v in prof["engines"].items() if v["launches"]}},
        "mfma_tflops_whole_step": st["mfma_flops"] / (ms_step / 1e3) / 1e12,
        "useful_tflops_whole_step": st["useful_flops"] / (ms_step / 1e3) / 1e12,
        "newton_iters": st["newton_iters"], "cg_iters_total": st["cg_iters_total"],
        "step_seconds": [b - a for a, b in zip([0.0] + marks[:-1], marks)],
        "accuracy": acc,
    }
    ctx.close()
    del P0, P1, P2, out
    if not args.no_fp64_compare:
        out64, f64 = fp64_gpu(dm, c, H0, H1, d, order)
        f64["accuracy"] = accuracy(name, out64[0], out64[1], out64[2], out64[3], out64[4]) if name else None
        f64["speedup_of_this_run"] = value / f64["value"]
        res["fp64_gpu"] = f64
        del out64
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(min(args.cpu_sample_n, N), N, d)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
