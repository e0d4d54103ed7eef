"""Benchmark: unknowns solved per second for series of symmetric
tridiagonal systems on one MI355X, FP32-refined path vs plain FP64 path at
equal residual, with the fraction of the HBM roofline.

Default run (`--workload suite`): the headline is the ADI-shaped line solves
(M = N = 8192, b = 2.05, a = -1, right-hand sides = the grid lines of a
smooth Gaussian random field, correlation length 64 cells, stored FP32;
P = 128 blocks), the workload the metric's FP32-refined vs FP64 comparison
is stated on.  Nested under "workloads": the uneven batch (256 matrices of
M log-uniform in [128, 16384], N uniform in [1, 2048], block counts from the
batch autotuner) and the 1-D Poisson series (M = N = 4096, 8 sine modes +
noise, P = 64), each with its own roofline, comparison and CPU baseline.

One step = one full solve (beta weights, interface step, block sweeps) from
inputs already resident in device memory.  Buffer sets are rotated so that
consecutive steps do not find their data in the 256 MB last-level cache.
Single workloads: `--workload adi|poisson|batch|gradient|fourier`.  The
preliminary step (host FP64 tables + upload) is timed separately
(`prepare_ms`).

Prints one JSON line.  --gpus above 1 is refused: the build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
F_BYTES = {"f32_refined": 4, "f32_wide": 4, "f32": 4, "f64": 8}
X_BYTES = {"f32_refined": 8, "f32_wide": 8, "f32": 4, "f64": 8}
DTYPE = {"f32_refined": "f32+f64", "f64": "f64", "f32_wide": "f32->f64", "f32": "f32"}
METRIC = "unknowns solved/s + % HBM peak, FP32-refined vs FP64 plain at equal residual"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--mode", default="f32_refined",
                   choices=["f32_refined", "f64", "f32_wide", "f32"])
    p.add_argument("--workload", default="suite",
                   choices=["suite", "poisson", "adi", "batch", "gradient", "fourier"],
                   help="suite (default): adi as the headline, batch and poisson nested; "
                        "poisson: 1-D Poisson series 4096x4096, P=64; "
                        "adi: ADI line solves 8192x8192, b=2.05, P=128; "
                        "batch: 256 uneven matrices, autotuned block counts; "
                        "gradient: 2048x1024 forward + adjoint, P=32; "
                        "fourier: series of 256 2-D Poisson problems on a 1024^2 mesh")
    p.add_argument("--M", type=int, default=0)
    p.add_argument("--N", type=int, default=0)
    p.add_argument("--P", type=int, default=0)
    p.add_argument("--passes", type=int, default=None,
                   help="refinement passes of the f32_refined mode; default: the autotuner's "
                        "(the fewest whose residual on the workload's right-hand sides stays "
                        "within 1.25 times that of the FP64-arithmetic solve)")
    p.add_argument("--interface", default="auto",
                   choices=["auto", "recurrence", "dichotomy", "dense"],
                   help="evaluation order of the interface values (single-matrix workloads); "
                        "auto: the autotuner's measured choice")
    p.add_argument("--batch-fused", type=int, default=16,
                   help="lag (tiles of 256 right-hand sides) of the uneven batch's one-launch "
                        "order when it is timed beside the autotuner's choice of the separate "
                        "launches (0: not timed)")
    p.add_argument("--fused", type=int, default=None,
                   help="lag of the fused order (single-matrix workloads; 0: three launches "
                        "per solve); default: the autotuner's measured choice")
    p.add_argument("--batch-rows", type=int, default=0, choices=[0, 32, 64],
                   help="rows per block of the uneven batch (0: the batch autotuner's choice; "
                        "32 or 64 fix it, e.g. to profile one configuration)")
    p.add_argument("--launch", default="auto", choices=["auto", "eager", "graph"],
                   help="time eager launches or replays of a captured HIP graph per step; auto: "
                        "graph replays for the uneven batch, eager launches for the "
                        "single-matrix workloads (replays measured slower there: Poisson "
                        "56.1 against 51.0 us per step, ADI 231.6 against 227.5 us)")
    p.add_argument("--sets", type=int, default=0,
                   help="buffer sets rotated across steps (0: enough to exceed 512 MB)")
    p.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison runs")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="first stream this many MiB through a plain elementwise kernel (read + "
                        "write of known size) to calibrate rocprofv3 FETCH_SIZE/WRITE_SIZE")
    return p.parse_args()


def oracle_one_thread(a, b, F, seconds):
    """unknowns/s of the oracle on one host thread: a child process (OpenMP's
    thread count is fixed when the library loads) that touches no GPU."""
    import subprocess
    import tempfile

    import numpy as np
    with tempfile.TemporaryDirectory() as d:
        for name, arr in (("a", a), ("b", b), ("F", F)):
            np.save(os.path.join(d, name + ".npy"), np.ascontiguousarray(arr))
        code = (
            "import sys, time, numpy as np\n"
            f"sys.path.insert(0, {ROOT!r})\n"
            "import oracle\n"
            f"d = {d!r}\n"
            "a, b, F = (np.load(d + '/' + n + '.npy') for n in ('a', 'b', 'F'))\n"
            "reps, t0 = 0, time.perf_counter()\n"
            "while True:\n"
            "    oracle.thomas(a, b, F)\n"
            "    reps += 1\n"
            f"    if time.perf_counter() - t0 >= {float(seconds)}:\n"
            "        break\n"
            "print(reps * F.shape[0] * F.shape[1] / (time.perf_counter() - t0))\n")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=seconds + 120, env=dict(os.environ, OMP_NUM_THREADS="1"))
    if r.returncode != 0:
        return None
    return float(r.stdout.strip().splitlines()[-1])


def copy_bandwidth(torch, dev, mib=512, reps=20):
    """Measured HBM rate of a plain device copy (torch's copy kernel, `mib`
    MiB read and written per launch), the practical ceiling the sweeps are
    read against; GB/s counts the bytes read plus the bytes written."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(src)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    gbs = 2 * src.numel() * 4 / (ms * 1e-3) / 1e9
    del src, dst
    return {"kernel": "torch copy_", "bytes_per_launch": 2 * (mib << 20), "ms_per_launch": round(ms, 5),
            "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def graph_for(args, kind):
    """Whether a workload of `kind` ('single' or 'batch') is timed from graph
    replays."""
    return args.launch == "graph" or (args.launch == "auto" and kind == "batch")


def time_steps(solve, n_sets, steps, warmup, graph, timed_plan, torch):
    """ms per step over `steps` calls of solve(k) (eager launches, or replays
    of one captured HIP graph per buffer set), then the per-phase split from
    a separate eager run with the library's phase events on."""
    for k in range(max(warmup, n_sets)):
        solve(k)
    torch.cuda.synchronize()
    graphs = []
    if graph:
        for k in range(n_sets):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                solve(k)
            graphs.append(g)
        for k in range(warmup):
            graphs[k % n_sets].replay()

        def step(k):
            graphs[k % n_sets].replay()
    else:
        step = solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(steps):
        step(k)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    # per-step distribution, in a separate pass (events around every step)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        step(k)
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    del graphs
    # phase split (events between the launches of each solve)
    timed_plan.timing(True)
    timed_plan.timing_read()                 # clear
    for k in range(min(steps, 20)):
        solve(k)
    torch.cuda.synchronize()
    ms_beta, ms_iface, ms_sweep, calls = timed_plan.timing_read()
    timed_plan.timing(False)
    return dict(ms_per_step=ms_total / steps, wall_s=wall,
                ms_step_median=per[steps // 2], ms_step_min=per[0],
                ms_beta=ms_beta / calls, ms_iface=ms_iface / calls,
                ms_sweep=ms_sweep / calls, launch="graph" if graph else "eager")


class Single:
    """One matrix, rotated buffer sets."""

    def __init__(self, args, t, wl, torch):
        self.args, self.t, self.torch = args, t, torch
        if args.workload == "poisson":
            M, N, P = args.M or 4096, args.N or 4096, args.P or 64
            w = wl.poisson_series(M=M, N=N, P=P)
            self.name = ("1-D Poisson series (sum of 8 sine modes + noise), FP32 storage with "
                         "FP64 refinement")
        else:
            M, N, P = args.M or 8192, args.N or 8192, args.P or 128
            w = wl.adi_lines(M=M, N=N, P=P)
            self.name = ("ADI line solves on a smooth Gaussian random field (b=2.05), "
                         "FP32 storage")
        self.M, self.N, self.P = M, N, P
        self.a, self.b, self.F32 = w["a"], w["b"], w["F"]
        t0 = time.perf_counter()
        self.plan = t.Plan(self.a, self.b, P)
        torch.cuda.synchronize()
        self.prepare_ms = (time.perf_counter() - t0) * 1e3
        # interface order, fused order and refinement passes: measured by the
        # autotuner on the workload's own right-hand sides (the block count
        # is the workload's)
        self.tuning = None
        if args.interface == "auto" or args.fused is None or args.passes is None:
            Fd = torch.from_numpy(self.F32).to("cuda:0")
            if F_BYTES[args.mode] == 8:
                Fd = Fd.double()
            self.tuning = t.autotune_plan(self.a, self.b, N, args.mode, P=P, F=Fd)
            del Fd
        order = self.tuning["order"] if args.interface == "auto" else args.interface
        self.plan.set_interface(order)
        if args.passes is not None:
            self.passes = args.passes
        elif args.mode == "f32_refined":
            self.passes = self.tuning["passes"]
        else:
            self.passes = 2
        self.plan.set_refinement(self.passes)
        if args.fused is None:
            lag, tile = self.tuning["fuse_lag"], self.tuning["fuse_tile"]
        else:
            lag, tile = args.fused, 512
        self.plan.set_fused(lag, tile or 512)
        self.unknowns = M * N
        self.config = {"workload": self.name, "M": M, "N": N, "P": P, "interface": order,
                       "fused_lag": lag, "fused_tile": tile if lag else 0,
                       "tuning": self.tuning}

    def sweep_bytes(self, mode):
        # the block sweep reads F, writes X, reads two interface values per
        # block and right-hand side
        return self.unknowns * (F_BYTES[mode] + X_BYTES[mode]) + 2 * (self.P - 1) * self.N * 8

    def run(self, mode, steps, warmup):
        torch, args = self.torch, self.args
        dev = torch.device("cuda:0")
        per_set = self.unknowns * (F_BYTES[mode] + X_BYTES[mode])
        n_sets = args.sets or max(1, -(-(512 << 20) // per_set) + 1)
        Fd = torch.from_numpy(self.F32).to(dev)
        if F_BYTES[mode] == 8:
            Fd = Fd.double()
        xdt = torch.float64 if X_BYTES[mode] == 8 else torch.float32
        Fs = [Fd] + [Fd.clone() for _ in range(n_sets - 1)]
        Xs = [torch.empty((self.M, self.N), dtype=xdt, device=dev) for _ in range(n_sets)]

        def solve(k):
            self.plan.solve(Fs[k % n_sets], Xs[k % n_sets], mode=mode)

        r = time_steps(solve, n_sets, steps, warmup, graph_for(args, "single"), self.plan, torch)
        if n_sets > 1:
            # warm: one buffer set, which the last-level cache may hold
            warm = time_steps(lambda k: self.plan.solve(Fs[0], Xs[0], mode=mode), 1,
                              max(10, steps // 2), 3, graph_for(args, "single"), self.plan, torch)
            r["warm_ms_per_step"] = warm["ms_per_step"]
        eta, r2 = self.plan.residual(Fs[0], Xs[0], mode=mode)
        torch.cuda.synchronize()
        r["eta_max"], r["r2_max"], r["sets"] = float(eta.max()), float(r2.max()), n_sets
        del Fs, Xs
        torch.cuda.empty_cache()
        return r

    def cpu_baseline(self, seconds):
        import numpy as np
        import oracle
        Fw = self.F32.astype(np.float64)
        reps, t0 = 0, time.perf_counter()
        while True:
            oracle.thomas(self.a, self.b, Fw)
            reps += 1
            if time.perf_counter() - t0 >= seconds:
                break
        el = time.perf_counter() - t0
        one = oracle_one_thread(self.a, self.b, Fw[:, :512], seconds / 2)
        return {"value": reps * self.unknowns / el, "unit": "unknowns/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"FP64 sequential sweep per RHS (OpenMP over RHS) on the full "
                          f"{self.M}x{self.N} series, repeated {reps}x over {el:.1f} s",
                "value_1_thread": one,
                "sample_1_thread": f"the first 512 right-hand sides, one thread "
                                   f"(OMP_NUM_THREADS=1 in a child process), about "
                                   f"{seconds / 2:.0f} s"}


class Batch:
    """256 matrices of uneven sizes and series lengths in one batch plan."""

    def __init__(self, args, t, wl, torch):
        self.args, self.t, self.torch = args, t, torch
        w = wl.uneven_batch()
        self.items = w["items"]
        self.a = [it["a"] for it in self.items]
        self.b = [it["b"] for it in self.items]
        self.Ms = [it["M"] for it in self.items]
        self.Ns = [it["N"] for it in self.items]
        self.P, tuned_passes, self.lag, self.tune_ms = t.batch_autotune(
            self.a, self.b, self.Ns, args.mode, with_order=True)
        if args.batch_rows:
            self.P = [1 if m < 4 else max(1, min(-(-m // args.batch_rows), m // 2, 65535))
                      for m in self.Ms]
        if args.passes is not None:
            self.passes = args.passes
        elif args.mode == "f32_refined":
            self.passes = tuned_passes
        else:
            self.passes = 2
        t0 = time.perf_counter()
        self.plan = t.BatchPlan(self.a, self.b, self.P)
        self.plan.set_refinement(self.passes)
        if args.batch_rows:
            self.lag = 0
        self.plan.set_fused(self.lag)
        torch.cuda.synchronize()
        self.prepare_ms = (time.perf_counter() - t0) * 1e3
        self.unknowns = sum(m * n for m, n in zip(self.Ms, self.Ns))
        self.name = ("uneven batch: 256 matrices, M log-uniform [128, 16384], b = 2 + U[0.01, 1], "
                     "a = -1, N uniform [1, 2048], FP32 storage")
        # matrices per register row bucket (32 or 64 rows per block)
        per_bucket = {"32": sum(1 for m, p in zip(self.Ms, self.P) if -(-m // p) <= 32)}
        per_bucket["64"] = len(self.P) - per_bucket["32"]
        self.config = {"workload": self.name, "K": len(self.items), "unknowns": self.unknowns,
                       "matrices_by_rows_per_block": per_bucket,
                       "launch_order": ("one launch, lag %d tiles" % self.lag) if self.lag
                       else "separate launches",
                       "tuning": {"matrices_by_rows_per_block": per_bucket,
                                  "passes": tuned_passes, "fuse_lag": self.lag,
                                  "ms": self.tune_ms}}

    def sweep_bytes(self, mode):
        return sum(m * n * (F_BYTES[mode] + X_BYTES[mode]) + 2 * (p - 1) * n * 8
                   for m, n, p in zip(self.Ms, self.Ns, self.P))

    def run(self, mode, steps, warmup):
        torch, args = self.torch, self.args
        dev = torch.device("cuda:0")
        Fs = []
        for it in self.items:
            F = torch.from_numpy(it["F"]).to(dev)
            Fs.append(F.double() if F_BYTES[mode] == 8 else F)
        xdt = torch.float64 if X_BYTES[mode] == 8 else torch.float32
        Xs = [torch.empty((m, n), dtype=xdt, device=dev) for m, n in zip(self.Ms, self.Ns)]

        def solve(k):
            self.plan.solve(Fs, Xs, mode=mode)

        r = time_steps(solve, 1, steps, warmup, graph_for(args, "batch"), self.plan, torch)
        # the other launch order of the same batch (bitwise the same X),
        # timed the same way: the one-launch order (tdsolve_batch_set_fused,
        # lag --batch-fused) beside the separate launches or the reverse,
        # when every matrix has blocks of at most 32 rows (otherwise the
        # library runs the separate launches)
        r["other_order"] = None
        alt = args.batch_fused if self.lag == 0 else 0
        if (alt > 0 or self.lag > 0) and all(-(-m // p) <= 32 for m, p in zip(self.Ms, self.P)):
            self.plan.set_fused(alt)
            f = time_steps(solve, 1, max(10, steps // 2), max(3, warmup // 2),
                           graph_for(args, "batch"), self.plan, torch)
            self.plan.set_fused(self.lag)
            r["other_order"] = {"launch_order": ("one launch, lag %d tiles" % alt) if alt
                                else "separate launches",
                                "ms_per_step": round(f["ms_per_step"], 5), "launch": f["launch"]}
        # residuals of every matrix of the batch: the largest normwise
        # backward error from the library (tdsolve_status, which recomputes
        # the last batch solve's residuals), and the relative 2-norm residual
        # of every right-hand side by torch ops on the device (a check of
        # the result, outside the timed solve)
        solve(0)
        eta, _ = self.plan.status()
        r2 = 0.0
        for a, b, F, X in zip(self.a, self.b, Fs, Xs):
            a_d = torch.from_numpy(a).to(dev)[:, None]
            b_d = torch.from_numpy(b).to(dev)[:, None]
            Fw = F.double()
            R = Fw - b_d * X
            R[:-1] -= a_d * X[1:]
            R[1:] -= a_d * X[:-1]
            r2 = max(r2, float((R.norm(dim=0) / Fw.norm(dim=0).clamp_min(1e-300)).max()))
        r["eta_max"], r["r2_max"], r["sets"] = float(eta), r2, 1
        del Fs, Xs
        torch.cuda.empty_cache()
        return r

    def cpu_baseline(self, seconds):
        import numpy as np
        import oracle
        done, t0, k = 0, time.perf_counter(), 0
        while time.perf_counter() - t0 < seconds and k < len(self.items):
            it = self.items[k]
            oracle.thomas(it["a"], it["b"], it["F"].astype(np.float64))
            done += it["M"] * it["N"]
            k += 1
        el = time.perf_counter() - t0
        return {"value": done / el, "unit": "unknowns/s", "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": f"FP64 sequential sweep per RHS on the first {k} of the "
                          f"{len(self.items)} matrices ({done} unknowns) in {el:.1f} s"}


class Gradient(Single):
    """Forward solve and adjoint of loss = sum(W * X): one step computes X,
    then gF = A^{-1} W and the reductions ga, gb with the same plan."""

    def __init__(self, args, t, wl, torch):
        self.args, self.t, self.torch = args, t, torch
        w = wl.gradient_case()
        self.M, self.N, self.P = w["M"], w["N"], w["P"]
        self.a, self.b, self.F32, self.W = w["a"], w["b"], w["F"], w["W"]
        t0 = time.perf_counter()
        self.plan = t.Plan(self.a, self.b, self.P)
        self.passes = args.passes if args.passes is not None else 2
        self.plan.set_refinement(self.passes)
        torch.cuda.synchronize()
        self.prepare_ms = (time.perf_counter() - t0) * 1e3
        self.unknowns = self.M * self.N
        self.name = ("differentiation: b = 3 + U[0, 1], a ~ U[-1, -0.5], FP32 storage, "
                     "forward + adjoint (gF, ga, gb) per step")
        self.config = {"workload": self.name, "M": self.M, "N": self.N, "P": self.P}

    def run(self, mode, steps, warmup):
        torch = self.torch
        dev = torch.device("cuda:0")
        F = torch.from_numpy(self.F32).to(dev)
        if F_BYTES[mode] == 8:
            F = F.double()
        xdt = torch.float64 if X_BYTES[mode] == 8 else torch.float32
        X = torch.empty((self.M, self.N), dtype=xdt, device=dev)
        W = torch.from_numpy(self.W).to(dev).to(xdt)

        def solve(k):
            self.plan.solve(F, X, mode=mode)
            self.plan.backward(X, W, mode=mode)

        r = time_steps(solve, 1, steps, warmup, graph_for(self.args, "single"), self.plan, torch)
        eta, r2 = self.plan.residual(F, X, mode=mode)
        torch.cuda.synchronize()
        r["eta_max"], r["r2_max"], r["sets"] = float(eta.max()), float(r2.max()), 1
        return r


class Fourier:
    """Series of S 2-D Poisson problems by the variable separation method."""

    def __init__(self, args, t, wl, torch):
        from paper_0901_2859_amd.fourier import FourierPoisson2D
        self.args, self.t, self.torch = args, t, torch
        self.n = args.M or 1024
        self.S = args.N or 256
        self.unknowns = self.S * (self.n - 1) ** 2
        self.name = (f"variable separation (Fourier) method: {self.S} 2-D Poisson problems "
                     f"on a {self.n}x{self.n} mesh, 5-point operator, uniform random sources")
        self.config = {"workload": self.name, "mesh": self.n, "problems": self.S}
        self.cls = FourierPoisson2D
        self.solvers = {}
        t0 = time.perf_counter()
        self.solver(args.mode)
        torch.cuda.synchronize()
        self.prepare_ms = (time.perf_counter() - t0) * 1e3
        self.P = self.solvers[args.mode].P

    def solver(self, mode):
        if mode not in self.solvers:
            self.solvers[mode] = self.cls(self.n, self.n, self.S, mode=mode)
            self.passes = self.args.passes if self.args.passes is not None else 2
            self.solvers[mode].plan.set_refinement(self.passes)
        return self.solvers[mode]

    def sweep_bytes(self, mode):
        M, N = self.n - 1, self.S
        return sum(M * N * (F_BYTES[mode] + X_BYTES[mode]) + 2 * (p - 1) * N * 8 for p in self.P)

    def run(self, mode, steps, warmup):
        torch = self.torch
        import numpy as np
        fp = self.solver(mode)
        rng = np.random.default_rng(6)
        f = torch.from_numpy(rng.uniform(-1, 1, size=(self.S, self.n - 1, self.n - 1))).cuda()
        if mode != "f64":
            f = f.float()

        def solve(k):
            fp.solve(f)

        r = time_steps(solve, 1, steps, warmup, graph_for(self.args, "batch"), fp.plan, torch)
        r["eta_max"], r["r2_max"], r["sets"] = None, None, 1
        return r

    def cpu_baseline(self, seconds):
        import numpy as np
        from oracle import poisson2d
        import oracle
        rng = np.random.default_rng(6)
        h = 1.0 / self.n
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds and done < self.S:
            poisson2d.solve_direct(rng.uniform(-1, 1, size=(self.n - 1, self.n - 1)), h, h)
            done += 1
        el = time.perf_counter() - t0
        return {"value": done * (self.n - 1) ** 2 / el, "unit": "unknowns/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"direct sparse LU of the 5-point problem, {done} of the "
                          f"{self.S} problems in {el:.1f} s"}


def equal_residual(reports):
    """The fastest mode whose largest relative residual reaches the plain
    FP64 sweep's (r2 <= r2_f64 + 1e-10, the residual reading of the
    accuracy target); a mode's time is that of its faster launch order
    where two were timed (the batch: both give bitwise the same X)."""
    ref = reports.get("f64", {}).get("r2_max")
    if ref is None:
        return None

    def ms(r):
        o = r.get("other_order")
        return min(r["ms_per_step"], o["ms_per_step"]) if o else r["ms_per_step"]

    ok = {m: r for m, r in reports.items() if r.get("r2_max") is not None
          and r["r2_max"] <= ref + 1e-10}
    best = min(ok, key=lambda m: ms(ok[m]))
    return {"r2_max": {m: r.get("r2_max") for m, r in reports.items()},
            "ms_per_step": {m: round(ms(r), 5) for m, r in reports.items()},
            "fastest_at_fp64_residual": best}


def workload_report(name, args, t, wl, torch, dev, mode, steps, warmup, passes=None):
    """Time one workload in `mode` (and the comparison modes), with its
    roofline, path fraction and CPU baseline."""
    from paper_0901_2859_amd import profdigest
    a2 = argparse.Namespace(**vars(args))
    a2.workload = name
    a2.mode = mode
    a2.passes = passes if passes is not None else args.passes
    W = {"batch": Batch, "gradient": Gradient, "fourier": Fourier}.get(name, Single)(
        a2, t, wl, torch)

    def run(m, k, w):
        r = W.run(m, k, w)
        r["unknowns_per_s"] = W.unknowns / (r["ms_per_step"] * 1e-3)
        alg = W.unknowns * (F_BYTES[m] + X_BYTES[m])
        r["path_gbs"] = alg / (r["ms_per_step"] * 1e-3) / 1e9
        r["path_bytes"] = alg
        return r

    main_r = run(mode, steps, warmup)
    # dominant kernel: the block sweep
    sweep_bytes = W.sweep_bytes(mode)
    ms_sweep = main_r["ms_sweep"]
    achieved = sweep_bytes / (ms_sweep * 1e-3) / 1e9
    batched = name in ("batch", "fourier")
    if batched:
        # the batch sweeps one launch per register row bucket (32, 64 rows);
        # the phase time covers both when the autotuner mixed them
        buckets = sorted({32 if -(-m // p) <= 32 else 64 for m, p in zip(W.Ms, W.P)}) \
            if name == "batch" else [0]
        if name == "batch":
            by = {r: sum(m * n for m, n, p in zip(W.Ms, W.Ns, W.P)
                         if (32 if -(-m // p) <= 32 else 64) == r) for r in buckets}
            rows = max(by, key=by.get)
        else:
            rows = 0
        kname = "k_sweep_batch_halves" if rows == 64 and mode != "f32" else "k_sweep_batch"
        shape = (f"{name}_r{rows}" if len(buckets) == 1 else f"{name}_mixed") \
            if name == "batch" else name
        if getattr(W, "lag", 0) > 0:
            # the whole step in one launch (timed as the sweep phase): its
            # algorithmic bytes are the path's, F read once and X written once
            kname = "k_fused_batch"
            sweep_bytes = W.unknowns * (F_BYTES[mode] + X_BYTES[mode])
            achieved = sweep_bytes / (ms_sweep * 1e-3) / 1e9
    elif mode != "f32" and W.plan.info().sweep_halves:
        kname = "k_sweep_halves"
        shape = f"{name}_{W.M}x{W.N}_P{W.P}"
    else:
        kname = "k_sweep_reg"
        shape = f"{name}_{W.M}x{W.N}_P{W.P}"
    # HBM bytes per launch measured by rocprofv3 counters for this kernel,
    # mode and workload; null unless taken from the current kernel sources
    tr = profdigest.read_traffic(os.path.join(
        ROOT, "profiles", f"{kname}_{mode}_{shape}_traffic.txt"))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if tr is None else round(tr[0]),
                "kernel": kname, "bytes_per_launch": sweep_bytes,
                "ms_per_launch": round(ms_sweep, 5)}
    compare = {}
    if not args.no_compare:
        for m in ("f64", "f32_wide"):
            if m != mode:
                compare[m] = run(m, max(10, steps // 2), max(3, warmup // 2))
    cpu = None if args.no_cpu else W.cpu_baseline(args.cpu_seconds)
    rep = {
        "config": dict(W.config, mode=mode, refine_passes=W.passes,
                       layout="RHS-interleaved [M][N]",
                       buffer_sets=main_r["sets"], launch=main_r["launch"]),
        "value": main_r["unknowns_per_s"],
        "unit": "unknowns/s",
        "ms_per_step": main_r["ms_per_step"],
        "dtype": DTYPE[mode],
        "hbm_frac_path": round(main_r["path_gbs"] / HBM_PEAK_GBS, 4),
        "path_gbs": round(main_r["path_gbs"], 1),
        # every kernel of a step: algorithmic bytes (F read once, X written
        # once) over the whole step time
        "roofline_path": {"bound": "hbm", "achieved": round(main_r["path_gbs"], 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(main_r["path_gbs"] / HBM_PEAK_GBS, 4),
                          "bytes_per_step": main_r["path_bytes"],
                          "ms_per_step": round(main_r["ms_per_step"], 5)},
        "phases_ms": {"beta": round(main_r["ms_beta"], 5),
                      "interface": round(main_r["ms_iface"], 5),
                      "sweep": round(main_r["ms_sweep"], 5)},
        "warm_ms_per_step": main_r.get("warm_ms_per_step"),
        "ms_per_step_median": round(main_r["ms_step_median"], 5),
        "ms_per_step_min": round(main_r["ms_step_min"], 5),
        "r2_max": main_r["r2_max"],
        "eta_max": main_r["eta_max"],
        "prepare_ms": round(W.prepare_ms, 3),
        "roofline": roofline,
        "compare": compare,
        "cpu_baseline": cpu,
    }
    if "other_order" in main_r:
        rep["other_order"] = main_r["other_order"]
    modes = dict(compare)
    modes[mode] = main_r
    rep["equal_residual"] = equal_residual(modes)
    del W
    torch.cuda.empty_cache()
    return rep


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_0901_2859_amd import tdsolve as t
    from paper_0901_2859_amd import workloads as wl

    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    head_name = "adi" if args.workload == "suite" else args.workload
    head = workload_report(head_name, args, t, wl, torch, dev, args.mode, args.steps, args.warmup)
    nested = {}
    if args.workload == "suite":
        for name in ("batch", "poisson"):
            nested[name] = workload_report(name, args, t, wl, torch, dev, args.mode, args.steps,
                                           args.warmup)
    copy = None if args.no_compare else copy_bandwidth(torch, dev)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
    }
    out.update({k: v for k, v in head.items() if k not in ("value", "unit", "ms_per_step", "dtype")})
    out["copy"] = copy
    if nested:
        out["workloads"] = nested
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
