"""Benchmark of the direct N-body force path on one MI355X.

Workload: 131072-body equal-mass Plummer sphere (standard units), softening eps2 = 1e-6, every
source with its own time t_j = -2^-k (k uniform in 3..10) and seeded Taylor data so the predictor
does real work; 4th-order Hermite forces: acceleration, jerk, potential and nearest neighbour.

One step = one pass of the hot path on device-resident data: copy the N_i updated sources into
the library (copy kernel), select the prediction time, and compute forces on the N_i active sinks
(fused predictor + gravity kernel), results left in device memory.  The headline line is the
mixed-precision path with every sink active (N_i = N = 131072); the same run sweeps
N_i = 1, 2, 4, ..., N in FP64 and mixed precision.

Printed: one JSON line with the metric, the roofline of the gravity kernel (algorithmic flops,
42 per 4th-order interaction, over the kernel's HIP-event time, at the shader clock measured over
the timed region), the FP64 oracle's throughput on a bounded sample of host cores, the per-N_i
sweep, and compact legs of the other workloads (6th order with neighbour lists at N = 1048576,
4096 batched few-body systems, the adjoint at N = 65536).  Every timed result states its error
against the FP64 oracle on a seeded sample of its sinks (max, p99 and median relative error of
acc and pot, the condition-normalised jerk error, and the condition number at the worst sink).
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 131072
EPS2 = 1e-6
BS_EPS2 = 1e-6  # softening of the block time-step runs
# First step eta_start |a|/|j| (order 6: at most eta_start sqrt(|a|/|s|)), as eta4.  A larger
# value (0.03) gives some particles first steps long enough that the crude start (crackle zero)
# costs energy: 1.2e-7 after one time unit at N = 131072 (seed 7) against 5e-12 with 0.01.
BS_ETA_START = 0.01
FLOPS_4TH = 42  # algorithmic flops per 4th-order acc+jerk+pot interaction (FMA = 2, rsqrt = 1)
FLOPS_2ND = 20  # algorithmic flops per 2nd-order acc+pot interaction (3 dx, 6 R^2, 1 rsqrt, 3 powers, 6 acc, 1 pot)
PEAK_FP32 = 157.3  # TFLOP/s, MI355X FP32 vector
PEAK_FP64 = 78.6  # TFLOP/s, MI355X FP64 vector
BOUND = {"fp64": 1e-13, "mixed": 1e-6}  # max relative error on acc (and pot) against the oracle
CLOCK_GROUPS = 256  # workgroups of one clock sample (every XCD gets many)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_force_mixed_plummer131072_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1510_04068_amd", "csrc", f)
                  for f in ("nbx_kernels.hip", "nbx_internal.h", "nbx_predict.h", "nbx_bs_device.h")]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per gravity launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-sweep", action="store_true", help="skip the N_i sweep")
    ap.add_argument("--no-e2e", action="store_true",
                    help="skip the end-to-end host-path timing (transfers included) at five N_i")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--sweep-reps", type=int, default=20, help="minimum timed steps per sweep point")
    ap.add_argument("--oracle-sinks", type=int, default=4096,
                    help="largest oracle sample per sweep point (timing and errors; all sinks below it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the compact 6th-order (N=1048576), batched few-body and adjoint legs")
    ap.add_argument("--sweep-ni", type=str, default="", metavar="N,N,...",
                    help="time only these N_i in the sweep (default: 2^0 .. 2^17)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape tuner (nbx_tune) and its tuned N_i sweep")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device-to-device copy kernel of MIB MiB first (HBM counter calibration)")
    ap.add_argument("--batch", action="store_true",
                    help="(part of the default run) 4096 independent few-body Plummer systems (3..96 particles, "
                         "eps2=0, 4th order) in one persistent launch, default and autotuned lane mappings")
    ap.add_argument("--adjoint", action="store_true",
                    help="(part of the default run) the adjoint on a 65536-body Plummer sphere (eps2=1e-6): "
                         "forward forces, the vector-Jacobian product, and the gradient through 16 checkpointed "
                         "Hermite steps (dt=1/512)")
    ap.add_argument("--order2", action="store_true",
                    help="also time the 2nd-order (GRAPE-5) mode, acc+pot+NN, on the same N=131072 sources, "
                         "N_i in {1024, 16384, 131072}")
    ap.add_argument("--blockstep", type=str, default="", metavar="N,N,...",
                    help="also run the 6th-order block time-step Hermite integrator for one N-body time unit "
                         "(eta4=0.01, eta6=0.1, eps2=1e-6) on Plummer spheres of these sizes, FP64 and mixed")
    ap.add_argument("--blockstep-precisions", type=str, default="fp64,mixed", metavar="P,P,...",
                    help="precisions of the --blockstep / --blockstep4 runs: fp64, mixed and ds (double-single, "
                         "the paper's DS; about ten times the FP64 pair cost on this GPU)")
    ap.add_argument("--blockstep4", type=str, default="", metavar="N,N,...",
                    help="also run the 4th-order block time-step Hermite integrator (Aarseth criterion, eta4=0.01, "
                         "eps2=1e-6) for one N-body time unit on Plummer spheres of these sizes, FP64 and mixed")
    ap.add_argument("--order6", action="store_true",
                    help="6th-order leg at N_i in {1024, 65536, 1048576} (the default run times 1024 and 65536): "
                         "forces with neighbour lists on a 1048576-body Plummer/Salpeter cluster (eps2=1e-8, "
                         "h2=1e-4, at most 256 neighbours)")
    ap.add_argument("--order8", action="store_true",
                    help="also time 8th-order forces (acc, jerk, snap, crackle) on the --order6 workload")
    return ap.parse_args()


class Workload:
    def __init__(self, torch, nbx, ics, dev):
        self.torch, self.nbx = torch, nbx
        src = ics.make_sources(N, seed=2)
        self.src = src
        self.ics = ics
        import numpy as np

        T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        f64, i64, i32 = torch.float64, torch.int64, torch.int32
        self.d = dict(addr=T(np.arange(N), i32), id=T(src.ids, i64), m=T(src.m, f64), t=T(src.t, f64),
                      x=T(src.x, f64), v=T(src.v, f64), a=T(src.a, f64), jerk=T(src.jerk, f64))
        self.out = dict(acc=torch.empty((N, 3), dtype=f64, device=dev), jerk=torch.empty((N, 3), dtype=f64, device=dev),
                        pot=torch.empty(N, dtype=f64, device=dev), nn_id=torch.empty(N, dtype=i64, device=dev),
                        nn_r2=torch.empty(N, dtype=f64, device=dev))
        self.sets = {}
        self.np = np
        self.T = T

    def active(self, ni):
        """Sorted addresses of the first ni entries of the seeded permutation, plus the gathered
        per-source inputs of those addresses (the updated sources of this block step)."""
        if ni not in self.sets:
            np, T, torch = self.np, self.T, self.torch
            sel = self.ics.active_set(N, ni, seed=1002)
            s = self.src
            self.sets[ni] = dict(
                addr=T(sel, torch.int32), id=T(s.ids[sel], torch.int64), m=T(s.m[sel], torch.float64),
                t=T(s.t[sel], torch.float64), x=T(s.x[sel], torch.float64), v=T(s.v[sel], torch.float64),
                a=T(s.a[sel], torch.float64), jerk=T(s.jerk[sel], torch.float64))
        return self.sets[ni]


def _q(x):
    """Summary figure of an error array: 3 significant digits."""
    return float("%.3g" % x)


def err_stats(gpu, ref, bound, label_n=None):
    """Errors of GPU outputs against the oracle on the same sinks (reading of the error metric:
    per sink |q_gpu - q_ref| / |q_ref| for acc and pot, |d jerk| / sum_j |jerk_ij| for the jerk, and
    kappa = sum_j |a_ij| / |a| at the worst acc sink).  gpu and ref hold acc, pot and optionally
    jerk, snap [n][3]; ref also holds cond [n][>=2]."""
    acc_r = ref["acc"]
    den = np.linalg.norm(acc_r, axis=1)
    e_acc = np.linalg.norm(gpu["acc"] - acc_r, axis=1) / np.where(den > 0, den, 1.0)
    e_pot = np.abs(gpu["pot"] - ref["pot"]) / np.abs(ref["pot"])
    kappa = ref["cond"][:, 0] / np.where(den > 0, den, 1.0)
    worst = int(np.argmax(e_acc))
    over = e_acc > bound
    out = {"n": int(acc_r.shape[0]),
           "acc": {"max": _q(e_acc.max()), "p99": _q(np.quantile(e_acc, 0.99)), "median": _q(np.median(e_acc))},
           "pot": {"max": _q(e_pot.max()), "p99": _q(np.quantile(e_pot, 0.99)), "median": _q(np.median(e_pot))},
           "kappa_at_max_acc": _q(kappa[worst]), "bound": bound, "n_acc_above_bound": int(over.sum())}
    if over.any():
        out["min_kappa_above_bound"] = _q(kappa[over].min())
    for k, c in (("jerk", 1), ("snap", 2)):
        if gpu.get(k) is not None and ref.get(k) is not None:
            e = np.linalg.norm(gpu[k] - ref[k], axis=1) / np.where(ref["cond"][:, c] > 0, ref["cond"][:, c], 1.0)
            out[k + "_cond"] = {"max": _q(e.max()), "median": _q(np.median(e))}
    return out


def fetch(out, rows, keys=("acc", "jerk", "pot")):
    """Host copies of the given rows of device output tensors (a dict of [n][3] / [n] tensors)."""
    import torch

    idx = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=next(iter(out.values())).device)
    return {k: out[k].index_select(0, idx).cpu().numpy() for k in keys if out.get(k) is not None}


class Clock:
    """Mean shader clock over a region, per XCD, from two clock samples of the library (the
    cycle counter against the constant-rate counter)."""

    def __init__(self, torch, nbx, ctx, dev):
        self.torch, self.nbx, self.ctx = torch, nbx, ctx
        self.buf = [torch.zeros(3 * CLOCK_GROUPS, dtype=torch.int64, device=dev) for _ in range(2)]
        self.wall_khz, self.sclk_max_khz = nbx.nbx_clock_rates(ctx.ctx)

    def sample(self, k, stream):
        self.nbx.nbx_clock_sample(self.ctx.ctx, stream, CLOCK_GROUPS, self.buf[k])

    def result(self):
        a, b = (x.cpu().numpy().reshape(-1, 3) for x in self.buf)
        per = {}
        for xcd in sorted(set(a[:, 0].tolist()) & set(b[:, 0].tolist())):
            ca, cb = a[a[:, 0] == xcd], b[b[:, 0] == xcd]
            cyc = float(np.median(cb[:, 1]) - np.median(ca[:, 1]))
            wall = float(np.median(cb[:, 2]) - np.median(ca[:, 2]))
            if wall > 0:
                per[int(xcd)] = round(cyc / wall * self.wall_khz * 1e-3, 1)
        mhz = list(per.values())
        return {"mean_mhz": round(sum(mhz) / len(mhz), 1) if mhz else None, "per_xcd_mhz": per,
                "nominal_max_mhz": round(self.sclk_max_khz * 1e-3, 1),
                "method": "cycle counter / constant-rate counter (%d kHz), median over %d workgroups per "
                          "sample, samples just before and after the timed steps" % (self.wall_khz, CLOCK_GROUPS)}


def step(nbx, ctx, w, ni, stream, ev=None):
    """One pass of the hot path: copy the ni updated sources, predict, forces on the ni sinks."""
    a = w.active(ni)
    nbx.nbx_set_j_dev(ctx.ctx, stream, ni, a["addr"], a["id"], a["m"], a["t"], a["x"], a["v"], a["a"], a["jerk"])
    nbx.nbx_predict(ctx.ctx, 0.0)
    if ev is not None:
        ev[0].record(stream)
    o = w.out
    nbx.nbx_force_dev(ctx.ctx, stream, ni, a["addr"], EPS2, None, o["acc"], o["jerk"], None, o["pot"], o["nn_id"],
                      o["nn_r2"])
    if ev is not None:
        ev[1].record(stream)


def timed(torch, nbx, ctx, w, ni, stream, steps, warmup, times=None, flush=None, clock=None):
    """Returns (seconds per step, mean force-kernel seconds per launch); `times` (a list) receives
    every launch's seconds.  With `flush` (a large device tensor) each step first overwrites it,
    which evicts the sources from L2 and the MALL, so the launch reads them from HBM.  With `clock`
    (a Clock) a clock sample runs just before and just after the timed steps."""
    for _ in range(warmup):
        step(nbx, ctx, w, ni, stream)
    if clock is not None:
        clock.sample(0, stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        if flush is not None:
            flush.fill_(float(k))
        step(nbx, ctx, w, ni, stream, evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if clock is not None:
        clock.sample(1, stream)
        torch.cuda.synchronize()
    ks = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    if times is not None:
        times.extend(ks)
    return (t1 - t0) / steps, sum(ks) / steps


def launch_floor(torch, stream, reps=200):
    """Median time of two dependent minimal kernels on the stream, HIP events around them: the
    floor under a force launch (gravity kernel + combine kernel) that does no work."""
    x = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(10):
        x.add_(1.0)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        x.add_(1.0)
        x.add_(1.0)
        e1.record(stream)
        ts.append((e0, e1))
    torch.cuda.synchronize()
    us = sorted(a.elapsed_time(b) * 1e3 for a, b in ts)
    return us[len(us) // 2]


def timed_sweep(torch, nbx, ctx, w, ni, stream, min_reps, budget_s=0.02, times=None):
    """timed() for one sweep point: warm up for ~budget/4 (at least 2 steps) so that the clocks have
    settled after the previous point, then time enough steps for ~budget of force-kernel time."""
    _, k = timed(torch, nbx, ctx, w, ni, stream, 2, 1)
    warm = max(0, int(0.25 * budget_s / k) - 3)
    reps = max(min_reps, min(400, int(budget_s / k)))
    return timed(torch, nbx, ctx, w, ni, stream, reps, warm, times=times)


def end_to_end(nbx, ics, src, prec, ni_list, reps):
    """The host-pointer path with its transfers (the scope of the paper's timings that include
    PCIe): per step nbx_set_j of the ni updated sources from host arrays, nbx_predict, nbx_force
    with host sink addresses, nbx_get_force back to host arrays; wall time per step."""
    import numpy as np

    rows = []
    with nbx.Context(order=4, precision=prec, nj_max=N, ni_max=N) as ctx:
        ctx.set_sources(src)
        for ni in ni_list:
            sel = ics.active_set(N, ni, seed=1002)
            arrs = [np.ascontiguousarray(a[sel]) for a in (src.ids, src.m, src.t, src.x, src.v, src.a, src.jerk)]

            def go():
                nbx.nbx_set_j(ctx.ctx, sel, *arrs)
                nbx.nbx_predict(ctx.ctx, 0.0)
                nbx.nbx_force(ctx.ctx, sel, EPS2)
                return nbx.nbx_get_force(ctx.ctx, ni)

            for _ in range(3):
                go()
            n_rep = max(3, min(reps, int(0.2 / max(1e-6, 1e-9 * ni * N))))
            t0 = time.perf_counter()
            for _ in range(n_rep):
                go()
            dt = (time.perf_counter() - t0) / n_rep
            rows.append({"ni": ni, "ms": round(dt * 1e3, 4), "int_s": float("%.4g" % (ni * float(N) / dt))})
    return rows



ORACLE_THREADS = [0]  # host threads of the oracle runs (all cores), taken before any one-thread run


def oracle_run(src, sel, nthreads=None):
    """The FP64 oracle as it stands: predict every source to t = 0, then acc/jerk/pot/NN of the
    sinks sel (addresses) against all sources.  Returns (seconds, outputs)."""
    import oracle

    if nthreads is None:
        nthreads = ORACLE_THREADS[0]
    t0 = time.perf_counter()
    xq, vq, _ = oracle.predict(4, 0.0, src.t, src.x, src.v, src.a, src.jerk)
    ref = oracle.force(4, EPS2, src.ids, src.m, xq, vq, src.ids[sel], xq[sel], vq[sel], nthreads=nthreads)
    return time.perf_counter() - t0, ref


def cpu_baseline(src, seconds):
    """FP64 oracle (predict all sources + forces on a sample of sinks) on the host cores.  Returns
    the baseline record plus the sample's addresses and oracle outputs (the reference of the
    headline launch's error)."""
    import oracle

    oracle.build(force_rebuild=False)
    rng = np.random.Generator(np.random.PCG64(7))

    def run(ns, nthreads=0):
        sel = np.sort(rng.choice(N, size=ns, replace=False))
        dt, ref = oracle_run(src, sel, nthreads)
        return dt, sel, ref

    cores = ORACLE_THREADS[0] or oracle.max_threads()
    probe = 256
    dt, _, _ = run(probe)
    ns = int(min(N, max(probe, probe * seconds / max(dt, 1e-6))))
    dt, sel_main, ref_main = run(ns)
    # one thread, on a sample a fifth as long (the oracle keeps the thread count it was last given,
    # so this runs last)
    ns1 = max(16, int(ns / max(cores, 1) / 5))
    dt1, _, _ = run(ns1, nthreads=1)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    rec = {"value": ns * N / dt, "unit": "interactions/s", "cores": cores, "kind": "oracle",
           "host": {"cpu": model, "nproc": os.cpu_count()},
           "sample": "FP64 oracle, predictor on all %d sources + acc/jerk/pot/NN of %d seeded random sinks "
                     "against all %d sources (%.2e interactions, %.1f s)" % (N, ns, N, ns * float(N), dt),
           "single_thread": {"value": ns1 * N / dt1, "cores": 1,
                             "sample": "same, %d sinks (%.2e interactions, %.1f s)" % (ns1, ns1 * float(N), dt1)}}
    return rec, sel_main, ref_main


def oracle_sweep(src, sweep, gpu_rows, cap):
    """Per sweep point: the oracle timed on the point's own sinks (all of them up to `cap`, else a
    seeded sample of `cap`), and the errors of every timed GPU variant of the point on those sinks.
    gpu_rows[ni][variant] holds the GPU outputs for the sample positions."""
    for row in sweep:
        ni = row["ni"]
        pos = sample_positions(ni, cap)
        sel = nbody_ics_active(ni)[pos]
        dt, ref = oracle_run(src, sel)
        row["oracle_sinks"] = int(len(pos))
        row["oracle_int_s"] = float("%.4g" % (len(pos) * float(N) / dt))
        row["oracle_s_per_step"] = float("%.4g" % (dt * ni / len(pos)))
        row["oracle_scope"] = ("predictor on all sources + the %s sinks" %
                               ("%d" % ni if len(pos) == ni else "seeded sample of %d of the %d" % (len(pos), ni)))
        errs = {}
        for name, out in gpu_rows.get(ni, {}).items():
            errs[name] = err_stats(out, ref, BOUND["fp64" if name.startswith("fp64") else "mixed"])
        row["err"] = errs
        print("bench: oracle ni=%d sinks=%d %.3g int/s errs %s" % (
            ni, len(pos), row["oracle_int_s"],
            " ".join("%s:%.2e" % (k, v["acc"]["max"]) for k, v in errs.items())), file=sys.stderr, flush=True)


def same_state_check(torch, nbx, w, dev, stream, n_check=16384):
    """The force kernels on the headline sources with every t_j = 0 predicted to t = 0 (the
    predictor is then the identity on both sides, so GPU and oracle see bit-identical positions and
    velocities): all N sinks active, errors on n_check seeded sinks.  This isolates the force
    arithmetic from the last-bit differences of two independent FP64 predictors."""
    src = w.src
    sel = np.sort(np.random.Generator(np.random.PCG64(8)).choice(N, size=n_check, replace=False))
    import oracle

    ref = oracle.force(4, EPS2, src.ids, src.m, src.x, src.v, src.ids[sel], src.x[sel], src.v[sel],
                       nthreads=ORACLE_THREADS[0])
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    f64 = torch.float64
    res = {"scope": "headline sources with t_j = 0 at t = 0 (identical inputs on both sides), N_i = N, %d "
                    "seeded sinks" % n_check}
    with nbx.Context(order=4, precision=nbx.NBX_FP64, nj_max=N, ni_max=N) as c:
        d = w.d
        nbx.nbx_set_j_dev(c.ctx, stream, N, d["addr"], d["id"], d["m"], T(np.zeros(N), f64), d["x"], d["v"],
                          d["a"], d["jerk"])
        nbx.nbx_set_nj(c.ctx, N)
        nbx.nbx_predict(c.ctx, 0.0)
        for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
            c.set_precision(prec)
            o = w.out
            nbx.nbx_force_dev(c.ctx, stream, N, d["addr"], EPS2, None, o["acc"], o["jerk"], None, o["pot"],
                              o["nn_id"], o["nn_r2"])
            nbx.nbx_sync(c.ctx, stream)
            res[name] = err_stats(fetch(o, sel), ref, BOUND[name])
    print("bench: same-state errors %s" % json.dumps(res), file=sys.stderr, flush=True)
    return res


def sample_positions(ni, cap):
    """Positions (rows of the output) of the sweep point's oracle sample: all below cap."""
    if ni <= cap:
        return np.arange(ni)
    rng = np.random.Generator(np.random.PCG64(4000 + ni))
    return np.sort(rng.choice(ni, size=cap, replace=False))


def nbody_ics_active(ni):
    import nbody_ics

    return nbody_ics.active_set(N, ni, seed=1002)


def order6(torch, nbx, ics, dev, steps, order=6, ni_list=(1024, 65536, 1 << 20), n_check=64):
    """Config-3 points: 6th (or 8th) order, Salpeter masses, neighbour lists; kernel time per
    precision, and each precision's error against the oracle on n_check seeded sinks of every
    active set."""
    import oracle

    n, eps2, h2, nbr_max = 1 << 20, 1e-8, 1e-4, 256
    flops = 128 if order == 8 else 79
    src = ics.make_sources(n, seed=3, order=order, masses="salpeter")
    stream = torch.cuda.current_stream()
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    ctx = nbx.Context(order=order, precision=nbx.NBX_MIXED, nj_max=n, ni_max=n, nbr_max=nbr_max)
    nbx.nbx_set_j_dev(ctx.ctx, stream, n, T(np.arange(n), i32), T(src.ids, i64), T(src.m, f64), T(src.t, f64),
                      T(src.x, f64), T(src.v, f64), T(src.a, f64), T(src.jerk, f64), T(src.snap, f64),
                      T(src.crackle, f64))
    nbx.nbx_set_nj(ctx.ctx, n)
    nbx.nbx_predict(ctx.ctx, 0.0)
    out = [torch.empty((n, 3), dtype=f64, device=dev) for _ in range(4 if order == 8 else 3)]
    pot, nnr2 = torch.empty(n, dtype=f64, device=dev), torch.empty(n, dtype=f64, device=dev)
    nnid, cnt = torch.empty(n, dtype=i64, device=dev), torch.empty(n, dtype=i32, device=dev)
    ids = torch.empty((n, nbr_max), dtype=i64, device=dev)
    d_h2 = torch.full((n,), h2, dtype=f64, device=dev)
    xp, vp, ap = oracle.predict(order, 0.0, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    jp = oracle.predict_jerk(0.0, src.t, src.jerk, src.snap, src.crackle) if order == 8 else None
    rows = []
    for ni in ni_list:
        sel_h = ics.active_set(n, ni, seed=1003)
        sel = T(sel_h, i32)
        pos = np.sort(np.random.Generator(np.random.PCG64(5000 + ni)).choice(ni, size=min(ni, n_check),
                                                                             replace=False))
        ca = sel_h[pos]
        if order == 8:
            ref = oracle.force8(eps2, src.ids, src.m, xp, vp, ap, jp, src.ids[ca], xp[ca], vp[ca], ap[ca], jp[ca])
        else:
            ref = oracle.force(6, eps2, src.ids, src.m, xp, vp, src.ids[ca], xp[ca], vp[ca], aj=ap, ai=ap[ca])
        row = {"ni": ni}
        for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
            ctx.set_precision(prec)
            reps = 1 if ni == n else steps

            def go():
                if order == 8:
                    nbx.nbx_force8_dev(ctx.ctx, stream, ni, sel, eps2, d_h2, out[0], out[1], out[2], out[3], pot,
                                       nnid, nnr2, cnt, ids)
                else:
                    nbx.nbx_force_dev(ctx.ctx, stream, ni, sel, eps2, d_h2, out[0], out[1], out[2], pot, nnid,
                                      nnr2, cnt, ids)

            go()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                go()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row[name + "_kernel_ms"] = round(ms, 4)
            row[name + "_int_s"] = float("%.4g" % (ni * float(n) / (ms * 1e-3)))
            peak = PEAK_FP64 if prec == nbx.NBX_FP64 else PEAK_FP32
            row[name + "_roofline_frac"] = round(flops * ni * float(n) / (ms * 1e-3) / 1e12 / peak, 4)
            got = fetch({"acc": out[0], "jerk": out[1], "snap": out[2], "pot": pot}, pos,
                        ("acc", "jerk", "snap", "pot"))
            row[name + "_err"] = err_stats(got, ref, BOUND[name])
        row["speedup"] = round(row["fp64_kernel_ms"] / row["mixed_kernel_ms"], 3)
        row["mean_neighbours"] = round(float(cnt[:ni].double().mean().item()), 3)
        rows.append(row)
        print("bench: order%d %s" % (order, json.dumps(row)), file=sys.stderr, flush=True)
    status = nbx.nbx_sync(ctx.ctx, stream)
    ctx.close()
    what = "8th-order acc+jerk+snap+crackle" if order == 8 else "6th-order acc+jerk+snap"
    return {"workload": "Plummer N=1048576, Salpeter masses (slope -2.35, 0.1-100, total 1), eps2=1e-8, "
                        "%s+pot+NN+neighbour lists (h2=1e-4, max 256)" % what,
            "flops_per_interaction": flops, "rows": rows, "list_status": status,
            "err_sample": "%d seeded sinks of each active set against the FP64 oracle" % n_check}


def order2(torch, nbx, ics, dev, steps):
    """2nd-order (GRAPE-5) mode on the headline sources: acc + pot + NN; kernel time per precision."""
    import numpy as np

    src = ics.make_sources(N, seed=2)
    stream = torch.cuda.current_stream()
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    ctx = nbx.Context(order=2, precision=nbx.NBX_MIXED, nj_max=N, ni_max=N)
    nbx.nbx_set_j_dev(ctx.ctx, stream, N, T(np.arange(N), i32), T(src.ids, i64), T(src.m, f64), T(src.t, f64),
                      T(src.x, f64), T(src.v, f64), T(src.a, f64), None)
    nbx.nbx_set_nj(ctx.ctx, N)
    nbx.nbx_predict(ctx.ctx, 0.0)
    acc = torch.empty((N, 3), dtype=f64, device=dev)
    pot, nnr2 = torch.empty(N, dtype=f64, device=dev), torch.empty(N, dtype=f64, device=dev)
    nnid = torch.empty(N, dtype=i64, device=dev)
    rows = []
    for ni in (1024, 16384, N):
        sel = T(ics.active_set(N, ni, seed=1002), i32)
        sh = ctx.launch_shape(ni)
        row = {"ni": ni, "shape": "L%d P%d S%d wg%d" % (sh["lanes_per_sink"], sh["sinks_per_lane"], sh["splits"],
                                                      sh["workgroups"])}
        for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
            ctx.set_precision(prec)

            def go():
                nbx.nbx_force_dev(ctx.ctx, stream, ni, sel, EPS2, None, acc, None, None, pot, nnid, nnr2)

            go()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                go()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[name + "_kernel_ms"] = round(ms, 4)
            row[name + "_int_s"] = float("%.4g" % (ni * float(N) / (ms * 1e-3)))
            peak = PEAK_FP32 if prec == nbx.NBX_MIXED else PEAK_FP64
            row[name + "_roofline_frac"] = round(FLOPS_2ND * ni * float(N) / (ms * 1e-3) / 1e12 / peak, 4)
        row["speedup"] = round(row["fp64_kernel_ms"] / row["mixed_kernel_ms"], 3)
        rows.append(row)
        print("bench: order2 %s" % json.dumps(row), file=sys.stderr, flush=True)
    nbx.nbx_sync(ctx.ctx, stream)
    ctx.close()
    return {"workload": "Plummer N=131072 (seed 2), eps2=1e-6, per-source times, 2nd-order (GRAPE-5) acc+pot+NN",
            "flops_per_interaction": FLOPS_2ND, "rows": rows}


def blockstep(torch, nbx, ics, sizes, tune=True, order=6, precisions=("fp64", "mixed")):
    """Block time-step runs (6th order by default; 4th order with the Aarseth criterion), one N-body
    time unit, in the given precisions (fp64: the paper's DP; ds: its double-single DS; mixed: this
    library's FP32 pair arithmetic): wall time from the start to the end of the integration,
    energy error, block steps and mean N_active."""
    codes = {"fp64": nbx.NBX_FP64, "mixed": nbx.NBX_MIXED, "ds": nbx.NBX_DS}
    rows = []
    for n in sizes:
        m, x, v = ics.plummer(n, seed=7)
        for name in precisions:
            prec = codes[name]
            ctx = nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nbx.nbx_bs_init(ctx.ctx, np.arange(n), m, x, v, BS_EPS2, eta4=0.01, eta6=0.1, eta_start=BS_ETA_START)
            e0 = sum(nbx.nbx_bs_energy(ctx.ctx))
            tt = time.perf_counter()
            if tune:  # launch shapes per N_i class for these sources (setup, not part of the run)
                ctx.tune(n)
                print("bench: blockstep order %d n=%d %s shapes tuned in %.1f s" % (
                    order, n, name, time.perf_counter() - tt), file=sys.stderr, flush=True)
            t1 = time.perf_counter()
            parts = 16 if n >= 262144 else 8  # one time unit in parts, with a progress line each
            for k in range(1, parts + 1):
                st = nbx.nbx_bs_run(ctx.ctx, k / float(parts))
                print("bench: blockstep order %d n=%d %s t=%g blocks=%d status=%d" % (
                    order, n, name, st["t"], st["block_steps"], st["status"]), file=sys.stderr, flush=True)
                if st["status"] != nbx.NBX_OK:
                    break
            t2 = time.perf_counter()
            e1 = sum(nbx.nbx_bs_energy(ctx.ctx))
            ctx.close()
            row = {"n": n, "precision": name, "init_s": round(tt - t0, 4), "tune_s": round(t1 - tt, 3),
                   "run_s": round(t2 - t1, 4),
                   "block_steps": st["block_steps"], "particle_steps": st["particle_steps"],
                   "mean_n_active": round(st["particle_steps"] / max(st["block_steps"], 1), 2),
                   "energy_error": float("%.3e" % abs((e1 - e0) / e0)), "status": st["status"],
                   "interactions_per_s": float("%.4g" % (st["particle_steps"] * float(n) / (t2 - t1)))}
            rows.append(row)
            print("bench: blockstep %s" % json.dumps(row), file=sys.stderr, flush=True)
    crit = ("averaged Aarseth/6th-order criterion eta4=0.01 eta6=0.1" if order == 6 else
            "Aarseth criterion eta4=0.01")
    return {"workload": "Plummer spheres (seed 7), %s-order Hermite block time steps, %s, first step %g |a|/|j|, "
                        "eps2=%g, dt_max=1/8, one N-body time unit" % ("6th" if order == 6 else "4th", crit,
                                                                      BS_ETA_START, BS_EPS2),
            "rows": rows}


def batch(torch, nbx, ics, dev, steps):
    """Batched few-body systems: one persistent launch; FP64 and mixed; default and tuned L; every
    particle's error against the oracle (each system on its own)."""
    import oracle

    n_sys, eps2 = 4096, 0.0
    sizes = ics.few_body_sizes(n_sys, 4)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    parts = [ics.plummer(int(n), seed=10000 + s) for s, n in enumerate(sizes)]
    ref = {"acc": [], "jerk": [], "pot": [], "cond": []}
    for mm, xx, vv in parts:
        ids = np.arange(len(mm), dtype=np.int64)
        r = oracle.force(4, eps2, ids, mm, xx, vv, ids, xx, vv)
        for k in ref:
            ref[k].append(r[k])
    ref = {k: np.concatenate(v) for k, v in ref.items()}
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    m = T(np.concatenate([p[0] for p in parts]))
    x, v = T(np.concatenate([p[1] for p in parts])), T(np.concatenate([p[2] for p in parts]))
    n = int(off[-1])
    acc, jrk = torch.empty((n, 3), dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    inter = float(np.sum(sizes.astype(np.float64) ** 2))
    stream = torch.cuda.current_stream()
    res = {"workload": "4096 Plummer systems, N uniform in [3,96] (seed 4), eps2=0, 4th-order acc+jerk+pot, one "
                       "persistent launch", "interactions": inter, "particles": n}
    for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
        ctx = nbx.Context(order=4, precision=prec, nj_max=1, ni_max=1)
        nbx.nbx_batch_setup(ctx.ctx, off)
        for tuned in (False, True):
            if tuned:
                lanes = nbx.nbx_batch_tune(ctx.ctx, stream, m, x, v, eps2, acc, jrk, pot)
                res[name + "_lanes_per_class"] = [int(l) for l in lanes]
            for _ in range(3):
                nbx.nbx_batch_force_dev(ctx.ctx, stream, m, x, v, eps2, acc, jrk, pot)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                nbx.nbx_batch_force_dev(ctx.ctx, stream, m, x, v, eps2, acc, jrk, pot)
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / steps * 1e3
            key = name + ("_tuned" if tuned else "_default")
            res[key + "_us"] = round(us, 3)
            res[key + "_int_s"] = float("%.4g" % (inter / (us * 1e-6)))
            got = {"acc": acc.cpu().numpy(), "jerk": jrk.cpu().numpy(), "pot": pot.cpu().numpy()}
            res[key + "_err"] = err_stats(got, ref, BOUND[name])
        ctx.close()
    print("bench: batch %s" % json.dumps(res), file=sys.stderr, flush=True)
    return res


def adjoint(torch, nbx, ics, dev, steps, n_check=128):
    """Config-5 timings: forward, adjoint kernel, and a 16-step checkpointed Hermite gradient; the
    forward and the adjoint's errors against the oracle on n_check seeded particles (adjoint: the
    gradient error per particle over the largest reference gradient of the sample)."""
    import oracle

    from paper_1510_04068_amd.autograd import ForceContext, forces, hermite4

    n, eps2 = 65536, 1e-6
    src = ics.make_sources(n, seed=5)
    rng = np.random.default_rng(5005)
    wa_h, wj_h = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    wa, wj = T(wa_h), T(wj_h)
    stream = torch.cuda.current_stream()
    sel = np.sort(np.random.Generator(np.random.PCG64(5006)).choice(n, n_check, replace=False)).astype(np.int32)
    ref_f = oracle.force(4, eps2, src.ids, src.m, src.x, src.v, src.ids[sel], src.x[sel], src.v[sel])
    ref_g = oracle.force_vjp(eps2, src.m, src.x, src.v, wa_h, wj_h, 0.5 * src.m, sel=sel)
    res = {"workload": "Plummer N=65536, eps2=1e-6, loss = seeded weights . (acc, jerk) + total potential energy; "
                       "16 checkpointed 4th-order Hermite steps, dt=1/512", "n": n,
           "err_sample": "%d seeded particles against the FP64 oracle (forward: per-sink relative error; "
                         "adjoint: |g - g_ref| / max |g_ref| over the sample)" % n_check}
    for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
        fc = ForceContext(n, precision=prec)
        x, v, m = T(src.x), T(src.v), T(src.m)

        def ev_time(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        g = [torch.empty((n, 3), dtype=torch.float64, device=dev) for _ in range(2)] + [torch.empty(n, dtype=torch.float64, device=dev)]
        gp = 0.5 * m
        res[name + "_forward_ms"] = round(ev_time(lambda: forces(x, v, m, eps2, fc), steps), 4)
        res[name + "_vjp_ms"] = round(ev_time(lambda: nbx.nbx_force_vjp_dev(fc.ctx.ctx, stream, n, m, x, v, eps2, wa, wj, gp,
                                                                           g[0], g[1], g[2]), steps), 4)
        acc_f, jrk_f, pot_f = forces(x, v, m, eps2, fc)
        torch.cuda.synchronize()
        res[name + "_forward_err"] = err_stats(fetch({"acc": acc_f, "jerk": jrk_f, "pot": pot_f}, sel), ref_f,
                                               BOUND[name])
        ge = {}
        for k, (gd, gr) in zip(("x", "v", "m"), zip(g, ref_g)):
            d = gd.index_select(0, torch.as_tensor(sel.astype(np.int64), device=dev)).cpu().numpy() - gr
            e = (np.linalg.norm(d, axis=1) if d.ndim == 2 else np.abs(d)) / np.abs(gr).max()
            ge[k] = _q(e.max())
        res[name + "_vjp_err_max"] = ge

        def traj():
            xx, vv, mm = x.clone().requires_grad_(), v.clone().requires_grad_(), m.clone().requires_grad_()
            x1, v1 = hermite4(xx, vv, mm, eps2, 1.0 / 512, 16, fc, checkpoint=True)
            ((wa * x1).sum() + (wj * v1).sum()).backward()

        res[name + "_hermite16_grad_ms"] = round(ev_time(traj, 1), 3)
        res[name + "_vjp_pairs_s"] = float("%.4g" % (float(n) * n / (res[name + "_vjp_ms"] * 1e-3)))
        fc.close()
    print("bench: adjoint %s" % json.dumps(res), file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: nbx runs on one GPU only (the source-sharded multi-GPU design is described in the "
              "documentation, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import nbody_ics
    import paper_1510_04068_amd as nbx

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        evict = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB: pushes a out of the 256 MB MALL
        del evict
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("bench: copy calibration read %d B, wrote %d B" % (nbytes, nbytes), file=sys.stderr, flush=True)
        del a, b
    import oracle

    oracle.build(force_rebuild=False)
    ORACLE_THREADS[0] = oracle.max_threads()
    w = Workload(torch, nbx, nbody_ics, dev)
    ctx = nbx.Context(order=4, precision=nbx.NBX_MIXED, nj_max=N, ni_max=N)
    d = w.d
    nbx.nbx_set_j_dev(ctx.ctx, stream, N, d["addr"], d["id"], d["m"], d["t"], d["x"], d["v"], d["a"], d["jerk"])
    nbx.nbx_set_nj(ctx.ctx, N)
    nbx.nbx_sync(ctx.ctx, stream)

    # headline: mixed precision, every sink active; the shader clock is sampled around the timed steps
    clock = Clock(torch, nbx, ctx, dev)
    ctx.set_precision(nbx.NBX_MIXED)
    print("bench: mixed N_i=N warmup=%d steps=%d" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    head_times = []
    sec, kern = timed(torch, nbx, ctx, w, N, stream, args.steps, args.warmup, times=head_times, clock=clock)
    nbx.nbx_sync(ctx.ctx, stream)
    sclk = clock.result()
    print("bench: clock %s" % json.dumps(sclk), file=sys.stderr, flush=True)
    inter = float(N) * N
    value = inter / sec
    achieved = FLOPS_4TH * inter / kern / 1e12
    shape = ctx.launch_shape(N)
    # outputs of the last timed step (row q = address q at N_i = N), kept for the error check
    head_out = {"mixed": {k: w.out[k].cpu().numpy() for k in ("acc", "jerk", "pot")}}

    # FP64 at the same point
    ctx.set_precision(nbx.NBX_FP64)
    print("bench: fp64 N_i=N", file=sys.stderr, flush=True)
    sec64, kern64 = timed(torch, nbx, ctx, w, N, stream, max(20, args.steps), 1)
    head_out["fp64"] = {k: w.out[k].cpu().numpy() for k in ("acc", "jerk", "pot")}
    same_state = same_state_check(torch, nbx, w, dev, stream)
    gpu_rows = {}  # sweep outputs at the oracle sample positions: gpu_rows[ni][variant]

    def shape_str(cx, ni):
        sh = cx.launch_shape(ni)
        return "L%d P%d S%d wg%d" % (sh["lanes_per_sink"], sh["sinks_per_lane"], sh["splits"], sh["workgroups"])

    def time_row(cx, row, ni, suffix):
        for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
            cx.set_precision(prec)
            row[name + suffix + "_shape"] = shape_str(cx, ni)
            ts = []
            s, k = timed_sweep(torch, nbx, cx, w, ni, stream, args.sweep_reps, times=ts)
            gpu_rows.setdefault(ni, {})[name + suffix] = fetch(w.out, sample_positions(ni, args.oracle_sinks))
            row[name + suffix + "_kernel_ms"] = round(k * 1e3, 5)
            if not suffix:
                ts.sort()
                row[name + "_kernel_ms_median"] = round(ts[len(ts) // 2] * 1e3, 5)
                row[name + "_kernel_ms_min"] = round(ts[0] * 1e3, 5)
                row[name + "_reps"] = len(ts)
                row[name + "_step_ms"] = round(s * 1e3, 5)
            row[name + suffix + "_int_s"] = float("%.4g" % (ni * float(N) / k))
        row[suffix.lstrip("_") + ("_" if suffix else "") + "speedup"] = round(
            row["fp64" + suffix + "_kernel_ms"] / row["mixed" + suffix + "_kernel_ms"], 3)

    sweep, tune_s = [], None
    if not args.no_sweep:
        # a second context on the same sources gets the library's tuner (a shape per N_i class from
        # timed candidates); each N_i is then timed with the static rule and the tuned shapes back to
        # back, so that clock drift over the sweep does not bias the comparison
        ctx_t = None
        if not args.no_tune:
            ctx_t = nbx.Context(order=4, precision=nbx.NBX_MIXED, nj_max=N, ni_max=N)
            nbx.nbx_set_j_dev(ctx_t.ctx, stream, N, d["addr"], d["id"], d["m"], d["t"], d["x"], d["v"], d["a"],
                              d["jerk"])
            nbx.nbx_set_nj(ctx_t.ctx, N)
            t0 = time.perf_counter()
            nbx.nbx_predict(ctx_t.ctx, 0.0)
            for prec in (nbx.NBX_MIXED, nbx.NBX_FP64):
                ctx_t.set_precision(prec)
                ctx_t.tune(N)
            nbx.nbx_sync(ctx_t.ctx, stream)
            tune_s = time.perf_counter() - t0
            print("bench: tuned launch shapes in %.1f s" % tune_s, file=sys.stderr, flush=True)
        sweep_ni = [int(k) for k in args.sweep_ni.split(",")] if args.sweep_ni else [1 << e for e in range(18)]
        floor_us = launch_floor(torch, stream)
        print("bench: launch floor (two dependent empty-work kernels) %.2f us" % floor_us, file=sys.stderr,
              flush=True)
        for ni in sweep_ni:
            row = {"ni": ni}
            time_row(ctx, row, ni, "")
            if ctx_t is not None:
                time_row(ctx_t, row, ni, "_tuned")
            for name in ("fp64", "mixed"):
                row[name + "_above_floor_us"] = round(row[name + "_kernel_ms_median"] * 1e3 - floor_us, 3)
            sweep.append(row)
            print("bench: sweep %s" % json.dumps(row), file=sys.stderr, flush=True)
        if ctx_t is not None:
            nbx.nbx_sync(ctx_t.ctx, stream)
            ctx_t.close()
        # the sweep runs with the sources warm in L2 / the 256 MB MALL; small N_i read them from
        # HBM when a 512 MiB write precedes every launch
        flush = torch.empty(1 << 26, dtype=torch.float64, device=dev)
        for row in sweep:
            if row["ni"] not in (1, 64, 1024):
                continue
            for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
                ctx.set_precision(prec)
                ts = []
                timed(torch, nbx, ctx, w, row["ni"], stream, 50, 5, times=ts, flush=flush)
                ts.sort()
                row[name + "_flushed_kernel_ms_median"] = round(ts[len(ts) // 2] * 1e3, 5)
            print("bench: flushed %s" % json.dumps({k: v for k, v in row.items() if "flushed" in k or k == "ni"}),
                  file=sys.stderr, flush=True)
        del flush
    nbx.nbx_sync(ctx.ctx, stream)
    ctx.close()

    e2e = None
    if not args.no_e2e:
        e2e = {"scope": "host arrays: nbx_set_j of the N_i updated sources, nbx_predict, nbx_force with host "
                        "sink addresses, nbx_get_force to host arrays; wall time per step", "rows": {}}
        for prec, name in ((nbx.NBX_FP64, "fp64"), (nbx.NBX_MIXED, "mixed")):
            e2e["rows"][name] = end_to_end(nbx, nbody_ics, w.src, prec, (1, 64, 1024, 16384, N), 50)
            print("bench: end-to-end %s %s" % (name, json.dumps(e2e["rows"][name])), file=sys.stderr, flush=True)

    o2 = order2(torch, nbx, nbody_ics, dev, max(3, args.steps // 2)) if args.order2 else None
    bs_prec = tuple(args.blockstep_precisions.split(","))
    bsr = (blockstep(torch, nbx, nbody_ics, [int(k) for k in args.blockstep.split(",")], tune=not args.no_tune,
                     precisions=bs_prec) if args.blockstep else None)
    bs4 = (blockstep(torch, nbx, nbody_ics, [int(k) for k in args.blockstep4.split(",")], tune=not args.no_tune,
                     order=4, precisions=bs_prec) if args.blockstep4 else None)
    extras = not args.no_extras
    o6 = (order6(torch, nbx, nbody_ics, dev, max(2, args.steps // 10),
                 ni_list=(1024, 65536, 1 << 20) if args.order6 else (1024, 65536))
          if (args.order6 or extras) else None)
    o8 = order6(torch, nbx, nbody_ics, dev, max(2, args.steps // 10), order=8) if args.order8 else None
    bt = batch(torch, nbx, nbody_ics, dev, max(20, args.steps)) if (args.batch or extras) else None
    adj = adjoint(torch, nbx, nbody_ics, dev, max(3, args.steps // 5)) if (args.adjoint or extras) else None

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu, sel_main, ref_main = cpu_baseline(w.src, args.cpu_seconds)
        err_scope = "the cpu_baseline sample: %d seeded sinks" % len(sel_main)
    else:
        import oracle

        sel_main = np.sort(np.random.Generator(np.random.PCG64(7)).choice(N, size=2048, replace=False))
        ref_main = oracle_run(w.src, sel_main)[1]
        err_scope = "2048 seeded sinks"
    head_err = {name: err_stats({k: v[sel_main] for k, v in head_out[name].items()}, ref_main, BOUND[name])
                for name in ("mixed", "fp64")}
    head_err["scope"] = ("outputs of the last timed N_i=N launch of each precision against the FP64 oracle on " +
                         err_scope + "; end to end, so each side predicts the sources with its own FP64 "
                         "predictor, whose last-bit differences close pairs amplify (see same_state)")
    head_err["same_state"] = same_state
    print("bench: headline errors %s" % json.dumps(head_err), file=sys.stderr, flush=True)
    if sweep:
        print("bench: oracle per sweep point", file=sys.stderr, flush=True)
        oracle_sweep(w.src, sweep, gpu_rows, args.oracle_sinks)

    line = {
        "metric": "interactions/s (acc+jerk+pot) vs active N_i at N=128k, mixed vs FP64",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "Plummer sphere N=131072, eps2=1e-6, per-source times, 4th-order acc+jerk+pot+nearest "
                        "neighbour, all sinks active (N_i=N), mixed precision (FP64 predictor, double-single "
                        "position differences, FP32 arithmetic, compensated FP32 sums)",
            "n_sources": N, "n_active": N, "eps2": EPS2, "order": 4, "precision": "mixed",
            "launch_shape": shape,
            "step": "copy N_i updated sources + predict + forces on N_i sinks, device-resident",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": load_traffic(),
            "kernel": "k_force<4,mixed> shape L%d P%d S%d (+ k_combine; HIP events around both on the launch "
                      "stream)" % (shape["lanes_per_sink"], shape["sinks_per_lane"], shape["splits"]),
            "kernel_ms": kern * 1e3,
            "kernel_ms_median": sorted(head_times)[len(head_times) // 2] * 1e3,
            "launches": len(head_times),
            "flops_per_interaction": FLOPS_4TH,
            "sclk_mhz": sclk["mean_mhz"],
            "frac_of_peak_at_sclk": (achieved / (PEAK_FP32 * sclk["mean_mhz"] / 2400.0)
                                     if sclk["mean_mhz"] else None),
        },
        "clock": sclk,
        "max_rel_err": head_err,
        "fp64": {
            "value": inter / sec64,
            "ms_per_step": sec64 * 1e3,
            "kernel_ms": kern64 * 1e3,
            "roofline_frac": FLOPS_4TH * inter / kern64 / 1e12 / PEAK_FP64,
            "speedup_mixed_over_fp64": kern64 / kern,
        },
        "cpu_baseline": cpu,
        "sweep": sweep,
        "launch_floor_us": floor_us if sweep else None,
        "tune_seconds": tune_s,
    }
    if o2 is not None:
        line["order2"] = o2
    if e2e is not None:
        line["end_to_end"] = e2e
    if bsr is not None:
        line["blockstep"] = bsr
    if bs4 is not None:
        line["blockstep4"] = bs4
    if o6 is not None:
        line["order6"] = o6
    if o8 is not None:
        line["order8"] = o8
    if bt is not None:
        line["batch"] = bt
    if adj is not None:
        line["adjoint"] = adj
    print(json.dumps(line), flush=True)
    reap_children()


def reap_children():
    """Leave no process behind: end any child this process started (none is expected)."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for k in kids:
        print("bench: ending child process %d (%s)" % (k.pid, " ".join(k.cmdline()[:3])), file=sys.stderr,
              flush=True)
        k.terminate()
    psutil.wait_procs(kids, timeout=5)


if __name__ == "__main__":
    main()
