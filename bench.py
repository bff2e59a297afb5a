"""Benchmark of the ion PIC/MCC step on one MI355X.

Workload: 2M argon ions in FP64 on the 64x64x128 mesh (sort every 50 steps,
dt = 1e-9 s, synthetic ECRIS-shaped inputs).  A step is one pass of the whole
path: sort (every 50th step), Coulomb collisions, push + wall/aperture loss +
ionisation/charge exchange, and the density deposit.  The ions are created
on the GPU before the timed region.

Order: init; a fixed settling run (50 000 steps by default, whatever
--warmup is) so that the timed state has ions reaching the walls and the
aperture and atoms recycled at the gas inlet; --warmup steps; a short pass
with HIP events around every launch that picks the dominant kernel; steps up
to the next sort; then the timed window: --steps rounded up to whole sort
periods, starting with a sort, bracketed by device synchronisations.

Prints one JSON line: throughput in particle-steps/s, the roofline of the
dominant kernel (algorithmic bytes per launch / its mean launch time, timed
with HIP events on the run's stream around one in `stride` of its launches
in the timed window, at least ten of them) and of the whole step (the fused
step's algorithmic bytes plus the sort's share, over the mean step time),
the HBM traffic the committed rocprofv3 counters give for that kernel, and
the CPU oracle timed on a bounded sample of the same workload, alone on one
core and as one copy per usable core at once.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "ion particle-steps/s (push+MCC+deposit) at 2M ions; p50/p99 scan latency"


def describe(name, p):
    prec = "FP32-mixed (binary32 state, binary64 accumulators)" if p.get("precision", 0) else "FP64"
    mix = " + ".join(f"{round(100 * s['fraction'])}% {'O' if s['z_max'] == 8 else 'Ar'} (Q<={s['z_max']})"
                     for s in p["species"])
    ne = "self-consistent electrons (n_e = ion charge density per cell)" if p.get("self_ne") else \
        "fixed electron background"
    if p.get("self_n0"):
        ne += ", neutrals from the tracked atoms per cell"
    if p.get("cx_partner"):
        ne += ", each charge exchange ionises a tracked atom"
    return (f"{name}: {p['n']} ions, {mix}, born Q=1 in the ECR-zone ellipsoid, {prec}, {ne}, "
            f"mesh {p['nx']}x{p['ny']}x{p['nz']}, dt {p['dt']:g} s, sort every {p['sort_every']}, "
            + ("all processes on" if (p["process_mask"] & 31) == 31 else f"process mask {p['process_mask']}")
            + (", with the electron-ion heating kick" if p["process_mask"] & 32 else ""))

# algorithmic HBM bytes per particle per launch (FP64 structure of arrays:
# x y z vx vy vz 8 B each, qs 1 B, pid 4 B, birth step 4 B (moved by the sort
# only), collision cell 4 B)
ALG_BYTES_FP64 = {
    # the fused step (Coulomb pairing and collisions, push, loss, MCC,
    # deposit): read x, v, qs, pid and the collision cell; write x, v, qs
    "step": 48 + 1 + 4 + 4 + 48 + 1,
    # read x, v, qs, pid; write x, v, qs
    "push": 48 + 1 + 4 + 48 + 1,
    # read qs, pid, cell; write one 12-byte work item per pair (half a particle)
    "coul_order": 1 + 4 + 4 + 6,
    # per particle (half a pair): read the item, both velocities and charges, write both velocities
    "coul_pairs": 6 + 24 + 1 + 24,
    # read x, qs
    "deposit": 24 + 1,
    # count pass (read x; write key, rank) + scatter (read record, key, rank; write record, cell)
    "sort": (24 + 8) + (57 + 8) + (57 + 4),
    # push + deposit in one kernel: the deposit reads nothing more from HBM
    "push_deposit": 48 + 1 + 4 + 48 + 1,
    # exchange partners: read each slot's collision cell, qs and birth (the
    # requesting cells' atoms add a few bytes more)
    "cx_partner": 4 + 1 + 4,
}
ALG_BYTES_FP32 = {
    "step": 24 + 1 + 4 + 4 + 24 + 1,
    "push": 24 + 1 + 4 + 24 + 1,
    "coul_order": 1 + 4 + 4 + 6,
    "coul_pairs": 6 + 12 + 1 + 12,
    "deposit": 12 + 1,
    "sort": (12 + 8) + (33 + 8) + (33 + 4),
    "push_deposit": 24 + 1 + 4 + 24 + 1,
    "cx_partner": 4 + 1 + 4,
}


def kernel_sources_sha256():
    """Hash of every kernel source and the boundary header (what the traffic
    counters measured): any change to them voids a committed summary."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1507_03392_amd", "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    for path in [os.path.join(csrc, f) for f in files] + [os.path.join(ROOT, "include", "ecrpic.h")]:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when there is none for this kernel and workload or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", " ", "#", "`")):
                k, _, v = line.partition(":")
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_sources_sha256() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_sample(workload, steps):
    """The oracle on a bounded sample of the workload: init, one step (the
    first sort), then `steps` timed steps.  Run in a child process that
    never touches the GPU; prints one JSON line."""
    import workloads as W
    from oracle.binding import OracleSim
    params, _ = W.config(workload)
    o = OracleSim(params)
    o.init_ions()
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    print(json.dumps({"seconds": dt, "steps": steps, "n": params["n"]}), flush=True)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    use = min(avail, int(cap)) if cap and cap.isdigit() and int(cap) > 0 else avail
    return model, os.cpu_count() or avail, avail, max(1, use)


def cpu_baseline(workload, params, steps):
    """The oracle as it stands (single-threaded C, FP64) timed on the host:
    one process alone (1 core), then one process per usable core, each on
    its own copy of the same sample, all at once; the all-core figure is
    their summed throughput (independent runs, as a scan would use the
    cores)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-sample", workload, "--cpu-steps", str(steps)]
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")

    def run_many(k):
        t0 = time.perf_counter()
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, env=env, text=True) for _ in range(k)]
        outs = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
        if any(p.returncode != 0 for p in procs):
            raise RuntimeError("oracle sample failed")
        return outs, time.perf_counter() - t0

    model, ncpu, avail, use = host_cpu()
    one, _ = run_many(1)
    v1 = one[0]["n"] * one[0]["steps"] / one[0]["seconds"]
    log(f"bench: oracle 1 core {v1:.3e} particle-steps/s; now {use} processes at once")
    many, wall = run_many(use)
    # the timed windows overlap (same work after the same set-up): summed
    # work over the slowest window
    slowest = max(o["seconds"] for o in many)
    vall = sum(o["n"] * o["steps"] for o in many) / slowest
    return dict(value=vall, unit="particle-steps/s", cores=use, kind="oracle",
                sample=f"{params['n']} ions, {params['nx']}x{params['ny']}x{params['nz']} mesh, steps 1..{steps} "
                       f"after init (one sort); single-threaded FP64 C oracle, {use} independent copies at once "
                       f"(all usable cores), slowest timed window {slowest:.1f} s",
                value_1core=v1, seconds_1core=one[0]["seconds"], cpu_model=model, nproc=ncpu,
                usable_cpus=avail)


def serve_bench(args):
    """The serving workload: the 256-request scan trace through the
    continuous-batching server; value = served particle-steps/s."""
    import torch

    import workloads as W
    from paper_1507_03392_amd.serve import Request, Server, summary

    prec = W.PREC_FP64 if args.fp64 else W.PREC_FP32
    trace = W.c5_trace(precision=prec, rate_hz=args.rate, n_hi=args.n_hi)
    reqs = [Request(rid=i, arrival=a, params=p, steps=st) for i, (a, p, st) in enumerate(trace)]
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    # warm-up: two small requests (code objects, graph capture path)
    warm = [Request(rid=i, arrival=0.0, params=W.with_(trace[i][1], n=20_000), steps=100) for i in range(2)]
    Server(hbm_budget=budget, max_active=args.slots, batch_max_n=args.batch_max_n).serve(warm)
    torch.cuda.synchronize()
    log(f"bench: serving {len(reqs)} requests at {args.rate:g}/s, {args.slots} slots, batch of runs up to "
        f"{args.batch_max_n} particles, HBM budget {budget / 2**30:.1f} GiB")
    srv = Server(hbm_budget=budget, max_active=args.slots, batch_max_n=args.batch_max_n)
    res = srv.serve(reqs)
    torch.cuda.synchronize()
    s = summary(res)
    # time-weighted number of resident runs
    ev = srv.log
    occ = sum((ev[i + 1][0] - ev[i][0]) * ev[i][3] for i in range(len(ev) - 1)) / max(1e-9, ev[-1][0] - ev[0][0])
    # resident runs over time: time-weighted mean per one-second bin
    t_end = ev[-1][0]
    bins = []
    for b0 in range(int(t_end) + 1):
        acc_t = 0.0
        for i in range(len(ev) - 1):
            lo, hi = max(ev[i][0], b0), min(ev[i + 1][0], b0 + 1)
            if hi > lo:
                acc_t += (hi - lo) * ev[i][3]
        bins.append(round(acc_t / max(1e-9, min(1.0, t_end - b0)), 2))
    total_steps = sum(r.steps for r in reqs)
    offered = sum(r.params["n"] * r.steps for r in reqs) / max(r.arrival for r in reqs)
    log(f"bench: served {s['completed']}/{s['requests']} in {s['span_s']:.2f} s, p50 {s['p50_s']:.3f} s, "
        f"p99 {s['p99_s']:.3f} s, {s['throughput']:.3e} particle-steps/s")
    out = {
        "metric": METRIC,
        "value": s["throughput"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": total_steps,
        "warmup": 0,
        "ms_per_step": s["span_s"] / total_steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"c5: {len(reqs)} scan requests, Poisson arrivals at {args.rate:g}/s, N log-uniform "
                               f"10k-{args.n_hi / 1e6:g}M, n0 3e10-3e11 cm^-3, T_e 0.3-3 keV with n_e scaled, 2000 steps each, "
                               f"mesh 64x64x128, {'FP64' if args.fp64 else 'FP32-mixed'}, {args.slots} slots"
                               + (f", runs up to {args.batch_max_n} particles batched" if args.batch_max_n else ""),
                   "requests": len(reqs), "slots": args.slots, "hbm_budget_bytes": budget,
                   "arrival_rate_hz": args.rate, "batch_max_n": args.batch_max_n, "n_hi": args.n_hi},
        "roofline": None,
        "serving": {"p50_s": s["p50_s"], "p99_s": s["p99_s"], "completed": s["completed"],
                    "span_s": s["span_s"], "particle_steps": s["particle_steps"],
                    "offered_particle_steps_per_s": offered, "mean_resident_runs": occ,
                    "max_resident_runs": max(e[3] for e in ev),
                    "resident_runs_per_second": bins,
                    "max_resident_bytes": max(e[4] for e in ev)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--prof-steps", type=int, default=200,
                    help="steps of the all-kernel timing pass (after warm-up) that picks the dominant kernel")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--event-stride", type=int, default=0,
                    help="time one launch of the dominant kernel in this many with HIP events (1: every launch; "
                         "default: 10, fewer when the window has under 100 steps, for ten timed launches)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-drift", action="store_true", help="FP32-mixed workloads: skip the FP64 comparison run")
    ap.add_argument("--self-ne", action="store_true",
                    help="electron density = ion charge density per cell (self-consistent electrons)")
    ap.add_argument("--cx-partner", action="store_true",
                    help="every charge exchange takes its electron from a tracked atom of the cell (implies --self-n0)")
    ap.add_argument("--self-n0", action="store_true",
                    help="neutral gas of charge exchange and elastic scattering from the tracked atoms per cell")
    ap.add_argument("--pressure", action="store_true",
                    help="also deposit the ion pressure moment (its own kernel after the step)")
    ap.add_argument("--process-mask", type=int, default=None,
                    help="run only the processes in this mask (push 1, ionisation 2, exchange 4, Coulomb 8, "
                         "deposit 16): a profiling aid for counters by process, not the benchmark's step")
    ap.add_argument("--heat", action="store_true",
                    help="add the electron-ion heating kick (diamagnetic bias with --self-ne)")
    ap.add_argument("--fp64", action="store_true", help="c5: serve the scan in FP64 instead of FP32-mixed")
    ap.add_argument("--slots", type=int, default=16, help="c5: run slots (one HIP stream each)")
    ap.add_argument("--rate", type=float, default=20.0, help="c5: mean arrival rate of the requests (1/s)")
    ap.add_argument("--n-hi", type=int, default=2_000_000, help="c5: largest request (particles)")
    ap.add_argument("--batch-max-n", type=int, default=0,
                    help="c5: requests of at most this many particles are batched (ecr_step_batch; 0: none)")
    ap.add_argument("--split", action="store_true",
                    help="run push and deposit as two kernels (per-kernel timing; the default fuses them)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--settle", type=int, default=None,
                    help="steps run after init and before warm-up, fixed whatever --warmup is, so that the timed "
                         "state has its losses and recycling going (default: 50000; c4: 20000)")
    ap.add_argument("--oracle-sample", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_sample:
        oracle_sample(args.oracle_sample, args.cpu_steps)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the ion step is not "
              "sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5":
        serve_bench(args)
        return

    import torch

    import paper_1507_03392_amd as ecr
    import workloads as W

    if args.copy_mb > 0:
        a = torch.ones(args.copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_mb} MiB device to device (counter calibration)")
        del a, b

    params, _ = W.config(args.workload)
    if args.self_ne:
        params["self_ne"] = True
    if args.process_mask is not None:
        params["process_mask"] = args.process_mask
    if args.heat:
        params["process_mask"] |= ecr.P_HEAT
    if args.pressure:
        params["deposit_mask"] |= 1 << W.F_ION_P
    if args.self_n0 or args.cx_partner:
        params["self_n0"] = True
    if args.cx_partner:
        params["cx_partner"] = True
    n = params["n"]
    fp32 = params.get("precision", 0) == ecr.FP32_MIXED
    log(f"bench: workload {args.workload}, {n} ions, grid {params['nx']}x{params['ny']}x{params['nz']}")
    period = params["sort_every"]
    settle = args.settle if args.settle is not None else (20_000 if args.workload == "c4" else 50_000)
    run = ecr.Run(params, split=args.split)
    run.init_ions()
    t_s = time.perf_counter()
    done = 0
    while done < settle:
        k = min(10_000, settle - done)
        run.step_graph(k)
        torch.cuda.synchronize()
        done += k
        log(f"bench: settled {done}/{settle} steps ({time.perf_counter() - t_s:.1f} s)")
    run.step(args.warmup)
    torch.cuda.synchronize()
    log(f"bench: warmup {args.warmup} steps done")

    # per-kernel launch times over a short pass (HIP events around every
    # launch on the run's stream) pick the dominant kernel ...
    run.profile(True)
    run.step(args.prof_steps)
    kt = run.kernel_times()
    run.profile(False)
    per = {k: (ms / c if c else 0.0, c) for k, (ms, c) in kt.items()}
    tot = {k: ms for k, (ms, c) in kt.items()}
    dom = max(tot, key=lambda k: tot[k])
    kernels = {k: {"avg_us": round(per[k][0] * 1e3, 2), "launches": per[k][1],
                   "share": round(tot[k] / max(1e-12, sum(tot.values())), 3)} for k in tot if per[k][1]}
    log(f"bench: kernels {json.dumps(kernels)}")

    # the timed window starts at a sort and holds whole sort periods, so it
    # carries its share of sorts whatever --steps is (rounded up)
    step_now = settle + args.warmup + args.prof_steps
    pad = (-step_now) % period
    if pad:
        run.step(pad)
    steps = -(-args.steps // period) * period
    # ... the dominant kernel is then timed with events over the timed region
    # itself, on one launch in `stride` (the event packets around a launch
    # hold up the queue, so timing every launch would slow the step it
    # measures), with at least ten timed launches
    stride = args.event_stride if args.event_stride else min(10, max(1, steps // 10))
    run.profile(True, kinds=[dom], stride=stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches = run.kernel_times()[dom]
    run.profile(False)
    elapsed = t1 - t0
    value = n * steps / elapsed
    log(f"bench: timed {steps} steps (from step {step_now + pad}, {steps // period} sorts) in {elapsed:.3f} s "
        f"({value:.3e} particle-steps/s)")
    tal = run.tallies()
    table = ALG_BYTES_FP32 if fp32 else ALG_BYTES_FP64
    alg = table[dom] * n
    avg_s = ms * 1e-3 / max(1, launches)
    achieved = alg / avg_s / 1e9
    # the whole step against the roofline: the fused step's bytes plus the
    # sort's amortised over its period
    step_bytes = (table["step"] + table["sort"] / period) * n
    step_frac = step_bytes / (elapsed / steps) / 1e9 / HBM_PEAK_GBS
    # the counters were taken on the default step (fixed electron background,
    # no optional physics, fused deposit): another configuration runs other code
    default_step = not (args.self_ne or args.heat or args.split or args.self_n0 or args.cx_partner or args.pressure
                        or args.process_mask is not None)
    traffic = measured_traffic(args.workload, dom) if default_step else None

    drift = None
    if fp32 and not args.no_drift:
        # the FP32-mixed run against the same workload in FP64 on the same
        # GPU (the FP64 path matches the oracle to 1e-12), same steps from init
        done = step_now + pad + steps
        ref = ecr.Run(W.with_(params, precision=0))
        ref.init_ions()
        ref.step_graph(done)
        tr = ref.tallies()
        t32 = run.tallies()
        a32, a64 = run.get_state(), ref.get_state()
        d32, d64 = run.density(W.F_ION_N)[0], ref.density(W.F_ION_N)[0]
        ion32, ion64 = t32["ionized"].sum(axis=0), tr["ionized"].sum(axis=0)
        q = [int(i) for i in np.nonzero(ion64 >= 100)[0]]
        e32 = float(np.mean(a32["vx"] ** 2 + a32["vy"] ** 2 + a32["vz"] ** 2))
        e64 = float(np.mean(a64["vx"] ** 2 + a64["vy"] ** 2 + a64["vz"] ** 2))
        drift = {"reference": "same workload in FP64 on this GPU", "steps": done,
                 "ionized_rel_err_by_q": {str(i): float(ion32[i] / ion64[i] - 1) for i in q},
                 "ionized_total": [int(ion32.sum()), int(ion64.sum())],
                 "extracted_total": [int(t32["extracted"].sum()), int(tr["extracted"].sum())],
                 "wall_total": [int(t32["wall"].sum()), int(tr["wall"].sum())],
                 "cx_total": [int(t32["cx"].sum()), int(tr["cx"].sum())],
                 "mean_v2_rel_diff": e32 / e64 - 1,
                 "ion_density_rel_l1": float(np.abs(d32 - d64).sum() / np.abs(d64).sum())}
        log(f"bench: FP32-mixed drift vs FP64 {json.dumps(drift)}")
        del ref

    cpu = None
    if not args.no_cpu:
        log(f"bench: CPU oracle sample, {args.cpu_steps} steps of the same workload")
        cpu = cpu_baseline(args.workload, params, args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload, params),
                   "n_particles": n, "mesh": [params["nx"], params["ny"], params["nz"]],
                   "sort_every": period, "steps_requested": args.steps,
                   "timed_window": [step_now + pad, step_now + pad + steps], "settle_steps": settle},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg, "avg_launch_us": avg_s * 1e6, "timed_launches": launches,
                     "event_stride": stride, "step_alg_bytes": step_bytes, "step_frac": step_frac},
        "kernels": kernels,
        "tallies": {"ionized": int(tal["ionized"].sum()), "wall": int(tal["wall"].sum()),
                    "extracted": int(tal["extracted"].sum()), "cx": int(tal["cx"].sum()),
                    "anomalies": tal["anomalies"]},
        "cpu_baseline": cpu,
    }
    if drift is not None:
        out["drift_vs_fp64"] = drift
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
