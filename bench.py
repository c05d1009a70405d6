"""Benchmark: spin-flip attempts/s and time-to-converged-weights of the
parallel multicanonical method on one MI355X.

Workload (the paper's scale, Sec. 3): 2D Ising model, L = 32 (1024 spins,
1025 energy bins), 16384 walkers, random +-1 starts, log weights 0 at the
start, weight iterations of 200 recorded sweeps until min H / mean H >= 0.5
over the reachable bins, then a 10^4-sweep production run and ln g.

One step = one full solve with its own seed: create the instance (initial
spins on the device), iterate to flatness, production run, ln g.  ``value``
is every attempted spin flip of the timed steps divided by their wall time,
inputs resident on the device.  ``ttc_p50_s`` / ``ttc_p99_s`` are the
nearest-rank percentiles over the timed steps of the wall time from instance
creation to the return of the first weight iteration that reaches flatness.

roofline: the sweep kernel's device time comes from HIP events the library
records around its launches on the stream it launches them on; its
algorithmic work per attempt is counted in 32-bit integer operations (see
``ALU_OPS_PER_ATTEMPT``) against the chip's integer issue peak.

cpu_baseline: the CPU oracle (plain C, OpenMP over walkers) on a bounded
sample of the same workload, at the exact weights omega = -ln g.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from muca_inputs import WORKLOADS  # noqa: E402

WORKLOAD = "ising_L32_W16384"
METRIC = "spin-flip attempts/s at L=32, 16384 walkers; p50/p99 time-to-converged-weights"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = one wave64 32-bit VALU
# instruction per SIMD every 4 clocks, in lane-operations per second.  Measured
# on gfx950 (bench.py --issue-probe): the 32-bit multiplies (lo, hi, the
# 32x32->64 mad) and the three-input xor issue at 0.94-0.98 of it with eight
# waves per SIMD; a 32-bit add issues faster (up to 1.5x).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic 32-bit integer operations per attempt: a quarter of a
# Philox4x32-10 block (5 products 32x32->64 and 10 two-input XORs; the key
# schedule is per walker and precomputed) plus the Metropolis step (4
# neighbour reads, 3 adds, the energy change, the table index, the compare,
# the conditional flip, the energy update, the histogram increment: 13).
ALU_OPS_PER_ATTEMPT = 5 + 10 + 13
# The second roof: LDS bytes per attempt the chain needs -- the threshold
# gather (4 B) and the histogram counter's read-modify-write (4 + 4 B) -- plus
# the random words handed over through LDS in the two-wave form (4 B written,
# 4 B read).  Peak: 128 B per clock per CU.
LDS_BYTES_PER_ATTEMPT = {2: 4 + 8 + 8, 5: 4 + 8 + 8, 1: 4 + 8, 0: 8 + 8, 3: 8, 4: 8 + 8}


def lds_bytes_per_attempt(variant, L):
    return LDS_BYTES_PER_ATTEMPT[variant]
LDS_PEAK_BYTES = 256 * 128 * 2.4e9


def nearest_rank(values, q):
    v = sorted(values)
    if not v:
        return None
    idx = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[idx]


def exact_ln_g(L):
    """Exact ln g from the golden tables (exact integers, or ln g for large L)."""
    path = os.path.join(ROOT, "tests", "golden", "ising_dos_L%d.txt" % L)
    if os.path.exists(path):
        with open(path) as f:
            g = [int(x) for x in f if not x.startswith("#")]
        return np.array([math.log(v) if v > 0 else -math.inf for v in g])
    path = os.path.join(ROOT, "tests", "golden", "ising_lndos_L%d.txt" % L)
    if os.path.exists(path):
        with open(path) as f:
            return np.array([float(x) for x in f if not x.startswith("#")])
    return None


KERNEL_NAMES = {0: "sweep_kernel", 1: "sweep_fast_kernel", 2: "sweep_split_kernel", 3: "sweep_wide_kernel",
                4: "sweep_wide_split_kernel", 5: "sweep_pair_kernel"}


def solve(Solver, wl, seed, iter_cap):
    L, W = wl["L"], wl["walkers"]
    t0 = time.perf_counter()
    s = Solver(L, W, seed)
    t_created = time.perf_counter()
    attempts = 0
    kernel_ms = 0.0
    launches = 0
    variant_ms = {}
    it = 0
    converged = False

    def account(info):
        nonlocal attempts, kernel_ms, launches
        attempts += info["attempts"]
        kernel_ms += info["kernel_ms"]
        launches += info["kernel_launches"]
        v = info["kernel_variant"]
        variant_ms[v] = variant_ms.get(v, 0.0) + info["kernel_ms"]

    last_note = time.perf_counter()
    while it < iter_cap:
        info = s.iterate(wl["therm_sweeps"], wl["iter_sweeps"])
        it += 1
        account(info)
        if info["flatness"] >= wl["min_flat"]:
            converged = True
            break
        if time.perf_counter() - last_note > 30.0:
            print("  seed %d: iteration %d, visited %d bins, flatness %.3f" %
                  (seed, it, info["visited_bins"], info["flatness"]), file=sys.stderr, flush=True)
            last_note = time.perf_counter()
    t_conv = time.perf_counter()
    account(s.production(wl["prod_therm_sweeps"], wl["prod_sweeps"]))
    lng = s.log_dos(0) if converged else None
    s.close()
    t_end = time.perf_counter()
    return dict(seed=seed, iterations=it, converged=converged, attempts=attempts,
                kernel_ms=kernel_ms, launches=launches, variant_ms=variant_ms,
                ttc_s=t_conv - t_created, wall_s=t_end - t0, ln_g=lng)


def hardware_rate(Solver, wl, ln_g, warm_sweeps=20, timed_sweeps=200):
    """The paper's hardware measurement (Sec. 3.1): start from the exact
    weights, skip equilibration, time a fixed number of sweeps."""
    L, W = wl["L"], wl["walkers"]
    s = Solver(L, W, 12345)
    om = np.where(np.isfinite(ln_g), -ln_g, 0.0)
    s.set_log_weights(om)
    s.production(0, warm_sweeps)
    info = s.production(0, timed_sweeps)
    s.close()
    return info["attempts"] / (info["kernel_ms"] * 1e-3), info["kernel_ms"] / info["kernel_launches"]


KERNEL_SOURCES = ["muca_kernels.hip", "muca_sweep_fast.hip", "muca_sweep_split.hip", "muca_sweep_wide.hip",
                  "muca_chain.h", "muca_rowbits.h", "philox.h", "muca_device.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_L32_W16384.txt")
# The chain wave's instruction count per attempt of the headline kernel (from
# its gfx950 assembly, checked against SQ_INSTS_* counters), for the third
# roof: one chain wave per 64 walkers issues at most one instruction every 4
# clocks, so no launch of W walkers beats (W / 64) * 64 * 2.4e9 / (4 * count)
# attempts/s while each chain wave has a SIMD to itself.
CHAIN_FILE = os.path.join(ROOT, "profiles", "chain_issue_sweep_split_L32.md")
COPY_BYTES = 256 << 20


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_00919_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per sweep launch of the benchmark shape from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads
    for a plain copy) and a note of where they came from; the bytes are None
    if the kernel sources changed since the counters were taken.  The
    lattices stay in L2 during a launch, so the count does not grow with the
    sweeps per launch."""
    rel = os.path.relpath(TRAFFIC_FILE, ROOT)
    src = kernel_source_hash()
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary (%s missing)" % rel
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    taken = vals.get("kernel_source_sha256_16")
    if taken != src:
        return None, ("%s was taken on kernel sources %s, not the current %s: not used" % (rel, taken, src))
    return float(vals["hbm_bytes_per_launch"]), (
        "rocprofv3 FETCH_SIZE + WRITE_SIZE from %s (kernel sources %s, the ones built here), "
        "not measured in this run" % (rel, src))


def summary_values(path):
    """key = value lines of a committed profile summary."""
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith(("#", "|", "`")) and line.count("=") == 1:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    return vals


def chain_roof(attempts_per_s, walkers):
    """The chain-issue roof of the headline kernel from the committed
    instruction count (None and a note if the kernel sources changed since)."""
    rel = os.path.relpath(CHAIN_FILE, ROOT)
    src = kernel_source_hash()
    if not os.path.exists(CHAIN_FILE):
        return None, "no instruction count (%s missing)" % rel
    vals = summary_values(CHAIN_FILE)
    if vals.get("kernel_source_sha256_16") != src:
        return None, "%s was taken on kernel sources %s, not the current %s: not used" % (
            rel, vals.get("kernel_source_sha256_16"), src)
    per = float(vals["chain_instructions_per_attempt"])
    waves = -(-walkers // 64)
    peak = min(waves, 256) * 64 * 2.4e9 / (4.0 * per)
    return {"bound": "chain issue", "achieved": attempts_per_s, "peak": peak, "unit": "attempts/s",
            "frac": attempts_per_s / peak, "chain_instructions_per_attempt": per, "chain_waves": waves,
            "clocks_per_instruction": 4}, "instruction count from %s (kernel sources %s)" % (rel, src)


def scaled_log_weights(L):
    """Near-flat log weights for a lattice with no exact table: the exact
    entropy of the L/2 lattice scaled to L (ln g_L(E) ~ 4 ln g_{L/2}(E/4),
    the entropy per spin hardly depending on L); None if that table is missing."""
    half = exact_ln_g(L // 2)
    if half is None:
        return None
    ok = np.isfinite(half)
    k = np.arange(half.size)
    om = -4.0 * np.interp(np.arange(L * L + 1) / 4.0, k[ok], half[ok])
    return om - om.max()


def profile_pass(Solver, wl, ln_g, sweeps=50, warm=0):
    """Short run for counter collection: one sweep launch of the benchmark
    shape at exact weights (near-flat scaled ones where no exact table
    exists), after `warm` unrecorded sweeps that spread the walkers over the
    energy range (their launches come first in a trace), then a plain device
    copy of COPY_BYTES bytes that calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch
    s = Solver(wl["L"], wl["walkers"], 12345)
    if ln_g is not None:
        s.set_log_weights(np.where(np.isfinite(ln_g), -ln_g, 0.0))
    else:
        s.set_log_weights(scaled_log_weights(wl["L"]))
    if warm:
        s.production(0, warm)
    info = s.production(0, sweeps)
    s.close()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": True, "warm_sweeps": warm, "width": info["width"], "attempts": info["attempts"],
                      "kernel_variant": info["kernel_variant"], "copy_bytes": COPY_BYTES,
                      "kernel_source_sha256_16": kernel_source_hash()}), flush=True)


def cpu_full_solve(wl, iter_cap, seed=1):
    """The weight iteration of one solve of the workload on the CPU oracle (all
    host threads), to the first flat iteration: its wall time (the oracle's
    time to converged weights).  The production run is left out: at 10^4 +
    10^4 sweeps it would take the oracle about ten more minutes."""
    import oracle
    L, W = wl["L"], wl["walkers"]
    t0 = time.perf_counter()
    o = oracle.OracleMuca(L, W, seed)
    it = 0
    while it < iter_cap:
        info = o.iterate(wl["therm_sweeps"], wl["iter_sweeps"])
        it += 1
        print("oracle iteration %d: flatness %.3f, %.0f s" % (it, info["flatness"],
              time.perf_counter() - t0), file=sys.stderr, flush=True)
        if info["flatness"] >= wl["min_flat"]:
            break
    t_w = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"seed": seed, "iterations": it, "ttcw_s": t_w, "cores": threads, "kind": "oracle"}


def host_cpu():
    """The host CPU the oracle ran on: model name and the logical CPUs this
    process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "usable_cpus": len(os.sched_getaffinity(0)), "nproc": os.cpu_count()}


def cpu_baseline(wl, ln_g, sweeps, warm, nthreads=0):
    import oracle
    L, W = wl["L"], wl["walkers"]
    o = oracle.OracleMuca(L, W, 12345, nthreads=nthreads)
    o.set_log_weights(np.where(np.isfinite(ln_g), -ln_g, 0.0))
    o.production(0, warm)
    t = time.perf_counter()
    info = o.production(0, sweeps)
    dt = time.perf_counter() - t
    threads = nthreads or int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {
        "value": info["attempts"] / dt,
        "unit": "attempts/s",
        "cores": threads,
        "kind": "oracle",
        "host": host_cpu(),
        "sample": "L=%d, %d walkers, %d sweeps after %d warm-up sweeps at exact weights "
                  "omega = -ln g (%.2e attempts, %.1f s)" % (L, W, sweeps, warm, info["attempts"], dt),
    }


# ------------------------------------------------------------ other workloads
def _solo_solve(Solver, L, W, seed, iter_sweeps, min_flat, max_it, prod_therm, prod_sweeps):
    """One instance alone: weight iterations to the flatness bound, then the
    production run in one call; returns (attempts, iterations, ln g, wall s)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = Solver(L, W, seed)
    att, it = 0, 0
    while it < max_it:
        info = s.iterate(0, iter_sweeps)
        att += info["attempts"]
        it += 1
        if info["flatness"] >= min_flat:
            break
    att += s.production(prod_therm, prod_sweeps)["attempts"]
    lng = _log_dos_or_zeros(s)
    s.close()
    torch.cuda.synchronize()
    return att, it, lng, time.perf_counter() - t0


def _log_dos_or_zeros(s):
    from paper_1707_00919_amd import MucaError
    try:
        return s.log_dos(0)
    except MucaError:
        return np.zeros(s.N + 1)


def batched_solve(Batch, Solver, inst, flags, iter_sweeps, min_flat, max_it, prod_therm, prod_sweeps):
    """The instances solved together in batched rounds.  Every round runs, for
    each member, a weight iteration until its flatness bound, then slices of
    its production run (at most iter_sweeps sweeps each, the unrecorded ones
    first) from the next round on, so that early members do not wait for the
    slowest one.  The slices' histograms are summed and ln g taken from the
    sum (ln g(E_min) = ln 2), which equals one production call of the same
    sweeps.  Returns (attempts, iterations, ln g list, rounds, device ms of
    every round)."""
    from paper_1707_00919_amd import MucaError
    from paper_1707_00919_amd.analysis import jackknife_log_dos
    members = [Solver(L, W, sd) for L, W, sd in inst]
    b = Batch(members, flags=flags)
    n = len(members)
    iters = [0] * n
    phase = [0] * n              # 0 iterating, 1 production, 2 done
    therm_left = [prod_therm] * n
    prod_left = [prod_sweeps] * n
    acc = [np.zeros(m.N + 1, dtype=np.uint64) for m in members]
    att, round_ms, rounds = 0, [], 0
    while any(ph != 2 for ph in phase):
        mode = np.zeros(n, dtype=np.uint32)
        th = np.zeros(n, dtype=np.uint32)
        sw = np.zeros(n, dtype=np.uint32)
        for i in range(n):
            if phase[i] == 0:
                mode[i], sw[i] = 1, iter_sweeps
            elif phase[i] == 1:
                mode[i] = 2
                th[i] = min(therm_left[i], iter_sweeps)
                sw[i] = min(prod_left[i], iter_sweeps - th[i])
        infos = b.run(mode, th, sw)
        rounds += 1
        round_ms.append(next(i for i in infos if i is not None)["kernel_ms"])
        for i, inf in enumerate(infos):
            if inf is None:
                continue
            att += inf["attempts"]
            if phase[i] == 0:
                iters[i] += 1
                if inf["flatness"] >= min_flat or iters[i] >= max_it:
                    phase[i] = 1
            else:
                therm_left[i] -= int(th[i])
                prod_left[i] -= int(sw[i])
                if sw[i]:
                    acc[i] += members[i].histogram()
                if therm_left[i] == 0 and prod_left[i] == 0:
                    phase[i] = 2
    lngs = []
    for m, h in zip(members, acc):
        try:
            lngs.append(jackknife_log_dos(m.L, h, m.log_weights(), normalization=0)[0])
        except MucaError:
            lngs.append(np.zeros(m.N + 1))
    b.close()
    for m in members:
        m.close()
    return att, iters, lngs, rounds, round_ms


def bench_batched(args):
    """48 instances of uneven size (muca_inputs.batch_instances) solved in
    batched rounds, against the same instances solved one per launch."""
    import torch
    from paper_1707_00919_amd import Batch, Solver, _abi
    from muca_inputs import BATCH_WORKLOAD as C, batch_instances
    inst = batch_instances(C["instances"])
    flags = _abi.MUCA_BATCH_GRAPH | _abi.MUCA_BATCH_AUTOTUNE

    def batched():
        return batched_solve(Batch, Solver, inst, flags, C["iter_sweeps"], C["min_flat"], C["max_iterations"],
                             C["prod_therm_sweeps"], C["prod_sweeps"])

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    att_b, iters_b, lng_b, rounds, round_ms = batched()
    kms = float(sum(round_ms))
    tenths = np.array_split(np.asarray(round_ms), 10)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    print("batched: %.2f s, %d rounds" % (wall_b, rounds), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    att_s, same = 0, True
    iters_s, solo_wall = [], []
    for (L, W, sd), lb in zip(inst, lng_b):
        a, it, lng, ws = _solo_solve(Solver, L, W, sd, C["iter_sweeps"], C["min_flat"],
                                     C["max_iterations"], C["prod_therm_sweeps"], C["prod_sweeps"])
        att_s += a
        iters_s.append(it)
        solo_wall.append(ws)
        same &= bool(np.array_equal(lng.view(np.uint64), lb.view(np.uint64)))
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    slow = int(np.argmax(solo_wall))
    print("one per launch: %.2f s; slowest member alone %.2f s (L=%d, %d walkers)" %
          (wall_s, solo_wall[slow], inst[slow][0], inst[slow][1]), file=sys.stderr, flush=True)
    out = {
        "metric": "aggregate spin-flip attempts/s, 48 uneven instances, batched rounds",
        "value": att_b / wall_b, "unit": "attempts/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": wall_b * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched48", "instances": len(inst),
                   "L": sorted(set(L for L, _, _ in inst)),
                   "walkers_total": sum(W for _, W, _ in inst),
                   "iter_sweeps": C["iter_sweeps"], "min_flatness": C["min_flat"],
                   "production": [C["prod_therm_sweeps"], C["prod_sweeps"]],
                   "production_slices": C["iter_sweeps"],
                   "batch_flags": "graph|autotune"},
        "one_per_launch_attempts_per_s": att_s / wall_s,
        "speedup_vs_one_per_launch": (att_b / wall_b) / (att_s / wall_s),
        "bit_identical_to_one_per_launch": same and iters_b == iters_s,
        "rounds": rounds, "iterations_max": max(iters_b),
        "batched_wall_s": wall_b, "one_per_launch_wall_s": wall_s,
        "slowest_member_alone_s": solo_wall[slow],
        "slowest_member": {"L": inst[slow][0], "walkers": inst[slow][1], "seed": inst[slow][2],
                           "iterations": iters_s[slow]},
        "makespan_over_slowest_alone": wall_b / solo_wall[slow],
        "batched_device_ms": kms,
        "device_share_of_wall": kms * 1e-3 / wall_b,
        "round_device_ms_by_tenth": [round(float(t.mean()), 2) for t in tenths if t.size],
    }
    print(json.dumps(out), flush=True)


def bench_served(args):
    """Poisson request arrivals (muca_inputs.serving_requests) into the
    continuous-batching server; request latency percentiles and throughput."""
    import torch
    from paper_1707_00919_amd import Server, Solver
    from muca_inputs import SERVE_REQUEST as Q, serving_requests
    reqs = serving_requests(duration=args.serve_duration)
    srv = Server(64 << 30, max_active_walkers=args.serve_max_walkers, batch_flags=1, policy=args.serve_policy,
                 max_wait_s=args.serve_max_wait)
    t0 = time.perf_counter()
    # the server's clock (seconds since it was created) on this loop's clock
    clock_off = (time.perf_counter() - t0) - srv.stats()["clock_s"]
    tickets = {}
    nxt = 0
    results = {}
    lng_served = {}
    last_note = t0
    while len(results) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt][0] <= now:
            _, L, W, sd = reqs[nxt]
            tickets[srv.submit(L, W, sd, **Q)] = nxt
            nxt += 1
        if not srv.progress():
            time.sleep(2e-4)
        for t in list(tickets):
            r = srv.take(t)
            if r is not None:
                i = tickets.pop(t)
                results[i] = r[0]
                if i < args.serve_solo_sample:
                    lng_served[i] = r[1]
        if time.perf_counter() - last_note > 30.0:
            st = srv.stats()
            print("served %d/%d, active %d, queued %d, %.0f s" %
                  (len(results), len(reqs), st["active"], st["queued"], st["clock_s"]),
                  file=sys.stderr, flush=True)
            last_note = time.perf_counter()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    # one request per launch, in turn, for the first requests of the stream:
    # the same solves alone (bit-identical results), timed back to back
    solo = None
    if args.serve_solo_sample:
        t1 = time.perf_counter()
        att_s, same = 0, True
        for i in range(min(args.serve_solo_sample, len(reqs))):
            _, L, W, sd = reqs[i]
            a, _, lng, _ = _solo_solve(Solver, L, W, sd, Q["iter_sweeps"], Q["min_flatness"],
                                    Q["max_iterations"], Q["prod_therm"], Q["prod_sweeps"])
            att_s += a
            same &= bool(np.array_equal(lng.view(np.uint64), lng_served[i].view(np.uint64)))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        solo = {"requests": min(args.serve_solo_sample, len(reqs)), "attempts_per_s": att_s / dt,
                "wall_s": dt, "bit_identical_to_served": same}
    # latency from each request's scheduled arrival, not from the moment the
    # loop got round to submitting it (progress() can block briefly), so a
    # late submission does not hide waiting time
    lat = [r["t_done"] + clock_off - reqs[i][0] for i, r in results.items()]
    ttcw = [r["t_weights"] + clock_off - reqs[i][0] for i, r in results.items()]
    submit_lag = [r["t_submit"] + clock_off - reqs[i][0] for i, r in results.items()]
    att = sum(r["attempts"] for r in results.values())
    out = {
        "metric": "served multicanonical solves: aggregate attempts/s; p50/p99 latency",
        "value": att / wall, "unit": "attempts/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "served_poisson20", "requests": len(reqs),
                   "arrival_rate_per_s": 20.0, "arrival_window_s": args.serve_duration,
                   "L": [16, 24, 32, 48, 64], "walkers": [1024, 16384],
                   "mem_cap_bytes": 64 << 30, "max_active_walkers": args.serve_max_walkers,
                   "admission": args.serve_policy, "max_wait_s": args.serve_max_wait,
                   **Q},
        "latency_p50_s": nearest_rank(lat, 50), "latency_p99_s": nearest_rank(lat, 99),
        "latency_from": "scheduled arrival",
        "submit_lag_max_s": max(submit_lag), "submit_lag_p99_s": nearest_rank(submit_lag, 99),
        "ttcw_p50_s": nearest_rank(ttcw, 50), "ttcw_p99_s": nearest_rank(ttcw, 99),
        "converged": sum(1 for r in results.values() if r["status"] == 0),
        "failed": sum(1 for r in results.values() if r["status"] not in (0, 5)),
        "makespan_s": wall, "peak_counters": st,
        "one_per_launch_sample": solo,
        "speedup_vs_one_per_launch": (att / wall) / solo["attempts_per_s"] if solo else None,
    }
    print(json.dumps(out), flush=True)


def bench_schedule(args):
    """The paper's iteration schedule (Sec. 3: Eq. 7 update counts, f_therm
    = 30, growth 1.1, stop at d_k < 1e-4 -- or at d_c < 0.05, App. A) at
    L = 32, 16384 walkers, then a production run; time to converged weights,
    ln g accuracy, and seed 1's d_k and d_c per iteration (the quantities of
    the paper's f_therm study, App. A, for the f_therm given)."""
    import torch
    from paper_1707_00919_amd import Solver
    L, W = 32, 16384
    ln_g = exact_ln_g(L)
    runs = []
    for seed in range(1, args.steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Solver(L, W, seed)
        ok, steps = s.run_schedule(max_iterations=args.schedule_max_iterations, stop=args.schedule_stop,
                                   f_therm=args.f_therm)
        t_w = time.perf_counter() - t0
        if seed == 1:
            trace = [[st["kl_divergence"], st["chebyshev"]] for st in steps]
        err = None
        if ok:  # production only at converged weights
            s.production(10000, 10000)
            lng = s.log_dos(0)
            m = np.isfinite(ln_g)
            err = float(np.max(np.abs(lng[m] - ln_g[m])))
        wall = time.perf_counter() - t0
        pos = s.last_info()["position"]
        s.close()
        runs.append(dict(ok=ok, iterations=len(steps), ttcw=t_w, wall=wall, err=err, position=pos,
                         first_full=next((i for i, st in enumerate(steps)
                                          if st["width"] == L * L + 1), None),
                         attempts=W * pos))
        print("seed %d: converged %s, %d iterations, %.2f s to weights, ln g err %s" %
              (seed, ok, len(steps), t_w, "%.3f" % err if err is not None else "-"), file=sys.stderr,
              flush=True)
    wall = sum(r["wall"] for r in runs)
    out = {
        "metric": "time to converged weights, paper's schedule, L=32, 16384 walkers",
        "value": nearest_rank([r["ttcw"] for r in runs], 50), "unit": "s", "n_gpus": 1,
        "steps": len(runs), "warmup": 0, "ms_per_step": wall * 1e3 / len(runs),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "paper_schedule_L32", "L": L, "walkers": W, "z": 2.25,
                   "f_therm": args.f_therm, "growth": 1.1, "stop": args.schedule_stop,
                   "max_iterations": args.schedule_max_iterations,
                   "dk_flat": 1e-4, "dc_flat": 0.05, "production": [10000, 10000]},
        "ttcw_p50_s": nearest_rank([r["ttcw"] for r in runs], 50),
        "ttcw_p99_s": nearest_rank([r["ttcw"] for r in runs], 99),
        "iterations": [r["iterations"] for r in runs],
        "first_full_range_iteration": [r["first_full"] for r in runs],
        "converged": sum(r["ok"] for r in runs),
        "ln_g_max_abs_err": max((r["err"] for r in runs if r["err"] is not None), default=None),
        "attempts_per_s": sum(r["attempts"] for r in runs) / wall,
        "seed1_dk_dc_per_iteration": trace,
    }
    print(json.dumps(out), flush=True)


def bench_production(args):
    """Production analysis at L = 32 (Sec. 3.3): at the exact weights, a
    production run of 16384 walkers in 100 blocks, jackknife errors of ln g,
    <E>/N and C/N at three temperatures against their exact values, and the
    paper's statistical gain: squared jackknife errors of the oracle on the
    host cores (24 walkers, as the paper's CPU node) over those of the GPU,
    scaled to equal run time."""
    import torch
    from paper_1707_00919_amd import Solver, analysis
    import oracle
    from oracle import analysis as oracle_analysis
    L, W, blocks = 32, 16384, 100
    ln_g = exact_ln_g(L)
    omega = np.where(np.isfinite(ln_g), -ln_g, 0.0)
    betas = [0.3, 0.4406867935, 0.6]
    s = Solver(L, W, 1)
    s.set_log_weights(omega)
    s.production(10000, 0)   # the walkers start from random spins (reading 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = analysis.production_blocks(s, 0, args.block_sweeps, blocks)
    t_gpu = time.perf_counter() - t0
    s.close()
    est, err = analysis.jackknife_log_dos(L, h, omega, 1)
    e, ee, c, ce = analysis.canonical(L, h, omega, betas)
    ex, cx = oracle_analysis.canonical(ln_g, betas)
    m = np.isfinite(ln_g)
    dev = np.abs(est[m] - ln_g[m])
    # the oracle: 24 walkers on the host cores, same weights, bounded time
    o = oracle.OracleMuca(L, 24, 1)
    o.set_log_weights(omega)
    o.production(10000, 0)
    tw = time.perf_counter()
    o.production(0, 100)
    rate = 24 * L * L * 100 / (time.perf_counter() - tw)
    t1 = time.perf_counter()
    hc = []
    per_block = max(1, int(args.cpu_seconds * rate / (24 * L * L * blocks)))
    for _ in range(blocks):
        o.production(0, per_block)
        hc.append(o.hist.copy())
    t_cpu = time.perf_counter() - t1
    est_c, err_c = oracle_analysis.jackknife_log_dos(np.array(hc), omega, 1)
    both = m & np.isfinite(err) & np.isfinite(err_c) & (err > 0) & (err_c > 0)
    gain = float(np.mean((err_c[both] ** 2 * t_cpu) / (err[both] ** 2 * t_gpu)))
    out = {
        "metric": "production analysis at L=32: jackknife errors, canonical averages, "
                  "statistical gain over the CPU oracle at equal time",
        "value": gain, "unit": "x (eps_cpu^2 / eps_gpu^2 at equal run time)", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": t_gpu * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "production_L32", "L": L, "walkers": W, "blocks": blocks,
                   "block_sweeps": args.block_sweeps, "weights": "exact, omega = -ln g",
                   "cpu": "oracle, 24 walkers, %d sweeps per block" % per_block},
        "gpu_production_s": t_gpu, "gpu_attempts_per_s": W * L * L * blocks * args.block_sweeps / t_gpu,
        "cpu_production_s": t_cpu,
        "ln_g_max_abs_dev": float(dev.max()),
        "ln_g_jackknife_err_mean": float(np.mean(err[m & np.isfinite(err)])),
        "ln_g_frac_within_2_err": float(np.mean(dev < 2 * err[m])),
        "betas": betas,
        "energy_per_spin": list(map(float, e)), "energy_err": list(map(float, ee)),
        "energy_exact": list(map(float, ex)),
        "specific_heat_per_spin": list(map(float, c)), "specific_heat_err": list(map(float, ce)),
        "specific_heat_exact": list(map(float, cx)),
        "cpu_cores": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(),
    }
    print(json.dumps(out), flush=True)


def bench_issue_probe(args):
    """Issue rates of the integer vector instructions the sweep is made of
    (muca_probe_issue_rate): lane-operations per second of each, with one and
    with eight waves per SIMD, against the ALU peak the roofline uses."""
    import ctypes
    from paper_1707_00919_amd import _abi
    lib = _abi.lib()
    rows = []
    for name, op in _abi.MUCA_PROBE_OPS.items():
        for wps in (1, 2, 8):
            ms, ops = ctypes.c_double(), ctypes.c_uint64()
            rc = lib.muca_probe_issue_rate(op, wps, args.probe_iterations, ctypes.byref(ms), ctypes.byref(ops))
            if rc != 0:
                raise RuntimeError("muca_probe_issue_rate failed: %d" % rc)
            rate = ops.value / (ms.value * 1e-3)
            rows.append({"instruction": name, "waves_per_simd": wps, "ms": ms.value, "lane_ops": ops.value,
                         "lane_ops_per_s": rate, "frac_of_peak": rate / VALU_PEAK_OPS})
            print("%-22s %d waves/SIMD: %.3e lane-ops/s (%.3f of %.3e)" %
                  (name, wps, rate, rate / VALU_PEAK_OPS, VALU_PEAK_OPS), file=sys.stderr, flush=True)
    print(json.dumps({"issue_probe": rows, "peak_lane_ops_per_s": VALU_PEAK_OPS,
                      "iterations": args.probe_iterations}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iter-cap", type=int, default=2000)
    ap.add_argument("--cpu-attempts", type=float, default=6.7e9,
                    help="size of the oracle's CPU-baseline sample (about ten seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hardware-rate", action="store_true")
    ap.add_argument("--cpu-full-solve", action="store_true",
                    help="also time one whole solve of the workload on the CPU oracle (minutes)")
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[WORKLOAD, "ising_L64_W65536", "ising_L128_W16384", "batched48",
                             "served_poisson20", "paper_schedule_L32", "production_L32"],
                    help="the headline workload (default) or one of the batched, served "
                         "and paper-schedule workloads, each with its own JSON line")
    ap.add_argument("--schedule-stop", choices=["kl", "chebyshev"], default="kl",
                    help="paper_schedule_L32: stop at d_k < 1e-4 (Eq. 6) or d_c < 0.05 (App. A)")
    ap.add_argument("--f-therm", type=int, default=30,
                    help="paper_schedule_L32: thermalisation attempts per walker per bin of w")
    ap.add_argument("--schedule-max-iterations", type=int, default=1000,
                    help="paper_schedule_L32: give up after this many iterations (the update "
                         "counts grow by 1.1 per iteration once the full range is covered)")
    ap.add_argument("--serve-duration", type=float, default=60.0)
    ap.add_argument("--block-sweeps", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serve-max-walkers", type=int, default=1 << 19)
    ap.add_argument("--serve-policy", choices=["fifo", "smallest-first"], default="fifo",
                    help="served_poisson20: admission order of queued requests")
    ap.add_argument("--serve-max-wait", type=float, default=30.0,
                    help="served_poisson20 with smallest-first: a request queued longer than this "
                         "goes first")
    ap.add_argument("--serve-solo-sample", type=int, default=24,
                    help="solve this many of the first requests alone, one per launch, "
                         "for the comparison rate")
    ap.add_argument("--issue-probe", action="store_true",
                    help="measure the issue rate of the sweep's integer instructions (the ALU roof)")
    ap.add_argument("--probe-iterations", type=int, default=16384)
    ap.add_argument("--profile-warm", type=int, default=0,
                    help="unrecorded sweeps before the profiled launch of --profile-pass")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short sweep + calibration copy for rocprofv3 counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the walkers and the histogram of an instance live on a "
              "single device (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1707_00919_amd import Solver

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.issue_probe:
        return bench_issue_probe(args)
    if args.workload == "batched48":
        return bench_batched(args)
    if args.workload == "served_poisson20":
        return bench_served(args)
    if args.workload == "paper_schedule_L32":
        return bench_schedule(args)
    if args.workload == "production_L32":
        return bench_production(args)
    wl = WORKLOADS[args.workload]
    ln_g = exact_ln_g(wl["L"])
    if args.profile_pass:
        profile_pass(Solver, wl, ln_g, warm=args.profile_warm)
        return

    for i in range(args.warmup):
        r = solve(Solver, wl, 100000 + i, args.iter_cap)
        print("warmup step %d: %d iterations, %.2f s" % (i, r["iterations"], r["wall_s"]),
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        r = solve(Solver, wl, 1 + i, args.iter_cap)
        runs.append(r)
        print("step %d: seed %d, %d iterations, ttc %.3f s, wall %.3f s" %
              (i, r["seed"], r["iterations"], r["ttc_s"], r["wall_s"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    attempts = sum(r["attempts"] for r in runs)
    kernel_ms = sum(r["kernel_ms"] for r in runs)
    launches = sum(r["launches"] for r in runs)
    variant_ms = {}
    for r in runs:
        for v, ms in r["variant_ms"].items():
            variant_ms[v] = variant_ms.get(v, 0.0) + ms
    main_variant = max(variant_ms, key=variant_ms.get)
    # the committed counter summary covers the headline shape only
    traffic, traffic_source = traffic_per_launch() if args.workload == WORKLOAD else (
        None, "counters are kept for the headline shape only")
    avg_launch_s = kernel_ms * 1e-3 / launches
    attempts_per_launch = attempts / launches
    achieved = ALU_OPS_PER_ATTEMPT * attempts_per_launch / avg_launch_s
    ttc = [r["ttc_s"] for r in runs]
    errs = []
    if ln_g is not None:
        m = np.ones(wl["L"] ** 2 + 1, dtype=bool)
        m[1] = m[-2] = False
        for r in runs:
            if r["ln_g"] is not None:
                errs.append(float(np.max(np.abs(r["ln_g"][m] - ln_g[m]))))

    out = {
        "metric": METRIC if args.workload == WORKLOAD else
        "spin-flip attempts/s at L=%d, %d walkers; p50/p99 time-to-converged-weights" % (wl["L"], wl["walkers"]),
        "value": attempts / wall,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "L": wl["L"], "walkers": wl["walkers"],
                   "iter_sweeps": wl["iter_sweeps"], "min_flatness": wl["min_flat"],
                   "production_sweeps": wl["prod_sweeps"],
                   "production_therm_sweeps": wl["prod_therm_sweeps"],
                   "therm_sweeps": wl["therm_sweeps"],
                   "seeds": "1..%d" % args.steps},
        "ttc_p50_s": nearest_rank(ttc, 50),
        "ttc_p99_s": nearest_rank(ttc, 99),
        "iterations_p50": nearest_rank([r["iterations"] for r in runs], 50),
        "iterations_max": max(r["iterations"] for r in runs),
        "converged": sum(r["converged"] for r in runs),
        "ln_g_max_abs_err": max(errs) if errs else None,
        "ln_g_note": "with production_therm_sweeps unrecorded sweeps at the final weights before the "
                     "recorded production sweeps; they are counted in value",
        "sweep_kernel_attempts_per_s": attempts / (kernel_ms * 1e-3),
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved / VALU_PEAK_OPS,
            "traffic": traffic,
            "traffic_source": traffic_source,
            "kernel": KERNEL_NAMES[main_variant] + "<%d>" % wl["L"],
            "kernel_time_share": variant_ms[main_variant] / kernel_ms,
            "avg_launch_ms": avg_launch_s * 1e3,
            "launches": launches,
            "ops_per_attempt": ALU_OPS_PER_ATTEMPT,
        },
    }
    if args.workload == WORKLOAD:
        roof, note = chain_roof(attempts / (kernel_ms * 1e-3), wl["walkers"])
        out["roofline_chain"] = roof
        out["roofline_chain_source"] = note
    lds_b = lds_bytes_per_attempt(main_variant, wl["L"])
    lds_rate = lds_b * attempts_per_launch / avg_launch_s
    out["roofline_lds"] = {"achieved": lds_rate / 1e12, "peak": LDS_PEAK_BYTES / 1e12, "unit": "TB/s",
                           "frac": lds_rate / LDS_PEAK_BYTES,
                           "bytes_per_attempt": lds_b}
    if not args.no_hardware_rate and ln_g is not None:
        rate, ms = hardware_rate(Solver, wl, ln_g)
        out["exact_weights_attempts_per_s"] = rate
    if not args.no_cpu_baseline and ln_g is not None:
        sweeps = max(1, int(round(args.cpu_attempts / (wl["walkers"] * wl["L"] ** 2))))
        out["cpu_baseline"] = cpu_baseline(wl, ln_g, sweeps, 2)
        one = cpu_baseline(wl, ln_g, max(1, sweeps // 16), 1, nthreads=1)
        out["cpu_baseline_one_core"] = {"value": one["value"], "unit": one["unit"], "cores": 1,
                                        "sample": one["sample"]}
    if args.cpu_full_solve:
        out["cpu_full_solve"] = cpu_full_solve(wl, args.iter_cap)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
