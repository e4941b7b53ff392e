"""Benchmark: site-update attempts/s of the octahedron model with DTr on one MI355X.

Default workload: one L = 2^17 lattice (2^34 sites, 4 GiB bit-packed) from the
flat zig-zag surface, DTrDB (device-level DTr, block-level single-hit dead
border with delayed borders), 256 x 256-site device domains, TC=1,1 (8 x 8-site
thread cells), p = 0.95, q = 0.05.  One step = one MCS (2^34 update attempts:
4 device-step launches) + the exact W^2 measurement + the height
autocorrelation C_h(t, s) against a snapshot taken after warm-up (one fused
measurement pass).

Prints ONE JSON line.  `value` is attempts/s over the timed steps (inputs
resident in HBM); `roofline` reports the device-step kernel, timed with HIP
events on the stream it runs on; `cpu_baseline` times the CPU oracle (the DTr
emulation) on a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CUS, SIMDS_PER_CU = 256, 4
CLOCK_GHZ = 2.4
# VALU issue peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (32-bit integer lane ops)
VALU_PEAK_GOPS = CUS * SIMDS_PER_CU * 16 * CLOCK_GHZ


# Counters of the benchmark's device-step kernel, per launch, from rocprofv3
# runs of the commands in profiles/step_kernel_L131072_DTrDB.md (one counter
# group per run): HBM bytes from FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch), scaled by what the same counters read for the 4 GiB lattice copy
# in the same runs (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00), and the SQ / GRBM
# counters behind rocprofv3's VALUBusy, LdsUtil and LDSBankConflict.  Valid
# only for the device sources they were taken on (hash of the files below);
# otherwise the bench reports them as null.
DEVICE_SOURCES = ("paper_1705_01022_amd/csrc/kernels.hpp", "paper_1705_01022_amd/csrc/db_rows.hpp",
                  "paper_1705_01022_amd/csrc/okpz.hip", "paper_1705_01022_amd/csrc/philox.hpp",
                  "paper_1705_01022_amd/csrc/internal.hpp")
MEASURED = {"sources": "db81be07e6f37fc1", "workload": "L131072",
            # per launch of step_db_rows_kernel<true, 4, 8, 3>, averages of 12 dispatches
            "FETCH_SIZE_KiB": 922611.0, "WRITE_SIZE_KiB": 1584208.0,
            "SQ_INSTS_VALU": 2.69274e9, "SQ_ACTIVE_INST_VALU": 2.69274e9, "SQ_INSTS_SALU": 1.87680e9,
            "SQ_INSTS_LDS": 5.85401e8, "SQ_LDS_IDX_ACTIVE": 2.47391e9, "SQ_LDS_BANK_CONFLICT": 8.60797e8,
            "SQ_WAIT_INST_LDS": 3.21385e9,
            # GRBM_GUI_ACTIVE summed over the 8 XCDs, divided by 8: the dispatch's GPU cycles
            "GRBM_GUI_ACTIVE": 108021000.0 / 8, "launch_ms": 5.7300}


def device_sources_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in DEVICE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(workload: str):
    """The stored per-launch counters, or None if they were taken on other
    sources or another workload."""
    if workload != MEASURED["workload"] or device_sources_hash() != MEASURED["sources"]:
        return None
    return MEASURED


def counter_rates(m: dict, launch_s: float, wave_attempts: float) -> dict:
    """Rates against the chip from stored per-launch counters (rocprofv3's
    derived-metric definitions; CU_NUM = 256, GRBM_GUI_ACTIVE = GPU cycles of
    the dispatch):
      valu_busy       = SQ_ACTIVE_INST_VALU / (CU_NUM x GRBM_GUI_ACTIVE)
                        (quad-cycles of VALU work per SIMD-quad-cycle: 1 = every
                        SIMD issues a VALU instruction every 4 cycles)
      lds_util        = SQ_LDS_IDX_ACTIVE / (CU_NUM x GRBM_GUI_ACTIVE)
      lds_bank_conflict_frac = SQ_LDS_BANK_CONFLICT / (CU_NUM x GRBM_GUI_ACTIVE)
                        (share of the LDS's cycles lost to bank conflicts)
      lds_conflicts_per_access = SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)
      hbm_measured_frac = (FETCH x 2.00 + WRITE x 1.00) bytes / launch time / 8 TB/s
    plus instruction counts per wave-attempt (64 update attempts)."""
    gui = m["GRBM_GUI_ACTIVE"]
    traffic = 1024.0 * (m["FETCH_SIZE_KiB"] * 2.00 + m["WRITE_SIZE_KiB"] * 1.00)
    return {
        "valu_busy": m["SQ_ACTIVE_INST_VALU"] / (CUS * gui),
        "lds_util": m["SQ_LDS_IDX_ACTIVE"] / (CUS * gui),
        "lds_bank_conflict_frac": m["SQ_LDS_BANK_CONFLICT"] / (CUS * gui),
        "lds_conflicts_per_access": m["SQ_LDS_BANK_CONFLICT"] / (m["SQ_LDS_IDX_ACTIVE"] - m["SQ_LDS_BANK_CONFLICT"]),
        "valu_insts_per_wave_attempt": m["SQ_INSTS_VALU"] / wave_attempts,
        "salu_insts_per_wave_attempt": m["SQ_INSTS_SALU"] / wave_attempts,
        "lds_insts_per_wave_attempt": m["SQ_INSTS_LDS"] / wave_attempts,
        "lds_conflict_cycles_per_wave_attempt": m["SQ_LDS_BANK_CONFLICT"] / wave_attempts,
        "traffic_bytes": traffic,
        "hbm_measured_GBs": traffic / launch_s / 1e9,
        "hbm_measured_frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS,
        "counter_launch_ms": m["launch_ms"],
        "gpu_clock_GHz": gui / (m["launch_ms"] * 1e-3) / 1e9,
    }


def ops_per_attempt(scheme: int, cell: int, accept: bool) -> float:
    """A hand-counted model (kept for comparison with the measured counters):
    32-bit VALU issue slots one update attempt needs -- its share of a
    Philox4x32-10 block (100 slots: 10 rounds of two quarter-rate 32x32->64
    multiplies and two 3-input XORs) for an F-bit field, plus field extraction
    (1), site selection (4 for a fixed cell grid, 8 with the per-round cell
    shift), word/bit addressing (5), reading the four slopes (6), the decision
    (1, or 5 with an acceptance draw) and the flip masks (3)."""
    sites = cell * cell if scheme == 1 else cell * cell // 4
    s_bits = max(0, sites.bit_length() - 1)
    if accept:
        F = 1 << (s_bits + 8 - 1).bit_length()
    else:
        F = 1 << (max(s_bits, 1) - 1).bit_length()
    rng = 100.0 * F / 128.0
    select = 4 if scheme == 0 else 8
    return rng + 1 + select + 5 + 6 + (5 if accept else 1) + 3

WORKLOADS = {
    # name: (L, D, C, scheme, p, q, label)
    "L131072": (1 << 17, 256, 8, 1, 0.95, 0.05,
                "octahedron L=131072 (4 GiB packed), DTrDB, D=256x256, TC=1,1, p=0.95 q=0.05"),
    "L4096": (4096, 256, 8, 0, 1.0, 0.0,
              "octahedron L=4096 (4 MiB packed), DTrDT, D=256x256, TC=1,1, p=1 q=0"),
    "L64": (64, 16, 8, 0, 1.0, 0.0, "octahedron L=64, DTrDT, D=16x16, TC=1,1, p=1 q=0"),
}
SCHEME_NAME = {0: "DTrDT", 1: "DTrDB", 2: "DTrDTr"}


def _cpu_window_worker(job):
    """One worker of the CPU baseline: the oracle's DTr emulation of MCS
    m = 0, 1, ... on its own flat window (8 x 8 tiles) of the lattice, for
    about budget_s seconds.  Returns (attempts, seconds)."""
    L, D, C, scheme, p, q, budget_s, k = job
    import oracle

    tiles = 8
    W = min(L, tiles * 2 * D)
    off = (k * W) % L  # disjoint windows along the diagonal
    window = (off, off, W, W)
    emu = oracle.Emu(L=L, Dx=D, Dy=D, Cx=C, Cy=C, scheme=scheme, p=p, q=q, seed=1, stream=0)
    attempts, m, el = 0, 0, 0.0
    while el < budget_s and m < 64:
        s, valid = oracle.init_flat_window(L, window)
        t0 = time.perf_counter()
        if L == W:
            attempts += emu.mcs(s, m)
        else:
            attempts += emu.mcs_window(s, valid, window, m)
        el += time.perf_counter() - t0
        m += 1
    return attempts, el, m


def cpu_baseline(L, D, C, scheme, p, q, budget_s=15.0, workers=None):
    """Time the oracle's DTr emulation (unchanged, one process per core) on
    windows of 8 x 8 tiles of the same lattice (same global tile ids and random
    streams), counting the attempts of the domains wholly inside each window.
    Must run before anything in this process touches the GPU (it forks)."""
    import multiprocessing as mp

    if workers is None:
        workers = max(1, min(16, os.cpu_count() or 1))
    jobs = [(L, D, C, scheme, p, q, budget_s, k) for k in range(workers)]
    t0 = time.perf_counter()
    if workers == 1:
        res = [_cpu_window_worker(jobs[0])]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_cpu_window_worker, jobs)
    wall = time.perf_counter() - t0
    attempts = sum(r[0] for r in res)
    busy = max(r[1] for r in res)  # the workers' timed emulation, concurrent
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    W = min(L, 8 * 2 * D)
    return {"value": attempts / busy, "unit": "attempts/s", "cores": workers, "kind": "oracle",
            "cpu": model, "host_cpus": os.cpu_count(),
            "sample": "DTr emulation of the oracle, %d processes, each MCS 0..%d on its own flat %dx%d-site "
                      "window (8 x 8 tiles) of the L=%d lattice; %d attempts in %.1f s of concurrent emulation "
                      "(%.1f s wall with window set-up)"
                      % (workers, max(r[2] for r in res) - 1, W, W, L, attempts, busy, wall)}


def batched_comparison(okpz, n_batched=200, n_plain=4, tune_mcs=10):
    """The batched workload (512 realisations, L in {256..2048}, (1,0) or
    (1/2,1/2), DTrDT, D = min(256, L/2), TC=1,1): one persistent launch per
    run (graph-captured, launch shape autotuned) against the plain path that
    runs one lattice per launch (okpz_run, 4 device-step launches per MCS)."""
    from workloads import batched_composition

    comp = batched_composition(512, 1)
    b = okpz.Batch()
    lats = [b.lattice(c.L, c.Dx, c.Dy, c.Cx, c.Cy, c.scheme, seed=1, stream=c.stream) for c in comp]
    P, Q = [c.p for c in comp], [c.q for c in comp]
    sites = sum(c.L * c.L for c in comp)
    n = len(comp)
    tuned = b.tune([tune_mcs] * n, P, Q)
    b.sync()
    b.timing(True)
    t0 = time.perf_counter()
    b.run([n_batched] * n, P, Q)
    b.sync()
    el_b = time.perf_counter() - t0
    gpu_ms = b.get_timing()["ms"]
    b.timing(False)
    # measuring the whole ensemble: one batched pass (W^2, C_h, C_s of every
    # member in three launches) against one pass per member
    b.snapshot()
    b.observe(with_autocorr=True)  # warm-up
    t0 = time.perf_counter()
    b.observe(with_autocorr=True)
    el_ob = time.perf_counter() - t0
    t0 = time.perf_counter()
    for lat in lats:
        lat.observe(with_autocorr=True)
    el_ol = time.perf_counter() - t0
    t0 = time.perf_counter()
    for lat, c in zip(lats, comp):
        lat.run(n_plain, c.p, c.q)
    b.sync()
    el_p = time.perf_counter() - t0
    b.close()
    batched = sites * n_batched / el_b
    plain = sites * n_plain / el_p
    best = tuned["best"]
    return {"workload": "512 realisations, L uniform in {256,512,1024,2048}, (p,q)=(1,0)|(1/2,1/2), "
                        "DTrDT, D=min(256,L/2), TC=1,1",
            "sites": sites, "batched_attempts_per_s": batched, "batched_mcs": n_batched,
            "batched_kernel_ms": gpu_ms, "plain_attempts_per_s": plain, "plain_mcs": n_plain,
            "batched_over_plain": batched / plain,
            "launch_shape": {"threads": best[0], "grid_fraction": best[1], "graph": best[2]},
            "tuner_ms": {"%d/%.2f/%s" % k: v for k, v in tuned["times_ms"].items()},
            "observe_all_ms": {"batched": 1e3 * el_ob, "per_member": 1e3 * el_ol}}


def config2_comparison(okpz, n_batched=100, n_plain=20):
    """The L = 4096 workload (DTrDT, 256 x 256-site domains, TC=1,1, p=1,
    q=0): its 64 realisations (streams 0..63, seed 1) as one batch against one
    lattice on the plain path (okpz_run, 4 device-step launches per MCS).
    The 4 MiB lattices are cache-resident, so only attempts/s is reported."""
    L, D, C = 4096, 256, 8
    b = okpz.Batch()
    for st in range(64):
        b.lattice(L, D, D, C, C, okpz.BLOCK_DT, seed=1, stream=st)
    n = 64
    b.run([2] * n, [1.0] * n, [0.0] * n)
    b.sync()
    t0 = time.perf_counter()
    b.run([n_batched] * n, [1.0] * n, [0.0] * n)
    b.sync()
    el_b = time.perf_counter() - t0
    b.close()
    with okpz.Lattice(L, D, D, C, C, okpz.BLOCK_DT, seed=1, stream=0) as lat:
        lat.run(2, 1.0, 0.0)
        lat.sync()
        t0 = time.perf_counter()
        lat.run(n_plain, 1.0, 0.0)
        lat.sync()
        el_p = time.perf_counter() - t0
    batched = 64 * L * L * n_batched / el_b
    plain = L * L * n_plain / el_p
    return {"workload": "L=4096 (4 MiB packed), DTrDT, D=256x256, TC=1,1, p=1 q=0; 64 realisations "
                        "(streams 0..63) as one batch vs one lattice on the plain path",
            "batched_attempts_per_s": batched, "batched_mcs": n_batched,
            "plain_attempts_per_s": plain, "plain_mcs": n_plain, "batched_over_plain": batched / plain}


def _serve_window(okpz, reqs, time_scale=1.0, chunk_mcs=64):
    """Replay the requests' arrival times (scaled) against a fresh server and
    return per-request latencies and the throughput of the window."""
    srv = okpz.Server(chunk_mcs=chunk_mcs)
    t0 = time.perf_counter()
    for r in reqs:
        wait = r.arrival * time_scale - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        srv.submit(r.L, r.Dx, r.Dy, r.Cx, r.Cy, r.scheme, 1, r.rid, r.n_mcs, r.p, r.q)
    # collect results as they finish (a line every 25 finished requests)
    res, reported, t_end = [], 0, time.perf_counter() + 1200.0
    while len(res) < len(reqs) and time.perf_counter() < t_end:
        time.sleep(0.2)
        res += srv.poll(len(reqs) + 8)
        if len(res) >= reported + 25:
            reported = len(res) - len(res) % 25
            print("bench: served %d of %d requests" % (len(res), len(reqs)), file=sys.stderr, flush=True)
    srv.drain(60.0)
    res += srv.poll(len(reqs) + 8)
    st = srv.stats()
    srv.close()
    assert len(res) == len(reqs) and all(x["status"] == 0 for x in res)
    lat = sorted(x["t_finish"] - x["t_submit"] for x in res)
    span = max(x["t_finish"] for x in res) - min(x["t_submit"] for x in res)
    attempts = sum(r.L * r.L * r.n_mcs for r in reqs)
    import numpy as np

    return {"requests": len(reqs), "attempts_per_s": attempts / span, "span_s": span,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "ticks": st["ticks"], "max_members": st["max_members"],
            "offered_req_per_s": 1.0 / (time_scale * (reqs[-1].arrival / len(reqs)))}


def served_comparison(okpz, n_requests=200, plain_mcs=20):
    """The serving workload (Poisson arrivals at 200/s, L = 2^U{9..13}, 10^3 or
    10^4 MCS, p ~ U[0.5,1], q = 1-p, DTrDB, D = min(256, L/2), TC=1,1): a
    bounded window of the first requests replayed in real time (overloaded by
    construction), then the same requests at about 70 % of the measured
    capacity; against the plain path (each request alone, one lattice per
    launch), timed on plain_mcs MCS of every request."""
    from workloads import serving_requests

    reqs = serving_requests(2000, 200.0, 1)[:n_requests]
    over = _serve_window(okpz, reqs)
    per_req = sum(r.L * r.L * r.n_mcs for r in reqs) / len(reqs)
    capacity = over["attempts_per_s"] / per_req  # requests/s
    target = 0.7 * capacity
    scale = (reqs[-1].arrival / len(reqs)) * target
    at70 = _serve_window(okpz, reqs, time_scale=1.0 / scale)
    t_plain, a_plain = 0.0, 0
    for r in reqs:
        with okpz.Lattice(r.L, r.Dx, r.Dy, r.Cx, r.Cy, r.scheme, seed=1, stream=r.rid) as lat:
            lat.run(1, r.p, r.q)
            lat.sync()
            t0 = time.perf_counter()
            lat.run(plain_mcs, r.p, r.q)
            lat.sync()
            t_plain += time.perf_counter() - t0
            a_plain += r.L * r.L * plain_mcs
    plain = a_plain / t_plain
    return {"workload": "serving: first %d requests of a Poisson stream at 200/s, L=2^U{9..13}, "
                        "MCS in {1e3,1e4}, p~U[0.5,1], q=1-p, DTrDB, D=min(256,L/2), TC=1,1" % n_requests,
            "overload": over, "at_70pct_capacity": at70, "capacity_req_per_s": capacity,
            "plain_attempts_per_s": plain, "plain_mcs_per_request": plain_mcs,
            "served_over_plain": over["attempts_per_s"] / plain}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="L131072", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-served", action="store_true", help="skip the serving window")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-config2", action="store_true", help="skip the L=4096 batch-vs-plain comparison")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the benchmark runs on exactly one GPU (the lattice and its kernels live on one "
              "MI355X; sharding across GPUs is a design, not an implementation); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one process only", file=sys.stderr)
        sys.exit(2)

    L, D, C, scheme, p, q, label = WORKLOADS[args.workload]
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the baseline forks worker processes
        print("bench: CPU oracle baseline (about %.0f s)" % args.cpu_budget, file=sys.stderr, flush=True)
        cpu = cpu_baseline(L, D, C, scheme, p, q, args.cpu_budget)

    import paper_1705_01022_amd as okpz

    print("bench: workload %s, warmup %d, steps %d" % (args.workload, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    lat = okpz.Lattice(L, D, D, C, C, scheme, seed=1, stream=0)
    lat.run(args.warmup, p, q)
    lat.snapshot()
    lat.sync()
    print("bench: warm-up done", file=sys.stderr, flush=True)

    lat.timing(True)
    lat.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lat.run(1, p, q)
        mo, ac = lat.observe(True)
    lat.sync()
    elapsed = time.perf_counter() - t0
    tm = lat.get_timing()
    lat.timing(False)
    print("bench: timed %d steps in %.3f s (W^2=%.6f, C_h=%.6f)" % (args.steps, elapsed, mo["w2"],
                                                                   ac["c_h"]),
          file=sys.stderr, flush=True)

    sites = L * L
    attempts = args.steps * sites
    value = attempts / elapsed
    step_avg_s = tm["step_ms"] / tm["step_launches"] / 1e3
    # one device step moves the active quarter of the lattice in and out once:
    # algorithmic bytes = 2 * (L^2/4 sites * 2 bits / 8) = L^2 / 8
    bytes_per_launch = sites / 8
    attempts_per_launch = sites / 4
    accept = not (p in (0.0, 1.0) and q in (0.0, 1.0))
    ops = ops_per_attempt(scheme, C, accept)
    alu_model = attempts_per_launch * ops / step_avg_s / 1e9
    cells = (D // C) * (D // C)
    cpt = max(1, cells // 256)
    if scheme == 1 and cpt in (2, 4) and C == 8 and D in (128, 256):
        kernel_name = "step_db_rows_kernel<accept=%s, %d cells/lane, D=%d, C=%d> (%s)" % (
            accept, cpt, D, C, SCHEME_NAME[scheme])
    elif scheme == 1 and cpt >= 2 and D // C <= 64:
        kernel_name = "step_db_columns_kernel<accept=%s, %d cells/lane> (%s)" % (accept, cpt, SCHEME_NAME[scheme])
    else:
        kernel_name = "step_kernel<%s, accept=%s, %d cells/lane>" % (SCHEME_NAME[scheme], accept, cpt)
    hbm_achieved = bytes_per_launch / step_avg_s / 1e9
    ctr = measured_counters(args.workload)
    rates = counter_rates(ctr, step_avg_s, attempts_per_launch / 64) if ctr else None
    line = {
        "metric": "site-update attempts/s",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": label,
            "L": L, "dom": [D, D], "cell": [C, C], "scheme": SCHEME_NAME[scheme], "p": p, "q": q,
            "step": "1 MCS (L^2 attempts, 4 device-step launches) + exact W^2 and C_h(t,s) in one pass",
            "parallelism": "single GPU",
        },
        # HBM roofline of the device-step kernel: algorithmic bytes (each
        # launch reads and writes the active quarter of the lattice once, 0.5 B
        # per attempt) over its mean launch time (HIP events on the lattice's
        # stream), against 8 TB/s.  The kernel is bound by instruction issue and
        # LDS, not by HBM: the counter-derived rates beside it say how busy
        # those units are (valid for the sources the counters were taken on).
        "roofline": {
            "kernel": kernel_name,
            "bound": "hbm",
            "achieved": hbm_achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_achieved / HBM_PEAK_GBS,
            "traffic": rates["traffic_bytes"] if rates else None,
            "traffic_unit": "B/launch (HBM, rocprofv3 FETCH_SIZE x2.00 + WRITE_SIZE x1.00)",
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": step_avg_s * 1e3,
            "launches": tm["step_launches"],
            "counters": rates,
            "alu_model": {"ops_per_attempt": ops, "achieved_Gops": alu_model, "peak_Gops": VALU_PEAK_GOPS,
                          "alu_model_frac": alu_model / VALU_PEAK_GOPS,
                          "note": "hand-counted op model, not a measurement"},
        },
        "kernel_attempts_per_s": attempts_per_launch / step_avg_s,
        "measure_ms_per_step": tm["measure_ms"] / max(1, args.steps),
        "paper_context": {"value": 9e9, "unit": "attempts/s",
                          "hardware": "Kepler GTX Titan Black / Tesla K80, DTrDB, L=2^16",
                          "cpu_sequential": 5.5e7, "cpu_parallel_12_threads": 2.8e8,
                          "cpu_hardware": "Intel i7-4930k",
                          "paper_speedup_vs_one_socket": 30, "paper_speedup_vs_sequential": ">=180",
                          "this_value_over_paper_gpu": value / 9e9},
    }
    lat.close()
    if not args.no_batched:
        print("bench: batched vs plain", file=sys.stderr, flush=True)
        line["batched"] = batched_comparison(okpz)
    if not args.no_config2:
        print("bench: L=4096 batch vs plain", file=sys.stderr, flush=True)
        line["config2"] = config2_comparison(okpz)
    if not args.no_served:
        print("bench: serving window", file=sys.stderr, flush=True)
        line["served"] = served_comparison(okpz, args.serve_requests)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
