#!/usr/bin/env python
"""Benchmark of the pool-boiling LBM step on one MI355X.

Default workload: the roofline case, a 4096x2048 fluid domain over a 4096x64
heater, FP32-deviation population storage (populations as deviations from
w_i rho, rho and v in FP32, T in FP64); the flow step computes in FP64, the
energy equation in FP32 increments over FP64 T (with FP64 EOS derivative and
stage-1 differences); one +2% hot spot per 64 heater columns (seed 0),
heater-bottom superheat 0.1 Tc, heat flux sampled every 10 steps.  A step is one full time step of the
method (flow launch + thermal launch [+ flux sample]).  Inputs are resident in
HBM when the timed region starts.

Prints ONE JSON line with MLUPS (fluid-node updates per second), the roofline
of the step against the 8 TB/s HBM peak and the FP64 oracle timed on the host
on a bounded sample of the same workload; beside them the serving legs
(32-job boiling curve, Poisson job stream at three loads) and the smaller
single-domain set-ups.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (nx, nyf, nys, precision, description)
    "roofline": (4096, 2048, 64, 1, "pool boiling 4096x2048 fluid + 4096x64 heater, FP32-deviation populations, "
                                    "FP64 flow/EOS/T, FP32 rho, FP32 energy-equation increments, 1 hot spot per 64 "
                                    "columns, superheat 0.1 Tc"),
    "roofline_fp64": (4096, 2048, 64, 0, "pool boiling 4096x2048 fluid + 4096x64 heater, FP64 populations, "
                                         "1 hot spot per 64 columns, superheat 0.1 Tc"),
    "paper": (400, 400, 20, 1, "pool boiling 400x400 fluid + 400x20 heater, FP32-deviation populations, "
                               "superheat 0.1 Tc"),
}


def algorithmic_bytes(nx, nyf, nys, precision):
    """Bytes the method must move per step: populations read + written
    (9 x 8 x 2 FP64 or 9 x 4 x 2 FP32) and T read + written (16) per fluid
    node, T read + written per heater node."""
    per_fluid = (144 if precision == 0 else 72) + 16
    return per_fluid * nx * nyf + 16 * nx * nys


TRAFFIC_FILES = {"roofline": "pmc_traffic_step_4096x2048_fp32dev.txt"}


def source_sha256():
    """Hash of the kernels and of the host library that builds their work
    lists (both decide what a launch reads and writes)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1911_10747_amd", "csrc")
    h = hashlib.sha256()
    for name in ("pb_kernels.hip", "pb_api.cpp"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_profile(workload):
    """Per-step HBM bytes (both launches) and per-kernel bytes and wavefront
    VALU instructions, measured with rocprofv3 (FETCH_SIZE / WRITE_SIZE scaled
    by a copy-kernel calibration, SQ_INSTS_VALU), if the measurement was taken
    on the current kernel and host-library source (hash match); else None."""
    if workload not in TRAFFIC_FILES:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[workload])
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_sha256():
        return None
    return rec


def _pmc_per_dispatch(path, counter):
    """Per-kernel lists of one counter's value per dispatch from a rocprofv3
    --pmc CSV (rows of one dispatch summed)."""
    import csv
    import re
    per = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"]
            m = re.search(r"(k_\w+<[^>]*>|__amd_rocclr_\w+)", name)
            key = m.group(1) if m else name
            disp = row.get("Dispatch_Id") or row.get("Correlation_Id")
            per.setdefault(key, {}).setdefault(disp, 0.0)
            per[key][disp] += float(row["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def write_traffic_profile(fetch_csv, write_csv, valu_csv, copy_bytes, out, workload, command):
    """Summarise three rocprofv3 --pmc runs of the same command (FETCH_SIZE,
    WRITE_SIZE, SQ_INSTS_VALU; KiB / instructions per dispatch) into the
    per-launch HBM bytes and VALU instructions that load_profile reads.  The
    byte counters are scaled by what they read for the device-to-device copy
    of copy_bytes the command starts with (the runtime's copy kernel), so
    that the copy reads and writes exactly copy_bytes."""
    import numpy as np
    fetch = _pmc_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _pmc_per_dispatch(write_csv, "WRITE_SIZE")
    valu = _pmc_per_dispatch(valu_csv, "SQ_INSTS_VALU")
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the FETCH_SIZE run: run the command with --copy-calibration")
    fk = max(max(fetch[k]) for k in copy)
    wk = max(max(write[k]) for k in copy if k in write)
    cal = dict(copy_bytes=copy_bytes, fetch_kib=fk, write_kib=wk, fetch_factor=copy_bytes / (fk * 1024.0),
               write_factor=copy_bytes / (wk * 1024.0))
    rec = dict(calibration=cal)
    total = 0
    for key in sorted(fetch):
        if not key.startswith(("k_flow", "k_thermal")):
            continue
        rd = float(np.mean(fetch[key])) * 1024.0 * cal["fetch_factor"]
        wr = float(np.mean(write.get(key, [0.0]))) * 1024.0 * cal["write_factor"]
        rec[key] = dict(read_bytes=int(rd), write_bytes=int(wr), total_bytes=int(rd + wr), launches=len(fetch[key]),
                        valu_insts=int(np.mean(valu[key])) if key in valu else None)
        total += int(rd + wr)
    rec.update(roofline_bytes_per_step=total, source_sha256=source_sha256(), workload=workload, command=command,
               method="per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) averaged over each kernel's launches and scaled by "
                      "true/measured for the device-to-device copy of the same run; valu_insts: SQ_INSTS_VALU "
                      "(wavefront VALU instructions) per dispatch, averaged; source_sha256: SHA-256 of "
                      "pb_kernels.hip followed by pb_api.cpp")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def kernel_record(rec, prefix):
    """The profile entry of the kernel whose name starts with prefix."""
    if rec is None:
        return None
    for k, v in rec.items():
        if k.startswith(prefix) and isinstance(v, dict):
            return v
    return None


# VALU issue: 256 CUs x 4 SIMDs at 2.4 GHz, one wavefront-64 instruction every
# 4 cycles per SIMD (16 lanes) -> 614.4 G wavefront instructions/s, for FP64
# (78.6 TFLOP/s of FP64 FMA) and for non-packed FP32 alike (the 157.3 TFLOP/s
# FP32 figure counts packed FP32, two operations per lane, which this build
# does not use).  Measured on the box with independent FMA chains at 3-8 waves
# per SIMD: 0.22-0.24 wave instructions per SIMD-cycle for both.
VALU_PEAK_GINST = 256 * 4 / 4 * 2.4


def per_kernel(nx, nyf, nys, prec, prof, rec):
    """Each launch against the roof that bounds it: k_flow against HBM
    (algorithmic bytes: populations in + out and the T read per fluid node;
    measured bytes from the counters), k_thermal_sweep against VALU issue
    (measured wavefront VALU instructions per launch over the chip's issue
    rate) with its HBM figures beside."""
    flow_alg = ((144 if prec == 0 else 72) + 8) * nx * nyf
    th_alg = 16 * nx * (nyf + nys)
    out = {}
    for name, ms, alg, bound in (("k_flow", prof["flow_ms"], flow_alg, "hbm"),
                                 ("k_thermal_sweep", prof["thermal_ms"], th_alg, "alu")):
        k = {"bound": bound, "ms": round(ms, 5), "algorithmic_bytes": alg,
             "achieved_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
             "frac_hbm": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        kr = kernel_record(rec, name)
        if kr is not None:
            k["traffic"] = kr["total_bytes"]
            k["traffic_gbs"] = round(kr["total_bytes"] / (ms * 1e-3) / 1e9, 1)
            if kr.get("valu_insts"):
                k["valu_ginst_s"] = round(kr["valu_insts"] / (ms * 1e-3) / 1e9, 1)
                k["valu_peak_ginst_s"] = round(VALU_PEAK_GINST, 1)
                k["frac_valu"] = round(kr["valu_insts"] / (ms * 1e-3) / 1e9 / VALU_PEAK_GINST, 4)
        out[name] = k
    return out


def _oracle_pool_domain(nx, nyf, nys, superheat, n_spots, seed):
    """The oracle set up on the standard pool-boiling start (liquid layer at
    the Maxwell density below 40% of the height, heater-bottom superheat with
    +2% hot spots, wall adhesion -0.7 psi_L, top wall -psi_V), constants from
    the oracle's own thermodynamics."""
    from paper_1911_10747_amd import workloads as W
    from oracle import eos, orc
    import numpy as np
    P = dict(W.BASE_PARAMS)
    Tc = eos.critical_temperature(P["a"], P["b"], P["R"])
    Ts = W.T_SAT_OVER_TC * Tc
    rl, rv, _ = eos.maxwell(Ts, P["a"], P["b"], P["R"], P["omega"], Tc)
    P.update(nx=nx, nyf=nyf, nys=nys, Tc=Tc, rho_L=rl, rho_V=rv, rho_S=W.RHO_S_OVER_RHO_L * rl,
             g=W.gravity_for_height(nyf))
    dom = orc.Domain(**P)
    Tb = W.spot_Tb(nx, Ts + superheat * Tc, n_spots, seed)
    gam = np.full(nx, -0.7 * eos.psi(rl, Ts, P["a"], P["b"], P["R"], P["omega"], Tc))
    gtop = np.full(nx, -eos.psi(rv, Ts, P["a"], P["b"], P["R"], P["omega"], Tc))
    dom.set_bc(Ts, Tb, gamma_bot=gam, gamma_top=gtop)
    dom.set_fields(W.layered_rho(nx, nyf, int(round(0.4 * nyf)), rl, rv), W.thermal_init(nx, nys, nyf, Ts, Tb))
    return dom


def cpu_baseline(nx, nyf, nys, steps):
    """The FP64 oracle, as it stands, on `steps` steps of the same workload
    (serial C, one core)."""
    dom = _oracle_pool_domain(nx, nyf, nys, 0.1, max(1, nx // 64), 0)
    t0 = time.perf_counter()
    dom.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=nx * nyf * steps / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"{steps} steps of the full {nx}x{nyf}+{nys} domain, serial FP64 C oracle, one core, "
                       f"{dt:.1f} s")


def _oracle_job_step_time(job):
    """Worker of cpu_jobs_baseline: seconds per oracle step of one job,
    measured over its window of steps (in a process of its own, so the
    jobs' windows run concurrently, one per core)."""
    dom = _oracle_pool_domain(job["nx"], job["nyf"], job["nys"], job["superheat"],
                              max(1, job["nx"] // 64), job["seed"])
    dom.step(2)
    t0 = time.perf_counter()
    dom.step(job["window"])
    return (time.perf_counter() - t0) / job["window"]


def _fifo_schedule(durations, arrivals, cores):
    """Finish times of jobs served first come first served on `cores`
    single-thread workers."""
    import heapq
    free = [0.0] * cores
    heapq.heapify(free)
    finish = []
    for a, dur in sorted(zip(arrivals, durations), key=lambda p: p[0]):
        start = max(a, heapq.heappop(free))
        heapq.heappush(free, start + dur)
        finish.append((a, start + dur))
    return finish


def cpu_jobs_baseline(jobs, window, cores, rates=()):
    """The oracle on a boiling-curve job mix, one single-thread oracle
    process per host core: every job's step time is measured on its own
    domain over `window` steps, all jobs' windows running concurrently on
    `cores` processes, and scaled to the job's full number of steps; the
    jobs are then served first come first served on `cores` workers, all
    submitted at once (jobs/hour, p50/p99 latency) and, for each rate in
    `rates` (jobs/s), on the seeded arrival trace replayed at that rate."""
    import multiprocessing as mp
    import numpy as np
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        per_step = pool.map(_oracle_job_step_time, [dict(j, window=window) for j in jobs], chunksize=1)
    wall = time.perf_counter() - t0
    dur = [ps * j["steps"] for ps, j in zip(per_step, jobs)]

    def served(arrivals):
        fin = _fifo_schedule(dur, arrivals, cores)
        lat = np.array([f - a for a, f in fin])
        span = max(f for _, f in fin) - min(arrivals)
        return dict(jobs_per_hour=round(len(jobs) / span * 3600.0, 3), p50_latency_s=round(float(np.percentile(lat, 50)), 1),
                    p99_latency_s=round(float(np.percentile(lat, 99)), 1))

    out = dict(cores=cores, kind="oracle", all_at_once=served([0.0] * len(jobs)),
               mlups_per_core=round(float(np.mean([j["nx"] * j["nyf"] / ps for ps, j in zip(per_step, jobs)])) / 1e6, 3),
               sample=f"each job's oracle step time measured over {window} steps of its own domain, the {len(jobs)} "
                      f"jobs' windows run concurrently on {cores} single-thread processes ({wall:.1f} s), scaled to "
                      f"the job's full steps")
    if rates and all("arrival" in j for j in jobs):
        base = [j["arrival"] for j in jobs]
        out["trace"] = [dict(rate_jobs_per_s=r, **served([a / r for a in base])) for r in rates]
    return out


def small_configs(log):
    """Single-domain rates of the smaller set-ups (one domain per launch, so
    launch overhead shows): the 100x100 + 100x10 pool in FP64 and the
    400x400 + 400x20 paper-scale pool in both storage modes; 4 hot spots / 6
    hot spots, superheat 0.1 Tc.  (The oracle's rate on the 100x100 pool is in
    the cpu_baseline leg.)  Each is timed with plain launches and as a batch of
    one replayed from captured graphs of 100 steps."""
    from paper_1911_10747_amd import autotune, poolboil as pb, presets
    out = {}
    for name, nx, nyf, nys, prec, spc, steps in (("pool_100x100+10_fp64", 100, 100, 10, 0, 25, 4000),
                                                 ("pool_400x400+20_fp32dev", 400, 400, 20, 1, 67, 4000),
                                                 ("pool_400x400+20_fp64", 400, 400, 20, 0, 67, 4000)):
        spec = presets.JobSpec(nx=nx, nyf=nyf, nys=nys, superheat=0.1, steps=steps, precision=prec,
                               spots_per_columns=spc)
        rates = []
        for graph in (False, True):
            dom = presets.make_domain(spec, with_window=False)
            b = pb.Batch([dom], steps_per_graph=100) if graph else None
            stepper = b if graph else dom
            autotune.settle(stepper.step, dom.sync)
            stepper.step(200)
            dom.sync()
            t0 = time.perf_counter()
            stepper.step(steps)
            dom.sync()
            rates.append(time.perf_counter() - t0)
            if b is not None:
                b.close()
            dom.close()
        out[name] = dict(gpu_mlups=round(nx * nyf * steps / rates[0] / 1e6, 1),
                         gpu_mlups_graph_replay=round(nx * nyf * steps / rates[1] / 1e6, 1),
                         ms_per_step=round(rates[0] / steps * 1e3, 4),
                         ms_per_step_graph_replay=round(rates[1] / steps * 1e3, 4), steps=steps)
        log(f"small configs: {name}: {out[name]['gpu_mlups']} MLUPS, "
            f"{out[name]['gpu_mlups_graph_replay']} with graph replay")
    return out


def _serve_jobs(jobs, precision, batching, max_slots, mem_budget, realtime, time_scale=1.0, tiles=None):
    from paper_1911_10747_amd import presets, serve
    # batched runs take the shapes tuned on the batched mix; a job run alone
    # takes the library's choice for its own size (thermal_tile 0)
    tile, tv = (tiles["tile"], tiles["thermal_tile"]) if (tiles and batching) else ((0, 0), 0)
    srv = serve.Server(mem_budget=mem_budget, max_slots=max_slots, precision=precision, chunk_steps=2000,
                       graph_steps=100 if batching else 0, batching=batching, tile=tile, thermal_tile=tv)
    if realtime:
        res, wall = serve.run_trace(srv, jobs, time_scale=time_scale, max_wall_s=900)
    else:
        t0 = time.perf_counter()
        ids = [srv.submit(presets.JobSpec(nx=j["nx"], nyf=j["nyf"], nys=j["nys"], superheat=j["superheat"],
                                          steps=j["steps"], seed=j["seed"]), arrival=t0) for j in jobs]
        srv.drain(max_wall_s=900)
        wall = time.perf_counter() - t0
        res = [srv.result(i) for i in ids]
    lat = serve.latency_stats(res)
    return dict(jobs=len(res), wall_s=round(wall, 3), jobs_per_hour=round(len(res) / wall * 3600.0, 1),
                p50_latency_s=round(lat["p50_s"], 4), p99_latency_s=round(lat["p99_s"], 4),
                mlups=round(srv.stats.node_updates / wall / 1e6, 1), max_resident=srv.stats.max_resident,
                chunks=srv.stats.chunks, errors=sum(1 for r in res if r.error)), [r.q_mean for r in res]


def serving_legs(log):
    """Boiling-curve jobs: (1) 32 jobs of log-uniform size 128..1024 x 128..512
    (heater 1/20 of the height), superheat U[0.02, 0.30] Tc, 20000 steps, all
    submitted at once; (2) a Poisson stream of 48 jobs, sizes 64..2048 x
    64..1024, 5000-20000 steps, 4 GiB of device memory for resident jobs, at
    three loads relative to the FP32 capacity on these jobs.  FP32-deviation
    continuous batching against FP64 one job at a time, same jobs (the curve
    also FP32 one job at a time, to separate batching from precision), the
    stream replayed at 0.5, 0.8 and 1.2 x the measured FP32 capacity.  The
    curve's batched run takes the tile shapes of the batch autotuner run on its
    job mix (outside the timed legs); the stream's batches take the tuned flow
    tile and the energy strips the library chooses for each batch's total size;
    a job run alone takes the library's choice for its size."""
    import numpy as np
    from paper_1911_10747_amd import workloads as W
    from paper_1911_10747_amd import autotune, presets
    out = {}
    curve = W.batch_jobs(seed=0, n=32, steps=20000)
    specs = [presets.JobSpec(nx=j["nx"], nyf=j["nyf"], nys=j["nys"], superheat=j["superheat"], steps=j["steps"],
                             seed=j["seed"], precision=1) for j in curve]
    tiles = autotune.tune_batch(specs, log=log)
    log(f"serving: batched FP32 tiles: flow {tiles['tile']}, thermal {tiles['thermal_tile']}")
    log("serving: boiling curve, 32 jobs, FP32 batched")
    b32, q32 = _serve_jobs(curve, 1, True, 64, 32 << 30, realtime=False, tiles=tiles)
    # the whole job mix's algorithmic bytes over the batched run's wall clock
    alg = sum(algorithmic_bytes(j["nx"], j["nyf"], j["nys"], 1) * j["steps"] for j in curve)
    b32["hbm_frac_algorithmic"] = round(alg / b32["wall_s"] / 1e9 / HBM_PEAK_GBS, 4)
    log("serving: boiling curve, 32 jobs, FP32 one at a time")
    b32s, _ = _serve_jobs(curve, 1, False, 1, 32 << 30, realtime=False)
    log("serving: boiling curve, 32 jobs, FP64 one at a time")
    b64, q64 = _serve_jobs(curve, 0, False, 1, 32 << 30, realtime=False)
    dq = np.abs(np.array(q32) - np.array(q64)) / np.maximum(np.abs(np.array(q64)), 1e-30)
    out["boiling_curve"] = dict(fp32_batched=b32, fp32_one_at_a_time=b32s, fp64_one_at_a_time=b64,
                                speedup_jobs_per_hour=round(b32["jobs_per_hour"] / b64["jobs_per_hour"], 2),
                                batching_gain_fp32=round(b32["jobs_per_hour"] / b32s["jobs_per_hour"], 2),
                                mean_job_fluid_node_updates=float(np.mean([j["nx"] * j["nyf"] * j["steps"]
                                                                           for j in curve])),
                                heat_flux_rel_diff_median=float(np.median(dq)), heat_flux_rel_diff_max=float(dq.max()),
                                within_3pct=int((dq <= 0.03).sum()))
    out["batched_tiles"] = dict(flow=list(tiles["tile"]), thermal=tiles["thermal_tile"],
                                ms_per_step_curve_mix=round(tiles["ms_per_step"], 4))
    # the same mix with the launches' grids capped (blocks loop over the work
    # lists): 768 blocks hold every flow block the chip runs at once, 3072 one
    # energy wavefront per SIMD slot; 0 = one block per tile
    tuned = [dataclasses.replace(s, tile=tiles["tile"], thermal_tile=tiles["thermal_tile"]) for s in specs]
    grid = {}
    for pblocks in (0, 768, 3072):
        grid[str(pblocks)] = round(autotune.time_batch(tuned, 300, 50, 100, persistent_blocks=pblocks), 4)
        log(f"serving: curve mix, persistent grid {pblocks}: {grid[str(pblocks)]} ms/step")
    out["batched_tiles"]["ms_per_step_by_persistent_grid"] = grid
    # Poisson stream: one job mix (arrival gaps drawn at 1 job/s), replayed at
    # 0.5, 0.8 and 1.2 x the FP32 capacity measured on the same jobs submitted
    # at once.  The resident set changes from chunk to chunk, so the batches
    # take the tuned flow tile and the energy strips the library sizes for
    # each batch.
    stream = W.job_stream(seed=0, n=48, rate_per_s=1.0)
    stiles = dict(tiles, thermal_tile=0)
    log("serving: Poisson stream jobs, FP32 capacity (all submitted at once)")
    cap, _ = _serve_jobs(stream, 1, True, 32, 4 << 30, realtime=False, tiles=stiles)
    cap_per_s = cap["jobs_per_hour"] / 3600.0
    levels = []
    for load in (0.5, 0.8, 1.2):
        rate = load * cap_per_s
        log(f"serving: Poisson stream, 48 jobs at {rate:.2f} jobs/s ({load} x capacity), FP32 continuous batching")
        s32, q32 = _serve_jobs(stream, 1, True, 32, 4 << 30, realtime=True, time_scale=rate, tiles=stiles)
        log(f"serving: Poisson stream, 48 jobs at {rate:.2f} jobs/s, FP64 one at a time")
        s64, q64 = _serve_jobs(stream, 0, False, 1, 4 << 30, realtime=True, time_scale=rate)
        dq = np.abs(np.array(q32) - np.array(q64)) / np.maximum(np.abs(np.array(q64)), 1e-30)
        levels.append(dict(load=load, rate_jobs_per_s=round(rate, 3), fp32_batched=s32, fp64_one_at_a_time=s64,
                           heat_flux_rel_diff_median=float(np.median(dq)), heat_flux_rel_diff_max=float(dq.max()),
                           within_3pct=int((dq <= 0.03).sum())))
    out["poisson_stream"] = dict(jobs=len(stream), mem_budget_gib=4, fp32_capacity=cap,
                                 fp32_capacity_jobs_per_s=round(cap_per_s, 3), levels=levels)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="roofline", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-job-window", type=int, default=10,
                    help="oracle steps timed per job for the CPU jobs/hour baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default="0x0")
    ap.add_argument("--thermal-tile", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the tile autotuner; use --tile/--thermal-tile")
    ap.add_argument("--no-serving", action="store_true", help="skip the boiling-curve / job-stream legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--traffic-profile", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "VALU_CSV"),
                    help="summarise three rocprofv3 --pmc runs of this command into profiles/ (no GPU work)")
    args = ap.parse_args()
    if args.traffic_profile:
        out = os.path.join(ROOT, "profiles", TRAFFIC_FILES[args.workload])
        cmd = ("cd /tmp && timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> -o fetch -- "
               "python3 <repo>/bench.py --no-tune --tile 64x8 --thermal-tile 0 --steps 10 --warmup 2 "
               "--no-cpu-baseline --no-serving --copy-calibration 1024   (and the same with --pmc WRITE_SIZE and "
               "--pmc SQ_INSTS_VALU SQ_WAVES); then python3 <repo>/bench.py --traffic-profile <fetch.csv> "
               "<write.csv> <valu.csv>")
        rec = write_traffic_profile(*args.traffic_profile, 1 << 30, out, WORKLOADS[args.workload][4], cmd)
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU x-slab sharding is design-only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10747_amd import poolboil as pb
    from paper_1911_10747_amd import presets

    nx, nyf, nys, prec, desc = WORKLOADS[args.workload]
    tx, ty = (int(v) for v in args.tile.split("x"))
    thermal_tile = args.thermal_tile
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {n} bytes done", file=sys.stderr, flush=True)
        del src, dst
    tuned = None
    if not args.no_tune:
        from paper_1911_10747_amd import autotune
        tuned = autotune.tune(nx, nyf, nys, prec, use_cache=False,
                              log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        (tx, ty), thermal_tile = tuned["tile"], tuned["thermal_tile"]
    spec = presets.JobSpec(nx=nx, nyf=nyf, nys=nys, superheat=0.1, steps=args.warmup + args.steps, seed=0,
                           precision=prec, tile=(tx, ty), thermal_tile=thermal_tile)
    dom = presets.make_domain(spec)
    dom.flux_window(0, 1 << 62, 10)
    # untimed steps until 50 ms of GPU work have run, so that the clocks have
    # ramped up from the idle of the set-up before the warmup and the timed
    # steps (a short timed run would otherwise measure the ramp)
    from paper_1911_10747_amd import autotune as _at
    settle_steps = _at.settle(dom.step, dom.sync)
    print(f"bench: {args.workload} {nx}x{nyf}+{nys} prec={prec}: {settle_steps} settle steps, warmup {args.warmup}",
          file=sys.stderr, flush=True)
    dom.step(args.warmup)
    dom.profile_reserve(args.steps)     # the timed steps' HIP events, created before the clock starts
    dom.sync()
    torch.cuda.synchronize()
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    prof = dom.profile_steps(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom.sync()
    ms_step = wall / args.steps * 1e3
    mlups = nx * nyf * args.steps / wall / 1e6
    alg = algorithmic_bytes(nx, nyf, nys, prec)
    kern_ms = prof["flow_ms"] + prof["thermal_ms"]
    achieved = alg / (kern_ms * 1e-3) / 1e9
    rec = load_profile(args.workload)
    traffic = rec.get("roofline_bytes_per_step") if rec else None
    kernels = per_kernel(nx, nyf, nys, prec, prof, rec)
    out = {
        "metric": "MLUPS (fused pool-boiling step, fluid-node updates per second) and fraction of HBM peak",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": settle_steps,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec else "f64",
        "data": "synthetic (seeded pool-boiling start: Maxwell liquid layer, +2% heater hot spots)",
        "config": {"workload": desc, "nx": nx, "ny_fluid": nyf, "ny_solid": nys,
                   "storage": "fp32-deviation" if prec else "fp64",
                   "arithmetic": "fp64 flow; fp32 energy-equation increments on fp64 T" if prec else "fp64",
                   "tile": [tx, ty], "thermal_tile": thermal_tile, "autotuned": tuned is not None,
                   "parallelism": "single GPU"},
        "roofline": {
            "bound": "hbm",
            "kernel": "one step = k_flow + k_thermal (algorithmic bytes of the whole step over the summed "
                      "mean launch durations)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # the same bytes over the wall-clock time per step (launch gaps and
            # the heat-flux samples included)
            "achieved_wall": round(alg / (ms_step * 1e-3) / 1e9, 1),
            "frac_wall": round(alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_gbs": round(traffic / (kern_ms * 1e-3) / 1e9, 1) if traffic else None,
            "traffic_frac": round(traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "algorithmic_bytes_per_step": alg,
            "flow_ms": round(prof["flow_ms"], 5),
            "thermal_ms": round(prof["thermal_ms"], 5),
            "kernels": kernels,
        },
    }
    dom.close()
    if not args.no_serving:
        out["serving"] = serving_legs(lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        out["small_configs"] = small_configs(lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        print(f"bench: oracle on {args.cpu_steps} steps", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(nx, nyf, nys, args.cpu_steps)
        if "small_configs" in out:
            out["cpu_baseline"]["pool_100x100+10"] = cpu_baseline(100, 100, 10, 2000)
        if "serving" in out:
            # the same job mixes on the oracle, one single-thread process per
            # host core (at most 16: the host's share for one GPU)
            from paper_1911_10747_amd import workloads as W
            cores = max(1, min(16, len(os.sched_getaffinity(0))))
            sv = out["serving"]
            print(f"bench: oracle jobs/hour on {cores} cores", file=sys.stderr, flush=True)
            curve = cpu_jobs_baseline(W.batch_jobs(seed=0, n=32, steps=20000), args.cpu_job_window, cores)
            rates = [lv["rate_jobs_per_s"] for lv in sv["poisson_stream"]["levels"]]
            stream = cpu_jobs_baseline(W.job_stream(seed=0, n=48, rate_per_s=1.0), args.cpu_job_window, cores,
                                       rates=rates)
            out["cpu_baseline"]["boiling_curve_jobs"] = curve
            out["cpu_baseline"]["poisson_stream_jobs"] = stream
            bc = sv["boiling_curve"]
            bc["cpu_oracle_jobs_per_hour"] = curve["all_at_once"]["jobs_per_hour"]
            bc["cpu_oracle_cores"] = cores
            bc["speedup_vs_cpu_oracle"] = round(bc["fp32_batched"]["jobs_per_hour"] /
                                                curve["all_at_once"]["jobs_per_hour"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
