"""Tile autotuner for the flow and thermal kernels.

The two launches of a step are independent in their tiling, so each is tuned
on its own: every flow tile shape is timed with the default thermal variant and
every thermal variant with the default flow tile, using HIP events around each
launch (pb_profile_steps).  Results are cached per (nx, ny_fluid, ny_solid,
precision) in a JSON file.  Tiling never changes results: per-node arithmetic
is the same for every variant (checked bit for bit by the GPU tests).
"""
import dataclasses
import json
import os

from . import poolboil as pb
from . import presets

FLOW_TILES = [(64, 4), (64, 8), (32, 8), (128, 4), (32, 16), (64, 16)]
THERMAL_VARIANTS = list(range(1, 8))   # config values: strips of 28, 20, 24, 16, 12, 8, 36 rows (0 = by size)
CACHE = os.environ.get("POOLBOIL_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                            "tune_cache.json"))


def _key(nx, nyf, nys, precision):
    return f"{nx}x{nyf}+{nys}:p{precision}"


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def save_cache(c):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(c, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def settle(step, sync, min_s=0.05, chunk=20):
    """Untimed steps (step(chunk), then sync()) until min_s of wall time has
    passed with the GPU busy, and return how many ran.  The GPU's clocks ramp
    up over some 30 ms after an idle spell such as a domain's set-up: on
    4096x2048+64 the first 20 steps after 2 s of idle ran at 195/81 us
    (flow/energy launch) against 181/66 us from about 120 steps on, so a
    timing taken right after set-up measures the ramp."""
    import time
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s:
        step(chunk)
        sync()
        n += chunk
    return n


def _time(spec, steps, warmup):
    dom = presets.make_domain(spec, with_window=False)
    settle(dom.step, dom.sync)
    dom.step(warmup)
    prof = dom.profile_steps(steps)
    dom.close()
    return prof


def tune(nx, nyf, nys, precision=pb.PB_FP32_DEV, steps=30, warmup=5, use_cache=True, log=None):
    """Return dict(tile=(bx, by), thermal_tile=v, flow_ms=..., thermal_ms=...)."""
    key = _key(nx, nyf, nys, precision)
    cache = load_cache() if use_cache else {}
    if key in cache:
        r = cache[key]
        r["tile"] = tuple(r["tile"])
        return r
    base = dict(nx=nx, nyf=nyf, nys=nys, superheat=0.1, precision=precision, steps=steps + warmup)
    flow = {}
    for tile in FLOW_TILES:
        flow[tile] = _time(presets.JobSpec(tile=tile, **base), steps, warmup)["flow_ms"]
        if log:
            log(f"autotune {key} flow tile {tile}: {flow[tile]:.4f} ms")
    best_tile = min(flow, key=flow.get)
    therm = {}
    for v in THERMAL_VARIANTS:
        therm[v] = _time(presets.JobSpec(tile=best_tile, thermal_tile=v, **base), steps, warmup)["thermal_ms"]
        if log:
            log(f"autotune {key} thermal variant {v}: {therm[v]:.4f} ms")
    best_v = min(therm, key=therm.get)
    r = dict(tile=best_tile, thermal_tile=best_v, flow_ms=flow[best_tile], thermal_ms=therm[best_v],
             flow_all={f"{a}x{b}": v for (a, b), v in flow.items()}, thermal_all={str(k): v for k, v in therm.items()})
    if use_cache:
        cache = load_cache()
        cache[key] = dict(r, tile=list(best_tile))
        save_cache(cache)
    return r


def time_batch(specs, steps, warmup, steps_per_graph, persistent_blocks=0):
    """Wall time per step (ms) of the domains of specs stepped as one batch:
    warmup steps, then steps timed, graph replay of steps_per_graph; with
    persistent_blocks > 0 the launches' grids are capped at that many blocks."""
    import time
    doms = [presets.make_domain(s, with_window=False) for s in specs]
    try:
        b = pb.Batch(doms, steps_per_graph=steps_per_graph, persistent_blocks=persistent_blocks)
        try:
            settle(b.step, lambda: [dm.sync() for dm in doms])
            b.step(warmup)
            for dm in doms:
                dm.sync()
            t0 = time.perf_counter()
            b.step(steps)
            for dm in doms:
                dm.sync()
            return (time.perf_counter() - t0) / steps * 1e3
        finally:
            b.close()
    finally:
        for dm in doms:
            dm.close()


def tune_batch(specs, steps=300, warmup=50, steps_per_graph=100, log=None):
    """Tile shapes for a batch of domains stepped together (a job mix): every
    flow tile shape timed with the default thermal variant, then every thermal
    variant with the best flow tile, each as the wall time per step of the
    whole batch (graph replay, as the server runs it).  Small and ragged
    domains favour other shapes than one large domain.  Returns
    dict(tile=(bx, by), thermal_tile=v, ms_per_step=..., all=...)."""
    specs = list(specs)

    def with_tiles(tile, tv):
        return [dataclasses.replace(s, tile=tile, thermal_tile=tv) for s in specs]

    flow = {}
    for tile in FLOW_TILES:
        flow[tile] = time_batch(with_tiles(tile, 0), steps, warmup, steps_per_graph)
        if log:
            log(f"autotune batch of {len(specs)}: flow tile {tile}: {flow[tile]:.4f} ms/step")
    best_tile = min(flow, key=flow.get)
    therm = {}
    for v in THERMAL_VARIANTS:
        therm[v] = time_batch(with_tiles(best_tile, v), steps, warmup, steps_per_graph)
        if log:
            log(f"autotune batch of {len(specs)}: thermal variant {v}: {therm[v]:.4f} ms/step")
    best_v = min(therm, key=therm.get)
    return dict(tile=best_tile, thermal_tile=best_v, ms_per_step=therm[best_v],
                all={f"{a}x{b}/0": t for (a, b), t in flow.items()} | {f"{best_tile[0]}x{best_tile[1]}/{v}": t
                                                                        for v, t in therm.items()})
