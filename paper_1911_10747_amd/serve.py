"""Continuous-batching server for boiling-curve jobs.

A job is one pool-boiling run (domain size, heater superheat, number of
steps, seed); its result is the time-mean wall heat flux of Eq. 38 over the
second half of the run, reported with its Jakob number (Eq. 37).

Scheduling.  Resident jobs keep their whole state in HBM and are stepped in
lock-step by one shared launch per kernel (pb_batch), replayed from a
captured HIP graph when a chunk has the full graph length.  Jobs join and
leave that one batch in place (pb_batch_add / pb_batch_remove).  Work proceeds in
chunks: each chunk ends exactly when the first resident job finishes (or
after `chunk_steps`), so every job runs exactly its own number of steps.
While a chunk runs on the GPU the host admits waiting jobs whose device
footprint fits in the memory budget and a free slot; they join at the next
chunk boundary, when finished jobs retire and free their memory.  Per-node
arithmetic does not depend on the mix, so a job's result is bit-identical
whether it ran alone or with others.

Latency = finish time - arrival time (host wall clock).
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import poolboil as pb
from . import presets


@dataclass
class JobResult:
    job_id: int
    q_mean: float = float("nan")
    q_top_mean: float = float("nan")
    T_w_mean: float = float("nan")
    n_samples: int = 0
    Ja: float = float("nan")
    superheat: float = float("nan")
    steps: int = 0
    arrival: float = 0.0
    start: float = 0.0
    finish: float = 0.0
    error: str = ""

    @property
    def latency_s(self):
        return self.finish - self.arrival


@dataclass
class _Job:
    job_id: int
    spec: presets.JobSpec
    arrival: float
    nbytes: int
    dom: object = None
    stream: object = None
    done_steps: int = 0
    start: float = 0.0


@dataclass
class ServerStats:
    chunks: int = 0
    graph_chunks: int = 0
    steps: int = 0
    admitted: int = 0
    retired: int = 0
    max_resident: int = 0
    batch_changes: int = 0        # pb_batch_add / pb_batch_remove calls
    node_updates: float = 0.0
    busy_s: float = 0.0
    occupancy: list = field(default_factory=list)


class Server:
    """Continuous batching over one GPU.

    mem_budget: device bytes available for resident jobs.
    max_slots: maximum number of resident jobs.
    precision: pb.PB_FP32_DEV or pb.PB_FP64 (all jobs of a server share it).
    chunk_steps: upper bound on the steps between scheduling points.
    graph_steps: length of the captured step batch (even; 0 disables graphs).
    batching: False steps each resident job alone (one job at a time when
    max_slots is 1) instead of in shared launches.
    """

    def __init__(self, mem_budget, max_slots=64, precision=pb.PB_FP32_DEV, chunk_steps=1000, graph_steps=100,
                 batching=True, tile=(0, 0), thermal_tile=0, clock=time.perf_counter):
        self.mem_budget = int(mem_budget)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.chunk_steps = int(chunk_steps)
        self.graph_steps = int(graph_steps)
        self.batching = batching
        self.tile, self.thermal_tile = tile, thermal_tile
        self.clock = clock
        self.derived = presets.derived()
        self.h_fg = pb.latent_heat(presets.W.BASE_PARAMS["a"], presets.W.BASE_PARAMS["b"],
                                   presets.W.BASE_PARAMS["R"], presets.W.BASE_PARAMS["omega"], self.derived.Tc,
                                   self.derived.Tsat)
        self.waiting = []
        self.resident = []
        self.results = {}
        self.used = 0
        self.next_id = 0
        self.stats = ServerStats()
        self._batch = None
        self._batch_members = None
        self._inflight = None     # (chunk steps, start time, member jobs) of the chunk on the GPU

    # ------------------------------------------------------------------ API
    def footprint(self, spec):
        return pb.domain_bytes(presets.make_config(self._spec(spec), self.derived))

    def submit(self, spec, arrival=None):
        spec = self._spec(spec)
        nbytes = self.footprint(spec)
        if nbytes > self.mem_budget:
            raise ValueError(f"job needs {nbytes} bytes, budget is {self.mem_budget}")
        jid = self.next_id
        self.next_id += 1
        self.waiting.append(_Job(jid, spec, self.clock() if arrival is None else arrival, nbytes))
        return jid

    def result(self, job_id):
        return self.results.get(job_id)

    def idle(self):
        return not self.waiting and not self.resident and self._inflight is None

    def poll(self):
        """Advance the schedule by one chunk: finish the chunk in flight (if
        any), retire finished jobs, launch the next chunk, and admit waiting
        jobs while it runs.  Returns the ids of jobs finished by this call."""
        finished = self._complete_chunk()
        if not self.resident:
            self._admit()
        self._launch_chunk()
        self._admit()
        return finished

    def drain(self, max_wall_s=None):
        t0 = self.clock()
        while not self.idle():
            self.poll()
            if max_wall_s is not None and self.clock() - t0 > max_wall_s:
                raise TimeoutError("server did not drain in time")

    # ------------------------------------------------------------ internals
    def _spec(self, spec):
        if spec.precision != self.precision or spec.tile != self.tile or spec.thermal_tile != self.thermal_tile:
            spec = presets.JobSpec(**{**spec.__dict__, "precision": self.precision, "tile": self.tile,
                                      "thermal_tile": self.thermal_tile})
        return spec

    def _admit(self):
        while self.waiting and len(self.resident) < self.max_slots:
            job = self.waiting[0]
            if self.used + job.nbytes > self.mem_budget:
                break
            self.waiting.pop(0)
            # each job gets its own stream: its set-up then overlaps the chunk in
            # flight instead of queueing behind the batch on a shared stream
            import torch
            job.stream = torch.cuda.Stream()
            job.dom = presets.make_domain(job.spec, self.derived, stream=job.stream.cuda_stream)
            job.start = self.clock()
            self.used += job.nbytes
            self.resident.append(job)
            self.stats.admitted += 1
            self.stats.max_resident = max(self.stats.max_resident, len(self.resident))

    def _launch_chunk(self):
        if not self.resident:
            return
        n = min([self.chunk_steps] + [j.spec.steps - j.done_steps for j in self.resident])
        t0 = self.clock()
        if self.batching:
            if self._batch is None:
                self._batch = pb.Batch([j.dom for j in self.resident], steps_per_graph=self.graph_steps)
                self._batch_members = {j.job_id for j in self.resident}
            else:
                # admitted jobs join the running batch (pb_batch_add: the work
                # lists change in place, no member waits)
                for j in self.resident:
                    if j.job_id not in self._batch_members:
                        self._batch.add(j.dom)
                        self._batch_members.add(j.job_id)
                        self.stats.batch_changes += 1
            self._batch.step(n)
            if self.graph_steps and n >= self.graph_steps:
                self.stats.graph_chunks += 1
        else:
            for j in self.resident:
                j.dom.step(n)
        self._inflight = (n, t0, list(self.resident))
        self.stats.chunks += 1
        self.stats.steps += n
        self.stats.occupancy.append(len(self.resident))
        self.stats.node_updates += n * sum(j.spec.nx * j.spec.nyf for j in self.resident)

    def _complete_chunk(self):
        if self._inflight is None:
            return []
        n, t0, members = self._inflight
        self._inflight = None
        finished = []
        keep = []
        for j in self.resident:
            if any(j is m for m in members):      # jobs admitted during the chunk did not run it
                j.done_steps += n
            if j.done_steps >= j.spec.steps:
                finished.append(j)
            else:
                keep.append(j)
        # wait for the chunk
        err = {}
        for j in members:
            try:
                j.dom.sync()
            except pb.NonFiniteError as e:
                err[j.job_id] = str(e)
        now = self.clock()
        self.stats.busy_s += now - t0
        for j in list(keep):
            if j.job_id in err:   # a failed job retires early; the others continue
                keep.remove(j)
                finished.append(j)
        for j in finished:
            self._retire(j, now, err.get(j.job_id, ""))
        self.resident = keep
        return [j.job_id for j in finished]

    def _retire(self, j, now, error):
        fl = j.dom.heat_flux()
        d = self.derived
        r = JobResult(job_id=j.job_id, q_mean=fl["q_bottom_mean"], q_top_mean=fl["q_top_mean"],
                      T_w_mean=fl["T_w_mean"], n_samples=fl["n_samples"], superheat=j.spec.superheat,
                      Ja=j.spec.overrides.get("Cv", presets.W.BASE_PARAMS["Cv"]) * j.spec.superheat * d.Tc / self.h_fg,
                      steps=j.done_steps, arrival=j.arrival, start=j.start, finish=now, error=error)
        self.results[j.job_id] = r
        if self._batch is not None and j.job_id in self._batch_members:
            # it leaves the batch; the work already queued for it has run
            # (the chunk was synchronised above), so it can go at once
            self._batch.remove(j.dom)
            self._batch_members.discard(j.job_id)
            self.stats.batch_changes += 1
        j.dom.close()
        j.dom = None
        j.stream = None
        self.used -= j.nbytes
        self.stats.retired += 1


def run_trace(server, jobs, time_scale=1.0, max_wall_s=600.0):
    """Feed a job stream (dicts with 'arrival' seconds and JobSpec fields) to
    the server in real time (arrival times divided by time_scale) and run it
    to completion.  Returns (results list, wall seconds)."""
    clock = server.clock
    t0 = clock()
    pending = sorted(jobs, key=lambda j: j["arrival"])
    ids = []
    i = 0
    while i < len(pending) or not server.idle():
        now = clock() - t0
        while i < len(pending) and pending[i]["arrival"] / time_scale <= now:
            j = pending[i]
            spec = presets.JobSpec(nx=j["nx"], nyf=j["nyf"], nys=j["nys"], superheat=j["superheat"],
                                   steps=j["steps"], seed=j["seed"])
            ids.append(server.submit(spec, arrival=t0 + j["arrival"] / time_scale))
            i += 1
        if server.idle() and i < len(pending):
            time.sleep(max(0.0, min(0.01, pending[i]["arrival"] / time_scale - (clock() - t0))))
            continue
        server.poll()
        if clock() - t0 > max_wall_s:
            raise TimeoutError("trace did not finish in time")
    wall = clock() - t0
    return [server.result(k) for k in ids], wall


def latency_stats(results):
    lat = np.array([r.latency_s for r in results if r is not None])
    return dict(n=int(lat.size), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()))
