"""Host logic of the continuous-batching server, on the CPU: the device side
is replaced by fakes that record what they are asked to do."""
import pytest

from paper_1911_10747_amd import presets, serve
from paper_1911_10747_amd import poolboil as pb


class FakeDomain:
    def __init__(self, spec):
        self.spec, self.t, self.closed = spec, 0, False

    def step(self, n):
        assert not self.closed
        self.t += n

    def sync(self):
        pass

    def heat_flux(self):
        return dict(q_bottom_mean=float(self.spec.superheat), q_top_mean=0.0, T_w_mean=0.0, n_samples=self.t // 10)

    def close(self):
        self.closed = True


class FakeBatch:
    log = []
    made = 0

    def __init__(self, domains, steps_per_graph=0, persistent_blocks=0, stream=None):
        self.domains = list(domains)
        FakeBatch.made += 1
        FakeBatch.log.append(len(self.domains))

    def add(self, dom):
        assert all(d is not dom for d in self.domains) and not dom.closed
        self.domains.append(dom)
        FakeBatch.log.append(len(self.domains))

    def remove(self, dom):
        assert any(d is dom for d in self.domains) and not dom.closed
        self.domains = [d for d in self.domains if d is not dom]
        FakeBatch.log.append(len(self.domains))

    def step(self, n):
        for d in self.domains:
            d.step(n)

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    made = []

    def make_domain(spec, d=None, use_torch=True, stream=None, with_window=True):
        dom = FakeDomain(spec)
        made.append(dom)
        return dom

    class FakeStream:
        cuda_stream = None

    import types
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(Stream=FakeStream))
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)
    monkeypatch.setattr(presets, "make_domain", make_domain)
    monkeypatch.setattr(pb, "Batch", FakeBatch)
    FakeBatch.log = []
    FakeBatch.made = 0
    return made


def test_every_job_runs_exactly_its_steps_and_budget_holds(fake):
    srv = serve.Server(mem_budget=10**12, max_slots=3, chunk_steps=700, graph_steps=100)
    specs = [presets.JobSpec(nx=64, nyf=64, nys=3, superheat=0.01 * k, steps=s, seed=k)
             for k, s in enumerate([1000, 250, 3000, 1200, 90, 2000])]
    ids = [srv.submit(sp) for sp in specs]
    srv.drain(max_wall_s=30)
    for jid, sp, dom in zip(ids, specs, fake):
        r = srv.result(jid)
        assert r.steps == sp.steps and dom.t == sp.steps and dom.closed
        assert r.q_mean == pytest.approx(sp.superheat)
    assert srv.stats.max_resident == 3
    assert max(FakeBatch.log) <= 3
    assert srv.used == 0
    # one batch for the whole run: jobs joined and left it in place
    assert FakeBatch.made == 1
    assert srv.stats.batch_changes == (len(specs) - 3) + len(specs)


def test_memory_budget_limits_residency(fake):
    one = presets.JobSpec(nx=128, nyf=128, nys=6, superheat=0.1, steps=500)
    srv = serve.Server(mem_budget=10**15, max_slots=10)
    need = srv.footprint(one)
    srv = serve.Server(mem_budget=int(2.5 * need), max_slots=10)
    for k in range(5):
        srv.submit(presets.JobSpec(**{**one.__dict__, "seed": k}))
    srv.drain(max_wall_s=30)
    assert srv.stats.max_resident == 2
    assert srv.stats.retired == 5
    with pytest.raises(ValueError):
        srv.submit(presets.JobSpec(nx=4096, nyf=4096, nys=10, superheat=0.1, steps=10))


def test_latency_percentiles():
    rs = [serve.JobResult(job_id=i, arrival=0.0, finish=float(i + 1)) for i in range(100)]
    st = serve.latency_stats(rs)
    assert st["n"] == 100 and st["p50_s"] == pytest.approx(50.5) and st["p99_s"] == pytest.approx(99.01)


def test_settle_steps_until_the_time_has_passed():
    """autotune.settle runs whole chunks, syncing after each, until min_s of
    wall time has passed, and returns the steps it ran."""
    import time
    from paper_1911_10747_amd import autotune
    calls = []

    def step(n):
        calls.append(("step", n))
        time.sleep(0.004)

    def sync():
        calls.append(("sync", 0))

    t0 = time.perf_counter()
    n = autotune.settle(step, sync, min_s=0.02, chunk=7)
    assert time.perf_counter() - t0 >= 0.02
    steps = [c for c in calls if c[0] == "step"]
    assert n == 7 * len(steps) and len(steps) >= 2
    assert calls[0][0] == "step" and calls[-1][0] == "sync"
    assert all(a[0] == "step" and b[0] == "sync" for a, b in zip(calls[::2], calls[1::2]))
