"""Host logic of the serving driver (paper_2410_04001_amd/serving.py) on the
CPU: the Poisson replay submits every request no earlier than its arrival
time, in arrival order, polls until all have completed and reports the wall
time from the first arrival to the last completion; latency_summary's
percentiles and rates follow from the completion records.  The engine is a
stand-in with one FIFO server of fixed service time on the engine's own
clock (lrnr_srv_clock, a host function of liblrnr.so)."""
import types

import numpy as np
import pytest

from paper_2410_04001_amd import serving


class FifoEngine:
    """submit / poll / take_done with the engine's record fields; requests
    are served one at a time, service_s each, in submission order."""

    def __init__(self, service_s):
        self.service = service_s
        self.free_at = 0.0
        self.pending = []      # submitted, not yet delivered
        self.finished = []     # completed, not yet taken
        self.submitted = []    # (id, arrival, clock at submission)

    def submit(self, req, arrival=None):
        now = serving.clock()
        arrival = now if arrival is None else float(arrival)
        admitted = max(arrival, self.free_at)
        self.free_at = admitted + self.service
        req.record = {"id": req.id, "arrival": arrival, "admitted": admitted,
                      "done": self.free_at, "model": 0, "tiles": 1}
        self.pending.append(req)
        self.submitted.append((req.id, arrival, now))

    def poll(self):
        now = serving.clock()
        still = []
        for r in self.pending:
            (self.finished if r.record["done"] <= now else still).append(r)
        self.pending = still
        active = sum(1 for r in still if r.record["admitted"] <= now)
        return len(still) - active, active

    def take_done(self):
        out, self.finished = self.finished, []
        return out


def make_requests(n, seed=0):
    rng = np.random.default_rng(seed)
    return [types.SimpleNamespace(id=i, n=int(rng.integers(1024, 65536)), record=None)
            for i in range(n)]


@pytest.mark.parametrize("rate,service", [(400.0, 0.001), (200.0, 0.008)])
def test_replay_submits_on_time_and_completes_all(rate, service):
    n = 40
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    arrivals -= arrivals[0]
    eng = FifoEngine(service)
    reqs = make_requests(n)
    done, wall = serving.replay(eng, reqs, arrivals, timeout=10.0)
    assert sorted(r.id for r in done) == list(range(n))
    # submitted in arrival order, never before the scheduled arrival
    ids = [s[0] for s in eng.submitted]
    assert ids == list(range(n))
    for (_, arrival, at), a in zip(eng.submitted, arrivals):
        assert at >= arrival
    sched = np.array([s[1] for s in eng.submitted])
    assert np.allclose(np.diff(sched), np.diff(arrivals), atol=1e-9)
    # every latency covers the service time; FIFO completions are ordered
    lat = np.array([r.record["done"] - r.record["arrival"] for r in reqs])
    assert np.all(lat >= service - 1e-9)
    dones = np.array([r.record["done"] for r in reqs])
    assert np.all(np.diff(dones) > 0)
    # wall: first arrival to last completion
    assert wall == pytest.approx(dones.max() - sched[0], abs=1e-9)
    assert wall >= arrivals[-1]


def test_latency_summary_matches_the_records():
    reqs = make_requests(101, seed=3)
    rng = np.random.default_rng(5)
    for i, r in enumerate(reqs):
        a = 0.01 * i
        adm = a + rng.uniform(0, 0.002)
        r.record = {"arrival": a, "admitted": adm, "done": adm + rng.uniform(0.005, 0.02)}
    wall = 2.0
    s = serving.latency_summary(reqs, wall)
    lat = np.array([r.record["done"] - r.record["arrival"] for r in reqs])
    q = np.array([r.record["admitted"] - r.record["arrival"] for r in reqs])
    assert s["requests"] == 101
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert s["mean_ms"] == pytest.approx(lat.mean() * 1e3)
    assert s["queue_p99_ms"] == pytest.approx(np.percentile(q, 99) * 1e3)
    assert s["req_per_s"] == pytest.approx(101 / wall)
    assert s["colloc_pts_per_s"] == pytest.approx(sum(r.n for r in reqs) / wall)
    assert s["p50_ms"] <= s["p99_ms"]
