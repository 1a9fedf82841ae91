"""Host-side tests of the solve engine and the serving loop (no GPU).

  * the engine's C ABI validates options and jobs before touching a device,
    and sizes jobs consistently (size queries need no GPU);
  * the serving loop's continuous batching, admission order, memory budget
    and latency bookkeeping, driven by a simulated engine and clock;
  * the one-at-a-time FIFO baseline against a direct event simulation.
"""
import ctypes
import os

import numpy as np
import pytest

import synth
from paper_2305_18643_amd import serving


@pytest.fixture(scope="module")
def b():
    from paper_2305_18643_amd import _binding as b
    if not os.path.exists(b.LIB_PATH):
        from paper_2305_18643_amd import build
        build.build()
    b.load_library()
    return b


def _job(b, m, orbs=(0, 1, 2, 3)):
    spec = b.JobSpec((m.t, m.U), m.nup, m.ndn, orbs=orbs)
    return spec, spec.c_job(64, 100, 0)


def test_engine_defaults_and_validation(b):
    lib = b.load_library()
    o = b.EngineOpts()
    assert lib.qcm_engine_default_opts(ctypes.byref(o)) == 0
    assert o.prec == b.QCM_FP32V and o.reorth == 1 and o.max_iter == 600 and o.gf_steps == 100
    assert o.max_jobs == 256 and o.tol == 0.0
    need = ctypes.c_size_t(0)
    m = synth.impurity_model(np.random.default_rng(1), 4)
    spec, j = _job(b, m)
    assert lib.qcm_engine_job_bytes(ctypes.byref(o), ctypes.byref(j), ctypes.byref(need)) == 0
    assert need.value > 0
    o2 = b.EngineOpts.from_buffer_copy(o)
    o2.prec = 5
    assert lib.qcm_engine_job_bytes(ctypes.byref(o2), ctypes.byref(j), ctypes.byref(need)) == b.QCM_EARG
    o2 = b.EngineOpts.from_buffer_copy(o)
    o2.gf_steps = 0
    assert lib.qcm_engine_job_bytes(ctypes.byref(o2), ctypes.byref(j), ctypes.byref(need)) == b.QCM_EARG
    # repeated orbital
    spec, j = _job(b, m, orbs=(0, 1, 1))
    assert lib.qcm_engine_job_bytes(ctypes.byref(o), ctypes.byref(j), ctypes.byref(need)) == b.QCM_EARG
    # an up-spin sector beyond the engine's row limit
    big = synth.cluster_4x4()
    spec, j = _job(b, big)
    rc = lib.qcm_engine_job_bytes(ctypes.byref(o), ctypes.byref(j), ctypes.byref(need))
    assert rc == b.QCM_ERANGE and b"row limit" in lib.qcm_last_error()
    # 15 orbitals at half filling are inside it
    spec, j = _job(b, synth.chain(15, nup=7, ndn=8))
    assert lib.qcm_engine_job_bytes(ctypes.byref(o), ctypes.byref(j), ctypes.byref(need)) == 0


def test_engine_create_validation(b):
    lib = b.load_library()
    o, zz = b.engine_opts(prec="fp64", z=synth.omega_grid())
    h = ctypes.c_void_p()
    assert lib.qcm_engine_create(ctypes.byref(o), None, 1 << 20, None, ctypes.byref(h)) == b.QCM_EARG
    assert lib.qcm_engine_create(ctypes.byref(o), ctypes.c_void_p(4096 + 8), 1 << 20, None,
                                 ctypes.byref(h)) == b.QCM_EARG
    assert b"aligned" in lib.qcm_last_error()
    assert lib.qcm_engine_create(ctypes.byref(o), ctypes.c_void_p(4096), 1024, None,
                                 ctypes.byref(h)) == b.QCM_EWORKSPACE
    assert not h.value
    assert lib.qcm_engine_destroy(None) == 0


def test_job_bytes_scale_with_the_sectors(b):
    # footprint: psi (FP64) plus max(ground-state vectors, chain vectors);
    # FP32 vectors take about half of the FP64 footprint for large sectors
    ms = synth.batched_solves(18643, 256)
    by_L = {}
    for m in ms:
        by_L.setdefault(m.L, m)
    last = 0
    for L in sorted(by_L):
        spec = b.JobSpec((by_L[L].t, by_L[L].U), by_L[L].nup, by_L[L].ndn, orbs=range(4))
        b64 = b.batch_bytes([spec], prec="fp64", z=synth.omega_grid())
        b32 = b.batch_bytes([spec], prec="fp32v", z=synth.omega_grid())
        assert b32 < b64
        assert b64 > last
        last = b64
    m = by_L[14]
    d = synth_dim(m)
    spec = b.JobSpec((m.t, m.U), m.nup, m.ndn, orbs=range(4))
    b64 = b.batch_bytes([spec], prec="fp64", gf_steps=100)
    # ten chains per part, three vectors each, both parts, FP64
    du = [_binom(14, m.nup + 1) * _binom(14, m.ndn), _binom(14, m.nup - 1) * _binom(14, m.ndn)]
    chains = 3 * 8 * 10 * sum(du)
    assert chains + 8 * d <= b64 <= 1.05 * (chains + 8 * d) + (64 << 20)


def _binom(n, k):
    from math import comb
    return comb(n, k) if 0 <= k <= n else 0


def synth_dim(m):
    return _binom(m.L, m.nup) * _binom(m.L, m.ndn)


def test_batch_solve_size_is_the_sum(b):
    ms = synth.batched_solves(18643, 12)
    specs = [b.JobSpec((m.t, m.U), m.nup, m.ndn, orbs=range(4)) for m in ms]
    one = [b.batch_bytes([s], prec="fp32v") for s in specs]
    allb = b.batch_bytes(specs, prec="fp32v")
    hdr1 = b.batch_bytes([], prec="fp32v")
    assert allb == hdr1 + sum(x - hdr1 for x in one)


# ---------------------------------------------------------------- serving loop

class FakeClock:
    def __init__(self):
        self.now = 0.0

    def __call__(self):
        return self.now

    def sleep(self, dt):
        self.now += max(dt, 0.0)


class FakeEngine:
    """Jobs need `bytes` of a pool and `rounds` rounds; a round takes dt."""

    def __init__(self, clock, pool, slots, dt=0.001):
        self.clock, self.pool, self.slots, self.dt = clock, pool, slots, dt
        self.used = 0
        self.active = {}
        self.done = []
        self.peak = 0
        self.log = []

    def submit(self, spec):
        if len(self.active) >= self.slots or self.used + spec.bytes > self.pool:
            return False
        self.used += spec.bytes
        self.peak = max(self.peak, self.used)
        self.active[spec.tag] = [spec, spec.rounds]
        self.log.append(spec.tag)
        return True

    def step(self, rounds):
        self.clock.now += self.dt
        for tag in list(self.active):
            self.active[tag][1] -= 1
            if self.active[tag][1] == 0:
                spec, _ = self.active.pop(tag)
                self.used -= spec.bytes
                self.done.append({"tag": tag})
        return len(self.active)

    def poll(self):
        out, self.done = self.done, []
        return out


class Spec:
    def __init__(self, tag, bytes_, rounds):
        self.tag, self.bytes, self.rounds = tag, bytes_, rounds


def test_serve_continuous_batching_and_budget():
    clk = FakeClock()
    eng = FakeEngine(clk, pool=100, slots=4)
    rng = np.random.default_rng(3)
    specs = [Spec(i, int(rng.integers(10, 60)), int(rng.integers(5, 40))) for i in range(40)]
    arr = serving.poisson_arrivals(200.0, 40, seed=9)
    rep = serving.serve(eng, specs, arr, clock=clk, sleep=clk.sleep)
    assert sorted(rep.results) == list(range(40))
    assert eng.peak <= 100
    # admitted strictly in arrival order (lookahead 0)
    assert eng.log == list(range(40))
    # overlapping work: more than one request in flight at some point
    assert rep.max_in_flight > 1
    for t in range(40):
        assert rep.latency[t] >= specs[t].rounds * eng.dt - 1e-12
        assert rep.admitted_at[t] >= arr[t] - 1e-12
    lat = np.array([rep.latency[t] for t in range(40)])
    assert rep.percentile(50) == serving.nearest_rank(lat, 50)
    assert rep.percentile(100) == lat.max()


def test_serve_lookahead_admits_past_a_blocked_head():
    clk = FakeClock()
    eng = FakeEngine(clk, pool=100, slots=8)
    specs = [Spec(0, 70, 50), Spec(1, 60, 5), Spec(2, 10, 5), Spec(3, 10, 5)]
    rep = serving.serve(eng, specs, [0.0, 0.0, 0.0, 0.0], clock=clk, sleep=clk.sleep,
                        lookahead=0)
    assert eng.log == [0, 1, 2, 3]
    clk2 = FakeClock()
    eng2 = FakeEngine(clk2, pool=100, slots=8)
    specs = [Spec(0, 70, 50), Spec(1, 60, 5), Spec(2, 10, 5), Spec(3, 10, 5)]
    rep2 = serving.serve(eng2, specs, [0.0, 0.0, 0.0, 0.0], clock=clk2, sleep=clk2.sleep,
                         lookahead=2)
    assert eng2.log[:3] == [0, 2, 3]
    assert rep2.latency[2] < rep.latency[2]


def test_serve_rejects_a_request_larger_than_the_pool():
    clk = FakeClock()
    eng = FakeEngine(clk, pool=50, slots=2)
    with pytest.raises(RuntimeError):
        serving.serve(eng, [Spec(0, 80, 3)], [0.0], clock=clk, sleep=clk.sleep)


def test_fifo_baseline_matches_event_simulation():
    rng = np.random.default_rng(4)
    s = rng.uniform(0.1, 1.0, 200)
    a = np.cumsum(rng.exponential(0.4, 200))
    lat = serving.fifo_one_at_a_time(s, a)
    # event simulation: one server, first come first served
    t = 0.0
    ref = []
    for ai, si in zip(a, s):
        t = max(t, ai) + si
        ref.append(t - ai)
    assert np.allclose(lat, ref, rtol=0, atol=1e-12)
    # a single FIFO server never finishes a request before its arrival plus service
    assert np.all(lat >= s - 1e-12)


def test_nearest_rank():
    x = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert serving.nearest_rank(x, 50) == 3.0
    assert serving.nearest_rank(x, 99) == 5.0
    assert serving.nearest_rank(x, 20) == 1.0
    assert serving.nearest_rank(x, 21) == 2.0
