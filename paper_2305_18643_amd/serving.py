"""Continuous-batching serving loop over the solve engine (qcm_engine_*).

Requests (ground state + Green-function block of a cluster) arrive at given
times.  The loop admits every request that has arrived, in arrival order,
as soon as the engine has a free slot and enough pool memory for it (the
engine's own admission test), runs one engine round (one Lanczos step of
every admitted solve, in one set of launches), and collects the solves that
completed.  A request's latency runs from its arrival to the poll that
returns its result.

The engine is any object with ``submit(spec) -> bool``, ``step(rounds) ->
n_active`` and ``poll() -> list of results`` (each with a ``tag``), so the
scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeReport:
    latency: dict                      # tag -> seconds (arrival -> result)
    results: dict                      # tag -> engine result
    admitted_at: dict                  # tag -> seconds since start
    wall: float                        # start -> last result
    max_in_flight: int
    rounds: int
    head_blocked: int                  # ticks where the oldest waiting request did not fit
    extra: dict = field(default_factory=dict)

    def percentile(self, q: float) -> float:
        """Nearest-rank percentile of the latencies, q in (0, 100]."""
        lat = np.sort(np.fromiter(self.latency.values(), dtype=float))
        if lat.size == 0:
            return float("nan")
        k = int(np.ceil(q / 100.0 * lat.size)) - 1
        return float(lat[min(max(k, 0), lat.size - 1)])

    def throughput(self) -> float:
        return len(self.latency) / self.wall if self.wall > 0 else float("nan")


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of `count` requests."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def serve(engine, specs, arrivals, *, clock=time.perf_counter, sleep=time.sleep,
          lookahead: int = 0, progress=None, progress_every: int = 100) -> ServeReport:
    """Serve specs[i] arriving at arrivals[i] seconds (non-decreasing).

    lookahead = 0 admits strictly in arrival order (the oldest waiting request
    blocks the others until it fits); lookahead = k also tries the next k
    waiting requests when the oldest does not fit.  progress, if given, is
    called with the number of completed requests after every progress_every
    completions.
    """
    n = len(specs)
    arrivals = np.asarray(arrivals, dtype=float)
    if n != arrivals.shape[0]:
        raise ValueError("one arrival time per request")
    if n and np.any(np.diff(arrivals) < 0):
        raise ValueError("arrival times must be non-decreasing")
    tags = [s.tag for s in specs]
    if len(set(tags)) != n:
        raise ValueError("request tags must be unique")
    arr_of = {t: a for t, a in zip(tags, arrivals)}
    t0 = clock()
    nxt = 0                      # next request not yet arrived
    waiting: list = []           # arrived, not admitted (arrival order)
    latency, results, admitted_at = {}, {}, {}
    in_flight = max_in_flight = rounds = blocked = 0
    last_done = 0.0
    while len(results) < n:
        now = clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            waiting.append(specs[nxt])
            nxt += 1
        # admission: arrival order, optionally looking past a blocked head
        k = 0
        tried = 0
        while k < len(waiting):
            if engine.submit(waiting[k]):
                admitted_at[waiting[k].tag] = clock() - t0
                waiting.pop(k)
                in_flight += 1
                continue
            if k == 0:
                blocked += 1
            tried += 1
            if tried > lookahead:
                break
            k += 1
        max_in_flight = max(max_in_flight, in_flight)
        if in_flight == 0:
            if nxt >= n and not waiting:
                break
            if not waiting:
                # idle until the next arrival
                wait = arrivals[nxt] - (clock() - t0)
                if wait > 0:
                    sleep(wait)
                continue
            raise RuntimeError(f"request {waiting[0].tag} cannot be admitted by an idle engine "
                               "(larger than the pool)")
        engine.step(1)
        rounds += 1
        for r in engine.poll():
            done = clock() - t0
            tag = r["tag"]
            results[tag] = r
            latency[tag] = done - arr_of[tag]
            last_done = done
            in_flight -= 1
            if progress is not None and len(results) % progress_every == 0:
                progress(len(results))
    return ServeReport(latency, results, admitted_at, last_done, max_in_flight, rounds, blocked)


def fifo_one_at_a_time(service_times, arrivals) -> np.ndarray:
    """Latencies of a first-come first-served queue that runs one request at
    a time, given each request's measured service time (Lindley recursion:
    start = max(arrival, previous finish))."""
    s = np.asarray(service_times, dtype=float)
    a = np.asarray(arrivals, dtype=float)
    fin = np.empty_like(s)
    prev = -np.inf
    for i in range(s.shape[0]):
        start = max(a[i], prev)
        fin[i] = start + s[i]
        prev = fin[i]
    return fin - a


def nearest_rank(x, q: float) -> float:
    x = np.sort(np.asarray(x, dtype=float))
    if x.size == 0:
        return float("nan")
    k = int(np.ceil(q / 100.0 * x.size)) - 1
    return float(x[min(max(k, 0), x.size - 1)])
