"""Python handle on the native query server (mpr_server_* in include/mpr.h).

The engine (batching, admission, ladders, streams) is C++ inside libmpr;
this module only marshals arguments and drives an open-loop arrival
process for measurements.
"""
from __future__ import annotations

import ctypes
import threading
import time

from . import MprError, QueryResult, ServerOptions, ServerStats, lib


class Server:
    def __init__(self, device: int = 0, baby: int = 32, max_n: int = 1000, max_batch: int = 256,
                 slots: int = 4, hbm_budget_bytes: int = 200 << 30, wide_only: bool = False,
                 busy_poll: bool = False, period_mode: bool = False, request_timeout_s: float = 0.0):
        self.opt = ServerOptions(device, baby, max_n, max_batch, slots, hbm_budget_bytes, int(bool(wide_only)),
                                 int(bool(busy_poll)), int(bool(period_mode)), float(request_timeout_s))
        h = ctypes.c_void_p()
        st = lib().mpr_server_create(ctypes.byref(self.opt), ctypes.byref(h))
        if st != 0:
            raise MprError(st, "mpr_server_create")
        self.h = h
        self._buf = (QueryResult * 1024)()
        self._held = []  # results query() read while waiting for its own

    def submit(self, m: int, n: int, tag: int):
        st = lib().mpr_server_submit(self.h, m, n, tag)
        if st != 0:
            raise MprError(st, "mpr_server_submit")

    def cancel(self, tag: int):
        """Requests with this tag still waiting complete with MPR_ECANCELED."""
        st = lib().mpr_server_cancel(self.h, tag)
        if st != 0:
            raise MprError(st, "mpr_server_cancel")

    def poll(self, wait_ms: int = 10):
        if self._held:
            out, self._held = self._held, []
            return out
        return self._poll(wait_ms)

    def _poll(self, wait_ms: int):
        cnt = ctypes.c_int()
        st = lib().mpr_server_poll(self.h, self._buf, len(self._buf), ctypes.byref(cnt), wait_ms)
        if st != 0:
            raise MprError(st, "mpr_server_poll")
        out = []
        for i in range(cnt.value):
            r = self._buf[i]
            out.append({"tag": r.tag, "m": r.m, "n": r.n, "gamma": r.gamma, "status": r.status, "cold": r.cold,
                        "t_submit": r.t_submit_s, "t_start": r.t_start_s, "t_done": r.t_done_s})
        return out

    def now(self) -> float:
        return lib().mpr_server_now(self.h)

    def stats(self) -> dict:
        s = ServerStats()
        lib().mpr_server_stats_get(self.h, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def query(self, m: int, n: int, timeout_s: float = 600.0) -> dict:
        """Submit one request and wait for its answer; other results that
        arrive meanwhile are kept for the next poll()."""
        tag = int(time.monotonic_ns() & 0x7FFFFFFFFFFF)
        self.submit(m, n, tag)
        t_end = time.monotonic() + timeout_s
        while time.monotonic() < t_end:
            for r in self._poll(50):
                if r["tag"] == tag:
                    return r
                self._held.append(r)  # someone else's: returned by the next poll()
        raise TimeoutError("query (%d, %d) did not complete" % (m, n))

    def close(self):
        if self.h:
            lib().mpr_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def ladder_bytes(m: int, baby: int = 32, max_n: int = 1000, wide_only: bool = False) -> int:
    return int(lib().mpr_server_ladder_bytes(m, baby, max_n, int(bool(wide_only))))


def period_build_bytes(m: int) -> int:
    """Device bytes a period-mode build of m holds while it runs."""
    return int(lib().mpr_server_period_bytes(m))


def run_open_loop(server: Server, arrivals, timeout_s: float = 600.0):
    """Submits (t, m, n) arrivals at their times (seconds from now) from a
    separate thread and collects every result.  Returns the results in
    submission order (tag = index)."""
    t0 = time.monotonic()
    done = {}

    def feeder():
        for k, (t, m, n) in enumerate(arrivals):
            d = t0 + t - time.monotonic()
            if d > 0:
                time.sleep(d)
            server.submit(m, n, k)

    th = threading.Thread(target=feeder, daemon=True)
    th.start()
    t_end = t0 + timeout_s
    while len(done) < len(arrivals) and time.monotonic() < t_end:
        for r in server.poll(20):
            done[r["tag"]] = r
    th.join(timeout=1.0)
    if len(done) < len(arrivals):
        raise TimeoutError("%d of %d queries unanswered" % (len(arrivals) - len(done), len(arrivals)))
    return [done[k] for k in range(len(arrivals))]
