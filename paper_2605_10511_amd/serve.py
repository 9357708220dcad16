"""Serving loop over the fused query path.

Requests arrive over time (Poisson in the benchmark).  The server

* prepares each request on arrival: dimension hash tables come from a cache
  keyed by (dimension, key, filter, payloads) and are built once, on the
  device (paper Section 3.1, Kernel #1); the plan is compiled against the
  resident fact columns;
* admits prepared requests while the device state fits the state budget:
  the in-flight plans' own workspaces (``dpf_plan_footprint``) plus the
  cached dimension hash tables, each charged once however many plans probe
  it; an in-flight slot must also be free;
* batches whatever is admitted into ONE fused launch per free stream
  (continuous batching: a new batch starts as soon as a stream drains, it
  does not wait for a full batch), so queries that arrive together share a
  launch and the work queue of one persistent kernel (Section 3.2);
* completes a batch when its stream event fires, decodes the records and
  records arrival-to-result latency.

``place_table`` decides where a table rests: in HBM while the tables placed
so far and this one fit the residency budget, otherwise in pinned host
memory mapped into the device, scanned over the host link (Section 3.1's
zero-copy path).  The server finds such tables by their columns' placement.  Requests on such tables run on a stream of their own and never
share a batch with resident-table requests: a launch finishes when its
slowest plan does, and a host-link scan takes tens of milliseconds.  They
also run with one workgroup per CU (``host_knobs``): the host link, not the
CUs, bounds such a scan, and a full grid of persistent workgroups would hold
every slot of every CU for the scan's whole duration.
"""
from __future__ import annotations

import collections
import json
import time

import numpy as np

from . import dpf


class Request:
    __slots__ = ("t", "template", "spec", "plan", "footprint", "rows", "done", "issued", "table")

    def __init__(self, t: float, template: str, spec: dict, table: str):
        self.t = t
        self.template = template
        self.spec = spec
        self.table = table
        self.plan = None
        self.footprint = 0
        self.rows = None
        self.done = None
        self.issued = None


class _Batch:
    __slots__ = ("stream", "event", "reqs", "result", "footprint")


class Server:
    def __init__(self, ctx: dpf.Context, db: dpf.Database, nstreams: int = 4, slots: int = 8,
                 state_budget: int = 4 << 30, placements: dict | None = None, host_tables=None,
                 host_knobs: dict | None = None, max_batch: int = 64):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.db = db
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]  # default priority
        self.slots = slots
        self.state_budget = state_budget
        self.hashes: dict[str, dpf.Hash] = {}
        self.placements = placements or {}
        self.hash_builds = 0
        self.hash_build_s = 0.0
        self.hash_bytes = 0  # device bytes of the cached hash tables, charged once
        if host_tables is None:  # the tables whose columns rest in host memory
            host_tables = [t for t, cols in db.tables.items()
                           if cols and next(iter(cols.values())).info().placement == dpf.DPF_PLACE_HOST_MAPPED]
        self.host_tables = set(host_tables)
        self.host_knobs = dict(host_knobs) if host_knobs is not None else {"max_workgroups": 64}
        self.host_stream = torch.cuda.Stream() if self.host_tables else None  # default priority
        self.max_batch = max(1, min(64, max_batch))  # plans per fused launch
        # what the loop did: plans per launched batch, and the most batches
        # that were on the device at the same time
        self.batch_sizes: list[int] = []
        self.max_inflight = 0

    # -- preparation -------------------------------------------------------
    def _hash(self, pr: dict) -> dpf.Hash:
        key = json.dumps([pr["dim"], pr["key"], pr.get("filters", []), pr.get("payloads", [])], sort_keys=True)
        h = self.hashes.get(key)
        if h is None:
            t0 = time.perf_counter()
            s = self.streams[0]
            h = self.db.build_hash(pr, self.placements.get(pr["dim"], "AUTO"), s)
            s.synchronize()  # later batches on other streams read it
            self.hashes[key] = h
            self.hash_bytes += h.info().device_bytes
            self.hash_builds += 1
            self.hash_build_s += time.perf_counter() - t0
        return h

    def warm(self, reqs: list):
        """Build (cache) every dimension hash table ``reqs`` will probe."""
        for r in reqs:
            for pr in r.spec.get("probes", []):
                self._hash(pr)

    def prepare(self, r: Request):
        hashes = [self._hash(pr) for pr in r.spec.get("probes", [])]
        r.plan = self.db.plan(r.spec, hashes=hashes)
        r.footprint = r.plan.footprint()

    # -- the loop ----------------------------------------------------------
    def run(self, reqs: list, log=None, t_limit: float | None = None) -> list:
        """Serve ``reqs`` (ascending arrival times, seconds from the start);
        returns the completed requests with ``done`` and ``rows`` set."""
        torch = self.torch
        reqs = sorted(reqs, key=lambda r: r.t)
        ready = collections.deque()
        ready_host = collections.deque()
        host_busy = False
        inflight: list[_Batch] = []
        free = list(range(len(self.streams)))
        used = 0
        nin = 0
        done = []
        i = 0
        t0 = time.perf_counter()
        while i < len(reqs) or ready or ready_host or inflight:
            now = time.perf_counter() - t0
            if t_limit is not None and now > t_limit and not inflight:
                break
            progressed = False
            # arrivals: prepare in arrival order
            while i < len(reqs) and reqs[i].t <= now:
                self.prepare(reqs[i])
                (ready_host if reqs[i].table in self.host_tables else ready).append(reqs[i])
                i += 1
                progressed = True
            # completions
            for b in list(inflight):
                if b.event.query():
                    t = time.perf_counter() - t0
                    for k, r in enumerate(b.reqs):
                        r.rows = b.result.get(k)
                        r.done = t
                        r.plan.release()
                        r.plan = None
                    b.result.release()
                    used -= b.footprint
                    if b.stream >= 0:
                        nin -= len(b.reqs)
                        free.append(b.stream)
                    else:
                        host_busy = False
                    inflight.remove(b)
                    done.extend(b.reqs)
                    progressed = True
            # admission + launch: one fused batch per free stream
            while free and ready and nin < self.slots:
                batch = []
                fp = 0
                while ready and nin + len(batch) < self.slots and len(batch) < self.max_batch:
                    r = ready[0]
                    if used + self.hash_bytes + fp + r.footprint > self.state_budget and (batch or inflight):
                        break  # wait for state to drain
                    batch.append(ready.popleft())
                    fp += r.footprint
                if not batch:
                    break
                si = free.pop(0)
                s = self.streams[si]
                b = _Batch()
                b.stream = si
                b.reqs = batch
                b.footprint = fp
                issued = time.perf_counter() - t0
                for r in batch:
                    r.issued = issued
                b.result = dpf.execute(self.ctx, [r.plan for r in batch], stream=s)
                b.event = torch.cuda.Event()
                b.event.record(s)
                inflight.append(b)
                used += fp
                nin += len(batch)
                self.batch_sizes.append(len(batch))
                self.max_inflight = max(self.max_inflight, len(inflight))
                progressed = True
            # host-table requests: one at a time on their own stream
            if ready_host and not host_busy:
                r = ready_host.popleft()
                b = _Batch()
                b.stream = -1
                b.reqs = [r]
                b.footprint = r.footprint
                r.issued = time.perf_counter() - t0
                b.result = dpf.execute(self.ctx, [r.plan], stream=self.host_stream, **self.host_knobs)
                b.event = torch.cuda.Event()
                b.event.record(self.host_stream)
                inflight.append(b)
                used += r.footprint
                host_busy = True
                self.batch_sizes.append(1)
                self.max_inflight = max(self.max_inflight, len(inflight))
                progressed = True
            if not progressed:
                nxt = reqs[i].t - (time.perf_counter() - t0) if i < len(reqs) else 0.0
                if not inflight and nxt > 0:
                    time.sleep(min(nxt, 0.002))
                else:
                    time.sleep(20e-6)
        for r in list(ready) + list(ready_host):
            if r.plan is not None:
                r.plan.release()
                r.plan = None
        return done

    def close(self):
        for h in self.hashes.values():
            h.release()
        self.hashes.clear()
        self.hash_bytes = 0
        self.host_stream = None


def place_table(db: dpf.Database, name: str, columns: dict, encodings: dict | None, residency_budget: int,
                chunk_rows: int = 65536, sample_rows: int = 1 << 20) -> str:
    """Encode a table where the residency budget allows: HBM when the
    compressed bytes of the tables already resident in HBM plus this one fit
    ``residency_budget``, else pinned host memory mapped into the device.
    The table's compressed size is estimated from its first ``sample_rows``
    rows, encoded on the host with the same encodings.  Returns the
    placement chosen ("HBM" or "HOST_MAPPED")."""
    n = len(next(iter(columns.values())).offsets) - 1 if hasattr(next(iter(columns.values())), "offsets") \
        else len(next(iter(columns.values())))
    k = min(n, sample_rows)
    host_ctx = dpf.Context(-1)
    est = 0
    enc = encodings or {}
    for c, v in columns.items():
        part = v[:k] if not hasattr(v, "offsets") else type(v)(v.offsets[:k + 1], v.data[:int(v.offsets[k])])
        col = dpf.Column(host_ctx, part, enc.get(c, "AUTO"), chunk_rows, "HOST")
        est += col.info().compressed_bytes
        col.release()
    host_ctx.close()
    est = int(est * (n / max(1, k)))
    resident = sum(col.info().compressed_bytes for t in db.tables.values() for col in t.values()
                   if col.info().placement == dpf.DPF_PLACE_HBM)
    placement = "HBM" if resident + est <= residency_budget else "HOST_MAPPED"
    db.add_table(name, columns, encodings, chunk_rows=chunk_rows, placement=placement)
    return placement


def latency_stats(done: list, seconds: float) -> dict:
    lat = np.array([(r.done - r.t) * 1e3 for r in done]) if done else np.zeros(0)
    out = {"completed": len(done), "qps": len(done) / seconds if seconds > 0 else 0.0}
    if len(lat):
        wait = np.array([(r.issued - r.t) * 1e3 for r in done])
        serv = np.array([(r.done - r.issued) * 1e3 for r in done])
        out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                    "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                    "queue_wait_p50_ms": float(np.percentile(wait, 50)),
                    "queue_wait_p99_ms": float(np.percentile(wait, 99)),
                    "service_p50_ms": float(np.percentile(serv, 50)),
                    "service_p99_ms": float(np.percentile(serv, 99))})
    for tmpl in ("FA", "SJ"):
        sel = np.array([(r.done - r.t) * 1e3 for r in done if r.template == tmpl])
        if len(sel):
            out[tmpl] = {"n": int(len(sel)), "p50_ms": float(np.percentile(sel, 50)),
                         "p99_ms": float(np.percentile(sel, 99))}
    return out
