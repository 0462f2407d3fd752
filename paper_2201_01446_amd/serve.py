"""Continuous-batching serving loop over the batched C-ABI.

A request is one cell (coordinates, and a box when periodic); the answer is
its energy, forces and virial.  The server keeps `slots` batches in flight,
each on its own HIP stream with its own resident neighbor list and scratch
(`dp_batch`), sized so that all slots together stay within an HBM budget.
Whenever a slot is free it takes the waiting requests in arrival order, as
many as fit its atom capacity, and launches them as one batch: pinned host
staging, one chain of kernels over all of the batch's atoms, results copied
back asynchronously.  The loop then goes straight back to admitting, so
requests that arrive while others run are taken as soon as a slot frees up,
and the batches of different slots overlap on the device.  Completion is
detected with HIP events; a request's latency runs from its arrival to the
moment its results are on the host, split into the wait for a slot (arrival
to launch) and the service (launch to results on the host).  A request larger
than a slot's capacity is rejected on its own (its result says why); the
others are served.
"""
import ctypes
import gc
import time
from collections import deque

import numpy as np
import torch

from ._lib import FP32, check, lib


class Request(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int), ("offset", ctypes.c_int), ("periodic", ctypes.c_int),
                ("box", ctypes.c_double * 9)]


def footprint_bytes(model, natoms):
    b = ctypes.c_size_t()
    check(lib.dp_footprint_bytes(model.h, int(natoms), ctypes.byref(b)))
    return b.value


class Batch:
    """A resident batch (device neighbor list and scratch for max_atoms)."""

    def __init__(self, model, max_atoms, max_requests=4096, skin=2.0):
        self.h = ctypes.c_void_p()
        check(lib.dp_batch_create(model.h, int(max_atoms), int(max_requests), skin, ctypes.byref(self.h)))
        self.model, self.max_atoms, self.max_requests = model, max_atoms, max_requests

    def compute(self, cells, coords_dev, precision=FP32, out=None, stream=None):
        """cells: list of (natoms, box or None) in the order of coords_dev rows.
        Returns device tensors E (nreq), F (total, 3), W (nreq, 3, 3)."""
        n = len(cells)
        reqs = (Request * n)()
        off = 0
        for r, (na, box) in enumerate(cells):
            reqs[r].natoms, reqs[r].offset = int(na), off
            reqs[r].periodic = 0 if box is None else 1
            if box is not None:
                b = np.asarray(box, dtype=np.float64).reshape(9)
                for k in range(9):
                    reqs[r].box[k] = b[k]
            off += int(na)
        dev = coords_dev.device
        if out is None:
            out = dict(E=torch.empty(n, dtype=torch.float64, device=dev),
                       F=torch.empty((off, 3), dtype=torch.float64, device=dev),
                       W=torch.empty((n, 3, 3), dtype=torch.float64, device=dev))
        st = stream if stream is not None else torch.cuda.current_stream()
        check(lib.dp_batch_compute(self.model.h, self.h, n, ctypes.cast(reqs, ctypes.c_void_p),
                                   ctypes.c_void_p(coords_dev.data_ptr()), precision,
                                   ctypes.c_void_p(out["E"].data_ptr()), ctypes.c_void_p(out["F"].data_ptr()),
                                   ctypes.c_void_p(out["W"].data_ptr()), None, ctypes.c_void_p(st.cuda_stream)))
        return out

    def stats(self):
        v = [ctypes.c_int() for _ in range(4)]
        check(lib.dp_batch_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(max_nei=v[0].value, sel_overflow=v[1].value, table_oob=v[2].value, cap_overflow=v[3].value)

    def __del__(self):
        if getattr(self, "h", None):
            lib.dp_batch_destroy(self.h)
            self.h = None


class _Slot:
    def __init__(self, model, cap_atoms, max_requests, skin, device):
        self.batch = Batch(model, cap_atoms, max_requests, skin)
        self.stream = torch.cuda.Stream(device=device)
        self.cap = cap_atoms
        self.x_host = torch.empty((cap_atoms, 3), dtype=torch.float64).pin_memory()
        # staging goes through this numpy view: a plain single-threaded copy
        # (a torch slice assignment took up to 8 ms now and then, stalling
        # the loop)
        self.x_host_np = self.x_host.numpy()
        self.x_dev = torch.empty((cap_atoms, 3), dtype=torch.float64, device=device)
        self.E_host = torch.empty(max_requests, dtype=torch.float64).pin_memory()
        self.W_host = torch.empty((max_requests, 3, 3), dtype=torch.float64).pin_memory()
        self.F_host = torch.empty((cap_atoms, 3), dtype=torch.float64).pin_memory()
        self.out = dict(E=torch.empty(max_requests, dtype=torch.float64, device=device),
                        F=torch.empty((cap_atoms, 3), dtype=torch.float64, device=device),
                        W=torch.empty((max_requests, 3, 3), dtype=torch.float64, device=device))
        self.event = torch.cuda.Event()
        self.busy = False
        self.members = []
        self.launched = 0.0


class Server:
    """Continuous batching over `slots` streams; see the module docstring.

    The HBM budget is split evenly over the slots: each slot's resident
    batch is created for the largest atom count whose device footprint
    (neighbor list and scratch, dp_footprint_bytes) fits its share, so the
    whole server never holds more than the budget.  Admission is then a
    capacity check: a free slot takes waiting requests in arrival order while
    their atoms fit."""

    def __init__(self, model, precision=FP32, slots=3, hbm_budget=8 << 30, skin=2.0, max_requests=1024,
                 device="cuda"):
        self.model, self.precision = model, precision
        share = hbm_budget // slots
        lo, hi = 1, 1 << 24
        if footprint_bytes(model, lo) > share:
            raise ValueError("HBM budget too small for one atom per slot")
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if footprint_bytes(model, mid) <= share:
                lo = mid
            else:
                hi = mid - 1
        self.slot_atoms = lo
        self.hbm_budget = hbm_budget
        self.max_requests = max_requests
        self.slots = [_Slot(model, lo, max_requests, skin, device) for _ in range(slots)]

    def _launch(self, slot, reqs):
        """reqs: list of (rid, coords[n,3], box)."""
        slot.launched = time.perf_counter()
        off = 0
        cells = []
        for rid, x, box in reqs:
            n = x.shape[0]
            slot.x_host_np[off:off + n] = x
            cells.append((n, box))
            off += n
        with torch.cuda.stream(slot.stream):
            slot.x_dev[:off].copy_(slot.x_host[:off], non_blocking=True)
            nreq = len(cells)
            out = {k: v[: (nreq if k != "F" else off)] for k, v in slot.out.items()}
            slot.batch.compute(cells, slot.x_dev[:off], self.precision, out=out, stream=slot.stream)
            slot.E_host[:nreq].copy_(out["E"], non_blocking=True)
            slot.W_host[:nreq].copy_(out["W"], non_blocking=True)
            slot.F_host[:off].copy_(out["F"], non_blocking=True)
            slot.event.record(slot.stream)
        slot.members = [(rid, x.shape[0]) for rid, x, _ in reqs]
        slot.busy = True

    def _collect(self, slot, results, done_at, launched_at):
        now = time.perf_counter()
        off = 0
        for r, (rid, n) in enumerate(slot.members):
            results[rid] = dict(E=float(slot.E_host[r]), W=slot.W_host[r].numpy().copy(),
                                F=slot.F_host[off:off + n].numpy().copy())
            done_at[rid] = now
            launched_at[rid] = slot.launched
            off += n
        slot.busy = False
        slot.members = []

    def run(self, requests, arrivals=None, max_batch_atoms=None):
        """requests: list of (coords, box); arrivals: seconds after start at
        which each request arrives (None: all at once, a closed loop);
        max_batch_atoms: most atoms a slot takes into one batch (None: its
        capacity; a larger request still goes alone).  Full slots give the most throughput; under a latency
        target a smaller cap keeps a burst of arrivals from becoming a few
        large batches that share the GPU and return late.  Returns (results
        by request, stats).  Python's cyclic garbage collector is paused while
        the loop runs (a full collection over a large heap stalls admission
        and completion for tens of ms)."""
        enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, arrivals, max_batch_atoms)
        finally:
            if enabled:
                gc.enable()

    def _run(self, requests, arrivals, max_batch_atoms):
        nreq = len(requests)
        arrivals = np.zeros(nreq) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
        order = np.argsort(arrivals, kind="stable")
        results, done_at, launched_at = [None] * nreq, [None] * nreq, [None] * nreq
        # a request no slot can hold is answered at once with the reason
        rejected = [rid for rid, (x, _) in enumerate(requests) if x.shape[0] > self.slot_atoms]
        for rid in rejected:
            results[rid] = dict(error=f"{requests[rid][0].shape[0]} atoms exceed the slot capacity "
                                      f"{self.slot_atoms}")
        skip = set(rejected)
        order = np.array([o for o in order if int(o) not in skip], dtype=np.int64)
        nserve = len(order)
        waiting = deque()
        nxt = 0
        batch_atoms = []
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            while nxt < nserve and arrivals[order[nxt]] <= now:
                waiting.append(int(order[nxt]))
                nxt += 1
            progressed = False
            for s in self.slots:   # completions free their slot
                if s.busy and s.event.query():
                    self._collect(s, results, done_at, launched_at)
                    progressed = True
            for s in self.slots:   # admission in arrival order
                if s.busy or not waiting:
                    continue
                take, atoms = [], 0
                cap = s.cap if max_batch_atoms is None else max(1, min(s.cap, max_batch_atoms))
                while waiting and len(take) < self.max_requests:
                    n = requests[waiting[0]][0].shape[0]
                    if atoms + n > cap and take:
                        break
                    take.append(waiting.popleft())
                    atoms += n
                self._launch(s, [(rid, requests[rid][0], requests[rid][1]) for rid in take])
                batch_atoms.append(atoms)
                progressed = True
            if nxt >= nserve and not waiting and not any(s.busy for s in self.slots):
                break
            if not progressed:
                time.sleep(2e-5)
        wall = time.perf_counter() - t0
        served = [int(i) for i in order]
        lat = np.array([done_at[i] - t0 - arrivals[i] for i in served])
        wait = np.array([launched_at[i] - t0 - arrivals[i] for i in served])
        size = np.array([requests[i][0].shape[0] for i in served])
        total_atoms = int(size.sum())
        stats = dict(requests=nreq, rejected=len(rejected), atoms=total_atoms, wall_s=wall,
                     atoms_per_s=total_atoms / wall, batches=len(batch_atoms),
                     mean_batch_atoms=float(np.mean(batch_atoms)) if batch_atoms else 0.0,
                     slot_atoms=self.slot_atoms, slots=len(self.slots))
        if served:
            p99 = np.percentile(lat, 99)
            tail = lat >= p99
            stats.update(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(p99 * 1e3),
                         mean_ms=float(lat.mean() * 1e3), mean_wait_ms=float(wait.mean() * 1e3),
                         mean_service_ms=float((lat - wait).mean() * 1e3),
                         # the slowest 1 %: what their latency was made of
                         tail_wait_ms=float(wait[tail].mean() * 1e3),
                         tail_service_ms=float((lat - wait)[tail].mean() * 1e3),
                         tail_mean_atoms=float(size[tail].mean()), mean_atoms=float(size.mean()))
        return results, stats


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of n requests of a Poisson process of `rate` per s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
