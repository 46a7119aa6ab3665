"""Continuous-batching encode server for images of mixed sizes.

Requests carry one image each.  Every window of an image is a patch to code
(sliding windows as in the paper's patch coding, Sec. III-A).  The scheduler

* admits requests in arrival order while their pixels fit the HBM budget (an arena
  preallocated once; step buffers are preallocated too, so nothing is allocated on
  the device per request or per step); requests that can never fit the budget, or
  whose window row is wider than a step, are rejected,
* cuts admitted images into row ranges ("chunks") and fills each device step with
  up to ``step_windows`` windows: every ready request first gets an equal share of
  the step, the rest goes to the oldest ones, so requests that arrive while others
  run join the next step and a huge image never starves small ones,
* runs a step as one image projection and one encode over all its chunks (any mix
  of requests and sizes), overlapped with the host-to-device copies of newly
  admitted images and the device-to-host copies of finished codes on separate
  streams,
* completes a request when all its windows are coded and its codes are on the host.

A window's code depends only on its own pixels, so a request's codes are the same
alone or in any mix.  The scheduling logic is independent of the device: ``Backend``
is implemented by ``DeviceBackend`` (HIP, via the C ABI) and by test backends.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds on the server clock
    pixels: object                 # host image [H, W] float32 (numpy or pinned torch)
    H: int
    W: int
    windows: int = 0
    done_rows: int = 0             # window rows handed to steps
    coded_rows: int = 0            # window rows whose codes reached the host
    served_step: int = -1          # last step that coded rows of it (admission step at first)
    t_admit: float | None = None
    t_done: float | None = None
    slot: object = None            # backend memory handle
    codes: object = None           # host (atom, angle, coef) arrays [windows, K]


@dataclasses.dataclass
class Chunk:
    req: Request
    y0: int                        # first window row
    rows: int                      # window rows in this chunk
    out_start: int                 # first window index within the request


class Arena:
    """First-fit allocator over [0, capacity) in units of elements (for admission)."""

    def __init__(self, capacity: int, align: int = 64):
        self.capacity = capacity
        self.align = align
        self.free = [(0, capacity)]   # sorted (start, length)

    def alloc(self, n: int):
        n = (n + self.align - 1) // self.align * self.align
        for i, (s, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, l - n)
                return (s, n)
        return None

    def release(self, block):
        s, n = block
        self.free.append((s, n))
        self.free.sort()
        merged = []
        for a, b in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + b)
            else:
                merged.append((a, b))
        self.free = merged

    @property
    def used(self) -> int:
        return self.capacity - sum(l for _, l in self.free)


class Backend:
    """Device interface used by the scheduler."""

    N: int
    K: int

    def request_elems(self, req: Request) -> int:            # arena elements a request needs
        raise NotImplementedError

    def upload(self, req: Request, block) -> None:             # copy pixels into its arena block
        raise NotImplementedError

    def uploaded(self, req: Request) -> bool:                  # pixels are on the device
        raise NotImplementedError

    def launch(self, chunks: list[Chunk]) -> object:           # start a step, return a token
        raise NotImplementedError

    def finished(self, token) -> bool:                         # step done and codes on the host
        raise NotImplementedError

    def wait(self, token) -> None:
        raise NotImplementedError


class Scheduler:
    """Admission, chunking and completion; drives a Backend."""

    def __init__(self, backend: Backend, budget_elems: int, step_windows: int, max_inflight: int = 2,
                 clock=time.perf_counter):
        self.be = backend
        self.arena = Arena(budget_elems)
        self.step_windows = step_windows
        self.max_inflight = max_inflight
        self.clock = clock
        self.t0 = clock()
        self.queue: collections.deque[Request] = collections.deque()   # arrived, not admitted
        self.active: list[Request] = []                                # admitted, not finished
        self.inflight: collections.deque = collections.deque()         # (token, chunks)
        self.finished: list[Request] = []
        self.lock = threading.Lock()
        self.max_active = 0
        self.steps = 0
        self.rejected: list[Request] = []

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        n = self.be.N
        req.windows = max(req.H - n + 1, 0) * max(req.W - n + 1, 0)
        with self.lock:
            self.queue.append(req)

    def _admit(self):
        with self.lock:
            while self.queue:
                req = self.queue[0]
                need = self.be.request_elems(req)
                row = req.W - self.be.N + 1
                if need > self.arena.capacity or (req.windows > 0 and row > self.step_windows):
                    self.queue.popleft()
                    self.rejected.append(req)          # can never fit the budget or one step
                    continue
                block = self.arena.alloc(need)
                if block is None:
                    break                              # wait for memory (arrival order kept)
                self.queue.popleft()
                req.slot = block
                req.served_step = self.steps
                req.t_admit = self.now()
                self.be.upload(req, block)
                self.active.append(req)
        self.max_active = max(self.max_active, len(self.active))

    def _next_chunks(self) -> list[Chunk]:
        """Fill one step of at most ``step_windows`` windows: every ready request first
        gets an equal share of the step (at least one window row while a row still fits),
        then the rest goes to the oldest requests.  Shares are handed out longest-unserved
        first; admission rejects images whose window row is wider than a step, so the first
        of them always gets a row and no request waits behind others for ever."""
        n = self.be.N
        ready = []
        for req in self.active:                        # oldest first
            wr, wc = req.H - n + 1, req.W - n + 1
            if wr > 0 and wc > 0 and req.done_rows < wr and self.be.uploaded(req):
                ready.append(req)
        if not ready:
            return []
        budget = self.step_windows
        share = max(budget // len(ready), 1)
        take = {}
        age = {req.rid: i for i, req in enumerate(ready)}
        for req in sorted(ready, key=lambda r: (r.served_step, age[r.rid])):
            if budget <= 0:
                break
            wc = req.W - n + 1
            left = req.H - n + 1 - req.done_rows
            rows = min(left, max(min(share, budget) // wc, 1 if wc <= budget else 0))
            if rows > 0:
                take[req.rid] = rows
                budget -= rows * wc
        for req in ready:
            if budget <= 0:
                break
            wc = req.W - n + 1
            left = req.H - n + 1 - req.done_rows - take.get(req.rid, 0)
            extra = min(left, budget // wc)
            if extra > 0:
                take[req.rid] = take.get(req.rid, 0) + extra
                budget -= extra * wc
        chunks = []
        for req in ready:
            rows = take.get(req.rid, 0)
            if rows > 0:
                wc = req.W - n + 1
                chunks.append(Chunk(req, req.done_rows, rows, req.done_rows * wc))
                req.done_rows += rows
                req.served_step = self.steps
        return chunks

    def _retire(self, chunks: list[Chunk]):
        n = self.be.N
        for c in chunks:
            c.req.coded_rows += c.rows
        for req in list(self.active):
            wr = req.H - n + 1
            if wr <= 0 or req.W - n + 1 <= 0 or req.coded_rows >= wr:
                req.t_done = self.now()
                self.active.remove(req)
                self.arena.release(req.slot)
                self.finished.append(req)

    def poll(self) -> bool:
        """One scheduling round; returns True if it did anything."""
        did = False
        while self.inflight and self.be.finished(self.inflight[0][0]):
            _, chunks = self.inflight.popleft()
            self._retire(chunks)
            did = True
        self._admit()
        # requests without windows complete as soon as they are admitted
        for req in list(self.active):
            if req.windows == 0:
                self._retire([])
                did = True
                break
        if len(self.inflight) < self.max_inflight:
            chunks = self._next_chunks()
            if chunks:
                self.inflight.append((self.be.launch(chunks), chunks))
                self.steps += 1
                did = True
        return did

    def drain(self, total: int, idle_sleep: float = 2e-4):
        """Run until ``total`` requests have finished or been rejected."""
        while len(self.finished) + len(self.rejected) < total:
            if not self.poll():
                if self.inflight:
                    self.be.wait(self.inflight[0][0])
                else:
                    time.sleep(idle_sleep)


def replay(scheduler: Scheduler, requests: list[Request], realtime: bool = True):
    """Open-loop client: submits each request at its arrival time (server clock)."""
    def client():
        for r in requests:
            if realtime:
                dt = r.arrival - scheduler.now()
                if dt > 0:
                    time.sleep(dt)
            scheduler.submit(r)
    th = threading.Thread(target=client, daemon=True)
    th.start()
    scheduler.drain(len(requests))
    th.join()


def latency_report(reqs: list[Request], warmup: float = 0.0) -> dict:
    lat = np.array([r.t_done - r.arrival for r in reqs if r.arrival >= warmup and r.t_done is not None])
    wait = np.array([r.t_admit - r.arrival for r in reqs if r.arrival >= warmup and r.t_admit is not None])
    if lat.size == 0:
        return {"requests": 0}
    return {"requests": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "max_s": float(lat.max()), "admit_wait_p50_s": float(np.percentile(wait, 50)),
            "admit_wait_p99_s": float(np.percentile(wait, 99))}


# --------------------------------------------------------------------------- device backend
class DeviceBackend(Backend):
    """HIP backend: arena of pixels in HBM, one projection + encode per step."""

    def __init__(self, h, K: int, budget_bytes: int, step_windows: int, device="cuda:0", slots: int = 2,
                 keep_codes=lambda req: True):
        import torch
        from . import rsc
        self.rsc = rsc
        self.torch = torch
        self.h = h
        self.N = h.N
        self.K = K
        self.dev = torch.device(device)
        self.pool = torch.empty(budget_bytes // 4, dtype=torch.float32, device=self.dev)
        self.copy_in = torch.cuda.Stream(self.dev)
        self.compute = torch.cuda.Stream(self.dev)
        self.copy_out = torch.cuda.Stream(self.dev)
        self.step_windows = step_windows
        # per in-flight step slot: coordinates, codes on device and pinned on host
        self.slots = []
        for _ in range(slots):
            self.slots.append({
                "xhat": torch.empty((step_windows, h.B), dtype=torch.float32, device=self.dev),
                "atom": torch.empty((step_windows, K), dtype=torch.int32, device=self.dev),
                "angle": torch.empty((step_windows, K), dtype=torch.int32, device=self.dev),
                "coef": torch.empty((step_windows, K), dtype=torch.float32, device=self.dev),
                "h_atom": torch.empty((step_windows, K), dtype=torch.int32, pin_memory=True),
                "h_angle": torch.empty((step_windows, K), dtype=torch.int32, pin_memory=True),
                "h_coef": torch.empty((step_windows, K), dtype=torch.float32, pin_memory=True),
                "busy": False,
            })
        self.ready = {}
        self.keep_codes = keep_codes

    def request_elems(self, req):
        return req.H * req.W

    def upload(self, req, block):
        torch = self.torch
        start, _ = block
        src = req.pixels if isinstance(req.pixels, torch.Tensor) else torch.from_numpy(req.pixels)
        with torch.cuda.stream(self.copy_in):
            self.pool[start:start + req.H * req.W].copy_(src.reshape(-1), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_in)
        self.ready[req.rid] = ev
        K = self.K
        if self.keep_codes(req):
            req.codes = (np.empty((req.windows, K), np.int32), np.empty((req.windows, K), np.int32),
                         np.empty((req.windows, K), np.float32))

    def uploaded(self, req):
        ev = self.ready.get(req.rid)
        return ev is not None and ev.query()

    def launch(self, chunks):
        torch, rsc = self.torch, self.rsc
        slot = next(s for s in self.slots if not s["busy"])
        slot["busy"] = True
        n = self.N
        sizes, offs = [], []
        for c in chunks:
            start, _ = c.req.slot
            sizes.append((c.rows + n - 1, c.req.W))
            offs.append(start + c.y0 * c.req.W)
        with torch.cuda.stream(self.compute):      # small descriptor copies ordered on this stream
            batch = rsc.ImageBatch(sizes, n, self.dev, offsets=offs)
        P = batch.P_total
        xh = slot["xhat"][:P]
        out = (slot["atom"][:P], slot["angle"][:P], slot["coef"][:P], None)
        rsc.rsc_project_images(self.h, self.pool, batch, xhat=xh, stream=self.compute)
        rsc.rsc_omp_encode(self.h, xh, self.K, out=out, stream=self.compute)
        done = torch.cuda.Event()
        done.record(self.compute)
        with torch.cuda.stream(self.copy_out):
            self.copy_out.wait_event(done)
            for name in ("atom", "angle", "coef"):
                slot["h_" + name][:P].copy_(slot[name][:P], non_blocking=True)
            fin = torch.cuda.Event()
            fin.record(self.copy_out)
        return {"slot": slot, "fin": fin, "chunks": chunks, "batch": batch, "P": P}

    def _complete(self, tok):
        slot = tok["slot"]
        if not slot["busy"]:
            return
        pos = 0
        for c in tok["chunks"]:
            wc = c.req.W - self.N + 1
            n = c.rows * wc
            if c.req.codes is not None:
                for i, name in enumerate(("h_atom", "h_angle", "h_coef")):
                    c.req.codes[i][c.out_start:c.out_start + n] = slot[name][pos:pos + n].numpy()
            pos += n
        slot["busy"] = False

    def finished(self, tok):
        if tok["fin"].query():
            self._complete(tok)
            return True
        return False

    def wait(self, tok):
        tok["fin"].synchronize()


def encode_one_at_a_time(h, K: int, requests: list[Request], device="cuda:0", realtime: bool = True,
                         clock=time.perf_counter, keep_codes=lambda req: True):
    """Baseline: each request alone, in arrival order (copy in, project, encode, copy out)."""
    import torch
    from . import rsc
    dev = torch.device(device)
    t0 = clock()
    for req in requests:
        if realtime:
            dt = req.arrival - (clock() - t0)
            if dt > 0:
                time.sleep(dt)
        req.t_admit = max(clock() - t0, req.arrival)
        n = h.N
        req.windows = max(req.H - n + 1, 0) * max(req.W - n + 1, 0)
        if req.windows:
            src = req.pixels if isinstance(req.pixels, torch.Tensor) else torch.from_numpy(req.pixels)
            pix = src.reshape(-1).to(dev, non_blocking=True)
            batch = rsc.ImageBatch([(req.H, req.W)], n, dev)
            xh = rsc.rsc_project_images(h, pix, batch)
            atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh, K)
            codes = (atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy())
            if keep_codes(req):
                req.codes = codes
        req.t_done = clock() - t0
    return requests
