"""Continuous-batching request loop for the Mojette erasure code on one GPU.

Writes (encode an object of k data packets into n projections, Section 2.3)
and degraded reads (rebuild an object from the projections that survive,
Section 2.2) arrive as a Poisson stream.  Projections stay resident in HBM in
per-class arenas; a class is one code (k, m) and one row length P from a
geometric grid, and an object of S bytes is stored in the smallest class with
P * k * 8 >= S.

Admission works against a fixed HBM budget, carved at start-up into the
arenas, a pre-staged payload pool per class (the images writes encode) and
an output ring per class (where reads land):
  - a write needs an arena slot: a free one, or the oldest resident object if
    no in-flight read uses it; otherwise it waits;
  - a read needs a resident object of its class and a row of the output ring;
  - an iteration takes at most `cap` requests of each kind per class.
Every loop turn retires the iterations whose completion event has fired,
admits what has arrived and fits, and issues ONE descriptor-driven encode
call for every write and ONE descriptor-driven decode call for every
short-row read of every class (a 24-byte descriptor per request: where its
image and its arena slot sit in the server's one word pool, its row length,
code and erasure mask).  Reads of long rows either run as chunked decode
jobs on side streams, joined into the iteration, or (long_reads="both_ends")
as one more descriptor-driven decode on a side stream, every block swept
from both ends, that completes on its own event; long_reads="auto" takes
the chunked decode (short chains, twice the sweep work) at low load and the
decode from both ends (the sweep work once, chains of half a row) once
requests arrive faster than `auto_rate` per second (over the last 10 ms)
or more than `auto_backlog` wait.  Up to `depth` iterations
are in flight, so requests join while earlier ones are still running on the
device.

Latency is arrival to the GPU completion event of the request's iteration,
read on the GPU clock from a start event that had completed before the host
clock started: never shorter than the true latency.  The host work is
bookkeeping only (slot rings, masks, timestamps); every pixel and bin is read
and written by the HIP kernels.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass

import numpy as np

import paper_1504_07038_amd as mj

CODES = ((4, 2), (8, 4))
READ_FRACTION = 0.7
LOG2_MIN, LOG2_MAX = 12, 20     # object sizes 4 KB .. 1 MB


@dataclass
class Geometry:
    k: int
    m: int
    P: int
    dirs: list
    words: int          # projection words per object (one arena slot)

    @property
    def Q(self):
        return self.k

    @property
    def img_words(self):
        return self.P * self.k


def class_grid(k: int, per_octave: int = 4):
    """Row lengths of the classes of code k: P_min * 2^(j / per_octave),
    rounded up, from 4 KB objects to 1 MB objects."""
    pmin = (1 << LOG2_MIN) // (8 * k)
    steps = (LOG2_MAX - LOG2_MIN) * per_octave
    return sorted({int(np.ceil(pmin * 2.0 ** (j / per_octave) - 1e-9)) for j in range(steps + 1)})


def geometries(codes=CODES, per_octave: int = 4):
    out = []
    for k, m in codes:
        n = k + m
        dirs = [i - n // 2 for i in range(n)]
        for P in class_grid(k, per_octave):
            out.append(Geometry(k, m, P, dirs, mj.mojette_block_words(dirs, P, k)))
    return out


@dataclass
class Trace:
    """A request stream, sorted by arrival."""
    arrival: np.ndarray     # seconds
    size: np.ndarray        # object bytes
    cls: np.ndarray         # class index
    read: np.ndarray        # 1 = degraded read, 0 = write
    mask: np.ndarray        # reads: erased projections (bit i = projection i)


def make_trace(qps: float, duration: float, geos, seed: int, codes=CODES) -> Trace:
    """Poisson arrivals at `qps` for `duration` s.  Per request: code uniform
    over `codes`; size 2^U[12, 20] bytes rounded up to a multiple of 8k; 70%
    reads, each losing a uniform number 0..m of its n projections (a uniform
    subset, so every read is decodable, Section 2.3)."""
    import synth

    rng = np.random.default_rng(seed)
    N = max(1, int(rng.poisson(qps * duration)))
    arrival = np.sort(rng.uniform(0.0, duration, N))
    code = rng.integers(0, len(codes), N)
    ks = np.array([k for k, _ in codes])[code]
    raw = 2.0 ** rng.uniform(LOG2_MIN, LOG2_MAX, N)
    size = (np.ceil(raw / (8 * ks)) * (8 * ks)).astype(np.int64)
    read = (rng.random(N) < READ_FRACTION).astype(np.int64)
    cls = np.empty(N, dtype=np.int64)
    mask = np.zeros(N, dtype=np.uint16)
    for ci, (k, m) in enumerate(codes):
        ids = np.array([g for g, geo in enumerate(geos) if (geo.k, geo.m) == (k, m)])
        Ps = np.array([geos[g].P for g in ids])
        sel = np.flatnonzero(code == ci)
        pos = np.searchsorted(Ps, size[sel] // (8 * k), side="left")
        if (pos >= len(Ps)).any():
            raise ValueError("object larger than the largest class")
        cls[sel] = ids[pos]
        mask[sel] = synth.erasure_masks(seed * 7 + ci, len(sel), k + m, (0, m))
    return Trace(arrival, size, cls, read, mask)


class SlotStore:
    """Arena slot bookkeeping of one class (host side, no device memory):
    free slots on a stack, resident objects in a FIFO ring (oldest at head),
    in-flight read counts per slot, and the payload row each object holds."""

    def __init__(self, slots: int):
        self.slots = slots
        self.free = np.arange(slots - 1, -1, -1, dtype=np.int64)
        self.nfree = slots
        self.ring = np.zeros(slots, dtype=np.int64)
        self.head = 0
        self.count = 0
        self.refs = np.zeros(slots, dtype=np.int32)
        self.source = np.full(slots, -1, dtype=np.int64)

    def push_resident(self, slots: np.ndarray, rows: np.ndarray) -> None:
        k = len(slots)
        idx = (self.head + self.count + np.arange(k)) % self.slots
        self.ring[idx] = slots
        self.count += k
        self.source[slots] = rows

    def take_write_slots(self, want: int) -> np.ndarray:
        """Up to `want` slots: free ones first, then the oldest resident
        objects in ring order that no in-flight read holds; a held object
        met on the way goes to the young end of the ring (a second chance)
        instead of stopping the eviction there."""
        take = min(want, self.nfree)
        got = self.free[self.nfree - take:self.nfree][::-1].copy()
        self.nfree -= take
        want -= take
        if want > 0 and self.count > 0:
            idx = (self.head + np.arange(self.count)) % self.slots
            cand = self.ring[idx]
            idle = np.flatnonzero(self.refs[cand] == 0)
            k = min(want, len(idle))
            if k:
                scanned = int(idle[k - 1]) + 1          # objects looked at, oldest first
                held = cand[:scanned][self.refs[cand[:scanned]] != 0]
                ev = cand[idle[:k]]
                self.head = (self.head + scanned) % self.slots
                self.count -= scanned
                self.source[ev] = -1
                if len(held):
                    back = (self.head + self.count + np.arange(len(held))) % self.slots
                    self.ring[back] = held
                    self.count += len(held)
                got = np.concatenate([got, ev])
        return got

    def pick_resident(self, k: int, rng) -> np.ndarray:
        """k resident objects drawn uniformly (with repeats); holds them."""
        idx = (self.head + rng.integers(0, self.count, k)) % self.slots
        slots = self.ring[idx]
        np.add.at(self.refs, slots, 1)
        return slots

    def release(self, slots: np.ndarray) -> None:
        np.add.at(self.refs, slots, -1)

    def resident(self) -> np.ndarray:
        return self.ring[(self.head + np.arange(self.count)) % self.slots]


class _Class(SlotStore):
    """Device buffers of one class (views into the server's word pool, at the
    given word offsets) on top of its slot bookkeeping."""

    def __init__(self, geo: Geometry, slots: int, cap: int, depth: int, pool, offs):
        super().__init__(slots)
        self.geo = geo
        self.cap = cap
        self.pay = 2 * cap
        self.arena_off, self.payload_off, self.out_off = offs
        self.arena = pool[self.arena_off:self.arena_off + slots * geo.words]
        self.payload = pool[self.payload_off:self.payload_off + self.pay * geo.img_words]
        self.out = pool[self.out_off:self.out_off + depth * cap * geo.img_words]
        self.arena_ptr = self.arena.data_ptr()
        self.payload_ptr = self.payload.data_ptr()
        self.out_ptr = self.out.data_ptr()
        tmpl = mj.MojetteJob()
        tmpl.P, tmpl.Q, tmpl.n = geo.P, geo.Q, len(geo.dirs)
        for i, p in enumerate(geo.dirs):
            tmpl.dirs[i] = p
        self.template = tmpl


class Server:
    """The store and the loop.  `budget_bytes` covers the arenas, payload
    pools, output rings and staging; `per_iter_bytes` bounds one class's
    image bytes per kind per iteration (sets `cap`)."""

    def __init__(self, budget_bytes: int = 64 << 30, depth: int = 3, seed: int = 1,
                 geos=None, prefill: float = 0.5, per_iter_bytes: int = 16 << 20,
                 chunk_min_P: int = 1024, chunk_cols: int = 256, side_streams: int = 3,
                 chunk_max_reads: int = 1 << 30, long_reads: str = "chunked",
                 auto_backlog: int = 50000, auto_rate: float = float("inf")):
        import torch

        self.torch = torch
        self.dev = torch.device("cuda:0")
        self.geos = geos if geos is not None else geometries()
        self.depth = depth
        self.rng = np.random.default_rng(seed)
        self.stream = torch.cuda.Stream()
        self.stream_ptr = self.stream.cuda_stream
        self.L = mj.lib()
        caps = [int(max(4, min(4096, per_iter_bytes // (g.img_words * 8)))) for g in self.geos]
        stage_words = sum(2 * c + c // 4 + 1 for c in caps) + 64
        # Reads of long rows (P >= chunk_min_P) take one of two paths (with
        # "auto", per iteration: both ends while requests arrive faster than
        # auto_rate per second or more than auto_backlog wait, else chunked):
        #   "chunked"    chunked decode jobs (one chunk plan per code, a
        #                workspace per class and in-flight iteration) on side
        #                streams, joined into the iteration: short chains,
        #                twice the sweep work;
        #   "both_ends"  one descriptor-driven decode of every long read of
        #                the iteration, each block swept from both ends, on a
        #                side stream with a completion event of its own: the
        #                sweep work once, and the iteration's writes and
        #                short reads complete without waiting for it.
        # Measured (66 classes, 3 iterations in flight): with 64 MiB per
        # class and kind in an iteration, chunked keeps pace up to 1M req/s
        # and moves 322 GB/s at 2M with a growing queue (every iteration
        # full); with 128 MiB (96 GiB budget) it keeps pace at 2M (374 GB/s,
        # p99 22 ms).  Both ends at 3 in flight peaks at 126 GB/s: an
        # iteration's long reads take ~25 ms to sweep (chains of up to 16k
        # columns), and the iterations waiting on them hold the in-flight
        # window; with 6 in flight and 128 MiB it also keeps pace at 2M, at
        # a p99 of 38 ms (37 ms already at 1M).  With 384 MiB iterations (160
        # GiB budget, 3 in flight), "auto" switching at 1.5M arrivals/s keeps
        # pace at 3M req/s (555 GB/s, p99 33 ms) with the chunked path's
        # latency below (p50 0.9 ms at 10k req/s); switching on the backlog
        # alone came too late (3M: p99 186 ms).
        if long_reads not in ("chunked", "both_ends", "auto"):
            raise ValueError("long_reads is 'chunked', 'both_ends' or 'auto'")
        self.long_reads = long_reads
        self.auto_backlog = auto_backlog
        self.auto_rate = auto_rate
        self.busy = long_reads == "both_ends"   # this iteration's long reads from both ends
        self.chunk_min_P = chunk_min_P
        self.plans = {}
        ws_words = []
        for g, cap in zip(self.geos, caps):
            w = 0
            if chunk_min_P and g.P >= chunk_min_P and long_reads != "both_ends":
                key = (tuple(g.dirs), g.Q)
                if key not in self.plans:
                    self.plans[key] = mj.ChunkPlan(g.dirs, g.Q, chunk_cols)
                w = self.plans[key].workspace_words(g.P, cap)
            ws_words.append(w)
        # Writes and whole-block reads go through the descriptor-driven calls:
        # one plan over the codes, a descriptor per request (24 bytes) staged
        # with the slot lists, one workspace (the calls run in stream order).
        codes = []
        for g in self.geos:
            if (g.Q, tuple(g.dirs)) not in codes:
                codes.append((g.Q, tuple(g.dirs)))
        self.geom_id = [codes.index((g.Q, tuple(g.dirs))) for g in self.geos]
        # long rows that are not chunked decode from both ends in the
        # descriptor call (half the chain of a whole-block sweep, the same work)
        two = [{"decode_two_corner_min_P": chunk_min_P} for _ in codes] if chunk_min_P else None
        self.plan = mj.GeomPlan([(q, list(d)) for q, d in codes], two)
        self.max_desc = 2 * sum(caps)
        desc_words = 3 * self.max_desc
        stage_words += desc_words
        ws_bytes = self.plan.workspace_bytes(self.max_desc)
        # both ends: a descriptor-call workspace per side stream
        n_side_ws = side_streams if long_reads != "chunked" else 0
        fixed = sum((depth + 2) * c * g.img_words * 8 for c, g in zip(caps, self.geos))
        fixed += 2 * depth * stage_words * 8 + depth * 8 * sum(ws_words) + ws_bytes
        fixed += n_side_ws * ws_bytes
        if fixed >= budget_bytes:
            raise ValueError("budget too small for the payload pools and output rings")
        share = (budget_bytes - fixed) // len(self.geos)
        # one word pool holds every class's arena, payload pool and output ring
        layout, at = [], 0
        for c, (g, cap) in enumerate(zip(self.geos, caps)):
            slots = share // (g.words * 8)
            if slots < 2 * cap:
                raise ValueError(f"budget leaves class {c} fewer than {2 * cap} slots")
            offs = (at, at + slots * g.words, at + slots * g.words + 2 * cap * g.img_words)
            at = offs[2] + depth * cap * g.img_words
            layout.append((int(slots), offs))
        self.pool = torch.empty(at, dtype=torch.int64, device=self.dev)
        self.ws = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device=self.dev)
        self.ws_side = [torch.empty(max(1, ws_bytes), dtype=torch.uint8, device=self.dev)
                        for _ in range(n_side_ws)]
        self.cs = []
        for c, (g, cap) in enumerate(zip(self.geos, caps)):
            slots, offs = layout[c]
            st = _Class(g, slots, cap, depth, self.pool, offs)
            st.plan = self.plans.get((tuple(g.dirs), g.Q)) if ws_words[c] else None
            st.long = bool(chunk_min_P) and g.P >= chunk_min_P
            st.ws_words = ws_words[c]
            st.ws = (torch.empty(depth * ws_words[c], dtype=torch.int64, device=self.dev)
                     if ws_words[c] else None)
            self.cs.append(st)
        self.side = [torch.cuda.Stream() for _ in range(side_streams)]
        # Long-row reads are chunked in iterations of at most this many
        # reads (by default all): chunks cut a read's latency the most (a
        # 1 MB read in ~0.2 ms) at twice the sweep work.  Above the limit
        # long rows decode from both ends in the descriptor call, half the
        # chain of a one-sided sweep (~8 ms for a 1 MB object however many
        # share the chip).  Measured, sustained rate of the loop: always
        # chunked 188 GB/s at 1M requests/s; both ends above 1,024 reads
        # 93 GB/s at 500k; one-sided above 512 reads 89 GB/s.
        self.chunk_max_reads = chunk_max_reads
        for c, st in enumerate(self.cs):
            mj.mojette_fill_splitmix64(st.payload, st.payload.numel(), seed * 1000 + c,
                                       stream=self.stream_ptr)
        self.stage_words = stage_words
        self.h_stage = torch.empty(depth * stage_words, dtype=torch.int64).pin_memory()
        self.h_np = self.h_stage.numpy()
        self.d_stage = torch.empty(depth * stage_words, dtype=torch.int64, device=self.dev)
        self.d_stage_ptr = self.d_stage.data_ptr()
        self.status = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.jobs = [(mj.MojetteJob * mj.MAX_CLASSES)() for _ in range(2)]
        self.chunk_jobs = (mj.MojetteJob * mj.MAX_CLASSES)()
        self.iter_no = 0
        self._prefill(prefill)
        self.stream.synchronize()

    @property
    def budget_used(self) -> int:
        b = (self.h_stage.numel() + self.d_stage.numel()) * 8 + self.ws.numel()
        b += sum(w.numel() for w in self.ws_side)
        b += self.pool.numel() * 8
        for st in self.cs:
            b += st.ws.numel() * 8 if st.ws is not None else 0
        return b

    # ---- launches -----------------------------------------------------------

    def _run_chunked(self, entries, ring: int, stream_ptr: int) -> None:
        """Long-row classes' reads: chunked decode jobs in one call on
        `stream_ptr` (the library merges up to 8 classes per launch)."""
        arr = self.chunk_jobs
        size = ctypes.sizeof(mj.MojetteJob)
        for i, (c, nb, img, slots, erased) in enumerate(entries):
            st = self.cs[c]
            ctypes.memmove(ctypes.addressof(arr[i]), ctypes.addressof(st.template), size)
            a = arr[i]
            a.nblocks, a.images, a.projs, a.slots, a.erased = nb, img, st.arena_ptr, slots, erased
            a.plan = st.plan.handle
            a.workspace = st.ws.data_ptr() + ring * st.ws_words * 8
        rc = self.L.mojette_decode_jobs(arr, len(entries), self.status.data_ptr(), stream_ptr)
        if rc != mj.MOJETTE_OK:
            raise mj.MojetteError(rc, "mojette_decode_jobs")

    def _run_jobs(self, kind: str, entries) -> None:
        """entries: (class, nblocks, images ptr, slots ptr, erased ptr)."""
        arr = self.jobs[0 if kind == "w" else 1]
        size = ctypes.sizeof(mj.MojetteJob)
        for s in range(0, len(entries), mj.MAX_CLASSES):
            chunk = entries[s:s + mj.MAX_CLASSES]
            for i, (c, nb, img, slots, erased) in enumerate(chunk):
                st = self.cs[c]
                ctypes.memmove(ctypes.addressof(arr[i]), ctypes.addressof(st.template), size)
                a = arr[i]
                a.nblocks, a.images, a.projs, a.slots, a.erased = nb, img, st.arena_ptr, slots, erased
            if kind == "w":
                rc = self.L.mojette_encode_jobs(arr, len(chunk), self.stream_ptr)
            else:
                rc = self.L.mojette_decode_jobs(arr, len(chunk), self.status.data_ptr(),
                                                self.stream_ptr)
            if rc != mj.MOJETTE_OK:
                raise mj.MojetteError(rc, f"mojette_{'encode' if kind == 'w' else 'decode'}_jobs")

    def _prefill(self, frac: float) -> None:
        """Write objects into a fraction of every arena (set-up, untimed)."""
        torch = self.torch
        for c, st in enumerate(self.cs):
            want = int(st.slots * frac)
            while want > 0:
                b = min(want, st.pay)
                slots = st.take_write_slots(b)
                d = torch.from_numpy(slots).to(self.dev)
                with torch.cuda.stream(self.stream):
                    self._run_jobs("w", [(c, b, st.payload_ptr, d.data_ptr(), None)])
                self.stream.synchronize()
                st.push_resident(slots, np.arange(b))
                want -= b

    def _descriptors(self, at: int, entries) -> int:
        """Write descriptors (image_off, proj_off, P | geom_id | mask) at word
        `at` of the host stage; entries: (class, image word offsets, slots,
        masks or None).  Returns the number written."""
        hs = self.h_np
        k0 = 0
        for c, img_off, slots, masks in entries:
            st = self.cs[c]
            k = len(slots)
            d = hs[at + 3 * k0:at + 3 * (k0 + k)].reshape(k, 3)
            d[:, 0] = img_off
            d[:, 1] = st.arena_off + slots * st.geo.words
            w = np.full(k, st.geo.P | (self.geom_id[c] << 32), dtype=np.int64)
            if masks is not None:
                w |= masks.astype(np.int64) << 48
            d[:, 2] = w
            k0 += k
        return k0

    def _launch(self, writes, reads, trace: Trace):
        """Stage descriptors, slot lists and masks, copy them over, launch,
        record the completion events.  writes: (class, ids, slots, first
        payload row); reads: (class, ids, slots).  Writes and whole-block
        reads are one descriptor-driven encode and one decode over every
        class; long-row reads are chunked decode jobs on side streams, or
        (both ends) one more decode on a side stream.  Returns (begin event,
        completion event, ring slot, long-read completion event or None,
        classes whose reads it covers)."""
        torch = self.torch
        ring = self.iter_no % self.depth
        self.iter_no += 1
        base = ring * self.stage_words
        hs = self.h_np
        wd, rd, rl, ld = [], [], [], []
        for c, ids, slots, row0 in writes:
            st = self.cs[c]
            img = st.payload_off + (row0 + np.arange(len(slots))) * st.geo.img_words
            wd.append((c, img, slots, None))
        both = self.busy
        chunking = not both and sum(len(r[2]) for r in reads) <= self.chunk_max_reads
        for c, ids, slots in reads:
            st = self.cs[c]
            img = st.out_off + (ring * st.cap + np.arange(len(slots))) * st.geo.img_words
            if both and st.long:
                ld.append((c, img, slots, trace.mask[ids]))
            elif st.plan is None or not chunking:
                rd.append((c, img, slots, trace.mask[ids]))
        nw = self._descriptors(base, wd)
        nr = self._descriptors(base + 3 * nw, rd)
        nl = self._descriptors(base + 3 * (nw + nr), ld)
        pos = base + 3 * (nw + nr + nl)
        for c, ids, slots in reads:
            st = self.cs[c]
            if st.plan is None or not chunking:
                continue
            k = len(slots)
            hs[pos:pos + k] = slots
            nmw = (k + 3) // 4
            hs[pos + k + nmw - 1] = 0
            hs[pos + k:pos + k + nmw].view(np.uint16)[:k] = trace.mask[ids]
            out = st.out_ptr + ring * st.cap * st.geo.img_words * 8
            rl.append((c, k, out, self.d_stage_ptr + pos * 8, self.d_stage_ptr + (pos + k) * 8))
            pos += k + nmw
        begin = torch.cuda.Event(enable_timing=True)
        done = torch.cuda.Event(enable_timing=True)
        chunked = rl
        stage_u8 = self.d_stage.view(torch.uint8)
        with torch.cuda.stream(self.stream):
            begin.record(self.stream)
            self.d_stage[base:pos].copy_(self.h_stage[base:pos], non_blocking=True)
            joins = []
            if chunked:
                staged = torch.cuda.Event()
                staged.record(self.stream)
                # groups of 8 classes (one merged launch each), spread over the side streams
                groups = [chunked[i:i + 8] for i in range(0, len(chunked), 8)]
                per_side = [groups[k::len(self.side)] for k in range(len(self.side))]
                for side, grps in zip(self.side, per_side):
                    if not grps:
                        continue
                    side.wait_event(staged)
                    for g in grps:
                        self._run_chunked(g, ring, side.cuda_stream)
                    ev = torch.cuda.Event()
                    ev.record(side)
                    joins.append(ev)
            if nw:
                d = stage_u8[8 * base:8 * (base + 3 * nw)]
                mj.mojette_encode_batched(self.plan, d, nw, self.pool, self.ws, self.status,
                                          stream=self.stream_ptr)
            if nr:
                d = stage_u8[8 * (base + 3 * nw):8 * (base + 3 * (nw + nr))]
                mj.mojette_decode_batched(self.plan, d, nr, self.pool, self.ws, self.status,
                                          stream=self.stream_ptr)
            long_ev = None
            if nl:
                # every long read of the iteration, on a side stream of its own
                k = ring % len(self.side)
                side = self.side[k]
                staged = torch.cuda.Event()
                staged.record(self.stream)
                side.wait_event(staged)
                d = stage_u8[8 * (base + 3 * (nw + nr)):8 * (base + 3 * (nw + nr + nl))]
                mj.mojette_decode_batched(self.plan, d, nl, self.pool, self.ws_side[k],
                                          self.status, stream=side.cuda_stream)
                long_ev = torch.cuda.Event(enable_timing=True)
                long_ev.record(side)
            for ev in joins:
                self.stream.wait_event(ev)
            done.record(self.stream)
        return begin, done, ring, long_ev, {c for c, _, _, _ in ld}

    # ---- the loop -----------------------------------------------------------

    def run(self, trace: Trace, track=None, max_wall: float = 120.0):
        """Serve `trace` in real time.  Returns (completion times on the
        trace's clock, tracked results, counters).  `track`: request ids whose
        results are copied out at completion (tests)."""
        torch = self.torch
        N = len(trace.arrival)
        nq = 2 * len(self.cs)
        qid = trace.cls * 2 + trace.read
        order = np.argsort(qid, kind="stable")
        bounds = np.searchsorted(qid[order], np.arange(nq + 1))
        queues = [order[bounds[q]:bounds[q + 1]] for q in range(nq)]
        arrived = np.zeros(nq, dtype=np.int64)
        heads = np.zeros(nq, dtype=np.int64)
        done_t = np.full(N, np.nan)
        results = {}
        inflight = []
        seen = 0
        stats = {"iterations": 0, "max_queued": 0, "admitted": 0, "blocked_writes": 0,
                 "both_ends_iterations": 0}
        gpu_ms = 0.0
        rate_win = []   # (time, arrivals so far), about one a millisecond over 10 ms
        start = torch.cuda.Event(enable_timing=True)
        start.record(self.stream)
        start.synchronize()
        t0 = time.perf_counter()
        while True:
            # retire finished iterations (the oldest regardless, if the window is full)
            # (an iteration is done when its long reads are too: its ring
            # slot of staging and output rows is then free)
            while inflight and (len(inflight) >= self.depth or (
                    inflight[0][1].query() and (inflight[0][3] is None or inflight[0][3].query()))):
                begin, ev, ring, long_ev, long_cs, writes, reads = inflight.pop(0)
                ev.synchronize()
                gpu_ms += begin.elapsed_time(ev)
                t_long = None
                if long_ev is not None:
                    long_ev.synchronize()
                    gpu_ms += max(0.0, begin.elapsed_time(long_ev) - begin.elapsed_time(ev))
                    t_long = start.elapsed_time(long_ev) / 1e3
                self._retire(start.elapsed_time(ev) / 1e3, ring, writes, reads, done_t,
                             track, results, t_long, long_cs)
            now = time.perf_counter() - t0
            n_arr = int(np.searchsorted(trace.arrival, now, side="right"))
            if n_arr > seen:
                arrived += np.bincount(qid[seen:n_arr], minlength=nq)
                seen = n_arr
            if not rate_win or now - rate_win[-1][0] >= 1e-3:
                rate_win.append((now, seen))
                # keep the newest sample at least 10 ms old (a wait on a
                # completion event can leave no sample inside the window)
                while len(rate_win) > 1 and now - rate_win[1][0] >= 10e-3:
                    rate_win.pop(0)
            pending = arrived - heads
            stats["max_queued"] = max(stats["max_queued"], int(pending.sum()))
            writes, reads = [], []
            for q in np.flatnonzero(pending):
                c, is_read = divmod(int(q), 2)
                st = self.cs[c]
                h = int(heads[q])
                if is_read:
                    if st.count == 0:
                        continue
                    k = min(int(pending[q]), st.cap)
                    slots = st.pick_resident(k, self.rng)
                    reads.append((c, queues[q][h:h + k], slots))
                else:
                    slots = st.take_write_slots(min(int(pending[q]), st.cap))
                    k = len(slots)
                    if k == 0:
                        stats["blocked_writes"] += 1
                        continue
                    row0 = int(self.rng.integers(0, st.pay - k + 1))
                    writes.append((c, queues[q][h:h + k], slots, row0))
                heads[q] = h + k
                stats["admitted"] += k
            if writes or reads:
                if self.long_reads == "auto":
                    # the arrival rate over the last 10 ms, and the requests
                    # still waiting once this iteration is admitted
                    t_old, n_old = rate_win[0]
                    rate = (seen - n_old) / (now - t_old) if now - t_old >= 1e-3 else 0.0
                    self.busy = (rate > self.auto_rate or
                                 int((arrived - heads).sum()) > self.auto_backlog)
                    stats["both_ends_iterations"] += int(self.busy)
                inflight.append((*self._launch(writes, reads, trace), writes, reads))
                stats["iterations"] += 1
            elif seen == N and not inflight and (heads == arrived).all():
                break
            elif inflight:
                time.sleep(10e-6)
            else:
                nxt = trace.arrival[seen] if seen < N else now
                time.sleep(max(0.0, min(nxt - now, 1e-3)))
            if time.perf_counter() - t0 > max_wall:
                raise RuntimeError("serving loop exceeded its wall-clock limit")
        self.stream.synchronize()
        stats["gpu_busy_s"] = round(gpu_ms / 1e3, 4)
        stats["wall_s"] = round(time.perf_counter() - t0, 4)
        return done_t, results, stats

    def _retire(self, t_done, ring, writes, reads, done_t, track, results, t_long=None,
                long_cs=()) -> None:
        for c, ids, slots, row0 in writes:
            st = self.cs[c]
            done_t[ids] = t_done
            rows = row0 + np.arange(len(slots))
            st.push_resident(slots, rows)
            if track:
                g = st.geo
                for rid, s, row in zip(ids, slots, rows):
                    if int(rid) in track:
                        results[int(rid)] = ("w", c, int(s), int(row),
                                             st.arena[s * g.words:(s + 1) * g.words].cpu())
        for c, ids, slots in reads:
            st = self.cs[c]
            done_t[ids] = t_long if c in long_cs else t_done
            st.release(slots)
            if track:
                g = st.geo
                for j, (rid, s) in enumerate(zip(ids, slots)):
                    if int(rid) in track:
                        o = (ring * st.cap + j) * g.img_words
                        results[int(rid)] = ("r", c, int(s), int(st.source[s]),
                                             st.out[o:o + g.img_words].cpu())


def summarize(trace: Trace, done_t: np.ndarray, stats: dict) -> dict:
    """p50/p99 latency (arrival to completion), sustained user GB/s."""
    lat = done_t - trace.arrival
    ok = np.isfinite(lat)
    span = float(np.nanmax(done_t)) if ok.any() else float("nan")
    rd = ok & (trace.read == 1)
    wr = ok & (trace.read == 0)

    def pct(x, q):
        return round(float(np.percentile(x, q)) * 1e6, 1) if len(x) else None

    return {
        "requests": int(len(lat)),
        "completed": int(ok.sum()),
        "offered_qps": round(len(lat) / float(trace.arrival[-1]), 1) if len(lat) > 1 else None,
        "p50_us": pct(lat[ok], 50), "p99_us": pct(lat[ok], 99),
        "read_p50_us": pct(lat[rd], 50), "read_p99_us": pct(lat[rd], 99),
        "write_p50_us": pct(lat[wr], 50), "write_p99_us": pct(lat[wr], 99),
        "GBps": round(float(trace.size[ok].sum()) / span / 1e9, 3) if span > 0 else None,
        "span_s": round(span, 4),
        **stats,
    }
