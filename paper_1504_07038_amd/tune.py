"""Decode schedule autotuner with a learned cost model.

A decode workload is a code (k, m), a row length P, a batch of nblocks
blocks and a number of erasures per block.  Its schedules:
  ("whole", nb)      every block swept whole, nb blocks per wavefront
                     (mojette_decode_batch_tuned);
  ("two_corner", 0)  every block swept from both ends, half the chain
                     (mojette_decode_batch_two_corner);
  ("chunked", cols)  the sweep of every block cut into chunks of about cols
                     columns (mojette_decode_batch_chunked).
The best one depends on the workload: few long blocks want chunks, many
short blocks want full wavefronts.  The tuner measures schedules with HIP
events; its cost model, a small perceptron trained on the GPU by the
library's own forward/backward/Adam kernels, predicts log(time) from the
workload and the schedule, so that a new workload is tuned by measuring only
the few schedules the model ranks best instead of all of them.

This module only picks launch parameters; every schedule it can pick
decodes bit-identically.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import paper_1504_07038_amd as mj

TILE = 16                          # decode tile width (columns)
CHUNK_COLS = (128, 256, 512, 1024, 2048)
N_FEATURES = 9


@dataclass(frozen=True)
class Workload:
    k: int
    m: int
    P: int
    nblocks: int
    erasures: int

    @property
    def dirs(self):
        n = self.k + self.m
        return [i - n // 2 for i in range(n)]

    @property
    def user_bytes(self) -> int:
        return self.nblocks * self.P * self.k * 8


def candidates(w: Workload):
    """Every schedule the tuner considers for w."""
    full = mj.mojette_decode_max_blocks_per_wave(w.dirs, w.P, w.k)
    out = [("whole", mj.mojette_decode_default_blocks_per_wave(w.dirs, w.P, w.k))]
    nb = full
    while nb >= 1 and len(out) < 5:
        if ("whole", nb) not in out:
            out.append(("whole", nb))
        nb //= 2
    out.append(("two_corner", 0))
    for cols in CHUNK_COLS:
        if (w.P // TILE) // (cols // TILE) >= 2:
            out.append(("chunked", cols))
    return out


def rule_schedule(w: Workload):
    """A two-line rule for comparison with the learned model: chunks of 256
    columns for a few long blocks, the library's default otherwise."""
    if w.nblocks <= 32 and w.P >= 1024:
        return ("chunked", 256)
    return default_schedule(w)


def default_schedule(w: Workload):
    """The untuned method: whole blocks, the library's blocks per wavefront."""
    return ("whole", mj.mojette_decode_default_blocks_per_wave(w.dirs, w.P, w.k))


def features(w: Workload, s) -> np.ndarray:
    kind, val = s
    f = np.zeros(N_FEATURES, dtype=np.float64)
    f[0] = math.log2(w.P) / 8.0
    f[1] = w.k / 8.0
    f[2] = (w.k + w.m) / 8.0
    f[3] = math.log2(w.nblocks + 1) / 8.0
    f[4] = 1.0 if kind == "chunked" else 0.0
    if kind == "whole":
        f[5] = math.log2(val) / 5.0
        f[7] = math.log2(max(1, math.ceil(w.nblocks / val))) / 8.0   # wavefronts
    elif kind == "two_corner":
        f[8] = 1.0
        half = max(1, mj.mojette_decode_max_blocks_per_wave(w.dirs, w.P, w.k) // 2)
        f[5] = math.log2(half) / 5.0
        f[7] = math.log2(max(1, math.ceil(2 * w.nblocks / half))) / 8.0
    else:
        f[6] = math.log2(val) / 8.0
        chunks = (w.P // TILE) // (val // TILE)
        f[7] = math.log2(w.nblocks * chunks) / 8.0                    # parallel chunks
    return f


class Bench:
    """Device data of workloads and event-timed runs of their schedules."""

    def __init__(self, seed: int = 1504, reps: int = 5):
        import torch

        self.torch = torch
        self.seed = seed
        self.reps = reps
        self.plans = {}
        self.cur = None

    def plan(self, w: Workload, cols: int):
        key = (tuple(w.dirs), w.k, cols)
        if key not in self.plans:
            self.plans[key] = mj.ChunkPlan(w.dirs, w.k, cols)
        return self.plans[key]

    def prepare(self, w: Workload):
        import synth

        torch = self.torch
        if self.cur is not None and self.cur[0] == w:
            return self.cur
        words = mj.mojette_block_words(w.dirs, w.P, w.k)
        img = torch.empty(w.nblocks * w.P * w.k, dtype=torch.int64, device="cuda")
        mj.mojette_fill_splitmix64(img, img.numel(), self.seed)
        proj = torch.empty(w.nblocks * words, dtype=torch.int64, device="cuda")
        mj.mojette_encode_batch(img, w.nblocks, w.P, w.k, w.dirs, proj)
        masks = synth.erasure_masks(self.seed + 1, w.nblocks, w.k + w.m, w.erasures)
        d_mask = torch.from_numpy(masks.view(np.int16)).cuda()
        out = torch.empty_like(img)
        self.cur = (w, img, proj, d_mask, out)
        return self.cur

    def run(self, w: Workload, s, check: bool = False) -> float:
        """Median time (ms) of schedule s on w."""
        torch = self.torch
        _, img, proj, d_mask, out = self.prepare(w)
        kind, val = s
        if kind == "whole":
            def call():
                mj.mojette_decode_batch_tuned(proj, d_mask, w.nblocks, w.P, w.k, w.dirs, out, val)
        elif kind == "two_corner":
            def call():
                mj.mojette_decode_batch_two_corner(proj, d_mask, w.nblocks, w.P, w.k, w.dirs, out,
                                                   blocks_per_wave=val)
        else:
            plan = self.plan(w, val)
            ws = torch.empty(max(1, plan.workspace_words(w.P, w.nblocks)), dtype=torch.int64,
                             device="cuda")

            def call():
                mj.mojette_decode_batch_chunked(plan, proj, d_mask, w.nblocks, w.P, out, ws)
        st = torch.cuda.current_stream()
        call()
        torch.cuda.synchronize()
        if check and not torch.equal(out, img):
            raise AssertionError(f"schedule {s} decoded {w} wrongly")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(self.reps)]
        for a, b in evs:
            a.record(st)
            call()
            b.record(st)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in evs]))


class CostModel:
    """log(time) predictor: the library's fp32 perceptron, trained with its
    own gradient and Adam kernels (full batch)."""

    def __init__(self, hidden: int = 32, seed: int = 0):
        import torch

        self.torch = torch
        self.D, self.H = N_FEATURES, hidden
        n = mj.mojette_mlp_params(self.D, self.H)
        rng = np.random.default_rng(seed)
        # He-scaled normal weights, zero biases
        p = np.concatenate([rng.normal(0, math.sqrt(2.0 / self.D), self.H * self.D),
                            np.zeros(self.H),
                            rng.normal(0, math.sqrt(2.0 / self.H), self.H * self.H),
                            np.zeros(self.H), rng.normal(0, math.sqrt(1.0 / self.H), self.H),
                            np.zeros(1)])
        assert len(p) == n
        self.params = torch.from_numpy(p.astype(np.float32)).cuda()
        self.mu, self.sd = 0.0, 1.0
        self.losses = []

    def fit(self, X: np.ndarray, y: np.ndarray, steps: int = 2000, lr: float = 3e-3) -> float:
        torch = self.torch
        self.mu, self.sd = float(np.mean(y)), float(np.std(y) + 1e-9)
        d_x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        d_t = torch.from_numpy(((y - self.mu) / self.sd).astype(np.float32)).cuda()
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        g = torch.empty(self.params.numel() + 1, dtype=torch.float32, device="cuda")
        ws = torch.empty(mj.mojette_mlp_grad_workspace(self.D, self.H, len(y)),
                         dtype=torch.float32, device="cuda")
        for step in range(1, steps + 1):
            mj.mojette_mlp_grad(self.params, self.D, self.H, d_x, d_t, g, ws)
            mj.mojette_mlp_adam(self.params, g[:-1], m, v, lr, 0.9, 0.999, 1e-8, step)
            if step % 250 == 0 or step == steps:
                self.losses.append(float(g[-1]))
        return self.losses[-1]

    def predict(self, X: np.ndarray) -> np.ndarray:
        torch = self.torch
        d_x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        d_y = torch.empty(len(X), dtype=torch.float32, device="cuda")
        mj.mojette_mlp_forward(self.params, self.D, self.H, d_x, d_y)
        return d_y.cpu().numpy().astype(np.float64) * self.sd + self.mu


class Tuner:
    def __init__(self, bench: Bench, model: CostModel | None = None):
        self.bench = bench
        self.model = model

    def measure_all(self, w: Workload):
        """Exhaustive tuning: {schedule: ms}."""
        return {s: self.bench.run(w, s) for s in candidates(w)}

    def dataset(self, table):
        """table: {workload: {schedule: ms}} -> (X, log ms)."""
        X, y = [], []
        for w, times in table.items():
            for s, t in times.items():
                X.append(features(w, s))
                y.append(math.log(t))
        return np.array(X), np.array(y)

    def rank(self, w: Workload):
        """Candidates ordered by predicted time."""
        cands = candidates(w)
        pred = self.model.predict(np.array([features(w, s) for s in cands]))
        return [cands[i] for i in np.argsort(pred)]

    def choose(self, w: Workload, budget: int = 2, times=None):
        """Measure the `budget` best-ranked schedules (from `times` when they
        were measured already) and keep the fastest."""
        best = None
        for s in self.rank(w)[:max(1, budget)]:
            t = times[s] if times is not None else self.bench.run(w, s)
            if best is None or t < best[1]:
                best = (s, t)
        return best


# ---- schedules of a plan over codes (descriptor-driven batched calls) ----
#
# A plan gives every code one schedule for all of its blocks, whatever their
# row length: the decode's blocks per wavefront, ring split and the row
# length from which blocks decode from both ends, the encode's tile width.  The tuner starts from the library's choices and accepts a
# change only when a step of the actual workload (encode + decode of a
# sample of its blocks, the launches the plan makes) measures faster, so the
# schedule it returns is never slower than the untuned one on that sample.
# The cost model ranks the decode candidates of each code over the code's
# row-length classes, so that only the best-ranked ones are measured.

ENCODE_TILES = (64, 128, 256)
TWO_CORNER_MIN_P = (8192, 1024)    # rows at least this long decode from both ends


def decode_candidates(k: int, m: int):
    """Blocks per wavefront the tuner tries for code (k, m) (0: the library's)."""
    n = k + m
    dirs = [i - n // 2 for i in range(n)]
    full = mj.mojette_decode_max_blocks_per_wave(dirs, 64, k)
    out, nb = [], max(1, full // 2)
    while nb >= 1 and len(out) < 4:
        out.append(nb)
        nb //= 2
    return out


class PlanTuner:
    """measure(tune) -> median step ms of the workload sample with a plan made
    with that tune (a list of per-code mojette_tune dicts)."""

    def __init__(self, codes, classes, measure, model: CostModel | None = None,
                 budget: int = 2, margin: float = 0.01):
        self.codes = list(codes)            # [(k, m)]
        self.classes = classes              # {code index: [(P, nblocks)]}
        self.measure = measure
        self.model = model
        self.budget = budget
        self.margin = margin
        self.history = []

    def rank_decode(self, g: int):
        k, m = self.codes[g]
        cands = decode_candidates(k, m)
        if self.model is None or not self.classes.get(g):
            return cands
        totals = []
        for nb in cands:
            X = np.array([features(Workload(k, m, P, cnt, m), ("whole", nb))
                          for P, cnt in self.classes[g]])
            totals.append(float(np.sum(np.exp(self.model.predict(X)))))
        return [cands[i] for i in np.argsort(totals)]

    def _try(self, tune, g, key, val, best_ms):
        trial = [dict(t) for t in tune]
        trial[g][key] = val
        ms = self.measure(trial)
        self.history.append((g, key, val, ms))
        if ms < best_ms * (1.0 - self.margin):
            return trial, ms
        return tune, best_ms

    def tune(self):
        tune = [dict() for _ in self.codes]
        default_ms = self.measure(tune)
        self.history.append((None, "default", None, default_ms))
        best_ms = default_ms
        for g in range(len(self.codes)):
            for nb in self.rank_decode(g)[:self.budget]:
                tune, best_ms = self._try(tune, g, "decode_blocks_per_wave", nb, best_ms)
            tune, best_ms = self._try(tune, g, "decode_ring_split", -1, best_ms)
            for pmin in TWO_CORNER_MIN_P:
                tune, best_ms = self._try(tune, g, "decode_two_corner_min_P", pmin, best_ms)
            for w in ENCODE_TILES:
                if w != 128:
                    tune, best_ms = self._try(tune, g, "encode_tile_cols", w, best_ms)
        return tune, best_ms, default_ms
