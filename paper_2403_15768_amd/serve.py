"""Continuous-batching serving loop for nanotube design queries.

A query is a nanotube design: radius R (box 512 x (2R+8)^2), relaxation time,
pressure-gradient force and the spectral parameters of its wall friction
(paper Sec. 5.1: permeability of carbon nanotubes against diameter and
charge-carrier density).  The server

* admits arrived queries, first come first served, while their device
  footprint fits the HBM budget (each admitted query owns a context whose
  state stays resident on the GPU);
* computes each query's wall friction with the GPU quadrature once;
* advances every active query in rounds of 64 steps (one graph replay per
  group of a batch), and between rounds lets queries join and leave the
  running batch (lbm_batch_add / lbm_batch_remove: only the groups they
  touch get new work lists, the batch itself is never rebuilt);
* checks each query on its own step counter every ``check_every`` steps (a
  multiple of 64) and retires it when its flux changed by less than
  ``rel_tol`` relative over that interval, freeing its memory.

``mode="f32"`` runs every query in FP32 storage (FP64 arithmetic).
``mode="mixed"`` runs a query first with half-precision storage (FP32
arithmetic) until its flux change per check falls below ``switch_tol`` or
stops shrinking, then hands its state to an FP32 context
(``lbm_transfer_state``) which joins the FP32 batch and converges to the same
``rel_tol``: both modes end at the same accuracy.

A query's trajectory depends only on its own parameters and step counter,
so its result is the same alone and in any mix, bit for bit.

Scheduling, admission and bookkeeping are host logic here; every numerical
step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time
from collections import deque
from dataclasses import asdict, dataclass, field

import numpy as np

from . import inputs, lbm


@dataclass
class Result:
    qid: int
    radius: int
    tau: float
    arrival_s: float
    admitted_s: float
    done_s: float
    steps: int
    steps_half: int
    flux: float
    status: str  # "ok", "not_converged", "diverged"
    # the final u_x field [z][y][x], kept only when the server is asked to
    ux: np.ndarray | None = field(default=None, repr=False, compare=False)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclass
class _Slot:
    query: inputs.Query
    ch: lbm.Channel
    phase: str  # "half" or "f32"
    admitted_s: float
    reserved: int
    prev_q: float | None = None
    prev_rel: float | None = None
    steps_half: int = 0
    steps: int = 0  # the context's step counter, kept on the host side
    cells: int = 0  # fluid cells


def tube_params(q: inputs.Query):
    ny, nz, cy, cz = inputs.tube_box(q.radius)
    return dict(lattice=lbm.D3Q19, geometry=lbm.TUBE, nx=q.nx, ny=ny, nz=nz, tau=q.tau,
                force=(q.g, 0.0, 0.0), tube_radius=float(q.radius), tube_cy=cy, tube_cz=cz)


class TubeQueries:
    """Nanotube design queries: friction from the spectral quadrature."""

    @staticmethod
    def params(q) -> dict:
        return tube_params(q)

    @staticmethod
    def set_friction(ch: lbm.Channel, q) -> None:
        kw = tube_params(q)
        om = inputs.tube_plasmon_frequencies(ch.wall_coords(), kw["nx"], q.radius, kw["tube_cy"],
                                             kw["tube_cz"], q.spectral.omega0,
                                             inputs.rng_for("serving", 1000 + q.qid))
        ch.set_friction_spectral(q.spectral, om)


class DuctQueries:
    """Rectangular ducts (inputs.Channel specs): smooth random friction field."""

    @staticmethod
    def params(q) -> dict:
        return dict(lattice=lbm.D3Q19, geometry=lbm.DUCT, nx=q.nx, ny=q.ny, nz=q.nz, tau=q.tau,
                    force=(q.g, 0.0, 0.0), tube_radius=0.0, tube_cy=0.0, tube_cz=0.0)

    @staticmethod
    def set_friction(ch: lbm.Channel, q) -> None:
        ch.set_friction(inputs.duct_friction(ch.wall_coords(), q.nx, q.ny, q.nz,
                                             inputs.rng_for("batch", q.seed_index)))


def footprint(q, precision: str, kind=TubeQueries) -> int:
    kw = kind.params(q)
    p = lbm.make_params(kw["lattice"], kw["geometry"], kw["nx"], kw["ny"], kw["nz"], kw["tau"],
                        kw["force"], precision, 1.0, kw["tube_radius"], kw["tube_cy"], kw["tube_cz"])
    return lbm.footprint(p)


def open_channel(q, precision: str, kind=TubeQueries) -> lbm.Channel:
    kw = kind.params(q)
    ch = lbm.Channel(kw["lattice"], kw["geometry"], kw["nx"], kw["ny"], kw["nz"], kw["tau"],
                     kw["force"], precision, 1.0, kw["tube_radius"], kw["tube_cy"], kw["tube_cz"])
    kind.set_friction(ch, q)
    return ch


ROUND = 64  # steps per round: one graph replay per batch group


class Server:
    def __init__(self, mode: str = "f32", hbm_budget: int = 32 << 30, check_every: int = 1024,
                 rel_tol: float = 1e-8, switch_tol: float = 1e-5, max_steps: int = 500_000,
                 tune: bool = True, realtime: bool = True, log=None, kind=TubeQueries,
                 keep_fields: bool = False, max_members: int = 2048):
        assert mode in ("f32", "mixed")
        if check_every % ROUND or check_every < 2 * ROUND:
            raise ValueError(f"check_every must be a multiple of {ROUND}, at least {2 * ROUND}")
        self.kind = kind
        self.mode = mode
        self.budget = int(hbm_budget)
        self.check_every = int(check_every)
        self.rel_tol = rel_tol
        self.switch_tol = switch_tol
        self.max_steps = max_steps
        self.tune = tune
        self.realtime = realtime
        self.log = log
        self.keep_fields = keep_fields
        self.max_members = int(max_members)
        self.shape = None  # workgroup shape chosen by the autotuner
        self.tuning = {}   # per phase: the autotuner's choice
        self.stats = {"batch_rebuilds": 0, "rounds": 0, "joins": 0, "leaves": 0,
                      "max_active": 0, "lattice_updates": 0, "batch_bytes": 0,
                      "host_wait_s": 0.0, "check_s": 0.0}

    # ------------------------------------------------------------- helpers
    def _say(self, *a):
        if self.log:
            self.log(" ".join(str(x) for x in a))

    def _reserve(self, q) -> int:
        # mixed mode ends in FP32 and holds both contexts during the hand-off
        f32 = footprint(q, "f32", self.kind)
        return f32 + (footprint(q, "f16s", self.kind) if self.mode == "mixed" else 0)

    def _open(self, q, precision) -> lbm.Channel:
        kw = self.kind.params(q)
        return lbm.Channel(kw["lattice"], kw["geometry"], kw["nx"], kw["ny"], kw["nz"], kw["tau"],
                           kw["force"], precision, 1.0, kw["tube_radius"], kw["tube_cy"],
                           kw["tube_cz"])

    def _admit(self, q, now) -> _Slot:
        ch = self._open(q, "f16s" if self.mode == "mixed" else "f32")
        self.kind.set_friction(ch, q)
        s = _Slot(query=q, ch=ch, phase="half" if self.mode == "mixed" else "f32",
                  admitted_s=now, reserved=self._reserve(q), steps=ch.step_count,
                  cells=ch.fluid_count)
        return s

    # the batches: one per phase, of a capacity for what the budget can hold
    def _capacity(self, phase: str, need_items: int = 0, need_cols: int = 0) -> dict:
        bytes_per_cell = 2 * 19 * (2 if phase == "half" else 4)
        cells = self.budget // bytes_per_cell
        return dict(max_members=self.max_members,
                    max_items=max(2 * need_items, cells // 24 + 4096),
                    max_columns=max(2 * need_cols, cells // 32 + 1024))

    def _join(self, phase: str, s: _Slot) -> None:
        b = self._batches.get(phase)
        it, co = lbm.member_cost(s.ch)
        load = self._load.setdefault(phase, [0, 0])
        if b is not None and (load[0] + it > b.cap["max_items"] or
                              load[1] + co > b.cap["max_columns"]):
            # out of room (more than the budget estimate held): a bigger batch
            # takes the members over
            members = [c for c in b.channels if c is not None]
            cap = self._capacity(phase, load[0] + it, load[1] + co)
            nb = self._new_batch(phase, cap)
            for c in members:
                b.remove(c)
                nb.add(c)
            self._drop_batch(b)
            self.stats["batch_rebuilds"] += 1
            b = nb
        if b is None:
            b = self._new_batch(phase, self._capacity(phase))
        b.add(s.ch)
        load[0] += it
        load[1] += co
        self.stats["joins"] += 1

    def _leave(self, phase: str, s: _Slot) -> None:
        b = self._batches[phase]
        b.remove(s.ch)
        it, co = lbm.member_cost(s.ch)
        self._load[phase][0] -= it
        self._load[phase][1] -= co
        self.stats["leaves"] += 1

    def _new_batch(self, phase: str, cap: dict) -> lbm.Batch:
        prec = "f16s" if phase == "half" else "f32"
        kw = self.kind.params(self._any_query)
        b = lbm.Batch.empty(kw["lattice"], prec, kw["geometry"] == lbm.TUBE, **cap)
        b.cap = cap
        b.tuned = False
        self._batches[phase] = b
        self._batch_bytes += b.arena.numel()
        self.stats["batch_bytes"] = max(self.stats["batch_bytes"], self._batch_bytes)
        return b

    def _drop_batch(self, b) -> None:
        self._batch_bytes -= b.arena.numel()
        b.close()

    def _hand_off(self, s: _Slot) -> None:
        self._leave("half", s)
        f32 = self._open(s.query, "f32")
        f32.transfer_from(s.ch)
        s.ch.close()
        s.ch = f32
        s.phase = "f32"
        s.steps_half = f32.step_count
        self._join("f32", s)

    def _maybe_tune(self, phase: str, b: lbm.Batch, waiting: int) -> None:
        # once per phase, when the batch holds a representative mix (or all
        # that will come at once)
        if not self.tune or b.tuned or (b.members < 4 and waiting):
            return
        b.tune()
        b.tuned = True
        self.tuning[phase] = b.tuning
        if phase == ("half" if self.mode == "mixed" else "f32"):
            self.shape = b.shape

    # ------------------------------------------------------------- the loop
    def run(self, trace: list) -> list[Result]:
        import torch

        trace = sorted(trace, key=lambda q: getattr(q, "arrival_s", 0.0))
        if not self.realtime:  # saturation: every query is there at t = 0
            trace = [dataclasses.replace(q, arrival_s=0.0) for q in trace]
        if not trace:
            return []
        self._any_query = trace[0]
        self._batches: dict = {}
        self._load: dict = {}
        self._batch_bytes = 0
        clock = time.perf_counter
        t0 = clock()
        now = lambda: clock() - t0
        i, n = 0, len(trace)
        waiting: deque = deque()
        active: list[_Slot] = []
        used = 0
        results: list[Result] = []
        # The checks after a round are enqueued with it (flux and mass into
        # pinned host rows) and read one round later, after the next round
        # has been queued: the GPU never waits for the host's bookkeeping.  A
        # query's decision therefore lands one round after its check, alone
        # or in any mix alike.  At most two rounds are queued ahead of the
        # GPU, so that a query joins within a round or two of its admission.
        ring = torch.empty((4 * self.max_members, 3), dtype=torch.float64, pin_memory=True)
        next_row = 0
        pending = None  # (event, [(slot, row, steps at the check)])
        while i < n or waiting or active:
            t = now()
            while i < n and getattr(trace[i], "arrival_s", 0.0) <= t:
                waiting.append(trace[i])
                i += 1
            # admission by device footprint (the batches' own arenas counted),
            # first come first served
            while waiting and (used + self._batch_bytes + self._reserve(waiting[0])
                               <= self.budget):
                q = waiting.popleft()
                s = self._admit(q, now())
                used += s.reserved
                active.append(s)
                self._join(s.phase, s)
            if waiting and not active:
                raise RuntimeError(f"query {waiting[0].qid} does not fit the HBM budget")
            if not active:
                if i < n and self.realtime:
                    time.sleep(max(0.0, min(0.05, trace[i].arrival_s - now())))
                continue
            self.stats["max_active"] = max(self.stats["max_active"], len(active))
            # one round for every active query
            for phase, b in self._batches.items():
                if b.members:
                    self._maybe_tune(phase, b, len(waiting) + (n - i))
                    b.step(ROUND)
            self.stats["rounds"] += 1
            self.stats["lattice_updates"] += ROUND * sum(s.cells for s in active)
            # checks on each query's own step counter, enqueued behind the round
            enq = []
            for s in active:
                s.steps += ROUND
                if s.steps % self.check_every == 0:
                    row = ring[next_row]
                    next_row = (next_row + 1) % ring.shape[0]
                    s.ch.invariants_async(row)
                    enq.append((s, row, s.steps))
            ev = torch.cuda.Event()
            ev.record()
            done, pending = pending, (ev, enq)
            if done is None:
                continue
            t_w = clock()
            done[0].synchronize()
            self.stats["host_wait_s"] += clock() - t_w
            if not done[1]:
                continue
            t_c = clock()
            retire: list[tuple[_Slot, str]] = []
            for s, row, steps in done[1]:
                q = float(row[0])
                if not math.isfinite(q):
                    retire.append((s, "diverged"))
                    continue
                rel = abs(q - s.prev_q) / abs(q) if s.prev_q is not None and q != 0 else math.inf
                if s.phase == "f32" and rel < self.rel_tol:
                    retire.append((s, "ok"))
                elif steps >= self.max_steps:
                    retire.append((s, "not_converged"))
                elif s.phase == "half" and (rel < self.switch_tol or (
                        rel < 1e-4 and s.prev_rel is not None and rel > 0.7 * s.prev_rel)):
                    s.prev_rel = rel
                    s.prev_q = q
                    self._hand_off(s)
                    continue
                s.prev_rel = rel
                s.prev_q = q
            t_done = now()
            for s, status in retire:
                active.remove(s)
                used -= s.reserved
                self._leave(s.phase, s)  # after the queued round: the final state
                try:
                    q = s.ch.invariants()[0]
                except lbm.LBMError:
                    q = math.nan
                steps = s.ch.step_count
                results.append(Result(qid=s.query.qid, radius=getattr(s.query, "radius", 0),
                                      tau=s.query.tau,
                                      arrival_s=getattr(s.query, "arrival_s", 0.0),
                                      admitted_s=s.admitted_s,
                                      done_s=t_done, steps=steps,
                                      steps_half=s.steps_half, flux=q, status=status,
                                      ux=s.ch.field(1) if self.keep_fields else None))
                s.ch.close()
                self._say(f"done q{s.query.qid} steps={steps} "
                          f"half={s.steps_half} t={t_done:.2f}s active={len(active)}")
            self.stats["check_s"] += clock() - t_c
        torch.cuda.synchronize()
        for b in list(self._batches.values()):
            self._drop_batch(b)
        self._batches = {}
        return sorted(results, key=lambda r: r.qid)


def summarize(results: list[Result], wall_s: float) -> dict:
    lat = np.array([r.latency_s for r in results])
    ok = [r for r in results if r.status == "ok"]
    first = min(r.arrival_s for r in results)
    last = max(r.done_s for r in results)
    return {"queries": len(results), "converged": len(ok),
            "solves_per_s": round(len(ok) / max(last - first, 1e-9), 4),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
            "makespan_s": round(last - first, 3), "wall_s": round(wall_s, 3),
            "mean_steps": round(float(np.mean([r.steps for r in results])), 1),
            "mean_steps_half": round(float(np.mean([r.steps_half for r in results])), 1)}


def main(argv=None):
    ap = argparse.ArgumentParser(description="serve a Poisson trace of nanotube queries")
    ap.add_argument("--queries", type=int, default=500)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--mode", default="f32", choices=["f32", "mixed"])
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--rmin", type=int, default=8)
    ap.add_argument("--rmax", type=int, default=32)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--check-every", type=int, default=1024)
    ap.add_argument("--out", default=None)
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args(argv)
    import torch

    lbm.load()
    torch.cuda.set_device(0)
    trace = inputs.serving_trace(args.queries, args.rate, args.nx, (args.rmin, args.rmax))
    srv = Server(mode=args.mode, hbm_budget=int(args.budget_gb * (1 << 30)),
                 check_every=args.check_every,
                 log=(lambda m: print(m, flush=True)) if args.verbose else None)
    t0 = time.perf_counter()
    res = srv.run(trace)
    wall = time.perf_counter() - t0
    summ = summarize(res, wall)
    summ.update(mode=args.mode, rate=args.rate, budget_gb=args.budget_gb,
                radius=[args.rmin, args.rmax], shape=srv.shape, **srv.stats)
    print(json.dumps(summ), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summ,
                       "results": [{k: v for k, v in asdict(r).items() if k != "ux"} for r in res]},
                      f)


if __name__ == "__main__":
    main()
