#!/usr/bin/env python3
"""Benchmark of the lattice-Boltzmann nanochannel hot path on one MI355X.

Headline: D3Q19 MLUPS (fluid-cell lattice updates per second) of the fused
pull stream-collide with the Navier-slip friction wall on the 256 x 128 x 64
rectangular duct (tau 0.7, g 1e-6, smooth random wall friction, FP32
population storage), with the HBM roofline fraction of the stream-collide
kernel and the CPU oracle timed on the same workload.

A "step" is one lattice time step of the whole duct; every ``--check-every``
steps the flux and mass are reduced in FP64 and brought to the host, as the
run-to-steady loop does (the last step of each chunk sums them as it goes).
Per-query set-up (geometry, friction field -> wall weights, rest state)
happens before the timed region.

The same line carries the rest of the metric: the 256-duct batch run to
steady (solves/s, p50 / p99 time-to-steady) and short serving traces of
nanotube queries, each in FP32 storage and in mixed precision.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 MLUPS + % of HBM roofline; batched solves/s and p99 time-to-steady"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 152, "f64": 304, "f16s": 76}  # 19 reads + 19 writes
DUCT = (256, 128, 64)
KERNEL_SOURCES = ["paper_2403_15768_amd/csrc/lbm_device.h",
                  "paper_2403_15768_amd/csrc/lbm_kernels.hip"]
# counter-measured HBM bytes per launch of the dominant kernel, per workload
# and storage (no noise, periodic ends); used while the kernel sources match
COUNTERS = {
    ("duct", "f32"): os.path.join(ROOT, "profiles",
                                  "stream_collide_duct_256x128x64_f32.counters.json"),
    ("duct", "f64"): os.path.join(ROOT, "profiles",
                                  "stream_collide_duct_256x128x64_f64.counters.json"),
    ("corrugated", "f32"): os.path.join(ROOT, "profiles",
                                        "stream_collide_masked_corrugated_256x128x64_f32"
                                        ".counters.json"),
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_duct(lbm, inputs, precision):
    nx, ny, nz = DUCT
    ch = lbm.Channel(lbm.D3Q19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0.0, 0.0),
                     precision=precision)
    lam = inputs.duct_friction(ch.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 0))
    ch.set_friction(lam)
    return ch


def make_corrugated(lbm, inputs, precision):
    """The 256 x 128 x 64 slab with wrinkled walls (amplitude 4, wavelength 64
    along x) and the duct's smooth random friction field."""
    nx, ny, nz = DUCT
    solid = inputs.corrugated_mask(nx, ny, inputs.rng_for("corrugated", 0))
    ch = lbm.Channel(lbm.D3Q19, lbm.MASKED, nx, ny, nz, tau=0.7, force=(1e-6, 0.0, 0.0),
                     precision=precision, solid=solid)
    lam = inputs.duct_friction(ch.wall_coords(), nx, ny, nz, inputs.rng_for("corrugated", 1))
    ch.set_friction(lam)
    return ch


def timed_run(torch, ch, steps, check_every):
    """Run `steps` steps with an FP64 flux/mass check every `check_every`
    (the last step of each chunk also sums the flux and mass of the state it
    reads; the reduction then finishes and the host reads it, as the
    run-to-steady loop does).  Returns the wall seconds of exactly those
    steps and `steps` times the average step-kernel duration, from HIP events
    on the stream the kernels run on.  Each chunk's first launch is enqueued
    before its start event: the GPU idles until the host submits it (after a
    synchronisation), which is launch latency, not kernel time; the events
    then bracket the chunk's other launches, which run back to back."""
    stream = ch.stream
    nchunks = (steps + check_every - 1) // check_every
    # the events exist before the clock starts: only their records are timed
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(nchunks)]
    # one untimed step: each chunk then starts on the buffer parity whose
    # step graphs the warm-up built
    ch.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, timed = 0, []
    for a, b in ev:
        k = min(check_every, steps - done)
        if k == 1:  # a one-step chunk: its launch latency stays in the window
            a.record(stream)
            ch.step_checked(1)
        else:
            ch.step(1)
            a.record(stream)
            ch.step_checked(k - 1)
        b.record(stream)
        timed.append((a, b, max(k - 1, 1)))
        ch.checked_invariants()  # finishes the FP64 reduction, host check
        done += k
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n = sum(k for _, _, k in timed)
    kernel_ms = sum(a.elapsed_time(b) for a, b, _ in timed) / n * steps
    return t1 - t0, kernel_ms


def copy_ceiling(torch, lbm, nbytes, reps=10):
    """Plain streaming copy of nbytes (read nbytes + write nbytes), ping-pong
    between two buffers like the step's two population buffers."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(3):
        lbm.copy_probe(src, dst, nbytes, s)
        src, dst = dst, src
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        lbm.copy_probe(src, dst, nbytes, s)
        src, dst = dst, src
    b.record(s)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(steps):
    import oracle
    from paper_2403_15768_amd import inputs

    nx, ny, nz = DUCT
    o = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0, 0))
    o.set_friction(inputs.duct_friction(o.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 0)))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": round(o.fluid_count * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1,
            "host_cores": host_cores(), "kind": "oracle",
            "sample": f"{steps} steps of the 256x128x64 duct (D3Q19, FP64, single-threaded "
                      f"scalar C: one of the host's {host_cores()} cores), {dt:.1f} s"}


def extras(torch, lbm, inputs, args):
    """Secondary measurements: FP64 duct, the R = 32 nanotube with its
    spectral friction quadrature, and the other wall kinds, ends, noise forms
    and line species."""
    import numpy as np

    out = {}
    ch = make_duct(lbm, inputs, "f64")
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    cells = ch.fluid_count
    out["duct_f64"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                       "kernel_us": round(kms * 1e3 / 2000, 2),
                       "hbm_frac": round(304 * cells / (kms * 1e-3 / 2000) / 1e9 / HBM_PEAK_GBS, 4)}
    ch.close()
    del ch
    # the duct far beyond the 256 MB last-level cache (512 x 256 x 128: 2.55
    # GB of FP32 state, 1.27 GB of half state; nontemporal stores): the step
    # kernel against HBM alone, in float and half storage
    nx, ny, nz = 512, 256, 128
    for prec in ("f32", "f16s"):
        ch = lbm.Channel(lbm.D3Q19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0.0, 0.0),
                         precision=prec)
        ch.set_friction(inputs.duct_friction(ch.wall_coords(), nx, ny, nz,
                                             inputs.rng_for("duct", 0)))
        ch.step(100)
        wall, kms = timed_run(torch, ch, 1000, 1000)
        cells = ch.fluid_count
        bpu = BYTES_PER_UPDATE[prec]
        out[f"duct_512x256x128_{prec}"] = {
            "mlups": round(cells * 1000 / wall / 1e6, 1), "kernel_us": round(kms * 1e3 / 1000, 2),
            "hbm_frac": round(bpu * cells / (kms * 1e-3 / 1000) / 1e9 / HBM_PEAK_GBS, 4),
            "state_gb": round(bpu * cells / 1e9, 2)}
        ch.close()
        del ch
        torch.cuda.empty_cache()
    R, nx = 32, 512
    ny, nz, cy, cz = inputs.tube_box(R)
    tb = lbm.Channel(lbm.D3Q19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0), precision="f32",
                     tube_radius=float(R), tube_cy=cy, tube_cz=cz)
    sp = inputs.draw_spectral(inputs.rng_for("tube", 0))
    om = inputs.tube_plasmon_frequencies(tb.wall_coords(), nx, R, cy, cz, sp.omega0,
                                         inputs.rng_for("tube", 1))
    tb.set_friction_spectral(sp, om)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb.set_friction_spectral(sp, om)
    qs = time.perf_counter() - t0
    n = tb.wall_count
    out["quadrature"] = {"nodes": n, "grid": [sp.nq, sp.nw], "s": round(qs, 4),
                         "gpoints_per_s": round((n + 1) * sp.nq * sp.nw / qs / 1e9, 2)}
    # the screened form (|1 - g_s g_l e^{-2qd}|^2, dispersive liquid mode)
    sp.coupling, sp.v_l = 1, 0.5
    tb.set_friction_spectral(sp, om)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb.set_friction_spectral(sp, om)
    qs = time.perf_counter() - t0
    out["quadrature_screened"] = {"nodes": n, "grid": [sp.nq, sp.nw], "s": round(qs, 4),
                                  "gpoints_per_s": round((n + 1) * sp.nq * sp.nw / qs / 1e9, 2)}
    sp.coupling, sp.v_l = 0, 0.0
    tb.set_friction_spectral(sp, om)
    tb.step(200)
    wall, kms = timed_run(torch, tb, 2000, 1000)
    cells = tb.fluid_count
    out["tube_r32_f32"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                           "kernel_us": round(kms * 1e3 / 2000, 2),
                           "hbm_frac_fluid_bytes": round(152 * cells / (kms * 1e-3 / 2000) / 1e9
                                                         / HBM_PEAK_GBS, 4)}
    tb.close()
    # the slab with electron sheets on both walls (electron wind): water step
    # plus the sheets' step, against the same slab without them
    nx, ny, nz = DUCT
    for name, elec in (("slab_f32", False), ("slab_f32_electrons", True)):
        ch = lbm.Channel(lbm.D3Q19, lbm.SLAB, nx, ny, nz, tau=0.7, force=(1e-6, 0.0, 0.0),
                         precision="f32")
        ch.set_friction(0.05)
        if elec:
            ch.set_electrons(0.9, 1.0, 0.05, 1e-6)
        ch.step(200)
        wall, kms = timed_run(torch, ch, 2000, 1000)
        cells = ch.fluid_count
        out[name] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                     "step_us": round(kms * 1e3 / 2000, 2),
                     "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9 / HBM_PEAK_GBS, 4)}
        ch.close()
    # one rank's share of the duct split into 8 x-slabs (32 x 128 x 64, x
    # periodic in place of the halo exchange): the channel kernel (one
    # workgroup per 32-cell x-line) and the batch kernel (64-lane waves
    # packed across x-lines), as a sharded run would step it
    for name, batched in (("duct_share_32x128x64_f32", False),
                          ("duct_share_32x128x64_f32_batch_kernel", True)):
        ch = lbm.Channel(lbm.D3Q19, lbm.DUCT, 32, 128, 64, tau=0.7, force=(1e-6, 0.0, 0.0),
                         precision="f32")
        ch.set_friction(0.05)
        cells = ch.fluid_count
        if batched:
            b = lbm.Batch([ch])
            b.tune()
            b.step(64)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(b.stream)
            b.step(2048)
            e1.record(b.stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 2048
            b.close()
        else:
            ch.step(200)
            _, kms = timed_run(torch, ch, 2048, 1024)
            us = kms * 1e3 / 2048
        out[name] = {"mlups": round(cells / us, 1), "step_us": round(us, 2),
                     "hbm_frac": round(152 * cells / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        ch.close()
    # open x ends (Neumann-like inlet and outlet): the benchmark duct with a
    # density drop besides its body force; the step kernel plus the kernel
    # that recomputes the end nodes with the ghost pulls
    ch = make_duct(lbm, inputs, "f32")
    ch.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    cells = ch.fluid_count
    out["duct_f32_open_ends"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                 "step_us": round(kms * 1e3 / 2000, 2),
                                 "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9
                                                   / HBM_PEAK_GBS, 4)}
    ch.close()
    # the R = 32 nanotube (512 x 72 x 72) with open ends: a pressure-driven
    # tube, the interpolated wall links at both ends reading the ghosts
    R, nx = 32, 512
    ny, nz, cy, cz = inputs.tube_box(R)
    tb = lbm.Channel(lbm.D3Q19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(0.0, 0, 0), precision="f32",
                     tube_radius=float(R), tube_cy=cy, tube_cz=cz)
    tb.set_friction(0.05)
    tb.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    tb.step(200)
    wall, kms = timed_run(torch, tb, 2000, 1000)
    cells = tb.fluid_count
    out["tube_r32_f32_open_ends"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                     "kernel_us": round(kms * 1e3 / 2000, 2),
                                     "hbm_frac_fluid_bytes": round(152 * cells / (kms * 1e-3 / 2000)
                                                                   / 1e9 / HBM_PEAK_GBS, 4)}
    tb.close()
    # the R = 32 nanotube with electron lines in the solid around its wall
    # (the electron wind of a carbon nanotube): water step plus line step
    tb = lbm.Channel(lbm.D3Q19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0), precision="f32",
                     tube_radius=float(R), tube_cy=cy, tube_cz=cz)
    tb.set_friction(0.05)
    tb.set_electrons(0.9, 1.0, 0.05, 1e-6)
    tb.step(200)
    wall, kms = timed_run(torch, tb, 2000, 1000)
    cells = tb.fluid_count
    out["tube_r32_f32_electrons"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                     "step_us": round(kms * 1e3 / 2000, 2),
                                     "shells": tb.shell_count}
    tb.close()
    # walls that vary along x: the wrinkled slab (masked walls)
    ch = make_corrugated(lbm, inputs, "f32")
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    cells = ch.fluid_count
    out["corrugated_f32"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                             "kernel_us": round(kms * 1e3 / 2000, 2),
                             "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9
                                               / HBM_PEAK_GBS, 4)}
    ch.close()
    # a wrinkled slab of the same size whose last row repeats its first (255
    # rows of the mask above, then the first again), between two reservoirs
    # at a density drop: masked walls with open ends
    nx, ny, nz = DUCT
    m = inputs.corrugated_mask(nx - 1, ny, inputs.rng_for("corrugated", 0))
    solid = np.concatenate([m, m[:, :1]], axis=1)
    ch = lbm.Channel(lbm.D3Q19, lbm.MASKED, nx, ny, nz, tau=0.7, force=(0.0, 0.0, 0.0),
                     precision="f32", solid=solid)
    ch.set_friction(0.05)
    ch.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    cells = ch.fluid_count
    out["corrugated_f32_open_ends"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                       "kernel_us": round(kms * 1e3 / 2000, 2),
                                       "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9
                                                         / HBM_PEAK_GBS, 4)}
    ch.close()
    # the benchmark duct with electron lines on all four walls
    ch = make_duct(lbm, inputs, "f32")
    ch.set_electrons(0.9, 1.0, 0.05, 1e-6)
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    cells = ch.fluid_count
    out["duct_f32_electrons"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                 "step_us": round(kms * 1e3 / 2000, 2),
                                 "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9
                                                   / HBM_PEAK_GBS, 4)}
    # with phonon lines beside the electron lines (solved in the same kernel)
    ch.set_phonons(0.7, 1.3, 0.02, 0.08)
    ch.step(200)
    wall, kms = timed_run(torch, ch, 2000, 1000)
    out["duct_f32_electrons_phonons"] = {"mlups": round(cells * 2000 / wall / 1e6, 1),
                                         "step_us": round(kms * 1e3 / 2000, 2),
                                         "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000)
                                                           / 1e9 / HBM_PEAK_GBS, 4)}
    ch.close()
    # the fluctuating update (thermal noise, kT = 1e-6) on the FP32 duct,
    # both noise forms
    for mode, name in ((1, "stress"), (2, "all")):
        ch = make_duct(lbm, inputs, "f32")
        ch.set_thermal(1e-6, mode, 1)
        ch.step(200)
        wall, kms = timed_run(torch, ch, 2000, 1000)
        cells = ch.fluid_count
        out[f"duct_f32_thermal_{name}"] = {
            "mlups": round(cells * 2000 / wall / 1e6, 1),
            "kernel_us": round(kms * 1e3 / 2000, 2),
            "hbm_frac": round(152 * cells / (kms * 1e-3 / 2000) / 1e9 / HBM_PEAK_GBS, 4)}
        ch.close()
    return out


def batch_throughput(args, specs):
    """256 uneven ducts in one batch: throughput and per-channel error after
    1000 steps for FP64 / FP32 / half storage."""
    import numpy as np
    import torch

    from paper_2403_15768_amd import lbm, serve

    cells = sum(c.nx * c.ny * c.nz for c in specs)
    out = {}
    fields, fluxes = {}, {}
    precs = args.batch_precisions.split(",")
    for prec in precs:
        log("batch:", prec)
        chs = [serve.open_channel(c, prec, serve.DuctQueries) for c in specs]
        if args.thermal:  # the fluctuating update, each channel its own seed
            for k, ch in enumerate(chs):
                ch.set_thermal(1e-6, args.thermal, k)
        b = lbm.Batch(chs)
        if args.no_tune:
            shape = 4
            b.tuning = {"group_bytes": b.settings()["group_bytes"], "streams": 2,
                        "us_per_step": 0.0, "us_per_step_default": 0.0}
        else:
            shape = b.tune()
        b.step(64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(args.batch_steps - 64)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        n = args.batch_steps - 64
        inv = b.invariants()
        fluxes[prec] = inv[:, 0].copy()
        fields[prec] = [ch.field(1) for ch in chs]
        bpu = BYTES_PER_UPDATE[prec]
        t = b.tuning
        out[prec] = {"mlups": round(cells * n / (ms * 1e-3) / 1e6, 1),
                     "us_per_step": round(ms * 1e3 / n, 2),
                     "hbm_frac": round(bpu * cells * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "groups": b.groups,
                     "tuned": {"waves_per_group": shape, "group_mib": t["group_bytes"] >> 20,
                               "streams": t["streams"], "us_per_step": round(t["us_per_step"], 2),
                               "us_per_step_default_setting":
                                   round(t["us_per_step_default"], 2)}}
        b.close()
        for ch in chs:
            ch.close()
        del chs
        torch.cuda.empty_cache()
    for prec in [p for p in ("f32", "f16s") if p in precs and "f64" in precs]:
        fe = [float(np.max(np.abs(a - r)) / np.max(np.abs(r)))
              for a, r in zip(fields[prec], fields["f64"])]
        qe = np.abs(fluxes[prec] / fluxes["f64"] - 1)
        out[prec].update(field_err_max=float(np.max(fe)), field_err_median=float(np.median(fe)),
                         flux_err_max=float(np.max(qe)), flux_err_median=float(np.median(qe)))
    return out


def batch_steady(specs, modes=("f32", "mixed")):
    """Run every channel of the batch to steady (flux change < 1e-8 per
    check), FP32 storage against mixed precision at the same tolerance:
    solves/s, p50 / p99 time-to-steady and the spread of the final fluxes.
    The mixed-precision solve ends in FP32 storage, so both modes meet the
    same accuracy; the 'FP32' path stores float and computes in double."""
    from paper_2403_15768_amd import serve

    out, flux = {}, {}
    for mode in modes:
        log("batch: run to steady", mode)
        srv = serve.Server(mode=mode, hbm_budget=64 << 30, realtime=False, kind=serve.DuctQueries)
        t0 = time.perf_counter()
        res = srv.run(specs)
        wall = time.perf_counter() - t0
        sm = serve.summarize(res, wall)
        sm["lattice_updates"] = srv.stats["lattice_updates"]
        sm["glups"] = round(srv.stats["lattice_updates"] / wall / 1e9, 2)
        sm["batch_rebuilds"] = srv.stats["batch_rebuilds"]
        sm["joins"] = srv.stats["joins"]
        sm["rounds"] = srv.stats["rounds"]
        sm["host_wait_s"] = round(srv.stats["host_wait_s"], 3)
        sm["check_s"] = round(srv.stats["check_s"], 3)
        sm["tuning"] = {k: {"waves_per_group": v["waves_per_group"],
                            "group_mib": v["group_bytes"] >> 20, "streams": v["streams"]}
                        for k, v in srv.tuning.items()}
        out[mode] = sm
        flux[mode] = {r.qid: r.flux for r in res}
    if "f32" in flux and "mixed" in flux:
        fa, fb = flux["f32"], flux["mixed"]
        out["mixed_vs_f32_flux_diff_max"] = float(max(abs(fb[k] / fa[k] - 1) for k in fa))
        out["speedup_mixed_over_f32"] = round(out["f32"]["makespan_s"] /
                                              out["mixed"]["makespan_s"], 3)
    return out


def batch_workload(args):
    """The batch line of its own: throughput and errors after 1000 steps,
    then run-to-steady solves/s."""
    from paper_2403_15768_amd import inputs

    specs = inputs.batch_channels(256)
    out = {"workload": "batch_256_ducts" + ("", "_thermal_stress", "_thermal_all")[args.thermal],
           "channels": len(specs), "cells": sum(c.nx * c.ny * c.nz for c in specs)}
    if args.batch_precisions:
        out.update(batch_throughput(args, specs))
    if not args.no_steady:
        out["steady"] = batch_steady(specs)
    print(json.dumps(out), flush=True)


def serving_run(trace, modes=("f32", "mixed"), budget_gb=32.0):
    """One Poisson trace of nanotube queries through the continuous-batching
    server, FP32 storage against mixed precision."""
    import torch

    from paper_2403_15768_amd import serve

    out = {}
    for mode in modes:
        log(f"serving: {mode}, {len(trace)} queries")
        srv = serve.Server(mode=mode, hbm_budget=int(budget_gb * (1 << 30)), realtime=True)
        t0 = time.perf_counter()
        res = srv.run(trace)
        wall = time.perf_counter() - t0
        sm = serve.summarize(res, wall)
        sm.update(max_active=srv.stats["max_active"], batch_rebuilds=srv.stats["batch_rebuilds"],
                  joins=srv.stats["joins"], rounds=srv.stats["rounds"],
                  glups=round(srv.stats["lattice_updates"] / wall / 1e9, 2))
        out[mode] = sm
        torch.cuda.empty_cache()
    if "f32" in out and "mixed" in out:
        out["speedup_mixed_over_f32"] = round(out["f32"]["makespan_s"] /
                                              out["mixed"]["makespan_s"], 3)
    return out


def serving_workload(args):
    """Poisson-arriving nanotube queries (radius 8..32), continuous batching,
    FP32 storage against mixed precision on the same trace."""
    from paper_2403_15768_amd import inputs

    trace = inputs.serving_trace(args.queries, args.rate)
    out = {"workload": "serving_tubes", "queries": len(trace), "rate_per_s": args.rate,
           "radius": [8, 32], "box": "512 x (2R+8)^2"}
    out.update(serving_run(trace, budget_gb=args.budget_gb))
    print(json.dumps(out), flush=True)


def whole_metric(args):
    """The rest of the headline metric, bounded to a few minutes: the 256-duct
    batch run to steady (solves/s, p50 / p99 time-to-steady, FP32 storage
    against mixed precision) and two short serving traces of nanotube queries
    (radius 8..32), one at the 50/s arrival rate (oversubscribed: one GPU
    serves about 2 such queries per second) and one at 2/s."""
    from paper_2403_15768_amd import inputs

    specs = inputs.batch_channels(256)
    out = {"batch_steady": {"workload": "batch_256_ducts", "channels": len(specs),
                            "cells": sum(c.nx * c.ny * c.nz for c in specs)}}
    out["batch_steady"].update(batch_steady(specs))
    out["serving"] = {}
    for rate in (50.0, 2.0):
        trace = inputs.serving_trace(args.serving_queries, rate)
        key = f"rate_{rate:g}_per_s"
        out["serving"][key] = {"queries": len(trace), "radius": [8, 32],
                               "box": "512 x (2R+8)^2", "budget_gb": args.budget_gb}
        out["serving"][key].update(serving_run(trace, budget_gb=args.budget_gb))
    return out


def permeability_workload(args):
    """Sec. 5.1: steady permeability enhancement of x-periodic nanotubes
    against radius and carrier density (plasmon frequency), friction from the
    quadrature; continuum Navier slip predicts 1 + 4 nu / (lambda R)."""
    import numpy as np

    from paper_2403_15768_amd import permeability

    radii, scales = [4, 6, 8, 12, 16, 24, 32], [0.5, 1.0, 2.0]
    t0 = time.perf_counter()
    res = permeability.sweep(radii, scales, precision=args.precision)
    dt = time.perf_counter() - t0
    nu = (0.8 - 0.5) / 3
    rows = [{"R": r.radius, "omega_scale": r.omega_scale, "lambda": round(r.lam, 6),
             "enhancement": round(r.enhancement, 5),
             "slip_length_fit_over_nu_lambda": round(r.slip_length_fit() * r.lam / nu, 4),
             "steps": r.steps} for r in res]
    slopes = {}
    for s in scales:
        e = np.array([r.enhancement for r in res if r.omega_scale == s])
        slopes[str(s)] = round(float(np.polyfit(np.log(radii), np.log(e - 1), 1)[0]), 4)
    rec = {"metric": "nanotube permeability enhancement vs radius (Sec. 5.1)",
           "value": round(len(res) / dt, 3), "unit": "tubes solved per s (each also with no-slip walls)",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64" if args.precision != "f16s" else "f32",
           "data": "synthetic",
           "config": {"workload": "tube_permeability_sweep", "radii": radii,
                      "omega_scales": scales, "nx": 16, "tau": 0.8, "g": 1e-6,
                      "storage": args.precision, "steady": "flux change < 1e-9 per 500 steps"},
           "loglog_slope_of_enhancement_minus_1": slopes, "tubes": rows,
           "wall_s": round(dt, 3)}
    # the wall's shape (same section): wrinkled walls against flat ones
    t0 = time.perf_counter()
    wr = permeability.wrinkle_sweep([1.0, 2.0, 4.0], [float("inf"), 0.05],
                                    precision=args.precision)
    rec["wrinkles"] = {"config": {"lattice": "D2Q9", "nx": 128, "mean_gap": 24,
                                  "wavelength": 64, "tau": 0.8, "g": 1e-6},
                       "wall_s": round(time.perf_counter() - t0, 3),
                       "rows": [{"amplitude": w.amplitude, "meander": w.meander,
                                 "no_slip": bool(np.isinf(w.lam)),
                                 "lambda": None if np.isinf(w.lam) else w.lam,
                                 "flux_over_flat": round(w.relative, 5),
                                 "steps": w.steps} for w in wr]}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16s"])
    ap.add_argument("--cpu-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--thermal", type=int, default=0, choices=[0, 1, 2],
                    help="thermal noise (kT = 1e-6) on the duct or the batch: 1 stress "
                         "source, 2 every non-conserved direction")
    ap.add_argument("--open-ends", action="store_true",
                    help="duct or slab: Neumann-like inlet and outlet (densities 1 +- 1e-5) "
                         "in place of periodic x")
    ap.add_argument("--phonons", action="store_true",
                    help="slab with --electrons: phonon lines beside the electron lines")
    ap.add_argument("--electrons", action="store_true",
                    help="with --workload slab: electron sheets on both walls")
    ap.add_argument("--workload", default="duct",
                    choices=["duct", "slab", "corrugated", "batch", "serving", "permeability"],
                    help="duct: the headline line; batch / serving: their own JSON line")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-precisions", default="f64,f32,f16s",
                    help="storage precisions timed by --workload batch")
    ap.add_argument("--no-steady", action="store_true",
                    help="--workload batch: skip the run-to-steady comparison")
    ap.add_argument("--queries", type=int, default=500)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--serving-queries", type=int, default=40,
                    help="queries per serving trace in the headline line")
    ap.add_argument("--no-tune", action="store_true",
                    help="default kernel shapes (no autotuner launches: for counter runs)")
    ap.add_argument("--no-whole-metric", action="store_true",
                    help="headline line without the batch run-to-steady and serving parts")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path "
              "(the per-GPU kernel is measured at N = 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_15768_amd import inputs, lbm

    lbm.load()
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return batch_workload(args)
    if args.workload == "serving":
        return serving_workload(args)
    if args.workload == "permeability":
        if args.precision == "f32" and "--precision" not in sys.argv:
            args.precision = "f64"
        return permeability_workload(args)
    slab = args.workload == "slab"
    corr = args.workload == "corrugated"
    log("bench:", args.workload, "256x128x64", args.precision, "steps", args.steps)
    if slab:  # walls on y only (z periodic), uniform friction, optional electron sheets
        nx, ny, nz = DUCT
        ch = lbm.Channel(lbm.D3Q19, lbm.SLAB, nx, ny, nz, tau=0.7, force=(1e-6, 0.0, 0.0),
                         precision=args.precision)
        ch.set_friction(0.05)
        if args.electrons:
            ch.set_electrons(0.9, 1.0, 0.05, 1e-6)
            if args.phonons:
                ch.set_phonons(0.7, 1.3, 0.02, 0.08)
    elif corr:
        ch = make_corrugated(lbm, inputs, args.precision)
    else:
        ch = make_duct(lbm, inputs, args.precision)
    if args.thermal:
        ch.set_thermal(1e-6, args.thermal, 1)
    if args.open_ends:
        ch.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    cells = ch.fluid_count
    # the step kernel's block width from the autotuner (searched here, once)
    block = 0 if args.no_tune else ch.tune(retime=True)[0]
    ch.step(args.warmup)
    ch.invariants()
    wall, kernel_ms = timed_run(torch, ch, args.steps, args.check_every)
    q, m, dm = ch.invariants()
    # the tuned and the default block width over runs of the same length, for
    # the tuner's gain (the timed region above may be too short to compare)
    _, kms_tuned = timed_run(torch, ch, 1000, 1000)
    ch.set_block(0)
    _, kms_default = timed_run(torch, ch, 1000, 1000)
    ch.close()
    del ch

    mlups = cells * args.steps / wall / 1e6
    kern_s = kernel_ms * 1e-3 / args.steps
    bpu = BYTES_PER_UPDATE[args.precision]
    achieved = bpu * cells / kern_s / 1e9
    log(f"bench: {mlups:.1f} MLUPS, step kernel {kern_s * 1e6:.2f} us, {achieved:.0f} GB/s")

    traffic = None
    cfile = COUNTERS.get((args.workload, args.precision))
    if cfile and os.path.exists(cfile) and not args.thermal and not args.open_ends:
        c = json.load(open(cfile))
        if c.get("kernel_hash") == kernel_hash():
            traffic = c.get("bytes_per_launch")

    # the same footprint as one step (a population buffer read, the other
    # written; partly held by the 256 MB last-level cache), and a 1 GiB copy
    copy_gbs = copy_ceiling(torch, lbm, bpu // 2 * cells)
    copy_big = copy_ceiling(torch, lbm, 1 << 30)
    log(f"bench: copy ceiling {copy_gbs:.0f} GB/s (same footprint), {copy_big:.0f} GB/s (1 GiB)")
    ext = {} if args.no_extras else extras(torch, lbm, inputs, args)
    ext["copy_same_footprint_GBs"] = round(copy_gbs, 1)
    ext["copy_1GiB_GBs"] = round(copy_big, 1)
    ext["frac_of_copy_same_footprint"] = round(achieved / copy_gbs, 4)
    ext["final_flux"] = q
    ext["mass_deviation"] = dm
    ext["step_block_width"] = {"tuned": block, "kernel_us_tuned": round(kms_tuned * 1e3 / 1000, 3),
                               "kernel_us_default_width": round(kms_default * 1e3 / 1000, 3)}

    arith = "f32" if args.precision == "f16s" else "f64"  # half storage computes in float
    whole = None
    if (args.workload == "duct" and not args.no_whole_metric and not args.thermal
            and not args.open_ends):
        whole = whole_metric(args)
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(args.cpu_steps)

    rec = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": arith,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_256x128x64_d3q19_{args.precision}storage"
                               + ("", "_thermal_stress", "_thermal_all")[args.thermal]
                               + ("_electrons" if slab and args.electrons else "")
                               + ("_phonons" if slab and args.electrons and args.phonons else "")
                               + ("_open_ends" if args.open_ends else ""),
                   "lattice": "D3Q19", "box": list(DUCT), "fluid_cells": cells, "tau": 0.7,
                   "g": 1e-6, "storage": args.precision, "arithmetic": arith,
                   "friction": ("uniform lambda 0.05" if slab else
                                "smooth random lambda(x,s): mean 0.05, std 0.02, corr. length 16"),
                   "walls": ("wrinkled: staircase sinusoids, amplitude 4, wavelength 64"
                             if corr else "planar"),
                   "electrons": ("sheets on both walls: tau_e 0.9, rho_e0 1, gamma_e 0.05, "
                                 "force_e 1e-6"
                                 + ("; phonon lines: tau_p 0.7, rho_p0 1.3, gamma_pc 0.02, "
                                    "gamma_ep 0.08" if args.phonons else ""))
                                if slab and args.electrons else None,
                   "check_every": args.check_every,
                   "thermal": [None, "stress source, kT 1e-6", "all directions, kT 1e-6"][args.thermal]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_GBs": None if traffic is None else round(traffic / kern_s / 1e9, 1),
                     "kernel": ("k_step_masked<D3Q19>" if corr else
                                "k_step<D3Q19>" if not args.thermal else
                                f"k_step<D3Q19, noise {args.thermal}>")
                               + (" + k_electron_step (time per step covers both)"
                                  if slab and args.electrons else "")
                               + (" + k_open_ends (time per step covers both)"
                                  if args.open_ends else ""),
                     "kernel_us": round(kern_s * 1e6, 3), "bytes_per_update": bpu},
        "cpu_baseline": cpu,
        "extras": ext,
    }
    if whole:
        rec.update(whole)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
