"""Throughput of the S-fraction multiscale ROM time stepping on one MI355X.

Runs the whole hot path on the 512^3 layered-plus-inclusions workload (16^3 subdomains
of 32^3 cells, m = 16 boundary functions per face, k = 16 S-fraction levels, FP32):
device ROM build for every subdomain (timed separately: ROM builds/s), the CFL step of
the coupled ROM, W untimed warm-up steps and K timed leapfrog steps with all 65,536
surface receivers recorded every step.  Prints one JSON line.

value = fine-grid-equivalent cell updates per second:
    N_cells * K * (dt_ROM / dt_fine) / wall,   dt_fine = 0.9 h / (sqrt(3) c_max)
(the fine grid's leapfrog limit for the same medium), inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# The library records hipEvents around the kernels of one step in TIMING_EVERY; an event record
# between two kernels costs device time of its own, so the other steps run as they would untimed.
# Odd, so that the timed steps fall on every position of the 64-step (32 for shots) receiver
# windows and the window flushes are sampled in proportion.
TIMING_EVERY = 17
COUNTERS = os.path.join(ROOT, "profiles", "step_main_counters.json")
STEP_SRC = os.path.join(ROOT, "paper_1406_6923_amd", "csrc", "step_kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name: str) -> W.Workload:
    if name == "large":
        return W.CFG_LARGE
    if name == "small":
        return W.CFG_SMALL
    if name.startswith("scaled"):
        n = int(name[len("scaled"):] or 4)
        return W.scaled_large((n, n, n), nsteps=2000)
    raise SystemExit(f"unknown workload {name}")


def step_kernel_sha() -> str:
    with open(STEP_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profiles(launch_bytes_alg: float):
    """HBM bytes per main-kernel launch from committed rocprofv3 counters, if they match this kernel."""
    if not os.path.exists(COUNTERS):
        return None, "no committed counters"
    with open(COUNTERS) as fh:
        rec = json.load(fh)
    if rec.get("kernel_sha") != step_kernel_sha():
        return None, "counters predate the current step kernel"
    return rec.get("bytes_per_launch"), rec.get("note", "")


def cpu_baseline(cfg: W.Workload, c_full: np.ndarray, dt_ratio: float, nsub=(1, 1, 1), nsteps=2000):
    """The FP64 oracle on a bounded sample of the same workload (host cores)."""
    from oracle import coupled, rom, subdomains
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    sx, sy, sz = cfg.sub_cells
    box = c_full[:nsub[2] * sz + 1, :nsub[1] * sy + 1, :nsub[0] * sx + 1].astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    subs = subdomains.decompose(box, cfg.h, cfg.sub_cells, cfg.m)
    roms = rom.build_all(subs, cfg.k)
    t_build = time.perf_counter() - t0
    cs = coupled.CoupledSystem(subs, roms)
    rng = np.random.default_rng(0)
    U = cs.scatter(rng.standard_normal(cs._dof_layout()[1]) * 1e-6)
    dt = 0.9 * cs.cfl_dt()
    t0 = time.perf_counter()
    cs.run(dt, np.zeros((nsteps, 0)), U0=U, U_prev=U)
    t_step = time.perf_counter() - t0
    cells = nsub[0] * sx * nsub[1] * sy * nsub[2] * sz
    one_thread = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            cs.run(dt, np.zeros((nsteps, 0)), U0=U, U_prev=U)
            one_thread = cells * nsteps * dt_ratio / (time.perf_counter() - t0) / 1e9
    except Exception:  # pragma: no cover
        pass
    # the oracle's fine-grid FDTD on the same box, at its own stability limit
    from oracle import grid
    fg = grid.FineGrid(box, cfg.h)
    nf = 200
    dtf = 0.9 * fg.cfl_dt()
    src = np.array([[box.shape[2] // 2, box.shape[1] // 2, box.shape[0] // 2]])
    t0 = time.perf_counter()
    fg.fdtd(dtf, W.ricker(cfg.f_peak, dtf, nf)[:, None], src, np.array([[1, 1, 0]]))
    fdtd_rate = cells * nf / (time.perf_counter() - t0) / 1e9
    value = cells * nsteps * dt_ratio / t_step / 1e9
    # The step loop's per-subdomain products are small: if one BLAS thread runs it as fast as the
    # whole pool, the oracle effectively used one core.
    used = 1 if (one_thread is not None and one_thread >= 0.85 * value) else int(threads)
    return {
        "value": value,
        "unit": "Gcell-updates/s (fine-grid-equivalent)",
        "cores": used,
        "blas_threads": int(threads),
        "kind": "oracle",
        "sample": (f"{nsub[0]}x{nsub[1]}x{nsub[2]} subdomains ({cells} cells) cut from the same velocity model, "
                   f"same subdomain size and ROM sizes; oracle ROM build of those subdomains "
                   f"({len(subs) / t_build:.3f} builds/s, not in value) then {nsteps} FP64 leapfrog steps "
                   f"of the coupled ROMs timed; dt ratio taken from the GPU run; cores = 1 when the "
                   f"one-thread rate matches the {int(threads)}-thread rate (the products are too small to "
                   f"parallelise)"),
        "builds_per_s": len(subs) / t_build,
        "step_seconds": t_step,
        "value_one_thread": one_thread,
        "oracle_fine_fdtd_gcell_per_s": fdtd_rate,
    }


def finite_shift_probe(torch, sfm, dev, stream, n: int = 4, steps: int = 200, sigma_factors=(16.0, 32.0, 64.0)):
    """Finite-shift ROMs on an n^3-subdomain sample with the large workload's subdomain and ROM
    shape (33^3 nodes, m = 16, k = 16): device build rate (Jacobi-PCG shifted solves), the CFL
    step against sigma = infinity ROMs of the same sample, and the FP64-coefficient step rate.
    The shift is the first of sigma_factors * (2 pi f_peak)^2 whose S-fraction is positive definite
    at the FP64 level in every subdomain (the build reports a breakdown otherwise: the deepest
    level of a small shift can sit at rounding level, e.g. a Gamma-hat_16 pivot at 1.6e-14 of its
    diagonal at factor 16); the refused factors are listed."""
    cfg = W.scaled_large((n, n, n), nsteps=steps)
    c = cfg.velocity_model()
    vel = torch.from_numpy(c.astype(np.float32)).to(dev)
    out = {"workload": cfg.name, "subdomains": n ** 3, "coefficients": "f64", "refused_sigma_factors": []}
    h_inf = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_build_roms(h_inf.ctx, vel, stream=stream)
    torch.cuda.synchronize()
    out["sigma_inf_builds_per_s"] = n ** 3 / (time.perf_counter() - t0)
    dt_inf = sfm.sfm_cfl_dt(h_inf.ctx, 200, stream=stream)
    h_inf.close()
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
    iters = None
    for factor in sigma_factors:
        sigma = factor * (2.0 * math.pi * cfg.f_peak) ** 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            iters = sfm.sfm_build_roms_shifted(h.ctx, sigma, vel, stream=stream)
        except sfm.SfmError as e:
            if e.status != sfm.SFM_EBREAKDOWN:
                raise
            log(f"[bench] finite shift {factor} (2 pi f_peak)^2: {e.message}")
            out["refused_sigma_factors"].append(factor)
            continue
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        out.update(sigma=sigma, sigma_over_peak_omega_sq=factor)
        break
    if iters is None:
        h.close()
        out["error"] = "every shift factor broke down"
        return out
    out.update(build_seconds=t_b, builds_per_s=n ** 3 / t_b, cg_iters_max=iters)
    dt_sh = sfm.sfm_cfl_dt(h.ctx, 200, stream=stream)
    out["dt_ratio_vs_sigma_inf"] = dt_sh / dt_inf
    dt = 0.9 * dt_sh
    wav = torch.tensor(W.ricker(cfg.f_peak, dt, steps)[:, None], dtype=torch.float32, device=dev)
    sfm.sfm_step(h.ctx, 20, dt, wav[:20].contiguous(), None, stream=stream)
    sfm.sfm_set_timing(h.ctx, True, every=TIMING_EVERY)
    sfm.sfm_step(h.ctx, steps, dt, wav, None, stream=stream)
    torch.cuda.synchronize()
    info = h.info()
    main_ms = info["timed_main_ms"] / max(info["timed_steps"], 1)
    k, p = info["k"], info["p"]
    bytes_per_launch = n ** 3 * ((2 * k - 1) * p * (p + 1) // 2 * 8 + 3 * k * p * 4)
    out.update(fp64_main_ms=main_ms, fp64_main_gbs=bytes_per_launch / (main_ms * 1e-3) / 1e9)
    h.close()
    log(f"[bench] finite shift sigma = {sigma:.3g}: {out['builds_per_s']:.1f} builds/s "
        f"(sigma = inf {out['sigma_inf_builds_per_s']:.1f}), at most {iters} CG iterations, "
        f"dt x{out['dt_ratio_vs_sigma_inf']:.3f}, FP64 step kernel {main_ms:.4f} ms ({out['fp64_main_gbs']:.0f} GB/s)")
    return out


def fp64_stream_probe(torch, sfm, h, cfg: W.Workload, dt: float, dt_ratio: float, finite_dt_gain, steps: int = 100):
    """The FP64 coefficient stream (the finite-shift path's step) at the full workload's scale: the
    run's own ROMs loaded into an FP64-storage context, the step kernel timed over `steps` steps.
    Combined with the finite-shift probe's dt gain this is the finite-shift stepping rate at scale."""
    gam, hat = sfm.sfm_export_roms(h.ctx)
    h64 = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
    sfm.sfm_load_roms(h64.ctx, gam, hat)
    del gam, hat
    sfm.sfm_set_state(h64.ctx, None, None, 0)      # zero state, no sources: the stream is the same
    sfm.sfm_step(h64.ctx, 10, dt, None, None)
    sfm.sfm_set_timing(h64.ctx, True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_step(h64.ctx, steps, dt, None, None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = h64.info()
    h64.close()
    S, k, p = info["n_subdomains"], info["k"], info["p"]
    main_ms = info["timed_main_ms"] / max(info["timed_steps"], 1)
    launch_bytes = S * ((2 * k - 1) * p * (p + 1) // 2 * 8 + 3 * k * p * 4)
    out = {"subdomains": S, "main_ms": main_ms, "main_gbs": launch_bytes / (main_ms * 1e-3) / 1e9,
           "ms_per_step": wall / steps * 1e3,
           "gcell_per_s_at_sigma_inf_dt": cfg.n_cells * steps * dt_ratio / wall / 1e9}
    if finite_dt_gain:
        out["finite_shift_gcell_per_s_estimate"] = out["gcell_per_s_at_sigma_inf_dt"] * finite_dt_gain
    log(f"[bench] FP64 coefficient stream at {S} subdomains: main kernel {main_ms:.4f} ms "
        f"({out['main_gbs']:.0f} GB/s), {out['ms_per_step']:.4f} ms/step")
    return out


FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6


def shot_sources(cfg: W.Workload, n: int, seed: int = 2024):
    """n shot positions uniformly random on the surface (depth 2 nodes), off every interface plane."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        i = int(rng.integers(1, cfg.ncell[0]))
        j = int(rng.integers(1, cfg.ncell[1]))
        if i % cfg.sub_cells[0] == 0 or j % cfg.sub_cells[1] == 0 or (i, j, 2) in out:
            continue
        out.append((i, j, 2))
    return out


def shots_probe(torch, sfm, h, cfg, dev, stream, dt, ratio, nshot, first_src, warmup, steps, nrec, single_ms):
    """nshot shots (sources first_src..) stepped together through the same ROMs, all receivers recorded."""
    sfm.sfm_shots_init(h.ctx, nshot, np.arange(first_src, first_src + nshot), stream=stream)
    chosen, variants = sfm.sfm_shots_tuning(h.ctx)
    log(f"[bench] shot kernel autotuner: {variants} (waves per SIMD, ms per step) -> {chosen}")
    total = warmup + steps
    w = W.ricker(cfg.f_peak, dt, total)
    wav = torch.tensor(np.repeat(w[:, None], nshot, axis=1), dtype=torch.float32, device=dev)
    tr = torch.zeros((nshot, max(nrec, 1), steps), dtype=torch.float32, device=dev) if nrec else None
    if warmup:
        sfm.sfm_shots_step(h.ctx, warmup, dt, wav[:warmup].contiguous(), None, stream=stream)
    torch.cuda.synchronize()
    sfm.sfm_shots_timing(h.ctx)
    sfm.sfm_set_timing(h.ctx, True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    sfm.sfm_shots_step(h.ctx, steps, dt, wav[warmup:].contiguous(), tr, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sfm.sfm_set_timing(h.ctx, False)
    nt, ms = sfm.sfm_shots_timing(h.ctx)
    info = h.info()
    S, k, p = info["n_subdomains"], info["k"], info["p"]
    main_ms = ms[0] / max(nt, 1)
    flops = S * 2.0 * (2 * k - 1) * p * p * nshot
    hbm = S * ((2 * k - 1) * p * (p + 1) // 2 * 4 + 4 * k * p * nshot * 4)
    achieved = flops / (main_ms * 1e-3) / 1e12
    out = {
        "nshot": nshot, "steps": steps, "warmup": warmup, "receivers": nrec,
        "ms_per_step": wall / steps * 1e3,
        "value": cfg.n_cells * nshot * steps * ratio / wall / 1e9,
        "unit": "Gcell-updates/s (all shots)",
        "speedup_vs_single_shot_runs": nshot * single_ms / (wall / steps * 1e3),
        "main_kernel_ms": main_ms, "face_kernel_ms": ms[1] / max(nt, 1), "record_kernel_ms": ms[2] / max(nt, 1),
        # the roof that binds: at flops / hbm ≈ 17 flop/B, below the FP32 matrix ridge of
        # 157.3 / 8 ≈ 20 flop/B, the attainable rate is set by HBM
        "roofline": ({"bound": "hbm", "achieved": hbm / (main_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": hbm / (main_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
                     if flops / hbm < FP32_MFMA_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS else
                     {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved / FP32_MFMA_PEAK_TFLOPS}) | {
                     "kernel": "shots_main_kernel", "intensity_flop_per_byte": flops / hbm,
                     "mfma_tflops": achieved, "mfma_frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                     "flops_per_launch": flops, "algorithmic_bytes_per_launch": hbm,
                     "hbm_gbs": hbm / (main_ms * 1e-3) / 1e9},
        "traces_finite": bool(torch.isfinite(tr).all().item()) if tr is not None else True,
        "autotune": {"chosen_waves_per_simd": chosen,
                     "variants": [{"waves_per_simd": w, "ms": m} for w, m in variants]},
    }
    log(f"[bench] {nshot} shots: {out['ms_per_step']:.3f} ms/step, {out['value']:.1f} Gcell-updates/s, main kernel "
        f"{main_ms:.3f} ms = {achieved:.1f} TFLOP/s FP32 MFMA ({100 * achieved / FP32_MFMA_PEAK_TFLOPS:.1f}%), "
        f"{out['roofline']['hbm_gbs']:.0f} GB/s")
    del tr
    return out


def uneven_shots_probe(torch, sfm, dev, stream, nsteps: int, nshot: int = 64, compare_steps: int = 192):
    """Many-shot workload: uneven boxes, a ROM size per subdomain, 64 shots, all receivers; the
    step loop replayed from a hipGraph, then the same steps with every kernel launched directly."""
    cfg = W.CFG_SHOTS
    log(f"[bench] many-shot workload {cfg.name}: generating velocity {cfg.nodes}")
    c = cfg.velocity_model()
    c_max = float(c.max())
    vel = torch.from_numpy(c.astype(np.float32)).to(dev)
    del c
    srcs = np.asarray(W.surface_shots(cfg, nshot))
    rec = cfg.receivers()
    # FP64 coefficient storage: at k = 24 and 32 the S-fraction blocks of the 48-cell boxes do not
    # survive FP32 rounding (the rounded operator's spectral radius grows by up to 1e6)
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=sfm.SFM_PREC_FP64)
    S = h.info()["n_subdomains"]
    ks = W.level_choices(S, seed=W.SHOTS_LEVEL_SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_build_roms_levels(h.ctx, ks, vel, srcs, rec, stream=stream)   # k_s Lanczos steps per subdomain
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    del vel
    dt = 0.9 * sfm.sfm_cfl_dt(h.ctx, 200, stream=stream)
    ratio = dt / (0.9 * cfg.h / (math.sqrt(3.0) * c_max))
    sfm.sfm_shots_init(h.ctx, nshot, np.arange(nshot), stream=stream)
    chosen, variants = sfm.sfm_shots_tuning(h.ctx)
    total = nsteps + 64
    wav = torch.tensor(np.repeat(W.ricker(cfg.f_peak, dt, total)[:, None], nshot, axis=1), dtype=torch.float32,
                       device=dev)
    tr = torch.zeros((nshot, len(rec), nsteps), dtype=torch.float32, device=dev)
    sfm.sfm_shots_step(h.ctx, 64, dt, wav[:64].contiguous(), None, stream=stream)       # warm-up, graph capture
    torch.cuda.synchronize()
    r0 = sfm.sfm_shots_graph(h.ctx)
    t0 = time.perf_counter()
    sfm.sfm_shots_step(h.ctx, nsteps, dt, wav[64:].contiguous(), tr, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    replays = sfm.sfm_shots_graph(h.ctx) - r0
    finite = bool(torch.isfinite(tr).all().item())
    del tr
    # graph replay against direct launches on the same number of steps (6 windows)
    tr2 = torch.zeros((nshot, len(rec), compare_steps), dtype=torch.float32, device=dev)
    w2 = wav[:compare_steps].contiguous()
    per = {}
    for mode in (1, 0):
        sfm.sfm_shots_graph(h.ctx, mode)
        sfm.sfm_shots_step(h.ctx, compare_steps, dt, w2, tr2, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sfm.sfm_shots_step(h.ctx, compare_steps, dt, w2, tr2, stream=stream)
        torch.cuda.synchronize()
        per["graph" if mode else "direct"] = (time.perf_counter() - t0) / compare_steps * 1e3
    sfm.sfm_shots_graph(h.ctx, 1)
    # per-kernel device times (direct launches with events)
    sfm.sfm_shots_timing(h.ctx)
    sfm.sfm_set_timing(h.ctx, True)
    sfm.sfm_shots_step(h.ctx, 32, dt, w2[:32].contiguous(), tr2, stream=stream)
    torch.cuda.synchronize()
    sfm.sfm_set_timing(h.ctx, False)
    nt, ms = sfm.sfm_shots_timing(h.ctx)
    del tr2
    p = cfg.p
    main_ms = ms[0] / max(nt, 1)
    flops = float(sum(2.0 * (2 * int(k) - 1) * p * p * nshot for k in ks))
    hbm = float(sum((2 * int(k) - 1) * p * (p + 1) // 2 * 4 + 4 * int(k) * p * nshot * 4 for k in ks))
    achieved = flops / (main_ms * 1e-3) / 1e12
    hbm = float(sum((2 * int(k) - 1) * p * (p + 1) // 2 * 8 + 4 * int(k) * p * nshot * 4 for k in ks))
    box = [list(cfg.box_cells(d)) for d in range(3)]
    out = {
        "workload": cfg.name, "subdomains": S, "box_cells": box,
        "box_shapes": len({(a, b, c_) for a in box[0] for b in box[1] for c_ in box[2]}),
        "m": cfg.m, "k_max": cfg.k, "k_levels": sorted(set(int(x) for x in ks)), "k_mean": float(ks.mean()),
        "nshot": nshot, "steps": nsteps, "receivers": len(rec), "dt_ratio": ratio,
        "build_seconds": t_build, "builds_per_s": S / t_build,
        "ms_per_step": wall / nsteps * 1e3, "graph_replays": replays,
        "value": cfg.n_cells * nshot * nsteps * ratio / wall / 1e9, "unit": "Gcell-updates/s (all shots)",
        "graph_ms_per_step": per["graph"], "direct_ms_per_step": per["direct"],
        "main_kernel_ms": main_ms, "face_kernel_ms": ms[1] / max(nt, 1), "record_kernel_ms": ms[2] / max(nt, 1),
        "coefficients": "fp64 (FP64 MFMA), states fp32",
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "kernel": "shots_main_kernel<double>",
                     "flops_per_launch": flops, "algorithmic_bytes_per_launch": hbm,
                     "hbm_gbs": hbm / (main_ms * 1e-3) / 1e9},
        "traces_finite": finite,
        "autotune": {"chosen_waves_per_simd": chosen,
                     "variants": [{"waves_per_simd": w, "ms": m} for w, m in variants]},
    }
    log(f"[bench] many-shot workload: build {t_build:.1f} s ({S} subdomains), {out['ms_per_step']:.3f} ms/step "
        f"over {nsteps} steps, {out['value']:.1f} Gcell-updates/s; graph {per['graph']:.3f} vs direct "
        f"{per['direct']:.3f} ms/step; main kernel {main_ms:.3f} ms = {achieved:.1f} TFLOP/s")
    h.close()
    return out


def surrogate_probe(torch, sfm, dev, stream, n_samples: int, epochs: int, tol: float = 1e-3):
    """Learned ROMs: a training set of n_samples 32^3-cell subdomains (m = 8, k = 16) of seeded
    layered / lognormal / blob media labelled by the device Lanczos build, the network trained on
    the device, then the learned build (judge and fallback) of a 256^3 grid of unseen media."""
    m, k, cells, h = 8, 16, 32, 10.0
    p = 6 * m
    n_out = 2 * k * p * (p + 1) // 2
    nn = cells + 1
    per_domain = (16, 16, 16)
    n_dom = max(1, -(-n_samples // int(np.prod(per_domain))))
    xs = torch.empty((n_dom * int(np.prod(per_domain)), nn ** 3), dtype=torch.float32, device=dev)
    ts = torch.empty((xs.shape[0], n_out), dtype=torch.float32, device=dev)
    t_label = 0.0
    for d in range(n_dom):
        ncell = tuple(cells * b for b in per_domain)
        c = W.surrogate_velocity(tuple(x + 1 for x in ncell), seed=5000 + d).astype(np.float32)
        vel = torch.from_numpy(c).to(dev)
        del c
        hd = sfm.Sfm(ncell, (cells, cells, cells), h, m, k, precision=sfm.SFM_PREC_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sfm.sfm_build_roms(hd.ctx, vel, stream=stream)
        torch.cuda.synchronize()
        t_label += time.perf_counter() - t0
        S = int(np.prod(per_domain))
        sfm.sfm_rom_inputs(hd.ctx, vel, xs[d * S:(d + 1) * S], stream=stream)
        sfm.sfm_rom_targets(hd.ctx, ts[d * S:(d + 1) * S], stream=stream)
        hd.close()
        del vel
        log(f"[bench] surrogate training set: domain {d + 1}/{n_dom} labelled")
    xs, ts = xs[:n_samples], ts[:n_samples]
    net = sfm.Cnn(nn, 32, n_out, max_batch=64, seed=11)
    net.fit_scale(ts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(xs, ts, batch=64, epochs=epochs, lr=1e-3, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del xs, ts
    log(f"[bench] surrogate: {n_samples} samples, {epochs} epochs in {t_train:.1f} s, loss {losses[0]:.3f} -> "
        f"{losses[-1]:.3f}")
    ncell = (256, 256, 256)
    c = W.surrogate_velocity(tuple(x + 1 for x in ncell), seed=777).astype(np.float32)
    vel = torch.from_numpy(c).to(dev)
    hs = sfm.Sfm(ncell, (cells, cells, cells), h, m, k, precision=sfm.SFM_PREC_FP64)
    acc, err, secs = sfm.sfm_build_roms_surrogate(hs.ctx, net, tol, 12.0, vel, stream=stream)
    S = len(acc)
    out = {
        "training_subdomains": n_samples, "m": m, "k": k, "box_cells": cells, "n_out": n_out,
        "params": net.n_params, "epochs": epochs, "batch": 64,
        "label_seconds": t_label, "train_seconds": t_train,
        "train_samples_per_s": n_samples * epochs / t_train, "loss_first_epoch": float(losses[0]),
        "loss_last_epoch": float(losses[-1]),
        "eval_workload": "256^3 cells, 512 subdomains of unseen seeded media", "tol": tol,
        "accepted": int(acc.sum()), "subdomains": S,
        "ntd_error_min": float(err.min()), "ntd_error_median": float(np.median(err)),
        "ntd_error_max": float(err.max()),
        "lanczos_seconds": float(secs[0]), "network_seconds": float(secs[1]), "judge_seconds": float(secs[2]),
        "network_roms_per_s": S / max(float(secs[1]), 1e-9), "lanczos_roms_per_s": S / max(float(secs[0]), 1e-9),
    }
    log(f"[bench] learned build of {S} subdomains: accepted {out['accepted']} at tol {tol}, NtD errors median "
        f"{out['ntd_error_median']:.2e}; Lanczos {secs[0]:.3f} s, network {secs[1]:.4f} s, judge {secs[2]:.3f} s")
    hs.close()
    net.close()
    return out


def adjoint_probe(torch, sfm, dev, stream, nsteps: int, checkpoint_every: int):
    """Misfit gradient on the gradient workload: observed traces from the medium with the Gaussian
    anomaly, ROMs of the background medium, J = 1/2 ||traces - observed||^2, dJ/d(Gamma, Gamma-hat)
    by the discrete adjoint with checkpoints; timed forward and gradient.  A checkpoint interval
    below nsteps is timed beside the run that holds every forward state and (-K X) in HBM (2 x 4001
    states of 2.6 MB at 4000 steps; the forward then runs once).  Then the sound-speed gradient
    through a network of the surrogate's architecture."""
    cfg = W.CFG_ADJOINT
    c_bg = cfg.velocity_model()
    c_true = W.gaussian_anomaly(c_bg, **W.ADJOINT_ANOMALY)
    src, rec = cfg.sources(), cfg.receivers()
    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    out = {"workload": cfg.name, "subdomains": cfg.n_subdomains, "m": cfg.m, "k": cfg.k, "p": cfg.p,
           "steps": nsteps, "receivers": len(rec), "checkpoint_every": checkpoint_every,
           "anomaly": "+5% Gaussian, radius 30 cells, domain centre"}
    tr_obs = torch.zeros((len(rec), nsteps), dtype=torch.float32, device=dev)
    tr = torch.zeros_like(tr_obs)
    h_obs = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k)
    sfm.sfm_build_roms(h_obs.ctx, torch.from_numpy(c_true.astype(np.float32)).to(dev), src, rec, stream=stream)
    dt_true = sfm.sfm_cfl_dt(h_obs.ctx, 100, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_build_roms(h.ctx, torch.from_numpy(c_bg.astype(np.float32)).to(dev), src, rec, stream=stream)
    torch.cuda.synchronize()
    out["build_seconds"] = time.perf_counter() - t0
    dt = 0.9 * min(dt_true, sfm.sfm_cfl_dt(h.ctx, 100, stream=stream))
    wav = torch.tensor(W.ricker(cfg.f_peak, dt, nsteps)[:, None], dtype=torch.float32, device=dev)
    sfm.sfm_step(h_obs.ctx, nsteps, dt, wav, tr_obs, stream=stream)      # observed data
    h_obs.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_step(h.ctx, nsteps, dt, wav, tr, stream=stream)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    resid = (tr - tr_obs).contiguous()
    J = 0.5 * float((resid.double() ** 2).sum().item())
    t0 = time.perf_counter()
    g_gam, g_hat = sfm.sfm_adjoint_gradient(h.ctx, nsteps, dt, wav, resid, checkpoint_every, stream=stream)
    t_grad = time.perf_counter() - t0
    t_hbm = None
    if checkpoint_every < nsteps:       # the same gradient with every forward state held in HBM
        t0 = time.perf_counter()
        g2, _ = sfm.sfm_adjoint_gradient(h.ctx, nsteps, dt, wav, resid, nsteps, stream=stream)
        t_hbm = time.perf_counter() - t0
        out["all_in_hbm_gradient_seconds"] = t_hbm
        out["all_in_hbm_vs_checkpointed_rel_l2"] = float(np.linalg.norm(g2 - g_gam) / np.linalg.norm(g_gam))
        del g2
    # the sound-speed gradient through a network of the surrogate's architecture (seeded weights:
    # the cost does not depend on them)
    ntri = cfg.p * (cfg.p + 1) // 2
    net = sfm.Cnn(cfg.sub_cells[0] + 1, 32, 2 * cfg.k * ntri, max_batch=64, seed=17)
    gvel = torch.zeros(c_bg.shape, dtype=torch.float32, device=dev)
    vel_bg = torch.from_numpy(c_bg.astype(np.float32)).to(dev)
    sfm.sfm_surrogate_velocity_gradient(h.ctx, net, vel_bg, g_gam, g_hat, gvel, stream=stream)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_surrogate_velocity_gradient(h.ctx, net, vel_bg, g_gam, g_hat, gvel, stream=stream)
    t_vel = time.perf_counter() - t0
    out.update(velocity_gradient_seconds=t_vel, velocity_gradient_finite=bool(torch.isfinite(gvel).all().item()),
               velocity_gradient_network=f"3D CNN {cfg.sub_cells[0] + 1}^3 -> 4 conv x 32 ch -> "
                                         f"{2 * cfg.k * ntri} outputs, batches of 64")
    net.close()
    h.close()
    out.update(dt=dt, misfit=J, forward_seconds=t_fwd, forward_ms_per_step=t_fwd / nsteps * 1e3,
               gradient_seconds=t_grad, gradient_over_forward=t_grad / t_fwd,
               grad_gamma_norm=float(np.linalg.norm(g_gam)), grad_gamma_hat_norm=float(np.linalg.norm(g_hat)),
               gradient_finite=bool(np.isfinite(g_gam).all() and np.isfinite(g_hat).all()),
               fine_equiv_gcell_per_s_gradient=cfg.n_cells * nsteps / t_grad / 1e9)
    log(f"[bench] adjoint ({cfg.name}, {nsteps} steps): forward {t_fwd:.3f} s, gradient {t_grad:.3f} s "
        f"({t_grad / t_fwd:.2f}x the forward, checkpoints every {checkpoint_every})"
        + (f", {t_hbm:.3f} s with every state in HBM" if t_hbm else "")
        + f", sound-speed gradient through the network {t_vel:.3f} s, misfit {J:.4e}")
    return out


def main():
    global TIMING_EVERY
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--build-batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-receivers", action="store_true")
    ap.add_argument("--cfl-iters", type=int, default=200)
    ap.add_argument("--copy-probe-mib", type=int, default=2048,
                    help="size of the device copy timed as the practical HBM bandwidth reference")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--shots", type=int, default=64,
                    help="shots stepped together through the same ROMs after the single-shot run (0: skip)")
    ap.add_argument("--shot-steps", type=int, default=100)
    ap.add_argument("--surrogate-samples", type=int, default=20000,
                    help="training subdomains of the learned ROMs (0: skip)")
    ap.add_argument("--surrogate-epochs", type=int, default=6)
    ap.add_argument("--uneven-steps", type=int, default=1500,
                    help="steps of the many-shot uneven-box workload (0: skip it)")
    ap.add_argument("--adjoint-steps", type=int, default=4000,
                    help="steps of the misfit-gradient probe on the 256^3 gradient workload (0: skip)")
    ap.add_argument("--adjoint-checkpoint", type=int, default=100,
                    help="checkpoint interval of the gradient probe (0: every forward state held in HBM); "
                         "a shorter interval is timed beside the all-in-HBM run")
    ap.add_argument("--timing-every", type=int, default=TIMING_EVERY,
                    help="time the kernels of one step in this many (1 = every step)")
    ap.add_argument("--no-finite-shift", action="store_true",
                    help="skip the finite-shift ROM probe (4^3-subdomain sample of the same ROM shape)")
    args = ap.parse_args()
    TIMING_EVERY = max(1, args.timing_every)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); splitting the subdomains over "
              f"several GPUs (one boundary exchange per cut face per step) is designed but not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1406_6923_amd import sfm

    cfg = workload(args.workload)
    prec = {"fp32": sfm.SFM_PREC_FP32, "bf16": sfm.SFM_PREC_BF16_FP32ACC, "fp64": sfm.SFM_PREC_FP64}[args.precision]
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    log(f"[bench] workload {cfg.name}: generating velocity {cfg.nodes}")
    t0 = time.perf_counter()
    c = cfg.velocity_model()
    c_max = float(c.max())
    vel = torch.from_numpy(c.astype(np.float32)).to(dev)
    log(f"[bench] velocity ready ({time.perf_counter() - t0:.1f} s), c in [{c.min():.0f}, {c_max:.0f}]")
    src = cfg.sources()
    rec = cfg.receivers()
    n_main_src = len(src)
    nshot = args.shots if prec == sfm.SFM_PREC_FP32 else 0
    if nshot:
        # the shot sources ride along in the build; they stay silent in the single-shot run
        src = np.concatenate([np.asarray(src).reshape(-1, 3), np.asarray(shot_sources(cfg, nshot))])

    h = sfm.Sfm(cfg.ncell, cfg.sub_cells, cfg.h, cfg.m, cfg.k, precision=prec, build_batch=args.build_batch)
    info = h.info()
    S = info["n_subdomains"]
    log(f"[bench] building {S} ROMs (p = {info['p']}, k = {info['k']}) on the GPU")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sfm.sfm_build_roms(h.ctx, vel, src, rec, stream=stream)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    log(f"[bench] build {t_build:.2f} s ({S / t_build:.1f} builds/s)")

    t0 = time.perf_counter()
    dt_max = sfm.sfm_cfl_dt(h.ctx, args.cfl_iters, stream=stream)
    t_cfl = time.perf_counter() - t0
    log(f"[bench] certified stability limit {dt_max:.6e} s in {t_cfl:.2f} s")
    dt = 0.9 * dt_max
    dt_fine = 0.9 * cfg.h / (math.sqrt(3.0) * c_max)
    ratio = dt / dt_fine
    log(f"[bench] dt_ROM = {dt:.4e} s, dt_fine = {dt_fine:.4e} s, ratio {ratio:.3f}")

    nrec = 0 if args.no_receivers else len(rec)
    total = args.warmup + args.steps
    wav_np = np.zeros((total, len(src)))
    wav_np[:, :n_main_src] = W.ricker(cfg.f_peak, dt, total)[:, None]
    wav = torch.tensor(wav_np, dtype=torch.float32, device=dev)
    traces = torch.zeros((max(nrec, 1), max(args.steps, 1)), dtype=torch.float32, device=dev) if nrec else None
    warm_tr = torch.zeros((max(nrec, 1), max(args.warmup, 1)), dtype=torch.float32, device=dev) if nrec else None

    if args.warmup:
        sfm.sfm_step(h.ctx, args.warmup, dt, wav[:args.warmup].contiguous(), warm_tr, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] warm-up {args.warmup} steps done; timing {args.steps} steps")
    # Per-kernel device times are taken live in the timed region: the library records a
    # hipEvent pair around every kernel of one step in TIMING_EVERY on the stream it launches on.
    sfm.sfm_set_timing(h.ctx, True, every=TIMING_EVERY)
    t0 = time.perf_counter()
    sfm.sfm_step(h.ctx, args.steps, dt, wav[args.warmup:].contiguous(), traces, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps: {wall:.3f} s")
    info = h.info()
    sfm.sfm_set_timing(h.ctx, False)
    main_ms = info["timed_main_ms"] / max(info["timed_steps"], 1)
    face_ms = info["timed_face_ms"] / max(info["timed_steps"], 1)
    rec_ms = info["timed_record_ms"] / max(info["timed_steps"], 1)
    k, p = info["k"], info["p"]
    elem = {sfm.SFM_PREC_FP32: 4, sfm.SFM_PREC_BF16_FP32ACC: 2, sfm.SFM_PREC_FP64: 8}[prec]
    bytes_per_sub = (2 * k - 1) * p * (p + 1) // 2 * elem + 3 * k * p * 4
    launch_bytes = S * bytes_per_sub
    achieved = launch_bytes / (main_ms * 1e-3) / 1e9
    if prec == sfm.SFM_PREC_FP32:
        traffic, traffic_note = traffic_from_profiles(launch_bytes)
    else:
        traffic, traffic_note = None, "committed counters cover the FP32 kernel only"
    log(f"[bench] main kernel {main_ms:.4f} ms ({achieved:.0f} GB/s algorithmic), face {face_ms:.4f} ms, "
        f"receivers {rec_ms:.4f} ms")

    finite = bool(torch.isfinite(traces).all().item()) if traces is not None else True

    # Measured device-copy bandwidth (reads + writes) as the practical HBM reference.
    n = max(args.copy_probe_mib, 2048) * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * 4 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    log(f"[bench] device copy {copy_gbs:.0f} GB/s")
    # Sustained FP64 matrix-core rate on register operands: the practical ceiling of the build's
    # products and of the FP64 many-shot kernel, beside the published peak.
    pbuf = torch.empty(4096 * 256, dtype=torch.float64, device=dev)
    sfm.sfm_probe_fp64_matrix_rate(pbuf, 4096, 200, stream=stream)
    fp64_mfma = sfm.sfm_probe_fp64_matrix_rate(pbuf, 4096, 2000, stream=stream)
    del pbuf
    log(f"[bench] FP64 matrix cores sustain {fp64_mfma:.1f} TFLOP/s (published peak {FP64_MFMA_PEAK_TFLOPS})")

    comparators = {}
    if not args.no_comparators:
        # fine-grid FDTD on the same grid at its own stability limit
        nf = min(args.steps, 200)
        wf = torch.tensor(W.ricker(cfg.f_peak, dt_fine, nf)[:, None], dtype=torch.float32, device=dev)
        secs = sfm.sfm_fdtd_run(cfg.ncell, cfg.h, vel, dt_fine, nf, cfg.sources(), wf, None, None, stream=stream)
        fdtd_rate = cfg.n_cells * nf / secs / 1e9
        log(f"[bench] fine-grid FDTD: {secs / nf * 1e3:.4f} ms/step, {fdtd_rate:.1f} Gcell-updates/s")
        # plain per-subdomain ROM stepping (same math, one launch per subdomain per step)
        npl = 3
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sfm.sfm_step_plain(h.ctx, npl, dt, wav[:npl].contiguous(), stream=stream)
        torch.cuda.synchronize()
        tpl = (time.perf_counter() - t1) / npl
        plain_rate = cfg.n_cells * ratio / tpl / 1e9
        log(f"[bench] plain per-subdomain stepping: {tpl * 1e3:.2f} ms/step")
        comparators = {
            "fine_fdtd_gcell_per_s": fdtd_rate, "fine_fdtd_ms_per_step": secs / nf * 1e3,
            "plain_rom_gcell_per_s": plain_rate, "plain_rom_ms_per_step": tpl * 1e3,
        }
    ms_per_step = wall / max(args.steps, 1) * 1e3
    value = cfg.n_cells * args.steps * ratio / wall / 1e9
    out = {
        "metric": "fine-grid-equiv Gcell-updates/s",
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {sfm.SFM_PREC_FP32: "f32", sfm.SFM_PREC_BF16_FP32ACC: "bf16-coef/f32-acc",
                  sfm.SFM_PREC_FP64: "f64-coef/f32-state"}[prec],
        "data": "synthetic",
        "config": {
            "workload": cfg.name,
            "ncell": list(cfg.ncell), "sub_cells": list(cfg.sub_cells), "subdomains": S,
            "m": cfg.m, "k": cfg.k, "p": p, "h": cfg.h, "receivers": nrec, "sources": n_main_src,
            "silent_shot_sources_in_build": nshot,
            "velocity": "seeded 20-layer model (1500-4500 m/s) + 50 spheres (+-30%)",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "step_main_kernel",
            "algorithmic_bytes_per_launch": launch_bytes,
            "avg_launch_ms": main_ms,
            "timed_launches": info["timed_steps"],
            "timed_one_step_in": TIMING_EVERY,
            "traffic_note": traffic_note,
        },
        "rom_builds_per_s": S / t_build,
        "stability_certificate_seconds": t_cfl,
        "build_seconds": t_build,
        "dt_rom": dt,
        "dt_fine": dt_fine,
        "dt_ratio": ratio,
        "raw_gcell_per_s": cfg.n_cells * args.steps / wall / 1e9,
        "face_kernel_ms": face_ms,
        "receiver_kernel_ms": rec_ms,
        "traces_finite": finite,
        "copy_gbs": copy_gbs,
        "frac_of_copy": achieved / copy_gbs,
        "fp64_matrix_probe_tflops": fp64_mfma,
    }
    if comparators:
        comparators["speedup_vs_fine_fdtd"] = value / comparators["fine_fdtd_gcell_per_s"]
        comparators["speedup_vs_plain_rom"] = value / comparators["plain_rom_gcell_per_s"]
        out["comparators"] = comparators
    if nshot:
        out["shots"] = shots_probe(torch, sfm, h, cfg, dev, stream, dt, ratio, nshot, n_main_src, 10,
                                   args.shot_steps, nrec, ms_per_step)
    if args.uneven_steps:
        out["many_shots_uneven"] = uneven_shots_probe(torch, sfm, dev, stream, args.uneven_steps)
        rf = out["many_shots_uneven"]["roofline"]
        rf["measured_fp64_matrix_tflops"] = fp64_mfma
        rf["frac_of_measured"] = rf["achieved"] / fp64_mfma
    if args.surrogate_samples:
        out["learned_roms"] = surrogate_probe(torch, sfm, dev, stream, args.surrogate_samples, args.surrogate_epochs)
    if not args.no_finite_shift:
        out["finite_shift"] = finite_shift_probe(torch, sfm, dev, stream)
        if prec == sfm.SFM_PREC_FP32 and "dt_ratio_vs_sigma_inf" in out["finite_shift"]:
            out["finite_shift"]["fp64_stream_at_scale"] = fp64_stream_probe(
                torch, sfm, h, cfg, dt, ratio, out["finite_shift"]["dt_ratio_vs_sigma_inf"])
    if args.adjoint_steps:
        out["adjoint"] = adjoint_probe(torch, sfm, dev, stream, args.adjoint_steps,
                                       args.adjoint_checkpoint or args.adjoint_steps)
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: oracle on a one-subdomain sample")
        out["cpu_baseline"] = cpu_baseline(cfg, c, ratio)
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
