"""Throughput benchmark of the D2Q9 LBGK hot path on one MI355X.

One benchmark step = one pass of the whole path over the forced-turbulence
workload: 500 fused stream+collide steps of a 4096^2 FP32 grid with Guo
forcing and linear drag, the moments at the last step, and the sub-volume
energy/enstrophy balance at box sizes 8..256 (the workload's diagnostic
cadence is one balance every 500 steps).  Inputs are resident in HBM before
the timed region; the timed region is bracketed by torch.cuda.synchronize().
The step-kernel shape, including how many steps one launch advances
(temporal blocking), is chosen by the library's autotuner.

Prints ONE JSON line on stdout (everything else goes to stderr):
value = lattice updates per second of the whole pass (MLUPS), with the
dominant kernel's roofline (HIP events around its launches on the library's
stream; algorithmic bytes of one launch = every population read and written
once plus the force field read once, whatever the number of steps fused) and
the FP64 CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--tau T]
                       [--no-cpu-baseline] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9 MLUPS/GPU + % HBM roofline; batched-ensemble & adjoint MLUPS vs plain"
HBM_PEAK_GBS = 8000.0
STEPS_PER_PASS = 500
SIZES = (8, 16, 32, 64, 128, 256)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"k_step": ("lbm_step.hip", "lbm_site.h"),
                  "k_step_fused": ("lbm_step_fused.hip", "lbm_fused.h", "lbm_site.h"),
                  "k3_step": ("lbm3d.hip",)}


def step_source_digest(kernel="k_step_fused"):
    """Digest of a step kernel's sources (its counters are valid only for them)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1809_06735_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profile_record(kernel, workload, tile):
    """The committed counter record of a step kernel in this launch shape, or None when
    it is missing or was taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("TRAFFIC_JSON:"):
            continue
        rec = json.loads(line.split(":", 1)[1])
        if rec.get("source_sha256_16") != step_source_digest(kernel):
            return None
        rt, tl = list(rec.get("tile", [])), list(tile)
        if rt == tl:
            return rec
        # band heights that give the same number of bands are the same launch
        lo, hi = rec.get("ry_range", (None, None))
        if lo is not None and len(rt) == len(tl) == 8 and rt[:3] + rt[4:] == tl[:3] + tl[4:] and lo <= tl[3] <= hi:
            return rec
    return None


def traffic_from_profile(kernel, workload, tile):
    """Per-launch HBM bytes of a step kernel from the committed counter summary, or None."""
    rec = profile_record(kernel, workload, tile)
    return rec.get("bytes_per_launch") if rec else None


# VALU issue of the chip: one wavefront instruction per CU and clock, 256 CUs at 2.4 GHz,
# 64 lanes (FP32 without packed instructions, which this library does not use).
VALU_LANE_OPS_PER_S = 256 * 2.4e9 * 64


def method_valu_per_update(workload="forced4096"):
    """VALU lane-instructions per lattice update of the method itself: the counted
    instructions of the one-step kernel (one collision per site, no halo recomputation),
    the leanest shape among the committed counter records of the current source; None if
    no record is current."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_traffic.md")
    if not os.path.exists(path):
        return None, None
    best = (None, None)
    for line in open(path):
        if not line.startswith("TRAFFIC_JSON:"):
            continue
        rec = json.loads(line.split(":", 1)[1])
        v = rec.get("valu_lane_instructions_per_update")
        if rec.get("source_sha256_16") != step_source_digest("k_step") or not v:
            continue
        if best[0] is None or v < best[0]:
            best = (v, rec.get("tile"))
    return best


def single_step_kernel(n, tau, alpha, fx, fy, steps=400):
    """The one-step-per-launch kernel on the same workload, in its tuned shape."""
    import numpy as np
    import torch
    from paper_1809_06735_amd import Simulation
    z = np.zeros((n, n))
    s = Simulation(np.ones((n, n)), z, z, tau, dtype="f32", fx=fx, fy=fy, alpha=alpha)
    best = None
    for shape in ((512, 1, 1, 1, 1), (256, 1, 1, 1, 1), (512, 1, 1, 1, 0)):
        s.set_tile(*shape)
        s.step(22)
        torch.cuda.synchronize()
        s.step_time(reset=True)
        s.step_timing(True)
        s.step(steps + 2)
        torch.cuda.synchronize()
        s.step_timing(False)
        ms, nl = s.step_time(reset=True)
        per = ms * 1e-3 / nl
        if best is None or per < best[1]:
            best = (shape, per)
    s.close()
    shape, per = best
    gbs = 80 * n * n / per / 1e9
    tile = tuple(shape) + (1, 0, 0)
    return {"shape": list(tile), "avg_launch_us": round(per * 1e6, 2), "GBps": round(gbs, 1),
            "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4), "kernel_MLUPS": round(n * n / per / 1e6, 1),
            "traffic": traffic_from_profile("k_step", "forced4096", tile)}


def paper_set_up_256(log, steps=20000, every=100):
    """The paper's own forced workload (Sec. 3 and 5): 256^2 FP32, exact-difference forcing
    with the constant-phase stream-function force on 5 <= |k| <= 7 and the damping of
    1 <= |k| <= 2, for every tau0 of Sec. 5: `steps` steps from rest with the sub-volume
    balance every `every` steps (all box sides of the workload)."""
    import math
    import numpy as np
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation
    w = inp.WORKLOADS["paper256"]
    n = w.n
    fx, fy = inp.paper_forcing(n)
    z = np.zeros((n, n))
    runs = {}
    for tau in w.taus:
        sim = Simulation(np.ones((n, n)), z, z, tau, dtype="f32", fx=fx, fy=fy, scheme="edm",
                         damp_f0=inp.PAPER_DAMPING_F0, damp_shell=inp.PAPER_DAMPING_SHELL,
                         with_balance=True)
        sim.step(2 * every)  # spin-up, untimed
        torch.cuda.synchronize()
        sim.step_timing(True)
        t0 = time.perf_counter()
        stats = []
        for _ in range(steps // every - 2):
            sim.step(every)
            stats.append(sim.balance(w.sizes)["stats"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, nl = sim.step_time(reset=True)
        sim.step_timing(False)
        _, ux, uy, sc = sim.moments()
        urms = math.sqrt(float((ux.double() ** 2 + uy.double() ** 2).mean()))
        nu = (tau - 0.5) / 3
        nsamp = len(stats)
        mean = lambda L, q: float(np.nanmean([st[k][q]["mean"] for st in stats
                                              for k in range(len(w.sizes)) if st[k]["L"] == L]))
        runs[str(tau)] = {
            "steps_timed": nsamp * every, "balance_samples": nsamp,
            "wall_s": round(wall, 3),
            "MLUPS_with_balance": round(n * n * nsamp * every / wall / 1e6, 1),
            "step_us": round(kms * 1e3 / max(nl, 1), 2),
            "step_MLUPS": round(n * n * nl / (kms * 1e-3) / 1e6, 1) if kms > 0 else None,
            "U_rms": round(urms, 4), "U_rms_exact": urms, "Re_UN_over_nu": round(urms * n / nu, 0),
            "min_rho": round(sc["min_rho"], 4),
            "mean_dE": {str(L): mean(L, "dE") for L in (4, 16, 64, 181, 256)},
            "mean_dZ": {str(L): mean(L, "dZ") for L in (4, 16, 64, 181, 256)},
            "mean_Ma": {str(L): mean(L, "Ma") for L in (4, 256)}}
        log(f"[bench] paper set-up tau0={tau}: {runs[str(tau)]['step_us']} us/step, "
            f"U_rms {urms:.4f}, Re {urms * n / nu:.0f}")
        sim.close()
    # the same runs stepped together: one launch of the Fourier sums, one of the
    # coefficients and one of the step kernel per step for all of them (no balance)
    from paper_1809_06735_amd.ensemble import Ensemble
    mem = [{"rho": np.ones((n, n)), "ux": z, "uy": z, "tau": tau, "scheme": "edm", "fx": fx, "fy": fy,
            "damp_f0": inp.PAPER_DAMPING_F0, "damp_shell": inp.PAPER_DAMPING_SHELL} for tau in w.taus]
    ens = Ensemble(mem, dtype="f32", chunk=every)
    ens.step(2 * every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(steps - 2 * every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nb = steps - 2 * every
    same = []
    for r, tau in enumerate(w.taus):
        _, ux, uy, _ = ens.moments(r)
        urms = math.sqrt(float((ux.double() ** 2 + uy.double() ** 2).mean()))
        same.append(urms == runs[str(tau)]["U_rms_exact"])
    for v in runs.values():
        v.pop("U_rms_exact")
    batched = {"runs": len(w.taus), "steps_timed": nb,
               "us_per_step_all_runs": round(wall / nb * 1e6, 2),
               "us_per_run_step": round(wall / nb / len(w.taus) * 1e6, 2),
               "MLUPS": round(n * n * len(w.taus) * nb / wall / 1e6, 1),
               "U_rms_equal_to_single_runs": all(same)}
    log(f"[bench] paper set-up, {len(w.taus)} runs batched: {batched['us_per_run_step']} us per run-step "
        f"({batched['MLUPS']} MLUPS); final U_rms equal to the single runs: {all(same)}")
    ens.close()
    return {"workload": w.name, "damping_rate_F0R": inp.PAPER_DAMPING_F0,
            "forcing_F0T_lattice": inp.PAPER_FORCING_F0_LATTICE, "runs": runs, "batched": batched}


def paper_statistics_256(log, tau=0.52, nconf=25, every=100, spin_up=4000):
    """The statistics of Sec. 5 as the paper presents them, on the paper's set-up at
    tau0 = 0.52: 25 configurations every `every` steps after a spin-up, each restarted from
    its checkpoint; all-corner statistics and PDFs at ~40 box sides (l = L/256 from 1/256
    to 1), the Table-1 random windows with their own PDFs, pooled over the configurations,
    and the energy spectrum of every configuration."""
    import numpy as np
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation, configuration_statistics, sample_configurations
    n = 256
    fx, fy = inp.paper_forcing(n)
    z = np.zeros((n, n))
    sim = Simulation(np.ones((n, n)), z, z, tau, dtype="f32", fx=fx, fy=fy, scheme="edm",
                     damp_f0=inp.PAPER_DAMPING_F0, with_balance=True)
    sim.step(spin_up)
    cfgs = sample_configurations(sim, nconf, every)
    sizes = tuple(sorted({int(v) for v in np.round(np.logspace(0, np.log10(n), 40))} | {181}))
    e = inp.log_edges(1e-7, 10.0, 10)
    edges = np.stack([e, e, np.linspace(0.0, 0.5, len(e))])
    samples = [inp.table1_corners(n, sizes, seed=i) for i in range(nconf)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = configuration_statistics(sim, cfgs, sizes, edges=edges, sample=lambda i: samples[i],
                                   spectrum_shells=182)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nwin_all = nconf * n * n * (len(sizes) - 1) + nconf
    nwin_smp = nconf * sum(samples[0][1])
    sim.close()
    pick = {3: "l~0.01", 181: "l~0.707", 256: "l=1"}
    out = {"tau0": tau, "configurations": nconf, "box_sides": len(sizes),
           "seconds_for_all_configurations": round(dt, 3),
           "ms_per_configuration": round(dt * 1e3 / nconf, 2),
           "all_corner_windows": nwin_all, "table1_windows": nwin_smp,
           "windows_per_s": round((nwin_all + nwin_smp) / dt, 0)}
    for L, tag in pick.items():
        k = sizes.index(L)
        out[tag] = {"all_mean_dE": res["stats"][k]["dE"]["mean"], "all_mean_dZ": res["stats"][k]["dZ"]["mean"],
                    "table1_mean_dE": res["sample_stats"][k]["dE"]["mean"],
                    "table1_count": res["sample_stats"][k]["dE"]["count"],
                    "mean_Ma": res["stats"][k]["Ma"]["mean"]}
    spec = res["spectra"].mean(0)
    out["spectrum_k1_k6_k32"] = [float(spec[1]), float(spec[6]), float(spec[32])]
    log(f"[bench] paper statistics: {nconf} configurations x {len(sizes)} sides in {dt:.2f} s")
    return out


def entropic_1024(log, n=1024, tau0=0.5005, steps=400):
    """The entropic collision (Sec. 1) on a decaying 1024^2 FP32 field at tau0 = 0.5005,
    autotuned single-step shape, against the BGK step on the same field: the cost of the
    per-site alpha solve (FP64 Newton iterations on the entropy equality)."""
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation
    rho, ux, uy = inp.spectrum_velocity(n, seed=0, max_mach=0.1)
    out = {"grid": n, "tau0": tau0, "dtype": "f32"}
    for coll in ("entropic", "bgk"):
        sim = Simulation(rho, ux, uy, tau0, dtype="f32", collision=coll)
        tile = sim.autotune(trial_steps=4) if coll == "entropic" else None
        sim.step(20)
        torch.cuda.synchronize()
        sim.step_timing(True)
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kms, nl = sim.step_time(reset=True)
        rec = {"MLUPS": round(n * n * steps / dt / 1e6, 1)}
        if nl:
            rec["kernel_MLUPS"] = round(n * n * nl * max(sim.get_tile()[5], 1) / (kms * 1e-3) / 1e6, 1)
        if coll == "entropic":
            a, _ = sim.relaxation()
            rec["shape"] = list(tile)
            rec["alpha_min"], rec["alpha_max"] = float(a.min()), float(a.max())
            _, _, _, sc = sim.moments()
            rec["finite"] = sc["nonfinite"] == 0
        out[coll] = rec
        sim.close()
    log(f"[bench] entropic {out['entropic']['MLUPS']} MLUPS vs BGK {out['bgk']['MLUPS']} at {n}^2")
    return out


def decay1024(log, passes=20):
    """The decaying-turbulence workload (1024^2 FP32, tau = 0.51, spectrum field of max Mach
    0.05, the balance at L = 8..256 every 100 steps): `passes` passes of 100 steps and one
    balance each, the balance beside the next pass's steps as in the main measurement.  The
    populations (75.5 MB) stay in the 256 MB Infinity Cache, so this rate is not an HBM
    figure."""
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation
    w = inp.WORKLOADS["decay1024"]
    _, ux, uy = inp.spectrum_velocity(w.n, seed=w.seed, max_mach=0.05)
    import numpy as np
    sim = Simulation(np.ones((w.n, w.n)), ux, uy, w.tau, dtype="f32", with_balance=True)
    tile = sim.autotune(trial_steps=5)
    sim.step(w.balance_every)
    sim.balance(w.sizes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pending = False
    for _ in range(passes):
        sim.step(w.balance_every)
        if pending:
            sim.balance_end()
        sim.balance_begin(w.sizes)
        pending = True
    res = sim.balance_end()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = w.n * w.n * w.balance_every * passes / dt / 1e6
    _, _, _, sc = sim.moments()
    out = {"grid": w.n, "dtype": "f32", "tau": w.tau, "steps": w.balance_every * passes,
           "balance_every": w.balance_every, "sizes": list(w.sizes), "shape": list(tile),
           "MLUPS_with_balance": round(mlups, 1), "finite": sc["nonfinite"] == 0,
           "mean_dE": {str(st["L"]): st["dE"]["mean"] for st in res["stats"]}}
    sim.close()
    log(f"[bench] decay1024: {out['MLUPS_with_balance']} MLUPS with the balance every {w.balance_every} steps")
    return out


def d3q19_256(log, n=256, tau=0.52, steps=200, lattice="d3q19"):
    """The three-dimensional extension: a forced 256^3 FP32 run on D3Q19 (or D3Q27) (one
    launch per step, 164 (228) algorithmic bytes per site: 19 (27) populations read and
    written, 3 force values read), timed with HIP events on the handle's stream, then the 3D
    balance with the stretching term at L = 16, 64, 256 over every cube corner.  `traffic`:
    HBM bytes per launch from the committed counter summary, if it was taken on the current
    kernel source (D3Q19 only)."""
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation3D
    shape = (n, n, n)
    rho, ux, uy, uz = inp.fields3(shape, seed=0, max_mach=0.1)
    fx, fy, fz = inp.force3(shape, seed=0, amp=1e-6)
    sim = Simulation3D(rho, ux, uy, uz, tau, dtype="f32", fx=fx, fy=fy, fz=fz, with_balance=True,
                       lattice=lattice)
    q = 27 if lattice == "d3q27" else 19
    del rho, ux, uy, uz, fx, fy, fz
    tile = sim.autotune(3)  # one step per launch, or 2..4 steps per launch (temporal blocking)
    sim.step(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sites = n ** 3
    gbs = (8 * q + 12) * sites / (ms * 1e-3) / 1e9
    out = {"grid": [n, n, n], "lattice": lattice, "dtype": "f32", "steps": steps, "shape": list(tile),
           "ms_per_step": round(ms, 4), "algorithmic_bytes_per_site": 8 * q + 12,
           "MLUPS": round(sites / (ms * 1e-3) / 1e6, 1), "kernel_GBps": round(gbs, 1),
           "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
           "traffic": (traffic_from_profile("k3_step", "d3q19_256", ["rows", "nt"])
                       if tile[0] == 1 and q == 19 else None)}
    sizes = (16, 64, 256)
    t0 = time.perf_counter()
    res = sim.balance(sizes)
    out["balance_s"] = round(time.perf_counter() - t0, 3)
    out["balance"] = {str(st["L"]): {"mean_dE": st["dE"]["mean"], "mean_dZ": st["dZ"]["mean"],
                                     "mean_Ma": st["Ma"]["mean"]} for st in res["stats"]}
    _, _, _, _, sc = sim.moments()
    out["finite"] = sc["nonfinite"] == 0
    sim.close()
    log(f"[bench] {lattice} {n}^3: {out['MLUPS']} MLUPS ({out['kernel_GBps']} GB/s), balance {out['balance_s']} s")
    return out


# Algorithmic HBM bytes per site of one balance call (FP64 fields, 13 term fields): the
# level-n moments (nine FP32 populations and the FP32 force in; FP64 rho, u and total
# force out), the term passes (pass A: levels n-2..n of rho, u and the force in, 7 terms
# and the auxiliary omega, sigma_xx, sigma_yy, sigma_xy out; pass B: level-n rho, u, the
# force and those four in, 5 terms and H out; pass C: omega and H in, 1 term out; the
# field means come from their workgroup sums), the prefix table's one read and one write
# after the passes, and one read of the table per walk over the window corners (a side L
# whose double 2 L is also asked for shares one walk with it).
BAL_BYTES_MOMENTS = (9 * 4 + 2 * 4) + (3 * 8 + 2 * 8)
BAL_BYTES_TERMS = (11 * 8 + 11 * 8) + (9 * 8 + 7 * 8) + (3 * 8 + 8)
BAL_BYTES_TABLES = 13 * 8 + 13 * 8
BAL_BYTES_PER_WALK = 13 * 8


def table_walks(sizes, nx, ny):
    """Walks over the window corners for these box sides, paired as the library pairs them."""
    m = min(nx, ny)
    twin = [None] * len(sizes)
    for k, L in enumerate(sizes):
        if twin[k] is not None or 2 * L > m or (2 * L == nx and 2 * L == ny):
            continue
        for k2, L2 in enumerate(sizes):
            if k2 != k and twin[k2] is None and L2 == 2 * L:
                twin[k], twin[k2] = k2, -1
                break
    return sum(1 for t in twin if t != -1)


def balance4096(log, calls=5):
    """Workload forced4096's diagnostic alone: the balance at L = 8..256 of a 4096^2 FP32
    run after 600 steps, in line (nothing beside it), time per call against the algorithmic
    bytes of its passes."""
    import numpy as np
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation
    w = inp.WORKLOADS["forced4096"]
    n = w.n
    fx, fy = inp.forcing_field(n, seed=w.seed, alpha=w.alpha)
    z = np.zeros((n, n))
    sim = Simulation(np.ones((n, n)), z, z, 0.51, dtype="f32", fx=fx, fy=fy, alpha=w.alpha,
                     with_balance=True)
    sim.step(600)
    sim.balance(SIZES)
    ts = []
    for _ in range(calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.balance(SIZES)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    sim.close()
    ms = float(np.median(ts)) * 1e3
    walks = table_walks(SIZES, n, n)
    per_site = BAL_BYTES_MOMENTS + BAL_BYTES_TERMS + BAL_BYTES_TABLES + walks * BAL_BYTES_PER_WALK
    gbs = per_site * n * n / (ms * 1e-3) / 1e9
    out = {"grid": n, "sizes": list(SIZES), "table_walks": walks, "calls": calls, "ms_per_call": round(ms, 3),
           "algorithmic_bytes_per_site": per_site, "GBps": round(gbs, 1),
           "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] balance at 4096^2 alone: {ms:.2f} ms per call, {gbs:.0f} GB/s of algorithmic bytes "
        f"({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    return out


def tau_sweep_4096(log, tile=None, steps=5000, every=500):
    """The forced 4096^2 workload's tau sweep {0.5005, 0.501, 0.505, 0.51, 0.55}: from rest,
    `steps` steps per tau with the balance at L = 8..256 every `every` steps (in line), in
    the launch shape of the headline run.  Per tau: MLUPS of the whole run, U_rms and max
    Mach at the end, mean delta^E / delta^Omega at L = 8 and 256, and, if the run diverges,
    the step at which the library reported it (LBM_E_DIVERGED), as data."""
    import numpy as np
    import torch
    import lbm_inputs as inp
    from paper_1809_06735_amd import LBMError, Simulation
    from paper_1809_06735_amd import _lib as L
    w = inp.WORKLOADS["forced4096"]
    n = w.n
    fx, fy = inp.forcing_field(n, seed=w.seed, alpha=w.alpha)
    z = np.zeros((n, n))
    out = {"grid": n, "steps_per_tau": steps, "balance_every": every, "balance_sizes": list(SIZES),
           "shape": list(tile) if tile else None, "runs": {}}
    for tau in w.taus:
        sim = Simulation(np.ones((n, n)), z, z, tau, dtype="f32", fx=fx, fy=fy, alpha=w.alpha,
                         with_balance=True)
        if tile:
            sim.set_tile(*tile)
        rec = {"diverged_at": None}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        try:
            for _ in range(steps // every):
                sim.step(every)
                res = sim.balance(SIZES)
            torch.cuda.synchronize()
        except LBMError as e:
            if e.code != L.LBM_E_DIVERGED:
                raise
            rec["diverged_at"] = sim.time
            rec["error"] = str(e)
        dt = time.perf_counter() - t0
        rec["MLUPS_with_balance"] = round(n * n * sim.time / dt / 1e6, 1)
        rec["steps_run"] = sim.time
        if rec["diverged_at"] is None:
            _, _, _, sc = sim.moments()
            rec["U_rms"] = float(np.sqrt(2 * sc["energy"] / sc["mass"]))
            rec["max_Mach"] = float(sc["max_speed"] * np.sqrt(3.0))
            st = {s["L"]: s for s in res["stats"]}
            rec["mean_dE"] = {str(k): st[k]["dE"]["mean"] for k in (SIZES[0], SIZES[-1])}
            rec["mean_dZ"] = {str(k): st[k]["dZ"]["mean"] for k in (SIZES[0], SIZES[-1])}
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out["runs"][str(tau)] = rec
        log(f"[bench] tau sweep {tau}: {rec['MLUPS_with_balance']} MLUPS, diverged_at {rec['diverged_at']}, "
            f"U_rms {rec.get('U_rms')}")
    return out


def cpu_baseline(n, tau, alpha, fx, fy, steps):
    import torch
    from oracle import ref
    import numpy as np
    f = ref.init_populations(np.ones((n, n)), np.zeros((n, n)), np.zeros((n, n)))
    fxt, fyt = ref.t64(fx), ref.t64(fy)
    f = ref.step(f, tau, fxt, fyt, alpha)          # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        f = ref.step(f, tau, fxt, fyt, alpha)
    dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps (PyTorch CPU) of the {n}^2 forced grid, "
                      f"{dt:.1f} s; step only, no balance"}


EXTRAS = {"paper_set_up_256": paper_set_up_256, "paper_statistics_256": paper_statistics_256,
          "entropic_1024": entropic_1024, "d3q19_256": d3q19_256, "decay1024": decay1024,
          "tau_sweep_4096": tau_sweep_4096,
          "d3q27_256": lambda log, steps=200: d3q19_256(log, steps=steps, lattice="d3q27"),
          "balance4096": balance4096}


def _ensemble_extra(log, steps=500):
    from paper_1809_06735_amd import ensemble as ens_mod
    return ens_mod.bench_ensemble(steps=steps, log=log)


def _ensemble_fixed_extra(log, steps=204):
    """The 64-run ensemble in every mode at fixed shapes (the autotuner's picks on MI355X:
    1024 threads x 1 site x 2 groups for the one-step modes; K = 6, 128-lane strips with the
    packed halo, 32-row bands for the multi-step modes), without the autotuner's trial
    launches: the run that kernel profiles are taken from."""
    from paper_1809_06735_amd import ensemble as ens_mod
    return ens_mod.bench_ensemble(steps=steps, log=log, tile=(1024, 1, 2), multi=(6, 128, 32, 1, 1),
                                  one_by_one=False)


def _adjoint_extra(log, steps=None):
    from paper_1809_06735_amd import adjoint as adj_mod
    return adj_mod.bench_adjoint(log=log, steps=steps)


EXTRAS["ensemble"] = _ensemble_extra
EXTRAS["ensemble_fixed"] = _ensemble_fixed_extra
EXTRAS["adjoint"] = _adjoint_extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tau", type=float, default=0.51)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only launch the step kernel of the workload (20 times, autotuned shape) "
                         "and the 1 GiB copy kernel (5 times), for hardware-counter runs")
    ap.add_argument("--only-extra", choices=sorted(EXTRAS),
                    help="run one extra measurement alone and print its JSON (profiling runs)")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --only-extra: also run the 1 GiB copy kernel 5 times (counter scale)")
    ap.add_argument("--extra-steps", type=int, default=None,
                    help="with --only-extra: the extra's step count (shorter profiling runs of the "
                         "extras that take one)")
    a = ap.parse_args()
    if a.only_extra:
        import inspect
        import torch
        fn = EXTRAS[a.only_extra]
        kw = {}
        if a.extra_steps is not None:
            if "steps" not in inspect.signature(fn).parameters:
                print(f"--extra-steps: {a.only_extra} takes no step count", file=sys.stderr)
                sys.exit(2)
            kw["steps"] = a.extra_steps
        res = fn(log, **kw)
        if a.with_copy:
            from paper_1809_06735_amd import _lib as L
            lib = L.load()
            buf = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
            for _ in range(5):
                L.check(lib.lbm_copy(buf[1 << 30:].data_ptr(), buf[:1 << 30].data_ptr(), 1 << 30,
                                     torch.cuda.current_stream().cuda_stream), "lbm_copy")
            torch.cuda.synchronize()
        print(json.dumps({a.only_extra: res}), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is "
              "described in the design notes but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lbm_inputs as inp
    from paper_1809_06735_amd import Simulation, copy_bandwidth

    w = inp.WORKLOADS["forced4096"]
    n = w.n
    log(f"[bench] building inputs {n}^2 (force field seed {w.seed})")
    fx, fy = inp.forcing_field(n, seed=w.seed, alpha=w.alpha)
    z = np.zeros((n, n))
    sim = Simulation(np.ones((n, n)), z, z, a.tau, dtype="f32", fx=fx, fy=fy, alpha=w.alpha,
                     with_balance=True)
    tile = sim.autotune(trial_steps=5)
    log(f"[bench] step kernel shape {tile}")
    if a.kernels_only:
        torch.cuda.synchronize()
        sim.step(20)
        torch.cuda.synchronize()
        sim.close()
        buf = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
        from paper_1809_06735_amd import _lib as L
        lib = L.load()
        for _ in range(5):
            L.check(lib.lbm_copy(buf[1 << 30:].data_ptr(), buf[:1 << 30].data_ptr(), 1 << 30,
                                 torch.cuda.current_stream().cuda_stream), "lbm_copy")
        torch.cuda.synchronize()
        log("[bench] kernels-only run done: 20 step launches, 5 copies of 1 GiB")
        return

    # One pass: STEPS_PER_PASS steps, then the balance of that time.  The balance runs on the
    # library's second stream beside the next pass's steps (lbm_balance_begin); its statistics
    # are collected once the next pass's steps are enqueued, and the last one before the clock
    # stops, so every pass's balance is inside the timed region.
    pending = [False]

    def one_pass():
        sim.step(STEPS_PER_PASS)
        res = sim.balance_end() if pending[0] else None
        sim.balance_begin(SIZES)
        pending[0] = True
        return res

    def drain():
        pending[0] = False
        return sim.balance_end()

    log(f"[bench] warmup {a.warmup} passes")
    for _ in range(a.warmup):
        one_pass()
    if pending[0]:
        drain()
    torch.cuda.synchronize()
    sim.step_time(reset=True)
    sim.step_timing(True)
    log(f"[bench] timing {a.steps} passes x {STEPS_PER_PASS} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(a.steps):
        one_pass()
    last = drain()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sim.step_timing(False)
    kern_ms, launches = sim.step_time(reset=True)
    lu = n * n * STEPS_PER_PASS * a.steps
    mlups = lu / elapsed / 1e6
    spl = max(tile[5], 1)                     # steps per launch of the bulk shape
    kernel = "k_step_fused" if spl > 1 else "k_step"
    avg_launch_s = kern_ms * 1e-3 / max(launches, 1)
    bytes_per_site = 9 * 4 * 2 + 2 * 4        # 9 reads + 9 writes + 2 force reads, FP32
    alg_bytes = bytes_per_site * n * n        # per launch, whatever the steps fused
    achieved = alg_bytes / avg_launch_s / 1e9
    traffic = traffic_from_profile(kernel, "forced4096", tile)
    # VALU instructions per lattice update: of this kernel in this shape (halo recomputation
    # and LDS addressing included) and of the method alone (the one-step kernel), from the
    # committed counters of the current sources
    rec = profile_record(kernel, "forced4096", tile)
    vpl = rec.get("valu_lane_instructions_per_update") if rec else None
    vpl_method, vpl_method_tile = method_valu_per_update()
    # the same kernel alone on the GPU (no balance beside it): 64 bulk launches, one graph
    torch.cuda.synchronize()
    sim.step_time(reset=True)
    sim.step_timing(True)
    sim.step(64 * spl + 2)
    torch.cuda.synchronize()
    sim.step_timing(False)
    alone_ms, alone_n = sim.step_time(reset=True)
    alone_s = alone_ms * 1e-3 / max(alone_n, 1)
    kern_mlups = n * n * spl / avg_launch_s / 1e6
    alone_mlups = n * n * spl / alone_s / 1e6
    peak_valu = VALU_LANE_OPS_PER_S / 1e12
    st = last["stats"]
    log(f"[bench] {mlups:.0f} MLUPS whole pass; {kernel} ({spl} steps/launch) "
        f"{avg_launch_s * 1e6:.1f} us/launch = {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.1%} "
        f"of 8 TB/s), {n * n * spl / avg_launch_s / 1e6:.0f} MLUPS in the kernel")

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed * 1e3 / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: fluid at rest, seeded random-phase divergence-free force on shells 4<=|k|<=6",
        "config": {"workload": f"forced4096: D2Q9 BGK {n}x{n} periodic FP32, Guo force + drag "
                               f"alpha={w.alpha}, tau={a.tau}; one step = {STEPS_PER_PASS} LBGK "
                               f"steps + moments + sub-volume balance at L={list(SIZES)} (the balance on a second "
                               f"stream, beside the next pass's steps)",
                   "grid": n, "tau": a.tau, "lbgk_steps_per_step": STEPS_PER_PASS,
                   "balance_sizes": list(SIZES), "step_kernel_shape": list(tile),
                   "parallelism": "single GPU"},
        # With K steps per launch (temporal blocking) the kernel moves 80/K B per lattice
        # update and is limited by VALU issue, not HBM: the headline view is the method's
        # VALU instructions (the one-step kernel's count per update) issued per second
        # against the chip's issue rate; the HBM views per launch and per update follow.
        "roofline": {"bound": "alu",
                     "achieved": round(kern_mlups * vpl_method / 1e6, 3) if vpl_method else None,
                     "peak": round(peak_valu, 3), "unit": "T VALU lane-instr/s",
                     "frac": round(kern_mlups * vpl_method / 1e6 / peak_valu, 4) if vpl_method else None,
                     "traffic": traffic,
                     "kernel": f"{kernel}<float, K={spl}> (pull stream + BGK collide + Guo force, "
                               f"{spl} steps per launch)" if spl > 1 else
                               "k_step (fused pull stream + BGK collide + Guo force)",
                     "steps_per_launch": spl,
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "kernel_MLUPS": round(kern_mlups, 1),
                     "method_valu_per_lattice_update": vpl_method,
                     "method_valu_counted_on": vpl_method_tile,
                     "kernel_valu_per_lattice_update": vpl,
                     "kernel_valu_frac": round(kern_mlups * vpl / 1e6 / peak_valu, 4) if vpl else None,
                     "peak_derivation": "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one wave64 VALU "
                                        "instruction per CU and clock (FP32 without packed "
                                        "instructions)",
                     "hbm_per_launch": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                                        "algorithmic_bytes_per_launch": alg_bytes,
                                        "note": "80 B per site per launch (9 populations read and "
                                                "written, the force read), whatever K"},
                     "hbm_per_lattice_update": {
                         "bytes_per_lattice_update": bytes_per_site,
                         "achieved": round(bytes_per_site * kern_mlups * 1e6 / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(bytes_per_site * kern_mlups * 1e6 / 1e9 / HBM_PEAK_GBS, 4),
                         "note": "the single-step roofline (80 B per lattice update); above 1 because "
                                 "temporal blocking advances K steps per HBM round trip"},
                     "alone": {"avg_launch_us": round(alone_s * 1e6, 2),
                               "kernel_MLUPS": round(alone_mlups, 1),
                               "frac": round(alone_mlups * vpl_method / 1e6 / peak_valu, 4) if vpl_method else None,
                               "hbm_per_launch_frac": round(alg_bytes / alone_s / 1e9 / HBM_PEAK_GBS, 4),
                               "note": "the same kernel timed without the balance running beside it"}},
        "balance_at_end": {str(s["L"]): {"mean_dE": s["dE"]["mean"], "mean_dZ": s["dZ"]["mean"],
                                         "mean_Ma": s["Ma"]["mean"]} for s in st},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()

    if not a.no_extras:
        extras = {}
        try:
            extras["single_step_kernel_forced4096"] = single_step_kernel(n, a.tau, w.alpha, fx, fy)
        except Exception as e:  # noqa: BLE001
            extras["single_step_kernel_forced4096"] = f"error: {e}"
        try:
            gbs, _ = copy_bandwidth(1 << 30, iters=10)
            extras["copy_kernel_GBps"] = round(gbs, 1)
        except Exception as e:  # noqa: BLE001
            extras["copy_kernel_GBps"] = f"error: {e}"
        try:
            rho0, ux0, uy0 = inp.spectrum_velocity(n, seed=0, max_mach=0.05)
            plain = Simulation(rho0, ux0, uy0, a.tau, dtype="f32")
            ptile = plain.autotune(trial_steps=5)
            plain.step(200)
            torch.cuda.synchronize()
            plain.step_timing(True)
            t1 = time.perf_counter()
            plain.step(1000)
            torch.cuda.synchronize()
            dtp = time.perf_counter() - t1
            kms, nl = plain.step_time(reset=True)
            per = kms * 1e-3 / nl                  # per launch of ptile[5] steps
            extras["plain_unforced_4096_fp32"] = {
                "MLUPS": round(n * n * 1000 / dtp / 1e6, 1), "shape": list(ptile),
                "kernel_GBps": round(72 * n * n / per / 1e9, 1),
                "frac_of_8TBps": round(72 * n * n / per / 1e9 / HBM_PEAK_GBS, 4)}
            plain.close()
            del plain
        except Exception as e:  # noqa: BLE001
            extras["plain_unforced_4096_fp32"] = f"error: {e}"
        try:
            extras["paper_set_up_256"] = paper_set_up_256(log)
        except Exception as e:  # noqa: BLE001
            extras["paper_set_up_256"] = f"error: {e}"
        try:
            extras["paper_statistics_256"] = paper_statistics_256(log)
        except Exception as e:  # noqa: BLE001
            extras["paper_statistics_256"] = f"error: {e}"
        try:
            extras["entropic_1024"] = entropic_1024(log)
        except Exception as e:  # noqa: BLE001
            extras["entropic_1024"] = f"error: {e}"
        try:
            extras["decay1024"] = decay1024(log)
        except Exception as e:  # noqa: BLE001
            extras["decay1024"] = f"error: {e}"
        try:
            extras["balance4096"] = balance4096(log)
        except Exception as e:  # noqa: BLE001
            extras["balance4096"] = f"error: {e}"
        try:
            extras["tau_sweep_4096"] = tau_sweep_4096(log, tile=tile)
        except Exception as e:  # noqa: BLE001
            extras["tau_sweep_4096"] = f"error: {e}"
        try:
            extras["d3q19_256"] = d3q19_256(log)
        except Exception as e:  # noqa: BLE001
            extras["d3q19_256"] = f"error: {e}"
        try:
            extras["d3q27_256"] = d3q19_256(log, lattice="d3q27")
        except Exception as e:  # noqa: BLE001
            extras["d3q27_256"] = f"error: {e}"
        try:
            from paper_1809_06735_amd import ensemble as ens_mod
            extras["ensemble"] = ens_mod.bench_ensemble(log=log)
        except Exception as e:  # noqa: BLE001
            extras["ensemble"] = f"unavailable: {e}"
        try:
            from paper_1809_06735_amd import adjoint as adj_mod
            extras["adjoint"] = adj_mod.bench_adjoint(log=log)
        except Exception as e:  # noqa: BLE001
            extras["adjoint"] = f"unavailable: {e}"
        out["extras"] = extras

    if not a.no_cpu_baseline:
        log(f"[bench] cpu baseline: {a.cpu_steps} oracle steps at {n}^2")
        out["cpu_baseline"] = cpu_baseline(n, a.tau, w.alpha, fx, fy, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
