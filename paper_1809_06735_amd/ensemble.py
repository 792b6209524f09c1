"""Batched ensemble of independent D2Q9 grids (lbm_batch_* of the C ABI)."""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _lib as L
from .sim import _dev64, _ptr, _require_gpu, _stream_handle

MODES = {"persistent": L.LBM_BATCH_PERSISTENT, "per_step": L.LBM_BATCH_PER_STEP,
         "multi_step": L.LBM_BATCH_MULTI_STEP, "persistent_multi": L.LBM_BATCH_PERSISTENT_MULTI}


class Ensemble:
    """Runs of possibly different sizes, tau, drag and force, stepped together.

    members: list of dicts with keys rho, ux, uy (arrays [ny, nx]), tau, and
    optionally fx, fy, alpha.  dtype: "f32" or "f64" for every run.

    Exact-difference runs (member key scheme = "edm", optional damp_f0 and
    damp_shell as for Simulation): every member on one grid size with the same
    force flag and damped shell; tau, damp_f0 and the force fields may differ.
    They step in the per-step mode, every run's Fourier sums, coefficients and
    step in one launch each.
    """

    def __init__(self, members, dtype="f32", device="cuda", stream=None, mode=None,
                 chunk=100, layout="rows"):
        _require_gpu()
        self._lib = L.load()
        self.device = torch.device(device)
        self.n = len(members)
        dt = {"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype]
        cfgs = (L.Config * self.n)()
        dev_inputs = []
        self.shapes = []
        sh = _stream_handle(stream)
        for r, m in enumerate(members):
            rho = _dev64(m["rho"], self.device)
            ux = _dev64(m["ux"], self.device)
            uy = _dev64(m["uy"], self.device)
            has_f = m.get("fx") is not None
            fx = _dev64(m["fx"], self.device) if has_f else None
            fy = _dev64(m["fy"], self.device) if has_f else None
            ny, nx = rho.shape
            self.shapes.append((ny, nx))
            shell = m.get("damp_shell", (1.0, 2.0))
            cfgs[r] = L.Config(nx=nx, ny=ny, dtype=dt, has_force=int(has_f), with_balance=0,
                               layout=L.LAYOUTS[layout], tau=float(m["tau"]),
                               drag_alpha=float(m.get("alpha", 0.0)),
                               force_scheme=L.SCHEMES[m.get("scheme", "guo")],
                               damp_f0=float(m.get("damp_f0", 0.0)), damp_kmin=float(shell[0]),
                               damp_kmax=float(shell[1]), stream=sh)
            dev_inputs.append((rho, ux, uy, fx, fy))
        nbytes = C.c_size_t()
        L.check(self._lib.lbm_batch_workspace_bytes(cfgs, self.n, C.byref(nbytes)),
                "lbm_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        arr = lambda k: (C.c_void_p * self.n)(*[  # noqa: E731
            (d[k].data_ptr() if d[k] is not None else None) for d in dev_inputs])
        h = C.c_void_p()
        L.check(self._lib.lbm_batch_init(cfgs, self.n, _ptr(self.workspace), nbytes.value, arr(0), arr(1),
                                         arr(2), arr(3), arr(4), C.byref(h)), "lbm_batch_init")
        self._h = h
        (stream or torch.cuda.current_stream(self.device)).synchronize()
        del dev_inputs
        if mode is None:
            mode = "per_step" if members[0].get("scheme", "guo") == "edm" else "persistent"
        self.set_mode(mode, chunk)

    def close(self):
        if getattr(self, "_h", None):
            L.check(self._lib.lbm_batch_destroy(self._h), "lbm_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def sites(self) -> int:
        return int(self._lib.lbm_batch_sites(self._h))

    @property
    def time(self) -> int:
        t = C.c_int64()
        L.check(self._lib.lbm_batch_time(self._h, C.byref(t)), "lbm_batch_time")
        return t.value

    def set_mode(self, mode="persistent", chunk=100):
        L.check(self._lib.lbm_batch_set_mode(self._h, MODES[mode], int(chunk)), "lbm_batch_set_mode")
        self.mode = mode

    def set_tile(self, vx, groups, block_threads=256):
        L.check(self._lib.lbm_batch_set_tile(self._h, int(block_threads), int(vx), int(groups)),
                "lbm_batch_set_tile")

    def set_multi(self, steps_per_launch, strip, band, nt=1, halo=0):
        """Shape of the multi-step mode (K steps per launch over strip x band tiles; halo=1
        packs the 2 (K - 1) halo columns into the `strip` lanes of a workgroup)."""
        t = L.Tile(int(strip), 1, 1, int(band), int(nt), int(steps_per_launch), 1, int(halo))
        L.check(self._lib.lbm_batch_set_multi(self._h, C.byref(t)), "lbm_batch_set_multi")

    def get_multi(self):
        """(steps_per_launch, strip, band, nt, halo) of the multi-step mode."""
        t = L.Tile()
        L.check(self._lib.lbm_batch_get_multi(self._h, C.byref(t)), "lbm_batch_get_multi")
        return t.fuse, t.bx, t.ry, t.nt, t.halo

    def get_mode(self):
        m, c = C.c_int32(), C.c_int32()
        L.check(self._lib.lbm_batch_get_mode(self._h, C.byref(m), C.byref(c)), "lbm_batch_get_mode")
        return {v: k for k, v in MODES.items()}[m.value], c.value

    def autotune(self, trial_steps=10):
        """Search mode and work-item shape; returns (block_threads, vx, groups)."""
        bt, vx, g = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self._lib.lbm_batch_autotune(self._h, int(trial_steps), C.byref(bt), C.byref(vx),
                                             C.byref(g)), "lbm_batch_autotune")
        self.mode = self.get_mode()[0]
        return bt.value, vx.value, g.value

    def step(self, n=1):
        L.check(self._lib.lbm_batch_step(self._h, int(n)), "lbm_batch_step")
        return self

    def moments(self, run, out_dtype=torch.float64, scalars=True):
        ny, nx = self.shapes[run]
        od = L.LBM_F64 if out_dtype == torch.float64 else L.LBM_F32
        rho = torch.empty((ny, nx), dtype=out_dtype, device=self.device)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        sc = (C.c_double * 8)() if scalars else None
        L.check(self._lib.lbm_batch_moments(self._h, int(run), _ptr(rho), _ptr(ux), _ptr(uy), od, sc),
                "lbm_batch_moments")
        if scalars:
            return rho, ux, uy, dict(zip(L.SCALAR_NAMES, list(sc)))
        return rho, ux, uy


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def bench_ensemble(nruns=64, steps=500, log=print, tile=None, multi=None, one_by_one=True):
    """MLUPS of the 64-run decaying ensemble (sizes 256^2..1024^2, FP32) in the persistent,
    per-step, multi-step and persistent multi-step modes, against the plain single-grid step
    (autotuned, multi-step shapes included) run member by member.  With tile =
    (block_threads, vx, groups) and multi = (K, strip, band, nt, halo) given, those shapes
    are set instead of autotuned."""
    import lbm_inputs as inp
    from .sim import Simulation

    log(f"[ensemble] building {nruns} members")
    members = inp.ensemble_members(nruns)
    ens = Ensemble(members, dtype="f32", mode="persistent", chunk=100)
    sites = ens.sites
    if tile is None or multi is None:
        tile = ens.autotune(trial_steps=12)
        multi = ens.get_multi()
        how = "autotuned"
    else:
        ens.set_tile(tile[1], tile[2], tile[0])
        ens.set_multi(*multi)
        how = "fixed"
    shapes = {"block_threads": tile[0], "vx": tile[1], "groups": tile[2],
              "multi_step": {"steps_per_launch": multi[0], "strip": multi[1], "band": multi[2],
                             "nt": multi[3], "halo": multi[4]}}
    if how == "autotuned":
        shapes["mode"] = ens.mode
    out = {"runs": nruns, "sites": sites, how: shapes}
    for mode in ("persistent", "per_step", "multi_step", "persistent_multi"):
        chunk = 100
        if mode in ("multi_step", "persistent_multi"):
            # a whole number of K-step rounds per graph replay (chunk is even)
            k = multi[0]
            chunk = k * -(-100 // k)
            chunk += k if chunk % 2 else 0
        n = chunk * max(1, round(steps / chunk))
        ens.set_mode(mode, chunk)
        ens.step(chunk)                    # warm-up, builds the graph
        dt = _timed(lambda: ens.step(n))
        out[f"{mode}_MLUPS"] = round(sites * n / dt / 1e6, 1)
        shape = multi if mode in ("multi_step", "persistent_multi") else tile
        log(f"[ensemble] {mode} (shape {shape}, {n} steps): {out[f'{mode}_MLUPS']} MLUPS")
    r, _, _, sc = ens.moments(0)
    out["finite"] = bool(sc["nonfinite"] == 0)
    ens.close()
    del ens
    torch.cuda.empty_cache()
    if not one_by_one:
        return out
    # plain single-grid step, one member of each size
    per_size = {}
    for m in members:
        n = m["n"]
        if n in per_size:
            continue
        s = Simulation(m["rho"], m["ux"], m["uy"], m["tau"], dtype="f32")
        s.autotune(trial_steps=5)
        s.step(100)
        dt = _timed(lambda: s.step(steps))
        per_size[n] = n * n * steps / dt / 1e6
        s.close()
    t_seq = sum(m["n"] ** 2 * steps / (per_size[m["n"]] * 1e6) for m in members)
    out["members_one_by_one_MLUPS"] = round(sites * steps / t_seq / 1e6, 1)
    out["single_grid_MLUPS_by_size"] = {str(k): round(v, 1) for k, v in sorted(per_size.items())}
    log(f"[ensemble] members one by one: {out['members_one_by_one_MLUPS']} MLUPS")
    return out
