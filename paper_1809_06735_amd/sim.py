"""Python front end of the HIP library: device memory and streams from PyTorch,
every computation in the library's kernels.

Classes / functions
-------------------
Simulation      one periodic D2Q9 grid (lbm_init / lbm_step / lbm_moments /
                lbm_subvolume_balance and the checkpoint, tuning and timing calls)
balance_fields  the sub-volume balance of caller-given (rho, u) levels
Simulation3D    one periodic D3Q19 grid with the 3D balance (lbm3_*)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1809_06735_amd needs a ROCm GPU (gfx950); none is visible")


def _dev64(a, device):
    """Host/torch array -> contiguous FP64 tensor on `device`."""
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def stats_to_dict(s: L.BalanceStats):
    """lbm_balance_stats -> {'L', 'dE': {...}, 'dZ': {...}, 'Ma': {...}}."""
    def one(pfx, count, nan):
        return {"count": int(count), "n_nan": int(nan), "mean": s.__getattribute__("mean_" + pfx),
                "std": s.__getattribute__("std_" + pfx), "min": s.__getattribute__("min_" + pfx),
                "max": s.__getattribute__("max_" + pfx)}
    return {"L": int(s.L), "dE": one("dE", s.count_dE, s.nan_dE),
            "dZ": one("dZ", s.count_dZ, s.nan_dZ), "Ma": one("Ma", s.count_Ma, 0)}


def _balance_args(nx, ny, sizes, windows):
    sizes = [int(v) for v in sizes]
    sz = (C.c_int32 * max(1, len(sizes)))(*sizes)
    out = (L.BalanceStats * max(1, len(sizes)))()
    if windows is not None and len(windows) > 0:
        flat = [int(v) for w in windows for v in w]
        win = (C.c_int32 * len(flat))(*flat)
        nwin = len(windows)
        wterms = (C.c_double * (L.NWVALS * nwin))()
    else:
        win, nwin, wterms = None, 0, None
    return sizes, sz, out, win, nwin, wterms


class _Extra:
    """Marshalling of the optional balance outputs (histograms on given edges,
    randomly placed windows, pooling over calls) into lbm_balance_extra."""

    def __init__(self, nsizes, edges=None, accumulate=False, sample=None, device="cuda",
                 all_corners=True):
        self.x = L.BalanceExtra()
        self.nsizes = nsizes
        self.ne = 0
        self.keep = []
        self.x.accumulate = int(bool(accumulate))
        if edges is not None:
            e = np.ascontiguousarray(edges, dtype=np.float64)
            if e.ndim == 1:
                e = np.stack([e, e, e])
            if e.shape[0] != 3:
                raise ValueError("edges: one row per quantity (delta^E, delta^Omega, Ma) or one row for all")
            self.ne = e.shape[1]
            self.e = np.ascontiguousarray(e)
            self.x.edges = self.e.ctypes.data_as(C.POINTER(C.c_double))
            self.x.nedges = self.ne
            if all_corners:
                self.h = np.zeros((nsizes, 3, self.ne + 1), dtype=np.int64)
                self.x.hist = self.h.ctypes.data_as(C.POINTER(C.c_int64))
        self.sample = sample is not None
        if self.sample:
            corners, counts = sample
            xy = torch.as_tensor(np.ascontiguousarray(corners, dtype=np.int32) if not
                                 isinstance(corners, torch.Tensor) else corners,
                                 dtype=torch.int32, device=device).contiguous()
            if len(counts) != nsizes or xy.dim() != 2 or xy.shape[1] != 2 or \
                    xy.shape[0] != sum(int(c) for c in counts):
                raise ValueError("sample: corners [sum(counts), 2] and one count per size")
            self.keep.append(xy)
            self.cnt = (C.c_int32 * max(1, nsizes))(*[int(c) for c in counts])
            self.sout = (L.BalanceStats * max(1, nsizes))()
            self.x.sample_xy = C.c_void_p(xy.data_ptr())
            self.x.sample_counts = self.cnt
            self.x.sample_out = self.sout
            if edges is not None:
                self.sh = np.zeros((nsizes, 3, self.ne + 1), dtype=np.int64)
                self.x.sample_hist = self.sh.ctypes.data_as(C.POINTER(C.c_int64))

    def into(self, res):
        if self.ne and hasattr(self, "h"):
            res["hist"] = self.h
        if self.sample:
            res["sample_stats"] = [stats_to_dict(self.sout[k]) for k in range(self.nsizes)]
            if self.ne:
                res["sample_hist"] = self.sh
        return res


def _balance_result(sizes, out, maps, nwin, wterms, terms, nx, ny):
    res = {"stats": [stats_to_dict(out[k]) for k in range(len(sizes))] if out is not None else []}
    if maps is not None:
        res["maps"] = maps
    if nwin:
        wv = np.frombuffer(wterms, dtype=np.float64).reshape(nwin, L.NWVALS).copy()
        res["window_terms"] = wv[:, :L.NTERMS]
        res["window_errors"] = wv[:, L.NTERMS:]  # delta^E, delta^Omega, Ma per window
    if terms is not None:
        res["terms"] = {k: terms[i] for i, k in enumerate(L.TERM_NAMES)}
    return res


class Simulation:
    """One periodic D2Q9 BGK grid on the current GPU.

    rho0, ux0, uy0: [ny, nx] initial fields (NumPy or torch, converted to FP64
    on the device); fx, fy: optional static external force; alpha: linear drag.
    dtype: "f32" or "f64" population storage.  layout: "rows" (the nine
    populations of a grid row contiguous, the faster one on MI355X) or "planes".
    scheme: "guo" (Guo's forcing term) or "edm" (the exact-difference method of
    the paper's Sec. 3); with "edm", damp_f0 > 0 adds the spectral damping
    F^R = -damp_f0 sum u^(k) e^{i k.x} of the modes damp_shell[0] <= |k| <=
    damp_shell[1] (Eq. 16, u^ the Fourier-series coefficients, so damp_f0 is
    a rate per step).  collision: "bgk" (Eq. 1) or "entropic" (the entropic
    scheme of Sec. 1, unforced: relaxation time 2 tau / alpha towards the
    minimiser of H, alpha per site from the entropy equality).
    """

    def __init__(self, rho0, ux0, uy0, tau, dtype="f32", fx=None, fy=None, alpha=0.0,
                 with_balance=False, device="cuda", stream=None, layout="rows", scheme="guo",
                 damp_f0=0.0, damp_shell=(1.0, 2.0), collision="bgk"):
        _require_gpu()
        self._lib = L.load()
        self.device = torch.device(device)
        r = _dev64(rho0, self.device)
        vx = _dev64(ux0, self.device)
        vy = _dev64(uy0, self.device)
        self.ny, self.nx = r.shape
        self.dtype = {"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype]
        self.dtype_name = dtype
        self.tau = float(tau)
        self.alpha = float(alpha)
        has_force = fx is not None
        self._stream = stream
        self.layout = layout
        cfg = L.Config(nx=self.nx, ny=self.ny, dtype=self.dtype, has_force=int(has_force),
                       with_balance=int(with_balance), layout=L.LAYOUTS[layout], tau=self.tau,
                       drag_alpha=self.alpha, force_scheme=L.SCHEMES[scheme],
                       damp_f0=float(damp_f0), damp_kmin=float(damp_shell[0]),
                       damp_kmax=float(damp_shell[1]), collision=L.COLLISIONS[collision],
                       stream=_stream_handle(stream))
        self.scheme = scheme
        self.collision = collision
        self._cfg = cfg
        nbytes = C.c_size_t()
        L.check(self._lib.lbm_workspace_bytes(C.byref(cfg), C.byref(nbytes)), "lbm_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        f_x = _dev64(fx, self.device) if has_force else None
        f_y = _dev64(fy, self.device) if has_force else None
        h = C.c_void_p()
        L.check(self._lib.lbm_init(C.byref(cfg), _ptr(self.workspace), nbytes.value, _ptr(r),
                                   _ptr(vx), _ptr(vy), _ptr(f_x), _ptr(f_y), C.byref(h)), "lbm_init")
        self._h = h
        # keep the inputs alive until the stream has consumed them
        self._inputs = (r, vx, vy, f_x, f_y)
        torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
        self._inputs = None

    # -- lifecycle ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            L.check(self._lib.lbm_destroy(self._h), "lbm_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- stepping ---------------------------------------------------------------------------
    def step(self, n: int = 1):
        L.check(self._lib.lbm_step(self._h, int(n)), "lbm_step")
        return self

    @property
    def time(self) -> int:
        t = C.c_int64()
        L.check(self._lib.lbm_time(self._h, C.byref(t)), "lbm_time")
        return t.value

    def moments(self, out_dtype=torch.float64, scalars=True):
        """(rho, ux, uy[, scalars dict]) at the current time."""
        od = L.LBM_F64 if out_dtype == torch.float64 else L.LBM_F32
        shape = (self.ny, self.nx)
        rho = torch.empty(shape, dtype=out_dtype, device=self.device)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        if scalars:
            sc = (C.c_double * 8)()
            rc = self._lib.lbm_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy), od, sc)
            d = dict(zip(L.SCALAR_NAMES, list(sc)))
            if rc == L.LBM_E_DIVERGED:
                raise L.LBMError(rc, self._lib.lbm_last_error().decode())
            L.check(rc, "lbm_moments")
            return rho, ux, uy, d
        L.check(self._lib.lbm_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy), od, None), "lbm_moments")
        return rho, ux, uy

    def balance(self, sizes, windows=None, maps=False, term_fields=False, edges=None,
                accumulate=False, sample=None, all_corners=True):
        """Sub-volume balance statistics at the current time (needs with_balance).

        edges: bin edges (one row, or one per quantity delta^E, delta^Omega, Ma) for
        histograms over the windows of each size; sample: (corners [total, 2], counts per
        size) of randomly placed windows (Table 1), statistics in 'sample_stats';
        accumulate: pool with the earlier calls since the last one without it;
        all_corners=False skips the all-corner statistics (sampled windows only)."""
        sizes, sz, out, win, nwin, wterms = _balance_args(self.nx, self.ny, sizes, windows)
        if not all_corners:
            out = None
        dm = torch.empty((len(sizes), 3, self.ny, self.nx), dtype=torch.float64,
                         device=self.device) if maps else None
        tf = torch.empty((L.NTERMS, self.ny, self.nx), dtype=torch.float64,
                         device=self.device) if term_fields else None
        if edges is None and not accumulate and sample is None:
            L.check(self._lib.lbm_subvolume_balance(self._h, sz, len(sizes), out, _ptr(dm), win, nwin,
                                                    wterms, _ptr(tf)), "lbm_subvolume_balance")
            return _balance_result(sizes, out, dm, nwin, wterms, tf, self.nx, self.ny)
        ex = _Extra(len(sizes), edges, accumulate, sample, self.device, all_corners)
        L.check(self._lib.lbm_subvolume_balance_ex(self._h, sz, len(sizes), out, _ptr(dm), win, nwin,
                                                   wterms, _ptr(tf), C.byref(ex.x)),
                "lbm_subvolume_balance_ex")
        return ex.into(_balance_result(sizes, out, dm, nwin, wterms, tf, self.nx, self.ny))

    def balance_begin(self, sizes):
        """Start the all-corner balance statistics of the current time on the library's
        second stream; steps issued afterwards overlap with it.  balance_end() returns
        {'stats': [...]} exactly as balance(sizes) would have."""
        self._bal_sizes = [int(v) for v in sizes]
        sz = (C.c_int32 * max(1, len(self._bal_sizes)))(*self._bal_sizes)
        L.check(self._lib.lbm_balance_begin(self._h, sz, len(self._bal_sizes)), "lbm_balance_begin")

    def balance_end(self):
        out = (L.BalanceStats * max(1, len(self._bal_sizes)))()
        L.check(self._lib.lbm_balance_end(self._h, out), "lbm_balance_end")
        return {"stats": [stats_to_dict(out[k]) for k in range(len(self._bal_sizes))]}

    def window_series(self, windows, every, count):
        """Balance of explicit windows (x0, y0, L) sampled every `every` (>= 2) steps,
        `count` times: the time series of one sub-volume's balance of Sec. 3 (Figs. 1-2).
        Returns {'time': [count], 'terms': [count, nwin, 13] box means (LHS and each
        right-hand-side term), 'errors': [count, nwin, 3] delta^E, delta^Omega, Ma_V}."""
        every, count = int(every), int(count)
        if every < 2:
            raise ValueError("every must be >= 2 (the time derivative needs two recorded steps)")
        times, terms, errs = [], [], []
        for _ in range(count):
            self.step(every)
            r = self.balance((), windows=windows)
            times.append(self.time)
            terms.append(r["window_terms"])
            errs.append(r["window_errors"])
        return {"time": np.array(times), "terms": np.stack(terms), "errors": np.stack(errs)}

    def enstrophy(self):
        """Global enstrophy 1/2 sum omega^2 of the current moments (omega by Eq. 18)."""
        v = C.c_double()
        L.check(self._lib.lbm_enstrophy(self._h, C.byref(v)), "lbm_enstrophy")
        return v.value

    def relaxation(self):
        """(alpha, nu_eff) FP64 [ny, nx] of the current populations: the entropic
        collision's alpha and nu_eff = c_s^2 (2 tau / alpha - 1/2) (alpha = 2, nu_eff = nu
        for the BGK collision)."""
        a = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        v = torch.empty_like(a)
        L.check(self._lib.lbm_relaxation(self._h, _ptr(a), _ptr(v)), "lbm_relaxation")
        return a, v

    def energy_spectrum(self, nshells=None):
        """Shell-summed kinetic-energy spectrum E(s) of the current velocity (Figs. 5 and 10),
        s = 0 .. nshells - 1 (default: up to the shell of (nx/2, ny/2)); needs with_balance."""
        ns = int(nshells) if nshells is not None else _default_shells(self.nx, self.ny)
        out = (C.c_double * ns)()
        L.check(self._lib.lbm_energy_spectrum(self._h, out, ns), "lbm_energy_spectrum")
        return np.frombuffer(out, dtype=np.float64).copy()

    # -- checkpoints ------------------------------------------------------------------------------
    def state_bytes(self) -> int:
        n = C.c_size_t()
        L.check(self._lib.lbm_state_bytes(self._h, C.byref(n)), "lbm_state_bytes")
        return n.value

    def save(self, out=None):
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        L.check(self._lib.lbm_save(self._h, _ptr(out)), "lbm_save")
        return out

    def load(self, state):
        """Restore a state written by :meth:`save` of a handle with the same grid, dtype and
        layout (the library checks its header; the size and device are checked here)."""
        dev = self.device
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        if not torch.is_tensor(state) or state.device != dev or not state.is_contiguous():
            raise ValueError("state must be a contiguous tensor on " + str(dev))
        if state.numel() * state.element_size() != self.state_bytes():
            raise ValueError(f"state holds {state.numel() * state.element_size()} bytes, "
                             f"this handle's state {self.state_bytes()}")
        L.check(self._lib.lbm_load(self._h, _ptr(state)), "lbm_load")
        return self

    # -- launch shape / graphs / timing ---------------------------------------------------------
    def set_tile(self, bx, by, vx, ry, nt=0, fuse=1, pf=0, halo=0):
        """Step-kernel shape; fuse = 2..6 selects the multi-step kernel (ry = band
        height, by = vx = 1; halo = 0: strip of bx columns plus a halo wavefront,
        halo = 1: bx threads holding the strip and its halo columns)."""
        t = L.Tile(bx, by, vx, ry, nt, fuse, pf, halo)
        L.check(self._lib.lbm_set_tile(self._h, C.byref(t)), "lbm_set_tile")

    def get_tile(self):
        t = L.Tile()
        L.check(self._lib.lbm_get_tile(self._h, C.byref(t)), "lbm_get_tile")
        return (t.bx, t.by, t.vx, t.ry, t.nt, max(t.fuse, 1), t.pf, t.halo)

    def autotune(self, trial_steps=10):
        """Time every candidate shape (per step) and keep the fastest; returns it
        as (bx, by, vx, ry, nt, fuse, pf, halo)."""
        t = L.Tile()
        L.check(self._lib.lbm_autotune(self._h, int(trial_steps), C.byref(t)), "lbm_autotune")
        return (t.bx, t.by, t.vx, t.ry, t.nt, max(t.fuse, 1), t.pf, t.halo)

    def set_graph(self, chunk):
        L.check(self._lib.lbm_set_graph(self._h, int(chunk)), "lbm_set_graph")

    def step_timing(self, enable=True):
        L.check(self._lib.lbm_step_timing(self._h, int(bool(enable))), "lbm_step_timing")

    def step_time(self, reset=False):
        """(milliseconds, launches) of the device-timed step kernels."""
        ms = C.c_double()
        n = C.c_int64()
        L.check(self._lib.lbm_step_time(self._h, C.byref(ms), C.byref(n), int(bool(reset))),
                "lbm_step_time")
        return ms.value, n.value


def balance_fields_noalloc(rho, ux, uy, nu, sizes, fx=None, fy=None, windows=None, maps=False,
                           term_fields=False, device="cuda", stream=None):
    """balance_fields through lbm_balance_fields_noalloc: the library's static per-GPU
    scratch instead of a workspace (grids up to about 590^2).  rho/ux/uy: three levels
    (n-2, n-1, n) as device FP64 [ny, nx] tensors or host arrays; nu a scalar."""
    _require_gpu()
    lib = L.load()
    dev = torch.device(device)
    rs = [_dev64(a, dev) for a in rho]
    xs = [_dev64(a, dev) for a in ux]
    ys = [_dev64(a, dev) for a in uy]
    ny, nx = rs[2].shape
    f_x = _dev64(fx, dev) if fx is not None else None
    f_y = _dev64(fy, dev) if fy is not None else None
    inp = L.BalanceInput()
    inp.nx, inp.ny, inp.nu = nx, ny, float(nu)
    for k in range(3):
        inp.rho[k] = rs[k].data_ptr()
        inp.ux[k] = xs[k].data_ptr()
        inp.uy[k] = ys[k].data_ptr()
    inp.fx = f_x.data_ptr() if f_x is not None else None
    inp.fy = f_y.data_ptr() if f_y is not None else None
    inp.stream = _stream_handle(stream).value
    sizes, sz, out, win, nwin, wterms = _balance_args(nx, ny, sizes, windows)
    dm = torch.empty((len(sizes), 3, ny, nx), dtype=torch.float64, device=dev) if maps else None
    tf = torch.empty((L.NTERMS, ny, nx), dtype=torch.float64, device=dev) if term_fields else None
    L.check(lib.lbm_balance_fields_noalloc(C.byref(inp), sz, len(sizes), out, _ptr(dm), win, nwin, wterms,
                                           _ptr(tf)), "lbm_balance_fields_noalloc")
    return _balance_result(sizes, out, dm, nwin, wterms, tf, nx, ny)


def balance_fields(rho, ux, uy, nu, sizes, fx=None, fy=None, windows=None, maps=False,
                   term_fields=False, device="cuda", stream=None, edges=None, sample=None,
                   all_corners=True, workspace=None, accumulate=False):
    """Sub-volume balance of given fields: rho/ux/uy are three levels (n-2, n-1, n).
    edges / sample / accumulate / all_corners as Simulation.balance; pooling needs the
    same `workspace` (a uint8 device tensor of lbm_balance_workspace_bytes) across calls."""
    _require_gpu()
    lib = L.load()
    dev = torch.device(device)
    rs = [_dev64(a, dev) for a in rho]
    xs = [_dev64(a, dev) for a in ux]
    ys = [_dev64(a, dev) for a in uy]
    ny, nx = rs[2].shape
    f_x = _dev64(fx, dev) if fx is not None else None
    f_y = _dev64(fy, dev) if fy is not None else None
    inp = L.BalanceInput()
    nu_f = None
    if np.ndim(nu) == 0 and not (isinstance(nu, torch.Tensor) and nu.dim() > 0):
        inp.nx, inp.ny, inp.nu = nx, ny, float(nu)
    else:  # a viscosity field at level n
        nu_f = _dev64(nu, dev)
        if tuple(nu_f.shape) != (ny, nx):
            raise ValueError("nu field must be [ny, nx]")
        inp.nx, inp.ny, inp.nu = nx, ny, 0.0
        inp.nu_field = nu_f.data_ptr()
    for k in range(3):
        inp.rho[k] = rs[k].data_ptr()
        inp.ux[k] = xs[k].data_ptr()
        inp.uy[k] = ys[k].data_ptr()
    inp.fx = f_x.data_ptr() if f_x is not None else None
    inp.fy = f_y.data_ptr() if f_y is not None else None
    inp.stream = _stream_handle(stream).value
    nbytes = C.c_size_t()
    L.check(lib.lbm_balance_workspace_bytes(nx, ny, C.byref(nbytes)), "lbm_balance_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    if ws.numel() < nbytes.value:
        raise ValueError("balance workspace too small")
    sizes, sz, out, win, nwin, wterms = _balance_args(nx, ny, sizes, windows)
    if not all_corners:
        out = None
    dm = torch.empty((len(sizes), 3, ny, nx), dtype=torch.float64, device=dev) if maps else None
    tf = torch.empty((L.NTERMS, ny, nx), dtype=torch.float64, device=dev) if term_fields else None
    if edges is None and sample is None and not accumulate:
        L.check(lib.lbm_balance_fields(C.byref(inp), _ptr(ws), nbytes.value, sz, len(sizes), out,
                                       _ptr(dm), win, nwin, wterms, _ptr(tf)), "lbm_balance_fields")
        return _balance_result(sizes, out, dm, nwin, wterms, tf, nx, ny)
    ex = _Extra(len(sizes), edges, accumulate, sample, dev, all_corners)
    L.check(lib.lbm_balance_fields_ex(C.byref(inp), _ptr(ws), ws.numel(), sz, len(sizes), out,
                                      _ptr(dm), win, nwin, wterms, _ptr(tf), C.byref(ex.x)),
            "lbm_balance_fields_ex")
    return ex.into(_balance_result(sizes, out, dm, nwin, wterms, tf, nx, ny))


def sample_configurations(sim, count, every):
    """Advance `sim` and keep `count` configurations `every` (>= 2) steps apart, the way a
    statistically stationary run is sampled into configurations (Sec. 4-5, Figs. 4 and 9):
    a list of (time, device checkpoint); Simulation.load restarts from any of them with
    the moment history the balance needs."""
    if int(every) < 2:
        raise ValueError("every must be >= 2 (the balance needs the two preceding steps)")
    out = []
    for _ in range(int(count)):
        sim.step(int(every))
        out.append((sim.time, sim.save()))
    return out


def configuration_statistics(sim, configs, sizes, edges=None, sample=None, spectrum_shells=None):
    """Balance statistics pooled over configurations (Sec. 4-5: 25 configurations per
    ensemble): `sim` is restarted from each checkpoint of `configs` (as returned by
    sample_configurations) and its balance evaluated with pooling; sample is None,
    (corners, counts) for every configuration, or a callable i -> (corners, counts).
    Returns the pooled balance result (as Simulation.balance) plus 'times' and, with
    spectrum_shells, 'spectra' [nconf, spectrum_shells]."""
    res, spectra, times = None, [], []
    for i, (t, state) in enumerate(configs):
        sim.load(state)
        smp = sample(i) if callable(sample) else sample
        res = sim.balance(sizes, edges=edges, accumulate=i > 0, sample=smp)
        times.append(int(t))
        if spectrum_shells:
            spectra.append(sim.energy_spectrum(spectrum_shells))
    res = dict(res or {})
    res["times"] = times
    if spectrum_shells:
        res["spectra"] = np.stack(spectra)
    return res


def _default_shells(nx, ny):
    return int(np.floor(np.hypot(nx // 2, ny // 2) + 0.5)) + 1


def energy_spectrum(ux, uy, nshells=None, device="cuda", stream=None):
    """Shell-summed kinetic-energy spectrum of given [ny, nx] velocity fields (powers of two)."""
    _require_gpu()
    lib = L.load()
    dev = torch.device(device)
    vx, vy = _dev64(ux, dev), _dev64(uy, dev)
    ny, nx = vx.shape
    ns = int(nshells) if nshells is not None else _default_shells(nx, ny)
    nbytes = C.c_size_t()
    L.check(lib.lbm_spectrum_workspace_bytes(nx, ny, C.byref(nbytes)), "lbm_spectrum_workspace_bytes")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    out = (C.c_double * ns)()
    L.check(lib.lbm_spectrum_fields(nx, ny, _ptr(vx), _ptr(vy), _ptr(ws), nbytes.value, out, ns,
                                    _stream_handle(stream)), "lbm_spectrum_fields")
    return np.frombuffer(out, dtype=np.float64).copy()


def copy_bandwidth(nbytes=1 << 30, iters=20, device="cuda"):
    """GB/s of the library's plain copy kernel (read + write bytes / time)."""
    _require_gpu()
    lib = L.load()
    a = torch.empty(nbytes, dtype=torch.uint8, device=device)
    b = torch.empty_like(a)
    s = _stream_handle()
    L.check(lib.lbm_copy(_ptr(b), _ptr(a), nbytes, s), "lbm_copy")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        L.check(lib.lbm_copy(_ptr(b), _ptr(a), nbytes, s), "lbm_copy")
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / iters
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def set_tuned_tile(nx, ny, dtype="f32", forced=False, layout="rows", tile=(512, 1, 1, 1, 1, 1, 0),
                   scheme="guo"):
    """Record a step-kernel shape for a grid as if the autotuner had chosen it
    (tile = (bx, by, vx, ry, nt, fuse, pf)); forced with scheme "edm" means a
    static force or the damping."""
    lib = L.load()
    edm = scheme == "edm"
    cfg = L.Config(nx=int(nx), ny=int(ny), dtype={"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype],
                   has_force=0, with_balance=0, layout=L.LAYOUTS[layout], tau=0.6,
                   drag_alpha=1e-3 if forced and not edm else 0.0, force_scheme=L.SCHEMES[scheme],
                   damp_f0=1e-5 if forced and edm else 0.0, damp_kmin=1.0, damp_kmax=2.0,
                   stream=None)
    t = L.Tile(*[int(v) for v in tile])
    L.check(lib.lbm_set_tuned_tile(C.byref(cfg), C.byref(t)), "lbm_set_tuned_tile")



class Simulation3D:
    """One periodic D3Q19 or D3Q27 BGK grid on the current GPU (the method of Sec. 1 in
    three dimensions, with the 3D balance of Sec. 2 and its vortex-stretching term).

    rho0, ux0, uy0, uz0: [nz, ny, nx] initial fields; fx, fy, fz: optional static force;
    dtype: "f32" or "f64" population storage; lattice: "d3q19" or "d3q27".
    """

    def __init__(self, rho0, ux0, uy0, uz0, tau, dtype="f32", fx=None, fy=None, fz=None,
                 with_balance=False, device="cuda", stream=None, lattice="d3q19"):
        _require_gpu()
        self._lib = L.load()
        self.device = torch.device(device)
        r, vx, vy, vz = (_dev64(a, self.device) for a in (rho0, ux0, uy0, uz0))
        self.nz, self.ny, self.nx = r.shape
        self.dtype = {"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype]
        self.dtype_name = dtype
        self.tau = float(tau)
        has_force = fx is not None
        self.lattice = lattice
        cfg = L.Config3(nx=self.nx, ny=self.ny, nz=self.nz, dtype=self.dtype, has_force=int(has_force),
                        with_balance=int(with_balance), tau=self.tau, stream=_stream_handle(stream),
                        lattice=L.LATTICES3[lattice])
        self._cfg = cfg
        nbytes = C.c_size_t()
        L.check(self._lib.lbm3_workspace_bytes(C.byref(cfg), C.byref(nbytes)), "lbm3_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        f = [_dev64(a, self.device) if has_force else None for a in (fx, fy, fz)]
        h = C.c_void_p()
        L.check(self._lib.lbm3_init(C.byref(cfg), _ptr(self.workspace), nbytes.value, _ptr(r), _ptr(vx),
                                    _ptr(vy), _ptr(vz), _ptr(f[0]), _ptr(f[1]), _ptr(f[2]), C.byref(h)),
                "lbm3_init")
        self._h = h
        torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()

    def close(self):
        if getattr(self, "_h", None):
            L.check(self._lib.lbm3_destroy(self._h), "lbm3_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def sites(self) -> int:
        return self.nx * self.ny * self.nz

    def step(self, n: int = 1):
        L.check(self._lib.lbm3_step(self._h, int(n)), "lbm3_step")
        return self

    @property
    def time(self) -> int:
        t = C.c_int64()
        L.check(self._lib.lbm3_time(self._h, C.byref(t)), "lbm3_time")
        return t.value

    def set_tile(self, fuse, bx=0, by=0, bz=0):
        """Bulk launch shape: fuse = 1 one step per launch; fuse = 2..4 steps per launch on
        workgroups of bx x by lanes (tiles of (bx - 2 (fuse - 1)) x (by - 2 (fuse - 1))
        columns) over bands of bz planes."""
        t = L.Tile3(int(fuse), int(bx), int(by), int(bz))
        L.check(self._lib.lbm3_set_tile(self._h, C.byref(t)), "lbm3_set_tile")

    def get_tile(self):
        t = L.Tile3()
        L.check(self._lib.lbm3_get_tile(self._h, C.byref(t)), "lbm3_get_tile")
        return (t.fuse, t.bx, t.by, t.bz)

    def autotune(self, trial_launches=5):
        t = L.Tile3()
        L.check(self._lib.lbm3_autotune(self._h, int(trial_launches), C.byref(t)), "lbm3_autotune")
        return (t.fuse, t.bx, t.by, t.bz)

    def moments(self, scalars=True):
        """(rho, ux, uy, uz[, scalars dict]) at the current time, FP64 [nz, ny, nx]."""
        shape = (self.nz, self.ny, self.nx)
        out = [torch.empty(shape, dtype=torch.float64, device=self.device) for _ in range(4)]
        if not scalars:
            L.check(self._lib.lbm3_moments(self._h, *(_ptr(t) for t in out), None), "lbm3_moments")
            return tuple(out)
        sc = (C.c_double * 9)()
        rc = self._lib.lbm3_moments(self._h, *(_ptr(t) for t in out), sc)
        if rc == L.LBM_E_DIVERGED:
            raise L.LBMError(rc, self._lib.lbm_last_error().decode())
        L.check(rc, "lbm3_moments")
        return (*out, dict(zip(L.SCALAR_NAMES3, list(sc))))

    def balance(self, sizes, term_fields=False):
        """Statistics of delta^E, delta^Omega and Ma_V over the L^3 cubes at every corner
        for each L in sizes (needs with_balance and two recorded steps)."""
        sizes = [int(v) for v in sizes]
        sz = (C.c_int32 * max(1, len(sizes)))(*sizes)
        out = (L.BalanceStats * max(1, len(sizes)))()
        tf = torch.empty((L.NTERMS3, self.nz, self.ny, self.nx), dtype=torch.float64,
                         device=self.device) if term_fields else None
        L.check(self._lib.lbm3_subvolume_balance(self._h, sz, len(sizes), out, _ptr(tf)),
                "lbm3_subvolume_balance")
        res = {"stats": [stats_to_dict(out[k]) for k in range(len(sizes))]}
        if tf is not None:
            res["terms"] = {name: tf[k] for k, name in enumerate(L.TERM_NAMES3)}
        return res
