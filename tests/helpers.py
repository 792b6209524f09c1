"""Shared test helpers: error measures and oracle runs on periodic patches."""
import numpy as np
import torch

from oracle import ref


def rel_err(got, want):
    """max |got - want| / max |want| (per field; robust to zero crossings)."""
    g = torch.as_tensor(got).detach().cpu().to(torch.float64)
    w = torch.as_tensor(want).detach().cpu().to(torch.float64)
    den = float(w.abs().max())
    return float((g - w).abs().max()) / (den if den > 0 else 1.0)


def wrap_patch(a, y0, x0, size):
    """size x size block of a periodic [ny, nx] array starting at (y0, x0)."""
    a = np.asarray(a)
    ny, nx = a.shape
    ys = (np.arange(size) + y0) % ny
    xs = (np.arange(size) + x0) % nx
    return a[np.ix_(ys, xs)]


def oracle_patch_moments(fields, tau, steps, y0, x0, core, fx=None, fy=None, alpha=0.0):
    """Oracle moments after `steps` steps on the core x core block at (y0, x0).

    The oracle runs on a periodic patch with a margin of steps + 1 cells: the
    patch's artificial wrap travels at most one cell per step, so the core is
    exactly what the full periodic grid computes.
    """
    m = steps + 1
    size = core + 2 * m
    pr = [wrap_patch(a, y0 - m, x0 - m, size) for a in fields]
    f = ref.init_populations(*pr)
    kw = {}
    if fx is not None:
        kw = dict(fx_ext=ref.t64(wrap_patch(fx, y0 - m, x0 - m, size)),
                  fy_ext=ref.t64(wrap_patch(fy, y0 - m, x0 - m, size)), alpha=alpha)
    elif alpha:
        kw = dict(alpha=alpha)
    f = ref.run(f, steps, tau, **kw)
    r, vx, vy = ref.moments(f, kw.get("fx_ext"), kw.get("fy_ext"), kw.get("alpha", 0.0))
    sl = (slice(m, m + core), slice(m, m + core))
    return r[sl], vx[sl], vy[sl]


def gpu_patch(t, y0, x0, core):
    return torch.as_tensor(wrap_patch(t.detach().cpu().numpy(), y0, x0, core))
