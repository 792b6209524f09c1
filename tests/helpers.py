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


def moment_err(name, got, want, dtype):
    """Parity measure of one moment field.  With FP32 storage the density is compared as
    rho - 1 against max |rho - 1|: its variation (1e-8 .. 1e-3 of rho in these runs) sits
    far below max |rho| = 1, where a comparison of rho itself could not see it.  FP64
    density (whose oracle rho - 1 carries ~1e-16 absolute rounding) and the velocities
    use :func:`rel_err`."""
    if name == "rho" and dtype == "f32":
        g = torch.as_tensor(got).detach().cpu().to(torch.float64)
        w = torch.as_tensor(want).detach().cpu().to(torch.float64)
        return rel_err(g - 1.0, w - 1.0)
    return rel_err(got, want)


def rho_floor32(rho, us, steps, q=9):
    """Absolute error floor of rho - 1 with FP32 population storage.  Each of the q stored
    deviations d_l = f_l - w_l is rounded once per step (relative 2^-24), and nothing
    restores the lost mass, so after t steps rho - 1 at a site is off by up to about
    t q 2^-24 max|d| (linear accumulation; independent roundings give ~sqrt(t) of it).
    max|d| is estimated by the largest equilibrium deviation of the given moments,
    w_l (|rho - 1| + rho (3 |c.u| + 4.5 (c.u)^2 + 1.5 |u|^2)) over the D2Q9 weights (which
    bound the D3Q19 ones; q = 19 there).  us = the velocity components."""
    r = torch.as_tensor(rho, dtype=torch.float64)
    u = torch.sqrt(sum(torch.as_tensor(a, dtype=torch.float64) ** 2 for a in us))
    dr, um, rm = float((r - 1).abs().max()), float(u.max()), float(r.abs().max())
    dmax = max(4 / 9 * (dr + 1.5 * rm * um * um),
               1 / 9 * (dr + rm * (3 * um + 4.5 * um * um + 1.5 * um * um)),
               1 / 36 * (dr + rm * (3 * 1.4142135623730951 * um + 9 * um * um + 1.5 * um * um)))
    return steps * q * 2.0 ** -24 * dmax


def moment_tol(name, want, dtype, steps, base, q=None):
    """Tolerance of :func:`moment_err` for one field: `base` (1e-12 FP64, 1e-5 FP32), except
    FP32 density, whose rho - 1 cannot be more exact than :func:`rho_floor32` allows: there
    max(base, floor / max|rho - 1|).  want = (rho, ux, uy[, uz]) of the oracle; q the
    populations per site (9 in 2D, 19 in 3D unless given)."""
    if name != "rho" or dtype != "f32":
        return base
    dr = float((torch.as_tensor(want[0], dtype=torch.float64) - 1).abs().max())
    floor = rho_floor32(want[0], want[1:], steps, q or (9 if len(want) == 3 else 19))
    return max(base, floor / dr) if dr > 0 else float("inf")


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


def _perturb(a, rel, rng):
    a = np.asarray(a, dtype=np.float64)
    return a * (1.0 + rel * rng.standard_normal(a.shape))


def balance_sensitivity(lv, nu, sizes, fx=None, fy=None, rel=2.2e-16, trials=2, seed=0):
    """Conditioning of the balance on these inputs, measured with the oracle.

    Every input value is multiplied by (1 + rel * N(0, 1)) and the oracle rerun;
    returns (fields, stats, kappa_terms, kappa_stats) where kappa_* is the
    largest observed change relative to the unperturbed value (terms: relative
    to the field's max |value|).  Rounding inside any correct implementation
    moves the results by about this much, so parity tolerances scale with it.
    """
    flds = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], fx, fy, nu)
    stats = ref.subvolume_balance(flds, sizes) if sizes else []
    rng = np.random.default_rng(seed)
    kt = {k: 0.0 for k in ref.TERM_NAMES}
    ks = [{q: {s: 0.0 for s in ("mean", "std", "min", "max")} for q in ("dE", "dZ", "Ma")}
          for _ in stats]
    for _ in range(trials):
        p = {k: [_perturb(a, rel, rng) for a in lv[k]] for k in ("rho", "ux", "uy")}
        pf = (_perturb(fx, rel, rng), _perturb(fy, rel, rng)) if fx is not None else (None, None)
        f2 = ref.balance_fields(p["rho"], p["ux"], p["uy"], pf[0], pf[1], nu)
        for k in ref.TERM_NAMES:
            den = float(flds[k].abs().max()) or 1.0
            kt[k] = max(kt[k], float((f2[k] - flds[k]).abs().max()) / den)
        if stats:
            s2 = ref.subvolume_balance(f2, sizes)
            for j, (a, b) in enumerate(zip(stats, s2)):
                for q in ("dE", "dZ", "Ma"):
                    for s in ("mean", "std", "min", "max"):
                        va, vb = a[q][s], b[q][s]
                        if np.isfinite(va) and va != 0:
                            ks[j][q][s] = max(ks[j][q][s], abs(vb - va) / abs(va))
    return flds, stats, kt, ks
