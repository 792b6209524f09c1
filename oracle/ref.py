"""FP64 CPU oracle for the D2Q9 LBGK step and the sub-volume balance diagnostic.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the library never does.  It is
plain PyTorch on the CPU in float64, written to be read against the paper
(Tauzin et al., "A numerical tool for the study of the hydrodynamic recovery
of the Lattice Boltzmann Method", Computers & Fluids 172 (2018)), with no
blocking, fusion or reordering beyond the formulas themselves.

Arrays are indexed [y, x]; populations are [9, ny, nx].  Lattice units
(dx = dt = 1).

Parts and where they come from
------------------------------
* D2Q9 lattice, equilibrium (Sec. 1, Eq. 2), moments rho = sum f,
  rho u = sum f c (Sec. 1, text after Eq. 2), LBGK update (Sec. 1, Eq. 1),
  nu = c_s^2 (tau - 1/2) (Sec. 1, Eq. 5).
* Forcing term F_l: Guo's scheme (Guo, Zheng & Shi, Phys. Rev. E 65, 046308,
  2002) with the half-force velocity u = (sum f c + F/2) / rho, and a linear
  drag -alpha rho u folded into the force implicitly.  (The paper itself uses
  the exact-difference method of Kupershtokh; see the readings list.)
* The paper's own forced set-up (Sec. 3, Eqs. 14-16): the exact-difference
  forcing (relax to f^eq(rho, j/rho), then add f^eq(rho, j/rho + F/rho) -
  f^eq(rho, j/rho)), the spectral damping of the wavevectors 1 <= |k| <= 2
  computed from the bare velocity j/rho with unnormalised transforms, and the
  physical velocity (j + F/2)/rho of that scheme for the balance.
* Time derivative: three-level backward formula (Sec. 3, Eq. 17).
* Space derivatives: 8th-order centred differences (Sec. 3, Eq. 18), periodic.
* Energy balance terms (Sec. 2, Eqs. 8 and 10), enstrophy balance terms
  (Sec. 2, Eqs. 9 and 11, 2D: the stretching term is identically zero),
  balancing errors (Sec. 2, Eqs. 12-13), sub-volume Mach number (Sec. 4,
  Eq. 20), sub-volume means over L x L boxes (Sec. 3, Fig. 3 and Table 1)
  with periodic wrap, statistics mu_l, sigma_l (Sec. 3).
* Entropic LBM (Sec. 1, Eq. 6 and tau_eff = 2 tau0 / alpha): the closed-form
  minimiser of H at fixed rho, rho u on D2Q9, alpha as the root of the entropy
  equality H(f + alpha (f^eq - f)) = H(f) by bisection, nu_eff = c_s^2 (tau_eff - 1/2);
  the balance takes the viscosity as a field.
* Statistics as presented (Sec. 3, Table 1; Figs. 5-13): histograms of
  delta^E, delta^Omega, Ma_V on given bin edges, the errors of windows at given
  random corners, pooling over configurations, and the shell-summed energy
  spectrum from FFTs.
* Adjoint (gradient of a sub-volume enstrophy-balance residual loss with
  respect to the initial velocity and tau): torch.autograd through the very
  same forward functions.  Pinned by central finite differences.

Readings of silent or ambiguous points (each is also listed in the design
notes): textbook D2Q9 with c_s^2 = 1/3; initial populations f = f^eq(rho0,
u0); moments at time t are taken from the pre-collision populations at t;
products inside a divergence are formed pointwise and then differenced; the
enstrophy equation's repeated flux term (Eq. 9, second line) is read as the
compressibility term of Eq. 11; the denominator of delta is the largest
|RHS term| only, and a zero denominator gives NaN, which is counted and left
out of mean and std; std is the population std (ddof 0); a box of side L = N
is a single window, smaller boxes take every corner of the periodic grid.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64

# ---------------------------------------------------------------------------
# D2Q9 lattice (Eq. 2 with the textbook D2Q9 set named in Sec. 3)
# ---------------------------------------------------------------------------
#: discrete velocities c_l = (c_x, c_y); order: rest, 4 axis, 4 diagonal
C = ((0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1))
#: weights t_l of Eq. 2
W = (4.0 / 9.0,) + (1.0 / 9.0,) * 4 + (1.0 / 36.0,) * 4
#: squared lattice speed of sound
CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)


def t64(a):
    """Any array-like -> float64 CPU tensor (no copy of an existing one)."""
    return torch.as_tensor(a, dtype=DT)


def viscosity(tau):
    """Eq. 5: nu = c_s^2 (tau - 1/2) dt, dt = 1."""
    return CS2 * (tau - 0.5)


# ---------------------------------------------------------------------------
# Equilibrium, moments, forcing, collision, streaming (Eqs. 1-2)
# ---------------------------------------------------------------------------
def equilibrium(rho, ux, uy):
    """Eq. 2: f^eq_l = t_l rho [1 + c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2)]."""
    usq = ux * ux + uy * uy
    out = []
    for (cx, cy), w in zip(C, W):
        cu = cx * ux + cy * uy
        out.append(w * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2)))
    return torch.stack(out)


def density(f):
    """rho = sum_l f_l."""
    return f.sum(0)


def momentum(f):
    """j = sum_l f_l c_l (components x, y)."""
    jx = sum(cx * f[l] for l, (cx, _) in enumerate(C) if cx != 0)
    jy = sum(cy * f[l] for l, (_, cy) in enumerate(C) if cy != 0)
    return jx, jy


def macroscopic(f, fx_ext=None, fy_ext=None, alpha=0.0):
    """Density, velocity and total body force at a site.

    Without force and drag: u = j / rho (Sec. 1).  With an external force
    F_ext and linear drag -alpha rho u the velocity is the half-force one,
    rho u = j + F/2 with F = F_ext - alpha rho u, solved in closed form:
    u = (j + F_ext/2) / (rho (1 + alpha/2)).
    Returns rho, ux, uy, Fx, Fy.
    """
    rho = density(f)
    jx, jy = momentum(f)
    zero = torch.zeros_like(rho)
    fx_ext = zero if fx_ext is None else fx_ext
    fy_ext = zero if fy_ext is None else fy_ext
    denom = rho * (1.0 + 0.5 * alpha)
    ux = (jx + 0.5 * fx_ext) / denom
    uy = (jy + 0.5 * fy_ext) / denom
    fx = fx_ext - alpha * rho * ux
    fy = fy_ext - alpha * rho * uy
    return rho, ux, uy, fx, fy


def guo_source(ux, uy, fx, fy, tau):
    """Guo forcing term F_l = (1 - 1/(2 tau)) t_l [(c_l - u)/c_s^2 + (c_l.u) c_l / c_s^4] . F."""
    pref = 1.0 - 0.5 / tau
    out = []
    for (cx, cy), w in zip(C, W):
        cu = cx * ux + cy * uy
        gx = (cx - ux) / CS2 + cu * cx / (CS2 * CS2)
        gy = (cy - uy) / CS2 + cu * cy / (CS2 * CS2)
        out.append(pref * w * (gx * fx + gy * fy))
    return torch.stack(out)


def collide(f, tau, fx_ext=None, fy_ext=None, alpha=0.0):
    """Right-hand side of Eq. 1 added to f: f* = f - (f - f^eq)/tau + F_l (per site)."""
    rho, ux, uy, fx, fy = macroscopic(f, fx_ext, fy_ext, alpha)
    post = f - (f - equilibrium(rho, ux, uy)) / tau
    if fx_ext is not None or fy_ext is not None or alpha != 0.0:
        post = post + guo_source(ux, uy, fx, fy, tau)
    return post


def stream(fpost):
    """Left-hand side of Eq. 1: f_l(x + c_l, t + 1) = f*_l(x, t), periodic."""
    return torch.stack([torch.roll(fpost[l], shifts=(cy, cx), dims=(0, 1))
                        for l, (cx, cy) in enumerate(C)])


def step(f, tau, fx_ext=None, fy_ext=None, alpha=0.0):
    """One LBGK time step (Eq. 1): collide at every site, then stream."""
    return stream(collide(f, tau, fx_ext, fy_ext, alpha))


def init_populations(rho0, ux0, uy0):
    """Initial populations: the equilibrium of the given fields (Eq. 2)."""
    return equilibrium(t64(rho0), t64(ux0), t64(uy0))


def run(f, nsteps, tau, fx_ext=None, fy_ext=None, alpha=0.0):
    """nsteps applications of :func:`step`."""
    for _ in range(nsteps):
        f = step(f, tau, fx_ext, fy_ext, alpha)
    return f


def moments(f, fx_ext=None, fy_ext=None, alpha=0.0):
    """(rho, ux, uy) at the time of the pre-collision populations f."""
    rho, ux, uy, _, _ = macroscopic(f, fx_ext, fy_ext, alpha)
    return rho, ux, uy


def global_enstrophy(ux, uy):
    """Domain total of the enstrophy density, 1/2 sum omega^2, omega by Eq. 18."""
    w = vorticity(t64(ux), t64(uy))
    return float(0.5 * (w * w).sum())


# ---------------------------------------------------------------------------
# Discrete derivatives (Eqs. 17-18)
# ---------------------------------------------------------------------------
def _shift(a, m, dim):
    """a at index i + m along dim (periodic)."""
    return torch.roll(a, shifts=-m, dims=dim)


def _fd8(a, dim):
    p = lambda m: _shift(a, m, dim)  # noqa: E731
    return (-p(4) / 56.0 + 4.0 * p(3) / 21.0 - p(2) + 4.0 * p(1)
            - 4.0 * p(-1) + p(-2) - 4.0 * p(-3) / 21.0 + p(-4) / 56.0) / 5.0


def ddx(a):
    """Eq. 18, x direction (array axis 1), periodic, dx = 1."""
    return _fd8(a, 1)


def ddy(a):
    """Eq. 18, y direction (array axis 0), periodic, dy = 1."""
    return _fd8(a, 0)


def bdf2(a_n, a_nm1, a_nm2):
    """Eq. 17: dA/dt at level n ~ (3 A^n - 4 A^{n-1} + A^{n-2}) / (2 dt), dt = 1."""
    return (3.0 * a_n - 4.0 * a_nm1 + a_nm2) / 2.0


# ---------------------------------------------------------------------------
# Balance terms (Eqs. 8-11)
# ---------------------------------------------------------------------------
#: order of the 13 integrand fields
TERM_NAMES = ("lhs_E", "e1", "e2", "e3", "e4", "e5",
              "lhs_Z", "z1", "z2", "z3", "z4", "z5", "usq")


def vorticity(ux, uy):
    """omega = d_x u_y - d_y u_x (2D curl)."""
    return ddx(uy) - ddy(ux)


def balance_fields(rho, ux, uy, fx, fy, nu, p=None):
    """Pointwise integrands of the sub-volume balances at time level n.

    rho, ux, uy: sequences of three fields at levels (n-2, n-1, n).
    fx, fy: total body force at level n.  nu: kinematic viscosity, a number or a
    field at level n (the effective viscosity of the entropic scheme).
    p: pressure at level n; default the LBGK equation of state p = c_s^2 rho.

    Returns a dict with the 13 fields of TERM_NAMES:
    lhs_E = d_t E (Eq. 17) with E = rho |u|^2 / 2, and e1..e5 = the five
    right-hand-side integrands of Eq. 10 in its order (flux, pressure work,
    force work, dissipation, viscous diffusion); lhs_Z = d_t Omega with
    Omega = omega^2 / 2, and z1..z5 = the right-hand-side integrands of Eq. 11
    in its order (flux, compressibility, force curl, dissipation through H,
    diffusion through H; the 2D stretching term is zero); usq = |u|^2 at n.
    """
    r, vx, vy = t64(rho[2]), t64(ux[2]), t64(uy[2])
    fx = torch.zeros_like(r) if fx is None else t64(fx)
    fy = torch.zeros_like(r) if fy is None else t64(fy)
    p = CS2 * r if p is None else t64(p)

    dxux, dyux = ddx(vx), ddy(vx)
    dxuy, dyuy = ddx(vy), ddy(vy)
    energy = [0.5 * t64(rho[k]) * (t64(ux[k]) ** 2 + t64(uy[k]) ** 2) for k in range(3)]
    omega_lv = [vorticity(t64(ux[k]), t64(uy[k])) for k in range(3)]
    enst = [0.5 * w * w for w in omega_lv]
    e_n, om, z_n = energy[2], omega_lv[2], enst[2]

    # viscous stress sigma_ij = nu rho (d_j u_i + d_i u_j)
    sxx = 2.0 * nu * r * dxux
    syy = 2.0 * nu * r * dyuy
    sxy = nu * r * (dxuy + dyux)
    # H_i = (1/rho) d_j sigma_ij
    hx = (ddx(sxx) + ddy(sxy)) / r
    hy = (ddx(sxy) + ddy(syy)) / r

    out = {}
    out["lhs_E"] = bdf2(energy[2], energy[1], energy[0])
    out["e1"] = -(ddx(e_n * vx) + ddy(e_n * vy))
    out["e2"] = -(vx * ddx(p) + vy * ddy(p))
    out["e3"] = vx * fx + vy * fy
    out["e4"] = -(sxx * dxux + sxy * dyux + sxy * dxuy + syy * dyuy)
    out["e5"] = ddx(vx * sxx + vy * sxy) + ddy(vx * sxy + vy * syy)
    out["lhs_Z"] = bdf2(enst[2], enst[1], enst[0])
    out["z1"] = -(ddx(z_n * vx) + ddy(z_n * vy))
    out["z2"] = -z_n * (dxux + dyuy)
    out["z3"] = om * (ddx(fy / r) - ddy(fx / r))
    out["z4"] = hx * ddy(om) - hy * ddx(om)
    out["z5"] = ddx(om * hy) - ddy(om * hx)
    out["usq"] = vx * vx + vy * vy
    return out


# ---------------------------------------------------------------------------
# Sub-volume means and balancing errors (Eqs. 10-13, 20; Table 1)
# ---------------------------------------------------------------------------
def box_mean_map(g, L):
    """Mean of g over the L x L box with lower corner (y0, x0), for every corner.

    Periodic wrap; result[y0, x0] = (1/L^2) sum_{j<L, i<L} g[(y0+j)%ny, (x0+i)%nx].
    Uses running sums (cumsum) over the periodically doubled array.
    """
    g = t64(g)
    ny, nx = g.shape

    def window_sum(a, n, dim):
        ext = torch.cat([a, a], dim=dim)
        cs = torch.cumsum(ext, dim=dim)
        zero = torch.zeros_like(a.narrow(dim, 0, 1))
        cs = torch.cat([zero, cs], dim=dim)
        return cs.narrow(dim, L, n) - cs.narrow(dim, 0, n)

    s = window_sum(g, nx, 1)
    s = window_sum(s, ny, 0)
    return s / (L * L)


def box_mean_brute(g, L, y0, x0):
    """Mean over one L x L periodic box by a plain double loop (small cases only)."""
    g = t64(g)
    ny, nx = g.shape
    acc = 0.0
    for j in range(L):
        for i in range(L):
            acc += float(g[(y0 + j) % ny, (x0 + i) % nx])
    return acc / (L * L)


def window_means(fields, L):
    """Dict name -> [ny, nx] map of box means of every balance field."""
    return {k: box_mean_map(v, L) for k, v in fields.items()}


def balancing_errors(means):
    """Eqs. 12-13 and 20 from box means (any shape): returns (delta_E, delta_Z, Ma)."""
    e = [means[k] for k in ("e1", "e2", "e3", "e4", "e5")]
    z = [means[k] for k in ("z1", "z2", "z3", "z4", "z5")]
    z.append(torch.zeros_like(z[0]))   # z6: vortex stretching, zero in 2D
    rhs_e = sum(e)
    rhs_z = sum(z)
    den_e = torch.stack([t.abs() for t in e]).max(0).values
    den_z = torch.stack([t.abs() for t in z]).max(0).values
    nan = torch.full_like(rhs_e, float("nan"))
    d_e = torch.where(den_e > 0, (rhs_e - means["lhs_E"]).abs() / torch.where(den_e > 0, den_e, 1.0), nan)
    d_z = torch.where(den_z > 0, (rhs_z - means["lhs_Z"]).abs() / torch.where(den_z > 0, den_z, 1.0), nan)
    ma = means["usq"].sqrt() / CS
    return d_e, d_z, ma


def _stats(x):
    x = x.reshape(-1)
    finite = torch.isfinite(x)
    v = x[finite]
    n = int(v.numel())
    if n == 0:
        nanv = float("nan")
        return {"count": 0, "n_nan": int(x.numel()), "mean": nanv, "std": nanv, "min": nanv, "max": nanv}
    return {"count": n, "n_nan": int(x.numel() - n), "mean": float(v.mean()),
            "std": float(v.std(unbiased=False)), "min": float(v.min()), "max": float(v.max())}


def subvolume_balance(fields, sizes):
    """Statistics of delta^E, delta^Omega and Ma over all L x L boxes, per L.

    Every corner of the periodic grid is a window for L < N; L = N is a single
    window (the whole domain).  Returns a list of dicts, one per L, with keys
    L, dE, dZ, Ma (each a stats dict: count, n_nan, mean, std, min, max) and
    the full maps under 'maps' (delta_E, delta_Z, Ma).
    """
    ny, nx = next(iter(fields.values())).shape
    out = []
    for L in sizes:
        if not (1 <= L <= min(nx, ny)):
            raise ValueError(f"box size {L} outside [1, {min(nx, ny)}]")
        means = window_means(fields, L)
        if L == nx and L == ny:
            means = {k: v[:1, :1] for k, v in means.items()}
        d_e, d_z, ma = balancing_errors(means)
        out.append({"L": L, "dE": _stats(d_e), "dZ": _stats(d_z), "Ma": _stats(ma),
                    "maps": (d_e, d_z, ma)})
    return out


def window_terms(fields, windows):
    """Box means of the 13 fields at explicit windows (x0, y0, L): [nwin, 13]."""
    rows = []
    for (x0, y0, L) in windows:
        rows.append([float(box_mean_map(fields[k], L)[y0, x0]) for k in TERM_NAMES])
    return torch.tensor(rows, dtype=DT)


# ---------------------------------------------------------------------------
# Whole diagnostic from a run, and the differentiable loss
# ---------------------------------------------------------------------------
def run_with_history(f, nsteps, tau, fx_ext=None, fy_ext=None, alpha=0.0):
    """Advance nsteps (>= 2) and return (f_final, [m(n-2), m(n-1), m(n)]) with m = (rho, ux, uy)."""
    if nsteps < 2:
        raise ValueError("need at least two steps of history")
    hist = []
    for s in range(nsteps):
        if s >= nsteps - 2:
            hist.append(moments(f, fx_ext, fy_ext, alpha))
        f = step(f, tau, fx_ext, fy_ext, alpha)
    hist.append(moments(f, fx_ext, fy_ext, alpha))
    return f, hist


def fields_from_history(hist, tau, fx_ext=None, fy_ext=None, alpha=0.0, p=None):
    """Balance fields at the last level of a (rho, ux, uy) history of three levels."""
    rho = [h[0] for h in hist]
    ux = [h[1] for h in hist]
    uy = [h[2] for h in hist]
    r, vx, vy = rho[2], ux[2], uy[2]
    zero = torch.zeros_like(r)
    fxe = zero if fx_ext is None else t64(fx_ext)
    fye = zero if fy_ext is None else t64(fy_ext)
    fx = fxe - alpha * r * vx
    fy = fye - alpha * r * vy
    return balance_fields(rho, ux, uy, fx, fy, viscosity(tau), p=p)


def enstrophy_residual_loss(ux0, uy0, tau, nsteps, L, rho0=None):
    """Differentiable loss J = mean over all L x L windows of (RHS^Omega_V - LHS^Omega_V)^2.

    Unforced run of nsteps from f = f^eq(rho0, u0); the enstrophy balance at
    the final step (Eq. 11) uses levels nsteps-2, nsteps-1, nsteps.  ux0, uy0
    and tau may be tensors requiring grad.  A box of side L = N is one window.
    """
    ux0 = t64(ux0)
    uy0 = t64(uy0)
    rho0 = torch.ones_like(ux0) if rho0 is None else t64(rho0)
    tau_t = tau if torch.is_tensor(tau) else torch.tensor(float(tau), dtype=DT)
    f = equilibrium(rho0, ux0, uy0)
    _, hist = run_with_history(f, nsteps, tau_t)
    flds = fields_from_history(hist, tau_t)
    resid = flds["z1"] + flds["z2"] + flds["z3"] + flds["z4"] + flds["z5"] - flds["lhs_Z"]
    ny, nx = resid.shape
    box = box_mean_map(resid, L)
    if L == nx and L == ny:
        box = box[:1, :1]
    return (box * box).mean()


def enstrophy_residual_grad(ux0, uy0, tau, nsteps, L):
    """(J, dJ/dux0, dJ/duy0, dJ/dtau) by reverse-mode autodiff of the FP64 forward."""
    ux = t64(ux0).clone().requires_grad_(True)
    uy = t64(uy0).clone().requires_grad_(True)
    tt = torch.tensor(float(tau), dtype=DT, requires_grad=True)
    j = enstrophy_residual_loss(ux, uy, tt, nsteps, L)
    gx, gy, gt = torch.autograd.grad(j, (ux, uy, tt))
    return float(j.detach()), gx.detach(), gy.detach(), float(gt)


# ---------------------------------------------------------------------------
# The paper's own forced set-up (Sec. 3, Eqs. 14-16): exact-difference-method
# forcing and the spectral damping of the large scales
# ---------------------------------------------------------------------------
def wavevectors(kmin, kmax):
    """Integer wavevectors k with kmin <= |k| <= kmax."""
    r = int(math.ceil(kmax))
    return [(kx, ky) for ky in range(-r, r + 1) for kx in range(-r, r + 1)
            if kmin * kmin <= kx * kx + ky * ky <= kmax * kmax]


def shell_projection(a, kmin=1.0, kmax=2.0):
    """The part of the periodic field a [ny, nx] on the wavevectors
    kmin <= |k| <= kmax: ifft2(fft2(a) masked)."""
    ny, nx = a.shape
    mask = torch.zeros((ny, nx), dtype=DT)
    for kx, ky in wavevectors(kmin, kmax):
        mask[ky % ny, kx % nx] = 1.0
    return torch.real(torch.fft.ifft2(torch.fft.fft2(a) * mask))


def damping_force(ux, uy, amp, kmin=1.0, kmax=2.0):
    """Eq. 16, F^R = -F0^R sum_{kmin<=|k|<=kmax} u^(k) e^{i 2 pi k.x / N}, read with
    the imaginary unit restored in the exponent, u^ the Fourier-series
    coefficients (1/N^2) sum_x u(x) e^{-i 2 pi k.x / N} and the sum over +-k real:
    F^R = -F0^R P[u] with P the projection on those wavevectors.  amp = F0^R,
    a damping rate per step (1e-5 in the paper)."""
    return -amp * shell_projection(ux, kmin, kmax), -amp * shell_projection(uy, kmin, kmax)


def edm_total_force(f, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    """rho, bare velocity j/rho and the total force F = F_ext + F^R(j/rho) at a time."""
    rho = density(f)
    jx, jy = momentum(f)
    ux, uy = jx / rho, jy / rho
    fx = torch.zeros_like(rho) if fx_ext is None else fx_ext.clone()
    fy = torch.zeros_like(rho) if fy_ext is None else fy_ext.clone()
    if amp != 0.0:
        rx, ry = damping_force(ux, uy, amp, kmin, kmax)
        fx, fy = fx + rx, fy + ry
    return rho, ux, uy, fx, fy


def edm_collide(f, tau, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    """Kupershtokh's exact-difference method: after the BGK relaxation towards
    f^eq(rho, u), u = j/rho, add f^eq(rho, u + du) - f^eq(rho, u), du = F dt/rho."""
    rho, ux, uy, fx, fy = edm_total_force(f, fx_ext, fy_ext, amp, kmin, kmax)
    feq = equilibrium(rho, ux, uy)
    shifted = equilibrium(rho, ux + fx / rho, uy + fy / rho)
    return f - (f - feq) / tau + (shifted - feq)


def edm_step(f, tau, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    """One time step with the exact-difference forcing: collide, then stream."""
    return stream(edm_collide(f, tau, fx_ext, fy_ext, amp, kmin, kmax))


def edm_run(f, nsteps, tau, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    for _ in range(nsteps):
        f = edm_step(f, tau, fx_ext, fy_ext, amp, kmin, kmax)
    return f


def edm_moments(f, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    """(rho, ux, uy, Fx, Fy) at the time of f: the physical velocity of the
    exact-difference scheme, u = (j + F/2)/rho, and the total force."""
    rho, ux, uy, fx, fy = edm_total_force(f, fx_ext, fy_ext, amp, kmin, kmax)
    return rho, ux + 0.5 * fx / rho, uy + 0.5 * fy / rho, fx, fy


def edm_run_with_history(f, nsteps, tau, fx_ext=None, fy_ext=None, amp=0.0, kmin=1.0, kmax=2.0):
    """Populations after nsteps and the moments (rho, ux, uy) at t = nsteps-2,
    nsteps-1, nsteps, plus the total force at nsteps (for the balance)."""
    hist = []
    for t in range(nsteps + 1):
        if t >= nsteps - 2:
            hist.append(edm_moments(f, fx_ext, fy_ext, amp, kmin, kmax))
        if t < nsteps:
            f = edm_step(f, tau, fx_ext, fy_ext, amp, kmin, kmax)
    return f, hist


# ---------------------------------------------------------------------------
# Entropic LBM (Sec. 1: the H-functional of Eq. 6 and the effective relaxation
# time tau_eff = 2 tau0 / alpha towards the minimiser of H)
# ---------------------------------------------------------------------------
def h_function(f):
    """Eq. 6 per site: H(f) = sum_l f_l log(f_l / t_l)."""
    w = torch.tensor(W, dtype=DT).reshape(9, 1, 1)
    return (f * torch.log(f / w)).sum(0)


def entropic_equilibrium(rho, ux, uy):
    """The minimiser of H at fixed rho and rho u on D2Q9, in closed form:
    f_l = t_l rho prod_a (2 - s_a) ((2 u_a + s_a) / (1 - u_a))^{c_la},
    s_a = sqrt(1 + 3 u_a^2), a = x, y."""
    rho, ux, uy = t64(rho), t64(ux), t64(uy)
    sx = torch.sqrt(1.0 + 3.0 * ux * ux)
    sy = torch.sqrt(1.0 + 3.0 * uy * uy)
    zx = (2.0 * ux + sx) / (1.0 - ux)
    zy = (2.0 * uy + sy) / (1.0 - uy)
    base = rho * (2.0 - sx) * (2.0 - sy)
    return torch.stack([W[l] * base * zx ** C[l][0] * zy ** C[l][1] for l in range(9)])


def entropic_gain(f, delta, a):
    """H(f + a delta) - H(f) per site for delta = f^eq - f, f^eq the minimiser of H with
    the moments of f.  With t = a delta / f and phi(t) = (1 + t) log1p(t) - t,
    H(f + a delta) - H(f) = sum_l f_l phi(t_l) + a sum_l delta_l (1 + log(f_l / t_l));
    delta conserves mass and momentum and log(f^eq_l / t_l) is affine in c_l, so the
    second sum equals a sum_l delta_l log(f_l / f^eq_l) = -a sum_l delta_l log1p(delta_l / f_l):
    the same quantity with every first-order term cancelled analytically."""
    t = a * delta / f
    phi = (1.0 + t) * torch.log1p(t) - t
    return (f * phi).sum(0) - a * (delta * torch.log1p(delta / f)).sum(0)


#: below this max_l |feq_l - f_l| / f_l the populations count as equilibrium (alpha = 2)
ENTROPIC_NEAR_EQ = 1e-8


def entropic_alpha(f, feq, iters=200):
    """alpha of the entropic step per site: the root alpha > 1 of
    H(f + alpha (feq - f)) = H(f), by bisection on [1, alpha_max) with
    alpha_max the largest step keeping every population positive; alpha = 2 at
    equilibrium (max |feq - f| / f below ENTROPIC_NEAR_EQ), alpha = the top of the
    bracket when H is still below H(f) there (no root)."""
    delta = feq - f
    near = (delta.abs() / f).amax(0) < ENTROPIC_NEAR_EQ
    ratio = torch.where(delta < 0, -f / torch.where(delta < 0, delta, -torch.ones_like(delta)),
                        torch.full_like(f, float("inf")))
    amax = ratio.amin(0)
    hi = torch.where(torch.isfinite(amax), amax * (1.0 - 1e-12), torch.full_like(amax, 1e6))
    lo = torch.ones_like(hi)
    ghi = entropic_gain(f, delta, hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        below = entropic_gain(f, delta, mid) < 0
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    alpha = 0.5 * (lo + hi)
    alpha = torch.where(ghi < 0, hi, alpha)
    return torch.where(near, torch.full_like(alpha, 2.0), alpha)


def entropic_collide(f, tau0):
    """f* = f + alpha beta (f^eq - f), beta = 1 / (2 tau0): the relaxation time is
    tau_eff = 2 tau0 / alpha (tau0 for alpha = 2, the LBGK step); returns (f*, alpha)."""
    rho = density(f)
    jx, jy = momentum(f)
    feq = entropic_equilibrium(rho, jx / rho, jy / rho)
    alpha = entropic_alpha(f, feq)
    return f + alpha * (0.5 / tau0) * (feq - f), alpha


def entropic_step(f, tau0):
    return stream(entropic_collide(f, tau0)[0])


def entropic_run(f, nsteps, tau0):
    for _ in range(nsteps):
        f = entropic_step(f, tau0)
    return f


def effective_viscosity(alpha, tau0):
    """nu_eff = c_s^2 (tau_eff - 1/2), tau_eff = 2 tau0 / alpha (Eq. 5 with tau_eff)."""
    return CS2 * (2.0 * tau0 / t64(alpha) - 0.5)


def entropic_run_with_history(f, nsteps, tau0):
    """Populations after nsteps, the moments (rho, u) at nsteps-2, nsteps-1, nsteps and
    the effective viscosity field at nsteps (from the alpha of the populations then)."""
    hist = []
    for t in range(nsteps + 1):
        if t >= nsteps - 2:
            hist.append(moments(f))
        if t < nsteps:
            f = entropic_step(f, tau0)
    _, alpha = entropic_collide(f, tau0)
    return f, hist, effective_viscosity(alpha, tau0)


# ---------------------------------------------------------------------------
# Statistics as the paper presents them (Sec. 3, Table 1; Figs. 6-13)
# ---------------------------------------------------------------------------
def histogram(values, edges):
    """Counts of the finite values per bin: bin 0 below edges[0], bin i in
    [edges[i-1], edges[i]), bin n at or above edges[-1] (n = len(edges))."""
    v = t64(values).reshape(-1)
    v = v[torch.isfinite(v)]
    e = t64(edges)
    idx = torch.bucketize(v, e, right=True)  # number of edges <= v
    return torch.bincount(idx, minlength=len(e) + 1)


def sampled_errors(fields, L, corners):
    """delta^E, delta^Omega, Ma_V (Eqs. 12-13, 20) of the L x L windows whose lower
    corners (x0, y0) are given, taken modulo the grid (the randomly placed
    sub-volumes of Sec. 3, Fig. 3)."""
    ny, nx = next(iter(fields.values())).shape
    c = torch.as_tensor(corners, dtype=torch.int64).reshape(-1, 2)
    xs = torch.remainder(c[:, 0], nx)
    ys = torch.remainder(c[:, 1], ny)
    means = {k: v[ys, xs] for k, v in window_means(fields, L).items()}
    return balancing_errors(means)


def pooled_stats(value_sets):
    """Statistics (as _stats) of the union of several sets of values: the pooling
    over configurations of Sec. 4-5 (25 configurations per ensemble)."""
    return _stats(torch.cat([t64(v).reshape(-1) for v in value_sets]))


def shell_index(kx, ky):
    """Shell s of integer wavevectors: (2s - 1)^2 <= 4 |k|^2 < (2s + 1)^2 (shell 0:
    4 |k|^2 < 1), i.e. |k| rounded half up, decided in integer arithmetic."""
    k2 = 4 * (kx * kx + ky * ky)
    s = torch.floor(torch.sqrt(k2.to(DT)) / 2.0 + 0.5).to(torch.int64)
    s = torch.where((s > 0) & ((2 * s - 1) ** 2 > k2), s - 1, s)
    s = torch.where((2 * s + 1) ** 2 <= k2, s + 1, s)
    return s


def energy_spectrum(ux, uy, nshells):
    """Shell-summed kinetic energy spectrum (Figs. 5 and 10): E(s) = 1/2 sum over the
    wavevectors of shell s of |u^x(k)|^2 + |u^y(k)|^2, with u^ = fft2(u) / (nx ny) the
    Fourier-series coefficients and k the signed integer frequencies; s < nshells."""
    ux, uy = t64(ux), t64(uy)
    ny, nx = ux.shape
    ax = torch.fft.fft2(ux) / (nx * ny)
    ay = torch.fft.fft2(uy) / (nx * ny)
    p = 0.5 * (ax.abs() ** 2 + ay.abs() ** 2)
    kx = torch.round(torch.fft.fftfreq(nx, dtype=DT) * nx).to(torch.int64)
    ky = torch.round(torch.fft.fftfreq(ny, dtype=DT) * ny).to(torch.int64)
    s = shell_index(kx[None, :], ky[:, None])
    e = torch.zeros(nshells, dtype=DT)
    keep = s < nshells
    e.index_add_(0, s[keep], p[keep])
    return e


# ---------------------------------------------------------------------------
# Helpers for worked numbers of Sec. 3-4
# ---------------------------------------------------------------------------
def forcing_time_scale(f0, kf=6.0):
    """T_f = sqrt(2 pi / (k_f F0)) (Sec. 3)."""
    return math.sqrt(2.0 * math.pi / (kf * f0))


def ps_viscosity(tau0, dx, dt):
    """nu^PS = nu^LBGK dx^2 / dt with nu^LBGK = c_s^2 (tau0 - 1/2) (Sec. 4)."""
    return viscosity(tau0) * dx * dx / dt
