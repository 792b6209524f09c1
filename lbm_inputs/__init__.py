"""Seeded synthetic inputs for the D2Q9 LBGK runs and the balance diagnostic.

This module is shared by the oracle-side tests and the GPU side: it builds the
initial density/velocity fields and the static forcing field on the host, in
FP64 NumPy, so that both implementations consume bit-identical inputs.  It
holds none of the method's arithmetic (no equilibrium, collision, streaming,
finite differences or box averages).

The paper's runs are the authors' own 256^2 simulations (Sec. 3); their dumped
configurations are not available, so the workloads below stand in for them:

* Taylor-Green vortex (closed-form decaying solution of the Navier-Stokes
  equations) for the small FP64 case.
* A random-phase isotropic velocity field with energy spectrum
  E(k) ~ k^4 exp(-2 (k/8)^2), scaled to a given maximum Mach number, for the
  decaying-turbulence, ensemble and differentiable workloads.
* For the three-dimensional extension: sums of a few random low-wavenumber
  cosine modes (periodic on any box) for rho, u and a static force.
* A divergence-free stream-function force built like Sec. 3, Eqs. 14-15 (a sum
  of cosines over a shell of integer wavevectors, force = (d_y Psi, -d_x Psi)),
  with independent seeded phases, for the forced workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CS", "taylor_green", "spectrum_velocity", "forcing_field", "shell_vectors",
    "ensemble_members", "balance_levels", "WORKLOADS", "Workload", "random_modes3", "fields3",
    "force3",
]

#: lattice speed of sound of D2Q9 (used only to turn a Mach number into a speed)
CS = 1.0 / math.sqrt(3.0)


def taylor_green(n: int, u0: float = 0.01):
    """Taylor-Green vortex with one wavelength per box side.

    u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky), k = 2 pi / n, rho = 1,
    x, y the integer cell indices.  Returns (rho, ux, uy) as float64 [n, n]
    arrays indexed [y, x].
    """
    k = 2.0 * math.pi / n
    idx = np.arange(n, dtype=np.float64)
    y, x = np.meshgrid(idx, idx, indexing="ij")
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    rho = np.ones((n, n), dtype=np.float64)
    return rho, ux, uy


def _spectral_velocity(n: int, rng: np.random.Generator, k_peak: float):
    kint = np.fft.fftfreq(n, d=1.0 / n)               # integer wavenumbers
    ky, kx = np.meshgrid(kint, kint, indexing="ij")
    kmag = np.hypot(kx, ky)
    theta = rng.uniform(0.0, 2.0 * math.pi, size=(n, n))
    with np.errstate(divide="ignore", invalid="ignore"):
        energy = kmag ** 4 * np.exp(-2.0 * (kmag / k_peak) ** 2)
        amp = np.sqrt(energy / (math.pi * kmag)) / kmag
    amp[0, 0] = 0.0
    psi_hat = amp * np.exp(1j * theta)
    two_pi_n = 2.0 * math.pi / n
    ux = np.real(np.fft.ifft2(1j * two_pi_n * ky * psi_hat))
    uy = np.real(np.fft.ifft2(-1j * two_pi_n * kx * psi_hat))
    return ux, uy


def spectrum_velocity(n: int, seed=0, max_mach: float = 0.05, k_peak: float = 8.0):
    """Random-phase isotropic velocity field, divergence-free by construction.

    psi_hat(k) = sqrt(E(|k|) / (pi |k|)) / |k| * exp(i theta_k), theta_k drawn
    uniformly in [0, 2 pi) from ``np.random.default_rng(seed)`` in
    ``np.fft.fftfreq`` order, E(k) = k^4 exp(-2 (k / k_peak)^2); psi = Re IFFT;
    u = (d_y psi, -d_x psi) (spectral derivative, sign convention of Eq. 15);
    the field is scaled so that max |u| / c_s = max_mach.  rho = 1.

    ``seed`` may be an int or an existing ``np.random.Generator``.
    """
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    ux, uy = _spectral_velocity(n, rng, k_peak)
    scale = max_mach * CS / np.sqrt(ux * ux + uy * uy).max()
    ux *= scale
    uy *= scale
    rho = np.ones((n, n), dtype=np.float64)
    return rho, ux, uy


def shell_vectors(kmin: float, kmax: float):
    """All integer wavevectors k with kmin <= |k| <= kmax (both signs)."""
    r = int(math.ceil(kmax))
    out = []
    for ky in range(-r, r + 1):
        for kx in range(-r, r + 1):
            k2 = kx * kx + ky * ky
            if kmin * kmin <= k2 <= kmax * kmax:
                out.append((kx, ky))
    return out


def forcing_field(n: int, seed: int = 0, kmin: float = 4.0, kmax: float = 6.0,
                  max_force: float | None = None, alpha: float = 1e-4,
                  target_mach: float = 0.08):
    """Static divergence-free forcing field (shape of Sec. 3, Eqs. 14-15).

    Psi(x) = sum_{kmin<=|k|<=kmax} cos(2 pi k.x / n + phi_k), phi_k ~ U[0, 2pi)
    from ``default_rng(seed)`` in the order of :func:`shell_vectors`;
    F = (d_y Psi, -d_x Psi) analytically.  The amplitude is scaled so that
    max |F| = max_force, by default alpha * target_mach * c_s (the uniform
    drag-limited response F / (alpha rho) then has Mach ``target_mach``).
    Returns (fx, fy) float64 [n, n] indexed [y, x].
    """
    if max_force is None:
        max_force = alpha * target_mach * CS
    rng = np.random.default_rng(seed)
    vecs = shell_vectors(kmin, kmax)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=len(vecs))
    # The trigonometric sum is evaluated by one inverse FFT of its (sparse)
    # coefficient array: d/dy cos(w k.x + phi) = Re(i w k_y exp(i (w k.x + phi))).
    w = 2.0 * math.pi / n
    ax = np.zeros((n, n), dtype=np.complex128)
    ay = np.zeros((n, n), dtype=np.complex128)
    for (kx, ky), ph in zip(vecs, phases):
        e = np.exp(1j * ph) * n * n
        ax[ky % n, kx % n] += 1j * w * ky * e      # F_x = d_y Psi
        ay[ky % n, kx % n] += -1j * w * kx * e     # F_y = -d_x Psi
    fx = np.real(np.fft.ifft2(ax))
    fy = np.real(np.fft.ifft2(ay))
    scale = max_force / np.sqrt(fx * fx + fy * fy).max()
    return fx * scale, fy * scale


#: printed amplitudes of Sec. 3: F0^T of the stream function (Eq. 14) and F0^R of
#: the damping (Eq. 16)
PAPER_FORCING_F0 = 8e-4
PAPER_DAMPING_F0 = 1e-5
PAPER_DAMPING_SHELL = (1.0, 2.0)
#: F0^T in lattice units used for the paper's workload: the printed 8e-4 with
#: Psi and its derivatives in lattice units drives every tau0 of Sec. 5 to
#: divergence within 2000 steps; 0.0075 x 8e-4 reproduces the printed Reynolds
#: numbers (U_rms N / nu = 90 ... 1800 for tau0 = 0.60 ... 0.515) and the
#: stability limit (tau0 = 0.515 stable, 0.51 not) with the damping rate F0^R
PAPER_FORCING_F0_LATTICE = 8e-4 * 0.0075


def paper_forcing(n: int = 256, f0: float = PAPER_FORCING_F0_LATTICE, kmin: float = 5.0,
                  kmax: float = 7.0, phase: float = 0.0):
    """The turbulent forcing of Sec. 3 (Eqs. 14-15): stream function
    Psi = f0 sum_{kmin<=|k|<=kmax} cos(2 pi k.x / n + phase) with one phase for every
    wavevector, F = (d_y Psi, -d_x Psi) analytically in lattice units.  Returns
    (fx, fy) float64 [n, n] indexed [y, x]."""
    w = 2.0 * math.pi / n
    yy, xx = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    fx = np.zeros((n, n))
    fy = np.zeros((n, n))
    for kx, ky in shell_vectors(kmin, kmax):
        s = np.sin(w * (kx * xx + ky * yy) + phase)
        fx += -f0 * w * ky * s       # d_y cos(...) = -w k_y sin(...)
        fy += f0 * w * kx * s        # -d_x cos(...) = w k_x sin(...)
    return fx, fy


def table1_count(L: int, n: int = 256) -> int:
    """Sub-volumes processed per side L on an n x n grid (Sec. 3, Table 1): the whole
    domain once, 1000 for 100 <= L < 256, 5000 for 10 <= L < 100, 10000 below, the
    thresholds scaled by n / 256 on other grids."""
    if L >= n:
        return 1
    if L * 256 >= 100 * n:
        return 1000
    if L * 256 >= 10 * n:
        return 5000
    return 10000


def table1_corners(n: int, sizes, seed: int = 0):
    """Random lower corners (x0, y0) of the sub-volumes of Table 1 for each side in
    `sizes`, uniform over the grid, drawn with default_rng(seed) in the order of
    `sizes`; the whole-domain box has the corner (0, 0).  Returns (corners int32
    [total, 2], counts list) with the corners of sizes[k] in the k-th run."""
    rng = np.random.default_rng(seed)
    parts, counts = [], []
    for L in sizes:
        c = table1_count(int(L), n)
        if c == 1:
            xy = np.zeros((1, 2), dtype=np.int64)
        else:
            xy = rng.integers(0, n, size=(c, 2))
        parts.append(xy)
        counts.append(c)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.int32)), counts


def log_edges(lo: float = 1e-6, hi: float = 10.0, per_decade: int = 10):
    """Logarithmic bin edges lo * 10^(i / per_decade) up to hi (for the PDFs of the
    balancing errors, Figs. 6-7 and 11-12)."""
    nd = int(round(np.log10(hi / lo) * per_decade))
    return lo * 10.0 ** (np.arange(nd + 1) / per_decade)


ENSEMBLE_SIZES = (256, 384, 512, 768, 1024)


def ensemble_members(nruns: int = 64, sizes=ENSEMBLE_SIZES, tau_lo: float = 0.505,
                     tau_hi: float = 0.6, max_mach: float = 0.05, build_fields: bool = True):
    """Members of the batched decaying-turbulence ensemble.

    Run r uses ``default_rng(r)`` and draws, in order: its grid side from
    ``sizes`` (uniform), tau ~ U[tau_lo, tau_hi], then the spectrum phases.
    Returns a list of dicts {n, tau, seed, rho, ux, uy} (fields omitted when
    ``build_fields`` is False).
    """
    out = []
    for r in range(nruns):
        rng = np.random.default_rng(r)
        n = int(rng.choice(np.asarray(sizes)))
        tau = float(rng.uniform(tau_lo, tau_hi))
        m = {"n": n, "tau": tau, "seed": r}
        if build_fields:
            rho, ux, uy = spectrum_velocity(n, rng, max_mach=max_mach)
            m.update(rho=rho, ux=ux, uy=uy)
        out.append(m)
    return out


def balance_levels(n: int, seed: int = 3, max_mach: float = 0.05, drho: float = 1e-2,
                   dt_scale: float = 2e-3, compressive: float = 0.2, with_force: bool = True):
    """Three smooth time levels (n-2, n-1, n) of (rho, u) plus a force field.

    Synthetic inputs for checking the balance diagnostic on its own.  The
    velocity at level n-k is u * (1 + k dt_scale) + k dt_scale * v, where u and
    v are spectrum fields plus a compressive part ``compressive`` * grad(phi)
    (so that div u, and with it the compressibility terms, is not zero);
    rho = 1 + drho * s_k with smooth perturbations s_k.  Returns a dict with
    lists rho[3], ux[3], uy[3] ordered (n-2, n-1, n) and fx, fy (zeros when
    ``with_force`` is False).
    """
    rng = np.random.default_rng(seed)
    _, ux, uy = spectrum_velocity(n, rng, max_mach=max_mach)
    _, vx, vy = spectrum_velocity(n, rng, max_mach=max_mach)
    _, sx, sy = spectrum_velocity(n, rng, max_mach=1.0)
    _, gx, gy = spectrum_velocity(n, rng, max_mach=max_mach)
    # a curl-free field: rotate a divergence-free one by 90 degrees (grad phi)
    ux = ux + compressive * gy
    uy = uy - compressive * gx
    vx = vx - compressive * gx
    vy = vy - compressive * gy
    rhos, uxs, uys = [], [], []
    for lev in (2, 1, 0):
        a = 1.0 + lev * dt_scale
        uxs.append(ux * a + lev * dt_scale * vx)
        uys.append(uy * a + lev * dt_scale * vy)
        rhos.append(1.0 + drho * ((1.0 + 0.1 * lev) * sx + 0.5 * lev * sy) / CS)
    if with_force:
        fx, fy = forcing_field(n, seed=seed, max_force=1e-5)
    else:
        fx = np.zeros((n, n))
        fy = np.zeros((n, n))
    return {"rho": rhos, "ux": uxs, "uy": uys, "fx": fx, "fy": fy}


@dataclass(frozen=True)
class Workload:
    """One of the five workloads the library is measured and checked on."""
    name: str
    n: int
    dtype: str
    tau: float
    steps: int
    init: str
    seed: int = 0
    force: bool = False
    alpha: float = 0.0
    sizes: tuple = ()
    balance_every: int = 0
    taus: tuple = field(default_factory=tuple)


WORKLOADS = {
    "tg64": Workload("taylor-green 64^2 fp64", 64, "f64", 0.6, 1000, "tg",
                     sizes=(4, 8, 16, 32)),
    "decay1024": Workload("decaying turbulence 1024^2 fp32", 1024, "f32", 0.51, 10000, "spectrum",
                          seed=0, sizes=(8, 16, 32, 64, 128, 256), balance_every=100),
    "ensemble64": Workload("ensemble of 64 decaying runs 256^2..1024^2 fp32", 0, "f32", 0.0, 5000,
                           "ensemble"),
    "forced4096": Workload("forced turbulence 4096^2 fp32, Guo force + linear drag", 4096, "f32",
                           0.51, 50000, "rest", seed=0, force=True, alpha=1e-4,
                           sizes=(8, 16, 32, 64, 128, 256), balance_every=500,
                           taus=(0.5005, 0.501, 0.505, 0.51, 0.55)),
    "adjoint512": Workload("differentiable decaying run 512^2 fp32", 512, "f32", 0.51, 2000,
                           "spectrum", seed=7, sizes=(32,)),
    # the paper's own set-up (Sec. 3): exact-difference forcing, turbulent force on
    # 5 <= |k| <= 7 (one phase, lattice amplitude PAPER_FORCING_F0_LATTICE), damping
    # of 1 <= |k| <= 2 at the rate F0^R = 1e-5 per step, tau0 sweep of Sec. 5
    "paper256": Workload("the paper's forced 2D turbulence 256^2 fp32, exact-difference forcing", 256,
                         "f32", 0.52, 20000, "rest", seed=0, force=True,
                         sizes=(4, 8, 16, 32, 64, 128, 181, 256), balance_every=100,
                         taus=(0.60, 0.54, 0.53, 0.52, 0.515)),
}


# ---------------------------------------------------------------------------
# three dimensions ([nz, ny, nx] arrays)
# ---------------------------------------------------------------------------
def random_modes3(shape, rng: np.random.Generator, nmodes: int = 8, kmax: int = 2):
    """Sum of nmodes cosines cos(2 pi (a x / nx + b y / ny + c z / nz) + phase) with
    integer (a, b, c) in [-kmax, kmax] and standard-normal amplitudes, scaled to a
    maximum |value| of 1; [nz, ny, nx] FP64."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(nmodes):
        a, b, c = rng.integers(-kmax, kmax + 1, size=3)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        out += rng.standard_normal() * np.cos(2.0 * math.pi * (a * x / nx + b * y / ny + c * z / nz) + ph)
    m = np.abs(out).max()
    return out / m if m > 0 else out


def fields3(shape, seed: int = 0, max_mach: float = 0.05, drho: float = 0.01, nmodes: int = 8,
            kmax: int = 2):
    """Seeded smooth 3D initial fields (rho, ux, uy, uz), each velocity component with
    maximum |u| = max_mach c_s and rho = 1 + drho * (modes of max 1)."""
    rng = np.random.default_rng(seed)
    u = [max_mach * CS * random_modes3(shape, rng, nmodes, kmax) for _ in range(3)]
    rho = 1.0 + drho * random_modes3(shape, rng, nmodes, kmax)
    return rho, u[0], u[1], u[2]


def force3(shape, seed: int = 0, amp: float = 1e-5, nmodes: int = 4, kmax: int = 2):
    """Seeded static 3D force (fx, fy, fz), each component of maximum |value| amp."""
    rng = np.random.default_rng(seed + 7919)
    return tuple(amp * random_modes3(shape, rng, nmodes, kmax) for _ in range(3))
