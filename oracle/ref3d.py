"""FP64 CPU oracle for the three-dimensional extension: D2Q9's counterparts D3Q19 and
D3Q27 with the LBGK update and Guo's forcing term, and the sub-volume kinetic-energy and enstrophy
balances in 3D, where the enstrophy equation gains the vortex-stretching term.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it.  Plain PyTorch on the CPU in float64, written against the
paper (Tauzin et al., Computers & Fluids 172 (2018)): the LBGK update of Sec. 1 (Eqs.
1, 2, 5) on the textbook D3Q19 lattice, the balance equations of Sec. 2 in their index
form (Eqs. 8-11, written for any dimension; the paper's 2D runs drop the stretching
term, and Sec. 2 notes that 3D keeps it), the time and space derivatives of Sec. 3
(Eqs. 17-18) and the balancing errors of Eqs. 12-13 over cubic sub-volumes.

Arrays are indexed [z, y, x]; populations are [Q, nz, ny, nx], Q = 19 or 27 (the
lattice of a population array is read off its first extent).  Lattice units.

Readings (also in the design notes): D3Q19 with weights 1/3, 1/18, 1/36 and
c_s^2 = 1/3; D3Q27, the product of three D1Q3 lattices, with weights 8/27, 2/27, 1/54,
1/216 and the same c_s^2 and second-order equilibrium; Guo's force term with the half-force velocity (as the 2D hot path); the
vorticity omega = curl u; Eq. 11's terms in 3D: -d_j(Omega u_j), -Omega d_j u_j,
omega . curl(F / rho), H . curl(omega), div(H x omega) (H_i = d_j sigma_ij / rho) and the
stretching term omega_i omega_j d_j u_i; cubes L^3 at every corner with periodic wrap;
L = N is one window.
"""
from __future__ import annotations

import itertools

import torch

from . import ref

DT = torch.float64

# ---------------------------------------------------------------------------
# D3Q19 lattice
# ---------------------------------------------------------------------------
#: velocities (c_x, c_y, c_z): rest, 6 axis, 12 edge diagonals
C = ((0, 0, 0),
     (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
     (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
     (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1))
#: weights t_l
W = (1.0 / 3.0,) + (1.0 / 18.0,) * 6 + (1.0 / 36.0,) * 12
CS2 = 1.0 / 3.0
Q = 19

# ---------------------------------------------------------------------------
# D3Q27 lattice: every c in {-1, 0, 1}^3, weight prod_a (2/3 for c_a = 0, 1/6 otherwise)
# ---------------------------------------------------------------------------
#: rest, the 6 axis and 12 edge velocities in the D3Q19 order, then the 8 corners in
#: opposite pairs
C27 = C + ((1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
           (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1))
W27 = (8.0 / 27.0,) + (2.0 / 27.0,) * 6 + (1.0 / 54.0,) * 12 + (1.0 / 216.0,) * 8
LATTICES = {19: (C, W), 27: (C27, W27)}


def lattice(q):
    """(velocities, weights) of the lattice with q populations (19 or 27)."""
    return LATTICES[q]

t64 = ref.t64


def equilibrium(rho, ux, uy, uz, q=19):
    """Eq. 2 on D3Q19 (q = 19) or D3Q27 (q = 27): t_l rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)."""
    cs, ws = lattice(q)
    usq = ux * ux + uy * uy + uz * uz
    out = []
    for (cx, cy, cz), w in zip(cs, ws):
        cu = cx * ux + cy * uy + cz * uz
        out.append(w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq))
    return torch.stack(out)


def density(f):
    return f.sum(0)


def momentum(f):
    cs, _ = lattice(f.shape[0])
    jx = sum(cx * f[l] for l, (cx, _, _) in enumerate(cs))
    jy = sum(cy * f[l] for l, (_, cy, _) in enumerate(cs))
    jz = sum(cz * f[l] for l, (_, _, cz) in enumerate(cs))
    return jx, jy, jz


def macroscopic(f, fx=None, fy=None, fz=None):
    """rho and the half-force velocity u = (sum f c + F/2) / rho (u = j/rho unforced)."""
    rho = density(f)
    jx, jy, jz = momentum(f)
    if fx is not None:
        jx, jy, jz = jx + 0.5 * fx, jy + 0.5 * fy, jz + 0.5 * fz
    return rho, jx / rho, jy / rho, jz / rho


def guo_source(ux, uy, uz, fx, fy, fz, tau, q=19):
    """Guo's forcing term (1 - 1/(2 tau)) t_l [3 (c - u) + 9 (c.u) c] . F."""
    cs, ws = lattice(q)
    out = []
    for (cx, cy, cz), w in zip(cs, ws):
        cu = cx * ux + cy * uy + cz * uz
        gx = 3.0 * (cx - ux) + 9.0 * cu * cx
        gy = 3.0 * (cy - uy) + 9.0 * cu * cy
        gz = 3.0 * (cz - uz) + 9.0 * cu * cz
        out.append((1.0 - 0.5 / tau) * w * (gx * fx + gy * fy + gz * fz))
    return torch.stack(out)


def collide(f, tau, fx=None, fy=None, fz=None):
    """Eq. 1's collision: f - (f - f^eq) / tau (+ Guo's term)."""
    q = f.shape[0]
    rho, ux, uy, uz = macroscopic(f, fx, fy, fz)
    post = f - (f - equilibrium(rho, ux, uy, uz, q)) / tau
    if fx is not None:
        post = post + guo_source(ux, uy, uz, fx, fy, fz, tau, q)
    return post


def stream(fpost):
    """f_l(x + c_l, t + 1) = f*_l(x, t), periodic."""
    cs, _ = lattice(fpost.shape[0])
    return torch.stack([torch.roll(fpost[l], shifts=(cz, cy, cx), dims=(0, 1, 2))
                        for l, (cx, cy, cz) in enumerate(cs)])


def step(f, tau, fx=None, fy=None, fz=None):
    return stream(collide(f, tau, fx, fy, fz))


def init_populations(rho, ux, uy, uz, q=19):
    return equilibrium(t64(rho), t64(ux), t64(uy), t64(uz), q)


def run(f, nsteps, tau, fx=None, fy=None, fz=None):
    for _ in range(nsteps):
        f = step(f, tau, fx, fy, fz)
    return f


def run_with_history(f, nsteps, tau, fx=None, fy=None, fz=None):
    """Populations after nsteps (>= 2) and (rho, ux, uy, uz) at nsteps-2, nsteps-1, nsteps."""
    hist = []
    for s in range(nsteps):
        if s >= nsteps - 2:
            hist.append(macroscopic(f, fx, fy, fz))
        f = step(f, tau, fx, fy, fz)
    hist.append(macroscopic(f, fx, fy, fz))
    return f, hist


# ---------------------------------------------------------------------------
# Derivatives (Eq. 18 along each axis, periodic; Eq. 17 in time)
# ---------------------------------------------------------------------------
def ddx(a):
    return ref._fd8(a, 2)


def ddy(a):
    return ref._fd8(a, 1)


def ddz(a):
    return ref._fd8(a, 0)


def grad(a):
    return ddx(a), ddy(a), ddz(a)


def curl(ax, ay, az):
    return (ddy(az) - ddz(ay), ddz(ax) - ddx(az), ddx(ay) - ddy(ax))


def div(ax, ay, az):
    return ddx(ax) + ddy(ay) + ddz(az)


# ---------------------------------------------------------------------------
# Balance terms in 3D (Eqs. 8-11 in index form)
# ---------------------------------------------------------------------------
#: order of the 15 integrand fields: energy (LHS and five terms), enstrophy (LHS and six
#: terms, the sixth the vortex stretching), |u|^2
TERM_NAMES = ("lhs_E", "e1", "e2", "e3", "e4", "e5",
              "lhs_Z", "z1", "z2", "z3", "z4", "z5", "z6", "usq")


def balance_fields(rho, ux, uy, uz, fx, fy, fz, nu):
    """Pointwise integrands at level n from three levels (n-2, n-1, n) of rho, u.

    Energy, E = rho |u|^2 / 2: lhs_E = d_t E (Eq. 17); e1 = -div(E u); e2 = -u . grad p,
    p = rho / 3; e3 = u . F; e4 = -sigma_ij d_j u_i; e5 = d_j (u_i sigma_ij), with
    sigma_ij = nu rho (d_j u_i + d_i u_j).  Enstrophy, Omega = |omega|^2 / 2, omega = curl u:
    lhs_Z = d_t Omega; z1 = -div(Omega u); z2 = -Omega div u; z3 = omega . curl(F / rho);
    z4 = H . curl(omega); z5 = div(H x omega), H_i = d_j sigma_ij / rho; z6 = omega_i omega_j
    d_j u_i (vortex stretching).  usq = |u|^2.
    """
    r = t64(rho[2])
    v = [t64(ux[2]), t64(uy[2]), t64(uz[2])]
    zero = torch.zeros_like(r)
    F = [zero if fx is None else t64(fx), zero if fy is None else t64(fy), zero if fz is None else t64(fz)]
    d = [grad(vi) for vi in v]           # d[i][j] = d_j u_i
    energy = [0.5 * t64(rho[k]) * (t64(ux[k]) ** 2 + t64(uy[k]) ** 2 + t64(uz[k]) ** 2) for k in range(3)]
    vort = [curl(t64(ux[k]), t64(uy[k]), t64(uz[k])) for k in range(3)]
    enst = [0.5 * (w[0] ** 2 + w[1] ** 2 + w[2] ** 2) for w in vort]
    e_n, om, z_n = energy[2], vort[2], enst[2]
    p = CS2 * r
    sig = [[nu * r * (d[i][j] + d[j][i]) for j in range(3)] for i in range(3)]
    h = [sum(grad(sig[i][j])[j] for j in range(3)) / r for i in range(3)]
    out = {}
    out["lhs_E"] = ref.bdf2(energy[2], energy[1], energy[0])
    out["e1"] = -div(e_n * v[0], e_n * v[1], e_n * v[2])
    gp = grad(p)
    out["e2"] = -(v[0] * gp[0] + v[1] * gp[1] + v[2] * gp[2])
    out["e3"] = v[0] * F[0] + v[1] * F[1] + v[2] * F[2]
    out["e4"] = -sum(sig[i][j] * d[i][j] for i in range(3) for j in range(3))
    out["e5"] = div(*[sum(v[i] * sig[i][j] for i in range(3)) for j in range(3)])
    out["lhs_Z"] = ref.bdf2(enst[2], enst[1], enst[0])
    out["z1"] = -div(z_n * v[0], z_n * v[1], z_n * v[2])
    out["z2"] = -z_n * (d[0][0] + d[1][1] + d[2][2])
    cf = curl(F[0] / r, F[1] / r, F[2] / r)
    out["z3"] = om[0] * cf[0] + om[1] * cf[1] + om[2] * cf[2]
    cw = curl(*om)
    out["z4"] = h[0] * cw[0] + h[1] * cw[1] + h[2] * cw[2]
    hxw = (h[1] * om[2] - h[2] * om[1], h[2] * om[0] - h[0] * om[2], h[0] * om[1] - h[1] * om[0])
    out["z5"] = div(*hxw)
    out["z6"] = sum(om[i] * om[j] * d[i][j] for i in range(3) for j in range(3))
    out["usq"] = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    return out


# ---------------------------------------------------------------------------
# Cubic sub-volumes and balancing errors (Eqs. 12-13, 20)
# ---------------------------------------------------------------------------
def box_mean_map(g, L):
    """Mean of g over the L^3 cube with lower corner (z0, y0, x0), for every corner,
    periodic; running sums over the periodically doubled array along each axis."""
    g = t64(g)

    def window_sum(a, dim):
        n = a.shape[dim]
        ext = torch.cat([a, a], dim=dim)
        cs = torch.cumsum(ext, dim=dim)
        zero = torch.zeros_like(a.narrow(dim, 0, 1))
        cs = torch.cat([zero, cs], dim=dim)
        return cs.narrow(dim, L, n) - cs.narrow(dim, 0, n)

    s = window_sum(window_sum(window_sum(g, 2), 1), 0)
    return s / float(L) ** 3


def box_mean_brute(g, L, z0, y0, x0):
    g = t64(g)
    nz, ny, nx = g.shape
    acc = 0.0
    for k, j, i in itertools.product(range(L), range(L), range(L)):
        acc += float(g[(z0 + k) % nz, (y0 + j) % ny, (x0 + i) % nx])
    return acc / L ** 3


def balancing_errors(means):
    """delta^E, delta^Omega (Eqs. 12-13, largest |RHS term| as denominator, NaN for zero)
    and Ma_V = sqrt(<|u|^2>) / c_s (Eq. 20) from box means of any shape."""
    e = [means[k] for k in ("e1", "e2", "e3", "e4", "e5")]
    z = [means[k] for k in ("z1", "z2", "z3", "z4", "z5", "z6")]
    rhs_e, rhs_z = sum(e), sum(z)
    den_e = torch.stack([t.abs() for t in e]).max(0).values
    den_z = torch.stack([t.abs() for t in z]).max(0).values
    nan = torch.full_like(rhs_e, float("nan"))
    d_e = torch.where(den_e > 0, (rhs_e - means["lhs_E"]).abs() / torch.where(den_e > 0, den_e, 1.0), nan)
    d_z = torch.where(den_z > 0, (rhs_z - means["lhs_Z"]).abs() / torch.where(den_z > 0, den_z, 1.0), nan)
    return d_e, d_z, means["usq"].sqrt() / ref.CS


def subvolume_balance(fields, sizes):
    """Per L: statistics (count, n_nan, mean, std, min, max) of delta^E, delta^Omega, Ma_V
    over the cubes at every corner (L = N: the one whole-domain cube), and the maps."""
    nz, ny, nx = next(iter(fields.values())).shape
    out = []
    for L in sizes:
        if not (1 <= L <= min(nx, ny, nz)):
            raise ValueError(f"box size {L} outside [1, {min(nx, ny, nz)}]")
        means = {k: box_mean_map(v, L) for k, v in fields.items()}
        if L == nx == ny == nz:
            means = {k: v[:1, :1, :1] for k, v in means.items()}
        d_e, d_z, ma = balancing_errors(means)
        out.append({"L": L, "dE": ref._stats(d_e), "dZ": ref._stats(d_z), "Ma": ref._stats(ma),
                    "maps": (d_e, d_z, ma)})
    return out
