"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

None of these re-types an oracle formula: each checks a property that a
dropped term, a wrong sign, a wrong index or a swapped operand would break
(textbook lattice identities, conservation laws, closed-form solutions,
symmetries, brute force on small inputs, the paper's worked numbers).
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as inp
from oracle import ref

D = torch.float64


def rand_state(n=12, seed=0, mach=0.1):
    g = torch.Generator().manual_seed(seed)
    rho = 1.0 + 0.05 * torch.rand(n, n, generator=g, dtype=D)
    ux = mach * ref.CS * (2 * torch.rand(n, n, generator=g, dtype=D) - 1)
    uy = mach * ref.CS * (2 * torch.rand(n, n, generator=g, dtype=D) - 1)
    return rho, ux, uy


def lattice():
    c = torch.tensor(ref.C, dtype=D)
    w = torch.tensor(ref.W, dtype=D)
    return c, w


# --------------------------------------------------------------------------
# Lattice and equilibrium (Eq. 2)
# --------------------------------------------------------------------------
def test_d2q9_isotropy():
    """Textbook D2Q9 identities: weights sum to 1, odd moments vanish,
    sum w c_i c_j = c_s^2 delta_ij, 4th moment = c_s^4 (3 symmetric deltas)."""
    c, w = lattice()
    assert len(ref.C) == 9 and len(set(ref.C)) == 9
    assert torch.isclose(w.sum(), torch.tensor(1.0, dtype=D), atol=1e-15)
    assert torch.allclose((w[:, None] * c).sum(0), torch.zeros(2, dtype=D), atol=1e-16)
    m2 = torch.einsum("l,li,lj->ij", w, c, c)
    assert torch.allclose(m2, torch.eye(2, dtype=D) / 3.0, atol=1e-16)
    m3 = torch.einsum("l,li,lj,lk->ijk", w, c, c, c)
    assert torch.allclose(m3, torch.zeros(2, 2, 2, dtype=D), atol=1e-16)
    m4 = torch.einsum("l,li,lj,lk,lm->ijkm", w, c, c, c, c)
    dlt = torch.eye(2, dtype=D)
    iso = (torch.einsum("ij,km->ijkm", dlt, dlt) + torch.einsum("ik,jm->ijkm", dlt, dlt)
           + torch.einsum("im,jk->ijkm", dlt, dlt)) / 9.0
    assert torch.allclose(m4, iso, atol=1e-16)


def test_equilibrium_moments():
    """sum f^eq = rho, sum c f^eq = rho u, sum c_i c_j f^eq = rho c_s^2 delta_ij + rho u_i u_j."""
    rho, ux, uy = rand_state()
    feq = ref.equilibrium(rho, ux, uy)
    c, _ = lattice()
    assert torch.allclose(feq.sum(0), rho, rtol=1e-15, atol=0)
    jx = torch.einsum("l,lyx->yx", c[:, 0], feq)
    jy = torch.einsum("l,lyx->yx", c[:, 1], feq)
    assert torch.allclose(jx, rho * ux, atol=1e-16)
    assert torch.allclose(jy, rho * uy, atol=1e-16)
    pxx = torch.einsum("l,lyx->yx", c[:, 0] * c[:, 0], feq)
    pyy = torch.einsum("l,lyx->yx", c[:, 1] * c[:, 1], feq)
    pxy = torch.einsum("l,lyx->yx", c[:, 0] * c[:, 1], feq)
    assert torch.allclose(pxx, rho / 3 + rho * ux * ux, atol=1e-15)
    assert torch.allclose(pyy, rho / 3 + rho * uy * uy, atol=1e-15)
    assert torch.allclose(pxy, rho * ux * uy, atol=1e-16)


def test_guo_source_moments():
    """Guo's forcing term: zeroth moment 0, first moment (1 - 1/(2 tau)) F,
    second moment (1 - 1/(2 tau)) (u_i F_j + u_j F_i)."""
    rho, ux, uy = rand_state(seed=1)
    g = torch.Generator().manual_seed(5)
    fx = 1e-3 * torch.randn(rho.shape, generator=g, dtype=D)
    fy = 1e-3 * torch.randn(rho.shape, generator=g, dtype=D)
    tau = 0.57
    s = ref.guo_source(ux, uy, fx, fy, tau)
    c, _ = lattice()
    k = 1.0 - 0.5 / tau
    assert torch.allclose(s.sum(0), torch.zeros_like(rho), atol=1e-18)
    assert torch.allclose(torch.einsum("l,lyx->yx", c[:, 0], s), k * fx, atol=1e-18)
    assert torch.allclose(torch.einsum("l,lyx->yx", c[:, 1], s), k * fy, atol=1e-18)
    assert torch.allclose(torch.einsum("l,lyx->yx", c[:, 0] ** 2, s), k * 2 * ux * fx, atol=1e-18)
    assert torch.allclose(torch.einsum("l,lyx->yx", c[:, 1] ** 2, s), k * 2 * uy * fy, atol=1e-18)
    assert torch.allclose(torch.einsum("l,lyx->yx", c[:, 0] * c[:, 1], s),
                          k * (ux * fy + uy * fx), atol=1e-18)


# --------------------------------------------------------------------------
# Collision and streaming (Eq. 1)
# --------------------------------------------------------------------------
def test_collision_conserves_mass_and_adds_force():
    """Per site: sum f* = sum f and sum c (f* - f) = F (total force incl. drag)."""
    rho, ux, uy = rand_state(seed=2)
    g = torch.Generator().manual_seed(9)
    f = ref.equilibrium(rho, ux, uy) * (1 + 0.05 * torch.randn(9, *rho.shape, generator=g, dtype=D))
    fx = 1e-4 * torch.randn(rho.shape, generator=g, dtype=D)
    fy = 1e-4 * torch.randn(rho.shape, generator=g, dtype=D)
    alpha = 1e-2
    post = ref.collide(f, 0.53, fx, fy, alpha)
    assert torch.allclose(post.sum(0), f.sum(0), rtol=1e-15, atol=0)
    r, vx, vy, ftx, fty = ref.macroscopic(f, fx, fy, alpha)
    c, _ = lattice()
    dj_x = torch.einsum("l,lyx->yx", c[:, 0], post - f)
    dj_y = torch.einsum("l,lyx->yx", c[:, 1], post - f)
    assert torch.allclose(dj_x, ftx, atol=1e-17)
    assert torch.allclose(dj_y, fty, atol=1e-17)
    # the drag is included in the total force, opposed to the velocity
    assert torch.allclose(ftx, fx - alpha * r * vx, atol=0)


def test_equilibrium_is_fixed_point_unforced():
    """An unforced equilibrium population is unchanged by collision (uniform flow also by streaming)."""
    n = 8
    rho = torch.full((n, n), 1.02, dtype=D)
    ux = torch.full((n, n), 0.03, dtype=D)
    uy = torch.full((n, n), -0.01, dtype=D)
    f = ref.equilibrium(rho, ux, uy)
    assert torch.allclose(ref.step(f, 0.6), f, atol=1e-16)


def test_streaming_moves_centre_of_mass_with_momentum():
    """Streaming moves population l by +c_l (Eq. 1): the density first moment of a
    localised moving blob changes by exactly the total momentum per step (the fluid
    near the periodic seam stays at rest, so nothing crosses it)."""
    n = 48
    idx = torch.arange(n, dtype=D)
    y, x = torch.meshgrid(idx, idx, indexing="ij")
    blob = torch.exp(-((x - 22) ** 2 + (y - 25) ** 2) / 10.0)
    rho = 1.0 + 0.01 * blob
    ux = 0.05 * blob
    uy = -0.03 * blob
    f = ref.equilibrium(rho, ux, uy)
    jx0, jy0 = (rho * ux).sum(), (rho * uy).sum()

    def first_moment(ff):
        r = ref.density(ff)
        return (x * r).sum(), (y * r).sum()

    mx0, my0 = first_moment(f)
    t = 5
    mx1, my1 = first_moment(ref.run(f, t, 0.7))
    assert float((mx1 - mx0) / (t * jx0)) == pytest.approx(1.0, rel=1e-9)
    assert float((my1 - my0) / (t * jy0)) == pytest.approx(1.0, rel=1e-9)


def test_global_conservation():
    """Mass is conserved to roundoff with force and drag; momentum without them."""
    rho, ux, uy = inp.spectrum_velocity(32, seed=4, max_mach=0.1)
    f = ref.init_populations(rho, ux, uy)
    fx, fy = (ref.t64(a) for a in inp.forcing_field(32, seed=1, max_force=1e-4))
    m0 = float(ref.density(f).sum())
    ff = ref.run(f, 40, 0.55, fx, fy, 1e-3)
    assert float(ref.density(ff).sum()) == pytest.approx(m0, rel=1e-14)
    fu = ref.run(f, 40, 0.55)
    j0 = ref.momentum(f)
    j1 = ref.momentum(fu)
    scale = float(ref.density(f).sum()) * 0.1 * ref.CS
    assert abs(float(j1[0].sum() - j0[0].sum())) < 1e-13 * scale
    assert abs(float(j1[1].sum() - j0[1].sum())) < 1e-13 * scale


def test_uniform_force_with_drag_closed_form():
    """Uniform fluid at rest, uniform F_ext, drag alpha: momentum j^t = (F/alpha)(1 - r^t),
    r = (1 - alpha/2)/(1 + alpha/2); the velocity tends to F / (alpha rho)."""
    n = 4
    alpha = 0.05
    fx0, fy0 = 2e-4, -1e-4
    f = ref.equilibrium(torch.ones(n, n, dtype=D), torch.zeros(n, n, dtype=D), torch.zeros(n, n, dtype=D))
    fxf = torch.full((n, n), fx0, dtype=D)
    fyf = torch.full((n, n), fy0, dtype=D)
    r = (1 - alpha / 2) / (1 + alpha / 2)
    for t in range(1, 60):
        f = ref.step(f, 0.8, fxf, fyf, alpha)
        jx, jy = ref.momentum(f)
        assert float(jx[0, 0]) == pytest.approx(fx0 / alpha * (1 - r ** t), rel=1e-12)
        assert float(jy[0, 0]) == pytest.approx(fy0 / alpha * (1 - r ** t), rel=1e-12)


def _rot(a):
    """Rotate a [y, x] field so that the point (x, y) goes to (y, n-1-x)."""
    return torch.rot90(a, 1, (0, 1))


def test_shift_and_rotation_equivariance():
    """Translating the inputs translates the outputs; a quarter turn of the inputs
    (fields and velocity vectors) turns the outputs (step and balance fields)."""
    n = 24
    rho, ux, uy = (ref.t64(a) for a in inp.spectrum_velocity(n, seed=11, max_mach=0.1))
    rho = rho + 0.01 * ux / (0.1 * ref.CS)
    fx, fy = (ref.t64(a) for a in inp.forcing_field(n, seed=2, max_force=1e-4))
    tau, alpha = 0.56, 1e-3

    def evolve(r, vx, vy, gx, gy):
        f = ref.init_populations(r, vx, vy)
        _, hist = ref.run_with_history(f, 4, tau, gx, gy, alpha)
        return hist, ref.fields_from_history(hist, tau, gx, gy, alpha)

    hist, flds = evolve(rho, ux, uy, fx, fy)
    # shift
    sh = lambda a: torch.roll(a, (3, -5), (0, 1))  # noqa: E731
    hist_s, flds_s = evolve(sh(rho), sh(ux), sh(uy), sh(fx), sh(fy))
    for a, b in zip(hist[-1], hist_s[-1]):
        assert torch.allclose(sh(a), b, rtol=0, atol=1e-15)
    for k in ref.TERM_NAMES:
        assert torch.allclose(sh(flds[k]), flds_s[k], rtol=0, atol=1e-15 * float(flds[k].abs().max()) + 1e-30)
    # quarter turn: velocity (vx, vy) -> (vy, -vx) under (x, y) -> (y, n-1-x)
    hist_r, flds_r = evolve(_rot(rho), _rot(uy), -_rot(ux), _rot(fy), -_rot(fx))
    r_end, ux_end, uy_end = hist[-1]
    assert torch.allclose(_rot(r_end), hist_r[-1][0], atol=1e-15)
    assert torch.allclose(_rot(uy_end), hist_r[-1][1], atol=1e-15)
    assert torch.allclose(-_rot(ux_end), hist_r[-1][2], atol=1e-15)
    for k in ref.TERM_NAMES:   # all are scalars invariant under rotation
        scale = float(flds[k].abs().max()) + 1e-30
        assert torch.allclose(_rot(flds[k]), flds_r[k], atol=1e-13 * scale), k


def test_taylor_green_decay_rate():
    """Config tg64: energy of the Taylor-Green vortex decays as exp(-4 nu k^2 t) with
    nu = c_s^2 (tau - 1/2) (Eq. 5); E(1000)/E(0) = 0.2766 at N=64, tau=0.6."""
    n, tau, u0 = 64, 0.6, 0.01
    rho, ux, uy = inp.taylor_green(n, u0)
    f = ref.init_populations(rho, ux, uy)
    ts, es = [], []
    for t in range(1001):
        if t % 100 == 0:
            r, vx, vy = ref.moments(f)
            ts.append(t)
            es.append(float((0.5 * r * (vx * vx + vy * vy)).sum()))
        if t < 1000:
            f = ref.step(f, tau)
    k = 2 * math.pi / n
    rate_exact = 4 * (tau - 0.5) / 3 * k * k
    ts_a, es_a = np.array(ts[1:]), np.log(np.array(es[1:]))
    rate_fit = -np.polyfit(ts_a, es_a, 1)[0]
    assert rate_fit == pytest.approx(rate_exact, rel=1e-2)
    assert es[-1] / es[0] == pytest.approx(math.exp(-rate_exact * 1000), rel=2e-2)
    assert math.exp(-rate_exact * 1000) == pytest.approx(0.2766, abs=1e-4)


# --------------------------------------------------------------------------
# Derivative operators (Eqs. 17-18)
# --------------------------------------------------------------------------
def test_fd8_matches_textbook_stencil_on_sine():
    """FD8 on sin(kx) gives k* cos(kx), k* = 2 sum_m a_m sin(m k) with the textbook
    8th-order central weights a = (4/5, -1/5, 4/105, -1/280)."""
    n = 64
    idx = torch.arange(n, dtype=D)
    y, x = torch.meshgrid(idx, idx, indexing="ij")
    for kint in (1, 3, 7):
        k = 2 * math.pi * kint / n
        a = (4 / 5, -1 / 5, 4 / 105, -1 / 280)
        kstar = 2 * sum(am * math.sin((m + 1) * k) for m, am in enumerate(a))
        assert torch.allclose(ref.ddx(torch.sin(k * x)), kstar * torch.cos(k * x), atol=1e-14)
        assert torch.allclose(ref.ddy(torch.sin(k * y)), kstar * torch.cos(k * y), atol=1e-14)
        assert torch.allclose(ref.ddx(torch.sin(k * y)), torch.zeros(n, n, dtype=D), atol=1e-15)
    k = 2 * math.pi / 64
    kstar = 2 * sum(am * math.sin((m + 1) * k) for m, am in enumerate((4 / 5, -1 / 5, 4 / 105, -1 / 280)))
    assert kstar / k - 1 == pytest.approx(-1.4e-11, rel=0.1)


def test_fd8_exact_on_polynomials_to_degree_8():
    """An 8th-order centred difference differentiates polynomials of degree <= 8 exactly."""
    n = 40
    idx = torch.arange(n, dtype=D)
    y, x = torch.meshgrid(idx, idx, indexing="ij")
    s = (x - 20) / 4.0
    for deg in range(0, 9):
        g = s ** deg
        dg = deg * s ** max(deg - 1, 0) / 4.0 if deg > 0 else torch.zeros_like(s)
        got = ref.ddx(g)[:, 4:n - 4]
        assert torch.allclose(got, dg[:, 4:n - 4], rtol=1e-12, atol=1e-12), deg
    g = ((x - 20) / 4.0) ** 9   # degree 9 is not exact
    d9 = 9 * ((x - 20) / 4.0) ** 8 / 4.0
    assert (ref.ddx(g) - d9)[:, 4:n - 4].abs().max() > 1e-3


def test_fd8_telescopes():
    """Periodic central differences sum to zero over the domain."""
    g = torch.randn(16, 20, generator=torch.Generator().manual_seed(3), dtype=D)
    assert abs(float(ref.ddx(g).sum())) < 1e-13
    assert abs(float(ref.ddy(g).sum())) < 1e-13


def test_bdf2_exact_for_quadratics():
    """The three-level formula of Eq. 17 is exact for A(t) = a + b t + c t^2 at t = n."""
    a, b, c, nlev = 0.3, -1.7, 0.25, 10.0
    A = lambda t: a + b * t + c * t * t  # noqa: E731
    got = ref.bdf2(torch.tensor(A(nlev), dtype=D), torch.tensor(A(nlev - 1), dtype=D),
                   torch.tensor(A(nlev - 2), dtype=D))
    assert float(got) == pytest.approx(b + 2 * c * nlev, rel=1e-14)
    # relative error lambda^2/3 on exp(-lambda t)
    lam = 1e-2
    got = ref.bdf2(*(torch.tensor(math.exp(-lam * t), dtype=D) for t in (nlev, nlev - 1, nlev - 2)))
    exact = -lam * math.exp(-lam * nlev)
    assert float(got) / exact - 1 == pytest.approx(-lam * lam / 3, rel=2e-2)


# --------------------------------------------------------------------------
# Balance terms (Eqs. 8-13)
# --------------------------------------------------------------------------
def test_flux_terms_vanish_on_full_domain():
    """Divergence terms e1, e5, z1, z5 average to zero over the periodic domain."""
    lv = inp.balance_levels(32, seed=5)
    flds = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], lv["fx"], lv["fy"], nu=0.004)
    for k in ("e1", "e5", "z1", "z5"):
        scale = float(flds[k].abs().max())
        assert scale > 0
        assert abs(float(ref.box_mean_map(flds[k], 32)[0, 0])) < 1e-14 * scale, k
    for k in ("e2", "e3", "e4", "z2", "z3", "z4"):
        assert abs(float(flds[k].mean())) > 1e-10 * float(flds[k].abs().max()), k


def _tg_levels(n, U, nu, tlev, kstar):
    """Analytic TG fields (rho = 1) at times tlev with amplitude U exp(-2 nu k*^2 t)."""
    k = 2 * math.pi / n
    idx = torch.arange(n, dtype=D)
    y, x = torch.meshgrid(idx, idx, indexing="ij")
    rho, ux, uy = [], [], []
    for t in tlev:
        a = U * math.exp(-2 * nu * kstar * kstar * t)
        rho.append(torch.ones(n, n, dtype=D))
        ux.append(-a * torch.cos(k * x) * torch.sin(k * y))
        uy.append(a * torch.sin(k * x) * torch.cos(k * y))
    return rho, ux, uy, x, y, k


def test_taylor_green_balance_terms_closed_form():
    """Analytic Taylor-Green fields: <E> = U^2/4, <e4> = -nu U^2 k*^2, <Omega> = U^2 k*^2/2,
    <z4> = -2 nu U^2 k*^4, the other domain means vanish; z4 pointwise closed form.
    With the incompressible TG pressure the balances close on every sub-volume size."""
    n, U, nu = 64, 0.01, 0.1 / 3
    k = 2 * math.pi / n
    kstar = 2 * sum(am * math.sin((m + 1) * k) for m, am in enumerate((4 / 5, -1 / 5, 4 / 105, -1 / 280)))
    rho, ux, uy, x, y, _ = _tg_levels(n, U, nu, (98.0, 99.0, 100.0), kstar)
    a = U * math.exp(-2 * nu * kstar * kstar * 100.0)
    flds = ref.balance_fields(rho, ux, uy, None, None, nu)
    mean = lambda g: float(g.mean())  # noqa: E731
    E = 0.5 * (ux[2] ** 2 + uy[2] ** 2)
    assert mean(E) == pytest.approx(a * a / 4, rel=1e-13)
    assert mean(flds["e4"]) == pytest.approx(-nu * a * a * kstar ** 2, rel=1e-12)
    om = ref.vorticity(ux[2], uy[2])
    assert mean(0.5 * om * om) == pytest.approx(a * a * kstar ** 2 / 2, rel=1e-12)
    assert mean(flds["z4"]) == pytest.approx(-2 * nu * a * a * kstar ** 4, rel=1e-12)
    z4_exact = -4 * nu * a * a * kstar ** 4 * ((torch.cos(k * x) * torch.sin(k * y)) ** 2
                                               + (torch.sin(k * x) * torch.cos(k * y)) ** 2)
    assert torch.allclose(flds["z4"], z4_exact, atol=1e-12 * float(z4_exact.abs().max()))
    for key in ("e1", "e2", "e3", "e5", "z1", "z2", "z3", "z5"):
        assert abs(mean(flds[key])) < 1e-12 * float(flds["e4"].abs().max()), key
    # energy and enstrophy LHS match the dissipation on the full domain (BDF2 error lambda^2/3)
    assert mean(flds["lhs_E"]) / mean(flds["e4"]) == pytest.approx(1.0, abs=1e-5)
    assert mean(flds["lhs_Z"]) / mean(flds["z4"]) == pytest.approx(1.0, abs=1e-5)
    # local closure with the incompressible TG pressure
    p = [-(aa ** 2) / 4 * (torch.cos(2 * k * x) + torch.cos(2 * k * y))
         for aa in (a,)][0]
    fl_p = ref.balance_fields(rho, ux, uy, None, None, nu, p=p)
    for L in (4, 8, 16, 32, 64):
        means = ref.window_means(fl_p, L)
        for lhs, terms in (("lhs_E", ("e1", "e2", "e3", "e4", "e5")),
                           ("lhs_Z", ("z1", "z2", "z3", "z4", "z5"))):
            rhs = sum(means[t] for t in terms)
            big = max(float(means[t].abs().max()) for t in terms)
            assert float((rhs - means[lhs]).abs().max()) <= 1e-5 * big, (L, lhs)


def test_box_mean_matches_brute_force():
    """Running-sum box means equal plain double-loop sums, every L, many corners (N = 16)."""
    g = torch.randn(16, 16, generator=torch.Generator().manual_seed(8), dtype=D) + 0.3
    for L in range(1, 17):
        m = ref.box_mean_map(g, L)
        for (y0, x0) in ((0, 0), (3, 7), (15, 15), (9, 2), (15, 0)):
            assert float(m[y0, x0]) == pytest.approx(ref.box_mean_brute(g, L, y0, x0), abs=1e-13)
    # all corners for one L, against a rolled-sum construction
    L = 5
    m = ref.box_mean_map(g, L)
    acc = torch.zeros_like(g)
    for j in range(L):
        for i in range(L):
            acc += torch.roll(g, (-j, -i), (0, 1))
    assert torch.allclose(m, acc / L / L, atol=1e-14)


def test_balancing_error_definition_cases():
    """delta = |sum RHS - LHS| / max |RHS_i|; a zero denominator gives NaN (counted)."""
    z = torch.zeros(1, dtype=D)
    means = {k: z.clone() for k in ref.TERM_NAMES}
    means["e1"] = torch.tensor([2.0], dtype=D)
    means["e4"] = torch.tensor([-3.0], dtype=D)
    means["lhs_E"] = torch.tensor([-1.5], dtype=D)
    means["usq"] = torch.tensor([ref.CS2 * 0.04], dtype=D)
    d_e, d_z, ma = ref.balancing_errors(means)
    assert float(d_e) == pytest.approx(abs(2.0 - 3.0 + 1.5) / 3.0)
    assert math.isnan(float(d_z))
    assert float(ma) == pytest.approx(0.2)
    st = ref._stats(torch.tensor([1.0, float("nan"), 3.0], dtype=D))
    assert st["count"] == 2 and st["n_nan"] == 1 and st["mean"] == 2.0 and st["std"] == 1.0


def _full_domain_deltas(flds):
    """delta^E, delta^Omega of the one whole-domain box, from the plain domain means of the
    term fields (Eqs. 12-13 at L = N)."""
    m = {k: float(v.mean()) for k, v in flds.items()}
    e = [m[f"e{i}"] for i in range(1, 6)]
    z = [m[f"z{i}"] for i in range(1, 7) if f"z{i}" in m]
    return (abs(sum(e) - m["lhs_E"]) / max(abs(v) for v in e),
            abs(sum(z) - m["lhs_Z"]) / max(abs(v) for v in z))


def _lhs_one_level_late(flds, late):
    """Planted mistake: the time derivative (Eq. 17) taken over levels n-3, n-2, n-1 while
    the right-hand side stays at level n."""
    out = dict(flds)
    out["lhs_E"], out["lhs_Z"] = late["lhs_E"], late["lhs_Z"]
    return out


#: Whole-domain budget of the Taylor-Green vortex with the levels n-2, n-1, n aligned
#: (Eq. 17): measured 7.4e-5 / 4.4e-5 at 64^2, t = 200; a derivative one level late is
#: off by the energy's relative change per step, 2 nu k^2 = 6.4e-4 of the dissipation
#: (measured 1.9e-3 / 1.7e-3 with the acoustic part), so this bound separates the two.
TG_CLOSURE = 3e-4


def test_taylor_green_run_balance_closes_on_aligned_levels():
    """run_with_history returns (rho, u) at n-2, n-1, n (Eq. 17): the LBGK Taylor-Green
    vortex (config tg64 at t = 200) closes its whole-domain energy and enstrophy budgets
    to < 3e-4, and the same budget with the derivative one level late does not."""
    n, tau, steps = 64, 0.6, 200
    rho, ux, uy = inp.taylor_green(n, 0.01)
    f = ref.init_populations(rho, ux, uy)
    fend, hist = ref.run_with_history(f, steps, tau)
    flds = ref.fields_from_history(hist, tau)
    res = ref.subvolume_balance(flds, [64, 32])
    assert res[0]["dE"]["count"] == 1 and res[1]["dE"]["count"] == 64 * 64
    assert res[0]["dE"]["mean"] < TG_CLOSURE and res[0]["dZ"]["mean"] < TG_CLOSURE
    assert max(_full_domain_deltas(flds)) < TG_CLOSURE
    _, hist_late = ref.run_with_history(f, steps - 1, tau)
    late = _lhs_one_level_late(flds, ref.fields_from_history(hist_late, tau))
    assert min(_full_domain_deltas(late)) > 1e-3
    # the last level is the returned state
    for a, b in zip(hist[2], ref.moments(fend)):
        assert torch.equal(a, b)


def _uniform_force_levels(hist, steps, fvec):
    """From rest under a uniform force F with no drag every step adds exactly F to the
    momentum (Guo's term and the exact-difference term alike), so the physical velocity at
    time t is (t + 1/2) F / rho with rho = 1: level k of the history is t = steps - 2 + k.
    Rounding of the momentum sum leaves ~1e-16 absolute; a level one step off, or the bare
    velocity j/rho, is off by F/2 or more."""
    for k, lv in enumerate(hist):
        t = steps - 2 + k
        rho, us = lv[0], lv[1:1 + len(fvec)]
        assert float((rho - 1).abs().max()) < 1e-15
        for u, fc in zip(us, fvec):
            want = (t + 0.5) * fc
            assert float((u - want).abs().max()) <= 1e-9 * abs(fc), (k, t)


def test_history_levels_under_a_uniform_force():
    """run_with_history: levels t = n-2, n-1, n carry u = (t + 1/2) F exactly (Guo with the
    half-force velocity); a level off by one step is off by F / u ~ 1/t."""
    n, steps, fv = 12, 9, (2e-5, -1e-5)
    z = torch.zeros(n, n, dtype=D)
    f = ref.init_populations(z + 1, z, z)
    fx, fy = z + fv[0], z + fv[1]
    fend, hist = ref.run_with_history(f, steps, 0.7, fx, fy)
    _uniform_force_levels(hist, steps, fv)
    for a, b in zip(hist[2], ref.moments(fend, fx, fy)):
        assert torch.equal(a, b)


def test_exact_difference_physical_velocity_and_levels():
    """edm_moments returns the exact-difference scheme's physical velocity (j + F/2)/rho:
    from rest under a uniform force u(t) = (t + 1/2) F (the bare j/rho would give t F), at
    the levels t = n-2, n-1, n of edm_run_with_history, with the total force F."""
    n, steps, fv = 12, 9, (3e-5, 1e-5)
    z = torch.zeros(n, n, dtype=D)
    f = ref.init_populations(z + 1, z, z)
    fx, fy = z + fv[0], z + fv[1]
    _, hist = ref.edm_run_with_history(f, steps, 0.7, fx, fy)
    _uniform_force_levels(hist, steps, fv)
    for lv in hist:
        assert torch.equal(lv[3], fx) and torch.equal(lv[4], fy)
    # one step from rest: u(0) = F/2, u(1) = 3F/2
    r0, u0x, _, _, _ = ref.edm_moments(f, fx, fy)
    r1, u1x, _, _, _ = ref.edm_moments(ref.edm_step(f, 0.7, fx, fy), fx, fy)
    assert float((u0x - 0.5 * fv[0]).abs().max()) <= 1e-9 * fv[0]
    assert float((u1x - 1.5 * fv[0]).abs().max()) <= 1e-9 * fv[0]


def test_exact_difference_history_closes_the_taylor_green_budget():
    """edm_run_with_history without force is the LBGK run: the Taylor-Green budget closes on
    its levels as for run_with_history, and not one level late."""
    n, tau, steps = 64, 0.6, 200
    rho, ux, uy = inp.taylor_green(n, 0.01)
    f = ref.init_populations(rho, ux, uy)
    _, hist = ref.edm_run_with_history(f, steps, tau)
    flds = ref.fields_from_history([h[:3] for h in hist], tau)
    assert max(_full_domain_deltas(flds)) < TG_CLOSURE
    _, hist_late = ref.edm_run_with_history(f, steps - 1, tau)
    late = _lhs_one_level_late(flds, ref.fields_from_history([h[:3] for h in hist_late], tau))
    assert min(_full_domain_deltas(late)) > 1e-3


def test_entropic_history_closes_the_taylor_green_budget():
    """entropic_run_with_history near equilibrium (Taylor-Green at Ma 0.017: alpha within
    1e-5 of 2, nu_eff within 1e-6 of nu): the budget with its nu_eff field closes on its
    levels (< 3e-4; measured 3e-6 / 4e-5 at 32^2, t = 100) and not one level late (5.8e-3)."""
    n, tau, steps = 32, 0.6, 100
    rho, ux, uy = inp.taylor_green(n, 0.01)
    f = ref.init_populations(rho, ux, uy)
    _, hist, nu = ref.entropic_run_with_history(f, steps, tau)
    assert float((nu - ref.viscosity(tau)).abs().max()) < 1e-6
    lv = [[h[i] for h in hist] for i in range(3)]
    flds = ref.balance_fields(lv[0], lv[1], lv[2], None, None, nu)
    assert max(_full_domain_deltas(flds)) < TG_CLOSURE
    _, hist_late, nu_late = ref.entropic_run_with_history(f, steps - 1, tau)
    lv = [[h[i] for h in hist_late] for i in range(3)]
    late = _lhs_one_level_late(flds, ref.balance_fields(lv[0], lv[1], lv[2], None, None, nu_late))
    assert min(_full_domain_deltas(late)) > 1e-3


def test_worked_numbers():
    """nu^PS ~ 0.004 for tau0 = 0.52, dx = 2 pi/256, dt = 1e-3 (Sec. 4); T_f = 36.18 for
    F0 = 8e-4, k_f = 6 (Sec. 3)."""
    assert ref.ps_viscosity(0.52, 2 * math.pi / 256, 1e-3) == pytest.approx(0.004, rel=1.5e-2)
    assert ref.forcing_time_scale(8e-4) == pytest.approx(36.18, abs=5e-3)


# --------------------------------------------------------------------------
# Adjoint (gradient of the enstrophy-residual loss)
# --------------------------------------------------------------------------
def test_adjoint_matches_central_differences():
    """Autodiff gradient of J(u0, tau) agrees with central finite differences (FP64)."""
    n, steps, L = 16, 12, 8
    _, ux, uy = inp.spectrum_velocity(n, seed=7, max_mach=0.1)
    tau = 0.55
    J, gx, gy, gt = ref.enstrophy_residual_grad(ux, uy, tau, steps, L)
    assert J > 0
    rng = np.random.default_rng(0)
    vx = rng.standard_normal((n, n))
    vy = rng.standard_normal((n, n))
    h = 1e-6 * float(np.abs(ux).max())
    jp = float(ref.enstrophy_residual_loss(ux + h * vx, uy + h * vy, tau, steps, L))
    jm = float(ref.enstrophy_residual_loss(ux - h * vx, uy - h * vy, tau, steps, L))
    fd = (jp - jm) / (2 * h)
    ad = float((gx * ref.t64(vx)).sum() + (gy * ref.t64(vy)).sum())
    assert ad == pytest.approx(fd, rel=1e-5)
    ht = 1e-6
    jp = float(ref.enstrophy_residual_loss(ux, uy, tau + ht, steps, L))
    jm = float(ref.enstrophy_residual_loss(ux, uy, tau - ht, steps, L))
    assert gt == pytest.approx((jp - jm) / (2 * ht), rel=1e-5)
    # single-site derivative
    e = np.zeros((n, n))
    e[5, 9] = 1.0
    jp = float(ref.enstrophy_residual_loss(ux + h * e, uy, tau, steps, L))
    jm = float(ref.enstrophy_residual_loss(ux - h * e, uy, tau, steps, L))
    assert float(gx[5, 9]) == pytest.approx((jp - jm) / (2 * h), rel=1e-4)


# --------------------------------------------------------------------------
# Balance terms against independent routes (spectral derivatives, exact solutions)
# --------------------------------------------------------------------------
def _spec_d(a, axis):
    """Exact derivative of a periodic trigonometric polynomial (FFT), dx = 1."""
    a = np.asarray(a)
    n = a.shape[axis]
    k = 2 * np.pi * np.fft.fftfreq(n)
    shape = [1, 1]
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(a, axis=axis), axis=axis))


def _smooth_compressible_fields(n=128, seed=0):
    """Low-wavenumber rho, u = curl psi + grad phi (|k| <= 3), strong divergence."""
    rng = np.random.default_rng(seed)
    idx = np.arange(n)
    y, x = np.meshgrid(idx, idx, indexing="ij")
    w = 2 * np.pi / n

    def trig():
        out = np.zeros((n, n))
        for kx in range(-3, 4):
            for ky in range(-3, 4):
                if kx * kx + ky * ky <= 9:
                    out += rng.standard_normal() * np.cos(w * (kx * x + ky * y) + rng.uniform(0, 2 * np.pi))
        return out

    psi, phi, s = trig(), trig(), trig()
    ux = _spec_d(psi, 0) + _spec_d(phi, 1)
    uy = -_spec_d(psi, 1) + _spec_d(phi, 0)
    sc = 0.05 / np.abs(np.hypot(ux, uy)).max()
    ux, uy = ux * sc, uy * sc
    rho = 1.0 + 0.05 * s / np.abs(s).max()
    return rho, ux, uy


def test_enstrophy_advection_terms_match_vorticity_identity():
    """z1 + z2 equals -omega div(u omega), the advective part of d_t(omega^2/2) from the
    curl of u.grad u (2D identity), with exact spectral derivatives."""
    rho, ux, uy = _smooth_compressible_fields()
    lv = ([rho] * 3, [ux] * 3, [uy] * 3)
    fl = ref.balance_fields(*lv, None, None, nu=0.01)
    om = _spec_d(uy, 1) - _spec_d(ux, 0)
    expect = -om * (_spec_d(ux * om, 1) + _spec_d(uy * om, 0))
    got = (fl["z1"] + fl["z2"]).numpy()
    assert np.abs(fl["z2"].numpy()).max() > 0.3 * np.abs(expect).max()   # compressibility matters here
    assert np.abs(got - expect).max() < 1e-6 * np.abs(expect).max()


def test_energy_flux_term_matches_momentum_advection():
    """e1 = -div(E u) equals -(|u|^2/2) div(rho u) - rho u.(u.grad u) (spectral route)."""
    rho, ux, uy = _smooth_compressible_fields(seed=1)
    fl = ref.balance_fields([rho] * 3, [ux] * 3, [uy] * 3, None, None, nu=0.01)
    divm = _spec_d(rho * ux, 1) + _spec_d(rho * uy, 0)
    adv_x = ux * _spec_d(ux, 1) + uy * _spec_d(ux, 0)
    adv_y = ux * _spec_d(uy, 1) + uy * _spec_d(uy, 0)
    expect = -0.5 * (ux * ux + uy * uy) * divm - rho * (ux * adv_x + uy * adv_y)
    assert np.abs(fl["e1"].numpy() - expect).max() < 1e-6 * np.abs(expect).max()


def test_viscous_terms_match_divergence_of_stress():
    """e4 + e5 = u_i d_j sigma_ij and z4 + z5 = omega curl(H), H = div(sigma)/rho,
    sigma = nu rho (grad u + grad u^T) (spectral route)."""
    rho, ux, uy = _smooth_compressible_fields(seed=2)
    nu = 0.02
    fl = ref.balance_fields([rho] * 3, [ux] * 3, [uy] * 3, None, None, nu=nu)
    dxux, dyux, dxuy, dyuy = _spec_d(ux, 1), _spec_d(ux, 0), _spec_d(uy, 1), _spec_d(uy, 0)
    sxx, syy, sxy = 2 * nu * rho * dxux, 2 * nu * rho * dyuy, nu * rho * (dxuy + dyux)
    divx = _spec_d(sxx, 1) + _spec_d(sxy, 0)
    divy = _spec_d(sxy, 1) + _spec_d(syy, 0)
    expect_e = ux * divx + uy * divy
    got_e = (fl["e4"] + fl["e5"]).numpy()
    assert np.abs(got_e - expect_e).max() < 1e-6 * np.abs(expect_e).max()
    hx, hy = divx / rho, divy / rho
    om = dxuy - dyux
    expect_z = om * (_spec_d(hy, 1) - _spec_d(hx, 0))
    got_z = (fl["z4"] + fl["z5"]).numpy()
    assert np.abs(got_z - expect_z).max() < 1e-5 * np.abs(expect_z).max()


def test_kolmogorov_steady_state_closes_forced_balances():
    """Steady forced shear flow u_x = F0/(nu k*^2) sin(ky) with F_x = F0 sin(ky): the
    viscous force cancels the forcing, so e3 + e4 + e5 = 0 and z3 + z4 + z5 = 0
    pointwise (all other terms and both LHS vanish)."""
    n, nu, F0 = 64, 0.02, 1e-6
    k = 2 * math.pi * 2 / n
    kstar = 2 * sum(am * math.sin((m + 1) * k) for m, am in enumerate((4 / 5, -1 / 5, 4 / 105, -1 / 280)))
    idx = torch.arange(n, dtype=D)
    y, x = torch.meshgrid(idx, idx, indexing="ij")
    fx = F0 * torch.sin(k * y)
    fy = torch.zeros(n, n, dtype=D)
    ux = F0 / (nu * kstar ** 2) * torch.sin(k * y)
    uy = torch.zeros(n, n, dtype=D)
    rho = torch.ones(n, n, dtype=D)
    fl = ref.balance_fields([rho] * 3, [ux] * 3, [uy] * 3, fx, fy, nu)
    se = fl["e3"] + fl["e4"] + fl["e5"]
    sz = fl["z3"] + fl["z4"] + fl["z5"]
    assert float(fl["e3"].abs().max()) > 0 and float(fl["z3"].abs().max()) > 0
    assert float(se.abs().max()) < 1e-5 * float(fl["e3"].abs().max())
    assert float(sz.abs().max()) < 1e-5 * float(fl["z3"].abs().max())
    for key in ("lhs_E", "e1", "e2", "lhs_Z", "z1", "z2"):
        assert float(fl[key].abs().max()) < 1e-10 * float(fl["e3"].abs().max()), key


def test_acoustic_wave_pressure_work():
    """Linear standing sound wave rho = 1 + eps cos(kx) cos(W t), u = eps c_s sin(kx) sin(W t),
    W = c_s k*: the kinetic-energy change is the pressure work, d_t E = e2 = -u.grad p with
    p = c_s^2 rho (Eq. 8), to O(eps) and the BDF2 error."""
    nx, ny, eps = 256, 8, 1e-5
    k = 2 * math.pi / nx
    kstar = 2 * sum(am * math.sin((m + 1) * k) for m, am in enumerate((4 / 5, -1 / 5, 4 / 105, -1 / 280)))
    wfreq = math.sqrt(1 / 3) * kstar
    xs = torch.arange(nx, dtype=D)[None, :].expand(ny, nx)
    t0 = 37.0
    rho, ux, uy = [], [], []
    for t in (t0 - 2, t0 - 1, t0):
        rho.append(1 + eps * torch.cos(k * xs) * math.cos(wfreq * t))
        ux.append(eps * math.sqrt(1 / 3) * torch.sin(k * xs) * math.sin(wfreq * t))
        uy.append(torch.zeros(ny, nx, dtype=D))
    fl = ref.balance_fields(rho, ux, uy, None, None, nu=0.0)
    scale = float(fl["e2"].abs().max())
    assert scale > 0
    # BDF2 error on sin^2(W t): (2W)^2/3 ~ 2.7e-4 relative
    assert float((fl["lhs_E"] - fl["e2"]).abs().max()) < 1e-3 * scale


# ---------------------------------------------------------------------------
# The paper's own forced set-up: exact-difference forcing, Eqs. 14-16
# ---------------------------------------------------------------------------
def _near_eq_populations(ny, nx, seed):
    g = torch.Generator().manual_seed(seed)
    rho = 1 + 0.02 * torch.randn(ny, nx, generator=g, dtype=D)
    ux = 0.05 * torch.randn(ny, nx, generator=g, dtype=D)
    uy = 0.05 * torch.randn(ny, nx, generator=g, dtype=D)
    f = ref.equilibrium(rho, ux, uy) + 1e-3 * torch.randn(9, ny, nx, generator=g, dtype=D)
    return f, g


def test_edm_collision_conserves_mass_and_adds_the_force():
    """Per site: sum_l (f* - f) = 0 and sum_l c_l (f* - f) = F, the total force (turbulent
    force plus the damping of the large scales), to rounding."""
    f, g = _near_eq_populations(24, 32, 5)
    fx = 1e-3 * torch.randn(24, 32, generator=g, dtype=D)
    fy = 1e-3 * torch.randn(24, 32, generator=g, dtype=D)
    post = ref.edm_collide(f, 0.53, fx, fy, amp=0.4)
    _, _, _, Fx, Fy = ref.edm_total_force(f, fx, fy, amp=0.4)
    d = post - f
    assert float(d.sum(0).abs().max()) < 1e-15
    jx = sum(cx * d[l] for l, (cx, _) in enumerate(ref.C))
    jy = sum(cy * d[l] for l, (_, cy) in enumerate(ref.C))
    assert float((jx - Fx).abs().max()) < 1e-15
    assert float((jy - Fy).abs().max()) < 1e-15
    # with the damping off the total force is the given field
    _, _, _, Gx, Gy = ref.edm_total_force(f, fx, fy, amp=0.0)
    assert torch.equal(Gx, fx) and torch.equal(Gy, fy)


def test_edm_equilibrium_is_fixed_without_force():
    g = torch.Generator().manual_seed(6)
    rho = 1 + 0.02 * torch.randn(16, 16, generator=g, dtype=D)
    ux = 0.05 * torch.randn(16, 16, generator=g, dtype=D)
    uy = 0.05 * torch.randn(16, 16, generator=g, dtype=D)
    feq = ref.equilibrium(rho, ux, uy)
    assert float((ref.edm_collide(feq, 0.7) - feq).abs().max()) < 1e-15


def test_edm_velocity_shift_is_the_equilibrium_difference():
    """The forcing term is f^eq(rho, u + F/rho) - f^eq(rho, u) exactly: for tau = 1 the
    post-collision populations are the equilibrium at the shifted velocity."""
    f, g = _near_eq_populations(8, 12, 7)
    fx = 1e-3 * torch.randn(8, 12, generator=g, dtype=D)
    fy = 1e-3 * torch.randn(8, 12, generator=g, dtype=D)
    rho = f.sum(0)
    jx, jy = ref.momentum(f)
    want = ref.equilibrium(rho, (jx + fx) / rho, (jy + fy) / rho)
    assert float((ref.edm_collide(f, 1.0, fx, fy) - want).abs().max()) < 1e-15


def _count_shell(kmin, kmax):
    # independent count: for each k_x the k_y range from the circle inequalities
    n = 0
    r = int(math.floor(kmax))
    for kx in range(-r, r + 1):
        hi = math.floor(math.sqrt(kmax * kmax - kx * kx) + 1e-12)
        lo2 = kmin * kmin - kx * kx
        lo = 0 if lo2 <= 0 else math.ceil(math.sqrt(lo2) - 1e-12)
        n += sum(1 for ky in range(-hi, hi + 1) if abs(ky) >= lo)
    return n


def test_wavevector_shells():
    """12 wavevectors with 1 <= |k| <= 2 (the damped large scales of Eq. 16) and 80 with
    5 <= |k| <= 7 (the turbulent forcing of Eq. 14), counted two ways."""
    assert len(ref.wavevectors(1.0, 2.0)) == _count_shell(1.0, 2.0) == 12
    assert len(ref.wavevectors(5.0, 7.0)) == _count_shell(5.0, 7.0) == 80
    assert sorted(ref.wavevectors(5.0, 7.0)) == sorted(inp.shell_vectors(5.0, 7.0))


def test_shell_projection_keeps_exactly_the_shell():
    """A field built from modes inside and outside 1 <= |k| <= 2: the projection returns the
    inside part, and the damping force is -amp times it."""
    n = 32
    y, x = torch.meshgrid(torch.arange(n, dtype=D), torch.arange(n, dtype=D), indexing="ij")
    w = 2 * math.pi / n
    inside = 0.3 * torch.cos(w * x) + 0.2 * torch.sin(w * (x + y) + 0.4) - 0.1 * torch.cos(2 * w * y + 1.0)
    outside = 0.25 * torch.sin(w * (2 * x + y)) + 0.05 * torch.cos(3 * w * x) + 0.7
    p = ref.shell_projection(inside + outside)
    assert float((p - inside).abs().max()) < 1e-14
    fx, fy = ref.damping_force(inside + outside, outside, 0.65536)
    assert float((fx + 0.65536 * inside).abs().max()) < 1e-14
    assert float(fy.abs().max()) < 1e-14


def test_paper_amplitudes():
    """The printed amplitudes of Sec. 3 and the lattice amplitude of the workload."""
    assert inp.PAPER_FORCING_F0 == 8e-4 and inp.PAPER_DAMPING_F0 == 1e-5
    assert inp.PAPER_DAMPING_SHELL == (1.0, 2.0)
    assert inp.PAPER_FORCING_F0_LATTICE == pytest.approx(6e-6, rel=1e-12)
    # the damping of one in-shell mode is the rate times the mode (normalised coefficients)
    n = 32
    y, x = torch.meshgrid(torch.arange(n, dtype=D), torch.arange(n, dtype=D), indexing="ij")
    u = 0.01 * torch.cos(2 * math.pi * (x + y) / n)
    fx, _ = ref.damping_force(u, torch.zeros_like(u), inp.PAPER_DAMPING_F0)
    assert float((fx + 1e-5 * u).abs().max()) < 1e-20


def test_paper_forcing_is_the_curl_of_its_stream_function():
    """F^T = (d_y Psi, -d_x Psi) with Psi = F0 sum cos(2 pi k.x/256 + phi) (Eqs. 14-15):
    checked against spectral derivatives of Psi built independently, and divergence-free."""
    n, f0, ph = 64, 8e-4, 0.3
    fx, fy = inp.paper_forcing(n, f0=f0, kmin=5.0, kmax=7.0, phase=ph)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    psi = np.zeros((n, n))
    for kx, ky in ref.wavevectors(5.0, 7.0):
        psi += f0 * np.cos(2 * np.pi * (kx * x + ky * y) / n + ph)
    assert np.abs(fx - _spec_d(psi, 0)).max() < 1e-12 * np.abs(fx).max()
    assert np.abs(fy + _spec_d(psi, 1)).max() < 1e-12 * np.abs(fy).max()
    div = _spec_d(fx, 1) + _spec_d(fy, 0)
    assert np.abs(div).max() < 1e-12 * np.abs(fx).max()


def test_edm_run_with_damping_conserves_global_momentum():
    """The turbulent force and the damping both have zero domain mean, so the exact-
    difference scheme keeps the total momentum (and mass) to rounding over many steps."""
    n = 32
    fx, fy = inp.paper_forcing(n, f0=1e-4)
    fx, fy = ref.t64(fx), ref.t64(fy)
    f, _ = _near_eq_populations(n, n, 8)
    m0 = float(f.sum())
    j0 = [float(j.sum()) for j in ref.momentum(f)]
    f = ref.edm_run(f, 25, 0.56, fx, fy, amp=0.5)
    assert float(f.sum()) == pytest.approx(m0, rel=1e-13)
    j1 = [float(j.sum()) for j in ref.momentum(f)]
    assert abs(j1[0] - j0[0]) < 1e-12 and abs(j1[1] - j0[1]) < 1e-12
    # and the damping removes energy from the large scales: with amp the k = 1..2 content
    # of the velocity is smaller than without
    g, _ = _near_eq_populations(n, n, 8)
    a = ref.edm_run(g, 25, 0.56, fx, fy, amp=0.5)
    b = ref.edm_run(g, 25, 0.56, fx, fy, amp=0.0)
    ua = ref.edm_moments(a, fx, fy, 0.5)[1]
    ub = ref.edm_moments(b, fx, fy, 0.0)[1]
    assert float(ref.shell_projection(ua).abs().max()) < 0.5 * float(ref.shell_projection(ub).abs().max())


# ---------------------------------------------------------------------------
# Statistics as presented: histograms, Table-1 sampling, pooling, spectra
# ---------------------------------------------------------------------------
def test_histogram_bins_against_a_loop():
    """Bin 0 below the first edge, bin i in [e_{i-1}, e_i), the last bin at or above the
    last edge, NaN not counted; values exactly on an edge go to the bin it opens."""
    edges = [1e-3, 1e-2, 0.1, 1.0]
    g = torch.Generator().manual_seed(3)
    v = torch.cat([10 ** (-4 + 5 * torch.rand(500, generator=g, dtype=D)),
                   torch.tensor(edges, dtype=D), torch.tensor([float("nan"), 0.0, 5.0], dtype=D)])
    want = [0] * (len(edges) + 1)
    for x in v.tolist():
        if x != x:
            continue
        b = 0
        while b < len(edges) and x >= edges[b]:
            b += 1
        want[b] += 1
    got = ref.histogram(v, torch.tensor(edges, dtype=D))
    assert got.tolist() == want
    assert int(got.sum()) == 506


def test_sampled_window_errors_against_brute_force():
    """Errors of windows at random corners (modulo the grid) equal the errors of box means
    taken by a double loop."""
    lv = inp.balance_levels(24, seed=4)
    f = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], lv["fx"], lv["fy"], 0.004)
    corners = [(0, 0), (23, 5), (7, 19), (24 + 3, -2)]
    dE, dZ, ma = ref.sampled_errors(f, 6, corners)
    for i, (x0, y0) in enumerate(corners):
        m = {k: torch.tensor(ref.box_mean_brute(v, 6, y0 % 24, x0 % 24), dtype=D) for k, v in f.items()}
        e, z, a = ref.balancing_errors(m)
        assert float(abs(dE[i] - e)) <= 1e-12 * float(e) and float(abs(dZ[i] - z)) <= 1e-12 * float(z)
        assert float(abs(ma[i] - a)) <= 1e-13 * float(a)


def test_table1_counts_and_corners():
    """Table 1 on 256^2: 1 whole-domain box, 1000 for 100 <= L < 256, 5000 for 10 <= L < 100,
    10000 below; corners uniform on the grid and reproducible from the seed."""
    assert [inp.table1_count(L) for L in (256, 255, 100, 99, 10, 9, 1)] == \
        [1, 1000, 1000, 5000, 5000, 10000, 10000]
    c, n = inp.table1_corners(256, (3, 181, 256), seed=5)
    assert n == [10000, 1000, 1] and c.shape == (11001, 2) and c.dtype == np.int32
    assert c.min() >= 0 and c.max() < 256 and tuple(c[-1]) == (0, 0)
    c2, _ = inp.table1_corners(256, (3, 181, 256), seed=5)
    assert np.array_equal(c, c2)
    assert abs(c[:10000].mean() - 127.5) < 3  # uniform over [0, 256)


def test_pooled_statistics_merge():
    """Pooling two configurations equals the pairwise merge of their counts, means and
    second moments (Chan et al.'s formula, written out here)."""
    g = torch.Generator().manual_seed(8)
    a = torch.rand(300, generator=g, dtype=D)
    b = 2 + torch.rand(500, generator=g, dtype=D)
    b[7] = float("nan")
    p = ref.pooled_stats([a, b])
    bf = b[torch.isfinite(b)]
    na, nb = a.numel(), bf.numel()
    ma, mb = float(a.mean()), float(bf.mean())
    m2a = float(((a - ma) ** 2).sum())
    m2b = float(((bf - mb) ** 2).sum())
    n = na + nb
    mean = (na * ma + nb * mb) / n
    m2 = m2a + m2b + (mb - ma) ** 2 * na * nb / n
    assert p["count"] == n and p["n_nan"] == 1
    assert p["mean"] == pytest.approx(mean, rel=1e-14)
    assert p["std"] == pytest.approx(math.sqrt(m2 / n), rel=1e-13)


def test_shell_index_rounds_half_up_exactly():
    for kx in range(-40, 41):
        for ky in range(-40, 41):
            k2 = kx * kx + ky * ky
            s = int(ref.shell_index(torch.tensor(kx), torch.tensor(ky)))
            assert (2 * s - 1) ** 2 <= 4 * k2 < (2 * s + 1) ** 2 or (s == 0 and k2 == 0)


def test_energy_spectrum_single_modes_parseval_and_direct_sum():
    """A single mode puts its energy in its shell; the spectrum sums to half the mean |u|^2
    (Parseval); on an 8 x 12 grid it equals the spectrum from an explicit double-loop DFT."""
    n = 32
    y, x = torch.meshgrid(torch.arange(n, dtype=D), torch.arange(n, dtype=D), indexing="ij")
    ux = 0.3 * torch.cos(2 * math.pi * (3 * x + 4 * y) / n)   # |k| = 5
    uy = 0.2 * torch.sin(2 * math.pi * 7 * x / n)             # |k| = 7
    e = ref.energy_spectrum(ux, uy, 30)
    assert float(e[5]) == pytest.approx(0.3 ** 2 / 4, rel=1e-13)
    assert float(e[7]) == pytest.approx(0.2 ** 2 / 4, rel=1e-13)
    assert float(e.sum() - e[5] - e[7]) < 1e-28
    g = torch.Generator().manual_seed(9)
    vx = torch.randn(n, n, generator=g, dtype=D)
    vy = torch.randn(n, n, generator=g, dtype=D)
    e = ref.energy_spectrum(vx, vy, 40)
    assert float(e.sum()) == pytest.approx(0.5 * float((vx ** 2 + vy ** 2).mean()), rel=1e-13)
    ny, nx = 8, 12
    vx, vy = vx[:ny, :nx], vy[:ny, :nx]
    want = [0.0] * 12
    for ky in range(ny):
        for kx in range(nx):
            fx = kx if kx < nx / 2 else kx - nx   # signed frequencies (nx/2 counts as -nx/2)
            fy = ky if ky < ny / 2 else ky - ny
            cx = sum(complex(math.cos(-2 * math.pi * (kx * i / nx + ky * j / ny)),
                             math.sin(-2 * math.pi * (kx * i / nx + ky * j / ny))) * float(vx[j, i])
                     for j in range(ny) for i in range(nx)) / (nx * ny)
            cy = sum(complex(math.cos(-2 * math.pi * (kx * i / nx + ky * j / ny)),
                             math.sin(-2 * math.pi * (kx * i / nx + ky * j / ny))) * float(vy[j, i])
                     for j in range(ny) for i in range(nx)) / (nx * ny)
            k2 = fx * fx + fy * fy
            s = 0
            while (2 * s + 1) ** 2 <= 4 * k2:
                s += 1
            want[s] += 0.5 * (abs(cx) ** 2 + abs(cy) ** 2)
    got = ref.energy_spectrum(vx, vy, 12)
    for s in range(12):
        assert float(got[s]) == pytest.approx(want[s], rel=1e-12, abs=1e-17), s


# ---------------------------------------------------------------------------
# Entropic LBM: minimiser of H, alpha from the entropy equality, variable viscosity
# ---------------------------------------------------------------------------
def test_entropic_equilibrium_is_the_constrained_minimiser():
    """Moments rho, rho u exactly; log(f_l / t_l) affine in c_l (the conditions for a minimum
    of Eq. 6 under mass and momentum constraints); the textbook polynomial equilibrium to
    second order in u (difference O(u^3))."""
    g = torch.Generator().manual_seed(12)
    rho = 1 + 0.05 * torch.randn(6, 7, generator=g, dtype=D)
    ux = 0.1 * torch.randn(6, 7, generator=g, dtype=D)
    uy = 0.1 * torch.randn(6, 7, generator=g, dtype=D)
    f = ref.entropic_equilibrium(rho, ux, uy)
    assert float((f.sum(0) - rho).abs().max()) < 1e-15
    jx, jy = ref.momentum(f)
    assert float((jx - rho * ux).abs().max()) < 1e-15 and float((jy - rho * uy).abs().max()) < 1e-15
    lg = [torch.log(f[l] / ref.W[l]) for l in range(9)]
    bx, by = lg[1] - lg[0], lg[2] - lg[0]
    for l, (cx, cy) in enumerate(ref.C):
        assert float((lg[l] - lg[0] - cx * bx - cy * by).abs().max()) < 1e-14, l
    for s in (1e-2, 2e-2, 4e-2):
        d = float((ref.entropic_equilibrium(rho, s * ux / 0.1, s * uy / 0.1)
                   - ref.equilibrium(rho, s * ux / 0.1, s * uy / 0.1)).abs().max())
        if s == 1e-2:
            d1 = d
    assert d / d1 == pytest.approx(64, rel=0.05)  # cubic: 4x the velocity, 64x the difference


def test_entropic_gain_equals_the_literal_h_difference():
    """The rearranged H(f + a delta) - H(f) equals the difference of Eq. 6 summed exactly
    (math.fsum of the 18 per-population terms) at every site."""
    rho, ux, uy = inp.spectrum_velocity(16, seed=2, max_mach=0.15)
    f = ref.run(ref.init_populations(rho, ux, uy), 15, 0.52)
    feq = ref.entropic_equilibrium(ref.density(f), *[j / ref.density(f) for j in ref.momentum(f)])
    delta = feq - f
    for a in (0.7, 1.9, 2.3):
        got = ref.entropic_gain(f, delta, a)
        for (y, x) in [(0, 0), (3, 11), (15, 7), (8, 8)]:
            terms = []
            for l in range(9):
                fl, dl = float(f[l, y, x]), float(delta[l, y, x])
                terms.append((fl + a * dl) * math.log((fl + a * dl) / ref.W[l]))
                terms.append(-fl * math.log(fl / ref.W[l]))
            want = math.fsum(terms)
            assert float(got[y, x]) == pytest.approx(want, rel=1e-6, abs=1e-17), (a, y, x)


def test_entropic_alpha_entropy_equality_and_limits():
    """alpha solves the entropy equality, exceeds 1, is 2 at equilibrium and tends to 2 as
    the populations approach it (|alpha - 2| = O(epsilon))."""
    rho, ux, uy = inp.spectrum_velocity(16, seed=3, max_mach=0.15)
    f = ref.run(ref.init_populations(rho, ux, uy), 15, 0.51)
    r = ref.density(f)
    jx, jy = ref.momentum(f)
    feq = ref.entropic_equilibrium(r, jx / r, jy / r)
    a = ref.entropic_alpha(f, feq)
    assert float(a.min()) > 1.0
    scale = float((((feq - f) ** 2) / f).sum(0).max())
    assert float(ref.entropic_gain(f, feq - f, a).abs().max()) < 1e-12 * scale
    assert torch.equal(ref.entropic_alpha(feq, feq), torch.full_like(a, 2.0))
    devs = []
    for eps in (1e-2, 1e-3, 1e-4):
        fe = feq + eps * (f - feq)
        devs.append(float((ref.entropic_alpha(fe, feq) - 2).abs().max()))
    assert devs[1] < 0.2 * devs[0] and devs[2] < 0.2 * devs[1]


def test_entropic_collision_conserves_and_reduces_to_lbgk():
    rho, ux, uy = inp.spectrum_velocity(16, seed=4, max_mach=0.15)
    f = ref.run(ref.init_populations(rho, ux, uy), 10, 0.53)
    fp, a = ref.entropic_collide(f, 0.53)
    assert float((fp.sum(0) - f.sum(0)).abs().max()) < 1e-15
    for jp, j in zip(ref.momentum(fp), ref.momentum(f)):
        assert float((jp - j).abs().max()) < 1e-15
    r = ref.density(f)
    jx, jy = ref.momentum(f)
    feq = ref.entropic_equilibrium(r, jx / r, jy / r)
    # the step along feq - f is alpha / (2 tau0) of it; alpha = 2 is the LBGK step
    assert float((fp - (f + a * (feq - f) / (2 * 0.53))).abs().max()) < 1e-16
    assert ref.effective_viscosity(torch.tensor(2.0, dtype=D), 0.53) == pytest.approx(0.01, rel=1e-13)
    assert float(ref.effective_viscosity(a, 0.53).max()) > 0


def test_balance_with_a_viscosity_field():
    """A constant field equals the scalar; with a varying field, e4 + e5 = u . div(sigma)
    and z4 + z5 = omega curl(div(sigma) / rho) by spectral derivatives (sigma = rho nu(x) (du + du^T))."""
    rho, ux, uy = _smooth_compressible_fields(64, seed=6)
    lv = {"rho": [rho] * 3, "ux": [ux] * 3, "uy": [uy] * 3}
    a = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], None, None, 0.004)
    b = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], None, None, torch.full((64, 64), 0.004, dtype=D))
    for k in ref.TERM_NAMES:
        assert torch.equal(a[k], b[k]), k
    y, x = np.meshgrid(np.arange(64.0), np.arange(64.0), indexing="ij")
    nu = 0.004 * (1 + 0.3 * np.sin(2 * np.pi * (x + 2 * y) / 64))
    t = ref.balance_fields(lv["rho"], lv["ux"], lv["uy"], None, None, ref.t64(nu))
    r, u, v = [np.asarray(q, dtype=float) for q in (rho, ux, uy)]
    sxx = 2 * nu * r * _spec_d(u, 1)
    syy = 2 * nu * r * _spec_d(v, 0)
    sxy = nu * r * (_spec_d(v, 1) + _spec_d(u, 0))
    divx = _spec_d(sxx, 1) + _spec_d(sxy, 0)
    divy = _spec_d(sxy, 1) + _spec_d(syy, 0)
    want = u * divx + v * divy
    got = (t["e4"] + t["e5"]).numpy()
    assert np.abs(got - want).max() < 1e-5 * np.abs(want).max()


def test_global_enstrophy_of_a_taylor_green_field():
    """1/2 sum omega^2 for u = u0 (-cos kx sin ky, sin kx cos ky): omega = 2 u0 k* cos kx cos ky
    with the modified wavenumber of Eq. 18, k* = (2/5)(4 sin k - sin 2k + (4/21) sin 3k
    - (1/56) sin 4k), so the total is u0^2 k*^2 N^2 / 2; a uniform flow has none."""
    n, u0 = 48, 0.02
    k = 2 * math.pi / n
    kstar = 0.4 * (4 * math.sin(k) - math.sin(2 * k) + (4 / 21) * math.sin(3 * k) - math.sin(4 * k) / 56)
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    got = ref.global_enstrophy(ux, uy)
    assert got == pytest.approx(0.5 * u0 ** 2 * kstar ** 2 * n * n, rel=1e-12)
    assert ref.global_enstrophy(np.full((n, n), 0.03), np.full((n, n), -0.01)) == pytest.approx(0.0, abs=1e-25)
    # a shifted field has the same total
    assert ref.global_enstrophy(np.roll(ux, 5, 1), np.roll(uy, 5, 1)) == pytest.approx(got, rel=1e-13)
