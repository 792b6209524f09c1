"""GPU parity of the three-dimensional extension (D3Q19 and D3Q27 LBGK with Guo's forcing term, the
3D energy and enstrophy balances with the vortex-stretching term over cubic sub-volumes)
against the FP64 oracle (oracle/ref3d.py) on identical seeded inputs.

Tolerances.  Moments: FP64 storage within 1e-12 of the field's max |value|, FP32 within
1e-5 (as the 2D step).  Balance: the oracle's own sensitivity to a relative perturbation of
its inputs at the level the moments of the two runs differ (at least 1e-15) gives kappa per
term field and per statistic; terms must agree within max(1e-12, 30 kappa), statistics within
max(1e-9, 30 kappa) relative, window and NaN counts exactly.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from helpers import moment_err, moment_tol, rel_err
from oracle import ref3d

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def Sim3(*a, **k):
    from paper_1809_06735_amd import Simulation3D
    return Simulation3D(*a, **k)


def _oracle_run(fields, tau, steps, force, q=19):
    f = ref3d.init_populations(*fields, q=q)
    F = [ref3d.t64(a) for a in force] if force is not None else [None] * 3
    return ref3d.run_with_history(f, steps, tau, *F)


@pytest.mark.parametrize("lattice", ["d3q19", "d3q27"])
@pytest.mark.parametrize("shape", [(16, 20, 24), (17, 16, 272)])
@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
@pytest.mark.parametrize("forced", [False, True])
def test_3d_step_parity(gpu_lib, shape, dtype, tol, forced, lattice):
    """rho, u after 25 steps on a non-cubic grid (a ragged x extent, one and two workgroups
    per row) against the oracle on the same lattice; the scalars against the oracle's sums."""
    tau, steps = 0.56, 25
    q = 27 if lattice == "d3q27" else 19
    fields = inp.fields3(shape, seed=sum(shape), max_mach=0.15)
    force = inp.force3(shape, seed=3, amp=2e-5) if forced else None
    say(f"3d step {lattice} {shape} {dtype} forced={forced}")
    kw = dict(fx=force[0], fy=force[1], fz=force[2]) if forced else {}
    sim = Sim3(*fields, tau, dtype=dtype, lattice=lattice, **kw)
    sim.step(steps)
    r, vx, vy, vz, sc = sim.moments()
    _, hist = _oracle_run(fields, tau, steps, force, q)
    want = hist[-1]
    for name, g, w in zip(("rho", "ux", "uy", "uz"), (r, vx, vy, vz), want):
        e = moment_err(name, g, w, dtype)
        tol_f = moment_tol(name, want, dtype, steps, tol, q)
        say(f"  {name}: {e:.1e} (tol {tol_f:.1e})")
        assert e < tol_f, (name, e, tol_f)
    assert sc["time"] == steps
    assert abs(sc["mass"] - float(want[0].sum())) <= 1e-12 * float(want[0].sum()) * (1 if dtype == "f64" else 1e5)
    assert sc["nonfinite"] == 0 and sc["min_rho"] > 0


def test_3d_conservation_and_momentum_input(gpu_lib):
    """Unforced: mass and momentum stay at their initial totals to rounding (every D3Q19
    collision conserves them); forced: total momentum grows by sum(F) per step (Guo's term
    with the half-force velocity adds exactly F per step)."""
    shape = (32, 32, 32)
    fields = inp.fields3(shape, seed=11, max_mach=0.1)
    sim = Sim3(*fields, 0.52, dtype="f64")
    s0 = sim.moments()[-1]
    sim.step(100)
    s1 = sim.moments()[-1]
    assert abs(s1["mass"] - s0["mass"]) <= 1e-12 * s0["mass"]
    for k in ("mom_x", "mom_y", "mom_z"):
        assert abs(s1[k] - s0[k]) <= 1e-12 * s0["mass"] * 0.1, (k, s0[k], s1[k])
    # modes of zero mean plus a uniform part, so that the total force is not zero
    force = [f + c for f, c in zip(inp.force3(shape, seed=4, amp=1e-5), (2e-6, -1e-6, 5e-7))]
    fsum = [float(np.sum(f)) for f in force]
    sim = Sim3(*fields, 0.52, dtype="f64", fx=force[0], fy=force[1], fz=force[2])
    s0 = sim.moments()[-1]
    sim.step(50)
    s1 = sim.moments()[-1]
    for k, fs in zip(("mom_x", "mom_y", "mom_z"), fsum):
        # the reported momentum is rho u = j + F/2 at both ends: the difference is 50 sum(F)
        assert abs((s1[k] - s0[k]) - 50 * fs) <= 1e-10 * abs(50 * fs) + 1e-12 * s0["mass"] * 0.1, (
            k, s1[k] - s0[k], 50 * fs)


def _terms(hist, F, nu):
    return ref3d.balance_fields([h[0] for h in hist], [h[1] for h in hist], [h[2] for h in hist],
                                [h[3] for h in hist], *F, nu)


def _sensitivity(hist, F, nu, sizes, rel, seed=0):
    """Oracle term fields and statistics, and their relative change under a perturbation of
    every input by a factor 1 + rel * N(0, 1)."""
    base = _terms(hist, F, nu)
    rng = np.random.default_rng(seed)

    def pert(a):
        a = np.asarray(a)
        return ref3d.t64(a * (1 + rel * rng.standard_normal(a.shape)))

    ph = [tuple(pert(a) for a in h) for h in hist]
    pF = [None if f is None else pert(f) for f in F]
    p2 = _terms(ph, pF, nu)
    kt = {k: float((p2[k] - base[k]).abs().max() / (base[k].abs().max() or 1.0)) for k in ref3d.TERM_NAMES}
    want = ref3d.subvolume_balance(base, sizes)
    alt = ref3d.subvolume_balance(p2, sizes)
    ks = []
    for w, a in zip(want, alt):
        ks.append({q: {k: (abs(a[q][k] - w[q][k]) / max(abs(w[q][k]), 1e-300) if w[q]["count"] else 0.0)
                       for k in ("mean", "std", "min", "max")} for q in ("dE", "dZ", "Ma")})
    return base, want, kt, ks


def _compare_stats(got, want, kappa, label):
    assert got["L"] == want["L"]
    for q in ("dE", "dZ", "Ma"):
        g, w = got[q], want[q]
        assert g["count"] == w["count"], (label, q, g, w)
        if q != "Ma":
            assert g["n_nan"] == w["n_nan"], (label, q)
        if w["count"] == 0:
            continue
        for k in ("mean", "std", "min", "max"):
            r = max(1e-9, 30 * kappa[q][k])
            assert abs(g[k] - w[k]) <= r * max(abs(w[k]), 1e-300), (label, q, k, g[k], w[k], r)


@pytest.mark.parametrize("shape,sizes,forced,lattice", [((20, 20, 20), (1, 3, 8, 19, 20), True, "d3q19"),
                                                         ((16, 20, 24), (1, 5, 16), False, "d3q19"),
                                                         ((16, 16, 272), (2, 9, 16), True, "d3q19"),
                                                         ((20, 20, 20), (1, 4, 20), True, "d3q27")])
def test_3d_balance_parity(gpu_lib, shape, sizes, forced, lattice):
    """Balance of an FP64 run: the 14 integrand fields (with the stretching term z6) and the
    per-size statistics over every cube corner, against the oracle's run on the same lattice."""
    tau, steps = 0.53, 20
    q = 27 if lattice == "d3q27" else 19
    fields = inp.fields3(shape, seed=5 + shape[2], max_mach=0.2)
    force = inp.force3(shape, seed=9, amp=3e-5) if forced else None
    kw = dict(fx=force[0], fy=force[1], fz=force[2]) if forced else {}
    say(f"3d balance {lattice} {shape} sizes={sizes} forced={forced}")
    sim = Sim3(*fields, tau, dtype="f64", with_balance=True, lattice=lattice, **kw)
    sim.step(steps)
    res = sim.balance(sizes, term_fields=True)
    _, hist = _oracle_run(fields, tau, steps, force, q)
    r, vx, vy, vz, _ = sim.moments()
    dmom = max(rel_err(g, w) for g, w in zip((r, vx, vy, vz), hist[-1]))
    assert dmom < TOL64
    F = [None] * 3 if force is None else [ref3d.t64(f) for f in force]
    flds, want, kt, ks = _sensitivity(hist, F, (tau - 0.5) / 3, sizes, max(dmom, 1e-15))
    for name in ref3d.TERM_NAMES:
        e = rel_err(res["terms"][name], flds[name])
        tol = max(1e-12, 30 * kt[name])
        say(f"  {name}: {e:.1e} (tol {tol:.1e})")
        assert e <= tol, (name, e, tol)
    assert float(flds["z6"].abs().max()) > 1e-12  # the stretching term is really exercised
    for got, w, kk in zip(res["stats"], want, ks):
        say(f"  L={w['L']}: dE mean {got['dE']['mean']:.6e} / {w['dE']['mean']:.6e}, "
            f"dZ mean {got['dZ']['mean']:.6e} / {w['dZ']['mean']:.6e}")
        _compare_stats(got, w, kk, f"{shape} L={w['L']}")


def test_3d_cube_windows_properties(gpu_lib):
    """Properties of the cube windows that hold at any size, checked on the library's own
    term fields: L = 1 windows are the sites themselves (Ma_V extremes are those of
    sqrt(|u|^2) / c_s), L = N is the one whole-domain cube (its Ma_V and delta^E from the
    domain means), and every L in between has N^3 windows."""
    n = 24
    shape = (n, n, n)
    sizes = (1, 2, 7, 13, 23, 24)
    fields = inp.fields3(shape, seed=21, max_mach=0.2)
    force = inp.force3(shape, seed=2, amp=5e-5)
    sim = Sim3(*fields, 0.6, dtype="f64", with_balance=True, fx=force[0], fy=force[1], fz=force[2])
    sim.step(6)
    res = sim.balance(sizes, term_fields=True)
    tf = {k: v.double().cpu() for k, v in res["terms"].items()}
    ma = tf["usq"].sqrt() * 3 ** 0.5
    st = res["stats"]
    assert abs(st[0]["Ma"]["max"] - float(ma.max())) <= 1e-9 * float(ma.max())
    assert abs(st[0]["Ma"]["min"] - float(ma.min())) <= 1e-9 * float(ma.max())
    for s in st[:-1]:
        assert s["dE"]["count"] + s["dE"]["n_nan"] == n ** 3 and s["Ma"]["count"] == n ** 3
    whole = st[-1]
    assert whole["Ma"]["count"] == 1 and whole["dE"]["count"] + whole["dE"]["n_nan"] == 1
    m = {k: float(v.mean()) for k, v in tf.items()}
    assert abs(whole["Ma"]["mean"] - (m["usq"] ** 0.5) * 3 ** 0.5) <= 1e-9 * whole["Ma"]["mean"]
    rhs = sum(m[k] for k in ("e1", "e2", "e3", "e4", "e5"))
    den = max(abs(m[k]) for k in ("e1", "e2", "e3", "e4", "e5"))
    d_e = abs(rhs - m["lhs_E"]) / den
    assert abs(whole["dE"]["mean"] - d_e) <= 1e-6 * d_e + 1e-12, (whole["dE"]["mean"], d_e)


def test_d3q27_runs_one_step_per_launch(gpu_lib):
    """A D3Q27 handle refuses the multi-step shapes (written for D3Q19), its autotuner keeps
    one step per launch, and D3Q27 differs from D3Q19 on a fully three-dimensional field
    (the corner populations matter)."""
    from paper_1809_06735_amd import _lib as L
    shape = (16, 16, 32)
    fields = inp.fields3(shape, seed=2, max_mach=0.15)
    s27 = Sim3(*fields, 0.6, dtype="f64", lattice="d3q27")
    with pytest.raises(L.LBMError):
        s27.set_tile(2, 64, 4, 8)
    assert s27.autotune(2)[0] == 1
    s27.step(10)
    s19 = Sim3(*fields, 0.6, dtype="f64")
    s19.step(10)
    a, b = s27.moments(scalars=False), s19.moments(scalars=False)
    assert max(rel_err(x, y) for x, y in zip(a, b)) > 1e-6


def test_3d_errors(gpu_lib):
    from paper_1809_06735_amd import _lib as L
    shape = (16, 16, 16)
    fields = inp.fields3(shape, seed=1)
    sim = Sim3(*fields, 0.6, dtype="f32", with_balance=True)
    with pytest.raises(L.LBMError) as e:
        sim.balance((4,))
    assert e.value.code == L.LBM_E_STATE
    sim.step(2)
    with pytest.raises(L.LBMError) as e:
        sim.balance((17,))
    assert e.value.code == L.LBM_E_INVALID
    assert sim.balance((4,))["stats"][0]["L"] == 4
    plain = Sim3(*fields, 0.6, dtype="f32")
    plain.step(3)
    with pytest.raises(L.LBMError) as e:
        plain.balance((4,))
    assert e.value.code == L.LBM_E_STATE


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_3d_multistep_kernel_equals_single_steps(gpu_lib, dtype):
    """K = 2..4 steps per launch (tiles of lanes marching in z, levels exchanged through LDS)
    give bit-identical moments to one-step launches: forced and unforced, ragged tiles and
    bands (one plane), tiles wider than the grid, step counts that leave remainders."""
    from paper_1809_06735_amd import _lib as L
    shapes32 = [(2, 64, 4, 16), (2, 32, 8, 5), (3, 32, 8, 7), (3, 16, 16, 1), (4, 32, 16, 9), (4, 16, 16, 64),
                (2, 128, 4, 3), (3, 64, 8, 2)]
    shapes64 = [(2, 64, 4, 16), (2, 32, 8, 5), (3, 32, 8, 7), (3, 16, 16, 1), (4, 16, 16, 9)]
    for shape in ((16, 20, 24), (17, 16, 66)):
        fields = inp.fields3(shape, seed=41 + shape[2], max_mach=0.2)
        force = inp.force3(shape, seed=5, amp=3e-5)
        for forced in (False, True):
            kw = dict(fx=force[0], fy=force[1], fz=force[2]) if forced else {}
            base = Sim3(*fields, 0.54, dtype=dtype, **kw)
            base.step(13)
            want = base.moments(scalars=False)
            base.close()
            for tile in (shapes32 if dtype == "f32" else shapes64):
                s = Sim3(*fields, 0.54, dtype=dtype, **kw)
                s.set_tile(*tile)
                s.step(13)
                got = s.moments(scalars=False)
                for g, w in zip(got, want):
                    assert torch.equal(g, w), (shape, forced, tile)
                s.close()
            say(f"3d multi-step {dtype} {shape} forced={forced}: bit-identical")
    s = Sim3(*inp.fields3((16, 16, 16), seed=1), 0.6, dtype=dtype)
    for bad in ((5, 32, 8, 4), (2, 2, 64, 4), (4, 64, 4, 4), (2, 64, 4, 0), (2, 48, 1, 4), (2, 64, 16, 4)):
        with pytest.raises(L.LBMError):
            s.set_tile(*bad)


def test_3d_autotune_keeps_the_state(gpu_lib):
    shape = (32, 32, 64)
    fields = inp.fields3(shape, seed=8, max_mach=0.1)
    force = inp.force3(shape, seed=8, amp=1e-5)
    a = Sim3(*fields, 0.55, dtype="f32", fx=force[0], fy=force[1], fz=force[2])
    b = Sim3(*fields, 0.55, dtype="f32", fx=force[0], fy=force[1], fz=force[2])
    a.step(5)
    tile = a.autotune(2)
    say(f"3d autotuned shape {tile}")
    assert a.get_tile() == tile and 1 <= tile[0] <= 4
    a.step(20)
    b.step(25)
    for g, w in zip(a.moments(scalars=False), b.moments(scalars=False)):
        assert torch.equal(g, w)


def _wrap3(a, z0, y0, x0, size):
    a = np.asarray(a)
    nz, ny, nx = a.shape
    zs = (np.arange(size) + z0) % nz
    ys = (np.arange(size) + y0) % ny
    xs = (np.arange(size) + x0) % nx
    return a[np.ix_(zs, ys, xs)]


def test_3d_256_benchmark_run_on_oracle_patches(gpu_lib):
    """The 256^3 FP32 forced run the benchmark times (fields3 Ma 0.1, force3 amplitude 1e-6,
    tau 0.52, the autotuned launch shape): 12 steps, then rho, u on three 8^3 patches (one
    across the periodic corner) against the oracle run on periodic patches with a margin of
    steps + 1 cells on every side (information moves one cell per step, so the core is
    exactly what the full grid computes)."""
    n, tau, steps, core = 256, 0.52, 12, 8
    shape = (n, n, n)
    fields = inp.fields3(shape, seed=0, max_mach=0.1)
    force = inp.force3(shape, seed=0, amp=1e-6)
    say("3d 256^3 fp32 forced, autotune + 12 steps")
    sim = Sim3(*fields, tau, dtype="f32", fx=force[0], fy=force[1], fz=force[2])
    tile = sim.autotune(3)
    say(f"3d 256^3 autotuned shape {tile}")
    t0 = sim.time
    sim.step(steps)
    got = sim.moments(scalars=False)
    sim.close()
    # the autotuner advances the state; the oracle starts from the same initial fields and
    # runs t0 + steps steps
    total = t0 + steps
    m = total + 1
    for (z0, y0, x0) in ((250, 251, 249), (0, 128, 64), (100, 3, 200)):
        pf = [_wrap3(a, z0 - m, y0 - m, x0 - m, core + 2 * m) for a in fields]
        pF = [ref3d.t64(_wrap3(a, z0 - m, y0 - m, x0 - m, core + 2 * m)) for a in force]
        f = ref3d.run(ref3d.init_populations(*pf), total, tau, *pF)
        want = [w[m:m + core, m:m + core, m:m + core] for w in ref3d.macroscopic(f, *pF)]
        for name, g, w in zip(("rho", "ux", "uy", "uz"), got, want):
            e = moment_err(name, torch.as_tensor(_wrap3(g.cpu().numpy(), z0, y0, x0, core)), w, "f32")
            tol = moment_tol(name, want, "f32", total, TOL32)
            say(f"  patch ({z0},{y0},{x0}) {name} {e:.1e} (tol {tol:.1e})")
            assert e < tol, (name, e, tol)
