"""GPU parity of the paper's own forced set-up (Sec. 3, Eqs. 14-16): the exact-difference
step with a static force (the constant-phase stream-function force of Eqs. 14-15 or a
random one) and the spectral damping F^R of the modes kmin <= |k| <= kmax (Eq. 16), against
the FP64 oracle, which projects with FFTs where the library reduces direct Fourier sums.

Tolerances as for the Guo step: FP64 storage 1e-12 and FP32 storage 1e-5, both as
max |gpu - oracle| / max |oracle| per moment field; balance terms at the level that the
moment differences imply (perturbation of the oracle's own history).
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from helpers import moment_err, moment_tol, rel_err
from oracle import ref

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def Sim(*a, **k):
    from paper_1809_06735_amd import Simulation
    return Simulation(*a, **k)


def _fields(ny, nx, seed, mach=0.08):
    n = max(nx, ny)
    _, ux, uy = inp.spectrum_velocity(n, seed=seed, max_mach=mach)
    rng = np.random.default_rng(seed + 100)
    rho = 1.0 + 0.001 * rng.standard_normal((ny, nx))
    return rho, ux[:ny, :nx].copy(), uy[:ny, :nx].copy()


def _oracle(rho, ux, uy, steps, tau, fx, fy, amp, shell):
    f = ref.init_populations(rho, ux, uy)
    fxt = None if fx is None else ref.t64(fx)
    fyt = None if fy is None else ref.t64(fy)
    f = ref.edm_run(f, steps, tau, fxt, fyt, amp, *shell)
    return ref.edm_moments(f, fxt, fyt, amp, *shell)


def _check(sim, want, tol, label, dtype, steps):
    r, vx, vy, sc = sim.moments()
    for name, g, w in zip(("rho", "ux", "uy"), (r, vx, vy), want[:3]):
        e = moment_err(name, g, w, dtype)
        tol_f = moment_tol(name, want[:3], dtype, steps, tol)
        say(f"{label} {name} rel err {e:.2e} (tol {tol_f:.1e})")
        assert e < tol_f, (label, name, e, tol_f)
    return sc


def _run_case(ny, nx, dtype, steps, tau, amp, shell=(1.0, 2.0), force="random", seed=0, tol=TOL64,
              label="edm"):
    rho, ux, uy = _fields(ny, nx, seed)
    if force == "random":
        n = max(nx, ny)
        fx, fy = inp.forcing_field(n, seed=seed + 7, max_force=3e-5)
        fx, fy = fx[:ny, :nx].copy(), fy[:ny, :nx].copy()
    elif force == "paper":
        assert nx == ny
        fx, fy = inp.paper_forcing(nx)
    elif force == "paper-literal":
        assert nx == ny
        fx, fy = inp.paper_forcing(nx, f0=inp.PAPER_FORCING_F0)
    else:
        fx = fy = None
    f0 = amp
    say(f"{label}: {ny}x{nx} {dtype} {steps} steps tau {tau} amp {amp} shell {shell} force {force}")
    sim = Sim(rho, ux, uy, tau, dtype=dtype, fx=fx, fy=fy, scheme="edm", damp_f0=f0, damp_shell=shell)
    sim.step(steps)
    want = _oracle(rho, ux, uy, steps, tau, fx, fy, amp, shell)
    sc = _check(sim, want, tol, label, dtype, steps)
    assert sc["time"] == steps
    return sim, want


def test_edm_damped_fp64_nonsquare(gpu_lib):
    """FP64, 40 x 48, random static force plus damping of 1 <= |k| <= 2 at rate 0.5 per step."""
    _run_case(40, 48, "f64", 60, 0.56, 0.5, label="edm64 40x48")


def test_edm_paper_set_up_256(gpu_lib):
    """The paper's configuration on 256^2: the stream-function force on 5 <= |k| <= 7 with
    one phase (lattice amplitude of the workload), damping of 1 <= |k| <= 2 at the rate
    F0^R = 1e-5, tau0 = 0.52; FP64 and FP32 storage.  A second pair of runs takes the
    printed F0^T = 8e-4 in lattice units and a damping rate of 0.65 (both far stronger)
    so that every term is large."""
    amp = inp.PAPER_DAMPING_F0
    _run_case(256, 256, "f64", 30, 0.52, amp, force="paper", seed=3, label="paper256 f64")
    _run_case(256, 256, "f32", 30, 0.52, amp, force="paper", seed=3, tol=TOL32, label="paper256 f32")
    _run_case(256, 256, "f64", 30, 0.52, 0.65, force="paper-literal", seed=3, label="strong256 f64")
    _run_case(256, 256, "f32", 30, 0.52, 0.65, force="paper-literal", seed=3, tol=TOL32,
              label="strong256 f32")


@pytest.mark.parametrize("shell", [(1.0, 1.0), (2.0, 3.0), (0.5, 4.0)])
def test_edm_shells(gpu_lib, shell):
    """Other damped shells: |k| = 1 (2 modes of the half plane), 2 <= |k| <= 3 and every mode
    up to |k| = 4 (24 modes, the largest the library takes); odd grid extents."""
    _run_case(37, 44, "f64", 25, 0.6, 0.3, shell=shell, seed=5, label=f"shell {shell}")


def test_edm_without_damping(gpu_lib):
    """Exact-difference forcing with the static force only, and with no force at all (then
    it is the plain BGK step); FP64 and FP32."""
    _run_case(32, 64, "f64", 50, 0.53, 0.0, seed=8, label="edm force only f64")
    _run_case(32, 64, "f32", 50, 0.53, 0.0, seed=8, tol=TOL32, label="edm force only f32")
    _run_case(48, 32, "f64", 50, 0.7, 0.0, force=None, seed=9, label="edm unforced f64")


def test_edm_shapes_graphs_and_checkpoint_bitwise(gpu_lib):
    """Launch shapes, hipGraph replay and save/load change nothing: every variant gives the
    same bits as direct single launches of the default shape."""
    from paper_1809_06735_amd import _lib as L
    n = 64
    rho, ux, uy = _fields(n, n, 11)
    fx, fy = inp.paper_forcing(n, f0=1e-4)
    kw = dict(dtype="f32", fx=fx, fy=fy, scheme="edm", damp_f0=0.4)

    def run(tile=None, graph=0, steps=70, split=None):
        s = Sim(rho, ux, uy, 0.53, **kw)
        if tile is not None:
            s.set_tile(*tile)
        s.set_graph(graph)
        if split is None:
            s.step(steps)
        else:
            s.step(split)
            st = s.save()
            s.step(5)  # moved on, then restored
            s.load(st)
            s.step(steps - split)
        r, vx, vy = s.moments(scalars=False)
        return torch.stack([r, vx, vy]).cpu()

    base = run()
    for tile in [(64, 4, 1, 1, 0, 1, 0), (256, 1, 1, 3, 1, 1, 0), (128, 2, 1, 5, 0, 1, 0)]:
        assert torch.equal(run(tile), base), tile
    assert torch.equal(run(graph=8), base)
    assert torch.equal(run(split=31), base)
    s = Sim(rho, ux, uy, 0.53, **kw)
    with pytest.raises(L.LBMError):
        s.set_tile(128, 1, 1, 32, 0, 3, 1)  # multi-step shapes are for the Guo step
    with pytest.raises(L.LBMError):
        s.set_tile(64, 4, 2, 1, 0, 1, 0)  # one site per thread
    t = s.autotune(4)
    assert t[1] >= 1 and t[2] == 1 and t[5] == 1, t


def _edm_kappa(hist, nu, rel, seed=0):
    lv = [h[:3] for h in hist]
    fx, fy = hist[2][3], hist[2][4]
    base = ref.balance_fields([h[0] for h in lv], [h[1] for h in lv], [h[2] for h in lv], fx, fy, nu)
    rng = np.random.default_rng(seed)
    pert = [tuple(ref.t64(np.asarray(a) * (1 + rel * rng.standard_normal(a.shape))) for a in h)
            for h in hist]
    p2 = ref.balance_fields([h[0] for h in pert], [h[1] for h in pert], [h[2] for h in pert],
                            pert[2][3], pert[2][4], nu)
    return base, {k: float((p2[k] - base[k]).abs().max() / (base[k].abs().max() or 1.0))
                  for k in ref.TERM_NAMES}


def test_edm_balance_of_a_run(gpu_lib):
    """The sub-volume balance of a damped exact-difference run (FP64, 48^2): the handle's
    history and force are the scheme's physical velocity (j + F/2)/rho and total force
    F_ext + F^R, checked term by term against the oracle's run."""
    n, steps, tau = 48, 40, 0.6
    amp = 0.4
    rho, ux, uy = _fields(n, n, 13)
    fx, fy = inp.paper_forcing(n, f0=1e-4)
    sim = Sim(rho, ux, uy, tau, dtype="f64", fx=fx, fy=fy, scheme="edm", damp_f0=amp,
              with_balance=True)
    sim.step(steps)
    res = sim.balance((6, 24, 48), term_fields=True)
    r, vx, vy, _ = sim.moments()
    _, hist = ref.edm_run_with_history(ref.init_populations(rho, ux, uy), steps, tau, ref.t64(fx),
                                       ref.t64(fy), amp)
    dmom = max(rel_err(g, w) for g, w in zip((r, vx, vy), hist[-1][:3]))
    say(f"edm balance: moments agree to {dmom:.1e}")
    assert dmom < TOL64
    flds, kappa = _edm_kappa(hist, ref.viscosity(tau), max(dmom, 1e-16))
    for name in ref.TERM_NAMES:
        e = rel_err(res["terms"][name], flds[name])
        tol = max(1e-12, 10 * kappa[name])
        say(f"  {name}: {e:.1e} (tol {tol:.1e})")
        assert e <= tol, (name, e, tol)
    want = ref.subvolume_balance(flds, (6, 24, 48))
    for got, w in zip(res["stats"], want):
        for q in ("dE", "dZ", "Ma"):
            assert got[q]["count"] == w[q]["count"], (got["L"], q)


def test_edm_window_time_series(gpu_lib):
    """Time series of the balance over explicit windows (the single-sub-volume series of
    Sec. 3, Figs. 1-2) on a damped exact-difference run: box means of the 13 fields and each
    window's delta^E, delta^Omega, Ma_V at every sample, against the oracle's run."""
    n, tau, amp = 48, 0.6, 0.4
    rho, ux, uy = _fields(n, n, 21)
    fx, fy = inp.paper_forcing(n, f0=1e-4)
    sim = Sim(rho, ux, uy, tau, dtype="f64", fx=fx, fy=fy, scheme="edm", damp_f0=amp,
              with_balance=True)
    wins = [(5, 7, 34), (40, 44, 17), (0, 0, 48)]
    ser = sim.window_series(wins, every=6, count=3)
    assert list(ser["time"]) == [6, 12, 18]
    assert ser["terms"].shape == (3, 3, 13) and ser["errors"].shape == (3, 3, 3)
    nu = ref.viscosity(tau)
    for i, t in enumerate(ser["time"]):
        _, hist = ref.edm_run_with_history(ref.init_populations(rho, ux, uy), int(t), tau,
                                           ref.t64(fx), ref.t64(fy), amp)
        flds = ref.balance_fields([h[0] for h in hist], [h[1] for h in hist], [h[2] for h in hist],
                                  hist[2][3], hist[2][4], nu)
        wt = ref.window_terms(flds, wins)
        for k, name in enumerate(ref.TERM_NAMES):
            scale = float(flds[name].abs().max())
            d = float(np.abs(ser["terms"][i, :, k] - wt[:, k].numpy()).max())
            say(f"t={t} {name}: {d / scale:.1e}")
            assert d <= 1e-9 * scale, (t, name, d, scale)
        wm = {name: wt[:, k] for k, name in enumerate(ref.TERM_NAMES)}
        for q, o in enumerate(ref.balancing_errors(wm)):
            g = torch.as_tensor(ser["errors"][i, :, q])
            assert torch.allclose(g, o, rtol=1e-7, atol=1e-12), (t, q, g, o)


def test_configuration_sampling_and_pooled_statistics(gpu_lib):
    """The 25-configuration workflow of Sec. 4-5 in small: a damped exact-difference run is
    sampled into configurations, each restarted from its checkpoint; the pooled all-corner
    and Table-1 statistics, the pooled histograms and the per-configuration spectra equal the
    oracle's run sampled at the same times."""
    from paper_1809_06735_amd import configuration_statistics, sample_configurations
    n, tau, amp = 32, 0.6, 0.3
    rho, ux, uy = _fields(n, n, 31)
    fx, fy = inp.paper_forcing(n, f0=1e-4)
    sim = Sim(rho, ux, uy, tau, dtype="f64", fx=fx, fy=fy, scheme="edm", damp_f0=amp,
              with_balance=True)
    sim.step(10)
    cfgs = sample_configurations(sim, 3, every=7)
    assert [t for t, _ in cfgs] == [17, 24, 31]
    sim.step(50)  # moved on: the statistics restart from the checkpoints
    sizes = (3, 8, 32)
    edges = inp.log_edges(1e-6, 10.0, 5)
    smp = lambda i: inp.table1_corners(n, sizes, seed=100 + i)
    res = configuration_statistics(sim, cfgs, sizes, edges=edges, sample=smp, spectrum_shells=24)
    assert res["times"] == [17, 24, 31] and res["spectra"].shape == (3, 24)
    nu = ref.viscosity(tau)
    pools = {k: [[], [], []] for k in range(len(sizes))}
    spools = {k: [[], [], []] for k in range(len(sizes))}
    for i, (t, _) in enumerate(cfgs):
        f, hist = ref.edm_run_with_history(ref.init_populations(rho, ux, uy), t, tau, ref.t64(fx),
                                           ref.t64(fy), amp)
        flds = ref.balance_fields([h[0] for h in hist], [h[1] for h in hist], [h[2] for h in hist],
                                  hist[2][3], hist[2][4], nu)
        st = ref.subvolume_balance(flds, sizes)
        corners, counts = smp(i)
        off = 0
        for k, L in enumerate(sizes):
            sv = ref.sampled_errors(flds, L, corners[off:off + counts[k]])
            off += counts[k]
            for q in range(3):
                pools[k][q].append(st[k]["maps"][q].reshape(-1))
                spools[k][q].append(sv[q])
        want_spec = ref.energy_spectrum(hist[2][1], hist[2][2], 24).numpy()
        assert np.abs(res["spectra"][i] - want_spec).max() <= 1e-10 * want_spec.max()
    for k, L in enumerate(sizes):
        for kind, got, gh, src in (("all", res["stats"][k], res["hist"][k], pools),
                                   ("sampled", res["sample_stats"][k], res["sample_hist"][k], spools)):
            for q, name in enumerate(("dE", "dZ", "Ma")):
                vals = torch.cat([ref.t64(v).reshape(-1) for v in src[k][q]])
                w = ref.pooled_stats(src[k][q])
                g = got[name]
                assert g["count"] == w["count"], (kind, L, name)
                for m in ("mean", "std", "min", "max"):
                    assert g[m] == pytest.approx(w[m], rel=1e-7), (kind, L, name, m)
                hw = ref.histogram(vals, torch.as_tensor(edges)).numpy()
                assert int(np.abs(gh[q] - hw).sum()) <= 2, (kind, L, name, gh[q], hw)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_edm_runs_batched_equal_single_runs(gpu_lib, dtype):
    """Five exact-difference runs on one 64 x 48 grid (the five tau0 of the paper's set-up,
    different damping rates, force fields and initial states) stepped together: each run's
    moments equal, bit for bit, those of the same run stepped alone, after 9 steps (one
    graph replay of 8 plus one enqueued step) and after 40; one run also against the
    oracle.  Without force, the batch takes forceless runs as well."""
    from paper_1809_06735_amd.ensemble import Ensemble
    ny, nx = 64, 48
    taus = (0.5005, 0.501, 0.505, 0.51, 0.55)
    mem = []
    for k, tau in enumerate(taus):
        rho, ux, uy = _fields(ny, nx, 20 + k, mach=0.05)
        fx, fy = inp.forcing_field(max(nx, ny), seed=40 + k, max_force=2e-5)
        mem.append({"rho": rho, "ux": ux, "uy": uy, "tau": tau, "scheme": "edm",
                    "fx": fx[:ny, :nx].copy(), "fy": fy[:ny, :nx].copy(),
                    "damp_f0": 0.05 * (k + 1), "damp_shell": (1.0, 2.0)})
    ens = Ensemble(mem, dtype=dtype, chunk=8)
    assert ens.get_mode()[0] == "per_step"
    for steps in (9, 40):
        ens.step(steps - ens.time)
        for r, m in enumerate(mem):
            s = Sim(m["rho"], m["ux"], m["uy"], m["tau"], dtype=dtype, fx=m["fx"], fy=m["fy"], scheme="edm",
                    damp_f0=m["damp_f0"], damp_shell=m["damp_shell"])
            s.step(steps)
            want = s.moments(scalars=False)
            got = ens.moments(r, scalars=False)
            for name, g, w in zip(("rho", "ux", "uy"), got, want):
                assert torch.equal(g, w), (dtype, steps, r, name)
            s.close()
        say(f"edm batch {dtype}: 5 runs bitwise equal to single runs at {steps} steps")
    m = mem[3]
    want = _oracle(m["rho"], m["ux"], m["uy"], 40, m["tau"], m["fx"], m["fy"], m["damp_f0"], (1.0, 2.0))
    r, vx, vy, _ = ens.moments(3)
    for name, g, w in zip(("rho", "ux", "uy"), (r, vx, vy), want[:3]):
        e = moment_err(name, g, w, dtype)
        tol = moment_tol(name, want[:3], dtype, 40, TOL64 if dtype == "f64" else TOL32)
        say(f"edm batch {dtype} run 3 {name} vs oracle {e:.1e} (tol {tol:.1e})")
        assert e < tol, (name, e, tol)
    ens.close()
    plain = [{k: v for k, v in m.items() if k not in ("fx", "fy")} for m in mem[:2]]
    e2 = Ensemble(plain, dtype=dtype)
    e2.step(6)
    s = Sim(plain[1]["rho"], plain[1]["ux"], plain[1]["uy"], plain[1]["tau"], dtype=dtype, scheme="edm",
            damp_f0=plain[1]["damp_f0"])
    s.step(6)
    for g, w in zip(e2.moments(1, scalars=False), s.moments(scalars=False)):
        assert torch.equal(g, w)
    s.close()
    e2.close()


def test_edm_batch_rejects_what_it_does_not_run(gpu_lib):
    from paper_1809_06735_amd import LBMError
    from paper_1809_06735_amd.ensemble import Ensemble
    rho, ux, uy = _fields(32, 32, 1)
    a = {"rho": rho, "ux": ux, "uy": uy, "tau": 0.6, "scheme": "edm", "damp_f0": 0.1}
    b = dict(a, rho=_fields(32, 40, 2)[0], ux=_fields(32, 40, 2)[1], uy=_fields(32, 40, 2)[2])
    with pytest.raises(LBMError):
        Ensemble([a, b])                                  # two grid sizes
    with pytest.raises(LBMError):
        Ensemble([a, dict(a, damp_shell=(1.0, 3.0))])     # two damped shells
    with pytest.raises(LBMError):
        Ensemble([a, dict(a, scheme="guo", damp_f0=0.0)])  # two force schemes
    e = Ensemble([a, dict(a, tau=0.7)])
    for bad in (lambda: e.set_mode("persistent"), lambda: e.set_multi(4, 128, 32),
                lambda: e.set_tile(1, 1), lambda: e.autotune(4)):
        with pytest.raises(LBMError):
            bad()
    e.close()


def test_edm_damped_512_coefficient_launch(gpu_lib):
    """512^2: the step's workgroups would read too many Fourier partials to add them
    themselves, so the coefficients come from their own launch (the large-grid path); FP64
    against the oracle."""
    _run_case(512, 512, "f64", 8, 0.55, 0.3, seed=12, label="edm64 512^2")
