"""GPU parity of the D2Q9 step, initialisation and moments against the FP64 oracle.

Tolerances: FP64 storage 1e-12 and FP32 storage 1e-5, both as
max |gpu - oracle| / max |oracle| per moment field (the Taylor-Green velocity
has zero nodes, so a pointwise relative error is not meaningful).
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from helpers import gpu_patch, moment_err, moment_tol, oracle_patch_moments, rel_err
from oracle import ref

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def Sim(*a, **k):
    from paper_1809_06735_amd import Simulation
    return Simulation(*a, **k)


def check_moments(sim, want, tol, label, dtype="f64", steps=0):
    r, vx, vy, sc = sim.moments()
    for name, g, w in zip(("rho", "ux", "uy"), (r, vx, vy), want):
        e = moment_err(name, g, w, dtype)
        tol_f = moment_tol(name, want, dtype, steps, tol)
        say(f"{label} {name} rel err {e:.2e} (tol {tol_f:.1e})")
        assert e < tol_f, (label, name, e, tol_f)
    return sc


def test_taylor_green_64_fp64_1000_steps(gpu_lib):
    """Workload tg64: 64^2 FP64, tau 0.6, 1000 steps."""
    say("tg64 fp64 1000 steps")
    rho, ux, uy = inp.taylor_green(64, 0.01)
    sim = Sim(rho, ux, uy, 0.6, dtype="f64")
    sim.step(1000)
    f = ref.run(ref.init_populations(rho, ux, uy), 1000, 0.6)
    sc = check_moments(sim, ref.moments(f), TOL64, "tg64")
    assert sc["time"] == 1000
    assert sc["mass"] == pytest.approx(64 * 64, rel=1e-14)


def test_forced_drag_fp64_parity(gpu_lib):
    """FP64 with Guo forcing and drag, non-square grid, 120 steps."""
    say("forced fp64 96x80")
    ny, nx = 80, 96
    rng = np.random.default_rng(1)
    _, ux, uy = inp.spectrum_velocity(96, seed=2, max_mach=0.08)
    ux, uy = ux[:ny], uy[:ny]
    rho = 1.0 + 0.001 * rng.standard_normal((ny, nx))
    fx, fy = inp.forcing_field(96, seed=4, max_force=2e-5)
    fx, fy = fx[:ny], fy[:ny]
    tau, alpha = 0.53, 2e-3
    sim = Sim(rho, ux, uy, tau, dtype="f64", fx=fx, fy=fy, alpha=alpha)
    sim.step(120)
    f = ref.run(ref.init_populations(rho, ux, uy), 120, tau, ref.t64(fx), ref.t64(fy), alpha)
    check_moments(sim, ref.moments(f, ref.t64(fx), ref.t64(fy), alpha), TOL64, "forced64")


def test_spectrum_256_fp32_100_steps(gpu_lib):
    """FP32 storage, decaying spectrum, 256^2, 100 steps, whole grid."""
    say("spectrum 256 fp32 100 steps")
    rho, ux, uy = inp.spectrum_velocity(256, seed=0, max_mach=0.05)
    sim = Sim(rho, ux, uy, 0.51, dtype="f32")
    sim.step(100)
    f = ref.run(ref.init_populations(rho, ux, uy), 100, 0.51)
    check_moments(sim, ref.moments(f), TOL32, "spec256", "f32", 100)


def test_decay1024_fp32_sampled_patches(gpu_lib):
    """Workload decay1024 (1024^2 FP32, tau 0.51): 100 steps, oracle on sampled patches
    (one across the periodic corner)."""
    say("decay1024 fp32 100 steps, patches")
    rho, ux, uy = inp.spectrum_velocity(1024, seed=0, max_mach=0.05)
    sim = Sim(rho, ux, uy, 0.51, dtype="f32")
    sim.step(100)
    r, vx, vy = sim.moments(scalars=False)
    for (y0, x0) in ((1010, 1000), (400, 733)):
        want = oracle_patch_moments((rho, ux, uy), 0.51, 100, y0, x0, 24)
        for name, g, w in zip(("rho", "ux", "uy"), (r, vx, vy), want):
            e = moment_err(name, gpu_patch(g, y0, x0, 24), w, "f32")
            tol = moment_tol(name, want, "f32", 100, TOL32)
            say(f"decay1024 patch ({y0},{x0}) {name} {e:.2e} (tol {tol:.1e})")
            assert e < tol


@pytest.fixture(scope="module")
def forced4096():
    w = inp.WORKLOADS["forced4096"]
    fx, fy = inp.forcing_field(w.n, seed=w.seed, alpha=w.alpha)
    z = np.zeros((w.n, w.n))
    return w, np.ones((w.n, w.n)), z, z, fx, fy


def test_forced4096_fp32_sampled_patches_in_bench_launch_shape(gpu_lib, forced4096):
    """Workload forced4096 (4096^2 FP32, Guo force + drag, from rest) in the autotuned
    launch shape the benchmark uses: 20 steps, oracle on patches incl. the periodic seam."""
    w, rho, ux, uy, fx, fy = forced4096
    say("forced4096 fp32 autotune + 20 steps")
    sim = Sim(rho, ux, uy, w.tau, dtype="f32", fx=fx, fy=fy, alpha=w.alpha)
    tile = sim.autotune(trial_steps=3)
    say(f"forced4096 tile {tile}")
    sim.step(20)
    r, vx, vy, sc = sim.moments()
    assert sc["nonfinite"] == 0
    for (y0, x0) in ((4090, 4085), (0, 2048), (1234, 4091), (2000, 0)):
        want = oracle_patch_moments((rho, ux, uy), w.tau, 20, y0, x0, 16, fx=fx, fy=fy, alpha=w.alpha)
        for name, g, ww in zip(("rho", "ux", "uy"), (r, vx, vy), want):
            e = moment_err(name, gpu_patch(g, y0, x0, 16), ww, "f32")
            # from rest rho - 1 after 20 steps (~1e-11) lies below the FP32 storage's
            # resolution of the density: its tolerance is the rounding floor, reported
            tol = moment_tol(name, want, "f32", 20, TOL32)
            say(f"forced4096 patch ({y0},{x0}) {name} {e:.2e} (tol {tol:.1e})")
            assert e < tol, (name, e, tol)


@pytest.mark.parametrize("shape", [(16, 16), (33, 17), (50, 34), (64, 48), (20, 100)])
def test_ragged_grids_all_launch_shapes_agree(gpu_lib, shape):
    """Every launch shape gives bit-identical populations; one matches the oracle."""
    from paper_1809_06735_amd import _lib as L
    import ctypes as C
    ny, nx = shape
    say(f"ragged {ny}x{nx}")
    rng = np.random.default_rng(nx * 1000 + ny)
    rho = 1.0 + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.03 * rng.standard_normal((ny, nx))
    uy = 0.03 * rng.standard_normal((ny, nx))
    fx = 1e-5 * rng.standard_normal((ny, nx))
    fy = 1e-5 * rng.standard_normal((ny, nx))
    steps = 7
    ref_state = None
    f = ref.run(ref.init_populations(rho, ux, uy), steps, 0.7, ref.t64(fx), ref.t64(fy), 1e-3)
    want = ref.moments(f, ref.t64(fx), ref.t64(fy), 1e-3)
    for dt, tol in (("f64", TOL64), ("f32", TOL32)):
        lib = L.load()
        cand = []
        for vx_ in (1, 2, 4):
            for (bx, by) in ((64, 1), (64, 2), (128, 1), (64, 4)):
                for ry in (1, 3):
                    for nt in (0, 1):
                        cand.append((bx, by, vx_, ry, nt))
        # K steps per launch: strip width, band height, nt, K, prefetch
        for (w, h, k) in ((64, 1, 2), (64, 5, 3), (128, 16, 4), (64, 64, 2), (64, 2, 4)):
            for nt, pf in ((0, 0), (1, 1)):
                cand.append((w, 1, 1, h, nt, k, pf))
        # packed halo: the strip and its halo columns in the same lanes
        for (w, h, k) in ((64, 1, 4), (64, 5, 6), (128, 16, 5), (64, 3, 2)):
            cand.append((w, 1, 1, h, 1, k, 1, 1))
        ref_state = None
        checked = 0
        for tile in cand:
            if nx % tile[2]:
                continue
            sim = Sim(rho, ux, uy, 0.7, dtype=dt, fx=fx, fy=fy, alpha=1e-3)
            sim.set_tile(*tile)
            sim.step(steps)
            st = sim.save()
            if ref_state is None:
                ref_state = st
                check_moments(sim, want, tol, f"ragged {ny}x{nx} {dt} {tile}", dt, steps)
            else:
                assert torch.equal(st, ref_state), tile
            checked += 1
            sim.close()
        assert checked > 0


def test_graph_replay_equals_direct_launches(gpu_lib):
    rho, ux, uy = inp.spectrum_velocity(128, seed=5, max_mach=0.05)
    a = Sim(rho, ux, uy, 0.52, dtype="f32")
    a.set_graph(0)
    a.step(301)
    b = Sim(rho, ux, uy, 0.52, dtype="f32")
    b.set_graph(16)
    b.step(1)
    b.step(300)
    assert torch.equal(a.save(), b.save())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("layout", ["rows", "planes"])
def test_multi_step_kernel_equals_single_steps(gpu_lib, dtype, layout):
    """K = 2..6 steps per launch (temporal blocking through LDS) give bit-identical states
    to single-step launches: forced and unforced, ragged strips and bands (down to one row),
    step counts that leave remainders, direct launches and graph replay."""
    ny, nx = 75, 200
    rng = np.random.default_rng(21)
    rho = 1.0 + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.04 * rng.standard_normal((ny, nx))
    uy = 0.04 * rng.standard_normal((ny, nx))
    fx = 2e-5 * rng.standard_normal((ny, nx))
    fy = 2e-5 * rng.standard_normal((ny, nx))
    for forced in (False, True):
        kw = dict(fx=fx, fy=fy, alpha=2e-3) if forced else {}
        base = Sim(rho, ux, uy, 0.53, dtype=dtype, layout=layout, **kw)
        base.set_tile(64, 1, 1, 1, 0)
        base.set_graph(0)
        base.step(9)
        s9 = base.save().clone()
        base.step(52)
        s61 = base.save().clone()
        base.close()
        # last field: halo = 1 packs the halo columns into the workgroup (strip of
        # w - 2 (k - 1) columns: 58, 122, 182, 54, 246 here, ragged on 200 columns or
        # wider than the grid)
        for (k, w, h, nt, pf, chunk, halo) in (
                (2, 64, 16, 0, 0, 0, 0), (2, 128, 7, 1, 1, 0, 0), (2, 256, 75, 0, 1, 4, 0),
                (2, 64, 1, 1, 0, 2, 0), (2, 512, 32, 1, 1, 0, 0),
                (3, 64, 16, 1, 0, 0, 0), (3, 128, 5, 0, 1, 2, 0), (3, 256, 75, 1, 1, 0, 0),
                (4, 64, 3, 0, 0, 0, 0), (4, 192, 40, 1, 1, 4, 0), (4, 512, 64, 1, 0, 0, 0),
                (4, 64, 1, 1, 1, 0, 0), (5, 128, 20, 1, 1, 0, 0), (5, 64, 75, 0, 1, 2, 0),
                (6, 256, 9, 1, 1, 0, 0), (6, 64, 2, 0, 0, 4, 0),
                (4, 64, 3, 0, 0, 0, 1), (4, 128, 40, 1, 1, 4, 1), (5, 192, 20, 1, 1, 0, 1),
                (6, 64, 2, 0, 0, 4, 1), (6, 256, 9, 1, 1, 0, 1), (2, 512, 32, 1, 1, 0, 1)):
            s = Sim(rho, ux, uy, 0.53, dtype=dtype, layout=layout, **kw)
            s.set_tile(w, 1, 1, h, nt, k, pf, halo)
            s.set_graph(chunk)
            s.step(9)
            assert torch.equal(s.save(), s9), (forced, k, w, h, nt, pf, chunk, halo, 9)
            s.step(52)
            assert torch.equal(s.save(), s61), (forced, k, w, h, nt, pf, chunk, halo, 61)
            s.close()
        say(f"multi-step kernel {dtype} {layout} forced={forced}: bit-identical")


def test_multi_step_shapes_rejected_when_invalid(gpu_lib):
    from paper_1809_06735_amd import LBMError
    rho, ux, uy = inp.taylor_green(32, 0.01)
    s = Sim(rho, ux, uy, 0.6, dtype="f64")
    for bad in ((96, 1, 1, 8, 0, 2, 0), (0, 1, 1, 8, 0, 2, 0), (1024, 1, 1, 8, 0, 2, 0),
                (64, 2, 1, 8, 0, 2, 0), (64, 1, 2, 8, 0, 2, 0), (64, 1, 1, 0, 0, 2, 0),
                (64, 1, 1, 8, 0, 7, 0), (64, 1, 1, 8, 0, 1, 1), (960, 1, 1, 8, 0, 2, 0),
                (576, 1, 1, 8, 0, 2, 0), (64, 1, 1, 8, 0, 2, 0, 2), (64, 1, 1, 8, 0, 1, 0, 1),
                (64, 1, 1, 1, 0, 0, 0, 1), (576, 1, 1, 8, 0, 4, 1, 1)):
        with pytest.raises(LBMError):
            s.set_tile(*bad)
    s.close()


def test_save_load_resume_and_determinism(gpu_lib):
    rho, ux, uy = inp.spectrum_velocity(96, seed=6, max_mach=0.05)
    a = Sim(rho, ux, uy, 0.55, dtype="f32", with_balance=True)
    a.step(40)
    st = a.save().clone()
    a.step(25)
    b = Sim(rho, ux, uy, 0.55, dtype="f32", with_balance=True)
    b.load(st)
    assert b.time == 40
    b.step(25)
    assert torch.equal(a.save(), b.save())
    c = Sim(rho, ux, uy, 0.55, dtype="f32")
    c.step(65)
    assert torch.equal(c.save()[256:256 + 9 * 96 * 96 * 4], a.save()[256:256 + 9 * 96 * 96 * 4])
    ra = a.balance([8, 96])
    rb = b.balance([8, 96])
    assert ra["stats"] == rb["stats"]


def test_translation_equivariance_bitwise(gpu_lib):
    rho, ux, uy = inp.spectrum_velocity(64, seed=8, max_mach=0.05)
    sh = lambda a: np.roll(a, (5, -9), (0, 1))  # noqa: E731
    a = Sim(rho, ux, uy, 0.53, dtype="f32")
    b = Sim(sh(rho), sh(ux), sh(uy), 0.53, dtype="f32")
    a.step(30)
    b.step(30)
    ra = a.moments(scalars=False)
    rb = b.moments(scalars=False)
    for x, y in zip(ra, rb):
        assert torch.equal(torch.roll(x, (5, -9), (0, 1)), y)


def test_divergence_is_reported(gpu_lib):
    from paper_1809_06735_amd import LBMError
    rho, ux, uy = inp.taylor_green(32, 0.01)
    ux = ux.copy()
    ux[3, 4] = np.nan
    sim = Sim(rho, ux, uy, 0.6, dtype="f32", with_balance=True)
    sim.step(3)
    with pytest.raises(LBMError) as ei:
        sim.moments()
    assert ei.value.code == -4
    with pytest.raises(LBMError) as ei:
        sim.balance([8])
    assert ei.value.code == -4


def _oracle_divergence_step(rho, ux, uy, tau, limit):
    """First step after which the oracle's moments hold a non-finite value or rho <= 0 (the
    library's divergence criterion), or None within `limit` steps."""
    f = ref.init_populations(rho, ux, uy)
    for t in range(1, limit + 1):
        f = ref.step(f, tau)
        r, vx, vy = ref.moments(f)
        if not (torch.isfinite(r).all() and torch.isfinite(vx).all() and torch.isfinite(vy).all()):
            return t
        if float(r.min()) <= 0.0:
            return t
    return None


@pytest.mark.parametrize("seed,mach,tau", [(0, 0.5, 0.5001), (1, 0.6, 0.5001), (2, 0.5, 0.501)])
def test_divergence_window_matches_the_oracle(gpu_lib, seed, mach, tau):
    """An unstable run (32^2 at Mach 0.5-0.6 and tau near 1/2, FP64): the oracle's first
    diverged step t* lies in the window the library flags.  The library is finite at t* - 5
    and reports LBM_E_DIVERGED (-4) at t* + 5, with the step in its message; a state saved at
    t* - 5 restores a finite run (rollback to the last checkpoint)."""
    from paper_1809_06735_amd import LBMError
    n = 32
    _, ux, uy = inp.spectrum_velocity(n, seed=seed, max_mach=mach)
    rho = np.ones((n, n))
    ts = _oracle_divergence_step(rho, ux, uy, tau, 1000)
    say(f"divergence seed {seed} Ma {mach} tau {tau}: oracle diverges at step {ts}")
    assert ts is not None and ts > 10
    sim = Sim(rho, ux, uy, tau, dtype="f64")
    sim.step(ts - 5)
    r0, vx0, vy0, sc = sim.moments()
    assert sc["nonfinite"] == 0 and sc["min_rho"] > 0
    saved = sim.save()
    sim.step(10)
    with pytest.raises(LBMError) as ei:
        sim.moments()
    assert ei.value.code == -4
    assert str(ts + 5) in str(ei.value)
    sim.load(saved)
    r1, vx1, vy1, sc1 = sim.moments()
    assert sc1["nonfinite"] == 0 and sc1["time"] == ts - 5
    for a, b in zip((r0, vx0, vy0), (r1, vx1, vy1)):
        assert torch.equal(a, b)


def test_state_errors(gpu_lib):
    from paper_1809_06735_amd import LBMError
    rho, ux, uy = inp.taylor_green(32, 0.01)
    sim = Sim(rho, ux, uy, 0.6, dtype="f32")
    sim.step(3)
    with pytest.raises(LBMError) as ei:
        sim.balance([8])
    assert ei.value.code == -5        # no balance workspace
    sim2 = Sim(rho, ux, uy, 0.6, dtype="f32", with_balance=True)
    sim2.step(1)
    with pytest.raises(LBMError) as ei:
        sim2.balance([8])
    assert ei.value.code == -5        # no two levels of history yet
    with pytest.raises(LBMError):
        sim2.set_tile(64, 1, 3, 1)    # vx = 3 invalid
    with pytest.raises(LBMError):
        sim2.balance([64])            # L > N


def test_step_timing_counts_launches(gpu_lib):
    rho, ux, uy = inp.taylor_green(64, 0.01)
    sim = Sim(rho, ux, uy, 0.6, dtype="f32")
    sim.step_timing(True)
    sim.step(100)
    sim.step(5)
    ms, n = sim.step_time(reset=True)
    # the bulk launches are timed; the last two steps of each call record history
    assert n == 98 + 3 and ms > 0
    sim.set_tile(128, 1, 1, 16, 1, 2, 0)
    sim.step(100)
    sim.step(7)
    ms, n = sim.step_time(reset=True)
    assert n == 49 + 2 and ms > 0
    ms, n = sim.step_time()
    assert n == 0 and ms == 0


def test_copy_bandwidth_runs(gpu_lib):
    from paper_1809_06735_amd import copy_bandwidth
    gbs, ms = copy_bandwidth(1 << 26, iters=3)
    assert gbs > 100


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rows_layout_equals_planes_layout(gpu_lib, dtype):
    """The row-interleaved population layout gives bit-identical moments and balance to the
    plane layout (same arithmetic, other addresses), for several launch shapes."""
    ny, nx = 48, 80
    rng = np.random.default_rng(11)
    rho = 1.0 + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.03 * rng.standard_normal((ny, nx))
    uy = 0.03 * rng.standard_normal((ny, nx))
    fx = 1e-5 * rng.standard_normal((ny, nx))
    fy = 1e-5 * rng.standard_normal((ny, nx))
    ref_m = None
    for layout in ("planes", "rows"):
        for tile in ((64, 1, 1, 1, 0), (64, 4, 2, 3, 1), (64, 2, 4, 1, 1)):
            if dtype == "f64" and tile[2] == 4:
                continue
            s = Sim(rho, ux, uy, 0.57, dtype=dtype, fx=fx, fy=fy, alpha=1e-3, with_balance=True,
                    layout=layout)
            s.set_tile(*tile)
            s.step(17)
            m = s.moments(scalars=False)
            b = s.balance((4, 16, 48))["stats"]
            if ref_m is None:
                ref_m, ref_b = m, b
            else:
                for x, y in zip(m, ref_m):
                    assert torch.equal(x, y), (layout, tile)
                assert b == ref_b
            s.close()


def test_load_refuses_a_state_of_another_grid_dtype_or_layout(gpu_lib):
    """lbm_load checks the saved header (grid, dtype, layout, size) before copying anything;
    Simulation.load checks the buffer's size and device."""
    import ctypes as C
    from paper_1809_06735_amd import _lib as L
    say("save/load header checks")
    rho, ux, uy = inp.taylor_green(64, 0.01)
    a = Sim(rho, ux, uy, 0.6, dtype="f32")
    a.step(5)
    st = a.save()
    torch.cuda.synchronize()
    others = {
        "grid": Sim(rho[:48], ux[:48], uy[:48], 0.6, dtype="f32"),
        "dtype": Sim(rho, ux, uy, 0.6, dtype="f64"),
        "layout": Sim(rho, ux, uy, 0.6, dtype="f32", layout="planes"),
    }
    for what, b in others.items():
        before = b.save()
        rc = b._lib.lbm_load(b._h, C.c_void_p(st.data_ptr()))
        msg = b._lib.lbm_last_error().decode()
        say(f"  {what}: rc {rc}, {msg}")
        assert rc == L.LBM_E_INVALID, what
        assert ("nx" if what == "grid" else what) in msg or "ny" in msg
        assert torch.equal(b.save(), before), what  # nothing was copied
        if what != "layout":  # same size as this handle's state only for the layout case
            with pytest.raises(ValueError):
                b.load(st)
        b.close()
    bad = st.clone()
    bad[:8] = 0
    with pytest.raises(Exception):
        Sim(rho, ux, uy, 0.6, dtype="f32").load(bad)
    # the matching handle restores the state exactly
    c = Sim(rho, ux, uy, 0.6, dtype="f32")
    c.load(st)
    assert c.time == 5 and torch.equal(c.save(), st)
    a.step(3)
    c.step(3)
    assert torch.equal(a.save(), c.save())
    a.close()
    c.close()
