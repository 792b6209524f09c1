"""GPU checks of the batched ensemble: every run equals the single-grid path, and
the single-grid path equals the FP64 oracle (checked elsewhere), so the batch is
held to the oracle too; persistent and per-step modes agree bit for bit."""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from helpers import gpu_patch, moment_err, moment_tol, oracle_patch_moments, rel_err
from oracle import ref

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def small_members(seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(16, 16), (32, 48), (40, 24), (64, 64), (20, 36)]
    out = []
    for k, (ny, nx) in enumerate(shapes):
        rho = 1.0 + 0.01 * rng.standard_normal((ny, nx))
        ux = 0.04 * rng.standard_normal((ny, nx))
        uy = 0.04 * rng.standard_normal((ny, nx))
        m = {"rho": rho, "ux": ux, "uy": uy, "tau": float(rng.uniform(0.51, 0.8))}
        if k == 2:
            m["fx"] = 1e-5 * rng.standard_normal((ny, nx))
            m["fy"] = 1e-5 * rng.standard_normal((ny, nx))
            m["alpha"] = 1e-3
        if k == 4:
            m["alpha"] = 2e-3
        out.append(m)
    return out


@pytest.mark.parametrize("mode", ["persistent", "per_step", "multi_step", "persistent_multi"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ensemble_matches_single_grid_and_oracle(gpu_lib, mode, dtype):
    from paper_1809_06735_amd import Simulation
    from paper_1809_06735_amd.ensemble import Ensemble
    say(f"ensemble small {mode} {dtype}")
    mem = small_members()
    ens = Ensemble(mem, dtype=dtype, mode=mode, chunk=8)
    if mode in ("multi_step", "persistent_multi"):
        ens.set_multi(3, 64, 8)     # several strips and bands per member
    steps = 21                      # two graph replays + an odd remainder
    ens.step(steps)
    assert ens.time == steps
    tol = 1e-12 if dtype == "f64" else 1e-5
    for r, m in enumerate(mem):
        got = ens.moments(r)
        sim = Simulation(m["rho"], m["ux"], m["uy"], m["tau"], dtype=dtype, fx=m.get("fx"),
                         fy=m.get("fy"), alpha=m.get("alpha", 0.0))
        sim.step(steps)
        want_gpu = sim.moments()
        for a, b in zip(got[:3], want_gpu[:3]):
            assert rel_err(a, b) <= (1e-15 if dtype == "f64" else 1e-7), r
        kw = {}
        if m.get("fx") is not None:
            kw = dict(fx_ext=ref.t64(m["fx"]), fy_ext=ref.t64(m["fy"]))
        alpha = m.get("alpha", 0.0)
        f = ref.run(ref.init_populations(m["rho"], m["ux"], m["uy"]), steps, m["tau"], alpha=alpha, **kw)
        want = ref.moments(f, kw.get("fx_ext"), kw.get("fy_ext"), alpha)
        for name, a, b in zip(("rho", "ux", "uy"), got[:3], want):
            e = moment_err(name, a, b, dtype)
            tol_f = moment_tol(name, want, dtype, steps, tol)
            say(f"  run {r} {name} vs oracle {e:.1e} (tol {tol_f:.1e})")
            assert e < tol_f, (r, name, e, tol_f)
        sim.close()
    ens.close()


def test_persistent_and_per_step_modes_agree_bitwise(gpu_lib):
    from paper_1809_06735_amd.ensemble import Ensemble
    mem = small_members(1)
    a = Ensemble(mem, mode="persistent", chunk=10)
    b = Ensemble(mem, mode="per_step", chunk=4)
    a.step(37)
    b.step(37)
    for r in range(len(mem)):
        for x, y in zip(a.moments(r, scalars=False), b.moments(r, scalars=False)):
            assert torch.equal(x, y), r


def test_ensemble_tiles_and_autotune_keep_results(gpu_lib):
    from paper_1809_06735_amd.ensemble import Ensemble
    mem = small_members(2)
    base = Ensemble(mem, mode="persistent", chunk=6)
    base.set_tile(1, 1)
    base.step(30)
    ref_m = [base.moments(r, scalars=False) for r in range(len(mem))]
    for vx, g, bt in ((2, 1, 256), (4, 3, 256), (4, 8, 1024), (1, 2, 512)):
        e = Ensemble(mem, mode="persistent", chunk=6)
        e.set_tile(vx, g, bt)
        e.step(30)
        for r in range(len(mem)):
            for x, y in zip(e.moments(r, scalars=False), ref_m[r]):
                # FP32: differently shaped instances may round differently
                assert rel_err(x, y) <= 1e-5, (vx, g, r)
    t = Ensemble(mem, mode="persistent", chunk=6)
    bt, vx, g = t.autotune(trial_steps=4)
    assert bt in (256, 1024) and vx in (1, 2, 4) and 1 <= g <= 64
    assert t.get_mode()[0] in ("persistent", "per_step", "multi_step", "persistent_multi")
    k, w, h, nt, halo = t.get_multi()
    assert 2 <= k <= 6 and w in (128, 256, 512) and h in (32, 64, 128) and halo in (0, 1)
    assert t.time > 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_multi_step_mode_equals_per_step_bitwise(gpu_lib, dtype):
    """K steps per launch over (run, strip, band) tiles: bit-identical to one launch per
    step for every member, with forced and unforced members, ragged tiles, remainders and
    graph chunks whose launch count is odd (the buffer parity flips per replay)."""
    from paper_1809_06735_amd import LBMError
    from paper_1809_06735_amd.ensemble import Ensemble
    mem = small_members(3)
    ref_e = Ensemble(mem, dtype=dtype, mode="per_step", chunk=4)
    ref_e.step(7)
    r7 = [ref_e.moments(r, scalars=False) for r in range(len(mem))]
    ref_e.step(30)
    r37 = [ref_e.moments(r, scalars=False) for r in range(len(mem))]
    ref_e.close()
    for (k, w, h, nt, chunk, halo) in ((2, 64, 8, 1, 4, 0), (3, 64, 16, 0, 6, 0), (4, 128, 8, 1, 10, 0),
                                       (4, 64, 32, 1, 2, 0), (3, 512, 64, 1, 8, 0), (4, 64, 8, 1, 4, 1),
                                       (5, 128, 16, 0, 10, 1), (6, 256, 32, 1, 6, 1), (6, 64, 8, 1, 2, 1)):
        for mode in ("multi_step", "persistent_multi"):
            e = Ensemble(mem, dtype=dtype, mode=mode, chunk=chunk)
            e.set_multi(k, w, h, nt, halo)
            assert e.get_multi() == (k, w, h, nt, halo)
            e.step(7)
            for r in range(len(mem)):
                for x, y in zip(e.moments(r, scalars=False), r7[r]):
                    assert torch.equal(x, y), (mode, k, w, h, chunk, r, 7)
            e.step(30)
            for r in range(len(mem)):
                for x, y in zip(e.moments(r, scalars=False), r37[r]):
                    assert torch.equal(x, y), (mode, k, w, h, chunk, r, 37)
            e.close()
    e = Ensemble(mem, dtype=dtype, mode="multi_step", chunk=4)
    for bad in ((7, 64, 8), (1, 64, 8), (2, 96, 8), (2, 64, 4), (2, 1024, 8), (4, 64, 8, 1, 2)):
        with pytest.raises(LBMError):
            e.set_multi(*bad)
    e.close()


@pytest.mark.parametrize("mode", ["persistent", "multi_step_autotuned", "persistent_multi_autotuned"])
def test_ensemble64_workload_sampled(gpu_lib, mode):
    """Workload ensemble64 (64 runs, 256^2..1024^2, FP32, tau in [0.505, 0.6]): 20 steps in
    one graph replay chunk, in the persistent mode and in the multi-step shape that the
    autotuner picks for this workload (the shape the benchmark times), as separate launches
    and inside one persistent launch; three members (the largest and two others) checked on
    oracle patches, one across the periodic corner."""
    from paper_1809_06735_amd.ensemble import Ensemble
    say(f"ensemble64 build ({mode})")
    mem = inp.ensemble_members(64)
    if mode == "persistent":
        ens = Ensemble(mem, dtype="f32", mode="persistent", chunk=20)
    else:
        tuner = Ensemble(mem, dtype="f32", mode="persistent", chunk=20)
        tuner.autotune(trial_steps=6)
        shape = tuner.get_multi()
        tuner.close()
        del tuner
        torch.cuda.empty_cache()
        say(f"ensemble64 autotuned multi-step shape (K, strip, band, nt, halo) = {shape}")
        ens = Ensemble(mem, dtype="f32", mode=mode[:-len("_autotuned")], chunk=20)
        ens.set_multi(shape[0], shape[1], shape[2], shape[3], shape[4])
    assert ens.sites == sum(m["n"] ** 2 for m in mem)
    ens.step(20)
    big = max(range(len(mem)), key=lambda r: mem[r]["n"])
    for r in (0, 37, big):
        m = mem[r]
        got = ens.moments(r, scalars=False)
        n = m["n"]
        for (y0, x0) in ((n - 5, n - 7), (n // 3, n // 2)):
            want = oracle_patch_moments((m["rho"], m["ux"], m["uy"]), m["tau"], 20, y0, x0, 12)
            for name, g, w in zip(("rho", "ux", "uy"), got, want):
                e = moment_err(name, gpu_patch(g, y0, x0, 12), w, "f32")
                tol = moment_tol(name, want, "f32", 20, 1e-5)
                say(f"ensemble64 {mode} run {r} (n={n}) patch ({y0},{x0}) {name} {e:.1e} (tol {tol:.1e})")
                assert e < tol, (name, e, tol)
    ens.close()
