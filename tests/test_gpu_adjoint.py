"""GPU discrete adjoint against the FP64 oracle (autodiff of the oracle's forward,
itself pinned by central differences) and against central differences of the
GPU's own loss.

Tolerances: FP64 GPU vs FP64 oracle 1e-8 (max |diff| / max |oracle| for the
u0 gradient, relative for J and dJ/dtau); central differences 1e-4 relative
(the target stated for the differentiable workload) on 32^2 x 50 steps, and
1e-3 on the full 512^2 x 2000-step workload in FP64 (there the FD quotient
itself carries ~1e-4 of rounding: J ~ 1e-25 is a square of residuals that are
1e-3 of the terms they balance).

FP32: on a conditioned case (32^2, 50 steps, Ma 0.1, tau 0.55, where the
residual is ~1e-2 of the terms and the state changes by ~2 % per step) the
FP32 adjoint is compared element by element with the FP64 oracle's gradient.
Its error is set by FP32 rounding amplified by two cancellations: the BDF2
seeds of three levels that nearly cancel (1 / relative change per step) and
RHS - LHS (1 / relative residual); the tolerance is that amplification times
the FP32 unit roundoff, measured on these inputs from the oracle itself.  On
the full 512^2 x 2000 workload the same amplification exceeds 1 / eps32, so
there FP32 J is only required to be finite and within a factor of 2 of FP64,
and the FP64 gradient is the verified one.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as inp
from helpers import rel_err
from oracle import ref

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def tiny(seed=7, n=32):
    _, ux, uy = inp.spectrum_velocity(n, seed=seed, max_mach=0.1)
    return ux, uy


@pytest.mark.parametrize("box,ckpt", [(8, 7), (32, 50), (8, 1), (5, 13)])
def test_adjoint_fp64_matches_oracle(gpu_lib, box, ckpt):
    """Workload adjoint512's small check: 32^2, 50 steps, FP64."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    ux, uy = tiny()
    tau, steps = 0.55, 50
    say(f"adjoint fp64 32^2 box {box} ckpt {ckpt}")
    J, gx, gy, gt = adjoint_run(ux, uy, tau, steps, box, ckpt, dtype="f64")
    Jr, gxr, gyr, gtr = ref.enstrophy_residual_grad(ux, uy, tau, steps, box)
    say(f"  J {J:.6e} vs {Jr:.6e}; dJ/dtau {gt:.6e} vs {gtr:.6e}")
    assert J == pytest.approx(Jr, rel=1e-10)
    ex, ey = rel_err(gx, gxr), rel_err(gy, gyr)
    say(f"  grad u0 rel err {ex:.1e} {ey:.1e}")
    assert ex < 1e-8 and ey < 1e-8
    assert gt == pytest.approx(gtr, rel=1e-8)


def _fp32_amplification(ux, uy, tau, steps, box):
    """Amplification of FP32 rounding in the loss's gradient, from the FP64 oracle: the
    ratio of the largest level seed to the net sensitivity (BDF2 cancellation, Eq. 17) times
    the ratio of the terms to their residual (Eq. 11).  Both are read off the oracle's
    fields of these inputs."""
    f = ref.equilibrium(torch.ones(ux.shape, dtype=torch.float64), ref.t64(ux), ref.t64(uy))
    _, hist = ref.run_with_history(f, steps, tau)
    flds = ref.fields_from_history(hist, tau)
    om = [0.5 * ref.vorticity(h[1], h[2]) ** 2 for h in hist]
    change = float((om[2] - om[1]).abs().max()) / float(om[2].abs().max())
    terms = max(float(flds[k].abs().max()) for k in ("z1", "z2", "z3", "z4", "z5"))
    resid = sum(flds[k] for k in ("z1", "z2", "z3", "z4", "z5")) - flds["lhs_Z"]
    box_r = ref.box_mean_map(resid, box)
    box_t = max(float(ref.box_mean_map(flds[k], box).abs().max()) for k in ("z1", "z2", "z4", "z5"))
    return (1.0 / change) * max(terms / float(resid.abs().max()), box_t / float(box_r.abs().max()))


@pytest.mark.parametrize("box", [8, 32])
def test_adjoint_fp32_matches_oracle_on_a_conditioned_case(gpu_lib, box):
    """The FP32 adjoint (FP32 populations, FP32 adjoint populations) against the FP64
    oracle's gradient, element by element: 32^2, 50 steps, Ma 0.1, tau 0.55, checkpoints
    every 10.  Tolerance: 32 x eps32 x the measured amplification (see the module notes)."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    ux, uy = tiny()
    tau, steps = 0.55, 50
    say(f"adjoint fp32 32^2 box {box}")
    J, gx, gy, gt = adjoint_run(ux, uy, tau, steps, box, 10, dtype="f32")
    Jr, gxr, gyr, gtr = ref.enstrophy_residual_grad(ux, uy, tau, steps, box)
    amp = _fp32_amplification(ux, uy, tau, steps, box)
    tol = 32 * 2.0 ** -24 * amp
    ex, ey = rel_err(gx, gxr), rel_err(gy, gyr)
    et = abs(gt - gtr) / abs(gtr)
    a = torch.cat([gx.cpu().flatten(), gy.cpu().flatten()])
    b = torch.cat([gxr.flatten(), gyr.flatten()])
    cos = float((a @ b) / (a.norm() * b.norm()))
    say(f"  J {J:.6e} vs {Jr:.6e} ({abs(J / Jr - 1):.1e}); amplification {amp:.3g}, tol {tol:.2e}")
    say(f"  grad u0 rel err {ex:.2e} {ey:.2e}; dJ/dtau {gt:.6e} vs {gtr:.6e} ({et:.2e}); cosine {cos:.8f}")
    assert tol < 0.05, "case not conditioned for FP32"
    assert abs(J / Jr - 1) < tol
    assert ex < tol and ey < tol and et < tol


def test_adjoint_first_pass_in_multi_step_shapes_is_bitwise(gpu_lib):
    """The first forward pass runs in the grid's tuned shape, K steps per launch when that
    is the tuned choice; the loss and gradients do not change by a bit."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    from paper_1809_06735_amd.sim import set_tuned_tile
    ux, uy = tiny()
    set_tuned_tile(32, 32, "f64", tile=(64, 1, 1, 1, 0, 1, 0))
    J0, gx0, gy0, gt0 = adjoint_run(ux, uy, 0.55, 50, 8, 7, dtype="f64")
    for tile in ((64, 1, 1, 8, 1, 3, 1), (64, 1, 1, 5, 0, 4, 1), (128, 1, 1, 32, 1, 2, 0)):
        set_tuned_tile(32, 32, "f64", tile=tile)
        J, gx, gy, gt = adjoint_run(ux, uy, 0.55, 50, 8, 7, dtype="f64")
        assert J == J0 and gt == gt0, tile
        assert torch.equal(gx, gx0) and torch.equal(gy, gy0), tile
    set_tuned_tile(32, 32, "f64", tile=(64, 1, 1, 1, 0, 1, 0))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_launches_equal_single_steps(gpu_lib, dtype):
    """The backward sweep runs steps t, t - 1 (t odd, neither seeded) in one two-step
    launch when both lie in one checkpoint segment, else one step per launch.  Checkpoint
    intervals 3, 7 and 50 split the pairs differently (7: steps 7, 14, ... start segments,
    so pair (7, 6) straddles a boundary and both run alone), and 1 runs every step alone;
    the loss and the u0 gradient must be the same bits in all four, and dJ/dtau equal up
    to the order of its partial sums."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    ux, uy = tiny(seed=11)
    J0, gx0, gy0, gt0 = adjoint_run(ux, uy, 0.55, 50, 8, 1, dtype=dtype)
    for ck in (3, 7, 50):
        say(f"two-step launches {dtype} ckpt_every={ck}")
        J, gx, gy, gt = adjoint_run(ux, uy, 0.55, 50, 8, ck, dtype=dtype)
        assert J == J0, ck
        assert torch.equal(gx, gx0) and torch.equal(gy, gy0), ck
        assert gt == pytest.approx(gt0, rel=1e-12 if dtype == "f64" else 1e-5), ck


def test_two_step_launches_equal_single_steps_16_row_tiles(gpu_lib):
    """At 1024^2 in FP32 the two-step launches use 64 x 16 tiles (1024 of them) instead
    of 64 x 8: the same bits as one step per launch (checkpoint interval 1)."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    _, ux, uy = inp.spectrum_velocity(1024, seed=3, max_mach=0.1)
    say("two-step launches f32 1024^2, 64 x 16 tiles")
    J0, gx0, gy0, gt0 = adjoint_run(ux, uy, 0.55, 10, 16, 1, dtype="f32")
    J, gx, gy, gt = adjoint_run(ux, uy, 0.55, 10, 16, 10, dtype="f32")
    assert J == J0
    assert torch.equal(gx, gx0) and torch.equal(gy, gy0)
    assert gt == pytest.approx(gt0, rel=1e-5)
    assert bool(torch.isfinite(gx).all()) and float(gx.abs().max()) > 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_workspace_with_one_segment_buffer(gpu_lib, dtype):
    """A workspace one segment buffer smaller than the size the library asks for runs
    the recomputation in line instead of beside the sweep: the same bits."""
    import ctypes as C
    from paper_1809_06735_amd import _lib as L
    from paper_1809_06735_amd.adjoint import adjoint_run
    ux, uy = tiny(seed=5)
    n, steps, ck = 32, 50, 7
    cfg = L.AdjointConfig(nx=n, ny=n, dtype={"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype], box=8,
                          ckpt_every=ck, reserved=0, steps=steps, tau=0.55, stream=None)
    full = C.c_size_t()
    L.check(L.load().lbm_adjoint_workspace_bytes(C.byref(cfg), C.byref(full)), "workspace")
    es = 8 if dtype == "f64" else 4
    seg = ((ck + 1) * 9 * n * n * es + 255) // 256 * 256
    small = torch.empty(full.value - seg, dtype=torch.uint8, device="cuda")
    say(f"one segment buffer {dtype}: {full.value - seg} of {full.value} bytes")
    J0, gx0, gy0, gt0 = adjoint_run(ux, uy, 0.55, steps, 8, ck, dtype=dtype)
    J, gx, gy, gt = adjoint_run(ux, uy, 0.55, steps, 8, ck, dtype=dtype, workspace=small)
    assert J == J0 and gt == gt0
    assert torch.equal(gx, gx0) and torch.equal(gy, gy0)
    too_small = torch.empty(full.value - seg - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        adjoint_run(ux, uy, 0.55, steps, 8, ck, dtype=dtype, workspace=too_small)


def test_adjoint_matches_central_differences(gpu_lib):
    """dJ along a random direction and dJ/dtau against central differences of the GPU loss
    (FP64, 32^2, 50 steps): 1e-4 relative."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    ux, uy = tiny(seed=3)
    tau, steps, box = 0.52, 50, 8
    J, gx, gy, gt = adjoint_run(ux, uy, tau, steps, box, 10, dtype="f64")
    rng = np.random.default_rng(1)
    vx, vy = rng.standard_normal(ux.shape), rng.standard_normal(uy.shape)
    h = 1e-5 * np.abs(ux).max()
    jp = adjoint_run(ux + h * vx, uy + h * vy, tau, steps, box, 10, dtype="f64", need_grad=False)[0]
    jm = adjoint_run(ux - h * vx, uy - h * vy, tau, steps, box, 10, dtype="f64", need_grad=False)[0]
    fd = (jp - jm) / (2 * h)
    ad = float((gx.cpu() * torch.as_tensor(vx)).sum() + (gy.cpu() * torch.as_tensor(vy)).sum())
    say(f"directional: adjoint {ad:.8e} fd {fd:.8e}")
    assert ad == pytest.approx(fd, rel=1e-4)
    ht = 1e-5
    jp = adjoint_run(ux, uy, tau + ht, steps, box, 10, dtype="f64", need_grad=False)[0]
    jm = adjoint_run(ux, uy, tau - ht, steps, box, 10, dtype="f64", need_grad=False)[0]
    say(f"tau: adjoint {gt:.8e} fd {(jp - jm) / (2 * ht):.8e}")
    assert gt == pytest.approx((jp - jm) / (2 * ht), rel=1e-4)


def test_autograd_function(gpu_lib):
    from paper_1809_06735_amd.adjoint import adjoint_run, enstrophy_residual_loss
    ux, uy = tiny(seed=5)
    dev = torch.device("cuda")
    vx = torch.tensor(ux, device=dev, requires_grad=True)
    vy = torch.tensor(uy, device=dev, requires_grad=True)
    tau = torch.tensor(0.56, dtype=torch.float64, device=dev, requires_grad=True)
    J = enstrophy_residual_loss(vx, vy, tau, 30, 8, ckpt_every=8, dtype="f64")
    (3.0 * J).backward()
    J2, gx, gy, gt = adjoint_run(ux, uy, 0.56, 30, 8, 8, dtype="f64")
    assert float(J.detach()) == J2
    assert torch.allclose(vx.grad, 3.0 * gx) and torch.allclose(vy.grad, 3.0 * gy)
    assert float(tau.grad) == pytest.approx(3.0 * gt, rel=1e-15)


def test_adjoint512_fp64_central_differences(gpu_lib):
    """Workload adjoint512 (512^2, seed 7, tau 0.51, 2000 steps, checkpoints every 100, box 32)
    in FP64: adjoint directional derivative and dJ/dtau against central differences."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    w = inp.WORKLOADS["adjoint512"]
    _, ux, uy = inp.spectrum_velocity(w.n, seed=w.seed, max_mach=0.05)
    say("adjoint512 fp64 gradient + central differences")
    J, gx, gy, gt = adjoint_run(ux, uy, w.tau, w.steps, 32, 100, dtype="f64")
    rng = np.random.default_rng(2)
    vx, vy = rng.standard_normal(ux.shape), rng.standard_normal(uy.shape)
    h = 1e-4 * np.abs(ux).max()
    jp = adjoint_run(ux + h * vx, uy + h * vy, w.tau, w.steps, 32, 100, dtype="f64", need_grad=False)[0]
    jm = adjoint_run(ux - h * vx, uy - h * vy, w.tau, w.steps, 32, 100, dtype="f64", need_grad=False)[0]
    fd = (jp - jm) / (2 * h)
    ad = float((gx.cpu() * torch.as_tensor(vx)).sum() + (gy.cpu() * torch.as_tensor(vy)).sum())
    say(f"adjoint512 fp64 J {J:.6e}: directional adjoint {ad:.8e} fd {fd:.8e}")
    assert ad == pytest.approx(fd, rel=1e-3)
    ht = 1e-4
    jp = adjoint_run(ux, uy, w.tau + ht, w.steps, 32, 100, dtype="f64", need_grad=False)[0]
    jm = adjoint_run(ux, uy, w.tau - ht, w.steps, 32, 100, dtype="f64", need_grad=False)[0]
    say(f"adjoint512 fp64 dJ/dtau adjoint {gt:.8e} fd {(jp - jm) / (2 * ht):.8e}")
    assert gt == pytest.approx((jp - jm) / (2 * ht), rel=1e-3)


def test_adjoint512_fp32_runs(gpu_lib):
    """Workload adjoint512 in FP32: finite, J within a factor 2 of FP64; the gradient
    agreement with FP64 is reported (FP32 rounding exceeds the residual)."""
    from paper_1809_06735_amd.adjoint import adjoint_run
    w = inp.WORKLOADS["adjoint512"]
    _, ux, uy = inp.spectrum_velocity(w.n, seed=w.seed, max_mach=0.05)
    J32, gx32, gy32, gt32 = adjoint_run(ux, uy, w.tau, w.steps, 32, 100, dtype="f32")
    J64, gx64, gy64, gt64 = adjoint_run(ux, uy, w.tau, w.steps, 32, 100, dtype="f64")
    a = torch.cat([gx32.flatten(), gy32.flatten()])
    b = torch.cat([gx64.flatten(), gy64.flatten()])
    cos = float((a @ b) / (a.norm() * b.norm()))
    say(f"adjoint512 J fp32 {J32:.6e} fp64 {J64:.6e}; dJ/dtau {gt32:.6e} / {gt64:.6e}; "
        f"gradient cosine {cos:.4f}")
    assert np.isfinite(J32) and np.isfinite(gt32) and bool(torch.isfinite(a).all())
    assert 0.5 < J32 / J64 < 2.0
