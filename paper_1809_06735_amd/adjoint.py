"""Differentiable LBGK run: the library's discrete adjoint behind torch.autograd.

loss J(u0, tau) = mean over all box x box windows of (RHS^Omega_V - LHS^Omega_V)^2,
the enstrophy-balance residual (Eq. 11) after `steps` unforced BGK steps from
f = f^eq(rho = 1, u0).  Forward, checkpointing, recomputation and the backward
sweep all run in lbm_adjoint_run; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import time

import torch

from . import _lib as L
from .sim import _dev64, _ptr, _require_gpu, _stream_handle


def adjoint_run(ux0, uy0, tau, steps, box, ckpt_every=100, dtype="f32", need_grad=True,
                device="cuda", stream=None, workspace=None):
    """Returns (J, dJ/dux0, dJ/duy0, dJ/dtau); the gradients are None when need_grad is False."""
    _require_gpu()
    lib = L.load()
    dev = torch.device(device)
    vx = _dev64(ux0, dev)
    vy = _dev64(uy0, dev)
    ny, nx = vx.shape
    cfg = L.AdjointConfig(nx=nx, ny=ny, dtype={"f32": L.LBM_F32, "f64": L.LBM_F64}[dtype],
                          box=int(box), ckpt_every=int(ckpt_every), reserved=0, steps=int(steps),
                          tau=float(tau), stream=_stream_handle(stream))
    nbytes = C.c_size_t()
    L.check(lib.lbm_adjoint_workspace_bytes(C.byref(cfg), C.byref(nbytes)), "lbm_adjoint_workspace_bytes")
    # the size asked for holds two segment buffers; a caller's workspace one buffer smaller
    # also runs (without the overlapped recomputation), a smaller one is refused
    if workspace is None:
        workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    J = C.c_double()
    gt = C.c_double()
    gx = torch.empty_like(vx) if need_grad else None
    gy = torch.empty_like(vy) if need_grad else None
    L.check(lib.lbm_adjoint_run(C.byref(cfg), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                _ptr(vx), _ptr(vy),
                                C.byref(J), _ptr(gx), _ptr(gy), C.byref(gt) if need_grad else None),
            "lbm_adjoint_run")
    return J.value, gx, gy, (gt.value if need_grad else None)


class LBMAdjointFn(torch.autograd.Function):
    """J = LBMAdjointFn.apply(ux0, uy0, tau, steps, box, ckpt_every, dtype)."""

    @staticmethod
    def forward(ctx, ux0, uy0, tau, steps, box, ckpt_every, dtype):
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        J, gx, gy, gt = adjoint_run(ux0.detach(), uy0.detach(), float(tau), steps, box, ckpt_every,
                                    dtype, need_grad=need, device=ux0.device)
        if need:
            ctx.save_for_backward(gx, gy, torch.tensor(gt, dtype=torch.float64, device=ux0.device))
        ctx.need = need
        return torch.tensor(J, dtype=torch.float64, device=ux0.device)

    @staticmethod
    def backward(ctx, gJ):
        gx, gy, gt = ctx.saved_tensors
        # chain rule with the upstream scalar gradient
        return gJ * gx, gJ * gy, gJ * gt, None, None, None, None


def enstrophy_residual_loss(ux0, uy0, tau, steps, box, ckpt_every=100, dtype="f32"):
    """Differentiable loss; ux0, uy0 (and tau, if a tensor) may require grad."""
    tau_t = tau if torch.is_tensor(tau) else torch.tensor(float(tau), dtype=torch.float64,
                                                             device=ux0.device)
    return LBMAdjointFn.apply(ux0, uy0, tau_t, int(steps), int(box), int(ckpt_every), dtype)


def bench_adjoint(log=print, steps=None):
    """Workload adjoint512: 512^2 FP32 decaying spectrum (seed 7), tau 0.51, 2000 steps,
    checkpoints every 100, loss at box 32.  MLUPS of the loss-only run, of the whole
    gradient run and of its backward part, against the plain forward step.  `steps` (a
    multiple of 100) shortens every run, for profiling."""
    import lbm_inputs as inp
    from .sim import Simulation
    w = inp.WORKLOADS["adjoint512"]
    _, ux, uy = inp.spectrum_velocity(w.n, seed=w.seed, max_mach=0.05)
    dev = torch.device("cuda")
    vx = torch.as_tensor(ux, device=dev)
    vy = torch.as_tensor(uy, device=dev)
    sites = w.n * w.n
    nsteps = w.steps if steps is None else int(steps)
    out = {"grid": w.n, "steps": nsteps, "ckpt_every": 100, "box": 32, "dtype": "f32"}
    # tune the step-kernel shape for this grid once; the adjoint run reuses it
    s = Simulation(torch.ones_like(vx), vx, vy, w.tau, dtype="f32")
    out["tile"] = list(s.autotune(trial_steps=10))
    adjoint_run(vx, vy, w.tau, 20, 32, 10)          # warm-up (allocations, code load)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    t_fwd, _ = timed(lambda: adjoint_run(vx, vy, w.tau, nsteps, 32, 100, need_grad=False))
    t_all, res = timed(lambda: adjoint_run(vx, vy, w.tau, nsteps, 32, 100))
    out["loss"] = res[0]
    out["dJ_dtau"] = res[3]
    out["forward_and_loss_MLUPS"] = round(sites * nsteps / t_fwd / 1e6, 1)
    out["gradient_run_MLUPS"] = round(sites * nsteps / t_all / 1e6, 1)
    out["backward_part_MLUPS"] = round(sites * nsteps / max(t_all - t_fwd, 1e-9) / 1e6, 1)
    # the same gradient run in FP64 (the verified gradient of this workload: checked against
    # central differences at 1e-3; FP32 rounding exceeds this loss's residual, see the tests)
    adjoint_run(vx, vy, w.tau, 20, 32, 10, dtype="f64")
    t64_all, res64 = timed(lambda: adjoint_run(vx, vy, w.tau, nsteps, 32, 100, dtype="f64"))
    g32 = torch.cat([res[1].flatten(), res[2].flatten()])
    g64 = torch.cat([res64[1].flatten(), res64[2].flatten()])
    out["fp64"] = {"loss": res64[0], "dJ_dtau": res64[3],
                   "gradient_run_MLUPS": round(sites * nsteps / t64_all / 1e6, 1),
                   "verified": "central differences of the FP64 loss (1e-3) on this workload; "
                               "the oracle's autodiff at 32^2 (1e-8)"}
    out["fp32_vs_fp64"] = {"loss_ratio": res[0] / res64[0],
                           "gradient_cosine": float((g32 @ g64) / (g32.norm() * g64.norm())),
                           "verified": "FP32 adjoint checked against the oracle on a conditioned "
                                       "32^2 case; on this workload FP32 does not resolve the "
                                       "loss's residual, so its gradient direction is not meaningful"}
    # every state kept (one checkpoint segment: the backward pass recomputes nothing);
    # nsteps + 1 states of 9 FP32 populations fit easily in HBM (18.9 GB at 2000 steps)
    cfgk = dict(ckpt_every=nsteps, workspace=None)
    adjoint_run(vx, vy, w.tau, nsteps, 32, **cfgk)       # warm-up (allocation)
    t_keep, res_keep = timed(lambda: adjoint_run(vx, vy, w.tau, nsteps, 32, **cfgk))
    out["keep_every_state"] = {
        "ckpt_every": nsteps, "states_GB": round((nsteps + 1) * 9 * sites * 4 / 1e9, 2),
        "gradient_run_MLUPS": round(sites * nsteps / t_keep / 1e6, 1),
        "same_bits_as_checkpointed": bool(res_keep[0] == res[0] and torch.equal(res_keep[1], res[1])
                                          and torch.equal(res_keep[2], res[2]) and res_keep[3] == res[3])}
    torch.cuda.empty_cache()
    s.step(100)
    tp, _ = timed(lambda: s.step(nsteps))
    out["plain_forward_MLUPS"] = round(sites * nsteps / tp / 1e6, 1)
    s.close()
    log(f"[adjoint] gradient run {out['gradient_run_MLUPS']} MLUPS, backward part "
        f"{out['backward_part_MLUPS']} MLUPS, plain forward {out['plain_forward_MLUPS']} MLUPS; "
        f"every state kept: {out['keep_every_state']['gradient_run_MLUPS']} MLUPS")
    return out
