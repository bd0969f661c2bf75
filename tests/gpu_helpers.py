"""Shared helpers of the GPU tests: run one plan step through the C ABI on cuda:0."""
from __future__ import annotations

import numpy as np

# Parity bar (float32 path against the float64 oracle on identical inputs).
COST_RTOL = 1e-4      # per-rollout cost, relative
COST_ATOL = 1e-6      # absolute floor for costs near zero
U_ATOL = 1e-5         # updated controls, rad/s^2


def run_gpu(inp, *, planner=None, lam=None, U_alias=False, want_costs=True, want_weights=True,
            want_stats=True, stream=None, device="cuda:0"):
    """Run smpc_plan_step on a synth.workload.PlanInputs bundle; returns numpy results."""
    import torch

    from paper_2512_22575_amd import smpc as S
    own = planner is None
    if own:
        planner = S.Planner(inp.robot, device=0)
    dev = torch.device(device)
    grid = torch.from_numpy(np.ascontiguousarray(inp.grid)).to(dev)
    noise = torch.from_numpy(np.ascontiguousarray(inp.noise)).to(dev)
    U_in = torch.from_numpy(np.ascontiguousarray(inp.U_bar)).to(dev)
    U_out = U_in if U_alias else torch.full_like(U_in, float("nan"))
    K = inp.K
    costs = torch.full((K,), float("nan"), device=dev) if want_costs else None
    weights = torch.full((K,), float("nan"), device=dev) if want_weights else None
    stats = torch.full((4,), float("nan"), device=dev) if want_stats else None
    planner.plan_step(q0=inp.q0, qd0=inp.qd0, T_goal=inp.T_goal, grid=grid, origin=inp.origin,
                      voxel=inp.voxel, noise=noise, U_in=U_in, U_out=U_out, dt=inp.dt,
                      lam=inp.lam if lam is None else lam, weights=inp.weights,
                      costs_out=costs, weights_out=weights, stats_out=stats, stream=stream)
    torch.cuda.synchronize()
    out = dict(U_star=U_out.cpu().numpy().astype(np.float64))
    if costs is not None:
        out["S"] = costs.cpu().numpy().astype(np.float64)
    if weights is not None:
        out["w"] = weights.cpu().numpy().astype(np.float64)
    if stats is not None:
        out["stats"] = stats.cpu().numpy().astype(np.float64)
    if own:
        planner.close()
    return out


def assert_costs_close(S_gpu, S_ref, rtol=COST_RTOL, atol=COST_ATOL):
    S_gpu = np.asarray(S_gpu)
    S_ref = np.asarray(S_ref)
    finite = np.isfinite(S_ref)
    assert np.array_equal(finite, np.isfinite(S_gpu)), "finite/non-finite pattern differs"
    err = np.abs(S_gpu[finite] - S_ref[finite])
    bound = rtol * np.abs(S_ref[finite]) + atol
    worst = int(np.argmax(err / bound)) if err.size else 0
    assert np.all(err <= bound), (
        f"cost mismatch: max err/bound {float(np.max(err / bound)):.3g} at rollout {worst}: "
        f"gpu {S_gpu[finite][worst]!r} ref {S_ref[finite][worst]!r}")


def assert_controls_close(U_gpu, U_ref, atol=U_ATOL):
    err = np.abs(np.asarray(U_gpu) - np.asarray(U_ref))
    assert np.all(err <= atol), f"U* mismatch: max abs err {float(err.max()):.3g} > {atol}"


# One float32 rounding, relative: the least error any float32 evaluation of a cost has.
F32_ROUNDING = 2.0 ** -24


def control_conditioning_tolerance(ref, noise):
    """Change of U* that one float32 rounding of every cost can cause (oracle values only).

    U* - U_bar = sum_j w_j eps_j with w = softmax(-S / lambda), so to first order
    dU* = -sum_j (w_j / lambda) (eps_j - sum_i w_i eps_i) dS_j.  With |dS_j| <=
    F32_ROUNDING |S_j| this is at most sum_j (w_j / lambda) |eps_j - mean| |S_j|
    F32_ROUNDING per control.  It is negligible for spread-out weights and exceeds
    U_ATOL only when two or three rollouts with large S nearly tie for the minimum.
    """
    S = np.where(np.isfinite(ref["S"]), ref["S"], 0.0)
    w = ref["w"]
    eps = np.asarray(noise, np.float64)
    mean = np.tensordot(w, eps, axes=1)
    sens = np.tensordot(w * np.abs(S) / ref["lam"], np.abs(eps - mean[None]), axes=1)
    return sens * F32_ROUNDING


def weight_tolerance(ref):
    """Bound on |w_gpu - w_ref| implied by the cost bar.

    To first order dw_m = w_m (dS_m - sum_j w_j dS_j) / lambda; with per-rollout
    cost errors up to COST_RTOL |S| + COST_ATOL the weight error is at most
    2 w_m max|dS| / lambda.  A 1e-7 floor covers float32 rounding of w itself.
    """
    S = ref["S"]
    lam = ref["lam"]
    dS = COST_RTOL * np.max(np.abs(S[np.isfinite(S)])) + COST_ATOL
    return 2.0 * ref["w"] * dS / lam * 1.01 + 1e-7
