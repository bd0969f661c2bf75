"""GPU tests of the continuous-batching server.

* every request's result is bitwise the same when served alone (one request per
  batch) and in mixed batches;
* served results equal plain plan steps that replay the same warm-start chain;
* a budget that admits only one or two requests per batch still completes every
  request with the same results;
* the first step of a controller matches the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import rng as ORNG
from oracle import smpc_oracle as O
from synth import workload as W

pytestmark = pytest.mark.gpu


def _small_fleet(n_ctl=5, seed=50):
    """Controllers with different K, H and grids (small, so the oracle is quick)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_ctl):
        K = int(rng.choice([64, 200, 320, 513]))
        H = int(rng.choice([8, 16, 23, 40]))
        inp = W.make_inputs(seed + i, K=K, H=H, dt=0.02, n=int(rng.integers(24, 48)),
                            voxel=0.05, n_boxes=4, n_spheres=3, robot_seed=0)
        out.append(inp)
    return out


def _trace(fleet, n_req=24, seed=7):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(n_req):
        c = int(rng.integers(len(fleet)))
        q0 = fleet[c].q0 + W.f32(rng.normal(scale=0.05, size=7))
        reqs.append((t, c, W.f32(q0), W.f32(rng.normal(scale=0.2, size=7)),
                     fleet[c].T_goal, int(rng.integers(1 << 40))))
    return reqs


def _serve(fleet, reqs, max_batch, budget=256 << 20, submit_all_first=True):
    import torch

    from paper_2512_22575_amd import smpc as S
    planner = S.Planner(fleet[0].robot)
    srv = S.Server(planner, hbm_budget_bytes=budget, max_batch=max_batch)
    grids = [torch.from_numpy(f.grid).cuda() for f in fleet]
    ids = [srv.add_controller(g, f.origin, f.voxel, f.K, f.H, f.dt, f.lam, f.weights,
                              np.full(7, 0.5, np.float32)) for g, f in zip(grids, fleet)]
    done = {}
    pending = list(reqs)
    rounds = 0
    while pending or srv.queued() or srv.in_flight():
        rounds += 1
        assert rounds < 10000, "server made no progress"
        if pending and (submit_all_first or srv.queued() < 3):
            batch = pending if submit_all_first else pending[:3]
            for (tag, c, q0, qd0, T, seed) in batch:
                srv.submit(tag, ids[c], q0, qd0, T, seed)
            pending = pending[len(batch):]
        srv.pump()
        for comp in srv.poll():
            done[comp.tag] = (comp.status, np.array(comp.u0[:]), comp.S_min, comp.Z, comp.ess)
        torch.cuda.synchronize()
    srv.close()
    planner.close()
    return done


def test_alone_equals_mixed_bitwise():
    fleet = _small_fleet()
    reqs = _trace(fleet)
    alone = _serve(fleet, reqs, max_batch=1)
    mixed = _serve(fleet, reqs, max_batch=64)
    assert set(alone) == set(mixed) == {r[0] for r in reqs}
    for tag in alone:
        a, m = alone[tag], mixed[tag]
        assert a[0] == m[0] == 0
        np.testing.assert_array_equal(a[1], m[1])
        assert (a[2], a[3], a[4]) == (m[2], m[3], m[4])


def test_tiny_budget_still_serves_everything():
    fleet = _small_fleet()
    reqs = _trace(fleet, n_req=12)
    ref = _serve(fleet, reqs, max_batch=64)
    from paper_2512_22575_amd import smpc as S
    biggest = max(S.smpc_plan_workspace_bytes(f.K, f.H) for f in fleet)
    tight = _serve(fleet, reqs, max_batch=64, budget=2 * biggest + 4096)
    assert set(tight) == set(ref)
    for tag in ref:
        np.testing.assert_array_equal(ref[tag][1], tight[tag][1])


def test_served_steps_equal_plain_warm_started_steps():
    import torch

    from paper_2512_22575_amd import smpc as S
    fleet = _small_fleet(n_ctl=3)
    reqs = _trace(fleet, n_req=9)
    served = _serve(fleet, reqs, max_batch=8)
    planner = S.Planner(fleet[0].robot)
    ubar = {c: np.zeros((f.H, 7), np.float32) for c, f in enumerate(fleet)}
    for (tag, c, q0, qd0, T, seed) in reqs:
        f = fleet[c]
        dev = torch.device("cuda:0")
        U_in = torch.from_numpy(ubar[c]).to(dev)
        U_out = torch.empty_like(U_in)
        stats = torch.empty(4, device=dev)
        planner.plan_step(q0=q0, qd0=qd0, T_goal=T, grid=torch.from_numpy(f.grid).to(dev),
                          origin=f.origin, voxel=f.voxel, noise=None, K=f.K, H=f.H, U_in=U_in,
                          U_out=U_out, dt=f.dt, lam=f.lam, weights=f.weights, stats_out=stats,
                          seed=seed, sigma=np.full(7, 0.5, np.float32))
        torch.cuda.synchronize()
        U = U_out.cpu().numpy()
        np.testing.assert_array_equal(served[tag][1], U[0])
        st = stats.cpu().numpy()
        assert served[tag][2] == st[0] and served[tag][3] == st[1]
        ubar[c] = np.concatenate([U[1:], np.zeros((1, 7), np.float32)])
    planner.close()


def test_first_step_of_each_controller_matches_oracle():
    fleet = _small_fleet(n_ctl=3)
    reqs = [(i, i, f.q0, f.qd0, f.T_goal, 1000 + i) for i, f in enumerate(fleet)]
    served = _serve(fleet, reqs, max_batch=8)
    for (tag, c, q0, qd0, T, seed) in reqs:
        f = fleet[c]
        eps = ORNG.sample_noise(seed, f.K, f.H, np.full(7, 0.5))
        ref = O.plan_step(f.robot.rounded_f32(), q0, qd0, T, f.grid, f.origin, f.voxel, eps,
                          np.zeros((f.H, 7)), f.dt, f.lam, f.weights)
        np.testing.assert_allclose(served[tag][1], ref["U_star"][0], atol=1e-5)
        assert served[tag][2] == pytest.approx(ref["S_min"], rel=1e-4)


def test_serving_sizes_match_oracle_through_the_server():
    """One request per (K, H) class of the serving workload, K in {256, 1024, 2048, 4096}
    and H in {16, 32, 64}, on grids of 64^3 at 0.03 m, 112^3 at 0.02 m and 160^3 at
    0.01 m (10 to 60 primitives), all submitted together so they share batches: every
    rollout cost, the whole U* before the shift and u*_0 against the oracle run on the
    same counter-based disturbances."""
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import robot as RB
    from tests.gpu_helpers import U_ATOL, assert_costs_close, control_conditioning_tolerance

    rng = np.random.default_rng(55)
    rob = RB.make_robot(0)
    dev = torch.device("cuda:0")
    grids = []
    for n, voxel, n_prim in ((64, 0.03, 10), (112, 0.02, 30), (160, 0.01, 60)):
        g, origin, _, _ = W.make_scene_grid(rng, n, voxel, n_prim // 2, n_prim - n_prim // 2)
        grids.append((g, origin, W.f32s(voxel), torch.from_numpy(g).to(dev)))
    weights = {k: W.f32s(v) for k, v in W.DEFAULT_WEIGHTS.items()}
    dt, lam, sigma = W.f32s(0.02), 1.0, np.full(7, 0.5, np.float32)
    planner = S.Planner(rob)
    srv = S.Server(planner, hbm_budget_bytes=512 << 20, max_batch=64)
    cases = []
    for i, (K, H) in enumerate((K, H) for K in (256, 1024, 2048, 4096) for H in (16, 32, 64)):
        g, origin, voxel, gt = grids[i % 3]
        U_star = torch.full((H, 7), float("nan"), device=dev)
        costs = torch.full((K,), float("nan"), device=dev)
        cid = srv.add_controller(gt, origin, voxel, K, H, dt, lam, weights, sigma,
                                 U_star_out=U_star, costs_out=costs)
        q0 = W.f32(RB.random_joint_config(rng, rob))
        qd0 = W.f32(rng.normal(scale=0.1, size=7))
        T = W.f32(W.random_target_pose(rng))
        seed = int(rng.integers(1 << 40))
        srv.submit(i, cid, q0, qd0, T, seed)
        cases.append((K, H, g, origin, voxel, q0, qd0, T, seed, U_star, costs))
    done = {}
    for _ in range(10000):
        if not (srv.queued() or srv.in_flight()):
            break
        srv.pump()
        for comp in srv.poll():
            done[comp.tag] = comp
        torch.cuda.synchronize()
    for comp in srv.poll():
        done[comp.tag] = comp
    assert set(done) == set(range(len(cases)))
    for i, (K, H, g, origin, voxel, q0, qd0, T, seed, U_star, costs) in enumerate(cases):
        print(f"serving class K={K} H={H} grid {g.shape[0]}^3", flush=True)
        eps = ORNG.sample_noise(seed, K, H, sigma.astype(np.float64))
        ref = O.plan_step(rob.rounded_f32(), q0, qd0, T, g, origin, voxel, eps,
                          np.zeros((H, 7)), dt, lam, weights)
        ref["lam"] = lam
        U = U_star.cpu().numpy().astype(np.float64)
        assert done[i].status == 0
        assert_costs_close(costs.cpu().numpy().astype(np.float64), ref["S"])
        tol = U_ATOL + control_conditioning_tolerance(ref, eps)
        err = np.abs(U - ref["U_star"])
        assert np.all(err <= tol), (K, H, float(err.max()))
        np.testing.assert_array_equal(np.array(done[i].u0[:], np.float32), U[0].astype(np.float32))
        assert done[i].S_min == pytest.approx(ref["S_min"], rel=1e-4)
    srv.close()
    planner.close()
