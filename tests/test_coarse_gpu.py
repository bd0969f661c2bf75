"""GPU tests of the coarse lower bounds of the distance grid (smpc_grid.coarse).

* the bounds equal their definition (window minimum minus the rounding margin,
  -inf where the window holds a non-finite value), bit for bit;
* plan steps with bounds -- the whole table, or the table restricted to the robot's
  reach -- are bitwise identical to plan steps without them (a skipped lookup has a
  hinge of exactly 0), on the mid and the full-size reactive workloads, a float16 grid
  with on-device sampling, a ragged grid the arm leaves through every face, and through
  the server;
* a table restricted to a ball holds the full bound in every cell a lookup from the
  ball reaches, and the full bound or -inf elsewhere.
"""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu

CELL = 8


def coarse_reference(grid: np.ndarray) -> np.ndarray:
    g = grid.astype(np.float32)
    nz, ny, nx = g.shape
    nc = [(n - 2) // CELL + 1 for n in (nz, ny, nx)]
    out = np.empty(nc, np.float32)
    for cz in range(nc[0]):
        for cy in range(nc[1]):
            for cx in range(nc[2]):
                w = g[cz * CELL:min(cz * CELL + CELL, nz - 1) + 1,
                      cy * CELL:min(cy * CELL + CELL, ny - 1) + 1,
                      cx * CELL:min(cx * CELL + CELL, nx - 1) + 1]
                if not np.isfinite(w).all():
                    out[cz, cy, cx] = -np.inf
                    continue
                mn, mx = np.float32(w.min()), np.float32(np.abs(w).max())
                out[cz, cy, cx] = mn - (np.float32(1e-5) + mx * np.float32(2.0 ** -18))
    return out


def gpu_coarse(grid_t, dtype):
    import torch

    from paper_2512_22575_amd import smpc as S
    nz, ny, nx = grid_t.shape
    n = S.smpc_grid_coarse_cells(nx, ny, nz)
    out = torch.full((n,), float("nan"), device=grid_t.device)
    st = S.smpc_grid_coarse_min(grid_t, dtype, out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    assert st == S.SMPC_OK
    return out


# Rows of 16-byte multiples take the wide kernel (several x chunks at 520 columns);
# the others, and a grid that does not start on a 16-byte boundary, the row kernel.
@pytest.mark.parametrize("shape", [(17, 9, 33), (2, 2, 2), (40, 41, 42), (17, 9, 48), (2, 2, 8),
                                   (10, 12, 520), (40, 41, 200)])
def test_bounds_match_definition(shape):
    import torch

    from paper_2512_22575_amd import smpc as S
    rng = np.random.default_rng(sum(shape))
    grid = rng.normal(scale=0.3, size=shape).astype(np.float32)
    if shape in ((40, 41, 42), (40, 41, 200)):
        grid[5, 30, 7] = np.nan
        grid[33, 2, 40] = np.inf
        grid[39, 40, shape[2] - 1] = -np.inf
    got = gpu_coarse(torch.from_numpy(grid).cuda(), S.GRID_F32).cpu().numpy()
    want = coarse_reference(grid).reshape(-1)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    # float16 storage: bounds of the decoded values
    g16 = np.clip(grid, -2, 2).astype(np.float16)
    got16 = gpu_coarse(torch.from_numpy(g16.view(np.int16).copy()).cuda(), S.GRID_F16)
    want16 = coarse_reference(g16.astype(np.float32)).reshape(-1)
    np.testing.assert_array_equal(got16.cpu().numpy().view(np.uint32), want16.view(np.uint32))


def test_bounds_unaligned_grid_start():
    """A grid whose data starts 4 bytes past a 16-byte boundary (row kernel)."""
    import torch

    from paper_2512_22575_amd import smpc as S
    shape = (12, 10, 24)
    rng = np.random.default_rng(7)
    grid = rng.normal(scale=0.3, size=shape).astype(np.float32)
    buf = torch.zeros(grid.size + 1, device="cuda")
    buf[1:] = torch.from_numpy(grid.reshape(-1)).cuda()
    view = buf[1:].view(shape)
    assert view.data_ptr() % 16 == 4
    got = gpu_coarse(view, S.GRID_F32).cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32),
                                  coarse_reference(grid).reshape(-1).view(np.uint32))


def test_bounds_full_size_reactive_grid():
    """The 200^3 grid of the reactive workload, float32 and float16 (wide kernel)."""
    import torch

    from paper_2512_22575_amd import smpc as S
    sc = W.ReactiveScenario(seed=3, K=64)
    grid = sc.grid()
    got = gpu_coarse(torch.from_numpy(grid).cuda(), S.GRID_F32).cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32),
                                  coarse_reference(grid).reshape(-1).view(np.uint32))
    g16 = np.clip(grid, -2, 2).astype(np.float16)
    got16 = gpu_coarse(torch.from_numpy(g16.view(np.int16).copy()).cuda(), S.GRID_F16)
    want16 = coarse_reference(g16.astype(np.float32)).reshape(-1)
    np.testing.assert_array_equal(got16.cpu().numpy().view(np.uint32), want16.view(np.uint32))


def cells_reached(shape, origin, voxel, center, radius):
    """Cells (cz, cy, cx) holding lookups of points within `radius` of `center` (float64):
    cell k along an axis covers u in [8k, 8k + 8), extended to -inf for k = 0 and to +inf
    for the last cell, u = (p - origin) / voxel - 1/2 (R5's clamping)."""
    nz, ny, nx = shape
    u = (np.asarray(center, np.float64) - np.asarray(origin, np.float64)) / voxel - 0.5
    gaps = []
    for ax, n in enumerate((nx, ny, nz)):
        k = np.arange((n - 2) // CELL + 1)
        lo = np.where(k == 0, -np.inf, 8.0 * k)
        hi = np.where(k == k[-1], np.inf, 8.0 * (k + 1))
        gaps.append(np.maximum(np.maximum(lo - u[ax], u[ax] - hi), 0.0) ** 2)
    g2 = gaps[2][:, None, None] + gaps[1][None, :, None] + gaps[0][None, None, :]
    return g2 <= (radius / voxel) ** 2


def gpu_coarse_ball(grid_t, dtype, origin, voxel, center, radius):
    import torch

    from paper_2512_22575_amd import smpc as S
    nz, ny, nx = grid_t.shape
    out = torch.full((S.smpc_grid_coarse_cells(nx, ny, nz),), float("nan"), device=grid_t.device)
    st = S.smpc_grid_coarse_min_ball(grid_t, dtype, origin, voxel, center, radius, out.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert st == S.SMPC_OK
    return out


@pytest.mark.parametrize("shape", [(40, 41, 200), (17, 9, 33), (10, 12, 520)])
def test_ball_bounds_cover_every_reached_cell(shape):
    """Cells a lookup from the ball reaches hold the full bound bit for bit; every other
    cell holds the full bound or -inf; an infinite radius gives the full table."""
    import torch

    from paper_2512_22575_amd import smpc as S
    rng = np.random.default_rng(sum(shape) + 1)
    grid = rng.normal(scale=0.3, size=shape).astype(np.float32)
    origin, voxel = W.f32([-0.4, -0.3, 0.1]), W.f32s(0.01)
    extent = np.array(shape[::-1]) * voxel
    center = W.f32(origin + extent * np.array([0.3, 0.6, 0.5]))
    radius = float(0.35 * extent.min())
    full = coarse_reference(grid)
    reached = cells_reached(shape, origin, voxel, center, radius)
    assert 0 < reached.sum() < reached.size
    for dtype, g in ((S.GRID_F32, grid), (S.GRID_F16, np.clip(grid, -2, 2).astype(np.float16))):
        if dtype == S.GRID_F16:
            full = coarse_reference(g.astype(np.float32))
            gt = torch.from_numpy(g.view(np.int16).copy()).cuda()
        else:
            gt = torch.from_numpy(g).cuda()
        got = gpu_coarse_ball(gt, dtype, origin, voxel, center, radius).cpu().numpy()
        got = got.reshape(full.shape)
        np.testing.assert_array_equal(got[reached].view(np.uint32), full[reached].view(np.uint32))
        rest = got[~reached]
        assert np.all((rest == -np.inf) | (rest.view(np.uint32) == full[~reached].view(np.uint32)))
        if shape == (40, 41, 200):  # rows of cells wholly outside the ball are skipped
            assert np.any(rest == -np.inf)
        inf = gpu_coarse_ball(gt, dtype, origin, voxel, center, float("inf")).cpu().numpy()
        np.testing.assert_array_equal(inf.view(np.uint32), full.reshape(-1).view(np.uint32))


def _plan(inp, grid_t, coarse, **kw):
    import torch

    from paper_2512_22575_amd import smpc as S
    dev = grid_t.device
    noise = torch.from_numpy(inp.noise).to(dev) if inp.noise is not None else None
    U_in = torch.from_numpy(inp.U_bar).to(dev)
    U_out = torch.empty_like(U_in)
    K = kw["K"] if "K" in kw else inp.K
    costs = torch.empty((K,), device=dev)
    w = torch.empty((K,), device=dev)
    stats = torch.empty((4,), device=dev)
    planner = S.Planner(inp.robot)
    planner.plan_step(q0=inp.q0, qd0=inp.qd0, T_goal=inp.T_goal, grid=grid_t, origin=inp.origin,
                      voxel=inp.voxel, noise=noise, U_in=U_in, U_out=U_out, dt=inp.dt,
                      lam=inp.lam, weights=inp.weights, costs_out=costs, weights_out=w,
                      stats_out=stats, coarse=coarse, **kw)
    torch.cuda.synchronize()
    planner.close()
    return [t.cpu().numpy() for t in (U_out, costs, w, stats)]


def _check_same(inp, grid_t, dtype, **kw):
    """Plan steps without bounds, with the full table and with the table restricted to
    the robot's reach: bitwise the same."""
    from paper_2512_22575_amd import smpc as S
    planner = S.Planner(inp.robot)
    center, radius = planner.robot_reach()
    planner.close()
    a = _plan(inp, grid_t, None, grid_dtype=dtype, **kw)
    for coarse in (gpu_coarse(grid_t, dtype),
                   gpu_coarse_ball(grid_t, dtype, inp.origin, inp.voxel, center, radius)):
        b = _plan(inp, grid_t, coarse, grid_dtype=dtype, **kw)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.view(np.uint32), y.view(np.uint32))


def test_plan_step_identical_mid():
    import torch

    from paper_2512_22575_amd import smpc as S
    inp = W.mid()
    _check_same(inp, torch.from_numpy(inp.grid).cuda(), S.GRID_F32)


def test_plan_step_identical_reactive_full_size():
    import torch

    from paper_2512_22575_amd import smpc as S
    inp = W.ReactiveScenario(seed=3).inputs()
    _check_same(inp, torch.from_numpy(inp.grid).cuda(), S.GRID_F32)


def test_plan_step_identical_f16_sampling():
    import dataclasses

    import torch

    from paper_2512_22575_amd import smpc as S
    mid = W.mid()
    inp = dataclasses.replace(mid, noise=None)
    g16 = np.clip(inp.grid, -2, 2).astype(np.float16)
    grid_t = torch.from_numpy(g16.view(np.int16).copy()).cuda()
    _check_same(inp, grid_t, S.GRID_F16, seed=4, sigma=np.full(7, 0.5, np.float32), K=mid.K,
                H=mid.H)


def test_served_results_identical_with_bounds():
    import torch

    from paper_2512_22575_amd import smpc as S
    fleet = [W.make_inputs(70 + i, K=256, H=16, dt=0.02, n=40, voxel=0.05, n_boxes=6,
                           n_spheres=4, robot_seed=0) for i in range(3)]
    grids = [torch.from_numpy(f.grid).cuda() for f in fleet]
    out = {}
    for use in (False, True):
        planner = S.Planner(fleet[0].robot)
        srv = S.Server(planner, hbm_budget_bytes=64 << 20, max_batch=8)
        ids = [srv.add_controller(g, f.origin, f.voxel, f.K, f.H, f.dt, f.lam, f.weights,
                                  np.full(7, 0.5, np.float32),
                                  coarse=gpu_coarse(g, S.GRID_F32) if use else None)
               for g, f in zip(grids, fleet)]
        for t in range(9):
            f = fleet[t % 3]
            srv.submit(t, ids[t % 3], f.q0, f.qd0, f.T_goal, 100 + t)
        done = {}
        rounds = 0
        while len(done) < 9:
            rounds += 1
            assert rounds < 10000, "server made no progress"
            srv.pump()
            for c in srv.poll():
                done[c.tag] = (c.status, np.array(c.u0[:], np.float32), c.S_min, c.Z)
            torch.cuda.synchronize()
        srv.close()
        planner.close()
        out[use] = done
    for t in range(9):
        a, b = out[False][t], out[True][t]
        assert a[0] == b[0] == 0
        np.testing.assert_array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
        assert (a[2], a[3]) == (b[2], b[3])


def test_plan_step_identical_ragged_grid_spheres_outside_every_face():
    """Sides 41 x 33 x 17 (each 1 mod 8, so the last lookup corner n - 2 sits in the
    last cell with floor(u) = n - 1 clamped to it) and an origin that puts the grid
    across the arm, so that rollout spheres leave it through all six faces: bounds on
    and off give bitwise the same plan step, for float32 and float16 storage."""
    import dataclasses

    import torch

    from oracle import smpc_oracle as O
    from paper_2512_22575_amd import smpc as S
    from synth import scene as SC
    nx, ny, nz, voxel = 41, 33, 17, 0.012
    origin = W.f32([-0.566, -0.098, 0.453])
    rng = np.random.default_rng(1741)
    lo = origin + 0.02
    hi = origin + np.array([nx, ny, nz]) * voxel - 0.02
    prims = SC.random_primitives(rng, lo, hi, 5, 3, speed=0.0)
    grid = SC.signed_distance_grid(SC.occupancy(prims, (nx, ny, nz), origin, voxel), voxel)
    assert grid.shape == (nz, ny, nx)
    base = W.make_inputs(1741, K=384, H=24, dt=0.04, n=16, voxel=0.03, n_boxes=2, n_spheres=0)
    inp = dataclasses.replace(base, grid=grid, origin=origin, voxel=W.f32s(voxel))
    # Every face is crossed by some rollout sphere (oracle kinematics on the inputs).
    rob = inp.robot.rounded_f32()
    q = O.rollout(inp.q0, inp.qd0, inp.U_bar[None] + inp.noise, inp.dt)[0]
    centres = O.sphere_centres(rob, O.forward_kinematics(rob, q.reshape(-1, 7)))
    u = (centres.reshape(-1, 3) - origin) / voxel
    ext = np.array([nx, ny, nz])
    for ax in range(3):
        assert (u[:, ax] < 0).any() and (u[:, ax] > ext[ax]).any(), ax
    grid_t = torch.from_numpy(grid).cuda()
    _check_same(inp, grid_t, S.GRID_F32)
    g16 = np.clip(grid, -2, 2).astype(np.float16)
    _check_same(inp, torch.from_numpy(g16.view(np.int16).copy()).cuda(), S.GRID_F16)
