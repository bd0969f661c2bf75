"""GPU tests of smpc_plan_step_then_bounds: a receding-horizon loop in which each plan
step's launches also build the bounds of the next period's grid gives, period by
period, bitwise the plan-step outputs (U_out, costs, weights, statistics, u*_0, next
state) and bounds tables of the same loop run as smpc_grid_coarse_min_ball followed by
smpc_plan_step -- with the bounds written to a second table (built by the rollout
launch) or to the table the step reads (built by the merge launch); on float32 and
float16 grids; and on grids neither launch can take (another element type than the
step's grid, rows that are not a multiple of 16 bytes), which get the bounds from a
launch of their own.
"""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu


def _grids(base: np.ndarray, n: int, seed: int, dtype) -> list[np.ndarray]:
    """`n` grids: the scene's, then copies shifted by seeded noise (every period a new
    map, as in the closed loop)."""
    rng = np.random.default_rng(seed)
    out = [base] + [base + rng.normal(scale=0.02, size=base.shape).astype(np.float32)
                    for _ in range(n - 1)]
    from paper_2512_22575_amd import smpc as S
    if dtype == S.GRID_F16:
        return [np.clip(g, -2, 2).astype(np.float16).view(np.int16).copy() for g in out]
    return [np.ascontiguousarray(g, np.float32) for g in out]


def _loop(inp, grids_np, dtype, next_dtype, K, H, fused, alias, next_grids_np=None,
          step_reads_bounds=True):
    """Run len(grids_np) periods; return per-period outputs and the tables."""
    import torch

    from paper_2512_22575_amd import smpc as S
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    grids = [torch.from_numpy(g).to(dev) for g in grids_np]
    # The grids whose bounds the loop builds (the step's own, unless another type).
    bgrids = grids if next_grids_np is None else [torch.from_numpy(g).to(dev)
                                                  for g in next_grids_np]
    nz, ny, nx = grids_np[0].shape
    cells = S.smpc_grid_coarse_cells(nx, ny, nz)
    tabs = [torch.full((cells,), float("nan"), device=dev) for _ in range(1 if alias else 2)]
    planner = S.Planner(inp.robot)
    reach_c, reach_r = planner.robot_reach()
    rng = np.random.default_rng(11)
    U = [torch.from_numpy(inp.U_bar).to(dev), torch.zeros((H, 7), device=dev)]
    X = [torch.from_numpy(np.concatenate([inp.q0, inp.qd0]).astype(np.float32)).to(dev),
         torch.zeros((14,), device=dev)]
    costs = torch.empty((K,), device=dev)
    wts = torch.empty((K,), device=dev)
    stats = torch.empty((4,), device=dev)
    u0 = torch.empty((7,), device=dev)
    n = len(grids)
    tab = lambda i: tabs[i % len(tabs)]  # noqa: E731
    # When the step's grid differs in type from the bounded one, the step reads no table.
    reads_table = next_grids_np is None and step_reads_bounds
    results = []
    if fused:
        st = S.smpc_grid_coarse_min_ball(bgrids[0], next_dtype, inp.origin, inp.voxel, reach_c,
                                         reach_r, tab(0).data_ptr(), stream)
        assert st == S.SMPC_OK
    for i in range(n):
        if not fused:
            st = S.smpc_grid_coarse_min_ball(bgrids[i], next_dtype, inp.origin, inp.voxel,
                                             reach_c, reach_r, tab(i).data_ptr(), stream)
            assert st == S.SMPC_OK
        torch.cuda.synchronize()
        read = tab(i).cpu().numpy().copy()  # the bounds the step reads: grid i's
        noise = torch.from_numpy(W.sample_noise(rng, K, H)).to(dev)
        a = S.plan_args(inp.q0, inp.qd0, inp.T_goal, grids[i], inp.origin, inp.voxel, noise,
                        U[i % 2], U[(i + 1) % 2], K, H, inp.dt, inp.lam, inp.weights,
                        costs_out=costs, weights_out=wts, stats_out=stats, grid_dtype=dtype,
                        coarse=tab(i) if reads_table else None, receding=True, u0_out=u0,
                        state_in=X[i % 2], state_out=X[(i + 1) % 2])
        if fused:
            j = (i + 1) % n  # the last period bounds the first grid again
            st = S.smpc_plan_step_then_bounds(planner._ctx, a, bgrids[j], next_dtype, inp.origin,
                                              inp.voxel, reach_c, reach_r, tab(i + 1).data_ptr(),
                                              stream)
        else:
            st = S.smpc_plan_step(planner._ctx, a, stream)
        assert st == S.SMPC_OK, S.smpc_last_error(planner._ctx)
        torch.cuda.synchronize()
        results.append([t.cpu().numpy().copy() for t in
                        (U[(i + 1) % 2], costs, wts, stats, u0, X[(i + 1) % 2])] + [read])
    if not fused:  # the table the fused loop's last call leaves: grid 0's
        st = S.smpc_grid_coarse_min_ball(bgrids[0], next_dtype, inp.origin, inp.voxel, reach_c,
                                         reach_r, tab(n).data_ptr(), stream)
        assert st == S.SMPC_OK
    torch.cuda.synchronize()
    final = tab(n).cpu().numpy().copy()
    planner.close()
    return results, final


def _check(inp, grids_np, dtype, K, H, alias, next_dtype=None, next_grids_np=None,
           step_reads_bounds=True):
    nd = dtype if next_dtype is None else next_dtype
    a, fa = _loop(inp, grids_np, dtype, nd, K, H, False, alias, next_grids_np,
                  step_reads_bounds)
    b, fb = _loop(inp, grids_np, dtype, nd, K, H, True, alias, next_grids_np,
                  step_reads_bounds)
    names = ("U_out", "costs", "weights", "stats", "u0", "state", "table")
    for i, (ra, rb) in enumerate(zip(a, b)):
        for name, x, y in zip(names, ra, rb):
            np.testing.assert_array_equal(x.view(np.uint32), y.view(np.uint32),
                                          err_msg=f"period {i}: {name}")
        assert ra[3][3] == 0.0
    np.testing.assert_array_equal(fa.view(np.uint32), fb.view(np.uint32))
    # The tables hold bounds (some cells of the reach, and -inf outside it).
    assert np.isfinite(fa).any()


@pytest.mark.parametrize("alias", [False, True])
def test_fused_matches_separate_mid_f32(alias):
    inp = W.mid()
    from paper_2512_22575_amd import smpc as S
    print(f"mid f32 K={inp.K} H={inp.H} alias={alias}", flush=True)
    _check(inp, _grids(inp.grid, 4, 5, S.GRID_F32), S.GRID_F32, inp.K, inp.H, alias)


@pytest.mark.parametrize("alias", [False, True])
def test_fused_matches_separate_reactive_full_size(alias):
    """K = 4096, H = 40 on the 200^3 grid (the bench's period), ragged K too."""
    from paper_2512_22575_amd import smpc as S
    sc = W.ReactiveScenario(seed=3)
    inp = sc.inputs()
    grids = _grids(inp.grid, 3, 6, S.GRID_F32)
    for K in (sc.K, 1000):
        print(f"reactive f32 K={K} H={sc.H} alias={alias}", flush=True)
        _check(inp, grids, S.GRID_F32, K, sc.H, alias)


@pytest.mark.parametrize("alias", [False, True])
def test_fused_matches_separate_f16(alias):
    inp = W.mid()
    from paper_2512_22575_amd import smpc as S
    print(f"mid f16 alias={alias}", flush=True)
    _check(inp, _grids(inp.grid, 3, 7, S.GRID_F16), S.GRID_F16, 512, 24, alias)


def test_fused_step_without_bounds_of_its_own():
    """A step that reads no table (its grid's bounds not built) still builds the next
    grid's bounds in its rollout launch."""
    inp = W.mid()
    from paper_2512_22575_amd import smpc as S
    print("mid f32, step without bounds", flush=True)
    _check(inp, _grids(inp.grid, 3, 12, S.GRID_F32), S.GRID_F32, 700, 20, False,
           step_reads_bounds=False)


def test_unfusable_grids_get_their_own_launch():
    """Rows of 150 float32 (600 bytes) or float16 (300 bytes), and a next grid of another
    element type than the step's, take the unfused path with the same results."""
    from paper_2512_22575_amd import smpc as S
    inp = W.paper_shaped()
    print("paper-shaped f32 / f16", flush=True)
    _check(inp, _grids(inp.grid, 3, 8, S.GRID_F32), S.GRID_F32, inp.K, 40, False)
    _check(inp, _grids(inp.grid, 3, 9, S.GRID_F16), S.GRID_F16, inp.K, 40, True)
    mid = W.mid()
    print("mid f32 step, f16 next grid", flush=True)
    _check(mid, _grids(mid.grid, 3, 10, S.GRID_F32), S.GRID_F32, 256, 16, False,
           next_dtype=S.GRID_F16, next_grids_np=_grids(mid.grid, 3, 10, S.GRID_F16))


def test_fused_call_keeps_the_profile_events():
    """With profiling on, the fused call records its two kernels like smpc_plan_step."""
    import torch

    from paper_2512_22575_amd import smpc as S
    inp = W.mid()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    g = torch.from_numpy(inp.grid).to(dev)
    nz, ny, nx = inp.grid.shape
    tab = torch.empty((S.smpc_grid_coarse_cells(nx, ny, nz),), device=dev)
    planner = S.Planner(inp.robot)
    c, r = planner.robot_reach()
    noise = torch.from_numpy(inp.noise).to(dev)
    U_in = torch.from_numpy(inp.U_bar).to(dev)
    U_out = torch.empty_like(U_in)
    a = S.plan_args(inp.q0, inp.qd0, inp.T_goal, g, inp.origin, inp.voxel, noise, U_in, U_out,
                    inp.K, inp.H, inp.dt, inp.lam, inp.weights)
    planner.profile_enable(2)
    for _ in range(2):
        st = S.smpc_plan_step_then_bounds(planner._ctx, a, g, S.GRID_F32, inp.origin, inp.voxel,
                                          c, r, tab.data_ptr(), stream)
        assert st == S.SMPC_OK
    torch.cuda.synchronize()
    k1, k2 = planner.profile_read(4)
    assert len(k1) == 2 and np.all(k1 > 0) and np.all(k2 > 0)
    planner.close()


def test_receding_horizon_next_bounds():
    """RecedingHorizon.step with next_bounds (the next period's bounds built by the step,
    into the other of two tables) runs the same closed loop as steps that each build
    their own grid's bounds first."""
    import torch

    from paper_2512_22575_amd import smpc as S
    inp = W.mid()
    grids_np = _grids(inp.grid, 4, 13, S.GRID_F32)
    dev = torch.device("cuda:0")
    grids = [torch.from_numpy(g).to(dev) for g in grids_np]
    nz, ny, nx = grids_np[0].shape
    K, H = 512, inp.H

    def run(fused):
        planner = S.Planner(inp.robot)
        c, r = planner.robot_reach()
        stream = torch.cuda.current_stream(dev).cuda_stream
        tabs = [torch.empty((S.smpc_grid_coarse_cells(nx, ny, nz),), device=dev)
                for _ in range(2)]
        loop = S.RecedingHorizon(planner, H, inp.q0, inp.qd0)
        rng = np.random.default_rng(21)
        out = []
        if fused:
            assert S.smpc_grid_coarse_min_ball(grids[0], S.GRID_F32, inp.origin, inp.voxel, c, r,
                                               tabs[0].data_ptr(), stream) == S.SMPC_OK
        for i in range(len(grids)):
            if not fused:
                assert S.smpc_grid_coarse_min_ball(grids[i], S.GRID_F32, inp.origin, inp.voxel,
                                                   c, r, tabs[i % 2].data_ptr(),
                                                   stream) == S.SMPC_OK
            nb = None
            if fused and i + 1 < len(grids):
                nb = (grids[i + 1], S.GRID_F32, inp.origin, inp.voxel, tabs[(i + 1) % 2])
            noise = torch.from_numpy(W.sample_noise(rng, K, H)).to(dev)
            loop.step(T_goal=inp.T_goal, grid=grids[i], origin=inp.origin, voxel=inp.voxel,
                      dt=inp.dt, lam=inp.lam, weights=inp.weights, noise=noise,
                      coarse=tabs[i % 2], next_bounds=nb)
            torch.cuda.synchronize()
            out.append([t.cpu().numpy().copy() for t in (loop.U, loop.state, loop.u0)])
        planner.close()
        return out

    a, b = run(False), run(True)
    for i, (x, y) in enumerate(zip(a, b)):
        for name, u, v in zip(("U", "state", "u0"), x, y):
            np.testing.assert_array_equal(u.view(np.uint32), v.view(np.uint32),
                                          err_msg=f"period {i}: {name}")
