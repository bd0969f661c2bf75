"""C-ABI checks that need no GPU: exports, struct layout and argument validation.

Every invalid request must be rejected on the host before any HIP call, so these
run on a machine without a GPU.  No test here passes valid arguments with fake
device pointers while a GPU is present.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_22575_amd import smpc as S
from synth import robot as R
from synth import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smpc.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(smpc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    lib = S.load_library()
    names = header_functions()
    assert {"smpc_create", "smpc_destroy", "smpc_set_robot", "smpc_plan_step",
            "smpc_status_string", "smpc_last_error", "smpc_version"} <= set(names)
    for name in names:
        assert hasattr(lib, name), f"{name} declared in smpc.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}$", out, re.M), f"{name} is not a defined text symbol"


LAYOUT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "smpc.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("smpc_robot_desc sizeof %zu\n", sizeof(smpc_robot_desc));
  printf("smpc_plan_args sizeof %zu\n", sizeof(smpc_plan_args));
  printf("smpc_grid sizeof %zu\n", sizeof(smpc_grid));
  printf("smpc_cost_weights sizeof %zu\n", sizeof(smpc_cost_weights));
  F(smpc_robot_desc, a) F(smpc_robot_desc, q_ref) F(smpc_robot_desc, n_spheres)
  F(smpc_robot_desc, sphere_center) F(smpc_robot_desc, n_pairs) F(smpc_robot_desc, pairs)
  F(smpc_plan_args, T_goal) F(smpc_plan_args, esdf) F(smpc_plan_args, noise)
  F(smpc_plan_args, seed) F(smpc_plan_args, K) F(smpc_plan_args, weights)
  F(smpc_plan_args, U_in) F(smpc_plan_args, stats_out) F(smpc_plan_args, receding)
  F(smpc_plan_args, u0_out) F(smpc_plan_args, state_in) F(smpc_plan_args, state_out)
  F(smpc_grid, nx) F(smpc_grid, origin) F(smpc_grid, voxel) F(smpc_grid, coarse)
  printf("smpc_controller_desc sizeof %zu\n", sizeof(smpc_controller_desc));
  printf("smpc_request sizeof %zu\n", sizeof(smpc_request));
  printf("smpc_completion sizeof %zu\n", sizeof(smpc_completion));
  F(smpc_controller_desc, K) F(smpc_controller_desc, weights) F(smpc_controller_desc, sigma)
  F(smpc_controller_desc, U_star_out) F(smpc_controller_desc, costs_out)
  F(smpc_request, controller) F(smpc_request, q0) F(smpc_request, T_goal) F(smpc_request, seed)
  F(smpc_completion, status) F(smpc_completion, u0) F(smpc_completion, ess)
  printf("smpc_camera sizeof %zu\n", sizeof(smpc_camera));
  printf("smpc_ogm_params sizeof %zu\n", sizeof(smpc_ogm_params));
  F(smpc_camera, width) F(smpc_camera, T_wc) F(smpc_camera, max_depth)
  F(smpc_ogm_params, l_occ) F(smpc_ogm_params, robot_pad)
  return 0;
}
"""


def test_ctypes_structs_match_c_layout(tmp_path):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    src.write_text(LAYOUT_PROBE)
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    rename = {"lambda": "lambda_"}
    for line in out.splitlines():
        struct, field, value = line.split()
        cls = getattr(S, struct)
        if field == "sizeof":
            assert ctypes.sizeof(cls) == int(value), struct
        else:
            assert getattr(cls, rename.get(field, field)).offset == int(value), (struct, field)


def test_status_strings_and_version():
    assert S.smpc_status_string(S.SMPC_OK) == "ok"
    for st in (S.SMPC_E_INVALID_ARG, S.SMPC_E_OOM, S.SMPC_E_DEVICE, S.SMPC_E_NUMERIC,
               S.SMPC_E_UNSUPPORTED):
        assert S.smpc_status_string(st) not in ("ok", "unknown status")
    assert S.smpc_status_string(12345) == "unknown status"
    assert S.smpc_version() >= 100


# ---------------------------------------------------------------------------
# Validation (host-only paths)
# ---------------------------------------------------------------------------

@pytest.fixture()
def ctx():
    st, h = S.smpc_create(0)
    assert st == S.SMPC_OK and h.value
    yield h
    S.smpc_destroy(h)


def test_create_rejects_bad_arguments():
    lib = S.load_library()
    assert lib.smpc_create(None, 0) == S.SMPC_E_INVALID_ARG
    st, h = S.smpc_create(-1)
    assert st == S.SMPC_E_INVALID_ARG and not h.value
    S.smpc_destroy(None)   # no-op


def test_set_robot_validation(ctx):
    good = S.robot_desc(R.make_robot(0))
    assert S.smpc_set_robot(ctx, good) == S.SMPC_OK

    def check(mutate, expected, msg):
        d = S.robot_desc(R.make_robot(0))
        mutate(d)
        assert S.smpc_set_robot(ctx, d) == expected
        assert msg in S.smpc_last_error(ctx)

    check(lambda d: setattr(d, "n_dof", 6), S.SMPC_E_UNSUPPORTED, "n_dof")
    check(lambda d: d.a.__setitem__(2, float("nan")), S.SMPC_E_INVALID_ARG, "DH")
    check(lambda d: d.q_min.__setitem__(3, 5.0), S.SMPC_E_INVALID_ARG, "q_min[3]")
    check(lambda d: d.qdd_max.__setitem__(0, float("inf")), S.SMPC_E_INVALID_ARG, "qdd limit")
    check(lambda d: setattr(d, "n_spheres", 29), S.SMPC_E_INVALID_ARG, "n_spheres")
    check(lambda d: d.sphere_link.__setitem__(0, 8), S.SMPC_E_INVALID_ARG, "sphere_link")
    check(lambda d: d.sphere_link.__setitem__(0, 2), S.SMPC_E_UNSUPPORTED, "more than")
    check(lambda d: d.sphere_radius.__setitem__(5, -0.1), S.SMPC_E_INVALID_ARG, "radius")
    check(lambda d: setattr(d, "n_pairs", 379), S.SMPC_E_INVALID_ARG, "n_pairs")
    check(lambda d: d.pairs[0].__setitem__(1, d.pairs[0][0]), S.SMPC_E_INVALID_ARG, "pair 0")
    check(lambda d: d.pairs[3].__setitem__(0, 28), S.SMPC_E_INVALID_ARG, "pair 3")
    lib = S.load_library()
    assert lib.smpc_set_robot(ctx, None) == S.SMPC_E_INVALID_ARG
    assert lib.smpc_set_robot(None, ctypes.byref(good)) == S.SMPC_E_INVALID_ARG


class _FakeTensor:
    """Stands in for a device tensor in host-only validation tests (never dereferenced)."""

    def __init__(self, shape, ptr=0x1000):
        self.shape = shape
        self._ptr = ptr

    def data_ptr(self):
        return self._ptr


def _args(**over):
    inp = W.tiny()
    K, H = inp.K, inp.H
    kw = dict(q0=inp.q0, qd0=inp.qd0, T_goal=inp.T_goal, grid=_FakeTensor(inp.grid.shape),
              origin=inp.origin, voxel=inp.voxel, noise=_FakeTensor((K, H, 7)),
              U_in=_FakeTensor((H, 7)), U_out=_FakeTensor((H, 7)), K=K, H=H, dt=inp.dt,
              lam=inp.lam, weights=dict(inp.weights))
    kw.update(over)
    return S.plan_args(**kw)


def _expect(ctx, args, status, msg):
    st = S.smpc_plan_step(ctx, args, None)
    assert st == status, (st, S.smpc_last_error(ctx))
    assert msg in S.smpc_last_error(ctx)


def test_plan_step_requires_robot(ctx):
    _expect(ctx, _args(), S.SMPC_E_INVALID_ARG, "no robot")


@pytest.mark.parametrize("over,status,msg", [
    (dict(K=0), S.SMPC_E_INVALID_ARG, "K=0"),
    (dict(H=0), S.SMPC_E_INVALID_ARG, "H=0"),
    (dict(H=65), S.SMPC_E_INVALID_ARG, "H=65"),
    (dict(K=40_000_000, H=64), S.SMPC_E_INVALID_ARG, "2^31"),
    (dict(dt=0.0), S.SMPC_E_INVALID_ARG, "dt"),
    (dict(dt=float("nan")), S.SMPC_E_INVALID_ARG, "dt"),
    (dict(lam=0.0), S.SMPC_E_INVALID_ARG, "lambda"),
    (dict(lam=-1.0), S.SMPC_E_INVALID_ARG, "lambda"),
    (dict(lam=float("inf")), S.SMPC_E_INVALID_ARG, "lambda"),
    (dict(q0=np.full(7, np.nan)), S.SMPC_E_INVALID_ARG, "joint state"),
    (dict(qd0=np.array([0, 0, 0, np.inf, 0, 0, 0])), S.SMPC_E_INVALID_ARG, "joint state"),
    (dict(T_goal=np.diag([1.0, 1.0, 1.0, 2.0])), S.SMPC_E_INVALID_ARG, "last row"),
    (dict(T_goal=np.diag([1.0, 1.1, 1.0, 1.0])), S.SMPC_E_INVALID_ARG, "orthonormal"),
    (dict(voxel=0.0), S.SMPC_E_INVALID_ARG, "voxel"),
    (dict(origin=np.array([0, np.nan, 0])), S.SMPC_E_INVALID_ARG, "origin"),
    (dict(grid=_FakeTensor((1, 4, 4))), S.SMPC_E_INVALID_ARG, ">= 2"),
    (dict(grid=_FakeTensor((4, 4, 4), ptr=0)), S.SMPC_E_INVALID_ARG, "esdf.data"),
    (dict(grid=_FakeTensor((1024, 1024, 1024))), S.SMPC_E_INVALID_ARG, "2^31 bytes"),
    (dict(grid_dtype=7), S.SMPC_E_INVALID_ARG, "dtype"),
    (dict(grid_dtype=S.GRID_F16, grid=_FakeTensor((1024, 1024, 1024))), S.SMPC_E_INVALID_ARG,
     "2^31 bytes"),
    (dict(U_in=None), S.SMPC_E_INVALID_ARG, "U_in"),
    (dict(U_out=None), S.SMPC_E_INVALID_ARG, "U_out"),
    (dict(noise=None, sigma=[0.5, 0.5, -0.1, 0.5, 0.5, 0.5, 0.5]), S.SMPC_E_INVALID_ARG, "sigma"),
    (dict(noise=None, sigma=[0.5, 0.5, 0.5, np.nan, 0.5, 0.5, 0.5]), S.SMPC_E_INVALID_ARG, "sigma"),
])
def test_plan_step_rejects_invalid_arguments(ctx, over, status, msg):
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    _expect(ctx, _args(**over), status, msg)


_H = W.tiny().H
_UB = 7 * 4 * _H  # bytes of one nominal sequence


@pytest.mark.parametrize("over,msg", [
    # The shifted sequence is written while other blocks still read U_in.
    (dict(receding=True), "U_out overlaps U_in"),
    (dict(receding=True, U_out=_FakeTensor((_H, 7), ptr=0x1000 + _UB - 4)), "U_out overlaps U_in"),
    (dict(receding=True, U_out=_FakeTensor((_H, 7), ptr=0x1000 - _UB + 4)), "U_out overlaps U_in"),
    (dict(u0_out=_FakeTensor((7,), ptr=0x1000 + 8)), "overlaps an input"),
    (dict(state_in=_FakeTensor((14,), ptr=0x9000), state_out=_FakeTensor((14,), ptr=0x9000 + 52)),
     "overlaps an input"),
    (dict(state_in=_FakeTensor((14,), ptr=0x9000), u0_out=_FakeTensor((7,), ptr=0x9000 - 24)),
     "overlaps an input"),
    (dict(state_out=_FakeTensor((14,), ptr=0x1000 + _UB - 8)), "overlaps an input"),
])
def test_receding_outputs_must_not_overlap_inputs(ctx, over, msg):
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    _expect(ctx, _args(**over), S.SMPC_E_INVALID_ARG, msg)


def test_receding_flag_is_boolean(ctx):
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    a = _args(U_out=_FakeTensor((_H, 7), ptr=0x1000 + _UB))
    a.receding = 2
    _expect(ctx, a, S.SMPC_E_INVALID_ARG, "receding")


def test_adjacent_receding_buffers_pass_validation(ctx):
    # Touching but disjoint ranges are valid: the call gets past validation and, with
    # no GPU, fails at the first device call.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; this checks the GPU-less failure path")
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    a = _args(receding=True, U_out=_FakeTensor((_H, 7), ptr=0x1000 + _UB),
              u0_out=_FakeTensor((7,), ptr=0x1000 - 28), state_in=_FakeTensor((14,), ptr=0x9000),
              state_out=_FakeTensor((14,), ptr=0x9000 + 56))
    assert S.smpc_plan_step(ctx, a, None) == S.SMPC_E_DEVICE


@pytest.mark.parametrize("field,value", [
    ("w_env", -1.0), ("w_self", float("nan")), ("d_act", float("inf")),
    ("limit_margin_frac", 0.5), ("w_ns", -0.1)])
def test_plan_step_rejects_bad_weights(ctx, field, value):
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    w = dict(W.DEFAULT_WEIGHTS)
    w[field] = value
    _expect(ctx, _args(weights=w), S.SMPC_E_INVALID_ARG, "")


def test_valid_request_without_gpu_fails_loudly(ctx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; this checks the GPU-less failure path")
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    st = S.smpc_plan_step(ctx, _args(), None)
    assert st == S.SMPC_E_DEVICE
    assert S.smpc_last_error(ctx)


def _expect_noalloc(ctx, args, status, msg):
    st = S.smpc_plan_step_noalloc(ctx, args, None)
    assert st == status, (st, S.smpc_last_error(ctx))
    assert msg in S.smpc_last_error(ctx)


def test_noalloc_validates_like_plan_step(ctx):
    _expect_noalloc(ctx, _args(), S.SMPC_E_INVALID_ARG, "no robot")
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    _expect_noalloc(ctx, _args(K=0), S.SMPC_E_INVALID_ARG, "K=0")
    _expect_noalloc(ctx, _args(lam=-1.0), S.SMPC_E_INVALID_ARG, "lambda")
    _expect_noalloc(ctx, _args(receding=True), S.SMPC_E_INVALID_ARG, "U_out overlaps U_in")


def test_noalloc_rejects_a_workspace_beyond_the_static_scratch(ctx):
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    lib = S.load_library()
    limit = 4 << 20
    assert lib.smpc_plan_workspace_bytes(21247, 40) > limit >= lib.smpc_plan_workspace_bytes(21246, 40)
    big = dict(K=21247, H=40, noise=_FakeTensor((21247, 40, 7)), U_in=_FakeTensor((40, 7)),
               U_out=_FakeTensor((40, 7), ptr=0x100000))
    _expect_noalloc(ctx, _args(**big), S.SMPC_E_INVALID_ARG, "static scratch")
    # One rollout fewer fits, and the call stops at the next check (robot not resident).
    fits = dict(big, K=21246, noise=_FakeTensor((21246, 40, 7)))
    _expect_noalloc(ctx, _args(**fits), S.SMPC_E_INVALID_ARG, "not on the device")


def test_plan_step_then_bounds_validates_before_enqueueing(ctx):
    """Bad bounds arguments, then bad plan-step arguments, are refused on the host."""
    args = _args()
    grid = _FakeTensor((16, 16, 16), ptr=0x2000)
    good = dict(next_grid=grid, dtype=S.GRID_F32, origin=(0.0, 0.0, 0.0), voxel=0.05,
                center=(0.0, 0.0, 0.0), radius=1.0, coarse_out=0x3000)
    for bad in (dict(next_grid=_FakeTensor((16, 16, 16), ptr=0)), dict(radius=-1.0),
                dict(radius=float("nan")), dict(coarse_out=0), dict(voxel=0.0),
                dict(center=(float("inf"), 0.0, 0.0)), dict(dtype=7),
                dict(next_grid=_FakeTensor((16, 16, 1), ptr=0x2000))):
        kw = dict(good, **bad)
        st = S.smpc_plan_step_then_bounds(ctx, args, kw["next_grid"], kw["dtype"], kw["origin"],
                                          kw["voxel"], kw["center"], kw["radius"],
                                          kw["coarse_out"], None)
        assert st == S.SMPC_E_INVALID_ARG, bad
        assert "next grid" in S.smpc_last_error(ctx)
    # A table that overlaps the one the step reads without being it.
    import ctypes as C
    a_over = _args()
    a_over.esdf.coarse = C.c_void_p(0x3000)
    st = S.smpc_plan_step_then_bounds(ctx, a_over, grid, S.GRID_F32, (0.0, 0.0, 0.0), 0.05,
                                      (0.0, 0.0, 0.0), 1.0, 0x3004, None)
    assert st == S.SMPC_E_INVALID_ARG
    assert "overlaps" in S.smpc_last_error(ctx)
    # Valid bounds arguments: the plan step's own checks come next (no robot set).
    st = S.smpc_plan_step_then_bounds(ctx, args, grid, S.GRID_F32, (0.0, 0.0, 0.0), 0.05,
                                      (0.0, 0.0, 0.0), 1.0, 0x3000, None)
    assert st == S.SMPC_E_INVALID_ARG
    assert "robot" in S.smpc_last_error(ctx)


def test_noalloc_requires_the_robot_on_the_device(ctx):
    # Setting a robot makes no device call, so nothing is resident until a plan step.
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    _expect_noalloc(ctx, _args(), S.SMPC_E_INVALID_ARG, "run smpc_plan_step once")


def test_robot_reach_holds_every_sphere_centre(ctx):
    """The reach ball: the closed form of the modified-DH chain, and every sphere centre of
    the oracle's kinematics inside it at random joint values (limits ignored)."""
    from oracle import smpc_oracle as O
    st, c, r = S.smpc_robot_reach(ctx)
    assert st == S.SMPC_E_INVALID_ARG  # no robot yet
    rob = R.make_robot(0)
    assert S.smpc_set_robot(ctx, S.robot_desc(rob)) == S.SMPC_OK
    st, c, r = S.smpc_robot_reach(ctx)
    assert st == S.SMPC_OK and np.all(c == 0.0)
    f = rob.rounded_f32()
    chain = np.concatenate([[0.0], np.cumsum(np.hypot(f.a, f.d))])
    want = max(chain[f.sphere_link[i]] + np.linalg.norm(f.sphere_center[i])
               for i in range(f.n_spheres))
    assert r == pytest.approx(want + 1e-3, abs=1e-6)
    q = np.random.default_rng(3).uniform(-np.pi, np.pi, size=(2000, 7))
    centres = O.sphere_centres(f, O.forward_kinematics(f, q))
    reach = np.linalg.norm(centres, axis=-1).max()
    assert reach <= r - 1e-3 + 1e-9
    assert reach > 0.8 * (r - 1e-3)  # the bound is not loose by construction of the test


def test_coarse_ball_validates_on_host():
    lib = S.load_library()
    f3 = ctypes.c_float * 3

    def grid(voxel):
        return S.smpc_grid(ctypes.c_void_p(0x1000), 16, 16, 16, S.GRID_F32, f3(0.0, 0.0, 0.0),
                           voxel, None)

    def call(g, c, r, out=0x2000):
        return lib.smpc_grid_coarse_min_ball(ctypes.byref(g), c, r, ctypes.c_void_p(out), None)

    ok, bad = f3(0.0, 0.0, 0.0), f3(0.0, float("nan"), 0.0)
    assert call(grid(0.05), bad, 1.0) == S.SMPC_E_INVALID_ARG
    assert call(grid(0.05), ok, -1.0) == S.SMPC_E_INVALID_ARG
    assert call(grid(0.05), ok, float("nan")) == S.SMPC_E_INVALID_ARG
    assert call(grid(0.0), ok, 1.0) == S.SMPC_E_INVALID_ARG
    assert call(grid(0.05), ok, 1.0, out=0) == S.SMPC_E_INVALID_ARG


def test_planner_raises_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(OSError, match="missing"):
        S.load_library(str(tmp_path / "libsmpc.so"))


def test_sample_noise_and_grid_conversion_validate_on_host():
    ok_sigma = [0.5] * 7
    assert S.smpc_sample_noise(1, 0, 4, ok_sigma, 0x1000, 0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_sample_noise(1, 4, 0, ok_sigma, 0x1000, 0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_sample_noise(1, 4, 65, ok_sigma, 0x1000, 0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_sample_noise(1, 4, 4, ok_sigma, 0, 0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_sample_noise(1, 4, 4, [0.5] * 6 + [-1.0], 0x1000, 0, None) == \
        S.SMPC_E_INVALID_ARG
    assert S.smpc_sample_noise(1, 5_000_000, 64, ok_sigma, 0x1000, 0, None) == \
        S.SMPC_E_INVALID_ARG
    assert S.smpc_grid_to_f16(0, 0x1000, 8, 2.0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_grid_to_f16(0x1000, 0, 8, 2.0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_grid_to_f16(0x1000, 0x2000, -1, 2.0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_grid_to_f16(0x1000, 0x2000, 8, 0.0, None) == S.SMPC_E_INVALID_ARG
    assert S.smpc_grid_to_f16(0x1000, 0x2000, 0, 2.0, None) == S.SMPC_OK   # nothing to do


def test_server_create_validates_before_device_work(ctx):
    lib = S.load_library()
    assert lib.smpc_server_create(None, ctx, 1 << 20, 4) == S.SMPC_E_INVALID_ARG
    st, h = S.smpc_server_create(ctx, 1 << 20, 0)
    assert st == S.SMPC_E_INVALID_ARG and not h.value
    st, h = S.smpc_server_create(None, 1 << 20, 4)
    assert st == S.SMPC_E_INVALID_ARG
    st, h = S.smpc_server_create(ctx, 1 << 20, 4)      # no robot set yet
    assert st == S.SMPC_E_INVALID_ARG and "no robot" in S.smpc_last_error(ctx)
    S.smpc_server_destroy(None)
    assert S.smpc_server_queued(None) == 0 and S.smpc_server_in_flight(None) == 0


def test_server_create_without_gpu_fails_loudly(ctx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; this checks the GPU-less failure path")
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    st, h = S.smpc_server_create(ctx, 1 << 20, 4)
    assert st == S.SMPC_E_DEVICE and not h.value


def test_edt_validates_on_host():
    need = S.smpc_edt_workspace_bytes(10, 20, 30)
    assert need == 8 * 10 * 20 * 30
    assert S.smpc_edt_workspace_bytes(0, 5, 5) == 0
    assert S.smpc_edt_workspace_bytes(5, 513, 5) == 0
    assert S.smpc_edt_workspace_bytes(512, 512, 512) == 8 * 512 ** 3
    nvox = 6000
    occ, phi, d2, work = 0x10000000, 0x20000000, 0x30000000, 0x40000000
    ok = dict(occ=occ, nx=10, ny=20, nz=30, voxel=0.05, phi_out=phi, d2_out=d2, work=work,
              work_bytes=need, stream=None)
    bad = [dict(occ=0), dict(work=0), dict(phi_out=0, d2_out=0), dict(nx=0), dict(nz=513),
           dict(voxel=0.0), dict(voxel=float("nan")), dict(work_bytes=need - 1),
           dict(work=work + 2),                       # not 4-byte aligned
           dict(work=occ + 100),                      # overlaps the occupancy grid
           dict(phi_out=work + need - 4),             # overlaps the workspace
           dict(d2_out=phi + 4 * nvox - 8)]           # overlaps the field
    for over in bad:
        assert S.smpc_edt(**{**ok, **over}) == S.SMPC_E_INVALID_ARG, over


def test_coarse_bounds_validate_on_host():
    assert S.smpc_grid_coarse_cells(200, 200, 200) == 25 ** 3
    assert S.smpc_grid_coarse_cells(9, 10, 2) == 1 * 2 * 1
    assert S.smpc_grid_coarse_cells(1, 5, 5) == 0
    lib = S.load_library()
    import ctypes
    g = S.smpc_grid(ctypes.c_void_p(0x1000), 10, 10, 10, S.GRID_F32,
                    (ctypes.c_float * 3)(0, 0, 0), 0.1, None)
    assert lib.smpc_grid_coarse_min(ctypes.byref(g), ctypes.c_void_p(0), None) == S.SMPC_E_INVALID_ARG
    assert lib.smpc_grid_coarse_min(None, ctypes.c_void_p(0x2000), None) == S.SMPC_E_INVALID_ARG
    for field, value in (("data", None), ("nx", 1), ("dtype", 7)):
        bad = S.smpc_grid(ctypes.c_void_p(0x1000), 10, 10, 10, S.GRID_F32,
                          (ctypes.c_float * 3)(0, 0, 0), 0.1, None)
        setattr(bad, field, value)
        assert lib.smpc_grid_coarse_min(ctypes.byref(bad), ctypes.c_void_p(0x2000), None) == \
            S.SMPC_E_INVALID_ARG, field


def _ogm_call(ctx, **over):
    cam = S.make_camera(288.0, 288.0, 160.0, 120.0, 320, 240, np.eye(4), 0.1, 4.0)
    prm = S.make_ogm_params(0.025, 0.85, -0.4, -2.0, 3.5, 0.0, 0.01)
    kw = dict(ctx=ctx, q=None, depth=0x10000000, cam=cam, log_odds=0x20000000,
              occ_out=0x30000000, nx=10, ny=20, nz=30, origin=(0.0, 0.0, 0.0), voxel=0.05,
              prm=prm, work=0x40000000, work_bytes=S.smpc_ogm_workspace_bytes(320, 240),
              stream=None)
    for k, v in over.items():
        if k.startswith("cam."):
            setattr(cam, k[4:], v)
        elif k.startswith("prm."):
            setattr(prm, k[4:], v)
        else:
            kw[k] = v
    return S.smpc_ogm_update(**kw)


def test_ogm_validates_on_host(ctx):
    # cleaned image, then the 128-float sphere table
    assert S.smpc_ogm_workspace_bytes(320, 240) == (320 * 240 + 128) * 4
    assert S.smpc_ogm_workspace_bytes(0, 240) == 0
    assert S.smpc_ogm_workspace_bytes(16385, 1) == 0
    assert S.smpc_ogm_update(None, None, 0x1000, S.make_camera(1, 1, 0, 0, 1, 1, np.eye(4),
                             0.1, 1.0), 0x2000, None, 1, 1, 1, (0, 0, 0), 1.0,
                             S.make_ogm_params(0, 1, -1, -2, 2, 0), 0x3000, 1 << 20,
                             None) == S.SMPC_E_INVALID_ARG
    rot = np.eye(4)
    rot[0, 0] = 1.1
    shear = np.eye(4)
    shear[3, 0] = 0.5
    bad = [dict(depth=0), dict(log_odds=0), dict(work=0), dict(q=np.zeros(7)),  # no robot set
           {"cam.fx": 0.0}, {"cam.cy": float("inf")}, {"cam.width": 0},
           {"cam.height": 16385}, {"cam.min_depth": 0.0}, {"cam.max_depth": 0.05},
           {"cam.T_wc": (ctypes.c_float * 16)(*rot.reshape(-1))},
           {"cam.T_wc": (ctypes.c_float * 16)(*shear.reshape(-1))},
           dict(nx=0), dict(nx=2048, ny=1024, nz=1024), dict(voxel=0.0),
           dict(origin=(0.0, float("nan"), 0.0)), {"prm.tol": -0.1}, {"prm.robot_pad": -1e-3},
           {"prm.l_min": 4.0}, {"prm.l_hit": float("nan")},
           dict(work_bytes=S.smpc_ogm_workspace_bytes(320, 240) - 4),
           dict(work=0x40000002),                    # not 4-byte aligned
           dict(occ_out=0x20000000 + 100),           # overlaps the log-odds grid
           dict(work=0x10000000 + 8),                # overlaps the depth image
           ]
    for over in bad:
        assert _ogm_call(ctx, **over) == S.SMPC_E_INVALID_ARG, over
        assert S.smpc_last_error(ctx)
    assert S.smpc_set_robot(ctx, S.robot_desc(R.make_robot(0))) == S.SMPC_OK
    assert _ogm_call(ctx, q=np.full(7, np.nan)) == S.SMPC_E_INVALID_ARG
    assert "q" in S.smpc_last_error(ctx)


def test_ogm_without_gpu_fails_loudly(ctx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; this checks the GPU-less failure path")
    assert _ogm_call(ctx) == S.SMPC_E_DEVICE


def test_plan_workspace_bytes():
    assert S.smpc_plan_workspace_bytes(0, 10) == 0
    assert S.smpc_plan_workspace_bytes(10, 65) == 0
    a = S.smpc_plan_workspace_bytes(4096, 40)
    # costs (double) + per-block partials for 512 blocks of 8 rollouts
    assert a >= 4096 * 8 + 512 * (8 + 4 + 4 + 280 * 4)
    assert S.smpc_plan_workspace_bytes(8192, 40) > a
