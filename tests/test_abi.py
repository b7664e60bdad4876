"""The C-ABI library loads, exports every declared entry point, and rejects
malformed requests synchronously -- all without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2411_11833_amd import binding as B
from paper_2411_11833_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cutamp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ct_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 12
    lib = C.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    assert B.ct_status_string(0) == "ok"
    for s in range(1, 5):
        assert B.ct_status_string(s) not in ("ok", "unknown status")
    assert B.ct_status_string(99) == "unknown status"


def _descriptors(prob, **over):
    """C descriptors for a problem, with fields overridden for negative tests."""
    keep = []

    def dp(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def ip(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_int32))

    r, sc, sk = prob.robot, prob.scene, prob.skeleton
    spheres = over.get("spheres", r.spheres)
    robot = B.CtRobot(over.get("n_joints", 7), dp(r.dh), dp(r.q_lo), dp(over.get("q_hi", r.q_hi)), r.tool_d,
                      int(over.get("n_spheres", len(spheres))), dp(spheres),
                      ip(over.get("sphere_link", r.sphere_link)))
    scene = B.CtScene(dp(sc.table), len(sc.obstacles), dp(sc.obstacles), len(sc.objects), dp(sc.objects),
                      sc.obj_spheres.shape[1], dp(sc.obj_spheres), (C.c_double * 2)(*sc.region_lo),
                      (C.c_double * 2)(*over.get("region_hi", sc.region_hi)))
    K = over.get("n_steps", sk.n_steps)
    oos = over.get("object_of_step", sk.object_of_step)
    glo = np.array([prob.grasp_bounds(0)[0]] * max(K, 1))
    ghi = np.array([prob.grasp_bounds(0)[1]] * max(K, 1))
    skel = B.CtSkeleton(K, ip(oos), dp(glo), dp(ghi), over.get("goal", 0), over.get("waypoints", 0), dp(sk.q0),
                        over.get("self_collision", 0))
    w = B.CtWeights(1, 5, 1, 2, 1, over.get("w_coll", 1.0), 0.25, 0.1, 1, over.get("w_self", 1.0))
    e = B.CtTolerances(0.005, 0.05, 0, 0.001, 0, 0.001, 0.001, over.get("e_self", 0.0))
    return keep, robot, scene, skel, w, e


def _create(prob, **over):
    keep, robot, scene, skel, w, e = _descriptors(prob, **over)
    h = C.c_void_p()
    return B.LIB.ct_problem_create(C.byref(robot), C.byref(scene), C.byref(skel), C.byref(w), C.byref(e),
                                   C.byref(h)), h


@pytest.mark.parametrize("over, want", [
    ({"n_joints": 6}, B.CT_ERR_UNSUPPORTED),
    ({"n_steps": 7, "object_of_step": np.arange(7)}, B.CT_ERR_UNSUPPORTED),
    ({"n_steps": 0}, B.CT_ERR_INVALID_ARG),
    ({"object_of_step": np.array([5])}, B.CT_ERR_INVALID_ARG),          # no such object
    ({"q_hi": np.full(7, -3.0)}, B.CT_ERR_INVALID_ARG),                  # hi < lo
    ({"sphere_link": np.full(40, 9)}, B.CT_ERR_INVALID_ARG),             # no such link
    ({"spheres": np.tile([0, 0, 0, -0.05], (40, 1))}, B.CT_ERR_INVALID_ARG),   # negative radius
    ({"n_spheres": 0}, B.CT_ERR_INVALID_ARG),
    ({"region_hi": np.array([-9.0, -9.0])}, B.CT_ERR_INVALID_ARG),
    ({"w_coll": -1.0}, B.CT_ERR_INVALID_ARG),
    ({"goal": 3}, B.CT_ERR_INVALID_ARG),
    ({"waypoints": -1}, B.CT_ERR_INVALID_ARG),
    ({"self_collision": 2}, B.CT_ERR_INVALID_ARG),
    ({"self_collision": 1, "w_self": -1.0}, B.CT_ERR_INVALID_ARG),
    ({"self_collision": 1, "e_self": float("nan")}, B.CT_ERR_INVALID_ARG),
])
def test_create_rejects_bad_descriptors(over, want):
    rc, h = _create(I.single_pick_place(0, 0), **over)
    assert rc == want and h.value is None


def test_create_rejects_duplicate_objects():
    prob = I.packing(0, 0, n_objects=2, n_obstacles=1)
    rc, h = _create(prob, n_steps=2, object_of_step=np.array([1, 1]))
    assert rc == B.CT_ERR_INVALID_ARG


def test_null_arguments():
    h = C.c_void_p()
    assert B.LIB.ct_problem_create(None, None, None, None, None, C.byref(h)) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_problem_create(None, None, None, None, None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_problem_destroy(None) == B.CT_OK
    assert B.LIB.ct_problem_info(None, None, None, None) == B.CT_ERR_INVALID_ARG
    adam = B.CtAdam(1e-2, 0.9, 0.999, 1e-8, 1.0)
    assert B.LIB.ct_cost(None, None, 0, 64, None, None, None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_step(None, None, None, None, 0, 64, 1, C.byref(adam), None, None, None, None, None) == \
        B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_set_split(None, 2) == B.CT_ERR_INVALID_ARG
    with pytest.raises(B.CtError):
        B.ct_problem_info(None)


@pytest.mark.parametrize("bad", [
    dict(d_feat=3), dict(d_noise=6), dict(d_feat=0, d_noise=0), dict(hidden=100), dict(hidden=0),
    dict(depth=0), dict(depth=9), dict(d_out=0), dict(d_out=513), dict(max_rows=100), dict(max_rows=0),
])
def test_mlp_create_rejects_bad_shapes(bad):
    shape = dict(d_feat=120, d_noise=32, hidden=512, depth=3, d_out=84, max_rows=4096)
    shape.update(bad)
    h = C.c_void_p(1234)
    st = B.LIB.ct_mlp_create(C.byref(B.CtMlpShape(**shape)), C.byref(h))
    assert st == B.CT_ERR_INVALID_ARG
    assert h.value is None


def test_mlp_null_handles_rejected():
    adam = B.CtAdam(1e-3, 0.9, 0.999, 1e-8, 1.0)
    assert B.LIB.ct_mlp_create(None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_destroy(None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_info(None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_set_params(None, None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_forward(None, None, 0, None, None, 0, 0, None, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_backward(None, None, 64, None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_adam(None, 1, C.byref(adam), None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_imle_step(None, None, 1, None, None, None, 64, 8, 0, 1, C.byref(adam), None, None,
                                  None) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_mlp_sample(None, None, 0, None, None, None, None, None, None, None, None, 64, 64,
                               None) == B.CT_ERR_INVALID_ARG


def test_feasibility_rejects_bad_arguments():
    assert B.LIB.ct_feasibility(None, None, 0, 64, -1.0, None, None, None) == B.CT_ERR_INVALID_ARG


def test_term_weight_calls_reject_bad_arguments():
    assert B.LIB.ct_set_term_weights(None, None, 0) == B.CT_ERR_INVALID_ARG
    assert B.LIB.ct_al_update(None, None, 0, 64, C.c_float(1.0), None, None, None) == B.CT_ERR_INVALID_ARG
