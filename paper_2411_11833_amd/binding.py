"""Thin ctypes binding of libcutamp.so (include/cutamp.h), same names as the C ABI.

Argument marshalling only: device buffers are passed as integer addresses
(``tensor.data_ptr()``), streams as integer ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).  Every call raises
``CtError`` on a non-zero status.  Importing this module fails loudly when
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import inputs as I

LIB_PATH = os.environ.get("CUTAMP_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcutamp.so")

CT_OK, CT_ERR_INVALID_ARG, CT_ERR_UNSUPPORTED, CT_ERR_ALLOC, CT_ERR_DEVICE = range(5)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class CtRobot(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("dh", _dp), ("q_lo", _dp), ("q_hi", _dp), ("tool_d", C.c_double),
                ("n_spheres", C.c_int32), ("spheres", _dp), ("sphere_link", _ip)]


class CtScene(C.Structure):
    _fields_ = [("table", _dp), ("n_obstacles", C.c_int32), ("obstacles", _dp), ("n_objects", C.c_int32),
                ("objects", _dp), ("n_obj_spheres", C.c_int32), ("obj_spheres", _dp),
                ("region_lo", C.c_double * 2), ("region_hi", C.c_double * 2)]


class CtSkeleton(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("object_of_step", _ip), ("grasp_lo", _dp), ("grasp_hi", _dp),
                ("goal_cost", C.c_int32), ("waypoints", C.c_int32), ("q0", _dp), ("self_collision", C.c_int32)]


class CtWeights(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("kin_pos", "kin_rot", "grasp", "place", "jlim", "coll", "goal",
                                          "traj_len", "motion_coll", "self_coll")]


class CtTolerances(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("kin_pos", "kin_rot", "grasp", "place", "jlim", "coll",
                                          "motion_coll", "self_coll")]


class CtAdam(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("lr", "beta1", "beta2", "eps", "grad_scale")]


class CtMlpShape(C.Structure):
    _fields_ = [("d_feat", C.c_int32), ("d_noise", C.c_int32), ("hidden", C.c_int32), ("depth", C.c_int32),
                ("d_out", C.c_int32), ("max_rows", C.c_int64)]


class CtError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {ct_status_string(status)} ({status})")
        self.status = status


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2411_11833_amd.build`")
    # torch first: the library must bind to the HIP runtime that owns torch's
    # device memory and streams (the one torch loaded), not load a second one
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64
    sig = {
        "ct_status_string": (C.c_char_p, [C.c_int]),
        "ct_problem_create": (C.c_int, [C.POINTER(CtRobot), C.POINTER(CtScene), C.POINTER(CtSkeleton),
                                        C.POINTER(CtWeights), C.POINTER(CtTolerances), C.POINTER(vp)]),
        "ct_problem_destroy": (C.c_int, [vp]),
        "ct_problem_info": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "ct_seed_uniform": (C.c_int, [vp, u64, vp, vp, vp, i64, i64, vp]),
        "ct_seed_sampled": (C.c_int, [vp, u64, vp, vp, vp, i64, i64, vp]),
        "ct_cost": (C.c_int, [vp, vp, i64, i64, vp, vp, vp, vp]),
        "ct_cost_grad": (C.c_int, [vp, vp, i64, i64, vp, vp, vp, vp]),
        "ct_adam_apply": (C.c_int, [vp, vp, vp, vp, vp, i64, i64, i64, C.POINTER(CtAdam), vp, vp]),
        "ct_step": (C.c_int, [vp, vp, vp, vp, i64, i64, i64, C.POINTER(CtAdam), vp, vp, vp, vp, vp]),
        "ct_optimize": (C.c_int, [vp, vp, vp, vp, i64, i64, i64, i32, C.POINTER(CtAdam), vp, vp, vp, vp, i32, vp]),
        "ct_set_split": (C.c_int, [vp, i32]),
        "ct_get_split": (C.c_int, [vp, C.POINTER(i32)]),
        "ct_autotune": (C.c_int, [vp, vp, i64, i64, C.POINTER(i32), vp]),
        "ct_feasibility": (C.c_int, [vp, vp, i64, i64, C.c_float, vp, vp, vp]),
        "ct_step_mask": (C.c_int, [vp, vp, i64, i64, vp, i64, vp, vp]),
        "ct_penetrating_pairs": (C.c_int, [vp, vp, i64, i64, vp, vp]),
        "ct_feasibility_noalloc": (C.c_int, [vp, vp, i64, i64, C.c_float, vp, vp]),
        "ct_set_term_weights": (C.c_int, [vp, vp, i64]),
        "ct_al_update": (C.c_int, [vp, vp, i64, i64, C.c_float, vp, vp, vp]),
        "ct_al_weights": (C.c_int, [vp, vp, i64, i64, C.c_float, vp, vp, vp]),
        "ct_compact": (C.c_int, [vp, i64, vp, vp, vp]),
        "ct_gather_block": (C.c_int, [vp, i64, i32, i64, vp, vp, vp, vp, vp, i64, i32, i64, vp]),
        "ct_batch_create": (C.c_int, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(i64), C.POINTER(i64), C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]),
        "ct_batch_destroy": (C.c_int, [vp]),
        "ct_batch_set_tuning": (C.c_int, [vp, i32, i32, i32]),
        "ct_batch_step": (C.c_int, [vp, i64, C.POINTER(CtAdam), vp]),
        "ct_batch_optimize": (C.c_int, [vp, i64, i32, C.POINTER(CtAdam), vp]),
        "ct_batch_autotune": (C.c_int, [vp, C.POINTER(i32), vp]),
        "ct_mlp_create": (C.c_int, [C.POINTER(CtMlpShape), C.POINTER(vp)]),
        "ct_mlp_destroy": (C.c_int, [vp]),
        "ct_mlp_info": (C.c_int, [vp, C.POINTER(i64)]),
        "ct_mlp_set_params": (C.c_int, [vp, vp, vp]),
        "ct_mlp_get_params": (C.c_int, [vp, vp, vp]),
        "ct_mlp_get_grads": (C.c_int, [vp, vp, vp]),
        "ct_mlp_noise": (C.c_int, [vp, u64, vp, i64, vp, vp]),
        "ct_mlp_forward": (C.c_int, [vp, vp, i64, vp, vp, i64, u64, vp, vp]),
        "ct_mlp_infer": (C.c_int, [vp, vp, i64, vp, vp, i64, u64, vp, vp]),
        "ct_mlp_backward": (C.c_int, [vp, vp, i64, vp]),
        "ct_mlp_adam": (C.c_int, [vp, i64, C.POINTER(CtAdam), vp]),
        "ct_mlp_imle_step": (C.c_int, [vp, vp, i64, vp, vp, vp, i64, i32, u64, i64, C.POINTER(CtAdam), vp, vp,
                                       vp]),
        "ct_mlp_sample": (C.c_int, [vp, vp, u64, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    return lib


LIB = _load()


def _chk(status: int, what: str):
    if status != CT_OK:
        raise CtError(status, what)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def ct_status_string(status: int) -> str:
    return LIB.ct_status_string(int(status)).decode()


def ct_problem_create(prob: I.Problem) -> int:
    """Marshal an inputs.Problem into the C descriptors and create a handle
    (an opaque integer).  The numpy buffers only need to live for the call."""
    r, sc, sk, w, e = prob.robot, prob.scene, prob.skeleton, prob.weights, prob.tolerances
    keep = []

    def dp(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return _dptr(a)

    def ip(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(_ip)

    robot = CtRobot(7, dp(r.dh), dp(r.q_lo), dp(r.q_hi), float(r.tool_d), int(r.spheres.shape[0]),
                    dp(r.spheres), ip(r.sphere_link))
    scene = CtScene(dp(sc.table), int(sc.obstacles.shape[0]), dp(sc.obstacles.reshape(-1, 7)),
                    int(sc.objects.shape[0]), dp(sc.objects), int(sc.obj_spheres.shape[1]), dp(sc.obj_spheres),
                    (C.c_double * 2)(*sc.region_lo), (C.c_double * 2)(*sc.region_hi))
    K = sk.n_steps
    glo = np.array([prob.grasp_bounds(k)[0] for k in range(K)])
    ghi = np.array([prob.grasp_bounds(k)[1] for k in range(K)])
    skel = CtSkeleton(K, ip(sk.object_of_step), dp(glo), dp(ghi), int(sk.goal_cost), int(sk.waypoints),
                      dp(sk.q0), int(sk.self_collision))
    weights = CtWeights(w.kin_pos, w.kin_rot, w.grasp, w.place, w.jlim, w.coll, w.goal, w.traj_len,
                        w.motion_coll, w.self_coll)
    tols = CtTolerances(e.kin_pos, e.kin_rot, e.grasp, e.place, e.jlim, e.coll, e.motion_coll, e.self_coll)
    h = C.c_void_p()
    _chk(LIB.ct_problem_create(C.byref(robot), C.byref(scene), C.byref(skel), C.byref(weights),
                               C.byref(tols), C.byref(h)), "ct_problem_create")
    return h.value


def ct_problem_destroy(h: int) -> None:
    _chk(LIB.ct_problem_destroy(h), "ct_problem_destroy")


def ct_problem_info(h: int) -> tuple[int, int, int]:
    d, t, c = C.c_int32(), C.c_int32(), C.c_int32()
    _chk(LIB.ct_problem_info(h, C.byref(d), C.byref(t), C.byref(c)), "ct_problem_info")
    return d.value, t.value, c.value


def ct_seed_uniform(h, seed, X, M, V, n, ld, stream=0):
    _chk(LIB.ct_seed_uniform(h, int(seed) & (2 ** 64 - 1), X, M, V, n, ld, stream), "ct_seed_uniform")


def ct_seed_sampled(h, seed, X, M, V, n, ld, stream=0):
    _chk(LIB.ct_seed_sampled(h, int(seed) & (2 ** 64 - 1), X, M, V, n, ld, stream), "ct_seed_sampled")


def ct_cost(h, X, n, ld, cost, terms=None, mask=None, stream=0):
    _chk(LIB.ct_cost(h, X, n, ld, cost, terms, mask, stream), "ct_cost")


def ct_cost_grad(h, X, n, ld, cost, G, weights=None, stream=0):
    _chk(LIB.ct_cost_grad(h, X, n, ld, cost, G, weights, stream), "ct_cost_grad")


def _adam(lr, beta1, beta2, eps, grad_scale):
    return CtAdam(lr, beta1, beta2, eps, grad_scale)


def ct_adam_apply(h, X, M, V, G, n, ld, t, adam: CtAdam, frozen=None, stream=0):
    _chk(LIB.ct_adam_apply(h, X, M, V, G, n, ld, t, C.byref(adam), frozen, stream), "ct_adam_apply")


def ct_step(h, X, M, V, n, ld, t, adam: CtAdam, frozen=None, cost=None, mask=None, first_sat=None, stream=0):
    _chk(LIB.ct_step(h, X, M, V, n, ld, t, C.byref(adam), frozen, cost, mask, first_sat, stream), "ct_step")


def ct_optimize(h, X, M, V, n, ld, t0, iters, adam: CtAdam, frozen=None, cost=None, mask=None,
                first_sat=None, stop_at_first=0, stream=0):
    _chk(LIB.ct_optimize(h, X, M, V, n, ld, t0, iters, C.byref(adam), frozen, cost, mask, first_sat,
                         int(stop_at_first), stream), "ct_optimize")


def ct_set_split(h, split: int):
    _chk(LIB.ct_set_split(h, split), "ct_set_split")


def ct_get_split(h) -> int:
    s = C.c_int32()
    _chk(LIB.ct_get_split(h, C.byref(s)), "ct_get_split")
    return s.value


def ct_autotune(h, X, n, ld, stream=0) -> int:
    s = C.c_int32()
    _chk(LIB.ct_autotune(h, X, n, ld, C.byref(s), stream), "ct_autotune")
    return s.value


def ct_feasibility(h, terms, n, ld, penalty, counts=None, H=None, stream=0):
    _chk(LIB.ct_feasibility(h, terms, n, ld, penalty, counts, H, stream), "ct_feasibility")


def ct_penetrating_pairs(h, X, n, ld, pairs, stream=0):
    _chk(LIB.ct_penetrating_pairs(h, X, n, ld, pairs, stream), "ct_penetrating_pairs")


def ct_step_mask(h, terms, n, ld, step_mask, ld_mask, count, stream=0):
    _chk(LIB.ct_step_mask(h, terms, n, ld, step_mask, ld_mask, count, stream), "ct_step_mask")


def ct_feasibility_noalloc(h, terms, n, ld, penalty, H, stream=0):
    _chk(LIB.ct_feasibility_noalloc(h, terms, n, ld, penalty, H, stream), "ct_feasibility_noalloc")


def ct_set_term_weights(h, W, ld):
    _chk(LIB.ct_set_term_weights(h, W, ld), "ct_set_term_weights")


def ct_al_update(h, terms, n, ld, rho, mu, W, stream=0):
    _chk(LIB.ct_al_update(h, terms, n, ld, rho, mu, W, stream), "ct_al_update")


def ct_al_weights(h, terms, n, ld, rho, mu, W, stream=0):
    _chk(LIB.ct_al_weights(h, terms, n, ld, rho, mu, W, stream), "ct_al_weights")


def ct_compact(mask, n, idx, count, stream=0):
    _chk(LIB.ct_compact(mask, n, idx, count, stream), "ct_compact")


def ct_gather_block(Xs, lds, rows, n_src, idx, count, X, M, V, ld, row0, n, stream=0):
    _chk(LIB.ct_gather_block(Xs, lds, rows, n_src, idx, count, X, M, V, ld, row0, n, stream), "ct_gather_block")


def _ptrs(vals):
    arr = (C.c_void_p * len(vals))(*[v if v else None for v in vals])
    return arr


def ct_batch_create(problems, X, M, V, n, ld, cost=None, mask=None, first_sat=None, frozen=None) -> int:
    """All list arguments have one entry per skeleton (device addresses as ints)."""
    cnt = len(problems)
    nn = (C.c_int64 * cnt)(*n)
    ll = (C.c_int64 * cnt)(*ld)
    opt = lambda a: _ptrs(a) if a is not None else None  # noqa: E731
    h = C.c_void_p()
    _chk(LIB.ct_batch_create(cnt, _ptrs(problems), _ptrs(X), _ptrs(M), _ptrs(V), nn, ll, opt(cost), opt(mask),
                             opt(first_sat), opt(frozen), C.byref(h)), "ct_batch_create")
    return h.value


def ct_batch_destroy(h):
    _chk(LIB.ct_batch_destroy(h), "ct_batch_destroy")


def ct_batch_set_tuning(h, split=0, workgroups=0, persistent=1):
    _chk(LIB.ct_batch_set_tuning(h, split, workgroups, persistent), "ct_batch_set_tuning")


def ct_batch_step(h, t, adam: CtAdam, stream=0):
    _chk(LIB.ct_batch_step(h, t, C.byref(adam), stream), "ct_batch_step")


def ct_batch_optimize(h, t0, iters, adam: CtAdam, stream=0):
    _chk(LIB.ct_batch_optimize(h, t0, iters, C.byref(adam), stream), "ct_batch_optimize")


def ct_batch_autotune(h, stream=0) -> tuple[int, int]:
    out = (C.c_int32 * 2)()
    _chk(LIB.ct_batch_autotune(h, out, stream), "ct_batch_autotune")
    return out[0], out[1]


def ct_mlp_create(d_feat, d_noise, hidden, depth, d_out, max_rows) -> int:
    shape = CtMlpShape(d_feat, d_noise, hidden, depth, d_out, max_rows)
    h = C.c_void_p()
    _chk(LIB.ct_mlp_create(C.byref(shape), C.byref(h)), "ct_mlp_create")
    return h.value


def ct_mlp_destroy(h):
    _chk(LIB.ct_mlp_destroy(h), "ct_mlp_destroy")


def ct_mlp_info(h) -> int:
    n = C.c_int64()
    _chk(LIB.ct_mlp_info(h, C.byref(n)), "ct_mlp_info")
    return n.value


def ct_mlp_set_params(h, params, stream=0):
    _chk(LIB.ct_mlp_set_params(h, params, stream), "ct_mlp_set_params")


def ct_mlp_get_params(h, params, stream=0):
    _chk(LIB.ct_mlp_get_params(h, params, stream), "ct_mlp_get_params")


def ct_mlp_get_grads(h, grads, stream=0):
    _chk(LIB.ct_mlp_get_grads(h, grads, stream), "ct_mlp_get_grads")


def ct_mlp_noise(h, seed, draw, rows, out, stream=0):
    _chk(LIB.ct_mlp_noise(h, seed, draw, rows, out, stream), "ct_mlp_noise")


def ct_mlp_forward(h, feats, n_feats, feat_of_row, draw, rows, seed, Y, stream=0):
    _chk(LIB.ct_mlp_forward(h, feats, n_feats, feat_of_row, draw, rows, seed, Y, stream), "ct_mlp_forward")


def ct_mlp_infer(h, feats, n_feats, feat_of_row, draw, rows, seed, Y, stream=0):
    _chk(LIB.ct_mlp_infer(h, feats, n_feats, feat_of_row, draw, rows, seed, Y, stream), "ct_mlp_infer")


def ct_mlp_backward(h, dY, rows, stream=0):
    _chk(LIB.ct_mlp_backward(h, dY, rows, stream), "ct_mlp_backward")


def ct_mlp_adam(h, t, adam: CtAdam, stream=0):
    _chk(LIB.ct_mlp_adam(h, t, C.byref(adam), stream), "ct_mlp_adam")


def ct_mlp_imle_step(h, feats, n_feats, feat_of_row, targets, weights, rows, n_draws, seed, t, adam: CtAdam,
                     loss=None, chosen=None, stream=0):
    _chk(LIB.ct_mlp_imle_step(h, feats, n_feats, feat_of_row, targets, weights, rows, n_draws, seed, t,
                              C.byref(adam), loss, chosen, stream), "ct_mlp_imle_step")


def ct_mlp_sample(h, feats, seed, mean, std, lo, hi, wrap, X, M, V, n, ld, stream=0):
    _chk(LIB.ct_mlp_sample(h, feats, seed, mean, std, lo, hi, wrap, X, M, V, n, ld, stream), "ct_mlp_sample")
