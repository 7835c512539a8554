"""Python binding of libgsbs.so (include/gsbs.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all of
the method runs in the HIP kernels of the library.  PyTorch is used only to
own device buffers (tensors passed to gsbs_inject with device_ptrs=1) and to
provide the HIP stream.  Importing this module fails loudly if the library has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # load torch's HIP runtime first so that the library binds to the same one
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for host-only calls
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsbs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2509_03313_amd.build.build() "
                      "(or __graft_entry__.build()); there is no fallback path")

_lib = C.CDLL(LIB_PATH)

GSBS_OK = 0
ERRORS = {-1: "EINVAL", -2: "ESTATE", -3: "EMINIMAGE", -4: "ECAPACITY", -5: "EHIP", -6: "ENOMEM"}
MAX_SPECIES = 16
MAX_REACTIONS = 32


class GsbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gsbs error {ERRORS.get(code, code)}: {msg}")
        self.code = code


class gsbs_box(C.Structure):
    _fields_ = [("L_nm", C.c_double), ("capacity", C.c_int64)]


class gsbs_reaction(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("k_in", C.c_double), ("n_products", C.c_int32),
                ("products", C.c_int32 * 3), ("keep_b", C.c_int32)]


class gsbs_pulse(C.Structure):
    _fields_ = [("t_ns", C.c_double), ("n_tracks", C.c_int32), ("reserved", C.c_int32),
                ("spacing_nm", C.c_double), ("mol_per_spur", C.c_double), ("sigma_nm", C.c_double),
                ("let_kev_per_um", C.c_double), ("stream", C.c_uint64), ("frac", C.c_double * 16)]


class gsbs_first_order(C.Structure):
    _fields_ = [("a", C.c_int32), ("n_products", C.c_int32), ("products", C.c_int32 * 2), ("k_per_ns", C.c_double)]


class gsbs_source(C.Structure):
    _fields_ = [("rate_M_per_ns", C.c_double), ("n_products", C.c_int32), ("products", C.c_int32 * 3)]


class gsbs_params(C.Structure):
    _fields_ = [("c_cut", C.c_double), ("rounds", C.c_int32), ("contact_only", C.c_int32),
                ("dt0_ns", C.c_double), ("ratio", C.c_double), ("dt_max_ns", C.c_double),
                ("grid_config", C.c_int32), ("autotune", C.c_int32), ("search_split", C.c_int32),
                ("search_box", C.c_int32), ("step_graph", C.c_int32)]


class gsbs_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("molecule_steps", C.c_int64), ("reactions", C.c_int64),
                ("pair_candidates", C.c_int64), ("max_live", C.c_int64)]


_P = C.POINTER
_vp = C.c_void_p
_i32, _i64, _u64, _d = C.c_int32, C.c_int64, C.c_uint64, C.c_double
_SIGS = {
    "gsbs_default_params": [_P(gsbs_params)],
    "gsbs_create": [_P(gsbs_box), _i32, _u64, _vp, _P(_vp)],
    "gsbs_destroy": [_vp],
    "gsbs_set_species": [_vp, _i32, _P(_d)],
    "gsbs_set_reactions": [_vp, _i32, _P(gsbs_reaction)],
    "gsbs_set_params": [_vp, _P(gsbs_params)],
    "gsbs_get_radii": [_vp, _P(_d)],
    "gsbs_get_dt_max": [_vp, _i32, _P(_d)],
    "gsbs_inject": [_vp, _i32, _d, _i64, _vp, _vp, _d, _i32],
    "gsbs_set_records": [_vp, _i32, _i32, _P(_d)],
    "gsbs_advance_to": [_vp, _P(_d), _i32],
    "gsbs_set_surrogate": [_vp, _vp, _vp],
    "gsbs_get_handover_log": [_vp, _i32, _i64, _P(_d), _P(_d), _P(_d), _P(_i32), _P(_i64)],
    "gsbs_pair_corr": [_vp, _i32, _d, _i32, _P(C.c_float)],
    "gsbs_sync": [_vp],
    "gsbs_get_counts": [_vp, _i32, _P(_i64)],
    "gsbs_get_gvalues": [_vp, _i32, _P(_d)],
    "gsbs_get_current_counts": [_vp, _i32, _P(_i64)],
    "gsbs_get_time": [_vp, _i32, _P(_d)],
    "gsbs_get_n": [_vp, _i32, _P(_i64)],
    "gsbs_get_stats": [_vp, _P(gsbs_stats)],
    "gsbs_get_step_log": [_vp, _i64, _P(_i64), _P(_d), _P(_i32), _P(_i64), _P(_i64)],
    "gsbs_get_tuning": [_i32, _P(_i32), _P(_i32), _P(_d), _P(_i32)],
    "gsbs_set_profiling": [_vp, _i32],
    "gsbs_set_live_timing": [_vp, C.c_uint32],
    "gsbs_get_device_bytes": [_vp, _P(_i64)],
    "gsbs_get_profile": [_vp, _i32, C.c_char_p, _P(_d), _P(_i64), _P(_i64), _P(_i64), _P(_i32)],
    "gsbs_plan_schedule": [_d, _d, _i32, _P(_d), _i32, _P(_d), _d, _d, _d, _P(_d), _i64, _P(_i64)],
    "gsbs_debug_get_state": [_vp, _i32, _i64, _P(C.c_float), _P(C.c_uint8), _P(_u64), _P(_i64)],
    "gsbs_debug_set_state": [_vp, _i64, _P(C.c_float), _P(C.c_uint8), _P(_u64), _i64, _u64],
    "gsbs_debug_step": [_vp, _d, _i32, _P(C.c_float), _i32],
    "gsbs_debug_get_pairs": [_vp, _i64, _P(_u64), _P(C.c_float), _P(C.c_uint32), _P(_i32), _P(_i32),
                             _P(_i64)],
    "gsbs_debug_get_cells": [_vp, _i64, _P(_i32), _P(_u64), _P(_i32), _P(_i64)],
    "gsbs_features": [_vp, _i32, _d, _d, _i32, _d, _vp, _vp, _vp, _i32],
    "gsbs_repopulate": [_vp, _i32, _d, _vp, _i32, _vp, _vp, _d, _i32],
    "gsbs_numodes": [_vp, _i32, _i32, _vp, _vp, _vp, _d, _P(_i32), _i32],
    "gsbs_numodes_noalloc": [_vp, _i32, _i32, _vp, _vp, _vp, _d, _P(_i32)],
    "gsbs_set_sources": [_vp, _i32, _vp],
    "gsbs_set_first_order": [_vp, _i32, _vp],
    "gsbs_save": [_vp, _vp, _i64, _P(_i64)],
    "gsbs_inject_pulse": [_vp, _i32, _P(gsbs_pulse), _P(_i64)],
    "gsbs_load": [_vp, _vp, _i64],
    "gsbs_ssa": [_vp, _i32, _i32, _vp, _vp, _i32, _P(_d), _u64, _u64, _i64, _vp, _P(_i64), _i32],
    "gsbs_mlp_param_count": [_P(_i64)],
    "gsbs_mlp_create": [_i32, _vp, _P(_vp)],
    "gsbs_mlp_destroy": [_vp],
    "gsbs_mlp_set_weights": [_vp, _P(C.c_float), _i64],
    "gsbs_mlp_get_weights": [_vp, _P(C.c_float), _i64],
    "gsbs_mlp_forward": [_vp, _vp, _i32, _vp],
    "gsbs_mlp_get_activation": [_vp, _i32, _i32, _P(C.c_float)],
    "gsbs_mlp_backward": [_vp, _vp, _vp, _i32, _P(C.c_float)],
    "gsbs_mlp_get_grads": [_vp, _P(C.c_float), _i64],
    "gsbs_mlp_adam": [_vp, C.c_float, C.c_float, C.c_float, C.c_float],
    "gsbs_mlp_train_step": [_vp, _vp, _vp, _i32, C.c_float, C.c_float, C.c_float, C.c_float, _P(C.c_float)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.gsbs_last_error.argtypes = []
_lib.gsbs_last_error.restype = C.c_char_p

EXPORTED = sorted(list(_SIGS) + ["gsbs_last_error"])


def _chk(code):
    if code != GSBS_OK:
        raise GsbsError(code, _lib.gsbs_last_error().decode())


def _ptr(a, t):
    return a.ctypes.data_as(_P(t))


def gsbs_last_error() -> str:
    return _lib.gsbs_last_error().decode()


# ------------------------------------------------------ thin wrappers ---
def gsbs_default_params() -> gsbs_params:
    p = gsbs_params()
    _chk(_lib.gsbs_default_params(C.byref(p)))
    return p


def gsbs_create(boxes, seed: int, stream=None):
    arr = (gsbs_box * len(boxes))()
    for k, (L, cap) in enumerate(boxes):
        arr[k].L_nm = float(L)
        arr[k].capacity = int(cap)
    h = _vp()
    _chk(_lib.gsbs_create(arr, len(boxes), int(seed), stream, C.byref(h)))
    return h


def gsbs_destroy(ctx):
    _chk(_lib.gsbs_destroy(ctx))


def gsbs_set_species(ctx, D):
    d = np.ascontiguousarray(D, dtype=np.float64)
    _chk(_lib.gsbs_set_species(ctx, len(d), _ptr(d, _d)))


def gsbs_set_reactions(ctx, reactions):
    arr = (gsbs_reaction * max(len(reactions), 1))()
    for k, r in enumerate(reactions):
        arr[k].a, arr[k].b, arr[k].k_in = int(r.a), int(r.b), float(r.k_in)
        arr[k].n_products = len(r.products)
        for j, p in enumerate(r.products):
            arr[k].products[j] = int(p)
        arr[k].keep_b = 1 if getattr(r, "keep_b", False) else 0
    _chk(_lib.gsbs_set_reactions(ctx, len(reactions), arr))


def gsbs_set_params(ctx, p: gsbs_params):
    _chk(_lib.gsbs_set_params(ctx, C.byref(p)))


def gsbs_get_radii(ctx, n):
    out = np.zeros(max(n, 1))
    _chk(_lib.gsbs_get_radii(ctx, _ptr(out, _d)))
    return out[:n]


def gsbs_get_dt_max(ctx, inst):
    v = _d()
    _chk(_lib.gsbs_get_dt_max(ctx, inst, C.byref(v)))
    return v.value


def gsbs_inject(ctx, inst, t, xyz, species, edep_ev=0.0):
    """xyz (n,3) float32 and species (n,) uint8: numpy arrays (host) or torch
    tensors on the device (passed as device pointers)."""
    if torch is not None and isinstance(xyz, torch.Tensor):
        assert xyz.is_cuda and species.is_cuda and xyz.dtype == torch.float32 and species.dtype == torch.uint8
        xyz = xyz.contiguous()
        species = species.contiguous()
        n = species.numel()
        _chk(_lib.gsbs_inject(ctx, inst, float(t), n, C.c_void_p(xyz.data_ptr()),
                              C.c_void_p(species.data_ptr()), float(edep_ev), 1))
        return
    x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    s = np.ascontiguousarray(species, dtype=np.uint8)
    _chk(_lib.gsbs_inject(ctx, inst, float(t), len(s), x.ctypes.data_as(_vp), s.ctypes.data_as(_vp),
                          float(edep_ev), 0))


def gsbs_set_records(ctx, inst, times):
    t = np.ascontiguousarray(times, dtype=np.float64)
    _chk(_lib.gsbs_set_records(ctx, inst, len(t), _ptr(t, _d)))


GSBS_PLAIN, GSBS_SURROGATE = 0, 1


def gsbs_advance_to(ctx, targets, mode=GSBS_PLAIN):
    t = np.ascontiguousarray(targets, dtype=np.float64)
    _chk(_lib.gsbs_advance_to(ctx, _ptr(t, _d), int(mode)))


class gsbs_surrogate(C.Structure):
    _fields_ = [("settle_ns", C.c_double), ("min_gap_ns", C.c_double), ("tol", C.c_double), ("budget", C.c_double),
                ("guard_margin", C.c_double), ("r_max_nm", C.c_double), ("c_floor_M", C.c_double),
                ("n_ref_max", C.c_int32), ("n_dt", C.c_int32), ("n_c", C.c_int32), ("reserved", C.c_int32),
                ("mu", _vp), ("sd", _vp), ("lo", _vp), ("hi", _vp), ("mu_y", _vp), ("sd_y", _vp),
                ("dt_edges", _vp), ("c_edges", _vp), ("table", _vp)]


def gsbs_set_surrogate(ctx, net_handle, mu=None, sd=None, mu_y=None, sd_y=None, dt_edges=None, c_edges=None,
                       table=None, lo=None, hi=None, settle_ns=1000.0, min_gap_ns=0.0, tol=0.01, budget=0.0,
                       guard_margin=0.1, r_max_nm=200.0, c_floor_M=1e-10, n_ref_max=1024):
    """Set (net_handle not None) or clear the surrogate hand-over of a context
    (see gsbs_surrogate in gsbs.h).  Arrays are host arrays, copied."""
    if net_handle is None:
        _chk(_lib.gsbs_set_surrogate(ctx, None, None))
        return
    keep = []

    def arr(a, t):
        if a is None:
            return None
        v = np.ascontiguousarray(a, dtype=t)
        keep.append(v)
        return v.ctypes.data_as(_vp)

    tb = np.ascontiguousarray(table, dtype=np.float64)
    q = gsbs_surrogate(settle_ns, min_gap_ns, tol, budget, guard_margin, r_max_nm, c_floor_M, n_ref_max,
                       tb.shape[0], tb.shape[1], 0, arr(mu, np.float32), arr(sd, np.float32), arr(lo, np.float32),
                       arr(hi, np.float32), arr(mu_y, np.float32), arr(sd_y, np.float32), arr(dt_edges, np.float64),
                       arr(c_edges, np.float64), arr(tb, np.float64))
    _chk(_lib.gsbs_set_surrogate(ctx, net_handle, C.byref(q)))


def gsbs_get_handover_log(ctx, inst):
    """Hand-over points of an instance: dict of arrays t_switch, t_next, estimate, taken."""
    n = _i64()
    _chk(_lib.gsbs_get_handover_log(ctx, inst, 0, None, None, None, None, C.byref(n)))
    m = max(n.value, 1)
    ts, tn, es = np.zeros(m), np.zeros(m), np.zeros(m)
    tk = np.zeros(m, dtype=np.int32)
    _chk(_lib.gsbs_get_handover_log(ctx, inst, m, _ptr(ts, _d), _ptr(tn, _d), _ptr(es, _d), _ptr(tk, _i32),
                                    C.byref(n)))
    k = n.value
    return dict(t_switch=ts[:k], t_next=tn[:k], estimate=es[:k], taken=tk[:k].astype(bool))


def gsbs_pair_corr(ctx, inst, r_max_nm=200.0, n_ref_max=1024):
    """Pair-correlation function [9][32] of instance inst (see gsbs_features)."""
    out = np.zeros((9, 32), dtype=np.float32)
    _chk(_lib.gsbs_pair_corr(ctx, inst, float(r_max_nm), int(n_ref_max), _ptr(out, C.c_float)))
    return out


def gsbs_sync(ctx):
    _chk(_lib.gsbs_sync(ctx))


def gsbs_get_counts(ctx, inst, n_records, n_species):
    out = np.zeros((max(n_records, 1), n_species), dtype=np.int64)
    _chk(_lib.gsbs_get_counts(ctx, inst, _ptr(out, _i64)))
    return out[:n_records]


def gsbs_get_gvalues(ctx, inst, n_records, n_species):
    out = np.zeros((max(n_records, 1), n_species))
    _chk(_lib.gsbs_get_gvalues(ctx, inst, _ptr(out, _d)))
    return out[:n_records]


def gsbs_get_current_counts(ctx, inst, n_species):
    out = np.zeros(n_species, dtype=np.int64)
    _chk(_lib.gsbs_get_current_counts(ctx, inst, _ptr(out, _i64)))
    return out


def gsbs_get_time(ctx, inst):
    v = _d()
    _chk(_lib.gsbs_get_time(ctx, inst, C.byref(v)))
    return v.value


def gsbs_get_n(ctx, inst):
    v = _i64()
    _chk(_lib.gsbs_get_n(ctx, inst, C.byref(v)))
    return v.value


def gsbs_get_stats(ctx):
    s = gsbs_stats()
    _chk(_lib.gsbs_get_stats(ctx, C.byref(s)))
    return {k: getattr(s, k) for k, _ in gsbs_stats._fields_}


def gsbs_get_step_log(ctx):
    """Profiled steps: dict of arrays step, ms, nc, reach, by_species, cfg, n_est."""
    n = _i64()
    _chk(_lib.gsbs_get_step_log(ctx, 0, None, None, None, None, C.byref(n)))
    m = max(n.value, 1)
    st = np.zeros(m, dtype=np.int64)
    ms = np.zeros(m)
    gr = np.zeros(4 * m, dtype=np.int32)
    ne = np.zeros(m, dtype=np.int64)
    _chk(_lib.gsbs_get_step_log(ctx, m, _ptr(st, _i64), _ptr(ms, _d), _ptr(gr, _i32), _ptr(ne, _i64), C.byref(n)))
    k = n.value
    gr = gr.reshape(-1, 4)
    return dict(step=st[:k], ms=ms[:k], nc=gr[:k, 0], reach=gr[:k, 1], by_species=gr[:k, 2], cfg=gr[:k, 3],
                n_est=ne[:k])


def gsbs_get_tuning():
    """[(occupancy octave, molecule octave, best configuration, mean step ms)]."""
    n = _i32()
    _chk(_lib.gsbs_get_tuning(0, None, None, None, C.byref(n)))
    m = max(n.value, 1)
    keys = np.zeros(2 * m, dtype=np.int32)
    best = np.zeros(m, dtype=np.int32)
    ms = np.zeros(m)
    _chk(_lib.gsbs_get_tuning(m, _ptr(keys, _i32), _ptr(best, _i32), _ptr(ms, _d), C.byref(n)))
    return [(int(keys[2 * k]), int(keys[2 * k + 1]), int(best[k]), float(ms[k])) for k in range(n.value)]


def gsbs_set_profiling(ctx, on: bool):
    _chk(_lib.gsbs_set_profiling(ctx, 1 if on else 0))


KERNEL_SLOTS = ("k_bin", "k_scan", "k_scatter", "k_pairs", "k_pairs_sp", "k_react")


def gsbs_set_live_timing(ctx, kernels=()):
    """Live per-kernel timing of the named kernels (see KERNEL_SLOTS); () turns it off."""
    mask = 0
    for k in kernels:
        mask |= 1 << KERNEL_SLOTS.index(k)
    _chk(_lib.gsbs_set_live_timing(ctx, mask))


def gsbs_get_device_bytes(ctx) -> int:
    v = _i64()
    _chk(_lib.gsbs_get_device_bytes(ctx, C.byref(v)))
    return v.value


def gsbs_get_profile(ctx):
    """{kernel name: (total ms, launches, work units, candidate pairs)} of the profiled steps."""
    names = C.create_string_buffer(32 * 16)
    ms = np.zeros(16)
    nl = np.zeros(16, dtype=np.int64)
    wk = np.zeros(16, dtype=np.int64)
    cd = np.zeros(16, dtype=np.int64)
    n = _i32()
    _chk(_lib.gsbs_get_profile(ctx, 16, names, _ptr(ms, _d), _ptr(nl, _i64), _ptr(wk, _i64), _ptr(cd, _i64),
                               C.byref(n)))
    raw = names.raw
    out = {}
    for k in range(n.value):
        nm = raw[32 * k:32 * k + 32].split(b"\0")[0].decode()
        out[nm] = (float(ms[k]), int(nl[k]), int(wk[k]), int(cd[k]))
    return out


def gsbs_plan_schedule(t_start, t_end, anchors, events, dt0, ratio, dt_max):
    a = np.ascontiguousarray(anchors, dtype=np.float64)
    e = np.ascontiguousarray(events, dtype=np.float64)
    n = _i64()
    _chk(_lib.gsbs_plan_schedule(t_start, t_end, len(a), _ptr(a, _d), len(e), _ptr(e, _d), dt0, ratio, dt_max,
                                 None, 0, C.byref(n)))
    out = np.zeros(max(n.value, 1))
    _chk(_lib.gsbs_plan_schedule(t_start, t_end, len(a), _ptr(a, _d), len(e), _ptr(e, _d), dt0, ratio, dt_max,
                                 _ptr(out, _d), n.value, C.byref(n)))
    return out[:n.value]


def gsbs_debug_get_state(ctx, inst):
    n = _i64()
    _chk(_lib.gsbs_debug_get_state(ctx, inst, 0, None, None, None, C.byref(n)))
    m = n.value
    x = np.zeros((max(m, 1), 3), dtype=np.float32)
    s = np.zeros(max(m, 1), dtype=np.uint8)
    u = np.zeros(max(m, 1), dtype=np.uint64)
    _chk(_lib.gsbs_debug_get_state(ctx, inst, m, _ptr(x, C.c_float), _ptr(s, C.c_uint8), _ptr(u, _u64),
                                   C.byref(n)))
    return x[:m], s[:m], u[:m]


def gsbs_debug_set_state(ctx, xyz, species, uid, step=0, next_uid=None):
    x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    s = np.ascontiguousarray(species, dtype=np.uint8)
    u = np.ascontiguousarray(uid, dtype=np.uint64)
    nu = (int(u.max()) + 1 if len(u) else 0) if next_uid is None else int(next_uid)
    _chk(_lib.gsbs_debug_set_state(ctx, len(s), _ptr(x, C.c_float), _ptr(s, C.c_uint8), _ptr(u, _u64),
                                   int(step), nu))


def gsbs_debug_step(ctx, dt, flags=0, xyz0=None, nc_force=0):
    x0 = None
    if xyz0 is not None:
        x0 = np.ascontiguousarray(xyz0, dtype=np.float32).reshape(-1, 3)
    _chk(_lib.gsbs_debug_step(ctx, float(dt), int(flags), None if x0 is None else _ptr(x0, C.c_float),
                              int(nc_force)))


def gsbs_debug_get_pairs(ctx):
    n = _i64()
    _chk(_lib.gsbs_debug_get_pairs(ctx, 0, None, None, None, None, None, C.byref(n)))
    m = n.value
    uid2 = np.zeros((max(m, 1), 2), dtype=np.uint64)
    P = np.zeros(max(m, 1), dtype=np.float32)
    u24 = np.zeros(max(m, 1), dtype=np.uint32)
    rx = np.zeros(max(m, 1), dtype=np.int32)
    fl = np.zeros(max(m, 1), dtype=np.int32)
    _chk(_lib.gsbs_debug_get_pairs(ctx, m, _ptr(uid2, _u64), _ptr(P, C.c_float), _ptr(u24, C.c_uint32),
                                   _ptr(rx, _i32), _ptr(fl, _i32), C.byref(n)))
    return dict(uid=uid2[:m], P=P[:m], u24=u24[:m], rx=rx[:m], flag=fl[:m])


def gsbs_debug_get_cells(ctx):
    n = _i64()
    nc = _i32()
    _chk(_lib.gsbs_debug_get_cells(ctx, 0, None, None, C.byref(nc), C.byref(n)))
    m = n.value
    cell = np.zeros(max(m, 1), dtype=np.int32)
    u = np.zeros(max(m, 1), dtype=np.uint64)
    _chk(_lib.gsbs_debug_get_cells(ctx, m, _ptr(cell, _i32), _ptr(u, _u64), C.byref(nc), C.byref(n)))
    return cell[:m], u[:m], nc.value


DEBUG_FIXED = 1
DEBUG_LOG_ALL = 2
DEBUG_SEARCH_ONLY = 4
DEBUG_BY_SPECIES = 8
DEBUG_WHOLE_CELLS = 16


# ----------------------------------------------------- convenience layer ---
class Engine:
    """One context: n instances sharing a species/reaction table."""

    def __init__(self, L, seed, D, reactions, params: gsbs_params = None, stream=None, capacity=0):
        Ls = list(L) if np.ndim(L) else [float(L)]
        self.n_inst = len(Ls)
        self.ns = len(D)
        self.nr = len(reactions)
        self.records = [np.zeros(0)] * self.n_inst
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        caps = list(capacity) if np.ndim(capacity) else [capacity] * len(Ls)
        self.ctx = gsbs_create([(x, int(c)) for x, c in zip(Ls, caps)], seed, stream)
        gsbs_set_species(self.ctx, D)
        if params is not None:
            gsbs_set_params(self.ctx, params)
        gsbs_set_reactions(self.ctx, reactions)

    def close(self):
        if self.ctx:
            gsbs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def inject(self, inst, t, xyz, species, edep_ev=0.0):
        gsbs_inject(self.ctx, inst, t, xyz, species, edep_ev)

    def inject_pulse(self, inst, t, n_tracks, frac, **kw) -> int:
        """A pulse generated on the device (see gsbs_inject_pulse)."""
        return gsbs_inject_pulse(self.ctx, inst, t, n_tracks, frac, **kw)

    def set_records(self, inst, times):
        self.records[inst] = np.asarray(times, dtype=np.float64)
        gsbs_set_records(self.ctx, inst, self.records[inst])

    def advance_to(self, t, mode=GSBS_PLAIN):
        tt = np.full(self.n_inst, float(t)) if np.ndim(t) == 0 else np.asarray(t, dtype=np.float64)
        gsbs_advance_to(self.ctx, tt, mode)

    def counts(self, inst=0):
        return gsbs_get_counts(self.ctx, inst, len(self.records[inst]), self.ns)

    def gvalues(self, inst=0):
        return gsbs_get_gvalues(self.ctx, inst, len(self.records[inst]), self.ns)

    def current_counts(self, inst=0):
        return gsbs_get_current_counts(self.ctx, inst, self.ns)

    def time(self, inst=0):
        return gsbs_get_time(self.ctx, inst)

    def n(self, inst=0):
        return gsbs_get_n(self.ctx, inst)

    def stats(self):
        return gsbs_get_stats(self.ctx)

    def save(self) -> bytes:
        return gsbs_save(self.ctx)

    def load(self, blob: bytes, records=None):
        """Restore a checkpoint; records: the per-instance record times the
        saved engine had (kept on the Python side for counts())."""
        gsbs_load(self.ctx, blob)
        if records is not None:
            self.records = [np.asarray(r, dtype=np.float64) for r in records]

    def radii(self):
        return gsbs_get_radii(self.ctx, self.nr)

    def dt_max(self, inst=0):
        return gsbs_get_dt_max(self.ctx, inst)

    def load_workload(self, wl, inst=0, device=False):
        """Queue the injections and records of a workload.Workload."""
        for inj in wl.injections:
            xyz, sp = inj.xyz, inj.species
            if device:
                xyz = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float32)).cuda()
                sp = torch.from_numpy(np.ascontiguousarray(sp, dtype=np.uint8)).cuda()
            self.inject(inst, inj.t, xyz, sp, inj.edep_ev)
        self.set_records(inst, wl.records)


# ----------------------------------------------------------- surrogate state ---
N_FEATURES = 296


def _host_f32(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def gsbs_features(ctx, inst, dt_next, r_max=200.0, n_ref_max=1024, c_floor=1e-10, mu=None, sd=None, out=None):
    """Feature row of instance inst: a host numpy array, or written into the
    device tensor `out` (float32, 296 contiguous values)."""
    mu_h, sd_h = _host_f32(mu), _host_f32(sd)
    mu_p = mu_h.ctypes.data_as(_vp) if mu_h is not None else None
    sd_p = sd_h.ctypes.data_as(_vp) if sd_h is not None else None
    if out is None:
        host = np.zeros(N_FEATURES, dtype=np.float32)
        _chk(_lib.gsbs_features(ctx, inst, dt_next, r_max, n_ref_max, c_floor, mu_p, sd_p,
                                host.ctypes.data_as(_vp), 0))
        return host
    _chk(_lib.gsbs_features(ctx, inst, dt_next, r_max, n_ref_max, c_floor, mu_p, sd_p, C.c_void_p(out.data_ptr()), 1))
    return out


def gsbs_repopulate(ctx, inst, t_new, y, mu_y, sd_y, c_floor=1e-10, relative=False):
    """Homogeneous re-population from normalised log10 concentrations y (host
    array of 7 or a device tensor), or their change from the present state."""
    mu_h, sd_h = _host_f32(mu_y), _host_f32(sd_y)
    if hasattr(y, "data_ptr"):
        yp, dev = C.c_void_p(y.data_ptr()), 1
    else:
        yh = _host_f32(y)
        yp, dev = yh.ctypes.data_as(_vp), 0
    _chk(_lib.gsbs_repopulate(ctx, inst, t_new, yp, dev, mu_h.ctypes.data_as(_vp), sd_h.ctypes.data_as(_vp),
                              c_floor, 1 if relative else 0))


def gsbs_numodes(ctx, c0, dt_ns, rtol=1e-6):
    """Rate equations of the context's reaction table for n well-mixed
    solutions: c0 [n][n_species] mol/L and dt_ns [n] (host arrays or device
    float64 tensors).  Returns (c1, steps) -- c1 of the same kind as c0."""
    if hasattr(c0, "data_ptr"):
        import torch
        if c0.dim() != 2 or c0.dtype != torch.float64 or not c0.is_cuda or not c0.is_contiguous():
            raise ValueError("c0: a contiguous [n][n_species] float64 device tensor")
        n, ns = int(c0.shape[0]), int(c0.shape[1])
        c1 = torch.empty_like(c0)
        if hasattr(dt_ns, "data_ptr"):
            dtt = dt_ns
        else:
            dtt = torch.as_tensor(np.broadcast_to(np.asarray(dt_ns, np.float64), (n,)).copy(), device=c0.device)
        if (dtt.shape != (n,) or dtt.dtype != torch.float64 or dtt.device != c0.device
                or not dtt.is_contiguous()):
            raise ValueError("dt_ns: a contiguous [n] float64 tensor on c0's device")
        steps = np.zeros(max(n, 1), dtype=np.int32)
        _chk(_lib.gsbs_numodes(ctx, n, ns, C.c_void_p(c0.data_ptr()), C.c_void_p(dtt.data_ptr()),
                               C.c_void_p(c1.data_ptr()), float(rtol), _ptr(steps, _i32), 1))
        return c1, steps[:n]
    c0h = np.ascontiguousarray(c0, dtype=np.float64)
    if c0h.ndim != 2:
        raise ValueError("c0: [n][n_species]")
    n, ns = c0h.shape
    dth = np.ascontiguousarray(np.broadcast_to(np.asarray(dt_ns, np.float64), (n,)))
    c1 = np.empty_like(c0h)
    steps = np.zeros(max(n, 1), dtype=np.int32)
    _chk(_lib.gsbs_numodes(ctx, n, ns, c0h.ctypes.data_as(_vp), dth.ctypes.data_as(_vp), c1.ctypes.data_as(_vp),
                           float(rtol), _ptr(steps, _i32), 0))
    return c1, steps[:n]


def gsbs_numodes_noalloc(ctx, c0, dt_ns, c1, rtol=1e-6):
    """gsbs_numodes on device tensors without any allocation in the library:
    c0, c1 [n][n_species] and dt_ns [n] contiguous float64 device tensors (c1
    written in place).  Returns the accepted steps (host)."""
    n, ns = int(c0.shape[0]), int(c0.shape[1])
    for t, shape in ((c0, (n, ns)), (c1, (n, ns)), (dt_ns, (n,))):
        if tuple(t.shape) != shape or str(t.dtype) != "torch.float64" or not t.is_cuda or not t.is_contiguous():
            raise ValueError("c0, c1: [n][n_species], dt_ns: [n]; contiguous float64 device tensors")
    steps = np.zeros(max(n, 1), dtype=np.int32)
    _chk(_lib.gsbs_numodes_noalloc(ctx, n, ns, C.c_void_p(c0.data_ptr()), C.c_void_p(dt_ns.data_ptr()),
                                   C.c_void_p(c1.data_ptr()), float(rtol), _ptr(steps, _i32)))
    return steps[:n]


def gsbs_inject_pulse(ctx, inst, t_ns, n_tracks, frac, stream=0, spacing_nm=100.0, mol_per_spur=5.13,
                      sigma_nm=2.0, let_kev_per_um=0.8) -> int:
    """A pulse generated on the device from the counter-based spur model;
    returns the number of molecules queued."""
    p = gsbs_pulse()
    p.t_ns = float(t_ns)
    p.n_tracks = int(n_tracks)
    p.spacing_nm = float(spacing_nm)
    p.mol_per_spur = float(mol_per_spur)
    p.sigma_nm = float(sigma_nm)
    p.let_kev_per_um = float(let_kev_per_um)
    p.stream = int(stream)
    for k, f in enumerate(frac):
        p.frac[k] = float(f)
    n = _i64()
    _chk(_lib.gsbs_inject_pulse(ctx, int(inst), C.byref(p), C.byref(n)))
    return n.value


def gsbs_save(ctx) -> bytes:
    """Checkpoint of the whole context state (see gsbs_load)."""
    n = _i64()
    _chk(_lib.gsbs_save(ctx, None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _chk(_lib.gsbs_save(ctx, C.cast(buf, _vp), n.value, C.byref(n)))
    return buf.raw[:n.value]


def gsbs_load(ctx, blob: bytes):
    """Restore a checkpoint into a context with the same instances and edges."""
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _chk(_lib.gsbs_load(ctx, C.cast(buf, _vp), len(blob)))


def gsbs_set_first_order(ctx, channels):
    """First-order channels: objects with a, k (per ns) and products (at most
    two; see workload.FirstOrder)."""
    arr = (gsbs_first_order * max(len(channels), 1))()
    for q, f in enumerate(channels):
        arr[q].a = int(f.a)
        arr[q].k_per_ns = float(f.k)
        arr[q].n_products = len(f.products)
        for j, p in enumerate(f.products):
            arr[q].products[j] = int(p)
    _chk(_lib.gsbs_set_first_order(ctx, len(channels), C.cast(arr, _vp)))


def gsbs_set_sources(ctx, sources):
    """Zero-order sources: objects with rate (mol/L/ns) and products (see
    workload.Source); used by gsbs_numodes and gsbs_ssa."""
    arr = (gsbs_source * max(len(sources), 1))()
    for k, q in enumerate(sources):
        arr[k].rate_M_per_ns = float(q.rate)
        arr[k].n_products = len(q.products)
        for j, p in enumerate(q.products):
            arr[k].products[j] = int(p)
    _chk(_lib.gsbs_set_sources(ctx, len(sources), C.cast(arr, _vp)))


def gsbs_ssa(ctx, n0, volume_L, t_rec_ns, seed, stream0=0, max_events=1 << 32):
    """Gillespie runs of the context's reaction table in n volumes: n0
    [n][n_species] int32 counts and volume_L [n] litres (host arrays, or
    int32 / float64 device tensors), t_rec_ns the record times.  Returns
    (out [n][n_rec][n_species] of the kind of n0, events [n])."""
    t_rec = np.ascontiguousarray(np.atleast_1d(np.asarray(t_rec_ns, np.float64)))
    if hasattr(n0, "data_ptr"):
        import torch
        if n0.dim() != 2 or n0.dtype != torch.int32 or not n0.is_cuda or not n0.is_contiguous():
            raise ValueError("n0: a contiguous [n][n_species] int32 device tensor")
        n, ns = int(n0.shape[0]), int(n0.shape[1])
        if hasattr(volume_L, "data_ptr"):
            vol = volume_L
        else:
            vol = torch.as_tensor(np.broadcast_to(np.asarray(volume_L, np.float64), (n,)).copy(), device=n0.device)
        if vol.shape != (n,) or vol.dtype != torch.float64 or vol.device != n0.device or not vol.is_contiguous():
            raise ValueError("volume_L: a contiguous [n] float64 tensor on n0's device")
        out = torch.empty((n, len(t_rec), ns), dtype=torch.int32, device=n0.device)
        ev = np.zeros(max(n, 1), dtype=np.int64)
        _chk(_lib.gsbs_ssa(ctx, n, ns, C.c_void_p(n0.data_ptr()), C.c_void_p(vol.data_ptr()), len(t_rec),
                           _ptr(t_rec, _d), int(seed), int(stream0), int(max_events), C.c_void_p(out.data_ptr()),
                           _ptr(ev, _i64), 1))
        return out, ev[:n]
    n0h = np.ascontiguousarray(n0, dtype=np.int32)
    if n0h.ndim != 2:
        raise ValueError("n0: [n][n_species]")
    n, ns = n0h.shape
    volh = np.ascontiguousarray(np.broadcast_to(np.asarray(volume_L, np.float64), (n,)))
    out = np.zeros((n, len(t_rec), ns), dtype=np.int32)
    ev = np.zeros(max(n, 1), dtype=np.int64)
    _chk(_lib.gsbs_ssa(ctx, n, ns, n0h.ctypes.data_as(_vp), volh.ctypes.data_as(_vp), len(t_rec), _ptr(t_rec, _d),
                       int(seed), int(stream0), int(max_events), out.ctypes.data_as(_vp), _ptr(ev, _i64), 0))
    return out, ev[:n]


# ------------------------------------------------------------- surrogate MLP ---
MLP_IN, MLP_OUT, MLP_HIDDEN = 296, 7, 256


def mlp_param_count() -> int:
    n = _i64()
    _chk(_lib.gsbs_mlp_param_count(C.byref(n)))
    return n.value


class Mlp:
    """The surrogate perceptron on the device (gsbs_mlp_*).  x / t / y are
    device tensors (float32, contiguous, [batch][width])."""

    def __init__(self, max_batch: int, stream=None):
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        h = _vp()
        _chk(_lib.gsbs_mlp_create(int(max_batch), stream, C.byref(h)))
        self.h = h
        self.n = mlp_param_count()

    def close(self):
        if self.h:
            _chk(_lib.gsbs_mlp_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.n
        _chk(_lib.gsbs_mlp_set_weights(self.h, _ptr(w, C.c_float), self.n))

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.n, dtype=np.float32)
        _chk(_lib.gsbs_mlp_get_weights(self.h, _ptr(w, C.c_float), self.n))
        return w

    def get_grads(self) -> np.ndarray:
        g = np.zeros(self.n, dtype=np.float32)
        _chk(_lib.gsbs_mlp_get_grads(self.h, _ptr(g, C.c_float), self.n))
        return g

    def forward(self, x, y=None):
        B = int(x.shape[0])
        if y is None:
            y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=x.device)
        _chk(_lib.gsbs_mlp_forward(self.h, C.c_void_p(x.data_ptr()), B, C.c_void_p(y.data_ptr())))
        return y

    def activation(self, layer: int, batch: int) -> np.ndarray:
        width = MLP_IN if layer == 0 else MLP_HIDDEN
        out = np.zeros((batch, width), dtype=np.float32)
        _chk(_lib.gsbs_mlp_get_activation(self.h, int(layer), int(batch), _ptr(out, C.c_float)))
        return out

    def backward(self, x, t) -> float:
        loss = C.c_float()
        _chk(_lib.gsbs_mlp_backward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), int(x.shape[0]),
                                    C.byref(loss)))
        return loss.value

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _chk(_lib.gsbs_mlp_adam(self.h, lr, beta1, beta2, eps))

    def train_step(self, x, t, lr, beta1=0.9, beta2=0.999, eps=1e-8) -> float:
        loss = C.c_float()
        _chk(_lib.gsbs_mlp_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), int(x.shape[0]),
                                      lr, beta1, beta2, eps, C.byref(loss)))
        return loss.value
