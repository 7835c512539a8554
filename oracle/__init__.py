"""FP64 CPU oracle of the SBS diffusion-reaction method -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  The HIP engine never imports, links or calls it; the two share
no code.  The arithmetic lives in gsbs_oracle.c (plain C, FP64); this module
only marshals arguments through ctypes.  See gsbs_oracle.c for the passages of
arXiv 2509.03313 each function follows.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsbs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MAX_SPECIES = 16
MAX_REACT = 32


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE arithmetic, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Chem(C.Structure):
    _fields_ = [
        ("ns", C.c_int32), ("nr", C.c_int32),
        ("D", C.c_double * MAX_SPECIES),
        ("ra", C.c_int32 * MAX_REACT), ("rb", C.c_int32 * MAX_REACT),
        ("k_in", C.c_double * MAX_REACT),
        ("nprod", C.c_int32 * MAX_REACT),
        ("prod", (C.c_int32 * 3) * MAX_REACT),
        ("keep_b", C.c_int32 * MAX_REACT),
        ("c_cut", C.c_double),
        ("rounds", C.c_int32), ("contact_only", C.c_int32), ("brute", C.c_int32),
        ("fo_k", C.c_double * MAX_SPECIES), ("fo_nprod", C.c_int32 * MAX_SPECIES),
        ("fo_prod", (C.c_int32 * 2) * MAX_SPECIES),
    ]


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            _lib = _bind(C.CDLL(_LIB))
    return _lib


def compile_variant(source: str, path: str) -> str:
    """Compile C source text (a patched copy of gsbs_oracle.c) the way build()
    compiles the oracle; tests use it to plant a mistake and check that a pin
    catches it."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(source)
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", src,
                    "-o", path, "-lm"], check=True)
    return path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


@contextlib.contextmanager
def swapped(path: str):
    """Every wrapper below calls the library at `path` inside the block."""
    global _lib
    old = lib()
    with _lock:
        _lib = _bind(C.CDLL(path))
    try:
        yield
    finally:
        with _lock:
            _lib = old


def _bind(L):
    if True:
        if True:
            d, i32, i64, u64, f32 = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_float
            P = C.POINTER
            vp = C.c_void_p
            sig = {
                "orc_philox4x64_10": (None, [P(u64), P(u64), P(u64)]),
                "orc_u24": (d, [u64]),
                "orc_gauss3": (None, [P(u64), P(d)]),
                "orc_wrap": (d, [d, d]),
                "orc_minimg": (d, [d, d]),
                "orc_radius": (d, [d, d]),
                "orc_cutoff": (d, [d, d, d, d]),
                "orc_bridge": (d, [d, d, d, d]),
                "orc_dt_max": (d, [P(Chem), d]),
                "orc_schedule": (i64, [d, d, i32, P(d), i32, P(d), d, d, d, P(d), i64]),
                "orc_new": (vp, [d, u64, u64]),
                "orc_free": (None, [vp]),
                "orc_get_n": (i64, [vp]),
                "orc_get_step": (i64, [vp]),
                "orc_get_time": (d, [vp]),
                "orc_get_edep": (d, [vp]),
                "orc_get_diag": (None, [vp, P(i64)]),
                "orc_inject": (None, [vp, i64, P(d), P(i32), d]),
                "orc_set_state": (None, [vp, i64, P(d), P(d), P(i32), P(u64), i64, u64]),
                "orc_get_state": (None, [vp, P(d), P(d), P(i32), P(u64)]),
                "orc_counts": (None, [vp, i32, P(i64)]),
                "orc_set_log": (None, [vp, i32]),
                "orc_log_size": (i64, [vp]),
                "orc_get_log": (None, [vp, P(u64), P(d), P(C.c_uint32), P(i32), P(i32)]),
                "orc_step": (i64, [vp, P(Chem), d]),
                "orc_run": (i64, [vp, P(Chem), i32, P(d), P(i64), P(d), P(i32), P(d), i32, P(d),
                                  d, d, d, d, P(i64), P(d), P(i64)]),
                "orc_bin_f32": (None, [i64, P(f32), f32, i32, P(i32)]),
                "orc_rc2_f32": (None, [P(Chem), d, P(f32)]),
                "orc_cand_f32": (i64, [i64, P(f32), P(i32), f32, P(Chem), d, P(i64), i64]),
                "orc_ssa": (i64, [P(Chem), d, P(i64), i32, P(d), u64, u64, i64, P(i64), P(d), P(i32), i64,
                                  i32, P(d), P(i32), P(i32)]),
                "orc_spurs": (i64, [d, u64, u64, i32, d, d, d, i32, P(d), P(d), P(i32), i64]),
                "orc_match": (i64, [i64, i64, P(i64), P(i64), P(C.c_uint32), P(u64), i32, P(i64), P(i64)]),
                "orc_accept_f32": (i64, [i64, P(f32), P(f32), P(i32), P(u64), f32, P(Chem), d, u64, u64, u64,
                                         P(i64), P(d), P(C.c_uint32), i64, P(i64)]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
    return L


# ------------------------------------------------------------ chemistry ---
def make_chem(D, reactions, c_cut: float = 5.0, rounds: int = 4, contact_only: bool = False,
              brute: bool = False, first_order=()) -> Chem:
    """reactions: objects with a, b, k_in, products, keep_b (see
    workload.Reaction); first_order: objects with a, k (per ns) and products
    (at most two; see workload.FirstOrder), one per species."""
    c = Chem()
    c.ns = len(D)
    c.nr = len(reactions)
    for k, v in enumerate(D):
        c.D[k] = float(v)
    for r, rx in enumerate(reactions):
        c.ra[r] = rx.a
        c.rb[r] = rx.b
        c.k_in[r] = rx.k_in
        c.nprod[r] = len(rx.products)
        for k, p in enumerate(rx.products):
            c.prod[r][k] = p
        c.keep_b[r] = 1 if getattr(rx, "keep_b", False) else 0
    c.c_cut = c_cut
    c.rounds = rounds
    c.contact_only = 1 if contact_only else 0
    c.brute = 1 if brute else 0
    for f in first_order:
        assert c.fo_k[f.a] == 0.0 and len(f.products) <= 2
        c.fo_k[f.a] = f.k
        c.fo_nprod[f.a] = len(f.products)
        for k, p in enumerate(f.products):
            c.fo_prod[f.a][k] = p
    return c


# --------------------------------------------------------------- spurs ---
def spurs(L, seed, stream, n_tracks, spacing, mean, sigma, frac):
    """The counter-based spur model of orc_spurs: (xyz [n][3] float64, species int32)."""
    frac = np.ascontiguousarray(frac, dtype=np.float64)
    one = np.zeros(3)
    onei = np.zeros(1, dtype=np.int32)
    n = lib().orc_spurs(float(L), C.c_uint64(seed), C.c_uint64(stream), int(n_tracks), float(spacing), float(mean),
                        float(sigma), len(frac), _p(frac, C.c_double), _p(one, C.c_double), _p(onei, C.c_int32), 0)
    xyz = np.zeros((max(n, 1), 3))
    sp = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_spurs(float(L), C.c_uint64(seed), C.c_uint64(stream), int(n_tracks), float(spacing), float(mean),
                    float(sigma), len(frac), _p(frac, C.c_double), _p(xyz, C.c_double), _p(sp, C.c_int32), int(n))
    return xyz[:n], sp[:n]


def match(n, pairs, u24, uid, rounds=4):
    """Single-partner matching of accepted pairs (orc_match): pairs [k][2]
    molecule indices below n, u24[k] the pair uniforms' 24-bit integers, uid[n].
    Returns (partner [n] with -1 for unmatched, matched pair indices in match
    order, tie flag)."""
    pr = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    pi = np.ascontiguousarray(pr[:, 0])
    pj = np.ascontiguousarray(pr[:, 1])
    u = np.ascontiguousarray(u24, dtype=np.uint32)
    ud = np.ascontiguousarray(uid, dtype=np.uint64)
    partner = np.zeros(max(n, 1), dtype=np.int64)
    order = np.zeros(max(len(pi), 1), dtype=np.int64)
    r = lib().orc_match(int(n), len(pi), _p(pi, C.c_int64), _p(pj, C.c_int64), _p(u, C.c_uint32),
                        _p(ud, C.c_uint64), int(rounds), _p(partner, C.c_int64), _p(order, C.c_int64))
    tie = r < 0
    m = -r - 1 if tie else r
    return partner[:n], order[:m], bool(tie)


def accept_f32(xyz, xyz0, species, uid, L, chem, dt, step, seed, inst=0, max_pairs=50_000_000):
    """One step's decisions on fixed FP32 end (xyz) and start (xyz0) positions:
    (accepted pairs [k][2] of sorted indices, their P, u24, candidate count)."""
    x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    x0 = np.ascontiguousarray(xyz0, dtype=np.float32).reshape(-1, 3)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    u = np.ascontiguousarray(uid, dtype=np.uint64)
    n = len(sp)
    cap = 1 << 16
    while True:
        pr = np.zeros((cap, 2), dtype=np.int64)
        P = np.zeros(cap)
        u24 = np.zeros(cap, dtype=np.uint32)
        nc = C.c_int64()
        k = lib().orc_accept_f32(n, _p(x, C.c_float), _p(x0, C.c_float), _p(sp, C.c_int32), _p(u, C.c_uint64),
                                 float(L), C.byref(chem), float(dt), int(step), int(seed), int(inst),
                                 _p(pr, C.c_int64), _p(P, C.c_double), _p(u24, C.c_uint32), cap, C.byref(nc))
        if k <= cap or cap >= max_pairs:
            return pr[:min(k, cap)], P[:min(k, cap)], u24[:min(k, cap)], nc.value
        cap = min(max_pairs, 2 * k)


# ------------------------------------------------------------- scalars ---
def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def u24(w):
    return lib().orc_u24(int(w))


def gauss3(w):
    w = np.asarray(w, dtype=np.uint64)
    z = np.zeros(3)
    lib().orc_gauss3(_p(w, C.c_uint64), _p(z, C.c_double))
    return z


def wrap(x, L):
    return lib().orc_wrap(float(x), float(L))


def minimg(d, L):
    return lib().orc_minimg(float(d), float(L))


def radius(k_in, Dab):
    return lib().orc_radius(float(k_in), float(Dab))


def cutoff(R, Dab, dt, c):
    return lib().orc_cutoff(float(R), float(Dab), float(dt), float(c))


def bridge(r0, r1, R, s):
    return lib().orc_bridge(float(r0), float(r1), float(R), float(s))


def dt_max(chem: Chem, L: float) -> float:
    return lib().orc_dt_max(C.byref(chem), float(L))


def schedule(t_start, t_end, anchors, events, dt0, ratio, dt_max_):
    a = np.ascontiguousarray(anchors, dtype=np.float64)
    e = np.ascontiguousarray(events, dtype=np.float64)
    L = lib()
    n = L.orc_schedule(t_start, t_end, len(a), _p(a, C.c_double), len(e), _p(e, C.c_double),
                       dt0, ratio, dt_max_, None, 0)
    out = np.zeros(max(n, 1))
    L.orc_schedule(t_start, t_end, len(a), _p(a, C.c_double), len(e), _p(e, C.c_double),
                   dt0, ratio, dt_max_, _p(out, C.c_double), n)
    return out[:n]


# ------------------------------------------------------------ instance ---
class Instance:
    """One periodic cube of edge L (nm), Philox key (seed, inst)."""

    def __init__(self, L: float, seed: int, inst: int = 0):
        self.L = float(L)
        self._h = lib().orc_new(self.L, int(seed), int(inst))

    def close(self):
        if self._h:
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return lib().orc_get_n(self._h)

    @property
    def step_index(self):
        return lib().orc_get_step(self._h)

    @property
    def t(self):
        return lib().orc_get_time(self._h)

    @property
    def edep(self):
        return lib().orc_get_edep(self._h)

    def inject(self, xyz, species, edep_ev: float = 0.0):
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        s = np.ascontiguousarray(species, dtype=np.int32)
        lib().orc_inject(self._h, len(s), _p(x, C.c_double), _p(s, C.c_int32), float(edep_ev))

    def set_state(self, xyz, species, uid, x0=None, step: int = 0, next_uid: int = None):
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 3)
        s = np.ascontiguousarray(species, dtype=np.int32)
        u = np.ascontiguousarray(uid, dtype=np.uint64)
        nu = int(u.max()) + 1 if next_uid is None and len(u) else (next_uid or 0)
        lib().orc_set_state(self._h, len(s), _p(x, C.c_double),
                            None if x0a is None else _p(x0a, C.c_double),
                            _p(s, C.c_int32), _p(u, C.c_uint64), int(step), nu)

    def state(self):
        n = self.n
        x = np.zeros((n, 3))
        x0 = np.zeros((n, 3))
        s = np.zeros(n, dtype=np.int32)
        u = np.zeros(n, dtype=np.uint64)
        lib().orc_get_state(self._h, _p(x, C.c_double), _p(x0, C.c_double), _p(s, C.c_int32),
                            _p(u, C.c_uint64))
        return x, x0, s, u

    def counts(self, ns: int = 7):
        out = np.zeros(ns, dtype=np.int64)
        lib().orc_counts(self._h, ns, _p(out, C.c_int64))
        return out

    def set_log(self, mode: int):
        lib().orc_set_log(self._h, int(mode))

    def log(self):
        n = lib().orc_log_size(self._h)
        uid2 = np.zeros((n, 2), dtype=np.uint64)
        P = np.zeros(n)
        u = np.zeros(n, dtype=np.uint32)
        f = np.zeros(n, dtype=np.int32)
        rx = np.zeros(n, dtype=np.int32)
        if n:
            lib().orc_get_log(self._h, _p(uid2, C.c_uint64), _p(P, C.c_double),
                              _p(u, C.c_uint32), _p(f, C.c_int32), _p(rx, C.c_int32))
        return dict(uid=uid2, P=P, u24=u, flag=f, rx=rx)

    def diag(self):
        out = np.zeros(3, dtype=np.int64)
        lib().orc_get_diag(self._h, _p(out, C.c_int64))
        return dict(n_cand=int(out[0]), n_acc=int(out[1]), n_react=int(out[2]))

    def step(self, chem: Chem, dt: float) -> int:
        r = lib().orc_step(self._h, C.byref(chem), float(dt))
        if r < 0:
            raise RuntimeError("oracle: tied matching keys")
        return r


def run(workload, chem: Chem = None, inst: int = 0, dt0: float = None, ratio: float = None,
        dtmax: float = None, t_end: float = None, c_cut: float = 5.0, philox_seed: int = None):
    """Run a workload.Workload through the oracle (Philox key (philox_seed or
    workload.seed, inst)).  Returns dict with counts (n_records x n_species),
    edep (eV at each record) and stats."""
    if chem is None:
        chem = make_chem(workload.D, workload.reactions, c_cut=c_cut)
    dt0 = workload.dt0 if dt0 is None else dt0
    ratio = workload.ratio if ratio is None else ratio
    t_end = workload.t_end if t_end is None else t_end
    if dtmax is None:
        dtmax = dt_max(chem, workload.L)
    s = Instance(workload.L, workload.seed if philox_seed is None else philox_seed, inst)
    injs = [i for i in workload.injections if i.t <= t_end]
    n_inj = len(injs)
    inj_t = np.array([i.t for i in injs], dtype=np.float64)
    inj_n = np.array([len(i.species) for i in injs], dtype=np.int64)
    inj_x = np.ascontiguousarray(np.concatenate([i.xyz for i in injs]).astype(np.float64))
    inj_s = np.ascontiguousarray(np.concatenate([i.species for i in injs]).astype(np.int32))
    inj_e = np.array([i.edep_ev for i in injs], dtype=np.float64)
    rec = np.ascontiguousarray(workload.records[workload.records <= t_end], dtype=np.float64)
    ns = chem.ns
    counts = np.full((len(rec), ns), -1, dtype=np.int64)
    edep = np.zeros(len(rec))
    stats = np.zeros(4, dtype=np.int64)
    lib().orc_run(s._h, C.byref(chem), n_inj, _p(inj_t, C.c_double), _p(inj_n, C.c_int64),
                  _p(inj_x, C.c_double), _p(inj_s, C.c_int32), _p(inj_e, C.c_double),
                  len(rec), _p(rec, C.c_double), float(t_end), float(dt0), float(ratio),
                  float(dtmax), _p(counts, C.c_int64), _p(edep, C.c_double), _p(stats, C.c_int64))
    out = dict(times=rec, counts=counts, edep=edep, n_steps=int(stats[0]),
               molecule_steps=int(stats[1]), n_react=int(stats[2]), tie=bool(stats[3]),
               final_n=s.n, final_t=s.t)
    s.close()
    return out


# ------------------------------------------------------- FP32 emulation ---
def bin_f32(xyz, L: float, nc: int):
    x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    out = np.zeros(len(x), dtype=np.int32)
    lib().orc_bin_f32(len(x), _p(x, C.c_float), np.float32(L), int(nc), _p(out, C.c_int32))
    return out


def rc2_f32(chem: Chem, dt: float):
    out = np.zeros(MAX_REACT, dtype=np.float32)
    lib().orc_rc2_f32(C.byref(chem), float(dt), _p(out, C.c_float))
    return out[:chem.nr]


def cand_f32(xyz, species, L: float, chem: Chem, dt: float, max_pairs: int = 10_000_000):
    x = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    s = np.ascontiguousarray(species, dtype=np.int32)
    L_ = lib()
    n = L_.orc_cand_f32(len(x), _p(x, C.c_float), _p(s, C.c_int32), np.float32(L), C.byref(chem),
                        float(dt), None, 0)
    out = np.zeros((max(n, 1), 2), dtype=np.int64)
    L_.orc_cand_f32(len(x), _p(x, C.c_float), _p(s, C.c_int32), np.float32(L), C.byref(chem),
                    float(dt), _p(out, C.c_int64), n)
    return out[:n]
