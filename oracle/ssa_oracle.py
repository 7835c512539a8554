"""FP64 CPU oracle of homogeneous stochastic kinetics -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this module; the HIP engine never imports, links or calls it and shares no
code with it.  The arithmetic is orc_ssa in gsbs_oracle.c: Gillespie's direct
method, the stochastic reference the paper compares SBS + PBCs and its rate
equations against (section on the verification of periodic boundary
conditions and the discussion of its figure).  This module only marshals.
"""
from __future__ import annotations

import numpy as np

from . import _p, lib, make_chem

import ctypes as C

NA = 6.02214076e23


def ssa(reactions, ns, n0, volume_L, t_rec, seed, stream, max_events=1 << 40, log_events=0, sources=(),
        first_order=()):
    """One realisation.  Returns (counts [n_rec][ns] int64, events, (ev_t, ev_r))
    with events = -1 when max_events ran out before the last record.  sources:
    zero-order reactions (rate mol/L/ns, products), after the reactions in the
    propensity list; first_order: first-order channels (species order, between
    the reactions and the sources)."""
    src_rate = np.array([q.rate for q in sources] + [0.0], dtype=np.float64)
    src_np = np.array([len(q.products) for q in sources] + [0], dtype=np.int32)
    src_p = np.zeros(3 * (len(sources) + 1), dtype=np.int32)
    for k, q in enumerate(sources):
        src_p[3 * k:3 * k + len(q.products)] = q.products
    chem = make_chem([1.0] * ns, reactions, first_order=first_order)
    n0 = np.ascontiguousarray(n0, dtype=np.int64)
    assert n0.shape == (ns,)
    t_rec = np.ascontiguousarray(t_rec, dtype=np.float64)
    out = np.zeros((len(t_rec), ns), dtype=np.int64)
    ev_t = np.zeros(max(log_events, 1), dtype=np.float64)
    ev_r = np.zeros(max(log_events, 1), dtype=np.int32)
    ne = lib().orc_ssa(C.byref(chem), float(volume_L), _p(n0, C.c_int64), len(t_rec), _p(t_rec, C.c_double),
                       C.c_uint64(seed), C.c_uint64(stream), int(max_events), _p(out, C.c_int64),
                       _p(ev_t, C.c_double) if log_events else None,
                       _p(ev_r, C.c_int32) if log_events else None, int(log_events),
                       len(sources), _p(src_rate, C.c_double), _p(src_np, C.c_int32), _p(src_p, C.c_int32))
    k = min(max(ne, 0), log_events)
    return out, int(ne), (ev_t[:k], ev_r[:k])


def ensemble(reactions, ns, n0, volume_L, t_rec, seed, n_real, stream0=0, sources=(), first_order=()):
    """n_real realisations (streams stream0 ...).  Returns counts [n_real][n_rec][ns]."""
    res = np.zeros((n_real, len(t_rec), ns), dtype=np.int64)
    for m in range(n_real):
        out, ne, _ = ssa(reactions, ns, n0, volume_L, t_rec, seed, stream0 + m, sources=sources,
                         first_order=first_order)
        assert ne >= 0
        res[m] = out
    return res


def counts_from_conc(conc_M, volume_L):
    """Nearest-integer counts of concentrations (mol/L) in volume_L litres."""
    return np.rint(np.asarray(conc_M, dtype=np.float64) * NA * volume_L).astype(np.int64)
