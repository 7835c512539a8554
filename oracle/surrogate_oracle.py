"""FP64 CPU oracle of the surrogate's state functions -- TEST INFRASTRUCTURE.

Only tests/ (and the smoke check) may import this module; the HIP engine never
imports, links or calls it and shares no code with it.  Plain numpy, written
from the definitions of the feature vector and of the re-population:

  * features: log10 concentrations (mol/L), the pair-correlation function of
    each reaction's reactants in 32 log-spaced shells from the reaction radius
    R to min(L/2, r_max) -- counts of b molecules around a uid-subsampled set of
    a molecules over the ideal-gas expectation -- and log10 of the time to the
    next pulse.  Distances use the minimum image of Eq. 2 in IEEE binary32
    with the operation order dx = x_b - x_a, minimum image, (dx^2 + dy^2) + dz^2,
    so that the shell of every pair is decided exactly as on the device;
  * re-population counts: mean count C N_A V rounded down or up with the
    Philox uniform at counter (species, step, 0, 3).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox, radius

NA = 6.02214076e23
N_BINS = 32


def _minimg32(d, L):
    d = np.asarray(d, dtype=np.float32)
    L32, h32 = np.float32(L), np.float32(0.5 * L)
    return np.where(d >= h32, d - L32, np.where(d < -h32, d + L32, d)).astype(np.float32)


def shells(R, L, r_max):
    """FP64 edges e_k = R' (r_m / R')^(k/32) (R' = min(R, r_m / 2), r_m =
    min(L/2, r_max)), their FP32 squares, and the FP64 shell volumes (shell 0
    from r = 0)."""
    rm = min(0.5 * L, r_max)
    Rp = min(R, 0.5 * rm)
    e = np.array([Rp * (rm / Rp) ** (k / N_BINS) for k in range(N_BINS + 1)])
    e2 = (e * e).astype(np.float32)
    vol = np.empty(N_BINS)
    vol[0] = 4.0 / 3.0 * math.pi * e[1] ** 3
    vol[1:] = 4.0 / 3.0 * math.pi * (e[2:] ** 3 - e[1:-1] ** 3)
    return e, e2, vol


def pair_counts(xyz, species, uid, a, b, L, e2, n_ref_max):
    """Shell counts of species b around the references of species a, and the
    number of references."""
    xyz = np.asarray(xyz, dtype=np.float32)
    na = int(np.sum(species == a))
    m = max(1, -(-na // n_ref_max))
    refs = np.nonzero((species == a) & (uid % np.uint64(m) == 0))[0]
    hist = np.zeros(N_BINS, dtype=np.int64)
    bidx = np.nonzero(species == b)[0]
    for i in refs:
        j = bidx[bidx != i]
        d = [_minimg32(xyz[j, c] - xyz[i, c], L) for c in range(3)]
        d2 = ((d[0] * d[0] + d[1] * d[1]).astype(np.float32) + d[2] * d[2]).astype(np.float32)
        d2 = d2[d2 < e2[N_BINS]]
        k = np.searchsorted(e2, d2, side="right") - 1
        hist += np.bincount(np.maximum(k, 0), minlength=N_BINS)
    return hist, len(refs)


def features(xyz, species, uid, L, D, reactions, dt_next, r_max=200.0, n_ref_max=1024, c_floor=1e-10):
    species = np.asarray(species)
    uid = np.asarray(uid, dtype=np.uint64)
    counts = np.array([np.sum(species == s) for s in range(len(D))], dtype=np.float64)
    vol_litre = L ** 3 * 1e-24
    f = list(np.log10(counts / (NA * vol_litre) + c_floor))
    for r in reactions:
        R = radius(r.k_in, D[r.a] + D[r.b])
        _, e2, vol = shells(R, L, r_max)
        hist, nref = pair_counts(xyz, species, uid, r.a, r.b, L, e2, n_ref_max)
        nb = counts[r.b] - (1.0 if r.a == r.b else 0.0)
        if nref > 0 and nb > 0:
            f += list(hist / (nref * (nb / L ** 3) * vol))
        else:
            f += [1.0] * N_BINS
    f.append(math.log10(dt_next))
    return np.array(f)


def repop_counts(y, mu, sd, L, seed, inst, step, c_floor=1e-10, now=None):
    """now: present counts when y is the change of log10(C + c_floor)."""
    out = []
    for s in range(len(y)):
        lc = float(y[s]) * float(sd[s]) + float(mu[s])
        if now is not None:
            lc += math.log10(float(now[s]) / (NA * L ** 3 * 1e-24) + c_floor)
        conc = max(0.0, 10.0 ** lc - c_floor)
        mean = conc * NA * L ** 3 * 1e-24
        w = philox([s, step, 0, 3], [seed, inst])
        u = (float(int(w[0]) >> 11) + 0.5) * 2.0 ** -53
        fl = math.floor(mean)
        out.append(int(fl) + (1 if u < mean - fl else 0))
    return np.array(out, dtype=np.int64)
