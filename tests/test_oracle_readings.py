"""Pins of the oracle's readings that the paper leaves open, each against
something other than the oracle itself: hand-derived outcomes, a closed form,
the definition of an unbiased rounding, and the paper's volume-scaling check.
Every pin is also run against a copy of the oracle with a named, plausible
mistake planted in it (compiled from patched source, or a patched copy of a
Python function) and must fail there.

Readings pinned here:
  * single-partner matching (mutual best by the key (pair uniform, partner
    uid's low 40 bits), repeated over at most K rounds);
  * the step cap: the largest step keeping every reaction's candidate cutoff
    R + c sqrt(2 D_AB dt) within L/2 (Eq. 2's minimum image needs it);
  * re-population counts: C N_A V rounded down or up at random, unbiased;
  * PBCs (Eq. 1-2): a homogeneous mixture evolves at the same concentrations
    in cubes of 0.2 and 0.5 um (the paper's volume-scaling verification).
"""
import math
import multiprocessing as mp
import os
import types

import numpy as np
import pytest

from paper_2509_03313_amd import workload as W

NA = 6.02214076e23


def _variant(orc, tmp_path, name, *subs):
    """The oracle library with each (old, new) text substitution applied once."""
    src = orc.source()
    for old, new in subs:
        assert src.count(old) == 1, f"planted mistake {name}: pattern not unique: {old}"
        src = src.replace(old, new)
    return orc.compile_variant(src, os.path.join(str(tmp_path), f"orc_{name}.so"))


# --------------------------------------------------------------- matching ---
# Hand cases: (n, pairs, u24, uid, rounds) -> (partner, order of matched pairs).
# Keys compare the pair uniform first and the partner's uid (low 40 bits) second.
HAND = {
    # A-B (u 5), B-C (u 3): B's best is C (3 < 5) and C's is B; A's only partner
    # is taken, so A stays unmatched.
    "chain3": (3, [(0, 1), (1, 2)], [5, 3], [10, 11, 12], 4, [-1, 2, 1], [1]),
    # A-B (2), B-C (1), C-D (3): B-C mutual in round 1; A and D have no pair left.
    "chain4": (4, [(0, 1), (1, 2), (2, 3)], [2, 1, 3], [20, 21, 22, 23], 4, [-1, 2, 1, -1], [1]),
    # A-B (1), B-C (2), C-D (3): A-B in round 1 (C's best B is taken by A);
    # C-D only in round 2.
    "two_rounds": (4, [(0, 1), (1, 2), (2, 3)], [1, 2, 3], [30, 31, 32, 33], 4, [1, 0, 3, 2], [0, 2]),
    "two_rounds_k1": (4, [(0, 1), (1, 2), (2, 3)], [1, 2, 3], [30, 31, 32, 33], 1, [1, 0, -1, -1], [0]),
    # a path of 10 with uniforms falling to the right: each round matches only
    # the rightmost free pair, so K = 4 rounds leave (0, 1) unmatched, 5 do not
    "cascade_k4": (10, [(k, k + 1) for k in range(9)], [9 - k for k in range(9)], list(range(100, 110)), 4,
                   [-1, -1, 3, 2, 5, 4, 7, 6, 9, 8], [8, 6, 4, 2]),
    "cascade_k5": (10, [(k, k + 1) for k in range(9)], [9 - k for k in range(9)], list(range(100, 110)), 5,
                   [1, 0, 3, 2, 5, 4, 7, 6, 9, 8], [8, 6, 4, 2, 0]),
    # star: centre 0, leaves 1, 2 (u 7) and 3 (u 9); the equal uniforms are
    # decided by the partner uid (leaf 2, uid 30 < 31), before leaf 3's smaller uid
    "star_uid": (4, [(0, 1), (0, 2), (0, 3)], [7, 7, 9], [50, 31, 30, 29], 4, [2, -1, 0, -1], [1]),
    # only the partner uid's low 40 bits enter the key: leaf 1 (uid 2^63 + 7)
    # beats leaf 2 (uid 8)
    "uid_low40": (3, [(0, 1), (0, 2)], [5, 5], [60, (1 << 63) | 7, 8], 4, [1, 0, -1], [0]),
}


@pytest.mark.parametrize("case", sorted(HAND))
def test_matching_hand_cases(orc, case):
    n, pairs, u24, uid, rounds, partner, order = HAND[case]
    got, got_order, tie = orc.match(n, pairs, u24, uid, rounds)
    assert not tie
    assert got.tolist() == partner
    assert got_order.tolist() == order
    # the outcome does not depend on the order in which pairs are listed
    perm = np.random.default_rng(len(case)).permutation(len(pairs))
    got2, _, _ = orc.match(n, [pairs[k] for k in perm], [u24[k] for k in perm], uid, rounds)
    assert got2.tolist() == partner


def test_matching_identical_keys_flag_a_tie(orc):
    """Two pairs of one molecule whose keys are identical (equal uniforms,
    partner uids equal in their low 40 bits) both look mutual: flagged."""
    _, _, tie = orc.match(3, [(0, 1), (0, 2)], [4, 4], [70, 5, (1 << 63) | 5], 4)
    assert tie


MATCH_MISTAKES = {
    # each molecule prefers its largest key
    "max_key": [("            best[pi[k]] = UINT64_MAX;\n            best[pj[k]] = UINT64_MAX;",
                 "            best[pi[k]] = 0;\n            best[pj[k]] = 0;"),
                ("if (ki < best[pi[k]]) best[pi[k]] = ki;", "if (ki > best[pi[k]]) best[pi[k]] = ki;"),
                ("if (kj < best[pj[k]]) best[pj[k]] = kj;", "if (kj > best[pj[k]]) best[pj[k]] = kj;")],
    # the first listed pair of a molecule wins
    "first_pair": [("if (ki < best[pi[k]]) best[pi[k]] = ki;", "if (best[pi[k]] == UINT64_MAX) best[pi[k]] = ki;"),
                   ("if (kj < best[pj[k]]) best[pj[k]] = kj;", "if (best[pj[k]] == UINT64_MAX) best[pj[k]] = kj;")],
    # one round fewer than asked
    "rounds_minus_1": [("for (int round = 0; round < rounds; ++round)", "for (int round = 1; round < rounds; ++round)")],
    # the partner's whole uid in the key (its top bits overflow into the uniform)
    "full_uid": [("return ((uint64_t)u24 << 40) | (partner_uid & 0xFFFFFFFFFFULL);",
                  "return ((uint64_t)u24 << 40) | partner_uid;")],
}


@pytest.mark.parametrize("mistake", sorted(MATCH_MISTAKES))
def test_matching_pins_catch_planted_mistakes(orc, tmp_path, mistake):
    path = _variant(orc, tmp_path, mistake, *MATCH_MISTAKES[mistake])
    failed = []
    with orc.swapped(path):
        for case, (n, pairs, u24, uid, rounds, partner, order) in HAND.items():
            got, got_order, tie = orc.match(n, pairs, u24, uid, rounds)
            if tie or got.tolist() != partner or got_order.tolist() != order:
                failed.append(case)
    assert failed, f"no hand case catches {mistake}"


def _k_for_radius(R, Dab):
    """Rate constant (1e10 L/mol/s) whose steady-state radius is R (nm)."""
    return R * 4.0 * math.pi * Dab * 6.02214076e23 / 1e25


def test_step_reacts_the_mutual_best_of_a_chain(orc):
    """Three almost immobile molecules of one self-reacting species in a row,
    neighbours within R (both pairs accepted with P = 1, the outer pair not a
    candidate): the pair that reacts is the one with the smaller pair uniform,
    drawn from Philox at (lower uid, higher uid, step, 1)."""
    D = [1e-9]
    R = 0.3
    rx = [W.Reaction("A+A", 0, 0, _k_for_radius(R, 2e-9), ())]
    chem = orc.make_chem(D, rx)
    x = np.array([[0.0, 0.0, 0.0], [0.2, 0.0, 0.0], [0.4, 0.0, 0.0]])
    s = orc.Instance(100.0, 9, 0)
    s.set_state(x, np.zeros(3, dtype=np.int32), np.array([5, 6, 7], dtype=np.uint64), step=3)
    u = {}
    for a, b in ((5, 6), (6, 7)):
        w = orc.philox([a, b, 3, 1], [9, 0])
        u[(a, b)] = int(w[0]) >> 40
    assert u[(5, 6)] != u[(6, 7)]
    s.step(chem, 1e-3)
    _, _, _, left = s.state()
    gone = {5, 6} if u[(5, 6)] < u[(6, 7)] else {6, 7}
    assert set(left.tolist()) == {5, 6, 7} - gone


# --------------------------------------------------------------- step cap ---
@pytest.mark.parametrize("L", [200.0, 1000.0, 10000.0])
def test_dt_max_puts_the_binding_cutoff_at_half_the_edge(orc, L):
    """At dt_max every reaction's cutoff R + 5 sqrt(2 D_AB dt) is within L/2,
    and the binding one (R9 here: the largest R and D_AB) is at L/2."""
    chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
    dt = orc.dt_max(chem, L)
    rc = []
    for r in W.REACTIONS:
        Dab = W.D_CONFIG[r.a] + W.D_CONFIG[r.b]
        rc.append(orc.cutoff(orc.radius(r.k_in, Dab), Dab, dt, 5.0))
    assert max(rc) <= 0.5 * L * (1 + 1e-12)
    assert abs(max(rc) - 0.5 * L) <= 1e-12 * L
    assert int(np.argmax(rc)) == 8


def test_dt_max_pin_catches_a_one_sided_diffusion_coefficient(orc, tmp_path):
    path = _variant(orc, tmp_path, "dab_is_da",
                    ("        double Dab = c->D[c->ra[r]] + c->D[c->rb[r]];\n        if (Dab <= 0.0) continue;",
                     "        double Dab = c->D[c->ra[r]];\n        if (Dab <= 0.0) continue;"))
    with orc.swapped(path):
        chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
        dt = orc.dt_max(chem, 1000.0)
    rc = max(orc.cutoff(orc.radius(r.k_in, W.D_CONFIG[r.a] + W.D_CONFIG[r.b]), W.D_CONFIG[r.a] + W.D_CONFIG[r.b],
                        dt, 5.0) for r in W.REACTIONS)
    assert rc > 500.0 * (1 + 1e-6)


# --------------------------------------------------------- re-population ---
def _repop_check(repop, n_calls=1500):
    """Counts for concentrations chosen directly (mu = log10(C + floor), sd = 1,
    y = 0): every count is floor(m) or ceil(m), m = C N_A L^3, and the mean over
    the calls (different Philox counters) is m within 4 standard errors."""
    L = 100.0
    V = L ** 3 * 1e-24
    m = np.array([0.37, 2.5, 17.123, 1e-3, 41.0, 0.0, 7.77])
    C = m / (NA * V)
    mu = np.log10(C + 1e-10)
    sd = np.ones(7)
    y = np.zeros(7)
    out = np.array([repop(y, mu, sd, L, 11, 2, step) for step in range(n_calls)], dtype=np.float64)
    # m recomputed from the FP64 round trip through log10 / 10**
    m_eff = (10.0 ** mu - 1e-10) * NA * V
    lo, hi = np.floor(m_eff), np.ceil(m_eff)
    ok_vals = bool(np.all((out == lo) | (out == hi)))
    frac = m_eff - lo
    se = np.sqrt(np.maximum(frac * (1 - frac), 1e-12) / n_calls)
    ok_mean = bool(np.all(np.abs(out.mean(axis=0) - m_eff) <= 4 * se + 1e-12))
    return ok_vals, ok_mean


def test_repop_counts_are_unbiased_floor_or_ceil():
    from oracle import surrogate_oracle as SO
    ok_vals, ok_mean = _repop_check(SO.repop_counts)
    assert ok_vals and ok_mean


def test_repop_counts_relative_mode_keeps_the_present_state():
    """With relative = y = 0 the new mean equals the present count."""
    from oracle import surrogate_oracle as SO
    now = np.array([5, 0, 12, 3, 0, 9, 1])
    L = 200.0
    out = np.array([SO.repop_counts(np.zeros(7), np.zeros(7), np.ones(7), L, 3, 0, st, now=now)
                    for st in range(400)])
    # (C + floor) * 10**0 - floor = C: the mean count returns to the present one
    assert np.all(np.abs(out - now) <= 1)
    assert np.all(np.abs(out.mean(axis=0) - now) < 0.05)


@pytest.mark.parametrize("mistake", ["floor_only", "round_nearest", "inverted_draw"])
def test_repop_pins_catch_planted_mistakes(mistake):
    import oracle
    from oracle import surrogate_oracle as SO
    src = open(SO.__file__).read()
    old = "out.append(int(fl) + (1 if u < mean - fl else 0))"
    assert src.count(old) == 1
    new = {"floor_only": "out.append(int(fl))",
           "round_nearest": "out.append(int(math.floor(mean + 0.5)))",
           "inverted_draw": "out.append(int(fl) + (1 if u > mean - fl else 0))"}[mistake]
    mod = types.ModuleType("oracle._planted")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "planted", "exec"), mod.__dict__)
    assert oracle  # the package the planted copy imports from
    ok_vals, ok_mean = _repop_check(mod.repop_counts)
    assert not (ok_vals and ok_mean)


# ---------------------------------------------------------- volume scaling ---
# A homogeneous mixture (the spur model's species, a tenth of the
# volume-scaling concentration of the device check) with counts that scale
# exactly from the 0.2 um cube (x 15.625 in the 0.5 um cube), both cubes on
# the same step times (the 0.2 um cube's step cap), to 10 us.
VS_COUNTS_02 = {0: 56, 1: 64, 2: 8, 3: 64, 4: 8}
VS_T_END = 1e4


def _vs_run(args):
    path, L, seed = args
    import oracle
    cm = oracle.swapped(path) if path else None
    if cm:
        cm.__enter__()
    try:
        chem = oracle.make_chem(W.D_CONFIG, W.REACTIONS)
        dm = oracle.dt_max(chem, 200.0)
        conc = {s: n / 200.0 ** 3 for s, n in VS_COUNTS_02.items()}
        wl = W.homogeneous(seed, L, conc, VS_T_END, n_records=12)
        r = oracle.run(wl, chem=chem, inst=0, philox_seed=7, dtmax=dm)
        return r["counts"].astype(np.float64) / (L / 1000.0) ** 3
    finally:
        if cm:
            cm.__exit__(None, None, None)


def _vs_z(path, n_small=64, n_large=4):
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        a = np.array(pool.map(_vs_run, [(path, 200.0, s) for s in range(n_small)]))
        b = np.array(pool.map(_vs_run, [(path, 500.0, 100 + s) for s in range(n_large)]))
    ma, mb = a.mean(axis=0), b.mean(axis=0)
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    # per um^3: compare where the 0.5 um cube holds at least 20 molecules
    use = mb * 0.125 >= 20
    d = np.abs(ma - mb)
    return d, se, use


def test_volume_scaling_same_concentrations_in_02_and_05_um(orc):
    """The paper's PBC check on the oracle: the same mixture in 0.2 and 0.5 um
    cubes gives the same concentrations at every record (64 small, 4 large
    cubes; within 4.5 standard errors of the seed-to-seed scatter)."""
    d, se, use = _vs_z(None)
    assert use.sum() > 40
    assert np.all(d[use] <= 4.5 * se[use] + 1e-9), np.max((d / np.maximum(se, 1e-9))[use])


def test_volume_scaling_pin_catches_a_missing_wrap(orc, tmp_path):
    """Planted mistake: positions not wrapped back into the cube after a jump
    (PBC 1, Eq. 1, left out)."""
    path = _variant(orc, tmp_path, "no_wrap",
                    ("s->x[3 * i + a] = orc_wrap(s->x[3 * i + a] + sigma * z[a], L);",
                     "s->x[3 * i + a] = s->x[3 * i + a] + sigma * z[a];"))
    d, se, use = _vs_z(path)
    assert not np.all(d[use] <= 4.5 * se[use] + 1e-9)


# ------------------------------------------- full-size decisions (bucket grid) ---
@pytest.mark.parametrize("L,n,dt", [(400.0, 2500, 3.0), (600.0, 3000, 40.0), (1000.0, 4000, 60.0),
                                    (400.0, 2500, 40.0)])
def test_accept_f32_equals_all_pairs(orc, L, n, dt):
    """orc_accept_f32 (bucket grid, for full-size inputs) selects exactly the
    candidates of the all-pairs orc_cand_f32, and accepts exactly those whose
    pair uniform (Philox at (lower uid, higher uid, step, 1)) falls below the
    oracle's contact probability of their FP64 separations."""
    rng = np.random.default_rng(int(L + dt))
    x0 = rng.uniform(-L / 2, L / 2, size=(n, 3))
    m = (n // 30) * 10
    x0[:m] = rng.uniform(-L / 2, L / 2, size=(n // 30, 3)).repeat(10, axis=0) + rng.normal(0, 2.0, size=(m, 3))
    x0 = ((x0 + L / 2) % L - L / 2).astype(np.float32)
    x1 = ((x0 + rng.normal(0, math.sqrt(2 * 5 * dt), size=(n, 3)) + L / 2) % L - L / 2).astype(np.float32)
    sp = rng.integers(0, 7, size=n).astype(np.int32)
    uid = rng.permutation(np.arange(n, dtype=np.uint64) * 7 + 3)
    chem = orc.make_chem(W.D_CONFIG, W.REACTIONS)
    ref = orc.cand_f32(x1, sp, L, chem, dt)
    pr, P, u24, ncand = orc.accept_f32(x1, x0, sp, uid, L, chem, dt, 6, 21, 2)
    assert ncand == len(ref) and ncand > 100
    acc = set()
    for i, j in ref.tolist():
        r = W.REACTIONS[[k for k, q in enumerate(W.REACTIONS) if {q.a, q.b} == {sp[i], sp[j]}][0]]
        Dab = W.D_CONFIG[r.a] + W.D_CONFIG[r.b]
        d1 = [orc.minimg(float(x1[j, a]) - float(x1[i, a]), L) for a in range(3)]
        d0 = [orc.minimg(float(x0[j, a]) - float(x0[i, a]), L) for a in range(3)]
        p = orc.bridge(math.sqrt(sum(v * v for v in d0)), math.sqrt(sum(v * v for v in d1)), orc.radius(r.k_in, Dab),
                       Dab * dt)
        lo, hi = sorted((int(uid[i]), int(uid[j])))
        if ((int(orc.philox([lo, hi, 6, 1], [21, 2])[0]) >> 40) + 0.5) * 2.0 ** -24 < p:
            acc.add((min(i, j), max(i, j)))
    assert set(map(tuple, pr.tolist())) == acc and len(acc) > 0
