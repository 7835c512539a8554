"""Dose-rate study of the paper (section on the multiple-pulse set-up at SDR
and UHDR, and its H2O2-yield figure): trains of 1 us pulses at a pulse dose
rate of 2e5 or 1e6 Gy/s up to 20 Gy, the average dose rate set by the pulse
frequency, in a 2 um cube; SBS + PBCs while a pulse's spurs dissolve and the
rate equations between pulses (the paper's alternation).  Many pulse trains
run as the instances of one batched engine; the rate equations of all the
trains that hand over at a pulse are integrated in one launch.

Between pulses the mixture is homogeneous and nothing depends on absolute
time, so the engine's clock skips each inter-pulse interval: pulse p starts at
p * (width + settle + gap) on the engine clock while the rate equations cover
the true interval.  This keeps the engine's times small (its step lattice is
anchored at the pulse starts) even for pulse periods of 100 s.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List

import numpy as np

from . import gsbs
from . import workload as W

NA = 6.02214076e23
C_FLOOR = 1e-10
TAU_SETTLE = 1000.0  # ns after a pulse's last batch before the rate equations take over
GAP = 1.0            # ns of engine clock between the re-population and the next pulse
T_POST = 1e11        # ns (100 s) of rate equations after the last record: the post-irradiation yield


@dataclasses.dataclass
class Train:
    pulse_rate: float   # Gy/s during a pulse
    avg_rate: float     # Gy/s averaged over the train
    dose: float         # Gy per pulse
    n_pulses: int
    seed: int
    n_batches: int = 2
    plain: bool = False  # SBS through the whole train, no hand-over

    @property
    def width(self) -> float:  # ns
        return self.dose / self.pulse_rate * 1e9

    @property
    def period(self) -> float:  # ns, true time between pulse starts
        return self.dose / self.avg_rate * 1e9

    @property
    def hands_over(self) -> bool:
        return not self.plain and self.period > self.width + TAU_SETTLE + GAP

    @property
    def engine_period(self) -> float:  # ns on the engine clock
        return self.width + TAU_SETTLE + GAP if self.hands_over else self.period

    def injections(self, L: float) -> List[W.Injection]:
        rng = np.random.default_rng([self.seed, 11])
        n_tr = int(round(W.tracks_per_gray(L) * self.dose))
        out = []
        for p in range(self.n_pulses):
            arrive = rng.uniform(0.0, self.width, size=n_tr)
            batch = np.minimum((arrive / self.width * self.n_batches).astype(int), self.n_batches - 1)
            for b in range(self.n_batches):
                k = int(np.sum(batch == b))
                if k == 0:
                    continue
                pos, sp = W.tracks_z(rng, L, k)
                out.append(W.Injection(p * self.engine_period + b * self.width / self.n_batches,
                                       W._into_box(pos, L), sp, k * L * W.LET_KEV_PER_UM))
        return out


def paper_trains(seeds=(1, 2), avg_rates=(0.01, 1.0, 10.0, 100.0, 1e3, 1e4, 1e5), total_dose=20.0):
    """The paper's grid: 1 us pulses at 2e5 and 1e6 Gy/s (0.2 and 1 Gy per
    pulse) to 20 Gy, average dose rates 0.01 - 1e5 Gy/s."""
    out = []
    for dp in (2e5, 1e6):
        dose = dp * 1e-6
        for rate in avg_rates:
            for s in seeds:
                out.append(Train(dp, rate, dose, int(round(total_dose / dose)), seed=1000 * s + len(out)))
    return out


def run(trains: List[Train], L: float = 2000.0, seed: int = 1, numodes_rtol: float = 1e-6,
        ph7: bool = False, o2: bool = False) -> dict:
    """Run the trains as instances of one engine.  Returns, per train, the
    species counts, the H2O2 count and the deposited energy just before every
    pulse after the first and one period after the last, the H2O2 yield (slope
    of count against energy, molecules per 100 eV), the post-irradiation yield
    (the same slope of the H2O2 that each recorded mixture holds 100 s later,
    by the rate equations: the paper's post-irradiation concentrations after
    1, 2, ... pulses) and the wall time of the whole batch.

    ph7: pH 7 water (a chemistry extension): every cube starts with the
    1e-7 mol/L H3O+ / OH- background at uniform positions, and the rate
    equations carry R9's reverse (the water autoionisation) as a zero-order
    source.  The SBS stages (about 2 us per pulse) do not create ions; the
    background's turnover time, 1 / (k9 sqrt(Kw)) ~ 90 us, is much longer.

    o2: aerated water (the other extension): O2 at a fixed 2.5e-4 mol/L
    scavenges e_aq and H by first-order channels, superoxide (species 7)
    reacts with OH, e_aq and H."""
    import torch
    n = len(trains)
    V = L ** 3 * 1e-24
    if o2:
        e = gsbs.Engine([L] * n, seed, W.D_CONFIG_O2, W.REACTIONS_O2)
        gsbs.gsbs_set_first_order(e.ctx, W.FIRST_ORDER_O2)
    else:
        e = gsbs.Engine([L] * n, seed, W.D_CONFIG, W.REACTIONS)
    inj = [t.injections(L) for t in trains]
    if ph7:
        gsbs.gsbs_set_sources(e.ctx, W.SOURCES_PH7)
        n_bg = int(round(W.PH7_BACKGROUND_M * NA * V))
        for i, t in enumerate(trains):
            rng = np.random.default_rng([t.seed, 12])
            xyz = rng.uniform(-L / 2, L / 2, size=(2 * n_bg, 3))
            sp = np.repeat(np.array([W.H3O, W.OHM], dtype=np.uint8), n_bg)
            inj[i] = [W.Injection(0.0, W._into_box(xyz, L), sp, 0.0)] + inj[i]
    for i, js in enumerate(inj):
        for j in js:
            e.inject(i, j.t, j.xyz, j.species, j.edep_ev)
    n_max = max(t.n_pulses for t in trains)
    h2o2 = [[] for _ in range(n)]
    edep = [[] for _ in range(n)]
    counts = [[] for _ in range(n)]
    ode_steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in range(n_max):
        live = [i for i in range(n) if p < trains[i].n_pulses]
        nxt = {i: (p + 1) * trains[i].engine_period for i in live}
        sw = {i: p * trains[i].engine_period + trains[i].width + TAU_SETTLE for i in live if trains[i].hands_over}
        # SBS to the switch time (hand-over) or to the next pulse start
        target = np.array([e.time(i) for i in range(n)])
        for i in live:
            target[i] = sw.get(i, nxt[i])
        e.advance_to(target)
        ho = [i for i in live if i in sw]
        if ho:
            conc = np.stack([e.current_counts(i).astype(np.float64) for i in ho]) / (NA * V)
            dt = np.array([trains[i].period - trains[i].width - TAU_SETTLE for i in ho])
            c1, st = gsbs.gsbs_numodes(e.ctx, conc, dt, rtol=numodes_rtol)
            ode_steps += int(np.sum(st))
            for k, i in enumerate(ho):
                y = np.log10(np.maximum(c1[k], 0.0) + C_FLOOR).astype(np.float32)
                gsbs.gsbs_repopulate(e.ctx, i, nxt[i], y, np.zeros(len(y), np.float32), np.ones(len(y), np.float32),
                                     C_FLOOR, relative=False)
        for i in live:
            cnt = e.current_counts(i)
            if i not in sw:  # a step that ended at the next pulse start has injected its first batch
                for j in inj[i]:
                    if j.t == nxt[i]:
                        cnt = cnt - np.bincount(j.species, minlength=len(cnt))[:len(cnt)]
            h2o2[i].append(int(cnt[W.H2O2]))
            counts[i].append(np.asarray(cnt, dtype=np.int64))
            edep[i].append(float(sum(j.edep_ev for j in inj[i] if j.t < nxt[i] - 1e-9)))
    # post-irradiation: the rate equations carry every recorded mixture (the
    # cube just before each later pulse, and one period after the last)
    # T_POST further, radicals spent and slow superoxide dismutation done --
    # the H2O2 an irradiation of that many pulses leaves behind
    allc = np.concatenate([np.stack(counts[i]).astype(np.float64) for i in range(n)]) / (NA * V)
    post, _ = gsbs.gsbs_numodes(e.ctx, allc, np.full(len(allc), T_POST), rtol=numodes_rtol)
    post_h2o2, k0 = [], 0
    for i in range(n):
        post_h2o2.append(post[k0:k0 + len(counts[i]), W.H2O2] * NA * V)
        k0 += len(counts[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = e.stats()
    e.close()
    def slope(x, y):
        return float(np.polyfit(x, y, 1)[0]) if len(x) > 1 else float(y[0] / x[0])

    yields, g_post = [], []
    for i in range(n):
        x = np.array(edep[i]) / 100.0
        yields.append(slope(x, np.array(h2o2[i], dtype=np.float64)))
        g_post.append(slope(x, post_h2o2[i]))
    g_post = np.array(g_post)
    return dict(h2o2=h2o2, edep=edep, counts=[np.stack(c) for c in counts], g_h2o2=np.array(yields),
                g_h2o2_post=g_post, wall=wall,
                steps=st["steps"],
                molecule_steps=st["molecule_steps"], ode_steps=ode_steps)


RADICALS = (W.E_AQ, W.OH, W.H)


def build_up(train: Train, counts: np.ndarray, L: float = 2000.0, last: int = 5) -> float:
    """Radicals (e_aq, OH, H, and superoxide when the chemistry has it)
    standing at the next pulse start, over the radicals one pulse injects,
    averaged over the last pulses of a train: ~0 when the mixture reaches its
    steady state between pulses (the paper's SDR regime), growing with the
    average dose rate above the threshold (UHDR)."""
    per_pulse = W.tracks_per_gray(L) * train.dose * L / W.SPUR_SPACING_NM * W.SPUR_MEAN_MOLECULES * \
        float(sum(W.SPUR_FRACTIONS[s] for s in RADICALS))
    cols = list(RADICALS) + ([W.O2M] if counts.shape[1] > W.O2M else [])
    standing = counts[-last:, cols].sum(axis=1).mean()
    return float(standing / per_pulse)
