"""Seeded synthetic inputs for the SBS radiolysis engine and for its oracle.

This module only draws inputs: species tables, reaction tables, molecule
positions and species of the initial chemical stage, injection times and
record times.  It holds none of the method's arithmetic (no diffusion, no
periodic boundary handling beyond placing molecules inside the cube, no
reaction radii, no step schedule), so both the HIP engine and the CPU oracle
can take the same arrays.

Sources of the numbers (arXiv 2509.03313):
  * Table 1 -- the nine reactions R1-R9 and their rate constants in
    1e10 L/mol/s; for R1, R6 and R8 the printed number is 2k.
  * Table S2 -- diffusion coefficients in 1e-9 m^2/s (= nm^2/ns).
  * Eq. (5) -- D = (N / L^2) * (S / rho): number of primaries per dose.
  * Sec. "Workflow of gMicroMC extension" -- radiation events are sampled in
    time within each pulse according to the pulse structure; the pulse dose
    rate is the pulse dose over the FWHM, the average dose rate is the pulse
    dose times the frequency.

The physical and physico-chemical stages are outside the scope of this engine,
so the initial species come from a synthetic spur model instead: straight
tracks, spur centres at exponential spacing (mean 100 nm), a Poisson(5.13)
number of molecules per spur, each at a Gaussian offset (sigma 2 nm) from its
spur centre, with species drawn from fixed fractions.  At 0.8 keV/um this gives
6.4 molecules per 100 eV, i.e. about 400 molecules per um^3 per Gy.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------- species ---
SPECIES = ["e_aq", "OH", "H", "H3O+", "OH-", "H2O2", "H2"]
E_AQ, OH, H, H3O, OHM, H2O2, H2 = range(7)

# diffusion coefficients, nm^2/ns, of the synthetic workloads
D_CONFIG = [4.9, 2.2, 7.0, 9.0, 5.3, 2.3, 4.8]
# Table S2 (e_aq 4.82, OH 2.2, H 7.0, H+ 9.3, H2 4.8, OH- 5.3, H2O2 2.3),
# reordered to SPECIES
D_PAPER = [4.82, 2.2, 7.0, 9.3, 5.3, 2.3, 4.8]


@dataclasses.dataclass(frozen=True)
class Reaction:
    name: str
    a: int
    b: int
    k_in: float              # 1e10 L/mol/s as printed in Table 1 (2k for R1, R6, R8)
    products: tuple          # species indices, at most three
    keep_b: bool = False     # test-only sink: reactant b survives unchanged


@dataclasses.dataclass(frozen=True)
class Source:
    """A zero-order reaction (no reactants): products appear at a constant
    rate, mol/L/ns, anywhere in the volume."""
    name: str
    rate: float              # mol/L/ns
    products: tuple          # species indices, at most three


@dataclasses.dataclass(frozen=True)
class FirstOrder:
    """A first-order channel: a molecule of species a turns into its products
    (at most two, the first in its place) at rate k per ns -- e.g. scavenging
    by a solute held at a fixed concentration (pseudo-first order)."""
    name: str
    a: int
    k: float                 # per ns
    products: tuple


# Table 1; H2O is not tracked, R9 is taken in the forward direction only.
REACTIONS = [
    Reaction("R1", E_AQ, E_AQ, 1.3, (H2, OHM, OHM)),
    Reaction("R2", E_AQ, OH, 3.0, (OHM,)),
    Reaction("R3", E_AQ, H, 2.6, (H2, OHM)),
    Reaction("R4", E_AQ, H3O, 2.3, (H,)),
    Reaction("R5", E_AQ, H2O2, 1.4, (OH, OHM)),
    Reaction("R6", OH, OH, 0.95, (H2O2,)),
    Reaction("R7", OH, H, 1.5, ()),
    Reaction("R8", H, H, 1.1, (H2,)),
    Reaction("R9", H3O, OHM, 11.0, ()),
]

# Chemistry extension: pH 7 water.  R9 made reversible by its reverse, the
# autoionisation H2O -> H3O+ + OH-, at k9 * Kw (Kw = 1e-14 M^2 at 25 C), so that
# [H3O+][OH-] relaxes to Kw; the background starts at 1e-7 mol/L of each.
KW_M2 = 1e-14
PH7_BACKGROUND_M = 1e-7
SOURCES_PH7 = [Source("R9 reverse", 10.0 * 11.0 * KW_M2, (H3O, OHM))]  # 1e10 /M/s * 10 = /M/ns


# Chemistry extension: aerated water.  O2 at a fixed 2.5e-4 mol/L scavenges
# e_aq and H (pseudo-first order); superoxide is one species (O2- and HO2,
# pKa 4.8, lumped as O2- at pH 7: H + O2 -> HO2 -> O2- + H3O+).  Rate constants
# (1e10 L/mol/s) from the compilation of Buxton, Greenstock, Helman and Ross,
# J. Phys. Chem. Ref. Data 17 (1988) and Bielski et al., J. Phys. Chem. Ref.
# Data 14 (1985); the superoxide dismutation at pH 7 (observed 2e5 L/mol/s,
# entered like R1/R6/R8 as a self-recombination) gives H2O2 over seconds.
# D(O2-) = 1.75 nm^2/ns.
O2M = 7
SPECIES_O2 = SPECIES + ["O2-"]
D_CONFIG_O2 = D_CONFIG + [1.75]
O2_AERATED_M = 2.5e-4
REACTIONS_O2 = REACTIONS + [
    Reaction("O2- + OH", O2M, OH, 1.0, (OHM,)),
    Reaction("O2- + e_aq", O2M, E_AQ, 1.3, (H2O2, OHM, OHM)),
    Reaction("O2- + H", O2M, H, 2.0, (H2O2, OHM)),
    Reaction("O2- + O2-", O2M, O2M, 2e-5, (H2O2, OHM, OHM)),
]
FIRST_ORDER_O2 = [
    FirstOrder("e_aq + O2", E_AQ, 1.9e10 * O2_AERATED_M * 1e-9, (O2M,)),
    FirstOrder("H + O2", H, 2.1e10 * O2_AERATED_M * 1e-9, (O2M, H3O)),
]


# synthetic spur composition, molecules per 100 (charge and redox balance to 0)
SPUR_FRACTIONS = np.array([29, 35, 4, 30, 1, 0, 1], dtype=np.float64) / 100.0
SPUR_SPACING_NM = 100.0
SPUR_MEAN_MOLECULES = 5.13
SPUR_SIGMA_NM = 2.0
LET_KEV_PER_UM = 0.8           # 8 MeV cm^2/g, a 70 MeV-proton-like track
GY_UM3_IN_EV = 6.241509074e3   # 1 Gy deposited in 1 um^3 of water, in eV

# step lattice of the workloads: times 1 ps * 10^(6 j / 1999) after an injection
DT0_NS = 1e-3
RATIO = 10.0 ** (6.0 / 1999.0)


@dataclasses.dataclass
class Injection:
    t: float                 # ns
    xyz: np.ndarray          # (n, 3) float32 inside [-L/2, L/2)
    species: np.ndarray      # (n,) uint8
    edep_ev: float           # energy deposited by the tracks of this injection


@dataclasses.dataclass
class Workload:
    name: str
    L: float                 # nm
    seed: int
    injections: List[Injection]
    records: np.ndarray      # record times, ns
    t_end: float             # ns
    D: list = dataclasses.field(default_factory=lambda: list(D_CONFIG))
    reactions: list = dataclasses.field(default_factory=lambda: list(REACTIONS))
    dose_gy: float = 0.0
    dt0: float = DT0_NS      # first step after each injection, ns
    ratio: float = RATIO     # ratio of successive step end times after an injection

    @property
    def n_initial(self) -> int:
        return int(sum(len(i.species) for i in self.injections))


def _into_box(p: np.ndarray, L: float) -> np.ndarray:
    """float64 positions -> float32 inside [-L/2, L/2)."""
    q = np.mod(p + 0.5 * L, L) - 0.5 * L
    q = q.astype(np.float32)
    hi = np.float32(0.5 * L)
    lo = np.float32(-0.5 * L)
    q[q >= hi] = np.nextafter(hi, np.float32(0.0))
    q[q < lo] = lo
    return q


def spur_centres_along(rng, start: np.ndarray, direction: np.ndarray, length: float) -> np.ndarray:
    """Spur centres on a straight segment, exponential spacing (mean 100 nm)."""
    s = []
    pos = rng.exponential(SPUR_SPACING_NM)
    while pos < length:
        s.append(pos)
        pos += rng.exponential(SPUR_SPACING_NM)
    s = np.asarray(s, dtype=np.float64)
    return start[None, :] + s[:, None] * direction[None, :]


def spur_molecules(rng, centres: np.ndarray):
    """Poisson(5.13) molecules per spur at Gaussian offsets (sigma 2 nm)."""
    counts = rng.poisson(SPUR_MEAN_MOLECULES, size=len(centres))
    idx = np.repeat(np.arange(len(centres)), counts)
    pos = centres[idx] + rng.normal(0.0, SPUR_SIGMA_NM, size=(len(idx), 3))
    sp = rng.choice(len(SPUR_FRACTIONS), size=len(idx), p=SPUR_FRACTIONS).astype(np.uint8)
    return pos, sp


def _isotropic(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def tracks_z(rng, L: float, n_tracks: int):
    """Tracks parallel to z through the cube, (x, y) uniform on the face."""
    pos_all, sp_all = [], []
    for _ in range(n_tracks):
        start = np.array([rng.uniform(-L / 2, L / 2), rng.uniform(-L / 2, L / 2), -L / 2])
        c = spur_centres_along(rng, start, np.array([0.0, 0.0, 1.0]), L)
        p, s = spur_molecules(rng, c)
        pos_all.append(p)
        sp_all.append(s)
    if not pos_all:
        return np.zeros((0, 3)), np.zeros(0, np.uint8)
    return np.concatenate(pos_all), np.concatenate(sp_all)


def tracks_iso(rng, L: float, n_tracks: int, length: float):
    """Isotropic straight tracks of the given length (wrapping through the cube)."""
    pos_all, sp_all = [], []
    for _ in range(n_tracks):
        start = rng.uniform(-L / 2, L / 2, size=3)
        c = spur_centres_along(rng, start, _isotropic(rng), length)
        p, s = spur_molecules(rng, c)
        pos_all.append(p)
        sp_all.append(s)
    return np.concatenate(pos_all), np.concatenate(sp_all)


def tracks_per_gray(L: float) -> float:
    """Eq. (5) solved for N at 1 Gy: N = D L^2 / (S/rho), S/rho from the LET."""
    let_ev_per_nm = LET_KEV_PER_UM  # keV/um == eV/nm
    e_per_track = let_ev_per_nm * L
    return GY_UM3_IN_EV * (L / 1000.0) ** 3 / e_per_track


def log_times(t0: float, t1: float, n: int) -> np.ndarray:
    return t0 * (t1 / t0) ** (np.arange(n) / (n - 1))


# ------------------------------------------------------------ workloads ---
def single_pulse_small(seed: int, n_tracks: int = 5, track_nm: float = 39000.0) -> Workload:
    """~1e4 molecules along 5 isotropic tracks in a 1 um cube, 1 ps -> 1 us."""
    L = 1000.0
    rng = np.random.default_rng([seed, 0])
    pos, sp = tracks_iso(rng, L, n_tracks, track_nm)
    edep = n_tracks * track_nm * LET_KEV_PER_UM
    inj = Injection(0.0, _into_box(pos, L), sp, edep)
    # records: t = 0 and every 20th lattice time up to 1 us
    j = np.concatenate([np.arange(0, 2000, 20), [1999]])
    rec = np.concatenate([[0.0], DT0_NS * 10.0 ** (6.0 * j / 1999.0)])
    rec[-1] = 1000.0
    return Workload("single_pulse_1um_1e4", L, seed, [inj], rec, 1000.0,
                    dose_gy=edep / (GY_UM3_IN_EV * (L / 1000.0) ** 3))


def single_pulse_large(seed: int, dose_gy: float = 1.0, L: float = 10000.0,
                       t_end: float = 1.0e6, n_records: int = 100) -> Workload:
    """One 1 Gy pulse of z-parallel tracks (~4e5 molecules) in a 10 um cube."""
    rng = np.random.default_rng([seed, 1])
    n_tr = int(round(tracks_per_gray(L) * dose_gy))
    pos, sp = tracks_z(rng, L, n_tr)
    edep = n_tr * L * LET_KEV_PER_UM
    inj = Injection(0.0, _into_box(pos, L), sp, edep)
    rec = np.concatenate([[0.0], log_times(DT0_NS, t_end, n_records)])
    rec[-1] = t_end
    return Workload(f"single_pulse_{L/1000:g}um_{dose_gy:g}Gy", L, seed, [inj], rec, t_end,
                    dose_gy=dose_gy)


def multi_pulse(seed: int, n_pulses: int = 20, dose_per_pulse: float = 1.0, L: float = 10000.0,
                pulse_rate_gy_s: float = 1e6, avg_rate_gy_s: float = 1e3, n_batches: int = 10,
                n_records: int = 100, t_tail: Optional[float] = None) -> Workload:
    """Pulsed irradiation: width W = Dp / Ddot_p, period T = Dp / Ddot_av.

    Track arrival times are uniform within each pulse; tracks are grouped into
    n_batches equal sub-intervals and injected at the start of their
    sub-interval.  Records: n_records log-spaced times after each pulse start
    (1 ps to the period)."""
    rng = np.random.default_rng([seed, 2])
    W = dose_per_pulse / pulse_rate_gy_s * 1e9      # ns
    T = dose_per_pulse / avg_rate_gy_s * 1e9        # ns
    n_tr = int(round(tracks_per_gray(L) * dose_per_pulse))
    injections = []
    records = [0.0]
    for p in range(n_pulses):
        tp = p * T
        arrive = rng.uniform(0.0, W, size=n_tr)
        batch = np.minimum((arrive / W * n_batches).astype(int), n_batches - 1)
        for b in range(n_batches):
            k = int(np.sum(batch == b))
            if k == 0:
                continue
            pos, sp = tracks_z(rng, L, k)
            injections.append(Injection(tp + b * W / n_batches, _into_box(pos, L), sp,
                                        k * L * LET_KEV_PER_UM))
        span = T if p + 1 < n_pulses else (t_tail if t_tail is not None else T)
        records.extend(tp + log_times(DT0_NS, span, n_records))
    t_end = (n_pulses - 1) * T + (t_tail if t_tail is not None else T)
    rec = np.unique(np.asarray(records))
    return Workload(f"multi_pulse_{n_pulses}x{dose_per_pulse:g}Gy_{avg_rate_gy_s:g}Gys", L, seed,
                    injections, rec, t_end, dose_gy=n_pulses * dose_per_pulse)


def homogeneous(seed: int, L: float, conc_per_nm3: dict, t_end: float, n_records: int = 60,
                D=None, reactions=None) -> Workload:
    """Uniformly mixed molecules (volume-scaling and kinetics checks)."""
    rng = np.random.default_rng([seed, 3])
    pos_all, sp_all = [], []
    for s, c in conc_per_nm3.items():
        n = int(round(c * L ** 3))
        pos_all.append(rng.uniform(-L / 2, L / 2, size=(n, 3)))
        sp_all.append(np.full(n, s, dtype=np.uint8))
    pos = np.concatenate(pos_all)
    sp = np.concatenate(sp_all)
    inj = Injection(0.0, _into_box(pos, L), sp, 0.0)
    rec = np.concatenate([[0.0], log_times(DT0_NS, t_end, n_records)])
    rec[-1] = t_end
    return Workload(f"homogeneous_{L:g}nm", L, seed, [inj], rec, t_end,
                    D=list(D) if D is not None else list(D_CONFIG),
                    reactions=list(reactions) if reactions is not None else list(REACTIONS))


# Volume-scaling mixture: the species fractions of the spur model at a total
# of 2.5e5 molecules per um^3 (4.15e-4 mol/L), dense enough that a 0.2 um cube
# still holds 2000 molecules; the paper scales the single-pulse yields up in
# the same way so that its smallest cube is populated.
VOLUME_SCALING_TOTAL_PER_NM3 = 2.5e-4
VOLUME_SCALING_EDGES_NM = (200.0, 500.0, 1000.0)


def volume_scaling_conc() -> dict:
    """Species -> molecules per nm^3 of the volume-scaling mixture."""
    return {s: VOLUME_SCALING_TOTAL_PER_NM3 * f for s, f in enumerate(SPUR_FRACTIONS) if f > 0}


def volume_scaling(seed: int, L: float, t_end: float = 1e4, n_records: int = 40) -> Workload:
    """The homogeneous volume-scaling mixture in a cube of edge L nm."""
    return homogeneous(seed, L, volume_scaling_conc(), t_end, n_records=n_records)


def volume_scaling_counts(L: float) -> np.ndarray:
    """Initial counts of the volume-scaling mixture in a cube of edge L nm
    (the same rounding as volume_scaling)."""
    n = np.zeros(len(SPECIES), dtype=np.int64)
    for s, c in volume_scaling_conc().items():
        n[s] = int(round(c * L ** 3))
    return n


def batched_instances(seed: int, n_instances: int = 64):
    """Independent instances of uneven size for batched runs: box edge U(2,10) um,
    dose per pulse U(0.1, 2) Gy, 1-20 pulses, average dose rate log-uniform in
    0.01-1e5 Gy/s, pulse dose rate 1e6 Gy/s."""
    rng = np.random.default_rng([seed, 4])
    out = []
    for i in range(n_instances):
        L = float(rng.uniform(2000.0, 10000.0))
        dp = float(rng.uniform(0.1, 2.0))
        n_p = int(rng.integers(1, 21))
        dav = float(10.0 ** rng.uniform(-2.0, 5.0))
        out.append(dict(L=L, dose_per_pulse=dp, n_pulses=n_p, avg_rate=dav, seed=seed * 1000 + i))
    return out


def batched_first_pulses(seed: int, n_instances: int = 64):
    """The first pulse of every batched instance as one injection at t = 0
    (z-parallel tracks of that instance's dose): [(L, Injection)]."""
    out = []
    for p in batched_instances(seed, n_instances):
        rng = np.random.default_rng([p["seed"], 5])
        L = p["L"]
        n_tr = int(round(tracks_per_gray(L) * p["dose_per_pulse"]))
        pos, sp = tracks_z(rng, L, n_tr)
        out.append((L, Injection(0.0, _into_box(pos, L), sp, n_tr * L * LET_KEV_PER_UM)))
    return out


# Batched campaign: every instance of batched_instances with its whole pulse
# train, each pulse split into n_batches injection batches of z-parallel
# tracks drawn on the device by the counter-based spur model
# (gsbs_inject_pulse).  Only times and track counts are drawn here.
CAMPAIGN_STEP_BUDGET = 20000
CAMPAIGN_PULSE_RATE_GY_S = 1e6


@dataclasses.dataclass
class CampaignInstance:
    L: float                  # nm
    dose_per_pulse: float     # Gy
    n_pulses: int
    avg_rate: float           # Gy/s
    width: float              # ns, pulse width = dose / pulse rate
    period: float             # ns, dose / average rate
    batches: list             # [(t_ns, n_tracks, stream)], in time order
    records: np.ndarray       # ns
    t_end: float              # ns: one period after the last pulse starts


def campaign(seed: int, n_instances: int = 64, n_batches: int = 10, n_records: int = 20,
             pulse_rate_gy_s: float = CAMPAIGN_PULSE_RATE_GY_S) -> List[CampaignInstance]:
    """Instances of batched_instances(seed) as pulse trains: rectangular pulses
    of width Dp / Ddot_p every Dp / Ddot_av, track arrivals uniform in the
    pulse and grouped into n_batches equal sub-intervals (each injected at its
    start), records at n_records log-spaced times after every pulse start.
    Spur-model streams are (instance << 32) | (pulse * n_batches + batch)."""
    out = []
    for i, p in enumerate(batched_instances(seed, n_instances)):
        rng = np.random.default_rng([p["seed"], 6])
        L = p["L"]
        W = p["dose_per_pulse"] / pulse_rate_gy_s * 1e9
        T = p["dose_per_pulse"] / p["avg_rate"] * 1e9
        n_tr = int(round(tracks_per_gray(L) * p["dose_per_pulse"]))
        batches, records = [], [0.0]
        for q in range(p["n_pulses"]):
            tp = q * T
            arrive = rng.uniform(0.0, W, size=n_tr)
            b = np.minimum((arrive / W * n_batches).astype(int), n_batches - 1)
            cnt = np.bincount(b, minlength=n_batches)
            for k in range(n_batches):
                if cnt[k]:
                    batches.append((tp + k * W / n_batches, int(cnt[k]), (i << 32) | (q * n_batches + k)))
            records.extend(tp + log_times(DT0_NS, T, n_records))
        t_end = (p["n_pulses"] - 1) * T + T
        out.append(CampaignInstance(L, p["dose_per_pulse"], p["n_pulses"], p["avg_rate"], W, T, batches,
                                    np.unique(np.asarray(records)), t_end))
    return out
