"""Inter-pulse surrogate of the multi-pulse SBS run.

Between pulses the chemistry relaxes towards a homogeneous mixture; the paper
integrates that stretch with rate equations (its Eq. 3-4).  Here a perceptron
(device kernels behind gsbs_mlp_*) maps the state a settle time after a
pulse's last batch -- species concentrations, pair-correlation features of
the 9 reactions and the time to the next pulse (gsbs_features) -- to the
change of the log concentrations at the next pulse; the instance is then
re-populated homogeneously at those counts (gsbs_repopulate) and the next
pulse is injected into it.  Plain SBS is the fallback whenever a held-out
error table says the network's G(H2O2) error could exceed 1 %, and it is the
reference that error is measured against.

This module drives the library: it builds pulse plans from the synthetic track
generator, runs the engine to make training samples (features at the switch
time, log concentrations at the next pulse), trains the network with the
device kernels, fills the error table, and runs the hybrid or the plain
multi-pulse schedule.  All arithmetic of the step, the features, the network
and the re-population runs in the library's kernels; this file only prepares
inputs, normalisation constants and bookkeeping.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import gsbs
from . import workload as W

NA = 6.02214076e23
C_FLOOR = 1e-10       # mol/L added to a concentration before its logarithm
R_MAX = 200.0         # nm, outer edge of the pair-correlation shells
N_REF = 1024          # references per species for the pair correlations
TAU_SETTLE = 1000.0   # ns after a pulse's last batch before the network takes over
H2O2 = W.H2O2


@dataclasses.dataclass
class PulsePlan:
    """Pulsed irradiation of one cube (rectangular pulses, batches as in the
    workload generator)."""
    L: float
    seed: int
    n_pulses: int
    dose: float            # Gy per pulse
    pulse_rate: float      # Gy/s during a pulse
    avg_rate: float        # Gy/s averaged over the run
    n_batches: int = 2

    @property
    def width(self) -> float:  # ns
        return self.dose / self.pulse_rate * 1e9

    @property
    def period(self) -> float:  # ns
        return self.dose / self.avg_rate * 1e9

    def start(self, p: int) -> float:
        return p * self.period

    def switch(self, p: int) -> float:
        """Hand-over time after pulse p: the settle time after its last
        injection (the library's rule, gsbs_advance_to)."""
        self.injections()
        return self._last.get(p, self.start(p)) + TAU_SETTLE

    def injections(self) -> List[W.Injection]:
        if hasattr(self, "_inj"):
            return self._inj
        self._inj = self._make_injections()
        return self._inj

    def _make_injections(self) -> List[W.Injection]:
        self._last = {}  # pulse -> time of its last injection
        rng = np.random.default_rng([self.seed, 7])
        n_tr = int(round(W.tracks_per_gray(self.L) * self.dose))
        out = []
        for p in range(self.n_pulses):
            arrive = rng.uniform(0.0, self.width, size=n_tr)
            batch = np.minimum((arrive / self.width * self.n_batches).astype(int), self.n_batches - 1)
            for b in range(self.n_batches):
                k = int(np.sum(batch == b))
                if k == 0:
                    continue
                pos, sp = W.tracks_z(rng, self.L, k)
                out.append(W.Injection(self.start(p) + b * self.width / self.n_batches, W._into_box(pos, self.L), sp,
                                       k * self.L * W.LET_KEV_PER_UM))
                self._last[p] = out[-1].t
        return out

    def edep_until(self, t: float, inj: List[W.Injection]) -> float:
        return float(sum(i.edep_ev for i in inj if i.t <= t))


def log_conc(counts, L) -> np.ndarray:
    return np.log10(np.asarray(counts, dtype=np.float64) / (NA * L ** 3 * 1e-24) + C_FLOOR)


def _engine(Ls, seed, capacity=0):
    p = gsbs.gsbs_default_params()
    p.autotune = 1
    return gsbs.Engine(Ls, seed, W.D_CONFIG, W.REACTIONS, params=p, capacity=capacity)


# ------------------------------------------------------------- training data ---
def generate(plans: List[PulsePlan], seed: int, log=None, t_cap: Optional[float] = None) -> dict:
    """Run every plan with plain SBS as one batched context (one instance per
    plan) and collect, for every pulse but the last, the raw features at the
    switch time and the log concentrations there and at the next pulse.

    With t_cap (ns), an interval longer than t_cap after the switch time is
    simulated only to switch + t_cap: by then the radicals have recombined and
    the homogeneous mixture of inert products and a few ions no longer changes
    within the count noise, so its state there is the target, and the cube is
    carried to the next pulse start unchanged (re-populated at the same
    counts)."""
    n = len(plans)
    e = _engine([pl.L for pl in plans], seed)
    inj = [pl.injections() for pl in plans]
    for i, pl in enumerate(plans):
        for j in inj[i]:
            e.inject(i, j.t, j.xyz, j.species, j.edep_ev)
    events = []
    for i, pl in enumerate(plans):
        ev = []
        for p in range(pl.n_pulses - 1):
            ev.append((pl.switch(p), "switch", p))
            if t_cap is not None and pl.start(p + 1) - pl.switch(p) > t_cap:
                ev.append((pl.switch(p) + t_cap, "capped", p))
            else:
                ev.append((pl.start(p + 1), "next", p))
        events.append(ev)
    pos = [0] * n
    X, Y0, Y1, meta = [], [], [], []
    pending = {}
    t0 = time.perf_counter()
    while any(pos[i] < len(events[i]) for i in range(n)):
        tgt = [events[i][pos[i]][0] if pos[i] < len(events[i]) else e.time(i) for i in range(n)]
        e.advance_to(tgt)
        for i in range(n):
            if pos[i] >= len(events[i]):
                continue
            t, kind, p = events[i][pos[i]]
            pl = plans[i]
            if kind == "switch":
                x = gsbs.gsbs_features(e.ctx, i, pl.start(p + 1) - t, R_MAX, N_REF, C_FLOOR)
                pending[i] = (x, log_conc(e.current_counts(i), pl.L), pl.start(p + 1) - t)
            else:
                # the state just before the next pulse: the step that ends at t also
                # injected the molecules due at t, which are taken out again
                x, y0, dt = pending.pop(i)
                fresh = np.zeros(len(W.D_CONFIG), dtype=np.int64)
                for j in inj[i]:
                    if j.t == t:
                        fresh += np.bincount(j.species, minlength=len(W.D_CONFIG))[:len(W.D_CONFIG)]
                X.append(x)
                Y0.append(y0)
                Y1.append(log_conc(e.current_counts(i) - fresh, pl.L))
                meta.append((math.log10(dt), math.log10(pl.avg_rate), float(np.sum(10.0 ** y0))))
                if kind == "capped":  # carried unchanged to the next pulse start
                    z = np.zeros(7, np.float32)
                    gsbs.gsbs_repopulate(e.ctx, i, pl.start(p + 1), z, z, np.ones(7, np.float32), C_FLOOR,
                                         relative=True)
            pos[i] += 1
        if log:
            log(f"generate: {sum(pos)}/{sum(len(v) for v in events)} events, {time.perf_counter() - t0:.1f} s")
    e.close()
    return dict(X=np.array(X, dtype=np.float32), Y0=np.array(Y0), Y1=np.array(Y1), meta=np.array(meta))


def random_plans(seed: int, n: int, L: float = 2000.0, n_pulses: int = 6, rates=(300.0, 1e4),
                 doses=(0.5, 1.5)) -> List[PulsePlan]:
    rng = np.random.default_rng([seed, 11])
    out = []
    for k in range(n):
        rate = float(10 ** rng.uniform(math.log10(rates[0]), math.log10(rates[1])))
        dose = float(rng.uniform(*doses))
        out.append(PulsePlan(L, seed * 100003 + k, n_pulses, dose, 1e6, rate))
    return out


# ------------------------------------------------------------------ network ---
class Surrogate:
    """Network weights, normalisation constants and the held-out error table."""

    def __init__(self, max_batch: int = 4096):
        self.net = gsbs.Mlp(max_batch)
        self.max_batch = max_batch
        self.mu = self.sd = self.mu_y = self.sd_y = None
        self.lo = self.hi = None
        self.table = None       # 95th percentile of |dN_H2O2| / N_H2O2 per (log dt, log C_tot) bin
        self.dt_edges = self.c_edges = None
        self.bias = np.zeros(gsbs.MLP_OUT, dtype=np.float32)  # mean held-out log10 residual, subtracted

    def init_weights(self, seed: int):
        """Weights and biases uniform in +-1/sqrt(fan_in) (seeded)."""
        rng = np.random.default_rng(seed)
        parts = []
        sizes = [gsbs.MLP_IN] + [gsbs.MLP_HIDDEN] * 4 + [gsbs.MLP_OUT]
        for l in range(5):
            k, n = sizes[l], sizes[l + 1]
            lim = 1.0 / math.sqrt(k)
            parts += [rng.uniform(-lim, lim, size=n * k), rng.uniform(-lim, lim, size=n)]
        self.net.set_weights(np.concatenate(parts).astype(np.float32))

    def fit(self, data: dict, epochs: int = 60, batch: int = 64, lr: float = 5e-4, seed: int = 0, log=None,
            val: Optional[dict] = None, g_weight: float = 1.0):
        """Adam with a cosine learning-rate decay on the device kernels; with
        `val`, the weights of the epoch with the lowest validation loss are kept.
        g_weight scales the pair-correlation inputs after normalisation (0 hides
        them from the network)."""
        import torch
        X, Y = data["X"].astype(np.float64), (data["Y1"] - data["Y0"])
        self.mu = X.mean(axis=0).astype(np.float32)
        # features that barely vary in the training set are only centred, not
        # stretched: a small change elsewhere must not become a large input
        sd = X.std(axis=0)
        sd = np.where(sd < 1e-2 * (1.0 + np.abs(self.mu)), 1.0 + np.abs(self.mu), sd)
        sd[7:7 + 9 * 32] /= max(g_weight, 1e-30)
        self.sd = sd.astype(np.float32)
        self.g_weight = g_weight
        self.mu_y = Y.mean(axis=0).astype(np.float32)
        self.sd_y = np.maximum(Y.std(axis=0), 1e-4).astype(np.float32)
        Xn = np.clip((X - self.mu) / self.sd, -8.0, 8.0).astype(np.float32)
        Yn = ((Y - self.mu_y) / self.sd_y).astype(np.float32)
        self.lo, self.hi = Xn.min(axis=0), Xn.max(axis=0)
        xd = torch.from_numpy(Xn).cuda()
        yd = torch.from_numpy(Yn).cuda()
        n = len(Xn)
        rng = np.random.default_rng(seed)
        hist = []
        steps = 0
        total = epochs * max(1, n // batch)
        best = (np.inf, None)
        if val is not None:
            xv = torch.from_numpy(np.clip((val["X"].astype(np.float64) - self.mu) / self.sd, -8.0, 8.0)
                                  .astype(np.float32)).cuda()
            yv = ((val["Y1"] - val["Y0"]) - self.mu_y) / self.sd_y
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            ls = []
            for b0 in range(0, n - batch + 1 if n >= batch else 1, batch):
                idx = perm[b0:b0 + batch]
                rate = lr * 0.5 * (1.0 + math.cos(math.pi * steps / total))
                ls.append(self.net.train_step(xd[idx].contiguous(), yd[idx].contiguous(), rate))
                steps += 1
            hist.append(float(np.mean(ls)))
            vl = None
            if val is not None:
                vl = float(np.mean((self.net.forward(xv).cpu().numpy().astype(np.float64) - yv) ** 2))
                if vl < best[0]:
                    best = (vl, self.net.get_weights())
            if log and (ep % 20 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {hist[-1]:.5f}" + (f", validation {vl:.5f}" if vl is not None else ""))
        if best[1] is not None:
            self.net.set_weights(best[1])
            self.val_loss = best[0]
        return hist

    def predict_log(self, X_raw: np.ndarray, Y0: np.ndarray) -> np.ndarray:
        """Predicted log10 concentrations at the next pulse (for evaluation)."""
        import torch
        Xn = np.clip((X_raw.astype(np.float64) - self.mu) / self.sd, -8.0, 8.0).astype(np.float32)
        yn = self.net.forward(torch.from_numpy(Xn).cuda()).cpu().numpy().astype(np.float64)
        return Y0 + yn * self.sd_y + self.mu_y - self.bias

    def calibrate(self, data: dict) -> np.ndarray:
        """Mean signed residual of the predicted log10 concentrations on held-out
        samples, per species; later predictions subtract it.  A small systematic
        offset is harmless for one interval but adds up over consecutive
        intervals the network takes."""
        self.bias = np.zeros(gsbs.MLP_OUT, dtype=np.float32)
        r = self.predict_log(data["X"], data["Y0"]) - data["Y1"]
        self.bias = r.mean(axis=0).astype(np.float32)
        return self.bias

    def mu_out(self) -> np.ndarray:
        """Output offsets for the re-population (the calibration folded in)."""
        return (self.mu_y.astype(np.float64) - self.bias).astype(np.float32)

    def build_table(self, data: dict, n_dt: int = 4, n_c: int = 3):
        """95th percentile of the relative H2O2 error per (log dt, log C_tot) bin
        on held-out samples; empty bins get infinity (always plain SBS)."""
        pred = self.predict_log(data["X"], data["Y0"])
        n_true = 10.0 ** data["Y1"][:, H2O2]
        n_pred = 10.0 ** pred[:, H2O2]
        err = np.abs(n_pred - n_true) / np.maximum(n_true, 1e-30)
        ldt, lc = data["meta"][:, 0], np.log10(data["meta"][:, 2])
        self.dt_edges = np.quantile(ldt, np.linspace(0, 1, n_dt + 1))
        self.c_edges = np.quantile(lc, np.linspace(0, 1, n_c + 1))
        self.table = np.full((n_dt, n_c), np.inf)
        i = np.clip(np.searchsorted(self.dt_edges, ldt, side="right") - 1, 0, n_dt - 1)
        j = np.clip(np.searchsorted(self.c_edges, lc, side="right") - 1, 0, n_c - 1)
        for a in range(n_dt):
            for b in range(n_c):
                m = (i == a) & (j == b)
                if m.sum() >= 5:
                    self.table[a, b] = float(np.quantile(err[m], 0.95))
        return err

    def interval_error(self, log_dt: float, c_tot: float, x_norm: np.ndarray) -> float:
        """Held-out error estimate (95th percentile of |dN_H2O2| / N_H2O2) for an
        interval; infinity outside the table or the training inputs' range."""
        if self.table is None:
            return math.inf
        if log_dt < self.dt_edges[0] or log_dt > self.dt_edges[-1]:
            return math.inf
        lc = math.log10(c_tot)
        if lc < self.c_edges[0] or lc > self.c_edges[-1]:
            return math.inf
        span = self.hi - self.lo
        if np.any(x_norm < self.lo - 0.1 * span - 1e-3) or np.any(x_norm > self.hi + 0.1 * span + 1e-3):
            return math.inf
        a = int(np.clip(np.searchsorted(self.dt_edges, log_dt, side="right") - 1, 0, len(self.dt_edges) - 2))
        b = int(np.clip(np.searchsorted(self.c_edges, lc, side="right") - 1, 0, len(self.c_edges) - 2))
        return float(self.table[a, b])

    def usable(self, log_dt: float, c_tot: float, x_norm: np.ndarray, tol: float = 0.01) -> bool:
        return self.interval_error(log_dt, c_tot, x_norm) <= tol

    def save(self, path: str):
        np.savez(path, w=self.net.get_weights(), mu=self.mu, sd=self.sd, mu_y=self.mu_y, sd_y=self.sd_y, lo=self.lo,
                 hi=self.hi, table=self.table, dt_edges=self.dt_edges, c_edges=self.c_edges, bias=self.bias)

    def load(self, path: str):
        z = np.load(path)
        self.net.set_weights(z["w"])
        for k in ("mu", "sd", "mu_y", "sd_y", "lo", "hi", "table", "dt_edges", "c_edges"):
            setattr(self, k, z[k])
        self.bias = z["bias"] if "bias" in z.files else np.zeros(gsbs.MLP_OUT, dtype=np.float32)


# ------------------------------------------------------------ multi-pulse run ---
def set_on(e: gsbs.Engine, surrogate: "Surrogate", tol: float = 0.01, budget: Optional[float] = None):
    """Hand the surrogate to the library (gsbs_set_surrogate): normalisation
    (calibration folded into the output centres), training range, error table."""
    gsbs.gsbs_set_surrogate(e.ctx, surrogate.net.h, mu=surrogate.mu, sd=surrogate.sd, mu_y=surrogate.mu_out(),
                            sd_y=surrogate.sd_y, dt_edges=surrogate.dt_edges, c_edges=surrogate.c_edges,
                            table=surrogate.table, lo=surrogate.lo, hi=surrogate.hi, settle_ns=TAU_SETTLE, tol=tol,
                            budget=budget or 0.0, r_max_nm=R_MAX, c_floor_M=C_FLOOR, n_ref_max=N_REF)


def run(plan: PulsePlan, surrogate: Optional[Surrogate] = None, seed: int = 1, tol: float = 0.01,
        budget: Optional[float] = None, numodes_rtol: Optional[float] = None, log=None) -> dict:
    """Plain (surrogate None) or hybrid multi-pulse run of one cube.  Returns
    the H2O2 count and G(H2O2) at every pulse start after the first and at the
    end, the wall time and the number of intervals the network took.

    With a surrogate the whole run is one gsbs_advance_to in GSBS_SURROGATE
    mode: the library stops each interval's hand-over point, applies the
    error table, the input-range guard and the budget, and runs the network
    and the re-population (see gsbs.h).  Records at the hand-over points and
    at the pulse starts make those step ends in the plain run too, so both
    runs follow the same trajectory up to the first interval the network takes.

    With numodes_rtol (and no surrogate) every interval goes to the rate
    equations instead (the paper's SBS + NumODEs alternation): the counts at
    the switch time become concentrations, gsbs_numodes carries them to the
    next pulse start and the cube is re-populated homogeneously."""
    import torch
    inj = plan.injections()
    e = _engine(plan.L, seed)
    for j in inj:
        e.inject(0, j.t, j.xyz, j.species, j.edep_ev)
    n = plan.n_pulses
    t_sw = [plan.switch(p) for p in range(n - 1)]
    t_nx = [plan.start(p + 1) for p in range(n)]
    rec = np.unique(np.array(t_sw + t_nx))
    e.set_records(0, rec)
    used = np.zeros(n, dtype=bool)
    spent = 0.0
    handover = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if surrogate is not None:
        set_on(e, surrogate, tol, budget)
        # pulse by pulse (the hand-over points of each interval lie inside one call)
        for p in range(n):
            e.advance_to(t_nx[p], gsbs.GSBS_SURROGATE)
            if log:
                log(f"hybrid run: pulse {p + 1}/{n} started, {time.perf_counter() - t0:.1f} s")
        lg = gsbs.gsbs_get_handover_log(e.ctx, 0)
        handover = {k: np.asarray(v) for k, v in lg.items()}
        for ts, tk, est in zip(lg["t_switch"], lg["taken"], lg["estimate"]):
            p = int(np.argmin(np.abs(np.array(t_sw) - ts)))
            used[p] = bool(tk)
            spent += float(est) if tk else 0.0
    elif numodes_rtol is not None:
        for p in range(n):
            if p + 1 < n:
                e.advance_to(t_sw[p])
                now = e.current_counts(0)
                conc = now.astype(np.float64) / (NA * plan.L ** 3 * 1e-24)
                c1, _ = gsbs.gsbs_numodes(e.ctx, conc[None, :], [t_nx[p] - t_sw[p]], rtol=numodes_rtol)
                y = np.log10(np.maximum(c1[0], 0.0) + C_FLOOR).astype(np.float32)
                gsbs.gsbs_repopulate(e.ctx, 0, t_nx[p], y, np.zeros(len(y), np.float32),
                                     np.ones(len(y), np.float32), C_FLOOR, relative=False)
                used[p] = True
            else:
                e.advance_to(t_nx[p])
        e.advance_to(t_nx[-1])  # takes the records at the last pulse start
    else:
        for p in range(n):
            e.advance_to(t_nx[p])
            if log:
                log(f"plain run: pulse {p + 1}/{n} started, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = e.counts(0)
    at_switch = np.array([counts[int(np.searchsorted(rec, t))] for t in t_sw])
    n_h2o2, g_h2o2 = [], []
    for t in t_nx:
        cnt = counts[int(np.searchsorted(rec, t))].copy()
        for j in inj:  # the record at a pulse start follows that start's injection
            if j.t == t:
                cnt -= np.bincount(j.species, minlength=len(cnt))[:len(cnt)]
        ed = plan.edep_until(t - 1e-9, inj)
        n_h2o2.append(int(cnt[H2O2]))
        g_h2o2.append(cnt[H2O2] / (ed / 100.0))
    st = e.stats()
    e.close()
    return dict(t=np.array(t_nx), n_h2o2=np.array(n_h2o2), g_h2o2=np.array(g_h2o2), wall=wall,
                intervals_by_network=int(used.sum()), used=used, counts_at_switch=at_switch,
                error_estimate_spent=spent, steps=st["steps"], molecule_steps=st["molecule_steps"], handover=handover)
