"""Batched multi-pulse campaign: many independent cubes of uneven size, dose
per pulse, pulse count and average dose rate stepped together by one engine.

Each instance is a pulse train (workload.campaign): rectangular pulses, each
split into injection batches of z-parallel tracks that the library draws on
the device from the counter-based spur model (gsbs_inject_pulse).  Plain SBS
cannot cover inter-pulse intervals of up to 100 s, so every instance runs to
the end of its train or to the end of its budget-th step, whichever comes
first.  Step times follow from injection, record and target times alone
(gsbs_plan_schedule), so the budget fixes each instance's target time before
anything runs; only batches before the target are queued.

This module drives the library; it holds none of the method's arithmetic.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import gsbs
from . import workload as W


@dataclasses.dataclass
class Setup:
    engine: gsbs.Engine
    targets: np.ndarray        # ns, per instance
    planned_steps: np.ndarray  # SBS steps per instance up to its target
    batches: np.ndarray        # injection batches queued per instance
    molecules: int             # molecules queued over all instances
    edep_ev: np.ndarray        # energy of the queued batches per instance
    schedules: list            # step end times per instance up to its target

    def targets_after(self, g: int) -> np.ndarray:
        """Per instance, the end time of global step g (1-based; instances
        with fewer steps stop at their target)."""
        return np.array([s[min(g, len(s)) - 1] if len(s) else t for s, t in zip(self.schedules, self.targets)])


def targets_for(insts: List[W.CampaignInstance], dt_max: List[float], budget: int,
                dt0: float = W.DT0_NS, ratio: float = W.RATIO):
    """Per instance: the end of its train or of its budget-th step, and the
    number of steps up to there."""
    tg, ns, sc = [], [], []
    for x, dm in zip(insts, dt_max):
        anchors = np.array([b[0] for b in x.batches])
        events = np.concatenate([x.records, anchors])
        sched = gsbs.gsbs_plan_schedule(0.0, x.t_end, anchors, np.unique(events), dt0, ratio, dm)
        if len(sched) > budget:
            tg.append(float(sched[budget - 1]))
            ns.append(budget)
            sc.append(sched[:budget])
        else:
            tg.append(float(x.t_end))
            ns.append(len(sched))
            sc.append(sched)
    return np.array(tg), np.array(ns, dtype=np.int64), sc


def setup(insts: List[W.CampaignInstance], seed: int = 1000, budget: int = W.CAMPAIGN_STEP_BUDGET,
          params: Optional[gsbs.gsbs_params] = None, stream=None) -> Setup:
    """An engine with every instance's batches before its target queued (drawn
    on the device) and its records set."""
    e = gsbs.Engine([x.L for x in insts], seed, W.D_CONFIG, W.REACTIONS, params=params, stream=stream)
    dm = [e.dt_max(i) for i in range(len(insts))]
    tg, ns, sc = targets_for(insts, dm, budget)
    nb = np.zeros(len(insts), dtype=np.int64)
    ed = np.zeros(len(insts))
    mol = 0
    for i, x in enumerate(insts):
        for (t, n_tr, stream_id) in x.batches:
            if not t < tg[i]:
                break
            mol += e.inject_pulse(i, t, n_tr, W.SPUR_FRACTIONS, stream=stream_id, spacing_nm=W.SPUR_SPACING_NM,
                                  mol_per_spur=W.SPUR_MEAN_MOLECULES, sigma_nm=W.SPUR_SIGMA_NM,
                                  let_kev_per_um=W.LET_KEV_PER_UM)
            nb[i] += 1
            ed[i] += n_tr * x.L * W.LET_KEV_PER_UM
        e.set_records(i, x.records[x.records <= tg[i]])
    return Setup(e, tg, ns, nb, int(mol), ed, sc)
