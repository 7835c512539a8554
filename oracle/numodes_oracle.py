"""FP64 CPU oracle of the homogeneous rate equations -- TEST INFRASTRUCTURE.

Only tests/ (and the smoke check) may import this module; the HIP engine never
imports, links or calls it and shares no code with it.

The beam-off stage of the paper (its NumODEs, Eq. 3-4) integrates the
mass-action rate equations of the reaction table: every reaction r between
species a and b proceeds at the event rate

    rho_r = k_r [a][b]            (a != b)
    rho_r = (k_r / 2) [a]^2       (a == b: the table prints 2k for the
                                   self-recombinations, and each event
                                   removes two molecules of a, so that
                                   d[a]/dt = -k_r [a]^2 -- the paper's
                                   equation for the OH recombination)

and d[X]/dt = sum_r rho_r (products of r that are X - reactants of r that are
X), with k_r in L/mol/ns (the table's 1e10 L/mol/s times 10 / 1e9 ns) and
concentrations in mol/L.  A reaction flagged keep_b consumes only a.  The
integration uses SciPy's Radau (implicit Runge-Kutta, order 5) with the
analytic Jacobian and tight tolerances: a library routine as one step.

Extension (the paper prints R9 as an equilibrium and leaves its reverse and
the pH background aside): zero-order sources, each producing its products at
a constant rate in mol/L/ns -- with R9's reverse, the water autoionisation at
k9 Kw, [H3O+][OH-] relaxes to Kw; and first-order channels a -> products at
k [a] (scavenging by a solute at a fixed concentration, e.g. O2).
"""
from __future__ import annotations

import numpy as np


def table(reactions):
    """(ra, rb, k in L/mol/ns, products, keep_b) arrays of a reaction list."""
    ra = np.array([r.a for r in reactions], dtype=np.int64)
    rb = np.array([r.b for r in reactions], dtype=np.int64)
    k = np.array([10.0 * r.k_in for r in reactions], dtype=np.float64)  # 1e10 /M/s = 10 /M/ns
    prods = [tuple(r.products) for r in reactions]
    keep = np.array([bool(getattr(r, "keep_b", False)) for r in reactions])
    return ra, rb, k, prods, keep


def event_rates(c, ra, rb, k):
    c = np.asarray(c, dtype=np.float64)
    same = ra == rb
    return np.where(same, 0.5 * k * c[ra] * c[ra], k * c[ra] * c[rb])


def rhs(c, reactions, sources=(), first_order=()):
    """d[X]/dt.  sources: zero-order reactions (rate in mol/L/ns, products),
    each adding its rate to every product; first_order: channels a -> products
    at k [a] (k per ns)."""
    ra, rb, k, prods, keep = table(reactions)
    rho = event_rates(c, ra, rb, k)
    d = np.zeros(len(c))
    for f in first_order:
        r1 = f.k * c[f.a]
        d[f.a] -= r1
        for p in f.products:
            d[p] += r1
    for src in sources:
        for p in src.products:
            d[p] += src.rate
    for r in range(len(ra)):
        d[ra[r]] -= rho[r]
        if not keep[r]:
            d[rb[r]] -= rho[r]
        for p in prods[r]:
            d[p] += rho[r]
    return d


def jacobian(c, reactions, first_order=()):
    ra, rb, k, prods, keep = table(reactions)
    c = np.asarray(c, dtype=np.float64)
    J = np.zeros((len(c), len(c)))
    for f in first_order:
        J[f.a, f.a] -= f.k
        for p in f.products:
            J[p, f.a] += f.k
    for r in range(len(ra)):
        a, b = ra[r], rb[r]
        # d rho / d c
        g = np.zeros(len(c))
        if a == b:
            g[a] = k[r] * c[a]
        else:
            g[a] += k[r] * c[b]
            g[b] += k[r] * c[a]
        J[a] -= g
        if not keep[r]:
            J[b] -= g
        for p in prods[r]:
            J[p] += g
    return J


def integrate(c0, dt, reactions, rtol=1e-11, atol=1e-24, sources=(), first_order=()):
    """Concentrations (mol/L) after dt ns from c0 (a zero-order source adds a
    constant to the right-hand side and nothing to the Jacobian)."""
    from scipy.integrate import solve_ivp
    c0 = np.asarray(c0, dtype=np.float64)
    if dt <= 0:
        return c0.copy()
    sol = solve_ivp(lambda t, y: rhs(y, reactions, sources, first_order), (0.0, float(dt)), c0, method="Radau",
                    jac=lambda t, y: jacobian(y, reactions, first_order), rtol=rtol, atol=atol)
    assert sol.success, sol.message
    return sol.y[:, -1]
