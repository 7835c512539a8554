"""Pins of the rate-equation oracle (CPU only).

  * A + A with the printed 2k: 1/[A](t) = 1/[A]0 + k t, the product at half
    the consumed amount (closed form of the paper's self-recombination law);
  * A + B with unequal starts: ln([B][A]0 / ([A][B]0)) = ([B]0 - [A]0) k t;
  * the Jacobian equals central finite differences of the right-hand side;
  * the full water scheme conserves charge (H3O+ - e_aq - OH-) and the redox
    balance (OH + 2 H2O2 - e_aq - H - 2 H2) to rounding;
  * a test-only sink (keep_b) decays A exponentially at k [B];
  * a zero-order source alone grows its products linearly, and with R9 the
    ion concentration relaxes along the tanh / coth closed form to sqrt(Kw).
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import numodes_oracle as N  # noqa: E402
from paper_2509_03313_amd import workload as W  # noqa: E402


def test_self_recombination_closed_form():
    r = [W.Reaction("X", 0, 0, 0.95, (1,))]
    a0 = 3e-6
    for t in (1e2, 1e4, 1e6):
        c = N.integrate([a0, 0.0], t, r)
        a = 1.0 / (1.0 / a0 + 10.0 * 0.95 * t)
        assert abs(c[0] - a) <= 1e-8 * a, (t, c[0], a)
        assert abs(c[1] - (a0 - a) / 2) <= 1e-8 * a0


def test_a_plus_b_closed_form():
    r = [W.Reaction("Y", 0, 1, 3.0, ())]
    a0, b0 = 2e-6, 5e-6
    k = 30.0
    for t in (1e3, 1e4, 1e5):
        c = N.integrate([a0, b0], t, r)
        lhs = math.log(c[1] * a0 / (c[0] * b0))
        assert abs(lhs - (b0 - a0) * k * t) <= 1e-7 * max(1.0, lhs), (t, lhs)
        assert abs((b0 - c[1]) - (a0 - c[0])) <= 1e-9 * b0


def test_jacobian_is_derivative_of_rhs():
    rng = np.random.default_rng(0)
    c = 10.0 ** rng.uniform(-8, -5, size=7)
    J = N.jacobian(c, W.REACTIONS)
    for j in range(7):
        h = 1e-6 * c[j]
        cp, cm = c.copy(), c.copy()
        cp[j] += h
        cm[j] -= h
        fd = (N.rhs(cp, W.REACTIONS) - N.rhs(cm, W.REACTIONS)) / (2 * h)
        assert np.allclose(fd, J[:, j], rtol=1e-6, atol=1e-12 * np.abs(J).max())


def test_water_scheme_conserves_charge_and_redox():
    rng = np.random.default_rng(1)
    c0 = 10.0 ** rng.uniform(-7, -5, size=7)
    c = N.integrate(c0, 1e6, W.REACTIONS)
    Q = lambda x: x[W.H3O] - x[W.E_AQ] - x[W.OHM]  # noqa: E731
    R = lambda x: x[W.OH] + 2 * x[W.H2O2] - x[W.E_AQ] - x[W.H] - 2 * x[W.H2]  # noqa: E731
    scale = c0.sum()
    assert abs(Q(c) - Q(c0)) <= 1e-9 * scale and abs(R(c) - R(c0)) <= 1e-9 * scale
    assert np.all(c >= -1e-15 * scale)


def test_sink_decays_exponentially():
    r = [W.Reaction("S", 0, 1, 2.0, (), keep_b=True)]
    a0, b = 1e-7, 4e-6
    t = 2e4
    c = N.integrate([a0, b], t, r)
    assert abs(c[0] - a0 * math.exp(-20.0 * b * t)) <= 1e-8 * a0 and c[1] == b


def test_source_alone_is_linear():
    src = [W.Source("S", 2e-12, (0, 1))]
    c = N.integrate([1e-7, 0.0], 1e5, [], sources=src)
    assert np.allclose(c, [1e-7 + 2e-7, 2e-7], rtol=1e-10, atol=0)


def test_autoionisation_relaxes_along_tanh():
    # d c/dt = kb - kf c^2 for [H3O+] = [OH-] = c: c = ceq tanh(sqrt(kb kf) t + atanh(c0/ceq))
    # (coth and acoth above ceq), ceq = sqrt(Kw)
    r9 = [W.Reaction("R9", 0, 1, 11.0, ())]
    src = [W.Source("R9 reverse", W.SOURCES_PH7[0].rate, (0, 1))]
    kf = 110.0
    kb = src[0].rate
    ceq = math.sqrt(kb / kf)
    assert abs(ceq - 1e-7) <= 1e-15
    w = math.sqrt(kb * kf)
    for t in (1e3, 3e4, 1e5, 1e6):
        c = N.integrate([0.0, 0.0], t, r9, sources=src)
        want = ceq * math.tanh(w * t)
        assert abs(c[0] - want) <= 1e-8 * ceq and abs(c[1] - want) <= 1e-8 * ceq, (t, c, want)
        c = N.integrate([3e-7, 3e-7], t, r9, sources=src)
        want = ceq / math.tanh(w * t + math.atanh(ceq / 3e-7))
        assert abs(c[0] - want) <= 1e-8 * ceq, (t, c, want)
    # unequal starts: the ion product settles at Kw
    c = N.integrate([5e-7, 1e-8], 1e8, r9, sources=src)
    assert abs(c[0] * c[1] - W.KW_M2) <= 1e-6 * W.KW_M2


def test_first_order_channel_closed_form():
    # a -> p0 + p1 at k: a = a0 exp(-k t), each product a0 (1 - exp(-k t))
    fo = [W.FirstOrder("A", 0, 3e-3, (1, 2))]
    a0 = 2e-6
    for t in (10.0, 300.0, 3000.0):
        c = N.integrate([a0, 0.0, 0.0], t, [], first_order=fo)
        e = math.exp(-3e-3 * t)
        assert abs(c[0] - a0 * e) <= 1e-9 * a0 and abs(c[1] - a0 * (1 - e)) <= 1e-9 * a0
        assert abs(c[2] - c[1]) <= 1e-12 * a0
    # the Jacobian of the aerated scheme equals finite differences
    rng = np.random.default_rng(6)
    c = 10.0 ** rng.uniform(-8, -5, size=8)
    J = N.jacobian(c, W.REACTIONS_O2, W.FIRST_ORDER_O2)
    for j in range(8):
        h = 1e-6 * c[j]
        dp = c.copy(); dp[j] += h
        dm = c.copy(); dm[j] -= h
        fd = (N.rhs(dp, W.REACTIONS_O2, first_order=W.FIRST_ORDER_O2)
              - N.rhs(dm, W.REACTIONS_O2, first_order=W.FIRST_ORDER_O2)) / (2 * h)
        assert np.allclose(J[:, j], fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
