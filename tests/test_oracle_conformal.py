"""Pins of the conformal calibration oracle (Sec. 4.4): the order-statistic
index in closed form (including a level given as a decimal and the
infinite radius), the split-conformal coverage k / (n + 1) on exchangeable
scores by Monte Carlo, and the nonconformity score of a particle in free
fall, whose quasi-static step is known in closed form."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import conformal


def test_order_index_closed_forms():
    assert conformal.order_index(9, 0.1, 1) == 9            # ceil(10 * 0.9)
    assert conformal.order_index(99, 0.1, 1) == 90          # 100 * 0.9 is 90 in exact arithmetic
    assert conformal.order_index(19, 0.5, 10) == 19         # ceil(20 * 0.95)
    assert conformal.order_index(100, 0.3, 30) == 100       # ceil(101 * 0.99) = ceil(99.99)
    assert conformal.order_index(5, 0.1, 1) == 6            # beyond n: infinite radius
    with pytest.raises(ValueError):
        conformal.order_index(10, 1.0, 1)


def test_radius_is_the_kth_smallest_score():
    s = np.array([0.5, 0.1, 0.9, 0.3, 0.7, 0.2, 0.8, 0.4, 0.6])
    r, k = conformal.radius(s, 0.2, 1)                     # ceil(10 * 0.8) = 8
    assert k == 8 and r == 0.8
    r, k = conformal.radius(s, 0.05, 1)                    # ceil(9.5) = 10 > 9
    assert k == 10 and r == math.inf
    r, k = conformal.radius(np.array([0.3, 0.3, 0.1, 0.3]), 0.4, 1)   # ceil(5 * 0.6) = 3
    assert k == 3 and r == 0.3


def test_split_conformal_coverage():
    """For exchangeable scores the next score falls within the radius with
    probability k / (n + 1) exactly (continuous scores): 1 - delta / T when
    (n + 1)(1 - delta / T) is an integer."""
    rng = np.random.default_rng(7)
    n, delta, T, trials = 19, 0.5, 5, 40000
    k = conformal.order_index(n, delta, T)
    assert k == 18
    hits = 0
    for _ in range(trials):
        s = rng.exponential(size=n + 1)
        r, _ = conformal.radius(s[:n], delta, T)
        hits += s[n] <= r
    p = k / (n + 1)
    assert abs(hits / trials - p) <= 4.0 * math.sqrt(p * (1 - p) / trials)


def test_free_fall_score():
    """One free particle with no obstacle, quasi-static (gamma = 1):
    the step is x + dt^2 g, so the score of an observed next position is its
    distance from that point."""
    dt = 0.01
    inst = W.rope(1, dt=dt, gamma=1.0, T=1, grip_nodes=(), k=0.0, k_bend=0.0, h=0.01, ground=False,
                  s0=np.array([0.1, -0.2, 0.5, 0.0, 0.0, 0.0]))
    q = np.array([[0.1, -0.2, 0.5]])
    qn = q + np.array([[0.003, -0.004, -0.002]])
    s = conformal.scores([inst], [q], [np.zeros(0)], [qn])
    expect = np.linalg.norm(qn - (q + dt * dt * np.array([0.0, 0.0, -9.81])))
    assert abs(s[0] - expect) <= 1e-12


def test_calibration_recipe_scores_are_finite():
    cal = W.calibration_set(6, seed=11)
    insts = [c[0] for c in cal]
    s = conformal.scores(insts, [i.s0[:3 * i.n].reshape(-1, 3) for i in insts], [i.u[0] for i in insts],
                         [c[1] for c in cal])
    assert np.all(np.isfinite(s)) and np.all(s > 0)
