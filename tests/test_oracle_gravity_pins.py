"""Pins of the oracle's gravity (drainage) body force.

The paper's runs leave gravity out (Sec. 4) and name drainage as a stage of foaming (Sec. 3).
The body force is (rho - rho0) g, added to the Shan-Chen force: buoyancy relative to the
reference density rho0, by default the mean density of the seeded box (no net force on a periodic
box).  With the velocity-shift forcing a step moves every node's momentum by exactly its force,
which gives closed forms for a uniform box.
"""
import numpy as np
import pytest

from oracle import OracleSim
from oracle.oracle import OrcBubble


def _centroids(o):
    b = (OrcBubble * 8)()
    n = o._lib.orc_bubbles(o._h, b, 8)
    return [tuple(b[i].centroid) for i in range(n)]


@pytest.mark.parametrize("q,shape,tau", [(9, (16, 12, 1), 0.8), (19, (8, 6, 5), 1.3)])
def test_body_force_moves_momentum_by_its_closed_form(q, shape, tau):
    # G = 0, uniform rho: every node stays identical and gains (rho - rho0) g per step, so
    # J(t) = J(0) + t N (rho - rho0) g exactly in real arithmetic.
    nx, ny, nz = shape
    N = nx * ny * nz
    g = (2e-5, -1e-5, 3e-5)[: 2 if q == 9 else 3]
    o = OracleSim(q, nx, ny, nz, tau=tau, G=0.0, rho_l=1.3, rho_g=0.2, amp=0.0, K=0,
                  gravity=g, rho0=1.0)
    J0 = o.totals()[1:1 + len(g)]
    o.step(50)
    J = o.totals()[1:1 + len(g)]
    expect = J0 + 50 * N * (1.3 - 1.0) * np.asarray(g)
    assert np.allclose(J, expect, rtol=1e-11, atol=1e-15)


def test_uniform_box_at_the_reference_density_is_a_fixed_point():
    # rho0 = the node density itself (sum of f_eq(1.93), which is 1.93 up to rounding)
    o = OracleSim(9, 20, 16, 1, tau=0.9, G=-5.0, rho_l=1.93, amp=0.0, K=0)
    rho, _, _ = o.fields()
    assert np.all(rho == rho[0])
    o.set_gravity((1e-4, -2e-4), float(rho[0]))
    f0 = o.get_f()
    o.step(25)
    # as for the plain uniform state, only the rounding of sum f_eq remains (a force rho g
    # instead of (rho - rho0) g would move f by ~1e-5 per step)
    assert np.abs(o.get_f() - f0).max() <= 1e-14


def test_mean_density_reference_conserves_momentum():
    # rho0 = M/N: the body forces sum to zero, the Shan-Chen forces too, so J stays at J(0)
    o = OracleSim(9, 64, 48, 1, tau=1.0, G=-5.0, rho_l=1.93, rho_g=0.16, amp=1e-3, K=20,
                  gravity=(0.0, -5e-5))
    o.seed_nuclei(np.array([(20.5, 23.5, 0), (44.5, 23.5, 0)]), np.array([10.0, 8.0]),
                  np.zeros(2), 0.0)
    rho, _, tot0 = o.fields()
    assert abs(o.rho0 - rho.mean()) <= 1e-14 * rho.mean()
    o.step(200)
    tot = o.totals()
    assert np.max(np.abs(tot[1:3] - tot0[1:3])) <= 1e-12 * tot0[0]


@pytest.mark.parametrize("axis,sign", [(1, -1), (0, +1)])
def test_bubble_rises_against_gravity_at_a_rate_linear_in_g(axis, sign):
    # a radius-16 bubble in liquid: it drifts opposite to g, and in this slow (viscous) regime
    # the drift over a fixed time scales with |g| (factor 3 in g -> factor ~3 in drift)
    drift = []
    for mag in (1e-5, 3e-5):
        g = [0.0, 0.0]
        g[axis] = sign * mag
        o = OracleSim(9, 96, 96, 1, tau=1.0, G=-5.0, rho_l=1.93, rho_g=0.16, amp=0.0, K=100,
                      gravity=g)
        o.seed_nuclei(np.array([(47.5, 47.5, 0)]), np.array([16.0]), np.zeros(1), 0.0)
        c0 = _centroids(o)[0]
        o.step(1500)
        c1 = _centroids(o)[0]
        d = np.subtract(c1, c0)
        assert abs(d[1 - axis]) < 1e-9  # no drift across g (mirror symmetry)
        drift.append(-sign * d[axis])
    assert drift[0] > 0.2 and drift[1] > 0.2
    assert 2.5 < drift[1] / drift[0] < 3.5


def test_gravity_rejects_non_finite_input():
    o = OracleSim(9, 8, 8, 1)
    with pytest.raises(ValueError):
        o.set_gravity((float("nan"), 0.0))
