"""Pins of the oracle's two-component mode (a liquid and a gas component, Shan-Doolen mixture).

The paper grows bubbles by adding the blowing agent's gas (Sec. 3) and runs "two separate
simulations simultaneously for a two-phase model" (Sec. 3.1).  In one-component Shan-Chen added
mass shrinks bubbles; with a separate gas component it grows them.  Pins: conservation laws of
the mixture (per-component mass, total momentum), the uniform fixed point, the criterion's EOS
p = (rho_l + rho_v)/3 + (Gx/3) rho_l rho_v against the force the dynamics apply (the force is
minus the gradient of its nonideal part at long wavelength), and the volume a fed bubble gains.
"""
import numpy as np
import pytest

from oracle import OracleSim
from oracle.oracle import OrcBubble

TC = (1.5, 1.0, 1.0, 0.05)  # Gx, tau_v, rho_vapour, rho_dissolved


def _sim(q, shape, rho_l=1.0, rho_g=0.05, amp=1e-3, K=50, tc=TC, tau=1.0):
    nx, ny, nz = shape
    return OracleSim(q, nx, ny, nz, tau=tau, G=0.0, rho_l=rho_l, rho_g=rho_g, amp=amp, K=K,
                     two_component=tc)


def _bubbles(o):
    b = (OrcBubble * 8)()
    n = o._lib.orc_bubbles(o._h, b, 8)
    return [b[i] for i in range(n)]


def _slab(o, x0, x1, ny, nz=1):
    # paint a gas slab x0 <= x < x1 with radius-0 nuclei on every node
    cen = np.array([(x, y, z) for x in range(x0, x1) for y in range(ny) for z in range(nz)],
                   dtype=float)
    o.seed_nuclei(cen, np.zeros(len(cen)), np.zeros(len(cen)), 0.0)


@pytest.mark.parametrize("q,shape", [(9, (48, 40, 1)), (19, (20, 18, 16))])
def test_component_masses_and_total_momentum_are_conserved(q, shape):
    o = _sim(q, shape, tc=(1.5, 0.8, 1.0, 0.05))
    c = np.array(shape, dtype=float) / 2 - 0.5
    o.seed_nuclei(np.array([c]), np.array([6.0]), np.zeros(1), 0.0)
    rho0, _, t0 = o.fields()
    gas0 = o.gas_density().sum()
    o.step(150)
    rho1, _, t1 = o.fields()
    assert abs(rho1.sum() - rho0.sum()) <= 1e-12 * rho0.sum()
    assert abs(o.gas_density().sum() - gas0) <= 1e-12 * gas0
    assert np.max(np.abs(t1[1:] - t0[1:])) <= 1e-12 * t0[0]


def test_uniform_mixture_is_a_fixed_point():
    o = _sim(9, (12, 10, 1), rho_l=0.7, amp=0.0, tc=(1.5, 0.9, 1.0, 0.3))
    f0 = o.get_f()
    rv0 = o.gas_density()
    o.step(20)
    assert np.abs(o.get_f() - f0).max() <= 1e-15
    assert np.abs(o.gas_density() - rv0).max() <= 1e-14


@pytest.mark.parametrize("G", [1.5, 0.8])
def test_force_is_minus_the_gradient_of_the_eos_nonideal_part(G):
    # long-wavelength fields rho_a = a + eps_a cos(kx): the total interaction force is
    # -d/dx of the EOS's nonideal part (Gx/3) rho_l rho_v up to O(k^2), which pins the EOS the
    # criterion evaluates (from orc_laplacian_p) to the force the dynamics apply; a
    # coefficient Gx/6 would be off by a factor of 2
    nx, ny = 256, 4
    o = _sim(9, (nx, ny, 1), amp=0.0, K=0, tc=(G, 1.0, 1.0, 0.05))
    x = np.tile(np.arange(nx), ny)
    k = 2 * np.pi / nx
    rl = 1.0 + 0.01 * np.cos(k * x)
    rv = 0.5 + 0.02 * np.cos(k * x + 0.3)
    o.set_equilibrium(rl)
    o.set_gas_equilibrium(rv)
    p, _ = o.laplacian_p()
    nonideal = (p - (rl + rv) / 3.0).reshape(ny, nx)[0]
    grad = (np.roll(nonideal, -1) - np.roll(nonideal, 1)) / 2.0
    Fx = o.force()[0].reshape(ny, nx)[0]
    scale = np.abs(grad).max()
    assert np.max(np.abs(Fx + grad)) <= 1e-2 * scale


def test_fed_gas_grows_the_bubble():
    # the agent's gas goes to the gas component: a fed bubble gains about (added mass) /
    # (its gas density) nodes, an unfed one keeps its size (one-component SC shrinks it)
    areas = {}
    for rate in (0.0, 0.05):
        o = _sim(9, (64, 64, 1))
        o.seed_nuclei(np.array([(31.5, 31.5, 0.0)]), np.array([10.0]), np.array([1e9]), rate)
        n0 = _bubbles(o)[0].n
        rl0 = o.fields()[0].sum()
        gas0 = o.gas_density().sum()
        o.step(3000)
        b = _bubbles(o)
        assert len(b) == 1
        areas[rate] = (n0, b[0].n)
        # mass bookkeeping: all of it in the gas component, the liquid untouched
        assert abs(o.gas_density().sum() - gas0 - rate * 3000) <= 1e-9 * (gas0 + 1)
        assert abs(o.fields()[0].sum() - rl0) <= 1e-10 * rl0
    n0, n1 = areas[0.0]
    assert abs(n1 - n0) <= 0.1 * n0
    n0, n1 = areas[0.05]
    rv_in = 1.0
    assert 0.75 * 150 / rv_in <= n1 - n0 <= 1.25 * 150 / rv_in


def test_two_component_parameters_are_checked():
    with pytest.raises(ValueError):
        _sim(9, (8, 8, 1), tc=(1.5, 0.5, 1.0, 0.05))   # tau_v must exceed 1/2
    with pytest.raises(ValueError):
        _sim(9, (8, 8, 1), tc=(1.5, 1.0, 0.0, 0.05))   # densities must be positive
