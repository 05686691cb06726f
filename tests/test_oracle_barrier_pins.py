"""Pins of the oracle's modified Shan-Chen barrier (Sec. 3.1, Fig. 1 steps 3-6).

Each bubble keeps its own lattice and meets the others only through the liquid until the
criterion flips eta_m.  On one lattice: an owner id per node (a bubble's gas plus a corona of
liquid layers), and in the force a neighbour held by a different, un-merged bubble is seen as
bulk liquid, psi(rho_l).  The pins below tie that to facts that do not depend on the oracle's own
barrier code: the geometry of lattice-neighbour balls, the plain (already pinned) force on a
substituted density field, and exact equality with the plain model wherever the barrier cannot
act.
"""
import numpy as np
import pytest

from oracle import OracleSim, lattice
from paper_1708_01608_amd import workloads as W


def _sim(q, shape, barrier, corona=3, amp=0.0, K=10, rho_l=1.93, rho_g=0.16, tau=1.0, seed=1):
    nx, ny, nz = shape
    return OracleSim(q, nx, ny, nz, tau=tau, G=-5.0, rho_l=rho_l, rho_g=rho_g, amp=amp,
                     seed=seed, K=K, barrier=barrier, corona=corona)


def _seed(o, centres, radii):
    n = len(radii)
    o.seed_nuclei(np.asarray(centres, dtype=float), np.asarray(radii, dtype=float), np.zeros(n),
                  0.0)


def _offsets(q, shape, origin):
    """Minimal-image integer offsets of every node from `origin` (x fastest)."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = []
    for c, o, n in ((x, origin[0], nx), (y, origin[1], ny), (z, origin[2], nz)):
        v = (c - o + n // 2) % n - n // 2
        d.append(v.reshape(-1))
    return np.stack(d, axis=1)


@pytest.mark.parametrize("q,shape", [(9, (17, 15, 1)), (19, (13, 12, 11))])
@pytest.mark.parametrize("corona", [0, 1, 2, 3])
def test_corona_of_a_one_node_bubble_is_the_lattice_ball(q, shape, corona):
    # r layers of lattice-neighbour growth from one node reach exactly the nodes within r steps:
    # D2Q9 steps are the 8 king moves -> max-norm <= r; D3Q19 steps have max-norm 1 and L1 <= 2
    # -> max-norm <= r and L1 <= 2r.
    c = (6, 7, 5 if q == 19 else 0)
    o = _sim(q, shape, True, corona)
    _seed(o, [c], [0.0])
    own = o.owner()
    d = np.abs(_offsets(q, shape, c))
    inside = d.max(axis=1) <= corona
    if q == 19:
        inside &= d.sum(axis=1) <= 2 * corona
    assert set(np.unique(own)) <= {0, 1}
    assert np.array_equal(own == 1, inside)


def test_corona_ties_go_to_the_smaller_id():
    # one-node bubbles 6 apart on a row: the middle node is 3 steps from both
    o = _sim(9, (24, 9, 1), True, 3)
    _seed(o, [(5, 4, 0), (11, 4, 0)], [0.0, 0.0])
    row = o.owner().reshape(9, 24)[4]
    # x = 2..8 within 3 of x = 5 (x = 8 also of x = 11: the tie goes to id 1), x = 9..14 to id 2
    assert list(row[1:16]) == [0] + [1] * 7 + [2] * 6 + [0]


def test_barrier_off_by_default_and_owner_empty():
    o = _sim(9, (16, 16, 1), False)
    _seed(o, [(8, 8, 0)], [3.0])
    assert not np.any(o.owner())


@pytest.mark.parametrize("q,shape,centres,R,steps", [
    (9, (64, 32, 1), [(14.5, 15.5, 0), (46.5, 15.5, 0)], 5.0, 60),
    (19, (44, 24, 24), [(10.5, 11.5, 11.5), (32.5, 11.5, 11.5)], 7.0, 50),
])
def test_barrier_is_invisible_while_bubbles_are_apart(q, shape, centres, R, steps):
    # coronas more than one node apart: no node held by one bubble has a neighbour held by the
    # other, so the barrier never substitutes and the run equals the plain model bit for bit
    # (small spheres shrink fast in this liquid, hence R = 7 and 50 steps in 3D)
    runs = []
    for bar in (False, True):
        o = _sim(q, shape, bar, 3, amp=1e-3, tau=0.9)
        _seed(o, centres, [R, R])
        o.step(steps)
        runs.append(o.get_f())
        if bar:
            own = o.owner()
            assert set(np.unique(own)) == {0, 1, 2}
    assert np.array_equal(runs[0], runs[1])


def test_barrier_is_invisible_inside_one_component():
    # overlapping paints: both nuclei sit in one gas component from the start, which gets one
    # owner id, so again nothing is substituted
    runs = []
    for bar in (False, True):
        o = _sim(9, (48, 32, 1), bar, 3, amp=1e-3)
        _seed(o, [(20.5, 15.5, 0), (27.5, 15.5, 0)], [6.0, 6.0])
        o.step(40)
        runs.append(o.get_f())
        if bar:
            assert set(np.unique(o.owner())) == {0, 1}
    assert np.array_equal(runs[0], runs[1])


@pytest.mark.parametrize("q,shape,centres", [
    (9, (30, 14, 1), [(7.5, 6.5, 0), (19.5, 6.5, 0)]),
    (19, (18, 10, 8), [(4.5, 4.5, 3.5), (12.5, 4.5, 3.5)]),
])
def test_barrier_force_is_the_plain_force_of_the_substituted_field(q, shape, centres):
    # F_barrier(x) must equal the plain Shan-Chen force at x computed on the density field in
    # which every node held by another bubble (both owners nonzero and different) is replaced by
    # rho_l.  The plain force is pinned elsewhere (zero net force, coexistence, Laplace law).
    nx, ny, nz = shape
    N = nx * ny * nz
    o = _sim(q, shape, True, 3, amp=1e-3)
    _seed(o, centres, [3.0, 3.0])
    o.step(7)  # smooth profiles; no test pass yet (K = 10), owners from the seed pass
    own = o.owner()
    assert set(np.unique(own)) == {0, 1, 2}
    rho, _, _ = o.fields()
    F = o.force()
    plain = _sim(q, shape, False)
    e, _ = lattice(q)
    touched = 0
    for x in range(N):
        if own[x] == 0:
            continue
        sub = rho.copy()
        other = (own != 0) & (own != own[x])
        if not other.any():
            continue
        sub[other] = 1.93
        plain.set_equilibrium(sub)
        Fp = plain.force()[:, x]
        # the plain force at x on the unsubstituted densities: the barrier must matter somewhere
        plain.set_equilibrium(rho)
        F0 = plain.force()[:, x]
        scale = max(np.abs(F).max(), 1e-12)
        assert np.max(np.abs(F[:, x] - Fp)) <= 1e-12 * scale, x
        if np.max(np.abs(Fp - F0)) > 1e-9 * scale:
            touched += 1
    assert touched > 0  # the film nodes do feel the barrier


def test_criterion_merge_unifies_the_owners():
    # gap 3: the criterion fires at the first pass (t = 10); from then on both bubbles carry
    # owner id 1 and the film is plain Shan-Chen again
    spec = W.two_bubble(gap=3)
    o = OracleSim(spec.q, spec.nx, spec.ny, spec.nz, spec.tau, spec.G, spec.rho_l, spec.rho_g,
                  spec.amp, spec.seed, spec.theta, spec.K, spec.film_max, barrier=True, corona=3)
    o.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    assert set(np.unique(o.owner())) == {0, 1, 2}
    o.step(10)
    assert set(np.unique(o.owner())) == {0, 1}


def test_barrier_holds_a_four_node_film():
    # without the barrier the gap-4 film of the two-bubble box ruptures (criterion at t = 1700,
    # shared component at t = 1790); with it, the film neither fires nor ruptures by t = 1000
    spec = W.two_bubble()
    o = OracleSim(spec.q, spec.nx, spec.ny, spec.nz, spec.tau, spec.G, spec.rho_l, spec.rho_g,
                  spec.amp, spec.seed, spec.theta, spec.K, spec.film_max, barrier=True, corona=3)
    o.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    o.step(1000)
    from oracle.oracle import OrcEvent, OrcTopoEvent
    assert o._lib.orc_events(o._h, (OrcEvent * 4)(), 4) == 0
    assert o._lib.orc_topo_events(o._h, (OrcTopoEvent * 4)(), 4) == 0
