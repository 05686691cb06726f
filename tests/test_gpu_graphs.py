"""K-step blocks captured as HIP graphs give the same state, bit for bit, as the same steps
launched one by one (and the same registry: labels, merge and topological events)."""
import numpy as np
import pytest

from paper_1708_01608_amd import sc
from paper_1708_01608_amd import workloads as W

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _pair(make, steps):
    out = []
    for graphs in (True, False):
        g = make()
        g.step_graphs(graphs)
        g.step(steps)
        out.append(g)
    return out


def _same(a, b, two=False):
    assert np.array_equal(a.get_populations(), b.get_populations())
    if two:
        assert np.array_equal(a.get_gas_populations(), b.get_gas_populations())
    assert np.array_equal(a.last_labels(), b.last_labels())
    assert a.merge_events() == b.merge_events()
    assert a.topo_events() == b.topo_events()
    assert a.t == b.t


@pytest.mark.parametrize("K", [10, 7])
def test_two_bubble_graph_blocks_equal_single_launches(K):
    spec = W.two_bubble(K=K, gap=3)
    _announce(f"graphs two_bubble K={K} 303 steps")

    def make():
        g = sc.Sim.from_spec(spec)
        g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
        return g

    a, b = _pair(make, 303)  # ends mid-block: the tail runs step by step
    _same(a, b)
    assert a.merge_events()  # the gap-3 film fires early, so the registry path is exercised


def test_mixture_and_3d_graph_blocks_equal_single_launches():
    _announce("graphs mixture 64x64 and D3Q19 40x36x20")
    tc = (1.5, 1.0, 1.0, 0.05)

    def mix():
        g = sc.Sim(q=9, nx=64, ny=64, tau=1.0, G=0.0, rho_l=1.0, rho_g=0.05, amp=1e-3, seed=3,
                   K=20, two_component=tc)
        g.seed_nuclei(np.array([(31.5, 31.5, 0.0)]), np.array([10.0]), np.zeros(1), 0.0)
        return g

    a, b = _pair(mix, 200)
    _same(a, b, two=True)

    def box3d():
        g = sc.Sim(q=19, nx=40, ny=36, nz=20, tau=0.9, amp=1e-3, seed=9, K=25)
        g.seed_nuclei(np.array([(10.0, 12.0, 9.0), (27.0, 12.0, 9.0)]), np.array([6.0, 6.0]),
                      np.zeros(2), 0.0)
        return g

    a, b = _pair(box3d, 150)
    _same(a, b)


def test_graph_blocks_are_counted_as_launches_when_profiled():
    spec = W.two_bubble()
    _announce("graphs profiled two_bubble 100 steps")
    g = sc.Sim.from_spec(spec)
    g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    g.profile(True)
    g.step(100)
    ms, launches = g.profile_read(sc.SC_KERNEL_STEP)
    assert launches == 100 and ms > 0
