"""The blowing-agent source on every storage type (Sec. 3: gas is added to each bubble every step
until the agent is spent).

The mass the populations gain from the source is measured independently of the library's own
ledger: before every step a twin simulation (same parameters, no nuclei, hence no source) takes
the populations of the fed one, both run one step, and the difference of their FP64 totals is
what the source added; the step kernels see identical inputs and write identical outputs.  That
mass must equal what the nuclei released (within 1 %), and the library's ledger (released minus
undelivered) must agree with it.  With FP16/BF16 storage the per-step increments (~1e-7 per
population) lie far below the storage spacing at a gas node (~5e-4 in FP16), so this is the test
that rounding to nearest would fail.  In the mixture the agent's gas must also grow the bubble as
it does in the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1708_01608_amd import sc
from paper_1708_01608_amd import workloads as W

pytestmark = pytest.mark.gpu

STORAGES = [("f32", "f64"), ("f16", "f32"), ("bf16", "f32")]


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _delivered(g, twin, steps, two=False):
    """Mass the source added to g over `steps` steps, from the twin's totals (see above)."""
    got = 0.0
    for _ in range(steps):
        twin.set_populations(g.get_populations())
        if two:
            twin.set_gas_populations(g.get_gas_populations())
        g.step(1)
        twin.step(1)
        got += g.totals()[0] - twin.totals()[0]
    return got


@pytest.mark.parametrize("storage,compute", STORAGES)
def test_source_delivers_the_released_mass(storage, compute):
    # the two-bubble box (bubbles persist: the film ruptures at t ~ 1700); nucleus 1's budget
    # runs out at step 300, so the ledger also covers a bubble that stops being fed
    spec = W.two_bubble()
    spec.budgets = np.array([1.0, 0.03])
    spec.rate = 1e-4
    steps = 600
    _announce(f"source two_bubble storage={storage} compute={compute} {steps} steps")
    g = sc.Sim.from_spec(spec, storage=storage, compute=compute)
    g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    twin = sc.Sim.from_spec(spec, storage=storage, compute=compute)
    twin.seed_nuclei(np.zeros((0, 3)), np.zeros(0), np.zeros(0), 0.0)
    measured = _delivered(g, twin, steps)
    released, undelivered = g.source_ledger()
    print(f"{storage}: released {released:.9f} measured {measured:.9f} "
          f"undelivered {undelivered:.3e} ratio {measured / released:.6f}")
    assert released == pytest.approx(steps * 1e-4 + 0.03, rel=1e-12)
    assert len(g.bubbles()) == 2
    assert abs(measured / released - 1.0) <= 0.01
    # the ledger books exactly what the stored values gained (the twin totals carry the FP64
    # rounding of two ~3e4 sums per step)
    assert abs((released - undelivered) - measured) <= 1e-6
    comp, rem = g.nuclei(2)
    assert rem[1] == 0.0 and rem[0] == pytest.approx(1.0 - steps * 1e-4, rel=1e-12)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_agent_gas_grows_a_mixture_bubble(storage):
    # one bubble of the two-component mixture fed 0.05 gas per step (budget 1e3, small enough
    # that budget - remaining keeps its digits in FP64): it gains about
    # (added mass) / rho_vapour nodes in the oracle; the GPU must gain as much on every storage
    # and book every unit of the agent's gas into the gas component
    nx = ny = 64
    tc = (1.5, 1.0, 1.0, 0.05)
    kw = dict(tau=1.0, G=0.0, rho_l=1.0, rho_g=0.05, amp=1e-3, seed=3, K=50)
    centre, radius, rate, steps = np.array([(31.5, 31.5, 0.0)]), np.array([10.0]), 0.05, 1500
    _announce(f"source mixture 64x64 storage={storage} {steps} steps")
    o = OracleSim(9, nx, ny, 1, two_component=tc, **kw)
    o.seed_nuclei(centre, radius, np.array([1e3]), rate)
    n0 = o.bubbles()[0]["n"]
    o.step(steps)
    grow_o = o.bubbles()[0]["n"] - n0
    compute = "f64" if storage == "f32" else "f32"
    g = sc.Sim(q=9, nx=nx, ny=ny, two_component=tc, storage=storage, compute=compute, **kw)
    g.seed_nuclei(centre, radius, np.array([1e3]), rate)
    twin = sc.Sim(q=9, nx=nx, ny=ny, two_component=tc, storage=storage, compute=compute, **kw)
    twin.seed_nuclei(np.zeros((0, 3)), np.zeros(0), np.zeros(0), 0.0)
    n0g = g.bubbles()[0]["n"]
    measured = _delivered(g, twin, steps, two=True)
    released, undelivered = g.source_ledger()
    grow_g = g.bubbles()[0]["n"] - n0g
    print(f"{storage}: growth gpu {grow_g} oracle {grow_o} (from {n0g} / {n0}); released "
          f"{released:.6f} measured {measured:.6f} undelivered {undelivered:.3e}")
    assert n0g == n0
    assert released == pytest.approx(steps * rate, rel=1e-12)
    assert abs(measured / released - 1.0) <= 0.01
    assert abs((released - undelivered) - measured) <= 1e-6 * released
    assert grow_o >= 50
    assert abs(grow_g - grow_o) <= 0.1 * grow_o
