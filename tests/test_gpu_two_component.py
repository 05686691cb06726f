"""GPU parity of the two-component mode (liquid + gas, Shan-Doolen mixture) against the oracle."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1708_01608_amd import sc
from parity import RHO_TOL, U_TOL

pytestmark = pytest.mark.gpu

TC = (1.5, 1.0, 1.0, 0.05)  # G_cross, tau_vapour, rho_vapour, rho_dissolved

# 16-bit storage of the mixture (FP32 arithmetic), relative to the FP64 oracle: (rho_l and rho_v,
# u, mass drift without the agent).  One shift per component leaves the minority density inside
# and outside the bubbles (about 0.05 of the shift) with the absolute rounding of the majority
MIX16_TOL = {"f16": (0.1, 0.25, 5e-4), "bf16": (0.6, 1.5, 5e-3)}


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _pair(q, shape, centres, radii, budgets, rate, tc=TC, K=50, tau=1.0, amp=1e-3, **gkw):
    nx, ny, nz = shape
    kw = dict(tau=tau, G=0.0, rho_l=1.0, rho_g=0.05, amp=amp, seed=3, K=K)
    o = OracleSim(q, nx, ny, nz, two_component=tc, **kw)
    g = sc.Sim(q=q, nx=nx, ny=ny, nz=nz, two_component=tc, **kw, **gkw)
    for s in (o, g):
        s.seed_nuclei(np.asarray(centres, float), np.asarray(radii, float),
                      np.asarray(budgets, float), rate)
    return o, g


def _errors(g, o):
    rg, ug, _ = g.fields()
    ro, uo, _ = o.fields()
    e_rho = float(np.max(np.abs(rg - ro) / ro))
    e_u = float(np.max(np.abs(ug - uo)) / np.max(np.abs(uo)))
    vg, vo = g.gas_density(), o.gas_density()
    e_v = float(np.max(np.abs(vg - vo) / vo))
    return e_rho, e_u, e_v


def _case(case, **gkw):
    if case == "bubble_2d":
        return _pair(9, (64, 64, 1), [(31.5, 31.5, 0)], [10.0], [0.0], 0.0, **gkw), 100
    return _pair(19, (24, 24, 24), [(11.5, 11.5, 11.5)], [6.0], [0.0], 0.0,
                 tc=(1.5, 0.8, 1.0, 0.05), tau=0.9, **gkw), 50


@pytest.mark.parametrize("case", ["bubble_2d", "sphere_3d"])
def test_two_component_fields_match_oracle(case):
    # without the agent: every stored value is a collision result.  With it, each step adds a
    # small increment to FP32-stored populations, which rounds by ~1/2 ulp of a population
    # (~4e-9) per node and step whatever the increment; that storage effect is covered by the
    # growth test below (labels, sizes, mass), not by a field tolerance
    (o, g), steps = _case(case)
    _announce(f"two components {case} {steps} steps")
    g.step(steps)
    o.step(steps)
    e_rho, e_u, e_v = _errors(g, o)
    print(f"rho_l {e_rho:.3e} u {e_u:.3e} rho_v {e_v:.3e}")
    assert e_rho <= RHO_TOL and e_u <= U_TOL and e_v <= RHO_TOL
    assert np.array_equal(g.last_labels(), o.labels())


@pytest.mark.parametrize("q,shape,tile,variant", [
    (9, (150, 70, 1), (64, 1, 8), 3),      # 3 row tiles (the last 22 wide), 8 + 8 + ... + 6 rows
    (9, (96, 40, 1), (512, 1, 3), 1),      # one tile wider than the box, chunks of 3 rows
    (19, (40, 20, 18), (32, 4, 16), 3),    # 2 x-tiles (the last 8 wide), z chunks 16 + 2
    (19, (36, 18, 20), (64, 8, 7), 1),     # one x-tile wider than the box, y 8 + 8 + 2, z 7 + 7 + 6
    (19, (48, 20, 16), (128, 4, 64), 3),   # one z chunk covering the box
    # one component per wave
    (19, (40, 20, 18), (32, 4, 16), 4),
    (19, (36, 18, 20), (64, 8, 7), 5),
    (19, (70, 22, 9), (64, 4, 4), 5),      # x 64 + 6, y 4 x 5 + 2, z 4 + 4 + 1
    (19, (48, 20, 16), (128, 4, 64), 4),
])
def test_fused_kernel_shapes_match_oracle(q, shape, tile, variant):
    # a central bubble and one across the periodic corner, on tiles with ragged edges
    nx, ny, nz = shape
    R = 7.0 if q == 9 else 4.5
    zc = 0.0 if q == 9 else nz / 2 - 0.5
    centres = [(nx / 2 - 0.5, ny / 2 - 0.5, zc), (1.5, 2.5, 0.0 if q == 9 else 1.5)]
    kw = dict(tau=0.9, G=0.0, rho_l=1.0, rho_g=0.05, amp=1e-3, seed=11, K=20)
    tc = (1.5, 0.8, 1.0, 0.05)
    o = OracleSim(q, nx, ny, nz, two_component=tc, **kw)
    g = sc.Sim(q=q, nx=nx, ny=ny, nz=nz, tile=tile, variant=variant, two_component=tc, **kw)
    assert g.step_config() == (*tile, variant)
    for s in (o, g):
        s.seed_nuclei(np.asarray(centres), np.full(2, R), np.zeros(2), 0.0)
    _announce(f"fused mixture kernel q={q} box={shape} tile={tile} variant={variant}")
    g.step(40)
    o.step(40)
    e_rho, e_u, e_v = _errors(g, o)
    print(f"rho_l {e_rho:.3e} u {e_u:.3e} rho_v {e_v:.3e}")
    assert e_rho <= RHO_TOL and e_u <= U_TOL and e_v <= RHO_TOL
    assert np.array_equal(g.last_labels(), o.labels())


def test_autotune_of_the_mixture_keeps_the_state():
    o, g = _pair(19, (40, 24, 24), [(19.5, 11.5, 11.5)], [6.0], [0.0], 0.0, K=10)
    rho0, _, _ = g.fields()
    v0 = g.gas_density()
    _announce("mixture autotune")
    res = g.autotune(trials=1)
    assert len(res) == 60  # 5 tiles x 3 plane counts x 4 variants
    rho1, _, _ = g.fields()
    assert np.array_equal(rho0, rho1) and np.array_equal(v0, g.gas_density())
    best = min(res, key=lambda e: e["us"])
    assert g.step_config() == (*best["tile"], best["variant"])
    g.step(30)
    o.step(30)
    e_rho, e_u, e_v = _errors(g, o)
    assert e_rho <= RHO_TOL and e_u <= U_TOL and e_v <= RHO_TOL


def test_fed_bubble_grows_on_gpu_as_in_oracle():
    o, g = _pair(9, (64, 64, 1), [(31.5, 31.5, 0)], [10.0], [1e9], 0.05)
    n0 = g.bubbles()[0]["n"]
    g.step(1500)
    o.step(1500)
    bg, bo = g.bubbles(), o.bubbles()
    print("gpu", bg, "\noracle", bo)
    assert len(bg) == len(bo) == 1 and bg[0]["n"] == bo[0]["n"]
    assert bg[0]["n"] > n0 + 40  # the fed bubble grows
    assert np.array_equal(g.last_labels(), o.labels())
    _, _, tg = g.fields()
    _, _, to = o.fields()
    assert abs(tg[0] / to[0] - 1) <= 1e-6  # mixture mass, agent gas included


def test_two_component_pressure_and_laplacian_match_oracle():
    nx, ny = 48, 8
    x = np.tile(np.arange(nx), ny)
    k = 2 * np.pi / nx
    rl = 1.0 + 0.3 * np.cos(k * x)
    rv = 0.5 + 0.2 * np.cos(2 * k * x + 0.3)
    o = OracleSim(9, nx, ny, 1, G=0.0, amp=0.0, K=0, two_component=TC)
    g = sc.Sim(q=9, nx=nx, ny=ny, G=0.0, amp=0.0, K=0, two_component=TC)
    for s in (o, g):
        s.set_equilibrium(rl)
        s.set_gas_equilibrium(rv)
    po, lo = o.laplacian_p()
    pg, lg = g.laplacian_p()
    assert np.max(np.abs(pg - po)) <= 1e-6 * np.max(np.abs(po))
    assert np.max(np.abs(lg - lo)) <= 1e-5 * np.max(np.abs(lo))


def test_two_component_merge_events_match_oracle():
    # two gas bubbles, 3 liquid nodes apart
    o, g = _pair(9, (96, 64, 1), [(31.5, 31.5, 0), (63.5, 31.5, 0)], [14.0, 14.0], [0, 0], 0.0,
                 K=10)
    g.step(600)
    o.step(600)
    from parity import events_key
    from oracle.oracle import OrcEvent, OrcTopoEvent
    ev = (OrcEvent * 8)()
    n = o._lib.orc_events(o._h, ev, 8)
    te = (OrcTopoEvent * 8)()
    nt = o._lib.orc_topo_events(o._h, te, 8)
    crit = [(e.step, e.nucleus_a, e.nucleus_b, e.label_a, e.label_b, e.film_node, e.film_len)
            for e in ev[:n]]
    print("oracle", crit, [(e.step,) for e in te[:nt]], "\ngpu", g.merge_events(), g.topo_events())
    assert events_key(g.merge_events()) == crit
    assert [e["step"] for e in g.topo_events()] == [e.step for e in te[:nt]]


def test_mixture_3d_full_size_conservation():
    # the 256^3 mixture workload at full size in the benchmark's launch configuration: the
    # mixture's mass is initial + spent agent budgets and its momentum is unchanged (both exact in
    # real arithmetic, at any size)
    from paper_1708_01608_amd import workloads as W

    spec = W.mixture_3d()
    _announce("mixture_3d 256^3 40 steps conservation")
    g = sc.Sim.from_spec(spec)
    g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    t0 = g.totals()
    g.step(40)
    t1 = g.totals()
    _, rem = g.nuclei(len(spec.radii))
    spent = float((spec.budgets - rem).sum())
    dm = abs(t1[0] - (t0[0] + spent)) / t0[0]
    dj = float(np.max(np.abs(t1[1:] - t0[1:]))) / t0[0]
    print(f"mixture 256^3: mass {dm:.2e} momentum {dj:.2e} (spent {spent:.3e})")
    assert spent > 0 and dm <= 1e-7 and dj <= 1e-7
    g.close()


@pytest.mark.parametrize("case", ["bubble_2d", "sphere_3d"])
def test_two_component_shifted_fp32_storage_matches_oracle(case):
    # FP32 storage of f - w_i rho_ref (liquid) and f - w_i rho_dissolved (gas), FP64 arithmetic
    (o, g), steps = _case(case, rho_ref=1.0)
    _announce(f"two components {case} {steps} steps, shifted FP32 storage")
    g.step(steps)
    o.step(steps)
    e_rho, e_u, e_v = _errors(g, o)
    print(f"rho_l {e_rho:.3e} u {e_u:.3e} rho_v {e_v:.3e}")
    assert e_rho <= RHO_TOL and e_u <= U_TOL and e_v <= RHO_TOL
    assert np.array_equal(g.last_labels(), o.labels())


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", ["bubble_2d", "sphere_3d"])
def test_two_component_16bit_storage_error(case, storage):
    # 16-bit shifted storage, FP32 arithmetic: every stored value rounds to 11 (FP16) or 8
    # (BF16) significant bits; mass (no agent) is conserved up to that rounding, which does not
    # average out while the painted interface relaxes
    (o, g), steps = _case(case, storage=storage)
    _announce(f"two components {case} {steps} steps, storage {storage}")
    t0 = g.fields()[2][0]
    g.step(steps)
    o.step(steps)
    e_rho, e_u, e_v = _errors(g, o)
    dm = abs(g.fields()[2][0] / t0 - 1)
    print(f"{storage}: rho_l {e_rho:.3e} u {e_u:.3e} rho_v {e_v:.3e} mass drift {dm:.2e}")
    rt, ut, mt = MIX16_TOL[storage]
    assert e_rho <= rt and e_u <= ut and e_v <= rt
    assert dm <= mt


@pytest.mark.parametrize("storage,tile,variant", [
    ("f16", (64, 4, 4), 5), ("bf16", (32, 8, 16), 4), ("f16", (64, 8, 7), 3),
])
def test_two_component_16bit_fused_shapes(storage, tile, variant):
    # ragged tiles of the 16-bit kernels: x 64 + 6, y 4 x 5 + 2 (or 8 x 2 + 6), z chunks
    nx, ny, nz = 70, 22, 9
    centres = [(nx / 2 - 0.5, ny / 2 - 0.5, nz / 2 - 0.5), (1.5, 2.5, 1.5)]
    kw = dict(tau=0.9, G=0.0, rho_l=1.0, rho_g=0.05, amp=1e-3, seed=11, K=20)
    tc = (1.5, 0.8, 1.0, 0.05)
    o = OracleSim(19, nx, ny, nz, two_component=tc, **kw)
    g = sc.Sim(q=19, nx=nx, ny=ny, nz=nz, tile=tile, variant=variant, two_component=tc,
               storage=storage, **kw)
    assert g.step_config() == (*tile, variant)
    for s_ in (o, g):
        s_.seed_nuclei(np.asarray(centres), np.full(2, 4.0), np.zeros(2), 0.0)
    _announce(f"16-bit mixture kernel storage={storage} tile={tile} variant={variant}")
    g.step(40)
    o.step(40)
    e_rho, e_u, e_v = _errors(g, o)
    print(f"{storage}: rho_l {e_rho:.3e} u {e_u:.3e} rho_v {e_v:.3e}")
    rt, ut, _ = MIX16_TOL[storage]
    assert e_rho <= rt and e_u <= ut and e_v <= rt
