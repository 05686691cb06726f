"""GPU parity at the edges of the input space: the smallest boxes the library accepts, boxes one
node-row thin against the tile, runs without any nucleus, and the method's degenerate cases (no
interaction, a nucleus on no node, a nucleus filling the box, two nuclei at one centre)."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1708_01608_amd import sc
from paper_1708_01608_amd import workloads as W
from parity import RHO_TOL, TOL, U_TOL, events_key, field_errors, gpu_from_spec, oracle_from_spec

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _spec(q, shape, centres, radii, K=10):
    nx, ny, nz = shape
    n = len(radii)
    return W.SimSpec(name="edge", q=q, nx=nx, ny=ny, nz=nz, tau=0.9, G=-5.0, amp=1e-3, seed=5,
                     K=K, centres=np.asarray(centres, float).reshape(n, 3),
                     radii=np.asarray(radii, float), budgets=np.full(n, 1e-2), rate=1e-4)


# Near rest the velocity error is measured against max |u| plus an absolute floor: FP32 storage
# rounds each population by up to half an ulp (~3e-8 for f_i ~ 0.5), which moves u = j / rho by
# about 1e-8 per node whatever the flow, so a box whose noise has decayed to |u| ~ 1e-9 cannot
# be held to a relative bound.  The floor is ten times that shift.  FP32 arithmetic rounds the
# equilibria themselves (~6e-8 of w_i rho per step), measured 1.05e-7 on the 48x40x36 box at
# rest after 100 steps: its floor is ten times that.
U_FLOOR = 1e-7
U_FLOOR32 = 1e-6


def _compare(spec, steps, **kw):
    g, o = gpu_from_spec(spec, **kw), oracle_from_spec(spec)
    g.step(steps)
    o.step(steps)
    e_rho, _, tg, to = field_errors(g, o)
    ug, uo = g.fields()[1].astype(np.float64), o.fields()[1]
    du, umax = float(np.max(np.abs(ug - uo))), float(np.max(np.abs(uo)))
    print(f"rho {e_rho:.3e} |du| {du:.3e} max|u| {umax:.3e} mass {tg[0] / to[0] - 1:.2e}")
    return g, o, e_rho, (du, umax), tg, to


def _u_ok(u, tol, floor=U_FLOOR):
    du, umax = u
    return du <= tol * umax + floor


def _mass_ok(spec, steps, tg, to):
    # the agent's increments are added to FP32-stored populations (all below 1), each add
    # rounding by at most half an ulp, 2^-25: in a box of a few nodes that bound, not the 1e-7 of
    # the larger parity boxes, is what the mass can differ by
    n_adds = steps * spec.nx * spec.ny * spec.nz * spec.q if len(spec.radii) else 0
    return abs(tg[0] / to[0] - 1) <= max(1e-7, n_adds * 2.0 ** -25 / to[0])


# the smallest boxes (4 nodes per axis): the tile is far wider than the box, every ring node is
# a periodic image of an owned node; with no nucleus, and with one nucleus across the corner
@pytest.mark.parametrize("q,shape", [(9, (4, 4, 1)), (19, (4, 4, 4))])
@pytest.mark.parametrize("nuclei", [0, 1])
def test_smallest_boxes_match_oracle(q, shape, nuclei):
    centres, radii = ([(0.0, 0.0, 0.0)], [1.5]) if nuclei else (np.zeros((0, 3)), [])
    spec = _spec(q, shape, centres, radii)
    _announce(f"smallest box q={q} {shape} nuclei={nuclei}")
    g, o, e_rho, e_u, tg, to = _compare(spec, 40)
    assert e_rho <= RHO_TOL and _u_ok(e_u, U_TOL)
    assert _mass_ok(spec, 40, tg, to)
    assert np.array_equal(g.last_labels(), o.labels())
    assert events_key(g.merge_events()) == events_key(o.events())


# thin boxes: one row of tiles in y (ny = 4 = TY) and a ragged second x tile, in both lattices
@pytest.mark.parametrize("q,shape,tile", [
    (9, (300, 4, 1), (256, 1, 64)),
    (19, (300, 4, 4), (256, 4, 64)),
    (19, (4, 300, 6), (32, 8, 4)),
])
def test_thin_boxes_match_oracle(q, shape, tile):
    nx, ny, nz = shape
    c = [(nx / 3, ny / 2 - 0.5, (nz / 2 - 0.5) if q == 19 else 0.0)]
    spec = _spec(q, shape, c, [1.8])
    _announce(f"thin box q={q} {shape} tile={tile}")
    g, o, e_rho, e_u, tg, to = _compare(spec, 40, tile=tile)
    assert e_rho <= RHO_TOL and _u_ok(e_u, U_TOL)
    assert _mass_ok(spec, 40, tg, to)
    assert np.array_equal(g.last_labels(), o.labels())


@pytest.mark.parametrize("storage,compute", [("f32", "f64"), ("f32", "f32"), ("f16", "f32"),
                                             ("bf16", "f32")])
def test_no_nuclei_is_liquid_only(storage, compute):
    # without nuclei the box stays liquid: no gas label, no event, the fields follow the oracle
    spec = _spec(19, (48, 40, 36), np.zeros((0, 3)), [], K=25)
    _announce(f"no nuclei 48x40x36 storage={storage} compute={compute}")
    g, o, e_rho, e_u, tg, to = _compare(spec, 100, storage=storage, compute=compute)
    # FP32 storage with FP64 arithmetic is gated at 1e-5; the other combinations are reported,
    # not gated (their bounds only reject blown-up fields)
    rt, ut = TOL[(storage, compute)]
    tag = "gated" if (storage, compute) == ("f32", "f64") else "reported, not gated"
    print(f"[{tag}] no nuclei storage {storage} compute {compute}: rho {e_rho:.3e} u {e_u}")
    assert e_rho <= rt and _u_ok(e_u, ut, U_FLOOR if compute == "f64" else U_FLOOR32)
    assert not np.any(g.last_labels()) and not np.any(o.labels())
    assert g.bubbles() == [] and g.merge_events() == [] and o.events() == []


def test_mixture_smallest_box_matches_oracle():
    tc = (1.5, 0.8, 1.0, 0.05)
    kw = dict(tau=0.9, G=0.0, rho_l=1.0, rho_g=0.05, amp=1e-3, seed=7, K=10)
    o = OracleSim(19, 4, 4, 4, two_component=tc, **kw)
    g = sc.Sim(q=19, nx=4, ny=4, nz=4, two_component=tc, **kw)
    for s_ in (o, g):
        s_.seed_nuclei(np.zeros((1, 3)), np.array([1.5]), np.zeros(1), 0.0)
    _announce("mixture smallest box 4x4x4")
    g.step(40)
    o.step(40)
    rg, ug, _ = g.fields()
    ro, uo, _ = o.fields()
    e_rho = float(np.max(np.abs(rg - ro) / ro))
    e_v = float(np.max(np.abs(g.gas_density() - o.gas_density()) / o.gas_density()))
    du, umax = float(np.max(np.abs(ug - uo))), float(np.max(np.abs(uo)))
    print(f"rho_l {e_rho:.3e} |du| {du:.3e} max|u| {umax:.3e} rho_v {e_v:.3e}")
    assert e_rho <= RHO_TOL and _u_ok((du, umax), U_TOL) and e_v <= RHO_TOL
    assert np.array_equal(g.last_labels(), o.labels())


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_bandwidth_probes_report_rates(storage):
    # the ceilings the bench line quotes: positive rates, the pattern probe on a ragged box
    # (tiles overhang the box in x and y, planes in z)
    copy_gbs, read_gbs = sc.hbm_probe(1 << 26, 2)
    assert copy_gbs > 0 and read_gbs > 0
    flat, march = sc.pattern_probe(70, 40, 30, storage, (32, 8, 7), 2)
    assert np.isfinite(flat) and np.isfinite(march) and flat > 0 and march > 0


# ---- degenerate cases of the method ------------------------------------------------------------
def _degenerate(q, shape, centres, radii, G=-5.0, amp=1e-3):
    nx, ny, nz = shape
    n = len(radii)
    return W.SimSpec(name="degenerate", q=q, nx=nx, ny=ny, nz=nz, tau=0.9, G=G, amp=amp, seed=7,
                     K=10, centres=np.asarray(centres, float).reshape(n, 3),
                     radii=np.asarray(radii, float), budgets=np.full(n, 1e-2), rate=1e-4)


def _check_degenerate(spec, steps=40):
    g, o, e_rho, e_u, tg, to = _compare(spec, steps)
    assert e_rho <= RHO_TOL and _u_ok(e_u, U_TOL)
    assert _mass_ok(spec, steps, tg, to)
    assert np.array_equal(g.last_labels(), o.labels())
    n = len(spec.radii)
    if n:
        cg, rg = g.nuclei(n)
        co, ro = o.nuclei()
        assert np.array_equal(cg, co)
        np.testing.assert_array_equal(rg, ro)  # FP64 budgets, same order
    assert events_key(g.merge_events()) == events_key(o.events())
    return g, o


_DEG_BOXES = [(9, (40, 30, 1)), (19, (20, 16, 12))]


@pytest.mark.parametrize("q,shape", _DEG_BOXES)
def test_no_interaction(q, shape):
    # G = 0: the Shan-Chen force vanishes and the step is plain BGK; a gas nucleus then simply
    # diffuses into the liquid
    c = [(shape[0] / 2, shape[1] / 2, shape[2] / 2 if q == 19 else 0.0)]
    spec = _degenerate(q, shape, c, [4.0], G=0.0)
    _announce(f"degenerate: G = 0, q={q} {shape}")
    _check_degenerate(spec)


@pytest.mark.parametrize("q,shape", _DEG_BOXES)
def test_nucleus_covering_no_node(q, shape):
    # a nucleus smaller than the distance to the nearest node paints nothing: it belongs to no
    # gas component, so nothing is released for it and its budget stays whole
    c = [(10.5, 10.5, 6.5 if q == 19 else 0.0), (3.0, 4.0, 2.0 if q == 19 else 0.0)]
    spec = _degenerate(q, shape, c, [0.3, 2.5])
    _announce(f"degenerate: nucleus on no node, q={q} {shape}")
    g, o = _check_degenerate(spec)
    assert g.nuclei(2)[0][0] == 0 and g.nuclei(2)[1][0] == spec.budgets[0]


@pytest.mark.parametrize("q,shape", _DEG_BOXES)
def test_nucleus_filling_the_box(q, shape):
    # a nucleus larger than the box: every node is gas, one component across every periodic
    # seam, and the agent feeds the whole box
    c = [(1.0, 2.0, 3.0 if q == 19 else 0.0)]
    spec = _degenerate(q, shape, c, [1000.0])
    _announce(f"degenerate: nucleus filling the box, q={q} {shape}")
    g, o = _check_degenerate(spec)
    assert len(np.unique(g.last_labels())) == 1 and g.last_labels()[0] == 1


@pytest.mark.parametrize("q,shape,radius", [(9, (40, 30, 1), 5.0), (19, (24, 20, 20), 6.0)])
def test_two_nuclei_at_one_centre(q, shape, radius):
    # two nuclei painted over each other: one bubble that holds both, whose release pools the
    # two budgets (the 3D bubble is larger, so that it outlives the run)
    c = [(12.0, 9.0, 10.0 if q == 19 else 0.0)] * 2
    spec = _degenerate(q, shape, c, [radius, 3.0])
    _announce(f"degenerate: two nuclei at one centre, q={q} {shape}")
    g, o = _check_degenerate(spec)
    comp, _ = g.nuclei(2)
    assert comp[0] == comp[1] != 0
