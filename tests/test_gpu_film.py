"""GPU parity of the film geometry (h, R_d) against the oracle: line counts are integer work and
must be equal; h follows the densities (FP32 storage, FP64 arithmetic)."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1708_01608_amd import sc
from paper_1708_01608_amd import workloads as W
from parity import gpu_from_spec, oracle_from_spec

pytestmark = pytest.mark.gpu

RHO_L, RHO_G = 1.93, 0.16


def _two_balls(shape, ca, cb, R):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = np.full((nz, ny, nx), RHO_L)
    for c in (ca, cb):
        rho[(x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= R * R] = RHO_G
    return rho.reshape(-1)


@pytest.mark.parametrize("q,R,gap", [(9, 10, 2), (9, 14, 3), (19, 6, 2), (19, 7, 3)])
def test_film_geometry_of_synthetic_pairs(q, R, gap):
    if q == 9:
        shape = (4 * R + gap + 20, 2 * R + 14, 1)
        ca = (10 + R, shape[1] // 2, 0)
    else:
        shape = (4 * R + gap + 14, 2 * R + 10, 2 * R + 10)
        ca = (7 + R, shape[1] // 2, shape[2] // 2)
    cb = (ca[0] + 2 * R + gap + 1, ca[1], ca[2])
    rho = _two_balls(shape, ca, cb, R)
    nx, ny, nz = shape
    o = OracleSim(q, nx, ny, nz, tau=1.0, G=-5.0, rho_l=RHO_L, rho_g=RHO_G, amp=0.0, K=10)
    g = sc.Sim(q=q, nx=nx, ny=ny, nz=nz, tau=1.0, G=-5.0, rho_l=RHO_L, rho_g=RHO_G, amp=0.0,
               K=10)
    for s in (o, g):
        s.set_equilibrium(rho)
        s.seed_nuclei(np.array([ca, cb], float), np.array([-1.0, -1.0]), np.zeros(2), 0.0)
    ho, ro, no = o.film_geometry(0, 1)
    hg, rg, ng = g.film_geometry(0, 1)
    print(f"q{q} R{R} gap{gap}: oracle h {ho:.6f} R_d {ro:.3f} n {no}; gpu h {hg:.6f} "
          f"R_d {rg:.3f} n {ng}")
    assert ng == no and rg == ro
    assert abs(hg - ho) <= 1e-5 * max(1.0, abs(ho))


def test_film_geometry_at_the_two_bubble_rupture():
    spec = W.two_bubble()
    o, g = oracle_from_spec(spec), gpu_from_spec(spec)
    for s in (o, g):
        s.step(1700)  # the criterion fires at the test pass of t = 1700
    assert g.merge_events() and g.merge_events()[0]["step"] == 1700
    ho, ro, no = o.film_geometry(0, 1)
    hg, rg, ng = g.film_geometry(0, 1)
    print(f"rupture: oracle h {ho:.6f} R_d {ro} n {no}; gpu h {hg:.6f} R_d {rg} n {ng}")
    assert ng == no and abs(hg - ho) <= 1e-4 * ho


def test_film_geometry_rejects_one_bubble():
    g = sc.Sim(q=9, nx=32, ny=32, K=10, amp=0.0)
    g.seed_nuclei(np.array([(10.0, 16.0, 0.0), (12.0, 16.0, 0.0)]), np.array([4.0, 4.0]),
                  np.zeros(2), 0.0)
    with pytest.raises(sc.ScError):
        g.film_geometry(0, 1)


def test_fig3_sweep_point_matches_oracle():
    # one point of the size sweep (R_b = 12, gap 4, 84 x 56 box): firing step and geometry
    from paper_1708_01608_amd import fig3

    row = fig3.run([12], 4, 3000)[0]
    assert row["fired"]
    spec = W.two_bubble(nx=84, ny=56, radius=12.0, gap=4)
    o = oracle_from_spec(spec)
    o.step(row["step"])
    from oracle.oracle import OrcEvent
    ev = (OrcEvent * 4)()
    n = o._lib.orc_events(o._h, ev, 4)
    assert n == 1 and ev[0].step == row["step"]
    h, rd, nl = o.film_geometry(0, 1)
    print(f"sweep R_b 12: gpu {row}; oracle h {h:.6f} R_d {rd} n {nl}")
    assert nl == row["n_lines"] and abs(h - row["h_c"]) <= 1e-4 * h


@pytest.mark.parametrize("R,gap", [(8, 3), (12, 3)])
def test_fig3_sweep_point_3d_matches_oracle(R, gap):
    # the sweep's 3D form (two spheres, D3Q19): firing step, film node and geometry
    from paper_1708_01608_amd import fig3

    print(f"[gpu] 3D sweep point R_b {R} gap {gap}", flush=True)
    row = fig3.run([R], gap, 400, lattice=19)[0]
    assert row["fired"]
    nx, ny, _ = row["box"]
    spec = W.two_bubble_3d(nx=nx, ny=ny, nz=ny, radius=float(R), gap=gap)
    o = oracle_from_spec(spec)
    while o.t < row["step"]:
        o.step(spec.K)
        assert not o.events() or o.t == row["step"]
    ev = o.events()
    assert len(ev) == 1 and ev[0]["step"] == row["step"]
    assert ev[0]["film_len"] == row["film_len"]
    assert ev[0]["lap_p"] == pytest.approx(row["lap_p"], rel=1e-3)
    h, rd, nl = o.film_geometry(0, 1)
    print(f"3D sweep R_b {R}: gpu {row}; oracle h {h:.6f} R_d {rd} n {nl}")
    assert nl == row["n_lines"] and abs(h - row["h_c"]) <= 1e-4 * h
