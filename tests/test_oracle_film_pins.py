"""Pins of the oracle's film geometry (the film as a disc of radius R_d and thickness h between
two interfaces, Sec. 3; the h_c / R_d / R_b trends of Fig. 3).

h is pinned by hand-made density profiles whose rho = theta crossings follow from linear
interpolation; the line count behind R_d by a brute-force scan of the same label field written
independently in numpy (axis-aligned pairs, where the shifted lines are rows or x-lines).
"""
import numpy as np
import pytest

from oracle import OracleSim

RHO_L, RHO_G = 1.93, 0.16
THETA = 0.5 * (RHO_L + RHO_G)


def _box(q, shape, rho):
    nx, ny, nz = shape
    o = OracleSim(q, nx, ny, nz, tau=1.0, G=-5.0, rho_l=RHO_L, rho_g=RHO_G, amp=0.0, K=10)
    o.set_equilibrium(np.ascontiguousarray(rho.reshape(-1)))
    return o


def _two_balls(shape, ca, cb, R):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = np.full((nz, ny, nx), RHO_L)
    for c in (ca, cb):
        rho[(x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= R * R] = RHO_G
    return rho


def _seed_labels(o, ca, cb):
    # nuclei with negative radius: registered at the centres, nothing painted; the seed pass
    # labels the field as set
    o.seed_nuclei(np.array([ca, cb], dtype=float), np.array([-1.0, -1.0]), np.zeros(2), 0.0)


@pytest.mark.parametrize("gap,ramp", [(4, None), (3, None), (5, (1.3, 0.6))])
def test_thickness_is_the_distance_between_interpolated_crossings(gap, ramp):
    # a 1D-like film on the centre row of a 2D box: gas | liquid x gap | gas, optionally with one
    # ramp node value on each side; crossings by linear interpolation between node centres
    nx, ny = 40, 9
    rho = np.full((1, ny, nx), RHO_L)
    xa, xb = 14, 14 + gap + 1          # last gas node of A, first gas node of B
    rho[:, 2:7, 4:xa + 1] = RHO_G
    rho[:, 2:7, xb:xb + 11] = RHO_G
    if ramp:
        rho[:, 2:7, xa + 1] = ramp[0]  # first liquid node beside A
        rho[:, 2:7, xb - 1] = ramp[1]  # last node beside B: still gas-like (< theta)
    o = _box(9, (nx, ny, 1), rho)
    _seed_labels(o, (9.0, 4.0, 0.0), (xb + 5.0, 4.0, 0.0))
    h, rd, n = o.film_geometry(0, 1)
    if ramp is None:
        # both crossings halfway between the gas and liquid node centres
        assert h == pytest.approx(gap, abs=1e-12)
    else:
        # ramp[1] < theta joins bubble B's label: B starts at xb - 1
        sA = xa + (THETA - RHO_G) / (ramp[0] - RHO_G)
        sB = (xb - 2) + (RHO_L - THETA) / (RHO_L - ramp[1])
        assert h == pytest.approx(sB - sA, abs=1e-12)
    assert n >= 1 and rd == pytest.approx(0.5 * n)


def _brute_rows(lab, la, lb, ys, xs, film_max=8):
    """Count rows (y) where the x-ordered run from A to B is a film of 1..film_max liquid nodes."""
    count = 0
    for y in ys:
        row = lab[y]
        seg = list(row[xs[0]:xs[1] + 1])
        ia = [k for k, v in enumerate(seg) if v == la]
        if not ia:
            continue
        sa = ia[-1]
        ib = [k for k in range(sa + 1, len(seg)) if seg[k] == lb]
        if not ib:
            continue
        run = seg[sa + 1:ib[0]]
        if 1 <= len(run) <= film_max and all(v == 0 for v in run):
            count += 1
    return count


@pytest.mark.parametrize("R,gap", [(10, 2), (14, 3), (9, 5)])
def test_disc_line_count_2d_matches_brute_force(R, gap):
    nx, ny = 4 * R + gap + 20, 2 * R + 14
    cy = ny // 2
    ca = (10 + R, cy, 0)
    cb = (10 + 3 * R + gap + 1, cy, 0)  # surfaces gap nodes apart on the centre row
    rho = _two_balls((nx, ny, 1), ca, cb, R)
    o = _box(9, (nx, ny, 1), rho)
    _seed_labels(o, ca, cb)
    h, rd, n = o.film_geometry(0, 1)
    lab = o.labels().reshape(ny, nx)
    la, lb = lab[cy, ca[0]], lab[cy, cb[0]]
    bub = {b["label"]: b for b in o.bubbles()}
    K = int(np.floor(min(bub[la]["radius"], bub[lb]["radius"])))
    # centroids sit on the centre row (mirror symmetry), so line k is row cy + k
    ys = [cy + k for k in range(-K, K + 1)]
    assert n == _brute_rows(lab, la, lb, ys, (ca[0], cb[0]))
    assert rd == 0.5 * n
    assert h == pytest.approx(gap, abs=1e-9)


def test_disc_line_count_3d_matches_brute_force():
    R, gap = 6, 2
    shape = (4 * R + gap + 14, 2 * R + 10, 2 * R + 10)
    nx, ny, nz = shape
    cy, cz = ny // 2, nz // 2
    ca = (7 + R, cy, cz)
    cb = (7 + 3 * R + gap + 1, cy, cz)
    o = _box(19, shape, _two_balls(shape, ca, cb, R))
    _seed_labels(o, ca, cb)
    h, rd, n = o.film_geometry(0, 1)
    lab = o.labels().reshape(nz, ny, nx)
    la, lb = lab[cz, cy, ca[0]], lab[cz, cy, cb[0]]
    bub = {b["label"]: b for b in o.bubbles()}
    K = int(np.floor(min(bub[la]["radius"], bub[lb]["radius"])))
    # axis x: the perpendicular basis is n1 = -y, n2 = -z, so line (i, j) runs at (cy-i, cz-j)
    count = 0
    for i in range(-K, K + 1):
        for j in range(-K, K + 1):
            if i * i + j * j > K * K:
                continue
            count += _brute_rows(lab[cz - j], la, lb, [cy - i], (ca[0], cb[0]))
    assert n == count
    assert rd == pytest.approx(np.sqrt(n / np.pi))
    assert h == pytest.approx(gap, abs=1e-9)


def test_geometry_needs_two_distinct_bubbles():
    o = _box(9, (24, 12, 1), _two_balls((24, 12, 1), (6, 6, 0), (9, 6, 0), 3))
    _seed_labels(o, (6, 6, 0), (9, 6, 0))  # overlapping balls: one component
    with pytest.raises(ValueError):
        o.film_geometry(0, 1)
