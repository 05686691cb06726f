"""Seeded synthetic workloads (shapes, sizes and distributions only; no method arithmetic).

These generators feed both the HIP library and the FP64 oracle.  They draw nucleation sites,
radii, budgets and batch-instance parameters; every density field the method evolves is built
by each side itself from (seed, node index) with SplitMix64.

Workloads (the paper publishes no dataset; these stand in for its experiments):
  two_bubble      two bubbles of radius 15, gap 4, on a 128^2 D2Q9 box (Sec. 4, Fig. 2: two bubbles
                  approaching without gravity).
  two_bubble_3d   the same pair as two spheres in a D3Q19 box (film-size sweep in 3D).
  two_bubble_mixture  the pair with two components, optionally fed (film-size sweep of growing
                  bubbles).
  foam_2d         1024^2 D2Q9 with 64 random nuclei of radius 3 (Sec. 3.1: time-random nucleation
                  sites, blowing agent decomposed at them; Sec. 4, Fig. 4: foam structure).
  foam_3d         256^3 D3Q19 with 200 random nuclei (the 3D version of foam_2d).
  foam_3d_large   512^3 D3Q19 with 400 nuclei, for 16-bit population storage; a 128^3 box from the
                  same generator and seed (nucleus count scaled by volume) is the error run.
  batch           4096 independent two-bubble D2Q9 boxes of uneven size, G, radius and gap (Sec. 4,
                  Fig. 3: merging as a function of bubble size).
  mixture_2d      foam_2d's box and nuclei with a liquid and a gas component (Sec. 3: the agent's
                  gas grows the bubbles; Sec. 3.1: two simulations side by side).
  mixture_3d      foam_3d's box and nuclei with the two components.
"""
from dataclasses import dataclass, field
import math

import numpy as np

# Flat-interface coexistence densities of the scheme (psi = 1 - exp(-rho), cs^2 = 1/3) at five
# attraction strengths: (G, rho_gas, rho_liquid).  Used only to pick initial densities of batch
# instances; the test suite checks these values against the mechanical-stability condition and
# against the oracle's own flat-interface runs.
COEXISTENCE = (
    (-4.50, 0.254125, 1.494301),
    (-4.75, 0.196282, 1.724739),
    (-5.00, 0.156413, 1.932442),
    (-5.25, 0.127145, 2.125327),
    (-5.50, 0.104813, 2.307522),
)


def coexistence_densities(G):
    """Linear interpolation of COEXISTENCE at G (clamped to the tabulated range)."""
    gs = np.array([c[0] for c in COEXISTENCE])
    rg = np.array([c[1] for c in COEXISTENCE])
    rl = np.array([c[2] for c in COEXISTENCE])
    order = np.argsort(gs)
    return (float(np.interp(G, gs[order], rg[order])), float(np.interp(G, gs[order], rl[order])))


@dataclass
class SimSpec:
    """One periodic box and its nuclei; every field is plain data."""
    name: str
    q: int
    nx: int
    ny: int
    nz: int = 1
    tau: float = 1.0
    G: float = -5.0
    rho_l: float = 1.93
    rho_g: float = 0.16
    amp: float = 1e-3
    seed: int = 1
    theta: float = 0.0          # <= 0: midpoint of rho_l and rho_g
    K: int = 10                  # test cadence
    film_max: int = 8
    steps: int = 2000
    centres: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    radii: np.ndarray = field(default_factory=lambda: np.zeros(0))
    budgets: np.ndarray = field(default_factory=lambda: np.zeros(0))
    rate: float = 0.0
    # two components: (G_cross, tau_vapour, rho_vapour, rho_dissolved); None = one component
    two_component: tuple = None

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def d(self):
        return 2 if self.q == 9 else 3


def two_bubble(amp=1e-3, seed=1, nx=128, ny=128, radius=15.0, gap=4, K=10, steps=2000):
    """Two radius-15 bubbles with a 4-node liquid film on the x mid-line of a 128^2 box."""
    centres = pair_centres(nx, ny, radius, gap)
    return SimSpec(name="two_bubble", q=9, nx=nx, ny=ny, tau=1.0, G=-5.0, rho_l=1.93, rho_g=0.16,
                   amp=amp, seed=seed, K=K, steps=steps, centres=centres,
                   radii=np.array([radius, radius]), budgets=np.zeros(2), rate=0.0)


def two_bubble_3d(nx=96, ny=64, nz=64, radius=15.0, gap=4, K=10, steps=2000, amp=1e-3, seed=1):
    """Two spheres on the x axis of a D3Q19 box, `gap` liquid nodes apart on the four node rows
    nearest the axis (the 3D form of two_bubble, for the film-size sweep)."""
    c = pair_centres(nx, ny, radius, gap)
    c[:, 2] = nz / 2.0 - 0.5
    return SimSpec(name="two_bubble_3d", q=19, nx=nx, ny=ny, nz=nz, tau=1.0, G=-5.0, rho_l=1.93,
                   rho_g=0.16, amp=amp, seed=seed, K=K, steps=steps, centres=c,
                   radii=np.array([radius, radius]), budgets=np.zeros(2), rate=0.0)


def two_bubble_mixture(nx=128, ny=128, radius=15.0, gap=4, K=10, rate=0.0, steps=2000, amp=1e-3,
                       seed=1):
    """two_bubble with the liquid and gas components (MIXTURE); with rate > 0 the agent feeds
    each bubble `rate` mass of gas per step (unbounded budgets)."""
    centres = pair_centres(nx, ny, radius, gap)
    return SimSpec(name="two_bubble_mixture", q=9, nx=nx, ny=ny, tau=1.0, G=0.0, rho_l=1.0,
                   rho_g=0.05, amp=amp, seed=seed, K=K, steps=steps, centres=centres,
                   radii=np.array([radius, radius]), budgets=np.full(2, 1e12), rate=rate,
                   two_component=MIXTURE)


def pair_centres(nx, ny, radius, gap):
    """Centres of two equal bubbles on the x mid-line leaving exactly `gap` liquid nodes.

    The film is nodes s .. s+gap-1 with s = nx//2 - gap//2 on the rows y = ny/2 - 1 and ny/2;
    centres are half-integers (s - 1 - R + 1/2 and s + gap + R - 1/2, y = ny/2 - 1/2), so with
    gas iff |x - c|^2 <= R^2 the outermost gas node of each bubble on those rows is s-1 and
    s+gap (for the default 128^2, R = 15, gap = 4: centres 46.5 and 80.5, film x = 62..65).
    """
    s = nx // 2 - gap // 2
    cy = ny / 2.0 - 0.5
    return np.array([(s - 1 - radius + 0.5, cy, 0.0), (s + gap + radius - 0.5, cy, 0.0)],
                     dtype=np.float64)


def random_sites(rng, n, shape, min_spacing):
    """n integer sites, uniform on the periodic box, rejecting any closer than min_spacing
    (periodic distance) to an accepted one."""
    shape = np.asarray(shape)
    sites = []
    tries = 0
    while len(sites) < n:
        tries += 1
        if tries > 1000 * n + 100000:
            raise RuntimeError("could not place nuclei with the requested spacing")
        p = np.array([rng.integers(0, s) for s in shape], dtype=np.int64)
        ok = True
        for s in sites:
            dv = np.abs(p - s)
            dv = np.minimum(dv, shape - dv)
            if float(np.sqrt((dv * dv).sum())) < min_spacing:
                ok = False
                break
        if ok:
            sites.append(p)
    return np.array(sites, dtype=np.int64)


def _foam(name, q, shape, n_nuclei, seed, tau, K, steps, radius=3.0, min_spacing=12.0,
          amp=1e-3, rate=1e-4, rho_g=0.16, rho_l=1.93, G=-5.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    sites = random_sites(rng, n_nuclei, shape, min_spacing)
    centres = np.zeros((n_nuclei, 3))
    centres[:, : len(shape)] = sites
    if len(shape) == 2:
        scale = math.pi * 40.0 ** 2 * rho_g
    else:
        scale = 4.0 / 3.0 * math.pi * 40.0 ** 3 * rho_g
    budgets = rng.uniform(0.5, 2.0, size=n_nuclei) * scale
    nx, ny = shape[0], shape[1]
    nz = shape[2] if len(shape) == 3 else 1
    return SimSpec(name=name, q=q, nx=nx, ny=ny, nz=nz, tau=tau, G=G, rho_l=rho_l, rho_g=rho_g,
                   amp=amp, seed=seed, K=K, steps=steps, centres=centres,
                   radii=np.full(n_nuclei, radius), budgets=budgets, rate=rate)


def gas_rich_3d(n=256, n_nuclei=200, seed=3, steps=5000, K=50):
    """foam_3d's box and cadence with bubbles that persist, to measure the test pass on a gas
    mask that is not empty: 200 spheres of radius 12 (about 7,200 gas nodes each, 8.6 % of the
    box) at least 30 apart, in a slightly stretched liquid (rho_l = 1.80) that keeps them."""
    return _foam("gas_rich_3d", 19, (n, n, n), n_nuclei, seed, tau=0.9, K=K, steps=steps,
                 radius=12.0, min_spacing=30.0, rho_l=1.80)


def foam_2d(n=1024, n_nuclei=64, seed=2, steps=20000, K=100):
    return _foam("foam_2d", 9, (n, n), n_nuclei, seed, tau=1.0, K=K, steps=steps)


def foam_3d(n=256, n_nuclei=200, seed=3, steps=5000, K=50):
    return _foam("foam_3d", 19, (n, n, n), n_nuclei, seed, tau=0.9, K=K, steps=steps)


def foam_3d_large(n=512, n_nuclei=400, seed=4, steps=2000, K=50):
    """512^3; for the error run pass n=128 and the nucleus count scaled by volume (400/64 ~ 6)."""
    return _foam("foam_3d_large", 19, (n, n, n), n_nuclei, seed, tau=0.9, K=K, steps=steps)


def foam_3d_error_run(seed=4, steps=2000):
    return foam_3d_large(n=128, n_nuclei=max(1, round(400 / 64)), seed=seed, steps=steps)


def precision_error_box(seed=4, steps=2000, radius=12.0, gap=14, rho_l=1.80):
    """Two-phase error box of the precision workload (D3Q19, tau 0.9, G -5, K 50): two spheres of
    radius 12, 14 liquid nodes apart on the x axis of a 94 x 56 x 56 box.  At rho_l = 1.93 (the
    flat-interface coexistence density) a sphere's Laplace pressure condenses its gas, as it does
    the foam's radius-3 nuclei; a slightly stretched liquid at 1.80 keeps both spheres (about
    10,300 gas nodes each at t = 1000), so errors are stated on a box that holds gas."""
    nx, ny = int(4 * radius + gap + 32), int(2 * radius + 32)
    c = pair_centres(nx, ny, radius, gap)
    c[:, 2] = ny / 2.0 - 0.5
    return SimSpec(name="precision_error_box", q=19, nx=nx, ny=ny, nz=ny, tau=0.9, G=-5.0,
                   rho_l=rho_l, rho_g=0.16, amp=1e-3, seed=seed, K=50, steps=steps, centres=c,
                   radii=np.array([radius, radius]), budgets=np.zeros(2), rate=0.0)


# The mixture's parameters: cross repulsion G_cross, gas relaxation time (<= 0: the liquid's),
# gas density in the nuclei and dissolved in the liquid; the liquid component is 1.0 in the
# liquid and 0.05 in the nuclei.
MIXTURE = (1.5, 1.0, 1.0, 0.05)


def _mixture(spec, name):
    spec.name = name
    spec.G = 0.0
    spec.rho_l, spec.rho_g = 1.0, 0.05
    spec.two_component = MIXTURE
    return spec


def mixture_2d(n=1024, n_nuclei=64, seed=2, steps=20000, K=100):
    return _mixture(foam_2d(n, n_nuclei, seed, steps, K), "mixture_2d")


def mixture_3d(n=256, n_nuclei=200, seed=3, steps=5000, K=50):
    return _mixture(foam_3d(n, n_nuclei, seed, steps, K), "mixture_3d")


@dataclass
class BatchSpec:
    """Independent two-bubble D2Q9 boxes, one row per instance."""
    nx: np.ndarray
    ny: np.ndarray
    G: np.ndarray
    radius: np.ndarray
    gap: np.ndarray
    rho_l: np.ndarray
    rho_g: np.ndarray
    seed: np.ndarray
    tau: float = 1.0
    amp: float = 1e-3
    K: int = 10
    film_max: int = 8
    max_steps: int = 5000

    @property
    def n(self):
        return len(self.nx)

    def instance(self, k):
        """SimSpec of instance k (two bubbles on the x mid-line, as two_bubble)."""
        nx, ny = int(self.nx[k]), int(self.ny[k])
        R, g = float(self.radius[k]), int(self.gap[k])
        centres = pair_centres(nx, ny, R, g)
        return SimSpec(name=f"batch[{k}]", q=9, nx=nx, ny=ny, tau=self.tau, G=float(self.G[k]),
                       rho_l=float(self.rho_l[k]), rho_g=float(self.rho_g[k]), amp=self.amp,
                       seed=int(self.seed[k]), K=self.K, film_max=self.film_max,
                       steps=self.max_steps, centres=centres, radii=np.array([R, R]),
                       budgets=np.zeros(2), rate=0.0)


def batch(n=4096, seed=5, lo=64, hi=256, max_steps=5000):
    """nx, ny ~ U{lo..hi}; G ~ U[-5.5, -4.5]; R ~ U{8..40}; gap ~ U{2..10}; R is redrawn while the
    pair plus a margin does not fit (4R + gap + 16 > nx or 2R + 16 > ny)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = rng.integers(lo, hi + 1, size=n)
    ny = rng.integers(lo, hi + 1, size=n)
    G = rng.uniform(-5.5, -4.5, size=n)
    gap = rng.integers(2, 11, size=n)
    R = np.zeros(n, dtype=np.int64)
    for k in range(n):
        while True:
            r = int(rng.integers(8, 41))
            if 4 * r + gap[k] + 16 <= nx[k] and 2 * r + 16 <= ny[k]:
                R[k] = r
                break
    rg = np.zeros(n)
    rl = np.zeros(n)
    for k in range(n):
        rg[k], rl[k] = coexistence_densities(G[k])
    seeds = rng.integers(1, 2 ** 62, size=n, dtype=np.int64)
    return BatchSpec(nx=nx, ny=ny, G=G, radius=R.astype(np.float64), gap=gap, rho_l=rl, rho_g=rg,
                     seed=seeds, max_steps=max_steps)
