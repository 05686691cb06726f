"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

The oracle shares nothing with the HIP library; this module only marshals numpy arrays into
``libsc_oracle.so``.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None


class OrcEvent(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("nucleus_a", C.c_int32), ("nucleus_b", C.c_int32),
        ("label_a", C.c_uint32), ("label_b", C.c_uint32), ("film_node", C.c_int64),
        ("film_len", C.c_int32), ("pad", C.c_int32), ("lap_p", C.c_double),
        ("rho_film", C.c_double),
    ]


class OrcTopoEvent(C.Structure):
    _fields_ = [("step", C.c_int64), ("nucleus_a", C.c_int32), ("nucleus_b", C.c_int32)]


class OrcBubble(C.Structure):
    _fields_ = [
        ("label", C.c_uint32), ("nucleus", C.c_int32), ("n", C.c_int64),
        ("centroid", C.c_double * 3), ("radius", C.c_double), ("n_nuclei", C.c_int32),
        ("pad", C.c_int32),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build_oracle()
    lib = C.CDLL(LIB)
    P = C.c_void_p
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_double,
                               C.c_int, C.c_int]
    lib.orc_destroy.argtypes = [P]
    lib.orc_seed_nuclei.argtypes = [P, C.c_int, P, P, P, C.c_double]
    lib.orc_step.argtypes = [P, C.c_int]
    lib.orc_fields.argtypes = [P, P, P, P]
    lib.orc_laplacian_p.argtypes = [P, P, P]
    lib.orc_force.argtypes = [P, P]
    lib.orc_label_mask.restype = C.c_int64
    lib.orc_label_mask.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P]
    lib.orc_get_f.argtypes = [P, P]
    lib.orc_set_f.argtypes = [P, P]
    lib.orc_set_equilibrium.argtypes = [P, P, P]
    lib.orc_test_pass.argtypes = [P]
    lib.orc_time.restype = C.c_int64
    lib.orc_time.argtypes = [P]
    lib.orc_num_nodes.restype = C.c_int64
    lib.orc_num_nodes.argtypes = [P]
    lib.orc_labels.argtypes = [P, P]
    lib.orc_bubbles.argtypes = [P, P, C.c_int]
    lib.orc_events.argtypes = [P, P, C.c_int]
    lib.orc_topo_events.argtypes = [P, P, C.c_int]
    lib.orc_nuclei.argtypes = [P, P, P]
    lib.orc_lattice.argtypes = [C.c_int, P, P]
    lib.orc_feq.argtypes = [C.c_int, C.c_double, P, P]
    lib.orc_uniform.restype = C.c_double
    lib.orc_uniform.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_splitmix64.restype = C.c_uint64
    lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_set_two_component.restype = C.c_int
    lib.orc_set_two_component.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.orc_gas_density.argtypes = [P, P]
    lib.orc_set_gas_equilibrium.restype = C.c_int
    lib.orc_set_gas_equilibrium.argtypes = [P, P]
    lib.orc_film_geometry.restype = C.c_int
    lib.orc_film_geometry.argtypes = [P, C.c_int, C.c_int, P, P, P]
    lib.orc_set_gravity.restype = C.c_int
    lib.orc_set_gravity.argtypes = [P, P, C.c_double]
    lib.orc_rho0.restype = C.c_double
    lib.orc_rho0.argtypes = [P]
    lib.orc_set_barrier.restype = C.c_int
    lib.orc_set_barrier.argtypes = [P, C.c_int, C.c_int]
    lib.orc_owner.argtypes = [P, P]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_num_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def lattice(q):
    lib = _load()
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    lib.orc_lattice(q, _ptr(e), _ptr(w))
    return e, w


def feq(q, rho, u):
    lib = _load()
    uu = np.zeros(3, dtype=np.float64)
    uu[: len(u)] = u
    out = np.zeros(q, dtype=np.float64)
    lib.orc_feq(q, float(rho), _ptr(uu), _ptr(out))
    return out


def uniform(seed, idx):
    return _load().orc_uniform(seed, idx)


def splitmix64(seed, k):
    return _load().orc_splitmix64(seed, k)


def num_threads():
    return _load().orc_num_threads()


def label_mask(q, shape, mask):
    """Canonical labels of a gas mask (shape = (nx, ny, nz); mask flat in x-fastest order)."""
    lib = _load()
    nx, ny, nz = shape
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    lab = np.zeros(m.size, dtype=np.uint32)
    n = lib.orc_label_mask(q, nx, ny, nz, _ptr(m), _ptr(lab))
    return lab, int(n)


class OracleSim:
    """One FP64 oracle simulation (periodic box, x fastest)."""

    def __init__(self, q, nx, ny, nz=1, tau=1.0, G=-5.0, rho_l=1.93, rho_g=0.16, amp=1e-3,
                 seed=1, theta=0.0, K=10, film_max=8, barrier=False, corona=3, gravity=None,
                 rho0=0.0, two_component=None):
        self._lib = _load()
        self.q, self.nx, self.ny, self.nz = q, nx, ny, nz
        self.d = 2 if q == 9 else 3
        self.N = nx * ny * nz
        self.G = G
        h = self._lib.orc_create(q, nx, ny, nz, tau, G, rho_l, rho_g, amp, seed, theta, K,
                                 film_max)
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = C.c_void_p(h)
        if two_component is not None:  # (Gx, tau_v, rho_vapour, rho_dissolved)
            if self._lib.orc_set_two_component(self._h, *[float(v) for v in two_component]) != 0:
                raise ValueError("bad two-component parameters")
        if barrier:
            self.set_barrier(True, corona)
        if gravity is not None:
            self.set_gravity(gravity, rho0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and self._lib is not None:
            self._lib.orc_destroy(h)
            self._h = None

    def seed_nuclei(self, centres, radii, budgets, rate):
        c = np.zeros((len(radii), 3), dtype=np.float64)
        if len(radii) > 0:
            cc = np.asarray(centres, dtype=np.float64).reshape(len(radii), -1)
            c[:, : cc.shape[1]] = cc
        r = np.ascontiguousarray(radii, dtype=np.float64)
        b = np.ascontiguousarray(budgets, dtype=np.float64)
        rc = self._lib.orc_seed_nuclei(self._h, len(r), _ptr(c), _ptr(r), _ptr(b), float(rate))
        if rc != 0:
            raise RuntimeError(f"orc_seed_nuclei returned {rc}")

    def set_barrier(self, on, corona=3):
        if self._lib.orc_set_barrier(self._h, 1 if on else 0, int(corona)) != 0:
            raise ValueError("corona must be >= 0")

    def set_gas_equilibrium(self, rho_v):
        r = np.ascontiguousarray(rho_v, dtype=np.float64).reshape(self.N)
        if self._lib.orc_set_gas_equilibrium(self._h, _ptr(r)) != 0:
            raise ValueError("no gas component")

    def gas_density(self):
        rv = np.zeros(self.N)
        self._lib.orc_gas_density(self._h, _ptr(rv))
        return rv

    def film_geometry(self, a, b):
        """(h, R_d, n_lines) of the bubbles holding nuclei a and b at the last test pass."""
        h, r, n = C.c_double(), C.c_double(), C.c_int()
        rc = self._lib.orc_film_geometry(self._h, int(a), int(b), C.byref(h), C.byref(r),
                                         C.byref(n))
        if rc != 0:
            raise ValueError(f"orc_film_geometry returned {rc}")
        return h.value, r.value, n.value

    def set_gravity(self, g, rho0=0.0):
        gg = np.zeros(3)
        gg[: len(g)] = g
        if self._lib.orc_set_gravity(self._h, _ptr(gg), float(rho0)) != 0:
            raise ValueError("gravity and rho0 must be finite")

    @property
    def rho0(self):
        return float(self._lib.orc_rho0(self._h))

    def owner(self):
        o = np.zeros(self.N, dtype=np.int32)
        self._lib.orc_owner(self._h, _ptr(o))
        return o

    def step(self, n):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise FloatingPointError(f"orc_step returned {rc}")

    def test_pass(self):
        return self._lib.orc_test_pass(self._h)

    @property
    def t(self):
        return int(self._lib.orc_time(self._h))

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.d, self.N))
        tot = np.zeros(4)
        self._lib.orc_fields(self._h, _ptr(rho), _ptr(u), _ptr(tot))
        return rho, u, tot

    def totals(self):
        tot = np.zeros(4)
        self._lib.orc_fields(self._h, None, None, _ptr(tot))
        return tot

    def laplacian_p(self):
        p = np.zeros(self.N)
        lap = np.zeros(self.N)
        self._lib.orc_laplacian_p(self._h, _ptr(p), _ptr(lap))
        return p, lap

    def force(self):
        F = np.zeros((self.d, self.N))
        self._lib.orc_force(self._h, _ptr(F))
        return F

    def get_f(self):
        f = np.zeros((self.q, self.N))
        self._lib.orc_get_f(self._h, _ptr(f))
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        self._lib.orc_set_f(self._h, _ptr(f))

    def set_equilibrium(self, rho, u=None):
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.d, self.N)
        self._lib.orc_set_equilibrium(self._h, _ptr(r), _ptr(uu))

    def labels(self):
        lab = np.zeros(self.N, dtype=np.uint32)
        self._lib.orc_labels(self._h, _ptr(lab))
        return lab

    def bubbles(self):
        n = self._lib.orc_bubbles(self._h, None, 0)
        arr = (OrcBubble * max(n, 1))()
        self._lib.orc_bubbles(self._h, C.cast(arr, C.c_void_p), n)
        return [dict(label=b.label, nucleus=b.nucleus, n=b.n, centroid=tuple(b.centroid),
                     radius=b.radius, n_nuclei=b.n_nuclei) for b in arr[:n]]

    def events(self):
        n = self._lib.orc_events(self._h, None, 0)
        arr = (OrcEvent * max(n, 1))()
        self._lib.orc_events(self._h, C.cast(arr, C.c_void_p), n)
        return [dict(step=e.step, nucleus_a=e.nucleus_a, nucleus_b=e.nucleus_b,
                     label_a=e.label_a, label_b=e.label_b, film_node=e.film_node,
                     film_len=e.film_len, lap_p=e.lap_p, rho_film=e.rho_film) for e in arr[:n]]

    def topo_events(self):
        n = self._lib.orc_topo_events(self._h, None, 0)
        arr = (OrcTopoEvent * max(n, 1))()
        self._lib.orc_topo_events(self._h, C.cast(arr, C.c_void_p), n)
        return [dict(step=e.step, nucleus_a=e.nucleus_a, nucleus_b=e.nucleus_b) for e in arr[:n]]

    def nuclei(self):
        n = self._lib.orc_nuclei(self._h, None, None)
        comp = np.zeros(max(n, 1), dtype=np.uint32)
        rem = np.zeros(max(n, 1))
        self._lib.orc_nuclei(self._h, _ptr(comp), _ptr(rem))
        return comp[:n], rem[:n]
