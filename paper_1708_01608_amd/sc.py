"""Python binding of libsc (include/sc.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libsc.so.  PyTorch, when present, provides
the device memory (its caching allocator, through sc_allocator callbacks) and the stream.  If the
library is missing this module raises; there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsc.so")

SC_OK, SC_E_INVAL, SC_E_NOMEM, SC_E_DEVICE, SC_E_STATE, SC_E_NUMERIC, SC_E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
SC_D2Q9, SC_D3Q19 = 9, 19
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
COMPUTE = {"auto": 0, "f32": 1, "f64": 2}
SC_KERNEL_STEP, SC_KERNEL_SOURCE, SC_KERNEL_TEST = 0, 1, 2


class ScError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"sc error {code}: {message}")
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("lattice", C.c_int32), ("nx", C.c_int32),
        ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double), ("G", C.c_double),
        ("rho_liquid", C.c_double), ("rho_gas", C.c_double), ("noise_amp", C.c_double),
        ("noise_seed", C.c_uint64), ("gas_threshold", C.c_double), ("test_every", C.c_int32),
        ("film_max", C.c_int32), ("storage", C.c_int32), ("compute", C.c_int32),
        ("rho_ref", C.c_double), ("stream", C.c_void_p), ("allocator", C.POINTER(Allocator)),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32),
        ("step_variant", C.c_int32),
        ("barrier", C.c_int32), ("corona", C.c_int32),
        ("gravity", C.c_double * 3), ("rho_buoyancy", C.c_double),
        ("components", C.c_int32), ("reserved2", C.c_int32), ("G_cross", C.c_double),
        ("tau_vapour", C.c_double), ("rho_vapour", C.c_double), ("rho_dissolved", C.c_double),
    ]


class MergeEvent(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("nucleus_a", C.c_int32), ("nucleus_b", C.c_int32),
        ("label_a", C.c_uint32), ("label_b", C.c_uint32), ("film_node", C.c_int64),
        ("film_len", C.c_int32), ("reserved", C.c_int32), ("lap_p", C.c_double),
        ("rho_film", C.c_double),
    ]


class TopoEvent(C.Structure):
    _fields_ = [("step", C.c_int64), ("nucleus_a", C.c_int32), ("nucleus_b", C.c_int32)]


class Bubble(C.Structure):
    _fields_ = [
        ("label", C.c_uint32), ("nucleus", C.c_int32), ("n", C.c_int64),
        ("centroid", C.c_double * 3), ("radius", C.c_double), ("n_nuclei", C.c_int32),
        ("reserved", C.c_int32),
    ]


class TuneEntry(C.Structure):
    _fields_ = [("tile_x", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32),
                ("variant", C.c_int32), ("us_per_launch", C.c_double)]


class BatchInstance(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double), ("G", C.c_double),
        ("rho_liquid", C.c_double), ("rho_gas", C.c_double), ("noise_amp", C.c_double),
        ("noise_seed", C.c_uint64), ("gas_threshold", C.c_double),
        ("centre", (C.c_double * 3) * 2), ("radius", C.c_double * 2),
    ]


class BatchResult(C.Structure):
    _fields_ = [
        ("merge_step", C.c_int64), ("topo_step", C.c_int64), ("steps_run", C.c_int64),
        ("film_node", C.c_int64), ("film_len", C.c_int32), ("status", C.c_int32),
        ("lap_p", C.c_double), ("rho_film", C.c_double), ("totals", C.c_double * 3),
    ]


# Entry points declared in include/sc.h (checked by the CPU test suite).
EXPORTS = (
    "sc_abi_version", "sc_last_error", "sc_params_init", "sc_create", "sc_destroy",
    "sc_seed_nuclei", "sc_step", "sc_step_graphs", "sc_fields", "sc_fields_device", "sc_laplacian_p",
    "sc_laplacian_p_device", "sc_label_bubbles", "sc_label_bubbles_noalloc",
    "sc_merge_events", "sc_topo_events", "sc_bubbles", "sc_last_labels", "sc_nuclei",
    "sc_source_ledger", "sc_owner", "sc_buoyancy_density", "sc_film_geometry", "sc_gas_density",
    "sc_set_gas_equilibrium", "sc_time",
    "sc_lattice", "sc_get_populations", "sc_set_populations", "sc_set_equilibrium",
    "sc_get_gas_populations", "sc_set_gas_populations",
    "sc_test_pass", "sc_profile", "sc_profile_read", "sc_step_config", "sc_compute_type",
    "sc_batch_create", "sc_batch_run", "sc_batch_fields", "sc_batch_destroy", "sc_autotune",
    "sc_hbm_probe", "sc_pattern_probe", "sc_batch_tune",
)

_lib = None


def load_library(path=LIB_PATH):
    """Load libsc.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built (run __graft_entry__.build())")
    # PyTorch ships its own HIP runtime with the same soname as /opt/rocm's; loading torch first
    # makes libsc bind to that one, so the process holds a single HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "sc_abi_version": (C.c_uint32, []),
        "sc_last_error": (C.c_char_p, []),
        "sc_params_init": (C.c_int, [C.POINTER(Params)]),
        "sc_create": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_void_p)]),
        "sc_destroy": (C.c_int, [P]),
        "sc_seed_nuclei": (C.c_int, [P, C.c_int32, P, P, P, C.c_double]),
        "sc_step": (C.c_int, [P, C.c_int32]),
        "sc_fields": (C.c_int, [P, P, P, P]),
        "sc_fields_device": (C.c_int, [P, P, P]),
        "sc_laplacian_p": (C.c_int, [P, P, P]),
        "sc_laplacian_p_device": (C.c_int, [P, P, P]),
        "sc_label_bubbles": (C.c_int, [P, P, P, P]),
        "sc_merge_events": (C.c_int, [P, P, C.c_int32, P]),
        "sc_topo_events": (C.c_int, [P, P, C.c_int32, P]),
        "sc_bubbles": (C.c_int, [P, P, C.c_int32, P]),
        "sc_last_labels": (C.c_int, [P, P]),
        "sc_nuclei": (C.c_int, [P, P, P]),
        "sc_step_graphs": (C.c_int, [P, C.c_int32]),
        "sc_label_bubbles_noalloc": (C.c_int, [P, P, P, P]),
        "sc_source_ledger": (C.c_int, [P, P, P]),
        "sc_get_gas_populations": (C.c_int, [P, P]),
        "sc_set_gas_populations": (C.c_int, [P, P]),
        "sc_owner": (C.c_int, [P, P]),
        "sc_buoyancy_density": (C.c_int, [P, P]),
        "sc_film_geometry": (C.c_int, [P, C.c_int32, C.c_int32, P, P, P]),
        "sc_gas_density": (C.c_int, [P, P]),
        "sc_set_gas_equilibrium": (C.c_int, [P, P]),
        "sc_time": (C.c_int, [P, P]),
        "sc_lattice": (C.c_int, [C.c_int32, P, P]),
        "sc_get_populations": (C.c_int, [P, P]),
        "sc_set_populations": (C.c_int, [P, P]),
        "sc_set_equilibrium": (C.c_int, [P, P, P]),
        "sc_test_pass": (C.c_int, [P]),
        "sc_profile": (C.c_int, [P, C.c_int32]),
        "sc_profile_read": (C.c_int, [P, C.c_int32, P, P]),
        "sc_step_config": (C.c_int, [P, P, P, P, P]),
        "sc_compute_type": (C.c_int, [P, P]),
        "sc_batch_create": (C.c_int, [C.c_int32, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      P, P, C.POINTER(C.c_void_p)]),
        "sc_batch_run": (C.c_int, [P, P, P]),
        "sc_batch_fields": (C.c_int, [P, C.c_int32, P]),
        "sc_batch_destroy": (C.c_int, [P]),
        "sc_autotune": (C.c_int, [P, C.c_int32, P, C.c_int32, P]),
        "sc_hbm_probe": (C.c_int, [C.c_size_t, C.c_int32, P, P]),
        "sc_pattern_probe": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, C.c_int32, C.c_int32, P, P]),
        "sc_batch_tune": (C.c_int, [P, C.c_int32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc != SC_OK:
        msg = load_library().sc_last_error()
        raise ScError(rc, msg.decode() if msg else "")


def pattern_probe(nx, ny, nz, storage="f32", tile=(256, 4, 64), reps=5):
    """(flat GB/s, marching GB/s) of the D3Q19 step's memory pattern without its arithmetic."""
    lib = load_library()
    st = {"f32": 0, "f16": 1, "bf16": 2}[storage] if isinstance(storage, str) else int(storage)
    f, m = C.c_double(), C.c_double()
    _check(lib.sc_pattern_probe(int(nx), int(ny), int(nz), st, int(tile[0]), int(tile[1]),
                                int(tile[2]), int(reps), C.byref(f), C.byref(m)))
    return f.value, m.value


def hbm_probe(nbytes=2550136832, reps=5):
    """(copy GB/s, read GB/s) of the library's float4 probe kernels."""
    lib = load_library()
    c, r = C.c_double(), C.c_double()
    _check(lib.sc_hbm_probe(int(nbytes), int(reps), C.byref(c), C.byref(r)))
    return c.value, r.value


def lattice(q):
    lib = load_library()
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    _check(lib.sc_lattice(q, _ptr(e), _ptr(w)))
    return e, w


class TorchMemory:
    """Device memory and stream from PyTorch (caching allocator + a default-priority stream)."""

    def __init__(self, device=0):
        import torch

        self.torch = torch
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        stream = self.stream

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            except Exception:  # allocation failure is reported to the library as NULL
                return None

        delete = torch.cuda.caching_allocator_delete

        def _free(ptr, user):
            # at interpreter exit a handle may outlive torch's CUDA state: nothing to return
            try:
                delete(ptr)
            except Exception:
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = Allocator(self._alloc, self._free, None)


def _tuned_shape(q, nx, ny, nz, storage, compute, variant, components=1):
    """Step-kernel shape stored by paper_1708_01608_amd.tune for this box, if any."""
    from . import tune

    st = storage if isinstance(storage, str) else {0: "f32", 1: "f16", 2: "bf16"}[storage]
    comp = compute
    if comp == "auto":
        comp = "f64" if st == "f32" else "f32"
    e = tune.load().get(tune.key(q, nx, ny, nz, st, comp, components))
    if not e:
        return None, variant
    return tuple(e["tile"]), e["variant"]


def _check_disjoint(a, b, what):
    """Two output tensors of one call must not share memory: the kernels read neighbours of the
    nodes they write, so overlapping outputs would race (the library checks the same)."""
    if a is None or b is None:
        return
    a0, a1 = a.data_ptr(), a.data_ptr() + a.numel() * a.element_size()
    b0, b1 = b.data_ptr(), b.data_ptr() + b.numel() * b.element_size()
    if a0 < b1 and b0 < a1:
        raise ValueError(f"{what} overlap")


class Sim:
    """One periodic Shan-Chen box on the GPU (a handle of libsc)."""

    def __init__(self, q=9, nx=128, ny=128, nz=1, tau=1.0, G=-5.0, rho_l=1.93, rho_g=0.16,
                 amp=1e-3, seed=1, theta=0.0, K=10, film_max=8, storage="f32", compute="auto",
                 rho_ref=-1.0, tile=None, variant=0, memory="torch", tuned=True, barrier=False,
                 corona=3, gravity=None, rho0=0.0, two_component=None):
        self._lib = load_library()
        self._h = None
        p = Params()
        _check(self._lib.sc_params_init(C.byref(p)))
        p.lattice, p.nx, p.ny, p.nz = q, nx, ny, nz
        p.tau, p.G, p.rho_liquid, p.rho_gas = tau, G, rho_l, rho_g
        p.noise_amp, p.noise_seed, p.gas_threshold = amp, seed, theta
        p.test_every, p.film_max = K, film_max
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.compute = COMPUTE[compute] if isinstance(compute, str) else int(compute)
        p.rho_ref = rho_ref
        comp_name = compute if isinstance(compute, str) else {0: "auto", 1: "f32", 2: "f64"}[compute]
        if tile is None and tuned:
            tile, variant = _tuned_shape(q, nx, ny, nz, storage, comp_name, variant,
                                         2 if two_component is not None else 1)
            if gravity is not None and any(gravity) and variant == 2:
                variant = 3  # no pipelined gravity kernel: same tile, plain variant
        if tile is not None:
            p.tile_x, p.tile_y, p.tile_z = tile
        p.step_variant = int(variant)
        p.barrier, p.corona = (1 if barrier else 0), int(corona)
        if gravity is not None:
            for c, v in enumerate(gravity):
                p.gravity[c] = float(v)
        p.rho_buoyancy = float(rho0)
        if two_component is not None:  # (G_cross, tau_vapour, rho_vapour, rho_dissolved)
            p.components = 2
            p.G_cross, p.tau_vapour, p.rho_vapour, p.rho_dissolved = [float(v) for v in
                                                                       two_component]
        self.mem = None
        if memory == "torch":
            self.mem = TorchMemory()
            p.stream = self.mem.stream.cuda_stream
            p.allocator = C.pointer(self.mem.struct)
        self.q, self.nx, self.ny, self.nz = q, nx, ny, nz
        self.d = 2 if q == 9 else 3
        self.N = nx * ny * nz
        h = C.c_void_p()
        _check(self._lib.sc_create(C.byref(p), C.byref(h)))
        self._h = h
        self.params = p

    @classmethod
    def from_spec(cls, spec, **kw):
        if getattr(spec, "two_component", None) is not None:
            kw.setdefault("two_component", spec.two_component)
        return cls(q=spec.q, nx=spec.nx, ny=spec.ny, nz=spec.nz, tau=spec.tau, G=spec.G,
                   rho_l=spec.rho_l, rho_g=spec.rho_g, amp=spec.amp, seed=spec.seed,
                   theta=spec.theta, K=spec.K, film_max=spec.film_max, **kw)

    def close(self):
        if self._h is not None:
            self._lib.sc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def seed_nuclei(self, centres, radii, budgets, rate):
        n = len(radii)
        c = np.zeros((n, 3))
        if n > 0:
            cc = np.asarray(centres, dtype=np.float64).reshape(n, -1)
            c[:, : cc.shape[1]] = cc
        r = np.ascontiguousarray(radii, dtype=np.float64)
        b = np.ascontiguousarray(budgets, dtype=np.float64)
        _check(self._lib.sc_seed_nuclei(self._h, n, _ptr(c), _ptr(r), _ptr(b), float(rate)))

    def step(self, n):
        _check(self._lib.sc_step(self._h, int(n)))

    def step_graphs(self, enable):
        """K-step blocks of a small box as HIP graphs (default on) or launched step by step."""
        _check(self._lib.sc_step_graphs(self._h, 1 if enable else 0))

    def test_pass(self):
        _check(self._lib.sc_test_pass(self._h))

    @property
    def t(self):
        v = C.c_int64()
        _check(self._lib.sc_time(self._h, C.byref(v)))
        return v.value

    def fields(self, rho=True, u=True, totals=True):
        r = np.zeros(self.N, dtype=np.float32) if rho else None
        uu = np.zeros((self.d, self.N), dtype=np.float32) if u else None
        tot = np.zeros(4) if totals else None
        _check(self._lib.sc_fields(self._h, _ptr(r), _ptr(uu), _ptr(tot)))
        return r, uu, tot

    def fields_device(self, rho=None, u=None):
        """rho and u into caller-owned torch tensors on the sim's device (float32, contiguous,
        N and (d, N) elements); None skips one.  Returns (rho, u)."""
        import torch

        for t, n, name in ((rho, self.N, "rho"), (u, self.d * self.N, "u")):
            if t is None:
                continue
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and
                    t.is_contiguous() and t.numel() == n):
                raise ValueError(f"{name} must be a contiguous float32 device tensor of {n} "
                                 "elements")
        _check_disjoint(rho, u, "rho and u")
        # the tensors' pending work on the caller's stream comes first; the call itself returns
        # after the sim's stream has finished
        if self.mem is not None:
            self.mem.stream.wait_stream(torch.cuda.current_stream())
        else:
            torch.cuda.current_stream().synchronize()
        _check(self._lib.sc_fields_device(self._h, None if rho is None else rho.data_ptr(),
                                          None if u is None else u.data_ptr()))
        return rho, u

    def totals(self):
        return self.fields(rho=False, u=False, totals=True)[2]

    def laplacian_p(self):
        p = np.zeros(self.N)
        lap = np.zeros(self.N)
        _check(self._lib.sc_laplacian_p(self._h, _ptr(p), _ptr(lap)))
        return p, lap

    def laplacian_p_device(self, p=None, lap=None):
        """p and its lattice Laplacian into caller-owned float64 torch tensors of N elements on
        the sim's device; None skips one.  Returns (p, lap)."""
        import torch

        for t, name in ((p, "p"), (lap, "lap")):
            if t is None:
                continue
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and
                    t.is_contiguous() and t.numel() == self.N):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of "
                                 f"{self.N} elements")
        _check_disjoint(p, lap, "p and lap")
        if self.mem is not None:
            self.mem.stream.wait_stream(torch.cuda.current_stream())
        else:
            torch.cuda.current_stream().synchronize()
        _check(self._lib.sc_laplacian_p_device(self._h, None if p is None else p.data_ptr(),
                                               None if lap is None else lap.data_ptr()))
        return p, lap

    def label_bubbles(self, mask=None):
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        lab = np.zeros(self.N, dtype=np.uint32)
        nc = C.c_int64()
        _check(self._lib.sc_label_bubbles(self._h, _ptr(m), _ptr(lab), C.byref(nc)))
        return lab, nc.value

    def gas_density(self):
        """Density of the gas component (two-component mode; zeros otherwise)."""
        r = np.zeros(self.N, dtype=np.float32)
        _check(self._lib.sc_gas_density(self._h, _ptr(r)))
        return r

    def set_gas_equilibrium(self, rho_v):
        r = np.ascontiguousarray(rho_v, dtype=np.float64).reshape(self.N)
        _check(self._lib.sc_set_gas_equilibrium(self._h, _ptr(r)))

    def film_geometry(self, a, b):
        """(h, R_d, n_lines) of the bubbles holding nuclei a and b at the last test pass."""
        h, r, n = C.c_double(), C.c_double(), C.c_int32()
        _check(self._lib.sc_film_geometry(self._h, int(a), int(b), C.byref(h), C.byref(r),
                                          C.byref(n)))
        return h.value, r.value, n.value

    @property
    def rho0(self):
        """Buoyancy reference density of the gravity body force (0 when gravity is off)."""
        v = C.c_double()
        _check(self._lib.sc_buoyancy_density(self._h, C.byref(v)))
        return v.value

    def owner(self):
        """Owner field of the barrier (uint16, 0 = no bubble) as of the last test pass."""
        o = np.zeros(self.N, dtype=np.uint16)
        _check(self._lib.sc_owner(self._h, _ptr(o)))
        return o

    def last_labels(self):
        lab = np.zeros(self.N, dtype=np.uint32)
        _check(self._lib.sc_last_labels(self._h, _ptr(lab)))
        return lab

    def _list(self, fn, T, conv):
        n = C.c_int32()
        _check(fn(self._h, None, 0, C.byref(n)))
        arr = (T * max(n.value, 1))()
        _check(fn(self._h, C.cast(arr, C.c_void_p), n.value, C.byref(n)))
        return [conv(x) for x in arr[: n.value]]

    def merge_events(self):
        return self._list(self._lib.sc_merge_events, MergeEvent, lambda e: dict(
            step=e.step, nucleus_a=e.nucleus_a, nucleus_b=e.nucleus_b, label_a=e.label_a,
            label_b=e.label_b, film_node=e.film_node, film_len=e.film_len, lap_p=e.lap_p,
            rho_film=e.rho_film))

    def topo_events(self):
        return self._list(self._lib.sc_topo_events, TopoEvent, lambda e: dict(
            step=e.step, nucleus_a=e.nucleus_a, nucleus_b=e.nucleus_b))

    def bubbles(self):
        return self._list(self._lib.sc_bubbles, Bubble, lambda b: dict(
            label=b.label, nucleus=b.nucleus, n=b.n, centroid=tuple(b.centroid),
            radius=b.radius, n_nuclei=b.n_nuclei))

    def nuclei(self, n):
        comp = np.zeros(max(n, 1), dtype=np.uint32)
        rem = np.zeros(max(n, 1))
        _check(self._lib.sc_nuclei(self._h, _ptr(comp), _ptr(rem)))
        return comp[:n], rem[:n]

    def source_ledger(self):
        """(released, undelivered): agent mass the nuclei have given up, and the part of it the
        populations have not taken yet (FP64)."""
        rel, und = C.c_double(), C.c_double()
        _check(self._lib.sc_source_ledger(self._h, C.byref(rel), C.byref(und)))
        return rel.value, und.value

    def get_gas_populations(self):
        f = np.zeros((self.q, self.N))
        _check(self._lib.sc_get_gas_populations(self._h, _ptr(f)))
        return f

    def set_gas_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        _check(self._lib.sc_set_gas_populations(self._h, _ptr(f)))

    def get_populations(self):
        f = np.zeros((self.q, self.N))
        _check(self._lib.sc_get_populations(self._h, _ptr(f)))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        _check(self._lib.sc_set_populations(self._h, _ptr(f)))

    def set_equilibrium(self, rho, u=None):
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.N)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.d,
                                                                                     self.N)
        _check(self._lib.sc_set_equilibrium(self._h, _ptr(r), _ptr(uu)))

    def profile(self, enable=True):
        _check(self._lib.sc_profile(self._h, 1 if enable else 0))

    def profile_read(self, cls=SC_KERNEL_STEP):
        ms = C.c_double()
        n = C.c_int64()
        _check(self._lib.sc_profile_read(self._h, cls, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def step_config(self):
        v = [C.c_int32() for _ in range(4)]
        _check(self._lib.sc_step_config(self._h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def autotune(self, trials=5):
        """Times every step-kernel candidate on the current state, keeps the fastest."""
        cap = 128
        arr = (TuneEntry * cap)()
        n = C.c_int32()
        _check(self._lib.sc_autotune(self._h, int(trials), C.cast(arr, C.c_void_p), cap,
                                     C.byref(n)))
        return [dict(tile=(e.tile_x, e.tile_y, e.tile_z), variant=e.variant,
                     us=e.us_per_launch) for e in arr[: n.value]]

    def compute_type(self):
        v = C.c_int32()
        _check(self._lib.sc_compute_type(self._h, C.byref(v)))
        return {1: "f32", 2: "f64"}[v.value]

    @property
    def stream(self):
        return None if self.mem is None else self.mem.stream


class Batch:
    """Independent two-bubble D2Q9 boxes run by one persistent kernel (sc_batch_*)."""

    def __init__(self, spec, compute="auto", max_steps=None, memory="torch"):
        """spec: workloads.BatchSpec."""
        self._lib = load_library()
        self._h = None
        n = spec.n
        arr = (BatchInstance * n)()
        for k in range(n):
            s = spec.instance(k)
            I = arr[k]
            I.nx, I.ny, I.tau, I.G = s.nx, s.ny, s.tau, s.G
            I.rho_liquid, I.rho_gas, I.noise_amp, I.noise_seed = s.rho_l, s.rho_g, s.amp, s.seed
            I.gas_threshold = s.theta
            for b in range(2):
                for c in range(3):
                    I.centre[b][c] = float(s.centres[b][c])
                I.radius[b] = float(s.radii[b])
        self.n = n
        self.spec = spec
        self.mem = TorchMemory() if memory == "torch" else None
        stream = self.mem.stream.cuda_stream if self.mem else None
        alloc = C.pointer(self.mem.struct) if self.mem else None
        h = C.c_void_p()
        ms = spec.max_steps if max_steps is None else max_steps
        _check(self._lib.sc_batch_create(n, C.cast(arr, C.c_void_p), spec.K, spec.film_max, ms,
                                         COMPUTE[compute], stream, alloc, C.byref(h)))
        self._h = h

    def run(self):
        res = (BatchResult * self.n)()
        ms = C.c_double()
        _check(self._lib.sc_batch_run(self._h, C.cast(res, C.c_void_p), C.byref(ms)))
        out = [dict(merge_step=r.merge_step, topo_step=r.topo_step, steps_run=r.steps_run,
                    film_node=r.film_node, film_len=r.film_len, status=r.status, lap_p=r.lap_p,
                    rho_film=r.rho_film, totals=tuple(r.totals)) for r in res]
        return out, ms.value

    def tune(self, trial_steps=50):
        """Picks the rows per thread of the box step by timing a short run of every box."""
        rb = C.c_int32()
        ms = (C.c_double * 3)()
        _check(self._lib.sc_batch_tune(self._h, int(trial_steps), C.byref(rb),
                                       C.cast(ms, C.c_void_p)))
        return rb.value, list(ms)

    def density(self, k):
        nx, ny = int(self.spec.nx[k]), int(self.spec.ny[k])
        rho = np.zeros(nx * ny, dtype=np.float32)
        _check(self._lib.sc_batch_fields(self._h, int(k), _ptr(rho)))
        return rho

    def close(self):
        if self._h is not None:
            self._lib.sc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
