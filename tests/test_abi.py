"""C-ABI contract checks that need no GPU: exports, struct layouts, validation errors."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1708_01608_amd import sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sc.LIB_PATH):
        from paper_1708_01608_amd import build
        build.build()
    return sc.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(sc.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version(lib):
    assert lib.sc_abi_version() == 2


def test_params_layout_and_defaults(lib):
    p = sc.Params()
    assert lib.sc_params_init(C.byref(p)) == sc.SC_OK
    assert p.abi_version == 2 and p.lattice == 9 and (p.nx, p.ny, p.nz) == (128, 128, 1)
    assert p.tau == 1.0 and p.G == -5.0 and p.rho_liquid == 1.93 and p.rho_gas == 0.16
    assert p.test_every == 10 and p.film_max == 8 and p.storage == 0 and p.rho_ref == -1.0


def _c_layout(tmp_path, struct, fields):
    """offsetof / sizeof of a struct of include/sc.h as the C compiler lays it out."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sc.h"', 'int main(void){']
    lines.append(f'printf("%zu\\n", sizeof({struct}));')
    for f in fields:
        lines.append(f'printf("%zu\\n", offsetof({struct}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct,ctype", [("sc_params", sc.Params), ("sc_merge_event", sc.MergeEvent),
                                          ("sc_topo_event", sc.TopoEvent), ("sc_bubble", sc.Bubble),
                                          ("sc_allocator", sc.Allocator),
                                          ("sc_batch_instance", sc.BatchInstance),
                                          ("sc_batch_result", sc.BatchResult),
                                          ("sc_tune_entry", sc.TuneEntry)])
def test_binding_structs_match_c_layout(tmp_path, struct, ctype):
    names = [f[0] for f in ctype._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert C.sizeof(ctype) == size
    assert [getattr(ctype, n).offset for n in names] == offs


@pytest.mark.parametrize("field,value", [
    ("abi_version", 7), ("lattice", 15), ("nx", 3), ("nz", 2), ("tau", 0.5), ("tau", float("nan")),
    ("rho_liquid", 0.0), ("noise_amp", -1.0), ("test_every", -1), ("film_max", 0),
    ("storage", 3), ("tile_x", 48),
])
def test_invalid_parameters_are_rejected_before_any_device_work(lib, field, value):
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    setattr(p, field, value)
    h = C.c_void_p()
    assert lib.sc_create(C.byref(p), C.byref(h)) == sc.SC_E_INVAL
    assert not h.value
    assert lib.sc_last_error()


@pytest.mark.parametrize("field,value,code", [
    ("corona", -1, sc.SC_E_INVAL), ("corona", 65, sc.SC_E_INVAL), ("barrier", 2, sc.SC_E_INVAL),
])
def test_barrier_parameters_are_checked(lib, field, value, code):
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    assert p.barrier == 0 and p.corona == 3
    p.barrier = 1
    setattr(p, field, value)
    h = C.c_void_p()
    assert lib.sc_create(C.byref(p), C.byref(h)) == code
    assert not h.value


@pytest.mark.parametrize("storage,compute,ok", [(1, 0, True), (2, 1, True), (1, 2, False)])
def test_barrier_on_16bit_storage_runs_fp32_arithmetic(lib, storage, compute, ok):
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    p.barrier, p.storage, p.compute = 1, storage, compute
    h = C.c_void_p()
    rc = lib.sc_create(C.byref(p), C.byref(h))
    if ok:
        assert rc in (sc.SC_OK, sc.SC_E_DEVICE, sc.SC_E_NOMEM)
        if h.value:
            lib.sc_destroy(h)
    else:
        assert rc == sc.SC_E_UNSUPPORTED and not h.value


@pytest.mark.parametrize("g,storage,variant,code", [
    ((float("nan"), 0.0, 0.0), 0, 0, sc.SC_E_INVAL), ((0.0, 1e-5, 0.0), 0, 2, sc.SC_E_UNSUPPORTED),
    ((0.0, 1e-5, 0.0), 2, 0, None), ((0.0, 0.0, -1e-5), 1, 3, None),
])
def test_gravity_parameters_are_checked(lib, g, storage, variant, code):
    # D3Q19 (the pipelined variant 2 exists there); any storage; None: accepted by validation
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    assert list(p.gravity) == [0.0, 0.0, 0.0] and p.rho_buoyancy == 0.0
    p.lattice, p.nx, p.ny, p.nz = 19, 32, 32, 32
    for c in range(3):
        p.gravity[c] = g[c]
    p.storage, p.step_variant = storage, variant
    if variant:
        p.tile_x, p.tile_y, p.tile_z = 32, 4, 8
    h = C.c_void_p()
    rc = lib.sc_create(C.byref(p), C.byref(h))
    if code is None:
        assert rc in (sc.SC_OK, sc.SC_E_DEVICE, sc.SC_E_NOMEM)
        if h.value:
            lib.sc_destroy(h)
    else:
        assert rc == code and not h.value


@pytest.mark.parametrize("field,value,code", [
    ("components", 3, sc.SC_E_INVAL), ("rho_vapour", 0.0, sc.SC_E_INVAL),
    ("tau_vapour", 0.5, sc.SC_E_INVAL), ("compute", 1, sc.SC_E_UNSUPPORTED),
    ("barrier", 1, sc.SC_E_UNSUPPORTED), ("step_variant", 2, sc.SC_E_INVAL),
    ("tile_x", 32, sc.SC_E_INVAL),
])
def test_two_component_parameters_are_checked(lib, field, value, code):
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    assert p.components == 1 and p.G_cross == 1.5 and p.rho_dissolved == 0.05
    p.components = 2
    setattr(p, field, value)
    h = C.c_void_p()
    assert lib.sc_create(C.byref(p), C.byref(h)) == code
    assert not h.value


@pytest.mark.parametrize("storage,compute,rho_ref,ok", [
    (0, 0, -1.0, True), (0, 2, 1.0, True), (0, 1, -1.0, False),
    (1, 0, -1.0, True), (2, 1, -1.0, True), (1, 2, -1.0, False), (2, 2, 1.0, False),
])
def test_two_component_storage_pairings(lib, storage, compute, rho_ref, ok):
    # FP32 storage runs FP64 arithmetic, 16-bit storage FP32 arithmetic; any shift is accepted
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    p.components, p.storage, p.compute, p.rho_ref = 2, storage, compute, rho_ref
    h = C.c_void_p()
    rc = lib.sc_create(C.byref(p), C.byref(h))
    if ok:
        assert rc in (sc.SC_OK, sc.SC_E_DEVICE, sc.SC_E_NOMEM)
        if h.value:
            lib.sc_destroy(h)
    else:
        assert rc == sc.SC_E_UNSUPPORTED and not h.value


def test_boxes_past_32bit_byte_offsets_are_rejected(lib):
    # 1024 x 1024 x 1025 FP32 values need byte offsets past 2^32
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    p.lattice, p.nx, p.ny, p.nz = 19, 1024, 1024, 1025
    h = C.c_void_p()
    assert lib.sc_create(C.byref(p), C.byref(h)) == sc.SC_E_INVAL
    assert b"2^32" in lib.sc_last_error()
    assert not h.value


def test_d3q19_needs_depth(lib):
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    p.lattice, p.nz = 19, 1
    h = C.c_void_p()
    assert lib.sc_create(C.byref(p), C.byref(h)) == sc.SC_E_INVAL


def test_null_handles(lib):
    assert lib.sc_step(None, 1) == sc.SC_E_INVAL
    assert lib.sc_destroy(None) == sc.SC_E_INVAL
    assert lib.sc_fields(None, None, None, None) == sc.SC_E_INVAL
    assert lib.sc_fields_device(None, None, None) == sc.SC_E_INVAL
    assert lib.sc_laplacian_p_device(None, None, None) == sc.SC_E_INVAL


@pytest.mark.parametrize("q", [9, 19])
def test_library_lattice_is_a_valid_velocity_set(lib, q):
    e, w = sc.lattice(q)
    d = 2 if q == 9 else 3
    assert len({tuple(v) for v in e}) == q
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ e[:, :d]).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, e[:, :d], e[:, :d]) - np.eye(d) / 3).max() < 1e-15
    # opposite pairs sit next to each other
    for i in range(1, q, 2):
        assert np.array_equal(e[i], -e[i + 1])


@pytest.mark.parametrize("q,tile,variant,ok", [
    (9, (64, 1, 8), 1, True), (9, (512, 1, 3), 3, True), (9, (32, 1, 8), 1, False),
    (9, (64, 1, 8), 4, False), (19, (32, 4, 16), 1, True), (19, (128, 4, 64), 3, True),
    (19, (64, 8, 16), 4, True), (19, (32, 4, 16), 5, True), (19, (32, 4, 16), 2, False),
    (19, (32, 4, 16), 6, False), (19, (256, 4, 64), 1, False), (19, (16, 16, 16), 1, False),
])
def test_two_component_tiles_are_checked(lib, q, tile, variant, ok):
    # the fused two-component kernels have their own shape set (both densities' rings in LDS);
    # variants 4 and 5 (one component per wave) exist in D3Q19 only
    p = sc.Params()
    lib.sc_params_init(C.byref(p))
    p.components, p.lattice = 2, q
    p.nx, p.ny, p.nz = 64, 64, (1 if q == 9 else 64)
    p.tile_x, p.tile_y, p.tile_z = tile
    p.step_variant = variant
    h = C.c_void_p()
    rc = lib.sc_create(C.byref(p), C.byref(h))
    if ok:
        # accepted by validation: on a host without a GPU creation fails at the device instead
        assert rc in (sc.SC_OK, sc.SC_E_DEVICE, sc.SC_E_NOMEM)
        if rc == sc.SC_OK:
            lib.sc_destroy(h)
    else:
        assert rc == sc.SC_E_INVAL


class _FakeTensor:
    """Stands in for a device tensor in the binding's host-side overlap check."""

    def __init__(self, ptr, n, size):
        self._p, self._n, self._s = ptr, n, size

    def data_ptr(self):
        return self._p

    def numel(self):
        return self._n

    def element_size(self):
        return self._s


def test_binding_refuses_overlapping_outputs():
    a = _FakeTensor(0x10000, 100, 8)
    sc._check_disjoint(a, _FakeTensor(0x10000 + 800, 100, 8), "p and lap")   # adjacent: fine
    sc._check_disjoint(a, None, "p and lap")
    for start in (0x10000, 0x10000 + 8, 0x10000 - 8 * 99, 0x10000 + 799):
        with pytest.raises(ValueError):
            sc._check_disjoint(a, _FakeTensor(start, 100, 8), "p and lap")


@pytest.mark.parametrize("args", [
    (0, 8, 8, 0, 8, 8, 4, 1), (8, 8, 8, 3, 8, 8, 4, 1), (8, 8, 8, 0, 64, 32, 4, 1),
    (8, 8, 8, 0, 8, 8, 0, 1), (8, 8, 8, 0, 8, 8, 4, 0),
    ((1 << 30) + 1, 1, 1, 1, 256, 1, 1, 1), (8, 65536, 1, 1, 8, 8, 1, 1),
    (1025, 1024, 1024, 0, 256, 4, 64, 1),
])
def test_pattern_probe_arguments_are_checked(lib, args):
    # rejected before any device call: empty box, unknown storage, tile above 1024 threads or
    # without planes, no timed repetition, an axis too long, more than 2^32 bytes per direction
    f, m = C.c_double(-1.0), C.c_double(-1.0)
    assert lib.sc_pattern_probe(*args, C.byref(f), C.byref(m)) == sc.SC_E_INVAL
    assert f.value == -1.0 and m.value == -1.0
