"""sc_fields_device: the reported fields written into caller-owned device memory equal the host
copies of sc_fields bit for bit; buffers that are not memory of the sim's device are refused."""
import ctypes as C

import numpy as np
import pytest

from paper_1708_01608_amd import sc

pytestmark = pytest.mark.gpu

TC = (1.5, 0.8, 1.0, 0.05)


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _sim(components, storage="f32"):
    kw = dict(q=19, nx=40, ny=24, nz=20, tau=0.9, amp=1e-3, seed=3, K=10, storage=storage)
    if components == 2:
        g = sc.Sim(G=0.0, rho_l=1.0, rho_g=0.05, two_component=TC, **kw)
    else:
        g = sc.Sim(**kw)
    g.seed_nuclei(np.array([[19.5, 11.5, 9.5], [2.0, 3.0, 1.0]]), np.array([6.0, 4.0]),
                  np.array([1e-2, 1e-2]), 1e-4)
    return g


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("components", [1, 2])
def test_fields_device_equals_fields(components, storage):
    import torch

    _announce(f"fields_device components={components} storage={storage}")
    g = _sim(components, storage)
    g.step(30)
    rho = torch.full((g.N,), float("nan"), device="cuda", dtype=torch.float32)
    u = torch.full((g.d, g.N), float("nan"), device="cuda", dtype=torch.float32)
    g.fields_device(rho, u)
    r_h, u_h, _ = g.fields()
    assert np.array_equal(rho.cpu().numpy(), r_h)
    assert np.array_equal(u.cpu().numpy(), u_h)
    # one output only
    rho2 = torch.zeros(g.N, device="cuda", dtype=torch.float32)
    g.fields_device(rho=rho2)
    assert np.array_equal(rho2.cpu().numpy(), r_h)


def test_fields_device_refuses_other_memory():
    import torch

    _announce("fields_device refusals")
    g = _sim(1)
    with pytest.raises(ValueError):
        g.fields_device(rho=torch.zeros(g.N, dtype=torch.float32))             # host tensor
    with pytest.raises(ValueError):
        g.fields_device(rho=torch.zeros(g.N - 1, device="cuda", dtype=torch.float32))
    with pytest.raises(ValueError):
        g.fields_device(u=torch.zeros(g.N, device="cuda", dtype=torch.float32))  # d x N needed
    # through the C ABI: pinned host memory (reachable by the GPU, so even a missed check could
    # not fault) is not memory of the device, and the library says so before any kernel runs
    pinned = torch.zeros(g.N, dtype=torch.float32, pin_memory=True)
    rc = g._lib.sc_fields_device(g._h, C.c_void_p(pinned.data_ptr()), None)
    assert rc == sc.SC_E_INVAL
    assert b"device" in g._lib.sc_last_error()
    assert not torch.any(pinned)
    g.step(5)  # the handle stays usable


@pytest.mark.parametrize("components", [1, 2])
def test_laplacian_p_device_equals_host(components):
    import torch

    _announce(f"laplacian_p_device components={components}")
    g = _sim(components)
    g.step(20)
    p_h, lap_h = g.laplacian_p()
    p = torch.full((g.N,), float("nan"), device="cuda", dtype=torch.float64)
    lap = torch.full((g.N,), float("nan"), device="cuda", dtype=torch.float64)
    g.laplacian_p_device(p, lap)
    assert np.array_equal(p.cpu().numpy(), p_h) and np.array_equal(lap.cpu().numpy(), lap_h)
    lap2 = torch.zeros(g.N, device="cuda", dtype=torch.float64)
    g.laplacian_p_device(lap=lap2)  # the Laplacian alone
    assert np.array_equal(lap2.cpu().numpy(), lap_h)
    with pytest.raises(ValueError):
        g.laplacian_p_device(p=torch.zeros(g.N, device="cuda", dtype=torch.float32))


def test_device_outputs_that_overlap_are_refused():
    import torch

    _announce("device outputs overlap")
    g = _sim(1)
    g.step(5)
    buf = torch.zeros(2 * g.N, device="cuda", dtype=torch.float64)
    # the same memory as p and lap: refused by the binding and, underneath it, by the library
    with pytest.raises(ValueError):
        g.laplacian_p_device(buf[: g.N], buf[: g.N])
    rc = g._lib.sc_laplacian_p_device(g._h, C.c_void_p(buf.data_ptr()),
                                      C.c_void_p(buf.data_ptr() + 8 * (g.N // 2)))
    assert rc == sc.SC_E_INVAL and b"overlap" in g._lib.sc_last_error()
    assert not torch.any(buf)
    f = torch.zeros((g.d + 1) * g.N, device="cuda", dtype=torch.float32)
    rc = g._lib.sc_fields_device(g._h, C.c_void_p(f.data_ptr() + 4), C.c_void_p(f.data_ptr()))
    assert rc == sc.SC_E_INVAL and b"overlap" in g._lib.sc_last_error()
    # adjacent, disjoint halves are fine
    g.laplacian_p_device(buf[: g.N], buf[g.N:])
    p_h, lap_h = g.laplacian_p()
    assert np.array_equal(buf[: g.N].cpu().numpy(), p_h)
    assert np.array_equal(buf[g.N:].cpu().numpy(), lap_h)
