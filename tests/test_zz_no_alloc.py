"""sc_label_bubbles_noalloc, the allocation-free labelling entry point, against sc_label_bubbles.

Two calls in a row on different simulations, the second on a smaller box (the shared scratch
array keeps the first call's contents), each bit-exact against the allocating entry point; the
caching allocator's count does not move during the calls; boxes above the scratch's size and
buffers that are not device memory are refused before any kernel runs.  (A sub-buffer of a torch
segment is checked against the segment, as for sc_fields_device: the caller sizes it.)
"""
import ctypes as C

import numpy as np
import pytest

from paper_1708_01608_amd import sc

pytestmark = pytest.mark.gpu

MAX_NODES = 16777216


def _announce(msg):
    print(f"[gpu] {msg}", flush=True)


def _noalloc(g, mask_dev=None):
    import torch

    labels = torch.full((g.N,), -1, device="cuda", dtype=torch.int32)
    nc = C.c_int64(-1)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    rc = g._lib.sc_label_bubbles_noalloc(
        g._h, None if mask_dev is None else C.c_void_p(mask_dev.data_ptr()),
        C.c_void_p(labels.data_ptr()), C.byref(nc))
    after = torch.cuda.memory_allocated()
    assert rc == sc.SC_OK, g._lib.sc_last_error()
    assert after == before
    return labels.cpu().numpy().view(np.uint32), nc.value


def _foam_3d():
    g = sc.Sim(q=19, nx=48, ny=40, nz=36, tau=0.9, amp=1e-3, seed=4, K=0)
    rng = np.random.default_rng(11)
    centres = np.column_stack([rng.integers(0, 48, 7), rng.integers(0, 40, 7),
                               rng.integers(0, 36, 7)]).astype(float)
    g.seed_nuclei(centres, np.full(7, 6.0), np.zeros(7), 0.0)
    g.step(30)
    return g


def test_noalloc_labels_equal_the_allocating_entry_point():
    import torch

    _announce("noalloc labels: D3Q19 48x40x36 from rho, then D2Q9 37x23 from a device mask")
    g = _foam_3d()
    lab, nc = _noalloc(g)
    ref, nref = g.label_bubbles()
    assert nc == nref and nc >= 2
    assert np.array_equal(lab, ref)

    # second call: a smaller box and an explicit mask
    g2 = sc.Sim(q=9, nx=37, ny=23, K=0)
    rng = np.random.default_rng(5)
    mask = (rng.random(g2.N) < 0.45).astype(np.uint8)
    mask_dev = torch.from_numpy(mask).cuda()
    lab2, nc2 = _noalloc(g2, mask_dev)
    ref2, nref2 = g2.label_bubbles(mask)
    assert nc2 == nref2 and nc2 >= 2
    assert np.array_equal(lab2, ref2)

    # and the larger box again after the smaller one
    lab3, nc3 = _noalloc(g)
    assert nc3 == nref and np.array_equal(lab3, ref)


def test_noalloc_refuses_what_it_cannot_take():
    import torch

    _announce("noalloc refusals")
    g = sc.Sim(q=9, nx=32, ny=24, K=0)
    host = np.zeros(g.N, dtype=np.uint32)
    nc = C.c_int64()
    assert g._lib.sc_label_bubbles_noalloc(g._h, None, host.ctypes.data_as(C.c_void_p),
                                           C.byref(nc)) == sc.SC_E_INVAL
    # pinned host memory is reachable by the GPU (so even a missed check could not fault), but
    # it is not memory of the device
    pinned = torch.zeros(g.N, dtype=torch.int32, pin_memory=True)
    assert g._lib.sc_label_bubbles_noalloc(g._h, None, C.c_void_p(pinned.data_ptr()),
                                           C.byref(nc)) == sc.SC_E_INVAL
    assert not torch.any(pinned)
    assert g._lib.sc_label_bubbles_noalloc(g._h, None, None, C.byref(nc)) == sc.SC_E_INVAL
    # a box one row beyond the scratch's 16,777,216 nodes
    big = sc.Sim(q=9, nx=4096, ny=4097, K=0)
    assert big.N > MAX_NODES
    lab = torch.zeros(big.N, device="cuda", dtype=torch.int32)
    assert big._lib.sc_label_bubbles_noalloc(big._h, None, C.c_void_p(lab.data_ptr()),
                                             C.byref(nc)) == sc.SC_E_INVAL
    assert b"scratch" in big._lib.sc_last_error()
    big.close()
    # the handle stays usable
    _noalloc(g)
