"""The C-ABI library loads and exports every symbol include/dpd.h declares;
host-side validation rejects bad inputs before any device work.  No GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1807_09896_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libdpdphi.so is not built; run __graft_entry__.build()")
    return binding.load_library()


def test_exports_every_declared_symbol(lib):
    from paper_1807_09896_amd import binding
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == names


def test_kernel_names_and_error_text(lib):
    for i in range(9):
        assert lib.dpd_kernel_name(i)
    assert lib.dpd_kernel_name(9) == b""
    assert isinstance(lib.dpd_last_error(None), bytes)


def _create(lib, L=(6.0, 6.0, 6.0), n=4, gid=None, a=(25, 25, 25, 25), rc=1.0, dt=0.01,
            pos=None, types=None, grid_n=(12, 12, 12), h=0.5):
    from paper_1807_09896_amd import binding as b
    pos = np.full((n, 3), 1.0, np.float32) if pos is None else pos
    pos[:, 0] = np.linspace(0.5, 5.0, n)
    vel = np.zeros((n, 3), np.float32)
    typ = np.zeros(n, np.int32) if types is None else types
    parts = b.dpd_particles(n, pos.ctypes.data, vel.ctypes.data, typ.ctypes.data,
                            gid.ctypes.data if gid is not None else None, 0)
    phi = np.ones(grid_n[::-1], np.float32)
    grid = b.dpd_phi_grid((C.c_int32 * 3)(*grid_n), (C.c_double * 3)(h, h, h), 4,
                          phi.ctypes.data, 0)
    box = b.dpd_box((C.c_double * 3)(*L))
    prm = b.dpd_params((C.c_double * 4)(*a), 4.5, 1.0, rc, dt, 0.65, (C.c_double * 3)(0, 0, 0),
                       1, 0, 0)
    ctx = C.c_void_p()
    rc_ = lib.dpd_create(C.byref(box), C.byref(parts), C.byref(prm), C.byref(grid), None, None,
                         C.byref(ctx))
    return rc_, ctx


def test_host_validation_rejects_bad_inputs(lib):
    from paper_1807_09896_amd.binding import DPD_E_INVAL
    rc, ctx = _create(lib, gid=np.array([0, 1, 1, 2], np.uint32))
    assert rc == DPD_E_INVAL and ctx.value is None
    assert b"permutation" in lib.dpd_last_error(None)
    rc, _ = _create(lib, L=(2.5, 6.0, 6.0), grid_n=(5, 12, 12))
    assert rc == DPD_E_INVAL and b"3 cells" in lib.dpd_last_error(None)
    rc, _ = _create(lib, a=(25, 25, 30, 25))
    assert rc == DPD_E_INVAL and b"symmetric" in lib.dpd_last_error(None)
    rc, _ = _create(lib, dt=0.0)
    assert rc == DPD_E_INVAL
    rc, _ = _create(lib, grid_n=(10, 12, 12))
    assert rc == DPD_E_INVAL and b"n*h" in lib.dpd_last_error(None)
    bad = np.full((4, 3), 1.0, np.float32)
    bad[2, 1] = 7.0
    rc, _ = _create(lib, pos=bad)
    assert rc == DPD_E_INVAL and b"outside" in lib.dpd_last_error(None)
    rc, _ = _create(lib, types=np.array([0, 2, 0, 0], np.int32))
    assert rc == DPD_E_INVAL


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1807_09896_amd.binding import DPD_E_DEVICE
    rc, ctx = _create(lib)
    assert rc == DPD_E_DEVICE and ctx.value is None


def test_null_handles_are_rejected(lib):
    assert lib.dpd_step(None, 1) != 0
    assert lib.dpd_sync(None) != 0
    lib.dpd_destroy(None)
