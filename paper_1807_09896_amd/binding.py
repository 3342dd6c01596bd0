"""ctypes binding of libdpdphi.so (include/dpd.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Functions carry the C names; device buffers are torch tensors
on the current HIP device and the library runs on torch's current stream.
There is no CPU fallback: without the built library or a gfx950 device every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DPD_LIB overrides the library path (e.g. to compare builds of the kernels)
LIB_PATH = os.environ.get("DPD_LIB") or os.path.join(_HERE, "libdpdphi.so")

DPD_OK = 0
DPD_E_INVAL = -1
DPD_E_NOMEM = -2
DPD_E_DEVICE = -3
DPD_E_UNSTABLE = -4
DPD_E_STATE = -5
DPD_FLAG_NO_MASK = 1
DPD_FLAG_SPECULAR = 2
DPD_FLAG_SPH = 4
DPD_NUM_KERNELS = 9

_ERRNAMES = {DPD_E_INVAL: "DPD_E_INVAL", DPD_E_NOMEM: "DPD_E_NOMEM",
             DPD_E_DEVICE: "DPD_E_DEVICE", DPD_E_UNSTABLE: "DPD_E_UNSTABLE",
             DPD_E_STATE: "DPD_E_STATE"}

# Every exported symbol declared in include/dpd.h.
EXPORTED = ["dpd_create", "dpd_step", "dpd_forces", "dpd_get_state", "dpd_set_state",
            "dpd_neighbor_pairs", "dpd_profile", "dpd_counters", "dpd_kernel_times",
            "dpd_kernel_name", "dpd_sync", "dpd_last_error", "dpd_destroy", "dpd_copy_probe",
            "dpd_pair_random", "dpd_batch_create", "dpd_replica_count", "dpd_replica_forces",
            "dpd_replica_state", "dpd_replica_set_state", "dpd_replica_pairs",
            "dpd_replica_profile", "dpd_use_graph", "dpd_autotune", "dpd_set_params",
            "dpd_set_phi", "dpd_window_forward", "dpd_backward", "dpd_phi_relax",
            "dpd_snapshot_size", "dpd_snapshot_io", "dpd_valu_probe", "dpd_phi_relax_static",
            "dpd_window_trace", "dpd_use_persistent"]


class DPDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, str(code)), msg))
        self.code = code


class dpd_box(C.Structure):
    _fields_ = [("L", C.c_double * 3)]


class dpd_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("vel", C.c_void_p),
                ("type", C.c_void_p), ("gid", C.c_void_p), ("on_device", C.c_int32)]


class dpd_phi_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3), ("dtype", C.c_int32),
                ("data", C.c_void_p), ("on_device", C.c_int32)]


class dpd_params(C.Structure):
    _fields_ = [("a", C.c_double * 4), ("gamma", C.c_double), ("kBT", C.c_double),
                ("rc", C.c_double), ("dt", C.c_double), ("lambda_", C.c_double),
                ("g", C.c_double * 3), ("seed", C.c_uint64), ("replica", C.c_uint32),
                ("flags", C.c_int32), ("sr", C.c_double * 4), ("sa", C.c_double * 4),
                ("r0r", C.c_double), ("r0a", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class dpd_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libdpdphi.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1807_09896_amd.build)")
    L = C.CDLL(path)
    P = C.c_void_p
    L.dpd_create.argtypes = [P, P, P, P, P, P, C.POINTER(P)]
    L.dpd_create.restype = C.c_int
    L.dpd_step.argtypes = [P, C.c_int64]
    L.dpd_step.restype = C.c_int
    L.dpd_forces.argtypes = [P, P]
    L.dpd_forces.restype = C.c_int
    L.dpd_get_state.argtypes = [P, P, P, P, P]
    L.dpd_get_state.restype = C.c_int
    L.dpd_set_state.argtypes = [P, P, P, P, C.c_uint64, C.c_int32]
    L.dpd_set_state.restype = C.c_int
    L.dpd_neighbor_pairs.argtypes = [P, P, C.c_int64, C.POINTER(C.c_int64)]
    L.dpd_neighbor_pairs.restype = C.c_int
    L.dpd_profile.argtypes = [P, C.c_int32, C.c_int32, P]
    L.dpd_profile.restype = C.c_int
    L.dpd_counters.argtypes = [P, P]
    L.dpd_counters.restype = C.c_int
    L.dpd_kernel_times.argtypes = [P, C.c_int32, P, P]
    L.dpd_kernel_times.restype = C.c_int
    L.dpd_kernel_name.argtypes = [C.c_int32]
    L.dpd_kernel_name.restype = C.c_char_p
    L.dpd_sync.argtypes = [P]
    L.dpd_sync.restype = C.c_int
    L.dpd_last_error.argtypes = [P]
    L.dpd_last_error.restype = C.c_char_p
    L.dpd_destroy.argtypes = [P]
    L.dpd_destroy.restype = None
    L.dpd_copy_probe.argtypes = [P, P, C.c_size_t, P]
    L.dpd_copy_probe.restype = C.c_int
    L.dpd_snapshot_size.argtypes = [P]
    L.dpd_snapshot_size.restype = C.c_int64
    L.dpd_snapshot_io.argtypes = [P, C.c_int32, P]
    L.dpd_snapshot_io.restype = C.c_int
    L.dpd_phi_relax.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double), P]
    L.dpd_phi_relax.restype = C.c_int
    L.dpd_phi_relax_static.argtypes = [P, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.c_double, C.c_double, C.c_int32,
                                       C.POINTER(C.c_double), P]
    L.dpd_phi_relax_static.restype = C.c_int
    L.dpd_window_trace.argtypes = [P, P, P, P, P]
    L.dpd_window_trace.restype = C.c_int
    L.dpd_valu_probe.argtypes = [C.c_int32, C.c_int64, C.c_int32, P, P]
    L.dpd_valu_probe.restype = C.c_int
    L.dpd_pair_random.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, P, P, C.c_int64, P, P, P]
    L.dpd_pair_random.restype = C.c_int
    L.dpd_batch_create.argtypes = [C.c_int32, P, P, P, P, P, P, C.POINTER(P)]
    L.dpd_batch_create.restype = C.c_int
    L.dpd_replica_count.argtypes = [P]
    L.dpd_replica_count.restype = C.c_int
    L.dpd_replica_forces.argtypes = [P, C.c_int32, P]
    L.dpd_replica_forces.restype = C.c_int
    L.dpd_replica_state.argtypes = [P, C.c_int32, P, P, P, P]
    L.dpd_replica_state.restype = C.c_int
    L.dpd_replica_set_state.argtypes = [P, C.c_int32, P, P, P, C.c_uint64, C.c_int32]
    L.dpd_replica_set_state.restype = C.c_int
    L.dpd_replica_pairs.argtypes = [P, C.c_int32, P, C.c_int64, C.POINTER(C.c_int64)]
    L.dpd_replica_pairs.restype = C.c_int
    L.dpd_replica_profile.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
    L.dpd_replica_profile.restype = C.c_int
    L.dpd_use_graph.argtypes = [P, C.c_int32]
    L.dpd_use_graph.restype = C.c_int
    L.dpd_use_persistent.argtypes = [P, C.c_int32]
    L.dpd_use_persistent.restype = C.c_int
    L.dpd_autotune.argtypes = [P, C.c_int32, P, P]
    L.dpd_autotune.restype = C.c_int
    L.dpd_set_params.argtypes = [P, C.c_int32, P]
    L.dpd_set_params.restype = C.c_int
    L.dpd_set_phi.argtypes = [P, C.c_int32, P, C.c_int32]
    L.dpd_set_phi.restype = C.c_int
    L.dpd_window_forward.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
    L.dpd_window_forward.restype = C.c_int
    L.dpd_backward.argtypes = [P, P, P, P]
    L.dpd_backward.restype = C.c_int
    _lib = L
    return L


def _check(rc, ctx=None):
    if rc != DPD_OK:
        msg = load_library().dpd_last_error(ctx).decode()
        raise DPDError(rc, msg)


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    return C.c_void_p(t.ctypes.data)


class TorchAllocator:
    """dpd_allocator backed by torch's caching allocator on one device."""

    def __init__(self, device):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = dpd_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, user):
        t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _do_free(self, ptr, stream, user):
        self.live.pop(int(ptr or 0), None)


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# C-named entry points (thin marshalling)
# ---------------------------------------------------------------------------

def _marshal_box(L, pos, vel, type_, gid, params, phi, h, flags, keep):
    """ctypes structs of one box (host arrays are copied into `keep`)."""
    on_dev = int(hasattr(pos, "data_ptr"))
    n = int(pos.shape[0])

    def host(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    if on_dev:
        ppos, pvel, ptyp = pos, vel, type_
        pgid = gid
    else:
        ppos = host(pos, np.float32)
        pvel = host(vel, np.float32)
        ptyp = host(type_, np.int32)
        pgid = host(gid, np.uint32) if gid is not None else None
    parts = dpd_particles(n, _ptr(ppos), _ptr(pvel), _ptr(ptyp), _ptr(pgid), on_dev)
    box = dpd_box((C.c_double * 3)(*[float(x) for x in L]))
    phi_a = phi if hasattr(phi, "data_ptr") else np.ascontiguousarray(phi)
    if not hasattr(phi, "data_ptr"):
        keep.append(phi_a)
    dt = 8 if phi_a.dtype in (np.float64,) or str(phi_a.dtype) == "torch.float64" else 4
    nz, ny, nx = (int(x) for x in phi_a.shape)
    grid = dpd_phi_grid((C.c_int32 * 3)(nx, ny, nz), (C.c_double * 3)(*[float(x) for x in h]),
                        dt, _ptr(phi_a), int(hasattr(phi, "data_ptr")))
    return box, parts, _params_struct(params, flags), grid


def _params_struct(params, flags=0):
    """dpd_params from a parameter dict; a true params["specular"] adds
    DPD_FLAG_SPECULAR to flags, a params["sph"] dict (sr, sa, r0r, r0a)
    DPD_FLAG_SPH with its fields."""
    a = params["a"]
    if params.get("specular", False):
        flags = int(flags) | DPD_FLAG_SPECULAR
    sph = params.get("sph")
    sr = sa = ((0.0, 0.0), (0.0, 0.0))
    r0r = r0a = 0.0
    if sph:
        flags = int(flags) | DPD_FLAG_SPH
        sr, sa, r0r, r0a = sph["sr"], sph["sa"], sph["r0r"], sph["r0a"]
    return dpd_params((C.c_double * 4)(a[0][0], a[0][1], a[1][0], a[1][1]), params["gamma"],
                      params["kBT"], params["rc"], params["dt"], params["lam"],
                      (C.c_double * 3)(*params["g"]),
                      int(params["seed"]) & 0xFFFFFFFFFFFFFFFF, int(params["replica"]),
                      int(flags), (C.c_double * 4)(sr[0][0], sr[0][1], sr[1][0], sr[1][1]),
                      (C.c_double * 4)(sa[0][0], sa[0][1], sa[1][0], sa[1][1]), float(r0r),
                      float(r0a))


def dpd_create(L, pos, vel, type_, gid, params, phi, h, stream=None, use_torch_allocator=True,
               flags=0):
    """Create a context from host numpy arrays (or device tensors).

    params: dict with a (2x2), gamma, kBT, rc, dt, lam, g, seed, replica.
    phi: (nz, ny, nx) float32/float64 array; h: grid spacing (3,).
    Returns (ctx handle, keepalive) where keepalive must outlive the context.
    """
    import torch
    lib = load_library()
    if not torch.cuda.is_available():
        raise DPDError(DPD_E_DEVICE, "no HIP device visible to torch")
    keep = []
    box, parts, prm, grid = _marshal_box(L, pos, vel, type_, gid, params, phi, h, flags, keep)
    alloc = None
    if use_torch_allocator:
        alloc = TorchAllocator(torch.device("cuda", torch.cuda.current_device()))
        keep.append(alloc)
    ctx = C.c_void_p()
    rc = lib.dpd_create(C.byref(box), C.byref(parts), C.byref(prm), C.byref(grid),
                        C.byref(alloc.struct) if alloc else None, _stream_handle(stream),
                        C.byref(ctx))
    _check(rc, None)
    return ctx, keep


def dpd_batch_create(boxes, stream=None, use_torch_allocator=True, flags=0):
    """Create a batch context from a list of boxes, each a tuple
    (L, pos, vel, type, gid, params, phi, h) as taken by dpd_create.
    Returns (ctx handle, keepalive)."""
    import torch
    lib = load_library()
    if not torch.cuda.is_available():
        raise DPDError(DPD_E_DEVICE, "no HIP device visible to torch")
    nb = len(boxes)
    keep = []
    B = (dpd_box * nb)()
    Pp = (dpd_particles * nb)()
    Pr = (dpd_params * nb)()
    G = (dpd_phi_grid * nb)()
    for r, b in enumerate(boxes):
        B[r], Pp[r], Pr[r], G[r] = _marshal_box(*b, flags, keep)
    keep += [B, Pp, Pr, G]
    alloc = None
    if use_torch_allocator:
        alloc = TorchAllocator(torch.device("cuda", torch.cuda.current_device()))
        keep.append(alloc)
    ctx = C.c_void_p()
    rc = lib.dpd_batch_create(nb, B, Pp, Pr, G, C.byref(alloc.struct) if alloc else None,
                              _stream_handle(stream), C.byref(ctx))
    _check(rc, None)
    return ctx, keep


def dpd_replica_count(ctx):
    rc = load_library().dpd_replica_count(ctx)
    if rc < 0:
        _check(rc, ctx)
    return rc


def dpd_replica_forces(ctx, r, f_out):
    _check(load_library().dpd_replica_forces(ctx, int(r), _ptr(f_out)), ctx)


def dpd_replica_state(ctx, r, pos=None, vel=None, events=None, cell_of=None):
    _check(load_library().dpd_replica_state(ctx, int(r), _ptr(pos), _ptr(vel), _ptr(events),
                                            _ptr(cell_of)), ctx)


def dpd_replica_set_state(ctx, r, pos, vel, force, k):
    on_dev = int(hasattr(pos, "data_ptr"))
    if not on_dev:
        pos = np.ascontiguousarray(pos, np.float32)
        vel = np.ascontiguousarray(vel, np.float32)
        force = np.ascontiguousarray(force, np.float32)
    _check(load_library().dpd_replica_set_state(ctx, int(r), _ptr(pos), _ptr(vel), _ptr(force),
                                                int(k), on_dev), ctx)


def dpd_replica_pairs(ctx, r, pairs, cap):
    cnt = C.c_int64(0)
    _check(load_library().dpd_replica_pairs(ctx, int(r), _ptr(pairs), int(cap), C.byref(cnt)),
           ctx)
    return int(cnt.value)


def dpd_replica_profile(ctx, r, axis, nbins, out):
    _check(load_library().dpd_replica_profile(ctx, int(r), int(axis), int(nbins), _ptr(out)), ctx)


def dpd_use_graph(ctx, enable):
    _check(load_library().dpd_use_graph(ctx, int(enable)), ctx)


def dpd_use_persistent(ctx, enable):
    _check(load_library().dpd_use_persistent(ctx, int(enable)), ctx)


def dpd_autotune(ctx, steps):
    """Returns ((particles per thread, force block), ms per step of the four trials)."""
    shape = np.zeros(2, np.int32)
    ms = np.zeros(4, np.float64)
    _check(load_library().dpd_autotune(ctx, int(steps), _ptr(shape), _ptr(ms)), ctx)
    return (int(shape[0]), int(shape[1])), [float(x) for x in ms]


def dpd_step(ctx, n):
    _check(load_library().dpd_step(ctx, int(n)), ctx)


def dpd_forces(ctx, f_out):
    _check(load_library().dpd_forces(ctx, _ptr(f_out)), ctx)


def dpd_get_state(ctx, pos=None, vel=None, events=None, cell_of=None):
    _check(load_library().dpd_get_state(ctx, _ptr(pos), _ptr(vel), _ptr(events), _ptr(cell_of)), ctx)


def dpd_set_state(ctx, pos, vel, force, k):
    on_dev = int(hasattr(pos, "data_ptr"))
    if not on_dev:
        pos = np.ascontiguousarray(pos, np.float32)
        vel = np.ascontiguousarray(vel, np.float32)
        force = np.ascontiguousarray(force, np.float32)
    _check(load_library().dpd_set_state(ctx, _ptr(pos), _ptr(vel), _ptr(force), int(k), on_dev), ctx)


def dpd_neighbor_pairs(ctx, pairs, cap):
    cnt = C.c_int64(0)
    _check(load_library().dpd_neighbor_pairs(ctx, _ptr(pairs), int(cap), C.byref(cnt)), ctx)
    return int(cnt.value)


def dpd_profile(ctx, axis, nbins, out):
    _check(load_library().dpd_profile(ctx, int(axis), int(nbins), _ptr(out)), ctx)


def dpd_counters(ctx):
    out = np.zeros(10, np.int64)
    _check(load_library().dpd_counters(ctx, _ptr(out)), ctx)
    keys = ["steps", "k", "bounce", "fallback", "n_fluid", "n_wall", "cells", "mask_cells",
            "phi_lookups", "unstable"]
    return dict(zip(keys, (int(x) for x in out)))


def dpd_kernel_times(ctx, enable):
    ms = np.zeros(DPD_NUM_KERNELS, np.float64)
    cnt = np.zeros(DPD_NUM_KERNELS, np.int64)
    _check(load_library().dpd_kernel_times(ctx, int(enable), _ptr(ms), _ptr(cnt)), ctx)
    lib = load_library()
    return {lib.dpd_kernel_name(i).decode(): (float(ms[i]), int(cnt[i]))
            for i in range(DPD_NUM_KERNELS)}


def dpd_sync(ctx):
    _check(load_library().dpd_sync(ctx), ctx)


def dpd_last_error(ctx=None):
    return load_library().dpd_last_error(ctx).decode()


def dpd_destroy(ctx):
    load_library().dpd_destroy(ctx)


def dpd_copy_probe(dst, src, nbytes, stream=None):
    _check(load_library().dpd_copy_probe(_ptr(dst), _ptr(src), int(nbytes), _stream_handle(stream)))


def dpd_snapshot_size(ctx):
    n = load_library().dpd_snapshot_size(ctx)
    if n < 0:
        _check(int(n), ctx)
    return int(n)


def dpd_snapshot_io(ctx, dir_, blob):
    """dir_ 0 writes the context state into blob (a writable host uint8
    numpy array of dpd_snapshot_size bytes), 1 restores it from blob."""
    if blob.dtype != np.uint8 or not blob.flags["C_CONTIGUOUS"] or blob.nbytes < dpd_snapshot_size(ctx):
        raise ValueError("blob must be a contiguous uint8 array of dpd_snapshot_size bytes")
    _check(load_library().dpd_snapshot_io(ctx, int(dir_), C.c_void_p(blob.ctypes.data)), ctx)


def dpd_phi_relax(phi, work, h, eps, dtau, iters, residual=True, stream=None):
    """phi: contiguous device tensor (nz, ny, nx) of float32 or float64,
    relaxed in place; work: device tensor of the same dtype with at least
    phi.numel() + 1 elements.  Returns the last step's max |d phi / d t'|
    (synchronising) or None when residual is False."""
    import torch
    if phi.dim() != 3 or not phi.is_contiguous() or phi.dtype not in (torch.float32, torch.float64):
        raise ValueError("phi must be a contiguous (nz, ny, nx) float32 or float64 tensor")
    if work.dtype != phi.dtype or work.numel() < phi.numel() + 1 or not work.is_contiguous():
        raise ValueError("work must be contiguous, of phi's dtype, with phi.numel() + 1 elements")
    n = (C.c_int32 * 3)(int(phi.shape[2]), int(phi.shape[1]), int(phi.shape[0]))
    hh = (C.c_double * 3)(*[float(x) for x in h])
    res = C.c_double(0.0)
    _check(load_library().dpd_phi_relax(_ptr(phi), _ptr(work), int(phi.element_size()), n, hh,
                                        float(eps), float(dtau), int(iters),
                                        C.byref(res) if residual else None,
                                        _stream_handle(stream)))
    return res.value if residual else None


def dpd_phi_relax_static(phi, h, eps, dtau, iters, residual=True, stream=None):
    """dpd_phi_relax without a workspace: the library's static device scratch
    holds the ping-pong buffer (grids up to 64 MiB)."""
    import torch
    if phi.dim() != 3 or not phi.is_contiguous() or phi.dtype not in (torch.float32, torch.float64):
        raise ValueError("phi must be a contiguous (nz, ny, nx) float32 or float64 tensor")
    n = (C.c_int32 * 3)(int(phi.shape[2]), int(phi.shape[1]), int(phi.shape[0]))
    hh = (C.c_double * 3)(*[float(x) for x in h])
    res = C.c_double(0.0)
    _check(load_library().dpd_phi_relax_static(_ptr(phi), int(phi.element_size()), n, hh,
                                               float(eps), float(dtau), int(iters),
                                               C.byref(res) if residual else None,
                                               _stream_handle(stream)))
    return res.value if residual else None


def dpd_window_trace(ctx, pos_log=None, vel_log=None, frc_log=None, ev_log=None):
    """States (steps + 1, n, 3 float32: the window's start, then after each
    step) and event codes (steps, n int32) of the recorded window, in gid
    order (device tensors, any may be None)."""
    _check(load_library().dpd_window_trace(ctx, _ptr(pos_log), _ptr(vel_log), _ptr(frc_log),
                                           _ptr(ev_log)), ctx)


def dpd_valu_probe(kind, waves, iters, out, stream=None):
    """Run the VALU calibration kernel (see include/dpd.h); out: float32
    device tensor of waves * 64 elements."""
    if out.numel() < waves * 64:
        raise ValueError("out needs waves * 64 elements")
    _check(load_library().dpd_valu_probe(int(kind), int(waves), int(iters), _ptr(out),
                                         _stream_handle(stream)))


def dpd_pair_random(seed, k, replica, gi, gj, words=None, xi=None, stream=None):
    n = int(gi.shape[0])
    _check(load_library().dpd_pair_random(int(seed) & 0xFFFFFFFFFFFFFFFF, int(k), int(replica),
                                          _ptr(gi), _ptr(gj), n, _ptr(words), _ptr(xi),
                                          _stream_handle(stream)))


def dpd_set_params(ctx, r, params, flags=0):
    prm = _params_struct(params, flags)
    _check(load_library().dpd_set_params(ctx, int(r), C.byref(prm)), ctx)


def dpd_set_phi(ctx, r, phi):
    """phi: device tensor or host array of the create-time shape and dtype."""
    on_dev = int(hasattr(phi, "data_ptr"))
    if not on_dev:
        phi = np.ascontiguousarray(phi)
    _check(load_library().dpd_set_phi(ctx, int(r), _ptr(phi), on_dev), ctx)


def dpd_window_forward(ctx, steps, ckpt, axis, nbins, profile=None, counts=None):
    _check(load_library().dpd_window_forward(ctx, int(steps), int(ckpt), int(axis), int(nbins),
                                             _ptr(profile), _ptr(counts)), ctx)


def dpd_backward(ctx, dl_dprofile, dl_dphi=None):
    """Returns dL/d{a_ff, a_fw, gamma, g_x, g_y, g_z} (host float64[6])."""
    grads = np.zeros(6, np.float64)
    _check(load_library().dpd_backward(ctx, _ptr(dl_dprofile), _ptr(grads), _ptr(dl_dphi)), ctx)
    return grads
