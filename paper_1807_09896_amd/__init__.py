"""DPD time step with phase-field no-slip walls on MI355X (gfx950).

The method (Xu & Meakin): fluid DPD particles and frozen wall particles
interact by the conservative, dissipative and random pair forces (Sec. II.A,
Eq. 3-10) and are advanced by the Groot-Warren modified velocity-Verlet; a
fluid particle whose new position has phase field phi < 0 is bounced back
(Sec. II.C, Eq. 16-17).  The hot path runs in the HIP kernels of
libdpdphi.so behind the C ABI of include/dpd.h; this package is its Python
binding.
"""
from __future__ import annotations

import numpy as np

from . import binding
from .binding import (DPDError, dpd_autotune, dpd_batch_create, dpd_counters, dpd_create,
                      dpd_destroy, dpd_forces, dpd_get_state, dpd_kernel_times, dpd_last_error,
                      dpd_neighbor_pairs, dpd_profile, dpd_replica_count, dpd_replica_forces,
                      dpd_replica_pairs, dpd_replica_profile, dpd_replica_set_state,
                      dpd_phi_relax, dpd_replica_state, dpd_set_state, dpd_step, dpd_sync,
                      dpd_use_graph, dpd_use_persistent, load_library)

__all__ = ["Simulation", "DPDError", "load_library", "dpd_create", "dpd_batch_create",
           "dpd_step", "dpd_forces", "dpd_get_state", "dpd_set_state", "dpd_neighbor_pairs",
           "dpd_profile", "dpd_counters", "dpd_kernel_times", "dpd_sync", "dpd_last_error",
           "dpd_destroy", "dpd_replica_count", "dpd_replica_forces", "dpd_replica_state",
           "dpd_replica_set_state", "dpd_replica_pairs", "dpd_replica_profile",
           "dpd_use_graph", "dpd_use_persistent", "dpd_autotune", "dpd_phi_relax", "relax_phi"]


def relax_phi(phi, h, eps, dtau, iters, stream=None):
    """Relax a phase field on the GPU by Eq. 15 (Sec. II.B): `iters` explicit
    Euler steps of length dtau in the pseudo time, in place on the device
    tensor phi (nz, ny, nx).  Returns the last step's max |d phi / d t'|."""
    import torch
    work = torch.empty(phi.numel() + 1, dtype=phi.dtype, device=phi.device)
    return dpd_phi_relax(phi, work, h, eps, dtau, iters, residual=True, stream=stream)


def _box_args(system, params=None):
    return (system.L, system.pos, system.vel, system.type, system.gid,
            dict(system.params if params is None else params), system.phi, system.h)


class Simulation:
    """One box, or a batch of independent boxes, on the GPU.

    `system` is any object with L (3,), pos (N, 3) float32, vel (N, 3),
    type (N,) int32, gid (N,) uint32, phi (nz, ny, nx), h (3,) and params
    (dict: a, gamma, kBT, rc, dt, lam, g, seed, replica), such as the
    systems built by the `workloads` package, or a list of such objects for
    a batch context (one launch per kernel advances every box).  Per-box
    methods take the box index r (0 for a single box).
    """

    def __init__(self, system, params=None, flags=0, stream=None, graph=False):
        import torch
        self.torch = torch
        if isinstance(system, (list, tuple)):
            systems = list(system)
            self.ctx, self._keep = dpd_batch_create([_box_args(s) for s in systems],
                                                    stream=stream, flags=flags)
        else:
            systems = [system]
            self.ctx, self._keep = dpd_create(*_box_args(system, params), stream=stream,
                                              flags=flags)
        self.flags = flags
        self._phi_shape = tuple(systems[0].phi.shape)
        self.ns = [int(s.pos.shape[0]) for s in systems]
        self.n = self.ns[0]
        self.replicas = len(systems)
        self.params = dict(systems[0].params if params is None else params)
        self.device = torch.device("cuda", torch.cuda.current_device())
        if graph:
            self.use_graph(True)

    def close(self):
        if self.ctx is not None:
            dpd_destroy(self.ctx)
            self.ctx = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        dpd_step(self.ctx, n)

    def sync(self):
        dpd_sync(self.ctx)

    def use_graph(self, enable=True):
        dpd_use_graph(self.ctx, enable)

    def use_persistent(self, enable=True):
        """Each step as one persistent launch with per-box arrival counters."""
        dpd_use_persistent(self.ctx, enable)

    def autotune(self, steps=10):
        return dpd_autotune(self.ctx, steps)

    def forces(self, r=0):
        f = self.torch.empty((self.ns[r], 3), dtype=self.torch.float32, device=self.device)
        dpd_replica_forces(self.ctx, r, f)
        return f

    def state(self, r=0):
        t = self.torch
        n = self.ns[r]
        pos = t.empty((n, 3), dtype=t.float32, device=self.device)
        vel = t.empty((n, 3), dtype=t.float32, device=self.device)
        ev = t.empty((n,), dtype=t.int32, device=self.device)
        cell = t.empty((n,), dtype=t.int32, device=self.device)
        dpd_replica_state(self.ctx, r, pos, vel, ev, cell)
        return dict(pos=pos, vel=vel, events=ev, cell_of=cell)

    def set_state(self, pos, vel, force, k, r=0):
        dpd_replica_set_state(self.ctx, r, pos, vel, force, k)

    def pairs(self, r=0):
        n = dpd_replica_pairs(self.ctx, r, None, 0)
        buf = self.torch.empty((max(n, 1), 2), dtype=self.torch.int32, device=self.device)
        n2 = dpd_replica_pairs(self.ctx, r, buf, n)
        assert n2 == n
        return buf[:n].cpu().numpy().view(np.uint32)

    def profile(self, axis=2, nbins=100, r=0):
        out = self.torch.empty((nbins, 5), dtype=self.torch.float64, device=self.device)
        dpd_replica_profile(self.ctx, r, axis, nbins, out)
        return out

    def counters(self):
        return dpd_counters(self.ctx)

    def set_params(self, params, r=0):
        binding.dpd_set_params(self.ctx, r, params, self.flags)
        if r == 0:
            self.params = dict(params)

    def snapshot(self):
        """The complete dynamic state as bytes (checkpoint); restore() of it
        continues bit-identically."""
        blob = np.empty(binding.dpd_snapshot_size(self.ctx), dtype=np.uint8)
        binding.dpd_snapshot_io(self.ctx, 0, blob)
        return blob

    def restore(self, blob):
        binding.dpd_snapshot_io(self.ctx, 1, np.ascontiguousarray(blob, dtype=np.uint8))

    def set_phi(self, phi, r=0):
        binding.dpd_set_phi(self.ctx, r, phi)

    def kernel_times(self, enable):
        return dpd_kernel_times(self.ctx, enable)
