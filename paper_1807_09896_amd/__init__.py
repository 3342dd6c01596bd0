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
from .binding import (DPDError, dpd_counters, dpd_create, dpd_destroy, dpd_forces,
                      dpd_get_state, dpd_kernel_times, dpd_last_error, dpd_neighbor_pairs,
                      dpd_profile, dpd_set_state, dpd_step, dpd_sync, load_library)

__all__ = ["Simulation", "DPDError", "load_library", "dpd_create", "dpd_step", "dpd_forces",
           "dpd_get_state", "dpd_set_state", "dpd_neighbor_pairs", "dpd_profile",
           "dpd_counters", "dpd_kernel_times", "dpd_sync", "dpd_last_error", "dpd_destroy"]


class Simulation:
    """One box on the GPU.

    `system` is any object with L (3,), pos (N, 3) float32, vel (N, 3),
    type (N,) int32, gid (N,) uint32, phi (nz, ny, nx), h (3,) and params
    (dict: a, gamma, kBT, rc, dt, lam, g, seed, replica), such as the
    systems built by the `workloads` package.
    """

    def __init__(self, system, params=None, flags=0, stream=None):
        import torch
        self.torch = torch
        self.n = int(system.pos.shape[0])
        self.params = dict(system.params if params is None else params)
        self.ctx, self._keep = dpd_create(system.L, system.pos, system.vel, system.type,
                                          system.gid, self.params, system.phi, system.h,
                                          stream=stream, flags=flags)
        self.device = torch.device("cuda", torch.cuda.current_device())

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

    def forces(self):
        f = self.torch.empty((self.n, 3), dtype=self.torch.float32, device=self.device)
        dpd_forces(self.ctx, f)
        return f

    def state(self):
        t = self.torch
        pos = t.empty((self.n, 3), dtype=t.float32, device=self.device)
        vel = t.empty((self.n, 3), dtype=t.float32, device=self.device)
        ev = t.empty((self.n,), dtype=t.int32, device=self.device)
        cell = t.empty((self.n,), dtype=t.int32, device=self.device)
        dpd_get_state(self.ctx, pos, vel, ev, cell)
        return dict(pos=pos, vel=vel, events=ev, cell_of=cell)

    def set_state(self, pos, vel, force, k):
        dpd_set_state(self.ctx, pos, vel, force, k)

    def pairs(self):
        n = dpd_neighbor_pairs(self.ctx, None, 0)
        buf = self.torch.empty((max(n, 1), 2), dtype=self.torch.int32, device=self.device)
        n2 = dpd_neighbor_pairs(self.ctx, buf, n)
        assert n2 == n
        return buf[:n].cpu().numpy().view(np.uint32)

    def profile(self, axis=2, nbins=100):
        out = self.torch.empty((nbins, 5), dtype=self.torch.float64, device=self.device)
        dpd_profile(self.ctx, axis, nbins, out)
        return out

    def counters(self):
        return dpd_counters(self.ctx)

    def kernel_times(self, enable):
        return dpd_kernel_times(self.ctx, enable)
