"""Differentiable window of DPD steps (the adjoint form) for PyTorch.

`Window(sim, ...)` fixes a starting state of a single-box `Simulation`;
`window.profile(a_ff, a_fs, gamma, g_x, phi)` runs the window on the GPU
(`dpd_window_forward`) and returns the window-mean v_x per bin; its
backward calls the library's hand-written adjoint (`dpd_backward`).  The
starting positions and velocities are held fixed and not differentiated;
the carried force is recomputed from them with the given parameters.
"""
from __future__ import annotations

import torch

from . import binding


class _WindowFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, win, a_ff, a_fs, gamma, g_x, phi):
        sim = win.sim
        p = dict(win.params)
        a = float(a_ff)
        b = float(a_fs)
        p["a"] = [[a, b], [b, b]]
        p["gamma"] = float(gamma)
        p["g"] = [float(g_x), float(p["g"][1]), float(p["g"][2])]
        binding.dpd_set_state(sim.ctx, win.pos, win.vel, win.force, win.k0)
        binding.dpd_set_params(sim.ctx, 0, p, win.flags)
        binding.dpd_set_phi(sim.ctx, 0, phi.detach().contiguous())
        prof = torch.empty(win.nbins, dtype=torch.float64, device=sim.device)
        cnt = torch.empty(win.nbins, dtype=torch.int64, device=sim.device)
        binding.dpd_window_forward(sim.ctx, win.steps, win.ckpt, win.axis, win.nbins, prof, cnt)
        win.counts = cnt
        ctx.win = win
        ctx.phi_dtype = phi.dtype
        ctx.phi_shape = phi.shape
        return prof

    @staticmethod
    def backward(ctx, grad):
        win = ctx.win
        sim = win.sim
        dphi = torch.empty(ctx.phi_shape, dtype=torch.float64, device=sim.device)
        g = binding.dpd_backward(sim.ctx, grad.detach().to(torch.float64).contiguous(), dphi)
        t = lambda x: torch.tensor(float(x), dtype=torch.float64)
        return None, t(g[0]), t(g[1]), t(g[2]), t(g[3]), dphi.to(ctx.phi_dtype)


class Window:
    """A window of `steps` steps (checkpoint every `ckpt`) from the current
    state of `sim`, observed as `nbins` bins along `axis`."""

    def __init__(self, sim, steps=200, ckpt=20, axis=2, nbins=40, flags=0):
        if sim.replicas != 1:
            raise ValueError("the adjoint form needs a single-box Simulation")
        self.sim = sim
        self.steps, self.ckpt, self.axis, self.nbins = int(steps), int(ckpt), int(axis), int(nbins)
        self.flags = flags
        st = sim.state()
        self.pos, self.vel = st["pos"], st["vel"]
        self.force = sim.forces()
        self.k0 = sim.counters()["k"]
        self.params = dict(sim.params)
        self.counts = None

    def profile(self, a_ff, a_fs, gamma, g_x, phi):
        """Window-mean v_x per bin; differentiable in every argument
        (scalars as 0-d tensors, phi as the grid tensor)."""
        return _WindowFn.apply(self, a_ff, a_fs, gamma, g_x, phi)

    def run(self, params=None, phi=None):
        """Forward only (no graph), with the given parameter dict and grid."""
        p = dict(self.params if params is None else params)
        binding.dpd_set_state(self.sim.ctx, self.pos, self.vel, self.force, self.k0)
        binding.dpd_set_params(self.sim.ctx, 0, p, self.flags)
        if phi is not None:
            binding.dpd_set_phi(self.sim.ctx, 0, phi)
        prof = torch.empty(self.nbins, dtype=torch.float64, device=self.sim.device)
        cnt = torch.empty(self.nbins, dtype=torch.int64, device=self.sim.device)
        binding.dpd_window_forward(self.sim.ctx, self.steps, self.ckpt, self.axis, self.nbins,
                                   prof, cnt)
        self.counts = cnt
        return prof

    def backward(self, dl_dprofile, want_phi=True):
        """Gradients after `run`: (dict of scalars, dL/dphi tensor or None)."""
        dphi = None
        if want_phi:
            shape = tuple(self.sim._phi_shape)
            dphi = torch.empty(shape, dtype=torch.float64, device=self.sim.device)
        g = binding.dpd_backward(self.sim.ctx, dl_dprofile.to(torch.float64).contiguous(), dphi)
        names = ["a_ff", "a_fs", "gamma", "g_x", "g_y", "g_z"]
        return dict(zip(names, (float(x) for x in g))), dphi
