"""The adjoint over the full differentiation window against a frozen-decision
linearisation of the GPU's own forward.

Workload: the 20^3 sinusoidal slit (walls z = 3 + 2 sin(2 pi x / 20),
mirrored, ~16.4k fluid + 3.2k wall particles, an 80^3 float32 phase field),
a window of 200 steps with a checkpoint every 20, the window-mean v_x in 40
bins along z, loss = mean squared difference to a target profile (the GPU
window at a_ff = 20, gamma = 5, g_x = 0.025).

The window is a smooth function of the parameters only with its discrete
decisions held fixed (the pair sets r < rc, the bounce-back events of Eq.
16-17 and their codes, the bins), and even then it is chaotic: an FP64
trajectory from the same start, with the GPU's decisions, ends far from the
FP32 one after 200 steps, and the gradient along it is a different number
(measured: 45 % apart for a_ff).  The reference therefore follows the GPU's
trajectory: dpd_window_trace returns the GPU window's state before and after
every step and its decisions; the oracle's one-step map with those
decisions (pinned on the CPU: iterated, it is the oracle's replayed window
bit for bit) is linearised at each GPU state by FP64 central differences,
and the tangent of the window,
    delta_{t+1} = D step_t(x_t) [delta_t, dtheta],
starting from the tangent of the starting force, is carried over the 200
steps with the tangent of the bin sums.  That is the derivative of the
frozen-decision window along the GPU's trajectory, which is what the
adjoint computes backwards.  Parameters a_ff, a_fs, gamma, g_x, and three
random directions of the phase field (supported where |phi| < 0.9).  Bar:
1e-3 relative.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

NAMES = ["a_ff", "a_fs", "gamma", "g_x"]
TOL = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _perturbed(p0, what, h):
    p = dict(p0)
    a = [list(r) for r in p0["a"]]
    if what == "a_ff":
        a[0][0] += h
    elif what == "a_fs":
        a[0][1] += h
        a[1][0] += h
    elif what == "gamma":
        p["gamma"] = p0["gamma"] + h
    elif what == "g_x":
        p["g"] = [p0["g"][0] + h, p0["g"][1], p0["g"][2]]
    p["a"] = a
    return p


def _bins32(z, L, nbins):
    """The window's FP32 bin decision: clamp(floor(fl(z * fl32(nbins / L))))."""
    scale = np.float32(nbins / L)
    b = np.floor((np.asarray(z, np.float32) * scale).astype(np.float32)).astype(np.int64)
    return np.clip(b, 0, nbins - 1).astype(np.int32)


def test_full_window_against_the_linearised_gpu_trajectory(dpd, oracle_lib):
    import torch
    from paper_1807_09896_amd import binding
    from paper_1807_09896_amd.adjoint import Window
    s = workloads.sinusoid_slit_system()
    T, ckpt, nb = 200, 20, 40
    sim = dpd.Simulation(s, graph=True)
    win = Window(sim, steps=T, ckpt=ckpt, axis=2, nbins=nb)
    p0 = dict(sim.params)
    tgt_p = _perturbed(_perturbed(_perturbed(p0, "a_ff", 20.0 - p0["a"][0][0]), "gamma",
                                  5.0 - p0["gamma"]), "g_x", 0.025 - p0["g"][0])
    target = win.run(tgt_p).cpu().numpy()
    prof = win.run(p0).cpu().numpy()
    counts = win.counts.cpu().numpy().astype(np.float64)
    dldp = torch.tensor(2.0 * (prof - target) / nb, dtype=torch.float64, device="cuda")
    g, dphi = win.backward(dldp)
    dphi = dphi.cpu().numpy()
    n = s.n
    logs = {k: torch.empty((T + 1, n, 3), dtype=torch.float32, device="cuda")
            for k in ("pos", "vel", "frc")}
    ev = torch.empty((T, n), dtype=torch.int32, device="cuda")
    binding.dpd_window_trace(sim.ctx, logs["pos"], logs["vel"], logs["frc"], ev)
    rows = s.gid                      # row i of the system is gid rows[i]
    X = {k: v.cpu().numpy()[:, rows, :].astype(np.float64) for k, v in logs.items()}
    xs = np.ascontiguousarray(logs["pos"].cpu().numpy()[1:, rows, :])
    ev = np.ascontiguousarray(ev.cpu().numpy()[:, rows])
    bins = _bins32(xs[:, :, 2], s.L[2], nb)
    say("GPU window: %d particles, %d bounce-backs, %d returns to start"
        % (n, int((ev == 1).sum()), int((ev == 2).sum())))
    o = oracle_lib.Oracle(s, compute_forces=False)
    k0 = int(win.k0)
    fluid = o.type == 0
    # the bins of the GPU window are those of its decisions
    cnt = np.zeros(nb)
    for t in range(T):
        cnt += np.bincount(bins[t][fluid], minlength=nb)
    assert np.array_equal(cnt, counts)
    phi0 = o.phi64.copy()

    def set_theta(what, h, direc):
        if what == "phi":
            o.set_phi(phi0 + h * direc)
        else:
            o.params = _perturbed(p0, what, h)
            o.cparams = o._make_params(o.params)

    def reset():
        o.params = dict(p0)
        o.cparams = o._make_params(p0)
        o.set_phi(phi0)

    def tangent(what, direc=None):
        # tangent of the starting force (it does not depend on phi)
        if what == "phi":
            df = np.zeros((n, 3))
        else:
            h = 1e-6 * max(1.0, abs({"a_ff": p0["a"][0][0], "a_fs": p0["a"][0][1],
                                      "gamma": p0["gamma"], "g_x": p0["g"][0]}[what]))
            set_theta(what, h, direc)
            fp = o.window_start_force(X["pos"][0], X["vel"][0], k0)
            set_theta(what, -h, direc)
            fm = o.window_start_force(X["pos"][0], X["vel"][0], k0)
            reset()
            df = (fp - fm) / (2 * h)
        dr = np.zeros((n, 3))
        dv = np.zeros((n, 3))
        dS = np.zeros(nb)
        for t in range(T):
            size = max(1.0, np.abs(dr).max() + np.abs(dv).max() + 1e-2 * np.abs(df).max())
            e = 1e-6 / size
            out = []
            for sgn in (1.0, -1.0):
                set_theta(what, sgn * e, direc)
                out.append(o.window_step(X["pos"][t] + sgn * e * dr, X["vel"][t] + sgn * e * dv,
                                         X["frc"][t] + sgn * e * df, k0 + t + 1, ev[t], xs[t],
                                         bins[t], axis=2, nbins=nb))
            reset()
            (rp, vp, fp, sp, _), (rm, vm, fm, sm, _) = out
            dr, dv, df = (rp - rm) / (2 * e), (vp - vm) / (2 * e), (fp - fm) / (2 * e)
            dS += (sp - sm) / (2 * e)
        dprof = dS / np.maximum(counts, 1.0)
        return float((2.0 * (prof - target) / nb * dprof).sum())

    worst = 0.0
    for what in NAMES:
        ref = tangent(what)
        rel = abs(g[what] - ref) / abs(ref)
        worst = max(worst, rel)
        say("  %-6s adjoint % .8e  tangent % .8e  rel %.2e" % (what, g[what], ref, rel))
        assert rel < TOL, (what, g[what], ref)
    rng = np.random.default_rng(7)
    band = np.abs(s.phi) < 0.9
    for d in range(3):
        direc = rng.standard_normal(s.phi.shape) * band
        got = float((dphi * direc).sum())
        ref = tangent("phi", direc)
        rel = abs(got - ref) / abs(ref)
        worst = max(worst, rel)
        say("  phi direction %d: adjoint % .8e  tangent % .8e  rel %.2e" % (d, got, ref, rel))
        assert rel < TOL, ("phi", d, got, ref)
    say("worst relative difference %.2e" % worst)
    sim.close()
