"""GPU path (through the C ABI) against the FP64 oracle on the same seeded
inputs.

Bars: cell indices, interacting-pair sets and bounce-back event flags
bit-exact; per-particle FP32 forces within 2e-5 of the force-norm scale
F_scale (RMS |f| over fluid particles); positions and velocities after a
step within FP32 rounding of the FP64 values; long-run profiles within a few
standard errors.
"""
import math
import sys

import numpy as np
import pytest

import workloads
from gpu_helpers import by_gid, force_scale, require_gpu, sorted_pairs, trilinear_f64

pytestmark = pytest.mark.gpu

FORCE_TOL = 2e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpd():
    require_gpu()
    import paper_1807_09896_amd as dpd
    dpd.load_library()
    return dpd


def _stress_system(seed=70, width=0.02, vscale=3.0, crossers=80):
    """Slab channel whose phase field saturates to +-1 one grid node from the
    wall, hot fluid, and `crossers` fluid particles placed within 0.3 of a
    wall and aimed into it so that they cross in the next step: bounce-backs
    by Eq. 17, returns to the start position, and the atanh clamp at
    |phi| = 1 all occur in one step."""
    s = workloads.slab_system(L=(8.0, 6.0, 7.0), wall=1.0, width=width, grid_dtype=np.float32,
                              seed_fluid=seed, seed_wall=seed + 1,
                              params=workloads.default_params(g=(0.02, 0.0, 0.0), seed=seed))
    s.vel = (s.vel * vscale).astype(np.float32)
    rng = np.random.default_rng(seed + 5)
    fl = np.nonzero(s.type == 0)[0]
    pick = rng.choice(fl, size=min(crossers, len(fl)), replace=False)
    dt = s.params["dt"]
    for m, i in enumerate(pick):
        d0 = rng.uniform(0.001, 0.3)
        over = rng.uniform(0.01, 0.15)
        top = m % 2 == 1
        s.pos[i, 2] = np.float32(6.0 - d0 if top else 1.0 + d0)
        vz = (d0 + over) / dt
        s.vel[i, 2] = np.float32(vz if top else -vz)
    return s


def _small_curved(seed=12):
    """Sinusoidal channel with a cylinder in a 16 x 5 x 24 box (curved
    interfaces, several tiles of cells, ragged counts)."""
    return workloads.sinusoid_cylinder_system(L=(16.0, 5.0, 24.0), base=3.0, amp=1.5, radius=3.0,
                                              seed=seed,
                                              params=workloads.default_params(g=(0.01, 0, 0), seed=seed))


SYSTEMS = {
    "tiny": lambda: workloads.tiny_slab_system(),
    "slab_f64grid": lambda: workloads.slab_system(),
    "curved": _small_curved,
    "stress": _stress_system,
    "bulk": lambda: workloads.bulk_system(L=(5.0, 4.0, 3.0), params=workloads.default_params(seed=8)),
    # density 24: cells of up to about 30 particles, so that the per-cell
    # sort takes every run length (the register networks and the long runs)
    "dense": lambda: workloads.bulk_system(L=(5.0, 4.0, 3.0), rho=24.0,
                                           params=workloads.default_params(seed=21)),
    # cutoffs other than 1: the pair kernel's coarse-position pre-test scales
    # its bound with rc; with rc = 1.5 the cells are 1.6-1.75 wide, so row
    # candidates lie up to 3.5 apart per axis and their 10-bit code
    # differences wrap; at rc = 2 the pre-test keeps every candidate
    "rc15": lambda: workloads.slab_system(L=(8.0, 7.0, 9.0), wall=1.5, grid_dtype=np.float32,
                                          seed_fluid=31, seed_wall=32,
                                          params=workloads.default_params(rc=1.5,
                                                                          g=(0.02, 0, 0),
                                                                          seed=33)),
    "rc20": lambda: workloads.bulk_system(L=(8.0, 6.0, 7.0), rho=3.0,
                                          params=workloads.default_params(rc=2.0, seed=34)),
    # box edges whose 256 L is not an integer: the coarse codes' image
    # shifts are rounded, and the last cell of each axis is narrower
    "odd_box": lambda: workloads.bulk_system(L=(5.4, 4.8, 6.3), h=0.3, rho=4.0,
                                             params=workloads.default_params(seed=35)),
}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_initial_forces_cells_pairs(dpd, oracle_lib, name):
    s = SYSTEMS[name]()
    say("system", name, "n", s.n, "fluid", s.n_fluid)
    o = oracle_lib.Oracle(s)
    sim = dpd.Simulation(s)
    f_gpu = sim.forces().cpu().numpy().astype(np.float64)
    st = {k: v.cpu().numpy() for k, v in sim.state().items()}
    f_or = by_gid(o, o.f)
    fluid_g = by_gid(o, s.type) == 0
    scale = force_scale(f_or[fluid_g])
    err = np.abs(f_gpu - f_or).max(axis=1)
    assert err[fluid_g].max() <= FORCE_TOL * scale, (err.max(), scale)
    assert np.all(f_gpu[~fluid_g] == 0)
    assert np.array_equal(st["cell_of"], by_gid(o, o.cells()))
    assert np.array_equal(st["pos"], by_gid(o, s.pos))
    gp = sim.pairs()
    op = o.pairs()
    assert gp.shape == op.shape
    assert np.array_equal(sorted_pairs(gp), sorted_pairs(op))
    sim.close()


def _rounding_reach(s):
    """How far apart the kernel's and the oracle's reflected positions (Eq.
    17) can be: the kernel rounds x* - k2 u to FP32 once (half a unit in the
    last place of the largest edge per axis; k2's own FP32 error moves a
    step of at most 0.1 by ~1e-8), the oracle keeps FP64.  Returns that
    distance and the change it can make to phi (the trilinear field's
    largest slope times it, plus three FP32 roundings of a value <= 1)."""
    ulp = float(np.spacing(np.float32(max(s.L))))
    dx = np.sqrt(3.0) * (0.5 * ulp + 1e-8)
    phi = np.asarray(s.phi, np.float64)
    g2 = 0.0
    for axis, h in ((2, s.h[0]), (1, s.h[1]), (0, s.h[2])):
        g2 += (np.abs(np.roll(phi, -1, axis=axis) - phi).max() / h) ** 2
    return dx, np.sqrt(g2) * dx + 2e-7


def _min_image(d, L):
    d = np.abs(d)
    return np.minimum(d, np.asarray(L)[None, :] - d)


def _one_step_compare(dpd, oracle_lib, s, nsteps_before=0, sim=None, r=0):
    """One step of the GPU path from a common FP32 snapshot against the
    oracle.  With `sim` (a batch context holding s as box r) the snapshot is
    set into box r and the whole batch steps once."""
    own = sim is None
    o = oracle_lib.Oracle(s)
    if nsteps_before:
        o.step(nsteps_before)
    # a common FP32 snapshot: positions, velocities and the carried force
    pos32 = o.r.astype(np.float32)
    vel32 = o.v.astype(np.float32)
    f32 = o.f.astype(np.float32)
    for a in range(3):
        col = pos32[:, a]
        col[col < 0] += np.float32(s.L[a])
        col[col >= np.float32(s.L[a])] = np.float32(0.0)
    o.set_state(pos32, vel32, f32, o.k)
    if own:
        sim = dpd.Simulation(s)
    sim.set_state(by_gid(o, pos32), by_gid(o, vel32), by_gid(o, f32), o.k, r=r)
    ev_or = o.step(1)
    sim.step(1)
    st = {k: v.cpu().numpy() for k, v in sim.state(r).items()}
    f_gpu = sim.forces(r).cpu().numpy().astype(np.float64)
    fluid_g = by_gid(o, s.type) == 0
    ev_or_g = by_gid(o, ev_or)
    # events: bounce or not, bit-exact; the code (1 vs 2) wherever the
    # fallback test phi(r_bb) < 0 lies beyond the reach of the FP32 rounding
    # of the reflected position
    dx, dphi = _rounding_reach(s)
    assert np.array_equal(st["events"] > 0, ev_or_g > 0)
    both = (st["events"] > 0) & (ev_or_g > 0)
    if both.any():
        x_or = by_gid(o, o.r)[both]
        phib = trilinear_f64(s.phi, s.h, x_or)
        clear = np.abs(phib) > dphi
        assert np.array_equal(st["events"][both][clear], ev_or_g[both][clear])
        say("  events %d, codes compared %d (band %.2e)" % (both.sum(), clear.sum(), dphi))
    cells_or = by_gid(o, o.cells())
    bounced = ev_or_g > 0
    assert np.array_equal(st["cell_of"][~bounced], cells_or[~bounced])
    # a bounced particle's cell may differ only where its position lies
    # within that rounding of a cell face
    mism = np.nonzero(st["cell_of"] != cells_or)[0]
    if len(mism):
        x_m = by_gid(o, o.r)[mism]
        w = np.asarray(s.L) / np.floor(np.asarray(s.L) / s.params["rc"])
        face = np.abs(x_m / w[None, :] - np.round(x_m / w[None, :])) * w[None, :]
        assert np.all(face.min(axis=1) <= dx), face.min(axis=1)
    # positions and velocities
    r_or = by_gid(o, o.r)
    d = np.abs(st["pos"].astype(np.float64) - r_or)
    d = np.minimum(d, np.asarray(s.L)[None, :] - d)
    assert d[fluid_g].max() < 2e-5 * max(s.L)
    v_or = by_gid(o, o.v)
    f_or = by_gid(o, o.f)
    scale = force_scale(f_or[fluid_g])
    assert np.abs(st["vel"].astype(np.float64) - v_or)[fluid_g].max() < 1e-4 * (1 + np.abs(v_or).max())
    # The FP64 trajectory and the FP32 state differ by the rounding of the
    # drift (about 1e-6 at x ~ 20), which moves forces by more than the
    # force tolerance; the force kernel is therefore checked against the
    # oracle's FP64 forces at the oracle's own FP32 shadow positions (the
    # decision-form drift, identical to the GPU's by construction).
    f_sh = by_gid(o, o.forces(k=o.k, r=o.xs.astype(np.float64), vt=o.vt, xs=o.xs))
    err = np.abs(f_gpu - f_sh).max(axis=1)
    # every fluid particle at the same bar, bounced ones and their partners
    # included (their reflected positions differ by the FP32 rounding of Eq.
    # 17, which moves a pair force by ~1e-4 absolute: a few 1e-6 F_scale)
    near = np.zeros(len(err), bool)
    if bounced.any():
        pr = o.pairs().astype(np.int64)
        hit = bounced[pr[:, 0]] | bounced[pr[:, 1]]
        near[pr[hit, 0]] = True
        near[pr[hit, 1]] = True
        near |= bounced
    assert err[fluid_g].max() <= FORCE_TOL * scale, (err[fluid_g].max(), scale)
    if (fluid_g & near).any():
        say("  next to bounces: max |df| / F_scale %.2e (elsewhere %.2e)"
            % (err[fluid_g & near].max() / scale, err[fluid_g & ~near].max() / scale))
    # and against the FP64 trajectory within the drift rounding
    assert np.abs(f_gpu - f_or)[fluid_g].max() <= 2e-4 * scale
    # interacting pairs after the step, bit-exact except pairs of a bounced
    # particle whose FP64 distance lies within twice that rounding of rc
    gp = sim.pairs(r)
    op = o.pairs()
    if not bounced.any():
        assert np.array_equal(sorted_pairs(gp), sorted_pairs(op))
    else:
        rc = s.params["rc"]

        def edge(pairs):
            pi = pairs.astype(np.int64)
            b = bounced[pi[:, 0]] | bounced[pi[:, 1]]
            dist = np.sqrt((_min_image(r_or[pi[:, 0]] - r_or[pi[:, 1]], s.L) ** 2).sum(1))
            return b & (np.abs(dist - rc) <= 2 * dx)

        eg, eo = edge(gp), edge(op)
        say("  pairs: %d vs %d, %d / %d at the cutoff's rounding edge"
            % (len(gp), len(op), eg.sum(), eo.sum()))
        assert np.array_equal(sorted_pairs(gp[~eg]), sorted_pairs(op[~eo]))
    n_events = int((ev_or_g > 0).sum())
    if own:
        sim.close()
    return n_events


@pytest.mark.parametrize("name", ["tiny", "slab_f64grid", "curved", "stress", "dense", "rc15",
                                  "rc20", "odd_box"])
def test_one_step_parity(dpd, oracle_lib, name):
    s = SYSTEMS[name]()
    say("one-step", name, s.n)
    n_ev = _one_step_compare(dpd, oracle_lib, s)
    if name == "stress":
        assert n_ev >= 60


def test_one_step_parity_after_oracle_run(dpd, oracle_lib):
    s = _small_curved(seed=13)
    s.vel = (s.vel * 3).astype(np.float32)
    say("one-step after 20 oracle steps", s.n)
    _one_step_compare(dpd, oracle_lib, s, nsteps_before=20)


def test_mask_is_exact_and_runs_are_deterministic(dpd):
    s = _stress_system(seed=71, vscale=3.0)
    a = dpd.Simulation(s)
    b = dpd.Simulation(s, flags=1)          # DPD_FLAG_NO_MASK
    c = dpd.Simulation(s)
    for sim in (a, b, c):
        sim.step(40)
    sa, sb, sc = a.state(), b.state(), c.state()
    for k in ("pos", "vel", "events"):
        assert np.array_equal(sa[k].cpu().numpy(), sb[k].cpu().numpy()), k
        assert np.array_equal(sa[k].cpu().numpy(), sc[k].cpu().numpy()), k
    assert np.array_equal(a.forces().cpu().numpy(), b.forces().cpu().numpy())
    assert a.counters()["bounce"] > 0
    for sim in (a, b, c):
        sim.close()


def test_no_penetration_and_momentum_long_run(dpd):
    s = _small_curved(seed=14)
    sim = dpd.Simulation(s)
    fl = s.type == 0
    gid_fluid = s.gid[fl]
    for blk in range(5):
        sim.step(100)
        st = sim.state()
        pos = st["pos"].cpu().numpy()[gid_fluid]
        phi = trilinear_f64(s.phi, s.h, pos)
        assert phi.min() >= -1e-6, phi.min()
    c = sim.counters()
    say("counters", c)
    assert c["bounce"] > 0
    sim.close()


def test_momentum_balance_without_walls(dpd):
    p = workloads.default_params(g=(0.03, -0.01, 0.02), seed=5)
    s = workloads.bulk_system(L=(6.0, 6.0, 6.0), params=p)
    sim = dpd.Simulation(s)
    v0 = sim.state()["vel"].double().sum(0).cpu().numpy()
    sim.step(10)
    v1 = sim.state()["vel"].double().sum(0).cpu().numpy()
    expect = s.n_fluid * np.array([0.03, -0.01, 0.02]) * 0.01 * 10
    # FP32 forces: pair terms cancel up to rounding of each particle's sum
    assert np.allclose(v1 - v0, expect, atol=2e-3 * math.sqrt(s.n_fluid))
    sim.close()


def test_profile_observable(dpd, oracle_lib):
    s = workloads.slab_system()
    o = oracle_lib.Oracle(s)
    sim = dpd.Simulation(s)
    prof = sim.profile(axis=2, nbins=20).cpu().numpy()
    ref = o.profile(axis=2, nbins=20)
    assert np.array_equal(prof[:, 0], ref["count"])
    assert np.allclose(prof[:, 1], ref["sum_vx"], atol=1e-4)
    assert np.allclose(prof[:, 4], ref["sum_v2"], rtol=1e-6, atol=1e-3)
    sim.close()


def test_edge_cases(dpd, oracle_lib):
    # all walls, no fluid: create and step are no-ops
    s = workloads.tiny_slab_system()
    s.type[:] = 1
    sim = dpd.Simulation(s)
    sim.step(3)
    assert np.all(sim.forces().cpu().numpy() == 0)
    sim.close()
    # box of exactly 3 cells per axis, no walls
    p = workloads.default_params(seed=3)
    s = workloads.bulk_system(L=(3.0, 3.0, 3.0), h=0.5, params=p)
    o = oracle_lib.Oracle(s)
    sim = dpd.Simulation(s)
    f = sim.forces().cpu().numpy()
    fo = by_gid(o, o.f)
    assert np.abs(f - fo).max() <= FORCE_TOL * force_scale(fo)
    assert np.array_equal(sorted_pairs(sim.pairs()), sorted_pairs(o.pairs()))
    sim.close()
    # a fluid particle starting in the solid is rejected
    s = workloads.tiny_slab_system()
    fl = np.nonzero(s.type == 0)[0][0]
    s.pos[fl, 2] = 0.3
    with pytest.raises(dpd.DPDError, match="phi < 0"):
        dpd.Simulation(s)
    # non-finite phi grid is rejected
    s = workloads.tiny_slab_system()
    s.phi = s.phi.copy()
    s.phi[0, 0, 0] = np.nan
    with pytest.raises(dpd.DPDError, match="non-finite"):
        dpd.Simulation(s)
    # a particle that would jump more than half a cell: DPD_E_UNSTABLE
    s = workloads.tiny_slab_system()
    s.vel = s.vel.copy()
    s.vel[np.nonzero(s.type == 0)[0][3]] = [80.0, 0.0, 0.0]
    sim = dpd.Simulation(s)
    sim.step(1)
    with pytest.raises(dpd.DPDError, match="DPD_E_UNSTABLE"):
        sim.sync()
    sim.close()


def test_particle_on_the_interface_and_non_finite_state(dpd, oracle_lib):
    """A fluid particle exactly on the phi = 0 plane (a grid node of the
    slab interface, where phi interpolates to zero) is accepted (Sec. II.C:
    a bounce needs phi < 0) and, sent into the wall, bounces back with the
    oracle's event and position; a NaN velocity set into a running context
    is reported as DPD_E_UNSTABLE at the next synchronisation."""
    s = workloads.tiny_slab_system()
    i = int(np.nonzero(s.type == 0)[0][5])
    pos, vel = s.pos.copy(), s.vel.copy()
    lo = s.meta["lo"]
    pos[i] = np.asarray([1.0, 1.0, lo], np.float32)
    vel[i] = np.asarray([0.3, 0.0, -2.0], np.float32)
    s.pos, s.vel = pos, vel
    assert trilinear_f64(s.phi, s.h, pos[i:i + 1].astype(np.float64))[0] == 0.0
    n_ev = _one_step_compare(dpd, oracle_lib, s)
    assert n_ev >= 1
    sim = dpd.Simulation(workloads.tiny_slab_system())
    sim.step(2)
    st = {k: v.cpu().numpy() for k, v in sim.state().items()}
    f = sim.forces().cpu().numpy()
    v = st["vel"].copy()
    v[np.nonzero(workloads.tiny_slab_system().type == 0)[0][0]] = np.nan
    c = sim.counters()
    sim.set_state(st["pos"], v, f, c["k"])
    sim.step(1)
    with pytest.raises(dpd.DPDError, match="DPD_E_UNSTABLE"):
        sim.sync()
    sim.close()


def test_random_stream_matches_oracle(dpd, oracle_lib):
    """The GPU's Philox4x32-10 words equal the oracle's bit for bit, and its
    FP32 Box-Muller xi (hardware log2, sqrt and cos) stays within 3e-5 of the
    oracle's FP64 xi (|xi| <= 5.8)."""
    import torch
    rng = np.random.default_rng(2)
    n = 1 << 20
    gi = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    gj = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    gi[:10] = gj[:10]              # equal gids too
    dgi = torch.from_numpy(gi.view(np.int32)).cuda()
    dgj = torch.from_numpy(gj.view(np.int32)).cuda()
    worst = 0.0
    for seed, k, rep in [(1234, 0, 0), (2**40 + 7, 2**33 + 5, 17), (2**64 - 1, 2**48 - 1, 65535)]:
        words = torch.empty((n, 4), dtype=torch.int32, device="cuda")
        xi = torch.empty(n, dtype=torch.float32, device="cuda")
        dpd.binding.dpd_pair_random(seed, k, rep, dgi, dgj, words, xi)
        torch.cuda.synchronize()
        w_or, xi_or = oracle_lib.pairs_random(seed, gi, gj, k, rep)
        assert np.array_equal(words.cpu().numpy().view(np.uint32), w_or)
        d = np.abs(xi.cpu().numpy().astype(np.float64) - xi_or)
        worst = max(worst, float(d.max()))
        # symmetric in (i, j)
        xi_sw = torch.empty(n, dtype=torch.float32, device="cuda")
        dpd.binding.dpd_pair_random(seed, k, rep, dgj, dgi, None, xi_sw)
        assert torch.equal(xi, xi_sw)
    say("max |xi_gpu - xi_oracle| = %.3g" % worst)
    assert worst < 3e-5


def test_kernel_timing_and_copy_probe(dpd):
    import torch
    s = workloads.slab_system()
    sim = dpd.Simulation(s)
    sim.kernel_times(1)
    sim.step(5)
    t = sim.kernel_times(0)
    assert t["pair_force"][1] == 5 and t["pair_force"][0] > 0
    assert t["integrate_reflect_bin"][1] == 5
    sim.close()
    a = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    dpd.binding.dpd_copy_probe(b, a, a.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
