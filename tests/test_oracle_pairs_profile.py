"""Pins of the oracle's interacting-pair list and binned profile.

`Oracle.pairs` (the reference of every bit-exact pair-set comparison) is
checked against an independent O(N^2) enumeration written here from the
definition: the FP32 cell of each position, the image shift that the two
cells imply, the separation rounded once from the exact minimum-image
difference (evaluated in exact arithmetic), and the FP32 r^2 < rc^2 test
with correctly rounded fused multiply-adds.  Away from a thin band around
the cutoff, the set must also equal the pairs closer than rc by the FP64
minimum-image distance (Eq. 5: a pair interacts iff r < rc).

`Oracle.profile` (Sec. III.A's binned density, stream velocity and
temperature) is checked against direct binning with numpy and against
closed forms on a lattice.  No GPU is used.
"""
from fractions import Fraction

import numpy as np

import workloads


def _cell32(x, L, n):
    """FP32 cell coordinate: min(n - 1, floor(fl32(x * fl32(n / L))))."""
    invw = np.float32(n / L)
    g = np.floor((np.asarray(x, np.float32) * invw).astype(np.float32))
    return np.clip(g.astype(np.int64), 0, n - 1)


def _fma32(a, b, c):
    """fl32(a * b + c) with one rounding.  a * b is exact in float64 (two
    24-bit significands); where the float64 sum could sit on a float32
    rounding midpoint the exact value is rounded with fractions instead."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    c = np.asarray(c, np.float32)
    s64 = a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)
    out = s64.astype(np.float32)
    # float32 midpoints of the neighbourhood of s64: fix those cases exactly
    lo = np.nextafter(out, np.float32(-np.inf))
    hi = np.nextafter(out, np.float32(np.inf))
    mids = np.stack([(out.astype(np.float64) + lo) / 2, (out.astype(np.float64) + hi) / 2])
    risky = np.any(np.abs(mids - s64) <= np.abs(s64) * 2.0 ** -50, axis=0)
    for k in np.flatnonzero(risky.ravel()):
        ex = Fraction(float(a.flat[k])) * Fraction(float(b.flat[k])) + Fraction(float(c.flat[k]))
        out.flat[k] = _round_fraction32(ex)
    return out


def _round_fraction32(q):
    """Round an exact rational to the nearest float32 (ties to even)."""
    f = np.float32(float(q))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]
    best = min(cands, key=lambda v: (abs(Fraction(float(v)) - q),
                                     int(np.frombuffer(np.float32(v).tobytes(), np.uint32)[0]) & 1))
    return best


def _sep_exact32(xi, xj, s, L32):
    """fl32(x_i - x_j - s L), the exact difference rounded once.  For the
    positions used here (all coordinates either 0 or at least 2^-20) the
    float64 value of the difference is exact, which is asserted."""
    xi = np.asarray(xi, np.float64)
    xj = np.asarray(xj, np.float64)
    d = xi - xj - s * float(L32)
    # exactness: undo the operations and recover both operands
    assert np.all((d + s * float(L32)) + xj == xi)
    return d.astype(np.float32)


def _enumerate_pairs(system, rc):
    """Every (gid_i, gid_j), i fluid, j != i, with the FP32 decision of the
    definition; also the FP64 minimum-image distances of all such pairs."""
    pos = np.asarray(system.pos, np.float32)
    assert np.all((pos == 0) | (np.abs(pos) >= 2.0 ** -20))
    L = np.asarray(system.L, np.float64)
    L32 = L.astype(np.float32)
    nc = np.array([int(np.floor(x / rc)) for x in L])
    cells = np.stack([_cell32(pos[:, a], L[a], nc[a]) for a in range(3)], axis=1)
    rc2 = np.float32(rc * rc)
    fluid = np.flatnonzero(system.type == 0)
    out, dist = [], []
    for i in fluid:
        s = np.zeros((system.n, 3), np.int64)
        ok = np.ones(system.n, bool)
        for a in range(3):
            o = np.mod(cells[:, a] - cells[i, a] + 1, nc[a]) - 1   # offset in {-1, 0, 1}?
            ok &= (o >= -1) & (o <= 1)
            q = cells[i, a] + o
            s[:, a] = np.where(q < 0, -1, np.where(q >= nc[a], 1, 0))
        ok[i] = False
        j = np.flatnonzero(ok)
        d = np.stack([_sep_exact32(pos[i, a], pos[j, a], s[j, a], L32[a]) for a in range(3)],
                     axis=1)
        r2 = _fma32(d[:, 2], d[:, 2], _fma32(d[:, 1], d[:, 1], (d[:, 0] * d[:, 0]).astype(np.float32)))
        hit = j[r2 < rc2]
        out.append(np.stack([np.full(hit.size, system.gid[i]), system.gid[hit]], axis=1))
        # FP64 minimum image over all particles (not only the 27 cells)
        dd = pos[i].astype(np.float64)[None, :] - pos.astype(np.float64)
        dd -= L[None, :] * np.round(dd / L[None, :])
        r = np.sqrt((dd ** 2).sum(axis=1))
        r[i] = np.inf
        dist.append((np.full(system.n, system.gid[i]), system.gid, r))
    pairs = np.concatenate(out).astype(np.uint64) if out else np.zeros((0, 2), np.uint64)
    return pairs, dist


def _keys(p):
    p = np.asarray(p, np.uint64)
    return np.sort((p[:, 0] << np.uint64(32)) | p[:, 1])


def _systems():
    slab = workloads.slab_system()                      # 10^3 plane channel, walls at both z ends
    curved = workloads.sinusoid_cylinder_system(L=(16.0, 5.0, 24.0), base=3.0, amp=1.5,
                                               radius=3.0, seed=12)
    odd = workloads.bulk_system(L=(3.0, 4.5, 5.5), rho=3.0, seed=21)  # 3 cells, ragged widths
    return [slab, curved, odd]


def test_pairs_match_independent_enumeration_and_fp64_distances(oracle_lib):
    rc = 1.0
    for s in _systems():
        o = oracle_lib.Oracle(s, compute_forces=False)
        got = _keys(o.pairs())
        ref_pairs, dist = _enumerate_pairs(s, rc)
        ref = _keys(ref_pairs)
        assert got.size == ref.size and np.array_equal(got, ref), s.name
        # Eq. 5: r < rc away from a band of FP32 rounding around the cutoff
        band = 1e-5
        gset = set(got.tolist())
        n_in = n_out = 0
        for gi, gj, r in dist:
            key = (gi.astype(np.uint64) << np.uint64(32)) | gj.astype(np.uint64)
            inside = key[r < rc - band]
            outside = key[(r > rc + band) & np.isfinite(r)]
            assert all(int(k) in gset for k in inside), s.name
            assert not any(int(k) in gset for k in outside[:2000]), s.name
            n_in += inside.size
            n_out += outside.size
        assert n_in == got.size or n_in >= 0.999 * got.size
        # fluid-fluid pairs appear in both orders, fluid-wall pairs once
        typ = np.empty(s.n, np.int32)
        typ[s.gid] = s.type
        p = o.pairs().astype(np.int64)
        ff = (typ[p[:, 0]] == 0) & (typ[p[:, 1]] == 0)
        fw = (typ[p[:, 0]] == 0) & (typ[p[:, 1]] != 0)
        assert np.all(ff | fw)
        rev = _keys(p[ff][:, ::-1])
        assert np.array_equal(rev, _keys(p[ff]))


def test_pair_across_the_periodic_edge_rounds_once(oracle_lib):
    """Two particles 1 - 3e-6 apart across the periodic edge of a 168-long
    box interact: the separation is the exact difference rounded once
    (0.9999970 < rc).  Shifting the particle near 0 up by L first would
    round 168.249997 to 168.25 and put the pair exactly at the cutoff."""
    s = workloads.bulk_system(L=(168.0, 4.0, 4.0), rho=0.01, seed=2)
    xi = np.float32(0.25 - 3e-6)
    xj = np.float32(167.25)
    s.pos = np.array([[xi, 2.0, 2.0], [xj, 2.0, 2.0]], np.float32)
    s.vel = np.zeros((2, 3), np.float32)
    s.type = np.zeros(2, np.int32)
    s.gid = np.array([0, 1], np.uint32)
    exact = Fraction(float(xi)) + Fraction(168) - Fraction(float(xj))
    assert exact < 1 and np.float32(np.float32(xi + np.float32(168.0)) - xj) == 1.0
    o = oracle_lib.Oracle(s, compute_forces=False)
    assert sorted(map(tuple, o.pairs().tolist())) == [(0, 1), (1, 0)]
    ref, _ = _enumerate_pairs(s, 1.0)
    assert ref.shape[0] == 2


def test_fma32_is_correctly_rounded():
    rng = np.random.default_rng(4)
    a = rng.standard_normal(2000).astype(np.float32)
    b = rng.standard_normal(2000).astype(np.float32)
    c = rng.standard_normal(2000).astype(np.float32)
    got = _fma32(a, b, c)
    for k in range(0, 2000, 97):
        ex = Fraction(float(a[k])) * Fraction(float(b[k])) + Fraction(float(c[k]))
        assert got[k] == _round_fraction32(ex)


def test_profile_matches_direct_binning(oracle_lib):
    s = workloads.sinusoid_cylinder_system(L=(16.0, 5.0, 24.0), base=3.0, amp=1.5, radius=3.0,
                                           seed=13)
    o = oracle_lib.Oracle(s, compute_forces=False)
    o.step(3)
    fl = o.type == 0
    for axis, nbins in ((2, 24), (0, 7), (1, 1)):
        prof = o.profile(axis=axis, nbins=nbins)
        x = np.mod(o.r[fl, axis], s.L[axis])
        b = np.clip(np.floor(x / s.L[axis] * nbins).astype(np.int64), 0, nbins - 1)
        v = o.v[fl]
        assert np.array_equal(prof["count"], np.bincount(b, minlength=nbins).astype(float))
        np.testing.assert_allclose(prof["sum_vx"], np.bincount(b, v[:, 0], nbins),
                                   rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(prof["sum_v2"], np.bincount(b, (v ** 2).sum(1), nbins),
                                   rtol=1e-12, atol=1e-12)
        for a in range(3):
            np.testing.assert_allclose(prof["sum_v"][:, a], np.bincount(b, v[:, a], nbins),
                                       rtol=1e-12, atol=1e-12)
        # totals: every fluid particle once, the total momentum
        assert prof["count"].sum() == fl.sum()
        np.testing.assert_allclose(prof["sum_v"].sum(0), v.sum(0), rtol=1e-10, atol=1e-10)


def test_profile_closed_form_on_a_lattice(oracle_lib):
    """Fluid particles on a lattice with z = (k + 1/2) L / m, velocity
    (z, 0, 0): bin b of m bins holds the particles of plane b, its sum of
    v_x is count * z_b and its sum of |v|^2 count * z_b^2."""
    m, per = 8, 9
    L = (6.0, 6.0, 8.0)
    s = workloads.bulk_system(L=L, rho=0.01, seed=2)
    zs = (np.arange(m) + 0.5) * L[2] / m
    xy = [(0.5 + 2 * i, 0.5 + 2 * j) for i in range(3) for j in range(3)]
    pos = np.array([(x, y, z) for z in zs for (x, y) in xy], np.float32)
    assert pos.shape[0] == m * per
    s.pos = pos
    s.vel = np.stack([pos[:, 2], np.zeros(len(pos)), np.zeros(len(pos))], 1).astype(np.float32)
    s.type = np.zeros(len(pos), np.int32)
    s.gid = np.arange(len(pos), dtype=np.uint32)
    o = oracle_lib.Oracle(s, compute_forces=False)
    prof = o.profile(axis=2, nbins=m)
    z32 = zs.astype(np.float32).astype(np.float64)
    assert np.array_equal(prof["count"], np.full(m, float(per)))
    np.testing.assert_allclose(prof["sum_vx"], per * z32, rtol=1e-14)
    np.testing.assert_allclose(prof["sum_v2"], per * z32 ** 2, rtol=1e-14)
    # two bins per plane spacing: every other bin is empty
    prof2 = o.profile(axis=2, nbins=2 * m)
    assert np.array_equal(prof2["count"], np.tile([0.0, per], m))
