"""The pair kernel's candidate pre-test never drops a pair that the exact
FP32 decision keeps (host check of the bound, no GPU).

The kernel walks neighbour-row candidates on coarse position codes: per
axis q = rint(256 x) modulo 2^10, the lane's own code shifted by the row's
periodic image rint(256 s L), and keeps a candidate when the squared
signed code difference is at most (256 rc (1 + 1e-5) + 2.6)^2 (truncated
to an integer, computed in FP32).  The exact decision of Sec. II.A, taken
afterwards on the kept candidates, is r^2 < rc^2 in FP32 with each
separation component the FP32 rounding of the exact image difference.
Here the same integer and FP32 arithmetic runs in numpy on pairs drawn at
distances around rc, in boxes larger and smaller than the codes' 4-unit
period, with image shifts whose 256 L is not an integer, and every pair
that the exact decision keeps must pass the pre-test.
"""
import numpy as np
import pytest


def _code_axis(x):
    return np.rint(x.astype(np.float32) * np.float32(256.0)).astype(np.int64) & 1023


def _shift_axis(x, sL):
    a = np.rint(x.astype(np.float32) * np.float32(256.0)).astype(np.int64)
    b = np.rint(sL.astype(np.float32) * np.float32(256.0)).astype(np.int64)
    return (a - b) & 1023


def _signed10(v):
    v = v & 1023
    return np.where(v >= 512, v - 1024, v)


def _thresh(rc2):
    rc2 = np.float32(rc2)
    if not rc2 < np.float32(3.88):
        return np.iinfo(np.uint32).max
    r = np.float32(np.sqrt(rc2)) * np.float32(256.0 * 1.00001) + np.float32(2.6)
    return int(np.float32(r * r))


def _fp32_r2(xi, xj, sL):
    # each component: the exact difference x_i - x_j - s L rounded once
    d = (xi.astype(np.float64) - sL.astype(np.float64) - xj.astype(np.float64)).astype(np.float32)
    dx, dy, dz = (d[:, k].astype(np.float64) for k in range(3))
    r2 = (dx * dx).astype(np.float32).astype(np.float64)
    r2 = (dy * dy + r2).astype(np.float32).astype(np.float64)
    return (dz * dz + r2).astype(np.float32)


@pytest.mark.parametrize("rc,L", [(1.0, 168.0), (1.0, 3.3), (0.7, 12.37), (1.5, 9.1), (1.9, 41.3)])
def test_pretest_keeps_every_exact_pair(rc, L):
    rng = np.random.default_rng(int(rc * 100 + L))
    n = 400_000
    Lv = np.full(3, L, np.float32)
    xi = (rng.random((n, 3)) * L).astype(np.float32)
    # separations concentrated around rc (and some far inside)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = np.where(rng.random(n) < 0.8, rc * (1 + rng.uniform(-3e-3, 3e-3, n)),
                 rc * rng.random(n))
    xj_un = xi.astype(np.float64) - u * r[:, None]
    # the image shift s L that brings xj into [0, L): the row's shift
    s = np.floor(xj_un / L)
    xj = (xj_un - s * L).astype(np.float32)
    xj = np.where(xj >= np.float32(L), np.float32(0.0), xj).astype(np.float32)
    sL = (s * L).astype(np.float32)           # x_i - x_j - sL is the short difference
    r2 = _fp32_r2(xi, xj, sL)
    keep_exact = r2 < np.float32(rc * rc)
    assert keep_exact.sum() > n // 2
    # codes: candidate code minus the lane's shifted code, per 10-bit field
    dq = np.stack([_signed10(_code_axis(xj[:, k]) - _shift_axis(xi[:, k], sL[:, k]))
                   for k in range(3)], axis=1)
    q2 = (dq.astype(np.int64) ** 2).sum(axis=1)
    kept = q2 <= _thresh(rc * rc)
    missed = keep_exact & ~kept
    assert not missed.any(), (int(missed.sum()), r2[missed][:5])
    # the bound is tight enough to drop most of the candidates beyond 1.02 rc
    far = r2 > np.float32((1.02 * rc) ** 2)
    if far.any():
        assert kept[far].mean() < 0.05


def test_cutoff_too_large_keeps_everything():
    assert _thresh(4.0) == np.iinfo(np.uint32).max
    assert _thresh(3.8) < 2 ** 20
