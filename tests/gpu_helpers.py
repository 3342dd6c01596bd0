"""Shared helpers of the GPU parity tests (comparison utilities only)."""
import numpy as np


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a gfx950 device")


def force_scale(f_fluid):
    """F_scale: RMS over fluid particles of |f| (the force-norm scale)."""
    return float(np.sqrt((np.asarray(f_fluid, np.float64) ** 2).sum(axis=1).mean()))


def by_gid(oracle, arr):
    out = np.empty_like(arr)
    out[oracle.gid] = arr
    return out


def sorted_pairs(p):
    p = np.asarray(p, dtype=np.uint64)
    key = (p[:, 0] << np.uint64(32)) | p[:, 1]
    return np.sort(key)


def trilinear_f64(phi, h, x):
    """Test-side trilinear phi at positions x (N, 3), FP64 (a property check,
    independent of both the oracle and the kernels)."""
    phi = np.asarray(phi, np.float64)
    nz, ny, nx = phi.shape
    g = np.asarray(x, np.float64) / np.asarray(h)[None, :]
    i0 = np.floor(g).astype(np.int64)
    t = g - i0
    out = np.zeros(g.shape[0])
    for dz in (0, 1):
        wz = t[:, 2] if dz else 1 - t[:, 2]
        kk = np.mod(i0[:, 2] + dz, nz)
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1 - t[:, 1]
            jj = np.mod(i0[:, 1] + dy, ny)
            for dx in (0, 1):
                wx = t[:, 0] if dx else 1 - t[:, 0]
                ii = np.mod(i0[:, 0] + dx, nx)
                out += phi[kk, jj, ii] * wx * wy * wz
    return out
