"""FP64 oracle of the DPD step with phase-field bounce-back (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only users.  The GPU library never
imports, links or calls anything here, and this package imports nothing from
the GPU package; both take their inputs from `workloads`.

The arithmetic lives in `dpd_oracle.c` (plain C, FP64, OpenMP over
particles), built by `build_oracle()` with gcc and loaded through ctypes.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build_oracle(force: bool = True, sanitize=False, path: str | None = None) -> str:
    """Compile the oracle with gcc (no contraction, so FP32 decisions follow
    the written op order).  sanitize=True or "undefined" builds it with the
    undefined-behaviour sanitizer, "address" with the address sanitizer
    (a process that loads it must preload libasan), both aborting on the
    first report, into `path`."""
    out = path or _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        if sanitize:
            kind = "undefined" if sanitize is True else str(sanitize)
            cmd[1:1] = ["-g", "-fno-omit-frame-pointer", "-fsanitize=" + kind,
                        "-fno-sanitize-recover=all"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


class Geom(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("nc", C.c_int32 * 3), ("L32", C.c_float * 3),
                ("invw32", C.c_float * 3), ("ng", C.c_int32 * 3), ("h", C.c_double * 3),
                ("inv_h32", C.c_float * 3), ("inv_h64", C.c_double * 3),
                ("phi64", C.c_void_p), ("phi32", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("a", (C.c_double * 2) * 2), ("gamma", C.c_double), ("kBT", C.c_double),
                ("rc", C.c_double), ("dt", C.c_double), ("lam", C.c_double),
                ("g", C.c_double * 3), ("seed", C.c_uint64), ("replica", C.c_uint32),
                ("specular", C.c_int32), ("sph", C.c_int32), ("sr", (C.c_double * 2) * 2),
                ("sa", (C.c_double * 2) * 2), ("r0r", C.c_double), ("r0a", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("DPD_ORACLE_LIB")   # another build, e.g. the sanitized one
        if not path:
            if not os.path.exists(_LIB):
                build_oracle(force=False)
            path = _LIB
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_uniform_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, P]
        L.orc_xi.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32]
        L.orc_xi.restype = C.c_double
        L.orc_xi_fill.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, C.c_uint64,
                                  C.c_uint32, P]
        L.orc_pairs_random.argtypes = [C.c_uint64, P, P, C.c_int64, C.c_uint64, C.c_uint32, P, P]
        L.orc_cell_of.argtypes = [P, P]
        L.orc_cell_of.restype = C.c_int32
        L.orc_phi_decide32.argtypes = [P, P]
        L.orc_phi_decide32.restype = C.c_float
        L.orc_phi_decide64.argtypes = [P, P]
        L.orc_phi_decide64.restype = C.c_double
        L.orc_phi64.argtypes = [P, P, P]
        L.orc_phi64.restype = C.c_double
        L.orc_sph_w.argtypes = [C.c_double, C.c_double]
        L.orc_sph_w.restype = C.c_double
        L.orc_sph_dw.argtypes = [C.c_double, C.c_double]
        L.orc_sph_dw.restype = C.c_double
        L.orc_forces.argtypes = [P, P, C.c_int64, P, P, P, P, P, C.c_uint64, C.c_int, C.c_int, P]
        L.orc_forces.restype = C.c_int
        L.orc_cells_of.argtypes = [P, C.c_int64, P, P]
        L.orc_pairs.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_int64]
        L.orc_pairs.restype = C.c_int64
        L.orc_step.argtypes = [P, P, C.c_int64, P, P, P, P, P, P, P, P, C.c_int, P]
        L.orc_step.restype = C.c_int
        L.orc_potential.argtypes = [P, P, C.c_int64, P, P]
        L.orc_potential.restype = C.c_double
        L.orc_profile.argtypes = [P, C.c_int64, P, P, P, C.c_int, C.c_int, P, P, P, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_window.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_uint64, C.c_int, C.c_int,
                                 C.c_int, C.c_int, P, P, P, P, P, P, P]
        L.orc_window.restype = C.c_int
        L.orc_window_start_force.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_uint64, P]
        L.orc_window_start_force.restype = C.c_int
        L.orc_window_step.argtypes = [P, P, C.c_int64, P, P, P, P, P, C.c_uint64, C.c_int,
                                      C.c_int, P, P, P, P, P]
        L.orc_window_step.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def xi(seed, gi, gj, k, replica=0):
    return lib().orc_xi(seed, gi, gj, k, replica)


def xi_fill(seed, gi, gj0, count, k, replica=0):
    out = np.zeros(int(count), np.float64)
    lib().orc_xi_fill(seed, gi, gj0, int(count), k, replica, _p(out))
    return out


def pairs_random(seed, gi, gj, k, replica=0):
    """Philox words (n, 4) and xi (n,) of the pairs (gi[m], gj[m])."""
    gi = np.ascontiguousarray(gi, np.uint32)
    gj = np.ascontiguousarray(gj, np.uint32)
    n = gi.shape[0]
    words = np.zeros((n, 4), np.uint32)
    xi_out = np.zeros(n, np.float64)
    lib().orc_pairs_random(int(seed) & 0xFFFFFFFFFFFFFFFF, _p(gi), _p(gj), n, int(k),
                           int(replica), _p(words), _p(xi_out))
    return words, xi_out


def sph_w(r, r0):
    """Smoothing function of Eq. 23 (3-D) with support r0."""
    return lib().orc_sph_w(float(r), float(r0))


def sph_dw(r, r0):
    """dW/dr of Eq. 23 (3-D) with support r0."""
    return lib().orc_sph_dw(float(r), float(r0))


def cell_counts(L, rc):
    """Cells per axis: floor(L / rc), each at least rc wide."""
    return np.array([int(math.floor(float(x) / rc)) for x in L], dtype=np.int32)


class Oracle:
    """FP64 state of one box advanced by the oracle step.

    Takes a `workloads.System` (FP32 inputs, converted exactly to FP64) and
    keeps r, v, f, the force index k and the FP32 shadow positions on which
    the last discrete decisions were taken.  `mode` selects the force
    routine: 2 cell list (default), 1 brute force with the same FP32
    decisions, 0 brute force with the FP64 cutoff test.
    """

    def __init__(self, system, params=None, mode=2, compute_forces=True):
        self.system = system
        p = dict(system.params if params is None else params)
        self.params = p
        self.mode = mode
        self.n = system.n
        self.type = np.ascontiguousarray(system.type, dtype=np.int32)
        self.gid = np.ascontiguousarray(system.gid, dtype=np.uint32)
        self.r = np.ascontiguousarray(system.pos, dtype=np.float64).copy()
        # a wall particle's velocity is the velocity of its solid (it stays in place)
        self.v = np.ascontiguousarray(system.vel, dtype=np.float64).copy()
        self.f = np.zeros((self.n, 3), np.float64)
        self.vt = self.v.copy()
        self.xs = np.ascontiguousarray(system.pos, dtype=np.float32).copy()
        self.events = np.zeros(self.n, np.int32)
        self.k = 0
        phi = system.phi
        self.phi64 = np.ascontiguousarray(phi, dtype=np.float64)
        self.phi32 = np.ascontiguousarray(phi) if phi.dtype == np.float32 else None
        L = np.asarray(system.L, dtype=np.float64)
        h = np.asarray(system.h, dtype=np.float64)
        nc = cell_counts(L, p["rc"])
        if np.any(nc < 3):
            raise ValueError("box must hold at least 3 cells per axis")
        g = Geom()
        for a in range(3):
            g.L[a] = L[a]
            g.nc[a] = int(nc[a])
            g.L32[a] = float(np.float32(L[a]))
            g.invw32[a] = float(np.float32(nc[a] / L[a]))
            g.h[a] = h[a]
            g.inv_h32[a] = float(np.float32(1.0 / h[a]))
            g.inv_h64[a] = 1.0 / h[a]
        g.ng[0], g.ng[1], g.ng[2] = phi.shape[2], phi.shape[1], phi.shape[0]
        g.phi64 = self.phi64.ctypes.data
        g.phi32 = self.phi32.ctypes.data if self.phi32 is not None else None
        self.geom = g
        self.nc = nc
        self.cparams = self._make_params(p)
        if compute_forces:
            self.f = self.forces(k=0)

    @staticmethod
    def _make_params(p):
        cp = Params()
        for i in range(2):
            for j in range(2):
                cp.a[i][j] = float(p["a"][i][j])
        cp.gamma = float(p["gamma"])
        cp.kBT = float(p["kBT"])
        cp.rc = float(p["rc"])
        cp.dt = float(p["dt"])
        cp.lam = float(p["lam"])
        for a in range(3):
            cp.g[a] = float(p["g"][a])
        cp.seed = int(p["seed"]) & 0xFFFFFFFFFFFFFFFF
        cp.replica = int(p["replica"])
        cp.specular = 1 if p.get("specular", False) else 0
        sph = p.get("sph")
        if sph:
            # Eq. 22-24: strengths by type and the two ranges
            cp.sph = 1
            for i in range(2):
                for j in range(2):
                    cp.sr[i][j] = float(sph["sr"][i][j])
                    cp.sa[i][j] = float(sph["sa"][i][j])
            cp.r0r = float(sph["r0r"])
            cp.r0a = float(sph["r0a"])
        return cp

    def set_params(self, **kw):
        self.params.update(kw)
        self.cparams = self._make_params(self.params)

    def set_state(self, pos, vel, force, k):
        """Load an FP32 snapshot (exactly representable in FP64)."""
        self.r = np.ascontiguousarray(pos, dtype=np.float64).copy()
        self.v = np.ascontiguousarray(vel, dtype=np.float64).copy()
        self.f = np.ascontiguousarray(force, dtype=np.float64).copy()
        self.xs = np.ascontiguousarray(pos, dtype=np.float32).copy()
        self.k = int(k)

    def forces(self, k=None, mode=None, all_particles=False, vt=None, xs=None, r=None):
        """Forces at the current positions (Eq. 2) with predicted velocities vt."""
        k = self.k if k is None else k
        mode = self.mode if mode is None else mode
        vt = self.v if vt is None else vt
        xs = self.r.astype(np.float32) if xs is None else xs
        r = self.r if r is None else r
        f = np.zeros((self.n, 3), np.float64)
        rc = lib().orc_forces(C.byref(self.geom), C.byref(self.cparams), self.n,
                              _p(np.ascontiguousarray(r)), _p(np.ascontiguousarray(vt)),
                              _p(np.ascontiguousarray(xs, dtype=np.float32)),
                              _p(self.type), _p(self.gid), int(k), int(mode),
                              int(bool(all_particles)), _p(f))
        if rc != 0:
            raise MemoryError("oracle force allocation failed")
        return f

    def step(self, nsteps=1):
        """Advance nsteps; returns the event codes of the last step."""
        L = lib()
        for _ in range(int(nsteps)):
            k = C.c_uint64(self.k)
            rc = L.orc_step(C.byref(self.geom), C.byref(self.cparams), self.n,
                            _p(self.r), _p(self.v), _p(self.f), _p(self.type), _p(self.gid),
                            C.byref(k), _p(self.events), _p(self.xs), int(self.mode), _p(self.vt))
            if rc != 0:
                raise MemoryError("oracle step allocation failed")
            self.k = int(k.value)
        return self.events.copy()

    def set_phi(self, phi):
        """Replace the phase-field values (same shape); the FP64 copy drives the
        physics (Eq. 17 and its gradient), the FP32 copy the decisions of an
        FP32 grid."""
        phi = np.asarray(phi)
        assert phi.shape == self.phi64.shape
        self.phi64 = np.ascontiguousarray(phi, dtype=np.float64)
        self.geom.phi64 = self.phi64.ctypes.data
        if self.phi32 is not None:
            self.phi32 = np.ascontiguousarray(phi, dtype=np.float32)
            self.geom.phi32 = self.phi32.ctypes.data

    def window(self, T, axis=2, nbins=40, logs=None, k0=None):
        """Window of T steps from the current (r, v) at force index k0 (default
        the current k), the carried force refreshed first; the state itself is
        left unchanged.  Without `logs` every decision is taken and logged; with
        the logs of an earlier call they are replayed (frozen-event form).
        Returns dict(profile, sums, counts, logs, r, v): profile[b] =
        sums[b] / counts[b] is the window mean of v_x in bin b along `axis`."""
        n, T = self.n, int(T)
        if self.params.get("specular", False) or np.any(self.v[self.type != 0] != 0.0):
            raise ValueError("the window covers resting walls with bounce-back only")
        if self.params.get("sph"):
            raise ValueError("the window covers the a w conservative force only")
        record = logs is None
        if record:
            logs = dict(ev=np.zeros((T, n), np.int32), xs=np.zeros((T, n, 3), np.float32),
                        bin=np.zeros((T, n), np.int32), T=T, axis=axis, nbins=nbins)
        else:
            assert logs["T"] == T and logs["axis"] == axis and logs["nbins"] == nbins
        sums = np.zeros(nbins, np.float64)
        counts = np.zeros(nbins, np.float64)
        r_out = np.zeros((n, 3), np.float64)
        v_out = np.zeros((n, 3), np.float64)
        k0 = self.k if k0 is None else int(k0)
        rc = lib().orc_window(C.byref(self.geom), C.byref(self.cparams), n,
                              _p(np.ascontiguousarray(self.r)), _p(np.ascontiguousarray(self.v)),
                              _p(self.type), _p(self.gid), k0, T, int(axis), int(nbins),
                              int(record), _p(logs["ev"]), _p(logs["xs"]), _p(logs["bin"]),
                              _p(sums), _p(counts), _p(r_out), _p(v_out))
        if rc != 0:
            raise MemoryError("oracle window allocation failed")
        prof = sums / np.maximum(counts, 1.0)
        return dict(profile=prof, sums=sums, counts=counts, logs=logs, r=r_out, v=v_out)

    def window_start_force(self, r, v, k0):
        """f0 = F(r, v; k0) + g as the window starts: pairs decided at fl32(r),
        w = 1 - r/rc unclamped (rows in this oracle's particle order)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        f = np.zeros((self.n, 3), np.float64)
        rc = lib().orc_window_start_force(C.byref(self.geom), C.byref(self.cparams), self.n,
                                          _p(r), _p(v), _p(self.type), _p(self.gid), int(k0),
                                          _p(f))
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        return f

    def window_step(self, r, v, f, k, ev_t, xs_t, bin_t, axis=2, nbins=40):
        """One window step with every decision read from the step's logs
        (event codes ev_t, decision positions xs_t, bins bin_t), from the
        state (r, v, f); the new force at index k.  Returns (r, v, f, sums,
        counts) of the step (new arrays)."""
        r = np.array(r, dtype=np.float64, order="C")
        v = np.array(v, dtype=np.float64, order="C")
        f = np.array(f, dtype=np.float64, order="C")
        sums = np.zeros(nbins)
        counts = np.zeros(nbins)
        rc = lib().orc_window_step(C.byref(self.geom), C.byref(self.cparams), self.n, _p(r),
                                   _p(v), _p(f), _p(self.type), _p(self.gid), int(k), int(axis),
                                   int(nbins), _p(np.ascontiguousarray(ev_t, np.int32)),
                                   _p(np.ascontiguousarray(xs_t, np.float32)),
                                   _p(np.ascontiguousarray(bin_t, np.int32)), _p(sums),
                                   _p(counts))
        if rc != 0:
            raise MemoryError("oracle window step allocation failed")
        return r, v, f, sums, counts

    def cells(self, xs=None):
        xs = self.xs if xs is None else np.ascontiguousarray(xs, dtype=np.float32)
        out = np.zeros(self.n, np.int32)
        lib().orc_cells_of(C.byref(self.geom), self.n, _p(xs), _p(out))
        return out

    def pairs(self, xs=None):
        """Interacting (gid_i, gid_j) pairs from each fluid i (FP32 decision)."""
        xs = self.xs if xs is None else np.ascontiguousarray(xs, dtype=np.float32)
        cnt = lib().orc_pairs(C.byref(self.geom), C.byref(self.cparams), self.n, _p(xs),
                              _p(self.type), _p(self.gid), C.c_void_p(0), 0)
        out = np.zeros((max(cnt, 1), 2), np.uint32)
        cnt2 = lib().orc_pairs(C.byref(self.geom), C.byref(self.cparams), self.n, _p(xs),
                               _p(self.type), _p(self.gid), _p(out), cnt)
        assert cnt2 == cnt
        return out[:cnt]

    def phi_decide(self, x32):
        x = np.ascontiguousarray(x32, dtype=np.float32)
        if self.phi32 is not None:
            return lib().orc_phi_decide32(C.byref(self.geom), _p(x))
        return lib().orc_phi_decide64(C.byref(self.geom), _p(x))

    def phi(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros(3)
        val = lib().orc_phi64(C.byref(self.geom), _p(x), _p(g))
        return val, g

    def potential(self):
        return lib().orc_potential(C.byref(self.geom), C.byref(self.cparams), self.n,
                                   _p(self.r), _p(self.type))

    def kinetic(self):
        fl = self.type == 0
        return 0.5 * float((self.v[fl] ** 2).sum())

    def profile(self, axis=2, nbins=100):
        cnt = np.zeros(nbins); svx = np.zeros(nbins); sv2 = np.zeros(nbins)
        sv = np.zeros((nbins, 3))
        lib().orc_profile(C.byref(self.geom), self.n, _p(self.r), _p(self.v), _p(self.type),
                          int(axis), int(nbins), _p(cnt), _p(svx), _p(sv2), _p(sv))
        return dict(count=cnt, sum_vx=svx, sum_v2=sv2, sum_v=sv)

    def by_gid(self, arr):
        """Rows of a per-particle array reordered so that row g is gid g."""
        out = np.empty_like(arr)
        out[self.gid] = arr
        return out


def num_threads():
    return lib().orc_num_threads()
