"""FP64 CPU oracle for the SPH density / smoothing-length / force path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark use it; the GPU library never does.  It is a thin
ctypes binding over ``sph_oracle.c`` (plain C, FP64, OpenMP), which computes
the plain definitions of the density and force stages of Section II with an
exact neighbour search.  See the header of ``sph_oracle.c`` for what each
function follows.

Pinned by ``tests/test_oracle_pins.py`` (kernel normalisation and shape,
finite-difference derivatives, Lagrangian force and adiabatic du/dt,
conservation, lattice symmetry and counts, the paper's printed candidate
fractions, brute force vs grid vs an independent k-d tree, and the viscosity,
sound speed and signal velocity of an isolated approaching / receding pair,
also across a periodic face, written out from their definitions with the
kernel derivatives taken by finite differences of scipy's B-spline and the
sound speed from dP/drho along the adiabat).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "libsphoracle.so")

GAMMA = 5.0 / 3.0      # Section III-B constants
ALPHA = 2.0
N_NGB = 48.0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        d, i64, vp = C.c_double, C.c_int64, C.c_void_p
        L.ora_kernel_f.restype = d; L.ora_kernel_f.argtypes = [d]
        L.ora_kernel_df.restype = d; L.ora_kernel_df.argtypes = [d]
        L.ora_W.restype = d; L.ora_W.argtypes = [d, d]
        L.ora_dWdh.restype = d; L.ora_dWdh.argtypes = [d, d]
        L.ora_gradW_factor.restype = d; L.ora_gradW_factor.argtypes = [d, d]
        L.ora_mix.restype = C.c_uint64; L.ora_mix.argtypes = [C.c_uint64]
        L.ora_density.argtypes = [i64, vp, vp, vp, d, vp, vp, i64, vp, C.c_int] + [vp] * 6
        L.ora_solve_h.argtypes = [i64, vp, vp, vp, d, vp, vp, i64, vp, C.c_int, d, d, C.c_int, vp, vp]
        L.ora_ghost.argtypes = [i64, vp, vp, vp, vp, d, vp, vp, vp, vp]
        L.ora_force.argtypes = [i64, vp, vp, vp, d] + [vp] * 8 + [d, d, i64, vp, C.c_int] + [vp] * 8
        L.ora_sums.argtypes = [i64] + [vp] * 10
        L.ora_near_cutoff.argtypes = [i64, vp, vp, vp, d, vp, d, C.c_int, i64, vp, vp]
        L.ora_force_neighbours.argtypes = [i64, vp, vp, vp, d, vp, i64, vp, vp]
        L.ora_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.ndim == 0:
        a = np.full(n, float(a))
    return a


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _targets(targets):
    if targets is None:
        return 0, None
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    return t.size, t


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def W(r, h):
    return lib().ora_W(float(r), float(h))


def dWdh(r, h):
    return lib().ora_dWdh(float(r), float(h))


def gradW_factor(r, h):
    return lib().ora_gradW_factor(float(r), float(h))


def kernel_f(q):
    return lib().ora_kernel_f(float(q))


def kernel_df(q):
    return lib().ora_kernel_df(float(q))


def mix(j):
    return int(lib().ora_mix(int(j)))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def density(x, y, z, h, m, box=1.0, targets=None, brute=False):
    """Density stage at fixed h.  Returns dict of per-particle arrays
    (entries outside ``targets`` are zero)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    h, m = _f64(h, n), _f64(m, n)
    nt, t = _targets(targets)
    out = {k: np.zeros(n) for k in ("rho", "drho_dh", "nw", "dnw_dh")}
    out["nngb"] = np.zeros(n, dtype=np.int64)
    out["hash"] = np.zeros(n, dtype=np.uint64)
    st = lib().ora_density(n, _ptr(x), _ptr(y), _ptr(z), box, _ptr(h), _ptr(m), nt, _ptr(t),
                           int(brute), _ptr(out["rho"]), _ptr(out["drho_dh"]), _ptr(out["nw"]),
                           _ptr(out["dnw_dh"]), _ptr(out["nngb"]), _ptr(out["hash"]))
    if st:
        raise OracleError(st, "density")
    return out


def solve_h(x, y, z, m, h0, box=1.0, targets=None, brute=False, target_nw=N_NGB, tol=1e-9,
            max_iter=100, allow_noconv=False):
    """Per-particle safeguarded Newton on N_w(h) = target_nw.  Returns (h, iters)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    m = _f64(m, n)
    h = _f64(h0, n).copy()
    nt, t = _targets(targets)
    iters = np.zeros(n, dtype=np.int32)
    bad = np.zeros(1, dtype=np.int64)
    st = lib().ora_solve_h(n, _ptr(x), _ptr(y), _ptr(z), box, _ptr(m), _ptr(h), nt, _ptr(t),
                           int(brute), float(target_nw), float(tol), int(max_iter), _ptr(iters),
                           _ptr(bad))
    if st and not (allow_noconv and st == -5):
        raise OracleError(st, "solve_h")
    return h, iters


def ghost(h, rho, drho_dh, u, gamma=GAMMA):
    h, rho, drho_dh = _f64(h), _f64(rho), _f64(drho_dh)
    n = h.size
    u = _f64(u, n)
    out = {k: np.zeros(n) for k in ("P", "c", "f", "A")}
    lib().ora_ghost(n, _ptr(h), _ptr(rho), _ptr(drho_dh), _ptr(u), float(gamma), _ptr(out["P"]),
                    _ptr(out["c"]), _ptr(out["f"]), _ptr(out["A"]))
    return out


def force(x, y, z, h, m, vx, vy, vz, u, rho, drho_dh, box=1.0, gamma=GAMMA, alpha=ALPHA,
          targets=None, brute=False):
    """Force stage.  rho / drho_dh must be valid for every particle that is a
    neighbour of a target.  Returns dict of per-particle arrays."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    h, m = _f64(h, n), _f64(m, n)
    vx, vy, vz, u = _f64(vx, n), _f64(vy, n), _f64(vz, n), _f64(u, n)
    rho, drho_dh = _f64(rho, n), _f64(drho_dh, n)
    nt, t = _targets(targets)
    out = {k: np.zeros(n) for k in ("ax", "ay", "az", "dudt", "vsig", "S")}
    out["nforce"] = np.zeros(n, dtype=np.int64)
    out["hash"] = np.zeros(n, dtype=np.uint64)
    st = lib().ora_force(n, _ptr(x), _ptr(y), _ptr(z), box, _ptr(h), _ptr(m), _ptr(vx), _ptr(vy),
                         _ptr(vz), _ptr(u), _ptr(rho), _ptr(drho_dh), float(gamma), float(alpha),
                         nt, _ptr(t), int(brute), _ptr(out["ax"]), _ptr(out["ay"]), _ptr(out["az"]),
                         _ptr(out["dudt"]), _ptr(out["vsig"]), _ptr(out["S"]), _ptr(out["nforce"]),
                         _ptr(out["hash"]))
    if st:
        raise OracleError(st, "force")
    return out


def sums(m, vx, vy, vz, ax, ay, az, dudt, S):
    arrs = [_f64(a) for a in (m, vx, vy, vz, ax, ay, az, dudt, S)]
    out = np.zeros(5)
    lib().ora_sums(arrs[0].size, *[_ptr(a) for a in arrs], _ptr(out))
    return {"M": out[:3].copy(), "E": float(out[3]), "scale": float(out[4])}


def near_cutoff(x, y, z, h, box=1.0, rel=1e-6, brute=False, targets=None):
    """Per particle (or per target): True if some pair lies within rel of
    its own or the partner's cutoff."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    h = _f64(h, n)
    nt, t = _targets(targets)
    flag = np.zeros(n, dtype=np.uint8)
    st = lib().ora_near_cutoff(n, _ptr(x), _ptr(y), _ptr(z), box, _ptr(h), float(rel), int(brute), nt, _ptr(t),
                               _ptr(flag))
    if st:
        raise OracleError(st, "near_cutoff")
    return flag.astype(bool)


def force_neighbours(x, y, z, h, targets, box=1.0):
    """Mask of the targets and of all their force neighbours."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    h = _f64(h, n)
    nt, t = _targets(targets)
    mark = np.zeros(n, dtype=np.uint8)
    st = lib().ora_force_neighbours(n, _ptr(x), _ptr(y), _ptr(z), box, _ptr(h), nt, _ptr(t), _ptr(mark))
    if st:
        raise OracleError(st, "force_neighbours")
    return mark.astype(bool)


def run_all(ps, h, gamma=GAMMA, alpha=ALPHA, brute=False, targets=None):
    """Density then force at fixed h for a ParticleSet-like object."""
    d = density(ps.x, ps.y, ps.z, h, ps.m, ps.box, targets=None, brute=brute)
    f = force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"], d["drho_dh"],
              ps.box, gamma, alpha, targets=targets, brute=brute)
    return d, f
