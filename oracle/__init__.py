"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path (``paper_2009_07400_amd``)
never imports it and shares no code with it.

Every function takes and returns NumPy arrays in original atom order.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = C.c_double
_I = C.c_int
_L = C.c_long
_P = C.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(_LIB_PATH)
        lib.orc_pair_force.restype = _D
        lib.orc_pair_force.argtypes = [_D, _D, _D]
        lib.orc_pair_energy.restype = _D
        lib.orc_pair_energy.argtypes = [_D, _D, _D]
        lib.orc_cells_per_axis.restype = _I
        lib.orc_cells_per_axis.argtypes = [_D, _D]
        lib.orc_num_threads.restype = _I
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [_I]
        for name in ("orc_build_list", "orc_build_list_brute"):
            f = getattr(lib, name)
            f.restype = _L
            f.argtypes = [_I, _P, _P, _P, _D, _D, _I, _P, _P]
        lib.orc_atom_neighbors.restype = _L
        lib.orc_atom_neighbors.argtypes = [_I, _P, _P, _P, _D, _D, _I, _P, _L]
        lib.orc_forces.restype = None
        lib.orc_forces.argtypes = [_I, _P, _P, _P, _D, _P, _P, _I, _D, _D, _D, _P, _P, _P, _P, _P, _P]
        lib.orc_atom_force.restype = None
        lib.orc_atom_force.argtypes = [_I, _P, _P, _P, _D, _I, _D, _D, _D, _P, _P]
        lib.orc_half_list.restype = None
        lib.orc_half_list.argtypes = [_I, _P, _P, _I, _P, _P]
        lib.orc_forces_half.restype = None
        lib.orc_forces_half.argtypes = [_I, _P, _P, _P, _D, _P, _P, _I, _D, _D, _D, _P, _P, _P, _P, _P]
        lib.orc_run.restype = _L
        lib.orc_run.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I, _P, _P, _P, _P, _P,
                                _P]
        lib.orc_jvp.restype = None
        lib.orc_jvp.argtypes = [_I, _P, _P, _P, _D, _P, _P, _I, _D, _D, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        lib.orc_adjoint.restype = _L
        lib.orc_adjoint.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I,
                                    _P, _P, _P, _P, _P, _P, _P]
        lib.orc_tangent.restype = _L
        lib.orc_tangent.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I,
                                    _P, _P, _P, _P, _P, _P, _D, _D]
        lib.orc_sd_pair.restype = _D
        lib.orc_sd_pair.argtypes = [_D, _D, _D, _D, _D, _D, _D, _D, _D, _P]
        lib.orc_sd_forces.restype = None
        lib.orc_sd_forces.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _P, _P, _I, _D, _D, _D, _P, _P, _P, _P, _P, _P]
        lib.orc_sd_atom_force.restype = None
        lib.orc_sd_atom_force.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _I, _D, _D, _D, _P]
        lib.orc_sd_run.restype = _L
        lib.orc_sd_run.argtypes = [_I, _P, _P, _P, _P, _P, _P, _D, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I, _P, _P, _P,
                                   _P]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_P)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (for timing runs)."""
    _load().orc_set_threads(int(n))


def pair_force(s: float, eps: float = 1.0, sigma: float = 1.0) -> float:
    """f(s) with F_ij = f(s) x_ij."""
    return float(_load().orc_pair_force(s, eps, sigma))


def pair_energy(s: float, eps: float = 1.0, sigma: float = 1.0) -> float:
    return float(_load().orc_pair_energy(s, eps, sigma))


def cells_per_axis(L: float, r: float) -> int:
    return int(_load().orc_cells_per_axis(L, r))


def build_list(x, y, z, L: float, r: float, maxnb: int = 160, brute: bool = False):
    """Full Verlet list; returns (count[N], nbr[N, maxnb], longest list length)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    count = np.zeros(n, dtype=np.int32)
    nbr = np.full((n, maxnb), -1, dtype=np.int32)
    fn = _load().orc_build_list_brute if brute else _load().orc_build_list
    m = fn(n, _ptr(x), _ptr(y), _ptr(z), L, r, maxnb, _ptr(count), _ptr(nbr))
    return count, nbr, int(m)


def list_as_sets(count, nbr):
    return [tuple(nbr[i, : count[i]].tolist()) for i in range(count.shape[0])]


def atom_neighbors(x, y, z, L: float, r: float, i: int, cap: int = 512) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.zeros(cap, dtype=np.int32)
    m = _load().orc_atom_neighbors(x.shape[0], _ptr(x), _ptr(y), _ptr(z), L, r, int(i), _ptr(out), cap)
    if m > cap:
        raise ValueError("neighbor capacity exceeded")
    return out[:m].copy()


def forces(x, y, z, L, count, nbr, eps=1.0, sigma=1.0, rc=2.5):
    """Returns (F[N,3], scale[N], U, W) for the given list."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    count = np.ascontiguousarray(count, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    f = np.zeros((3, n))
    scale = np.zeros(n)
    U = C.c_double()
    W = C.c_double()
    _load().orc_forces(n, _ptr(x), _ptr(y), _ptr(z), L, _ptr(count), _ptr(nbr), nbr.shape[1], eps, sigma, rc,
                       _ptr(f[0]), _ptr(f[1]), _ptr(f[2]), _ptr(scale), C.byref(U), C.byref(W))
    return f.T.copy(), scale, U.value, W.value


def half_list(count, nbr):
    """Half list of a full list (each pair once, by the lower index);
    returns (hcount[N], hnbr[N, maxnb])."""
    count = np.ascontiguousarray(count, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    n, maxnb = nbr.shape
    hcount = np.zeros(n, dtype=np.int32)
    hnbr = np.full((n, maxnb), -1, dtype=np.int32)
    _load().orc_half_list(n, _ptr(count), _ptr(nbr), maxnb, _ptr(hcount), _ptr(hnbr))
    return hcount, hnbr


def forces_half(x, y, z, L, hcount, hnbr, eps=1.0, sigma=1.0, rc=2.5):
    """Forces from a half list by Newton's third law; returns (F[N,3], U, W)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    hcount = np.ascontiguousarray(hcount, dtype=np.int32)
    hnbr = np.ascontiguousarray(hnbr, dtype=np.int32)
    f = np.zeros((3, n))
    U = C.c_double()
    W = C.c_double()
    _load().orc_forces_half(n, _ptr(x), _ptr(y), _ptr(z), L, _ptr(hcount), _ptr(hnbr), hnbr.shape[1], eps, sigma,
                            rc, _ptr(f[0]), _ptr(f[1]), _ptr(f[2]), C.byref(U), C.byref(W))
    return f.T.copy(), U.value, W.value


def atom_force(x, y, z, L, i, eps=1.0, sigma=1.0, rc=2.5):
    """All-pairs force on one atom; returns (F[3], scale)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.zeros(3)
    sc = C.c_double()
    _load().orc_atom_force(x.shape[0], _ptr(x), _ptr(y), _ptr(z), L, int(i), eps, sigma, rc, _ptr(out),
                           C.byref(sc))
    return out, sc.value


def run(x, y, z, vx, vy, vz, L, nsteps, eps=1.0, sigma=1.0, mass=1.0, rc=2.5, skin=0.3, dt=0.005,
        rebuild_every=20, maxnb=160, thermo=True, hashes=False):
    """Velocity Verlet; returns dict(x, v, f, thermo[nsteps+1, 5], maxc, hashes, times).

    hashes[k] identifies the set of interacting pairs (s < rc^2) at step k;
    times = seconds in the force sums, the list builds and the rest."""
    st = [_f64(a).copy() for a in (x, y, z, vx, vy, vz)]
    n = st[0].shape[0]
    f = np.zeros((3, n))
    th = np.zeros((nsteps + 1, 5)) if thermo else None
    hs = np.zeros(nsteps + 1, dtype=np.uint64) if hashes else None
    tm = np.zeros(3)
    m = _load().orc_run(n, *[_ptr(a) for a in st], L, eps, sigma, mass, rc, skin, dt, rebuild_every, maxnb,
                        nsteps, _ptr(th) if thermo else None, _ptr(f[0]), _ptr(f[1]), _ptr(f[2]),
                        _ptr(hs) if hashes else None, _ptr(tm))
    if m > maxnb:
        raise ValueError(f"neighbor list overflow: {m} > {maxnb}")
    return {"x": np.stack(st[:3], 1), "v": np.stack(st[3:], 1), "f": f.T.copy(), "thermo": th, "maxc": int(m),
            "hashes": hs, "times": {"force": float(tm[0]), "neigh": float(tm[1]), "other": float(tm[2])}}


def jvp(x, y, z, L, count, nbr, w, eps=1.0, sigma=1.0, rc=2.5, a=None):
    """(J w) for J = dF/dx with the list fixed; with a given, also returns
    (sum_i a_i . dF_i/deps, sum_i a_i . dF_i/dsigma)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.shape[0]
    w = _f64(np.asarray(w).T)
    out = np.zeros((3, n))
    count = np.ascontiguousarray(count, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    gpar = np.zeros(2)
    if a is not None:
        aT = _f64(np.asarray(a).T)
        ap = (_ptr(aT[0]), _ptr(aT[1]), _ptr(aT[2]), _ptr(gpar))
    else:
        ap = (None, None, None, None)
    _load().orc_jvp(n, _ptr(x), _ptr(y), _ptr(z), L, _ptr(count), _ptr(nbr), nbr.shape[1], eps, sigma, rc,
                    _ptr(w[0]), _ptr(w[1]), _ptr(w[2]), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), *ap)
    return (out.T.copy(), gpar) if a is not None else out.T.copy()


def adjoint(x0, v0, L, nsteps, lam_x, lam_v, eps=1.0, sigma=1.0, mass=1.0, rc=2.5, skin=0.3, dt=0.005,
            rebuild_every=20, maxnb=160):
    """Reverse-mode derivative; returns (lam_x0[N,3], lam_v0[N,3], d_eps, d_sigma)."""
    x0 = _f64(np.asarray(x0).T)
    v0 = _f64(np.asarray(v0).T)
    lx = _f64(np.asarray(lam_x).T).copy()
    lv = _f64(np.asarray(lam_v).T).copy()
    n = x0.shape[1]
    g = np.zeros(2)
    m = _load().orc_adjoint(n, _ptr(x0[0]), _ptr(x0[1]), _ptr(x0[2]), _ptr(v0[0]), _ptr(v0[1]), _ptr(v0[2]), L,
                            eps, sigma, mass, rc, skin, dt, rebuild_every, maxnb, nsteps, _ptr(lx[0]),
                            _ptr(lx[1]), _ptr(lx[2]), _ptr(lv[0]), _ptr(lv[1]), _ptr(lv[2]), _ptr(g))
    if m > maxnb:
        raise ValueError("neighbor list overflow")
    return lx.T.copy(), lv.T.copy(), float(g[0]), float(g[1])


def tangent(x0, v0, L, nsteps, dx, dv, d_eps, d_sigma, eps=1.0, sigma=1.0, mass=1.0, rc=2.5, skin=0.3,
            dt=0.005, rebuild_every=20, maxnb=160):
    """Forward-mode derivative; returns (dx_T[N,3], dv_T[N,3])."""
    x0 = _f64(np.asarray(x0).T)
    v0 = _f64(np.asarray(v0).T)
    tx = _f64(np.asarray(dx).T).copy()
    tv = _f64(np.asarray(dv).T).copy()
    n = x0.shape[1]
    m = _load().orc_tangent(n, _ptr(x0[0]), _ptr(x0[1]), _ptr(x0[2]), _ptr(v0[0]), _ptr(v0[1]), _ptr(v0[2]), L,
                            eps, sigma, mass, rc, skin, dt, rebuild_every, maxnb, nsteps, _ptr(tx[0]),
                            _ptr(tx[1]), _ptr(tx[2]), _ptr(tv[0]), _ptr(tv[1]), _ptr(tv[2]), d_eps, d_sigma)
    if m > maxnb:
        raise ValueError("neighbor list overflow")
    return tx.T.copy(), tv.T.copy()


# ---------------------------------------------------------------- Spring-Dashpot (Eq. 3)

def sd_pair(d, dv, k, gamma, sigma):
    """Force on i of one pair (separation d = x_i - x_j, relative velocity
    dv = v_i - v_j); returns (F[3], magnitude along the unit vector)."""
    out = np.zeros(3)
    fm = _load().orc_sd_pair(float(d[0]), float(d[1]), float(d[2]), float(dv[0]), float(dv[1]), float(dv[2]),
                             k, gamma, sigma, _ptr(out))
    return out, float(fm)


def sd_forces(x, v, L, count, nbr, k, gamma, sigma):
    """Spring-Dashpot forces for the given list; x, v [N, 3].  Returns
    (F[N, 3], scale[N] = sum_j |F_ij|, U elastic, W virial)."""
    xT = _f64(np.asarray(x).T)
    vT = _f64(np.asarray(v).T)
    n = xT.shape[1]
    count = np.ascontiguousarray(count, dtype=np.int32)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    f = np.zeros((3, n))
    scale = np.zeros(n)
    U = C.c_double()
    W = C.c_double()
    _load().orc_sd_forces(n, _ptr(xT[0]), _ptr(xT[1]), _ptr(xT[2]), _ptr(vT[0]), _ptr(vT[1]), _ptr(vT[2]), L,
                          _ptr(count), _ptr(nbr), nbr.shape[1], k, gamma, sigma, _ptr(f[0]), _ptr(f[1]), _ptr(f[2]),
                          _ptr(scale), C.byref(U), C.byref(W))
    return f.T.copy(), scale, U.value, W.value


def sd_atom_force(x, v, L, i, k, gamma, sigma):
    """All-pairs Spring-Dashpot force on one sphere (no list)."""
    xT = _f64(np.asarray(x).T)
    vT = _f64(np.asarray(v).T)
    out = np.zeros(3)
    _load().orc_sd_atom_force(xT.shape[1], _ptr(xT[0]), _ptr(xT[1]), _ptr(xT[2]), _ptr(vT[0]), _ptr(vT[1]),
                              _ptr(vT[2]), L, int(i), k, gamma, sigma, _ptr(out))
    return out


def sd_run(x, v, L, nsteps, k, gamma, sigma=1.0, mass=1.0, cutoff=1.0, skin=0.3, dt=0.001, rebuild_every=20,
           maxnb=64, thermo=True):
    """Velocity Verlet of Spring-Dashpot spheres; x, v [N, 3].  Returns
    dict(x, v, f, thermo[nsteps+1, 5] = (KE, T, U elastic, W, KE + U), maxc)."""
    xT = _f64(np.asarray(x).T).copy()
    vT = _f64(np.asarray(v).T).copy()
    n = xT.shape[1]
    f = np.zeros((3, n))
    th = np.zeros((nsteps + 1, 5)) if thermo else None
    m = _load().orc_sd_run(n, _ptr(xT[0]), _ptr(xT[1]), _ptr(xT[2]), _ptr(vT[0]), _ptr(vT[1]), _ptr(vT[2]), L, k,
                           gamma, sigma, mass, cutoff, skin, dt, rebuild_every, maxnb, nsteps,
                           _ptr(th) if thermo else None, _ptr(f[0]), _ptr(f[1]), _ptr(f[2]))
    if m > maxnb:
        raise ValueError(f"neighbor list overflow: {m} > {maxnb}")
    return {"x": xT.T.copy(), "v": vT.T.copy(), "f": f.T.copy(), "thermo": th, "maxc": int(m)}
