"""Python marshalling for the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
links, loads or calls it, and it shares no code with the GPU path.

Every function here only converts numpy arrays to pointers and back; all
arithmetic happens in ``oracle.c``, which states the definition each routine
follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FMA contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64


def _declare(L):
    L.orc_min_image.argtypes = [P, P, P]
    L.orc_wrap.argtypes = [I64, P, P]
    L.orc_neighbor_counts.argtypes = [I64, P, P, P, C.c_double, C.c_double, P, I64, P, P, P]
    L.orc_neighbor_counts.restype = I64
    L.orc_neighbor_lists.argtypes = [I64, P, P, P, C.c_double, C.c_double, P, I64, P, P, P, P]
    L.orc_philox4x32_10.argtypes = [P, P, P]
    L.orc_dpd_theta.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
    L.orc_dpd_theta.restype = C.c_double
    L.orc_pair_forces.argtypes = [C.c_int, I64, P, P, P, P, P, P, C.c_uint64, P, I64, P, P,
                                  P, P, P, P]
    L.orc_pair_forces.restype = C.c_int
    L.orc_bond_forces.argtypes = [I64, P, P, P, I64, P, P, P, P, P]
    L.orc_bond_forces.restype = I64
    L.orc_thermo.argtypes = [I64, P, P, P, P]
    L.orc_run_nve.argtypes = [C.c_int, I64, P, P, P, P, P, I64, P, P, C.c_double, C.c_uint64,
                              I64, P, C.c_int, P]
    L.orc_run_nve.restype = C.c_int
    L.orc_run_nvt.argtypes = [C.c_int, I64, P, P, P, P, P, I64, P, P, C.c_double, C.c_uint64,
                              I64, P, P, P, P, P]
    L.orc_run_nvt.restype = C.c_int
    L.orc_cell_bins.argtypes = [P, C.c_double, P]
    L.orc_cell_list.argtypes = [I64, P, P, P, P, P, P, P]
    L.orc_morton_keys.argtypes = [I64, P, P, P]
    L.orc_stable_order.argtypes = [I64, P, P]
    L.orc_ghost_masks.argtypes = [I64, P, P, P, C.c_double, P]
    L.orc_ghost_list.argtypes = [I64, P, P, P, P]
    L.orc_ghost_list.restype = I64
    L.orc_ghost_receive.argtypes = [I64, P, P, C.c_int32, P, P, P, C.c_double, P, P, I64]
    L.orc_ghost_receive.restype = I64


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _per(periodic) -> np.ndarray:
    if periodic is None:
        periodic = (1, 1, 1)
    return _i32(np.broadcast_to(np.asarray(periodic, dtype=np.int32), (3,)))


def _box(L) -> np.ndarray:
    return _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))


def exclusions(n: int, bonds: Optional[np.ndarray]) -> Tuple[Optional[np.ndarray], Optional[np.ndarray]]:
    """Per-particle partner lists (CSR) from an (nb, 2) index-pair array."""
    if bonds is None or len(bonds) == 0:
        return None, None
    b = np.asarray(bonds, dtype=np.int64)
    a = np.concatenate([b[:, 0], b[:, 1]])
    p = np.concatenate([b[:, 1], b[:, 0]])
    order = np.lexsort((p, a))
    a, p = a[order], p[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, a + 1, 1)
    off = np.cumsum(off)
    return _i64(off), _i32(p)


def min_image(d, L, periodic=None) -> np.ndarray:
    d = _f64(np.array(d, dtype=np.float64).reshape(3))
    L_, per = _box(L), _per(periodic)
    lib().orc_min_image(_p(d), _p(L_), _p(per))
    return d


def wrap(pos, L) -> np.ndarray:
    x = _f64(np.array(pos, dtype=np.float64))
    L_ = _box(L)
    lib().orc_wrap(x.shape[0], _p(x), _p(L_))
    return x


def neighbors(pos, L, r_cut, r_buff, which=None, periodic=None, bonds=None):
    """Brute-force Verlet neighbour sets.  Returns (offsets, idx) in CSR form
    over the requested particles; each row is ascending."""
    pos = _f64(pos)
    n = pos.shape[0]
    w = None if which is None else _i64(which)
    m = n if w is None else w.shape[0]
    eo, ei = exclusions(n, bonds)
    counts = np.zeros(m, dtype=np.int64)
    L_, per = _box(L), _per(periodic)
    lib().orc_neighbor_counts(n, _p(pos), _p(L_), _p(per), r_cut, r_buff, _p(w), m,
                              _p(eo), _p(ei), _p(counts))
    off = np.zeros(m + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    idx = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
    lib().orc_neighbor_lists(n, _p(pos), _p(L_), _p(per), r_cut, r_buff, _p(w), m,
                             _p(eo), _p(ei), _p(off), _p(idx))
    return off, idx[: int(off[-1])]


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def dpd_theta(tag_i: int, tag_j: int, seed: int, timestep: int) -> float:
    return float(lib().orc_dpd_theta(tag_i, tag_j, seed, timestep))


KIND = {"lj": 0, "wca": 1, "dpd": 2}


def pair_forces(kind: str, pos, L, prm, vel=None, tag=None, timestep: int = 0, which=None,
                periodic=None, bonds=None):
    """Brute-force pair forces on the requested particles.
    Returns (F (m,3), u (m,), w (m,), nc (m,))."""
    pos = _f64(pos)
    n = pos.shape[0]
    vel = _f64(vel) if vel is not None else np.zeros_like(pos)
    tag = _i32(tag) if tag is not None else np.arange(n, dtype=np.int32)
    w_ = None if which is None else _i64(which)
    m = n if w_ is None else w_.shape[0]
    eo, ei = exclusions(n, bonds)
    F = np.zeros((m, 3))
    u = np.zeros(m)
    w = np.zeros(m)
    nc = np.zeros(m, dtype=np.int64)
    prm = _f64(prm)
    L_, per = _box(L), _per(periodic)
    rc = lib().orc_pair_forces(KIND[kind], n, _p(pos), _p(vel), _p(tag), _p(L_),
                               _p(per), _p(prm), timestep, _p(w_), m, _p(eo), _p(ei),
                               _p(F), _p(u), _p(w), _p(nc))
    if rc < 0:
        raise ValueError("unknown pair kind")
    return F, u, w, nc


def bond_forces(pos, L, bonds, K=30.0, R0=1.5, eps=1.0, sigma=1.0, with_wca=True, periodic=None):
    """FENE (+ WCA) bond forces.  Returns (F, u, w, n_stretched)."""
    pos = _f64(pos)
    n = pos.shape[0]
    b = _i32(bonds).reshape(-1, 2)
    F = np.zeros((n, 3))
    u = np.zeros(n)
    w = np.zeros(n)
    prm = _f64([K, R0, eps, sigma, 1.0 if with_wca else 0.0])
    L_, per = _box(L), _per(periodic)
    ns = lib().orc_bond_forces(n, _p(pos), _p(L_), _p(per), b.shape[0], _p(b),
                               _p(prm), _p(F), _p(u), _p(w))
    return F, u, w, int(ns)


def thermo(vel, u=None, w=None) -> np.ndarray:
    """{KE, PE, W, T} with compensated sums."""
    vel = _f64(vel)
    out = np.zeros(4)
    u_ = None if u is None else _f64(u)
    w_ = None if w is None else _f64(w)
    lib().orc_thermo(vel.shape[0], _p(vel), _p(u_), _p(w_), _p(out))
    return out


MODEL = {"lj": 0, "polymer": 1, "dpd": 2}


def run_nve(model: str, pos, vel, L, pair_prm, dt: float, nsteps: int, tag=None, bonds=None,
            bond_prm=(30.0, 1.5), t0: int = 0, force=None, with_thermo: bool = False):
    """Velocity-Verlet NVE with brute-force forces.
    Returns (pos, vel, F, thermo or None, status)."""
    x = _f64(np.array(pos, dtype=np.float64))
    v = _f64(np.array(vel, dtype=np.float64))
    n = x.shape[0]
    tag = _i32(tag) if tag is not None else np.arange(n, dtype=np.int32)
    b = _i32(bonds).reshape(-1, 2) if bonds is not None else np.zeros((0, 2), dtype=np.int32)
    F = _f64(np.array(force, dtype=np.float64)) if force is not None else np.zeros((n, 3))
    th = np.zeros((nsteps + 1, 4)) if with_thermo else None
    L_, pp, bp = _box(L), _f64(pair_prm), _f64(bond_prm)
    st = lib().orc_run_nve(MODEL[model], n, _p(x), _p(v), _p(tag), _p(L_), _p(pp),
                           b.shape[0], _p(b), _p(bp), dt, t0, nsteps, _p(F),
                           1 if force is not None else 0, _p(th))
    return x, v, F, th, int(st)


def run_nvt(model: str, pos, vel, L, pair_prm, dt: float, nsteps: int, T0: float, tau: float,
            xi: float = 0.0, eta: float = 0.0, tag=None, bonds=None, bond_prm=(30.0, 1.5),
            t0: int = 0):
    """Nose-Hoover NVT with brute-force forces.  Returns (pos, vel, F,
    thermo (nsteps+1, 4), ext (nsteps+1, 2) of {xi, eta}, status)."""
    x = _f64(np.array(pos, dtype=np.float64))
    v = _f64(np.array(vel, dtype=np.float64))
    n = x.shape[0]
    tag = _i32(tag) if tag is not None else np.arange(n, dtype=np.int32)
    b = _i32(bonds).reshape(-1, 2) if bonds is not None else np.zeros((0, 2), dtype=np.int32)
    F = np.zeros((n, 3))
    th = np.zeros((nsteps + 1, 4))
    ext = np.zeros((nsteps + 1, 2))
    xe = np.array([xi, eta], dtype=np.float64)
    nv = np.array([T0, tau], dtype=np.float64)
    L_, pp, bp = _box(L), _f64(pair_prm), _f64(bond_prm)
    st = lib().orc_run_nvt(MODEL[model], n, _p(x), _p(v), _p(tag), _p(L_), _p(pp),
                           b.shape[0], _p(b), _p(bp), dt, t0, nsteps, _p(nv), _p(xe), _p(F),
                           _p(th), _p(ext))
    return x, v, F, th, ext, int(st)


def nvt_conserved(thermo, ext, n: int, T0: float, tau: float):
    """KE + PE + g T0 (tau^2 xi^2 / 2 + eta), g = 3n - 3, per row."""
    g = 3.0 * n - 3.0
    return thermo[:, 0] + thermo[:, 1] + g * T0 * (0.5 * tau * tau * ext[:, 0] ** 2 + ext[:, 1])


def cell_bins(L, r_list: float) -> np.ndarray:
    b = np.zeros(3, dtype=np.int32)
    L_ = _box(L)
    lib().orc_cell_bins(_p(L_), r_list, _p(b))
    return b


def cell_list(pos, L, bins, lo=(0.0, 0.0, 0.0)):
    """Returns (cell_of (n,), cell_start (ncell+1,), cell_idx (n,))."""
    pos = _f64(pos)
    n = pos.shape[0]
    bins = _i32(bins)
    ncell = int(np.prod(bins.astype(np.int64)))
    cell_of = np.zeros(n, dtype=np.int32)
    start = np.zeros(ncell + 1, dtype=np.int32)
    idx = np.zeros(max(n, 1), dtype=np.int32)
    lo_, L_ = _box(lo), _box(L)
    lib().orc_cell_list(n, _p(pos), _p(lo_), _p(L_), _p(bins), _p(cell_of),
                        _p(start), _p(idx))
    return cell_of, start, idx[:n]


def morton_keys(pos, L) -> np.ndarray:
    pos = _f64(pos)
    k = np.zeros(pos.shape[0], dtype=np.uint32)
    L_ = _box(L)
    lib().orc_morton_keys(pos.shape[0], _p(pos), _p(L_), _p(k))
    return k


def stable_order(keys) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    o = np.zeros(k.shape[0], dtype=np.int32)
    lib().orc_stable_order(k.shape[0], _p(k), _p(o))
    return o


def ghost_masks(pos, lo, hi, width: float) -> np.ndarray:
    pos = _f64(pos)
    m = np.zeros(pos.shape[0], dtype=np.uint32)
    lo_, hi_ = _box(lo), _box(hi)
    lib().orc_ghost_masks(pos.shape[0], _p(pos), _p(lo_), _p(hi_), width, _p(m))
    return m


def ghost_list(mask):
    """Returns (counts[26], offsets[26], idx) ordered by direction then index."""
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    counts = np.zeros(26, dtype=np.int32)
    offs = np.zeros(26, dtype=np.int32)
    idx = np.zeros(max(26 * m.shape[0], 1), dtype=np.int32)
    k = lib().orc_ghost_list(m.shape[0], _p(m), _p(counts), _p(offs), _p(idx))
    return counts, offs, idx[:k]


def ghost_receive(pos, owner, self_id: int, L, lo, hi, width: float):
    """Brute-force receive set: (indices, images) of every foreign particle
    with an image inside [lo - width, hi + width)."""
    pos = _f64(pos)
    own = _i32(owner)
    n = pos.shape[0]
    cap = n
    idx = np.zeros(cap, dtype=np.int32)
    img = np.zeros((cap, 3))
    L_, lo_, hi_ = _box(L), _box(lo), _box(hi)
    k = lib().orc_ghost_receive(n, _p(pos), _p(own), self_id, _p(L_), _p(lo_),
                                _p(hi_), width, _p(idx), _p(img), cap)
    if k > cap:
        raise RuntimeError("receive set larger than the particle count")
    return idx[:k], img[:k]
