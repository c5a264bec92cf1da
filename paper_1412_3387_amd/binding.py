"""ctypes binding of libhoomd_mi355x.so with the same entry-point names.

Argument marshalling only: PyTorch provides device memory and the stream,
every step of the MD path runs in the library's HIP kernels.  Importing this
module does not load the library; the first use does, and fails loudly when
it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhoomd_mi355x.so")

FP64, MIXED = 0, 1
PAIR_LJ, PAIR_WCA, PAIR_DPD = 0, 1, 2
NVE, NVT = 0, 1
FORCE_AUTO, FORCE_SPLIT, FORCE_ONE = 0, 1, 2
ENERGY, VIRIAL = 1, 2
GHOST_SELECT, GHOST_UPDATE = 0, 1
FIELD_POS, FIELD_VEL, FIELD_TAG = 1, 2, 4
BOND_START, BOND_MIGRATE = 0, 1
BOND_RECORD_BYTES = 16

STATUS = {0: "OK", 1: "E_ARG", 2: "E_DEVICE", 3: "E_WORKSPACE", 4: "E_STATE",
          5: "E_NLIST_OVERFLOW", 6: "E_CELL_OVERFLOW", 7: "E_GHOST_OVERFLOW",
          8: "E_BOND_STRETCH", 9: "E_NAN", 10: "E_DANGEROUS_BUILD", 11: "E_HALO_OVERFLOW"}


class HoomdError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("pair", C.c_int32), ("r_cut", C.c_double),
                ("r_buff", C.c_double), ("dt", C.c_double), ("eps", C.c_double),
                ("sigma", C.c_double), ("dpd_A", C.c_double), ("dpd_gamma", C.c_double),
                ("dpd_kT", C.c_double), ("dpd_seed", C.c_uint32), ("bond_cap", C.c_int32),
                ("fene_K", C.c_double), ("fene_R0", C.c_double), ("nlist_cap", C.c_int32),
                ("cell_cap", C.c_int32), ("halo_cap", C.c_int32), ("sort_period", C.c_int32), ("check_period", C.c_int32),
                ("tpp_nlist", C.c_int32), ("tpp_force", C.c_int32), ("block_nlist", C.c_int32),
                ("block_force", C.c_int32), ("use_graph", C.c_int32), ("tune_period", C.c_int32),
                ("integrator", C.c_int32), ("nvt_group", C.c_int32), ("nvt_T0", C.c_double),
                ("nvt_tau", C.c_double), ("force_launch", C.c_int32), ("pad_", C.c_int32)]


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("L", C.c_double * 3), ("periodic", C.c_int32 * 3),
                ("pad_", C.c_int32), ("n_local", C.c_int64), ("n_cap", C.c_int64),
                ("n_bonds", C.c_int64)]


class Arrays(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("force", C.c_void_p),
                ("tag", C.c_void_p), ("bonds", C.c_void_p)]


class Subdomain(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("width", C.c_double)]


class Layout(C.Structure):
    _fields_ = [("nlist", C.c_void_p), ("nn", C.c_void_p), ("halo", C.c_void_p),
                ("halo_n", C.c_void_p), ("cell_idx", C.c_void_p), ("cell_size", C.c_void_p),
                ("nlist_cap", C.c_int32), ("cell_cap", C.c_int32), ("halo_cap", C.c_int32),
                ("bins", C.c_int32 * 3), ("row_offset", C.c_int64), ("cell_offset", C.c_int64),
                ("tile_offset", C.c_int64), ("general_tiles", C.c_void_p),
                ("rare_tiles", C.c_void_p), ("halo_lds", C.c_int32), ("bond_stride", C.c_int32),
                ("n_local", C.c_int64), ("n_total", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("tpp_nlist", C.c_int32), ("block_nlist", C.c_int32), ("tpp_force", C.c_int32),
                ("block_force", C.c_int32), ("force_ms", C.c_float * 5), ("build_ms", C.c_float * 4),
                ("scans", C.c_int32), ("from_cache", C.c_int32)]


BUILD_SHAPES = [(64, 512), (64, 256), (32, 512), (32, 256)]
FORCE_LANES = [1, 2, 4, 8, 16]


class Profile(C.Structure):
    _fields_ = [("force_ms", C.c_double), ("force_launches", C.c_int64),
                ("rebuild_ms", C.c_double), ("rebuild_launches", C.c_int64)]


EXPORTS = ["hoomd_workspace_bytes", "hoomd_init", "hoomd_destroy", "build_nlist",
           "compute_forces", "step", "pack_ghosts", "unpack_ghosts", "hoomd_thermo",
           "hoomd_thermo_log", "hoomd_sync_status", "hoomd_build_count", "hoomd_get_layout",
           "hoomd_autotune", "hoomd_profile", "hoomd_strerror", "pack_ghosts_noalloc",
           "integrate_half_step", "hoomd_rebuild_due", "migrate_particles", "receive_particles",
           "hoomd_thermostat", "hoomd_set_thermostat",
           "pack_bond_ranks", "unpack_bond_ranks"]

_lib = None


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1412_3387_amd/build.py "
                               "(there is no CPU fallback)")
        # torch ships its own HIP runtime (soname libamdhip64.so.7); loading it
        # first makes the library bind to that same runtime, so device
        # pointers from torch allocations are known to every HIP call here.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.hoomd_workspace_bytes.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(Box)]
        L.hoomd_workspace_bytes.restype = C.c_size_t
        L.hoomd_init.argtypes = [C.POINTER(P), C.POINTER(Params), C.c_int32, C.POINTER(Box),
                                 C.POINTER(Arrays), P, C.c_size_t, P]
        L.hoomd_destroy.argtypes = [P]
        L.hoomd_destroy.restype = None
        L.build_nlist.argtypes = [P, C.c_int32]
        L.compute_forces.argtypes = [P, C.c_uint64, C.c_uint32]
        L.step.argtypes = [P, C.c_uint64, C.c_int32, C.c_int32]
        L.pack_ghosts.argtypes = [P, C.c_int32, C.POINTER(Subdomain), C.c_int32, C.c_uint32, P,
                                  C.c_int64, P, P]
        L.unpack_ghosts.argtypes = [P, C.c_int32, P, C.c_int64, C.c_uint32, C.c_int32,
                                    C.POINTER(C.c_double)]
        L.hoomd_thermo.argtypes = [P, C.POINTER(C.c_double)]
        L.hoomd_thermostat.argtypes = [P, C.POINTER(C.c_double)]
        L.hoomd_set_thermostat.argtypes = [P, C.POINTER(C.c_double)]
        L.hoomd_thermo_log.argtypes = [P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]
        L.hoomd_sync_status.argtypes = [P, C.POINTER(C.c_int64)]
        L.hoomd_build_count.argtypes = [P, C.POINTER(C.c_int64)]
        L.hoomd_get_layout.argtypes = [P, C.c_int32, C.POINTER(Layout)]
        L.hoomd_autotune.argtypes = [P, C.c_int32, C.POINTER(Tuning)]
        L.hoomd_profile.argtypes = [P, C.c_int32, C.POINTER(Profile)]
        L.pack_ghosts_noalloc.argtypes = [P, P, P, C.c_int64, C.POINTER(Subdomain), C.c_uint32, P,
                                          C.c_int64, P, P, P]
        L.integrate_half_step.argtypes = [P, C.c_int32, C.c_uint64]
        L.hoomd_rebuild_due.argtypes = [P, C.POINTER(C.c_int32)]
        L.migrate_particles.argtypes = [P, C.c_int32, C.POINTER(Subdomain), P, C.c_int64, P, P,
                                        C.POINTER(C.c_int64)]
        L.receive_particles.argtypes = [P, C.c_int32, P, C.c_int64, C.POINTER(C.c_double)]
        L.pack_bond_ranks.argtypes = [P, C.c_int32, C.POINTER(Subdomain), C.c_int32, P, C.c_int64, P, P,
                                      C.POINTER(C.c_int64)]
        L.unpack_bond_ranks.argtypes = [P, C.c_int32, P, C.c_int64, C.c_int32]
        L.hoomd_strerror.argtypes = [C.c_int]
        L.hoomd_strerror.restype = C.c_char_p
        _lib = L
    return _lib


@dataclasses.dataclass
class ModelParams:
    """Python mirror of hoomd_params."""
    precision: int = MIXED
    pair: int = PAIR_LJ
    r_cut: float = 2.5
    r_buff: float = 0.4
    dt: float = 0.005
    eps: float = 1.0
    sigma: float = 1.0
    dpd_A: float = 25.0
    dpd_gamma: float = 4.5
    dpd_kT: float = 1.0
    dpd_seed: int = 0
    bond_cap: int = 0
    fene_K: float = 30.0
    fene_R0: float = 1.5
    nlist_cap: int = 0
    cell_cap: int = 0
    halo_cap: int = 0
    sort_period: int = 0
    check_period: int = 1
    tpp_nlist: int = 0
    tpp_force: int = 0
    block_nlist: int = 0
    block_force: int = 0
    use_graph: int = 1
    tune_period: int = 0
    integrator: int = 0
    nvt_group: int = 0
    nvt_T0: float = 1.0
    nvt_tau: float = 1.0
    force_launch: int = 0
    pad_: int = 0

    def list_radius(self) -> float:
        rc = 2.0 ** (1.0 / 6.0) * self.sigma if self.pair == PAIR_WCA else self.r_cut
        return rc + self.r_buff

    def to_c(self, density: float) -> Params:
        cap = self.nlist_cap
        if cap <= 0:
            # mean list length plus a wide margin, rounded to a multiple of 8
            mean = 4.0 / 3.0 * math.pi * self.list_radius() ** 3 * density
            cap = int(math.ceil((1.35 * mean + 24) / 8.0) * 8)
        p = Params()
        for f in dataclasses.fields(self):
            setattr(p, f.name, getattr(self, f.name))
        p.nlist_cap = cap
        return p


NOALLOC_MAX_ROWS = 2097152


def pack_ghosts_noalloc(pos, vel, tag, n_local: int, lo, hi, width: float, fields: int, send,
                        send_cap: int, counts, offsets, stream=None):
    """Context-free ghost selection + packing (C ABI pack_ghosts_noalloc)
    over device tensors: pos / vel (n, 4) float64, tag (n,) int32."""
    sd = Subdomain()
    for a in range(3):
        sd.lo[a] = float(lo[a])
        sd.hi[a] = float(hi[a])
    sd.width = float(width)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().pack_ghosts_noalloc(_ptr(pos), _ptr(vel), _ptr(tag), n_local, C.byref(sd), fields,
                                     _ptr(send), send_cap, _ptr(counts), _ptr(offsets), stream),
           "pack_ghosts_noalloc")


def _check(code: int, what: str):
    if code != 0:
        raise HoomdError(code, what)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """One library context over torch device tensors.

    systems: list of dicts with pos (n,3), vel (n,3), tag (n,), L (3,),
    optional bonds (nb,2) tag pairs, lo (3,), periodic (3,), n_cap.
    """

    def __init__(self, params: Sequence[ModelParams], systems: List[dict], device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.n_sys = len(systems)
        assert len(params) == self.n_sys
        self.mixed = params[0].precision == MIXED
        boxes = (Box * self.n_sys)()
        cparams = (Params * self.n_sys)()
        rows = 0
        self.offsets = []
        self.n_local = []
        self.n_cap = []
        bonds_all = []
        for s, (p, sy) in enumerate(zip(params, systems)):
            n = int(sy["pos"].shape[0])
            n_cap = int(sy.get("n_cap", n))
            L = np.asarray(sy["L"], dtype=np.float64)
            lo = np.asarray(sy.get("lo", (0.0, 0.0, 0.0)), dtype=np.float64)
            per = sy.get("periodic", (1, 1, 1))
            b = boxes[s]
            for a in range(3):
                b.lo[a] = float(lo[a])
                b.L[a] = float(L[a])
                b.periodic[a] = int(per[a])
            b.n_local = n
            b.n_cap = n_cap
            bonds = sy.get("bonds")
            b.n_bonds = 0 if bonds is None else int(len(bonds))
            if bonds is not None and len(bonds):
                bonds_all.append(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
            cparams[s] = p.to_c(density=n_cap / float(np.prod(L)))
            self.offsets.append(rows)
            self.n_local.append(n)
            self.n_cap.append(n_cap)
            rows += n_cap
        self.rows = rows
        dev = self.device
        f64 = torch.float64
        self.pos = torch.zeros((rows, 4), dtype=f64, device=dev)
        self.vel = torch.zeros((rows, 4), dtype=f64, device=dev)
        self.force = torch.zeros((rows, 4), dtype=torch.float32 if self.mixed else f64, device=dev)
        self.tag = torch.zeros(rows, dtype=torch.int32, device=dev)
        for s, sy in enumerate(systems):
            o, n = self.offsets[s], self.n_local[s]
            self.pos[o:o + n, :3] = torch.as_tensor(np.asarray(sy["pos"], dtype=np.float64), device=dev)
            self.vel[o:o + n, :3] = torch.as_tensor(np.asarray(sy["vel"], dtype=np.float64), device=dev)
            tg = sy.get("tag")
            tg = np.arange(n, dtype=np.int32) if tg is None else np.asarray(tg, dtype=np.int32)
            self.tag[o:o + n] = torch.as_tensor(tg, device=dev)
        self.bonds = None
        if bonds_all:
            self.bonds = torch.as_tensor(np.concatenate(bonds_all), device=dev).contiguous()
        self._cparams = cparams
        self._boxes = boxes
        nbytes = lib().hoomd_workspace_bytes(cparams, self.n_sys, boxes)
        if nbytes == 0:
            raise HoomdError(1, "hoomd_workspace_bytes")
        self.workspace = torch.zeros(int(nbytes), dtype=torch.uint8, device=dev)
        arr = Arrays(_ptr(self.pos), _ptr(self.vel), _ptr(self.force), _ptr(self.tag), _ptr(self.bonds))
        self._arrays = arr
        self.stream = torch.cuda.current_stream(dev)
        h = C.c_void_p()
        _check(lib().hoomd_init(C.byref(h), cparams, self.n_sys, boxes, C.byref(arr),
                                self.workspace.data_ptr(), nbytes, self.stream.cuda_stream),
               "hoomd_init")
        self.h = h

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().hoomd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points (same names as the C ABI) -----------------------------
    def build_nlist(self, force_rebuild: bool = True):
        _check(lib().build_nlist(self.h, 1 if force_rebuild else 0), "build_nlist")

    def compute_forces(self, timestep: int = 0, flags: int = 0):
        _check(lib().compute_forces(self.h, timestep, flags), "compute_forces")

    def step(self, first_timestep: int, n_steps: int, log_every: int = 0):
        _check(lib().step(self.h, first_timestep, n_steps, log_every), "step")

    def pack_ghosts(self, sys: int, lo, hi, width: float, mode: int, fields: int, send,
                    send_cap: int, counts, offsets):
        sd = Subdomain()
        for a in range(3):
            sd.lo[a] = float(lo[a])
            sd.hi[a] = float(hi[a])
        sd.width = float(width)
        _check(lib().pack_ghosts(self.h, sys, C.byref(sd), mode, fields, _ptr(send), send_cap,
                                 _ptr(counts), _ptr(offsets)), "pack_ghosts")

    def unpack_ghosts(self, sys: int, recv, n_recv: int, fields: int, mode: int, box_L):
        bl = (C.c_double * 3)(*[float(x) for x in box_L])
        _check(lib().unpack_ghosts(self.h, sys, _ptr(recv), n_recv, fields, mode, bl), "unpack_ghosts")

    def integrate_half_step(self, which: int, timestep: int = 0):
        _check(lib().integrate_half_step(self.h, which, timestep), "integrate_half_step")

    def rebuild_due(self) -> bool:
        v = C.c_int32()
        _check(lib().hoomd_rebuild_due(self.h, C.byref(v)), "hoomd_rebuild_due")
        return bool(v.value)

    def _refresh_counts(self, sys: int):
        self.n_local[sys] = int(self.layout(sys).n_local)

    def migrate_record_bytes(self) -> int:
        """Bytes of one migration record: position, velocity, tag, and with
        bonds the partner tags and owner directions."""
        return 56 + 8 * self.layout(0).bond_stride

    def pack_bond_ranks(self, sys: int, lo, hi, mode: int, send, send_cap: int, counts, offsets) -> int:
        """Bond owner-table messages of `sys` (16 bytes each); returns their number."""
        sd = Subdomain()
        for a in range(3):
            sd.lo[a] = float(lo[a])
            sd.hi[a] = float(hi[a])
        sd.width = 0.0
        n = C.c_int64()
        _check(lib().pack_bond_ranks(self.h, sys, C.byref(sd), mode, _ptr(send), send_cap, _ptr(counts),
                                     _ptr(offsets), C.byref(n)), "pack_bond_ranks")
        return n.value

    def unpack_bond_ranks(self, sys: int, recv, n_recv: int, mode: int):
        _check(lib().unpack_bond_ranks(self.h, sys, _ptr(recv), n_recv, mode), "unpack_bond_ranks")

    def migrate_particles(self, sys: int, lo, hi, send, send_cap: int, counts, offsets) -> int:
        """Pack and remove the locals of `sys` that left [lo, hi); returns how
        many left (records of migrate_record_bytes() each)."""
        sd = Subdomain()
        for a in range(3):
            sd.lo[a] = float(lo[a])
            sd.hi[a] = float(hi[a])
        sd.width = 0.0
        n = C.c_int64()
        code = lib().migrate_particles(self.h, sys, C.byref(sd), _ptr(send), send_cap, _ptr(counts),
                                       _ptr(offsets), C.byref(n))
        self._refresh_counts(sys)
        _check(code, "migrate_particles")
        return n.value

    def receive_particles(self, sys: int, recv, n_recv: int, box_L):
        bl = (C.c_double * 3)(*[float(x) for x in box_L])
        _check(lib().receive_particles(self.h, sys, _ptr(recv), n_recv, bl), "receive_particles")
        self._refresh_counts(sys)

    def thermostat(self) -> np.ndarray:
        """(n_sys, 2) Nose-Hoover {xi, eta} per system."""
        out = (C.c_double * (2 * self.n_sys))()
        _check(lib().hoomd_thermostat(self.h, out), "hoomd_thermostat")
        return np.array(out[:]).reshape(self.n_sys, 2)

    def set_thermostat(self, xi_eta):
        v = np.ascontiguousarray(np.asarray(xi_eta, dtype=np.float64).reshape(self.n_sys, 2))
        _check(lib().hoomd_set_thermostat(self.h, v.ctypes.data_as(C.POINTER(C.c_double))),
               "hoomd_set_thermostat")

    def thermo(self) -> np.ndarray:
        out = (C.c_double * (4 * self.n_sys))()
        _check(lib().hoomd_thermo(self.h, out), "hoomd_thermo")
        return np.array(out[:]).reshape(self.n_sys, 4)

    def thermo_log(self, max_rows: int = 4096) -> np.ndarray:
        out = (C.c_double * (5 * self.n_sys * max_rows))()
        rows = C.c_int32()
        _check(lib().hoomd_thermo_log(self.h, out, max_rows, C.byref(rows)), "hoomd_thermo_log")
        return np.array(out[: 5 * self.n_sys * rows.value]).reshape(rows.value, self.n_sys, 5)

    def sync_status(self):
        req = C.c_int64()
        code = lib().hoomd_sync_status(self.h, C.byref(req))
        return code, req.value

    def check(self):
        code, req = self.sync_status()
        if code != 0:
            raise HoomdError(code, f"device status (required capacity {req})")

    def build_count(self) -> int:
        v = C.c_int64()
        _check(lib().hoomd_build_count(self.h, C.byref(v)), "hoomd_build_count")
        return v.value

    def autotune(self, do_tune=True) -> Tuning:
        """do_tune: False/0 report, True/1 scan, 2 use the process-wide cache
        (scan only when it has nothing for this kind of context)."""
        t = Tuning()
        _check(lib().hoomd_autotune(self.h, int(do_tune), C.byref(t)), "hoomd_autotune")
        return t

    def profile(self, mode: int) -> Optional[Profile]:
        """mode 1 start, 0 stop, 2 read (returns the totals)."""
        pr = Profile()
        _check(lib().hoomd_profile(self.h, mode, C.byref(pr) if mode == 2 else None), "hoomd_profile")
        return pr if mode == 2 else None

    # -- inspection ---------------------------------------------------------
    def layout(self, sys: int = 0) -> Layout:
        lay = Layout()
        _check(lib().hoomd_get_layout(self.h, sys, C.byref(lay)), "hoomd_get_layout")
        return lay

    def _ws_view(self, ptr: int, count: int, itemsize: int = 4):
        base = self.workspace.data_ptr()
        off = ptr - base
        assert 0 <= off and off + itemsize * count <= self.workspace.numel()
        v = self.workspace[off:off + itemsize * count]
        return v.view(self.torch.int32) if itemsize == 4 else v.view(self.torch.int16)

    def neighbor_rows(self, sys: int = 0):
        """(nn (n,), rows as a list of int arrays of system-local row
        numbers), decoded through the per-tile halos."""
        lay = self.layout(sys)
        n = self.n_local[sys]
        o = self.offsets[sys]
        cap = lay.nlist_cap
        tiles = (n + 63) // 64
        nn = self._ws_view(lay.nn, n).cpu().numpy().copy()
        nl = self._ws_view(lay.nlist, tiles * 64 * cap, 2).cpu().numpy().view(np.uint16)
        nl = nl.reshape(tiles, cap, 64).astype(np.int64)
        halo = self._ws_view(lay.halo, tiles * lay.halo_cap).cpu().numpy().reshape(tiles, lay.halo_cap)
        rows = []
        for r in range(n):
            t, l = divmod(r, 64)
            rows.append(halo[t][nl[t, : nn[r], l]].astype(np.int64) - o)
        return nn, rows

    def general_tiles(self) -> int:
        """Tiles of the last build that went to the general (unframed) build."""
        lay = self.layout(0)
        return int(self._ws_view(lay.general_tiles, 1).cpu().item())

    def rare_tiles(self) -> int:
        """Tiles of the last build that the force pass handles in its second
        launch (per-pair images or a halo beyond its LDS stage)."""
        lay = self.layout(0)
        return int(self._ws_view(lay.rare_tiles, 1).cpu().item())

    def halo_n(self, sys: int = 0) -> np.ndarray:
        """Tile headers of the last build (halo size, longest row, per-pair
        image bit), as unsigned 32-bit words."""
        lay = self.layout(sys)
        tiles = (self.n_local[sys] + 63) // 64
        return self._ws_view(lay.halo_n, tiles).cpu().numpy().view(np.uint32)

    def halo_sizes(self, sys: int = 0) -> np.ndarray:
        lay = self.layout(sys)
        tiles = (self.n_local[sys] + 63) // 64
        return self._ws_view(lay.halo_n, tiles).cpu().numpy() & 0xFFFF

    def cells(self, sys: int = 0):
        """(bins, sizes (ncell,), members list per cell in system-local rows)."""
        lay = self.layout(sys)
        bins = np.array(lay.bins[:])
        ncell = int(np.prod(bins))
        size = self._ws_view(lay.cell_size, ncell).cpu().numpy().copy()
        idx = self._ws_view(lay.cell_idx, ncell * lay.cell_cap).cpu().numpy().reshape(ncell, lay.cell_cap)
        o = self.offsets[sys]
        return bins, size, [idx[c, : size[c]].astype(np.int64) - o for c in range(ncell)]

    def host_state(self, sys: int = 0):
        """(pos (n,3), vel (n,3), force (n,4), tag (n,)) of the locals of a system."""
        o, n = self.offsets[sys], self.n_local[sys]
        self.torch.cuda.synchronize(self.device)
        return (self.pos[o:o + n, :3].cpu().numpy().copy(), self.vel[o:o + n, :3].cpu().numpy().copy(),
                self.force[o:o + n].double().cpu().numpy().copy(), self.tag[o:o + n].cpu().numpy().copy())
