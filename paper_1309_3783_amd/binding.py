"""ctypes binding of libsphcell.so (include/sphcell.h), same names as the C-ABI.

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch provides the device memory (tensors) and the stream.  There is no
fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphcell.so")

SPH_OK, SPH_E_ARG, SPH_E_HIP, SPH_E_WORKSPACE, SPH_E_REBUILD, SPH_E_NOCONV, SPH_E_CAPACITY, SPH_E_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
SPH_FLAG_PAIR_HASH = 1
SPH_FLAG_RESUME = 2
SPH_FLAG_NO_BLOCK_SKIP = 4
SPH_FLAG_SORTED_ONLY = 8

# every function the header declares
EXPORTS = ["sph_version", "sph_status_str", "sph_params_default", "sph_ctx_create", "sph_ctx_destroy",
           "sph_last_error", "sph_ctx_sync", "sph_workspace_size", "sph_footprint", "sph_tree_create",
           "sph_tree_destroy", "sph_tree_bytes", "sph_tree_set_workspace", "sph_tree_workspace_needed",
           "sph_build_cells", "sph_build_cells_static", "sph_refresh_cells", "sph_sort_pairs", "sph_density",
           "sph_solve_h", "sph_force", "sph_set_halo", "sph_run_graph", "sph_last_timings", "sph_last_work",
           "sph_last_reads", "sph_enable_timing", "sph_tree_stats", "sph_kick", "sph_drift", "sph_cfl_dt"]


class sph_params(C.Structure):
    _fields_ = [("n_split", C.c_int32), ("split_frac", C.c_float), ("h_slack", C.c_float),
                ("max_depth", C.c_int32), ("top_grid", C.c_int32), ("n_target", C.c_float),
                ("h_tol", C.c_float), ("max_iter", C.c_int32), ("gamma", C.c_float), ("alpha", C.c_float),
                ("flags", C.c_uint32), ("blocks_per_cu", C.c_int32), ("max_replicas", C.c_int32),
                ("top_coarsen", C.c_int32), ("piece_records", C.c_int32),
                ("reserved", C.c_int32 * 1)]


class sph_input(C.Structure):
    _fields_ = [("nsets", C.c_int32), ("offsets", C.c_void_p), ("box", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("h", C.c_void_p),
                ("m", C.c_void_p), ("u", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("vz", C.c_void_p)]


class sph_density_out(C.Structure):
    _fields_ = [("rho", C.c_void_p), ("drho_dh", C.c_void_p), ("nw", C.c_void_p), ("dnw_dh", C.c_void_p),
                ("nngb", C.c_void_p), ("hash", C.c_void_p), ("h", C.c_void_p)]


class sph_force_out(C.Structure):
    _fields_ = [("ax", C.c_void_p), ("ay", C.c_void_p), ("az", C.c_void_p), ("dudt", C.c_void_p),
                ("vsig", C.c_void_p), ("S", C.c_void_p), ("nforce", C.c_void_p), ("hash", C.c_void_p),
                ("sums", C.c_void_p)]


_lib = None


def lib():
    """Load libsphcell.so; raise loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        # torch carries its own HIP runtime and the library links the
        # system's: torch's must find the GPU first (loaded the other way
        # round, the library's runtime sees no device)
        import torch
        torch.cuda.is_available()
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int32
        L.sph_version.restype = C.c_char_p
        L.sph_status_str.restype = C.c_char_p
        L.sph_status_str.argtypes = [st]
        L.sph_params_default.argtypes = [C.POINTER(sph_params)]
        L.sph_params_default.restype = None
        L.sph_ctx_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.sph_ctx_destroy.argtypes = [vp]
        L.sph_ctx_destroy.restype = None
        L.sph_last_error.argtypes = [vp]
        L.sph_last_error.restype = C.c_char_p
        L.sph_ctx_sync.argtypes = [vp]
        L.sph_footprint.argtypes = [C.c_int64, C.POINTER(sph_params), C.POINTER(C.c_size_t)]
        L.sph_workspace_size.argtypes = [C.c_int64, C.c_int32, C.POINTER(sph_params), C.POINTER(C.c_size_t)]
        L.sph_tree_set_workspace.argtypes = [vp, vp, vp, C.c_size_t]
        L.sph_tree_workspace_needed.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.sph_build_cells_static.argtypes = [vp, vp, C.POINTER(sph_input), C.POINTER(sph_params)]
        L.sph_tree_create.argtypes = [vp, C.POINTER(vp)]
        L.sph_tree_destroy.argtypes = [vp, vp]
        L.sph_tree_destroy.restype = None
        L.sph_tree_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.sph_build_cells.argtypes = [vp, vp, C.POINTER(sph_input), C.POINTER(sph_params)]
        L.sph_sort_pairs.argtypes = [vp, vp]
        L.sph_refresh_cells.argtypes = [vp, vp, C.POINTER(sph_input)]
        L.sph_density.argtypes = [vp, vp, C.POINTER(sph_density_out)]
        L.sph_solve_h.argtypes = [vp, vp, C.POINTER(sph_density_out), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
        L.sph_force.argtypes = [vp, vp, C.POINTER(sph_force_out)]
        L.sph_set_halo.argtypes = [vp, vp, vp, vp, vp]
        L.sph_run_graph.argtypes = [vp, vp, C.c_int32, C.POINTER(sph_density_out), C.POINTER(sph_force_out),
                                    vp]
        L.sph_last_timings.argtypes = [vp, C.POINTER(C.c_char_p), C.POINTER(C.c_double), C.c_int32]
        L.sph_last_timings.restype = C.c_int32
        L.sph_last_work.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.sph_last_reads.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.sph_enable_timing.argtypes = [vp, C.c_int32]
        L.sph_enable_timing.restype = None
        L.sph_tree_stats.argtypes = [vp, C.POINTER(C.c_int64), C.c_int32]
        L.sph_kick.argtypes = [vp, C.c_int64, C.c_float] + [vp] * 12
        L.sph_drift.argtypes = [vp, C.c_int32, vp, vp, C.c_double] + [vp] * 6
        L.sph_cfl_dt.argtypes = [vp, C.c_int64, vp, vp, C.c_float, C.POINTER(C.c_double)]
        for name in ("sph_ctx_create", "sph_ctx_sync", "sph_footprint", "sph_workspace_size", "sph_tree_create",
                     "sph_tree_bytes", "sph_tree_set_workspace", "sph_tree_workspace_needed", "sph_build_cells",
                     "sph_build_cells_static", "sph_refresh_cells", "sph_sort_pairs", "sph_density", "sph_solve_h",
                     "sph_force", "sph_run_graph", "sph_tree_stats", "sph_kick", "sph_drift", "sph_cfl_dt",
                     "sph_last_work", "sph_last_reads", "sph_set_halo"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def params(**kw) -> sph_params:
    p = sph_params()
    lib().sph_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def footprint(n: int, prm: sph_params | None = None) -> int:
    b = C.c_size_t(0)
    st = lib().sph_footprint(int(n), C.byref(prm or params()), C.byref(b))
    if st:
        raise SphError(st, "sph_footprint")
    return int(b.value)


def workspace_size(n: int, nsets: int = 1, prm: sph_params | None = None) -> int:
    b = C.c_size_t(0)
    st = lib().sph_workspace_size(int(n), int(nsets), C.byref(prm or params()), C.byref(b))
    if st:
        raise SphError(st, "sph_workspace_size")
    return int(b.value)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and one torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the SPH library runs only on the GPU (no CPU fallback)")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib().sph_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if st:
            raise SphError(st, "sph_ctx_create: " + lib().sph_last_error(None).decode(errors="replace"))
        self.h = h

    def check(self, st, what):
        if st:
            msg = lib().sph_last_error(self.h).decode(errors="replace")
            raise SphError(st, f"{what}: {msg}")

    def sync(self):
        """sph_ctx_sync: wait for the context's stream; raises on a stream error."""
        self.check(lib().sph_ctx_sync(self.h), "sph_ctx_sync")

    def enable_timing(self, on=True):
        lib().sph_enable_timing(self.h, 1 if on else 0)

    def timings(self):
        names = (C.c_char_p * 4096)()
        ms = (C.c_double * 4096)()
        k = lib().sph_last_timings(self.h, names, ms, 4096)
        return [(names[i].decode(), ms[i]) for i in range(k)]

    def work(self):
        """(density pair evaluations, force pair evaluations) of the last calls."""
        d, f = C.c_uint64(0), C.c_uint64(0)
        self.check(lib().sph_last_work(self.h, C.byref(d), C.byref(f)), "sph_last_work")
        return int(d.value), int(f.value)

    def reads(self):
        """(density records loaded, force records loaded) of the same calls."""
        d, f = C.c_uint64(0), C.c_uint64(0)
        self.check(lib().sph_last_reads(self.h, C.byref(d), C.byref(f)), "sph_last_reads")
        return int(d.value), int(f.value)

    def close(self):
        if getattr(self, "h", None):
            lib().sph_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Batch:
    """S particle sets concatenated on the device (caller order)."""
    x: object
    y: object
    z: object
    h: object
    m: object
    u: object
    vx: object
    vy: object
    vz: object
    offsets: np.ndarray
    box: np.ndarray
    keep: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def nsets(self) -> int:
        return int(self.offsets.size - 1)

    def as_input(self, h=None) -> sph_input:
        self._off = np.ascontiguousarray(self.offsets, dtype=np.int64)
        self._box = np.ascontiguousarray(self.box, dtype=np.float64)
        hh = self.h if h is None else h
        return sph_input(self.nsets, self._off.ctypes.data_as(C.c_void_p), self._box.ctypes.data_as(C.c_void_p),
                         _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(hh), _ptr(self.m), _ptr(self.u),
                         _ptr(self.vx), _ptr(self.vy), _ptr(self.vz))


def batch_from_sets(sets, device="cuda", h=None) -> Batch:
    """Upload ParticleSet-like objects (numpy, caller order) as one Batch."""
    import torch
    sizes = [s.n for s in sets]
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)

    def cat(attr, dt):
        arr = np.concatenate([np.asarray(getattr(s, attr)) for s in sets]) if sets else np.zeros(0)
        return torch.as_tensor(arr.astype(dt), device=device)

    hh = (torch.as_tensor(np.concatenate([np.asarray(x) for x in h]).astype(np.float32), device=device)
          if h is not None else cat("h0", np.float32))
    return Batch(cat("x", np.float64), cat("y", np.float64), cat("z", np.float64), hh,
                 cat("m", np.float32), cat("u", np.float32), cat("vx", np.float32), cat("vy", np.float32),
                 cat("vz", np.float32), off, np.array([s.box for s in sets], dtype=np.float64))


class DensityOut:
    def __init__(self, n, device, hash=False):
        import torch
        f = dict(dtype=torch.float32, device=device)
        self.rho = torch.empty(n, **f)
        self.drho_dh = torch.empty(n, **f)
        self.nw = torch.empty(n, **f)
        self.dnw_dh = torch.empty(n, **f)
        self.nngb = torch.empty(n, dtype=torch.int32, device=device)
        self.hash = torch.empty(n, dtype=torch.int64, device=device) if hash else None
        self.h = torch.empty(n, **f)

    def c(self) -> sph_density_out:
        return sph_density_out(_ptr(self.rho), _ptr(self.drho_dh), _ptr(self.nw), _ptr(self.dnw_dh),
                               _ptr(self.nngb), _ptr(self.hash), _ptr(self.h))


class ForceOut:
    def __init__(self, n, nsets, device, hash=False):
        import torch
        f = dict(dtype=torch.float32, device=device)
        self.ax = torch.empty(n, **f)
        self.ay = torch.empty(n, **f)
        self.az = torch.empty(n, **f)
        self.dudt = torch.empty(n, **f)
        self.vsig = torch.empty(n, **f)
        self.S = torch.empty(n, **f)
        self.nforce = torch.empty(n, dtype=torch.int32, device=device)
        self.hash = torch.empty(n, dtype=torch.int64, device=device) if hash else None
        self.sums = torch.zeros(max(nsets, 1) * 8, dtype=torch.float64, device=device)

    def c(self) -> sph_force_out:
        return sph_force_out(_ptr(self.ax), _ptr(self.ay), _ptr(self.az), _ptr(self.dudt), _ptr(self.vsig),
                             _ptr(self.S), _ptr(self.nforce), _ptr(self.hash), _ptr(self.sums))


class Tree:
    """A device-resident cell tree for one Batch (kept across density -> force).

    workspace=True (default): the tree's device memory is one torch uint8
    tensor handed to the library (sph_tree_set_workspace), sized by
    sph_workspace_size and grown (doubled, at least to what the library
    reports it needs) when a build fails with SPH_E_WORKSPACE; the library
    then never allocates inside a call.  workspace=False: the library owns
    the buffers."""

    def __init__(self, ctx: Context, workspace: bool = True):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(lib().sph_tree_create(ctx.h, C.byref(h)), "sph_tree_create")
        self.h = h
        self.batch = None
        self.prm = None
        self.use_ws = workspace
        self.ws = None          # the workspace tensor
        self._old_ws = []       # previous workspaces, kept until the stream has passed their last use

    def set_workspace(self, nbytes: int):
        """Attach a fresh workspace of nbytes (the tree must be built again)."""
        import torch
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        if self.ws is not None:
            self._old_ws.append(self.ws)
        self.ctx.check(lib().sph_tree_set_workspace(self.ctx.h, self.h, _ptr(ws), int(nbytes)),
                       "sph_tree_set_workspace")
        self.ws = ws
        if self._old_ws:
            # the saved Newton state (if any) is copied out of the old one
            self.ctx.stream.synchronize()
            self._old_ws.clear()

    def workspace_needed(self) -> int:
        b = C.c_size_t(0)
        self.ctx.check(lib().sph_tree_workspace_needed(self.h, C.byref(b)), "sph_tree_workspace_needed")
        return int(b.value)

    def close(self):
        if getattr(self, "h", None):
            lib().sph_tree_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_cells(self, batch: Batch, prm: sph_params | None = None, h=None):
        self.batch = batch
        self.prm = prm or params()
        self._h_ref = h
        self._in = batch.as_input(h)
        self.builds = getattr(self, "builds", 0) + 1
        self._built = False
        self._sorted = False
        if self.use_ws:
            want = workspace_size(batch.n, batch.nsets, self.prm)
            if self.ws is None or self.ws.numel() < want:
                self.set_workspace(max(want, 0 if self.ws is None else 2 * self.ws.numel()))
        self._call(lambda: lib().sph_build_cells(self.ctx.h, self.h, C.byref(self._in), C.byref(self.prm)),
                   "sph_build_cells")
        self._built = True

    def _call(self, fn, what, ok=(SPH_OK,)):
        """Run a library call; with a workspace, a call that ran out of it is
        repeated on a larger one (twice the size, at least what the library
        says it needs), after building -- and sorting -- the tree again."""
        st = fn()
        for _ in range(8):
            if st != SPH_E_WORKSPACE or not self.use_ws:
                break
            self.set_workspace(max(2 * self.ws.numel(), self.workspace_needed()))
            if fn is not self._rebuild:
                rs = self._rebuild()
                if rs != SPH_OK:
                    st = rs
                    continue
            st = fn()
        if st not in ok:
            self.ctx.check(st, what)
        return st

    def _rebuild(self):
        st = lib().sph_build_cells(self.ctx.h, self.h, C.byref(self._in), C.byref(self.prm))
        if st == SPH_OK and self._sorted:
            st = lib().sph_sort_pairs(self.ctx.h, self.h)
        return st

    def build_cells_static(self, batch: Batch, prm: sph_params | None = None, h=None):
        """sph_build_cells with the library's static scratch as workspace
        (no allocation in this or the later calls on the tree)."""
        self.batch = batch
        self.prm = prm or params()
        self._in = batch.as_input(h)
        self.ctx.check(lib().sph_build_cells_static(self.ctx.h, self.h, C.byref(self._in), C.byref(self.prm)),
                       "sph_build_cells_static")

    def refresh(self, batch: Batch, h=None) -> bool:
        """sph_refresh_cells: the tree's particles take the batch's new data
        (the sets and caller order of the last build) without a new build or
        sort.  Returns False when the cells no longer support the particles'
        h after their displacement since the build: the tree must then be
        built again."""
        self.batch = batch
        self._h_ref = h
        self._in = batch.as_input(h)
        st = self._call(lambda: lib().sph_refresh_cells(self.ctx.h, self.h, C.byref(self._in)),
                        "sph_refresh_cells", ok=(SPH_OK, SPH_E_REBUILD))
        if st == SPH_OK:
            self.refreshes = getattr(self, "refreshes", 0) + 1
        else:
            self._built = False      # the library left the tree unbuilt
        return st == SPH_OK

    def same_layout(self, batch: Batch) -> bool:
        """Built, and for sets with the batch's offsets and boxes."""
        b = self.batch
        return (getattr(self, "_built", False) and b is not None and b.nsets == batch.nsets and np.array_equal(b.offsets, batch.offsets)
                and np.array_equal(np.asarray(b.box, dtype=np.float64), np.asarray(batch.box, dtype=np.float64)))

    def sort_pairs(self):
        self._sorted = False
        self._call(lambda: lib().sph_sort_pairs(self.ctx.h, self.h), "sph_sort_pairs")
        self._sorted = True

    def density(self, out: DensityOut):
        self._dout = out.c()
        self._call(lambda: lib().sph_density(self.ctx.h, self.h, C.byref(self._dout)), "sph_density")

    def solve_h(self, out: DensityOut):
        """Returns (status, n_unconverged, iterations); REBUILD/NOCONV are returned, not raised."""
        self._dout = out.c()
        nu, it = C.c_int32(0), C.c_int32(0)
        st = self._call(lambda: lib().sph_solve_h(self.ctx.h, self.h, C.byref(self._dout), C.byref(nu),
                                                  C.byref(it)),
                        "sph_solve_h", ok=(SPH_OK, SPH_E_REBUILD, SPH_E_NOCONV))
        return st, int(nu.value), int(it.value)

    def force(self, out: ForceOut):
        self._fout = out.c()
        self._call(lambda: lib().sph_force(self.ctx.h, self.h, C.byref(self._fout)), "sph_force")

    def set_halo(self, owned, rho, drho_dh):
        """Mark the particles owned (uint8 tensor, 1) or read-only halo (0)
        and give the halo particles' rho and d rho/dh (caller order)."""
        self._halo = (owned, rho, drho_dh)
        self.ctx.check(lib().sph_set_halo(self.ctx.h, self.h, _ptr(owned), _ptr(rho), _ptr(drho_dh)),
                       "sph_set_halo")

    def run_graph(self, k_iter: int, dout: DensityOut, fout: ForceOut, unconv):
        self._gd, self._gf = dout.c(), fout.c()
        self._call(lambda: lib().sph_run_graph(self.ctx.h, self.h, int(k_iter), C.byref(self._gd),
                                               C.byref(self._gf), _ptr(unconv)), "sph_run_graph")

    def stats(self) -> dict:
        v = (C.c_int64 * 13)()
        self.ctx.check(lib().sph_tree_stats(self.h, v, 13), "sph_tree_stats")
        keys = ["particles", "cells", "leaves", "tasks", "pair_tasks", "sorted_entries", "chunks", "levels",
                "top_grid", "max_leaf", "graph_captures", "heavy_chunks", "pieces"]
        return dict(zip(keys, [int(x) for x in v]))

    def bytes(self) -> int:
        b = C.c_size_t(0)
        self.ctx.check(lib().sph_tree_bytes(self.h, C.byref(b)), "sph_tree_bytes")
        return int(b.value)


def solve_with_rebuild(tree: Tree, batch: Batch, prm: sph_params, dout: DensityOut, max_rebuilds: int = 4,
                       halo=None, refresh: bool = False):
    """build -> sort -> solve_h, rebuilding with the current h when h outgrows
    the cells (the library reports it; the rebuild itself runs on the GPU).
    halo: (owned, rho, drho_dh) of one GPU's share, set after every build.
    refresh: first try to keep the tree's cells and sorted lists (a tree
    built for the same sets, whose particles moved since): the build and sort
    run only if the refresh is refused or h then outgrows the cells."""
    h = batch.h
    total_it = 0
    p = prm
    for k in range(max_rebuilds + 1):
        if k == 0 and refresh and tree.same_layout(batch) and tree.refresh(batch, h=h):
            if halo is not None:
                tree.set_halo(*halo)
        else:
            tree.build_cells(batch, p, h=h)
            if halo is not None:
                tree.set_halo(*halo)
            tree.sort_pairs()
        st, nu, it = tree.solve_h(dout)
        total_it += it
        if st == SPH_E_REBUILD:
            # rebuild from the h reached and continue the same Newton state
            h = dout.h.clone()
            p = sph_params.from_buffer_copy(prm)
            p.flags |= SPH_FLAG_RESUME
            continue
        return st, nu, total_it
    return SPH_E_REBUILD, -1, total_it


def kick(ctx: Context, dt: float, v, u, a, dudt, v_out=None, u_out=None):
    """v_out = v + dt a, u_out = u + dt du/dt (v, a, v_out: triples of device
    tensors); in place when the outputs are omitted."""
    v_out = v if v_out is None else v_out
    u_out = u if u_out is None else u_out
    n = int(u.numel())
    ctx.check(lib().sph_kick(ctx.h, n, float(dt), *(_ptr(t) for t in v), _ptr(u), *(_ptr(t) for t in a),
                             _ptr(dudt), *(_ptr(t) for t in v_out), _ptr(u_out)), "sph_kick")


def drift(ctx: Context, batch: Batch, dt: float, v=None):
    """x += dt v for every set of the batch, wrapped into its box (v defaults
    to the batch velocities)."""
    vx, vy, vz = (batch.vx, batch.vy, batch.vz) if v is None else v
    off = np.ascontiguousarray(batch.offsets, dtype=np.int64)
    box = np.ascontiguousarray(batch.box, dtype=np.float64)
    ctx.check(lib().sph_drift(ctx.h, batch.nsets, off.ctypes.data_as(C.c_void_p), box.ctypes.data_as(C.c_void_p),
                              float(dt), _ptr(batch.x), _ptr(batch.y), _ptr(batch.z), _ptr(vx), _ptr(vy), _ptr(vz)),
              "sph_drift")


def cfl_dt(ctx: Context, h, vsig, c_cfl: float = 0.3) -> float:
    dt = C.c_double(0.0)
    ctx.check(lib().sph_cfl_dt(ctx.h, int(h.numel()), _ptr(h), _ptr(vsig), float(c_cfl), C.byref(dt)), "sph_cfl_dt")
    return float(dt.value)
