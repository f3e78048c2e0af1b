"""Python binding of librd (``include/rd.h``): argument marshalling only.

Every function named like the C entry points takes and returns plain
values, numpy arrays (host) or torch tensors (device, float64, contiguous,
on the current HIP device). All arithmetic runs in the library's HIP
kernels; if ``librd.so`` is missing this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librd.so")

RD_OK, RD_EINVAL, RD_ENOMEM, RD_EDEVICE, RD_ENONPHYS, RD_EUNSUPPORTED = range(6)
N, LDA, B, BMAX, BMIN, BX = range(6)
LUMP_GLOBAL, LUMP_SELECTIVE = 0, 1
EULER1, RK2 = 1, 2
FP64, FP32_ACC64 = 0, 1

_STATUS = {0: "RD_OK", 1: "RD_EINVAL", 2: "RD_ENOMEM", 3: "RD_EDEVICE", 4: "RD_ENONPHYS",
           5: "RD_EUNSUPPORTED"}


class RDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class rd_mesh_desc(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_triangles", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("tri", C.c_void_p),
                ("period_x", C.c_double), ("period_y", C.c_double),
                ("ghost", C.c_void_p), ("n_wall_edges", C.c_int64), ("wall_edges", C.c_void_p),
                ("gamma", C.c_double)]


class rd3_mesh_desc(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("tet", C.c_void_p),
                ("period_x", C.c_double), ("period_y", C.c_double), ("period_z", C.c_double),
                ("gamma", C.c_double)]


EXPORTS = ["rd_mesh_validate", "rd_mesh_create", "rd_mesh_destroy", "rd_mesh_info", "rd_set_stream",
           "rd_set_state", "rd_get_state", "rd_max_dt", "rd_step", "rd_step_cfl", "rd_step_timed", "rd_residual",
           "rd_adjoint_step", "rd_adjoint_step_noalloc", "rd_batch_create", "rd_batch_run", "rd_batch_destroy", "rd_sync",
           "rd_last_error", "rd_mesh_set_tile", "rd_mesh_get_tile", "rd_mesh_tile_info", "rd_tune",
           "rd_batch_set_tile", "rd_batch_tune", "rd_mesh_set_lumping", "rd_mesh_get_lumping",
           "rd_delaunay_flip", "rd_delaunay_refine", "rd3_mesh_create", "rd3_mesh_destroy", "rd3_set_state",
           "rd3_get_state", "rd3_max_dt", "rd3_step", "rd3_step_cfl", "rd3_step_timed", "rd3_sync"]

_lib = None


def lib():
    """The loaded librd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P, I, D, I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
        sig = {
            "rd_mesh_validate": [P],
            "rd_mesh_create": [P, P, P],
            "rd_mesh_destroy": [P],
            "rd_mesh_info": [P, P, P],
            "rd_set_stream": [P, P],
            "rd_set_state": [P, P, I],
            "rd_get_state": [P, P, I],
            "rd_max_dt": [P, D, P],
            "rd_step": [P, D, I, I, I],
            "rd_step_cfl": [P, I, D, I, I, I],
            "rd_step_timed": [P, D, I, I, I, P],
            "rd_residual": [P, I, P, P, I],
            "rd_adjoint_step": [P, P, D, I, I, P, P, I],
            "rd_adjoint_step_noalloc": [P, P, D, I, I, P, P, P],
            "rd_batch_create": [P, I, P, P],
            "rd_batch_run": [P, I, D, I, I, I],
            "rd_batch_destroy": [P],
            "rd_sync": [P],
            "rd_mesh_set_tile": [P, I],
            "rd_mesh_set_lumping": [P, I],
            "rd_delaunay_flip": [I64, P, P, D, D, I64, P, P, P],
            "rd_delaunay_refine": [P, P, P, I64, D, D, P, P, I64, D, D, P, I, I, I, I, P, P],
            "rd3_mesh_create": [P, P],
            "rd3_mesh_destroy": [P],
            "rd3_set_state": [P, P, I],
            "rd3_get_state": [P, P, I],
            "rd3_max_dt": [P, D, P],
            "rd3_step": [P, D, I, I],
            "rd3_step_cfl": [P, I, D, I, I],
            "rd3_step_timed": [P, I, D, I, I, P],
            "rd3_sync": [P],
            "rd_mesh_get_lumping": [P, P],
            "rd_mesh_get_tile": [P, P],
            "rd_mesh_tile_info": [P, P],
            "rd_tune": [P, D, I, I, I, I, P, I, P, P],
            "rd_batch_set_tile": [P, I],
            "rd_batch_tune": [P, D, I, I, I, I, P, I, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = I
        L.rd_last_error.restype = C.c_char_p
        L.rd_last_error.argtypes = []
        _ = I64
        _lib = L
    return _lib


def _check(st: int):
    if st != RD_OK:
        raise RDError(st, lib().rd_last_error().decode())


def _ptr(a, dev: bool):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if dev:
        if a.dtype.__str__() != "torch.float64" or not a.is_contiguous() or not a.is_cuda:
            raise ValueError("device arrays must be contiguous float64 tensors on the GPU")
        return a.data_ptr()
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError("host arrays must be C-contiguous float64")
    return a.ctypes.data


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def current_stream():
    """hipStream_t of torch's current stream (None when torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _desc(mesh: dict):
    keep = dict(x=np.ascontiguousarray(mesh["x"], np.float64),
                y=np.ascontiguousarray(mesh["y"], np.float64),
                tri=np.ascontiguousarray(mesh["tri"], np.int32),
                ghost=np.ascontiguousarray(mesh.get("ghost", np.zeros(mesh["nv"])), np.uint8),
                wall=np.ascontiguousarray(mesh.get("wall", np.zeros((0, 2))), np.int32))
    d = rd_mesh_desc(int(mesh["nv"]), int(mesh["nt"]), keep["x"].ctypes.data, keep["y"].ctypes.data,
                     keep["tri"].ctypes.data, float(mesh.get("px", 0.0)), float(mesh.get("py", 0.0)),
                     keep["ghost"].ctypes.data if keep["ghost"].any() else None,
                     int(keep["wall"].shape[0]), keep["wall"].ctypes.data if keep["wall"].size else None,
                     float(mesh.get("gamma", 1.4)))
    return d, keep


# ------------------------------------------------ C-named thin wrappers ----

def rd_mesh_validate(mesh: dict) -> None:
    d, keep = _desc(mesh)
    _check(lib().rd_mesh_validate(C.byref(d)))


def rd_mesh_create(mesh: dict, stream=None):
    d, keep = _desc(mesh)
    h = C.c_void_p()
    _check(lib().rd_mesh_create(C.byref(d), stream, C.byref(h)))
    return h


def rd_mesh_destroy(h) -> None:
    _check(lib().rd_mesh_destroy(h))


def rd_mesh_info(h):
    nv, nt = C.c_int64(), C.c_int64()
    _check(lib().rd_mesh_info(h, C.byref(nv), C.byref(nt)))
    return nv.value, nt.value


def rd_set_stream(h, stream) -> None:
    _check(lib().rd_set_stream(h, stream))


def rd_set_state(h, W) -> None:
    dev = _is_torch(W)
    _check(lib().rd_set_state(h, _ptr(W, dev), int(dev)))


def rd_get_state(h, out) -> None:
    dev = _is_torch(out)
    _check(lib().rd_get_state(h, _ptr(out, dev), int(dev)))


def rd_max_dt(h, cfl: float) -> float:
    dt = C.c_double()
    _check(lib().rd_max_dt(h, float(cfl), C.byref(dt)))
    return dt.value


def rd_step(h, dt: float, scheme: int = B, time: int = RK2, precision: int = FP64) -> None:
    _check(lib().rd_step(h, float(dt), int(scheme), int(time), int(precision)))


def rd_step_cfl(h, n_steps: int, cfl: float, scheme: int = B, time: int = RK2, precision: int = FP64) -> None:
    _check(lib().rd_step_cfl(h, int(n_steps), float(cfl), int(scheme), int(time), int(precision)))


KERNELS = ["wall1", "tri1", "shared1", "cfl", "gather1", "wall2", "tri2", "gather2"]
TUNE_DEFAULT = [0, 64, 128, 256, 512]


def rd_step_timed(h, cfl: float, scheme: int = B, time: int = RK2, precision: int = FP64) -> dict:
    ms = np.zeros(len(KERNELS))
    _check(lib().rd_step_timed(h, float(cfl), int(scheme), int(time), int(precision), ms.ctypes.data))
    return dict(zip(KERNELS, ms.tolist()))


def rd_mesh_set_tile(h, tile_triangles: int) -> None:
    _check(lib().rd_mesh_set_tile(h, int(tile_triangles)))


def rd_mesh_get_tile(h) -> int:
    t = C.c_int()
    _check(lib().rd_mesh_get_tile(h, C.byref(t)))
    return t.value


def rd_mesh_set_lumping(h, lumping: int) -> None:
    _check(lib().rd_mesh_set_lumping(h, int(lumping)))


def rd_mesh_get_lumping(h) -> int:
    t = C.c_int()
    _check(lib().rd_mesh_get_lumping(h, C.byref(t)))
    return t.value


def rd_delaunay_flip(mesh: dict):
    """Delaunay triangulation of the mesh's points by GPU edge flips: returns
    (tri [nt, 3] int32, n_flips, n_rounds); the input dict is not changed."""
    x = np.ascontiguousarray(mesh["x"], dtype=np.float64)
    y = np.ascontiguousarray(mesh["y"], dtype=np.float64)
    tri = np.array(mesh["tri"], dtype=np.int32, order="C", copy=True)
    nf, nr = C.c_int64(), C.c_int32()
    _check(lib().rd_delaunay_flip(int(mesh["nv"]), x.ctypes.data, y.ctypes.data, float(mesh["px"]),
                                  float(mesh["py"]), int(mesh["nt"]), tri.ctypes.data, C.byref(nf), C.byref(nr)))
    return tri, nf.value, nr.value


def rd_mesh_tile_info(h) -> dict:
    a = (C.c_int64 * 4)()
    _check(lib().rd_mesh_tile_info(h, a))
    return dict(tiles=a[0], local_vertices=a[1], shared_vertices=a[2], shared_parts=a[3])


def _tune(fn, h, cfl, scheme, time, precision, n_steps, candidates):
    cand = list(TUNE_DEFAULT if candidates is None else candidates)
    arr = (C.c_int * len(cand))(*cand)
    ms = np.zeros(len(cand))
    best = C.c_int()
    _check(fn(h, float(cfl), int(scheme), int(time), int(precision), int(n_steps), arr, len(cand),
              ms.ctypes.data, C.byref(best)))
    return best.value, dict(zip(cand, ms.tolist()))


def rd_tune(h, cfl: float, scheme: int = B, time: int = RK2, precision: int = FP64, n_steps: int = 5,
            candidates=None):
    """Returns (chosen tile size, {candidate: ms per step, negative if unusable})."""
    return _tune(lib().rd_tune, h, cfl, scheme, time, precision, n_steps, candidates)


def rd_batch_set_tile(b, tile_triangles: int) -> None:
    _check(lib().rd_batch_set_tile(b, int(tile_triangles)))


def rd_batch_tune(b, cfl: float, scheme: int = B, time: int = RK2, precision: int = FP64, n_steps: int = 20,
                  candidates=None):
    return _tune(lib().rd_batch_tune, b, cfl, scheme, time, precision, n_steps, candidates)


def rd_residual(h, scheme: int, R, phiT=None) -> None:
    dev = _is_torch(R)
    _check(lib().rd_residual(h, int(scheme), _ptr(R, dev), _ptr(phiT, dev) if phiT is not None else None,
                             int(dev)))


def rd_adjoint_step(h, W_n, dt: float, scheme: int, time: int, lam_np1, lam_n) -> None:
    dev = _is_torch(lam_n)
    _check(lib().rd_adjoint_step(h, _ptr(W_n, dev), float(dt), int(scheme), int(time),
                                 _ptr(lam_np1, dev), _ptr(lam_n, dev), int(dev)))


def rd_adjoint_step_noalloc(h, W_n, dt: float, scheme: int, time: int, lam_np1, lam_n, flags) -> None:
    """Device tensors only: W_n, lam_np1, lam_n float64 [4, nv]; flags int32 [2]
    (set on the device: non-physical, skipped solve column)."""
    if not (_is_torch(flags) and flags.is_cuda and str(flags.dtype) == "torch.int32" and flags.numel() >= 2
            and flags.is_contiguous()):
        raise ValueError("flags must be a contiguous int32 tensor of 2 elements on the GPU")
    _check(lib().rd_adjoint_step_noalloc(h, _ptr(W_n, True), float(dt), int(scheme), int(time),
                                         _ptr(lam_np1, True), _ptr(lam_n, True), flags.data_ptr()))


def rd_batch_create(handles, stream=None):
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    b = C.c_void_p()
    _check(lib().rd_batch_create(arr, len(handles), stream, C.byref(b)))
    return b


def rd_batch_run(b, n_steps: int, cfl: float, scheme: int = B, time: int = RK2, precision: int = FP64) -> None:
    _check(lib().rd_batch_run(b, int(n_steps), float(cfl), int(scheme), int(time), int(precision)))


def rd_batch_destroy(b) -> None:
    _check(lib().rd_batch_destroy(b))


def rd_sync(h) -> None:
    _check(lib().rd_sync(h))


def rd_last_error() -> str:
    return lib().rd_last_error().decode()


# ----------------------------------------------------- convenience class ---

class Mesh:
    """Owns an rd_mesh; host states are numpy [4, nv] float64 arrays."""

    def __init__(self, mesh: dict, stream=None):
        self.nv = int(mesh["nv"])
        self.nt = int(mesh["nt"])
        self.h = rd_mesh_create(mesh, stream if stream is not None else current_stream())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            rd_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, W):
        if not _is_torch(W):
            W = np.ascontiguousarray(W, dtype=np.float64)
        rd_set_state(self.h, W)

    def get_state(self, out=None):
        if out is None:
            out = np.zeros((4, self.nv))
        rd_get_state(self.h, out)
        return out

    def max_dt(self, cfl: float) -> float:
        return rd_max_dt(self.h, cfl)

    def step(self, dt, scheme=B, time=RK2, precision=FP64):
        rd_step(self.h, dt, scheme, time, precision)

    def step_cfl(self, n_steps, cfl, scheme=B, time=RK2, precision=FP64):
        rd_step_cfl(self.h, n_steps, cfl, scheme, time, precision)

    @property
    def tile(self) -> int:
        return rd_mesh_get_tile(self.h)

    @tile.setter
    def tile(self, tile_triangles: int):
        rd_mesh_set_tile(self.h, tile_triangles)

    def tune(self, cfl, scheme=B, time=RK2, precision=FP64, n_steps=5, candidates=None):
        return rd_tune(self.h, cfl, scheme, time, precision, n_steps, candidates)

    @property
    def lumping(self) -> int:
        return rd_mesh_get_lumping(self.h)

    @lumping.setter
    def lumping(self, lumping: int):
        rd_mesh_set_lumping(self.h, lumping)

    def residual(self, scheme=B, with_phiT=False):
        R = np.zeros((4, self.nv))
        phiT = np.zeros((4, self.nt)) if with_phiT else None
        rd_residual(self.h, scheme, R, phiT)
        return (R, phiT) if with_phiT else R

    def sync(self):
        rd_sync(self.h)


class Batch:
    """Owns an rd_batch over a list of ``Mesh`` objects (kept alive here)."""

    def __init__(self, meshes, stream=None):
        self.meshes = list(meshes)
        self.h = rd_batch_create([m.h for m in self.meshes],
                                 stream if stream is not None else current_stream())

    def run(self, n_steps, cfl, scheme=B, time=RK2, precision=FP64):
        rd_batch_run(self.h, n_steps, cfl, scheme, time, precision)

    def set_tile(self, tile_triangles: int):
        rd_batch_set_tile(self.h, tile_triangles)

    def tune(self, cfl, scheme=B, time=RK2, precision=FP64, n_steps=20, candidates=None):
        return rd_batch_tune(self.h, cfl, scheme, time, precision, n_steps, candidates)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            rd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rd_delaunay_refine(mesh: dict, max_radius: float = 0.0, max_ratio: float = 2 ** 0.5,
                       max_vertices: int | None = None, max_triangles: int | None = None,
                       max_iterations: int = 1000, morton: bool = False, size_grid=None):
    """Delaunay refinement of a triangulation on the GPU (rd_delaunay_refine):
    returns a new mesh dict (x, y, tri, nv, nt, px, py) with the iteration and
    flip counts (n_iterations, n_flips); with morton, vertices and triangles
    are renumbered in Morton order as the mesh grows; size_grid ([ny, nx]
    positive scale factors) makes the size bound max_radius * s(x) with s
    bilinear on that grid over the domain. Default capacities:
    room for triangles of circumradius down to max_radius / 3 over the
    domain's area, or 64 times the input when max_radius is 0."""
    nv, nt = int(mesh["nv"]), int(mesh["nt"])
    if max_vertices is None:
        if max_radius > 0:
            x, y = np.asarray(mesh["x"]), np.asarray(mesh["y"])
            w = mesh["px"] or (x.max() - x.min())
            h = mesh["py"] or (y.max() - y.min())
            max_vertices = nv + int(4 * w * h / (max_radius / 3) ** 2) + 64
        else:
            max_vertices = 64 * nv + 64
    if max_triangles is None:
        max_triangles = 2 * max_vertices + nt
    x = np.zeros(max(max_vertices, nv))
    y = np.zeros(max(max_vertices, nv))
    x[:nv] = mesh["x"]
    y[:nv] = mesh["y"]
    tri = np.zeros((max(max_triangles, nt), 3), dtype=np.int32)
    tri[:nt] = mesh["tri"]
    cv, ct = C.c_int64(nv), C.c_int64(nt)
    ni, nf = C.c_int32(), C.c_int64()
    grid = None if size_grid is None else np.ascontiguousarray(size_grid, np.float64)
    gny, gnx = (0, 0) if grid is None else grid.shape
    _check(lib().rd_delaunay_refine(C.byref(cv), x.ctypes.data, y.ctypes.data, int(max_vertices),
                                    float(mesh["px"]), float(mesh["py"]), C.byref(ct), tri.ctypes.data,
                                    int(max_triangles), float(max_radius), float(max_ratio),
                                    None if grid is None else grid.ctypes.data, int(gnx), int(gny),
                                    int(max_iterations), int(bool(morton)), C.byref(ni), C.byref(nf)))
    nv, nt = cv.value, ct.value
    return {"x": x[:nv].copy(), "y": y[:nv].copy(), "tri": tri[:nt].copy(), "nv": nv, "nt": nt,
            "px": float(mesh["px"]), "py": float(mesh["py"]), "n_iterations": ni.value, "n_flips": nf.value}


class Mesh3:
    """A tetrahedral mesh on the current GPU (the rd3_* entry points):
    states are [5, nv] float64 (rho, rho u, rho v, rho w, e)."""

    def __init__(self, mesh: dict):
        keep = [np.ascontiguousarray(mesh[k], np.float64) for k in ("x", "y", "z")]
        tet = np.ascontiguousarray(mesh["tet"], np.int32)
        d = rd3_mesh_desc(int(mesh["nv"]), int(mesh["nt"]), keep[0].ctypes.data, keep[1].ctypes.data,
                          keep[2].ctypes.data, tet.ctypes.data, float(mesh["px"]), float(mesh["py"]),
                          float(mesh["pz"]), float(mesh.get("gamma", 1.4)))
        h = C.c_void_p()
        _check(lib().rd3_mesh_create(C.byref(d), C.byref(h)))
        self.h = h
        self.nv, self.nt = int(mesh["nv"]), int(mesh["nt"])

    def close(self):
        if self.h:
            lib().rd3_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, W):
        dev = not isinstance(W, np.ndarray)
        if not dev:
            W = np.ascontiguousarray(W, np.float64)
            if W.shape != (5, self.nv):
                raise ValueError("state must be [5, nv]")
        _check(lib().rd3_set_state(self.h, W.data_ptr() if dev else W.ctypes.data, int(dev)))

    def get_state(self):
        out = np.zeros((5, self.nv))
        _check(lib().rd3_get_state(self.h, out.ctypes.data, 0))
        return out

    def max_dt(self, cfl):
        dt = C.c_double()
        _check(lib().rd3_max_dt(self.h, float(cfl), C.byref(dt)))
        return dt.value

    def step(self, dt, scheme, time):
        _check(lib().rd3_step(self.h, float(dt), int(scheme), int(time)))

    def step_cfl(self, n, cfl, scheme, time):
        _check(lib().rd3_step_cfl(self.h, int(n), float(cfl), int(scheme), int(time)))

    def step_timed(self, n, cfl, scheme, time):
        ms = np.zeros(5)
        _check(lib().rd3_step_timed(self.h, int(n), float(cfl), int(scheme), int(time), ms.ctypes.data))
        return ms

    def sync(self):
        _check(lib().rd3_sync(self.h))

