"""ctypes binding of the CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library. States are numpy arrays
of shape [4, nv] (rho, rho u, rho v, e), float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rd_oracle.cpp")
LIB = os.environ.get("RDO_LIB") or os.path.join(HERE, "liboracle.so")

N, LDA, B, BMAX, BMIN, BX = 0, 1, 2, 3, 4, 5
EULER1, RK2 = 1, 2


def host_sanitize_flags() -> list:
    """AddressSanitizer and UndefinedBehaviorSanitizer flags for a host build
    when RD_HOST_SANITIZE is set (the process must then preload libasan)."""
    if not os.environ.get("RD_HOST_SANITIZE"):
        return []
    return ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g"]


def compile_cmd(src: str, out: str) -> list:
    return ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", out, src] + host_sanitize_flags()


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        subprocess.run(compile_cmd(SRC, LIB), check=True)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.rdo_mesh_new.restype = P
        L.rdo_mesh_new.argtypes = [C.c_int64, C.c_int64, dp, dp, P, C.c_double, C.c_double,
                                   P, C.c_int64, P, C.c_double, C.c_char_p, C.c_int]
        L.rdo_mesh_free.argtypes = [P]
        L.rdo_set_lumping.argtypes = [P, C.c_int]
        L.rdo_domain_size.argtypes = [P]
        L.rdo_domain_size.restype = C.c_double
        L.rdo_geometry.argtypes = [P, dp, dp, dp, dp]
        L.rdo_residual.argtypes = [P, dp, C.c_int, dp, P]
        L.rdo_residual.restype = C.c_int
        L.rdo_parts.argtypes = [P, dp, C.c_int, dp]
        L.rdo_parts.restype = C.c_int
        L.rdo_step.argtypes = [P, dp, C.c_double, C.c_int, C.c_int]
        L.rdo_step.restype = C.c_int
        L.rdo_step_jvp.argtypes = [P, dp, dp, C.c_double, C.c_int, C.c_int]
        L.rdo_step_jvp.restype = C.c_int
        L.rdo_max_dt.argtypes = [P, dp, C.c_double]
        L.rdo_max_dt.restype = C.c_double
        L.rdo_triangle.argtypes = [dp, dp, C.c_double, C.c_int, dp]
        L.rdo_triangle.restype = C.c_int
        L.rdo_kmat.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.rdo_solve4.argtypes = [dp, dp, dp]
        L.rdo_set_threads.argtypes = [C.c_int]
        L.rdo_max_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().rdo_set_threads(int(n))


def max_threads() -> int:
    return int(lib().rdo_max_threads())


class OracleMesh:
    """A mesh (dict from ``paper_1705_02028_amd.inputs``) held by the oracle."""

    def __init__(self, mesh: dict):
        L = lib()
        self.nv = int(mesh["nv"])
        self.nt = int(mesh["nt"])
        self.gamma = float(mesh.get("gamma", 1.4))
        self._keep = [np.ascontiguousarray(mesh["tri"], dtype=np.int32),
                      np.ascontiguousarray(mesh["ghost"], dtype=np.uint8),
                      np.ascontiguousarray(mesh["wall"], dtype=np.int32)]
        tri, ghost, wall = self._keep
        err = C.create_string_buffer(256)
        self._h = L.rdo_mesh_new(self.nv, self.nt, np.ascontiguousarray(mesh["x"], np.float64),
                                 np.ascontiguousarray(mesh["y"], np.float64), tri.ctypes.data,
                                 float(mesh["px"]), float(mesh["py"]), ghost.ctypes.data,
                                 int(wall.shape[0]), wall.ctypes.data if wall.size else None,
                                 self.gamma, err, 256)
        if not self._h:
            raise ValueError(err.value.decode())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.rdo_mesh_free(h)
            self._h = None

    def set_lumping(self, selective: bool) -> None:
        """Stage-2 mass term: global lumping (default) or selective lumping."""
        lib().rdo_set_lumping(self._h, 1 if selective else 0)

    def domain_size(self) -> float:
        """L of the Bx sensor."""
        return float(lib().rdo_domain_size(self._h))

    def geometry(self):
        area = np.zeros(self.nt)
        nrm = np.zeros((self.nt, 3, 2))
        lmax = np.zeros(self.nt)
        V = np.zeros(self.nv)
        lib().rdo_geometry(self._h, area, nrm.reshape(-1), lmax, V)
        return dict(area=area, nrm=nrm, lmax=lmax, V=V)

    def residual(self, W, scheme=B, with_phiT=False):
        W = np.ascontiguousarray(W, dtype=np.float64)
        R = np.zeros((4, self.nv))
        phiT = np.zeros((4, self.nt)) if with_phiT else None
        rc = lib().rdo_residual(self._h, W.reshape(-1), int(scheme), R.reshape(-1),
                                phiT.ctypes.data if with_phiT else None)
        if rc:
            raise ValueError("bad arguments")
        return (R, phiT) if with_phiT else R

    def parts(self, W, scheme=B):
        W = np.ascontiguousarray(W, dtype=np.float64)
        out = np.zeros((self.nt, 3, 4))
        if lib().rdo_parts(self._h, W.reshape(-1), int(scheme), out.reshape(-1)):
            raise ValueError("bad arguments")
        return out

    def step(self, W, dt, scheme=B, time_order=RK2):
        out = np.array(W, dtype=np.float64, copy=True, order="C")
        if lib().rdo_step(self._h, out.reshape(-1), float(dt), int(scheme), int(time_order)):
            raise ValueError("bad arguments")
        return out

    def step_jvp(self, W, dW, dt, scheme=B, time_order=RK2):
        out = np.array(W, dtype=np.float64, copy=True, order="C")
        dout = np.array(dW, dtype=np.float64, copy=True, order="C")
        if lib().rdo_step_jvp(self._h, out.reshape(-1), dout.reshape(-1), float(dt),
                              int(scheme), int(time_order)):
            raise ValueError("bad arguments")
        return out, dout

    def max_dt(self, W, cfl):
        W = np.ascontiguousarray(W, dtype=np.float64)
        return float(lib().rdo_max_dt(self._h, W.reshape(-1), float(cfl)))


def triangle(W3, xy, gamma=1.4, scheme=B):
    """One triangle: returns dict(phiT[4], phiN[3,4], phiLDA[3,4], phiB[3,4], theta[4])."""
    out = np.zeros(52)
    lib().rdo_triangle(np.ascontiguousarray(W3, np.float64).reshape(-1),
                       np.ascontiguousarray(xy, np.float64).reshape(-1), float(gamma), int(scheme), out)
    return dict(phiT=out[0:4], phiN=out[4:16].reshape(3, 4), phiLDA=out[16:28].reshape(3, 4),
                phiB=out[28:40].reshape(3, 4), theta=out[40:44])


def kmat(W, nx, ny, gamma=1.4):
    """(K, K+, K-) for state W and length-scaled normal (nx, ny), factor 1/2 included."""
    K = np.zeros(16)
    Kp = np.zeros(16)
    Km = np.zeros(16)
    lib().rdo_kmat(np.ascontiguousarray(W, np.float64), float(nx), float(ny), float(gamma), K, Kp, Km)
    return K.reshape(4, 4), Kp.reshape(4, 4), Km.reshape(4, 4)


def solve4(A, b):
    x = np.zeros(4)
    lib().rdo_solve4(np.ascontiguousarray(A, np.float64).reshape(-1),
                     np.ascontiguousarray(b, np.float64), x)
    return x
