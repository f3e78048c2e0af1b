"""ctypes binding of the three-dimensional CPU oracle (``oracle/liboracle3.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's
CPU-baseline leg, never by the library. States are numpy arrays of shape
[5, nv] (rho, rho u, rho v, rho w, e), float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rd3_oracle.cpp")
LIB = os.environ.get("RDO3_LIB") or os.path.join(HERE, "liboracle3.so")

N, LDA, B, BMAX, BMIN = 0, 1, 2, 3, 4
EULER1, RK2 = 1, 2


def host_sanitize_flags() -> list:
    """AddressSanitizer and UndefinedBehaviorSanitizer flags for a host build
    when RD_HOST_SANITIZE is set (the process must then preload libasan)."""
    if not os.environ.get("RD_HOST_SANITIZE"):
        return []
    return ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g"]


def compile_cmd(src: str, out: str) -> list:
    return ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
            "-Wall", "-o", out, src] + host_sanitize_flags()


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
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.rdo3_mesh_new.restype = P
        L.rdo3_mesh_new.argtypes = [C.c_int64, C.c_int64, dp, dp, dp, ip, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_char_p, C.c_int]
        L.rdo3_mesh_free.argtypes = [P]
        L.rdo3_geometry.argtypes = [P, dp, dp, dp, dp]
        L.rdo3_residual.argtypes = [P, dp, C.c_int, dp]
        L.rdo3_step.argtypes = [P, dp, C.c_double, C.c_int, C.c_int]
        L.rdo3_max_dt.argtypes = [P, dp, C.c_double]
        L.rdo3_max_dt.restype = C.c_double
        L.rdo3_tet.argtypes = [dp, dp, C.c_double, C.c_int, dp]
        L.rdo3_kmat.argtypes = [dp, dp, C.c_double, dp, dp, dp]
        L.rdo3_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


class OracleMesh3:
    def __init__(self, mesh: dict):
        self.nv, self.nt = int(mesh["nv"]), int(mesh["nt"])
        err = C.create_string_buffer(256)
        self.h = lib().rdo3_mesh_new(self.nv, self.nt, np.ascontiguousarray(mesh["x"], np.float64),
                                     np.ascontiguousarray(mesh["y"], np.float64),
                                     np.ascontiguousarray(mesh["z"], np.float64),
                                     np.ascontiguousarray(mesh["tet"], np.int32), float(mesh["px"]),
                                     float(mesh["py"]), float(mesh["pz"]), float(mesh.get("gamma", 1.4)), err, 256)
        if not self.h:
            raise ValueError(err.value.decode())

    def __del__(self):
        if getattr(self, "h", None):
            lib().rdo3_mesh_free(self.h)
            self.h = None

    def geometry(self):
        vol, nrm, smax, V = np.zeros(self.nt), np.zeros(12 * self.nt), np.zeros(self.nt), np.zeros(self.nv)
        lib().rdo3_geometry(self.h, vol, nrm, smax, V)
        return vol, nrm.reshape(self.nt, 4, 3), smax, V

    def residual(self, W, scheme):
        R = np.zeros((5, self.nv))
        lib().rdo3_residual(self.h, np.ascontiguousarray(W, np.float64), int(scheme), R)
        return R

    def step(self, W, dt, scheme, order):
        out = np.array(W, dtype=np.float64, order="C", copy=True)
        lib().rdo3_step(self.h, out, float(dt), int(scheme), int(order))
        return out

    def max_dt(self, W, cfl):
        return lib().rdo3_max_dt(self.h, np.ascontiguousarray(W, np.float64), float(cfl))


def tet(W4, xyz, gamma, scheme):
    """One tetrahedron: dict of phiT [5], phiN [4, 5], phiLDA [4, 5], phi [4, 5], theta [5]."""
    out = np.zeros(70)
    lib().rdo3_tet(np.ascontiguousarray(W4, np.float64).ravel(), np.ascontiguousarray(xyz, np.float64).ravel(),
                   float(gamma), int(scheme), out)
    return {"phiT": out[:5], "phiN": out[5:25].reshape(4, 5), "phiLDA": out[25:45].reshape(4, 5),
            "phi": out[45:65].reshape(4, 5), "theta": out[65:70]}


def kmat(W, n, gamma):
    """(K, K+, K-) as [5, 5] arrays: |n| K(n / |n|) at the state W [5]."""
    K, Kp, Km = np.zeros(25), np.zeros(25), np.zeros(25)
    lib().rdo3_kmat(np.ascontiguousarray(W, np.float64), np.ascontiguousarray(n, np.float64), float(gamma),
                    K, Kp, Km)
    return K.reshape(5, 5), Kp.reshape(5, 5), Km.reshape(5, 5)
