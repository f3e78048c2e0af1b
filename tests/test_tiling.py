"""Host-side tile builder of the tiled step (rd_tiling.h), on the CPU.

Checks the invariants the tile kernels rely on: tiles partition the
triangles (Morton order within each mesh, never straddling two meshes), every
corner names its tile-local vertex, interior vertices have all their corners
in their tile with LDS slots in ascending triangle order, shared vertices own
exactly their corners' slots in the sliced buffer, and every index stays within
the sizes the kernels are launched with.
"""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1705_02028_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def shim():
    out = os.path.join(tempfile.mkdtemp(prefix="tiling_"), "libtiling.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-Wall",
                    "-I", os.path.join(ROOT, "paper_1705_02028_amd", "csrc"),
                    os.path.join(HERE, "cpp", "tiling_shim.cpp"), "-o", out] + oracle.host_sanitize_flags(),
                   check=True)
    L = C.CDLL(out)
    L.tiling_build.restype = C.c_int
    L.tiling_build.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                               C.c_int, C.c_void_p, C.c_void_p, C.c_int]
    L.tiling_sizes.argtypes = [C.c_void_p]
    L.tiling_arrays.argtypes = [C.c_void_p] * 12
    return L


def build(L, mesh, tt, voff=None, toff=None):
    nv, nt = mesh["nv"], mesh["nt"]
    voff = np.array([0, nv] if voff is None else voff, np.int64)
    toff = np.array([0, nt] if toff is None else toff, np.int64)
    tri = np.ascontiguousarray(mesh["tri"], np.int32)
    x = np.ascontiguousarray(mesh["x"], np.float64)
    y = np.ascontiguousarray(mesh["y"], np.float64)
    rc = L.tiling_build(nv, nt, tri.ctypes.data, x.ctypes.data, y.ctypes.data, mesh["px"], mesh["py"],
                        len(voff) - 1, voff.ctypes.data, toff.ctypes.data, tt)
    assert rc == 0
    sz = np.zeros(8, np.int64)
    L.tiling_sizes(sz.ctypes.data)
    ntiles, max_lv, max_lvi, max_slots, ntvl, nlp, nsv, nss = (int(v) for v in sz)
    a = dict(order=np.zeros(nt, np.int32), tbeg=np.zeros(ntiles + 1, np.int32), vbeg=np.zeros(ntiles + 1, np.int32),
             nvi=np.zeros(ntiles, np.int32), lpb=np.zeros(ntiles, np.int32), lp=np.zeros(nlp, np.int32),
             tvl=np.zeros(ntvl, np.int32), lv=np.zeros(3 * nt, np.uint16), dst=np.zeros(3 * nt, np.int32),
             tmesh=np.zeros(ntiles, np.int32), sv=np.zeros(nsv, np.int32), ssbeg=np.zeros(nsv, np.int32))
    L.tiling_arrays(*[a[k].ctypes.data for k in ("order", "tbeg", "vbeg", "nvi", "lpb", "lp", "tvl", "lv", "dst",
                                                  "tmesh", "sv", "ssbeg")])
    a.update(ntiles=ntiles, max_lv=max_lv, max_lvi=max_lvi, max_slots=max_slots, nss=nss, voff=voff, toff=toff)
    return a


def check(mesh, P, tt):
    nt, nv = mesh["nt"], mesh["nv"]
    tri = mesh["tri"]
    order = P["order"]
    assert np.array_equal(np.sort(order), np.arange(nt))          # a permutation of the triangles
    tbeg = P["tbeg"]
    assert tbeg[0] == 0 and tbeg[-1] == nt and np.all(np.diff(tbeg) >= 1) and np.all(np.diff(tbeg) <= tt)
    tile_of = np.empty(nt, np.int64)
    for k in range(P["ntiles"]):
        tile_of[order[tbeg[k]:tbeg[k + 1]]] = k
        # a tile never straddles two meshes, and its mesh id is right
        m = P["tmesh"][k]
        ts = order[tbeg[k]:tbeg[k + 1]]
        assert np.all((ts >= P["toff"][m]) & (ts < P["toff"][m + 1]))
    # vertex -> tiles of its corners
    vt = [set() for _ in range(nv)]
    inc = [[] for _ in range(nv)]
    for t in range(nt):
        for i in range(3):
            vt[tri[t, i]].add(int(tile_of[t]))
            inc[tri[t, i]].append((t, i))
    shared = np.array([len(s) > 1 for s in vt])
    assert np.array_equal(P["sv"], np.flatnonzero(shared))
    lv, dst = P["lv"].reshape(3, nt), P["dst"].reshape(3, nt)
    slot_of = {}                                                   # corner -> destination
    for k in range(P["ntiles"]):
        v0, v1, nvi = P["vbeg"][k], P["vbeg"][k + 1], P["nvi"][k]
        loc = P["tvl"][v0:v1]
        assert v1 - v0 <= P["max_lv"] and nvi <= P["max_lvi"]
        assert len(set(loc.tolist())) == len(loc)
        assert np.all(~shared[loc[:nvi]]) and np.all(shared[loc[nvi:]])
        lp = P["lp"][P["lpb"][k]:P["lpb"][k] + nvi + 1]
        assert lp[0] == 0 and np.all(np.diff(lp) >= 1) and lp[-1] <= P["max_slots"]
        for s in range(tbeg[k], tbeg[k + 1]):
            t = order[s]
            for i in range(3):
                v = tri[t, i]
                assert loc[lv[i, s]] == v                           # local vertex of the corner
                slot_of[(t, i)] = (k, int(dst[i, s]))
        for l in range(nvi):
            v = loc[l]
            corners = sorted(inc[v])                               # ascending triangle id
            got = [slot_of[c] for c in corners]
            assert all(g[0] == k for g in got)
            assert [-1 - g[1] for g in got] == list(range(lp[l], lp[l + 1]))
    # shared vertices: their j-th corner (ascending triangle id) at ssbeg + 64 j, all in range
    used = set()
    for kk, v in enumerate(P["sv"]):
        for j, c in enumerate(sorted(inc[v])):
            d = slot_of[c][1]
            assert d == P["ssbeg"][kk] + 64 * j and 0 <= d < P["nss"]
            used.add(d)
    assert len(used) == sum(len(inc[v]) for v in P["sv"])          # no two corners share a slot


@pytest.mark.parametrize("tt", [32, 64, 256])
def test_tiles_periodic_random_diagonals(shim, tt):
    m = I.split_square(23, diagonal="random", jitter=0.2, seed=3)
    P = build(shim, m, tt)
    check(m, P, tt)


@pytest.mark.parametrize("tt", [32, 100])
def test_tiles_walls_ghosts_random_numbering(shim, tt):
    m = I.split_square(19, periodic=(True, False), bc=("ghost", "wall"), renumber="random", seed=5)
    P = build(shim, m, tt)
    check(m, P, tt)


def test_tiles_of_a_batch_match_the_members_alone(shim):
    meshes = [I.split_square(n, periodic=(False, False), bc=("ghost", "ghost"), diagonal="random", seed=n)
              for n in (9, 14, 5)]
    flat = I.concat_meshes(meshes, spacing=0.0)
    voff = np.cumsum([0] + [mm["nv"] for mm in meshes])
    toff = np.cumsum([0] + [mm["nt"] for mm in meshes])
    P = build(shim, flat, 32, voff, toff)
    check(flat, P, 32)
    # member k's tiles are its own tiling, shifted by its offsets
    k0 = 0
    for k, mm in enumerate(meshes):
        Q = build(shim, mm, 32)
        n = Q["ntiles"]
        assert np.array_equal(P["tmesh"][k0:k0 + n], np.full(n, k))
        assert np.array_equal(P["order"][toff[k]:toff[k + 1]] - toff[k], Q["order"])
        assert np.array_equal(P["nvi"][k0:k0 + n], Q["nvi"])
        k0 += n
    assert k0 == P["ntiles"]


def test_morton_tiles_are_compact(shim):
    """On a structured mesh a Morton tile of 256 triangles covers a block of
    about 9 x 17 vertices: few shared vertices per tile."""
    m = I.split_square(129)
    P = build(shim, m, 256)
    lv_per_tile = np.diff(P["vbeg"])
    assert lv_per_tile.max() <= 200
    assert len(P["sv"]) < 0.4 * m["nv"]
