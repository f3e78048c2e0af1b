"""The C-ABI library loads on a machine without a GPU, exports exactly what
include/rd.h declares, and validates meshes on the host."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1705_02028_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rd():
    from paper_1705_02028_amd import rd as rdmod
    if not os.path.exists(rdmod.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build_hip()
    return rdmod


def declared():
    text = open(os.path.join(ROOT, "include", "rd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rd3?_[a-z_]+)\s*\(", text)))


def test_exports_match_header(rd):
    lib = rd.lib()
    names = declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", rd.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == names
    assert sorted(rd.EXPORTS) == names


def test_enum_values_match_header(rd):
    text = open(os.path.join(ROOT, "include", "rd.h")).read()
    for name, val in [("RD_N", rd.N), ("RD_LDA", rd.LDA), ("RD_B", rd.B), ("RD_BMAX", rd.BMAX),
                      ("RD_BMIN", rd.BMIN), ("RD_EULER1", rd.EULER1), ("RD_RK2", rd.RK2),
                      ("RD_FP64", rd.FP64), ("RD_FP32_ACC64", rd.FP32_ACC64), ("RD_OK", rd.RD_OK),
                      ("RD_EINVAL", rd.RD_EINVAL), ("RD_ENONPHYS", rd.RD_ENONPHYS), ("RD_BX", rd.BX),
                      ("RD_LUMP_GLOBAL", rd.LUMP_GLOBAL), ("RD_LUMP_SELECTIVE", rd.LUMP_SELECTIVE),
                      ("RD_EUNSUPPORTED", rd.RD_EUNSUPPORTED)]:
        assert re.search(rf"\b{name}\s*=\s*{val}\b", text), name


def test_desc_layout_matches_header(rd):
    # int64 x2, 3 pointers, 2 doubles, pointer, int64, pointer, double
    assert C.sizeof(rd.rd_mesh_desc) == 8 * 11


def test_host_validation_accepts_config_meshes(rd):
    for m in (I.split_square(64), I.split_square(33, periodic=(False, False), bc=("ghost", "wall")),
              I.split_square(20, diagonal="random", renumber="random", rotate_corners=True, jitter=0.2)):
        rd.rd_mesh_validate(m)


@pytest.mark.parametrize("case", ["clockwise", "index", "orphan", "gamma", "wall", "empty"])
def test_host_validation_rejects(rd, case):
    m = dict(I.split_square(6, periodic=(False, False), bc=("ghost", "wall")))
    if case == "clockwise":
        m["tri"] = np.ascontiguousarray(m["tri"][:, [0, 2, 1]])
        msg = "counter-clockwise"
    elif case == "index":
        t = m["tri"].copy()
        t[5, 2] = -1
        m["tri"] = t
        msg = "out of range"
    elif case == "orphan":
        m["x"] = np.append(m["x"], 3.0)
        m["y"] = np.append(m["y"], 3.0)
        m["ghost"] = np.append(m["ghost"], 0).astype(np.uint8)
        m["nv"] += 1
        msg = "no triangle"
    elif case == "gamma":
        m["gamma"] = 1.0
        msg = "gamma"
    elif case == "wall":
        w = m["wall"].copy()
        w[0, 1] = w[0, 0]
        m["wall"] = w
        msg = "wall edge"
    else:
        m["nt"] = 0
        msg = "empty"
    with pytest.raises(rd.RDError, match=msg) as e:
        rd.rd_mesh_validate(m)
    assert e.value.status == rd.RD_EINVAL


def test_periodic_unwrap_accepted_by_validation(rd):
    m = I.split_square(5)  # triangles straddle the periodic seam
    rd.rd_mesh_validate(m)
    m2 = dict(m)
    m2["px"] = 0.0  # without the period the seam triangles are inverted
    with pytest.raises(rd.RDError, match="counter-clockwise"):
        rd.rd_mesh_validate(m2)


def test_host_validation_limits_vertex_degree(rd):
    """A vertex may belong to at most 1023 triangles (the triangle's rank
    among a corner vertex's triangles is packed in 10 bits): a fan of n
    triangles around one centre vertex is accepted for n = 1023 and refused
    for n = 1024."""
    for n, ok in ((1023, True), (1024, False)):
        a = 2 * np.pi * np.arange(n) / n
        x = np.concatenate([[0.0], np.cos(a)])
        y = np.concatenate([[0.0], np.sin(a)])
        tri = np.array([[0, 1 + k, 1 + (k + 1) % n] for k in range(n)], dtype=np.int32)
        m = {"x": x, "y": y, "tri": tri, "nv": n + 1, "nt": n, "px": 0.0, "py": 0.0}
        if ok:
            rd.rd_mesh_validate(m)
        else:
            with pytest.raises(rd.RDError, match="at most 1023") as e:
                rd.rd_mesh_validate(m)
            assert e.value.status == rd.RD_EINVAL


def test_host_validation_rejects_sizes_beyond_32_bit_indices(rd):
    """3 n_triangles and n_vertices must stay below 2^31 (int32 corner and
    slot indices); the check runs before any array is read."""
    for nv, nt in ((16, 2 ** 31 // 3 + 1), (2 ** 31, 16)):
        d = rd.rd_mesh_desc(nv, nt, None, None, None, 0.0, 0.0, None, 0, None, 1.4)
        assert rd.lib().rd_mesh_validate(C.byref(d)) == rd.RD_EINVAL
        assert "too large" in rd.lib().rd_last_error().decode()
    d = rd.rd_mesh_desc(16, 2 ** 31 // 3, None, None, None, 0.0, 0.0, None, 0, None, 1.4)
    assert rd.lib().rd_mesh_validate(C.byref(d)) == rd.RD_EINVAL   # passes the size check, then
    assert "null" in rd.lib().rd_last_error().decode()             # stops at the missing arrays


def test_refinement_input_checks_run_on_the_host(rd):
    """rd_delaunay_refine refuses invalid bounds, capacities and domains
    before it touches a device."""
    sq = {"x": np.array([0.0, 1.0, 1.0, 0.0]), "y": np.array([0.0, 0.0, 1.0, 1.0]),
          "tri": np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32), "nv": 4, "nt": 2, "px": 0.0, "py": 0.0}
    skew = dict(sq, x=np.array([0.0, 1.0, 1.2, 0.0]))  # the right side is not axis-aligned
    per = I.split_square(6, periodic=(True, True), jitter=0.3, seed=1)  # coordinates below 0
    cases = [
        (sq, dict(max_ratio=0.5), "max_ratio"),
        (sq, dict(max_radius=-1.0), "max_radius"),
        (sq, dict(max_iterations=0), "max_iterations"),
        (sq, dict(max_vertices=3), "capacity"),
        (skew, dict(max_radius=0.1), "axis-aligned"),
        (per, dict(max_radius=0.1), "periodic axis"),
    ]
    for mesh, kw, msg in cases:
        kw = dict(kw)
        args = dict(max_radius=kw.pop("max_radius", 0.1), max_ratio=kw.pop("max_ratio", 2 ** 0.5))
        with pytest.raises(rd.RDError, match=msg) as e:
            rd.rd_delaunay_refine(mesh, **args, **kw)
        assert e.value.status == rd.RD_EINVAL


def test_3d_mesh_checks_run_on_the_host(rd):
    """rd3_mesh_create refuses invalid tetrahedral meshes before it touches a
    device."""
    import ctypes as C
    m = I.cube_tets(3, jitter=0.1, seed=1)

    def create(mesh):
        keep = [np.ascontiguousarray(mesh[k], np.float64) for k in ("x", "y", "z")]
        tet = np.ascontiguousarray(mesh["tet"], np.int32)
        d = rd.rd3_mesh_desc(int(mesh["nv"]), int(mesh["nt"]), keep[0].ctypes.data, keep[1].ctypes.data,
                             keep[2].ctypes.data, tet.ctypes.data, mesh["px"], mesh["py"], mesh["pz"],
                             mesh.get("gamma", 1.4))
        h = C.c_void_p()
        st = rd.lib().rd3_mesh_create(C.byref(d), C.byref(h))
        return st, rd.lib().rd_last_error().decode()

    flipped = dict(m, tet=m["tet"][:, [0, 2, 1, 3]])
    assert create(flipped) == (rd.RD_EINVAL, "tetrahedron 0 is not positively oriented")
    bad = dict(m, tet=np.where(m["tet"] == 5, m["nv"], m["tet"]))
    st, msg = create(bad)
    assert st == rd.RD_EINVAL and "out of range" in msg
    orphan = dict(m, x=np.append(m["x"], 0.5), y=np.append(m["y"], 0.5), z=np.append(m["z"], 0.5), nv=m["nv"] + 1)
    st, msg = create(orphan)
    assert st == rd.RD_EINVAL and "belongs to no tetrahedron" in msg
    st, msg = create(dict(m, gamma=1.0))
    assert st == rd.RD_EINVAL and "gamma" in msg


def test_refinement_capacity_limit_keeps_edge_keys_in_32_bits(rd):
    """Edge keys 3 t + i are 32-bit: a triangle capacity of 2^31 / 3 or more
    is refused before anything is allocated."""
    sq = {"x": np.array([0.0, 1.0, 1.0, 0.0]), "y": np.array([0.0, 0.0, 1.0, 1.0]),
          "tri": np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32), "nv": 4, "nt": 2, "px": 0.0, "py": 0.0}
    import ctypes as C
    x, y = sq["x"].copy(), sq["y"].copy()
    tri = sq["tri"].copy()
    nv, nt = C.c_int64(4), C.c_int64(2)
    st = rd.lib().rd_delaunay_refine(C.byref(nv), x.ctypes.data, y.ctypes.data, 4, 0.0, 0.0, C.byref(nt),
                                     tri.ctypes.data, (2 ** 31 - 1) // 3, 0.1, 2 ** 0.5, None, 0, 0, 10, 0,
                                     None, None)
    assert st == rd.RD_EINVAL and "32-bit" in rd.lib().rd_last_error().decode()
