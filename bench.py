"""Throughput of the residual-distribution step on one MI355X.

Workload: Kelvin-Helmholtz shear layer on a 2048x2048 periodic split-square
mesh (4,190,209 vertices, 8,380,418 triangles), B scheme, two-stage
Runge-Kutta, CFL 0.4 with the time step computed on the device every step.
The headline value is the FP32-distribution / FP64-accumulation variant (the
configuration's arithmetic); the FP64 variant is timed on the same mesh and
reported beside it. One step = CFL limit + both Runge-Kutta stages (two
triangle passes and two vertex gathers). Inputs are resident on the GPU
before timing starts. Also timed on the same workload: the Bx blend and the
B scheme with selective lumping (`variants`), the adjoint step against the
forward step, the GPU Delaunay refinement of a 1.3-million-vertex periodic
mesh (`mesh_generation`; alone with --meshgen), the three-dimensional path
on a 128^3-cell box of tetrahedra (`three_d`; alone with --three-d), and
(with --batch) many meshes in one graph.

Prints one JSON line. `--gpus N` with N > 1 exits: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12        # bytes/s, MI355X HBM3E
PEAK_FP64 = 78.6e12      # flop/s, vector FP64
PEAK_FP32 = 157.3e12     # flop/s, vector FP32


def method_bytes(nt, fp32):
    """The method's algorithmic HBM bytes per pass of an RK2/B step, per the
    cost model of the hot-path scope: ideal vertex reuse (half a vertex
    record per triangle), indices int32, reals of the triangle algebra's
    precision q (8 FP64, 4 FP32). Per triangle:
      triangle pass: corner ids 12 + coordinates 8 + Z 4q/2 + parts 12q,
        stage 1 also saves the N parts 12q, stage 2 reads them 12q and W^n 16;
      gather / update pass: CSR 14 + parts 12q + W read and written 32 +
        1/V 4 + Z written 4q/2.
    FP64: 228 / 244 B (stages 1 / 2), 162 B per gather; FP32 distribution:
    124 / 140 B, 106 B per gather; about 800 and 480 B per triangle-step.
    The CFL and wall passes are not in the model (0)."""
    q = 4 if fp32 else 8
    tri = 12 + 8 + 2 * q + 12 * q
    gat = 14 + 12 * q + 32 + 4 + 2 * q
    k = {"tri1": nt * (tri + 12 * q), "tri2": nt * (tri + 12 * q + 16), "gather1": nt * gat, "gather2": nt * gat,
         "shared1": 0, "cfl": 0, "wall1": 0, "wall2": 0}
    return k


def algorithmic_bytes(nt, nv, fp32):
    """Implementation bytes: what each kernel of this library's RK2/B step
    with the CFL limit moves at least once, with every vertex record read once
    per pass (ideal reuse). Larger than method_bytes by the library's own
    records (the packed slot ranks, the CFL term per triangle, the triangle
    of every part slot, the kept residual). q = bytes per real of the
    triangle algebra; a part or parameter vector is 4 reals; parts live in
    vertex-CSR order (one record per corner). The slice bases (4 bytes per
    64 vertices) are left out."""
    q = 4 if fp32 else 8
    r4 = 4 * q
    k = {}
    # stage 1: corner ids and packed slot ranks, coordinates, Z and |v|+c in;
    # parts, kept N parts (corners 0 and 1), phi^T and l_max lambda_max per
    # triangle out (the CFL term in the triangle algebra's precision)
    k["tri1"] = nt * (12 + 4 + 3 * r4 + 2 * r4 + r4 + q) + nv * (16 + r4 + 8)
    # CFL: CSR rows, V, the triangle of each of a vertex's slots and the
    # triangles' l_max lambda_max in, block minima out
    k["shared1"] = 0
    k["cfl"] = nv * (4 + 8) + nt * (3 * 4 + q)
    # gather 1: rows, parts in; W, V in; W*, W*-W, Z* out
    k["gather1"] = nt * 3 * r4 + nv * (4 + 32 + 8 + 32 + r4 + r4)
    # stage 2: ids, ranks, coordinates, Z*, W*-W, kept N parts, phi^T in; parts out
    k["tri2"] = nt * (12 + 4 + 2 * r4 + r4 + 3 * r4) + nv * (16 + r4 + r4)
    # gather 2: rows, parts in; W*, V in; W, Z, |v|+c out
    k["gather2"] = nt * 3 * r4 + nv * (4 + 32 + 8 + 32 + r4 + 8)
    k["wall1"] = k["wall2"] = 0
    return k


def algorithmic_bytes_tiled(nt, nv, fp32, info):
    """The same for the tiled form. info = rd_mesh_tile_info: L local vertex
    records over all tiles (a vertex on a tile border is loaded by each of its
    tiles), S shared vertices, P their parts; I = nv - S vertices are finished
    inside their tile. Parts of interior vertices never leave LDS."""
    q = 4 if fp32 else 8
    r4 = 4 * q
    L, S, P = info["local_vertices"], info["shared_vertices"], info["shared_parts"]
    I = nv - S
    k = {}
    # tile pass 1: corner tables, vertex records (id, xy, Z, |v|+c) in; kept N parts and phi^T,
    # interior R1 and CFL bound, shared parts and l_max lambda_max out
    k["tri1"] = nt * (18 + 2 * r4 + r4) + L * (4 + 16 + r4 + 8) + I * (4 + 8 + 32 + 8) + P * (r4 + 8)
    # shared pass 1: ids, slots, rows, V in; parts and CFL terms in; R1 and CFL bound out
    k["shared1"] = S * (4 + 4 + 8 + 8 + 32 + 8) + P * (r4 + 8)
    k["cfl"] = nv * 8
    k["gather1"] = 0
    # tile pass 2: corner tables, kept N parts and phi^T, vertex records (id, xy, W, R1, V) in;
    # interior W, Z, |v|+c and shared parts out
    k["tri2"] = nt * (18 + 2 * r4 + r4) + L * (4 + 16 + 32 + 32 + 8) + I * (4 + 32 + r4 + 8) + P * r4
    # shared pass 2: ids, slots, rows, V, W, R1, parts in; W, Z, |v|+c out
    k["gather2"] = S * (4 + 4 + 8 + 8 + 32 + 32 + 32 + r4 + 8) + P * r4
    k["wall1"] = k["wall2"] = 0
    return k


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_kh2048.txt")


# The sources that define the triangle kernels of both forms (their bodies,
# launch shapes and the translation units they are compiled in).
TRI_SOURCES = ("rd_device.h", "rd_kcommon.h", "rd_launch.h", "rd_kernels.hip", "rd_tiles.h", "rd_tiles.hip")


def source_hash():
    """Hash of the triangle kernels' sources: measured traffic is reported only
    for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in TRI_SOURCES:
        with open(os.path.join(ROOT, "paper_1705_02028_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of one kernel (FETCH_SIZE + WRITE_SIZE from
    rocprofv3 counter runs, scaled by the copy-kernel calibration), from
    profiles/hbm_traffic_kh2048.txt; None if absent or taken on other kernel
    sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    v = rec.get("bytes_per_launch", {}).get(key)
    return None if v is None else int(v)


def roofline_entry(name, mbytes, ibytes, ms, traffic_key=None):
    """Roofline of one kernel: `achieved` and `frac` from the method's
    algorithmic bytes (method_bytes) over the kernel's average duration; the
    implementation's own byte count beside it."""
    achieved = mbytes / (ms * 1e-3)
    impl = ibytes / (ms * 1e-3)
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved / 1e9, 1), "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 4),
            "traffic": measured_traffic(traffic_key) if traffic_key else None,
            "algorithmic_bytes": int(mbytes), "avg_ms": round(ms, 5),
            "implementation": {"bytes": int(ibytes), "achieved": round(impl / 1e9, 1),
                               "frac": round(impl / PEAK_HBM, 4)}}


def step_roofline(nt, fp32, ms_step):
    """The whole step against HBM: the method's bytes of all four passes over
    the measured time per step."""
    b = sum(method_bytes(nt, fp32).values())
    return {"bytes": int(b), "achieved": round(b / (ms_step * 1e-3) / 1e9, 1),
            "frac": round(b / (ms_step * 1e-3) / PEAK_HBM, 4)}


STAGE1 = ("wall1", "tri1", "shared1", "cfl", "gather1")


def stage_rates(per, nt):
    """Per-stage times (the sum of each stage's kernel times; the CFL pass
    counts with stage 1) and the triangle-updates/s of each stage alone."""
    s1 = sum(v for k, v in per.items() if k in STAGE1)
    s2 = sum(v for k, v in per.items() if k not in STAGE1)
    return {"stage1_ms": round(s1, 5), "stage2_ms": round(s2, 5),
            "stage1_triangle_updates_per_s": round(nt / (s1 * 1e-3), 1) if s1 > 0 else None,
            "stage2_triangle_updates_per_s": round(nt / (s2 * 1e-3), 1) if s2 > 0 else None}


def form_name(tile):
    return "two-pass" if tile == 0 else f"tiled-{tile}"


def time_variant(rd, torch, mesh, W0, prec, steps, warmup, cfl, timed_reps, tile, scheme=None, lump=0):
    scheme = rd.B if scheme is None else scheme
    g = rd.Mesh(mesh)
    g.set_state(W0)
    g.lumping = lump
    tuned = None
    if tile < 0:
        # twelve timed steps per candidate: the forms can differ by a few per
        # cent, about the spread of a three-step replay
        best, table = g.tune(cfl, scheme, rd.RK2, prec, n_steps=12)
        tuned = {"chosen": best, "ms_per_step": {str(k): round(v, 5) for k, v in table.items()}}
    else:
        g.tile = tile
    info = rd.rd_mesh_tile_info(g.h)
    if warmup:
        g.step_cfl(warmup, cfl, scheme, rd.RK2, prec)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step_cfl(steps, cfl, scheme, rd.RK2, prec)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g.sync()
    per = {}
    for _ in range(max(timed_reps, 1)):
        t = rd.rd_step_timed(g.h, cfl, scheme, rd.RK2, prec)
        for k, v in t.items():
            per[k] = per.get(k, 0.0) + v / max(timed_reps, 1)
    g.sync()
    tile_used = g.tile
    g.close()
    return ms, per, {"tile": tile_used, "tuner": tuned, "tile_info": info}


def adjoint_ratio(rd, torch, mesh, W0, cfl, reps, tile):
    """time(rd_adjoint_step) / time(rd_step) on the same mesh, FP64, B / RK2,
    fixed dt, device-resident states; each timed over `reps` calls. The
    forward step runs in the form the tuner picks (tile < 0) or `tile`."""
    g = rd.Mesh(mesh)
    g.set_state(W0)
    if tile < 0:
        g.tune(cfl, rd.B, rd.RK2, rd.FP64, n_steps=3)
    else:
        g.tile = tile
    dt = g.max_dt(cfl)
    W = torch.from_numpy(W0).cuda()
    lam = torch.randn_like(W)
    out = torch.empty_like(W)
    for _ in range(2):
        g.step(dt, rd.B, rd.RK2, rd.FP64)
        rd.rd_adjoint_step(g.h, W, dt, rd.B, rd.RK2, lam, out)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        g.step(dt, rd.B, rd.RK2, rd.FP64)
    e[1].record()
    for _ in range(reps):
        rd.rd_adjoint_step(g.h, W, dt, rd.B, rd.RK2, lam, out)
    e[2].record()
    torch.cuda.synchronize()
    fwd = e[0].elapsed_time(e[1]) / reps
    adj = e[1].elapsed_time(e[2]) / reps
    out = {"ratio": round(adj / fwd, 3), "forward_ms": round(fwd, 4), "adjoint_ms": round(adj, 4),
           "triangles": mesh["nt"], "forward_tile": g.tile}
    g.close()
    return out


def batch_vs_single(rd, torch, inputs, n_meshes, steps, cfl, tile, seed=0):
    """Four-quadrant problems of uneven size (side N ~ U{32..512}; rho, p ~
    U[0.1, 2], |u| <= 1 per quadrant): per-mesh rd_step_cfl launches vs one
    rd_batch_run graph, FP64, B / RK2, the same tile size for both (the batch
    autotuner's choice, timed on 20-step graphs, when tile < 0). Equal
    accuracy: every member's final state is bitwise the one its own run
    gives. The B scheme is not positivity preserving and some members of
    this draw go non-physical; they are listed (each member has its own
    latch), and both forms must agree on which."""
    import numpy as np
    meshes, states = inputs.batch_problem(seed=seed, n=n_meshes)
    nt = sum(m["nt"] for m in meshes)
    gm = [rd.Mesh(m) for m in meshes]
    b = rd.Batch(gm)
    tuned = None
    if tile < 0:
        for g, W in zip(gm, states):
            g.set_state(W)
        tile, table = b.tune(cfl, rd.B, rd.RK2, rd.FP64, n_steps=20)
        tuned = {str(k): round(v, 5) for k, v in table.items()}
    else:
        b.set_tile(tile)
    for g in gm:
        g.tile = tile
    for g, W in zip(gm, states):
        g.set_state(W)
        g.step_cfl(1, cfl, rd.B, rd.RK2, rd.FP64)   # warm-up
    torch.cuda.synchronize()
    for g, W in zip(gm, states):
        g.set_state(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in gm:
        g.step_cfl(steps, cfl, rd.B, rd.RK2, rd.FP64)
    torch.cuda.synchronize()
    single = time.perf_counter() - t0

    def finish():
        # final states (bit patterns, so NaNs compare too) and the members
        # whose latch is set; the copy is made even when the latch is set
        out, bad = [], []
        for k, g in enumerate(gm):
            st = np.zeros((4, g.nv))
            try:
                g.get_state(st)
            except rd.RDError as e:
                if e.status != rd.RD_ENONPHYS:
                    raise
                bad.append(k)
            out.append(st.view(np.uint64))
        return out, bad

    ref, bad_single = finish()
    for g, W in zip(gm, states):
        g.set_state(W)
    b.run(steps, cfl, rd.B, rd.RK2, rd.FP64)       # captures the graph
    for g, W in zip(gm, states):
        g.set_state(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps, cfl, rd.B, rd.RK2, rd.FP64)
    torch.cuda.synchronize()
    batched = time.perf_counter() - t0
    got, bad_batch = finish()
    equal = all(np.array_equal(a, r) for a, r in zip(got, ref))
    b.close()
    for g in gm:
        g.close()
    return {"meshes": n_meshes, "triangles": nt, "steps": steps,
            "draw": "rho, p ~ U[0.1, 2], |u| <= 1 per quadrant, side N ~ U{32..512}, seed %d" % seed,
            "per_instance_s": round(single, 4), "batched_graph_s": round(batched, 4),
            "speedup": round(single / batched, 3), "bitwise_equal": bool(equal),
            "nonphysical_members": bad_batch, "nonphysical_agree": bad_batch == bad_single,
            "batched_value": round(nt * steps / batched, 1), "tile": tile, "tuner_ms_per_step": tuned}


def _err(a, b):
    import numpy as np
    return float(max(np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-300) for k in range(4)))


def fp32_table(rd, inputs):
    """Error of the FP32-distribution / FP64-accumulation variant per
    workload: one step from the initial state against the FP64 oracle, and the
    end state of a run against the same run in FP64 on the GPU (which matches
    the oracle step by step). Kelvin-Helmholtz and Sod with the B scheme on
    these meshes amplify any perturbation exponentially (the oracle itself
    does: a 1e-15 relative input change grows to 1e-3 within ~150 steps on a
    129^2 Sod mesh), so their end-state differences measure that
    amplification more than the variant's rounding."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle

    def run(mesh, W0, n, cfl, scheme, time_, prec, t_end=None):
        g = rd.Mesh(mesh)
        g.set_state(W0)
        if t_end is None:
            g.step_cfl(n, cfl, scheme, time_, prec)
        else:
            t = 0.0
            while t < t_end * (1 - 1e-14):
                dt = min(g.max_dt(cfl), t_end - t)
                g.step(dt, scheme, time_, prec)
                t += dt
        out = g.get_state()
        g.close()
        return out

    rows = []
    cases = [
        ("advected sine 64^2, N / Euler, 100 steps", inputs.split_square(64), inputs.ic_advected_sine,
         rd.N, rd.EULER1, 0.5, 100, None),
        ("Sod 1024^2, B / RK2, to t = 0.2", inputs.split_square(1024, periodic=(False, False), bc=("ghost", "wall")),
         inputs.ic_sod, rd.B, rd.RK2, 0.4, None, 0.2),
        ("Kelvin-Helmholtz 2048^2, B / RK2, 500 steps", inputs.split_square(2048),
         lambda m: inputs.ic_kelvin_helmholtz(m, seed=0), rd.B, rd.RK2, 0.4, 500, None),
        ("four-quadrant 512^2, B / RK2, 200 steps", inputs.split_square(512, periodic=(False, False)),
         lambda m: inputs.ic_quadrants(m, inputs.quadrant_states(0, **inputs.NARROW_QUADRANTS)), rd.B, rd.RK2, 0.4, 200, None),
        ("Fourier density 256^2, B / RK2, 200 steps", inputs.split_square(256),
         lambda m: inputs.ic_fourier_density(m, seed=0), rd.B, rd.RK2, 0.4, 200, None),
    ]
    for name, mesh, icf, scheme, time_, cfl, n, t_end in cases:
        print(f"bench: fp32 table: {name}", file=sys.stderr, flush=True)
        W0 = icf(mesh)
        om = oracle.OracleMesh(mesh)
        dt = om.max_dt(W0, cfl)
        ref1 = om.step(W0, dt, scheme, time_)
        one = {}
        for prec in (rd.FP64, rd.FP32_ACC64):
            g = rd.Mesh(mesh)
            g.set_state(W0)
            g.step(dt, scheme, time_, prec)
            one[prec] = _err(g.get_state(), ref1)
            g.close()
        e64 = run(mesh, W0, n, cfl, scheme, time_, rd.FP64, t_end)
        e32 = run(mesh, W0, n, cfl, scheme, time_, rd.FP32_ACC64, t_end)
        rows.append({"workload": name, "one_step_fp64_vs_oracle": one[rd.FP64],
                     "one_step_fp32_vs_oracle": one[rd.FP32_ACC64], "end_fp32_vs_fp64": _err(e32, e64)})
    return rows


def cpu_baseline(mesh, W0, cfl):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    om = oracle.OracleMesh(mesh)
    dt = om.max_dt(W0, cfl)
    t0 = time.perf_counter()
    om.step(W0, dt, oracle.B, oracle.RK2)
    el = time.perf_counter() - t0
    out = {"value": round(mesh["nt"] / el, 1), "unit": "triangle-updates/s", "cores": oracle.max_threads(),
           "kind": "oracle", "seconds": round(el, 2), "us_per_triangle_step": round(el * 1e6 / mesh["nt"], 4),
           "sample": f"one FP64 RK2/B step of the same {mesh['N']}x{mesh['N']} mesh ({mesh['nt']} triangles)"}
    # one host thread, on a 512x512 mesh of the same workload (about a second of work)
    from paper_1705_02028_amd import inputs
    small = inputs.split_square(512)
    Ws = inputs.ic_kelvin_helmholtz(small, seed=0)
    os1 = oracle.OracleMesh(small)
    dts = os1.max_dt(Ws, cfl)
    threads = oracle.max_threads()
    oracle.set_threads(1)
    t0 = time.perf_counter()
    os1.step(Ws, dts, oracle.B, oracle.RK2)
    el1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    out["single_thread"] = {"value": round(small["nt"] / el1, 1), "unit": "triangle-updates/s", "cores": 1,
                            "us_per_triangle_step": round(el1 * 1e6 / small["nt"], 4),
                            "sample": f"one FP64 RK2/B step of the 512x512 mesh ({small['nt']} triangles)"}
    return out


def meshgen(rd, inputs, reps=3):
    """Delaunay refinement to a uniform periodic mesh of about 1.3 million
    vertices (the size of the paper's mesh-generation test) from a jittered
    32x32 lattice: circumradius bound 7.3e-4, quality bound sqrt 2; whole
    calls timed on the host (neighbour table, upload, GPU iterations,
    download), with and without Morton renumbering."""
    import numpy as np
    m0 = inputs.split_square(32, periodic=(True, True), jitter=0.3, seed=10)
    m0["x"], m0["y"] = np.mod(m0["x"], 1.0), np.mod(m0["y"], 1.0)
    rd.rd_delaunay_refine(m0, 0.05, 2 ** 0.5)  # first call: module load, allocator
    out = {}
    for morton in (False, True):
        best, m1 = None, None
        for _ in range(reps):
            t0 = time.perf_counter()
            m1 = rd.rd_delaunay_refine(m0, 7.3e-4, 2 ** 0.5, max_vertices=1600000, morton=morton)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        out["morton" if morton else "insertion_order"] = {
            "seconds": round(best, 4), "vertices": m1["nv"], "triangles": m1["nt"],
            "iterations": m1["n_iterations"], "flips": m1["n_flips"],
            "vertices_per_s": round(m1["nv"] / best, 1)}
    return out


def three_d(rd, inputs, N=128, steps=10, warmup=2):
    """The three-dimensional path (F4): Kelvin-Helmholtz shear layer in a
    periodic box of N^3 cells split into 6 N^3 tetrahedra (Morton order),
    B scheme, RK2, CFL 0.4 with dt on the device; FP64. Whole-step
    throughput from the host clock around `steps` steps (inputs resident),
    per-kernel times from HIP events; the oracle's single-step rate on a
    16^3 box beside it."""
    m = inputs.cube_tets(N, renumber="morton")
    W = inputs.ic3_kelvin_helmholtz(m, seed=0)
    g = rd.Mesh3(m)
    g.set_state(W)
    g.step_cfl(warmup, 0.4, rd.B, rd.RK2)
    g.sync()
    t0 = time.perf_counter()
    g.step_cfl(steps, 0.4, rd.B, rd.RK2)
    g.sync()
    el = time.perf_counter() - t0
    ms = g.step_timed(3, 0.4, rd.B, rd.RK2)
    g.close()
    nt, nv = m["nt"], m["nv"]
    names = ["cfl", "tet1", "gather1", "tet2", "gather2"]
    # algorithmic bytes per tetrahedron pass. First: corners and slots (32),
    # normals (96), the parts (160), the kept N parts of three corners and the
    # residual (160) per tetrahedron, Z once per vertex (40). Second: the same
    # with the kept values read instead of written (160), the volume (8), and
    # the first-stage rate besides Z per vertex (80).
    b_tet1 = nt * (32 + 96 + 160 + 160) + nv * 40
    b_tet2 = nt * (32 + 96 + 8 + 160 + 160) + nv * 80
    dom = 1 if ms[1] >= ms[3] else 3
    b_dom = b_tet1 if dom == 1 else b_tet2
    ach = b_dom / (ms[dom] * 1e-3)
    out = {"value": round(nt * steps / el, 1), "unit": "tetrahedron-updates/s", "ms_per_step": round(el * 1e3 / steps, 4),
           "workload": f"Kelvin-Helmholtz shear layer, {N}^3-cell periodic box, {nt} tetrahedra, {nv} vertices, "
                       "B scheme, RK2, CFL 0.4 (dt on device), FP64",
           "kernels_ms": {k: round(v, 4) for k, v in zip(names, ms)},
           "roofline": {"kernel": names[dom], "bound": "hbm", "achieved": round(ach / 1e9, 1),
                        "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": round(ach / PEAK_HBM, 4),
                        "bytes_per_launch": b_dom}}
    try:
        sys.path.insert(0, os.path.join(ROOT, "oracle"))
        import oracle3
        small = inputs.cube_tets(16, renumber="morton")
        Ws = inputs.ic3_kelvin_helmholtz(small, seed=0)
        om = oracle3.OracleMesh3(small)
        dts = om.max_dt(Ws, 0.4)
        t0 = time.perf_counter()
        om.step(Ws, dts, oracle3.B, oracle3.RK2)
        el1 = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(small["nt"] / el1, 1), "unit": "tetrahedron-updates/s",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"one FP64 RK2/B step of the 16^3 box ({small['nt']} tetrahedra)"}
    except Exception as e:  # the oracle is test infrastructure; report its absence
        out["cpu_baseline"] = {"error": str(e)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=2048)
    ap.add_argument("--cfl", type=float, default=0.4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--timed-reps", type=int, default=5)
    ap.add_argument("--renumber", choices=["none", "random", "morton"], default="none",
                    help="vertex and triangle numbering of the mesh (default: the lattice order)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="triangles per tile of the fused step (0: two-pass form; -1: run the autotuner)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batch", type=int, default=256, metavar="NMESH",
                    help="time NMESH four-quadrant meshes (32^2..512^2) per instance vs one batched graph (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the Bx blend and selective lumping")
    ap.add_argument("--fp32-table", action="store_true",
                    help="only print the FP32-variant error table per workload (JSON)")
    ap.add_argument("--meshgen", action="store_true",
                    help="only time the GPU Delaunay refinement of a 1.3M-vertex periodic mesh (JSON)")
    ap.add_argument("--no-meshgen", action="store_true", help="skip the mesh-generation timing")
    ap.add_argument("--three-d", action="store_true",
                    help="only time the three-dimensional path (128^3-cell box of tetrahedra, JSON)")
    ap.add_argument("--no-three-d", action="store_true", help="skip the three-dimensional timing")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise kernel of known traffic (2 GiB read, 2 GiB written) for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1705_02028_amd import inputs, rd

    torch.cuda.set_device(0)
    rd.lib()
    if args.calibrate_copy:
        # counter calibration: one elementwise kernel that reads 2 GiB and
        # writes 2 GiB, run after 1 GiB of other writes has replaced the
        # source in the 256 MB Infinity Cache
        src = torch.ones(256 * 2 ** 20, dtype=torch.float64, device="cuda")
        flush = torch.ones(128 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst, flush
    if args.fp32_table:
        print(json.dumps({"fp32_errors": fp32_table(rd, inputs)}), flush=True)
        return
    if args.meshgen:
        print(json.dumps({"mesh_generation": meshgen(rd, inputs)}), flush=True)
        return
    if args.three_d:
        print(json.dumps({"three_d": three_d(rd, inputs)}), flush=True)
        return
    mesh = inputs.split_square(args.N, renumber=None if args.renumber == "none" else args.renumber, seed=0)
    W0 = inputs.ic_kelvin_helmholtz(mesh, seed=0)
    nt, nv = mesh["nt"], mesh["nv"]

    print(f"bench: mesh {args.N}^2, {nt} triangles; fp32-acc64 {args.steps} steps", file=sys.stderr, flush=True)
    ms32, per32, form32 = time_variant(rd, torch, mesh, W0, rd.FP32_ACC64, args.steps, args.warmup, args.cfl,
                                       args.timed_reps, args.tile)
    value = nt * args.steps / (ms32 * 1e-3)
    b32 = (algorithmic_bytes_tiled(nt, nv, True, form32["tile_info"]) if form32["tile"]
           else algorithmic_bytes(nt, nv, True))
    dom32 = max(per32, key=per32.get)
    result = {
        "metric": "triangle-updates/sec (FP64 & FP32) at 2048^2 mesh; adjoint/forward time ratio",
        "value": round(value, 1),
        "unit": "triangle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (triangle algebra) + f64 (vertex sums, state)",
        "data": "synthetic",
        "config": {"workload": f"Kelvin-Helmholtz shear layer, {args.N}x{args.N} periodic split-square mesh, "
                               f"B scheme, RK2, CFL {args.cfl} (dt on device each step), "
                               "FP32 distribution + FP64 accumulation",
                   "triangles": nt, "vertices": nv, "seed": 0, "numbering": args.renumber},
        "roofline": roofline_entry(dom32, method_bytes(nt, True)[dom32], b32[dom32], per32[dom32],
                                   f"fp32/{form_name(form32['tile'])}/{dom32}"
                                   if args.renumber == "none" and args.N == 2048 else None),
        "step_roofline": step_roofline(nt, True, ms32 / args.steps),
        "vertex_updates_per_s": round(nv * args.steps / (ms32 * 1e-3), 1),
        "stages": stage_rates(per32, nt),
        "kernels_ms": {k: round(v, 5) for k, v in per32.items()},
        "kernels_GBps": {k: round(b32[k] / (v * 1e-3) / 1e9, 1) for k, v in per32.items()
                         if v > 0 and b32.get(k)},
        "form": form32,
    }
    if not args.no_fp64:
        print(f"bench: fp64 {args.steps} steps", file=sys.stderr, flush=True)
        ms64, per64, form64 = time_variant(rd, torch, mesh, W0, rd.FP64, args.steps, args.warmup, args.cfl,
                                           args.timed_reps, args.tile)
        b64 = (algorithmic_bytes_tiled(nt, nv, False, form64["tile_info"]) if form64["tile"]
               else algorithmic_bytes(nt, nv, False))
        dom64 = max(per64, key=per64.get)
        result["fp64"] = {"value": round(nt * args.steps / (ms64 * 1e-3), 1), "unit": "triangle-updates/s",
                          "ms_per_step": round(ms64 / args.steps, 5),
                          "vertex_updates_per_s": round(nv * args.steps / (ms64 * 1e-3), 1),
                          "stages": stage_rates(per64, nt),
                          "roofline": roofline_entry(dom64, method_bytes(nt, False)[dom64], b64[dom64], per64[dom64],
                                                     f"fp64/{form_name(form64['tile'])}/{dom64}"
                                                     if args.renumber == "none" and args.N == 2048 else None),
                          "step_roofline": step_roofline(nt, False, ms64 / args.steps),
                          "kernels_ms": {k: round(v, 5) for k, v in per64.items()},
                          "kernels_GBps": {k: round(b64[k] / (v * 1e-3) / 1e9, 1)
                                           for k, v in per64.items() if v > 0 and b64.get(k)},
                          "form": form64}
        if form64["tile"]:
            # the two-pass form beside the tuner's tiled pick: its triangle passes are the FP64
            # kernels with a per-triangle roofline of their own
            ms2, per2, _ = time_variant(rd, torch, mesh, W0, rd.FP64, args.steps, args.warmup, args.cfl,
                                        args.timed_reps, 0)
            b2 = algorithmic_bytes(nt, nv, False)
            dom2 = max(per2, key=per2.get)
            result["fp64"]["two_pass"] = {
                "ms_per_step": round(ms2 / args.steps, 5),
                "value": round(nt * args.steps / (ms2 * 1e-3), 1),
                "roofline": roofline_entry(dom2, method_bytes(nt, False)[dom2], b2[dom2], per2[dom2],
                                           f"fp64/two-pass/{dom2}"
                                           if args.renumber == "none" and args.N == 2048 else None),
                "kernels_ms": {k: round(v, 5) for k, v in per2.items()},
                "kernels_GBps": {k: round(b2[k] / (v * 1e-3) / 1e9, 1) for k, v in per2.items()
                                 if v > 0 and b2.get(k)}}
    if not args.no_variants:
        # the other blends and lumpings of Sections 3.3.3 and 3.4 on the same workload (two-pass form)
        print("bench: scheme variants", file=sys.stderr, flush=True)
        variants = {}
        for name, scheme, lump in (("Bx", rd.BX, 0), ("B, selective lumping", rd.B, 1)):
            entry = {}
            for pname, prec in (("fp32", rd.FP32_ACC64), ("fp64", rd.FP64)):
                ms, per, _ = time_variant(rd, torch, mesh, W0, prec, args.steps, args.warmup, args.cfl,
                                          args.timed_reps, 0, scheme=scheme, lump=lump)
                entry[pname] = {"ms_per_step": round(ms / args.steps, 5),
                                "triangle_updates_per_s": round(nt * args.steps / (ms * 1e-3), 1),
                                "kernels_ms": {k: round(v, 5) for k, v in per.items()}}
            variants[name] = entry
        result["variants"] = variants
    if not args.no_adjoint:
        print("bench: adjoint / forward", file=sys.stderr, flush=True)
        result["adjoint_forward_ratio"] = adjoint_ratio(rd, torch, mesh, W0, args.cfl, 10, args.tile)
        m256 = inputs.split_square(256)
        result["adjoint_forward_ratio_256"] = adjoint_ratio(rd, torch, m256, inputs.ic_fourier_density(m256, seed=0),
                                                            args.cfl, 20, args.tile)
    if not args.no_meshgen:
        print("bench: mesh generation", file=sys.stderr, flush=True)
        result["mesh_generation"] = meshgen(rd, inputs, reps=2)
    if not args.no_three_d:
        print("bench: three dimensions", file=sys.stderr, flush=True)
        result["three_d"] = three_d(rd, inputs)
    if args.batch:
        print(f"bench: batch of {args.batch} meshes", file=sys.stderr, flush=True)
        result["batch"] = batch_vs_single(rd, torch, inputs, args.batch, args.batch_steps, args.cfl, args.tile)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(mesh, W0, args.cfl)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
