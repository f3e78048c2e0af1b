"""Throughput of the residual-distribution step on one MI355X.

Workload: Kelvin-Helmholtz shear layer on a 2048x2048 periodic split-square
mesh (4,190,209 vertices, 8,380,418 triangles), B scheme, two-stage
Runge-Kutta, CFL 0.4 with the time step computed on the device every step.
The headline value is the FP32-distribution / FP64-accumulation variant (the
configuration's arithmetic); the FP64 variant is timed on the same mesh and
reported beside it. One step = CFL limit + both Runge-Kutta stages (two
triangle passes and two vertex gathers). Inputs are resident on the GPU
before timing starts.

Prints one JSON line. `--gpus N` with N > 1 exits: this build runs on one GPU.
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


def algorithmic_bytes(nt, nv, fp32):
    """Bytes each kernel of an RK2/B step with the CFL limit must move at
    least once, with every vertex record read once per pass (ideal reuse).
    q = bytes per real of the triangle algebra; a part or parameter vector is
    4 reals; parts live in vertex-CSR order (one record per corner)."""
    q = 4 if fp32 else 8
    r4 = 4 * q
    k = {}
    # stage 1: corner ids and CSR positions, coordinates, Z and |v|+c in;
    # parts, kept N parts, phi^T and l_max lambda_max per corner out
    k["tri1"] = nt * (12 + 12 + 3 * r4 + 3 * r4 + r4 + 24) + nv * (16 + r4 + 8)
    # CFL: CSR rows, V and the per-corner l_max lambda_max in, block minima out
    k["cfl_vertex"] = nv * (4 + 8) + nt * 24
    k["cfl_final"] = 0
    # gather 1: rows, parts in; W, V in; W*, W*-W, Z*, |v|+c out
    k["gather1"] = nt * 3 * r4 + nv * (4 + 32 + 8 + 32 + r4 + r4 + 8)
    # stage 2: ids, positions, coordinates, Z*, W*-W, kept N parts, phi^T in; parts out
    k["tri2"] = nt * (12 + 12 + 3 * r4 + r4 + 3 * r4) + nv * (16 + r4 + r4)
    # gather 2: rows, parts in; W*, V in; W, Z, |v|+c out
    k["gather2"] = nt * 3 * r4 + nv * (4 + 32 + 8 + 32 + r4 + 8)
    k["wall1"] = k["wall2"] = 0
    return k


def roofline_entry(name, bytes_, ms):
    achieved = bytes_ / (ms * 1e-3)
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved / 1e9, 1), "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM, 4), "traffic": None,
            "algorithmic_bytes": int(bytes_), "avg_ms": round(ms, 5)}


def time_variant(rd, torch, mesh, W0, prec, steps, warmup, cfl, timed_reps):
    g = rd.Mesh(mesh)
    g.set_state(W0)
    if warmup:
        g.step_cfl(warmup, cfl, rd.B, rd.RK2, prec)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step_cfl(steps, cfl, rd.B, rd.RK2, prec)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g.sync()
    per = {}
    for _ in range(max(timed_reps, 1)):
        t = rd.rd_step_timed(g.h, cfl, rd.B, rd.RK2, prec)
        for k, v in t.items():
            per[k] = per.get(k, 0.0) + v / max(timed_reps, 1)
    g.sync()
    g.close()
    return ms, per


def cpu_baseline(mesh, W0, cfl):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    om = oracle.OracleMesh(mesh)
    dt = om.max_dt(W0, cfl)
    t0 = time.perf_counter()
    om.step(W0, dt, oracle.B, oracle.RK2)
    el = time.perf_counter() - t0
    return {"value": round(mesh["nt"] / el, 1), "unit": "triangle-updates/s", "cores": oracle.max_threads(),
            "kind": "oracle", "seconds": round(el, 2),
            "sample": f"one FP64 RK2/B step of the same {mesh['N']}x{mesh['N']} mesh ({mesh['nt']} triangles)"}


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
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 512 MiB device-to-device copy (known bytes) for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1705_02028_amd import inputs, rd

    torch.cuda.set_device(0)
    rd.lib()
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    mesh = inputs.split_square(args.N)
    W0 = inputs.ic_kelvin_helmholtz(mesh, seed=0)
    nt, nv = mesh["nt"], mesh["nv"]

    print(f"bench: mesh {args.N}^2, {nt} triangles; fp32-acc64 {args.steps} steps", file=sys.stderr, flush=True)
    ms32, per32 = time_variant(rd, torch, mesh, W0, rd.FP32_ACC64, args.steps, args.warmup, args.cfl,
                               args.timed_reps)
    value = nt * args.steps / (ms32 * 1e-3)
    b32 = algorithmic_bytes(nt, nv, True)
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
                   "triangles": nt, "vertices": nv, "seed": 0},
        "roofline": roofline_entry(dom32, b32[dom32], per32[dom32]),
        "kernels_ms": {k: round(v, 5) for k, v in per32.items()},
        "kernels_GBps": {k: round(b32[k] / (v * 1e-3) / 1e9, 1) for k, v in per32.items() if v > 0 and b32[k]},
    }
    if not args.no_fp64:
        print(f"bench: fp64 {args.steps} steps", file=sys.stderr, flush=True)
        ms64, per64 = time_variant(rd, torch, mesh, W0, rd.FP64, args.steps, args.warmup, args.cfl,
                                   args.timed_reps)
        b64 = algorithmic_bytes(nt, nv, False)
        dom64 = max(per64, key=per64.get)
        result["fp64"] = {"value": round(nt * args.steps / (ms64 * 1e-3), 1), "unit": "triangle-updates/s",
                          "ms_per_step": round(ms64 / args.steps, 5),
                          "roofline": roofline_entry(dom64, b64[dom64], per64[dom64]),
                          "kernels_ms": {k: round(v, 5) for k, v in per64.items()},
                          "kernels_GBps": {k: round(b64[k] / (v * 1e-3) / 1e9, 1)
                                           for k, v in per64.items() if v > 0 and b64[k]}}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(mesh, W0, args.cfl)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
