"""Benchmark of the D2Q25 RK-3 step on one MI355X.

Default workload (the metric's configuration): 2048 x 2048 periodic lattice,
FP64, superposed shear and longitudinal waves (wavelength 64 cells), vdW
a = 9/49, b = 2/21, T = 1, tau = 0.005, dt = 5e-4.  A step is one full RK-3
step (three fused stage-kernel launches).  Inputs are resident in HBM before
the timed region starts.

Prints one JSON line with MLUPS (cells x steps / s / 1e6), the roofline of
the stage kernel (its average launch time from HIP events on the library's
stream over the timed region) and the CPU oracle timed on a bounded sample of
the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_VEC_PEAK_TFLOPS = 78.6  # MI355X vector FP64, published (FMA = 2 flops)
FP32_VEC_PEAK_TFLOPS = 157.3

# Algorithmic HBM bytes per cell per RK-3 step: 25 populations x 8 accesses
# (stage 1: read f^n, write f1; stages 2, 3: read f_src and f^n, write).
ALG_VALUES_PER_CELL_STEP = 25 * 8
# Algorithmic FP64/FP32 flops per cell per stage of the stage kernel (counted
# from its arithmetic; an FMA counts 2).  See the design notes for the tally.
ALG_FLOPS_PER_CELL_STAGE = 4230


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("olb_kernels.hip", "olb_consts.hpp", "olb_device.hpp", "olb_feq.hpp"):
        with open(os.path.join(ROOT, "paper_1702_01690_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """Measured HBM bytes per stage launch from committed rocprofv3 counter
    runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    entry = t.get(workload)
    if not entry or entry.get("kernel_hash") != kernel_source_hash():
        return None
    return entry.get("bytes_per_launch")


WORKLOADS = {
    "wave2048": "2048x2048 periodic FP64, shear + longitudinal waves, vdW a=9/49 b=2/21, T=1, "
                "tau=0.005, dt=5e-4, ds=1/64",
    "spinodal4096": "4096x4096 periodic FP32-mixed spinodal decomposition at T=0.9 T_c, "
                    "n=3.5(1+-1% noise), tau=0.005, dt=2e-4, ds=1/320",
    "channels": "256 walled channels (nx 64..512, ny 128..1024, 43.6 M nodes), FP32-mixed, "
                "T_w in [0.7, 0.95] T_c, one launch per stage over all channels, graphs of 10 steps",
}


def make_cases(workload):
    import olb_inputs as I
    if workload == "wave2048":
        c = I.wave2048()
        c.params["precision"] = 0
        return [c]
    if workload == "spinodal4096":
        c = I.spinodal(4096, 4096)
        c.params["precision"] = 1
        c.params["rho_ref"] = I.N_CRIT
        return [c]
    if workload == "channels":
        return I.channels()
    raise SystemExit(f"unknown workload {workload}")


def cpu_baseline(workload, sample_steps):
    """The oracle, as it stands, on the 64 x 64 crop of the wave workload (the
    2048^2 field is this crop tiled, so the per-cell work is identical)."""
    import olb_inputs as I
    import oracle
    if workload == "wave2048":
        case = I.wave64()
    elif workload == "spinodal4096":
        case = I.spinodal(64, 64)
    else:
        case = I.channel(64, 128, tw=0.8 * I.T_CRIT)
    o = oracle.Oracle(case.params)
    o.set_fields(*case.fields)
    o.step(1)
    t0 = time.perf_counter()
    o.step(sample_steps)
    dt = time.perf_counter() - t0
    cells = case.params["nx"] * case.params["ny"]
    return {"value": cells * sample_steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"{case.params['nx']}x{case.params['ny']} lattice of the same physics (FP64 oracle), "
                      f"{sample_steps} RK3 steps, {dt:.1f} s"}


def copy_kernel(gib, reps=10):
    """Device-to-device copy of a known size: calibrates the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE per dispatch) and measures the copy
    bandwidth this machine sustains."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    moved = 2 * n * 8
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                      "copy_GBps": round(moved / secs / 1e9, 1), "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="wave2048", choices=sorted(WORKLOADS))
    ap.add_argument("--graph", type=int, default=10, help="RK3 steps per HIP graph (batches)")
    ap.add_argument("--autotune", action="store_true", help="pick the tile height by trial (batches)")
    ap.add_argument("--tile", type=int, default=8, choices=[8, 16])
    ap.add_argument("--cpu-steps", type=int, default=2000,
                    help="oracle steps of the CPU-baseline sample (about 10-20 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_gib > 0:
        copy_kernel(args.copy_gib)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; multi-GPU runs are not part of it "
              "(see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1702_01690_amd import olb

    cases = make_cases(args.workload)
    precision = cases[0].params["precision"]
    batched = args.workload == "channels"
    cells = sum(c.params["nx"] * c.params["ny"] for c in cases)
    print(f"[bench] {args.workload} instances={len(cases)} nodes={cells} precision={precision} "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    if batched:
        lat = olb.Batch([c.params for c in cases], device="cuda:0")
        if args.autotune:
            lat.autotune(trial_steps=2)
        else:
            lat.set_tile(args.tile)
        if args.graph:
            lat.use_graph(args.graph)
        for i, c in enumerate(cases):
            lat.set_fields(i, *c.fields)
        n_stage, n_walls = 3, 3
        tile_by = lat.tiles()[1]
    else:
        lat = olb.Lattice(cases[0].params, device="cuda:0")
        lat.set_tile(args.tile)
        lat.set_fields(*cases[0].fields)
        n_stage, n_walls = lat.launch_counts()
        tile_by = args.tile
    stream = lat.stream

    lat.step(args.warmup)
    lat.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    lat.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = ev0.elapsed_time(ev1)
    secs = ms_events / 1e3
    mlups = cells * args.steps / secs / 1e6
    launches = n_stage * args.steps
    # the region holds the stage launches (and, with walls, the small ghost launches)
    avg_launch_s = secs / launches
    rb = 8 if precision == 0 else 4
    bytes_per_launch = ALG_VALUES_PER_CELL_STEP * rb * cells / n_stage
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    flops_per_launch = ALG_FLOPS_PER_CELL_STAGE * cells
    achieved_tflops = flops_per_launch / avg_launch_s / 1e12
    vec_peak = FP64_VEC_PEAK_TFLOPS if precision == 0 else FP32_VEC_PEAK_TFLOPS
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    alu_frac = achieved_tflops / vec_peak
    traffic = load_traffic(args.workload)
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": vec_peak,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": traffic,
                "hbm": {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(hbm_frac, 4)}}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic,
                "alu": {"achieved": round(achieved_tflops, 3), "peak": vec_peak, "unit": "TFLOP/s",
                        "frac": round(alu_frac, 4)}}
    lat.close()

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload, args.cpu_steps)

    out = {
        "metric": "MLUPS per full RK3 step (D2Q25)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_events / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "nodes": cells, "instances": len(cases), "tile": f"63x{tile_by - 1}",
                   "wall_s": round(wall, 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
