"""Benchmark of the particle time step on one MI355X.

Workload: FP64 periodic channel, 400 x 500 quads -> 400 000 triangles, 200 particles per
element (8e7 particles), dt = 2e-4; one timed step = pdf_step (advance, track, group,
bin, mix, statistics) + pdf_control(150, 250) (number control), inputs resident in HBM.
Prints one JSON line with whole-job throughput, the roofline of the dominant kernel
(timed with HIP events on the ensemble's stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# algorithmic HBM bytes per live particle (FP64 state): what each kernel must read and
# write once
BYTES_PER_PARTICLE = {
    # read x, y, U(3), omega, pid, elem; write x, y, U(3), omega, elem
    "advance": 6 * 8 + 8 + 4 + 6 * 8 + 4,
    # read idx, U(3), pid, x, y, omega, psi, w; write the 10 state arrays in canonical order
    "element_pass": 4 + 4 * 8 + 5 * 8 + (8 * 8 + 8 + 4),
    # read elem, write idx
    "scatter": 4 + 4,
}


KERNEL_NAMES = {"advance": "k_advance", "element_pass": "k_element_wave", "scatter": "k_scatter"}
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_channel_large.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1006_0532_amd", "csrc", "kernels.hip")


def counter_traffic(kernel, default_workload):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) from the committed rocprofv3
    counter summary of this workload, or None if the kernels changed since it was taken."""
    if not default_workload or not os.path.exists(COUNTERS):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    text = open(COUNTERS).read().splitlines()
    if f"kernels.hip sha256 prefix: {sha}" not in text:
        return None
    for line in text:
        f = line.split()
        if len(f) == 3 and f[0] == "traffic_bytes_per_launch" and f[1] == KERNEL_NAMES.get(kernel):
            return float(f[2])
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--nx", type=int, default=400)
    p.add_argument("--ny", type=int, default=500)
    p.add_argument("--ppe", type=int, default=200)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-calib", action="store_true",
                   help="run one 1 GiB device copy first (known-size kernel for HBM counter scaling)")
    return p.parse_args()


def cpu_baseline(args, dt, ctl):
    """The oracle on a reduced instance of the same generator (same grading, ppe, dt,
    control), timed for about cpu_seconds of host work."""
    import oracle as O
    from paper_1006_0532_amd import workloads as W
    nx, ny = 100, 126
    mesh = W.channel_mesh(nx, ny)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=args.ppe, bins=(4, 2, 2))
    g = O.Grid(mesh, f, mo)
    e = O.Ensemble(g, ini)
    done, t0 = 0, time.perf_counter()
    psteps = 0
    while True:
        n = e.count()
        e.step(dt)
        e.control(*ctl)
        psteps += n
        done += 1
        el = time.perf_counter() - t0
        if done >= 2 and el >= args.cpu_seconds:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": psteps / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"channel generator at {nx}x{ny} quads ({2 * nx * ny} triangles), "
                      f"{args.ppe} particles/element, {done} steps of dt={dt} with control "
                      f"{list(ctl)}, {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1006_0532_amd import pdfgpu, workloads as W

    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        s = a.sum()          # reads 1 GiB: fetch-side reference
        torch.cuda.synchronize()
        del a, b, s
    dt, ctl = 2.0e-4, (150, 250)
    t_setup = time.perf_counter()
    mesh = W.channel_mesh(args.nx, args.ny)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=args.ppe, bins=(4, 2, 2))
    n0 = mesh.n_elems * args.ppe
    grid = pdfgpu.Grid(mesh, f, mo)
    ens = pdfgpu.Ensemble(grid, ini, capacity=int(1.3 * n0) + 1024)
    ens.sync()
    print(f"[bench] set-up {time.perf_counter() - t_setup:.1f} s: {mesh.n_elems} triangles, "
          f"{n0} particles", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        ens.step(dt)
        ens.control(*ctl)
    ens.sync()
    torch.cuda.synchronize()

    live = []
    ens.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        live.append(ens.count())
        ens.step(dt)
        ens.control(*ctl)
    ens.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = ens.timing(False)
    elapsed = t1 - t0
    psteps = float(sum(live))
    value = psteps / elapsed

    # dominant kernel and its roofline (bytes per launch = bytes per particle x live)
    kern = {k: v for k, v in tim.items() if v[1] > 0}
    dom = max(kern, key=lambda k: kern[k][0])
    mean_live = psteps / args.steps
    roof = None
    if dom in BYTES_PER_PARTICLE:
        avg_ms = kern[dom][0] / kern[dom][1]
        achieved = BYTES_PER_PARTICLE[dom] * mean_live / (avg_ms * 1e-3) / 1e9
        default = (args.nx, args.ny, args.ppe) == (400, 500, 200)
        traffic = counter_traffic(dom, default)
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 3),
                "traffic_unit": "GB per launch",
                "avg_ms": round(avg_ms, 4), "bytes_per_particle": BYTES_PER_PARTICLE[dom]}
    per_kernel = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches": v[1]} for k, v in kern.items()}
    for k, bpp in BYTES_PER_PARTICLE.items():
        if k in kern:
            avg = kern[k][0] / kern[k][1]
            per_kernel[k]["GB/s"] = round(bpp * mean_live / (avg * 1e-3) / 1e9, 1)
    print(f"[bench] per kernel: {json.dumps(per_kernel)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, dt, ctl)

    out = {
        "metric": "particle-steps/s", "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "channel_large", "triangles": mesh.n_elems, "nodes": mesh.n_nodes,
                   "particles": n0, "ppe": args.ppe, "dt": dt, "control": list(ctl),
                   "bins": [4, 2, 2], "precision": "fp64", "parallelism": "single GPU"},
        "roofline": roof, "per_kernel": per_kernel, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
