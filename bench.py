"""Benchmark of the particle time step on one MI355X.

Workload: FP64 periodic channel, 400 x 500 quads -> 400 000 triangles, 200 particles per
element (8e7 particles), dt = 2e-4; one timed step = pdf_step (advance, track, group,
bin, mix, statistics) + pdf_control(150, 250) (number control), inputs resident in HBM.
Prints one JSON line with whole-job throughput, the roofline of the dominant kernel
(timed with HIP events on the ensemble's stream), the CPU oracle timed on a bounded
sample of the same workload, and the other forms: the same workload in mixed precision
(with its statistics against the FP64 form on the channel and on the 10^8-particle street
canyon, each field against its bound), 64 uneven independent problems advanced as one
batched ensemble against the same problems advanced one at a time, and the large street
canyon (4e6 triangles, about 4.8e8 particles) in mixed precision with per-kernel HBM rates.
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
# VALU issue of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
# (a wavefront instruction holds its SIMD for 4 cycles; FP64 arithmetic issues at this rate)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
FP64_PEAK_TFLOPS = 78.6

# algorithmic HBM bytes per live particle (FP64 state): what each kernel must read and
# write once
BYTES_PER_PARTICLE = {
    # read x, y, U(3), omega, pid, elem; write x, y, U(3), omega, elem and the arrival rank
    "advance": 6 * 8 + 8 + 4 + 6 * 8 + 4 + 4,
    # read idx, U(3), pid, x, y, omega, psi, w; write the 10 state arrays in canonical order
    "element_pass": 4 + 4 * 8 + 5 * 8 + (8 * 8 + 8 + 4),
    # placement in the grouped order: read elem and arrival rank, write idx
    "scatter": 4 + 4 + 4,
}


KERNEL_NAMES = {"advance": "k_advance", "element_pass": "k_element_wave", "scatter": "k_place"}
COUNTERS = os.path.join(ROOT, "profiles", "counters_channel_large.txt")
COUNTERS_HUGE = os.path.join(ROOT, "profiles", "counters_cavity_huge_mixed.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1006_0532_amd", "csrc", "kernels.hip")


def measured(kernel, name, default_workload, path=COUNTERS):
    """A figure measured by rocprofv3 counters on this workload (the committed summary's
    "measure <kernel> <name> <value>" lines), or None when the workload differs or the
    kernels changed since the counters were taken."""
    if not default_workload or not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    text = open(path).read().splitlines()
    if f"kernels.hip sha256 prefix: {sha}" not in text:
        return None
    for line in text:
        f = line.split()
        if len(f) == 4 and f[0] == "measure" and f[1] == KERNEL_NAMES.get(kernel, kernel) and f[2] == name:
            return float(f[3])
    return None


def counter_traffic(kernel, default_workload, path=COUNTERS):
    """HBM bytes per launch (32-, 64- and 128-byte read requests and 32- and 64-byte write
    requests of the L2 to memory, counted by rocprofv3) of this workload, or None."""
    rd = measured(kernel, "read_bytes_per_launch", default_workload, path)
    wr = measured(kernel, "write_bytes_per_launch", default_workload, path)
    return None if rd is None or wr is None else rd + wr


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    p.add_argument("--no-forms", action="store_true",
                   help="skip the mixed-precision and batched measurements")
    p.add_argument("--form-steps", type=int, default=10)
    p.add_argument("--large-mixed-only", action="store_true",
                   help="run only the large street canyon in the mixed form and print its figures")
    p.add_argument("--no-eulerian", action="store_true",
                   help="skip timing the elliptic-relaxation and pressure-projection solves")
    p.add_argument("--eulerian-only", action="store_true",
                   help="set up the channel, take the warm-up steps, then run only the Eulerian solves "
                        "and the closed loop and print their figures")
    p.add_argument("--batched-problems", type=int, default=64)
    p.add_argument("--batched-only", choices=("batched", "plain"), default=None,
                   help="run only the batched problems in FP64, as one ensemble or one ensemble at a time "
                        "(for per-kernel profiles of the two), and print their figures")
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
    one = cpu_baseline_one_thread(args, dt, ctl)
    return {"value": psteps / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"channel generator at {nx}x{ny} quads ({2 * nx * ny} triangles), "
                      f"{args.ppe} particles/element, {done} steps of dt={dt} with control "
                      f"{list(ctl)}, {el:.1f} s",
            "one_thread": one}


ONE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle as O
from paper_1006_0532_amd import workloads as W
nx, ny, ppe, dt, lo, hi, secs = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]), float(sys.argv[5]), \
    int(sys.argv[6]), int(sys.argv[7]), float(sys.argv[8])
m = W.channel_mesh(nx, ny)
e = O.Ensemble(O.Grid(m, W.channel_fields(m), W.model_constants()), W.init_desc(ppe=ppe, bins=(4, 2, 2)))
done, ps, t0 = 0, 0, time.perf_counter()
while True:
    n = e.count(); e.step(dt); e.control(lo, hi); ps += n; done += 1
    el = time.perf_counter() - t0
    if done >= 2 and el >= secs:
        break
print(json.dumps({"value": ps / el, "steps": done, "seconds": el}))
"""


def cpu_baseline_one_thread(args, dt, ctl):
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1) on a smaller
    sample of the same generator."""
    import subprocess
    nx, ny = 50, 62
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", ONE_THREAD, ROOT, str(nx), str(ny), str(args.ppe), str(dt),
                            str(ctl[0]), str(ctl[1]), str(max(2.0, args.cpu_seconds / 2))],
                           env=env, capture_output=True, text=True, timeout=300)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as ex:   # reported, not fatal: the baseline is context
        return {"error": str(ex)[:200]}
    return {"value": d["value"], "unit": "particle-steps/s", "cores": 1,
            "sample": f"channel generator at {nx}x{ny} quads ({2 * nx * ny} triangles), {args.ppe} "
                      f"particles/element, {d['steps']} steps with control {list(ctl)}, {d['seconds']:.1f} s"}


STAT_FIELDS = {"W": ([0], [1.0]), "U": ([1, 2, 3], [1.0] * 3), "omega": ([4], [1.0]), "psi": ([5], [1.0]),
               "R": ([6, 7, 8, 9, 10, 11], [1.0, 1.0, 1.0, 2.0, 2.0, 2.0]), "psi_var": ([12], [1.0])}


def field_errors(s, ref):
    """W-weighted relative L2 error ||s - ref||_{2,W} / ||ref||_{2,W} of every nodal field
    (mean velocity as a vector, Reynolds stresses as a tensor in the Frobenius norm)."""
    import numpy as np
    ok = ~np.isnan(ref).any(axis=1) & ~np.isnan(s).any(axis=1)
    W = ref[ok, 0]
    out = {}
    for name, (cols, wts) in STAT_FIELDS.items():
        d = sum(c * (s[ok, q] - ref[ok, q]) ** 2 for q, c in zip(cols, wts))
        r = sum(c * ref[ok, q] ** 2 for q, c in zip(cols, wts))
        num, den = float(np.sqrt(np.sum(W * d))), float(np.sqrt(np.sum(W * r)))
        out[name] = num / den if den > 0 else num
    return out


def timed_steps(ens, dt, steps, ctl=None):
    """Live particle-steps and wall time of `steps` steps (each followed by control when
    ctl is given), bracketed by device synchronisation."""
    import torch
    ens.sync()
    torch.cuda.synchronize()
    cur = ens.count()     # then from each control report; without control it is constant
    live, t0 = 0, time.perf_counter()
    if ctl:
        for _ in range(steps):
            live += cur
            ens.step(dt)
            cur = ens.control(*ctl)["live"]
    else:
        ens.step(dt, steps)
        live = cur * steps
    ens.sync()
    torch.cuda.synchronize()
    return live, time.perf_counter() - t0


def mixed_form(args, mesh, f, mo, ini, dt, ctl):
    """The same workload (step + control) in the mixed form."""
    from paper_1006_0532_amd import pdfgpu
    n0 = mesh.n_elems * args.ppe
    grid = pdfgpu.Grid(mesh, f, mo)
    ens = pdfgpu.Ensemble(grid, ini, capacity=int(1.3 * n0) + 1024, precision=pdfgpu.PDF_MIXED)
    for _ in range(args.warmup):
        ens.step(dt)
        ens.control(*ctl)
    ens.timing(True)
    live, el = timed_steps(ens, dt, args.form_steps, ctl)
    tim = ens.timing(False)
    out = {"value": live / el, "ms_per_step": 1e3 * el / args.form_steps, "steps": args.form_steps,
           "per_kernel_ms": {k: round(v[0] / v[1], 4) for k, v in tim.items() if v[1] > 0}}
    ens.close()
    grid.close()
    return out


# algorithmic bytes per particle of the mixed form (U, omega, psi, w in FP32)
MIXED_BYTES_PER_PARTICLE = {
    # read x, y (16), U, omega (16), pid 8, elem 4; write x, y, U, omega, elem, arrival rank
    "advance": 16 + 16 + 8 + 4 + 16 + 16 + 4 + 4,
    # read idx 4, U 12, pid 8, x, y 16, omega, psi, w 12; write the state (52)
    "element_pass": 4 + 12 + 8 + 16 + 12 + 52,
    "scatter": 4 + 4 + 4,
}


def large_mixed_form(args):
    """The large street canyon (4e6 triangles, 120 particles per element, about 4.8e8
    particles) in the mixed form with number control [90, 150]: throughput and per-kernel
    algorithmic HBM rates."""
    from paper_1006_0532_amd import pdfgpu, workloads as W
    mesh, f, mo, ini = W.cavity_huge()
    wl = W.WORKLOADS["cavity_huge"]
    dt, ctl = wl["dt"], wl["control"]
    n0 = mesh.n_elems * ini["ppe"]
    grid = pdfgpu.Grid(mesh, f, mo)
    ens = pdfgpu.Ensemble(grid, ini, capacity=int(1.3 * n0) + 1024, precision=pdfgpu.PDF_MIXED)
    for _ in range(2):
        ens.step(dt)
        ens.control(*ctl)
    ens.timing(True)
    live, el = timed_steps(ens, dt, args.form_steps, ctl)
    tim = ens.timing(False)
    mean_live = live / args.form_steps
    per = {}
    for k, v in tim.items():
        if v[1] == 0:
            continue
        avg = v[0] / v[1]
        per[k] = {"ms": round(avg, 4)}
        if k in MIXED_BYTES_PER_PARTICLE:
            gbs = MIXED_BYTES_PER_PARTICLE[k] * mean_live / (avg * 1e-3) / 1e9
            per[k].update({"GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
            tr = counter_traffic(k, True, COUNTERS_HUGE)
            if tr is not None:   # the counters' launch time, not this run's
                ms = measured(k, "avg_ms", True, COUNTERS_HUGE)
                per[k].update({"counter_GB_per_launch": round(tr / 1e9, 3),
                               "counter_bytes_per_particle": round(tr / mean_live, 1)})
                if ms:
                    per[k]["counter_GBs"] = round(tr / (ms * 1e-3) / 1e9, 1)
    out = {"workload": "cavity_huge", "triangles": mesh.n_elems, "particles": n0, "ppe": ini["ppe"],
           "bins": list(ini["bins"]), "control": list(ctl), "dt": dt, "steps": args.form_steps,
           "value": live / el, "ms_per_step": 1e3 * el / args.form_steps, "per_kernel": per}
    ens.close()
    grid.close()
    return out


def mixed_error(mesh, f, mo, ini, dt, steps):
    """Nodal statistics of the mixed form against the FP64 form on the full workload after
    `steps` steps without number control (control decisions on counts that differ by one
    edge-crossing particle would start different random streams): W-weighted relative L2
    per field."""
    from paper_1006_0532_amd import pdfgpu
    grid = pdfgpu.Grid(mesh, f, mo)
    st = {}
    for prec in (pdfgpu.PDF_FP64, pdfgpu.PDF_MIXED):
        ens = pdfgpu.Ensemble(grid, ini, precision=prec)
        ens.step(dt, steps)
        st[prec] = ens.stats()
        ens.close()
    grid.close()
    err = field_errors(st[pdfgpu.PDF_MIXED], st[pdfgpu.PDF_FP64])
    err["steps"] = steps
    return err


# the mixed form's bounds on each field's W-weighted relative L2 against the FP64 form:
# 1e-5 on the means of W, U and omega, 1e-4 on the scalar mean and the second moments
MIXED_BOUNDS = {"W": 1e-5, "U": 1e-5, "omega": 1e-5, "psi": 1e-4, "R": 1e-4, "psi_var": 1e-4}


def with_bounds(err):
    """Attach the mixed form's bounds to field errors and list the fields that exceed them."""
    err["bounds"] = dict(MIXED_BOUNDS)
    err["misses"] = sorted(k for k, b in MIXED_BOUNDS.items() if err[k] > b)
    return err


def mixed_error_cavity_large(steps=10):
    """The street canyon at 10^6 triangles x 100 particles (10^8), dt 1e-4: FP64 and mixed
    ensembles from the same streams, `steps` steps without control, the mixed statistics
    against the FP64 ones with the bounds they are held to (the test of the same case marks
    its miss on <omega> as expected)."""
    from paper_1006_0532_amd import pdfgpu, workloads as W
    mesh, f, mo, ini = W.cavity_large()
    dt = W.WORKLOADS["cavity_large"]["dt"]
    cap = int(1.3 * mesh.n_elems * ini["ppe"]) + 1024
    grid = pdfgpu.Grid(mesh, f, mo)
    st = {}
    for prec in (pdfgpu.PDF_FP64, pdfgpu.PDF_MIXED):
        ens = pdfgpu.Ensemble(grid, ini, capacity=cap, precision=prec)
        ens.step(dt, steps)
        st[prec] = ens.stats()
        ens.close()
    grid.close()
    err = with_bounds(field_errors(st[pdfgpu.PDF_MIXED], st[pdfgpu.PDF_FP64]))
    err.update(workload="cavity_large", steps=steps, dt=dt)
    return err


def batched_form(args, legs=("fp64", "mixed", "plain")):
    """64 independent channel / street-canyon problems of uneven size (triangles
    log-uniform in [1e3, 2e5], 20-400 particles per element): advanced together (one
    launch per kernel, the particle loop's wavefronts across the ends of two problems in a
    second small launch; graph-replayed steps, autotuned launch options) in FP64 and in the
    mixed form, against the same problems advanced one ensemble at a time (FP64)."""
    from paper_1006_0532_amd import pdfgpu, workloads as W
    probs = W.batched_problems(args.batched_problems)
    dts = [p[4] for p in probs]
    grids = [pdfgpu.Grid(m, f, mo) for m, f, mo, ini, dt in probs]
    inits = [ini for m, f, mo, ini, dt in probs]
    caps = [int(1.05 * m.n_elems * ini["ppe"]) + 1024 for m, f, mo, ini, dt in probs]
    n_total = sum(m.n_elems * ini["ppe"] for m, f, mo, ini, dt in probs)
    out = {"problems": len(probs), "triangles": int(sum(m.n_elems for m, *_ in probs)), "particles": int(n_total),
           "steps": args.form_steps}
    for name, prec in (("fp64", pdfgpu.PDF_FP64), ("mixed", pdfgpu.PDF_MIXED)):
        if name not in legs:
            continue
        ens = pdfgpu.Ensemble(grids, inits, capacity=caps, precision=prec)
        ens.set_options(use_graph=1)
        chosen, trials = ens.autotune(dts, steps_per_trial=2)
        live, el = timed_steps(ens, dts, args.form_steps)
        out[name] = {"value": live / el, "ms_per_step": 1e3 * el / args.form_steps, "options": chosen,
                     "autotune_trial_ms": [round(t, 3) for t in trials]}
        ens.close()
    if "plain" not in legs:
        for g in grids:
            g.close()
        return out
    # the same FP64 problems one ensemble at a time (seed ^ p << 32 gives the same streams)
    live_tot, el_tot = 0, 0.0
    for p, (g, ini, dt, cap) in enumerate(zip(grids, inits, dts, caps)):
        d = dict(ini)
        d["seed"] = int(ini["seed"]) ^ (p << 32)
        e = pdfgpu.Ensemble(g, d, capacity=cap)
        e.step(dt)
        live, el = timed_steps(e, dt, args.form_steps)
        live_tot += live
        el_tot += el
        e.close()
    out["plain_fp64_one_at_a_time"] = {"value": live_tot / el_tot, "ms_per_step": 1e3 * el_tot / args.form_steps}
    for g in grids:
        g.close()
    return out


def eulerian_leg(ens, dt, ctl):
    """Eulerian solves of Sec. 3.2 on the ensemble (a first call sets up the boundary
    geometry, work arrays, the assembled matrix and its multigrid hierarchy; the second is
    timed, results copied to the host included), then the closed loop of Table 1 with
    statistics feedback: Eq. (12) from the last statistics stored as the particles' wp, the
    particle step with number control, the pressure projection with the correction of
    Eq. (31), the fields fed back."""
    import torch
    eulerian = {}
    for name, fn in (("elliptic_relaxation", lambda: ens.elliptic_relaxation(tol=1e-10)),
                     ("pressure_projection", lambda: ens.pressure_projection(dt, cp=1e-3, tol=1e-10))):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, it = fn()
        torch.cuda.synchronize()
        eulerian[name] = {"ms": round(1e3 * (time.perf_counter() - t), 2), "cg_iterations": it, "tol": 1e-10}
    ens.set_feedback(True, 1.0, feed_rey=True, feed_omega=True)

    def loop_step():
        ens.elliptic_relaxation(tol=1e-10, store=True)
        ens.step(dt)
        ens.control(*ctl)
        ens.pressure_projection(dt, cp=1e-3, tol=1e-10)

    loop_step()
    ens.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        loop_step()
    ens.sync()
    torch.cuda.synchronize()
    eulerian["closed_loop_step"] = {"ms": round(1e3 * (time.perf_counter() - t) / 3, 2), "steps": 3,
                                    "order": "elliptic relaxation, particle step, control, pressure projection"}
    return eulerian


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1006_0532_amd import pdfgpu, workloads as W

    torch.cuda.set_device(0)
    if args.large_mixed_only:
        print(json.dumps(large_mixed_form(args)), flush=True)
        return
    if args.batched_only:
        legs = ("fp64",) if args.batched_only == "batched" else ("plain",)
        print(json.dumps(batched_form(args, legs)), flush=True)
        return
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
    if args.eulerian_only:
        print(json.dumps({"workload": "channel_large", "eulerian": eulerian_leg(ens, dt, ctl)}), flush=True)
        return

    # the live count of each step: the first from pdf_count before the timed region, the
    # others from the previous step's control report (one synchronisation per step)
    live = []
    cur = ens.count()
    ens.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        live.append(cur)
        ens.step(dt)
        cur = ens.control(*ctl)["live"]
    ens.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = ens.timing(False)
    elapsed = t1 - t0
    psteps = float(sum(live))
    value = psteps / elapsed

    # rooflines (bytes or operations per launch = per-particle figure x live particles);
    # the particle loop is bound by FP64 vector issue, the others by HBM
    kern = {k: v for k, v in tim.items() if v[1] > 0}
    mean_live = psteps / args.steps
    default = (args.nx, args.ny, args.ppe) == (400, 500, 200)

    def roofline(name):
        if name not in kern or name not in BYTES_PER_PARTICLE:
            return None
        avg_ms = kern[name][0] / kern[name][1]
        traffic = counter_traffic(name, default)
        hbm = BYTES_PER_PARTICLE[name] * mean_live / (avg_ms * 1e-3) / 1e9
        r = {"kernel": name, "avg_ms": round(avg_ms, 4),
             "traffic": None if traffic is None else round(traffic / 1e9, 3), "traffic_unit": "GB per launch",
             "hbm": {"bytes_per_particle": BYTES_PER_PARTICLE[name], "achieved_GBs": round(hbm, 1),
                     "frac": round(hbm / HBM_PEAK_GBS, 4)}}
        if traffic is not None:
            tg = traffic / (avg_ms * 1e-3) / 1e9
            r["hbm"].update(counter_GBs=round(tg, 1), counter_frac=round(tg / HBM_PEAK_GBS, 4),
                            counter_bytes_per_particle=round(traffic / mean_live, 1))
        valu = measured(name, "valu_per_wave", default)
        if name == "advance" and valu is not None:
            # one particle per lane: VALU lane-instructions per particle = instructions per wavefront
            ach = valu * mean_live / (avg_ms * 1e-3) / 1e12
            r.update(bound="alu", achieved=round(ach, 2), peak=round(VALU_PEAK_TOPS, 2),
                     unit="T VALU lane-instructions/s", frac=round(ach / VALU_PEAK_TOPS, 4),
                     valu_instructions_per_particle=valu, valu_busy=measured(name, "valu_busy", default))
            flop = measured(name, "fp64_flop_per_particle", default)
            if flop is not None:
                fa = flop * mean_live / (avg_ms * 1e-3) / 1e12
                r["fp64"] = {"flop_per_particle": flop, "achieved_TFLOPs": round(fa, 2), "peak_TFLOPs": FP64_PEAK_TFLOPS,
                             "frac": round(fa / FP64_PEAK_TFLOPS, 4)}
        else:
            r.update(bound="hbm", achieved=r["hbm"]["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=r["hbm"]["frac"], bytes_per_particle=BYTES_PER_PARTICLE[name])
        return r

    dom = max(kern, key=lambda k: kern[k][0])
    roof = roofline(dom)
    # the whole step against HBM: algorithmic bytes of its particle kernels per particle-step
    step_bpp = sum(BYTES_PER_PARTICLE.values())
    step_gbs = step_bpp * value / 1e9
    step_roof = {"bytes_per_particle_step": step_bpp, "achieved_GBs": round(step_gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                 "frac": round(step_gbs / HBM_PEAK_GBS, 4), "target_frac": 0.6}
    tr = [counter_traffic(k, default) for k in BYTES_PER_PARTICLE]
    if all(t is not None for t in tr):
        step_roof["counter_bytes_per_particle_step"] = round(sum(tr) / mean_live, 1)
    rooflines = [r for r in (roofline(k) for k in ("advance", "element_pass", "scatter")) if r]
    per_kernel = {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches": v[1]} for k, v in kern.items()}
    for k, bpp in BYTES_PER_PARTICLE.items():
        if k in kern:
            avg = kern[k][0] / kern[k][1]
            per_kernel[k]["GB/s"] = round(bpp * mean_live / (avg * 1e-3) / 1e9, 1)
    print(f"[bench] per kernel: {json.dumps(per_kernel)}", file=sys.stderr, flush=True)

    # Eulerian solves and the closed loop on the same ensemble after the timed steps
    eulerian = None
    if not args.no_eulerian:
        eulerian = eulerian_leg(ens, dt, ctl)
        print(f"[bench] eulerian: {json.dumps(eulerian)}", file=sys.stderr, flush=True)

    forms = None
    if not args.no_forms:
        forms = {"fp64": {"value": value, "ms_per_step": 1e3 * elapsed / args.steps}}
        ens.close()
        grid.close()
        forms["mixed"] = mixed_form(args, mesh, f, mo, ini, dt, ctl)
        forms["mixed"]["speedup_vs_fp64"] = forms["mixed"]["value"] / value
        forms["mixed"]["stat_error_vs_fp64"] = with_bounds(mixed_error(mesh, f, mo, ini, dt, args.form_steps))
        forms["mixed"]["cavity_large_error_vs_fp64"] = mixed_error_cavity_large(args.form_steps)
        print(f"[bench] mixed: {json.dumps(forms['mixed'])}", file=sys.stderr, flush=True)
        forms["batched"] = batched_form(args)
        b = forms["batched"]
        b["speedup_vs_plain"] = b["fp64"]["value"] / b["plain_fp64_one_at_a_time"]["value"]
        # against the channel's FP64 rate above (smaller problems, half of them street canyons)
        b["rate_vs_channel_fp64"] = b["fp64"]["value"] / value
        print(f"[bench] batched: {json.dumps(b)}", file=sys.stderr, flush=True)
        forms["cavity_huge_mixed"] = large_mixed_form(args)
        print(f"[bench] cavity_huge mixed: {json.dumps(forms['cavity_huge_mixed'])}", file=sys.stderr, flush=True)

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
        "roofline": roof, "rooflines": rooflines, "step_roofline": step_roof, "per_kernel": per_kernel,
        "cpu_baseline": cpu,
        "forms": forms, "eulerian": eulerian,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
