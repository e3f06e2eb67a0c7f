"""Benchmark of the planner's hot path: full three-weight iterations (App. B
steps 1-7) on the p=1024, eta=16, 32-wall random-box workload (8.4 M
collision factors), FP32 on one MI355X.

A step is one full iteration over every factor of the graph.  Prints one
JSON line: whole-job factor-updates/s (all factors, active or not), the
roofline of the dominant kernel from HIP events on the solver's stream, and
the FP64 reference timed on this host's cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3   # MI355X FP32 vector peak
KERNELS = ("k_stream", "k_queue", "k_nodes")


def workload(name):
    from paper_1311_4527_amd import instances as I
    if name == "box1024":
        return I.conf_box1024()
    if name == "swap100":
        return I.conf_swap100(0)
    if name == "swap8":
        return I.conf_small(0)
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(inst, dense: bool):
    """Bytes the factor-stream kernel must move per launch.

    dense: u of every edge is read and written (8+8 B per edge in 2-D), both
    node-record arrays are read once (16 B per node each), plus radii.
    otherwise: one activity bit per collision/wall factor read and written,
    energy and fixed edges' u read and written, the current node records."""
    c = inst.counts()
    d = inst.dim
    N = c["nodes"]
    if dense:
        return 2 * 4 * d * c["edges"] + 2 * 16 * N + 4 * inst.p
    bits = 2 * ((c["coll"] + 31) // 32 + (c["wall"] + 31) // 32) * 4
    small = 2 * 4 * d * (2 * c["energy"] + c["fixed"])
    return bits + small + 16 * N + 4 * inst.p


def activity_flops(inst):
    """FP32 operations of the closest-approach test of every collision
    factor (relative positions, clamp, squared distance: 28 ops in 2-D) and
    the segment distance of every wall factor (about 60 ops)."""
    c = inst.counts()
    return 28 * c["coll"] + 60 * c["wall"]


def run_gpu(inst, dense, steps, warmup):
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_DENSE
    S = Solver.from_instance(inst, flags=TWA_F_DENSE if dense else 0)
    S.twa_iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = S.twa_iterate_timed(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = S.twa_get_stats()
    z = S.twa_get_trajectories().cpu().numpy().astype("float64")
    import numpy as np
    J = float(np.sum(inst.C * np.sum(np.diff(z, axis=1) ** 2, axis=2)))
    S.close()
    return dict(seconds=t1 - t0, kernel_ms=kms, stats=stats, objective=J)


def cpu_baseline(inst, budget_s=12.0):
    """The FP64 reference, untouched, on this host's cores: one untimed
    iteration, then iterations until about budget_s seconds have passed."""
    import oracle as O
    P = O.Planner(inst)
    P.iterate(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        P.iterate(1)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    F = inst.counts()["factors"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    return dict(value=F * n / dt, unit="factor-updates/s", cores=cores, kind="oracle",
                sample=f"{n} reference iterations (after 1 untimed) of the same p=1024, eta=16, 32-wall "
                       f"instance from its straight-line start, {dt:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="box1024")
    ap.add_argument("--variant", choices=["dense", "skip"], default="dense")
    ap.add_argument("--also", action="store_true", help="also time the other variant")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (for hardware-counter scaling)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=4 * n, copy_bytes_written=4 * n, launches=5)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the planner's single-GPU hot path has no multi-GPU "
              "component (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    inst = workload(args.workload)
    c = inst.counts()
    dense = args.variant == "dense"
    r = run_gpu(inst, dense, args.steps, args.warmup)
    F = c["factors"]
    value = F * args.steps / r["seconds"]
    ms = r["kernel_ms"]
    avg = [m / args.steps for m in ms]
    dom = max(range(3), key=lambda k: avg[k])
    if dom == 0 and dense:
        A = algorithmic_bytes(inst, True) / (avg[0] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=A, peak=HBM_PEAK_GBS, unit="GB/s", frac=A / HBM_PEAK_GBS, traffic=None)
    elif dom == 0:
        A = activity_flops(inst) / (avg[0] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=A, peak=FP32_VALU_TFLOPS, unit="TFLOP/s", frac=A / FP32_VALU_TFLOPS,
                    traffic=None)
    else:
        roof = dict(bound="alu", achieved=None, peak=FP32_VALU_TFLOPS, unit="TFLOP/s", frac=None, traffic=None)
    roof["kernel"] = KERNELS[dom]
    roof["avg_us"] = {KERNELS[k]: avg[k] * 1e3 for k in range(3)}
    roof["algorithmic_bytes_per_launch"] = algorithmic_bytes(inst, dense)
    out = dict(metric="TWA factor-prox updates/s (all factors, one full iteration = one step)",
               value=value, unit="factor-updates/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * r["seconds"] / args.steps, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"{inst.name}: random box p={inst.p}, eta={inst.eta}, {inst.n_walls} walls, "
                                    f"r=0.005, FP32 ({c['coll']} collision + {c['wall']} wall + {c['energy']} "
                                    f"energy + {c['fixed']} fixed factors, {c['edges']} edges)",
                           variant=args.variant, iterations_per_s=args.steps / r["seconds"]),
               roofline=roof,
               active=r["stats"], objective=r["objective"])
    if args.also:
        r2 = run_gpu(inst, not dense, args.steps, args.warmup)
        out["other_variant"] = dict(variant="skip" if dense else "dense",
                                    value=F * args.steps / r2["seconds"],
                                    ms_per_step=1e3 * r2["seconds"] / args.steps,
                                    avg_us={KERNELS[k]: r2["kernel_ms"][k] / args.steps * 1e3 for k in range(3)},
                                    objective=r2["objective"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
