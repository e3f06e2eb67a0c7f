"""Benchmark of the planner's hot path: full three-weight iterations (App. B
steps 1-7) on the p=1024, eta=16, 32-wall random-box workload (8.4 M
collision factors), FP32 on one MI355X.

A step is one full iteration over every factor of the graph.  Prints one
JSON line: whole-job factor-updates/s (all factors, active or not) of the
plain dense-state iteration, the roofline of its dominant kernel from HIP
events on the solver's stream, the activity-bit variant, the batched
launch of 256 ragged instances against the same instances solved one after
another, the adjoint of 500 unrolled iterations against the forward run,
and the FP64 reference timed on this host's cores on a bounded sample.
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

# HBM bytes per launch of the factor-stream kernel on the 1024-agent box,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE (median KiB per dispatch) scaled
# by the same counters over a 512 MiB device copy (read x2.000, write
# x1.000).  Valid only for the kernel sources they were taken on.
MEASURED_TRAFFIC = {
    "dense": dict(fetch_kib=142758.5, write_kib=1176.4, sources="235194436a4501f6"),
    "skip": dict(fetch_kib=4353.5, write_kib=2318.2, sources="235194436a4501f6"),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
KERNEL_SOURCES = ("paper_1311_4527_amd/csrc/twa.hip", "paper_1311_4527_amd/csrc/prox.h",
                  "paper_1311_4527_amd/csrc/solver.h")


def kernel_sources_digest():
    """Digest of the kernel sources with comments and blank space removed, so
    that it changes exactly when the code the counters were taken on does."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(variant):
    m = MEASURED_TRAFFIC[variant]
    if m["sources"] != kernel_sources_digest():
        return None
    return (m["fetch_kib"] * FETCH_SCALE + m["write_kib"] * WRITE_SCALE) * 1024.0


def workload(name):
    from paper_1311_4527_amd import instances as I
    if name == "box1024":
        return I.conf_box1024()
    if name == "swap100":
        return I.conf_swap100(0)
    if name == "swap8":
        return I.conf_small(0)
    if name == "single1":
        # one agent in free space from a noisy start (eta=8): the optimum is
        # the straight line between its end points
        return I.circle_swap(1, 0.1, 8, sigma=0.3, seed=1, alpha=1.0, C=1.0, name="single1_eta8_s1")
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(inst, dense: bool, active=(0, 0)):
    """Bytes the factor-stream kernel must move per launch.

    dense: u of every collision and wall edge is read (8 B per edge in 2-D);
    it is written back only where it changes, i.e. where a factor that sent
    weight rho0 in the previous iteration turns inactive and its u resets to
    zero (at most active = (collision, wall) factors active in the last
    iteration); energy and fixed edges' u read and written; both node-record
    arrays read once (16 B per node each), plus radii.
    otherwise: one activity bit per collision/wall factor read and written,
    energy and fixed edges' u read and written, the current node records."""
    c = inst.counts()
    d = inst.dim
    N = c["nodes"]
    small = 2 * 4 * d * (2 * c["energy"] + c["fixed"])
    if dense:
        reads = 4 * d * (4 * c["coll"] + 2 * c["wall"])
        resets = 4 * d * (4 * active[0] + 2 * active[1])
        return reads + resets + small + 2 * 16 * N + 4 * inst.p
    bits = 2 * ((c["coll"] + 31) // 32 + (c["wall"] + 31) // 32) * 4
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
    q = S.twa_get_quality()  # objective, clearance and last move, on the device
    S.close()
    return dict(seconds=t1 - t0, kernel_ms=kms, stats=stats, objective=q["objective"],
                min_clearance=q["min_clearance"], max_move=q["max_move"])


def roofline(inst, variant, avg_ms, stats):
    """Roofline object of the dominant kernel (avg_ms: per-launch device ms of
    the three kernels; stats: the solver's, for the active factor counts)."""
    dom = max(range(3), key=lambda k: avg_ms[k])
    dense = variant == "dense"
    active = (stats["active_coll"], stats["active_wall"])
    if dom == 0 and dense:
        A = algorithmic_bytes(inst, True, active) / (avg_ms[0] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=A, peak=HBM_PEAK_GBS, unit="GB/s", frac=A / HBM_PEAK_GBS,
                    traffic=measured_traffic("dense"))
    elif dom == 0:
        A = activity_flops(inst) / (avg_ms[0] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=A, peak=FP32_VALU_TFLOPS, unit="TFLOP/s", frac=A / FP32_VALU_TFLOPS,
                    traffic=measured_traffic("skip"))
    else:
        roof = dict(bound="alu", achieved=None, peak=FP32_VALU_TFLOPS, unit="TFLOP/s", frac=None, traffic=None)
    roof["kernel"] = KERNELS[dom]
    roof["avg_us"] = {KERNELS[k]: avg_ms[k] * 1e3 for k in range(3)}
    roof["algorithmic_bytes_per_launch"] = algorithmic_bytes(inst, dense, active)
    return roof


def objective(inst, z):
    import numpy as np
    z = np.asarray(z, dtype=np.float64)
    return float(np.sum(inst.C * np.sum(np.diff(z, axis=1) ** 2, axis=2)))


def run_batched(K, warmup):
    """256 ragged instances (p ~ U{4..128}, eta in {4, 8, 16}, swaps and
    boxes, 2-D and 3-D) in one persistent launch, against the same instances
    solved one after another with the plain solver for the same iterations."""
    import numpy as np
    import torch
    from paper_1311_4527_amd import autotune, instances as I
    from paper_1311_4527_amd.twa import Batch, Solver, TWA_F_DENSE
    insts = I.conf_batch()
    F = sum(i.counts()["factors"] for i in insts)
    tuner = Batch(insts)
    log = []
    block, groups = autotune.tune(tuner, iters=20, use_cache=False, log=log)
    tuner.close()
    B = Batch(insts)
    B.twa_batch_config(block, groups)
    B.twa_batch_iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = B.twa_batch_iterate_timed(K)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    zb = [B.twa_batch_get_trajectories(i).cpu().numpy() for i in range(len(insts))]
    B.close()
    t_plain = 0.0
    worst = 0.0
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst)
        S.twa_iterate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.twa_iterate(K)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        zp = S.twa_get_trajectories().cpu().numpy()
        S.close()
        Jb, Jp = objective(inst, zb[i]), objective(inst, zp)
        worst = max(worst, abs(Jb - Jp) / max(Jp, 1e-30))
    # the literal dense form of the same batch in the phased launch: every
    # edge's u read, so HBM-bound; its whole iterations (three phases)
    # against the algorithmic bytes of all instances
    D = Batch(insts, flags=TWA_F_DENSE)
    D.twa_batch_config(0, 1)
    D.twa_batch_iterate(warmup)
    Kd = min(K, 500)
    d_ms = D.twa_batch_iterate_timed(Kd)
    act = [D.twa_batch_solver(i).twa_get_stats() for i in range(len(insts))]
    D.close()
    bytes_it = sum(algorithmic_bytes(i, True, (a["active_coll"], a["active_wall"])) for i, a in zip(insts, act))
    A = bytes_it / (d_ms * 1e-3 / Kd) / 1e9
    dense = dict(iterations=Kd, device_ms=d_ms, us_per_iteration=d_ms * 1e3 / Kd, value=F * Kd / (d_ms * 1e-3),
                 roofline=dict(bound="hbm", achieved=A, peak=HBM_PEAK_GBS, unit="GB/s", frac=A / HBM_PEAK_GBS,
                               traffic=None, kernel="kp_stream + kp_queue + kp_nodes (whole iteration)",
                               algorithmic_bytes_per_iteration=bytes_it))
    return dict(instances=len(insts), factors=F, iterations=K, warmup=warmup,
                value=F * K / t_batch, unit="factor-updates/s", seconds=t_batch, device_ms=dev_ms,
                plain_sequential=dict(value=F * K / t_plain, seconds=t_plain),
                speedup=t_plain / t_batch, max_rel_objective_diff=worst,
                autotune=dict(block=block, groups=groups, candidates=log), dense_phased=dense)


def profile_batched(K, warmup=50, block=0, groups=1):
    """The 256-instance batch in one launch form only (default: phased), K
    iterations after a warm-up, for a kernel trace."""
    import torch
    from paper_1311_4527_amd import instances as I
    from paper_1311_4527_amd.twa import Batch
    insts = I.conf_batch()
    F = sum(i.counts()["factors"] for i in insts)
    B = Batch(insts)
    B.twa_batch_config(block, groups)
    B.twa_batch_iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.twa_batch_iterate(K)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    B.close()
    return dict(instances=len(insts), factors=F, iterations=K, block=block, groups=groups,
                value=F * K / t, unit="factor-updates/s", us_per_iteration=t / K * 1e6)


def min_clearance_pairs(radii, z):
    """Smallest closest-approach distance minus r_i + r_j over every pair and
    segment of trajectories z [p][eta+1][dim] (constant velocity per segment)."""
    import numpy as np
    z = np.asarray(z, dtype=np.float64)
    p = z.shape[0]
    iu, ju = np.triu_indices(p, 1)
    d0 = z[ju, :-1] - z[iu, :-1]
    d1 = z[ju, 1:] - z[iu, 1:]
    e = d1 - d0
    ee = np.sum(e * e, axis=-1)
    a = np.clip(-np.sum(d0 * e, axis=-1) / np.where(ee > 0, ee, 1.0), 0.0, 1.0)
    v = d0 + a[..., None] * e
    dist = np.sqrt(np.sum(v * v, axis=-1))
    return float(np.min(dist - (radii[iu] + radii[ju])[:, None]))


def run_admm_vs_twa(max_iters=20000, every=50):
    """Iterations until the trajectories are collision-free (clearance
    >= -1e-6, checked every 50 iterations) for the three-weight algorithm and
    for standard ADMM (all weights rho0) on antipodal circle swaps."""
    import torch
    from paper_1311_4527_amd import instances as I
    from paper_1311_4527_amd.twa import Solver, TWA_F_ADMM
    out = []
    for p, r, eta in ((8, 0.05, 4), (16, 0.05, 6), (32, 0.03, 6)):
        inst = I.circle_swap(p, r, eta, sigma=1e-3, seed=0, alpha=0.1, C=1.0 / (p * 4), name=f"swap{p}")
        row = dict(p=p, eta=eta, r=r)
        for flags, name in ((0, "twa"), (TWA_F_ADMM, "admm")):
            S = Solver.from_instance(inst, flags=flags)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done, free_at = 0, None
            while done < max_iters:
                S.twa_iterate(every)
                done += every
                if min_clearance_pairs(inst.radii, S.twa_get_trajectories().cpu().numpy()) >= -1e-6:
                    free_at = done
                    break
            torch.cuda.synchronize()
            row[name] = dict(iterations_to_collision_free=free_at, seconds=time.perf_counter() - t0)
            S.close()
        out.append(row)
    return out


def run_feasible_vs_energy(max_iters=20000, every=25):
    """Sec. 4 (CONF2): random starts and goals in the plane.  Iterations to a
    collision-free plan with no cost term, against iterations until the
    energy run is collision-free and its objective has settled (within 1e-3
    of the value after max_iters), and the feasibility restart from the
    energy run stopped at 10% of that."""
    import numpy as np
    import torch
    from paper_1311_4527_amd import instances as I
    from paper_1311_4527_amd.twa import Solver, TWA_F_COST_NONE
    out = []
    for p in (16, 32, 64):
        inst = I.random_box(p, 0.02, 8, min_sep=0.05, sigma=1e-3, seed=100 + p, alpha=0.1, C=1.0 / (p * 8))
        row = dict(p=p, eta=8, r=0.02)
        # feasibility only
        S = Solver.from_instance(inst, flags=TWA_F_COST_NONE)
        free = None
        for k in range(every, max_iters + 1, every):
            S.twa_iterate(every)
            if min_clearance_pairs(inst.radii, S.twa_get_trajectories().cpu().numpy()) >= -1e-6:
                free = k
                break
        row["feasible_iterations"] = free
        S.close()
        # energy: objective trace
        E = Solver.from_instance(inst)
        trace = []
        for k in range(every, max_iters + 1, every):
            E.twa_iterate(every)
            z = E.twa_get_trajectories().cpu().numpy()
            trace.append((k, objective(inst, z), min_clearance_pairs(inst.radii, z)))
        E.close()
        Jf = trace[-1][1]
        row["energy_iterations"] = next((k for k, J, c in trace if abs(J - Jf) <= 1e-3 * Jf and c >= -1e-6), None)
        # stop the energy run early, then solve the feasibility problem from its state
        stop = max(every, (row["energy_iterations"] or max_iters) // 10)
        E = Solver.from_instance(inst)
        E.twa_iterate(stop)
        zz, uu, ll, _ = E.twa_get_state()
        row["energy_stopped_at"] = stop
        row["stopped_clearance"] = min_clearance_pairs(inst.radii, zz.cpu().numpy())
        F = Solver.from_instance(inst, flags=TWA_F_COST_NONE)
        F.twa_set_state(zz, uu, ll, 0)
        restart = None
        for k in range(every, max_iters + 1, every):
            F.twa_iterate(every)
            if min_clearance_pairs(inst.radii, F.twa_get_trajectories().cpu().numpy()) >= -1e-6:
                restart = k
                break
        row["restart_iterations"] = restart
        row["restart_objective"] = objective(inst, F.twa_get_trajectories().cpu().numpy())
        row["converged_objective"] = Jf
        E.close()
        F.close()
        out.append(row)
    torch.cuda.synchronize()
    return out


def run_vo(p=16, r=0.05):
    """Sec. 5: the velocity-obstacle local planner on an antipodal swap of p
    agents; wall time of every epoch's joint solve (eq. rec_col_avoi_pos) on
    the GPU, iterated to a collision-free plan, as the paper times it."""
    import numpy as np
    import torch
    from paper_1311_4527_amd.vo import VOPlanner
    ang = 2 * np.pi * np.arange(p) / p
    pos = np.stack([np.cos(ang), np.sin(ang)], 1)
    V = VOPlanner(pos, -pos, np.full(p, r), tau=1.0, fraction=0.5, vmax=0.25)
    V.solve_epoch()  # warm
    warm = V.last_iterations
    times, its = [], []
    for _ in range(200):
        if V.arrived():
            break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V.step()
        times.append(time.perf_counter() - t0)
        its.append(V.last_iterations)
    V.close()
    t = np.array(times)
    conv = [n for n in its if n > 0]
    return dict(p=p, r=r, epochs=len(times), arrived=V.arrived(), epochs_at_cap=len(its) - len(conv),
                iterations_median=float(np.median(conv)) if conv else None, iterations_total=int(sum(conv)),
                warm_iterations=int(warm),
                epoch_ms_median=float(np.median(t) * 1e3), epoch_ms_p90=float(np.percentile(t, 90) * 1e3),
                epoch_ms_max=float(t.max() * 1e3))


def run_sizes(sizes=(256, 512, 1024, 2048), steps=200, warmup=300):
    """The benchmark's random box (eta = 16, 32 walls, r = 0.005) at other
    agent counts: whole-iteration throughput, dense and activity bits, in the
    steady state (warmup iterations first), with the dominant kernel's
    roofline fraction (algorithmic bytes or operations of that size; the
    counter traffic is measured for 1024 agents only)."""
    from paper_1311_4527_amd import instances as I
    out = []
    for p in sizes:
        inst = I.conf_box1024(p=p)
        F = inst.counts()["factors"]
        row = dict(p=p, factors=F)
        for variant in ("dense", "skip"):
            r = run_gpu(inst, variant == "dense", steps, warmup)
            avg = [m / steps for m in r["kernel_ms"]]
            roof = roofline(inst, variant, avg, r["stats"])
            row[variant] = dict(value=F * steps / r["seconds"], ms_per_step=1e3 * r["seconds"] / steps,
                                kernel=roof["kernel"], bound=roof["bound"], frac=roof["frac"],
                                avg_us=roof["avg_us"])
        print(f"# p={p}: dense {row['dense']['value']:.4g}, skip {row['skip']['value']:.4g} factor-updates/s",
              file=sys.stderr, flush=True)
        out.append(row)
    return out


def run_adjoint(K=500):
    """Forward K iterations alone, then forward with the start remembered plus
    the adjoint on the p=256, eta=8 swap.  The TAPE solver's first backward
    (untimed) sizes its forward tape; the timed forward records checkpoints
    into it, and the timed backward reads them instead of re-running the
    forward."""
    import numpy as np
    import torch
    from paper_1311_4527_amd import instances as I
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = I.conf_adjoint(7)
    S = Solver.from_instance(inst)
    S.twa_iterate(K)                     # warm (graphs, clocks)
    S.twa_set_init(inst.z0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.twa_iterate(K)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    S.close()
    T = Solver.from_instance(inst, flags=TWA_F_TAPE)
    v = torch.from_numpy(np.random.default_rng(0).normal(size=inst.z0.shape).astype(np.float32)).cuda()
    T.twa_iterate(K)
    T.twa_backward(v)                    # warm
    T.twa_set_init(inst.z0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.twa_iterate(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dx0, dxT, dr, _ = T.twa_backward(v)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = bool(torch.isfinite(dx0).all() and torch.isfinite(dr).all())
    taped = T.twa_get_stats()["tape_checkpoints"]   # recorded by the timed forward
    T.close()
    c = inst.counts()
    every = 32 * max(1, round(np.sqrt(K) / 32)) if taped else int(np.ceil(np.sqrt(K)))
    return dict(workload=f"{inst.name}: p={inst.p}, eta={inst.eta}, {c['edges']} edges", K=K,
                checkpoint_every=every, forward_tape_checkpoints=taped, forward_s=t_fwd,
                forward_taped_s=t1 - t0, backward_s=t2 - t1, backward_over_forward=(t2 - t1) / t_fwd,
                forward_taped_plus_backward_over_forward=(t2 - t0) / t_fwd, finite=ok)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(P, budget_s):
    """Reference iterations per second over about budget_s seconds (after one
    untimed iteration)."""
    P.iterate(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        P.iterate(1)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return n, time.perf_counter() - t0


def cpu_baseline(inst, budget_s=8.0):
    """The FP64 reference, untouched, on this host's cores: all of the threads
    it is given (OMP_NUM_THREADS), then one thread, each over about budget_s
    seconds of iterations of the same instance from its straight-line start."""
    import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1))
    F = inst.counts()["factors"]
    O.set_threads(cores)
    n, dt = _oracle_rate(O.Planner(inst), budget_s)
    O.set_threads(1)
    n1, dt1 = _oracle_rate(O.Planner(inst), budget_s)
    O.set_threads(cores)
    out = dict(value=F * n / dt, unit="factor-updates/s", cores=cores, kind="oracle",
               sample=f"{n} reference iterations on {cores} threads (after 1 untimed) of the same p=1024, eta=16, "
                      f"32-wall instance from its straight-line start, {dt:.1f} s wall; and {n1} iterations on "
                      f"one thread, {dt1:.1f} s",
               cpu_model=cpu_model(), host_threads=os.cpu_count(), single_thread=dict(value=F * n1 / dt1, unit="factor-updates/s", cores=1,
                                                         iterations=n1, seconds=dt1))
    # the two small circle swaps and one free agent, beside the GPU's small_workloads leg
    small = {}
    for name, K in (("swap8", 2000), ("swap100", 100), ("single1", 200)):
        si = workload(name)
        Ps = O.Planner(si)
        t0 = time.perf_counter()
        Ps.iterate(K)
        ds = time.perf_counter() - t0
        small[name] = dict(iterations=K, iterations_per_s=K / ds,
                           factor_updates_per_s=si.counts()["factors"] * K / ds)
    out["small_workloads"] = small
    return out


def run_small(warmup=50):
    """The circle swaps of 8 agents (eta=4, 2000 iterations) and 100 agents
    (eta=8, 5000 iterations): launch- and latency-bound, so iterations/s."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    out = {}
    for name, K in (("swap8", 2000), ("swap100", 5000)):
        inst = workload(name)
        S = Solver.from_instance(inst)
        S.twa_iterate(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.twa_iterate(K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(p=inst.p, eta=inst.eta, iterations=K, iterations_per_s=K / dt,
                         factor_updates_per_s=inst.counts()["factors"] * K / dt,
                         objective=objective(inst, S.twa_get_trajectories().cpu().numpy()))
        S.close()
    # one agent in free space, 200 iterations from a fresh solver (the
    # convergence run the paper times on its own single-agent example)
    import numpy as np
    inst = workload("single1")
    S = Solver.from_instance(inst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.twa_iterate(200)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    z = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    s = np.arange(inst.eta + 1) / inst.eta
    line = inst.x0[:, None, :] + s[None, :, None] * (inst.xT - inst.x0)[:, None, :]
    out["single1"] = dict(p=1, eta=inst.eta, iterations=200, ms=dt * 1e3, iterations_per_s=200 / dt,
                          max_distance_to_line=float(np.abs(z - line).max()))
    S.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="box1024")
    ap.add_argument("--variant", choices=["dense", "skip"], default="dense")
    ap.add_argument("--only", action="store_true", help="time the chosen variant only (for profiling)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (for hardware-counter scaling)")
    ap.add_argument("--leg", choices=["batched", "adjoint", "vo", "sizes"], default=None,
                    help="only run one side leg, without its comparison runs (for profiling)")
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
    if args.leg == "batched":
        print(json.dumps(profile_batched(args.batch_steps)), flush=True)
        return
    if args.leg == "adjoint":
        print(json.dumps(run_adjoint(500)), flush=True)
        return
    if args.leg == "vo":
        print(json.dumps(run_vo()), flush=True)
        return
    if args.leg == "sizes":
        print(json.dumps(run_sizes()), flush=True)
        return
    inst = workload(args.workload)
    c = inst.counts()
    F = c["factors"]
    r = run_gpu(inst, args.variant == "dense", args.steps, args.warmup)
    avg = [m / args.steps for m in r["kernel_ms"]]
    out = dict(metric="TWA factor-prox updates/s (all factors, one full iteration = one step)",
               value=F * args.steps / r["seconds"], unit="factor-updates/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=1e3 * r["seconds"] / args.steps, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"{inst.name}: random box p={inst.p}, eta={inst.eta}, {inst.n_walls} walls, "
                                    f"r={float(inst.radii[0])}, FP32 ({c['coll']} collision + {c['wall']} wall + "
                                    f"{c['energy']} energy + {c['fixed']} fixed factors, {c['edges']} edges)",
                           variant=args.variant, iterations_per_s=args.steps / r["seconds"]),
               roofline=roofline(inst, args.variant, avg, r["stats"]),
               active=r["stats"], objective=r["objective"], min_clearance=r["min_clearance"],
               max_move=r["max_move"])
    print(f"# main {args.variant}: {out['value']:.4g} factor-updates/s", file=sys.stderr, flush=True)
    if not args.only:
        other = "skip" if args.variant == "dense" else "dense"
        r2 = run_gpu(inst, other == "dense", args.steps, args.warmup)
        avg2 = [m / args.steps for m in r2["kernel_ms"]]
        out["variants"] = {other: dict(value=F * args.steps / r2["seconds"],
                                       ms_per_step=1e3 * r2["seconds"] / args.steps,
                                       roofline=roofline(inst, other, avg2, r2["stats"]), objective=r2["objective"])}
        print(f"# variant {other}: {out['variants'][other]['value']:.4g}", file=sys.stderr, flush=True)
        out["batched"] = run_batched(args.batch_steps, 50)
        print(f"# batched: {out['batched']['value']:.4g} (x{out['batched']['speedup']:.1f} vs sequential)",
              file=sys.stderr, flush=True)
        out["small_workloads"] = run_small()
        print(f"# small: {[(k, round(v['iterations_per_s'])) for k, v in out['small_workloads'].items()]} iterations/s",
              file=sys.stderr, flush=True)
        out["admm_vs_twa"] = run_admm_vs_twa()
        print(f"# admm vs twa: {[(r['p'], r['twa']['iterations_to_collision_free'], r['admm']['iterations_to_collision_free']) for r in out['admm_vs_twa']]}",
              file=sys.stderr, flush=True)
        out["feasible_vs_energy"] = run_feasible_vs_energy()
        print(f"# feasible vs energy: {[(r['p'], r['feasible_iterations'], r['energy_iterations'], r['restart_iterations']) for r in out['feasible_vs_energy']]}",
              file=sys.stderr, flush=True)
        out["vo_local_planner"] = run_vo()
        print(f"# vo: {out['vo_local_planner']}", file=sys.stderr, flush=True)
        out["adjoint"] = run_adjoint(500)
        print(f"# adjoint: backward/forward {out['adjoint']['backward_over_forward']:.2f}", file=sys.stderr,
              flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
