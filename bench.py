"""Throughput of the whole FMM hot path on one MI355X.

A step is one full evaluation: fmm_build_tree (bounding cube, keys, radix
sort, octree, dual tree traversal, CSR lists) + fmm_upward (P2M, M2M) +
fmm_evaluate (M2L and P2P through the work queue, L2L, L2P, outputs), on
inputs already resident in HBM.  Metric: particles per second per FMM
evaluation at N = 2^20 uniform particles, p = 8, 64 particles per leaf,
theta = 1/2, with the relative L2 error against the FP64 direct sum checked
on a 4096-particle sample.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK = {"fp32_valu": 157.3e12, "fp32_mfma": 157.3e12, "bf16_mfma": 2.5e15, "fp64": 78.6e12, "hbm": 8.0e12}
P2P_FLOP = 20          # per particle pair: potential + field, one reciprocal square root counted once
M2L_SPLIT_PRODUCTS = 3  # bf16 products per FP32-accurate product in the mixed M2L (hi.hi, hi.lo, lo.hi)
# the work queue's kernels and the build of the task tables they run
QUEUE_SOURCES = ("paper_1203_0889_amd/csrc/queue.hip", "paper_1203_0889_amd/csrc/queue.h",
                 "paper_1203_0889_amd/csrc/m2l_mfma.hip", "paper_1203_0889_amd/csrc/near_far.hip")
TRAFFIC_PROFILE = "profiles/k_queue_uniform1m_p8_traffic.txt"


def source_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_counters(workload, tuning):
    """Fields of the committed PMC summary of the work queue, if it was
    taken on this workload, on the current queue kernel source and at this
    work-queue tuning (the file holds one block per profiled tuning; else
    None)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    head, blocks = {}, []
    with open(path) as f:
        for line in f:
            if ":" not in line or line.startswith("#"):
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k == "tuning":
                blocks.append({})
            (blocks[-1] if blocks else head)[k] = v
    if head.get("workload") != workload or head.get("source_sha256_16") != source_hash(QUEUE_SOURCES):
        return None
    fields = next((b for b in blocks if b.get("tuning") == tuning_text(tuning)), None)
    if fields is None:
        return None
    out = {}
    for k in ("hbm_bytes_per_launch", "mfma_flop_executed", "mfma_busy_simd_cycles", "p2p_valu_wave_insts",
              "clock_ghz"):
        try:
            out[k] = float(fields[k])
        except (KeyError, ValueError):
            pass
    return out


def tuning_text(t):
    return "m2l_task_entries=%d,grid_per_cu=%d,p2p_per_cu=%d,early_p2p_per_cu=%d" % (
        t["m2l_task_entries"], t["grid_per_cu"], t["p2p_per_cu"], t.get("early_p2p_per_cu", 0))


def fixed_tuning(text):
    """Parse 'key=value,...' into set_tuning keyword arguments."""
    out = {}
    for item in text.split(","):
        k, v = item.split("=")
        out[k.strip()] = int(v)
    return out


def m2l_flop(p):
    P = (p + 1) ** 2
    return 2 * P * P   # dense real operator applied to one multipole


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform1m_p8",
                    help="uniform1m_p8 (default), plummer1m_p8, plummer4m_p10, uniform4k_p4 or batch256_p6")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--p", type=int, default=None,
                    help="expansion order instead of the workload's (accuracy comparisons across orders)")
    ap.add_argument("--adjoint", action="store_true", help="time forward energy + fmm_backward per step")
    ap.add_argument("--mutual", nargs="?", const="both", default=None, choices=["both", "m2l", "p2p"],
                    help="FP64 path: the mutual interaction for M2L, P2P or both (each pair listed both ways once)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing leg")
    ap.add_argument("--no-error", action="store_true", help="skip the error check against the direct sum")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default work-queue tuning")
    ap.add_argument("--tuning", default=None,
                    help="fixed work-queue tuning, e.g. m2l_task_entries=128,grid_per_cu=1,p2p_per_cu=3 "
                         "(skips the autotuner; counter runs serialise kernels, which skews its timing)")
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="particles in the all-core CPU oracle sample (default: the workload's N)")
    ap.add_argument("--cpu-n-1core", type=int, default=16384,
                    help="particles in the single-core CPU oracle sample")
    ap.add_argument("--sweep", action="store_true",
                    help="granularity sweep (the paper's Q experiment): M2L entries per task x N x p, one JSON line")
    ap.add_argument("--trace", action="store_true",
                    help="after the timed steps, one evaluation with the device task trace: summary in the line")
    ap.add_argument("--timestep", type=int, default=0,
                    help="time stepping: this many steps of straight-line motion per mode (full rebuild, "
                         "incremental, incremental + step graph, incremental + cost reuse), one JSON line")
    ap.add_argument("--drift", type=float, default=0.004,
                    help="time stepping: largest move per step and axis, in units of the particle's leaf side")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_cpu, n_1core):
    """CPU leg: the FP64 oracle FMM on the host (same generator, p, ncrit,
    theta): on all the cores OpenMP is given, at n_cpu particles (the
    workload's N by default), and on one core at n_1core particles."""
    import oracle
    from paper_1203_0889_amd import workloads as W

    def inputs(n):
        if w["dist"] == "uniform":
            return W.uniform_cube(n, w["seed"])
        return W.plummer(n, w["seed"], equal_charges=w["dist"] == "plummer_equal")

    sub_pos, sub_q = inputs(n_cpu)
    t0 = time.perf_counter()
    oracle.fmm(sub_pos, sub_q, w["p"], w["ncrit"], *w["theta"])
    t1 = time.perf_counter()
    cores = oracle.num_threads()
    out = {"value": n_cpu / (t1 - t0), "unit": "particles/s", "cores": cores, "kind": "oracle",
           "sample": "oracle FMM (FP64, Cartesian Taylor, OpenMP over targets; same p/ncrit/theta, %s) on N=%d "
                     "(the workload has N=%d): %.2f s" % (w["dist"], n_cpu, w["n"], t1 - t0),
           "cpu_model": cpu_model(), "nproc": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    if n_1core > 0:
        one_pos, one_q = inputs(n_1core)
        oracle.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.fmm(one_pos, one_q, w["p"], w["ncrit"], *w["theta"])
            t1 = time.perf_counter()
        finally:
            oracle.set_num_threads(cores)
        out["one_core"] = {"value": n_1core / (t1 - t0), "unit": "particles/s", "n": n_1core, "s": t1 - t0}
    return out


def cpu_leg_error(pos, q, outs, w, n, grads=None):
    """CPU leg, second part: the error of the GPU outputs against the
    oracle's direct sum on a seeded sample of targets."""
    import oracle
    from paper_1203_0889_amd import workloads as W
    sample = W.error_sample(n, w["seed"])
    phi_d, fld_d = oracle.direct(pos, q, sample)
    err = {"phi_rel_l2": rel_l2(outs["phi"].cpu().numpy()[sample], phi_d),
           "field_rel_l2": rel_l2(outs["field"].cpu().numpy()[sample], fld_d), "sample": len(sample)}
    if grads is not None:
        # dE/dq = phi, dE/dx = -F of the exact (symmetric) direct sum
        err["grad_q_rel_l2"] = rel_l2(grads[1].cpu().numpy()[sample], phi_d)
        err["grad_pos_rel_l2"] = rel_l2(grads[0].cpu().numpy()[sample], -q[sample, None] * fld_d)
    return err


def cpu_leg_error_batch(pos, q, offs, phi, field):
    """CPU leg for a batch: every 32nd instance against the oracle's direct
    sum (all targets up to 8192 particles, else 1024 seeded targets)."""
    import oracle
    errs = []
    ph, fl = phi.cpu().numpy(), field.cpu().numpy()
    for k in range(0, len(offs) - 1, 32):
        lo, hi = offs[k], offs[k + 1]
        nk = hi - lo
        tg = np.arange(nk) if nk <= 8192 else np.sort(np.random.default_rng(k).choice(nk, 1024, replace=False))
        pd, fd = oracle.direct(pos[lo:hi], q[lo:hi], tg)
        errs.append((rel_l2(ph[lo:hi][tg], pd), rel_l2(fl[lo:hi][tg], fd)))
    return {"phi_rel_l2_max": max(e[0] for e in errs), "field_rel_l2_max": max(e[1] for e in errs),
            "instances_checked": len(errs)}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def queue_roofline(plan, stage_avg, p, n, precision, workload, tuning):
    """Roofline of the dominant kernel and the algorithmic work of one evaluation."""
    counts = plan.counts()
    _, _, cells = plan.copy_tree()
    mp, ms_, pp, ps = plan.copy_lists()
    cnt = cells[:, 5]
    tgt = np.repeat(np.arange(len(cnt)), np.diff(pp))
    inter = int(np.sum(cnt[tgt] * cnt[ps])) - n
    p2p_flop = P2P_FLOP * inter
    m2l_f = m2l_flop(p) * counts["nm2l"]
    t_p2p = stage_avg.get("p2p", 0.0) * 1e-3
    t_m2l = stage_avg.get("m2l", 0.0) * 1e-3
    if precision == "mixed":
        # M2L and P2P run in the work queue: k_queue on the plan's stream
        # with the P2P-only k_p2p_side beside it on forked streams (stage
        # "queue": HIP events from before k_queue on the plan's stream to
        # the join of the side streams).  Its ALU bound on the method's own
        # work: P2P flops on the FP32 vector units and M2L flops (2 P^2 per
        # pair) on the bf16 matrix cores, the dtype of the contraction; the
        # two do not issue concurrently on a SIMD, so their minimum times add.
        tq = stage_avg.get("queue", 0.0) * 1e-3
        flops = p2p_flop + m2l_f
        t_min = p2p_flop / PEAK["fp32_valu"] + m2l_f / PEAK["bf16_mfma"]
        ctr = committed_counters(workload, tuning) or {}
        roof = {"bound": "alu", "achieved": flops / tq / 1e12 if tq > 0 else None,
                "peak": flops / t_min / 1e12, "unit": "TFLOP/s", "traffic": ctr.get("hbm_bytes_per_launch"),
                "kernel": "k_queue + k_p2p_side (P2P FP32 VALU + M2L split-bf16 MFMA)", "kernel_ms": tq * 1e3,
                "peak_basis": "P2P flop / 157.3 TF fp32 vector + M2L flop (2 P^2 per pair) / 2.5 PF bf16 dense MFMA"}
        # the bound the implementation's own instruction mix allows: three
        # bf16 products per FP32-accurate M2L product (split operands), and
        # the FP32 vector rate without packed FP32 (half of 157.3 TF; packed
        # FP32 instructions are disabled at compile time)
        t_split = p2p_flop / PEAK["fp32_valu"] + m2l_f * M2L_SPLIT_PRODUCTS / PEAK["bf16_mfma"]
        t_np = p2p_flop / (PEAK["fp32_valu"] / 2) + m2l_f * M2L_SPLIT_PRODUCTS / PEAK["bf16_mfma"]
        roof["split_products"] = {"peak": flops / t_split / 1e12, "basis": "3 bf16 products per M2L product"}
        roof["split_products_nonpacked_fp32"] = {"peak": flops / t_np / 1e12,
                                                 "basis": "3 bf16 products per M2L product, FP32 vector rate 78.65 TF"}
        if tq > 0:
            for k in ("split_products", "split_products_nonpacked_fp32"):
                roof[k]["frac"] = flops / tq / 1e12 / roof[k]["peak"]
        # from the committed counters of this workload, tuning and queue
        # source: what the matrix cores and vector units actually executed
        if "mfma_flop_executed" in ctr:
            roof["m2l_mfma"] = {"flop_executed": ctr["mfma_flop_executed"], "method_flop": m2l_f,
                                "executed_per_method_flop": ctr["mfma_flop_executed"] / m2l_f}
            if tq > 0 and "mfma_busy_simd_cycles" in ctr and "clock_ghz" in ctr:
                simd_cycles = tq * ctr["clock_ghz"] * 1e9 * 1024
                roof["m2l_mfma"]["busy_frac_of_queue"] = ctr["mfma_busy_simd_cycles"] / simd_cycles
        if "p2p_valu_wave_insts" in ctr and inter > 0:
            roof["p2p_valu_insts_per_interaction"] = ctr["p2p_valu_wave_insts"] * 64 / inter
    else:
        dom, t, f = ("p2p", t_p2p, p2p_flop) if t_p2p >= t_m2l else ("m2l", t_m2l, m2l_f)
        roof = {"bound": "alu", "achieved": f / t / 1e12 if t > 0 else None, "peak": PEAK["fp64"] / 1e12,
                "unit": "TFLOP/s", "traffic": None, "kernel": "%s fp64" % dom}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    work = {"ncell": counts["ncell"], "nleaf": counts["nleaf"], "m2l_pairs": counts["nm2l"],
            "p2p_pairs": counts["np2p"], "p2p_interactions": inter, "p2p_flop": p2p_flop, "m2l_flop": m2l_f,
            "m2l_tables": plan.queue_info()}
    return roof, work


def timed(step, plan, steps, warmup, torch):
    """Mean wall time of `steps` steps (synchronised before and after, no
    synchronisation inside), then the per-stage HIP-event times averaged over
    `max(warmup, 1)` further steps, read after each of those steps."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_sum = {}
    nstage = max(warmup, 1)
    for _ in range(nstage):
        step()
        for k, v in plan.stage_times().items():    # HIP events on the plan's stream
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    return (t1 - t0) * 1e3 / steps, {k: v / nstage for k, v in stage_sum.items()}


def calib_copy(mib, torch, dev):
    if mib <= 0:
        return
    nel = mib * (1 << 20) // 4
    src = torch.ones(nel, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def base_result(a, value, ms, unit_metric):
    return {"metric": unit_metric, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16x3-mfma+f32+f64" if a.precision == "mixed" else "f64",
            "data": "synthetic"}


def run_single(a, torch, fmm, W):
    pos, q, w = W.make(a.workload)
    if a.p is not None:
        w = dict(w, p=a.p)
    n = len(q)
    print("bench: workload %s N=%d precision %s%s" % (a.workload, n, a.precision, " + adjoint" if a.adjoint else ""),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    dpos = torch.from_numpy(pos).to(dev)
    dq = torch.from_numpy(q).to(dev)
    plan = fmm.Plan(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0,
                    mutual=a.mutual or False)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    field = torch.empty((n, 3), dtype=torch.float64, device=dev)
    force = torch.empty((n, 3), dtype=torch.float64, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)
    gE = torch.ones(1, dtype=torch.float64, device=dev)
    grads = [None, None]
    bw_ms = [0.0]
    calib_copy(a.copy_calib_mib, torch, dev)

    tuning = plan.get_tuning()
    if a.tuning:
        plan.set_tuning(**fixed_tuning(a.tuning))
        tuning = plan.get_tuning()
    elif not a.no_autotune:
        # set-up, not timed: pick the work-queue setting (FP64: the task
        # size of its matrix-core M2L) on this workload
        plan.build_tree(dpos, dq)
        plan.upward()
        tuning, tq_ms = plan.autotune(repeats=2)
        print("bench: autotuned %s (evaluation %.3f ms)" % (tuning, tq_ms), file=sys.stderr, flush=True)

    ev = [torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]

    def step():
        plan.build_tree(dpos, dq)
        plan.upward()
        plan.evaluate_into(phi=phi, field=field, force=force, energy=energy)
        if a.adjoint:
            ev[0].record()
            grads[0], grads[1] = plan.backward(gE)
            ev[1].record()
            ev[1].synchronize()
            bw_ms[0] += ev[0].elapsed_time(ev[1])

    ms, stage_avg = timed(step, plan, a.steps, a.warmup, torch)
    if a.adjoint:
        stage_avg["backward"] = bw_ms[0] / (a.steps + a.warmup + max(a.warmup, 1))
    print("bench: %.3f ms/step; stages %s" % (ms, json.dumps({k: round(v, 4) for k, v in stage_avg.items()})),
          file=sys.stderr, flush=True)
    roof, work = queue_roofline(plan, stage_avg, w["p"], n, a.precision, a.workload, tuning)
    if a.adjoint:
        metric = "particles/s per FMM energy + gradient (forward + fmm_backward), %s" % a.workload
    else:
        metric = "particles/s per FMM evaluation at N=1M, rel. L2 error \u22641e-4 vs FP64 direct"
        if a.workload != "uniform1m_p8":
            metric = "particles/s per FMM evaluation, %s" % a.workload
    result = base_result(a, n / (ms * 1e-3), ms, metric)
    result["config"] = {"workload": a.workload if a.p is None else "%s_at_p%d" % (a.workload, a.p), "n": n, "p": w["p"], "ncrit": w["ncrit"],
                        "theta": "%d/%d" % tuple(w["theta"]), "precision": a.precision, "distribution": w["dist"],
                        "adjoint": bool(a.adjoint)}
    if a.mutual:
        result["config"]["mutual"] = a.mutual
    result["stages_ms"] = {k: round(v, 4) for k, v in stage_avg.items()}
    result["tuning"] = tuning
    result["work"] = work
    result["roofline"] = roof
    if a.trace and a.precision == "mixed":
        # outside the timed region: a second plan with the task trace on,
        # writing into outputs of its own (the error check below reads the
        # timed plan's outputs)
        from paper_1203_0889_amd import trace as T
        tp = fmm.Plan(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0, trace=True)
        tp.set_tuning(**tuning)
        t_phi, t_field = torch.empty_like(phi), torch.empty_like(field)
        for _ in range(2):
            tp.build_tree(dpos, dq)
            tp.upward()
            tp.evaluate_into(phi=t_phi, field=t_field)
        result["trace"] = T.summarize(tp.trace())
        print("bench: task trace %s" % json.dumps(result["trace"]), file=sys.stderr, flush=True)
        tp.close()
    if not a.no_cpu:
        result["cpu_baseline"] = cpu_baseline(w, min(a.cpu_n, n) if a.cpu_n > 0 else n, a.cpu_n_1core)
    if not a.no_error:
        result["error"] = cpu_leg_error(pos, q, {"phi": phi, "field": field}, w, n,
                                        grads if a.adjoint else None)
    return result


def run_batch(a, torch, fmm, W):
    """256 instances (N_k = round(2^(10 + 6u)), even k uniform, odd k Plummer),
    p = 6, ncrit = 64, theta = 1/2: one batched solve (one forest, one build,
    one queue launch) per step, against 256 sequential single-instance solves
    and against replays of the batched plan's captured graph."""
    n_inst, p, ncrit, theta = 256, 6, 64, (1, 2)
    pos, q, offsets = W.batch(n_inst, 5)
    n = len(q)
    offs = [int(o) for o in offsets]
    print("bench: workload batch256_p6 N=%d in %d instances" % (n, n_inst), file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    dpos = torch.from_numpy(pos).to(dev)
    dq = torch.from_numpy(q).to(dev)
    plan = fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=a.precision, device=0)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    field = torch.empty((n, 3), dtype=torch.float64, device=dev)
    energy = torch.empty(n_inst, dtype=torch.float64, device=dev)
    tuning = plan.get_tuning()
    if a.tuning:
        plan.set_tuning(**fixed_tuning(a.tuning))
        tuning = plan.get_tuning()
    elif not a.no_autotune and a.precision == "mixed":
        plan.build_tree(dpos, dq, offs)
        plan.upward()
        tuning, _ = plan.autotune(repeats=2)

    def step():
        plan.build_tree(dpos, dq, offs)
        plan.upward()
        plan.evaluate_into(phi=phi, field=field, energy=energy)

    ms, stage_avg = timed(step, plan, a.steps, a.warmup, torch)
    roof, work = queue_roofline(plan, stage_avg, p, n, a.precision, "batch256_p6", tuning)
    # graph replay of upward + evaluate on the built forest
    plan.graph_capture(phi=phi, field=field, energy=energy)
    for _ in range(a.warmup):
        plan.graph_launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        plan.graph_launch()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / a.steps
    # a whole step in one graph on a kept topology (rebuild from the
    # positions and charges through the stored permutation, upward,
    # evaluate): a second plan with FMM_FLAG_KEEP_TOPOLOGY
    kplan = fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=a.precision, device=0, keep_topology=True)
    kplan.set_tuning(**tuning)
    kplan.build_tree(dpos, dq, offs)
    kphi, kfield = torch.empty_like(phi), torch.empty_like(field)
    kenergy = torch.empty_like(energy)
    kplan.graph_capture_step(dpos, dq, phi=kphi, field=kfield, energy=kenergy)
    for _ in range(a.warmup):
        kplan.graph_launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        kplan.graph_launch()
    torch.cuda.synchronize()
    step_graph_ms = (time.perf_counter() - t0) * 1e3 / a.steps
    kplan.sync()
    del kplan
    # 256 sequential single-instance solves (same tuning), one warm pass first
    singles = [fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=a.precision, device=0) for _ in range(n_inst)]
    for s_ in singles:
        s_.set_tuning(**tuning)
    views = [(dpos[offs[k]:offs[k + 1]], dq[offs[k]:offs[k + 1]]) for k in range(n_inst)]
    sphi = torch.empty(n, dtype=torch.float64, device=dev)
    sfld = torch.empty((n, 3), dtype=torch.float64, device=dev)

    def sequential():
        for k, s_ in enumerate(singles):
            s_.build_tree(views[k][0], views[k][1])
            s_.upward()
            s_.evaluate_into(phi=sphi[offs[k]:offs[k + 1]], field=sfld[offs[k]:offs[k + 1]])

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    print("bench: batched %.3f ms, graph replay %.3f ms, step graph (kept topology) %.3f ms, sequential %.3f ms"
          % (ms, graph_ms, step_graph_ms, seq_ms), file=sys.stderr, flush=True)
    result = base_result(a, n / (ms * 1e-3), ms, "particles/s, 256 instances solved as one batch (sum N_k / time)")
    result["config"] = {"workload": "batch256_p6", "n": n, "instances": n_inst, "p": p, "ncrit": ncrit,
                        "theta": "1/2", "precision": a.precision, "distribution": "even k uniform, odd k Plummer"}
    result["stages_ms"] = {k: round(v, 4) for k, v in stage_avg.items()}
    result["tuning"] = tuning
    result["work"] = work
    result["roofline"] = roof
    result["sequential"] = {"ms": seq_ms, "particles_per_s": n / (seq_ms * 1e-3), "speedup_of_batch": seq_ms / ms}
    result["graph_replay_upward_evaluate"] = {"ms": graph_ms, "particles_per_s": n / (graph_ms * 1e-3)}
    result["graph_replay_kept_topology_step"] = {"ms": step_graph_ms,
                                                 "particles_per_s": n / (step_graph_ms * 1e-3)}
    if not a.no_error:
        result["error"] = cpu_leg_error_batch(pos, q, offs, phi, field)
    return result


def run_sweep(a, torch, fmm, W):
    """The paper's granularity experiment (Sec. 5) on the GPU queue: uniform
    cubes of N = 1e5, 1e6, 1e7 particles, p = 6 and 9 (ncrit 64, theta 1/2,
    mixed), M2L class entries per task in {16, 32, 64, 128} (the task size,
    the analogue of Q) with the default launch shape.  Per point: the mean of
    3 timed steps (build + upward + evaluate, HIP events per stage), the
    number of M2L tasks, and the balance of one traced evaluation."""
    from paper_1203_0889_amd import trace as T
    dev = torch.device("cuda", 0)
    rows = []
    for n in (100000, 1000000, 10000000):
        pos, q = W.uniform_cube(n, 2)
        dpos, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
        for p in (6, 9):
            for entries in (16, 32, 64, 128):
                row = {"n": n, "p": p, "m2l_task_entries": entries}
                for traced in (False, True):
                    plan = fmm.Plan(p=p, ncrit=64, theta=(1, 2), precision="mixed", device=0, trace=traced)
                    plan.set_tuning(m2l_task_entries=entries, grid_per_cu=1, p2p_per_cu=2)

                    def step():
                        plan.build_tree(dpos, dq)
                        plan.upward()
                        plan.evaluate(force=False, energy=False)
                    if traced:
                        step()
                        s = T.summarize(plan.trace())
                        row.update({"m2l_tasks": plan.queue_info()["ntask"], "m2l_task_median_us": s["m2l"]["median_us"],
                                    "cu_busy_imbalance": s["cu_busy_imbalance"],
                                    "tail_us": s["cu_last_end_us"]["max"] - s["cu_last_end_us"]["min"]})
                    else:
                        ms, st = timed(step, plan, 3, 1, torch)
                        row.update({"ms_per_step": ms, "particles_per_s": n / (ms * 1e-3), "queue_ms": st["queue"]})
                    plan.close()
                print("bench: sweep %s" % json.dumps(row), file=sys.stderr, flush=True)
                rows.append(row)
    return {"sweep": "M2L class entries per task x N x p, uniform, ncrit 64, theta 1/2, mixed", "rows": rows}


def run_timestep(a, torch, fmm, W):
    """Time stepping on one workload: every particle moves along a straight
    line, at most `drift` of its leaf side per step and axis; each mode runs
    `warmup` untimed then `timestep` timed steps of (tree, upward, evaluate)
    from the step's positions, which sit in device memory beforehand.
    Modes: full rebuild every step; FMM_FLAG_INCREMENTAL (the topology is
    kept while every particle stays inside its leaf widened by 1/8 of a side);
    the same with the whole step replayed from a captured graph (the step's
    positions are copied into the graph's input first); both again with
    FMM_FLAG_COST_REUSE (P2P tasks ordered by the durations measured in the
    previous step).  `value` is the last mode's rate (mixed), else that of
    the step graph."""
    from paper_1203_0889_amd import trace as T
    pos, q, w = W.make(a.workload)
    n = len(q)
    dev = torch.device("cuda", 0)
    k_all = a.warmup + a.timestep
    print("bench: time stepping %s N=%d, %d + %d steps, drift %.4g leaf sides per step"
          % (a.workload, n, a.warmup, a.timestep, a.drift), file=sys.stderr, flush=True)
    probe = fmm.Plan(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0)
    dpos0, dq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    probe.build_tree(dpos0, dq)
    _, perm, cells = probe.copy_tree()
    tuning = probe.get_tuning()
    if a.tuning:
        tuning.update(fixed_tuning(a.tuning))
    elif a.precision == "mixed" and not a.no_autotune:
        probe.upward()
        tuning, _ = probe.autotune(repeats=2)
    probe.close()
    # leaf side of every particle (input order): the tight cube's side over 2^level
    side0 = float(np.max(pos.max(axis=0) - pos.min(axis=0)))
    side = np.zeros(n)
    for c in np.nonzero(cells[:, 6] < 0)[0]:
        side[perm[cells[c, 4]:cells[c, 4] + cells[c, 5]]] = side0 / 2.0 ** cells[c, 0]
    vel = torch.from_numpy(W.velocities(n, w["seed"] + 1000, a.drift * side)).to(dev)
    steps_pos = [(dpos0 + k * vel).contiguous() for k in range(1, k_all + 1)]
    outs = {"phi": torch.empty(n, dtype=torch.float64, device=dev),
            "field": torch.empty((n, 3), dtype=torch.float64, device=dev),
            "force": torch.empty((n, 3), dtype=torch.float64, device=dev),
            "energy": torch.empty(1, dtype=torch.float64, device=dev)}
    modes = {}
    mode_names = ["rebuild", "incremental", "incremental_graph"]
    if a.precision == "mixed":
        mode_names += ["incremental_cost_reuse", "incremental_graph_cost_reuse"]
    for mode in mode_names:
        kw = dict(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0)
        if mode != "rebuild":
            kw["incremental"] = True
        if mode.endswith("cost_reuse"):
            kw["cost_reuse"] = True
        plan = fmm.Plan(**kw)
        plan.set_tuning(**tuning)
        plan.build_tree(dpos0, dq)
        gpos = None
        if "graph" in mode:
            gpos = steps_pos[0].clone()
            plan.graph_capture_step(gpos, dq, **outs)

        def step(k):
            if gpos is not None:
                gpos.copy_(steps_pos[k])
                plan.graph_launch()
            else:
                plan.build_tree(steps_pos[k], dq)
                plan.upward()
                plan.evaluate_into(**outs)

        for k in range(a.warmup):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(a.warmup, k_all):
            step(k)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if gpos is not None:
            plan.sync()          # the replays' leaf checks
        ms = (t1 - t0) * 1e3 / a.timestep
        modes[mode] = {"ms_per_step": ms, "particles_per_s": n / (ms * 1e-3), "builds": plan.build_info()}
        print("bench: %s %s" % (mode, json.dumps(modes[mode])), file=sys.stderr, flush=True)
        plan.close()
    if a.precision == "mixed":
        # the same steps with the task trace on, with and without cost
        # reuse: the balance of the work queue in the last step
        balance = {}
        for reuse in (False, True):
            tp = fmm.Plan(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0,
                          incremental=True, trace=True, cost_reuse=reuse)
            tp.set_tuning(**tuning)
            tp.build_tree(dpos0, dq)
            for k in range(k_all):
                tp.build_tree(steps_pos[k], dq)
                tp.upward()
                tp.evaluate_into(**outs)
            balance["cost_reuse" if reuse else "estimated_costs"] = T.summarize(tp.trace())
            tp.close()
        modes["queue_balance_last_step"] = balance
        print("bench: balance %s" % json.dumps(balance), file=sys.stderr, flush=True)
    best = "incremental_graph_cost_reuse" if a.precision == "mixed" else "incremental_graph"
    result = base_result(a, modes[best]["particles_per_s"], modes[best]["ms_per_step"],
                         "particles/s per time step (tree, upward, evaluate) on a kept topology, %s" % a.workload)
    result["steps"] = a.timestep
    result["config"] = {"workload": "%s_timestep" % a.workload, "n": n, "p": w["p"], "ncrit": w["ncrit"],
                        "theta": "%d/%d" % tuple(w["theta"]), "precision": a.precision, "distribution": w["dist"],
                        "drift_leaf_sides_per_step": a.drift}
    result["tuning"] = tuning
    result["modes"] = modes
    if not a.no_error:
        result["error"] = cpu_leg_error(steps_pos[-1].cpu().numpy(), q, outs, w, n)   # the last step's outputs
    return result


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus %d refused)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.mutual and (a.precision != "fp64" or a.sweep or a.timestep > 0 or a.workload == "batch256_p6"):
        print("bench.py: --mutual is an FP64-path option of a single workload", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1203_0889_amd import fmm, workloads as W
    if a.sweep:
        result = run_sweep(a, torch, fmm, W)
    elif a.timestep > 0:
        result = run_timestep(a, torch, fmm, W)
    elif a.workload == "batch256_p6":
        result = run_batch(a, torch, fmm, W)
    else:
        result = run_single(a, torch, fmm, W)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
