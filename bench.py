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
QUEUE_SOURCES = ("paper_1203_0889_amd/csrc/queue.hip", "paper_1203_0889_amd/csrc/queue.h")
TRAFFIC_PROFILE = "profiles/k_queue_uniform1m_p8_traffic.txt"


def source_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(workload):
    """HBM bytes per queue launch from the committed PMC summary, if it was
    taken on this workload and on the current queue kernel source."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("workload") != workload or fields.get("source_sha256_16") != source_hash(QUEUE_SOURCES):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def m2l_flop(p):
    P = (p + 1) ** 2
    return 2 * P * P   # dense real operator applied to one multipole


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform1m_p8")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default work-queue tuning")
    ap.add_argument("--cpu-n", type=int, default=524288, help="particles in the CPU oracle sample")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(pos, q, w, sample_idx, n_cpu):
    """CPU leg: the FP64 oracle timed on a bounded sample of the same
    workload, plus the oracle direct sum on the error sample."""
    import oracle
    from paper_1203_0889_amd import workloads as W
    sub_pos, sub_q = W.uniform_cube(n_cpu, w["seed"]) if w["dist"] == "uniform" else W.plummer(n_cpu, w["seed"])
    t0 = time.perf_counter()
    oracle.fmm(sub_pos, sub_q, w["p"], w["ncrit"], *w["theta"])
    t1 = time.perf_counter()
    phi_d, fld_d = oracle.direct(pos, q, sample_idx)
    base = {"value": n_cpu / (t1 - t0), "unit": "particles/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "oracle FMM (FP64, Cartesian Taylor, same p/ncrit/theta, %s) on N=%d instead of %d; %.2f s"
                      % (w["dist"], n_cpu, len(q), t1 - t0)}
    return base, phi_d, fld_d


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d refused)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1203_0889_amd import fmm, workloads as W

    pos, q, w = W.make(a.workload)
    n = len(q)
    print("bench: workload %s N=%d precision %s" % (a.workload, n, a.precision), file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    dpos = torch.from_numpy(pos).to(dev)
    dq = torch.from_numpy(q).to(dev)
    plan = fmm.Plan(p=w["p"], ncrit=w["ncrit"], theta=w["theta"], precision=a.precision, device=0)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    field = torch.empty((n, 3), dtype=torch.float64, device=dev)
    energy = torch.empty(1, dtype=torch.float64, device=dev)

    if a.copy_calib_mib > 0:
        nel = a.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        plan.build_tree(dpos, dq)
        plan.upward()
        plan.evaluate_into(phi=phi, field=field, energy=energy)

    tuning = plan.get_tuning()
    if not a.no_autotune and a.precision == "mixed":
        # set-up, not timed: pick the work-queue setting on this workload
        plan.build_tree(dpos, dq)
        plan.upward()
        tuning, tq_ms = plan.autotune(repeats=2)
        print("bench: autotuned %s (queue %.3f ms)" % (tuning, tq_ms), file=sys.stderr, flush=True)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    stage_sum = {}
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
        for k, v in plan.stage_times().items():    # HIP events on the plan's stream
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / a.steps
    stage_avg = {k: v / a.steps for k, v in stage_sum.items()}
    print("bench: %.3f ms/step; stages %s" % (ms, json.dumps({k: round(v, 4) for k, v in stage_avg.items()})),
          file=sys.stderr, flush=True)

    counts = plan.counts()
    # algorithmic work of one evaluation
    _, _, cells = plan.copy_tree()
    mp, ms_, pp, ps = plan.copy_lists()
    cnt = cells[:, 5]
    tgt = np.repeat(np.arange(len(cnt)), np.diff(pp))
    inter = int(np.sum(cnt[tgt] * cnt[ps])) - n
    p2p_flop = P2P_FLOP * inter
    m2l_f = m2l_flop(w["p"]) * counts["nm2l"]
    t_p2p = stage_avg.get("p2p", 0.0) * 1e-3
    t_m2l = stage_avg.get("m2l", 0.0) * 1e-3
    if a.precision == "mixed":
        # M2L and P2P run in one work-queue launch (stage "queue", HIP events
        # on the plan's stream).  Its ALU bound: P2P on the FP32 vector units
        # plus M2L on the bf16 matrix cores at three products per FP32-accurate
        # product; the two do not issue concurrently on a SIMD, so their
        # minimum times add.
        tq = stage_avg.get("queue", 0.0) * 1e-3
        t_min = p2p_flop / PEAK["fp32_valu"] + m2l_f * M2L_SPLIT_PRODUCTS / PEAK["bf16_mfma"]
        traffic = committed_traffic(a.workload)
        roof = {"bound": "alu", "achieved": (p2p_flop + m2l_f) / tq / 1e12 if tq > 0 else None,
                "peak": (p2p_flop + m2l_f) / t_min / 1e12, "unit": "TFLOP/s", "traffic": traffic,
                "kernel": "k_queue (P2P FP32 VALU + M2L split-bf16 MFMA)", "kernel_ms": tq * 1e3,
                "peak_basis": "P2P flop / 157.3 TF fp32 vector + 3 x M2L flop / 2.5 PF bf16 dense MFMA"}
    else:
        dom, t, f = ("p2p", t_p2p, p2p_flop) if t_p2p >= t_m2l else ("m2l", t_m2l, m2l_f)
        roof = {"bound": "alu", "achieved": f / t / 1e12 if t > 0 else None, "peak": PEAK["fp64"] / 1e12,
                "unit": "TFLOP/s", "traffic": None, "kernel": "%s fp64" % dom}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]

    result = {
        "metric": "particles/s per FMM evaluation at N=1M, rel. L2 error <=1e-4 vs FP64 direct",
        "value": n / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": n, "p": w["p"], "ncrit": w["ncrit"],
                   "theta": "%d/%d" % tuple(w["theta"]), "precision": a.precision,
                   "distribution": w["dist"]},
        "stages_ms": {k: round(v, 4) for k, v in stage_avg.items()},
        "tuning": tuning,
        "work": {"ncell": counts["ncell"], "nleaf": counts["nleaf"], "m2l_pairs": counts["nm2l"],
                 "p2p_pairs": counts["np2p"], "p2p_interactions": inter, "p2p_flop": p2p_flop, "m2l_flop": m2l_f},
        "roofline": roof,
    }
    if not a.no_cpu:
        sample = W.error_sample(n, w["seed"])
        base, phi_d, fld_d = cpu_baseline(pos, q, w, sample, a.cpu_n)
        result["cpu_baseline"] = base
        ph = phi.cpu().numpy()[sample]
        fl = field.cpu().numpy()[sample]
        result["error"] = {"phi_rel_l2": float(np.linalg.norm(ph - phi_d) / np.linalg.norm(phi_d)),
                           "field_rel_l2": float(np.linalg.norm(fl - fld_d) / np.linalg.norm(fld_d)),
                           "sample": len(sample)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
