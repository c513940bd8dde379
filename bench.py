"""Benchmark of the RBSOG per-step force path on one MI355X.

Workload: the 300,000-ion +-1 electrolyte at number density 0.1 (random
sequential addition, d_min = 1), r_c = 3.5 with Table 1 row 2 scaled to the
cutoff, P = 200 wave vectors per step, velocity-Verlet dt = 1e-3 from a
Maxwellian at T = 1, wave vectors drawn on the device.  A step is one whole
pass of the path: kick, drift, wrap/quantise, near-list check (and, when
due, cell list and list build), near part, k staging, structure factor, far
force, energies, kick.

Prints one JSON line: particle-steps/s of the FP32C form (``value``) and of
the FP64 form, the FP32C force error against FP64, the roofline of the
dominant kernel measured with HIP events on the library's stream, and the
CPU oracle timed on the host on one force evaluation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s, RBSOG forces FP32-comp vs FP64, at <=1e-5 rel RMS force err"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = VALU lane-op slots per
# second for non-packed instructions (FP32 FMA counts one slot)
PEAK_VALU_SLOTS = 256 * 4 * 16 * 2.4e9
# issue slots of one FP32 transcendental (sin, cos, exp, rsqrt): gfx950 issues
# them at half the FMA rate (measured: 16.5 vs 31.9 T lane-ops/s)
TRANS_SLOTS = 2
# algorithmic VALU slots per unit of work (the method's arithmetic, not the
# implementation's: candidate rejects and the full-list doubling are overhead)
WORK = {
    # per (particle, k): phase 3 + accumulate 2, sin + cos
    "rho": 5 + 2 * TRANS_SLOTS,
    # per (particle, k): phase 3 + Im 2 + accumulate 3, sin + cos
    "far": 8 + 2 * TRANS_SLOTS,
    # per unique pair inside r_c: rsqrt, M+1 = 17 exp, ~40 FMA-class (direct Gaussian sum)
    "near": 40 + 18 * TRANS_SLOTS,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    # tune the main workload's launch shapes during its warm-up (the other
    # workloads are always tuned); off by default so that a kernel trace of the
    # run holds only the timed shapes
    ap.add_argument("--autotune", action="store_true")
    # the ensemble, 2e7-ion and water workloads (reported next to the main line)
    ap.add_argument("--no-other", action="store_true")
    ap.add_argument("--other-steps", type=int, default=100)
    ap.add_argument("--n", type=int, default=300_000, help=argparse.SUPPRESS)
    # after the bench: device-to-device copies of this many MiB, the reference
    # kernel against which rocprofv3's FETCH_SIZE / WRITE_SIZE are scaled
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    # near-list skin (fraction of r_c); 0 builds at every step (the fused
    # cell kernel), as the adaptive skin does while lists last under two steps
    ap.add_argument("--skin", type=float, default=None)
    return ap.parse_args()


def run_precision(R, torch, wl, prec, args, near_table=False, device_chains=0):
    n = len(wl["q"])
    P = wl["P"]
    stream = torch.cuda.Stream()
    sysm = R.System(wl["pos"], wl["q"], wl["box"], wl["rc"], P, seed=2022, precision=prec,
                    stream=stream.cuda_stream, autotune=args.autotune, near_table=near_table,
                    device_chains=device_chains, skin=args.skin)
    label = f"prec={prec}{' core-shell' if near_table else ''}{f' device-chains={device_chains}' if device_chains else ''}"
    if not device_chains:
        batches = 1 + args.warmup + args.steps + args.profile_steps
        t0 = time.time()
        sysm.sample_k(batches)
        log(f"[bench] prec={prec}: sampled {batches * P} wave vectors in {time.time() - t0:.2f} s")
    F0, E0 = sysm.forces()
    Fn0, Ff0 = sysm.components()
    # neighbour pairs inside r_c at step 0 (full list, both orders), for the near roofline
    row, _ = R.rbsog_debug_neighbors(sysm.ctx, n)
    near_pairs = int(row[-1])
    R.rbsog_set_velocities(sysm.ctx, None, T=1.0, seed=7)
    # the first warm-up steps are profiled (one kernel at a time, HIP events):
    # the start of the run, where the near list lasts many steps; the last
    # warm-up steps (at least two) replay the step graph, so that its capture
    # stays out of the timed steps
    w_prof = max(0, min(args.profile_steps, args.warmup - 2))
    kernels_start = {}
    if w_prof > 0:
        R.rbsog_profile(sysm.ctx, True)
        sysm.step(w_prof, 1e-3)
        kernels_start = read_profile(R, sysm)
        R.rbsog_profile(sysm.ctx, False)
    sysm.step(args.warmup - w_prof, 1e-3)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    sysm.step(args.steps, 1e-3)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    log(f"[bench] {label}: {args.steps} steps in {ms:.2f} ms "
        f"(wall {wall * 1e3:.2f} ms)")
    info_end = R.rbsog_info(sysm.ctx)
    # and steps after the timed ones: the state the timed run ended in
    kernels = {}
    if args.profile_steps > 0:
        R.rbsog_profile(sysm.ctx, True)
        sysm.step(args.profile_steps, 1e-3)
        kernels = read_profile(R, sysm)
        R.rbsog_profile(sysm.ctx, False)
    E = R.rbsog_get_energy(sysm.ctx)
    info = R.rbsog_info(sysm.ctx)
    shapes = {k: info[k] for k in ("rho_chunk", "far_block", "tuned", "list_capacity", "list_builds")}
    sysm.close()
    return dict(ms=ms, wall=wall, F0=F0, Fn0=Fn0, Ff0=Ff0, E0=E0, E_end=E, kernels=kernels,
                kernels_start=kernels_start, near_pairs=near_pairs, value=n * args.steps / (ms * 1e-3),
                shapes=shapes, builds=info_end["list_builds"], skin_end=info_end["skin"])


def read_profile(R, sysm):
    prof = R.rbsog_profile_read(sysm.ctx)
    return {k: {"ms_total": v[0], "launches": v[1], "us_per_launch": 1e3 * v[0] / max(v[1], 1)}
            for k, v in prof.items() if v[1] > 0}


DEVICE_CHAINS = 64
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_electrolyte300k.md")
# the counters are valid for the sources they were taken on
KERNEL_SOURCES = ("paper_2205_13824_amd/csrc/kernels_near.hip", "paper_2205_13824_amd/csrc/kernels_far.hip",
                  "paper_2205_13824_amd/csrc/kernels_md.hip", "paper_2205_13824_amd/csrc/rbsog_internal.h")


def kernel_traffic(kernel):
    """HBM bytes per launch of an FP32C kernel from the committed rocprofv3
    counters (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    the kernel sources changed since the counters were taken or the kernel is
    not in the file."""
    import hashlib

    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("source-", "traffic-")))
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if vals.get("source-sha256", "").strip() != h.hexdigest():
        return None
    v = vals.get(f"traffic-{kernel}-bytes-per-launch")
    return int(v) if v is not None else None


# library profile names -> kernel symbols in the rocprofv3 summaries (FP32C; the
# kernels templated on a slot count appear there as e.g. k_near_cells<false, 3>)
KERNEL_SYMBOL = {"near": "k_near_list<false>", "near_cells": "k_near_cells<false>", "rho": "k_rho<false>",
                 "far": "k_far<false>"}


def roofline(kernels, n, P, near_pairs, nexp32=3, ntail32=7):
    # near: units are unique pairs (the list holds both orders); both near
    # kernels evaluate the same pairs
    units = {"rho": n * P, "far": n * P, "near": near_pairs // 2, "near_cells": near_pairs // 2}
    work = dict(WORK, near_cells=WORK["near"])
    cands = {k: v for k, v in kernels.items() if k in units}
    if not cands:
        return None
    dom = max(cands, key=lambda k: cands[k]["ms_total"])
    t = cands[dom]["us_per_launch"] * 1e-6
    achieved = units[dom] * work[dom] / t
    out = {"kernel": KERNEL_SYMBOL[dom], "bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_VALU_SLOTS / 1e9,
           "unit": "Gop/s (VALU lane slots)", "frac": achieved / PEAK_VALU_SLOTS, "traffic": None,
           "units_per_launch": units[dom], "slots_per_unit": work[dom], "us_per_launch": t * 1e6}
    out["traffic"] = kernel_traffic(KERNEL_SYMBOL[dom])
    if dom in ("near", "near_cells"):
        # the same pairs priced as this library evaluates them (both orders;
        # rsqrt, nexp exponentials, two tail polynomials, ~15 FMA-class)
        ev = 2 * (TRANS_SLOTS * (1 + nexp32) + 3 * nexp32 + 2 * ntail32 + 15)
        out["as_evaluated"] = {"slots_per_unit": ev, "frac": units[dom] * ev / t / PEAK_VALU_SLOTS}
    return out


def timed_steps(R, torch, obj, stream, steps, dt):
    """HIP-event time of `steps` velocity-Verlet steps on the library's stream (ms)."""
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    obj.step(steps, dt)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def other_workloads(R, W, torch, args):
    """The other workloads the path is built for, each in the launch shapes the
    autotuner picks: the 256-replica ensemble, about 2e7 ions, 3e6 water sites.
    Wave vectors come from the device chains (a refill every DEVICE_CHAINS
    steps, so the shorter runs below time steps between refills)."""
    out = {}
    # replica ensemble: 256 systems, log-uniform sizes 500..50000, P = 100, FP32C
    t0 = time.time()
    ens = W.c4_ensemble()
    sysl = ens["systems"]
    stream = torch.cuda.Stream()
    b = R.Batch([x["pos"] for x in sysl], [x["q"] for x in sysl], [x["box"] for x in sysl], ens["rc"], ens["P"],
                ens["seeds"], precision=R.RBSOG_FP32C, stream=stream.cuda_stream, autotune=True,
                device_chains=DEVICE_CHAINS)
    steps = args.other_steps
    b.forces()
    R.rbsog_set_velocities(b.ctx, None, T=1.0, seed=7)
    b.step(args.warmup, 1e-3)
    ms = timed_steps(R, torch, b, stream, steps, 1e-3)
    out["ensemble_256"] = {"workload": f"256 replicas, {b.n} ions in all (500..50000 each, log-uniform), density "
                                       f"0.1, r_c=3.5, P=100, FP32C, velocity-Verlet",
                           "value": b.n * steps / (ms * 1e-3), "unit": "particle-steps/s", "steps": steps,
                           "ms_per_step": ms / steps, "setup_s": time.time() - t0}
    b.close()
    log(f"[bench] ensemble: {out['ensemble_256']['value']:.3e} particle-steps/s")
    # about 2e7 ions, P = 1000, both precisions
    c5 = W.c5_large()
    for prec, name in ((R.RBSOG_FP32C, "fp32c"), (R.RBSOG_FP64, "fp64")):
        stream = torch.cuda.Stream()
        sm = R.System(c5["pos"], c5["q"], c5["box"], c5["rc"], c5["P"], seed=5, precision=prec,
                      stream=stream.cuda_stream, autotune=True, device_chains=DEVICE_CHAINS)
        steps5 = max(5, steps // 10)
        sm.forces()
        R.rbsog_set_velocities(sm.ctx, None, T=1.0, seed=7)
        sm.step(2, 1e-3)
        ms = timed_steps(R, torch, sm, stream, steps5, 1e-3)
        out[f"ions_20M_{name}"] = {"workload": f"{len(c5['q'])} ions, density 0.1, jittered lattice, r_c=3.5, "
                                               f"P=1000, velocity-Verlet",
                                   "value": len(c5["q"]) * steps5 / (ms * 1e-3), "unit": "particle-steps/s",
                                   "steps": steps5, "ms_per_step": ms / steps5}
        sm.close()
        log(f"[bench] 2e7 ions {name}: {out[f'ions_20M_{name}']['value']:.3e} particle-steps/s")
    del c5
    # 3e6 water sites (10^6 rigid 3-site molecules as point charges), r_c = 10, P = 500
    pos, q, box = W.water(100, 0.0334, seed=3)
    for prec, name in ((R.RBSOG_FP32C, "fp32c"), (R.RBSOG_FP64, "fp64")):
        stream = torch.cuda.Stream()
        sm = R.System(pos, q, box, 10.0, 500, seed=3, precision=prec, stream=stream.cuda_stream, autotune=True,
                      device_chains=DEVICE_CHAINS)
        sm.forces()
        sm.step(1, 1e-4)
        ms = timed_steps(R, torch, sm, stream, 5, 1e-4)
        out[f"water_3M_{name}"] = {"workload": "3,000,000 water sites (SPC/E-shaped charges), r_c=10, P=500",
                                   "value": len(q) * 5 / (ms * 1e-3), "unit": "particle-steps/s", "steps": 5,
                                   "ms_per_step": ms / 5}
        sm.close()
        log(f"[bench] water {name}: {out[f'water_3M_{name}']['value']:.3e} particle-steps/s")
    return out


def cpu_baseline(wl, budget_s=12.0):
    import oracle

    sog = oracle.sog_row2(wl["rc"])
    pos, q, box, rc, P = wl["pos"], wl["q"], wl["box"], wl["rc"], wl["P"]
    S = oracle.S_product(sog, box)
    m = oracle.mh_sample(sog, box, seed=99, stream=0, n=P)[0]
    evals = 0
    t0 = time.perf_counter()
    while True:
        oracle.near_cells(pos, q, box, rc, sog)
        oracle.far_rb(pos, q, box, sog, m, P, S)
        evals += 1
        if time.perf_counter() - t0 > budget_s or evals >= 60:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(q) * evals / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{evals} full force evaluation(s) (near part over the cell list + random-batch far part, "
                      f"P={P}) of the same {len(q)}-ion system, FP64, OpenMP; the VV update is omitted",
            "seconds": dt}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              f"by spatial domains with one all-reduce of rho per step, which this build does not run).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2205_13824_amd import rbsog as R
    from paper_2205_13824_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    t0 = time.time()
    wl = W.c2_electrolyte(args.n)
    n, P = len(wl["q"]), wl["P"]
    log(f"[bench] workload built in {time.time() - t0:.1f} s: n={n} L={wl['box'][0]:.4f} P={P}")

    # every leg draws its wave vectors inside the timed steps (device chains,
    # identical sequences in both precisions); one more leg takes them from a
    # host-sampled sequence uploaded before timing
    r32 = run_precision(R, torch, wl, R.RBSOG_FP32C, args, device_chains=DEVICE_CHAINS)
    r64 = run_precision(R, torch, wl, R.RBSOG_FP64, args, device_chains=DEVICE_CHAINS)
    r32t = run_precision(R, torch, wl, R.RBSOG_FP32C, args, near_table=True, device_chains=DEVICE_CHAINS)
    r32h = run_precision(R, torch, wl, R.RBSOG_FP32C, args)
    err = math.sqrt(float(np.sum((r32["F0"] - r64["F0"]) ** 2) / np.sum(r64["F0"] ** 2)))
    err_near = math.sqrt(float(np.sum((r32["Fn0"] - r64["Fn0"]) ** 2) / np.sum(r64["Fn0"] ** 2)))
    err_far = math.sqrt(float(np.sum((r32["Ff0"] - r64["Ff0"]) ** 2) / np.sum(r64["Ff0"] ** 2)))
    log(f"[bench] FP32C vs FP64 force relrms: total {err:.3e} near {err_near:.3e} far {err_far:.3e}")
    err_t = math.sqrt(float(np.sum((r32t["F0"] - r64["F0"]) ** 2) / np.sum(r64["F0"] ** 2)))
    log(f"[bench] FP32C core-shell vs FP64 force relrms: total {err_t:.3e}")

    # the kernel that dominates the end of the run (where its steps spend
    # most of their time), and the near-list pass of the run's start
    roof = roofline(r32["kernels"], n, P, r32["near_pairs"])
    roof_start = roofline({k: v for k, v in r32["kernels_start"].items() if k == "near"}, n, P, r32["near_pairs"])
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}-ion +-1 electrolyte, density 0.1, RSA d_min=1, r_c=3.5, P={P}, "
                               f"Table 1 row 2, velocity-Verlet dt=1e-3, T=1, "
                               f"wave vectors sampled on the device ({DEVICE_CHAINS} chains)",
                   "n": n, "P": P, "rc": wl["rc"], "box": float(wl["box"][0])},
        "fp64": {"value": r64["value"], "ms_per_step": r64["ms"] / args.steps, "dtype": "f64"},
        "fp32c_speedup_vs_fp64": r32["value"] / r64["value"],
        "fp32c_coreshell": {"value": r32t["value"], "ms_per_step": r32t["ms"] / args.steps, "dtype": "f32",
                            "force_relrms_vs_fp64": err_t,
                            "near_us_per_launch": r32t["kernels"].get("near", {}).get("us_per_launch"),
                            "note": "near part by the core-shell table of Sec. 3.4 (opts.near_table)"},
        "sampling": {"chains": DEVICE_CHAINS,
                     "refill_us_per_launch": r32["kernels"].get("sample_refill", {}).get("us_per_launch"),
                     "note": "wave vectors drawn inside the timed steps by on-device Metropolis-Hastings chains "
                             f"(opts.device_chains = {DEVICE_CHAINS}): one refill launch every {DEVICE_CHAINS} "
                             "steps advances every chain by P states"},
        "fp32c_host_sequence": {"value": r32h["value"], "ms_per_step": r32h["ms"] / args.steps, "dtype": "f32",
                                "note": "wave vectors from the host chain, sampled and uploaded before timing"},
        "fp32c_force_relrms_vs_fp64": {"total": err, "near": err_near, "far": err_far},
        "energy_step0": {"fp32c": list(map(float, r32["E0"])), "fp64": list(map(float, r64["E0"]))},
        "roofline": roof,
        "roofline_list_pass": roof_start,
        "near_list": {"builds": r32["builds"], "evaluations": 1 + args.warmup + args.steps,
                      "skin_at_end": r32["skin_end"],
                      "note": "list builds over the run; skin 0 at the end means the adaptive skin found lists "
                              "lasting under two steps (the ions without a repulsive core collapse after about "
                              "300 steps) and builds at every step with the fused cell kernel"},
        "kernels_fp32c_start": r32["kernels_start"],
        "kernels_fp32c": r32["kernels"],
        "kernels_fp64": r64["kernels"],
        "launch_shapes": {"fp32c": r32["shapes"], "fp64": r64["shapes"]},
    }
    if not args.no_other:
        out["other_workloads"] = other_workloads(R, W, torch, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 x {args.copy_probe_mib} MiB device-to-device")


if __name__ == "__main__":
    main()
