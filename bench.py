"""Benchmark of the RBSOG per-step force path on one MI355X.

Headline workload: about 2e7 ions (272^3 = 20,123,648 +-1 charges at number
density 0.1 on a jittered simple-cubic lattice, charges shuffled), r_c = 3.5
with Table 1 row 2 scaled to the cutoff, P = 1000 wave vectors per step drawn
on the device, velocity Verlet with dt = 1e-3 from a Maxwellian at T = 1.  A
step is one whole pass of the path: kick, drift, wrap/quantise, near-list
check (and, when due, cell list and list build), near part, k staging,
structure factor, far force, energies, kick.

Prints one JSON line: particle-steps/s of the FP32C form (``value``) and of
the FP64 form, the FP32C force error against FP64 (total, near, far), the
roofline of the dominant kernel against MI355X's published peaks (with its
duration measured by HIP events on the library's stream over profiled steps
of the same run), the CPU oracle timed on the host on a bounded sample of the
same workload, and the other workloads (300,000-ion electrolyte, 3e6 water
sites, 256-replica ensemble) with their own figures.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s, RBSOG forces FP32-comp vs FP64, at <=1e-5 rel RMS force err"

# MI355X published peaks: vector FP32 157.3 TFLOP/s (packed FMA counted as 2
# flops per lane), vector FP64 78.6 TFLOP/s, HBM3E 8 TB/s
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# Algorithmic work per unit as the method states it (candidate rejects and
# the full list's second evaluation of a pair are overhead): FMA-class
# operations and transcendentals
#   structure factor per (particle, k): phase 3 + accumulate 2, sin + cos
#   far force per (particle, k): phase 3 + Im 2 + accumulate 3, sin + cos
#   near part per unique pair inside r_c: ~40 FMA-class, rsqrt + M+1 = 17 exp
OPS = {"rho": (5, 2), "far": (8, 2), "near": (40, 18)}
# flops: an FMA-class operation 2, a transcendental 1
FLOPS = {k: 2 * f + t for k, (f, t) in OPS.items()}

DEVICE_CHAINS = 64
DT = 1e-3

# workloads the timed legs can run on: (generator in workloads.py, description)
WORKLOADS = {
    "ions20M": ("c5_large", "+-1 ions (272^3 jittered simple-cubic lattice), density 0.1, r_c=3.5"),
    "electrolyte300k": ("c2_electrolyte", "+-1 electrolyte, density 0.1, RSA d_min=1, r_c=3.5"),
    "water3M": ("c3_water", "water sites (10^6 SPC/E-shaped 3-site molecules as point charges), r_c=10"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    # steps after the timed ones that run kernel by kernel with HIP events
    ap.add_argument("--profile-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other", action="store_true")
    ap.add_argument("--other-steps", type=int, default=200)
    ap.add_argument("--no-autotune", action="store_true")
    # after the bench: device-to-device copies of this many MiB, the reference
    # kernel against which rocprofv3's FETCH_SIZE / WRITE_SIZE are scaled
    ap.add_argument("--copy-probe-mib", type=int, default=0)
    # the workload of the two timed legs (profiling runs of the other
    # workloads name them here; the reported headline is ions20M)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="ions20M")
    return ap.parse_args()


def relrms(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def profile_steps_split(R, obj, mode, steps):
    """Per-kernel HIP-event times over `steps` single steps in profile mode
    `mode`: ({kernel: mean over the steps without a near-list build},
    {kernel: mean over the steps with one})."""
    acc = ({}, {})
    for _ in range(steps):
        nb0 = R.rbsog_info(obj.ctx)["list_builds"]
        R.rbsog_profile(obj.ctx, mode)
        obj.step(1, DT)
        prof = R.rbsog_profile_read(obj.ctx)
        built = R.rbsog_info(obj.ctx)["list_builds"] > nb0
        for k, (t, cnt) in prof.items():
            if cnt > 0:
                a = acc[1 if built else 0].setdefault(k, [0.0, 0])
                a[0] += t
                a[1] += cnt
    R.rbsog_profile(obj.ctx, 0)
    return tuple({k: {"ms_total": v[0], "launches": v[1], "us_per_launch": 1e3 * v[0] / v[1]} for k, v in d.items()}
                 for d in acc)


def timed_steps(torch, obj, stream, steps):
    """HIP-event time (ms) of `steps` velocity-Verlet steps on the stream the
    library launches on (torch's stream object, passed to the library)."""
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    obj.step(steps, DT)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def run_leg(R, torch, wl, prec, args, steps, near_table=False, autotune=True, profile_steps=None):
    """One precision on one workload: first evaluation (forces kept), tuning,
    warm-up (step graphs captured), timed steps, profiled steps."""
    n, P = len(wl["q"]), wl["P"]
    stream = torch.cuda.Stream()
    t0 = time.time()
    sysm = R.System(wl["pos"], wl["q"], wl["box"], wl["rc"], P, seed=2022, precision=prec,
                    stream=stream.cuda_stream, near_table=near_table, device_chains=DEVICE_CHAINS)
    F0, E0 = sysm.forces()
    Fn0, Ff0 = sysm.components()
    tune = None
    if autotune:
        t1 = time.time()
        info = R.rbsog_autotune(sysm.ctx, 3)
        tune = {k: info[k] for k in ("rho_chunk", "far_block", "rho_ktile", "build_slots", "cell_slots", "tuned")}
        tune["seconds"] = time.time() - t1
    R.rbsog_set_velocities(sysm.ctx, None, T=1.0, seed=7)
    sysm.step(args.warmup, DT)
    setup = time.time() - t0
    ms = timed_steps(torch, sysm, stream, steps)
    info_end = R.rbsog_info(sysm.ctx)
    kernels, alone, build_step = {}, {}, {}
    ps = args.profile_steps if profile_steps is None else profile_steps
    if ps > 0:
        # kernel by kernel with HIP events on the stream each kernel runs on:
        # first as in the timed steps (the structure factor beside the near
        # part on the second stream for systems with little far work), then
        # every kernel alone; steps that built a near list kept apart
        kernels, build_step = profile_steps_split(R, sysm, 2, ps)
        alone, _ = profile_steps_split(R, sysm, 1, ps)
        for k, v in kernels.items():
            if k in alone:
                v["us_alone"] = alone[k]["us_per_launch"]
    info = R.rbsog_info(sysm.ctx)
    sysm.close()
    label = f"{n} prec={prec}{' core-shell' if near_table else ''}"
    log(f"[bench] {label}: {steps} steps in {ms:.2f} ms ({ms / steps:.4f} ms/step), setup {setup:.1f} s")
    return dict(ms=ms, steps=steps, F0=F0, Fn0=Fn0, Ff0=Ff0, E0=E0, kernels=kernels, build_step=build_step,
                value=n * steps / (ms * 1e-3), ms_per_step=ms / steps, tune=tune,
                shapes={k: info[k] for k in ("rho_chunk", "far_block", "rho_ktile", "build_slots", "cell_slots", "tuned", "list_capacity")},
                builds=info_end["list_builds"], skin_end=info_end["skin"], setup_s=setup)


def count_near_pairs(R, wl):
    """Unique pairs inside r_c at the start (the near kernels' algorithmic units)."""
    sysm = R.System(wl["pos"], wl["q"], wl["box"], wl["rc"], wl["P"], seed=1, precision=R.RBSOG_FP32C,
                    device_chains=1)
    sysm.forces()
    row, _ = R.rbsog_debug_neighbors(sysm.ctx)
    sysm.close()
    return int(row[-1]) // 2


# kernel names (as rocprofv3 shows them, without the template's later
# arguments) of the profile keys
KERNEL_NAMES = {"rho": "k_rho", "far": "k_far", "far_side": "k_far_side", "near": "k_near_list",
                "near_cells": "k_near_cells", "list_build": "k_list_build"}


def traffic_table(workload):
    """HBM bytes per launch from the committed counter summary of the
    workload, for the kernels whose sources have not changed since (else
    none)."""
    from paper_2205_13824_amd import profsummary

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return {}
    return profsummary.read_traffic(path)


def traffic_of(tab, key, fp64):
    """HBM bytes per launch of the kernel the profile steps time for `key`:
    the first template argument is the precision, and the variant whose
    remaining flags are all false is the one timed (the far kernel of the
    single profiled steps does not open the next step; the near list pass
    records no pairs and sums no energies there)."""
    want = f"{KERNEL_NAMES[key]}<{'true' if fp64 else 'false'}"
    cands = [k for k in tab if k == want + ">" or k.startswith(want + ",")]
    plain = [k for k in cands if all(x.strip() == "false" for x in k[len(want) + 1:-1].split(",") if x.strip())]
    pick = plain[0] if plain else (cands[0] if cands else None)
    if pick is None:
        return None
    rd, wr = tab[pick]
    return rd + wr


def rooflines(kernels, n, P, near_pairs, fp64, traffic=None, rates=None):
    """Per kernel: algorithmic flops per launch / measured launch time (HIP
    events, as in the timed steps) against the published vector peak of the
    precision; the same with the kernel alone on the device; and (FP32) the
    time the algorithmic operations take at this device's measured issue
    rates (FMA-class at the FP32 FMA rate, transcendentals at the sin/cos
    rate), as a fraction of the launch time."""
    units = {"rho": n * P, "far": n * P, "far_side": n * P, "near": near_pairs, "near_cells": near_pairs}
    kind = {"rho": "rho", "far": "far", "far_side": "far", "near": "near", "near_cells": "near"}
    peak = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    out = {}
    for k, v in kernels.items():
        if k not in units:
            continue
        t = v["us_per_launch"] * 1e-6
        flops = units[k] * FLOPS[kind[k]]
        achieved = flops / t / 1e12
        out[k] = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                  "traffic": traffic_of(traffic or {}, k, fp64), "units_per_launch": units[k],
                  "flops_per_unit": FLOPS[kind[k]], "us_per_launch": v["us_per_launch"], "launches": v["launches"]}
        if "us_alone" in v:
            a = flops / (v["us_alone"] * 1e-6) / 1e12
            out[k]["alone"] = {"us_per_launch": v["us_alone"], "achieved": a, "frac": a / peak}
        if rates and not fp64:
            f, tr = OPS[kind[k]]
            tb = units[k] * (f / rates["v_fma_f32"] + tr / rates["v_sin_f32"])
            out[k]["measured_rates"] = {"us_at_rates": tb * 1e6, "frac": tb / t,
                                        "fma_per_unit": f, "trans_per_unit": tr}
    return out


def dominant(rl):
    """The kernel with the largest time per step among those with a roofline."""
    if not rl:
        return None
    k = max(rl, key=lambda k: rl[k]["us_per_launch"] * rl[k]["launches"])
    return dict(rl[k], kernel=k)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, P):
    """The oracle on the host, on a bounded sample of the headline workload,
    scaled to particle-steps/s: one full near evaluation (cell list over all
    ions), the structure factor of P_s of the step's P wave vectors over all
    ions (scaled by P / P_s), and the far force of T sampled ions over all P
    wave vectors (scaled by N / T).  Once with every OpenMP thread, once with
    one thread on smaller samples (the near part on the same lattice
    generator's 136^3 system, whose per-ion cost is the same)."""
    import oracle
    from paper_2205_13824_amd import workloads as W

    sog = oracle.sog_row2(wl["rc"])
    pos, q, box, rc = wl["pos"], wl["q"], wl["box"], wl["rc"]
    n = len(q)
    S = oracle.S_product(sog, box)
    m = oracle.mh_sample(sog, box, seed=99, stream=0, n=P)[0]
    w = oracle.rb_weights(S, P, box, P)

    def sample(ps, t_targets, near_sys):
        rng = np.random.default_rng(5)
        t0 = time.perf_counter()
        oracle.near_cells(near_sys[0], near_sys[1], box if near_sys[2] is None else near_sys[2], rc, sog)
        t_near = (time.perf_counter() - t0) * (n / len(near_sys[1]))
        t0 = time.perf_counter()
        re, im = oracle.structure_factor(pos, q, box, m[:ps])
        t_rho = (time.perf_counter() - t0) * (P / ps)
        tg = np.sort(rng.choice(n, size=t_targets, replace=False))
        re_full = np.resize(re, P)
        im_full = np.resize(im, P)
        t0 = time.perf_counter()
        oracle.far_force(pos[tg], q[tg], box, m, w, re_full, im_full)
        t_far = (time.perf_counter() - t0) * (n / t_targets)
        tot = t_near + t_rho + t_far
        return {"value": n / tot, "seconds_per_step_estimated": tot,
                "parts_s": {"near": t_near, "rho": t_rho, "far": t_far}}

    threads = oracle.max_threads()
    t0 = time.perf_counter()
    allc = sample(40, 100_000, (pos, q, None))
    wall_all = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        small = W.ions_lattice(136, 0.1, seed=5)
        t0 = time.perf_counter()
        one = sample(2, 10_000, small)
        wall_one = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return {"value": allc["value"], "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{n}-ion headline system, FP64 oracle (C, OpenMP): one near evaluation over all ions, "
                      f"rho of 40 of the step's {P} wave vectors over all ions (x {P}/40), far force of "
                      f"100,000 sampled ions over all {P} (x N/1e5); velocity update omitted",
            "parts_s": allc["parts_s"], "seconds": wall_all,
            "one_core": {"value": one["value"], "unit": "particle-steps/s", "cores": 1, "parts_s": one["parts_s"],
                         "seconds": wall_one,
                         "sample": "one OpenMP thread: near evaluation of the same generator's 136^3-ion lattice "
                                   "(same density and jitter; x N/2.5e6), rho of 2 wave vectors over all ions "
                                   f"(x {P}/2), far force of 10,000 sampled ions (x N/1e4)"}}


def other_workloads(R, W, torch, args, near_pairs_c2=None):
    out = {}
    steps = args.other_steps
    # 300,000-ion electrolyte (RSA, P = 200): both precisions and the core-shell near table
    t0 = time.time()
    c2 = W.c2_electrolyte()
    log(f"[bench] 300k electrolyte built in {time.time() - t0:.1f} s")
    n2 = len(c2["q"])
    r32 = run_leg(R, torch, c2, R.RBSOG_FP32C, args, steps, autotune=not args.no_autotune, profile_steps=5)
    r64 = run_leg(R, torch, c2, R.RBSOG_FP64, args, steps, autotune=not args.no_autotune, profile_steps=5)
    r32t = run_leg(R, torch, c2, R.RBSOG_FP32C, args, steps, near_table=True, autotune=not args.no_autotune,
                   profile_steps=5)
    pairs2 = count_near_pairs(R, c2)
    rl2 = rooflines(r32["kernels"], n2, c2["P"], pairs2, False, traffic_table("electrolyte300k"))
    out["electrolyte_300k"] = {
        "workload": f"{n2}-ion +-1 electrolyte, density 0.1, RSA d_min=1, r_c=3.5, P={c2['P']}, velocity-Verlet",
        "fp32c": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "shapes": r32["shapes"]},
        "fp64": {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "shapes": r64["shapes"]},
        "fp32c_coreshell": {"value": r32t["value"], "ms_per_step": r32t["ms_per_step"],
                            "force_relrms_vs_fp64": relrms(r32t["F0"], r64["F0"])},
        "fp32c_force_relrms_vs_fp64": {"total": relrms(r32["F0"], r64["F0"]),
                                       "near": relrms(r32["Fn0"], r64["Fn0"]),
                                       "far": relrms(r32["Ff0"], r64["Ff0"])},
        "unit": "particle-steps/s", "steps": steps, "near_pairs": pairs2,
        "near_list": {"builds": r32["builds"], "skin_at_end": r32["skin_end"]},
        "roofline": dominant(rl2), "rooflines": rl2, "kernels_fp32c": r32["kernels"],
        "kernels_fp64": r64["kernels"]}
    del c2
    # 3e6 water sites (10^6 rigid 3-site molecules as point charges), r_c = 10, P = 500
    c3 = W.c3_water()
    n3 = len(c3["q"])
    w32 = run_leg(R, torch, c3, R.RBSOG_FP32C, args, 5, profile_steps=2)
    w32t = run_leg(R, torch, c3, R.RBSOG_FP32C, args, 5, near_table=True, profile_steps=2)
    w64 = run_leg(R, torch, c3, R.RBSOG_FP64, args, 5, profile_steps=2)
    near_us = {k: v["kernels"].get("near", v["kernels"].get("list_build", {})).get("us_per_launch")
               for k, v in (("fp32c", w32), ("fp32c_coreshell", w32t), ("fp64", w64))}
    out["water_3M"] = {
        "workload": f"{n3} water sites (10^6 SPC/E-shaped 3-site molecules), r_c=10, P=500, velocity-Verlet dt=1e-3",
        "fp32c": {"value": w32["value"], "ms_per_step": w32["ms_per_step"],
                  "force_relrms_vs_fp64": {"total": relrms(w32["F0"], w64["F0"]),
                                           "near": relrms(w32["Fn0"], w64["Fn0"]),
                                           "far": relrms(w32["Ff0"], w64["Ff0"])}},
        "fp32c_coreshell": {"value": w32t["value"], "ms_per_step": w32t["ms_per_step"],
                            "force_relrms_vs_fp64": {"total": relrms(w32t["F0"], w64["F0"]),
                                                     "near": relrms(w32t["Fn0"], w64["Fn0"])}},
        "fp64": {"value": w64["value"], "ms_per_step": w64["ms_per_step"]},
        "near_kernel_us_per_launch": near_us, "unit": "particle-steps/s", "steps": 5,
        "kernels_fp32c": w32["kernels"], "kernels_fp32c_coreshell": w32t["kernels"]}
    del c3
    # replica ensemble: 256 systems, log-uniform sizes 500..50000, P = 100, FP32C
    t0 = time.time()
    ens = W.c4_ensemble()
    sysl = ens["systems"]
    stream = torch.cuda.Stream()
    b = R.Batch([x["pos"] for x in sysl], [x["q"] for x in sysl], [x["box"] for x in sysl], ens["rc"], ens["P"],
                ens["seeds"], precision=R.RBSOG_FP32C, stream=stream.cuda_stream, device_chains=DEVICE_CHAINS)
    b.forces()
    if not args.no_autotune:
        R.rbsog_autotune(b.ctx, 3)
    R.rbsog_set_velocities(b.ctx, None, T=1.0, seed=7)
    b.step(args.warmup, DT)
    ms = timed_steps(torch, b, stream, steps)
    info = R.rbsog_info(b.ctx)
    out["ensemble_256"] = {"workload": f"256 replicas, {b.n} ions in all (500..50000 each, log-uniform), density "
                                       f"0.1, r_c=3.5, P=100, FP32C, velocity-Verlet",
                           "value": b.n * steps / (ms * 1e-3), "unit": "particle-steps/s", "steps": steps,
                           "ms_per_step": ms / steps, "setup_s": time.time() - t0,
                           "shapes": {k: info[k] for k in ("rho_chunk", "far_block", "rho_ktile", "build_slots", "cell_slots", "tuned")}}
    b.close()
    log(f"[bench] ensemble: {out['ensemble_256']['value']:.3e} particle-steps/s")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path would shard "
              f"by spatial domains with one all-reduce of rho per step, which this build does not run).",
              file=sys.stderr)
        sys.exit(2)
    # torch first: the library then runs on the HIP runtime torch has loaded,
    # so torch's streams and events are the library's
    import torch

    from paper_2205_13824_amd import rbsog as R
    from paper_2205_13824_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    t0 = time.time()
    gen, desc = WORKLOADS[args.workload]
    wl = getattr(W, gen)()
    n, P = len(wl["q"]), wl["P"]
    log(f"[bench] headline workload built in {time.time() - t0:.1f} s: n={n} L={wl['box'][0]:.4f} P={P}")

    # this device's issue rates (lane-instructions/s) for the measured-rate bounds
    rates = R.rbsog_probe_rates(0, 3)
    r32 = run_leg(R, torch, wl, R.RBSOG_FP32C, args, args.steps, autotune=not args.no_autotune)
    r64 = run_leg(R, torch, wl, R.RBSOG_FP64, args, args.steps, autotune=not args.no_autotune)
    err = {"total": relrms(r32["F0"], r64["F0"]), "near": relrms(r32["Fn0"], r64["Fn0"]),
           "far": relrms(r32["Ff0"], r64["Ff0"])}
    log(f"[bench] FP32C vs FP64 force relrms: {err}")
    pairs = count_near_pairs(R, wl)
    traffic = traffic_table(args.workload)
    rl32 = rooflines(r32["kernels"], n, P, pairs, False, traffic, rates)
    rl64 = rooflines(r64["kernels"], n, P, pairs, True, traffic, rates)
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n} {desc}, P={P}, Table 1 row 2, velocity-Verlet dt=1e-3 from a Maxwellian "
                               f"at T=1, wave vectors drawn on the device ({DEVICE_CHAINS} Metropolis-Hastings chains)",
                   "name": args.workload,
                   "n": n, "P": P, "rc": wl["rc"], "box": float(wl["box"][0])},
        "fp64": {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                 "roofline": dominant(rl64), "rooflines": rl64},
        "fp32c_speedup_vs_fp64": r32["value"] / r64["value"],
        "fp32c_force_relrms_vs_fp64": err,
        "energy_step0": {"fp32c": list(map(float, r32["E0"])), "fp64": list(map(float, r64["E0"]))},
        "roofline": dominant(rl32),
        "rooflines": rl32,
        "near_pairs": pairs,
        "measured_rates": {"unit": "lane-instructions/s", **rates},
        "near_list": {"builds": r32["builds"], "evaluations": 1 + args.warmup + args.steps,
                      "skin_at_end": r32["skin_end"]},
        "launch_shapes": {"fp32c": r32["shapes"], "fp64": r64["shapes"],
                          "tuning": {"fp32c": r32["tune"], "fp64": r64["tune"]}},
        "kernels_fp32c": r32["kernels"],
        "kernels_fp64": r64["kernels"],
        "kernels_fp32c_build_steps": r32["build_step"],
        "setup_s": {"fp32c": r32["setup_s"], "fp64": r64["setup_s"]},
    }
    if not args.no_cpu_baseline and args.workload == "ions20M":
        out["cpu_baseline"] = cpu_baseline(wl, P)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3e} particle-steps/s")
    del wl
    if not args.no_other:
        out["other_workloads"] = other_workloads(R, W, torch, args)
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
