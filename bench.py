#!/usr/bin/env python3
"""Throughput of the Lees-Edwards shear-flow MD step on one MI355X.

Workload (default): LJ fluid, N = 256,000 particles on 256,000 of the sites
of a 64^3 simple-cubic lattice (seeded choice, jitter U(-0.05, 0.05)), density 0.8442, cutoff 2.5, T = 1, Langevin
gamma = 1 on the peculiar velocity, shear rate 0.1 (flow x, gradient y),
dt = 0.005, skin 0.3, float64, shear stress sampled every 10 steps.  One
"step" is a full pass of the hot path: offset, rebuild test (and rebuild when
due: crossing/wrap, sort, Lees-Edwards stencil, neighbour lists), pair forces,
Langevin force, velocity Verlet, stress sample.

Prints ONE JSON line.  `value` is particle-steps/s with the state resident in
HBM.  The roofline entry is for the dominant kernel (the fused force /
thermostat / integrator kernel), timed with HIP events on the simulation's
stream during the timed region.  The CPU baseline is the FP64 oracle
(oracle/) on a bounded sample of the same workload, single thread.
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

METRIC = "particle-steps/s per GPU + p50/p99 sweep latency; mixed vs FP64 at viscosity tol"
PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 vector (also the unpacked FP32 vector rate)
PEAK_HBM_GBS = 8000.0
PAIR_FLOPS = 26.0             # per in-cutoff pair, counted once per unordered pair
STEP_FLOPS = 40.0             # thermostat + velocity Verlet per particle
BYTES_FUSED = 100.0           # fused step, per particle: read x, u, tag; write x, u
TIMING_FORCE = 0x1 | (8 << 8)  # event-time every 8th plain-step force launch (phase 0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# friction per thermostat on the LJ fluid (the paper's xi = 1 Langevin, xi_DPD = 5)
LJ_GAMMA = {"langevin": 1.0, "langevin_abs": 1.0, "dpd": 5.0}
DPD_PAIR_FLOPS = 30.0         # DPD dissipative + random pair terms (Philox is integer work)


def lj_params(n, shear_rate, precision, seed=21, skin=0.3, thermostat="langevin"):
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.sim import Params
    w = inputs.lj_workload(n=n, shear_rate=shear_rate, seed=seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=shear_rate, seed=seed, skin=skin,
               precision=precision, rc=2.5, dt=0.005, kT=1.0, gamma=LJ_GAMMA[thermostat],
               thermostat=thermostat)
    return w, p


KG_CHAINS, KG_LEN = 2000, 200


def kg_params(shear_rate, precision, seed=31, skin=0.3, n_chains=KG_CHAINS, chain_len=KG_LEN):
    """Kremer-Grest melt: WCA + FENE(30, 1.5), density 0.85, T=1, gamma=0.5, dt=0.01,
    overlap-free lattice-path start (stands in for the warmed-up random-walk melt)."""
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.sim import Params
    w = inputs.kg_workload(n_chains, chain_len, shear_rate=shear_rate, seed=seed, layout="snake")
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=shear_rate, seed=seed, skin=skin,
               precision=precision, rc=2.0 ** (1.0 / 6.0), pair="wca", n_chains=n_chains,
               chain_len=chain_len, dt=0.01, kT=1.0, gamma=0.5)
    return w, p


def pick_skin(n, shear_rate, precision, workload, thermostat="langevin"):
    """Autotuned skin for a workload (short bursts; see paper_2109_11083_amd.tune)."""
    from paper_2109_11083_amd.tune import autotune
    if workload == "kg":
        w, p = kg_params(shear_rate, precision)
    else:
        w, p = lj_params(n, shear_rate, precision, thermostat=thermostat)
    best, table = autotune(p, w.x, w.u)
    return best.skin, [dict(skin=a, tune=b, value=round(c, 1)) for a, b, c in table]


def run_gpu(n, shear_rate, precision, steps, warmup, sample_every=10, timing=TIMING_FORCE, skin=0.3,
            workload="lj", thermostat="langevin"):
    """One timed run.  timing: le_timing_enable mask for HIP-event timing inside the
    timed region (bit 0: the plain-step force kernel; 0xF: every phase; bits 8..: stride)."""
    import torch
    from paper_2109_11083_amd import binding as B
    from paper_2109_11083_amd.sim import Sim
    if workload == "kg":
        w, p = kg_params(shear_rate, precision, skin=skin)
    else:
        w, p = lj_params(n, shear_rate, precision, skin=skin, thermostat=thermostat)
    sim = Sim(p, w.x, w.u, step0=0)
    ring = torch.zeros((max(steps // sample_every, 1), 6), dtype=torch.float64, device="cuda")
    if warmup > 0:
        wring = torch.zeros((max(warmup // sample_every, 1), 6), dtype=torch.float64, device="cuda")
        sim.step(warmup, sample_every=sample_every, ring=wring)
    sim.sync()
    st0 = sim.stats()
    B.le_timing_enable(sim.handle, timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, sample_every=sample_every, ring=ring)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = B.le_timing_read(sim.handle)
    st1 = sim.stats()
    sig = ring.cpu().numpy()
    # steady-state window: the second half of the timed steps (25 tau at 10,000
    # steps of dt 0.005), ten blocks of 2.5 tau, much longer than the decay of
    # the shear-stress correlations, for the standard error
    tail = sig[int(0.5 * len(sig)):]
    eta = float(tail[:, 3].mean() / shear_rate) if shear_rate != 0 else None
    eta_se = None
    if len(tail) >= 20:
        blocks = tail[: len(tail) // 10 * 10, 3].reshape(10, -1).mean(axis=1) / shear_rate
        eta_se = float(blocks.std(ddof=1) / math.sqrt(10))
    prof = sim.observables(50)
    out = dict(n=p.n, seconds=t1 - t0, steps=steps, value=p.n * steps / (t1 - t0),
               ms_per_step=1e3 * (t1 - t0) / steps, phases=phases,
               rebuilds=st1["rebuilds"] - st0["rebuilds"], max_neighbors=st1["max_neighbors"],
               eta=eta, eta_se=eta_se, box=p.box, rc=p.rc,
               ux_profile=[float(v) for v in prof["sum_ux"] / prof["count"]], kT=prof["kT"])
    sim.close()
    return out


def copy_probe(mib=1024, reps=5):
    """Plain device-to-device copy of a known size (calibrates HBM byte counters)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": reps}),
          flush=True)


def serving_bench(count=64):
    """Sweep requests (N ~ U{2000..64000}, shear rate log-uniform in [1e-3, 1], 5000 steps,
    Poisson arrivals at 4/s): continuous batching in mixed precision against FP64 one request at a
    time (FIFO), on the same trace; plus the same requests all at once (sweep throughput)."""
    from paper_2109_11083_amd.serve import Server, sweep_trace
    out = {}
    runs = [("batched_mixed", "mixed", 16, False), ("fifo_fp64", "fp64", 1, False),
            ("batched_mixed_burst", "mixed", 16, True), ("fifo_fp64_burst", "fp64", 1, True)]
    etas, ses = {}, {}
    for name, prec, slots, burst in runs:
        trace = sweep_trace(count=count, precision=prec, burst=burst)
        res, summ = Server(max_active=slots).run(trace, realtime=not burst)
        etas[name] = np.array([r.eta for r in res])
        ses[name] = np.array([r.eta_se if r.eta_se is not None else np.nan for r in res])
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"bench: serving {name}: p50 {summ['p50_s']:.3f} s p99 {summ['p99_s']:.3f} s "
            f"throughput {summ['throughput']:.3e} particle-steps/s")
    d = np.abs(etas["batched_mixed"] - etas["fifo_fp64"])
    z = d / np.hypot(ses["batched_mixed"], ses["fifo_fp64"])
    z = z[np.isfinite(z)]
    out["eta_mixed_vs_fp64"] = dict(median_abs_diff=float(np.median(d)), max_abs_diff=float(d.max()),
                                    median_diff_in_se=float(np.median(z)) if len(z) else None,
                                    frac_within_2se=float((z <= 2.0).mean()) if len(z) else None,
                                    frac_within_3se=float((z <= 3.0).mean()) if len(z) else None,
                                    note="per request, 5000 steps, eta over the second half with its "
                                         "10-block standard error; the two runs of a request are "
                                         "independent trajectories, so the differences are statistical")
    out["trace"] = dict(requests=count, n="U{2000..64000}", shear_rate="log-U[1e-3, 1]", steps=5000,
                        arrivals="Poisson 4/s (burst: all at t=0)", skin=0.4)
    return out


def cpu_baseline(n, shear_rate, nsteps, thermostat="langevin", workload="lj"):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    if workload == "kg":
        w, p = kg_params(shear_rate, "fp64")
        what = f"{p.n_chains} x {p.chain_len} Kremer-Grest melt"
    else:
        w, p = lj_params(n, shear_rate, "fp64", thermostat=thermostat)
        what = f"{p.n}-particle LJ system"
    op = O.make_params(p.n, p.box, shear_rate=p.shear_rate, dt=p.dt, kT=p.kT, gamma=p.gamma,
                       rc=p.rc, fene_k=p.fene_k, fene_r0=p.fene_r0, seed=p.seed,
                       chain_len=p.chain_len, n_chains=p.n_chains, thermostat=thermostat)
    sim = O.Sim(w.x, w.u, op, step0=0, method=1)
    t0 = time.perf_counter()
    sim.run(nsteps)
    t1 = time.perf_counter()
    return dict(value=p.n * nsteps / (t1 - t0), unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{nsteps} steps of the same {what} (FP64 cell-list oracle, "
                       f"1 thread, {t1 - t0:.1f} s)")


def kernel_hash():
    """Hash of the kernel source: le_kernels.hip followed by le_internal.h (its
    compile-time tile and halo sizes)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("le_kernels.hip", "le_internal.h"):
        with open(os.path.join(ROOT, "paper_2109_11083_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(name, skin):
    """HBM bytes per launch of a kernel from a committed rocprofv3 PMC summary
    (profiles/<name>.md), or None if it was taken on another kernel source or
    at another skin (other list lengths, other traffic)."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256 prefix") != kernel_hash():
        return None
    try:
        if abs(float(vals["skin"]) - float(skin)) > 1e-9:
            return None
    except (KeyError, ValueError):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--shear-rate", type=float, default=None,
                    help="default 0.1 (LJ) / 0.01 (KG)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--n", type=int, default=256000,
                    help="LJ particles: n sites of a ceil(n^(1/3))^3 lattice (256000 -> 64^3)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps of the CPU baseline (default 12 for LJ, 40 for the KG melt: 10-20 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="no HIP events in the timed region (then no per-kernel roofline)")
    ap.add_argument("--skin", default="auto",
                    help="neighbour-list skin, or 'auto' (autotuned per workload, short bursts)")
    ap.add_argument("--workload", default="lj", choices=["lj", "kg"],
                    help="lj: 256,000-particle LJ fluid (the headline); kg: 2000 x 200 Kremer-Grest melt")
    ap.add_argument("--thermostat", default="langevin", choices=["langevin", "dpd", "langevin_abs"],
                    help="LJ workload: Langevin on the peculiar velocity (gamma 1), DPD (gamma 5) or "
                         "Langevin on the lab velocity (gamma 1)")
    ap.add_argument("--serve", action=argparse.BooleanOptionalAction, default=True,
                    help="shear-rate sweep serving: p50/p99 time-to-result and sweep throughput")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (byte-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU decomposition is a design, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        copy_probe()
        return
    kg = args.workload == "kg"
    sr = args.shear_rate if args.shear_rate is not None else (0.01 if kg else 0.1)

    tune_table = None
    th = "langevin" if kg else args.thermostat
    dpd = th == "dpd"
    if args.skin == "auto":
        skin, tune_table = pick_skin(args.n, sr, args.precision, args.workload, thermostat=th)
        log(f"bench: autotuned skin {skin}: {tune_table}")
    else:
        skin = float(args.skin)
    args.skin = skin
    size = f"{KG_CHAINS}x{KG_LEN}" if kg else f"n={args.n}"
    log(f"bench: {args.workload} {size} shear_rate={sr} {args.precision} "
        f"steps={args.steps} warmup={args.warmup} skin={skin}")
    r = run_gpu(args.n, sr, args.precision, args.steps, args.warmup,
                timing=0 if args.no_timing else TIMING_FORCE, skin=args.skin, workload=args.workload,
                thermostat=th)
    log(f"bench: {r['value']:.4e} particle-steps/s, {r['ms_per_step']:.4f} ms/step, "
        f"rebuilds={r['rebuilds']}, force={r['phases']['force']}")

    # roofline of the dominant kernel: the fused force / thermostat / integrator
    # kernel of plain steps (timing phase 0), from its event-timed average over
    # every 8th launch of the timed region
    force_ms, force_n = r["phases"]["force"]
    roofline = None
    kname = ("k_force_kg400k_" if kg else ("k_force_dpd_lj256k_" if dpd else "k_force_lj256k_")) + args.precision
    if force_n > 0:
        avg_s = force_ms / 1e3 / force_n
        traffic = read_traffic(kname + "_traffic", args.skin)
        if kg:
            # HBM-bound: algorithmic bytes of the fused step per particle
            achieved = r["n"] * BYTES_FUSED / avg_s / 1e9
            roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                            frac=round(achieved / PEAK_HBM_GBS, 5), traffic=traffic,
                            bytes_per_particle=BYTES_FUSED)
        else:
            rho = r["n"] / (r["box"][0] * r["box"][1] * r["box"][2])
            pairs_pp = 4.0 / 3.0 * math.pi * r["rc"] ** 3 * rho
            flops_pp = (PAIR_FLOPS + (DPD_PAIR_FLOPS if dpd else 0.0)) * pairs_pp / 2.0 + STEP_FLOPS
            achieved = r["n"] * flops_pp / avg_s / 1e12
            roofline = dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP64_TFLOPS,
                            unit="TFLOP/s", frac=round(achieved / PEAK_FP64_TFLOPS, 5), traffic=traffic,
                            flops_per_particle=round(flops_pp, 1))
        roofline.update(kernel=("k_force<kDpdForce> (LJ + DPD pair terms; the kicks and drift follow in "
                                "k_integrate), plain steps") if dpd else
                        "k_force (fused pair force + Langevin + velocity Verlet), plain steps",
                        avg_kernel_us=round(avg_s * 1e6, 3), launches=force_n,
                        hbm_GBs_if_traffic=(round(traffic / avg_s / 1e9, 1) if traffic else None))

    extra = {}
    # per-phase device time of the same workload (all phases event-timed; a separate, shorter run)
    b = run_gpu(args.n, sr, args.precision, min(args.steps, 2000), 100, timing=0xF, skin=args.skin,
                workload=args.workload, thermostat=th)
    extra["phase_us_per_step"] = {k: round(1e3 * v[0] / b["steps"], 2) for k, v in b["phases"].items()}
    log(f"bench: phases {extra['phase_us_per_step']}")
    if not args.no_extra and not dpd:
        if not kg:
            for sr2 in (0.01, 1.0):
                e = run_gpu(args.n, sr2, args.precision, 2000, 100, skin=args.skin)
                extra[f"lj_shear_rate_{sr2}"] = dict(value=e["value"],
                                                    rebuilds_per_1000=1000 * e["rebuilds"] / 2000,
                                                    eta=e["eta"])
                log(f"bench: shear_rate={sr2}: {e['value']:.4e} p-steps/s rebuilds={e['rebuilds']}")
        # the other precision on the same workload: throughput and viscosity with its error bar
        other = "mixed" if args.precision == "fp64" else "fp64"
        m = run_gpu(args.n, sr, other, args.steps, args.warmup, skin=args.skin, workload=args.workload)
        fm, fn = m["phases"]["force"]
        extra[f"{args.workload}_{other}"] = dict(
            value=m["value"], force_kernel_us=1e3 * fm / max(fn, 1), eta=m["eta"], eta_se=m["eta_se"],
            eta_diff_vs_main=(m["eta"] - r["eta"]) if (r["eta"] is not None and m["eta"] is not None)
            else None,
            eta_diff_in_se=(abs(m["eta"] - r["eta"]) / math.hypot(m["eta_se"], r["eta_se"])
                            if (m["eta_se"] and r["eta_se"]) else None))
        log(f"bench: {other}: {m['value']:.4e} p-steps/s eta={m['eta']}")
        if not kg:
            # Kremer-Grest melt, 2000 chains x 200 beads (HBM-bound pair kernel)
            kskin, _ = pick_skin(0, 0.01, args.precision, "kg")
            k = run_gpu(0, 0.01, args.precision, 2000, 100, skin=kskin, workload="kg")
            kf, kn = k["phases"]["force"]
            kus = 1e3 * kf / max(kn, 1)
            extra["kg_2000x200"] = dict(value=k["value"], force_kernel_us=kus,
                                        force_kernel_GBs_algorithmic=k["n"] * BYTES_FUSED / (kus * 1e-6) / 1e9,
                                        rebuilds_per_1000=1000 * k["rebuilds"] / 2000, shear_rate=0.01,
                                        skin=kskin)
            log(f"bench: kg: {k['value']:.4e} p-steps/s force {kus:.1f} us")

    if args.serve and not kg and th == "langevin":
        extra["serving"] = serving_bench(args.serve_requests)

    cpu = None
    if not args.no_cpu_baseline:
        cpu_steps = args.cpu_steps if args.cpu_steps else (40 if kg else 12)
        cpu = cpu_baseline(args.n, sr, cpu_steps, thermostat=th, workload=args.workload)
        log(f"bench: cpu oracle {cpu['value']:.4e} particle-steps/s")

    if kg:
        wl = (f"Kremer-Grest melt {KG_CHAINS} chains x {KG_LEN} beads (N={r['n']}), density 0.85, "
              f"WCA + FENE(30, 1.5), T=1, Langevin gamma=0.5 on peculiar velocity, shear_rate={sr}, "
              f"dt=0.01, skin {args.skin}, {args.precision}; overlap-free lattice-path start")
    else:
        tdesc = {"langevin": "Langevin gamma=1 on peculiar velocity",
                 "langevin_abs": "Langevin gamma=1 on lab velocity",
                 "dpd": "DPD gamma=5, r_c 2.5"}[th]
        wl = (f"LJ fluid N={r['n']} (64^3 lattice sites, N chosen), density 0.8442, rc 2.5, "
              f"T=1, {tdesc}, shear_rate={sr}, "
              f"dt=0.005, skin {args.skin}, {args.precision}")
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": wl,
            "n_particles": r["n"],
            "shear_rate": sr,
            "precision": args.precision,
            "stress_sample_every": 10,
            "skin": args.skin,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rebuilds_per_1000_steps": round(1000.0 * r["rebuilds"] / args.steps, 2),
        "skin_autotune": tune_table,
        "viscosity": {"eta": r["eta"], "block_se": r["eta_se"],
                      "window": "second half of the timed steps, 10 blocks"},
        "ux_profile_50_bins": [round(v, 5) for v in r["ux_profile"]],
        "kT_kinetic": r["kT"],
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
