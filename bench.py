#!/usr/bin/env python3
"""Throughput of the Lees-Edwards shear-flow MD step on one MI355X.

Headline workload: the Kremer-Grest melt of 2000 linear chains x 200 beads
(N = 400,000), built as random walks of bond 0.97 (non-reversal) at density
0.85, WCA (r_c 2^(1/6)) + FENE (K 30, R0 1.5), kT 1, Langevin gamma 0.5 on
the peculiar velocity, dt 0.01, shear rate 0.01 (flow x, gradient y), FP64,
shear stress sampled every 10 steps.  Before the timed region the overlapping
random-walk start is warmed up without shear with capped pair forces until
the largest force is below 10^3 (paper Section 2.4: systems are equilibrated
before shear); the list skin is autotuned on the warmed state.  One "step" is
a full pass of the hot path: offset, rebuild test (and rebuild when due:
crossing/wrap, sort, Lees-Edwards stencil, neighbour lists), pair + bond
forces, Langevin force, velocity Verlet, stress sample.

Prints ONE JSON line.  `value` is particle-steps/s with the state resident in
HBM.  The roofline entry is for the dominant kernel (the fused force /
thermostat / integrator kernel), timed with HIP events on the simulation's
stream during the timed region.  The CPU baseline is the FP64 oracle
(oracle/, its OpenMP timing build on all host cores) on a bounded sample of
the same workload.  Extras: the 256,000-particle LJ fluid (throughput, force
kernel roofline, three shear rates), its viscosity in FP64 and mixed
precision from fixed-length runs, the KG melt's viscosity at two shear rates
in both precisions, the shear-rate sweep serving trace, and the oracle on
every configuration with one thread and with all cores.
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

ETA_STEPS = 25000             # fixed length of each viscosity run (independent of --steps)
ETA_WARMUP = 2000
ETA_WINDOW = 0.2              # last 20% of the samples (Fig. profile caption)

LJ_GAMMA = {"langevin": 1.0, "langevin_abs": 1.0, "dpd": 5.0}
DPD_PAIR_FLOPS = 30.0         # DPD dissipative + random pair terms (Philox is integer work)
KG_CHAINS, KG_LEN = 2000, 200


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ workloads
def lj_params(n, shear_rate, precision, seed=21, skin=0.3, thermostat="langevin"):
    """LJ fluid: n of the sites of a ceil(n^(1/3))^3 lattice, density 0.8442, r_c 2.5."""
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.sim import Params
    w = inputs.lj_workload(n=n, shear_rate=shear_rate, seed=seed)
    p = Params(n=w.x.shape[1], box=w.box, shear_rate=shear_rate, seed=seed, skin=skin,
               precision=precision, rc=2.5, dt=0.005, kT=1.0, gamma=LJ_GAMMA[thermostat],
               thermostat=thermostat)
    return w.x, w.u, p


def kg_params(shear_rate, precision, skin=0.3, seed=31):
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.sim import Params
    L = inputs.box_for(KG_CHAINS * KG_LEN, inputs.KG_DENSITY)
    return Params(n=KG_CHAINS * KG_LEN, box=(L, L, L), shear_rate=shear_rate, seed=seed, skin=skin,
                  precision=precision, rc=2.0 ** (1.0 / 6.0), pair="wca", n_chains=KG_CHAINS,
                  chain_len=KG_LEN, dt=0.01, kT=1.0, gamma=0.5)


_KG_WARM = {}


def kg_state(shear_rate, seed=31):
    """The warmed random-walk melt (warm-up once per process, on the GPU, untimed),
    with the streaming profile of `shear_rate` added to its thermal velocities."""
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.warmup import warm_up
    if seed not in _KG_WARM:
        w = inputs.kg_workload(KG_CHAINS, KG_LEN, shear_rate=0.0, seed=seed, layout="walk")
        t0 = time.perf_counter()
        x, c, info = warm_up(kg_params(0.0, "fp64", seed=seed), w.x, w.u)
        log(f"bench: KG warm-up {info.steps} steps in {time.perf_counter() - t0:.1f} s, "
            f"max force {info.max_force:.1f}")
        _KG_WARM[seed] = (x, c, info)
    x, c, info = _KG_WARM[seed]
    u = inputs.streaming_initial_velocity(x, c, shear_rate, kg_params(0.0, "fp64").box[1])
    return x, u, info


def workload(name, shear_rate, precision, skin=0.3, n=256000, thermostat="langevin"):
    """(x, u, Params) of a named workload; skin may be a (skin, pair layout) pair."""
    import dataclasses
    skin, tune = skin if isinstance(skin, tuple) else (skin, 0)
    if name == "kg":
        x, u, _ = kg_state(shear_rate)
        return x, u, dataclasses.replace(kg_params(shear_rate, precision, skin=skin), tune=tune)
    x, u, p = lj_params(n, shear_rate, precision, skin=skin, thermostat=thermostat)
    return x, u, dataclasses.replace(p, tune=tune)


def pick_skin(name, shear_rate, precision, n=256000, thermostat="langevin"):
    """Autotuned skin and pair layout (short bursts of the cell-filling skins with the
    LDS-halo and the global-memory layouts; paper_2109_11083_amd.tune)."""
    from paper_2109_11083_amd.tune import autotune
    x, u, p = workload(name, shear_rate, precision, n=n, thermostat=thermostat)
    tunes = (2,) if thermostat == "dpd" else (1, 2)
    best, table = autotune(p, x, u, tunes=tunes)
    return (best.skin, best.tune), [dict(skin=a, tune=b, value=round(c, 1)) for a, b, c in table]


# ------------------------------------------------------------------ one timed run
def eta_of(sig, shear_rate, window=ETA_WINDOW):
    """Viscosity (Eq. viscosity) over the last `window` of the samples, with the
    standard error of 10 block means."""
    if shear_rate == 0 or len(sig) == 0:
        return None, None
    tail = sig[int(round((1.0 - window) * len(sig))):]
    if len(tail) == 0:
        return None, None
    eta = float(tail[:, 3].mean() / shear_rate)
    se = None
    if len(tail) >= 20:
        blocks = tail[: len(tail) // 10 * 10, 3].reshape(10, -1).mean(axis=1) / shear_rate
        se = float(blocks.std(ddof=1) / math.sqrt(10))
    return eta, se


def run_gpu(x, u, p, steps, warmup, sample_every=10, timing=TIMING_FORCE):
    """One timed run.  timing: le_timing_enable mask for HIP-event timing inside the
    timed region (bit 0: the plain-step force kernel; 0xF: every phase; bits 8..: stride)."""
    import torch
    from paper_2109_11083_amd import binding as B
    from paper_2109_11083_amd.sim import Sim
    sim = Sim(p, x, u, step0=0)
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
    sig = ring.cpu().numpy()[: steps // sample_every]
    eta, eta_se = eta_of(sig, p.shear_rate)
    prof = sim.observables(50)
    out = dict(n=p.n, seconds=t1 - t0, steps=steps, value=p.n * steps / (t1 - t0),
               ms_per_step=1e3 * (t1 - t0) / steps, phases=phases,
               rebuilds=st1["rebuilds"] - st0["rebuilds"], max_neighbors=st1["max_neighbors"],
               eta=eta, eta_se=eta_se, box=p.box, rc=p.rc,
               ux_profile=[float(v) for v in prof["sum_ux"] / np.maximum(prof["count"], 1)],
               kT=prof["kT"])
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


# ------------------------------------------------------------------ roofline
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
    (profiles/<name>.md: one `hbm_bytes_per_launch@<skin>` line per profiled skin),
    or None if it was taken on another kernel source or at another skin (other
    list lengths, other traffic)."""
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
    for k, v in vals.items():
        if k.startswith("hbm_bytes_per_launch@"):
            try:
                if abs(float(k.split("@", 1)[1]) - float(skin)) <= 1e-6:
                    return float(v)
            except ValueError:
                continue
    return None


def roofline_of(r, kind, precision, skin, dpd=False):
    """Roofline entry of the fused force kernel of run r (event-timed plain steps)."""
    force_ms, force_n = r["phases"]["force"]
    if force_n == 0:
        return None
    avg_s = force_ms / 1e3 / force_n
    if kind == "kg":
        name = "k_force_kg400k_" + precision
        traffic = read_traffic(name + "_traffic", skin)
        achieved = r["n"] * BYTES_FUSED / avg_s / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 5), traffic=traffic,
                    bytes_per_particle=BYTES_FUSED,
                    kernel="k_force (fused WCA + FENE force, Langevin, velocity Verlet), plain steps")
    else:
        name = ("k_force_dpd_lj256k_" if dpd else "k_force_lj256k_") + precision
        traffic = read_traffic(name + "_traffic", skin)
        rho = r["n"] / (r["box"][0] * r["box"][1] * r["box"][2])
        pairs_pp = 4.0 / 3.0 * math.pi * r["rc"] ** 3 * rho
        flops_pp = (PAIR_FLOPS + (DPD_PAIR_FLOPS if dpd else 0.0)) * pairs_pp / 2.0 + STEP_FLOPS
        achieved = r["n"] * flops_pp / avg_s / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP64_TFLOPS, 5), traffic=traffic,
                    flops_per_particle=round(flops_pp, 1),
                    kernel=("k_force_dpd (LJ + DPD pair terms; the kicks and drift follow in "
                            "k_integrate), plain steps") if dpd else
                    "k_force (fused LJ force, Langevin, velocity Verlet), plain steps")
    roof.update(avg_kernel_us=round(avg_s * 1e6, 3), launches=force_n,
                hbm_GBs_if_traffic=(round(traffic / avg_s / 1e9, 1) if traffic else None))
    return roof


# ------------------------------------------------------------------ legs
def viscosity_pair(name, shear_rate, skin, steps=ETA_STEPS, warmup=ETA_WARMUP, dt=None):
    """FP64 and mixed runs of the same start, fixed length: eta +- block SE each,
    their difference in units of the combined error, and the throughputs
    (dt: the workload's own time step unless given)."""
    import dataclasses
    out = {}
    for prec in ("fp64", "mixed"):
        x, u, p = workload(name, shear_rate, prec, skin=skin)
        if dt is not None:
            p = dataclasses.replace(p, dt=dt)
        out["dt"] = p.dt
        r = run_gpu(x, u, p, steps, warmup)
        out[prec] = dict(eta=r["eta"], eta_se=r["eta_se"], value=r["value"],
                         force_kernel_us=1e3 * r["phases"]["force"][0] / max(r["phases"]["force"][1], 1))
        log(f"bench: {name} shear_rate={shear_rate} {prec}: eta={r['eta']:.4f} +- {r['eta_se']:.4f} "
            f"{r['value']:.4e} p-steps/s")
    a, b = out["fp64"], out["mixed"]
    out["eta_diff"] = b["eta"] - a["eta"]
    out["eta_diff_in_se"] = abs(b["eta"] - a["eta"]) / math.hypot(a["eta_se"], b["eta_se"])
    out["mixed_speedup"] = b["value"] / a["value"]
    out["window"] = (f"{steps} timed steps after {warmup}, stress every 10 steps, eta over the last "
                     f"{int(ETA_WINDOW * 100)}% of the samples, standard error of 10 block means")
    return out


def serving_bench(count=64):
    """Sweep requests (N ~ U{2000..64000}, shear rate log-uniform in [1e-3, 1], 5000 steps,
    Poisson arrivals at 4/s): continuous batching through le_step_batch in mixed precision
    against FP64 one request at a time (FIFO) on the same trace; then all requests at once
    (sweep throughput), batched in both precisions and FIFO.  The cell size and pair
    layout of the requests come from the batch autotuner on the first 8 requests."""
    from paper_2109_11083_amd.serve import Server, request_params, sweep_trace
    from paper_2109_11083_amd.tune import autotune_batch
    probe = [request_params(r) for r in sweep_trace(count=8, precision="mixed", burst=True)]
    (skin, tune), table = autotune_batch([(w.x, w.u, p) for w, p in probe])
    log(f"bench: serving autotune: skin {skin} tune {tune}: "
        f"{[(a, b, round(c / 1e9, 3)) for a, b, c in table]}")
    out = dict(autotune=dict(skin=skin, tune=tune,
                             table=[dict(skin=a, tune=b, value=round(c, 1)) for a, b, c in table]))
    runs = [("batched_mixed", "mixed", "batched", 64, False), ("fifo_fp64", "fp64", "streams", 1, False),
            ("batched_mixed_burst", "mixed", "batched", 64, True),
            ("batched_fp64_burst", "fp64", "batched", 64, True),
            ("fifo_fp64_burst", "fp64", "streams", 1, True)]
    etas, ses = {}, {}
    for name, prec, mode, slots, burst in runs:
        trace = sweep_trace(count=count, precision=prec, burst=burst, skin=skin, tune=tune)
        res, summ = Server(max_active=slots, mode=mode).run(trace, realtime=not burst)
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
    out["speedup_burst_batched_mixed_vs_fifo_fp64"] = (out["batched_mixed_burst"]["throughput"]
                                                       / out["fifo_fp64_burst"]["throughput"])
    out["trace"] = dict(requests=count, n="U{2000..64000}", shear_rate="log-U[1e-3, 1]", steps=5000,
                        arrivals="Poisson 4/s (burst: all at t=0)", skin=f"cell-filling skin of {skin}",
                        tune=tune, batched="le_step_batch chunks of 500 steps (batch graphs)",
                        fifo="one simulation at a time, le_step chunks (single graphs)")
    return out


def c5_sweep(scale=0.1, steps=30000, warmup=1000, seed=51, dt=0.005):
    """The mixed-precision batched sweep: 16 Kremer-Grest melts (chains ~ U{500..2000} x scale,
    lengths ~ U{100..400}, density 0.85, WCA + FENE, random walks warmed up together with
    capped forces), shear rate 10^(-4 + 3k/15) for melt k, advanced as ONE batch
    (le_step_batch) in FP64 and again in mixed precision from the same warmed states.
    Reports both batch throughputs and, per melt, eta +- block SE in each precision with
    their difference in combined standard errors (the FP64 path is the reference: the
    oracle checks it on short windows, and no CPU run reaches these lengths).  dt = 0.005: at
    0.01 the gamma_dot = 0.1 melt of the longest chains stretches a FENE bond past R0 after
    ~1.1e4 steps, in either precision; at 0.005 every melt runs 3e4 steps.  A member that
    still latches an error is reported and left out of the comparison."""
    import dataclasses
    import torch
    from paper_2109_11083_amd import inputs
    from paper_2109_11083_amd.sim import Params, Sim, step_batch
    from paper_2109_11083_amd.tune import autotune_batch, filling_skin
    from paper_2109_11083_amd.warmup import warm_up_many
    rng = np.random.default_rng(seed)
    melts = []
    for k in range(16):
        nc = max(2, int(round(int(rng.integers(500, 2001)) * scale)))
        cl = int(rng.integers(100, 401))
        sr = 10.0 ** (-4.0 + 3.0 * k / 15.0)
        w = inputs.kg_workload(nc, cl, shear_rate=0.0, seed=seed * 100 + k, layout="walk")
        p = Params(n=w.x.shape[1], box=w.box, shear_rate=sr, seed=seed * 100 + k, rc=2.0 ** (1.0 / 6.0),
                   pair="wca", n_chains=nc, chain_len=cl, dt=dt, kT=1.0, gamma=0.5)
        melts.append((p, w.x, w.u))
    t0 = time.perf_counter()
    warmed = warm_up_many(melts)
    log(f"bench: c5 warm-up of 16 melts ({sum(p.n for p, _, _ in melts)} beads) in "
        f"{time.perf_counter() - t0:.1f} s")
    states = []
    for (p, _, _), (x, c, _) in zip(melts, warmed):
        states.append((x, inputs.streaming_initial_velocity(x, c, p.shear_rate, p.box[1]), p))
    (skin, tune), table = autotune_batch(states, skins=(0.4, 0.5, 0.6, 0.8), tunes=(2,), steps=300)
    log(f"bench: c5 batch autotune skin {skin}: {[(a, round(v / 1e9, 3)) for a, _, v in table]}")
    out = dict(melts=[], skin=skin, tune=tune, steps=steps, warmup=warmup)
    etas = {}
    for prec in ("fp64", "mixed"):
        stream = torch.cuda.Stream()
        sims = []
        for x, u, p in states:
            f = filling_skin(p, skin)
            sims.append(Sim(dataclasses.replace(p, precision=prec, skin=f if f else skin, tune=tune), x, u,
                            stream=stream))
        step_batch(sims, warmup)
        stream.synchronize()
        t0 = time.perf_counter()
        rings = step_batch(sims, steps, sample_every=10)
        stream.synchronize()
        t1 = time.perf_counter()
        failed = {}
        for k, s in enumerate(sims):
            try:
                s.sync()
            except Exception as exc:  # noqa: BLE001 - a latched device error of one melt
                failed[k] = str(exc)
        out[f"failed_{prec}"] = failed
        ntot = sum(s.params.n for s in sims)
        out[f"throughput_{prec}"] = ntot * steps / (t1 - t0)
        etas[prec] = [eta_of(r.cpu().numpy(), s.params.shear_rate) if k not in failed else (None, None)
                      for k, (r, s) in enumerate(zip(rings, sims))]
        for s in sims:
            s.close()
        log(f"bench: c5 batch {prec}: {ntot} beads, {out[f'throughput_{prec}']:.4e} p-steps/s")
    zs = []
    for k, (x, u, p) in enumerate(states):
        (e64, s64), (e32, s32) = etas["fp64"][k], etas["mixed"][k]
        z = abs(e32 - e64) / math.hypot(s64, s32) if (s64 and s32 and e64 is not None and e32 is not None) else None
        if z is not None:
            zs.append(z)
        out["melts"].append(dict(chains=p.n_chains, length=p.chain_len, n=p.n, shear_rate=p.shear_rate,
                                 strain=p.shear_rate * p.dt * steps, eta_fp64=e64, se_fp64=s64,
                                 eta_mixed=e32, se_mixed=s32, diff_in_se=z))
    zs = np.array(zs)
    out["mixed_speedup"] = out["throughput_mixed"] / out["throughput_fp64"]
    out["eta_agreement"] = dict(median_diff_in_se=float(np.median(zs)), frac_within_2se=float((zs <= 2).mean()),
                                frac_within_3se=float((zs <= 3).mean()),
                                note="eta over the last 20% of each run, 10-block SE; the two runs "
                                     "of a melt are independent trajectories (statistical differences)")
    out["scale"] = scale
    return out


def batch_probe(count=64, steps=500, alone=8):
    """The first `count` requests of the serving trace (FP64, cell-filling skin of 0.4,
    LDS-halo layout) created together and advanced as one batch with le_step_batch,
    then `alone` of them one by one with le_step: ms per step and particle-steps/s."""
    import torch
    from paper_2109_11083_amd.serve import request_params, sweep_trace
    from paper_2109_11083_amd.sim import Sim, step_batch
    trace = sweep_trace(count=count, precision="fp64", burst=True, skin=0.4, tune=1)
    reqs = [request_params(r) for r in trace]
    stream = torch.cuda.Stream()
    sims = [Sim(p, w.x, w.u, stream=stream) for w, p in reqs]
    ntot = sum(s.params.n for s in sims)
    step_batch(sims, 100)
    stream.synchronize()
    t0 = time.perf_counter()
    step_batch(sims, steps)
    stream.synchronize()
    t1 = time.perf_counter()
    out = dict(members=count, n_total=ntot, steps=steps, ms_per_step=1e3 * (t1 - t0) / steps,
               value=ntot * steps / (t1 - t0), alone=[])
    for s in sims:
        s.close()
    for w, p in reqs[:alone]:
        s = Sim(p, w.x, w.u)
        s.step(100)
        s.sync()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        dt = time.perf_counter() - t0
        out["alone"].append(dict(n=p.n, ms_per_step=1e3 * dt / steps, value=p.n * steps / dt))
        s.close()
    return out


def host_info():
    info = dict(nproc=os.cpu_count())
    try:
        aff = sorted(os.sched_getaffinity(0))
        info["affinity"] = f"{len(aff)} cpus: {aff[0]}-{aff[-1]}" if aff else ""
        info["usable_cpus"] = len(aff)
    except AttributeError:
        info["usable_cpus"] = os.cpu_count()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    info["OMP_NUM_THREADS"] = os.environ.get("OMP_NUM_THREADS")
    return info


def cpu_runs():
    """The FP64 cell-list oracle (oracle/) on bounded samples of C1 (LJ N=1000), C2 (LJ
    N=256,000) and C3 (KG 400,000 beads; the overlap-free lattice-path start, since no
    oracle input comes from the GPU path), single-threaded and with its OpenMP timing build
    on every usable core.  ~15-25 s in total."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    from paper_2109_11083_amd import inputs
    hi = host_info()
    cores = int(os.environ.get("OMP_NUM_THREADS") or hi.get("usable_cpus") or 1)
    cores = max(1, min(cores, hi.get("usable_cpus") or cores))
    threads = O.timing_threads(cores)
    cases = []
    w1 = inputs.lj_workload(n_side=10, shear_rate=0.1, seed=11)
    c1 = (w1.x, w1.u, O.make_params(1000, w1.box, shear_rate=0.1, seed=11))
    x2, u2, p2 = lj_params(256000, 0.1, "fp64")
    c2 = (x2, u2, O.make_params(p2.n, p2.box, shear_rate=0.1, seed=21))
    w3 = inputs.kg_workload(KG_CHAINS, KG_LEN, shear_rate=0.01, seed=31, layout="snake")
    p3 = kg_params(0.01, "fp64")
    c3 = (w3.x, w3.u, O.make_params(p3.n, p3.box, shear_rate=0.01, dt=0.01, gamma=0.5, rc=p3.rc,
                                    seed=31, chain_len=KG_LEN, n_chains=KG_CHAINS))
    plan = [("C1 LJ N=1000", c1, 400, 1000), ("C2 LJ N=256000", c2, 4, 16),
            ("C3 KG 2000x200", c3, 10, 20)]
    for name, (x, u, op), n1, nall in plan:
        for timing, steps in ((False, n1), (True, nall)):
            sim = O.Sim(x, u, op, step0=0, timing=timing)
            t0 = time.perf_counter()
            sim.run(steps)
            dt = time.perf_counter() - t0
            n = x.shape[1]
            cases.append(dict(config=name, threads=threads if timing else 1, steps=steps,
                              seconds=round(dt, 3), value=n * steps / dt))
            log(f"bench: cpu oracle {name} {threads if timing else 1} thread(s): {n * steps / dt:.4e} "
                f"p-steps/s ({steps} steps, {dt:.1f} s)")
    return dict(host=hi, runs=cases, threads_all=threads)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--shear-rate", type=float, default=None, help="default 0.01 (KG) / 0.1 (LJ)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--n", type=int, default=256000,
                    help="LJ particles: n sites of a ceil(n^(1/3))^3 lattice (256000 -> 64^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="no HIP events in the timed region (then no per-kernel roofline)")
    ap.add_argument("--skin", default="auto",
                    help="neighbour-list skin, or 'auto' (autotuned per workload, short bursts)")
    ap.add_argument("--tune", type=int, default=0,
                    help="pair layout with an explicit --skin: 0 from density, 1 LDS halo, 2 global")
    ap.add_argument("--c5-scale", type=float, default=0.1,
                    help="chain counts of the 16-melt mixed-precision sweep as a fraction of "
                         "U{500..2000} (1.0: the full sweep, up to 800k beads per melt)")
    ap.add_argument("--c5-steps", type=int, default=30000)
    ap.add_argument("--workload", default="kg", choices=["kg", "lj"],
                    help="kg: 2000 x 200 Kremer-Grest melt (the headline); lj: 256,000-particle LJ fluid")
    ap.add_argument("--thermostat", default="langevin", choices=["langevin", "dpd", "langevin_abs"],
                    help="LJ workload: Langevin on the peculiar velocity (gamma 1), DPD (gamma 5) or "
                         "Langevin on the lab velocity (gamma 1)")
    ap.add_argument("--serve", action=argparse.BooleanOptionalAction, default=True,
                    help="shear-rate sweep serving: p50/p99 time-to-result and sweep throughput")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (byte-counter calibration) and exit")
    ap.add_argument("--batch-probe", type=int, default=0, metavar="COUNT",
                    help="only advance the first COUNT serving requests as one batch (then 8 alone), "
                         "print their timings and exit")
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
    if args.batch_probe:
        print(json.dumps(batch_probe(args.batch_probe, steps=args.steps if args.steps != 10000 else 500)),
              flush=True)
        return
    kg = args.workload == "kg"
    sr = args.shear_rate if args.shear_rate is not None else (0.01 if kg else 0.1)
    th = "langevin" if kg else args.thermostat
    dpd = th == "dpd"

    tune_table = None
    if args.skin == "auto":
        skin, tune_table = pick_skin(args.workload, sr, args.precision, n=args.n, thermostat=th)
        log(f"bench: autotuned skin, layout {skin}: {tune_table}")
    else:
        skin = (float(args.skin), args.tune)
    x, u, p = workload(args.workload, sr, args.precision, skin=skin, n=args.n, thermostat=th)
    log(f"bench: {args.workload} n={p.n} shear_rate={sr} {args.precision} steps={args.steps} "
        f"warmup={args.warmup} skin={skin}")
    r = run_gpu(x, u, p, args.steps, args.warmup, timing=0 if args.no_timing else TIMING_FORCE)
    log(f"bench: {r['value']:.4e} particle-steps/s, {r['ms_per_step']:.4f} ms/step, "
        f"rebuilds={r['rebuilds']}, force={r['phases']['force']}")
    roofline = roofline_of(r, args.workload, args.precision, skin[0], dpd=dpd)

    extra = {}
    # per-phase device time of the same workload (all phases event-timed; a separate, shorter run)
    b = run_gpu(x, u, p, 2000, 100, timing=0xF)
    extra["phase_us_per_step"] = {k: round(1e3 * v[0] / b["steps"], 2) for k, v in b["phases"].items()}
    extra["rebuilds_per_1000_steps_2000_step_run"] = 1000 * b["rebuilds"] / 2000
    log(f"bench: phases {extra['phase_us_per_step']}")
    viscosity = None

    def guarded(name, fn):
        """An extra leg; a failure (e.g. a latched device error) is recorded, not fatal."""
        try:
            return fn()
        except Exception as exc:  # noqa: BLE001 - reported in the JSON line
            log(f"bench: {name} failed: {exc}")
            return dict(error=str(exc))

    if not args.no_extra and not dpd:
        if kg:
            # the 256,000-particle LJ fluid: throughput and force-kernel roofline at its own skin
            ljskin, ljtable = pick_skin("lj", 0.1, "fp64")
            x2, u2, p2 = workload("lj", 0.1, "fp64", skin=ljskin)
            e = run_gpu(x2, u2, p2, 2000, 100)
            extra["lj_256k"] = dict(value=e["value"], ms_per_step=e["ms_per_step"], skin=ljskin[0],
                                    tune=ljskin[1], rebuilds_per_1000=1000 * e["rebuilds"] / 2000,
                                    roofline=roofline_of(e, "lj", "fp64", ljskin[0]), skin_autotune=ljtable)
            log(f"bench: lj 256k: {e['value']:.4e} p-steps/s")
        else:
            ljskin = skin
        for sr2 in (0.01, 1.0):
            x2, u2, p2 = workload("lj", sr2, "fp64", skin=ljskin)
            e = run_gpu(x2, u2, p2, 2000, 100)
            extra[f"lj_256k_shear_rate_{sr2}"] = dict(value=e["value"],
                                                     rebuilds_per_1000=1000 * e["rebuilds"] / 2000)
            log(f"bench: lj shear_rate={sr2}: {e['value']:.4e} p-steps/s rebuilds={e['rebuilds']}")
        # viscosity in FP64 and mixed precision from fixed-length runs (Eq. viscosity)
        viscosity = dict(lj_256k_shear_rate_0_1=guarded("lj viscosity", lambda: viscosity_pair("lj", 0.1, ljskin)))
        kskin = skin if kg else pick_skin("kg", 0.01, "fp64")[0]
        extra["c5_mixed_batched_kg_sweep"] = guarded(
            "c5 sweep", lambda: c5_sweep(scale=args.c5_scale, steps=args.c5_steps))
        # 200 time units each: dt 0.01 at shear rate 0.01; at 0.1 the melt can
        # stretch a bond to R0 within 2e4 steps of dt 0.01 (a latched LE_E_BOND),
        # so that run takes 4e4 steps of dt 0.005
        for sr3, dt3, n3 in ((0.01, None, 20000), (0.1, 0.005, 40000)):
            viscosity[f"kg_400k_shear_rate_{sr3}"] = guarded(
                "kg viscosity", lambda: viscosity_pair("kg", sr3, kskin, steps=n3, warmup=1000, dt=dt3))
    if args.serve and not args.no_extra and th == "langevin":
        extra["serving"] = guarded("serving", lambda: serving_bench(args.serve_requests))

    cpu = None
    if not args.no_cpu_baseline:
        runs = cpu_runs()
        extra["cpu_oracle"] = runs
        want = "C3 KG 2000x200" if kg else "C2 LJ N=256000"
        best = [c for c in runs["runs"] if c["config"] == want and c["threads"] == runs["threads_all"]][-1]
        hi = runs["host"]
        cpu = dict(value=best["value"], unit="particle-steps/s", cores=best["threads"], kind="oracle",
                   sample=(f"{best['steps']} steps of the {want} system (FP64 cell-list oracle, OpenMP "
                           f"timing build, {best['threads']} threads, {best['seconds']:.1f} s; host "
                           f"{hi.get('model', '?')}, nproc {hi.get('nproc')}, affinity "
                           f"{hi.get('affinity', '?')}"
                           + ("; lattice-path start of the same melt" if kg else "") + ")"))

    if kg:
        info = _KG_WARM[31][2]
        wl = (f"Kremer-Grest melt {KG_CHAINS} chains x {KG_LEN} beads (N={r['n']}), random walks of "
              f"bond 0.97, density 0.85, WCA + FENE(30, 1.5), T=1, Langevin gamma=0.5 on peculiar "
              f"velocity, shear_rate={sr}, dt=0.01, skin {skin}, {args.precision}; warmed up without "
              f"shear with capped forces ({info.steps} steps, max force {info.max_force:.0f} < 1e3) "
              f"before the timed region")
    else:
        tdesc = {"langevin": "Langevin gamma=1 on peculiar velocity",
                 "langevin_abs": "Langevin gamma=1 on lab velocity",
                 "dpd": "DPD gamma=5, r_c 2.5"}[th]
        wl = (f"LJ fluid N={r['n']} (64^3 lattice sites, N chosen), density 0.8442, rc 2.5, "
              f"T=1, {tdesc}, shear_rate={sr}, dt=0.005, skin {skin}, {args.precision}")
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
            "skin": skin[0],
            "pair_layout": {0: "from density", 1: "LDS halo", 2: "global"}[skin[1]],
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rebuilds_per_1000_steps": round(1000.0 * r["rebuilds"] / args.steps, 2),
        "skin_autotune": tune_table,
        "viscosity": viscosity,
        "ux_profile_50_bins": [round(v, 5) for v in r["ux_profile"]],
        "kT_kinetic": r["kT"],
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
