"""Benchmark of the APIC augury contact step on one MI355X.

Workload (the headline): the 64x64x16-particle block pressed onto and
sliding over a 256x256x16-particle slab (1,114,112 particles, sparse grid
h = 1, mu = 0.3, 4 augury iterations), stepped by the resident driver with
state resident in HBM.  One "step" is one pass of the whole hot path: cell
keys, radix sort, gather, segments and sparse node-block maps, mass and Vbar
P2G, four fused G2P + friction-rule + P2G rounds, and the final G2P,
position update and momentum drift.

The timed steps keep the geometry of the scene's initial configuration
(driver time step 0: x += 0 * v), so every step does the work of the same
input.  With a nonzero time step the bodies here have no internal forces:
the block's particles keep moving into its own contact layer, cell
occupancy climbs step after step, and the step cost drifts with it
(--free-flight-steps reports that rate).

Prints ONE JSON line: FP32-mixed throughput (the headline value, graph
replay), the plain FP64 throughput on the same scene, the same scene at
mu = 0 and 1, the 256-sphere scene, the roofline of the dominant kernel (the
fused round kernel, timed with HIP events on its stream) and the HBM
fraction of every transfer kernel, the batched form (1,024 two-body scenes)
and the serving loop (Poisson request streams, p50/p99 step latency,
admitted/deferred counts), each with a teacher-forced parity error against
the FP64 oracle, and the CPU oracle timed on this host on bounded samples of
every workload.  Launch tunings come from the committed autotuner cache
(--tune auto re-tunes).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import platform
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contact particle-steps/s (FP32-mixed vs plain FP64) at 2e-5 tol; %HBM peak; p99"
HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2 (packed
# FP32) x 2.4 GHz); the kernels here issue unpacked FP32, whose rate is half.
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Algorithmic flops of one H application per particle with separable weights
# (P2G about 64 x 14, G2P about 64 x 24, weights about 60).
ROUND_FLOPS_PER_PARTICLE = 2500

# Algorithmic bytes per launch of each transfer kernel, FP32-mixed: per
# particle and per active node of the shared grid (body-grid node blocks are
# counted at the shared grid's rate; FP64 doubles all but 4-byte keys).
#  round: read t 12 + key 4 + m 4 + normal 12 + series state Y 48, write Y 48;
#         per node read velocity 12, write momentum 12
#  mass:  read t 12 + key 4 + m 4; per node write mass 4 + body mass 4
#  p2g0:  read t 12 + key 4 + m 4 + Vbar 48, write normal 12; per node read
#         body mass 4 and mass 4, write momentum 12 and 1/m 8 (FP64)
#  final: read t 12 + key 4 + m 4 + normal 12 + Y 16 + Vbar 48 + x 12, write
#         v, C 48 + x 12; per node read velocity 12 and 1/m 8
KERNEL_BYTES = {
    "round": {"fp32": (128, 24), "fp64": (252, 48)},
    "mass": {"fp32": (20, 8), "fp64": (36, 16)},
    "p2g0": {"fp32": (80, 28), "fp64": (156, 48)},
    "final": {"fp32": (168, 20), "fp64": (332, 32)},
}
ROUND_BYTES_PER_PARTICLE = {k: v[0] for k, v in KERNEL_BYTES["round"].items()}
ROUND_BYTES_PER_NODE = {k: v[1] for k, v in KERNEL_BYTES["round"].items()}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the transfer and layout kernel sources with comments and blank
    lines removed, so that counters taken on a kernel stay valid while only
    its comments change."""
    h = hashlib.sha256()
    for f in ("transfer.hip", "layout.hip", "apic_internal.h"):
        with open(os.path.join(ROOT, "paper_2108_02259_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, name: str = "round_kernel_slab_block_counters.json"):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash() or d.get("kernel") != kernel:
        return None
    return d.get("hbm_bytes_per_launch")


def kernel_traffic_from_profiles(name: str = "round_kernel_slab_block_counters.json"):
    """Counter bytes per launch of every transfer kernel of the counted run
    (kernel name -> bytes), if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return {}
    return {k: v["hbm_bytes_per_launch"] for k, v in d.get("per_kernel", {}).items()}


def sq_counters_from_profiles(kernel: str, name: str = "slab_block_sq_counters.json"):
    """VALU/LDS/L2 utilisation of `kernel` from the committed SQ counter runs,
    if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    k = d.get("kernels", {}).get(kernel)
    if d.get("source_hash") != source_hash() or k is None:
        return None
    return {"valu_busy": k["valu_busy"], "lds_active": k["lds_active"],
            "lds_bank_conflict": k["lds_bank_conflict"],
            "wave_time_waiting": k["wave_time_waiting"], "l2_hit_rate": k["l2_hit_rate"]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def host_cores():
    """(cores this process may run on, cores the host reports)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return usable, os.cpu_count() or usable


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def parity(vg, Cg, vr, Cr, h):
    """max(|dv|_inf, h |dC|_inf) / |v_ref|_inf."""
    import numpy as np
    scale = max(float(np.abs(vr).max()), 1e-300)
    return float(max(np.abs(vg - vr).max(), h * np.abs(Cg - Cr).max()) / scale)


def oracle_step64(sc, x, v, C, m, mu=None, n_iter=None, origin=None, dims=None):
    """One FP64 oracle contact step of a scene on the given state."""
    import numpy as np
    from oracle import oracle as ora
    f = lambda a: np.asarray(a, dtype=np.float64)
    g = ora.Grid(h=sc.h, origin=sc.origin if origin is None else origin,
                 dims=sc.dims if dims is None else dims)
    return ora.contact_step(g, f(x), f(v), f(C), f(m), sc.body,
                            sc.mu if mu is None else mu, sc.n_iter if n_iter is None else n_iter)


def serve(ctx, pool, lam, duration, steps, seed, max_particles, max_scenes, budget):
    """Poisson arrivals at rate lam for `duration` seconds of wall time; each
    arrival is a request for `steps` driver steps of a pool scene.  Every
    tick steps all resident requests once; a request's step latency is the
    duration of the tick that stepped it."""
    import numpy as np
    import torch
    from paper_2108_02259_amd.contact import Server
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / lam, size=int(lam * duration * 2) + 16)
    t_arr = np.cumsum(gaps)
    t_arr = t_arr[t_arr < duration]
    which = rng.integers(0, len(pool), size=len(t_arr))
    srv = Server(ctx, torch.float32, max_particles, max_scenes, budget)
    step_lat, req_lat, arrive = [], [], {}
    stepped = 0
    ticks = admitted = deferred_ticks = replayed_ticks = 0
    i = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        if now >= duration:
            break
        while i < len(t_arr) and t_arr[i] <= now:
            e = pool[which[i]]
            srv.submit(i, e["row"], e["dt"], steps, *e["ins"], e["body"], *e["outs"])
            arrive[i] = t_arr[i]
            i += 1
        ts = time.perf_counter()
        info, done = srv.tick()
        te = time.perf_counter()
        admitted += info["admitted"]
        deferred_ticks += 1 if info["deferred"] else 0
        replayed_ticks += info["replayed"]
        if info["resident"] == 0:
            if i < len(t_arr):
                time.sleep(max(0.0, min(t_arr[i] - (te - t0), duration - (te - t0))))
            continue
        ticks += 1
        step_lat += [te - ts] * info["resident"]
        stepped += info["particles"]
        for tag in done:
            req_lat.append(te - t0 - arrive.pop(tag))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    failed = len(srv.failed)
    srv.close()
    mean_p = float(np.mean([e["n"] for e in pool]))
    return {"lambda_per_s": lam, "duration_s": duration, "arrived": int(i),
            "admitted": admitted, "completed": len(req_lat), "failed": failed,
            "queued_at_end": int(i) - admitted, "ticks": ticks,
            "ticks_with_requests_deferred": deferred_ticks,
            "ticks_replaying_a_graph": replayed_ticks,
            "offered_particle_steps_per_s": lam * steps * mean_p,
            "value": stepped / wall, "unit": "particle-steps/s",
            "p50_step_ms": None if not step_lat else 1e3 * percentile(step_lat, 50),
            "p99_step_ms": None if not step_lat else 1e3 * percentile(step_lat, 99),
            "p50_request_s": percentile(req_lat, 50), "p99_request_s": percentile(req_lat, 99)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--mu", type=float, default=0.3)
    ap.add_argument("--profile-steps", type=int, default=40)
    ap.add_argument("--fp64-steps", type=int, default=60)
    ap.add_argument("--mu-steps", type=int, default=60,
                    help="steps of the slab scene at mu = 0 and mu = 1 (0 = skip)")
    ap.add_argument("--spheres-steps", type=int, default=60,
                    help="steps of the 256-sphere scene (0 = skip)")
    ap.add_argument("--ramp-steps", type=int, default=200,
                    help="driver steps of the reduced ramp per friction value (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--tune", choices=("cache", "auto", "off"), default="cache",
                    help="launch tuning: the committed autotuner cache (autotuning what it "
                         "lacks), a fresh autotune of every workload, or the defaults")
    ap.add_argument("--free-flight-steps", type=int, default=0,
                    help="steps of the moving driver (physical dt) to report beside the "
                         "headline (its round kernels, slowed by growing cell occupancy, "
                         "would mix into a profile of the headline kernel)")
    ap.add_argument("--batched-steps", type=int, default=50,
                    help="steps of the 1,024-scene batched form (0 = skip)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched form (for profiling its kernels)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="wall time of each serving run (0 = skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the contact step runs on a single MI355X "
              "and has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_02259_amd import scenes
    from paper_2108_02259_amd.contact import Context, Server, Sim

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    # Two contexts, each with the launch tuning of its scene class: the slab
    # and sphere scenes of the single-scene legs, and the two-body scenes of
    # the batched form and the serving loop (whose tick sizes span many size
    # buckets).
    ctx = Context(0)
    ctx2 = Context(0)
    cache_path = os.path.join(ROOT, "paper_2108_02259_amd", "tuning_cache.json")
    cache = {}
    if args.tune == "cache" and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    for cls, c in (("slab_block", ctx), ("two_body", ctx2)):
        for prec, entries in cache.get(cls, {}).items():
            for b, t in entries.items():
                c.set_tuning(prec, 1 << int(b), t)
    new_cache = {}

    def bucket_of(count):
        return str(int(count).bit_length() - 1)

    def cached(cls, dtype_name, count):
        return cache.get(cls, {}).get(dtype_name, {}).get(bucket_of(count))

    def remember(cls, dtype_name, count, best):
        new_cache.setdefault(cls, {}).setdefault(dtype_name, {})[bucket_of(count)] = best

    def d(a, dtype=None):
        a = a if dtype is None else a.astype(dtype)
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def body_t(sc_):
        return torch.from_numpy(sc_.body.view(np.int16).copy()).to(dev)

    def table_of(sc_):
        return [dict(offset=0, count=sc_.n, h=sc_.h, origin=sc_.origin, dims=sc_.dims,
                     mu=sc_.mu, n_iter=sc_.n_iter, n_bodies=sc_.n_bodies)]

    def timed(sim, steps, graph):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps, graph=graph)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    use_graph = not args.no_graph

    def warmed(sc_, dtype, warmup):
        """A sim of this scene warmed up (the velocity field has spread, so no
        node is skipped as zero), tuned on that state (committed cache or
        autotune) and rebuilt from it with the tuning found."""
        table = table_of(sc_)
        bt_ = body_t(sc_)
        s0 = Sim(ctx, table, [0.0], *(d(a, dtype) for a in (sc_.x, sc_.v, sc_.C, sc_.m)), bt_)
        s0.step(warmup, graph=use_graph)
        x, v, C = s0.read()
        s0.close()
        m = d(sc_.m, dtype)
        tune = None
        name = np.dtype(dtype).name
        if args.tune != "off" and cached("slab_block", name, sc_.n):
            tune = {"best": cached("slab_block", name, sc_.n), "source": "cache"}
        elif args.tune != "off":
            best, tried = ctx.autotune(table, x, v, C, m, bt_, reps=2)
            tune = {"best": best, "best_ms": min(ms for _, ms in tried),
                    "candidates": len(tried), "source": "autotune"}
            remember("slab_block", name, sc_.n, best)
            log(f"autotune {sc_.name} {name}: {best}")
        s1 = Sim(ctx, table, [0.0], x, v, C, m, bt_)
        s1.step(2, graph=use_graph)
        return s1, tune

    def teacher_forced(sim, sc_, dtype, picks=None):
        """Parity of one resident step against the oracle stepping the same
        state (per scene of a batch when picks = [(scene, offset)...])."""
        x, v, C = (t.cpu().numpy() for t in sim.read())
        sim.step(1, graph=use_graph)
        _, vg, Cg = (t.cpu().numpy() for t in sim.read())
        errs = []
        for s_, off in (picks or [(sc_, 0)]):
            sl = slice(off, off + s_.n)
            ref = oracle_step64(s_, x[:, sl], v[:, sl], C[:, sl], s_.m.astype(dtype))
            errs.append(parity(vg[:, sl], Cg[:, sl], ref["v"], ref["C"], s_.h))
        return max(errs)

    out = {"metric": METRIC, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": "fp32-mixed (fp64 keys, grid velocity, normals, friction rule, reductions)",
           "data": "synthetic"}
    tuned = {}
    sc = scenes.slab_block(mu=args.mu)
    n = sc.n
    kt = None
    info = None

    if not args.batched_only:
        log(f"scene slab_block n={n} mu={sc.mu} N={sc.n_iter} dt={sc.dt:.4f}")
        # ---- FP32-mixed: headline (graph replay) ---------------------------
        sim, tuned["float32"] = warmed(sc, np.float32, args.warmup)
        t = timed(sim, args.steps, use_graph)
        value = n * args.steps / t
        ms_per_step = 1e3 * t / args.steps
        log(f"fp32-mixed: {ms_per_step:.3f} ms/step, {value:.3e} particle-steps/s "
            f"(graph={use_graph})")
        _, drift, _ = sim.report()
        # ---- kernel durations from HIP events: with profiling on, the steps
        # run eagerly and every launch is bracketed by a start/stop event pair
        # taken by the launch itself on the stream it runs on
        # (hipExtLaunchKernelGGL), summed per kernel class -----------------
        sim.profiling(True)
        sim.kernel_times()
        t_prof = timed(sim, args.profile_steps, use_graph)
        kt = sim.kernel_times()
        sim.profiling(False)
        log(f"fp32-mixed with kernel events: {1e3 * t_prof / args.profile_steps:.3f} ms/step")
        for k, (ms, cnt) in kt.items():
            if cnt:
                log(f"  {k:9s} {ms / cnt * 1e3:9.1f} us x {cnt / args.profile_steps:.0f}/step")
        info = sim.info()
        reps, _, _ = sim.report()
        slab_parity = teacher_forced(sim, sc, np.float32)
        log(f"fp32-mixed teacher-forced parity {slab_parity:.2e}")
        sim.close()
        nodes = info["shared_blocks"] * 64
        kus = {k: (1e3 * ms / cnt if cnt else None) for k, (ms, cnt) in kt.items()}
        round_us = kus["round"]
        achieved_tf = n * ROUND_FLOPS_PER_PARTICLE / (round_us * 1e-6) / 1e12
        hbm_kernels = {}
        best32 = (tuned.get("float32") or {}).get("best", {})
        group, pairs = best32.get("p2g_group", 4), "true" if best32.get("p2g_pairs") else "false"
        round_kernel = f"apic::k_iter<float, false, {group}, false, {pairs}>"
        names = {"round": round_kernel, "mass": f"apic::k_mass<float, {group}, {pairs}>",
                 "p2g0": f"apic::k_p2g0<float, {group}, {pairs}>",
                 "final": "apic::k_final<float, false>"}
        counted = kernel_traffic_from_profiles()
        for k, key in (("round", "round"), ("mass", "mass"), ("p2g0", "p2g0"),
                       ("final", "final")):
            per_p, per_node = KERNEL_BYTES[k]["fp32"]
            alg = n * per_p + nodes * per_node
            us = kus[key]
            gbs = alg / (us * 1e-6) / 1e9
            hbm_kernels[k] = {"kernel": names[k], "kernel_us": us, "alg_bytes_per_launch": alg,
                              "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
            line = f"  {k:6s} {us:7.1f} us  {gbs:7.0f} GB/s  {100 * gbs / HBM_PEAK_GBS:5.1f} % HBM"
            if names[k] in counted:  # measured bytes (rocprofv3 FETCH + WRITE, calibrated)
                cb = counted[names[k]]
                cg = cb / (us * 1e-6) / 1e9
                hbm_kernels[k].update({"counter_bytes_per_launch": cb, "counter_gbs": cg,
                                       "counter_frac": cg / HBM_PEAK_GBS})
                line += f"   counters {cb / 1e6:6.1f} MB {100 * cg / HBM_PEAK_GBS:5.1f} % HBM"
            log(line)
        out.update({
            "value": value, "ms_per_step": ms_per_step,
            "config": {"workload": "slab_block: 64x64x16 block moving at (2,0,-0.5) 0.5h above "
                                   "a 256x256x16 slab, 1,114,112 particles, sparse grid h=1, "
                                   "mu=0.3, N=4, resident driver, geometry held at the initial "
                                   "configuration (driver dt=0)", "particles": n,
                       "mu": sc.mu, "n_iter": sc.n_iter, "graph": use_graph},
            # the round kernel is bound by vector ALU issue (SQ counters: VALU
            # busy about 70 % of its cycles, HBM at about a quarter of peak)
            "roofline": {"bound": "alu", "achieved": achieved_tf,
                         "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved_tf / FP32_VECTOR_PEAK_TFLOPS,
                         "traffic": traffic_from_profiles(round_kernel),
                         "kernel": round_kernel + " (fused G2P + rule + P2G round)",
                         "kernel_us": round_us,
                         "alg_flops_per_launch": n * ROUND_FLOPS_PER_PARTICLE,
                         "hbm": {"achieved": hbm_kernels["round"]["achieved_gbs"],
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": hbm_kernels["round"]["frac"],
                                 "alg_bytes_per_launch": hbm_kernels["round"]["alg_bytes_per_launch"],
                                 "active_nodes": nodes},
                         "sq_counters": sq_counters_from_profiles(round_kernel)},
            "hbm_by_kernel": hbm_kernels,
            "max_drift_P": drift[0][0], "max_drift_L": drift[0][1],
            "max_bodies_per_node": reps[0]["max_bodies_per_node"],
            "parity": {"fp32_mixed_step_rel_err": slab_parity, "tol": 2e-5,
                       "pass": bool(slab_parity <= 2e-5),
                       "how": "teacher-forced: one resident step against the FP64 oracle "
                              "stepping the same state"},
            "kernels_us": kus, "plan": info})

        # ---- plain FP64 on the same scene -----------------------------------
        if args.fp64_steps > 0:
            sim64, tuned["float64"] = warmed(sc, np.float64, args.warmup)
            t64 = timed(sim64, args.fp64_steps, use_graph)
            _, drift64, _ = sim64.report()
            p64 = teacher_forced(sim64, sc, np.float64)
            sim64.close()
            out["fp64"] = {"value": n * args.fp64_steps / t64, "unit": "particle-steps/s",
                           "ms_per_step": 1e3 * t64 / args.fp64_steps, "steps": args.fp64_steps,
                           "max_drift_P": drift64[0][0], "max_drift_L": drift64[0][1],
                           "parity": p64, "tol": 1e-10}
            log(f"fp64: {out['fp64']['ms_per_step']:.3f} ms/step, "
                f"{out['fp64']['value']:.3e} particle-steps/s, parity {p64:.2e}")

        # ---- the slab scene at mu = 0 and mu = 1 ----------------------------
        if args.mu_steps > 0:
            out["slab_mu"] = {}
            for mu in (0.0, 1.0):
                s_mu = scenes.slab_block(mu=mu)
                sim_m, _ = warmed(s_mu, np.float32, args.warmup)
                tm = timed(sim_m, args.mu_steps, use_graph)
                pm = teacher_forced(sim_m, s_mu, np.float32)
                sim_m.close()
                out["slab_mu"][str(mu)] = {"value": n * args.mu_steps / tm,
                                           "ms_per_step": 1e3 * tm / args.mu_steps,
                                           "steps": args.mu_steps, "parity": pm}
                log(f"slab mu={mu}: {1e3 * tm / args.mu_steps:.3f} ms/step, parity {pm:.2e}")

        # ---- 256 spheres (2-8 bodies per node), N = 6, mu = 0.4 -------------
        if args.spheres_steps > 0:
            sp = scenes.spheres()
            sim_s, tsp = warmed(sp, np.float32, 10)
            ts_ = timed(sim_s, args.spheres_steps, use_graph)
            reps_s, drift_s, _ = sim_s.report()
            ps = teacher_forced(sim_s, sp, np.float32)
            sim_s.close()
            out["spheres"] = {"scene": "256 lattice spheres of radius 8h, random sequential "
                                       "packing in a 256h box, v ~ N(0,1), spin ~ N(0,0.5^2), "
                                       "mu 0.4, N 6, geometry held (dt 0)",
                              "particles": sp.n, "value": sp.n * args.spheres_steps / ts_,
                              "ms_per_step": 1e3 * ts_ / args.spheres_steps,
                              "steps": args.spheres_steps, "parity": ps, "tol": 2e-5,
                              "max_bodies_per_node": reps_s[0]["max_bodies_per_node"],
                              "max_drift_P": drift_s[0][0], "max_drift_L": drift_s[0][1],
                              "tuning": tsp}
            log(f"spheres n={sp.n}: {out['spheres']['ms_per_step']:.3f} ms/step, "
                f"{out['spheres']['value']:.3e} particle-steps/s, parity {ps:.2e}, "
                f"bodies/node {reps_s[0]['max_bodies_per_node']}")

    # ---- the reduced ramp (Section 3.3 without its FE solver): block slide
    # against the rigid block's analytic slide, FP64 ---------------------
    if not args.batched_only and args.ramp_steps > 0:
        from paper_2108_02259_amd import ramp
        out["ramp"] = {"workload": "6x6x6 block on a fixed heavy 20x10x3 ramp, gravity 10 tilted "
                                   "30 deg, grid h = particle spacing, N 4, dt 2e-3, rigid-body "
                                   "projection of the block after every contact step (FP64)",
                       "steps": args.ramp_steps, "t": args.ramp_steps * 2e-3, "by_mu": {}}
        for mu in (0.0, 0.2, 0.4, 0.7):
            _, disp, _ = ramp.run(ctx, mu, args.ramp_steps, trace_every=args.ramp_steps)
            t_end = args.ramp_steps * 2e-3
            out["ramp"]["by_mu"][str(mu)] = {"slide": float(disp[0, -1]),
                                             "analytic": float(ramp.analytic_slide(t_end, mu)),
                                             "sink": float(disp[2, -1])}
            log(f"ramp mu={mu}: slide {disp[0, -1]:.4f} (rigid-block analytic "
                f"{ramp.analytic_slide(t_end, mu):.4f}), sink {disp[2, -1]:.4f}")

    # ---- batched form: 1,024 independent two-body scenes in one set of
    # launches per phase, FP32-mixed, graph replay -------------------------
    scs = None
    if args.batched_steps > 0:
        t0 = time.perf_counter()
        scs = scenes.batch_scenes()
        bx, bv, bC, bm, bb, btable, bdts = scenes.pack(scs, np.float32)
        nb = bx.shape[1]
        log(f"batched: {len(scs)} scenes, {nb} particles (built in "
            f"{time.perf_counter() - t0:.1f} s)")
        arrs = [torch.from_numpy(a).to(dev) for a in (bx, bv, bC, bm)]
        bbt = torch.from_numpy(bb.view(np.int16)).to(dev)
        btune = None
        if args.tune != "off" and cached("two_body", "float32", nb):
            btune = {"best": cached("two_body", "float32", nb), "source": "cache"}
        elif args.tune != "off":
            best, tried = ctx2.autotune(btable, *arrs, bbt, reps=1)
            btune = {"best": best, "best_ms": min(ms for _, ms in tried),
                     "candidates": len(tried), "source": "autotune"}
            log(f"autotune batched: {best}")
            for bucket in range(10, 27):  # the serving loop's tick sizes too
                ctx2.set_tuning(torch.float32, 1 << bucket, best)
                remember("two_body", "float32", 1 << bucket, best)
        rng = np.random.default_rng(17)
        order = np.argsort([s_.n for s_ in scs])
        picks = [int(order[0]), int(rng.choice(order[400:600])), int(order[-1])]

        def run_batch(dts, label, with_parity):
            simb = Sim(ctx2, btable, dts, *arrs, bbt)
            simb.step(2, graph=use_graph)
            tb = timed(simb, args.batched_steps, use_graph)
            _, bdrift, _ = simb.report()
            binfo = simb.info()
            pb = None
            if with_parity:
                pb = teacher_forced(simb, None, np.float32,
                                    [(scs[i], btable[i]["offset"]) for i in picks])
            simb.close()
            r = {"scenes": len(scs), "particles": nb, "steps": args.batched_steps,
                 "value": nb * args.batched_steps / tb, "unit": "particle-steps/s",
                 "ms_per_step": 1e3 * tb / args.batched_steps, "dtype": "fp32-mixed",
                 "graph": use_graph, "tuning": btune,
                 "max_drift_P": max(x_[0] for x_ in bdrift),
                 "max_drift_L": max(x_[1] for x_ in bdrift), "plan": binfo}
            if pb is not None:
                r["parity"] = pb
                r["parity_scenes"] = [scs[i].n for i in picks]
            # the batched round kernel against its roofline: algorithmic bytes
            # over its average event-timed duration, with the committed counters
            simb2 = Sim(ctx2, btable, dts, *arrs, bbt)
            simb2.profiling(True)
            simb2.step(2)
            ktb = simb2.kernel_times()
            simb2.close()
            bbest = (btune or {}).get("best", {})
            rk = (f"apic::k_iter<float, false, {bbest.get('p2g_group', 1)}, false, "
                  f"{'true' if bbest.get('p2g_pairs') else 'false'}>")
            r_ms, r_cnt = ktb["round"]
            us = 1e3 * r_ms / max(r_cnt, 1)
            alg = nb * ROUND_BYTES_PER_PARTICLE["fp32"] + binfo["shared_blocks"] * 64 * ROUND_BYTES_PER_NODE["fp32"]
            r["roofline"] = {"kernel": rk, "kernel_us": us, "alg_bytes_per_launch": alg,
                             "achieved_gbs": alg / (us * 1e-6) / 1e9,
                             "frac": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                             "traffic": traffic_from_profiles(rk, "round_kernel_batched_1024_counters.json"),
                             "sq_counters": sq_counters_from_profiles(rk, "batched_1024_sq_counters.json")}
            log(f"batched ({label}): {r['ms_per_step']:.2f} ms/step, {r['value']:.3e} "
                f"particle-steps/s" + (f", parity {pb:.2e}" if pb is not None else ""))
            return r

        out["batched"] = run_batch([0.0] * len(scs), "geometry held", not args.no_cpu)
        out["batched"]["dt"] = "0 (geometry held at the initial configuration)"
        if not args.batched_only:
            out["batched_moving"] = run_batch(bdts, "moving", False)
            out["batched_moving"]["dt"] = "per scene, 0.2h / body speed"
        del arrs, bbt
        torch.cuda.empty_cache()

    # ---- serving: Poisson request streams, continuous batching -------------
    if args.serve_seconds > 0 and not args.batched_only:
        t0 = time.perf_counter()
        reqs = scenes.request_stream(lam=1.0, duration=1e9, max_requests=32)
        pool = []
        for r in reqs:
            sc_r = r.scene
            ins = [d(a, np.float32) for a in (sc_r.x, sc_r.v, sc_r.C, sc_r.m)]
            pool.append({"row": dict(h=sc_r.h, origin=sc_r.origin, dims=sc_r.dims, mu=sc_r.mu,
                                     n_iter=sc_r.n_iter, n_bodies=sc_r.n_bodies),
                         "dt": sc_r.dt, "ins": ins, "n": sc_r.n, "body": body_t(sc_r),
                         "outs": [torch.empty_like(ins[0]), torch.empty_like(ins[1]),
                                  torch.empty_like(ins[2])]})
        log(f"serving pool: {len(pool)} scenes, {sum(r.scene.n for r in reqs)} particles "
            f"({time.perf_counter() - t0:.1f} s)")
        cfg = dict(max_particles=32_000_000, max_scenes=512, budget=16 << 30)
        serve(ctx2, pool, 5000.0, min(1.0, args.serve_seconds), 50, 99, **cfg)  # warm-up
        serving = []
        for k, lam in enumerate((50.0, 200.0, 1000.0, 5000.0)):
            r = serve(ctx2, pool, lam, args.serve_seconds, 50, 100 + k, **cfg)
            log(f"serving lambda {lam:.0f}/s (offered {r['offered_particle_steps_per_s']:.2e}): "
                f"{r['value']:.3e} particle-steps/s, step p50 {r['p50_step_ms']:.2f} ms p99 "
                f"{r['p99_step_ms']:.2f} ms, {r['completed']}/{r['arrived']} done, "
                f"{r['admitted']} admitted, {r['ticks_replaying_a_graph']}/{r['ticks']} ticks "
                f"replayed a graph")
            serving.append(r)
        # parity of the served step: two pool requests stepped once through a
        # server against the oracle on the same inputs
        errs = []
        srv = Server(ctx2, torch.float32, 2_000_000, 4)
        for tag in (0, 1):
            e, sc_r = pool[tag], reqs[tag].scene
            srv.submit(tag, e["row"], e["dt"], 1, *e["ins"], e["body"], *e["outs"])
        srv.tick()
        for tag in (0, 1):
            e, sc_r = pool[tag], reqs[tag].scene
            ref = oracle_step64(sc_r, *(a.astype(np.float32) for a in (sc_r.x, sc_r.v, sc_r.C,
                                                                        sc_r.m)))
            errs.append(parity(e["outs"][1].cpu().numpy(), e["outs"][2].cpu().numpy(),
                               ref["v"], ref["C"], sc_r.h))
        srv.close()
        out["serving"] = serving
        out["serving_parity"] = {"value": max(errs), "tol": 2e-5,
                                 "requests": [reqs[0].scene.n, reqs[1].scene.n]}
        log(f"serving parity {max(errs):.2e}")
        del pool
        torch.cuda.empty_cache()

    # ---- free flight at the scene's time step (cost drifts with occupancy) --
    if args.free_flight_steps > 0 and not args.batched_only:
        simf = Sim(ctx, table_of(sc), [sc.dt],
                   *(d(a, np.float32) for a in (sc.x, sc.v, sc.C, sc.m)), body_t(sc))
        tf = timed(simf, args.free_flight_steps, use_graph)
        out["free_flight"] = {"steps": args.free_flight_steps, "dt": sc.dt,
                              "value": n * args.free_flight_steps / tf,
                              "ms_per_step": 1e3 * tf / args.free_flight_steps}
        simf.close()

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB device-to-device")
        del a, b

    # ---- CPU oracle baselines on bounded samples ---------------------------
    if not args.no_cpu and not args.batched_only:
        out["cpu_baseline"] = cpu_baselines(sc, scs, reqs if args.serve_seconds > 0 else None)

    if new_cache:
        log("tuning cache entries found by the autotuner in this run: " + json.dumps(new_cache))
    out["tuning"] = tuned
    print(json.dumps(out), flush=True)
    ctx2.close()
    ctx.close()


def cpu_baselines(slab, batch, reqs):
    """The FP64 oracle timed on this host's cores: configs 1-3 on one core,
    the batched and served workloads' independent scenes on one core and in
    parallel threads over all usable cores (the oracle releases the
    interpreter lock while it runs)."""
    import numpy as np
    from paper_2108_02259_amd import scenes
    usable, reported = host_cores()
    res = {}

    def clock(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    # config 2 (the headline workload): one full step
    t2 = clock(lambda: oracle_step64(slab, slab.x, slab.v, slab.C, slab.m))
    base = {"value": slab.n / t2, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 contact step of the full {slab.n}-particle slab+block scene (FP64, "
                      f"mu {slab.mu}, N {slab.n_iter}), {t2:.1f} s on one core of {cpu_model()}",
            "host_cores_usable": usable, "host_cores_reported": reported, "cpu": cpu_model()}
    log(f"cpu oracle slab_block: {t2:.1f} s/step ({slab.n / t2:.3e} particle-steps/s)")
    # config 1: two 12^3 cubes, all 200 driver steps, dense grid re-snapped
    tc = scenes.two_cubes()

    def run_cubes():
        x, v, C = tc.x.copy(), tc.v.copy(), tc.C.copy()
        for _ in range(tc.steps):
            origin, dims = scenes.snap_dense_grid(x, tc.h)
            r = oracle_step64(tc, x, v, C, tc.m, origin=origin, dims=dims)
            v, C = r["v"], r["C"]
            x = x + tc.dt * v
    t1 = clock(run_cubes)
    res["1_two_cubes"] = {"value": tc.n * tc.steps / t1, "cores": 1, "seconds": t1,
                          "sample": f"{tc.steps} driver steps of {tc.n} particles"}
    log(f"cpu oracle two_cubes: {t1:.1f} s for {tc.steps} steps")
    # config 3: one step of the 256 spheres
    sp = scenes.spheres()
    t3 = clock(lambda: oracle_step64(sp, sp.x, sp.v, sp.C, sp.m))
    res["3_spheres"] = {"value": sp.n / t3, "cores": 1, "seconds": t3,
                        "sample": f"1 contact step of {sp.n} particles, N 6"}
    log(f"cpu oracle spheres: {t3:.1f} s/step")

    def scene_parallel(samples, threads):
        """Each sample scene stepped once by the oracle; `threads` workers."""
        work = list(samples)
        lock = threading.Lock()

        def worker():
            while True:
                with lock:
                    if not work:
                        return
                    s_ = work.pop()
                oracle_step64(s_, s_.x, s_.v, s_.C, s_.m)
        ts = [threading.Thread(target=worker) for _ in range(threads)]
        t0 = time.perf_counter()
        for t_ in ts:
            t_.start()
        for t_ in ts:
            t_.join()
        return time.perf_counter() - t0

    for key, pool_, label in (("4_batched", batch, "two-body scenes of the batch"),
                              ("5_serving", None if reqs is None else [r.scene for r in reqs],
                               "requests of the serving pool")):
        if not pool_:
            continue
        rng = np.random.default_rng(5)
        idx = rng.choice(len(pool_), size=min(16, len(pool_)), replace=False)
        sample = [pool_[i] for i in idx]
        ps = sum(s_.n for s_ in sample)
        t_1 = scene_parallel(sample, 1)
        t_all = scene_parallel(sample, usable)
        res[key] = {"value_one_core": ps / t_1, "value_all_cores": ps / t_all,
                    "threads": usable, "seconds_one_core": t_1, "seconds_all_cores": t_all,
                    "sample": f"1 contact step each of {len(sample)} random {label} "
                              f"({ps} particles)"}
        log(f"cpu oracle {key}: 1 core {ps / t_1:.3e}, {usable} threads {ps / t_all:.3e} "
            f"particle-steps/s")
    base["configs"] = res
    return base


if __name__ == "__main__":
    main()
