#!/usr/bin/env python3
"""Throughput of the single-GPU MD hot path on the LJ bulk workload.

Workload: LJ liquid, N = 2,000,000 (fcc 80^3 with 48,000 seeded vacancies,
density 0.8442, T = 1.2), r_cut = 2.5, r_buff = 0.4, dt = 0.005, NVE velocity
Verlet, Morton reordering every 500 steps.  One step = the whole hot path
(fused force + integration + displacement check, and the neighbour-list
rebuilds and sorts that fall inside the window).  The reported value is the
mixed-precision rate (FP32 pair arithmetic, FP64 positions / integration /
reductions); the all-FP64 rate is measured on the same workload beside it.

Beside it (under "others", context only) the same path's mixed-precision rate
on the DPD fluid (N = 1,000,000) and on the 256-system batched ensemble.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-timesteps/sec, LJ 2M particles, mixed vs FP64 at stated force tolerance"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_lj2M_traffic.json")
KERNEL_SOURCES = ["paper_1412_3387_amd/csrc/forces.hip", "paper_1412_3387_amd/csrc/device.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run_precision(B, inputs, torch, s, prec, steps, warmup, tune, fixed=None, prof_steps=1000):
    """Two windows on one trajectory: the timed window runs the product path
    as a user runs it (captured step pairs replayed) and gives the throughput;
    the profiled window right after it launches the same kernels eagerly with
    HIP events around every force launch and every rebuild, and gives the
    per-launch durations."""
    kw = {}
    if fixed:
        kw = {k: int(fixed[k]) for k in ("tpp_nlist", "block_nlist", "tpp_force", "block_force")}
        tune = False
    p = B.ModelParams(precision=prec, pair=B.PAIR_LJ, r_cut=2.5, r_buff=0.4, dt=0.005,
                      sort_period=500, **kw)
    ctx = B.Context([p], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.build_nlist(True)
    tuning = ctx.autotune(tune)
    if warmup > 0:
        ctx.step(0, warmup)
    ctx.check()
    torch.cuda.synchronize()
    stream = ctx.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    b0 = ctx.build_count()
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.step(warmup, steps, log_every=steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.check()
    gpu_ms = e0.elapsed_time(e1)
    builds = ctx.build_count() - b0
    log = ctx.thermo_log()
    E0 = log[0, 0, 1] + log[0, 0, 2]
    E1 = log[-1, 0, 1] + log[-1, 0, 2]
    lay = ctx.layout()
    nn = ctx._ws_view(lay.nn, s.n)
    nbar = float(nn.double().mean().item())
    # profiled window
    ps = max(1, min(prof_steps, steps))
    b1 = ctx.build_count()
    ctx.profile(1)
    e0.record(stream)
    ctx.step(warmup + steps, ps)
    e1.record(stream)
    torch.cuda.synchronize()
    prof = ctx.profile(2)
    ctx.profile(0)
    ctx.check()
    prof_ms = e0.elapsed_time(e1)
    out = dict(ms=max(gpu_ms, 1e-9), wall=wall, prof=prof, prof_steps=ps, prof_ms=prof_ms,
               prof_builds=ctx.build_count() - b1, nbar=nbar, builds=builds,
               drift=abs(E1 - E0) / abs(E0), T_end=float(log[-1, 0, 4]),
               tuning=_tuning_dict(tuning))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def force_check(B, torch, s):
    """Mixed-precision forces against the FP64 path on the starting
    configuration: max over particles of |F_mixed - F_fp64| / F_rms.  Also
    returns both paths' forces (tag order) for the comparison with the
    oracle on the particles the CPU baseline computes."""
    import numpy as np
    out = {}
    for prec in (B.FP64, B.MIXED):
        p = B.ModelParams(precision=prec, pair=B.PAIR_LJ, r_cut=2.5, r_buff=0.4, dt=0.005,
                          sort_period=500)
        ctx = B.Context([p], [dict(pos=s.pos, vel=s.vel, L=s.L)])
        ctx.build_nlist(True)
        ctx.compute_forces(0, 0)
        ctx.check()
        x, v, f, tag = ctx.host_state()
        F = np.empty((s.n, 3))
        F[tag] = f[:, :3]
        out[prec] = F
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    ref = out[B.FP64]
    frms = float(np.sqrt(np.mean(ref ** 2)))
    err = float(np.max(np.linalg.norm(out[B.MIXED] - ref, axis=1))) / frms
    return {"max_err_over_Frms": err, "tolerance": 1e-5, "pass": err <= 1e-5, "F_rms": frms}, out


def _tuning_dict(t):
    return {"tpp_force": t.tpp_force, "block_force": t.block_force, "tpp_nlist": t.tpp_nlist,
            "block_nlist": t.block_nlist, "force_ms": [round(x, 4) for x in t.force_ms],
            "build_ms": [round(x, 4) for x in t.build_ms], "scans": t.scans, "from_cache": t.from_cache}


def other_workload(B, torch, label, params, systems, steps, warmup, t0=0):
    """Mixed-precision throughput of a secondary workload (context beside the
    headline: the same product path, captured steps replayed, launch shapes
    chosen by the autotuner): total particles x steps / device time of
    `steps` steps after `warmup` steps that start at step t0 (the context
    sorts the rows at init)."""
    ctx = B.Context(params, systems)
    ctx.build_nlist(True)
    tuning = ctx.autotune(1)
    ctx.step(t0, warmup)
    ctx.check()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    b0 = ctx.build_count()
    e0.record(ctx.stream)
    ctx.step(t0 + warmup, steps)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1)
    n = sum(int(sy["pos"].shape[0]) for sy in systems)
    builds = ctx.build_count() - b0
    # eager profiled window: HIP events around every force launch and rebuild
    ps = max(20, steps // 5)
    ctx.profile(1)
    ctx.step(t0 + warmup + steps, ps)
    torch.cuda.synchronize()
    prof = ctx.profile(2)
    ctx.profile(0)
    ctx.check()
    rows = sum(int(ctx._ws_view(ctx.layout(k).nn, ctx.n_local[k]).double().sum().item())
               for k in range(len(systems)))
    nbar = rows / n
    force_us = 1e3 * prof.force_ms / max(prof.force_launches, 1)
    alg = n * (4 * nbar + 124)  # the headline's per-particle bytes of the fused force pass
    out = {"workload": label, "value": n * steps / (ms / 1e3), "unit": "particle-timesteps/s",
           "steps_per_s": steps / (ms / 1e3), "particles": n, "systems": len(systems), "steps": steps,
           "rebuilds": builds, "precision": "mixed", "tuning": _tuning_dict(tuning),
           "profiled_window": {"steps": ps, "force_us_per_step": force_us,
                               "rebuild_ms_per_build": prof.rebuild_ms / max(ctx.build_count() - b0 - builds, 1),
                               "mean_row": nbar, "force_alg_GBps": alg / (force_us * 1e-6) / 1e9,
                               "force_frac_of_hbm": alg / (force_us * 1e-6) / 8e12}}
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def batch_per_system(B, torch, params, systems, steps, warmup):
    """The same ensemble with every system in a context of its own, stepped
    one context after another on one stream (per-system launches, each
    context's steps replayed as captured graphs), for comparison with the one
    batched context."""
    ctxs = [B.Context([p], [sy]) for p, sy in zip(params, systems)]
    for c in ctxs:
        c.build_nlist(True)
        c.autotune(2)
        c.step(0, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for c in ctxs:
        c.step(warmup, steps)
    e1.record()
    torch.cuda.synchronize()
    for c in ctxs:
        c.check()
    ms = e0.elapsed_time(e1)
    n = sum(int(sy["pos"].shape[0]) for sy in systems)
    for c in ctxs:
        c.close()
    del ctxs
    torch.cuda.empty_cache()
    return {"value": n * steps / (ms / 1e3), "unit": "particle-timesteps/s", "steps": steps,
            "launches": "one context per system, stepped in turn"}


def subdomain_phases(B, inputs, torch, reps=200):
    """The one-GPU share of the strong-scaling shape: subdomain 0 of the
    864,000-particle LJ box cut 3 x 3 x 3 (32,000 locals, ghost layer 2.9),
    mixed precision.  The ghost exchange between the 27 subdomains is done
    once as device copies on this GPU to obtain subdomain 0's receive
    buffer (a stand-in for the transport).  Per phase, the HIP-event time of
    one call averaged over `reps` calls: ghost selection + packing of
    subdomain 0's send list, the per-step re-gather (update) of that list,
    unpacking of its receive buffer (select, and update in place), the local
    forces; then one step's worth of subdomain 0 (update pack, update unpack,
    local forces) launched eagerly and replayed as a captured graph."""
    import numpy as np
    W, margin = 2.9, 0.25
    sd = inputs.lj_subdomain_box(grid=3, cells=60)
    full = sd.full
    frame = sd.side + 2 * (W + margin)
    rho = full.n / float(np.prod(full.L))
    n_cap = int(1.2 * rho * frame ** 3) + 64
    fields = B.FIELD_POS | B.FIELD_TAG
    rec = 32
    dev = torch.device("cuda:0")
    s_side = torch.cuda.Stream()
    with torch.cuda.stream(s_side):
        # all 27 subdomains in one context: every send list, then the slices
        # destined for subdomain 0
        systems, params = [], []
        for k in range(27):
            loc = sd.local(k)
            systems.append(dict(pos=full.pos[loc], vel=full.vel[loc], tag=loc.astype(np.int32),
                                L=np.full(3, frame), lo=sd.lo(k) - W - margin, periodic=(0, 0, 0), n_cap=n_cap))
            params.append(B.ModelParams(precision=B.MIXED, nlist_cap=160))
        ctx27 = B.Context(params, systems)
        cap = 8 * max(ctx27.n_local)
        sends, counts, offs = [], [], []
        for k in range(27):
            buf = torch.zeros(cap * rec, dtype=torch.uint8, device=dev)
            cnt = torch.zeros(26, dtype=torch.int32, device=dev)
            off = torch.zeros(26, dtype=torch.int32, device=dev)
            ctx27.pack_ghosts(k, sd.lo(k), sd.hi(k), W, B.GHOST_SELECT, fields, buf, cap, cnt, off)
            sends.append(buf)
            counts.append(cnt)
            offs.append(off)
        ctx27.check()
        hc = [c.cpu().numpy() for c in counts]
        ho = [o.cpu().numpy() for o in offs]
        pieces = []
        for k in range(1, 27):
            a = np.array([k % 3, (k // 3) % 3, k // 9])
            d = (np.zeros(3, dtype=np.int64) - a + 1) % 3 - 1
            dk = int((d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1))
            dk = dk if dk < 13 else dk - 1
            pieces.append(sends[k][int(ho[k][dk]) * rec:(int(ho[k][dk]) + int(hc[k][dk])) * rec])
        recv = torch.cat(pieces).contiguous()
        n_recv = recv.numel() // rec
        ctx27.close()
        del ctx27, sends
        # subdomain 0 alone: its own context on a stream that can be captured
        ctx = B.Context([B.ModelParams(precision=B.MIXED, nlist_cap=160)],
                        [systems[0]])
        send = torch.zeros(cap * rec, dtype=torch.uint8, device=dev)
        cnt = torch.zeros(26, dtype=torch.int32, device=dev)
        off = torch.zeros(26, dtype=torch.int32, device=dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)

        def timed(fn, n=reps):
            fn()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / n

        lo0, hi0 = sd.lo(0), sd.hi(0)
        out = {"workload": "lj_subdomain_32k", "locals": int(ctx.n_local[0]), "ghosts": int(n_recv),
               "send_entries": None, "precision": "mixed"}
        out["select_pack_us"] = timed(lambda: ctx.pack_ghosts(0, lo0, hi0, W, B.GHOST_SELECT, fields, send, cap,
                                                              cnt, off))
        out["send_entries"] = int(cnt.sum().item())
        out["update_pack_us"] = timed(lambda: ctx.pack_ghosts(0, lo0, hi0, W, B.GHOST_UPDATE, fields, send, cap,
                                                              cnt, off))
        out["unpack_select_us"] = timed(lambda: ctx.unpack_ghosts(0, recv, n_recv, fields, B.GHOST_SELECT, full.L),
                                        n=20)
        out["unpack_update_us"] = timed(lambda: ctx.unpack_ghosts(0, recv, n_recv, fields, B.GHOST_UPDATE, full.L))
        ctx.compute_forces(0, 0)
        out["local_forces_us"] = timed(lambda: ctx.compute_forces(0, 0))

        def one_step():
            ctx.pack_ghosts(0, lo0, hi0, W, B.GHOST_UPDATE, fields, send, cap, cnt, off)
            ctx.unpack_ghosts(0, recv, n_recv, fields, B.GHOST_UPDATE, full.L)
            ctx.compute_forces(0, 0)

        out["step_eager_us"] = timed(one_step)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s_side):
            one_step()
        out["step_graph_us"] = timed(g.replay)
        ctx.check()
        out["graph_speedup"] = out["step_eager_us"] / out["step_graph_us"]
        ctx.close()
        del g, ctx
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def other_workloads(B, inputs, torch, steps, warmup, only=None):
    """DPD fluid (N = 1,000,000, density 3, r_cut 1, A 25, gamma 4.5, kT 1,
    dt 0.02), the batched ensemble (128 LJ liquids of 500..20,000 particles
    and 128 bead-spring melts of 20..400 chains of 50, FENE + WCA), each in
    one context, the 32,000-particle NVT share of the weak-scaling fluid,
    and the per-phase times of the strong-scaling subdomain (`only`: one of
    them, by key).  A failing workload is reported, not fatal: the headline
    line still prints."""

    def dpd():
        # The configuration leaves r_buff and the sort period open; they are
        # the fastest pair of a preliminary scan (as the paper tunes r_buff):
        # DPD particles diffuse fast (dt = 0.02), and sorted every 100 steps
        # the tiles outgrow the framed build and the force pass's LDS stage
        d = inputs.dpd_bulk()
        p = B.ModelParams(precision=B.MIXED, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.5, dt=0.02, dpd_seed=33,
                          sort_period=20)
        return other_workload(B, torch, "dpd_1M", [p], [dict(pos=d.pos, vel=d.vel, L=d.L)], steps, warmup)

    def batch():
        ens = inputs.batch_ensemble()
        # launch shapes of the whole batch chosen by the autotuner
        params = [B.ModelParams(precision=B.MIXED, pair=B.PAIR_LJ, sort_period=500)
                  if sy.kind == "lj" else
                  B.ModelParams(precision=B.MIXED, pair=B.PAIR_WCA, bond_cap=2, sort_period=500)
                  for sy in ens]
        systems = [dict(pos=sy.pos, vel=sy.vel, L=sy.L, bonds=sy.bonds, tag=sy.tag) for sy in ens]
        r = other_workload(B, torch, "batch_256", params, systems, steps, warmup)
        if only is None:  # (a profiling run of the batch alone leaves the comparison out)
            r["per_system_launches"] = batch_per_system(B, torch, params, systems, max(steps // 5, 20), warmup)
            r["batched_over_per_system"] = r["value"] / r["per_system_launches"]["value"]
        return r

    def nvt():
        # one GPU's share of the weak-scaling runs: NVT (Nose-Hoover), packing
        # fraction 0.2, r_cut 3.0, dt 0.002
        w = inputs.lj_weak_share()
        p = B.ModelParams(precision=B.MIXED, r_cut=3.0, r_buff=0.4, dt=0.002, sort_period=500,
                          integrator=B.NVT, nvt_T0=1.2, nvt_tau=0.5)
        return other_workload(B, torch, "lj_nvt_32k", [p], [dict(pos=w.pos, vel=w.vel, L=w.L)], steps, warmup)

    res = {}
    for key, fn in (("dpd_1M", dpd), ("batch_256", batch), ("lj_nvt_32k", nvt),
                    ("subdomain_32k", lambda: subdomain_phases(B, inputs, torch))):
        if only is not None and only != key:
            continue
        try:
            res[key] = fn()
        except Exception as e:
            res[key] = {"error": repr(e)}
    return res


COPY_BYTES = 1 << 30


def pmc_pass(B, inputs, torch, s, fixed, steps, workload="lj"):
    """Workload for the hardware-counter passes: a plain streaming kernel of
    known size (an elementwise negation reading and writing COPY_BYTES each),
    then eager mixed-precision steps of the LJ bulk system (or, with
    workload "dpd", of the 1,000,000-particle DPD fluid)."""
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    kw = {k: int(fixed[k]) for k in ("tpp_nlist", "block_nlist", "tpp_force", "block_force")} if fixed else {}
    if workload == "dpd":
        s = inputs.dpd_bulk()
        p = B.ModelParams(precision=B.MIXED, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.5, dt=0.02, dpd_seed=33,
                          sort_period=20, use_graph=0, **kw)
    else:
        p = B.ModelParams(precision=B.MIXED, pair=B.PAIR_LJ, r_cut=2.5, r_buff=0.4, dt=0.005,
                          sort_period=500, use_graph=0, **kw)
    ctx = B.Context([p], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.build_nlist(True)
    ctx.step(0, steps)
    ctx.check()
    lay = ctx.layout()
    nbar = float(ctx._ws_view(lay.nn, s.n).double().mean().item())
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"pmc_pass": True, "workload": workload, "n": s.n, "steps": steps, "copy_bytes": COPY_BYTES,
                      "mean_row": nbar}), flush=True)


def _counter_rows(path):
    """Per-dispatch counter sums from a rocprofv3 counter_collection.csv."""
    import csv
    per = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            did = row.get("Dispatch_Id") or row.get("Correlation_Id")
            key = (did, name)
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    return per


def reduce_pmc(fetch_csv, write_csv, out_path, n):
    """HBM bytes per fused force launch from a FETCH_SIZE pass and a
    WRITE_SIZE pass (KiB per dispatch), each scaled by what the same counter
    reads for the streaming kernel of known size."""
    res = {"kernel_hash": kernel_hash(), "n": n}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        per = _counter_rows(path)
        copy = [v for (d, k), v in per.items() if "neg" in k]
        # one fused step = the main force launch plus the launch over rare tiles
        main = [v for (d, k), v in per.items() if "k_force<" in k]
        rare = [v for (d, k), v in per.items() if "k_force_rare<" in k]
        if not copy or not main:
            raise SystemExit(f"{path}: no copy ({len(copy)}) or force ({len(main)}) dispatches")
        copy_kib = sorted(copy)[len(copy) // 2]
        scale = (COPY_BYTES / 1024.0) / copy_kib
        force_kib = sum(main) / len(main) + (sum(rare) / len(rare) if rare else 0.0)
        res[label] = {"copy_kib_per_dispatch": copy_kib, "scale": scale,
                      "force_kib_per_step": force_kib, "main_dispatches": len(main),
                      "rare_dispatches": len(rare),
                      "bytes_per_launch": force_kib * 1024.0 * scale}
    res["bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def cpu_baseline(s, seconds):
    """The FP64 oracle on the host cores: brute-force forces of a bounded
    sample of particles against the whole box (its per-particle-step cost)."""
    import numpy as np
    import oracle
    oracle.build()
    rng = np.random.default_rng(0)
    lj = [1.0, 1.0, 2.5]
    m = 64
    t = 0.0
    while True:
        which = np.sort(rng.choice(s.n, m, replace=False))
        t0 = time.perf_counter()
        F_orc = oracle.pair_forces("lj", s.pos, s.L, lj, which=which)[0]
        t = time.perf_counter() - t0
        # the last, timed sample aims at `seconds` of CPU work (stops past
        # two thirds of it)
        if t > 0.66 * seconds or m >= s.n:
            break
        m = min(s.n, int(m * max(2.0, min(16.0, seconds / max(t, 1e-3)))))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": m / t, "unit": "particle-timesteps/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_logical_cpus": os.cpu_count(),
            "sample": (f"FP64 brute-force forces of {m} random particles against all {s.n} "
                       f"(O(N) each, minimum image), {t:.1f} s; the integration is negligible "
                       f"beside it")}, (which, F_orc)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-others", action="store_true",
                    help="skip the secondary workloads (DPD 1M, 256-system batch)")
    ap.add_argument("--other-steps", type=int, default=1000)
    ap.add_argument("--others-only", default=None,
                    choices=["dpd_1M", "batch_256", "lj_nvt_32k", "subdomain_32k"],
                    help="run one secondary workload (the batch without its per-system comparison), "
                         "print its JSON line and exit (for profiling)")
    ap.add_argument("--tuning-out", default=None,
                    help="write the lanes/block sizes chosen per precision to this JSON file")
    ap.add_argument("--tuning-from", default=None,
                    help="use lanes/block sizes from a file written by --tuning-out (no tuning)")
    ap.add_argument("--prof-steps", type=int, default=1000,
                    help="steps of the eager window timed per launch after the timed window")
    ap.add_argument("--pmc-workload", default="lj", choices=["lj", "dpd"],
                    help="workload of --pmc-pass")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run the workload of a hardware-counter pass instead of the benchmark")
    ap.add_argument("--reduce-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter_collection.csv of a FETCH_SIZE and a WRITE_SIZE pass "
                         "into the per-launch traffic file and exit")
    args = ap.parse_args()
    if args.reduce_pmc:
        reduce_pmc(args.reduce_pmc[0], args.reduce_pmc[1], TRAFFIC_FILE, args.n)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only (the hot path of one subdomain); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1412_3387_amd import binding as B
    from paper_1412_3387_amd import inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    B.lib()
    if args.others_only:
        print(json.dumps(other_workloads(B, inputs, torch, args.other_steps, 100, args.others_only)), flush=True)
        return
    s = inputs.lj_bulk(args.n)
    print(f"[bench] N={s.n} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    fixed = {}
    if args.tuning_from:
        with open(args.tuning_from) as f:
            fixed = json.load(f)
    if args.pmc_pass:
        pmc_pass(B, inputs, torch, s, fixed.get("mixed"), args.steps, args.pmc_workload)
        return
    mixed = run_precision(B, inputs, torch, s, B.MIXED, args.steps, args.warmup, not args.no_tune,
                          fixed.get("mixed"), args.prof_steps)
    print(f"[bench] mixed done {mixed['ms']:.1f} ms", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_precision(B, inputs, torch, s, B.FP64, args.steps, args.warmup, not args.no_tune,
                             fixed.get("fp64"), args.prof_steps)
        print(f"[bench] fp64 done {fp64['ms']:.1f} ms", file=sys.stderr, flush=True)
    if args.tuning_out:
        with open(args.tuning_out, "w") as f:
            json.dump({"mixed": mixed["tuning"], "fp64": fp64["tuning"] if fp64 else None}, f)

    K = args.steps
    value = s.n * K / (mixed["ms"] / 1e3)
    pr = mixed["prof"]
    PS = mixed["prof_steps"]
    force_avg_ms = pr.force_ms / max(pr.force_launches, 1)
    # algorithmic bytes of one fused force launch per particle, with 4-byte
    # neighbour indices and 24-byte vectors: the neighbour row and its length
    # (4 n + 4), position, velocity and position at the last build read
    # (3 x 24), position and velocity written (2 x 24); neighbour gathers are
    # served by caches and not counted
    bytes_per_particle = 4.0 * mixed["nbar"] + 4 + 3 * 24 + 2 * 24
    alg_bytes_per_launch = s.n * bytes_per_particle
    achieved = alg_bytes_per_launch / (force_avg_ms / 1e3) / 1e9
    # compulsory bytes of a whole step in the two-pass model (separate force
    # and integration passes, FP32 force array, rebuild every 10 steps)
    step_bytes = (4.0 * mixed["nbar"] + 4 + 24 + 12) + (24 + 24 + 12 + 24 + 24 + 24) \
        + (84 + 4.0 * mixed["nbar"]) / 10.0
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("n") == s.n:
            traffic = tr.get("bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-timesteps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair math + f64 state (mixed)",
        "data": "synthetic",
        "config": {"workload": "lj_bulk_2M", "N": s.n, "density": 0.8442, "T0": 1.2, "r_cut": 2.5,
                   "r_buff": 0.4, "dt": 0.005, "sort_period": 500, "precision": "mixed",
                   "parallelism": "single GPU"},
        "steps_per_s": K / (mixed["ms"] / 1e3),
        "energy_drift_rel": mixed["drift"],
        "T_end": mixed["T_end"],
        "rebuilds": mixed["builds"],
        "tuning": mixed["tuning"],
        "profiled_window": {"steps": PS, "ms_per_step": mixed["prof_ms"] / PS,
                            "rebuilds": mixed["prof_builds"],
                            "force_ms_per_step": pr.force_ms / PS,
                            "rebuild_ms_per_step": pr.rebuild_ms / PS,
                            "rebuild_ms_per_build": pr.rebuild_ms / max(mixed["prof_builds"], 1)},
        "step_alg_bytes_per_particle": step_bytes,
        "step_frac_of_hbm": step_bytes * s.n * K / (mixed["ms"] / 1e3) / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "kernel": "k_force (fused force + velocity Verlet)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes_per_launch,
                     "avg_launch_us": force_avg_ms * 1e3,
                     "alg_bytes_per_particle": bytes_per_particle, "mean_row": mixed["nbar"]},
    }
    if fp64 is not None:
        line["fp64"] = {"value": s.n * K / (fp64["ms"] / 1e3), "ms_per_step": fp64["ms"] / K,
                        "energy_drift_rel": fp64["drift"], "rebuilds": fp64["builds"],
                        "tuning": fp64["tuning"],
                        "force_avg_us": fp64["prof"].force_ms / max(fp64["prof"].force_launches, 1) * 1e3}
        line["mixed_over_fp64"] = line["value"] / line["fp64"]["value"]
    line["force_check"], gpu_forces = force_check(B, torch, s)
    if not args.no_others:
        print("[bench] other workloads", file=sys.stderr, flush=True)
        line["others"] = other_workloads(B, inputs, torch, args.other_steps, 100)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"], (which, F_orc) = cpu_baseline(s, args.cpu_seconds)
        # both GPU paths against the oracle on the particles it computed
        import numpy as np
        frms = float(np.sqrt(np.mean(np.sum(F_orc ** 2, axis=1))))
        line["force_check"]["vs_oracle"] = {
            name: float(np.max(np.linalg.norm(gpu_forces[prec][which] - F_orc, axis=1))) / frms
            for name, prec in (("fp64", B.FP64), ("mixed", B.MIXED))}
        line["force_check"]["vs_oracle"]["particles"] = int(len(which))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
