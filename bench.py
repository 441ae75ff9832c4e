"""Throughput benchmark of the elastic-wall D3Q19 update on one MI355X.

Workload (one step = one update of every fluid site, boundary links
included): the synthetic 4-generation Murray artery tree, seed 3
(7,484,227 fluid sites in a 1200 x 400 x 400 box, 79 stiffness segments,
48 fixed-density outlets), D3Q19 BGK tau = 0.8, FP32 deviation storage,
elastic walls (F = 0.5, stiffness log-uniform in [1e-3, 1e-1] per segment),
pulsatile parabolic velocity inlet u(t) = 0.02 (1 + 0.5 sin(2 pi t / 4000)).

Prints one JSON line: MLUPS over exactly --steps timed steps (whole job);
the HBM roofline of the update kernel (algorithmic bytes 2 * 19 * 4 per site
per launch over the kernel's average launch duration, HIP events on the
stream the library launches on, over a window of at least 2048
graph-replayed launches whatever --steps is); and the FP64 CPU oracle timed
on a bounded sample of the same workload.  Secondary figures (FP16/BF16
storage, the 64-instance sweep, bounce-back vs elastic, the cache-resident
tube, the paper's R = 100 cylinder, the network) ride in "secondary".
``--workload tube`` or ``--workload sweep`` makes one of those the main line
(for profiling them on their own; no oracle baseline then).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS & % of HBM roofline (FP32 vs FP16 storage); cycles-to-periodic, warm vs cold")
PEAK_GBS = 8000.0
# autotuner trial length of the main run (the other runs use 256 steps)
MAIN_TUNE_STEPS = 1024
# launches per roofline window (multiple of the library's 128-step graphs)
ROOF_MIN_LAUNCHES = 2048
BYTES_PER_POP = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def oracle_configure(o, wl, k=0):
    p = wl.params[k]
    o.set_wall(p.mode, F=p.F, P0=p.P0, k=p.k)
    for i, q in p.iolets.items():
        o.set_iolet(i, q["kind"], q["a0"], q.get("amp", 0.0), q.get("period", 1.0),
                    q.get("phase", 0.0), q.get("direction", (0.0, 0.0, 0.0)))
    o.init_fields()


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "d3q19.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2108_08783_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# the main workload: the headline tree, or the tube or the sweep (used to
# profile those on their own)
WORKLOADS = {
    "tube": ("tube32", "elastic straight cylinder R=32 L=512 (1,640,960 sites; FP32 working "
                       "set partly inside the 256 MB Infinity Cache), D3Q19 BGK tau=0.8, "
                       "pulsatile parabolic velocity inlet 0.02(1+0.5 sin(2 pi t/4000)), "
                       "density outlet, k log-uniform [1e-3,1e-1] seed 1, F=0.85"),
    "tree": ("tree", "elastic Murray tree seed 3 (7,484,227 sites), D3Q19 BGK tau=0.8, "
                     "pulsatile parabolic velocity inlet 0.02(1+0.5 sin(2 pi t/4000)), "
                     "density outlets, k log-uniform [1e-3,1e-1] per segment, F=0.5"),
    "sweep": ("sweep64", "64 elastic tubes and bifurcations seed 4 (19.7M sites), D3Q19 BGK "
                         "tau=0.8, pulsatile velocity inlets, density outlets, F=0.5"),
}


def make_workload(name):
    from paper_2108_08783_amd import workloads
    return {"tube": workloads.tube32, "tree": workloads.tree, "sweep": workloads.sweep}[name]()


def traffic_from_profiles(dtype, workload="tube"):
    """HBM bytes per launch from the committed counter summary of that
    workload, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"update_kernel_{WORKLOADS[workload][0]}_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    e = d.get("per_dtype", {}).get(dtype)
    return None if e is None else e.get("bytes_per_launch")


def copy_probe(gib=1.0, reps=20):
    """Achievable HBM bandwidth of plain device copies of known size: torch's
    copy and the library's streaming copy (normal and non-temporal); under
    rocprofv3 --pmc they also give the FETCH_SIZE / WRITE_SIZE scale."""
    import torch
    from paper_2108_08783_amd import lbm
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * 4 * n
    out = dict(bytes_per_copy=nbytes, torch_us=round(ms * 1e3, 2),
               torch_gbs=round(nbytes / (ms * 1e-3) / 1e9, 1))
    s = torch.cuda.current_stream().cuda_stream
    for nt in (0, 1):
        ms = lbm.lbm_copy_probe(b.data_ptr(), a.data_ptr(), 4 * n, nontemporal=nt, reps=reps,
                                stream=s)
        out[f"lib{'_nt' if nt else ''}_gbs"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    return out


def roof_window(steps):
    """Launches in a roofline window: at least ROOF_MIN_LAUNCHES, a multiple
    of 128 (whole graph replays); 0 when ROOF_MIN_LAUNCHES is 0 (profiling
    runs that want only the timed steps)."""
    if ROOF_MIN_LAUNCHES == 0:
        return 0
    n = max(ROOF_MIN_LAUNCHES, steps)
    return (n + 127) // 128 * 128


def gpu_run(wl, dtype, steps, warmup, bounceback=False, tune=True, launch=None, tune_steps=256):
    """Creates the lattice, autotunes, warms up, then times exactly `steps`
    steps (wall clock and HIP events) and, separately, a roofline window of
    graph-replayed launches (HIP events on the library's stream)."""
    import torch
    from paper_2108_08783_amd import lbm, workloads
    tc = time.perf_counter()
    lat = workloads.lattice(wl, dtype)
    t_create = time.perf_counter() - tc
    if bounceback:
        for k, p in enumerate(wl.params):
            lat.set_wall(k, lbm.BOUNCEBACK, F=0.0, P0=p.P0, k=p.k)
    if launch:
        lat.set_launch(**launch)
    elif tune:
        lat.autotune(tune_steps)
    t_tune = time.perf_counter() - tc - t_create
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = lat.time_steps(steps)          # HIP events on the library stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    win = roof_window(steps)
    roof_ms = lat.time_steps(win) if win else ms   # graph replays, HIP events
    info = lat.info()
    for k in range(len(wl.geoms)):
        lat.read_fields(k, wss=False, wall_dr=False)  # raises if diverged
    lat.close()
    n = info["n_sites"]
    print(f"[bench]   {dtype}: create {t_create:.1f}s, tune {t_tune:.1f}s, timed {t1 - t0:.3f}s, "
          f"roofline window {win} launches {roof_ms:.1f} ms", file=sys.stderr, flush=True)
    return dict(n=n, wall_s=t1 - t0, event_ms=ms, info=info,
                mlups=n * steps / (t1 - t0) / 1e6,
                launch_us=roof_ms * 1e3 / (win or steps), window=win or steps)


def update_kernel(info):
    """Name of the update kernel a launch configuration runs."""
    return "k_step_pair" if info["sites_per_lane"] == 2 else "k_step"


def summary(r, dtype, with_traffic=False):
    ach = 2 * 19 * BYTES_PER_POP[dtype] * r["n"] / (r["launch_us"] * 1e-6) / 1e9
    out = dict(sites=r["n"], mlups=round(r["mlups"], 1), us_per_step=round(r["launch_us"], 2),
               roofline_frac=round(ach / PEAK_GBS, 4), achieved_gbs=round(ach, 1),
               window_launches=r["window"],
               index_bits=r["info"]["index_bits"], block=r["info"]["block_size"],
               xcd_remap=r["info"]["xcd_remap"], nontemporal=r["info"]["nontemporal"],
               fused=r["info"]["boundary_fused"], sites_per_lane=r["info"]["sites_per_lane"],
               boundary_sites=r["info"]["n_boundary"])
    if with_traffic:
        out["traffic"] = traffic_from_profiles(dtype, with_traffic)
    return out


def cpu_one_thread(workload, target_s=6.0):
    """The oracle on the main workload with one OpenMP thread, in a child
    process (the thread count is fixed when the oracle library loads)."""
    import subprocess
    code = (
        "import json, sys, time; sys.path.insert(0, %r)\n"
        "import bench, oracle\n"
        "wl = bench.make_workload(%r); g = wl.geoms[0]\n"
        "o = oracle.Oracle(g.labels, wl.tau, segment=g.segment, normal=g.normal, iolet_weight=g.iolet_weight)\n"
        "bench.oracle_configure(o, wl); o.step(1)\n"
        "t0 = time.perf_counter(); o.step(1); dt = time.perf_counter() - t0\n"
        "n = max(2, int(%f / max(dt, 1e-6)))\n"
        "t0 = time.perf_counter(); o.step(n); el = time.perf_counter() - t0\n"
        "print(json.dumps(dict(value=o.n * n / el / 1e6, unit='MLUPS', cores=oracle.num_threads(), "
        "sample='%%d steps of the %%d-site workload (FP64), %%.1f s' %% (n, o.n, el))))\n"
    ) % (ROOT, workload, target_s)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(wl, target_s=15.0):
    """The FP64 oracle on the first instance of the workload, timed on this
    host's cores over a bounded number of steps."""
    import oracle
    g = wl.geoms[0]
    o = oracle.Oracle(g.labels, wl.tau, segment=g.segment, normal=g.normal,
                      iolet_weight=g.iolet_weight)
    oracle_configure(o, wl)
    o.step(2)
    t0 = time.perf_counter()
    o.step(3)
    dt = (time.perf_counter() - t0) / 3
    steps = max(3, int(target_s / max(dt, 1e-6)))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    return dict(value=o.n * steps / el / 1e6, unit="MLUPS", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"{steps} steps of the same {o.n}-site elastic workload (FP64, OpenMP), "
                       f"{el:.1f} s")


def main():
    global ROOF_MIN_LAUNCHES
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4096)
    ap.add_argument("--warmup", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--workload", default="tree", choices=sorted(WORKLOADS),
                    help="main workload (default: the tree the headline is quoted on)")
    ap.add_argument("--launch", default=None,
                    help="JSON launch configuration instead of autotuning")
    ap.add_argument("--probe-copy", action="store_true",
                    help="only run the plain-copy bandwidth probe")
    ap.add_argument("--window", type=int, default=2048,
                    help="minimum launches of the roofline window (0: use the timed steps; "
                         "for profiling runs)")
    args = ap.parse_args()
    ROOF_MIN_LAUNCHES = max(0, args.window)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (got --gpus {args.gpus}); "
              "a batch would shard by instance and one large domain by site ranges with a "
              "halo exchange, neither of which is built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.probe_copy:
        print(json.dumps(dict(copy_probe=copy_probe())), flush=True)
        return
    from paper_2108_08783_amd import workloads
    launch = json.loads(args.launch) if args.launch else None
    dtype = args.dtype
    main_wl = make_workload(args.workload)
    main_run = gpu_run(main_wl, dtype, args.steps, args.warmup, launch=launch,
                       tune_steps=MAIN_TUNE_STEPS)
    print(f"[bench] {args.workload} {dtype}: {main_run['mlups']:.0f} MLUPS over {args.steps} steps, "
          f"{main_run['launch_us']:.2f} us per launch over {main_run['window']}",
          file=sys.stderr, flush=True)
    n = main_run["n"]
    alg_bytes = 2 * 19 * BYTES_PER_POP[dtype] * n
    achieved = alg_bytes / (main_run["launch_us"] * 1e-6) / 1e9
    tr = traffic_from_profiles(dtype, args.workload)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_GBS, 4), traffic=tr,
                    kernel=update_kernel(main_run["info"]), window_launches=main_run["window"],
                    graph_replayed=True,
                    us_per_launch=round(main_run["launch_us"], 3),
                    algorithmic_bytes_per_launch=alg_bytes)

    secondary = {}
    if not args.no_secondary:
        secondary["copy_probe"] = copy_probe()
        sec_steps = min(args.steps, 1024)
        if args.workload != "tree":
            tree = workloads.tree()
        else:
            tree = main_wl
        for dt in ("f16", "bf16", "f32"):
            if args.workload == "tree" and dt == dtype:
                continue
            r = gpu_run(tree, dt, sec_steps, args.warmup)
            secondary["tree_" + dt] = summary(r, dt, with_traffic="tree")
            print(f"[bench] tree {dt}: {r['launch_us']:.2f} us per launch", file=sys.stderr,
                  flush=True)
        bb = gpu_run(tree, "f32", sec_steps, args.warmup, bounceback=True)
        elastic_us = (main_run if (args.workload == "tree" and dtype == "f32")
                      else gpu_run(tree, "f32", sec_steps, args.warmup))["launch_us"]
        secondary["tree_bounceback_f32"] = dict(
            summary(bb, "f32"), elastic_over_bb_time=round(elastic_us / bb["launch_us"], 4))
        if tree is not main_wl:
            del tree
        sw = main_wl if args.workload == "sweep" else workloads.sweep()
        for dt in ("f16", "f32"):
            if args.workload == "sweep" and dt == dtype:
                continue
            r = gpu_run(sw, dt, min(sec_steps, 512), args.warmup // 4)
            secondary["sweep64_" + dt] = summary(r, dt, with_traffic="sweep")
            print(f"[bench] sweep {dt}: {r['launch_us']:.2f} us per launch", file=sys.stderr,
                  flush=True)
        if sw is not main_wl:
            del sw
        tube = main_wl if args.workload == "tube" else workloads.tube32()
        for dt in ("f32", "f16"):
            if args.workload == "tube" and dt == dtype:
                continue
            r = gpu_run(tube, dt, sec_steps, args.warmup)
            secondary["tube_cache_resident_" + dt] = summary(r, dt, with_traffic="tube")
            print(f"[bench] tube {dt}: {r['launch_us']:.2f} us per launch", file=sys.stderr,
                  flush=True)
        del tube
        # the paper's R = 100 dx verification cylinder (41.9M sites, 6.4 GB
        # of FP32 populations): 1000 iterations beside its Table 1 entry
        from paper_2108_08783_amd import verification
        row = verification.timing([100], "f32")[0]
        secondary["paper_cylinder_R100_f32"] = dict(
            sites=row["sites"], elastic_s_per_1000=round(row["elastic_s"], 4),
            rigid_s_per_1000=round(row["rigid_s"], 4), elastic_glups=round(row["elastic_glups"], 2),
            roofline_frac=round(2 * 19 * 4 * row["elastic_glups"] * 1e9 / (PEAK_GBS * 1e9), 4),
            paper_elastic_s_per_1000=row["paper_elastic_s"], paper_cores=6000)
        print(f"[bench] paper cylinder R=100: {row['elastic_s']:.3f} s per 1000 iterations",
              file=sys.stderr, flush=True)
        # the warm-start network on one sample per tree site
        from paper_2108_08783_amd import mlp
        nb = mlp.bench(7_484_227, reps=5)
        secondary["mlp_7M_samples"] = nb
        print(f"[bench] network: {json.dumps(nb)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu and args.workload == "tree":
        cpu = cpu_baseline(main_wl)
        print(f"[bench] oracle: {cpu['value']:.1f} MLUPS on {cpu['cores']} threads",
              file=sys.stderr, flush=True)
        secondary["oracle_1_thread"] = cpu_one_thread(args.workload)
        print(f"[bench] oracle, 1 thread: {secondary['oracle_1_thread']['value']:.2f} MLUPS",
              file=sys.stderr, flush=True)

    info = main_run["info"]
    out = dict(
        metric=METRIC, value=round(main_run["mlups"], 1), unit="MLUPS", n_gpus=1,
        steps=args.steps, warmup=args.warmup,
        ms_per_step=round(main_run["wall_s"] * 1e3 / args.steps, 5),
        higher_is_better=True, scaling="strong", vs_baseline=None, dtype=dtype,
        data="synthetic",
        config=dict(workload=WORKLOADS[args.workload][1],
                    sites=n, boundary_sites=info["n_boundary"], storage=dtype,
                    index_bits=info["index_bits"], block=info["block_size"],
                    xcd_remap=info["xcd_remap"], nontemporal=info["nontemporal"],
                    boundary_fused=info["boundary_fused"], sites_per_lane=info["sites_per_lane"],
                    timed_steps_graph_replayed=args.steps >= 128, parallelism="single GPU",
                    autotune_trial_steps=MAIN_TUNE_STEPS),
        roofline=roofline,
        cpu_baseline=cpu,
        secondary=secondary,
        bytes_per_site=dict(algorithmic=2 * 19 * BYTES_PER_POP[dtype],
                            model=round(info["bytes_per_site_model"], 2)),
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
