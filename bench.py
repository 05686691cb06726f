"""Benchmark of the Shan-Chen hot path on one MI355X: MLUPS and the fraction of the HBM roofline.

A "step" of this benchmark is one test period of the workload: K lattice time steps (fused
stream-collide kernel + blowing-agent source) followed by the test pass (gas labelling, bubble
statistics, FP64 EOS/Laplacian merge criterion, FP64 totals), i.e. one pass of every part of the
hot path.  Inputs (the populations) are resident in HBM before timing starts.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload foam_3d] [--storage f32]
                  [--compute auto] [--variants]

Prints one JSON line.  `value` is MLUPS (million lattice-node updates per second) of the whole
job; `roofline` is the step kernel's algorithmic bytes per launch over its HIP-event-measured
average duration on the simulation stream, against the 8 TB/s HBM peak; `cpu_baseline` is the
FP64 CPU oracle timed on a bounded sample of the same workload on this host.  With the default
workload the same line also carries the two system patterns: `precision` (the 512^3 foam with
FP32, FP16 and BF16 storage, and each storage type's error against the FP64 oracle on a
two-phase box) and `batching` (the 4096-box batch in one persistent launch against the same kind
of boxes run one at a time).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = ("foam_3d", "foam_2d", "two_bubble", "foam_3d_large", "batch", "mixture_2d",
             "mixture_3d", "gas_rich_3d")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="foam_3d", choices=WORKLOADS)
    ap.add_argument("--storage", default="f32", choices=("f32", "f16", "bf16"))
    ap.add_argument("--compute", default="auto", choices=("auto", "f32", "f64"))
    ap.add_argument("--tile", default=None, help="tx,ty,tz[,variant] of the step kernel")
    ap.add_argument("--barrier", action="store_true",
                    help="run the modified Shan-Chen barrier (owners built at the test passes, "
                         "frontier nodes re-stepped by a fix-up kernel)")
    ap.add_argument("--gravity", default=None, metavar="GX,GY[,GZ]",
                    help="body force (rho - rho0) g in the step (drainage), e.g. 0,0,-1e-5")
    ap.add_argument("--autotune", action="store_true",
                    help="run the step-kernel autotuner before timing (default: the shape "
                         "stored by paper_1708_01608_amd.tune, else the built-in default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=0,
                    help="oracle steps timed for cpu_baseline after 10 untimed ones (0: 100, or "
                         "fewer where 100 would take over a minute)")
    ap.add_argument("--no-patterns", action="store_true",
                    help="default workload only: leave out the precision and batching keys")
    ap.add_argument("--precision-steps", type=int, default=4,
                    help="bench steps (K lattice steps each) timed per storage type at 512^3")
    ap.add_argument("--variants", action="store_true",
                    help="also time FP32-compute / 16-bit storage variants (extra JSON lines)")
    ap.add_argument("--batch-sample", type=int, default=32, metavar="N",
                    help="batch workload: boxes also run one at a time for comparison (0: none)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also run a plain device copy of BYTES bytes (calibrates the HBM "
                         "counters of a profiler run against a kernel of known traffic)")
    return ap.parse_args()


def workload_spec(name):
    from paper_1708_01608_amd import workloads as W

    return {"foam_3d": W.foam_3d, "foam_2d": W.foam_2d, "two_bubble": W.two_bubble,
            "foam_3d_large": W.foam_3d_large, "mixture_2d": W.mixture_2d,
            "mixture_3d": W.mixture_3d, "gas_rich_3d": W.gas_rich_3d}[name]()


METRIC_FULL = ("Shan-Chen MLUPS & % of HBM roofline; FP16-store/batched vs FP32 at fixed err")


def bytes_per_node(q, storage, components=1):
    """Algorithmic bytes per node and step: every population read once and written once."""
    return components * 2 * q * (4 if storage == "f32" else 2)


def kernel_hash(files=("sc_step.hip", "sc_stepcore.hpp", "sc_device.hpp")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1708_01608_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_kernel_hash():
    return kernel_hash()


def mixture_kernel_hash():
    return kernel_hash(("sc_step2c.hip", "sc_stepcore.hpp", "sc_device.hpp"))


def batch_kernel_hash():
    return kernel_hash(("sc_batch.hip", "sc_stepcore.hpp", "sc_device.hpp"))


def batch_traffic_from_profile(compute, rows_per_thread, node_steps):
    """HBM bytes of one whole-batch launch from the committed counter summary, if it was taken
    on the current batch kernel source, node-slot count and workload; else None."""
    path = os.path.join(ROOT, "profiles", f"batch_counters_{compute}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if (d.get("kernel_hash") != batch_kernel_hash() or d.get("rows_per_thread") != rows_per_thread
            or d.get("node_steps") != node_steps):
        return None
    return d.get("hbm_bytes_per_launch")


def traffic_from_profile(workload, storage, compute, tile):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current step kernel source with the same tile; else None."""
    path = os.path.join(ROOT, "profiles", f"step_counters_{workload}_{storage}_{compute}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    h = mixture_kernel_hash() if workload.startswith("mixture") else step_kernel_hash()
    if d.get("kernel_hash") != h or list(d.get("tile", [])) != list(tile):
        return None
    return d.get("hbm_bytes_per_launch")


def run_gpu(spec, args, storage, compute, steps, warmup, tile=None):
    import torch

    from paper_1708_01608_amd import sc

    variant = 0
    if tile is not None and len(tile) == 4:
        tile, variant = tile[:3], tile[3]
    gravity = [float(v) for v in args.gravity.split(",")] if args.gravity else None
    sim = sc.Sim.from_spec(spec, storage=storage, compute=compute, tile=tile, variant=variant,
                           barrier=args.barrier, gravity=gravity)
    sim.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    if tile is None and args.autotune:
        sim.autotune(trials=3)
    K = spec.K
    for _ in range(warmup):
        sim.step(K)
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K * steps)  # `steps` bench steps of K lattice steps and one test pass each
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms, launches = sim.profile_read(sc.SC_KERNEL_STEP)
    src_ms, src_n = sim.profile_read(sc.SC_KERNEL_SOURCE)
    test_ms, test_n = sim.profile_read(sc.SC_KERNEL_TEST)
    sim.profile(False)
    tile_used = sim.step_config()
    comp = sim.compute_type()
    sim.close()
    return dict(wall=wall, step_ms=step_ms, launches=launches, src_ms=src_ms, src_n=src_n,
                test_ms=test_ms, test_n=test_n, tile=tile_used, compute=comp)


def cpu_baseline_leg(spec, sample_steps, err_spec=None, err_steps=0, err_fields=None):
    """The FP64 CPU oracle on this host (the only part of the benchmark that runs it).

    (1) Its speed on a sample of the workload: 10 untimed steps, then `sample_steps` timed ones
    (100 unless that would take over a minute), test passes off.  (2) With err_fields, the FP64
    reference of the precision error box at err_steps, against which the GPU fields of each
    storage type (err_fields[(storage, compute)] = (rho, u)) are stated: rho as the maximum
    pointwise relative error, u as the maximum error over max |u| (u passes through zero)."""
    import numpy as np

    from oracle import OracleSim, num_threads

    o = OracleSim(spec.q, spec.nx, spec.ny, spec.nz, spec.tau, spec.G, spec.rho_l, spec.rho_g,
                  spec.amp, spec.seed, spec.theta, 0, spec.film_max,
                  two_component=spec.two_component)
    o.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    warm = 10
    t0 = time.perf_counter()
    o.step(warm)
    per_step = (time.perf_counter() - t0) / warm
    if sample_steps <= 0:
        sample_steps = int(max(10, min(100, 60.0 / max(per_step, 1e-6))))
    t0 = time.perf_counter()
    o.step(sample_steps)
    dt = time.perf_counter() - t0
    base = dict(value=round(spec.N * sample_steps / dt / 1e6, 3), unit="MLUPS",
                cores=num_threads(), kind="oracle",
                sample=f"{spec.name} {spec.nx}x{spec.ny}x{spec.nz}, {sample_steps} oracle steps "
                       f"after {warm} untimed (FP64 collide-stream + source; test passes off), "
                       f"{dt:.1f} s")
    del o
    errors = None
    if err_fields:
        e = OracleSim(err_spec.q, err_spec.nx, err_spec.ny, err_spec.nz, err_spec.tau,
                      err_spec.G, err_spec.rho_l, err_spec.rho_g, err_spec.amp, err_spec.seed,
                      err_spec.theta, err_spec.K, err_spec.film_max)
        e.seed_nuclei(err_spec.centres, err_spec.radii, err_spec.budgets, err_spec.rate)
        e.step(err_steps)
        ro, uo, _ = e.fields()
        umax = float(np.max(np.abs(uo)))
        errors = {}
        for (storage, compute), (rg, ug) in err_fields.items():
            errors[f"{storage} storage / {compute} compute"] = {
                "rho": float(f"{np.max(np.abs(rg - ro) / ro):.3e}"),
                "u": float(f"{np.max(np.abs(ug - uo)) / umax:.3e}")}
    return base, errors


def copy_probe(nbytes):
    """A device-to-device copy of a known size: under a counter run it calibrates the HBM
    counters (bytes each counter reports per byte really moved)."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_probe_bytes": nbytes,
                      "copy_GBps": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


def batch_measure(compute, runs, warmup, sample):
    """The batching pattern: every box of the 4096-box workload in one persistent launch (one
    run = the whole job, every box to its merge, topological merge or max_steps), then `sample`
    of the same boxes one at a time through sc_create/sc_step for comparison."""
    import torch

    from paper_1708_01608_amd import sc
    from paper_1708_01608_amd import workloads as W

    spec = W.batch()
    b = sc.Batch(spec, compute=compute)
    rows_per_thread, tune_ms = b.tune(trial_steps=50)
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = 0.0
    for _ in range(runs):
        res, ms = b.run()
        kms += ms
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    node_steps = sum(int(spec.nx[k]) * int(spec.ny[k]) * res[k]["steps_run"] for k in range(spec.n))
    mlups = node_steps * runs / wall / 1e6
    achieved = 72.0 * node_steps / (kms / runs / 1e3) / 1e9
    merged = sum(1 for r in res if r["merge_step"] >= 0)
    topo = sum(1 for r in res if r["topo_step"] >= 0 and r["merge_step"] < 0)
    b.close()
    ns = max(0, min(sample, spec.n))
    picks = list(range(0, spec.n, max(1, spec.n // max(ns, 1))))[:ns]
    t1 = time.perf_counter()
    ns1 = 0
    for k in picks:
        s = spec.instance(k)
        g = sc.Sim.from_spec(s, compute=compute)
        g.seed_nuclei(s.centres, s.radii, s.budgets, 0.0)
        while g.t < spec.max_steps and not g.merge_events() and not g.topo_events():
            g.step(spec.K)
        ns1 += s.N * g.t
        g.close()
    one_by_one = ns1 / (time.perf_counter() - t1) / 1e6 if picks else None
    return dict(spec=spec, mlups=mlups, wall=wall, kms=kms, achieved=achieved,
                node_steps=node_steps, merged=merged, topo=topo,
                rows_per_thread=rows_per_thread, tune_ms=tune_ms, one_by_one=one_by_one,
                sample=len(picks))


def run_batch(args):
    """--workload batch: the batching pattern as the benchmark's own line."""
    compute = "f64" if args.compute == "auto" else args.compute
    m = batch_measure(compute, args.steps, args.warmup, args.batch_sample)
    spec = m["spec"]
    out = {
        "metric": "Shan-Chen MLUPS & % of HBM roofline",
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["wall"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": compute,
        "data": "synthetic",
        "config": {"workload": "batch", "lattice": "D2Q9", "boxes": spec.n,
                   "nodes": int((spec.nx * spec.ny).sum()), "node_steps": m["node_steps"],
                   "max_steps": spec.max_steps, "test_every": spec.K, "storage": "f32",
                   "compute": compute, "rows_per_thread": m["rows_per_thread"],
                   "tune_ms_rb124": [round(v, 2) for v in m["tune_ms"]],
                   "merged_by_criterion": m["merged"],
                   "merged_topologically_first": m["topo"]},
        "roofline": {"bound": "hbm", "achieved": round(m["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": batch_traffic_from_profile(compute, m["rows_per_thread"],
                                                           m["node_steps"]),
                     "kernel": "k_batch", "bytes_per_node_step": 72,
                     "kernel_ms": round(m["kms"] / args.steps, 3)},
        "one_by_one_MLUPS": round(m["one_by_one"], 1) if m["one_by_one"] is not None else None,
        "one_by_one_sample": f"{m['sample']} boxes through sc_create/sc_step",
    }
    print(json.dumps(out), flush=True)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)


def precision_measure(args):
    """The precision pattern on the 512^3 foam (D3Q19, 400 nuclei, tau 0.9, K 50): the step kernel
    with FP32 storage (FP64 and FP32 arithmetic) against FP16 and BF16 shifted storage (FP32
    arithmetic), each timed over `precision_steps` bench steps after one untimed."""
    from paper_1708_01608_amd import sc

    spec = workload_spec("foam_3d_large")
    rows = {}
    march = {}
    for storage, compute in (("f32", "f64"), ("f32", "f32"), ("f16", "f32"), ("bf16", "f32")):
        r = run_gpu(spec, args, storage, compute, args.precision_steps, 1)
        b = bytes_per_node(spec.q, storage) * spec.N
        avg_s = r["step_ms"] / 1e3 / max(r["launches"], 1)
        # the storage type's own memory pattern, marched with the run's tiles, no arithmetic
        key = (storage, tuple(r["tile"][:3]))
        if key not in march:
            try:
                march[key] = sc.pattern_probe(spec.nx, spec.ny, spec.nz, storage, key[1], 3)[1]
            except sc.ScError as e:  # a ceiling, not the measurement: report null
                print(f"pattern probe failed: {e}", file=sys.stderr)
                march[key] = None
        rows[f"{storage} storage / {compute} compute"] = {
            "MLUPS": round(spec.N * args.precision_steps * spec.K / r["wall"] / 1e6, 1),
            "stencil_only_MLUPS": round(spec.N / avg_s / 1e6, 1),
            "bytes_per_node": bytes_per_node(spec.q, storage),
            "avg_launch_us": round(avg_s * 1e6, 1),
            "achieved_GBps": round(b / avg_s / 1e9, 1),
            "frac": round(b / avg_s / 1e9 / HBM_PEAK_GBS, 4),
            "pattern_march_GBps": round(march[key], 1) if march[key] else None,
            "frac_of_pattern_march": (round(b / avg_s / 1e9 / march[key], 4) if march[key]
                                      else None)}
    return spec, rows


def error_box_fields(steps):
    """GPU fields of the precision error box after `steps` steps, per storage type."""
    from paper_1708_01608_amd import sc
    from paper_1708_01608_amd import workloads as W

    spec = W.precision_error_box()
    fields = {}
    for storage, compute in (("f32", "f64"), ("f32", "f32"), ("f16", "f32"), ("bf16", "f32")):
        g = sc.Sim.from_spec(spec, storage=storage, compute=compute)
        g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
        g.step(steps)
        rho, u, _ = g.fields()
        g.close()
        fields[(storage, compute)] = (rho.astype("float64"), u.astype("float64"))
    return spec, fields


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; the multi-GPU path (slab "
                                   "domain decomposition) is a design note, not code",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    from paper_1708_01608_amd import sc

    if not os.path.exists(sc.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    if args.workload == "batch":
        run_batch(args)
        return
    spec = workload_spec(args.workload)
    comps = 1 if spec.two_component is None else 2
    if comps == 2 and (args.barrier or args.gravity or
                       (args.storage == "f32") == (args.compute == "f32") and
                       args.compute != "auto"):
        print(json.dumps({"error": "the mixture runs FP32 storage with FP64 arithmetic or 16-bit "
                                   "storage with FP32 arithmetic, no barrier, no gravity"}))
        sys.exit(2)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    r = run_gpu(spec, args, args.storage, args.compute, args.steps, args.warmup, tile)
    lattice_steps = args.steps * spec.K
    mlups = spec.N * lattice_steps / r["wall"] / 1e6
    # the barrier leaves the marching kernel as it is (its fix-up re-steps the few frontier nodes)
    bpn = bytes_per_node(spec.q, args.storage, comps)
    bytes_per_launch = bpn * spec.N
    avg_s = r["step_ms"] / 1e3 / max(r["launches"], 1)
    achieved = bytes_per_launch / avg_s / 1e9
    # the counters were taken on the plain kernels
    traffic = (None if args.barrier or args.gravity else
               traffic_from_profile(args.workload, args.storage, r["compute"], r["tile"]))
    out = {
        "metric": "Shan-Chen MLUPS & % of HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["compute"] if args.storage == "f32" else "f32",
        "data": "synthetic",
        "config": {
            "workload": spec.name,
            "lattice": f"D{spec.d}Q{spec.q}",
            "box": [spec.nx, spec.ny, spec.nz],
            "nodes": spec.N,
            "nuclei": int(len(spec.radii)),
            "storage": args.storage,
            "compute": r["compute"],
            "tau": spec.tau,
            "G": spec.G,
            "test_every": spec.K,
            "lattice_steps_per_step": spec.K,
            "step_tile": list(r["tile"]),
            "barrier": bool(args.barrier),
            "gravity": args.gravity,
            "components": comps,
            "shape_source": ("--tile" if args.tile else "autotune" if args.autotune
                             else "tuned_shapes.json or default"),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": ("k_mix" if comps == 2 else "k_step") + ("3d" if spec.q == 19 else "2d"),
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_s * 1e6, 2),
            "launches": r["launches"],
        },
        "stencil_only_MLUPS": round(spec.N / avg_s / 1e6, 1),
        "breakdown_ms": {
            "step_kernel": round(r["step_ms"], 3),
            "source": round(r["src_ms"], 3),
            "test_pass": round(r["test_ms"], 3),
            "wall": round(r["wall"] * 1e3, 3),
        },
    }
    # the copy ceiling on a buffer of the launch's size, at least 256 MiB so that it is HBM's
    copy_gbs, read_gbs = sc.hbm_probe(max(min(bytes_per_launch // 2, 2550136832), 1 << 28), 5)
    out["roofline"]["measured_copy_GBps"] = round(copy_gbs, 1)
    out["roofline"]["measured_read_GBps"] = round(read_gbs, 1)
    out["roofline"]["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    if spec.q == 19 and spec.two_component is None:
        # the step's own memory pattern with its arithmetic left out: flat (one node per
        # thread) and marching the step kernel's tiles
        tx, ty, tz = r["tile"][:3]
        try:
            flat_gbs, march_gbs = sc.pattern_probe(spec.nx, spec.ny, spec.nz, args.storage,
                                                   (tx, ty, tz), 5)
        except sc.ScError as e:  # a ceiling, not the measurement: report null
            print(f"pattern probe failed: {e}", file=sys.stderr)
            flat_gbs = march_gbs = None
        out["roofline"]["measured_pattern_flat_GBps"] = round(flat_gbs, 1) if flat_gbs else None
        out["roofline"]["measured_pattern_march_GBps"] = (round(march_gbs, 1) if march_gbs
                                                           else None)
        out["roofline"]["frac_of_pattern_march"] = (round(achieved / march_gbs, 4) if march_gbs
                                                    else None)
    patterns = (args.workload == "foam_3d" and not args.no_patterns and not args.barrier and
                not args.gravity and args.tile is None and args.storage == "f32")
    err_spec = err_fields = None
    err_steps = 100
    if patterns:
        pspec, rows = precision_measure(args)
        err_spec, err_fields = error_box_fields(err_steps)
        base = rows["f32 storage / f64 compute"]["MLUPS"]
        out["precision"] = {
            "workload": f"{pspec.name} {pspec.nx}^3 D3Q19, {len(pspec.radii)} nuclei, tau "
                        f"{pspec.tau}, K {pspec.K}; 16-bit storage holds f_i - w_i rho_l",
            "runs": rows,
            "f16_vs_f32_storage_MLUPS": round(rows["f16 storage / f32 compute"]["MLUPS"] / base, 3),
            "bf16_vs_f32_storage_MLUPS": round(rows["bf16 storage / f32 compute"]["MLUPS"] / base,
                                               3),
            "error_vs_fp64": None,
            "error_box": f"{err_spec.name}: two spheres R {err_spec.radii[0]:g}, "
                         f"{err_spec.nx}x{err_spec.ny}x{err_spec.nz}, tau {err_spec.tau}, "
                         f"rho_l {err_spec.rho_l}, after {err_steps} steps (both spheres persist)",
        }
        bm = batch_measure("f64", 1, 1, args.batch_sample)
        out["batching"] = {
            "workload": f"batch: {bm['spec'].n} D2Q9 two-bubble boxes 64..256 per side, "
                        f"to the merge or {bm['spec'].max_steps} steps, one persistent launch",
            "MLUPS": round(bm["mlups"], 1),
            "job_s": round(bm["wall"], 3),
            "frac": round(bm["achieved"] / HBM_PEAK_GBS, 4),
            "one_by_one_MLUPS": (round(bm["one_by_one"], 1) if bm["one_by_one"] is not None
                                 else None),
            "one_by_one_sample": f"{bm['sample']} boxes through sc_create/sc_step",
            "batched_vs_one_by_one": (round(bm["mlups"] / bm["one_by_one"], 1)
                                      if bm["one_by_one"] else None),
        }
        # the line now carries both halves of the metric: the FP32 roofline and the 16-bit /
        # batched forms against plain FP32 with their stated errors
        out["metric"] = METRIC_FULL
    if not args.no_cpu_baseline:
        out["cpu_baseline"], errors = cpu_baseline_leg(spec, args.cpu_sample_steps, err_spec,
                                                       err_steps, err_fields)
        if patterns:
            out["precision"]["error_vs_fp64"] = errors
    print(json.dumps(out), flush=True)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    if args.variants:
        # the mixture pairs 16-bit storage with FP32 arithmetic only
        combos = ((("f32", "f32"),) if comps == 1 else ()) + (("f16", "f32"), ("bf16", "f32"))
        for storage, compute in combos:
            rv = run_gpu(spec, args, storage, compute, args.steps, args.warmup, tile)
            b = bytes_per_node(spec.q, storage, comps) * spec.N
            a = b / (rv["step_ms"] / 1e3 / max(rv["launches"], 1)) / 1e9
            print(json.dumps({"variant": f"{storage} storage / {compute} compute",
                              "workload": spec.name,
                              "MLUPS": round(spec.N * lattice_steps / rv["wall"] / 1e6, 1),
                              "step_kernel_GBps": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                              "avg_launch_us": round(rv["step_ms"] * 1e3 / max(rv["launches"], 1), 2)}),
                  flush=True)


if __name__ == "__main__":
    main()
