"""Benchmark of the fused two-component D2Q9 step on one MI355X.

Workload (default): the batch of 256 uneven sinusoidal channels (lambda drawn
from {64, 128, 256, 512}, h0 = lambda/8, a = lambda/16, contact angle, viscosity
ratio and forcing drawn per instance with numpy default_rng(1601)), all
advanced together, FP32 populations.  One step = one pass of the whole hot path
(moments, density halo, interaction and wall force, mixture state, regularized
collision, streaming with bounce-back) over every instance.

Prints one JSON line: MLUPS (fluid-node updates per second, both species per
update), the HBM roofline of the step kernel, and the FP64 oracle timed on the
host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2-comp MLUPS & % HBM roofline; critical-pressure solves/hr batched vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per fluid-node update: 2 species x 9 populations, each
# read once and written once (4 bytes in FP32, 2 in the 16-bit formats).  The
# 16-bit formats also move a reference-density pair per node (8 bytes in
# D2Q9 and D3Q19); that is this design's overhead, not the method's, and is
# left out of the algorithmic count.
BYTES_PER_NODE = {"f32": 144, "f16": 72, "bf16": 72}
# D3Q19: 2 species x 19 populations read and written once per update.
BYTES_PER_NODE_3D = {"f32": 304, "f16": 152, "bf16": 152}


def workload(name):
    import synth
    if name == "batch":
        cfgs = synth.config_batch(n_inst=256, seed=1601)
        desc = ("batch of 256 sinusoidal channels, lambda ~ U{64,128,256,512}, h0 = lambda/8, "
                "a = lambda/16, theta ~ U(30,150) deg, viscosity ratio ~ logU(0.1,10), "
                "Bo ~ logU(10^-1.5,10^1.5), default_rng(1601)")
    elif name == "channel":
        cfgs = [synth.config_channel(lam=256, theta=90.0, g=2e-6)]
        desc = "sinusoidal channel lambda=256, h0=32, a=16, 1024x98, slug 1.5 lambda"
    elif name == "poiseuille":
        cfgs = [synth.config_poiseuille()]
        desc = "two-layer Poiseuille 256x64 (+2 wall rows), tau 0.6/1.5, g=1e-6"
    elif name == "droplet":
        cfgs = [synth.config_droplet(n=128, r=20.0)]
        desc = "free droplet 128x128 periodic, R=20"
    else:
        raise SystemExit("unknown workload %r" % name)
    return cfgs, desc


def tube_config():
    """The D3Q19 tube: 512 x 128 x 128, r(x) = 40 + 16 cos(2 pi x / 256), an oil
    slug of 384 nodes starting at x = 64."""
    import synth
    return synth.config_tube(lam=256, r0=40.0, a=16.0, nx=512, ny=128, nz=128, theta=60.0,
                             tau=(1.0, 1.0), g=1e-6, slug_len=384, slug_x0=64)


def cpu_baseline_tube(seconds):
    """The FP64 D3Q19 oracle on a bounded sample: a tube of the same shape
    family scaled down by 4 (128 x 34 x 34, r(x) = 10 + 4 cos(2 pi x / 64)),
    stepped until about `seconds` have passed."""
    import synth
    from oracle import lbm3d as o3
    from oracle import lbm as orc

    cfg = synth.config_tube(lam=64, r0=10.0, a=4.0, nx=128, ny=34, nz=34, theta=60.0,
                            tau=(1.0, 1.0), g=1e-6, slug_len=96, slug_x0=16)
    mask = synth.mask3_of(cfg)
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"])
    L = o3.Lattice3(p, mask, synth.rho03_of(cfg, mask))
    nf = int(mask.sum())
    L.step(1)
    t0 = time.perf_counter()
    L.step(3)
    dt = time.perf_counter() - t0
    n = max(3, int(seconds / max(dt / 3, 1e-6)))
    t0 = time.perf_counter()
    L.step(n)
    dt = time.perf_counter() - t0
    return {"value": nf * n / dt / 1e6, "unit": "MLUPS", "cores": orc.threads_used(),
            "kind": "oracle",
            "sample": "FP64 D3Q19 oracle, the tube scaled down by 4 (128x34x34, %d fluid nodes), "
                      "%d steps in %.1f s" % (nf, n, dt)}


def bench_tube(args):
    """MLUPS of the D3Q19 step on the 512 x 128 x 128 sinusoidal tube."""
    import torch
    import synth
    from paper_1601_00918_amd.binding3d import Simulation3D

    cfg = tube_config()
    if args.wall_interp:
        cfg = dict(cfg, wall_interp=True)
    nf = int(synth.mask3_of(cfg).sum())
    sim = Simulation3D(cfg, storage=args.storage)
    if args.tiling:
        bx, by, strip = (int(v) for v in args.tiling.split(","))
        sim.set_tiling(bx, by, strip)
    print("bench: tube3d, %d fluid nodes, workspace %.2f GB, tiling %s" %
          (nf, sim.workspace_bytes / 1e9, sim.tiling()), file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    sim.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    mlups = nf * args.steps / (ms / 1e3) / 1e6
    mon = sim.monitors()
    print("bench: %.4f ms/step (events), wall %.3f s, %.0f MLUPS, bad nodes %d" %
          (ms_per_step, wall, mlups, mon["bad_nodes"]), file=sys.stderr, flush=True)
    bytes_per_launch = BYTES_PER_NODE_3D[args.storage] * nf
    achieved = bytes_per_launch / (ms_per_step / 1e3) / 1e9
    traffic = (None if args.tiling or args.wall_interp else
               measured_traffic(args.storage, "step3_kernel_tube_traffic.txt", KERNEL3_SOURCES))
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "D3Q19 sinusoidal tube 512x128x128, r(x) = 40 + 16 cos(2 pi x/256), "
                               "oil slug 384, theta 60 deg, g = 1e-6" +
                               (", interpolated walls" if args.wall_interp else ""),
                   "fluid_nodes": nf, "storage": args.storage, "tiling": list(sim.tiling()[:3])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (round(traffic / (ms_per_step / 1e3) / 1e9, 1)
                                 if traffic else None),
                     "traffic_bytes_per_launch": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_tube(args.cpu_seconds)
    return out


def fluid_nodes(cfgs):
    import synth
    return int(sum(int(synth.mask_of(c).sum()) for c in cfgs))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_configs():
    """The oracle's timing set: C1 (droplet 128^2), C2 (two-layer Poiseuille
    256 x 64), C3 (channel lambda = 256, 1024 x 98) and a stratified subset of
    the 256-channel batch (its first two instances of each wavelength)."""
    import synth
    batch = synth.config_batch(n_inst=256, seed=1601)
    subset = []
    for lam in (64, 128, 256, 512):
        subset += [c for c in batch if c["lam"] == lam][:2]
    return [("C1 droplet 128x128 R=20", [synth.config_droplet(n=128, r=20.0)]),
            ("C2 two-layer Poiseuille 256x64", [synth.config_poiseuille()]),
            ("C3 channel lambda=256 1024x98", [synth.config_channel(lam=256, theta=90.0, g=2e-6)]),
            ("C4 subset: 8 channels of the batch, 2 per lambda", subset)]


def cpu_baseline(seconds):
    """The FP64 oracle on the host cores, as it stands, on bounded samples:
    each configuration of cpu_baseline_configs() at one thread and at every
    thread the oracle uses by default (OMP_NUM_THREADS, else all cores),
    stepped for about seconds / 8 each.  The reported value is the batch
    subset at the default thread count, the sample of the benchmark's own
    workload."""
    import numpy as np  # noqa: F401
    import synth
    from oracle import lbm as orc

    nthreads = orc.threads_used()
    per = seconds / 8.0
    runs = []
    for name, cfgs in cpu_baseline_configs():
        lats = []
        nf = 0
        for c in cfgs:
            mask = synth.mask_of(c)
            nf += int(mask.sum())
            lats.append(orc.Lattice(orc.Params(c["nx"], c["ny"], tau=c["tau"], G=c["G"],
                                               rho_s=c["rho_s"], g=c["g"],
                                               periodic_y=(c["kind"] == "box")),
                                    mask, synth.rho0_of(c, mask)))
        for threads in (1, nthreads):
            orc.set_threads(threads)
            for L in lats:
                L.step(1)
            t0 = time.perf_counter()
            for L in lats:
                L.step(1)
            dt1 = time.perf_counter() - t0
            n = max(1, int(per / max(dt1, 1e-6)))
            t0 = time.perf_counter()
            for L in lats:
                L.step(n)
            dt = time.perf_counter() - t0
            runs.append({"config": name, "threads": threads, "fluid_nodes": nf, "steps": n,
                         "seconds": round(dt, 2), "mlups": round(nf * n / dt / 1e6, 3)})
            if threads == nthreads == 1:
                break
    orc.set_threads(nthreads)
    main = next(r for r in runs if r["config"].startswith("C4") and r["threads"] == nthreads)
    return {"value": main["mlups"], "unit": "MLUPS", "cores": nthreads, "kind": "oracle",
            "sample": "FP64 oracle, %s (%d fluid nodes), %d steps in %.1f s at %d threads; "
                      "C1-C3 and 1-thread runs in 'runs'" % (
                          main["config"], main["fluid_nodes"], main["steps"], main["seconds"],
                          nthreads),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "runs": runs}


def gpu_configs_mlups(steps=200, warmup=20):
    """GPU MLUPS of the oracle's timing set (C1-C3 and the batch subset), FP32,
    each advanced alone (C1-C3 fit in the device cache, so no HBM fraction is
    claimed for them)."""
    import torch
    import synth
    from paper_1601_00918_amd import Simulation
    out = []
    for name, cfgs in cpu_baseline_configs():
        nf = sum(int(synth.mask_of(c).sum()) for c in cfgs)
        sim = Simulation(cfgs)
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        sim.step(steps)
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out.append({"config": name, "fluid_nodes": nf, "ms_per_step": round(ms, 5),
                    "mlups": round(nf / ms / 1e3, 1)})
        del sim
    return out


def other_workloads(steps=200, warmup=20):
    """The other step launches the project measures, timed in the default run
    like the headline one (HIP events on the launch stream): the 256-channel
    batch in binary16 deviation storage, and the D3Q19 tube in FP32 and
    binary16.  Each reports MLUPS, the fraction of 8 TB/s on its algorithmic
    bytes per node, and the measured HBM traffic rate when a counter record
    for the current kernel source exists."""
    import torch
    import synth
    from paper_1601_00918_amd import Simulation
    from paper_1601_00918_amd.binding3d import Simulation3D

    def timed(sim, n):
        sim.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        sim.step(n)
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    def entry(name, storage, nf, ms, bpn, traffic):
        return {"workload": name, "storage": storage, "fluid_nodes": nf,
                "ms_per_step": round(ms, 5), "mlups": round(nf / ms / 1e3, 1),
                "hbm_frac": round(bpn * nf / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": (round(traffic / (ms / 1e3) / 1e9, 1) if traffic else None)}

    out = []
    cfgs, desc = workload("batch")
    nf = fluid_nodes(cfgs)
    sim = Simulation(cfgs, storage="f16")
    ms = timed(sim, steps)
    del sim
    out.append(entry("256-channel batch", "f16", nf, ms, BYTES_PER_NODE["f16"],
                     measured_traffic("f16")))
    cfg = tube_config()
    nf3 = int(synth.mask3_of(cfg).sum())
    for storage in ("f32", "f16"):
        sim = Simulation3D(cfg, storage=storage)
        ms = timed(sim, steps)
        del sim
        out.append(entry("D3Q19 tube 512x128x128", storage, nf3, ms,
                         BYTES_PER_NODE_3D[storage],
                         measured_traffic(storage, "step3_kernel_tube_traffic.txt",
                                          KERNEL3_SOURCES)))
    return out


# Sources of the D2Q9 step kernel; the counter record names their hash.
KERNEL_SOURCES = ("lbm_kernels.hip", "lbm_store.h", "lbm_internal.h")
KERNEL3_SOURCES = ("lbm3d_kernels.hip", "lbm_store.h", "lbm3d_internal.h")


def measured_traffic(storage, record="step_kernel_batch256_traffic.txt",
                     sources=KERNEL_SOURCES):
    """HBM bytes per step launch from a committed FETCH_SIZE / WRITE_SIZE
    counter record (the 256-channel batch by default), scaled by the
    copy-kernel calibration; None when the kernel source has changed since the
    counters were taken or the format was not profiled."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", record)
    csrc = os.path.join(ROOT, "paper_1601_00918_amd", "csrc")
    try:
        rec = json.load(open(rec_path))
        h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                    for f in sources)).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != h or storage not in rec:
        return None
    r = rec[storage]
    return 1024.0 * (r["fetch_kib"] * rec["fetch_scale"] + r["write_kib"] * rec["write_scale"])


def copy_calibration(steps, warmup, nbytes=2 << 30):
    """The bandwidth ceiling: the library's streaming copy kernel
    (lbm_stream_copy: one contiguous chunk per workgroup, 16-byte nontemporal
    loads and stores, every byte read once and written once, like a step)
    over nbytes at several chunk sizes, and torch's own copy kernel beside it.
    Each moves exactly 2 * nbytes per launch, which also calibrates the
    profiler's FETCH_SIZE / WRITE_SIZE counters."""
    import ctypes

    import torch
    from paper_1601_00918_amd import _lib
    lib = _lib.load()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()

    def timed(launch):
        for _ in range(warmup):
            launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            launch()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    rows = []
    for chunk in (64 << 10, 256 << 10, 1 << 20):
        def own():
            st = lib.lbm_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(dst.data_ptr()), nbytes, chunk,
                                     ctypes.c_void_p(stream.cuda_stream))
            if st != 0:
                raise RuntimeError("lbm_stream_copy failed: %d" % st)
        ms = timed(own)
        rows.append({"kernel": "lbm_stream_copy", "chunk_bytes": chunk, "ms": round(ms, 5),
                     "GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1)})
    ms = timed(lambda: dst.copy_(src))
    rows.append({"kernel": "torch copy_", "ms": round(ms, 5),
                 "GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1)})
    assert torch.equal(src, dst)
    best = max(r["GBps"] for r in rows if r["kernel"] == "lbm_stream_copy")
    del src, dst
    return {"workload": "copy", "bytes_per_launch": 2 * nbytes, "runs": rows,
            "ceiling_GBps": best, "ceiling_frac_of_peak": round(best / HBM_PEAK_GBS, 4)}


def solves_per_hour(args):
    """Critical-pressure solves per hour: plain single-instance bisection vs
    batched solves with surrogate brackets, on channels of the batch family
    (lambda ~ U{--lams}, theta ~ U(30, 150) deg, viscosity ratio
    ~ logU(0.1, 10)).  The surrogate is trained first on batched plain solves
    of other channels of the same family; its cost is reported apart.  The
    gain is split into batching (batched plain vs single plain) and the
    surrogate (batched surrogate vs batched plain), each per wavelength class
    as well; single-instance results are checked against the batched ones on
    a stratified subset (--single-per-lam per wavelength)."""
    import numpy as np
    import torch
    import synth
    from paper_1601_00918_amd import _lib
    from paper_1601_00918_amd import surrogate as sg

    SIG, RHO = 0.161, 1.03
    # verbose: the driver prints a line per classified probe (progress of the
    # long phases)
    rules = dict(rel_tol=0.005, chunk_steps=500, still_chunks=3, verbose=1)
    lams = tuple(int(v) for v in args.lams.split(","))
    n_eval = args.solves
    train = synth.config_cp_set(args.train_solves or n_eval, seed=1611, lams=lams)
    evals = synth.config_cp_set(n_eval, seed=1612, lams=lams)
    stream = torch.cuda.Stream()

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = f()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def log(msg):
        print("solves: " + msg, file=sys.stderr, flush=True)

    # 1. training data: batched plain solves of the training channels
    tr, t_data = timed(lambda: sg.solve(train, [sg.plain_bracket(c, SIG, RHO) for c in train],
                                        SIG, RHO, stream=stream, autotune=1, **rules))
    ok = [i for i, r in enumerate(tr) if r["flags"] & ~_lib.CP_UNDECIDED == 0]
    F = np.stack([sg.features(train[i]) for i in ok])
    y = np.log10([tr[i]["bo_crit"] for i in ok])
    sur, t_fit = timed(lambda: sg.Surrogate(synth.mlp_init(918)).fit(
        F, y, np.random.default_rng(0), epochs=600))
    log("training data %d solves in %.1f s, fit %.1f s, validation rmse %.4f" % (
        len(train), t_data, t_fit, sur.sigma_val))
    # 2. batched + surrogate on the evaluation channels (inference included)
    def batched_sur():
        br = sur.brackets(evals, SIG, RHO, k=2.0)
        return sg.solve(evals, br, SIG, RHO, stream=stream, verify_bracket=2, autotune=1,
                        storage=args.storage, **rules)
    bs, t_bs = timed(batched_sur)
    log("batched surrogate %.1f s" % t_bs)
    # 3. batched plain (no surrogate), for the split of the gain
    bp, t_bp = timed(lambda: sg.solve(evals, [sg.plain_bracket(c, SIG, RHO) for c in evals],
                                      SIG, RHO, stream=stream, autotune=1,
                                      storage=args.storage, **rules))
    log("batched: surrogate %.1f s, plain %.1f s for %d solves" % (t_bs, t_bp, n_eval))
    # 4. plain single-instance solves: a stratified subset per wavelength
    subset = []
    for lam in lams:
        subset += [i for i, c in enumerate(evals) if c["lam"] == lam][:args.single_per_lam]
    per_lam = {lam: [] for lam in lams}
    single = {}
    for i in subset:
        c = evals[i]
        r, dt = timed(lambda: sg.solve([c], [sg.plain_bracket(c, SIG, RHO)], SIG, RHO,
                                       stream=stream, **rules)[0])
        single[i] = r
        per_lam[c["lam"]].append(dt)
        log("single lambda %d: %.1f s, %d probes, g_c %.4e (batched surrogate %.4e)" % (
            c["lam"], dt, r["probes"], r["g_crit"], bs[i]["g_crit"]))
    mix = {lam: sum(1 for c in evals if c["lam"] == lam) / n_eval for lam in lams}
    t_single = sum(mix[lam] * float(np.mean(per_lam[lam])) for lam in lams)
    diffs = [abs(bs[i]["g_crit"] / single[i]["g_crit"] - 1) for i in subset]
    plain_rate = 3600.0 / t_single
    rate = 3600.0 * n_eval / t_bs
    by_lam = {}
    for lam in lams:
        idx = [i for i, c in enumerate(evals) if c["lam"] == lam]
        by_lam[str(lam)] = {
            "solves": len(idx), "single_s_mean": round(float(np.mean(per_lam[lam])), 2),
            "probes_batched_surrogate": int(sum(bs[i]["probes"] for i in idx)),
            "probes_batched_plain": int(sum(bp[i]["probes"] for i in idx)),
            "steps_batched_surrogate": int(sum(bs[i]["steps"] for i in idx)),
            "steps_batched_plain": int(sum(bp[i]["steps"] for i in idx))}
    return {
        "metric": "critical-pressure solves/hr, batched + surrogate vs plain single-instance",
        "value": round(rate, 1), "unit": "solves/hr", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": "channels of the batch family, lambda ~ U{%s}, "
                               "theta ~ U(30,150) deg, viscosity ratio ~ logU(0.1,10), "
                               "default_rng(1612); bisection to 0.5 %%, 3-decade plain "
                               "bracket in Bo" % args.lams, "solves": n_eval},
        "plain_single_solves_per_hour": round(plain_rate, 1),
        "speedup": round(rate / plain_rate, 2),
        "batched_plain_solves_per_hour": round(3600.0 * n_eval / t_bp, 1),
        "gain_from_batching": round(t_single * n_eval / t_bp, 2),
        "gain_from_surrogate": round(t_bp / t_bs, 2),
        "probes": {"batched_surrogate": sum(r["probes"] for r in bs),
                   "batched_plain": sum(r["probes"] for r in bp)},
        "by_lambda": by_lam,
        # batched surrogate (args.storage) vs plain single-instance FP32
        "single_checked": len(subset),
        "max_rel_diff_vs_single": round(max(diffs), 5),
        "within_1pct_vs_single": sum(1 for d in diffs if d <= 0.01),
        "surrogate_training": {"solves": len(train), "data_s": round(t_data, 1),
                               "fit_s": round(t_fit, 2), "val_rmse_log10": sur.sigma_val},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--wall-interp", action="store_true",
                    help="--workload tube3d: the tube's wall at its analytic position "
                         "(interpolated bounce-back)")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tiling", default=None,
                    help="BX,STRIP for every instance (default: the library's default); "
                         "BX,BY,STRIP for --workload tube3d")
    ap.add_argument("--solves", type=int, default=128,
                    help="problems per set for --workload solves")
    ap.add_argument("--train-solves", type=int, default=0,
                    help="training problems for --workload solves (default: --solves)")
    ap.add_argument("--lams", default="64,128",
                    help="wavelengths of the --workload solves problems")
    ap.add_argument("--single-per-lam", type=int, default=2,
                    help="single-instance solves per wavelength for --workload solves")
    ap.add_argument("--reg-order", type=int, default=2, choices=(2, 3),
                    help="Hermite order of the regularization for the D2Q9 workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1601_00918_amd import Simulation

    if args.workload == "copy":
        print(json.dumps(copy_calibration(args.steps, args.warmup)), flush=True)
        return
    if args.workload == "solves":
        print(json.dumps(solves_per_hour(args)), flush=True)
        return
    if args.workload == "tube3d":
        print(json.dumps(bench_tube(args)), flush=True)
        return
    cfgs, desc = workload(args.workload)
    if args.reg_order != 2:
        cfgs = [dict(c, reg_order=args.reg_order) for c in cfgs]
        desc += "; third-order Hermite regularization"
    nf = fluid_nodes(cfgs)
    sim = Simulation(cfgs, storage=args.storage)
    if args.tiling:
        bx, strip = (int(v) for v in args.tiling.split(","))
        sim.set_tiling(bx, strip)
    print("bench: %s, %d instances, %d fluid nodes, workspace %.2f GB" %
          (args.workload, len(cfgs), nf, sim.workspace_bytes / 1e9), file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    sim.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    mlups = nf * args.steps / (ms / 1e3) / 1e6
    mon = sim.monitors()
    bad = sum(m["bad_nodes"] for m in mon)
    print("bench: %.4f ms/step (events), wall %.3f s, %.0f MLUPS, bad nodes %d" %
          (ms_per_step, wall, mlups, bad), file=sys.stderr, flush=True)

    bytes_per_launch = BYTES_PER_NODE[args.storage] * nf
    achieved = bytes_per_launch / (ms_per_step / 1e3) / 1e9
    traffic = (measured_traffic(args.storage)
               if args.workload == "batch" and not args.tiling and args.reg_order == 2
               else None)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": desc, "instances": len(cfgs), "fluid_nodes": nf,
                   "storage": args.storage, "tiling": list(sim.tiling()[:2]),
                   "reg_order": args.reg_order},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # measured HBM bytes per launch over the same launch time
                     "traffic": (round(traffic / (ms_per_step / 1e3) / 1e9, 1)
                                 if traffic else None),
                     "traffic_bytes_per_launch": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu:
        if args.workload == "batch" and args.reg_order == 2 and args.storage == "f32":
            del sim
            out["gpu_configs"] = gpu_configs_mlups()
            out["other_workloads"] = other_workloads()
            # the practical ceiling of a 50:50 read/write stream on this device
            cc = copy_calibration(20, 3)
            out["copy_ceiling"] = {"GBps": cc["ceiling_GBps"],
                                   "frac_of_peak": cc["ceiling_frac_of_peak"],
                                   "step_traffic_frac_of_ceiling":
                                       (round(out["roofline"]["traffic"] / cc["ceiling_GBps"], 4)
                                        if out["roofline"]["traffic"] else None)}
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
