"""Throughput of A-term IDG gridding + degridding on one MI355X.

One step = one gridding job and one degridding job over the whole MWA-like
observation (128 stations, 8128 baselines x 60 timesteps x 96 channels = 46.8M
4-pol visibilities; grid 8000^2 at 15 arcsec, subgrid 96^2, kernel support 24,
A-terms every 8 timesteps), inputs already resident in HBM:
    grid.zero_(); aidg_grid(V -> grid); aidg_degrid(grid -> V')
value = visibilities / (time per step), in Mvis/s gridded + degridded.

Also reported: grid and degrid rates separately, p50/p99 job latency over the
timed steps, the roofline position of the dominant kernel (per-kernel HIP event
times on the launch stream, algorithmic FMA work per visibility x pixel) and the
FP64 CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per (visibility, subgrid pixel) in the method's form: the 2x2
# complex multiply-accumulate is 16 FP32 FMAs, the phasor step ph <- ph * step is 4
# FP32 ops (2 mul + 2 FMA); each occupies one FMA issue slot, counted as 2 FLOP: 40.
# Both kernels pair a recurrence run's channels symmetrically about its centre, so
# two visibilities take 16 FMA per pixel with real multipliers and one complex phasor
# step (6 FLOP): 19 FLOP per (visibility, pixel) executed.  Rates are reported at both
# counts.
FLOP_PER_VP = 40
FLOP_PER_VP_EXECUTED = {"grid_dft": 19, "degrid_dft": 19}
# FP32 vector peak of MI355X: 256 CUs x 4 SIMDs x 2.4 GHz, each SIMD issuing up to
# two wave64 VALU instructions per 4 cycles (gfx950 VALU dual issue, counted by
# SQ_ACTIVE_INST_VALU2) = 128 FMA per clock per CU = 157.3 TFLOP/s at 2 FLOP/FMA.
# A single issue slot per 4 cycles would give half of it.
PEAK_FP32_TFLOPS = 256 * 4 * 32 * 2.4e9 * 2 / 1e12   # 157.3
PEAK_FP32_SINGLE_ISSUE_TFLOPS = PEAK_FP32_TFLOPS / 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mwa.json")


def library_source_hash() -> str:
    """SHA-256 over the library's sources (kernels, partitioner, plan and launches),
    what decides the kernels and how the workload is cut into launches, with
    comments and whitespace removed so that documentation edits keep it."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2502_17789_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".cpp", ".h")):
            text = open(os.path.join(csrc, name), encoding="utf-8").read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(name.encode())
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None once the library source has changed since."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        digest = library_source_hash()
    except OSError:
        return None
    if digest != rec.get("library_sha256"):
        return None
    k = rec["kernels"].get(kernel)
    return None if k is None else round(k["bytes_per_launch"])


def summarize_traffic(copy_fetch: str, copy_write: str, run_fetch: str, run_write: str, trace: str, out: str):
    """HBM bytes per launch of every kernel of a counter run, from rocprofv3 CSV output
    directories (FETCH_SIZE and WRITE_SIZE passes of the copy probe and of the run, and
    a --kernel-trace --stats run of the same command for the launch times, as CSV or as
    its SQLite database), scaled by
    what the counters read for the 1 GiB device-to-device copy.  Writes the JSON that
    measured_traffic() reads, keyed by the library's source hash."""
    import csv
    import glob

    def counters(d):
        tot, n = {}, {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                k = row["Kernel_Name"]
                tot[k] = tot.get(k, 0.0) + float(row["Counter_Value"])
                n[k] = n.get(k, 0) + 1
        return tot, n

    def short(name):
        for k in ("degrid_dft", "grid_dft", "fft_add", "split_ifft", "copyBuffer"):
            if k in name:
                return k
        return None

    cf, cn = counters(copy_fetch)
    cw, _ = counters(copy_write)
    copy_bytes = 1 << 30
    ck = [k for k in cf if "copyBuffer" in k]
    fetch_scale = copy_bytes / 1024 / (cf[ck[0]] / cn[ck[0]]) if ck else 1.0
    ck = [k for k in cw if "copyBuffer" in k]
    write_scale = copy_bytes / 1024 / (cw[ck[0]] / cn[ck[0]]) if ck else 1.0
    rf, rn = counters(run_fetch)
    rw, _ = counters(run_write)
    ms = {}
    for f in glob.glob(os.path.join(trace, "**", "*kernel_stats.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            k = short(row["Name"])
            if k:
                ms[k] = float(row["AverageNs"]) / 1e6
    for f in glob.glob(os.path.join(trace, "**", "*.db"), recursive=True):
        import sqlite3   # rocprofv3's default output: its top_kernels view holds microseconds
        for name, avg_us in sqlite3.connect(f).execute("select name, average from top_kernels"):
            k = short(name)
            if k:
                ms[k] = float(avg_us) / 1e3
    rec = {"library_sha256": library_source_hash(), "copy_probe_bytes": copy_bytes,
           "fetch_scale": fetch_scale, "write_scale": write_scale, "kernels": {}}
    for name, v in rf.items():
        k = short(name)
        if k is None or k == "copyBuffer":
            continue
        launches = rn[name]
        fk, wk = v / launches, rw.get(name, 0.0) / launches
        rec["kernels"][k] = {"launches": launches, "fetch_kib_raw": fk, "write_kib_raw": wk,
                             "read_bytes": fk * 1024 * fetch_scale, "write_bytes": wk * 1024 * write_scale,
                             "bytes_per_launch": (fk * fetch_scale + wk * write_scale) * 1024,
                             "launch_ms": ms.get(k)}
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-baselines", type=int, default=48)
    ap.add_argument("--serve", action="store_true",
                    help="served mixed workload instead of the MWA-like job (separate JSON line)")
    ap.add_argument("--jobs", type=int, default=300)
    ap.add_argument("--rho", type=float, nargs="+", default=[0.8, 1.2, 2.0])
    ap.add_argument("--rounds-in-flight", type=int, default=2)
    ap.add_argument("--range-subgrids", type=int, default=4096)
    ap.add_argument("--prepare-workers", type=int, default=4)
    ap.add_argument("--max-active", type=int, default=32)
    ap.add_argument("--precision", action="store_true",
                    help="precision study: FP32 path (reseed interval swept) against the FP64 path "
                         "on the MWA-like workload, over screen rms and w-range (JSON line per case)")
    ap.add_argument("--screens", type=float, nargs="+", default=[0.5, 2.0, 5.0])
    ap.add_argument("--wmax", type=float, nargs="+", default=[0.0, 250.0, 500.0],
                    help="largest |w| in wavelengths (0 = at transit)")
    ap.add_argument("--reseed", type=int, nargs="+", default=[8, 16, 32, 96])
    ap.add_argument("--kernel-sweep", action="store_true",
                    help="kernel-only grid/degrid throughput at subgrid sizes 32/64/96 (K = L/4), "
                         "FP32 and FP64, on the MWA-like observation (JSON line per case)")
    ap.add_argument("--lattice-cases", type=lambda t: tuple(int(x) for x in t.split(":")), nargs="*",
                    default=[], help="extra FP32 kernel-sweep cases L:lattice (centre lattice step)")
    ap.add_argument("--lattice-only", action="store_true", help="kernel sweep: only the --lattice-cases")
    ap.add_argument("--sweep-reseed", type=int, nargs="*", default=[],
                    help="kernel sweep: extra FP32 L = 96 cases at these re-seed intervals R")
    ap.add_argument("--degrid-forms", type=int, nargs="+", default=[0],
                    help="kernel sweep: degridder forms to run (0 automatic, 1 recurrence, 2 per visibility, "
                         "3 direct)")
    ap.add_argument("--occupancy-sweep", action="store_true",
                    help="degridder forms against subgrid occupancy: the MWA-like observation with every "
                         "k-th channel kept (k from --occupancy-decimation), FP32 (JSON line per case)")
    ap.add_argument("--occupancy-decimation", type=int, nargs="+", default=[1, 4, 12, 32, 96])
    ap.add_argument("--occupancy-L", type=int, nargs="+", default=[32, 96])
    ap.add_argument("--occupancy-forms", type=int, nargs="+", default=[1, 3, 2, 0],
                    help="occupancy sweep: degridder forms (1 recurrence, 3 direct, 2 per visibility, 0 auto)")
    ap.add_argument("--image", action="store_true",
                    help="image-level w-stacking (invert and predict) at the MWA-like size, FP32, at "
                         "max |w| of --image-wmax wavelengths (JSON line per case)")
    ap.add_argument("--image-wmax", type=float, nargs="+", default=[0.0, 250.0])
    ap.add_argument("--image-fold", type=int, nargs="+", default=[0, 1],
                    help="image mode: w_fold settings to run at max |w| > 0")
    ap.add_argument("--aterm-mode", type=int, choices=[0, 1], default=0,
                    help="A-term of gridding: 0 adjoint (A^H), 1 the paper's normalised A^-1")
    ap.add_argument("--stokes-i", action="store_true",
                    help="Stokes-I grids: one complex value per cell instead of four")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device 3 times (calibrates HBM byte counters)")
    ap.add_argument("--summarize-traffic", nargs=6, metavar=("COPY_FETCH", "COPY_WRITE", "FETCH", "WRITE",
                                                            "TRACE", "OUT"),
                    help="no GPU: write the per-kernel HBM traffic JSON from rocprofv3 CSV directories")
    return ap.parse_args()


def workload_description(wl, info):
    return {
        "workload": "MWA-like A-term IDG grid+degrid: 128 stations in a 5 km disc, 8128 baselines "
                    "x 60 x 2 s x 96 ch (140-170 MHz), 4-pol complex64; grid 8000^2 at 15 arcsec, "
                    "subgrid 96^2, K=24; A-terms 8 intervals x 128 stations (Gaussian beam x "
                    "Kolmogorov screen 2 rad rms)",
        "n_vis": int(wl.n_vis), "grid_size": wl.grid_size, "subgrid_size": wl.subgrid_size,
        "kernel_support": wl.kernel_support, "n_subgrids": int(info["n_subgrids"]),
        "n_wlayers": int(info["n_wlayers"]), "precision": "fp32 (fp64 phase origins)",
    }


def sample_table(wl, table, sel):
    """The plan's subgrids of baselines `sel`, renumbered for the sampled workload."""
    pos = -np.ones(wl.n_baselines, np.int64)
    pos[sel] = np.arange(len(sel))
    t = table[pos[table["bl"]] >= 0].copy()
    t["bl"] = pos[t["bl"]]
    t["vis_offset"] = (t["bl"].astype(np.int64) * wl.n_times + t["t0"]) * wl.n_chans + t["c0"]
    return t


def cpu_baseline(wl, n_bl: int, plan_table, V, G, Vout, w0, aterm_mode: int = 0, stokes_i: bool = False):
    """FP64 oracle (test infrastructure) on a fixed random subset of baselines, run on
    the timed step's own data: it grids the sampled baselines' input visibilities V
    with the plan's subgrids of those baselines (timed), and degrids the GPU's timed
    grid G for the same subgrids (timed), which also checks the timed degridding output
    Vout there visibility by visibility.  The timed grid itself is checked at 8 lattice
    directions against L^2 T times the direct A-term image of all visibilities (exact
    at lattice samples).  V, G, Vout: host arrays."""
    import oracle
    import synth
    rng = np.random.default_rng(2)
    sel = np.sort(rng.choice(wl.n_baselines, n_bl, replace=False))
    sub = synth.Workload("mwa-sample", wl.n_stations, np.ascontiguousarray(wl.baselines[sel]),
                         np.ascontiguousarray(wl.uvw[sel]), wl.freqs, wl.grid_size, wl.subgrid_size,
                         wl.kernel_support, wl.pixel_scale, wl.aterm_interval, wl.aterms)
    table = sample_table(wl, plan_table, sel)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    grid_fn = oracle.grid_stokes_i if stokes_i else oracle.grid
    degrid_fn = oracle.degrid_stokes_i if stokes_i else oracle.degrid
    t0 = time.perf_counter()
    grid_fn(sub, V[sel], table, W=G.shape[0], nthreads=threads, aterm_mode=aterm_mode)
    t1 = time.perf_counter()
    Vo = degrid_fn(sub, G, table, nthreads=threads)
    t2 = time.perf_counter()
    n = sub.n_vis
    out = {"value": round(n / (t2 - t0) / 1e6, 6), "unit": "Mvis/s", "cores": threads, "kind": "oracle",
           "sample": f"{n_bl} random baselines (seed 2) of the timed observation, all 60 x 96 "
                     f"visibilities each ({n} vis, the plan's {table.shape[0]} subgrids of them), grid "
                     f"of the timed input then degrid of the GPU's timed grid at full N, L, K; "
                     f"grid {t1 - t0:.2f} s, degrid {t2 - t1:.2f} s"}
    # the timed degridding output at the sampled baselines, every visibility
    d = np.linalg.norm(Vout[sel].astype(np.complex128) - Vo, axis=-1).ravel()
    r = np.linalg.norm(Vo, axis=-1).ravel()
    check = {"degrid_sampled": {"baselines": n_bl, "visibilities": int(d.size),
                                "normwise": float(np.linalg.norm(d) / np.linalg.norm(r)),
                                "max_over_rms": float(d.max() / np.sqrt(np.mean(r * r)))}}
    # the timed grid at 8 lattice directions: sum_w exp(2 pi i w0 n1) layer image = L^2 T direct image
    if aterm_mode == 0 and not stokes_i:
        L = wl.subgrid_size
        xs = rng.integers(0, L, 8).astype(np.int32)
        ys = rng.integers(0, L, 8).astype(np.int32)
        l, m = oracle.lattice_dirs(wl, xs, ys)
        n1 = -(l * l + m * m) / (1 + np.sqrt(1 - l * l - m * m))
        lhs = sum(oracle.layer_image_at(G[j], 1.0 / wl.fov, l, m, nthreads=threads)
                  * np.exp(2j * np.pi * w0[j] * n1)[:, None] for j in range(G.shape[0]))
        mask = oracle.coverage_mask(wl, plan_table)
        T = oracle.taper(L, wl.kernel_support)
        rhs = L * L * T[ys, xs][:, None] * oracle.direct_image(wl, V, l, m, xs, ys, mask=mask, nthreads=threads)
        check["grid_lattice"] = {"directions": 8,
                                 "normwise": float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)),
                                 "max_over_max": float(np.abs(lhs - rhs).max() / np.abs(rhs).max())}
    out["parity_of_timed_output"] = check
    return out


def serve_bench(args):
    """Mixed grid/degrid jobs with Poisson arrivals: served (continuous batching)
    vs sequential per-job launches on the same arrival trace."""
    import torch

    import paper_2502_17789_amd as aidg
    import synth
    from paper_2502_17789_amd.serve import GpuBackend, Job, Server

    torch.cuda.set_device(0)
    mix = synth.served_job_mix(args.jobs, seed=5)

    def make_job(d, tag):
        geo = aidg.Geometry(d["N"], d["L"], d["K"], d["dl"], aterm_interval=max(d["n_t"], 1))
        seed = d["seed"]

        def aterms():
            return synth.device_phase_screen_aterms(d["n_stations"], d["L"], d["screen_rms"], seed)

        def data(shape):
            g = torch.Generator(device="cuda")
            g.manual_seed(seed + 1)
            return torch.randn(shape, dtype=torch.complex64, device="cuda", generator=g)

        return Job(d["direction"], geo, d["n_stations"], d["baselines"], d["uvw"], d["freqs"],
                   aterms, data, tag=tag)

    def n_vis(d):
        return d["baselines"].shape[0] * d["uvw"].shape[1] * d["freqs"].shape[0]

    def run_sequential(arrivals):
        """One job at a time, each through its own plan (plain per-job launches)."""
        lat, service = [], []
        t0 = time.perf_counter()
        for d, arr in zip(mix, arrivals):
            now = time.perf_counter() - t0
            if now < arr:
                time.sleep(arr - now)
            s0 = time.perf_counter()
            job = make_job(d, None)
            A = job.aterms()
            geo = dataclasses_replace(job.geometry, workspace_bytes=256 << 20)
            with aidg.Plan(geo, job.n_stations, job.baselines, job.uvw, job.freqs, A) as p:
                del A
                if job.direction == "grid":
                    out = p.grid(job.data(p.vis_shape()))
                else:
                    out = p.degrid(job.data(p.grid_shape()))
                torch.cuda.synchronize()
                del out
            s1 = time.perf_counter()
            service.append(s1 - s0)
            lat.append(s1 - t0 - arr)
        return np.array(lat), np.array(service), time.perf_counter() - t0

    def run_served(arrivals):
        backend = GpuBackend(workspace_bytes=1 << 30, timing=True)
        srv = Server(backend, range_subgrids=args.range_subgrids,
                     rounds_in_flight=args.rounds_in_flight, prepare_workers=args.prepare_workers,
                     max_active=args.max_active)
        futs = []

        def consume(f):
            # the client takes its result and releases the device output, as the
            # sequential client does after each job
            f.result().output = None   # the job's work is complete when its future resolves

        with srv:
            t0 = time.perf_counter()
            for i, (d, arr) in enumerate(zip(mix, arrivals)):
                now = time.perf_counter() - t0
                if now < arr:
                    time.sleep(arr - now)
                f = srv.submit(make_job(d, i))
                f.add_done_callback(consume)
                futs.append(f)
            res = [f.result() for f in futs]
        lat = np.array([r.latency for r in res])
        span = max(r.finished for r in res) - min(r.arrival for r in res)
        stats = srv.stats()
        stats["busy_s"] = backend.busy_seconds()
        del res, futs, srv, backend
        torch.cuda.synchronize()
        torch.cuda.empty_cache()   # the next run starts from the same free memory
        return lat, span, stats

    total = sum(n_vis(d) for d in mix)
    run_sequential([0.0] * 6)   # warm-up: kernels of each subgrid size, allocator
    lat0, service, span0 = run_sequential([0.0] * len(mix))
    es = float(service.mean())
    out = {"metric": "served mixed grid/degrid jobs: Mvis/s and p50/p99 job latency",
           "jobs": len(mix), "total_vis": int(total), "mean_sequential_service_ms": round(es * 1e3, 3),
           "server": {"rounds_in_flight": args.rounds_in_flight, "range_subgrids": args.range_subgrids,
                      "prepare_workers": args.prepare_workers, "max_active": args.max_active},
           "sequential_back_to_back": {"mvis_s": round(total / span0 / 1e6, 3)}, "loads": []}
    rng = np.random.default_rng(6)
    for rho in list(args.rho) + ["saturated"]:
        if rho == "saturated":   # every job submitted at once: the server's own throughput
            arrivals = np.zeros(len(mix))
        else:
            gaps = rng.exponential(es / rho, len(mix))
            arrivals = np.concatenate([[0.0], np.cumsum(gaps)[:-1]])
        ls, span_s, st = run_served(arrivals)
        lq, _, span_q = (lat0, None, span0) if rho == "saturated" else run_sequential(arrivals)
        out["loads"].append({
            "rho": rho,
            "served": {"p50_ms": round(float(np.percentile(ls, 50)) * 1e3, 3),
                       "p99_ms": round(float(np.percentile(ls, 99)) * 1e3, 3),
                       "mvis_s": round(total / span_s / 1e6, 3), "rounds": st["rounds"],
                       "ranges_per_round": round(st["ranges_per_round"], 2),
                       "loop_wait_s": round(st["wait_s"], 3), "prepare_s": round(st["prepare_s"], 3),
                       "makespan_s": round(span_s, 3), "peak_admitted_bytes": st["peak_bytes"],
                       "gpu_busy_s": round(st["busy_s"], 3), "gpu_busy_frac": round(st["busy_s"] / span_s, 4),
                       "kernel_mvis_s": round(total / st["busy_s"] / 1e6, 3)},
            "sequential": {"p50_ms": round(float(np.percentile(lq, 50)) * 1e3, 3),
                           "p99_ms": round(float(np.percentile(lq, 99)) * 1e3, 3),
                           "mvis_s": round(total / span_q / 1e6, 3)}})
        print(f"# rho {rho}: {out['loads'][-1]}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def precision_study(args):
    """FP32 path (phasor recurrence re-seeded from FP64 every R channels) against the
    full-FP64 path on the MWA-like workload.  Visibilities: 300 point sources
    (0.01-30 Jy, log-uniform) plus unit noise, evaluated in FP64 on the device; the
    degridding input is the FP64 grid of those visibilities.  Per result: normwise
    relative error and max|d|/max|ref|; per visibility (|V_k|_F >= 1e-3 rms):
    max, p99 and rms of |dV_k|_F / |V_k|_F."""
    import torch

    import paper_2502_17789_amd as aidg
    import synth

    torch.cuda.set_device(0)

    def norm_err(x, ref):
        num = den = 0.0
        dmax = rmax = 0.0
        for j in range(ref.shape[0]):           # layer by layer: bounded temporaries
            d = x[j].to(torch.complex128) - ref[j]
            num += float(torch.linalg.vector_norm(d)) ** 2
            den += float(torch.linalg.vector_norm(ref[j])) ** 2
            dmax = max(dmax, float(d.abs().max()))
            rmax = max(rmax, float(ref[j].abs().max()))
        return num ** 0.5 / max(den ** 0.5, 1e-300), dmax / max(rmax, 1e-300)

    def vis_err(x, ref):
        d = (x.to(torch.complex128) - ref)
        nd = torch.linalg.vector_norm(d, dim=-1)
        nr = torch.linalg.vector_norm(ref, dim=-1)
        sel = nr >= 1e-3 * torch.sqrt((nr * nr).mean())
        r = (nd[sel] / nr[sel]).flatten()
        q = torch.quantile(r[torch.randperm(r.numel(), device=r.device)[:1 << 24]], 0.99)
        return {"normwise": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref)),
                "per_vis_max": float(r.max()), "per_vis_p99": float(q),
                "per_vis_rms": float(torch.sqrt((r * r).mean()))}

    for wmax in args.wmax:
        ha = synth.hour_angle_for_wmax(wmax) if wmax > 0 else 0.0
        for rms in args.screens:
            t0 = time.perf_counter()
            wl = synth.config_mwa(seed=2, screen_rms=rms, ha0_rad=ha)
            w_top = float(np.abs(wl.uvw[..., 2]).max() * wl.freqs.max() / 299792458.0)
            base = dict(grid_size=wl.grid_size, subgrid_size=wl.subgrid_size,
                        kernel_support=wl.kernel_support, pixel_scale=wl.pixel_scale,
                        aterm_interval=wl.aterm_interval)
            V64 = synth.device_point_source_vis(wl, 300, seed=3)
            A64 = torch.from_numpy(wl.aterms).cuda()
            with aidg.Plan(aidg.Geometry(precision=aidg.FP64, **base), wl.n_stations, wl.baselines,
                           wl.uvw, wl.freqs, A64) as p64:
                info = p64.info
                G64 = p64.grid(V64)
                Vd64 = p64.degrid(G64)
                torch.cuda.synchronize()
            del A64
            G32in = torch.empty(G64.shape, dtype=torch.complex64, device="cuda")
            for j in range(G64.shape[0]):
                G32in[j] = G64[j].to(torch.complex64)
            V32in = V64.to(torch.complex64)
            A32 = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
            for R in args.reseed:
                with aidg.Plan(aidg.Geometry(precision=aidg.FP32, reseed_channels=R, **base),
                               wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A32) as p32:
                    assert p32.info["n_wlayers"] == info["n_wlayers"]
                    G32 = p32.grid(V32in)
                    Vd32 = p32.degrid(G32in)
                    torch.cuda.synchronize()
                g_norm, g_max = norm_err(G32, G64)
                ve = vis_err(Vd32, Vd64)
                del G32, Vd32
                print(json.dumps({
                    "precision_case": {"screen_rms_rad": rms, "max_abs_w_lambda": round(w_top, 1),
                                       "hour_angle_rad": round(ha, 5), "n_wlayers": info["n_wlayers"],
                                       "w_step": round(info["w_step"], 3), "reseed_channels": R},
                    "grid_fp32_vs_fp64": {"normwise": g_norm, "max_over_max": g_max},
                    "degrid_fp32_vs_fp64": ve,
                    "elapsed_s": round(time.perf_counter() - t0, 1)}), flush=True)
            del G64, Vd64, G32in, V32in, V64, A32
            torch.cuda.empty_cache()


def _kernel_case(aidg, wl, prec, L, lattice=0, form=0, reps=2, reseed=0):
    """Kernel times of one plan of the observation `wl` at subgrid size L (K = L/4):
    HIP events around every launch, mean of `reps` grid + degrid calls after a
    warm-up.  Returns the JSON record of the case."""
    import torch

    import synth

    cdt = torch.complex64 if prec == aidg.FP32 else torch.complex128
    A = synth.device_phase_screen_aterms(wl.n_stations, L, 2.0, seed=7)
    n_int = (wl.n_times + wl.aterm_interval - 1) // wl.aterm_interval
    A = A.expand(n_int, -1, -1, -1, -1).contiguous().to(cdt)
    geo = aidg.Geometry(wl.grid_size, L, L // 4, wl.pixel_scale, aterm_interval=wl.aterm_interval,
                        precision=prec, center_lattice=lattice, degrid_form=form, reseed_channels=reseed)
    gen = torch.Generator(device="cuda")
    with aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A) as plan:
        del A
        gen.manual_seed(2)
        V = torch.randn(plan.vis_shape(), dtype=cdt, device="cuda", generator=gen)
        G = torch.zeros(plan.grid_shape(), dtype=cdt, device="cuda")
        Vo = torch.empty_like(V)
        plan.grid(V, G)
        plan.degrid(G, Vo)
        torch.cuda.synchronize()
        plan.set_profiling(True)
        for _ in range(reps):
            plan.grid(V, G)
            plan.degrid(G, Vo)
        torch.cuda.synchronize()
        kt = plan.kernel_times()
        info = plan.info
        del V, G, Vo
    torch.cuda.empty_cache()
    ms = {k: v["ms"] / reps for k, v in kt.items()}
    n = wl.n_vis
    t_grid = ms["grid_dft"] + ms["fft_add"]
    t_degrid = ms["split_ifft"] + ms["degrid_dft"]
    return {
        "subgrid_size": L, "kernel_support": L // 4, "center_lattice": lattice or "auto",
        "precision": "fp32" if prec == aidg.FP32 else "fp64",
        "degrid_form": ("auto", "recurrence", "per_vis", "direct")[form],
        "reseed_channels": reseed or 32,
        "n_vis": n, "n_chans": int(wl.n_chans), "n_subgrids": info["n_subgrids"], "n_groups": info["n_groups"],
        "n_subgrids_pervis": info["n_subgrids_pervis"], "n_subgrids_direct": info["n_subgrids_direct"],
        "mean_vis_per_subgrid": round(n / max(info["n_subgrids"], 1), 1),
        "grid_mvis_s": round(n / (t_grid * 1e-3) / 1e6, 1),
        "degrid_mvis_s": round(n / (t_degrid * 1e-3) / 1e6, 1),
        "ms": {k: round(v, 3) for k, v in ms.items() if v > 0},
        "dft_tflops": {k: round(kt[k]["vis_pixels"] * FLOP_PER_VP_EXECUTED[k] / (ms[k] * reps * 1e-3) / 1e12, 2)
                       for k in ("grid_dft", "degrid_dft")}}


def kernel_sweep(args):
    """Throughput against subgrid size, kernels only (HIP events around every launch):
    the MWA-like observation partitioned at L = 32, 64, 96 with K = L/4, in FP32
    and FP64, for each degridder form of --degrid-forms.  grid = grid_dft + fft_add,
    degrid = split_ifft + degrid_dft."""
    import torch

    import paper_2502_17789_amd as aidg
    import synth

    torch.cuda.set_device(0)
    wl = synth.config_mwa(seed=2)
    cases = [] if args.lattice_only else [(prec, L, 0) for prec in (aidg.FP32, aidg.FP64) for L in (32, 64, 96)]
    cases += [(aidg.FP32, L, lat) for L, lat in args.lattice_cases]
    for prec, L, lattice in cases:
        for form in args.degrid_forms:
            rec = _kernel_case(aidg, wl, prec, L, lattice, form)
            print(json.dumps({"kernel_sweep": rec}), flush=True)
    # the speed side of the re-seed interval (the precision side is --precision)
    for R in args.sweep_reseed:
        rec = _kernel_case(aidg, wl, aidg.FP32, 96, 0, 0, reseed=R)
        print(json.dumps({"kernel_sweep": rec}), flush=True)


def occupancy_sweep(args):
    """Degridder throughput against subgrid occupancy (Sec. 4.2, subgrid occupancy): the
    MWA-like observation with every k-th channel kept (rows of about 1/k the channels,
    subgrids of about 1/k the visibilities), degridded in each form of
    --occupancy-forms: the channel recurrence, direct phasors, per visibility (where a
    sub-table fits the workgroup) and the automatic choice per subgrid."""
    import torch

    import paper_2502_17789_amd as aidg
    import synth

    torch.cuda.set_device(0)
    base = synth.config_mwa(seed=2)
    for L in args.occupancy_L:
        for k in args.occupancy_decimation:
            wl = copy.copy(base)
            wl.freqs = np.ascontiguousarray(base.freqs[::k])
            for form in args.occupancy_forms:
                rec = _kernel_case(aidg, wl, aidg.FP32, L, 0, form)
                rec["channel_decimation"] = k
                print(json.dumps({"occupancy_sweep": rec}), flush=True)


def image_bench(args):
    """Image-level w-stacking (Eq. wstack) and its inverse (Eq. wunstack) on the
    MWA-like grid (N = 8000, the plan's w-layers), FP32: aidg_invert and aidg_predict
    timed with HIP events around every launch.  Each kernel class's effective
    bandwidth is the bytes its launches read and write (one N x N plane in and one
    out per row-FFT pass or transpose; the w-stacking pass also reads the image it
    adds to) over their time."""
    import torch

    import paper_2502_17789_amd as aidg
    import synth

    torch.cuda.set_device(0)
    cases = [(w, f) for w in args.image_wmax for f in (args.image_fold if w > 0 else [0])]
    for wmax, fold in cases:
        ha = synth.hour_angle_for_wmax(wmax) if wmax > 0 else 0.0
        wl = synth.config_mwa(seed=2, ha0_rad=ha)
        geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                            aterm_interval=wl.aterm_interval, w_fold=fold, aterm_mode=args.aterm_mode,
                            stokes_i=int(args.stokes_i))
        A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
        with aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A) as plan:
            del A
            W, N = plan.n_wlayers, wl.grid_size
            gen = torch.Generator(device="cuda")
            gen.manual_seed(4)
            G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
            I = torch.randn(plan.image_shape(), dtype=torch.complex64, device="cuda", generator=gen)
            Io = torch.empty_like(I)
            Go = torch.empty_like(G)
            plan.invert(G, Io)
            plan.predict(I, Go)
            torch.cuda.synchronize()
            plan.set_profiling(True)
            reps = 3
            stream = torch.cuda.current_stream()
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
            for r in range(reps):
                ev[r][0].record(stream)
                plan.invert(G, Io)
                ev[r][1].record(stream)
                plan.predict(I, Go)
                ev[r][2].record(stream)
            torch.cuda.synchronize()
            kt = plan.kernel_times()
            t_inv = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
            t_pred = float(np.median([e[1].elapsed_time(e[2]) for e in ev]))
            del G, I, Io, Go
        P = N * N * 8
        npol = geo.n_pol
        # per polarisation plane: invert reads + writes a plane in each of 2 row passes and
        # 1 transpose per layer, the first layer's w-stack pass reads 1 and writes 1, the
        # others read 2 and write 1; predict reads + writes in 2 row passes and 2 transposes
        by = {"image_fft": reps * npol * 4 * W * 2 * P,
              "image_wstack": reps * npol * ((W * 2 + 2 + (W - 1) * 3) + 2 * W * 2) * P}
        cls = {k: {"ms_per_launch": round(kt[k]["ms"] / max(kt[k]["launches"], 1), 4),
                   "launches_per_call_pair": kt[k]["launches"] // reps,
                   "gb_s": round(by[k] / (kt[k]["ms"] * 1e-3) / 1e9, 1)} for k in by}
        dom = max(by, key=lambda k: kt[k]["ms"])
        print(json.dumps({
            "image_level": {"grid_size": N, "n_wlayers": W, "max_abs_w_lambda": wmax or "transit",
                            "w_fold": fold, "aterm_mode": args.aterm_mode,
                            "grid_planes": 1 if args.stokes_i else 4, "precision": "fp32",
                            "plane_bytes": P},
            "invert_ms": round(t_inv, 3), "predict_ms": round(t_pred, 3),
            "classes": cls,
            "roofline": {"kernel": dom, "bound": "hbm", "achieved": cls[dom]["gb_s"], "peak": 8000.0,
                         "unit": "GB/s", "frac": round(cls[dom]["gb_s"] / 8000.0, 4)}}), flush=True)
        torch.cuda.empty_cache()


def dataclasses_replace(obj, **kw):
    import dataclasses
    return dataclasses.replace(obj, **kw)


def path_roofline(kt, wall_s):
    """Sustained rate of the whole timed step: both DFT kernels' executed FLOP (19 per
    vp in the paired-channel form) over the wall time, which also covers the FFTs, the
    adder, the splitter and the zeroing kernels."""
    flop = sum(kt[k]["vis_pixels"] * FLOP_PER_VP_EXECUTED[k] for k in ("grid_dft", "degrid_dft"))
    achieved = flop / wall_s / 1e12
    return {"achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 1), "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "scope": "grid_dft + degrid_dft executed FLOP (19 per vp each, paired-channel form) over the "
                     "wall time of the timed steps"}


# Rates of the survey's roofline definition: FP32 FMA at the dual-issue peak, FP64 FMA at
# the FP64 vector peak, and transcendental sin/cos at a quarter of the single-issue FP32
# rate (an assumed figure: the phasor seeds here are FMA polynomials, not TRANS).
R_PK_FMA = PEAK_FP32_TFLOPS * 1e12 / 2
R_F64_FMA = 78.6e12 / 2
R_TRANS = PEAK_FP32_SINGLE_ISSUE_TFLOPS * 1e12 / 2 / 4


def rdef_roofline(table, L: int, R: int, ms: float) -> dict:
    """The survey's roofline time of one DFT kernel launch over a plan's table,
    T_roof = N_vp 20 / R_pk + N_seed (2 / R_trans + 8 / R_f64) + N_sg L^2 72 / R_pk,
    with N_seed = sum over subgrids of nt L^2 (1 + ceil(nc / R)) phasor seeds (one step
    phasor and one origin per R channels, per row and pixel), against the measured
    launch time: frac = T_roof / T_meas."""
    nt = table["nt"].astype(np.int64)
    nc = table["nc"].astype(np.int64)
    n_vp = int((nt * nc).sum()) * L * L
    n_seed = int((nt * (1 + (nc + R - 1) // R)).sum()) * L * L
    t = n_vp * 20 / R_PK_FMA + n_seed * (2 / R_TRANS + 8 / R_F64_FMA) + len(table) * L * L * 72 / R_PK_FMA
    return {"t_roof_ms": round(t * 1e3, 3), "frac": round(t * 1e3 / ms, 4), "n_seed": n_seed,
            "seeds_per_vp": round(n_seed / max(n_vp, 1), 5)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the design "
              "would shard baselines across GPUs and all-reduce the grid); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_bench(args)
        return
    if args.precision:
        precision_study(args)
        return
    if args.kernel_sweep:
        kernel_sweep(args)
        return
    if args.occupancy_sweep:
        occupancy_sweep(args)
        return
    if args.image:
        image_bench(args)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return

    import torch

    import paper_2502_17789_amd as aidg
    import synth

    torch.cuda.set_device(0)
    wl = synth.config_mwa(seed=2)
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, aterm_mode=args.aterm_mode,
                        stokes_i=int(args.stokes_i))
    A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
    t0 = time.perf_counter()
    plan = aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A)
    plan_s = time.perf_counter() - t0
    info = plan.info
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    V = torch.randn(plan.vis_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    G = torch.zeros(plan.grid_shape(), dtype=torch.complex64, device="cuda")
    Vout = torch.empty_like(V)
    stream = torch.cuda.current_stream()

    def step():
        G.zero_()
        plan.grid(V, G)
        plan.degrid(G, Vout)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# plan {plan_s:.2f} s, {info['n_subgrids']} subgrids, {info['n_batches']} batches; "
          f"warmup done", file=sys.stderr, flush=True)

    plan.set_profiling(True)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        G.zero_()
        plan.grid(V, G)
        ev[i][1].record(stream)
        plan.degrid(G, Vout)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kt = plan.kernel_times()
    plan.set_profiling(False)
    t_grid = np.array([e[0].elapsed_time(e[1]) for e in ev])
    t_degrid = np.array([e[1].elapsed_time(e[2]) for e in ev])
    t_job = t_grid + t_degrid
    n = wl.n_vis
    ms_per_step = wall * 1e3 / args.steps

    dom = max(("grid_dft", "degrid_dft", "fft_add", "split_ifft"), key=lambda k: kt[k]["ms"])
    k = kt[dom]
    if dom in ("grid_dft", "degrid_dft"):
        achieved = k["vis_pixels"] * FLOP_PER_VP / (k["ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(PEAK_FP32_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": measured_traffic(dom),
                "frac_of_single_issue": round(achieved / PEAK_FP32_SINGLE_ISSUE_TFLOPS, 4),
                "frac_executed": round(k["vis_pixels"] * FLOP_PER_VP_EXECUTED[dom] / (k["ms"] * 1e-3) / 1e12
                                       / PEAK_FP32_TFLOPS, 4),
                "avg_launch_ms": round(k["ms"] / max(k["launches"], 1), 4),
                "launches": k["launches"]}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": 8000.0, "unit": "GB/s",
                "frac": None, "traffic": None}
    table = plan.subgrids()
    if dom in ("grid_dft", "degrid_dft"):
        roof["rdef"] = rdef_roofline(table, wl.subgrid_size, 32, roof["avg_launch_ms"])
    kernels = {name: {"ms_per_step": round(v["ms"] / args.steps, 3),
                      "launches_per_step": v["launches"] / args.steps,
                      **({"tflops": round(v["vis_pixels"] * FLOP_PER_VP / (v["ms"] * 1e-3) / 1e12, 3),
                          "tflops_executed": round(v["vis_pixels"] * FLOP_PER_VP_EXECUTED[name]
                                                   / (v["ms"] * 1e-3) / 1e12, 3)}
                         if name in ("grid_dft", "degrid_dft") and v["ms"] > 0 else {})}
               for name, v in kt.items()}
    out = {
        "metric": "Mvisibilities/sec gridded+degridded (with A-terms) at 1e-5 rel err; p50/p99 job latency",
        "value": round(n / (ms_per_step * 1e-3) / 1e6, 3),
        "unit": "Mvis/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {**workload_description(wl, info),
                   "aterm_mode": "inverse (normalised A^-1)" if args.aterm_mode else "adjoint (A^H)",
                   "grid_planes": 1 if args.stokes_i else 4},
        "grid_mvis_s": round(n / (np.median(t_grid) * 1e-3) / 1e6, 3),
        "degrid_mvis_s": round(n / (np.median(t_degrid) * 1e-3) / 1e6, 3),
        "latency_ms": {"p50": round(float(np.percentile(t_job, 50)), 3),
                       "p99": round(float(np.percentile(t_job, 99)), 3),
                       "job": "one grid job + one degrid job of the whole observation"},
        "plan_build_s": round(plan_s, 3),
        "roofline": roof,
        "path_roofline": path_roofline(kt, wall),
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        w0 = plan.wlayers()
        Vh, Gh, Vo = V.cpu().numpy(), G.cpu().numpy(), Vout.cpu().numpy()
        plan.close()
        del V, G, Vout, A
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_baselines, table, Vh, Gh, Vo, w0,
                                           args.aterm_mode, bool(args.stokes_i))
    else:
        plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
