"""Serving on the GPU: a mix of gridding and degridding jobs of different subgrid
sizes, grid sizes and lengths runs through the continuous-batching server (small
ranges, so every job is split over several rounds and shares launches with the
others).  Each result must equal the same job run alone through its own plan
(1e-6, normwise and on the worst element: only the order of FP32 atomic additions
differs), and jobs given the oracle's partition must match the FP64 oracle at the
1e-5 gate (tests/gates.py)."""
import numpy as np
import pytest

import synth
from gates import check_grid, check_vis

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def jobs_mix(orc):
    from paper_2502_17789_amd import Geometry
    from paper_2502_17789_amd.serve import Job
    specs = []
    rng = np.random.default_rng(77)
    for i in range(18):
        L = [32, 64, 96][i % 3]
        N = {32: 128, 64: 256, 96: 384}[L]
        K = L // 4
        wl = synth.config_tiny(300 + i, n_st=int(rng.integers(3, 7)), n_t=int(rng.integers(2, 8)),
                               n_c=int(rng.integers(1, 40)), L=L, K=K, N=N, fov_deg=12.0,
                               diameter_m=float(rng.uniform(200, 1200)), aterm_interval=2)
        direction = "grid" if i % 2 == 0 else "degrid"
        table = orc.partition(wl, 0.0) if i % 4 == 0 else None
        geo = Geometry(N, L, K, wl.pixel_scale, aterm_interval=2, w_step=-1.0 if table is not None else 0.0)
        if direction == "grid":
            data = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
        else:
            W = orc.n_layers(table) if table is not None else None
            data = None if W is None else synth.random_grid(W, N, rng)
        specs.append((Job(direction, geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs,
                          wl.aterms.astype(np.complex64), data, tag=i, table=table), wl))
    return specs


def test_served_results_equal_alone(orc):
    import paper_2502_17789_amd as aidg
    from paper_2502_17789_amd.serve import GpuBackend, Server
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    specs = jobs_mix(orc)
    rng = np.random.default_rng(5)
    # degrid jobs without a caller table need a grid with the plan's number of layers
    for job, wl in specs:
        if job.data is None:
            with aidg.Plan(job.geometry, job.n_stations, job.baselines, job.uvw, job.freqs,
                           torch.from_numpy(job.aterms).cuda()) as p:
                job.data = synth.random_grid(p.n_wlayers, job.geometry.grid_size, rng)
    srv = Server(GpuBackend(workspace_bytes=64 << 20), hbm_budget=8 << 30, range_subgrids=3)
    with srv:
        futs = [srv.submit(job) for job, _ in specs]
        results = [f.result(timeout=120) for f in futs]
    st = srv.stats()
    print(f"served {st}", flush=True)
    assert st["rounds"] > 3
    for (job, wl), res in zip(specs, results):
        A = torch.from_numpy(job.aterms).cuda()
        with aidg.Plan(job.geometry, job.n_stations, job.baselines, job.uvw, job.freqs, A,
                       table=job.table) as p:
            x = torch.from_numpy(np.asarray(job.data, np.complex64)).cuda()
            alone = p.grid(x) if job.direction == "grid" else p.degrid(x)
            torch.cuda.synchronize()
        got = res.output.cpu().numpy()
        check = check_grid if job.direction == "grid" else check_vis
        check(got, alone.cpu().numpy(), 1e-6, f"job {job.tag} ({job.direction}) served vs alone")
        if job.table is not None:
            ref = (orc.grid(wl, job.data, job.table) if job.direction == "grid"
                   else orc.degrid(wl, job.data, job.table))
            check(got, ref, 1e-5, f"job {job.tag} ({job.direction}) vs oracle")


@pytest.mark.parametrize("kind", ["mwa", "tiny_fold_inverse", "diff_stokes"])
def test_footprint_estimate_bounds_the_plan(kind):
    """The host estimate the admission uses (aidg_footprint_estimate) against the device
    memory plans actually take: within 0.9 and 1.5 times the plan's device bytes (the
    subgrid count is estimated), and exactly its grid size and layer count."""
    import paper_2502_17789_amd as aidg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if kind == "mwa":
        wl, kw = synth.config_mwa(seed=2), {}
    elif kind == "tiny_fold_inverse":
        wl, kw = synth.config_tiny(71, ha0_deg=-60.0, beam_fwhm_deg=15.0), dict(w_step=12.0, w_fold=1, aterm_mode=1)
    else:
        wl, kw = synth.config_diff(seed=4), dict(stokes_i=1)
    for ws in (0, 4 * wl.subgrid_size ** 2 * 8):
        geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                            aterm_interval=wl.aterm_interval, workspace_bytes=ws, **kw)
        f = aidg.footprint(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs)
        A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
        with aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A) as p:
            info = p.info
        del A
        print(f"{kind} workspace {ws}: estimate {f['plan_bytes']} B ({f['n_subgrids']} subgrids), plan "
              f"{info['device_bytes']} B ({info['n_subgrids']} subgrids)", flush=True)
        assert f["n_wlayers"] == info["n_wlayers"] and f["grid_bytes"] == info["grid_bytes"]
        assert f["vis_bytes"] == info["vis_bytes"]
        assert 0.9 * info["device_bytes"] <= f["plan_bytes"] <= 1.5 * info["device_bytes"]


def test_served_config5_jobs_equal_alone():
    """Jobs of the served mixed workload's own sizes (synth.served_job_mix, seed 5): two
    8000^2, L = 96 jobs of more than 3M visibilities (one gridding, one degridding), four
    more of other grid and subgrid sizes, and 18 small gridding jobs of one class (L = 32,
    FP32) that are active together, so that a round holds more than the 16 ranges of one
    launch.  The executor's workspace holds 6 group images of L = 96, so launches are
    flushed when it fills, also in the middle of a job's range.  Every served result must
    equal the job run alone through its own plan: degridding bitwise (the same kernels on
    the same subgrids, deterministic), gridding within 1e-6 element-wise (the order of the
    FP32 atomic additions onto the grid differs)."""
    import paper_2502_17789_amd as aidg
    from paper_2502_17789_amd.serve import GpuBackend, Job, Server
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mix = synth.served_job_mix(2000, seed=5)

    def n_vis(d):
        return d["baselines"].shape[0] * d["uvw"].shape[1] * d["freqs"].shape[0]

    big = [31, 301]
    assert all(mix[i]["N"] == 8000 and mix[i]["L"] == 96 and n_vis(mix[i]) >= 1e6 for i in big)
    assert {mix[i]["direction"] for i in big} == {"grid", "degrid"}
    others = []
    for N, L in ((4096, 64), (2048, 32), (1024, 96), (8000, 64)):
        others.append(next(i for i, d in enumerate(mix) if d["N"] == N and d["L"] == L and 2e4 <= n_vis(d) <= 1e6
                           and i not in others))
    small = [i for i, d in enumerate(mix) if d["L"] == 32 and d["direction"] == "grid" and n_vis(d) <= 3e4][:18]
    assert len(small) == 18
    picks = big + others + small

    def job_of(i):
        d = mix[i]
        geo = aidg.Geometry(d["N"], d["L"], d["K"], d["dl"], aterm_interval=max(d["n_t"], 1))

        def aterms():
            return synth.device_phase_screen_aterms(d["n_stations"], d["L"], d["screen_rms"], d["seed"])

        def data(shape):
            g = torch.Generator(device="cuda")
            g.manual_seed(d["seed"] + 1)
            return torch.randn(shape, dtype=torch.complex64, device="cuda", generator=g)

        return Job(d["direction"], geo, d["n_stations"], d["baselines"], d["uvw"], d["freqs"], aterms, data, tag=i)

    srv = Server(GpuBackend(workspace_bytes=6 * 4 * 96 * 96 * 8), hbm_budget=64 << 30, range_subgrids=256,
                 max_active=32)
    with srv:
        futs = [srv.submit(job_of(i)) for i in picks]
        results = {f.result(timeout=300).tag: f.result().output for f in futs}
    st = srv.stats()
    print(f"served {st}", flush=True)
    assert st["ranges_per_round"] > 2
    for i in picks:
        job = job_of(i)
        A = job.aterms()
        with aidg.Plan(job.geometry, job.n_stations, job.baselines, job.uvw, job.freqs, A) as p:
            del A
            if job.direction == "grid":
                alone = p.grid(job.data(p.vis_shape()))
            else:
                alone = p.degrid(job.data(p.grid_shape()))
            torch.cuda.synchronize()
        got = results.pop(i)
        tag = f"job {i} ({job.direction}, N={job.geometry.grid_size}, L={job.geometry.subgrid_size}, " \
              f"{n_vis(mix[i])} vis) served vs alone"
        if job.direction == "degrid":
            assert torch.equal(got, alone), tag
            print(tag + ": bitwise equal", flush=True)
        else:
            for j in range(alone.shape[0]):
                check_grid(got[j].cpu().numpy(), alone[j].cpu().numpy(), 1e-6, f"{tag}, layer {j}")
        del got, alone
