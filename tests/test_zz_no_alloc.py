"""aidg_execute_static, the entry point that allocates nothing (its group images live
in the library's static device workspace), against aidg_execute through an executor:
two calls in a row, the second with a smaller input, each with gridding and
degridding items of two plans (subgrid sizes 32 and 64), at the FP32 gates of
tests/gates.py (element-wise; gridding differs only in the order of FP32 atomic
additions, degridding not at all)."""
import numpy as np
import pytest

import synth
from gates import check_grid, check_vis

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(aidg, seed, L, K, N, n_t, n_c):
    wl = synth.config_tiny(seed, n_st=5, n_t=n_t, n_c=n_c, L=L, K=K, N=N, fov_deg=12.0, diameter_m=900.0)
    geo = aidg.Geometry(N, L, K, wl.pixel_scale, aterm_interval=wl.aterm_interval, center_lattice=4)
    A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
    return wl, aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A)


def run_both(aidg, jobs, budget):
    """jobs: list of (plan, direction, input); returns the outputs of aidg_execute_static
    and of aidg_execute for the same items."""
    outs = {}
    for kind in ("static", "executor"):
        items, res = [], []
        for plan, direction, x in jobs:
            if direction == aidg.DIR_GRID:
                out = torch.zeros(plan.grid_shape(), dtype=torch.complex64, device="cuda")
            else:
                out = torch.full(plan.vis_shape(), 3.0 + 3.0j, dtype=torch.complex64, device="cuda")
            n = plan.info["n_subgrids"]
            # two ranges per plan, the cut inside the table
            items += [(plan, direction, x, out, 0, n // 2), (plan, direction, x, out, n // 2, n)]
            res.append(out)
        if kind == "static":
            aidg.execute_static(items, workspace_bytes=budget)
        else:
            ex = aidg.Executor(workspace_bytes=budget)
            try:
                ex.execute(items)
            finally:
                ex.close()
        torch.cuda.synchronize()
        outs[kind] = [r.cpu().numpy() for r in res]
    return outs


def test_execute_static_matches_execute():
    import paper_2502_17789_amd as aidg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(61)
    wl1, p1 = make(aidg, 611, 32, 8, 128, 6, 24)
    wl2, p2 = make(aidg, 612, 64, 16, 256, 5, 20)
    wl3, p3 = make(aidg, 613, 32, 8, 128, 2, 5)   # the smaller second call
    try:
        def vis(wl):
            return torch.from_numpy(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
                                    .astype(np.complex64)).cuda()

        def grid(p):
            return torch.from_numpy(synth.random_grid(p.n_wlayers, p.geometry.grid_size, rng)
                                    .astype(np.complex64)).cuda()

        calls = [
            ("first call", [(p1, aidg.DIR_GRID, vis(wl1)), (p2, aidg.DIR_GRID, vis(wl2)),
                            (p1, aidg.DIR_DEGRID, grid(p1)), (p2, aidg.DIR_DEGRID, grid(p2))],
             5 * 4 * 64 * 64 * 8),                  # a few group images per launch: many launches
            ("second, smaller call", [(p3, aidg.DIR_GRID, vis(wl3)), (p3, aidg.DIR_DEGRID, grid(p3))], 0),
        ]
        for name, jobs, budget in calls:
            outs = run_both(aidg, jobs, budget)
            for i, ((plan, direction, _), s, e) in enumerate(zip(jobs, outs["static"], outs["executor"])):
                tag = f"{name}, item {i} ({'grid' if direction == aidg.DIR_GRID else 'degrid'})"
                if direction == aidg.DIR_GRID:
                    check_grid(s, e, 1e-5, tag)
                else:
                    check_vis(s, e, 1e-5, tag)
                    assert np.abs(s).max() > 0
    finally:
        for p in (p1, p2, p3):
            p.close()
