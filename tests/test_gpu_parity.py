"""GPU parity: the HIP gridder/degridder (through the C ABI) against the FP64 oracle.

Bar (tests/gates.py): per result the normwise relative error AND the worst element
(grids: max |dG| / max |G|; visibilities: max_k ||dV_k|| / rms_k ||V_k||):
  FP32 path  <= 1e-5     FP64 path <= 1e-10
  adjoint identity <grid(V), G> = <V, degrid(G)> on GPU outputs with G = grid(V), FP64
  sums: |lhs - rhs| / |lhs| <= 1e-5 (FP32), 1e-10 (FP64)
The oracle is fed the same partition as the library (the oracle's own partition,
passed to the library as a caller table), so element-by-element comparison is
meaningful; the library's own partition is checked through the partition-free
lattice identities instead.
"""
import math

import numpy as np
import pytest

import synth
from gates import check_grid, check_inner, check_vis

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aidg():
    import paper_2502_17789_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m.library()
    return m


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def dev(x, prec):
    dt = np.complex64 if prec == 0 else np.complex128
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()


def plan_for(aidg, wl, table=None, precision=0, **kw):
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision, **kw)
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, dev(wl.aterms, precision),
                     table=table)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


CASES = {
    "L32": dict(seed=101, L=32, K=8, N=128, n_st=6, n_t=6, n_c=9, w_step=12.0),
    "L64": dict(seed=102, L=64, K=16, N=256, n_st=5, n_t=7, n_c=20, fov_deg=15.0, diameter_m=800.0,
                w_step=20.0),
    "L96": dict(seed=103, L=96, K=24, N=384, n_st=4, n_t=5, n_c=33, fov_deg=12.0, diameter_m=1500.0,
                aterm_interval=2, w_step=0.0),
}


def case_workload(name):
    c = dict(CASES[name])
    w_step = c.pop("w_step")
    return synth.config_tiny(**c), w_step


@pytest.mark.parametrize("name", sorted(CASES))
def test_grid_matches_oracle(aidg, orc, name):
    wl, w_step = case_workload(name)
    table = orc.partition(wl, w_step)
    rng = np.random.default_rng(7)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    ref = orc.grid(wl, V, table)
    with plan_for(aidg, wl, table) as p:
        G = host(p.grid(dev(V, 0)))
    print(f"{name}: {table.shape[0]} subgrids")
    check_grid(G, ref, 1e-5, f"{name} grid")


@pytest.mark.parametrize("name", sorted(CASES))
def test_degrid_matches_oracle(aidg, orc, name):
    wl, w_step = case_workload(name)
    table = orc.partition(wl, w_step)
    rng = np.random.default_rng(8)
    G = synth.random_grid(orc.n_layers(table), wl.grid_size, rng)
    ref = orc.degrid(wl, G, table)
    with plan_for(aidg, wl, table) as p:
        V = host(p.degrid(dev(G, 0)))
    check_vis(V, ref, 1e-5, f"{name} degrid")


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_path_matches_oracle(aidg, orc, name):
    wl, w_step = case_workload(name)
    table = orc.partition(wl, w_step)
    rng = np.random.default_rng(9)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    G = synth.random_grid(orc.n_layers(table), wl.grid_size, rng)
    with plan_for(aidg, wl, table, precision=1) as p:
        Gg = host(p.grid(dev(V, 1)))
        Vg = host(p.degrid(dev(G, 1)))
    check_grid(Gg, orc.grid(wl, V, table), 1e-10, f"{name} fp64 grid")
    check_vis(Vg, orc.degrid(wl, G, table), 1e-10, f"{name} fp64 degrid")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_identity_on_gpu(aidg, name, precision):
    """<grid(V), G> = <V, degrid(G)> with G = grid(V): both sides are then of the order
    of ||grid(V)||^2, so the relative residual measures the adjoint mismatch itself."""
    wl, _ = case_workload(name)
    rng = np.random.default_rng(10)
    with plan_for(aidg, wl, precision=precision) as p:
        V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
        Vd = dev(V, precision)
        Gd = p.grid(Vd)
        Vg = host(p.degrid(Gd))
        Gv = host(Gd)
    Vr = np.asarray(Vd.cpu().numpy(), np.complex128)
    lhs, rhs = np.vdot(Gv, Gv), np.vdot(Vr, Vg)
    check_inner(lhs, rhs, 1e-5 if precision == 0 else 1e-10, f"{name} precision {precision} adjoint")


def n1(l, m):
    r2 = l * l + m * m
    return -r2 / (1 + np.sqrt(1 - r2))


@pytest.mark.parametrize("name", sorted(CASES))
def test_library_partition_lattice_identity(aidg, orc, name):
    """With the library's own partition: the gridded image at lattice directions
    equals L^2 T times the direct A-term image (Sec. 4.3: exact at lattice samples)."""
    wl, _ = case_workload(name)
    L = wl.subgrid_size
    rng = np.random.default_rng(11)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    with plan_for(aidg, wl) as p:
        G = host(p.grid(dev(V, 0)))
        table = p.subgrids()
        w0 = p.wlayers()
    assert orc.check_partition(wl, table, p.info["w_step"])[0] == 0
    xs = rng.integers(0, L, 40).astype(np.int32)
    ys = rng.integers(0, L, 40).astype(np.int32)
    l, m = orc.lattice_dirs(wl, xs, ys)
    lhs = sum(orc.layer_image_at(G[j], 1.0 / wl.fov, l, m) * np.exp(2j * np.pi * w0[j] * n1(l, m))[:, None]
              for j in range(G.shape[0]))
    T = orc.taper(L, wl.kernel_support)
    rhs = L * L * T[ys, xs][:, None] * orc.direct_image(
        wl, np.asarray(dev(V, 0).cpu().numpy(), np.complex128), l, m, xs, ys,
        mask=orc.coverage_mask(wl, table))
    check_grid(lhs, rhs, 1e-5, f"{name} lattice identity at 40 directions")


def test_grid_accumulates(aidg, orc):
    wl, w_step = case_workload("L32")
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), np.random.default_rng(1))
    with plan_for(aidg, wl) as p:
        g1 = p.grid(dev(V, 0))
        g2 = host(p.grid(dev(V, 0), out=g1.clone()))
        g1 = host(g1)
    assert rel(g2, 2 * g1) < 1e-6


EDGE = {
    "one_channel": dict(seed=201, n_c=1, n_t=4),
    "one_vis": dict(seed=202, n_st=2, n_t=1, n_c=1),
    "edges_excluded": dict(seed=203, N=64, diameter_m=700.0, n_t=6, n_c=8),
    "long_rows": dict(seed=204, n_st=3, n_t=3, n_c=70, f_lo=150e6, f_hi=151e6),
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases(aidg, orc, name):
    wl = synth.config_tiny(**EDGE[name])
    table = orc.partition(wl, 0.0)
    rng = np.random.default_rng(12)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    G = synth.random_grid(orc.n_layers(table), wl.grid_size, rng)
    with plan_for(aidg, wl, table, reseed_channels=16) as p:
        Gg = host(p.grid(dev(V, 0)))
        Vd = dev(np.full(V.shape, 7.0 + 7.0j), 0)  # degrid must overwrite everything
        Vg = host(p.degrid(dev(G, 0), out=Vd))
    check_grid(Gg, orc.grid(wl, V, table), 1e-5, f"{name} grid")
    check_vis(Vg, orc.degrid(wl, G, table), 1e-5, f"{name} degrid")
    mask = orc.coverage_mask(wl, table)
    assert np.abs(Vg[mask == 0]).max(initial=0.0) == 0.0


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("R", [1, 2, 3, 5, 8, 32])
def test_reseed_intervals(aidg, orc, R, precision):
    """Recurrence runs for re-seeding intervals from one channel up: rows of 23 channels
    split into runs of one channel (R = 1), of two, or of balanced even lengths with a
    ragged last run of odd length; grid and degrid against the oracle, FP32 and FP64."""
    wl = synth.config_tiny(206, n_st=4, n_t=5, n_c=23)
    table = orc.partition(wl, 0.0)
    rng = np.random.default_rng(13)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    G = synth.random_grid(orc.n_layers(table), wl.grid_size, rng)
    tol = 1e-5 if precision == 0 else 1e-10
    with plan_for(aidg, wl, table, precision=precision, reseed_channels=R,
                  degrid_form=aidg.DEGRID_RECURRENCE) as p:
        Gg = host(p.grid(dev(V, precision)))
        Vg = host(p.degrid(dev(G, precision)))
    check_grid(Gg, orc.grid(wl, V, table), tol, f"R={R} grid")
    check_vis(Vg, orc.degrid(wl, G, table), tol, f"R={R} degrid")


def test_nonuniform_channels_and_split_subgrids(aidg, orc):
    """Irregular channel spacing (phasors re-seeded every channel) and subgrids
    larger than the per-subgrid cap (split by the library)."""
    wl = synth.config_tiny(205, n_st=4, n_t=6, n_c=12, aterm_interval=6)
    wl.freqs = np.sort(140e6 + 20e6 * np.random.default_rng(3).random(12))
    table = orc.partition(wl, 0.0)
    rng = np.random.default_rng(13)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    G = synth.random_grid(orc.n_layers(table), wl.grid_size, rng)
    with plan_for(aidg, wl, table, max_subgrid_vis=5) as p:
        assert p.info["max_subgrid_vis"] <= 5
        Gg = host(p.grid(dev(V, 0)))
        Vg = host(p.degrid(dev(G, 0)))
    check_grid(Gg, orc.grid(wl, V, table), 1e-5, "irregular channels grid")
    check_vis(Vg, orc.degrid(wl, G, table), 1e-5, "irregular channels degrid")


def test_small_workspace_many_batches(aidg, orc):
    wl, w_step = case_workload("L32")
    table = orc.partition(wl, w_step)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), np.random.default_rng(14))
    with plan_for(aidg, wl, table, workspace_bytes=3 * 4 * 32 * 32 * 8) as p:
        assert p.info["n_batches"] == -(-p.info["n_groups"] // 3)
        G = host(p.grid(dev(V, 0)))
    check_grid(G, orc.grid(wl, V, table), 1e-5, "many batches grid")


def test_unsupported_subgrid_size(aidg):
    wl = synth.config_tiny(1, L=48, K=8, N=128)
    with pytest.raises(aidg.AidgError) as e:
        plan_for(aidg, wl)
    assert e.value.status == aidg.AIDG_E_UNSUPPORTED


def test_bad_caller_table_rejected(aidg, orc):
    wl, w_step = case_workload("L32")
    table = orc.partition(wl, w_step)
    dup = np.concatenate([table, table[:1]])
    with pytest.raises(aidg.AidgError) as e:
        plan_for(aidg, wl, dup)
    assert e.value.status == aidg.AIDG_E_INVALID
    off = table.copy()
    off["U0"][0] = 2
    with pytest.raises(aidg.AidgError):
        plan_for(aidg, wl, off)


GROUPED = {"L32": 4, "L64": 8, "L96": 16}


@pytest.mark.parametrize("name", sorted(GROUPED))
def test_grouped_centres_match_oracle(aidg, orc, name):
    """Library partition with centres on a coarse lattice, so that several subgrids
    share a centre and w-layer (one summed image, one FFT and one grid update per
    group); the oracle grids/degrids the same table subgrid by subgrid."""
    wl, w_step = case_workload(name)
    rng = np.random.default_rng(15)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    for prec, tol in ((0, 1e-5), (1, 1e-10)):
        with plan_for(aidg, wl, precision=prec, w_step=w_step, center_lattice=GROUPED[name]) as p:
            table = p.subgrids()
            info = p.info
            G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
            Gg = host(p.grid(dev(V, prec)))
            Vg = host(p.degrid(dev(G, prec)))
        assert orc.check_partition(wl, table, info["w_step"])[0] == 0
        assert info["n_groups"] < info["n_subgrids"]
        print(f"{name} precision {prec}: {info['n_subgrids']} subgrids in {info['n_groups']} groups")
        check_grid(Gg, orc.grid(wl, V, table), tol, f"{name} precision {prec} grid")
        check_vis(Vg, orc.degrid(wl, G, table), tol, f"{name} precision {prec} degrid")


def test_executor_ranges_split_groups(aidg, orc):
    """Executor ranges that start and end inside groups, and a workspace of two
    group images (many launches), give the plan's own result."""
    wl, w_step = case_workload("L64")
    rng = np.random.default_rng(16)
    V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 0)
    with plan_for(aidg, wl, w_step=w_step, center_lattice=8) as p:
        t = p.subgrids()
        n = t.shape[0]
        key = t["wlayer"].astype(np.int64) * 10**8 + t["V0"].astype(np.int64) * 10**4 + t["U0"]
        inner = [i for i in range(1, n) if key[i] == key[i - 1]]
        assert inner, "no group with two subgrids"
        cuts = sorted(set([0, n] + inner[:: max(1, len(inner) // 5)]))
        G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
        Gd = dev(G, 0)
        ref_g = host(p.grid(V))
        ref_v = host(p.degrid(Gd))
        ex = aidg.Executor(workspace_bytes=2 * 4 * 64 * 64 * 8)
        try:
            out_g = torch.zeros(p.grid_shape(), dtype=torch.complex64, device="cuda")
            out_v = torch.zeros(p.vis_shape(), dtype=torch.complex64, device="cuda")
            items = [(p, aidg.DIR_GRID, V, out_g, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
            items += [(p, aidg.DIR_DEGRID, Gd, out_v, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
            ex.execute(items)
            got_g, got_v = host(out_g), host(out_v)
        finally:
            ex.close()
    print(f"executor over {len(cuts) - 1} ranges")
    check_grid(got_g, ref_g, 1e-6, "executor grid")
    check_vis(got_v, ref_v, 1e-6, "executor degrid")
