"""GPU parity at the full MWA-like size, in the launch configuration bench.py times
(8128 baselines x 60 x 96 = 46.8M visibilities, grid 8000^2, L = 96, K = 24, the
library's own partition, default workspace and batching).

The oracle cannot redo a 46.8M-visibility job element by element, so each check
uses outputs it can compute one by one, or a property that holds at any size:
  * element by element on 128 random baselines (seed 2): degridding of a random
    full-size grid, compared visibility by visibility with the oracle's degridding of
    those baselines' subgrids (same table, same grid); and gridding of visibilities
    that are zero outside those baselines, compared cell by cell over the whole
    8000^2 grid with the oracle's gridding of their subgrids;
  * gridding at 256 lattice directions spread over the whole subgrid lattice (a
    16 x 16 sub-lattice, outer directions included) equals L^2 T times the direct
    A-term image of every gridded visibility (exact at lattice samples, Sec. 4.3);
  * degridding a grid made in closed form from lattice point sources gives the
    direct prediction of Eq. 1 on 128 baselines: sources over the whole lattice with
    their brightness scaled by T(x_s, y_s), so that every source's grid is of the
    same size (an unscaled grid of an outer source carries 1/T, up to 1e14 at K = 24,
    which FP32 cannot hold beside the others: the taper instability of Sec. 4.1), and
    unscaled sources where T >= 1e-2;
  * the adjoint identity <grid(V), G> = <V, degrid(G)> with G = grid(V);
  * image-level w-stacking of one polarisation against the oracle's FP64 transform,
    and the adjoint identity between invert and predict.
Gates (tests/gates.py): FP32 1e-5, normwise and on the worst element.
"""
import numpy as np
import pytest

import synth
from gates import check_grid, check_inner, check_vis

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    import paper_2502_17789_amd as aidg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = synth.config_mwa(seed=2)
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval)
    A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
    plan = aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A)
    print(f"plan: {plan.info}", flush=True)
    yield wl, plan
    plan.close()


def n1(l, m):
    r2 = l * l + m * m
    return -r2 / (1 + np.sqrt(1 - r2))


def sample_baselines(wl, n=128, seed=2):
    return np.sort(np.random.default_rng(seed).choice(wl.n_baselines, n, replace=False))


def sub_workload(wl, sel):
    return synth.Workload("sel", wl.n_stations, np.ascontiguousarray(wl.baselines[sel]),
                          np.ascontiguousarray(wl.uvw[sel]), wl.freqs, wl.grid_size, wl.subgrid_size,
                          wl.kernel_support, wl.pixel_scale, wl.aterm_interval, wl.aterms)


def sub_table(wl, table, sel):
    """The plan's subgrids of baselines `sel`, renumbered for the sub-workload."""
    pos = -np.ones(wl.n_baselines, np.int64)
    pos[sel] = np.arange(len(sel))
    t = table[pos[table["bl"]] >= 0].copy()
    t["bl"] = pos[t["bl"]]
    t["vis_offset"] = (t["bl"].astype(np.int64) * wl.n_times + t["t0"]) * wl.n_chans + t["c0"]
    return t


def test_fullsize_partition_valid(setup, orc):
    wl, plan = setup
    table = plan.subgrids()
    assert orc.check_partition(wl, table, plan.info["w_step"]) == (0, -1)


def test_fullsize_elementwise_128_baselines(setup, orc):
    wl, plan = setup
    sel = sample_baselines(wl)
    sub = sub_workload(wl, sel)
    table = sub_table(wl, plan.subgrids(), sel)
    W = plan.n_wlayers
    print(f"128 baselines: {table.shape[0]} of {plan.info['n_subgrids']} subgrids", flush=True)
    # degridding: a random full-size grid, the visibilities of the sampled baselines
    gen = torch.Generator(device="cuda")
    gen.manual_seed(26)
    G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    Vg = plan.degrid(G)
    torch.cuda.synchronize()
    Vsel = Vg[torch.from_numpy(sel).cuda()].cpu().numpy()
    del Vg
    Gh = G.cpu().numpy()
    del G
    Vo = orc.degrid(sub, Gh, table)
    del Gh
    check_vis(Vsel, Vo, 1e-5, "full-size degridding, 128 baselines, every visibility")
    mask = orc.coverage_mask(sub, table).astype(bool)
    assert np.abs(Vsel[~mask]).max(initial=0.0) == 0.0
    # gridding: visibilities zero outside the sampled baselines, every cell of the grid
    rng = np.random.default_rng(27)
    Vs = synth.random_vis((len(sel), wl.n_times, wl.n_chans), rng)
    Vfull = torch.zeros(plan.vis_shape(), dtype=torch.complex64, device="cuda")
    Vfull[torch.from_numpy(sel).cuda()] = torch.from_numpy(Vs.astype(np.complex64)).cuda()
    Gg = plan.grid(Vfull)
    torch.cuda.synchronize()
    del Vfull
    Go = orc.grid(sub, Vs, table, W=W)
    for j in range(W):
        check_grid(Gg[j].cpu().numpy(), Go[j], 1e-5, f"full-size gridding, 128 baselines, layer {j}, every cell")


def lattice_grid_16(L, rng):
    """A 16 x 16 sub-lattice spread over the whole L x L lattice, edges included."""
    base = np.linspace(0, L - 1, 16).round().astype(np.int32)
    jit = rng.integers(-1, 2, (2, 16))
    xs1 = np.clip(base + jit[0], 0, L - 1).astype(np.int32)
    ys1 = np.clip(base + jit[1], 0, L - 1).astype(np.int32)
    xs, ys = np.meshgrid(xs1, ys1)
    return xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)


def test_fullsize_grid_lattice_identity(setup, orc):
    wl, plan = setup
    L = wl.subgrid_size
    rng = np.random.default_rng(21)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng).astype(np.complex64)
    G = plan.grid(torch.from_numpy(V).cuda())
    torch.cuda.synchronize()
    Gh = G.cpu().numpy()
    del G
    w0 = plan.wlayers()
    xs, ys = lattice_grid_16(L, rng)
    l, m = orc.lattice_dirs(wl, xs, ys)
    lhs = sum(orc.layer_image_at(Gh[j], 1.0 / wl.fov, l, m) * np.exp(2j * np.pi * w0[j] * n1(l, m))[:, None]
              for j in range(Gh.shape[0]))
    del Gh
    mask = orc.coverage_mask(wl, plan.subgrids())
    T = orc.taper(L, wl.kernel_support)
    rhs = L * L * T[ys, xs][:, None] * orc.direct_image(wl, V, l, m, xs, ys, mask=mask)
    check_grid(lhs, rhs, 1e-5, f"full-size gridding, lattice identity at {len(xs)} directions")
    inner = T[ys, xs] >= 1e-2
    check_grid(lhs[inner], rhs[inner], 1e-5, f"same, the {inner.sum()} directions with T >= 1e-2")


def closed_form_grid(src, w0, N, L, du, scale):
    """Grid layers of lattice point sources in closed form: source s contributes
    scale_s B_s / (L^2 T_s) exp(-2 pi i [u l_s + v m_s + w0 n1_s]) at every cell."""
    g = torch.arange(N, dtype=torch.float64, device="cuda") - N // 2
    G = torch.zeros((len(w0), 4, N, N), dtype=torch.complex128, device="cuda")
    for s in range(len(src["l"])):
        eu = torch.exp(-2j * np.pi * g * du * float(src["l"][s]))
        ev = torch.exp(-2j * np.pi * g * du * float(src["m"][s]))
        ramp = torch.outer(ev, eu)
        for j in range(len(w0)):
            ph = np.exp(-2j * np.pi * w0[j] * n1(src["l"][s], src["m"][s])) * scale[s]
            for pol in range(4):
                G[j, pol] += complex(src["B"][s][pol] * ph) * ramp
        del ramp
    return G


@pytest.mark.parametrize("region", ["whole_lattice_scaled", "taper_above_1e-2"])
def test_fullsize_degrid_lattice_sources(setup, orc, region):
    wl, plan = setup
    L, N = wl.subgrid_size, wl.grid_size
    rng = np.random.default_rng(22)
    T = orc.taper(L, wl.kernel_support)
    n_src = 64 if region == "whole_lattice_scaled" else 16
    src = synth.point_sources(n_src, wl.fov, 0.5, 5.0, rng, L=L, on_lattice=True)
    if region == "whole_lattice_scaled":
        src["xs"] = rng.integers(0, L, n_src).astype(np.int32)
        src["ys"] = rng.integers(0, L, n_src).astype(np.int32)
    else:
        half = np.argwhere(T >= 1e-2)
        pick = half[rng.choice(len(half), n_src, replace=False)]
        src["ys"], src["xs"] = pick[:, 0].astype(np.int32), pick[:, 1].astype(np.int32)
    src["l"], src["m"] = orc.lattice_dirs(wl, src["xs"], src["ys"])
    Ts = T[src["ys"], src["xs"]]
    if region == "whole_lattice_scaled":
        src["B"] = src["B"] * Ts[:, None]     # every source's grid ~ B / L^2
    w0 = plan.wlayers()
    G = closed_form_grid(src, w0, N, L, 1.0 / wl.fov, 1.0 / (L * L * Ts))
    V = plan.degrid(G.to(torch.complex64))
    torch.cuda.synchronize()
    del G
    sel = sample_baselines(wl, seed=3)
    Vg = V.cpu().numpy()[sel].astype(np.complex128)
    del V
    sub = sub_workload(wl, sel)
    Vd = orc.direct_predict(sub, src["l"], src["m"], src["B"], src["xs"], src["ys"])
    mask = orc.coverage_mask(wl, plan.subgrids())[sel].astype(bool)
    check_vis(Vg[mask], Vd[mask], 1e-5,
              f"full-size degridding of {n_src} lattice sources ({region}, T from {Ts.min():.1e}), 128 baselines")
    assert np.abs(Vg[~mask]).max(initial=0.0) == 0.0


def test_fullsize_adjoint_identity(setup):
    wl, plan = setup
    gen = torch.Generator(device="cuda")
    gen.manual_seed(23)
    V = torch.randn(plan.vis_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    G = plan.grid(V)   # G = grid(V): <grid(V), G> = ||grid(V)||^2
    Vg = plan.degrid(G)
    torch.cuda.synchronize()
    c = torch.complex128
    lhs = sum(torch.vdot(G[j].flatten().to(c), G[j].flatten().to(c)).item() for j in range(G.shape[0]))
    rhs = torch.vdot(V.flatten().to(c), Vg.flatten().to(c)).item()
    check_inner(lhs, rhs, 1e-5, "full-size adjoint identity")


def test_fullsize_invert_matches_oracle(setup, orc):
    """Image-level w-stacking at 8000^2 (radices 4^3 5^3): one polarisation of a random
    grid against the oracle's FP64 transform."""
    wl, plan = setup
    N, L, K = wl.grid_size, wl.subgrid_size, wl.kernel_support
    gen = torch.Generator(device="cuda")
    gen.manual_seed(24)
    G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    I = plan.invert(G)
    torch.cuda.synchronize()
    pol = 1
    Ih = I[pol].cpu().numpy().astype(np.complex128)
    del I
    Gh = G[:, pol:pol + 1].cpu().numpy().astype(np.complex128)
    ref = orc.invert(Gh, plan.wlayers(), L, K, wl.pixel_scale)[0]
    check_grid(Ih, ref, 1e-5, f"full-size invert, W={plan.n_wlayers}, one polarisation")


def test_fullsize_image_adjoint_identity(setup):
    wl, plan = setup
    gen = torch.Generator(device="cuda")
    gen.manual_seed(25)
    G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    I = plan.invert(G)   # I = invert(G): <invert(G), I> = ||invert(G)||^2
    GI = plan.predict(I)
    torch.cuda.synchronize()
    c = torch.complex128
    lhs = torch.vdot(I.flatten().to(c), I.flatten().to(c)).item()
    rhs = sum(torch.vdot(G[j].flatten().to(c), GI[j].flatten().to(c)).item() for j in range(G.shape[0]))
    check_inner(lhs, rhs, 1e-5, "full-size image adjoint identity")
