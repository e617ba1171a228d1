"""GPU parity at the full MWA-like size, in the launch configuration bench.py times
(8128 baselines x 60 x 96 = 46.8M visibilities, grid 8000^2, L = 96, K = 24, the
library's own partition, default workspace and batching).

The oracle cannot redo a 46.8M-visibility job element by element, so each check
uses outputs it can compute one by one, or a property that holds at any size:
  * gridding at sampled lattice directions equals L^2 T times the direct A-term
    image of every gridded visibility (exact at lattice samples, Sec. 4.3);
  * degridding a grid made in closed form from lattice point sources gives the
    direct prediction of Eq. 1 for sampled baselines;
  * the adjoint identity <grid(V), G> = <V, degrid(G)>;
  * image-level w-stacking of one polarisation against the oracle's FP64 transform,
    and the adjoint identity between invert and predict.
All at the FP32 gate of 1e-5 (normwise relative).
"""
import numpy as np
import pytest

import synth

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


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def n1(l, m):
    r2 = l * l + m * m
    return -r2 / (1 + np.sqrt(1 - r2))


def test_fullsize_partition_valid(setup, orc):
    wl, plan = setup
    table = plan.subgrids()
    assert orc.check_partition(wl, table, plan.info["w_step"]) == (0, -1)


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
    xs = rng.integers(0, L, 8).astype(np.int32)
    ys = rng.integers(0, L, 8).astype(np.int32)
    l, m = orc.lattice_dirs(wl, xs, ys)
    lhs = sum(orc.layer_image_at(Gh[j], 1.0 / wl.fov, l, m) * np.exp(2j * np.pi * w0[j] * n1(l, m))[:, None]
              for j in range(Gh.shape[0]))
    mask = orc.coverage_mask(wl, plan.subgrids())
    T = orc.taper(L, wl.kernel_support)
    rhs = L * L * T[ys, xs][:, None] * orc.direct_image(wl, V, l, m, xs, ys, mask=mask)
    err = rel(lhs, rhs)
    print(f"full-size gridding, lattice identity at 8 directions: rel err {err:.3e}", flush=True)
    assert err <= 1e-5


def test_fullsize_degrid_lattice_sources(setup, orc):
    wl, plan = setup
    L, N = wl.subgrid_size, wl.grid_size
    rng = np.random.default_rng(22)
    src = synth.point_sources(4, wl.fov, 0.5, 5.0, rng, L=L, on_lattice=True)
    # The closed-form grid carries 1/T(x_s, y_s); with K = 24 the taper falls to ~4e-15 at
    # the lattice edge, so an FP32 grid built for an edge source holds values ~1e14 whose
    # rounding swamps every other pixel (the taper instability of Sec. 4.1).  Sources stay
    # in the central region |x - L/2| <= L/8, where T >= 0.3.
    src["xs"] = rng.integers(L // 2 - L // 8, L // 2 + L // 8 + 1, 4).astype(np.int32)
    src["ys"] = rng.integers(L // 2 - L // 8, L // 2 + L // 8 + 1, 4).astype(np.int32)
    src["l"], src["m"] = orc.lattice_dirs(wl, src["xs"], src["ys"])
    T = orc.taper(L, wl.kernel_support)
    w0 = plan.wlayers()
    du = 1.0 / wl.fov
    g = torch.arange(N, dtype=torch.float64, device="cuda") - N // 2
    G = torch.zeros((len(w0), 4, N, N), dtype=torch.complex128, device="cuda")
    for s in range(4):
        eu = torch.exp(-2j * np.pi * g * du * float(src["l"][s]))
        ev = torch.exp(-2j * np.pi * g * du * float(src["m"][s]))
        ramp = torch.outer(ev, eu)
        scale = 1.0 / (L * L * T[src["ys"][s], src["xs"][s]])
        for j in range(len(w0)):
            ph = np.exp(-2j * np.pi * w0[j] * n1(src["l"][s], src["m"][s])) * scale
            for pol in range(4):
                G[j, pol] += complex(src["B"][s][pol] * ph) * ramp
        del ramp
    V = plan.degrid(G.to(torch.complex64))
    torch.cuda.synchronize()
    del G
    sel = np.sort(rng.choice(wl.n_baselines, 16, replace=False))
    Vg = V.cpu().numpy()[sel].astype(np.complex128)
    sub = synth.Workload("sel", wl.n_stations, np.ascontiguousarray(wl.baselines[sel]),
                         np.ascontiguousarray(wl.uvw[sel]), wl.freqs, N, L, wl.kernel_support,
                         wl.pixel_scale, wl.aterm_interval, wl.aterms)
    Vd = orc.direct_predict(sub, src["l"], src["m"], src["B"], src["xs"], src["ys"])
    mask = orc.coverage_mask(wl, plan.subgrids())[sel].astype(bool)
    err = rel(Vg[mask], Vd[mask])
    per = np.linalg.norm(Vg[mask] - Vd[mask], axis=-1) / np.linalg.norm(Vd[mask], axis=-1)
    print(f"full-size degridding, 16 baselines: rel err {err:.3e}; per-vis max {per.max():.3e}, "
          f"p99 {np.percentile(per, 99):.3e}", flush=True)
    assert err <= 1e-5
    assert np.abs(Vg[~mask]).max(initial=0.0) == 0.0


def test_fullsize_adjoint_identity(setup):
    wl, plan = setup
    gen = torch.Generator(device="cuda")
    gen.manual_seed(23)
    V = torch.randn(plan.vis_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    Gv = plan.grid(V)
    Vg = plan.degrid(G)
    torch.cuda.synchronize()
    lhs = torch.vdot(Gv.flatten().to(torch.complex128), G.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(V.flatten().to(torch.complex128), Vg.flatten().to(torch.complex128)).item()
    scale = (Gv.to(torch.complex128).norm() * G.to(torch.complex128).norm()
             + V.to(torch.complex128).norm() * Vg.to(torch.complex128).norm()).item()
    print(f"full-size adjoint residual {abs(lhs - rhs) / scale:.3e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale


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
    err = rel(Ih, ref)
    print(f"full-size invert, W={plan.n_wlayers}, one polarisation: rel err {err:.3e}", flush=True)
    assert err <= 1e-5


def test_fullsize_image_adjoint_identity(setup):
    wl, plan = setup
    gen = torch.Generator(device="cuda")
    gen.manual_seed(25)
    G = torch.randn(plan.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    I = torch.randn(plan.image_shape(), dtype=torch.complex64, device="cuda", generator=gen)
    IG = plan.invert(G)
    GI = plan.predict(I)
    torch.cuda.synchronize()
    c = torch.complex128
    lhs = torch.vdot(IG.flatten().to(c), I.flatten().to(c)).item()
    rhs = torch.vdot(G.flatten().to(c), GI.flatten().to(c)).item()
    scale = (IG.to(c).norm() * I.to(c).norm() + G.to(c).norm() * GI.to(c).norm()).item()
    print(f"full-size image adjoint residual {abs(lhs - rhs) / scale:.3e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale
