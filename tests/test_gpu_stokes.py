"""GPU parity of Stokes-I grids (geometry stokes_i = 1): one complex value per grid cell,
I = (XX + YY) / 2 of each A-term-corrected subgrid image; degridding predicts the
visibilities of the unpolarised brightness I [[1, 0], [0, 1]].

  * gridding, degridding and invert match the oracle element by element (FP32 <= 1e-5,
    FP64 <= 1e-10, normwise), also with the w >= 0 fold and the inverse A-term mode;
  * grids are [W][1][N][N], a quarter of the four-plane size;
  * through the library alone, <grid(V), G> = <V, degrid(G)> / 2, and the autograd
    wrappers carry that factor;
  * a grouped launch mixing a Stokes-I plan and a four-plane plan gives each its own
    result.
"""
import numpy as np
import pytest

import synth
from gates import check_grid, check_vis

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def plan_for(aidg, wl, precision, w_step, stokes=1, fold=0, mode=0):
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision, w_step=w_step,
                        w_fold=fold, aterm_mode=mode, stokes_i=stokes)
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, dev(wl.aterms, precision))


CASES = {
    "one_layer": dict(wl=dict(seed=101), w_step=-1.0),
    "layers": dict(wl=dict(seed=102), w_step=12.0),
    "fold": dict(wl=dict(seed=103, ha0_deg=-60.0), w_step=12.0, fold=1),
    "inverse": dict(wl=dict(seed=104, beam_fwhm_deg=15.0), w_step=12.0, mode=1),
    "L64": dict(wl=dict(seed=105, N=256, L=64, K=16), w_step=12.0),
}
TOL = {0: 1e-5, 1: 1e-10}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_stokes_i_matches_oracle(aidg, orc, name, precision):
    c = CASES[name]
    wl = synth.config_tiny(**c["wl"])
    N, L, K = wl.grid_size, wl.subgrid_size, wl.kernel_support
    rng = np.random.default_rng(11)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    with plan_for(aidg, wl, precision, c["w_step"], fold=c.get("fold", 0), mode=c.get("mode", 0)) as p:
        W = p.n_wlayers
        assert p.grid_shape() == (W, 1, N, N) and p.image_shape() == (1, N, N)
        assert p.info["grid_bytes"] == W * N * N * (8 if precision == 0 else 16)
        table = p.subgrids()
        w0 = p.wlayers()
        GI = synth.random_grid(W, N, rng)[:, :1]
        Gt = p.grid(dev(V, precision))
        Ig = host(p.invert(Gt))
        Gg = host(Gt)
        Vg = host(p.degrid(dev(GI, precision)))
        nrm = p.aterm_norm() if c.get("mode", 0) else None
    Go = orc.grid_stokes_i(wl, V, table, W=W, aterm_mode=c.get("mode", 0))
    Vo = orc.degrid_stokes_i(wl, GI, table)
    Io = orc.invert(Go, w0, L, K, wl.pixel_scale,
                    norm=None if nrm is None else orc.aterm_norm(wl, table))
    q = N // 4
    tag = f"stokes {name} {'FP64' if precision else 'FP32'} W={W}"
    check_grid(Gg, Go, TOL[precision], tag + " grid")
    check_vis(Vg, Vo, TOL[precision], tag + " degrid")
    check_grid(Ig[:, q:3 * q, q:3 * q], Io[:, q:3 * q, q:3 * q], TOL[precision], tag + " image")


def test_stokes_i_adjoint_relation_and_autograd(aidg):
    """<grid(V), G> = <V, degrid(G)> / 2 on a Stokes-I plan, and the vector-Jacobian
    products of DegridFn and GridFn are the adjoints: <G, vjp_degrid(gV)> =
    <degrid(G), gV> and <V, vjp_grid(gG)> = <grid(V), gG>."""
    from paper_2502_17789_amd import autograd
    wl = synth.config_tiny(106)
    rng = np.random.default_rng(12)
    with plan_for(aidg, wl, 1, 12.0) as p:
        # excluded visibilities drop out of both sides: gridding ignores them and
        # degridding writes 0 for them
        V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 1)
        G = dev(synth.random_grid(p.n_wlayers, wl.grid_size, rng)[:, :1], 1)
        lhs = torch.vdot(p.grid(V).flatten(), G.flatten()).item()
        rhs = 0.5 * torch.vdot(V.flatten(), p.degrid(G).flatten()).item()
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
        Gr = G.clone().requires_grad_(True)
        gV = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 1)
        out = autograd.degrid(Gr, p)
        (g,) = torch.autograd.grad(out, Gr, grad_outputs=gV)
        a = torch.vdot(G.flatten(), g.flatten()).item()
        b = torch.vdot(p.degrid(G).flatten(), gV.flatten()).item()
        assert abs(a - b) <= 1e-10 * abs(b)
        Vr = V.clone().requires_grad_(True)
        gG = dev(synth.random_grid(p.n_wlayers, wl.grid_size, rng)[:, :1], 1)
        out = autograd.grid(Vr, p)
        (g,) = torch.autograd.grad(out, Vr, grad_outputs=gG)
        a = torch.vdot(V.flatten(), g.flatten()).item()
        b = torch.vdot(p.grid(V).flatten(), gG.flatten()).item()
        assert abs(a - b) <= 1e-10 * abs(b)


def test_grouped_launch_mixes_stokes_i_and_four_plane_plans(aidg):
    wl = synth.config_tiny(107)
    rng = np.random.default_rng(13)
    V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 0)
    with plan_for(aidg, wl, 0, 12.0, stokes=0) as p4, plan_for(aidg, wl, 0, 12.0, stokes=1) as p1:
        G4 = dev(synth.random_grid(p4.n_wlayers, wl.grid_size, rng), 0)
        G1 = dev(synth.random_grid(p1.n_wlayers, wl.grid_size, rng)[:, :1], 0)
        ref = [host(p4.grid(V)), host(p1.grid(V)), host(p4.degrid(G4)), host(p1.degrid(G1))]
        out = [torch.zeros_like(G4), torch.zeros_like(G1), torch.empty_like(V), torch.empty_like(V)]
        n4, n1 = p4.info["n_subgrids"], p1.info["n_subgrids"]
        ex = aidg.Executor()
        try:
            ex.execute([(p4, aidg.DIR_GRID, V, out[0], 0, n4), (p1, aidg.DIR_GRID, V, out[1], 0, n1)])
            ex.execute([(p4, aidg.DIR_DEGRID, G4, out[2], 0, n4), (p1, aidg.DIR_DEGRID, G1, out[3], 0, n1)])
            got = [host(t) for t in out]
        finally:
            ex.close()
    for i, (r, o) in enumerate(zip(ref, got)):
        (check_grid if i < 2 else check_vis)(o, r, 1e-6, f"grouped launch output {i}")


def test_library_adjoint_pair_on_stokes_i_plans(aidg):
    """aidg_grid_adjoint / aidg_degrid_adjoint are the exact adjoints of degridding and
    gridding also on a Stokes-I plan (the factors 2 and 1/2 inside the library), equal
    aidg_grid / aidg_degrid on a four-plane plan, and are refused in the inverse A-term
    mode."""
    wl = synth.config_tiny(108)
    rng = np.random.default_rng(14)
    with plan_for(aidg, wl, 1, 12.0) as p:
        V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 1)
        G = dev(synth.random_grid(p.n_wlayers, wl.grid_size, rng)[:, :1], 1)
        a = torch.vdot(p.grid_adjoint(V).flatten(), G.flatten()).item()
        b = torch.vdot(V.flatten(), p.degrid(G).flatten()).item()
        assert abs(a - b) <= 1e-12 * abs(b)
        a = torch.vdot(p.grid(V).flatten(), G.flatten()).item()
        b = torch.vdot(V.flatten(), p.degrid_adjoint(G).flatten()).item()
        assert abs(a - b) <= 1e-12 * abs(b)
        check_grid(host(p.grid_adjoint(V)), 2 * host(p.grid(V)), 1e-14, "Stokes-I grid_adjoint = 2 grid")
        check_vis(host(p.degrid_adjoint(G)), 0.5 * host(p.degrid(G)), 1e-14, "Stokes-I degrid_adjoint = degrid / 2")
    with plan_for(aidg, wl, 0, 12.0, stokes=0) as p:
        V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 0)
        G = dev(synth.random_grid(p.n_wlayers, wl.grid_size, rng), 0)
        assert torch.equal(p.degrid_adjoint(G), p.degrid(G))
        check_grid(host(p.grid_adjoint(V)), host(p.grid(V)), 1e-6, "four planes: grid_adjoint = grid")
    with plan_for(aidg, wl, 0, 12.0, mode=1) as p:
        V = dev(synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng), 0)
        with pytest.raises(aidg.AidgError) as e:
            p.grid_adjoint(V)
        assert e.value.status == aidg.AIDG_E_INVALID
