"""GPU parity of the inverse A-term mode and of Stokes-I grids at the full MWA-like size
(8128 baselines x 60 x 96 = 46.8M visibilities, grid 8000^2, L = 96, K = 24, the
library's own partition), in the launch configuration of `bench.py --aterm-mode 1` and
`bench.py --stokes-i`.  As for the default mode, each check uses outputs the oracle can
compute one by one:
  * inverse mode: the normalisation map against the oracle's, and gridding at sampled
    lattice directions against L^2 T sum_k f_k B_p^H V_k B_q exp(+2 pi i phi_k), the
    direct image with the Jones terms B = (A^-1)^H and the visibilities scaled by
    f = 1 / ||A_p^-1 A_q^-H||_F at that direction (B and f from numpy's inverse);
  * Stokes-I: gridding at sampled lattice directions against (XX + YY) / 2 of L^2 T
    times the direct A-term image, and <grid(V), G> = <V, degrid(G)> / 2.
All at the FP32 gate of 1e-5, normwise and on the worst element (tests/gates.py).
"""
import dataclasses

import numpy as np
import pytest

import synth
from gates import check_grid, check_inner

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mwa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return synth.config_mwa(seed=2)


def plan_for(wl, **kw):
    import paper_2502_17789_amd as aidg
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, **kw)
    A = torch.from_numpy(wl.aterms.astype(np.complex64)).cuda()
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def n1(l, m):
    r2 = l * l + m * m
    return -r2 / (1 + np.sqrt(1 - r2))


def layer_sum_at(orc, wl, Gh, w0, l, m):
    """sum_w exp(+2 pi i w0 n1) times each layer's image at (l, m)."""
    return sum(orc.layer_image_at(Gh[j], 1.0 / wl.fov, l, m) * np.exp(2j * np.pi * w0[j] * n1(l, m))[:, None]
               for j in range(Gh.shape[0]))


def grid_host(plan, V):
    G = plan.grid(torch.from_numpy(V).cuda())
    torch.cuda.synchronize()
    Gh = G.cpu().numpy()
    del G
    return Gh


def test_fullsize_inverse_mode(mwa, orc):
    wl = mwa
    L = wl.subgrid_size
    rng = np.random.default_rng(31)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng).astype(np.complex64)
    with plan_for(wl, aterm_mode=1) as p:
        table = p.subgrids()
        w0 = p.wlayers()
        M = p.aterm_norm()
        Gh = grid_host(p, V)
    check_grid(M, orc.aterm_norm(wl, table), 1e-5, "full-size inverse mode: normalisation map")
    # directions inside the beam's main lobe, where the inverse stays well conditioned
    xs = rng.integers(L // 2 - L // 6, L // 2 + L // 6, 4).astype(np.int32)
    ys = rng.integers(L // 2 - L // 6, L // 2 + L // 6, 4).astype(np.int32)
    l, m = orc.lattice_dirs(wl, xs, ys)
    lhs = layer_sum_at(orc, wl, Gh, w0, l, m)
    mask = orc.coverage_mask(wl, table)
    T = orc.taper(L, wl.kernel_support)
    A = wl.aterms.reshape(wl.aterms.shape[:-1] + (2, 2))
    t_int = np.arange(wl.n_times) // wl.aterm_interval
    p_st, q_st = wl.baselines[:, 0], wl.baselines[:, 1]
    rhs = np.zeros((len(xs), 4), np.complex128)
    Vd = V.astype(np.complex128)
    for d in range(len(xs)):
        Ai = np.linalg.inv(A[:, :, ys[d], xs[d]])                 # [n_int][n_st][2][2]
        B = np.conj(np.swapaxes(Ai, -1, -2))                        # (A^-1)^H
        prod = Ai[:, p_st] @ np.conj(np.swapaxes(Ai[:, q_st], -1, -2))  # [n_int][nbl][2][2]
        f = 1.0 / np.sqrt((np.abs(prod) ** 2).sum(axis=(-1, -2)))  # [n_int][nbl]
        Vs = Vd * f[t_int].T[:, :, None, None]                      # [nbl][nt][nc][4]
        Ab = wl.aterms.copy()
        Ab[:, :, ys[d], xs[d]] = B.reshape(B.shape[:2] + (4,))
        wlb = dataclasses.replace(wl, aterms=Ab)
        rhs[d] = L * L * T[ys[d], xs[d]] * orc.direct_image(wlb, Vs, l[d:d + 1], m[d:d + 1], xs[d:d + 1],
                                                           ys[d:d + 1], mask=mask)[0]
    check_grid(lhs, rhs, 1e-5, f"full-size inverse-mode gridding, lattice identity at {len(xs)} directions")


def test_fullsize_stokes_i(mwa, orc):
    wl = mwa
    L = wl.subgrid_size
    rng = np.random.default_rng(32)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng).astype(np.complex64)
    with plan_for(wl, stokes_i=1) as p:
        table = p.subgrids()
        w0 = p.wlayers()
        assert p.grid_shape()[1] == 1
        Gh = grid_host(p, V)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(33)
        Vt = torch.randn(p.vis_shape(), dtype=torch.complex64, device="cuda", generator=gen)
        Gt = p.grid(Vt)   # G = grid(V): <grid(V), G> = ||grid(V)||^2
        Vg = p.degrid(Gt).to(torch.complex128)
        Vt, Gt = Vt.to(torch.complex128), Gt.to(torch.complex128)
        lhs_a = torch.vdot(Gt.flatten(), Gt.flatten()).item()
        rhs_a = 0.5 * torch.vdot(Vt.flatten(), Vg.flatten()).item()
        del Vg, Vt, Gt
    check_inner(lhs_a, rhs_a, 1e-5, "full-size Stokes-I adjoint relation")
    xs = rng.integers(0, L, 6).astype(np.int32)
    ys = rng.integers(0, L, 6).astype(np.int32)
    l, m = orc.lattice_dirs(wl, xs, ys)
    lhs = layer_sum_at(orc, wl, Gh, w0, l, m)[:, 0]
    T = orc.taper(L, wl.kernel_support)
    ref = orc.direct_image(wl, V, l, m, xs, ys, mask=orc.coverage_mask(wl, table))
    rhs = L * L * T[ys, xs] * 0.5 * (ref[:, 0] + ref[:, 3])
    check_grid(lhs, rhs, 1e-5, f"full-size Stokes-I gridding, lattice identity at {len(xs)} directions")
