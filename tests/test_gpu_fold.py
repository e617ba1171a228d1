"""GPU parity of the w >= 0 fold (geometry w_fold = 1): rows with w < 0 are gridded
at (-u, -v, -w) by V(-u,-v,-w) = V(u,v,w)^H (Sec. 2.4 footnote), with the two
stations' A-terms swapped, and the w-layers sit at odd multiples of w_step / 2.

  * the library's fold partition passes the oracle's checker, and gridding and
    degridding on it match the oracle element by element (FP32 <= 1e-5,
    FP64 <= 1e-10, normwise);
  * through the library alone: the Hermitian part of invert(grid(V)) at lattice
    pixels is that of the direct A-term image (gated on the tapered image, the
    quantity the FP32 transform produces), and degrid(predict(I)) of lattice
    point sources with Hermitian brightness is their direct prediction.
"""
import numpy as np
import pytest

import synth
from gates import check_grid, check_image, check_vis

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
    return t.cpu().numpy().astype(np.complex128)


def plan_for(aidg, wl, precision=0):
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision, w_step=12.0, w_fold=1)
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, dev(wl.aterms, precision))


def herm_part(M):
    return 0.5 * (M + np.conj(M[..., [0, 2, 1, 3]]))


CASES = {"transit": dict(seed=51, ha0_deg=0.0), "west": dict(seed=52, ha0_deg=-60.0),
         "L64": dict(seed=53, ha0_deg=-5.0, N=256, L=64, K=16)}
TOL = {0: 1e-5, 1: 1e-10}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fold_matches_oracle(aidg, orc, name, precision):
    wl = synth.config_tiny(**CASES[name])
    rng = np.random.default_rng(3)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    with plan_for(aidg, wl, precision) as p:
        table = p.subgrids()
        assert table["folded"].sum() > 0
        assert orc.check_partition(wl, table, p.info["w_step"], fold=1) == (0, -1)
        W = p.n_wlayers
        assert np.allclose(p.wlayers()[np.unique(table["wlayer"])], np.unique(table["w0"]))
        G = synth.random_grid(W, wl.grid_size, rng)
        Gg = host(p.grid(dev(V, precision)))
        Vg = host(p.degrid(dev(G, precision)))
    tag = f"fold {name} {'FP64' if precision else 'FP32'} W={W}"
    check_grid(Gg, orc.grid(wl, V, table, W=W), TOL[precision], tag + " grid")
    check_vis(Vg, orc.degrid(wl, G, table), TOL[precision], tag + " degrid")


def lattice(wl, rng, n):
    N, L = wl.grid_size, wl.subgrid_size
    xs = rng.integers(1, L, n).astype(np.int32)
    ys = rng.integers(1, L, n).astype(np.int32)
    return xs, ys, N // 2 + (xs - L // 2) * (N // L), N // 2 + (ys - L // 2) * (N // L)


@pytest.mark.parametrize("name", ["transit", "west"])
def test_fold_image_and_prediction_are_exact_at_lattice_points(aidg, orc, name):
    wl = synth.config_tiny(**CASES[name])
    N, L = wl.grid_size, wl.subgrid_size
    rng = np.random.default_rng(4)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    src = synth.point_sources(4, wl.fov, 0.5, 5.0, rng, L=L, on_lattice=True)
    I = np.zeros((4, N, N), np.complex128)
    for s in range(4):
        I[:, N // 2 + (src["ys"][s] - L // 2) * (N // L), N // 2 + (src["xs"][s] - L // 2) * (N // L)] += src["B"][s]
    with plan_for(aidg, wl) as p:
        img = host(p.invert(p.grid(dev(V, 0))))
        Vp = host(p.degrid(p.predict(dev(I, 0))))
        table = p.subgrids()
    xs, ys, X, Y = lattice(wl, rng, 80)
    l, m = orc.lattice_dirs(wl, xs, ys)
    mask = orc.coverage_mask(wl, table)
    ref = orc.direct_image(wl, V, l, m, xs, ys, mask=mask)
    T = orc.taper(L, wl.kernel_support)[ys, xs]
    check_image(herm_part(img[:, Y, X].T), herm_part(ref), T, 1e-5, f"fold {name} Hermitian image")
    Vd = orc.direct_predict(wl, src["l"], src["m"], src["B"], src["xs"], src["ys"])
    check_vis(Vp[mask.astype(bool)], Vd[mask.astype(bool)], 1e-5, f"fold {name} prediction")
