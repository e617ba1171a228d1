"""GPU parity of the image-level step (w-stacking, Eq. wstack; its inverse for
prediction, Eq. wunstack) through the C ABI, against the FP64 oracle.

Bar (normwise relative error per result): FP32 <= 1e-5, FP64 <= 1e-10.
  * aidg_invert / aidg_predict against oracle.invert / oracle.predict on random
    grids and images, over N whose FFTs take every radix (4, 2, 3, 5) and several
    w-layers;
  * the adjoint identity <invert(G), I> = <G, predict(I)> on GPU outputs;
  * end to end through the library's own partition: invert(grid(V)) at subgrid-
    lattice pixels equals the direct A-term image of the gridded visibilities, and
    degrid(predict(I)) of point sources on lattice pixels equals their direct
    prediction (Eq. 1);
  * an N whose row FFT the library does not implement is refused.
"""
import numpy as np
import pytest

import synth
from gates import check_grid, check_image, check_inner, check_vis

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


def plan_for(aidg, wl, precision=0, w_step=0.0):
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision, w_step=w_step)
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, dev(wl.aterms, precision))


# N = 128: radices 4 4 4 2; N = 480: 4 4 2 3 5; N = 250: 2 5 5 5; N = 384: 4 4 4 2 3
CASES = {
    "N128": dict(seed=201, N=128, L=32, K=8, w_step=12.0),
    "N480": dict(seed=202, N=480, L=32, K=8, w_step=15.0),
    "N250": dict(seed=203, N=250, L=32, K=8, fov_deg=12.0, w_step=6.0),
    "N384": dict(seed=204, N=384, L=96, K=24, n_c=12, fov_deg=12.0, diameter_m=1500.0, w_step=0.0),
}
TOL = {0: 1e-5, 1: 1e-10}


def case(name):
    c = dict(CASES[name])
    w_step = c.pop("w_step")
    return synth.config_tiny(**c), w_step


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_invert_and_predict_match_oracle(aidg, orc, name, precision):
    wl, w_step = case(name)
    with plan_for(aidg, wl, precision, w_step) as p:
        w0 = p.wlayers()
        rng = np.random.default_rng(7)
        N, L, K = wl.grid_size, wl.subgrid_size, wl.kernel_support
        G = synth.random_grid(p.n_wlayers, N, rng)
        I = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
        Ig = host(p.invert(dev(G, precision)))
        Gg = host(p.predict(dev(I, precision)))
        tag = f"{name} {'FP64' if precision else 'FP32'} W={p.n_wlayers}"
        check_grid(Ig, orc.invert(G, w0, L, K, wl.pixel_scale), TOL[precision], tag + " invert")
        check_grid(Gg, orc.predict(I, w0, L, K, wl.pixel_scale), TOL[precision], tag + " predict")


@pytest.mark.parametrize("precision", [0, 1])
def test_image_adjoint_identity_on_gpu(aidg, precision):
    wl, w_step = case("N480")
    with plan_for(aidg, wl, precision, w_step) as p:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(3)
        dt = torch.complex64 if precision == 0 else torch.complex128
        G = torch.randn(p.grid_shape(), dtype=dt, device="cuda", generator=gen)
        # I = invert(G): then <invert(G), I> = ||invert(G)||^2 and the relative residual
        # measures the mismatch of the pair itself
        I = p.invert(G)
        GI = p.predict(I)
        torch.cuda.synchronize()
        c = torch.complex128
        lhs = torch.vdot(I.flatten().to(c), I.flatten().to(c)).item()
        rhs = torch.vdot(G.flatten().to(c), GI.flatten().to(c)).item()
        check_inner(lhs, rhs, TOL[precision], f"{'FP64' if precision else 'FP32'} image adjoint")


def lattice_pixels(wl, rng, n):
    N, L = wl.grid_size, wl.subgrid_size
    xs = rng.integers(1, L, n).astype(np.int32)
    ys = rng.integers(1, L, n).astype(np.int32)
    return xs, ys, N // 2 + (xs - L // 2) * (N // L), N // 2 + (ys - L // 2) * (N // L)


@pytest.mark.parametrize("precision", [0, 1])
def test_invert_of_gridded_visibilities_is_the_direct_image(aidg, orc, precision):
    wl, w_step = case("N480")
    rng = np.random.default_rng(11)
    V = synth.random_vis((wl.n_baselines, wl.n_times, wl.n_chans), rng)
    with plan_for(aidg, wl, precision, w_step) as p:
        assert p.n_wlayers >= 2
        I = host(p.invert(p.grid(dev(V, precision))))
        table = p.subgrids()
    xs, ys, X, Y = lattice_pixels(wl, rng, 80)
    l, m = orc.lattice_dirs(wl, xs, ys)
    ref = orc.direct_image(wl, V, l, m, xs, ys, mask=orc.coverage_mask(wl, table))
    check_image(I[:, Y, X].T, ref, orc.taper(wl.subgrid_size, wl.kernel_support)[ys, xs], TOL[precision],
                "invert(grid(V)) at lattice pixels vs direct image", untapered=precision == 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_degrid_of_predicted_lattice_sources_is_the_direct_prediction(aidg, orc, precision):
    wl, w_step = case("N480")
    N, L = wl.grid_size, wl.subgrid_size
    rng = np.random.default_rng(12)
    src = synth.point_sources(5, wl.fov, 0.5, 5.0, rng, L=L, on_lattice=True)
    I = np.zeros((4, N, N), np.complex128)
    for s in range(5):
        I[:, N // 2 + (src["ys"][s] - L // 2) * (N // L), N // 2 + (src["xs"][s] - L // 2) * (N // L)] += src["B"][s]
    with plan_for(aidg, wl, precision, w_step) as p:
        V = host(p.degrid(p.predict(dev(I, precision))))
        table = p.subgrids()
    Vd = orc.direct_predict(wl, src["l"], src["m"], src["B"], src["xs"], src["ys"])
    mask = orc.coverage_mask(wl, table).astype(bool)
    assert mask.sum() > 0.8 * mask.size
    check_vis(V[mask], Vd[mask], TOL[precision], "degrid(predict(I)) vs direct prediction")


def test_unsupported_image_size_is_refused(aidg):
    wl = synth.config_tiny(205, N=126, L=32, K=8)  # 126 = 2 x 3^2 x 7
    with plan_for(aidg, wl) as p:
        G = torch.zeros(p.grid_shape(), dtype=torch.complex64, device="cuda")
        with pytest.raises(RuntimeError, match="2\\^a 3\\^b 5\\^c"):
            p.invert(G)


@pytest.mark.parametrize("precision", [1, 0])
def test_image_to_visibilities_gradient(aidg, precision):
    """Loss Re sum conj(R) degrid(predict(I)) through autograd (backward: grid, then
    invert) against central finite differences at 40 image pixels of the inner half
    of the field.  The loss is linear in I, so the difference has no truncation
    error and a large step (1e3 against unit-variance pixels) keeps the rounding of
    the two loss evaluations small beside the change; errors are measured against
    the RMS gradient over the probes.  FP64: bound 1e-6; FP32: median <= 1e-2,
    max <= 5e-2."""
    from paper_2502_17789_amd import autograd
    wl, w_step = case("N480")
    N = wl.grid_size
    dt = torch.complex64 if precision == 0 else torch.complex128
    with plan_for(aidg, wl, precision, w_step) as p:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        I = torch.randn(p.image_shape(), dtype=dt, device="cuda", generator=gen).requires_grad_(True)
        Rv = torch.randn(p.vis_shape(), dtype=dt, device="cuda", generator=gen)

        def loss(img):
            return torch.real(torch.vdot(Rv.flatten(), autograd.predict_vis(img, p).flatten())).to(torch.float64)

        L0 = loss(I)
        L0.backward()
        grad = I.grad.detach().clone()
        rng = np.random.default_rng(6)
        probes = [(int(rng.integers(4)), int(rng.integers(N // 4, 3 * N // 4)), int(rng.integers(N // 4, 3 * N // 4)))
                  for _ in range(40)]
        h = 1e3
        errs, gs = [], []
        with torch.no_grad():
            for pol, y, x in probes:
                fd = []
                for unit in (1.0, 1.0j):
                    Ip = I.detach().clone()
                    Im = I.detach().clone()
                    Ip[pol, y, x] += h * unit
                    Im[pol, y, x] -= h * unit
                    fd.append((loss(Ip) - loss(Im)).item() / (2 * h))
                g = complex(grad[pol, y, x].item())
                errs.append(abs(complex(fd[0], fd[1]) - g))
                gs.append(abs(g))
        rms = float(np.sqrt(np.mean(np.square(gs))))
        e = np.array(errs) / rms
        print(f"{'FP64' if precision else 'FP32'} image->vis gradient: max {e.max():.2e} median {np.median(e):.2e}",
              flush=True)
        if precision:
            assert e.max() <= 1e-6
        else:
            assert np.median(e) <= 1e-2 and e.max() <= 5e-2


def test_invert_autograd_is_the_adjoint(aidg):
    """<invert(G), J> through autograd: its gradient with respect to G is predict(J)."""
    from paper_2502_17789_amd import autograd
    wl, w_step = case("N128")
    with plan_for(aidg, wl, 1, w_step) as p:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(8)
        G = torch.randn(p.grid_shape(), dtype=torch.complex128, device="cuda", generator=gen).requires_grad_(True)
        J = torch.randn(p.image_shape(), dtype=torch.complex128, device="cuda", generator=gen)
        torch.real(torch.vdot(J.flatten(), autograd.invert(G, p).flatten())).backward()
        ref = p.predict(J)
        assert rel(host(G.grad), host(ref)) <= 1e-12


def test_invert_at_the_largest_row_size(aidg, orc):
    """N = 8192 in FP32: a row fills exactly 64 KB of LDS, 7 passes (radix 4^6 and 2).
    One polarisation (all the plan's w-layers) against the oracle's FP64 transform."""
    wl = synth.config_tiny(206, N=8192, L=32, K=8, fov_deg=20.0)
    with plan_for(aidg, wl) as p:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(9)
        G = torch.randn(p.grid_shape(), dtype=torch.complex64, device="cuda", generator=gen)
        I = p.invert(G)
        torch.cuda.synchronize()
        Ih = I[2].cpu().numpy().astype(np.complex128)
        del I
        ref = orc.invert(G[:, 2:3].cpu().numpy().astype(np.complex128), p.wlayers(),
                         wl.subgrid_size, wl.kernel_support, wl.pixel_scale)[0]
        check_grid(Ih, ref, TOL[0], f"N=8192 invert, W={p.n_wlayers}, one polarisation")


def test_fp64_rows_beyond_64_kb_are_refused(aidg):
    """FP64 at N = 8000: a row of complex128 values would take 125 KB of LDS."""
    wl = synth.config_tiny(207, N=8000, L=32, K=8, fov_deg=20.0)
    with plan_for(aidg, wl, precision=1) as p:
        with pytest.raises(RuntimeError, match="64 KB"):
            p._image_workspace(torch.device("cuda"))
