"""Differentiable degrid/grid on the GPU: DegridFn's hand-written backward is the
gridder and GridFn's is the degridder.

Workload: 64 stations (2016 baselines) x 30 x 48 channels (2.9M visibilities),
grid 4096^2 at 15 arcsec, subgrid 64^2, K = 16, random complex grid.  Loss
L = Re sum conj(R) V(G) with complex Gaussian R.  Central finite differences on
the real and imaginary parts of 100 random grid cells (90 inside the footprint
the subgrid windows cover, 10 outside, where the gradient must be exactly zero)
are compared with autograd's gradient (PyTorch convention: dL/dRe + i dL/dIm).
L is linear in G, so the central difference is exact up to the rounding of the
two loss evaluations, an absolute error of about eps |L| / h per probe; it is
therefore measured against the RMS gradient over the probes inside the footprint
(a per-probe relative error would blow up at cells where the taper makes the
gradient tiny).  FP64 path: step h = 1e-3 rms(G), error <= 1e-6 rms(grad) per
probe.  FP32 path: the loss sums 2.9M visibilities whose FP32 rounding (~3e-7
normwise) makes it uncertain by about as much as a 1e-3 rms(G) step changes it,
so the step is h = 10 rms(G) (the step size trades nothing else); gates median
<= 1e-2 and max <= 5e-2 of rms(grad).  The adjoint residual is checked through
autograd as well.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(precision):
    import paper_2502_17789_amd as aidg
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = synth.config_diff(seed=4)
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision)
    cdt = np.complex64 if precision == 0 else np.complex128
    A = torch.from_numpy(wl.aterms.astype(cdt)).cuda()
    return wl, aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, A)


def footprint(plan, N, L):
    cover = np.zeros((N, N), bool)
    t = plan.subgrids()
    for U0, V0 in zip(t["U0"], t["V0"]):
        cover[V0 - L // 2:V0 + L // 2, U0 - L // 2:U0 + L // 2] = True
    return cover


@pytest.mark.parametrize("precision", [1, 0])
def test_degrid_backward_finite_differences(precision):
    from paper_2502_17789_amd.autograd import DegridFn
    wl, plan = make(precision)
    with plan:
        cdt = torch.complex64 if precision == 0 else torch.complex128
        gen = torch.Generator(device="cuda")
        gen.manual_seed(4)
        G = torch.randn(plan.grid_shape(), dtype=cdt, device="cuda", generator=gen)
        R = torch.randn(plan.vis_shape(), dtype=torch.complex128, device="cuda", generator=gen)
        Gv = G.clone().requires_grad_(True)
        V = DegridFn.apply(Gv, plan)
        loss = torch.real(torch.vdot(R.flatten(), V.flatten().to(torch.complex128)))
        loss.backward()
        grad = Gv.grad.detach()

        def L_of(Gp):
            return torch.real(torch.vdot(R.flatten(), plan.degrid(Gp).flatten().to(torch.complex128))).item()

        N, L = wl.grid_size, wl.subgrid_size
        cover = footprint(plan, N, L)
        rng = np.random.default_rng(44)
        inside = np.argwhere(cover)
        outside = np.argwhere(~cover)
        cells = [tuple(inside[i]) for i in rng.choice(len(inside), 90, replace=False)]
        cells += [tuple(outside[i]) for i in rng.choice(len(outside), 10, replace=False)]
        h = (1e-3 if precision == 1 else 10.0) * G.abs().pow(2).mean().sqrt().item()
        errs, outside_fd, inside_g = [], [], []
        for k, (gv, gu) in enumerate(cells):
            pol = int(rng.integers(0, 4))
            idx = (0, pol, int(gv), int(gu))
            g = grad[idx].item()
            orig = G[idx].clone()
            for part, unit in (("re", 1.0), ("im", 1j)):
                G[idx] = orig + unit * h
                Lp = L_of(G)
                G[idx] = orig - unit * h
                Lm = L_of(G)
                G[idx] = orig
                fd = (Lp - Lm) / (2 * h)
                ref = g.real if part == "re" else g.imag
                if k >= 90:
                    # no subgrid window covers the cell: the gradient is exactly zero and the
                    # difference is only the (order-dependent) rounding of the two degrids
                    assert ref == 0.0, (idx, part, ref)
                    outside_fd.append(abs(fd))
                else:
                    inside_g.append(abs(ref))
                    errs.append(abs(fd - ref))
        scale = float(np.sqrt(np.mean(np.square(inside_g))))
        assert max(outside_fd) <= (1e-8 if precision == 1 else 5e-2) * scale
        errs = np.array(errs) / scale
        print(f"precision {precision}: FD vs autograd median {np.median(errs):.3e} max {errs.max():.3e}",
              flush=True)
        if precision == 1:
            assert errs.max() <= 1e-6
        else:
            assert np.median(errs) <= 1e-2 and errs.max() <= 5e-2


@pytest.mark.parametrize("precision", [0, 1])
def test_autograd_adjoint_residuals(precision):
    """Directional derivatives through autograd: <dL/dG, dG> = Re<R, degrid(dG)> and
    <dL/dV, dV> = Re<Q, grid(dV)>, i.e. each backward is the adjoint of its forward."""
    from paper_2502_17789_amd.autograd import DegridFn, GridFn
    wl, plan = make(precision)
    with plan:
        cdt = torch.complex64 if precision == 0 else torch.complex128
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        G = torch.randn(plan.grid_shape(), dtype=cdt, device="cuda", generator=gen).requires_grad_(True)
        R = torch.randn(plan.vis_shape(), dtype=cdt, device="cuda", generator=gen)
        dG = torch.randn(plan.grid_shape(), dtype=cdt, device="cuda", generator=gen)
        torch.real(torch.vdot(R.flatten(), DegridFn.apply(G, plan).flatten())).backward()
        lhs = torch.real(torch.vdot(G.grad.flatten().to(torch.complex128), dG.flatten().to(torch.complex128)))
        rhs = torch.real(torch.vdot(R.flatten().to(torch.complex128),
                                    plan.degrid(dG).flatten().to(torch.complex128)))
        scale = (G.grad.to(torch.complex128).norm() * dG.to(torch.complex128).norm()).item()
        r1 = abs((lhs - rhs).item()) / scale

        V = torch.randn(plan.vis_shape(), dtype=cdt, device="cuda", generator=gen).requires_grad_(True)
        Q = torch.randn(plan.grid_shape(), dtype=cdt, device="cuda", generator=gen)
        dV = torch.randn(plan.vis_shape(), dtype=cdt, device="cuda", generator=gen)
        torch.real(torch.vdot(Q.flatten(), GridFn.apply(V, plan).flatten())).backward()
        lhs2 = torch.real(torch.vdot(V.grad.flatten().to(torch.complex128), dV.flatten().to(torch.complex128)))
        rhs2 = torch.real(torch.vdot(Q.flatten().to(torch.complex128),
                                     plan.grid(dV).flatten().to(torch.complex128)))
        scale2 = (V.grad.to(torch.complex128).norm() * dV.to(torch.complex128).norm()).item()
        r2 = abs((lhs2 - rhs2).item()) / scale2
        tol = 1e-5 if precision == 0 else 1e-12
        print(f"precision {precision}: adjoint residuals degrid {r1:.3e}, grid {r2:.3e}", flush=True)
        assert r1 <= tol and r2 <= tol
