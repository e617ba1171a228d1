"""Element-wise parity gates shared by the GPU tests.

Every parity check asserts the normwise error of a result AND a per-element bound,
so that one wrong subgrid, visibility or pixel cannot hide inside a large norm:

  grids and images:  ||x - ref|| / ||ref||            <= tol   (normwise)
                     max |x - ref| / max |ref|          <= tol   (worst cell, on the
                                                                  scale of the result)
  visibilities:      ||x - ref|| / ||ref||            <= tol   (normwise)
                     max_k ||dV_k||_F / rms_k ||V_k||_F <= tol   (worst visibility, 4 pols
                                                                  together, on the scale
                                                                  of a typical one)

tol is 1e-5 for the FP32 path and 1e-10 for the FP64 path.  The per-visibility
relative error |dV_k|_F / |V_k|_F (over visibilities with |V_k|_F >= 1e-3 rms) is
printed beside the gates: it is large only where |V_k| itself is small.
"""
from __future__ import annotations

import numpy as np


def _c128(a):
    return np.asarray(a, np.complex128)


def grid_errors(x, ref) -> dict:
    """Normwise and worst-element errors of a grid or image (any shape)."""
    x, ref = _c128(x), _c128(ref)
    assert x.shape == ref.shape, (x.shape, ref.shape)
    d = np.abs(x - ref)
    nr = float(np.linalg.norm(ref.ravel()))
    mr = float(np.abs(ref).max(initial=0.0))
    return {"normwise": float(np.linalg.norm(d.ravel())) / max(nr, 1e-300),
            "max_over_max": float(d.max(initial=0.0)) / max(mr, 1e-300)}


def vis_errors(x, ref) -> dict:
    """Normwise and worst-visibility errors of visibilities [..., 4]."""
    x, ref = _c128(x), _c128(ref)
    assert x.shape == ref.shape and x.shape[-1] == 4, (x.shape, ref.shape)
    nd = np.linalg.norm(x - ref, axis=-1).ravel()
    nr = np.linalg.norm(ref, axis=-1).ravel()
    rms = float(np.sqrt(np.mean(nr * nr))) if nr.size else 0.0
    out = {"normwise": float(np.linalg.norm(nd)) / max(float(np.linalg.norm(nr)), 1e-300),
           "max_over_rms": float(nd.max(initial=0.0)) / max(rms, 1e-300)}
    sel = nr >= 1e-3 * rms
    if sel.any():
        r = nd[sel] / nr[sel]
        out["per_vis_max"] = float(r.max())
        out["per_vis_p99"] = float(np.percentile(r, 99))
    return out


def _fmt(label, e):
    return label + ": " + ", ".join(f"{k} {v:.3e}" for k, v in e.items())


def check_grid(x, ref, tol: float, label: str = "grid") -> dict:
    e = grid_errors(x, ref)
    print(_fmt(label, e), flush=True)
    assert e["normwise"] <= tol, (label, e)
    assert e["max_over_max"] <= tol, (label, e)
    return e


def check_vis(x, ref, tol: float, label: str = "vis") -> dict:
    e = vis_errors(x, ref)
    print(_fmt(label, e), flush=True)
    assert e["normwise"] <= tol, (label, e)
    assert e["max_over_rms"] <= tol, (label, e)
    return e


def check_image(x, ref, T, tol: float, label: str = "image", untapered: bool = False) -> dict:
    """Gate for an image made by the image level (invert), which divides the sum of the
    layers' transforms by the taper T.  That division is exact scaling, but it lifts the
    transform's FP32 rounding by up to 1 / min T at the field's edge, so the element-wise
    gate applies to T x and T ref, the quantity the transform produces (T broadcast over
    the trailing polarisation axis).  The untapered error is printed; untapered=True
    (the FP64 path) gates it too."""
    Tc = np.asarray(T, np.float64)[..., None]
    e = check_grid(_c128(x) * Tc, _c128(ref) * Tc, tol, "T x " + label)
    u = grid_errors(x, ref)
    print(_fmt(label + " (untapered)", u), flush=True)
    if untapered:
        assert u["normwise"] <= tol and u["max_over_max"] <= tol, (label, u)
    return e


def check_inner(lhs: complex, rhs: complex, tol: float, label: str = "adjoint") -> float:
    """Relative residual of an inner-product identity, |lhs - rhs| / |lhs|.  The
    callers pick their inputs so that |lhs| is of the order of the product of the
    norms (for example <grid(V), G> with G = grid(V)), so the gate is not loosened
    by a near-orthogonal pair."""
    r = abs(lhs - rhs) / max(abs(lhs), 1e-300)
    print(f"{label}: |lhs - rhs| / |lhs| {r:.3e} (|lhs| {abs(lhs):.3e})", flush=True)
    assert r <= tol, (label, r)
    return r
