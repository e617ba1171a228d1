"""FP64 CPU oracle for A-term IDG gridding/degridding -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and the
two share no code: this wrapper drives ``oracle.cpp`` (plain C++17, double
precision, OpenMP over subgrids or directions) through ctypes on numpy arrays.

Pins (tests/test_oracle_*.py) tie every function here to something other than
itself: lattice identities against the brute-force direct DFT, a Dirichlet
closed form, numpy FFTs and scipy's Bessel function for special cases, and the
adjoint identity between gridding and degridding.

The image-level step (w-stacking, ``invert`` / ``predict``) is plain numpy in
FP64 on top of numpy's FFT; it is pinned by a brute-force DFT matrix, the adjoint
identity, and the direct imaging and prediction equations at the subgrid lattice.

Stokes-I grids (one complex value per cell, I = (XX + YY) / 2) are defined on top of
the 4-polarisation functions, and pinned by the direct image and prediction of
unpolarised lattice sources and by their adjoint relation.

The inverse A-term mode (Sec. 3.3: gridding with A_p^-1 . A_q^-H normalised by
||A_p^-1 A_q^-H||_F, the image divided by the weighted average of that factor) is
pinned by unitary Jones terms (where it is the adjoint mode over sqrt 2), a closed
form for diagonal Jones terms, and exact recovery of a lattice source's brightness.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

SUBGRID_DTYPE = np.dtype([
    ("bl", "<i4"), ("st1", "<i4"), ("st2", "<i4"), ("t0", "<i4"), ("nt", "<i4"),
    ("c0", "<i4"), ("nc", "<i4"), ("U0", "<i4"), ("V0", "<i4"), ("wlayer", "<i4"),
    ("aint", "<i4"), ("folded", "<i4"), ("w0", "<f8"), ("vis_offset", "<i8")])
assert SUBGRID_DTYPE.itemsize == 64

CHECK_CODES = {
    0: "ok", 1: "bad baseline/stations", 2: "sub-table outside table", 3: "A-term interval",
    4: "window off grid", 5: "uv beyond (L-K)/2", 6: "w beyond layer", 7: "visibility twice",
    8: "placeable visibility missing", 9: "inconsistent layer w0", 10: "vis_offset",
    11: "fold flag",
}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so (g++, -O2, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = ctypes.CDLL(LIB)
        _lib.oracle_partition.restype = ctypes.c_int64
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _geo(wl):
    return [ctypes.c_int(wl.grid_size), ctypes.c_int(wl.subgrid_size),
            ctypes.c_int(wl.kernel_support), ctypes.c_double(wl.pixel_scale)]


def _obs(wl):
    return [ctypes.c_int(wl.n_stations), ctypes.c_int(wl.n_baselines), ctypes.c_int(wl.n_times),
            ctypes.c_int(wl.n_chans), ctypes.c_int(wl.aterm_interval)]


def _arrs(wl):
    bl = np.ascontiguousarray(wl.baselines, np.int32)
    uvw = np.ascontiguousarray(wl.uvw, np.float64)
    f = np.ascontiguousarray(wl.freqs, np.float64)
    return bl, uvw, f


def taper(L: int, K: int, beta: float = 0.0) -> np.ndarray:
    T = np.zeros((L, L))
    lib().oracle_taper(ctypes.c_int(L), ctypes.c_int(K), ctypes.c_double(beta), _p(T))
    return T


def partition(wl, w_step: float, fold: int = 0) -> np.ndarray:
    bl, uvw, f = _arrs(wl)
    cap = max(1024, wl.n_vis)
    out = np.zeros(cap, SUBGRID_DTYPE)
    n = lib().oracle_partition(*_geo(wl), *_obs(wl), _p(bl), _p(uvw), _p(f),
                               ctypes.c_double(w_step), ctypes.c_int(fold), _p(out), ctypes.c_int64(cap))
    assert n >= 0
    return out[:n].copy()


def check_partition(wl, table: np.ndarray, w_step: float, fold: int = 0) -> tuple[int, int]:
    bl, uvw, f = _arrs(wl)
    table = np.ascontiguousarray(table, SUBGRID_DTYPE)
    bad = ctypes.c_int64(0)
    code = lib().oracle_check_partition(*_geo(wl), *_obs(wl), _p(bl), _p(uvw), _p(f),
                                        ctypes.c_double(w_step), ctypes.c_int(fold), _p(table),
                                        ctypes.c_int64(table.shape[0]), ctypes.byref(bad))
    return int(code), int(bad.value)


def n_layers(table: np.ndarray) -> int:
    return int(table["wlayer"].max()) + 1 if table.shape[0] else 1


def layer_w(table: np.ndarray) -> np.ndarray:
    W = n_layers(table)
    w = np.zeros(W)
    for j in range(W):
        sel = table["wlayer"] == j
        if sel.any():
            w[j] = table["w0"][sel][0]
    return w


def grid_subgrid(wl, vis: np.ndarray, sg, stage: int, beta: float = 0.0,
                 aterm_mode: int = 0) -> np.ndarray:
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    vis = _c128(vis)
    sgr = np.ascontiguousarray(np.asarray(sg, SUBGRID_DTYPE).reshape(1))
    L = wl.subgrid_size
    out = np.zeros((4, L, L), np.complex128)
    lib().oracle_grid_subgrid(*_geo(wl), ctypes.c_double(beta), *_obs(wl),
                              ctypes.c_int(A.shape[0]), _p(bl), _p(uvw), _p(f), _p(A), _p(vis),
                              _p(sgr), ctypes.c_int(stage), ctypes.c_int(aterm_mode), _p(out))
    return out


def grid(wl, vis: np.ndarray, table: np.ndarray, W: int | None = None, beta: float = 0.0,
         nthreads: int = 0, out: np.ndarray | None = None, aterm_mode: int = 0) -> np.ndarray:
    """Gridding; aterm_mode 0 applies A_p^H . A_q, 1 the normalised inverse
    A_p^-1 . A_q^-H / ||A_p^-1 A_q^-H||_F of Sec. 3.3."""
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    vis = _c128(vis)
    table = np.ascontiguousarray(table, SUBGRID_DTYPE)
    W = n_layers(table) if W is None else W
    N = wl.grid_size
    G = np.zeros((W, 4, N, N), np.complex128) if out is None else out
    rc = lib().oracle_grid(*_geo(wl), ctypes.c_double(beta), *_obs(wl), ctypes.c_int(A.shape[0]),
                           _p(bl), _p(uvw), _p(f), _p(A), _p(vis), _p(table),
                           ctypes.c_int64(table.shape[0]), ctypes.c_int(W), _p(G),
                           ctypes.c_int(nthreads), ctypes.c_int(aterm_mode))
    assert rc == 0
    return G


def stokes_i_reduce(G: np.ndarray) -> np.ndarray:
    """Stokes-I grid of a 4-polarisation grid (Sec. 5.5: one complex value per pixel for
    Stokes I): I = (XX + YY) / 2.  [W][4][N][N] -> [W][1][N][N]."""
    G = np.asarray(G)
    return 0.5 * (G[:, 0:1] + G[:, 3:4])


def stokes_i_expand(GI: np.ndarray) -> np.ndarray:
    """The 4-polarisation grid of an unpolarised brightness B = I [[1, 0], [0, 1]]:
    XX = YY = I, XY = YX = 0.  [W][1][N][N] -> [W][4][N][N]."""
    GI = np.asarray(GI, np.complex128)
    z = np.zeros_like(GI)
    return np.concatenate([GI, z, z, GI], axis=1)


def grid_stokes_i(wl, vis: np.ndarray, table: np.ndarray, W: int | None = None, beta: float = 0.0,
                  nthreads: int = 0, aterm_mode: int = 0) -> np.ndarray:
    """Gridding onto a Stokes-I grid: the Stokes-I part of the A-term-corrected 4-pol grid."""
    return stokes_i_reduce(grid(wl, vis, table, W=W, beta=beta, nthreads=nthreads, aterm_mode=aterm_mode))


def degrid_stokes_i(wl, GI: np.ndarray, table: np.ndarray, beta: float = 0.0, nthreads: int = 0) -> np.ndarray:
    """Degridding from a Stokes-I grid: the 4-pol visibilities of the unpolarised grid."""
    return degrid(wl, stokes_i_expand(GI), table, beta=beta, nthreads=nthreads)


def aterm_norm(wl, table: np.ndarray) -> np.ndarray:
    """Weighted average over the table's subgrids (weights: visibility counts) of the
    inverse mode's normalisation factor 1 / ||A_p^-1 A_q^-H||_F (Sec. 3.3), on the
    L x L subgrid lattice [y][x]."""
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    table = np.ascontiguousarray(table, SUBGRID_DTYPE)
    L = wl.subgrid_size
    out = np.zeros((L, L))
    lib().oracle_aterm_norm(ctypes.c_int(wl.grid_size), ctypes.c_int(L), ctypes.c_double(wl.pixel_scale),
                            *_obs(wl), ctypes.c_int(A.shape[0]), _p(bl), _p(uvw), _p(f), _p(A),
                            _p(table), ctypes.c_int64(table.shape[0]), _p(out))
    return out


def degrid(wl, G: np.ndarray, table: np.ndarray, beta: float = 0.0, nthreads: int = 0) -> np.ndarray:
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    G = _c128(G)
    table = np.ascontiguousarray(table, SUBGRID_DTYPE)
    V = np.zeros((wl.n_baselines, wl.n_times, wl.n_chans, 4), np.complex128)
    rc = lib().oracle_degrid(*_geo(wl), ctypes.c_double(beta), *_obs(wl), ctypes.c_int(A.shape[0]),
                             _p(bl), _p(uvw), _p(f), _p(A), _p(G), _p(table),
                             ctypes.c_int64(table.shape[0]), ctypes.c_int(G.shape[0]), _p(V),
                             ctypes.c_int(nthreads))
    assert rc == 0
    return V


def direct_image(wl, vis: np.ndarray, l, m, xs=None, ys=None, mask=None, nthreads: int = 0) -> np.ndarray:
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    vis = _c128(vis)
    l = np.ascontiguousarray(l, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    n = l.shape[0]
    xs = -np.ones(n, np.int32) if xs is None else np.ascontiguousarray(xs, np.int32)
    ys = -np.ones(n, np.int32) if ys is None else np.ascontiguousarray(ys, np.int32)
    mk = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    out = np.zeros((n, 4), np.complex128)
    lib().oracle_direct_image(ctypes.c_int(wl.grid_size), ctypes.c_int(wl.subgrid_size),
                              ctypes.c_double(wl.pixel_scale), *_obs(wl), ctypes.c_int(A.shape[0]),
                              _p(bl), _p(uvw), _p(f), _p(A), _p(vis),
                              None if mk is None else _p(mk), ctypes.c_int(n), _p(l), _p(m),
                              _p(xs), _p(ys), _p(out), ctypes.c_int(nthreads))
    return out


def direct_predict(wl, l, m, B, xs=None, ys=None, nthreads: int = 0) -> np.ndarray:
    bl, uvw, f = _arrs(wl)
    A = _c128(wl.aterms)
    l = np.ascontiguousarray(l, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    n = l.shape[0]
    xs = -np.ones(n, np.int32) if xs is None else np.ascontiguousarray(xs, np.int32)
    ys = -np.ones(n, np.int32) if ys is None else np.ascontiguousarray(ys, np.int32)
    B = _c128(B)
    V = np.zeros((wl.n_baselines, wl.n_times, wl.n_chans, 4), np.complex128)
    lib().oracle_direct_predict(ctypes.c_int(wl.grid_size), ctypes.c_int(wl.subgrid_size),
                                ctypes.c_double(wl.pixel_scale), *_obs(wl),
                                ctypes.c_int(A.shape[0]), _p(bl), _p(uvw), _p(f), _p(A),
                                ctypes.c_int(n), _p(l), _p(m), _p(xs), _p(ys), _p(B), _p(V),
                                ctypes.c_int(nthreads))
    return V


def layer_image_at(G_layer: np.ndarray, du: float, l, m, nthreads: int = 0) -> np.ndarray:
    G = _c128(G_layer)
    P, N = G.shape[0], G.shape[-1]
    l = np.ascontiguousarray(l, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    out = np.zeros((l.shape[0], P), np.complex128)
    lib().oracle_layer_image_at(_p(G), ctypes.c_int(P), ctypes.c_int(N), ctypes.c_double(du),
                                ctypes.c_int(l.shape[0]), _p(l), _p(m), _p(out), ctypes.c_int(nthreads))
    return out


def coverage_mask(wl, table: np.ndarray) -> np.ndarray:
    """1 for visibilities that belong to a subgrid of the table, else 0."""
    mask = np.zeros((wl.n_baselines, wl.n_times, wl.n_chans), np.uint8)
    for s in table:
        mask[s["bl"], s["t0"]:s["t0"] + s["nt"], s["c0"]:s["c0"] + s["nc"]] = 1
    return mask


def lattice_dirs(wl, xs, ys):
    """Direction cosines of subgrid-lattice pixels (xs, ys)."""
    L = wl.subgrid_size
    step = wl.fov / L
    xs = np.asarray(xs, np.int32)
    ys = np.asarray(ys, np.int32)
    return (xs - L // 2) * step, (ys - L // 2) * step


# ------------------------------------------------------------------ image level (w-stacking)


def image_taper(N: int, K: int, beta: float = 0.0) -> np.ndarray:
    """The Kaiser-Bessel taper of Sec. 4.2 at image resolution, one axis:
    t[X] = I0(beta sqrt(1 - (2 f)^2)) / I0(beta), f = (X - N/2) / N, beta = pi K / 4
    unless given.  The subgrid taper samples the same function at L points."""
    beta = beta if beta > 0 else math.pi * K / 4
    f = (np.arange(N) - N // 2) / N
    return np.i0(beta * np.sqrt(1.0 - (2.0 * f) ** 2)) / np.i0(beta)


def image_n1(N: int, dl: float) -> np.ndarray:
    """n - 1 = sqrt(1 - l^2 - m^2) - 1 at image pixel [Y][X], l = (X - N/2) dl,
    m = (Y - N/2) dl, in the cancellation-free form -r^2 / (1 + sqrt(1 - r^2))."""
    x = (np.arange(N) - N // 2) * dl
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def centred_dft2(a: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised centred DFT over the last two axes (Sec. 2.3):
    out[k1, k2] = sum_{x1, x2} a[x1, x2] exp(sign 2 pi i [(k1 - N/2)(x1 - N/2)
    + (k2 - N/2)(x2 - N/2)] / N), by numpy's FFT with the centre moved to index 0."""
    N = a.shape[-1]
    s = np.fft.ifftshift(a, axes=(-2, -1))
    t = np.fft.ifft2(s) * (N * N) if sign > 0 else np.fft.fft2(s)
    return np.fft.fftshift(t, axes=(-2, -1))


def lattice_to_image(M: np.ndarray, N: int) -> np.ndarray:
    """Bilinear interpolation of an L x L subgrid-lattice map [y][x] at the N x N image
    pixels, periodic over the field of view.  Image pixel X sits at lattice coordinate
    g = (X - N/2) L / N + L/2; the value mixes lattice points floor(g) and floor(g) + 1
    (mod L) with weights 1 - frac(g) and frac(g), per axis."""
    L = M.shape[-1]
    g = (np.arange(N) - N // 2) * (L / N) + L // 2
    i0 = np.floor(g).astype(np.int64)
    fr = g - i0
    i0 %= L
    i1 = (i0 + 1) % L
    rows = M[i0, :] * (1 - fr)[:, None] + M[i1, :] * fr[:, None]   # [Y][x]
    return rows[:, i0] * (1 - fr)[None, :] + rows[:, i1] * fr[None, :]


def invert(G: np.ndarray, w0, L: int, K: int, dl: float, beta: float = 0.0,
           norm: np.ndarray | None = None) -> np.ndarray:
    """Imaging by w-stacking (Sec. 2.4, Eq. wstack; Sec. 2.5 imaging step 3):
    I[p][Y][X] = 1 / (L^2 T(X, Y)) sum_w exp(+2 pi i w0_w n1(X, Y)) F+{G_w[p]}(Y, X),
    F+ the centred transform with exp(+2 pi i (u l + v m)) over (gv, gu).  The 1/L^2
    undoes the unnormalised subgrid transforms, so that at subgrid-lattice pixels the
    image of gridded visibilities is the direct A-term image.  G: [W][P][N][N].

    ``norm`` (the inverse A-term mode, Sec. 3.3): the L x L weighted-average
    normalisation map of ``aterm_norm``; the image is divided by its bilinear
    interpolation at every pixel, and set to 0 where that is 0."""
    G = np.asarray(G)
    N = G.shape[-1]
    t = image_taper(N, K, beta)
    n1 = image_n1(N, dl)
    out = np.zeros(G.shape[1:], np.complex128)
    for j in range(G.shape[0]):
        out += centred_dft2(G[j].astype(np.complex128), +1) * np.exp(2j * np.pi * w0[j] * n1)
    out = out / (L * L * np.outer(t, t))
    if norm is not None:
        c = lattice_to_image(np.asarray(norm, np.float64), N)
        out = np.where(c > 0, out / np.where(c > 0, c, 1.0), 0.0)
    return out


def predict(I: np.ndarray, w0, L: int, K: int, dl: float, beta: float = 0.0) -> np.ndarray:
    """Inverse w-stacking for prediction (Sec. 2.5 prediction step 2, Eq. wunstack),
    taken as the exact adjoint of ``invert`` (the degridder multiplies by T, so the
    image is divided by it here): G_w[p] = F-{ I[p] exp(-2 pi i w0_w n1) / (L^2 T) }.
    I: [P][N][N]; returns [W][P][N][N]."""
    I = np.asarray(I, np.complex128)
    N = I.shape[-1]
    t = image_taper(N, K, beta)
    n1 = image_n1(N, dl)
    base = I / (L * L * np.outer(t, t))
    return np.stack([centred_dft2(base * np.exp(-2j * np.pi * w * n1), -1) for w in w0])
