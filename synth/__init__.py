"""Seeded synthetic inputs for A-term image-domain gridding.

This module makes the *inputs* of the gridding and degridding operations:
station layouts, earth-rotation uvw tracks, channel frequencies, point-source
skies and per-station 2x2 Jones A-terms sampled on the subgrid lattice.  It
holds none of the gridding or degridding arithmetic itself; both the FP64
oracle (tests) and the HIP library (tests, bench) consume what it returns.

Shapes follow the paper's MWA-like workloads (Sec. 4 footnote, Sec. 6): a
disc of stations at latitude -26.7 deg, a phase centre at declination -27 deg
observed around transit, 2 s timesteps, 4-pol (XX, XY, YX, YY) visibilities.
The paper's MWA observations, beam model and sky catalogue are not available;
these generators stand in for them.

Layouts (all C-contiguous numpy arrays):
  baselines  int32   [nbl][2]            station pair (p, q), p < q
  uvw        float64 [nbl][nt][3]        metres
  freqs      float64 [nc]                Hz, increasing
  aterms     complex128 [n_int][n_st][L][L][4]   Jones (row-major 2x2) per
             A-term interval, station and subgrid-lattice pixel [y][x]
  vis        complex128 [nbl][nt][nc][4]
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SPEED_OF_LIGHT = 299792458.0
EARTH_ROTATION_RAD_S = 7.2921159e-5
ARCSEC = math.pi / (180.0 * 3600.0)


@dataclasses.dataclass
class Workload:
    """One synthetic observation plus the imaging geometry it is gridded with."""

    name: str
    n_stations: int
    baselines: np.ndarray
    uvw: np.ndarray
    freqs: np.ndarray
    grid_size: int
    subgrid_size: int
    kernel_support: int
    pixel_scale: float
    aterm_interval: int
    aterms: np.ndarray
    w_step: float = 0.0
    taper_beta: float = 0.0
    vis: np.ndarray | None = None
    sources: dict | None = None

    @property
    def n_baselines(self) -> int:
        return int(self.baselines.shape[0])

    @property
    def n_times(self) -> int:
        return int(self.uvw.shape[1])

    @property
    def n_chans(self) -> int:
        return int(self.freqs.shape[0])

    @property
    def n_vis(self) -> int:
        return self.n_baselines * self.n_times * self.n_chans

    @property
    def n_intervals(self) -> int:
        return int(self.aterms.shape[0])

    @property
    def fov(self) -> float:
        return self.grid_size * self.pixel_scale


# ---------------------------------------------------------------- geometry


def station_disc(n_st: int, diameter_m: float, rng: np.random.Generator) -> np.ndarray:
    """Stations uniform in a disc of the given diameter; ENU metres [n_st][3]."""
    r = 0.5 * diameter_m * np.sqrt(rng.random(n_st))
    th = 2.0 * math.pi * rng.random(n_st)
    enu = np.zeros((n_st, 3))
    enu[:, 0] = r * np.cos(th)
    enu[:, 1] = r * np.sin(th)
    return enu


def all_pairs(n_st: int) -> np.ndarray:
    p, q = np.triu_indices(n_st, k=1)
    return np.stack([p, q], axis=1).astype(np.int32)


def earth_rotation_uvw(enu: np.ndarray, baselines: np.ndarray, lat_rad: float,
                       dec_rad: float, hour_angles: np.ndarray) -> np.ndarray:
    """uvw [nbl][nt][3] in metres for baseline vector x_q - x_p.

    Standard local-ENU -> equatorial XYZ -> (u, v, w) rotation for a source at
    hour angle H and declination dec (Thompson, Moran & Swenson, Ch. 4).
    """
    e, n, u_ = enu[:, 0], enu[:, 1], enu[:, 2]
    sl, cl = math.sin(lat_rad), math.cos(lat_rad)
    X = -sl * n + cl * u_
    Y = e
    Z = cl * n + sl * u_
    bx = X[baselines[:, 1]] - X[baselines[:, 0]]
    by = Y[baselines[:, 1]] - Y[baselines[:, 0]]
    bz = Z[baselines[:, 1]] - Z[baselines[:, 0]]
    sh, ch = np.sin(hour_angles)[None, :], np.cos(hour_angles)[None, :]
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    bx, by, bz = bx[:, None], by[:, None], bz[:, None]
    uu = sh * bx + ch * by
    vv = -sd * ch * bx + sd * sh * by + cd * bz
    ww = cd * ch * bx - cd * sh * by + sd * bz
    return np.ascontiguousarray(np.stack([uu, vv, ww], axis=-1))


def transit_hour_angles(n_t: int, dt_s: float, ha0_rad: float = 0.0) -> np.ndarray:
    t = (np.arange(n_t) - 0.5 * (n_t - 1)) * dt_s
    return ha0_rad + t * EARTH_ROTATION_RAD_S


def channel_centres(f_lo: float, f_hi: float, n_c: int) -> np.ndarray:
    return f_lo + (np.arange(n_c) + 0.5) * (f_hi - f_lo) / n_c


# ---------------------------------------------------------------- A-terms


def lattice_lm(L: int, fov: float) -> tuple[np.ndarray, np.ndarray]:
    """Direction cosines of the L x L subgrid lattice, [y][x] arrays."""
    c = (np.arange(L) - L // 2) * (fov / L)
    l, m = np.meshgrid(c, c, indexing="xy")
    return l, m


def white_screen(coarse: int, rms: float, rng: np.random.Generator) -> np.ndarray:
    s = rng.standard_normal((coarse, coarse))
    s -= s.mean()
    return s * (rms / max(s.std(), 1e-30))


def kolmogorov_screen(coarse: int, rms: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random field with a k^(-11/3) power spectrum, scaled to rms."""
    k = np.fft.fftfreq(coarse)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    kk[0, 0] = np.inf
    amp = kk ** (-11.0 / 6.0)
    f = (rng.standard_normal((coarse, coarse)) + 1j * rng.standard_normal((coarse, coarse))) * amp
    s = np.fft.ifft2(f).real
    s -= s.mean()
    return s * (rms / max(s.std(), 1e-30))


def bilinear_on_fov(screen: np.ndarray, l: np.ndarray, m: np.ndarray, fov: float) -> np.ndarray:
    """Sample a coarse screen spanning [-fov/2, fov/2]^2 at directions (l, m)."""
    c = screen.shape[0]
    fx = np.clip((l / fov + 0.5) * (c - 1), 0.0, c - 1.0)
    fy = np.clip((m / fov + 0.5) * (c - 1), 0.0, c - 1.0)
    x0 = np.minimum(np.floor(fx).astype(int), c - 2)
    y0 = np.minimum(np.floor(fy).astype(int), c - 2)
    tx, ty = fx - x0, fy - y0
    return ((1 - tx) * (1 - ty) * screen[y0, x0] + tx * (1 - ty) * screen[y0, x0 + 1]
            + (1 - tx) * ty * screen[y0 + 1, x0] + tx * ty * screen[y0 + 1, x0 + 1])


def gaussian_beam(l: np.ndarray, m: np.ndarray, fwhm_rad: float) -> tuple[np.ndarray, np.ndarray]:
    """Analytic dipole-pair stand-in: x/y Gaussians elongated by +-5 %."""
    sig = fwhm_rad / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    bx = np.exp(-0.5 * ((l / (1.05 * sig)) ** 2 + (m / (0.95 * sig)) ** 2))
    by = np.exp(-0.5 * ((l / (0.95 * sig)) ** 2 + (m / (1.05 * sig)) ** 2))
    return bx, by


def make_aterms(n_int: int, n_st: int, L: int, fov: float, screen_rms: float, coarse: int,
                rng: np.random.Generator, kind: str = "white", beam_fwhm_rad: float | None = None,
                complex_jones: bool = False) -> np.ndarray:
    """Per-interval, per-station Jones on the L x L lattice: beam * exp(i phi) * I.

    ``complex_jones`` adds small random off-diagonal leakage and unequal
    diagonal gains, so that Jones ordering and conjugation are exercised.
    """
    l, m = lattice_lm(L, fov)
    if beam_fwhm_rad is not None:
        bx, by = gaussian_beam(l, m, beam_fwhm_rad)
    else:
        bx = by = np.ones_like(l)
    A = np.zeros((n_int, n_st, L, L, 4), dtype=np.complex128)
    gen = white_screen if kind == "white" else kolmogorov_screen
    for i in range(n_int):
        for s in range(n_st):
            ph = bilinear_on_fov(gen(coarse, screen_rms, rng), l, m, fov) if screen_rms > 0 else 0.0 * l
            e = np.exp(1j * ph)
            A[i, s, :, :, 0] = bx * e
            A[i, s, :, :, 3] = by * e
            if complex_jones:
                g = 1.0 + 0.1 * (rng.standard_normal(2) + 1j * rng.standard_normal(2))
                d = 0.05 * (rng.standard_normal(2) + 1j * rng.standard_normal(2))
                A[i, s, :, :, 0] *= g[0]
                A[i, s, :, :, 3] *= g[1]
                A[i, s, :, :, 1] = d[0] * bx * e
                A[i, s, :, :, 2] = d[1] * by * e
    return A


# ---------------------------------------------------------------- skies / visibilities


def point_sources(n: int, fov: float, flux_lo: float, flux_hi: float, rng: np.random.Generator,
                  L: int | None = None, on_lattice: bool = False, pol_frac: float = 0.1) -> dict:
    """Point sources: flux log-uniform, Q/U/V fractions ~ U(+-pol_frac).

    Returns l, m (direction cosines), lattice indices xs, ys (-1 when off the
    lattice) and brightness matrices B [n][4] = [[I+Q, U+iV], [U-iV, I-Q]].
    """
    flux = np.exp(rng.uniform(math.log(flux_lo), math.log(flux_hi), n))
    q, u, v = (rng.uniform(-pol_frac, pol_frac, (3, n)) * flux)
    B = np.stack([flux + q, u + 1j * v, u - 1j * v, flux - q], axis=1).astype(np.complex128)
    if on_lattice:
        assert L is not None
        xs = rng.integers(2, L - 1, n)
        ys = rng.integers(2, L - 1, n)
        l = (xs - L // 2) * (fov / L)
        m = (ys - L // 2) * (fov / L)
    else:
        xs = ys = -np.ones(n, dtype=np.int64)
        l = rng.uniform(-0.4, 0.4, n) * fov
        m = rng.uniform(-0.4, 0.4, n) * fov
    return {"l": l, "m": m, "xs": np.asarray(xs, np.int32), "ys": np.asarray(ys, np.int32), "B": B}


def random_vis(shape: tuple, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    return (scale * (rng.standard_normal(shape + (4,)) + 1j * rng.standard_normal(shape + (4,)))
            ).astype(np.complex128)


def random_grid(W: int, N: int, rng: np.random.Generator) -> np.ndarray:
    return (rng.standard_normal((W, 4, N, N)) + 1j * rng.standard_normal((W, 4, N, N))).astype(np.complex128)


# ---------------------------------------------------------------- configurations


def observation(n_st: int, diameter_m: float, n_t: int, dt_s: float, f_lo: float, f_hi: float,
                n_c: int, rng: np.random.Generator, ha0_rad: float = 0.0,
                freqs: np.ndarray | None = None):
    enu = station_disc(n_st, diameter_m, rng)
    bl = all_pairs(n_st)
    uvw = earth_rotation_uvw(enu, bl, math.radians(-26.7), math.radians(-27.0),
                             transit_hour_angles(n_t, dt_s, ha0_rad))
    f = channel_centres(f_lo, f_hi, n_c) if freqs is None else np.asarray(freqs, np.float64)
    return bl, uvw, f


def config_small(seed: int = 1) -> Workload:
    """CPU-sized: 16 stations in a 1 km disc, 8 x 2 s, 4 channels at 150..153 MHz,
    grid 512^2, subgrid 32^2, FOV 10 deg, identity Jones times a 0.5 rad white
    phase screen on an 8 x 8 coarse grid per station, 20 point sources."""
    rng = np.random.default_rng(seed)
    bl, uvw, f = observation(16, 1000.0, 8, 2.0, 0, 0, 4, rng,
                             freqs=np.array([150e6, 151e6, 152e6, 153e6]))
    N, L, K = 512, 32, 8
    dl = math.radians(10.0) / N
    A = make_aterms(1, 16, L, N * dl, 0.5, 8, rng, kind="white")
    src = point_sources(20, N * dl, 0.1, 10.0, rng)
    return Workload("small", 16, bl, uvw, f, N, L, K, dl, 8, A, sources=src)


def config_mwa(seed: int = 2, n_bl_subset: int | None = None, screen_rms: float = 2.0,
               ha0_rad: float = 0.0) -> Workload:
    """MWA-like: 128 stations in a 5 km disc (8128 baselines), 60 x 2 s, 96
    channels over 140..170 MHz, grid 8000^2 at 15 arcsec, subgrid 96^2, kernel
    support 24, A-terms every 8 timesteps = Gaussian beam times a Kolmogorov
    screen (2 rad rms, 16 x 16 coarse grid) per station."""
    rng = np.random.default_rng(seed)
    bl, uvw, f = observation(128, 5000.0, 60, 2.0, 140e6, 170e6, 96, rng, ha0_rad=ha0_rad)
    N, L, K = 8000, 96, 24
    dl = 15.0 * ARCSEC
    A = make_aterms(8, 128, L, N * dl, screen_rms, 16, rng, kind="kolmogorov",
                    beam_fwhm_rad=math.radians(25.0) * 155e6 / 155e6)
    if n_bl_subset is not None:
        sub = np.sort(np.random.default_rng(seed).choice(bl.shape[0], n_bl_subset, replace=False))
        bl, uvw = np.ascontiguousarray(bl[sub]), np.ascontiguousarray(uvw[sub])
    return Workload("mwa", 128, bl, uvw, f, N, L, K, dl, 8, A)


def config_diff(seed: int = 4) -> Workload:
    """Differentiable case: 64 stations in a 5 km disc (2016 baselines), 30 x 2 s,
    48 channels over 140..170 MHz, grid 4096^2 at 15 arcsec, subgrid 64^2, K=16."""
    rng = np.random.default_rng(seed)
    bl, uvw, f = observation(64, 5000.0, 30, 2.0, 140e6, 170e6, 48, rng)
    N, L, K = 4096, 64, 16
    dl = 15.0 * ARCSEC
    A = make_aterms(4, 64, L, N * dl, 2.0, 16, rng, kind="kolmogorov",
                    beam_fwhm_rad=math.radians(25.0))
    return Workload("diff", 64, bl, uvw, f, N, L, K, dl, 8, A)


def config_tiny(seed: int, n_st: int = 5, n_t: int = 6, n_c: int = 5, N: int = 128,
                L: int = 32, K: int = 8, fov_deg: float = 20.0, diameter_m: float = 300.0,
                aterm_interval: int = 3, screen_rms: float = 1.0, ha0_deg: float = 20.0,
                f_lo: float = 140e6, f_hi: float = 160e6, complex_jones: bool = True,
                w_step: float = 0.0, beam_fwhm_deg: float | None = None) -> Workload:
    """Small randomised geometry for exact-identity and property tests; with
    ``beam_fwhm_deg`` the Jones terms carry a Gaussian beam (non-unitary, varying over
    the field)."""
    rng = np.random.default_rng(seed)
    bl, uvw, f = observation(n_st, diameter_m, n_t, 30.0, f_lo, f_hi, n_c, rng,
                             ha0_rad=math.radians(ha0_deg))
    dl = math.radians(fov_deg) / N
    n_int = (n_t + aterm_interval - 1) // aterm_interval
    A = make_aterms(n_int, n_st, L, N * dl, screen_rms, 6, rng, kind="white",
                    complex_jones=complex_jones,
                    beam_fwhm_rad=None if beam_fwhm_deg is None else math.radians(beam_fwhm_deg))
    return Workload(f"tiny{seed}", n_st, bl, uvw, f, N, L, K, dl, aterm_interval, A,
                    w_step=w_step)


def max_uv_lambda(wl: Workload) -> float:
    return float(np.abs(wl.uvw[..., :2]).max() * wl.freqs.max() / SPEED_OF_LIGHT)


def served_job_mix(n_jobs: int, seed: int = 5, vis_lo: float = 1e3, vis_hi: float = 5e6):
    """Descriptions of a mixed serving workload: per job a direction (grid or
    degrid, 50/50), a visibility count log-uniform in [vis_lo, vis_hi], 16-128
    stations in a 5 km disc, 8/16/32/96 channels over 140-170 MHz (fewer
    baselines when the count is below one timestep), grid 1024^2..8000^2,
    subgrid 32/64/96 with K = L/4, pixel size min(15 arcsec, 0.45/u_max), one
    A-term interval with a 0-3 rad white phase screen.  Returns dicts with host
    arrays; A-terms and data are generated on the device when a job starts."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n_jobs):
        n_vis = float(np.exp(rng.uniform(math.log(vis_lo), math.log(vis_hi))))
        n_st = int(rng.integers(16, 129))
        n_c = int(rng.choice([8, 16, 32, 96]))
        L = int(rng.choice([32, 64, 96]))
        N = int(rng.choice([1024, 2048, 4096, 8000]))
        enu = station_disc(n_st, 5000.0, rng)
        bl = all_pairs(n_st)
        if n_vis < bl.shape[0] * n_c:
            keep = max(1, int(n_vis // n_c))
            bl = bl[np.sort(rng.choice(bl.shape[0], keep, replace=False))]
            n_t = 1
        else:
            n_t = max(1, int(round(n_vis / (bl.shape[0] * n_c))))
        uvw = earth_rotation_uvw(enu, bl, math.radians(-26.7), math.radians(-27.0),
                                 transit_hour_angles(n_t, 2.0))
        freqs = channel_centres(140e6, 170e6, n_c)
        umax = float(np.abs(uvw[..., :2]).max()) * freqs.max() / SPEED_OF_LIGHT
        dl = min(15.0 * ARCSEC, 0.45 / max(umax, 1.0), 0.6 / N)  # Nyquist; FOV/sqrt(2) < 1
        jobs.append({"direction": "grid" if rng.random() < 0.5 else "degrid", "n_stations": n_st,
                     "baselines": np.ascontiguousarray(bl, np.int32), "uvw": uvw, "freqs": freqs,
                     "N": N, "L": L, "K": L // 4, "dl": dl, "n_t": n_t, "screen_rms": float(rng.uniform(0, 3)),
                     "seed": int(rng.integers(1 << 31))})
    return jobs


def device_phase_screen_aterms(n_st: int, L: int, rms: float, seed: int, coarse: int = 8):
    """A-terms exp(i phi) I on the L x L lattice for one interval, made on the GPU:
    white coarse screens bilinearly upsampled.  Returns complex64 [1, n_st, L, L, 4]."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    c = torch.randn((n_st, 1, coarse, coarse), device="cuda", generator=g)
    c = c - c.mean(dim=(2, 3), keepdim=True)
    c = c * (rms / c.std(dim=(2, 3), keepdim=True).clamp_min(1e-12))
    phi = torch.nn.functional.interpolate(c, size=(L, L), mode="bilinear", align_corners=True)[:, 0]
    e = torch.polar(torch.ones_like(phi), phi)
    A = torch.zeros((1, n_st, L, L, 4), dtype=torch.complex64, device="cuda")
    A[0, :, :, :, 0] = e
    A[0, :, :, :, 3] = e
    return A


def hour_angle_for_wmax(w_target: float, seed: int = 2, lo: float = 0.0, hi: float = 1.0) -> float:
    """Phase-centre hour angle (rad) at which the MWA-like observation's largest
    |w| at the top channel reaches w_target wavelengths (bisection on ha0)."""
    c = 299792458.0

    def wmax(ha):
        _, uvw, f = observation(128, 5000.0, 60, 2.0, 140e6, 170e6, 96, np.random.default_rng(seed),
                                ha0_rad=ha)
        return float(np.abs(uvw[..., 2]).max() * f.max() / c)

    if wmax(lo) >= w_target:
        return lo
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if wmax(mid) < w_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def device_point_source_vis(wl: "Workload", n_src: int, seed: int, flux_lo: float = 0.01,
                            flux_hi: float = 30.0, noise_rms: float = 1.0, chunk: int = 32):
    """Visibilities of a point-source sky (identity Jones), evaluated in FP64 on the
    GPU: V = sum_s B_s exp(-2 pi i (u l_s + v m_s + w n1_s)) plus complex Gaussian
    noise of the given rms per component.  Returns complex128 [nbl, nt, nc, 4]."""
    import torch
    rng = np.random.default_rng(seed)
    src = point_sources(n_src, wl.fov, flux_lo, flux_hi, rng)
    l = torch.from_numpy(src["l"]).cuda()
    m = torch.from_numpy(src["m"]).cuda()
    n1 = -(l * l + m * m) / (1.0 + torch.sqrt(1.0 - l * l - m * m))
    B = torch.from_numpy(src["B"]).cuda()                               # [S, 4]
    fc = torch.from_numpy(wl.freqs / 299792458.0).cuda()               # [nc]
    uvw = torch.from_numpy(wl.uvw).cuda()                              # [nbl, nt, 3] metres
    out = torch.empty((wl.n_baselines, wl.n_times, wl.n_chans, 4), dtype=torch.complex128, device="cuda")
    for b0 in range(0, wl.n_baselines, chunk):
        u = uvw[b0:b0 + chunk]
        # phase in turns per metre of baseline, then per channel: [b, t, S] x [c]
        pm = u[..., 0:1] * l + u[..., 1:2] * m + u[..., 2:3] * n1
        turns = pm[:, :, None, :] * fc[None, None, :, None]             # [b, t, c, S]
        turns = turns - torch.round(turns)
        ph = torch.polar(torch.ones_like(turns), -2.0 * math.pi * turns)
        out[b0:b0 + chunk] = ph @ B
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    # torch draws complex normals with E|z|^2 = 1: scale to noise_rms per component
    out += noise_rms * math.sqrt(2.0) * torch.randn(out.shape, dtype=torch.complex128, device="cuda",
                                                    generator=g)
    return out
