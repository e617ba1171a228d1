"""GPU parity of the degridder's forms (Sec. 3.2, Degridder: a kernel design chosen per
subgrid by its occupancy).  geometry.degrid_form selects the recurrence form (lanes own
pixels, phasors step along each row's channels), the direct form (lanes own pixels,
every visibility's phasor seeded from FP64), the per-visibility form (lanes own
visibilities, for every sub-table that fits the workgroup) or the automatic choice per
subgrid.  Each is checked against the FP64 oracle's degridding on the plan's own
partition, element by element at the gates of tests/gates.py (FP32 1e-5, FP64 1e-10),
across subgrid sizes, precisions, the fold, Stokes-I grids, irregular channel spacing
and a channel-decimated observation whose subgrids hold a few visibilities each; the
forms agree with each other, each is deterministic (two calls bitwise equal), and the
plan reports how many subgrids took the direct and per-visibility forms.
"""
import numpy as np
import pytest

import synth
from gates import check_vis

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {0: 1e-5, 1: 1e-10}
LANES = {(32, 0): 128, (64, 0): 256, (96, 0): 256, (32, 1): 256, (64, 1): 256, (96, 1): 256}


@pytest.fixture(scope="module")
def aidg():
    import paper_2502_17789_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m.library()
    return m


def dev(x, prec):
    dt = np.complex64 if prec == 0 else np.complex128
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


CASES = {
    "L32": dict(seed=101, L=32, K=8, N=128, n_st=6, n_t=6, n_c=9),
    "L64": dict(seed=102, L=64, K=16, N=256, n_st=5, n_t=7, n_c=20, fov_deg=15.0, diameter_m=800.0),
    "L96": dict(seed=103, L=96, K=24, N=384, n_st=4, n_t=5, n_c=33, fov_deg=12.0, diameter_m=1500.0,
                aterm_interval=2),
    "one_channel": dict(seed=201, n_c=1, n_t=4),
    "one_vis": dict(seed=202, n_st=2, n_t=1, n_c=1),
}


def plan_for(aidg, wl, precision, form, **kw):
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                        aterm_interval=wl.aterm_interval, precision=precision, degrid_form=form, **kw)
    return aidg.Plan(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs, dev(wl.aterms, precision))


def eligible(table, L, precision):
    return int(np.sum(table["nt"].astype(np.int64) * table["nc"] <= LANES[(L, precision)]))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_degrid_forms_match_oracle(aidg, orc, name, precision):
    wl = synth.config_tiny(**CASES[name])
    L = wl.subgrid_size
    rng = np.random.default_rng(21)
    outs = {}
    forms = (aidg.DEGRID_RECURRENCE, aidg.DEGRID_DIRECT, aidg.DEGRID_PER_VIS, aidg.DEGRID_AUTO)
    for form in forms:
        with plan_for(aidg, wl, precision, form, w_step=12.0) as p:
            table = p.subgrids()
            if form == aidg.DEGRID_RECURRENCE:
                G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
                ref = orc.degrid(wl, G, table)
            n_pv, n_dir = p.info["n_subgrids_pervis"], p.info["n_subgrids_direct"]
            Vd = dev(np.full((wl.n_baselines, wl.n_times, wl.n_chans, 4), 5.0 + 5.0j), precision)
            V = host(p.degrid(dev(G, precision), out=Vd))
        n = len(table)
        if form == aidg.DEGRID_RECURRENCE:
            assert n_pv == 0 and n_dir == 0
        elif form == aidg.DEGRID_DIRECT:
            assert n_pv == 0 and n_dir == n
        elif form == aidg.DEGRID_PER_VIS:
            assert n_pv == eligible(table, L, precision) > 0 and n_dir == 0
        else:
            assert n_pv + n_dir <= n
        tag = (f"{name} {'FP64' if precision else 'FP32'} form {form} "
               f"({n_dir} direct, {n_pv} per visibility of {n})")
        check_vis(V, ref, TOL[precision], tag + " vs oracle")
        outs[form] = V
    for form in forms[1:]:
        check_vis(outs[form], outs[aidg.DEGRID_RECURRENCE], TOL[precision], f"{name} form {form} vs recurrence")


def test_irregular_channels_in_every_form(aidg, orc):
    """Channels without a common spacing: the recurrence form takes the direct form for
    them, and every form matches the oracle."""
    wl = synth.config_tiny(205, n_st=4, n_t=6, n_c=12, aterm_interval=6)
    wl.freqs = np.sort(140e6 + 20e6 * np.random.default_rng(3).random(12))
    rng = np.random.default_rng(25)
    for form in (aidg.DEGRID_RECURRENCE, aidg.DEGRID_DIRECT, aidg.DEGRID_PER_VIS, aidg.DEGRID_AUTO):
        with plan_for(aidg, wl, 0, form) as p:
            table = p.subgrids()
            G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
            V = host(p.degrid(dev(G, 0)))
            n_pv, n_dir = p.info["n_subgrids_pervis"], p.info["n_subgrids_direct"]
        assert n_pv + n_dir == len(table)  # no subgrid takes the recurrence
        check_vis(V, orc.degrid(wl, G, table), TOL[0], f"irregular channels, form {form}")


@pytest.mark.parametrize("kind", ["fold", "stokes_i", "inverse_mode"])
def test_per_visibility_form_in_plan_variants(aidg, orc, kind):
    """The per-visibility form's output conventions: a folded sub-table returns the
    conjugate transpose of its prediction at -uvw, a Stokes-I grid predicts from
    I diag(1, 1), and the inverse A-term mode degrids as the adjoint mode does."""
    wl = synth.config_tiny(71, ha0_deg=-60.0, beam_fwhm_deg=15.0, n_t=6, n_c=7)
    kw = {"fold": dict(w_fold=1, w_step=12.0), "stokes_i": dict(stokes_i=1, w_step=12.0),
          "inverse_mode": dict(aterm_mode=1, w_step=12.0)}[kind]
    rng = np.random.default_rng(22)
    with plan_for(aidg, wl, 0, aidg.DEGRID_PER_VIS, **kw) as p:
        table = p.subgrids()
        assert p.info["n_subgrids_pervis"] == eligible(table, wl.subgrid_size, 0) > 0
        G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
        if kind == "stokes_i":
            G = np.ascontiguousarray(G[:, :1])
        V = host(p.degrid(dev(G, 0)))
    ref = orc.degrid_stokes_i(wl, G, table) if kind == "stokes_i" else orc.degrid(wl, G, table)
    check_vis(V, ref, TOL[0], f"{kind}: per-visibility form vs oracle")


@pytest.mark.parametrize("form", [1, 2, 3])
def test_degrid_forms_are_deterministic(aidg, form):
    wl = synth.config_tiny(**CASES["L64"])
    rng = np.random.default_rng(23)
    with plan_for(aidg, wl, 0, form, w_step=20.0) as p:
        G = dev(synth.random_grid(p.n_wlayers, wl.grid_size, rng), 0)
        a = p.degrid(G).cpu().numpy()
        b = p.degrid(G).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_sparse_observation_takes_the_direct_form(aidg, orc):
    """A channel-decimated observation (rows of one or two channels, a few visibilities
    per subgrid: the low-occupancy regime of Sec. 4.2) in the automatic mode: most of its
    subgrids take the direct form, and the result is the oracle's."""
    wl = synth.config_tiny(31, n_st=8, n_t=6, n_c=24, L=64, K=16, N=512, fov_deg=10.0, diameter_m=2000.0,
                           f_lo=140e6, f_hi=170e6)
    wl.freqs = np.ascontiguousarray(wl.freqs[::12])
    rng = np.random.default_rng(24)
    with plan_for(aidg, wl, 0, aidg.DEGRID_AUTO, w_step=30.0) as p:
        table = p.subgrids()
        n_dir = p.info["n_subgrids_direct"]
        G = synth.random_grid(p.n_wlayers, wl.grid_size, rng)
        V = host(p.degrid(dev(G, 0)))
    print(f"sparse: {len(table)} subgrids, {np.mean(table['nt'] * table['nc']):.1f} visibilities each, "
          f"{n_dir} direct", flush=True)
    assert n_dir >= 0.5 * len(table)
    check_vis(V, orc.degrid(wl, G, table), TOL[0], "sparse observation, automatic form vs oracle")
