"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/aidg.h declares, validates geometry, and its own partitioner
(Sec. 3.1 sub-tables) produces partitions the oracle's independent checker accepts."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2502_17789_amd as aidg
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "aidg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aidg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(aidg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 11
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    header = open(os.path.join(ROOT, "include", "aidg.h")).read()
    version = int(re.search(r"#define AIDG_ABI_VERSION (\d+)", header).group(1))
    assert aidg.library().aidg_abi_version() == version


def geo_of(wl, **kw):
    return aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale,
                         aterm_interval=wl.aterm_interval, **kw)


def part(wl, **kw):
    return aidg.partition(geo_of(wl, **kw), wl.n_stations, wl.baselines, wl.uvw, wl.freqs)


@pytest.mark.parametrize("seed,w_step", [(1, 0.0), (2, 10.0), (3, -1.0), (4, 4.0)])
def test_partition_valid_tiny(orc, seed, w_step):
    wl = synth.config_tiny(seed, n_st=8, n_t=9, n_c=12, ha0_deg=30.0)
    table, ws = part(wl, w_step=w_step)
    assert orc.check_partition(wl, table, ws) == (0, -1)
    if w_step > 0:
        assert ws == w_step


def test_partition_valid_small_config(orc):
    wl = synth.config_small()
    table, ws = part(wl)
    assert orc.check_partition(wl, table, ws) == (0, -1)
    assert table.shape[0] <= wl.n_baselines * 2


def test_partition_respects_cap_and_edges(orc):
    wl = synth.config_tiny(9, N=64, diameter_m=700.0, n_t=12, n_c=16, aterm_interval=6)
    table, ws = part(wl, max_subgrid_vis=8)
    assert orc.check_partition(wl, table, ws) == (0, -1)
    assert (table["nt"] * table["nc"]).max() <= 8
    mask = orc.coverage_mask(wl, table)
    assert 0 < mask.sum() < mask.size  # some visibilities fall off the grid


def test_auto_w_step_formula():
    N, L, K, dl = 8000, 96, 24, 15.0 * synth.ARCSEC
    _, ws = aidg.partition(aidg.Geometry(N, L, K, dl), 2, np.array([[0, 1]]), np.zeros((1, 1, 3)),
                           np.array([150e6]))
    fov = N * dl
    r = fov / math.sqrt(2.0)
    rho = r / math.sqrt(1 - r * r)
    assert ws == pytest.approx(2 * K / (4 * fov * rho), rel=1e-12)


@pytest.mark.parametrize("bad", [dict(subgrid_size=33), dict(kernel_support=32), dict(grid_size=30),
                                 dict(pixel_scale=-1.0), dict(aterm_interval=0),
                                 dict(pixel_scale=math.radians(120) / 512), dict(max_subgrid_vis=2049),
                                 dict(max_subgrid_vis=-1), dict(center_lattice=-2), dict(w_fold=2),
                                 dict(aterm_mode=2), dict(stokes_i=2)])
def test_invalid_geometry_rejected(bad):
    kw = dict(grid_size=512, subgrid_size=32, kernel_support=8, pixel_scale=math.radians(10) / 512)
    kw.update(bad)
    with pytest.raises(aidg.AidgError) as e:
        aidg.partition(aidg.Geometry(**kw), 2, np.array([[0, 1]]), np.zeros((1, 1, 3)), np.array([1e8]))
    assert e.value.status == aidg.AIDG_E_INVALID


@pytest.mark.parametrize("seed,ha0_deg", [(51, 0.0), (52, -60.0)])
def test_fold_partition_valid_and_fewer_layers(orc, seed, ha0_deg):
    """w_fold: the library's partition passes the oracle's checker in fold mode, holds
    folded sub-tables, puts every layer at w0 = (j + 1/2) w_step > 0, and needs no
    more layers than the unfolded partition (about half when w takes both signs)."""
    wl = synth.config_tiny(seed, ha0_deg=ha0_deg)
    geo = dict(grid_size=wl.grid_size, subgrid_size=wl.subgrid_size, kernel_support=wl.kernel_support,
               pixel_scale=wl.pixel_scale, aterm_interval=wl.aterm_interval, w_step=12.0)
    t1, ws = aidg.partition(aidg.Geometry(**geo, w_fold=1), wl.n_stations, wl.baselines, wl.uvw, wl.freqs)
    t0, _ = aidg.partition(aidg.Geometry(**geo), wl.n_stations, wl.baselines, wl.uvw, wl.freqs)
    assert orc.check_partition(wl, t1, ws, fold=1) == (0, -1)
    assert t1["folded"].sum() > 0 and (t1["w0"] > 0).all()
    assert np.allclose(((t1["w0"] / ws) - 0.5) % 1.0, 0.0)
    assert len(np.unique(t1["w0"])) <= len(np.unique(t0["w0"]))


def test_strict_range_reports_range_error():
    wl = synth.config_tiny(9, N=64, diameter_m=700.0)
    with pytest.raises(aidg.AidgError) as e:
        part(wl, strict_range=1)
    assert e.value.status == aidg.AIDG_E_RANGE


@pytest.mark.slow
def test_partition_valid_mwa_full_size(orc):
    """Full MWA-like observation (8128 baselines x 60 x 96, 46.8M visibilities)."""
    wl = synth.config_mwa()
    table, ws = part(wl)
    assert orc.check_partition(wl, table, ws) == (0, -1)
    occ = table["nt"] * table["nc"]
    assert occ.sum() == wl.n_vis
    assert 5e4 < table.shape[0] < 5e5


def test_autograd_refuses_the_inverse_aterm_mode():
    """Inverse-mode gridding is not the adjoint of degridding: the differentiable
    wrappers refuse such plans before touching the device."""
    import types
    from paper_2502_17789_amd import autograd
    geo = aidg.Geometry(64, 32, 8, 1e-3, aterm_mode=aidg.ATERM_INVERSE)
    with pytest.raises(ValueError):
        autograd._adjoint_plan(types.SimpleNamespace(geometry=geo))
    ok = types.SimpleNamespace(geometry=aidg.Geometry(64, 32, 8, 1e-3))
    assert autograd._adjoint_plan(ok) is ok


def test_missing_library_fails_loudly(monkeypatch):
    """Without libaidg.so every entry point raises: there is no CPU fallback."""
    monkeypatch.setattr(aidg, "LIB_PATH", "/nonexistent/libaidg.so")
    monkeypatch.setattr(aidg, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        aidg.library()
    wl = synth.config_tiny(1)
    geo = aidg.Geometry(wl.grid_size, wl.subgrid_size, wl.kernel_support, wl.pixel_scale)
    with pytest.raises(RuntimeError, match="not built"):
        aidg.partition(geo, wl.n_stations, wl.baselines, wl.uvw, wl.freqs)


def test_product_never_imports_the_oracle():
    """The library package, its sources and the build script name no oracle module."""
    root = os.path.dirname(aidg.__file__)
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text and "oracle.cpp" not in text, f


def test_execute_static_rejects_budgets_beyond_its_workspace():
    """aidg_execute_static checks its workspace budget before any device call: beyond
    AIDG_STATIC_WORKSPACE_BYTES (and below 0) it returns AIDG_E_INVALID with a message;
    an empty item list within the budget is a no-op."""
    lib = aidg.library()
    header = open(os.path.join(ROOT, "include", "aidg.h")).read()
    assert "#define AIDG_STATIC_WORKSPACE_BYTES ((int64_t)128 << 20)" in header
    assert aidg.STATIC_WORKSPACE_BYTES == 128 << 20
    for bad in (aidg.STATIC_WORKSPACE_BYTES + 1, -1, 1 << 40):
        assert lib.aidg_execute_static(None, 0, bad, None) == aidg.AIDG_E_INVALID
        assert b"AIDG_STATIC_WORKSPACE_BYTES" in lib.aidg_last_error()
    assert lib.aidg_execute_static(None, 0, 0, None) == aidg.AIDG_OK
    assert lib.aidg_execute_static(None, 0, aidg.STATIC_WORKSPACE_BYTES, None) == aidg.AIDG_OK
    assert lib.aidg_execute_static(None, -1, 0, None) == aidg.AIDG_E_INVALID
