// Host-side plan logic: geometry validation, w-layer spacing, the sub-table
// partitioner of Sec. 3.1, adoption of caller partitions and the taper.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "aidg_internal.h"

namespace aidg {

aidg_status validate_geometry(const aidg_geometry* g, Geometry* o, std::string* err) {
  if (!g) {
    *err = "geometry is NULL";
    return AIDG_E_INVALID;
  }
  const int N = g->grid_size, L = g->subgrid_size, K = g->kernel_support;
  if (L < 4 || (L & 1)) {
    *err = "subgrid_size must be even and >= 4";
    return AIDG_E_INVALID;
  }
  if (N < L || (N & 1)) {
    *err = "grid_size must be even and >= subgrid_size";
    return AIDG_E_INVALID;
  }
  if (K < 0 || (K & 1) || K >= L) {
    *err = "kernel_support must be even with 0 <= K < L";
    return AIDG_E_INVALID;
  }
  if (g->aterm_interval < 1) {
    *err = "aterm_interval must be >= 1";
    return AIDG_E_INVALID;
  }
  if (!(g->pixel_scale > 0) || !std::isfinite(g->pixel_scale)) {
    *err = "pixel_scale must be positive";
    return AIDG_E_INVALID;
  }
  const double fov = N * g->pixel_scale;
  // the corner pixel of the subgrid lattice, (-FOV/2, -FOV/2), must be above the horizon
  if (fov * fov / 2.0 >= 1.0) {
    *err = "field of view reaches the horizon (FOV/sqrt(2) >= 1)";
    return AIDG_E_INVALID;
  }
  if (g->precision != AIDG_FP32 && g->precision != AIDG_FP64) {
    *err = "precision must be AIDG_FP32 or AIDG_FP64";
    return AIDG_E_INVALID;
  }
  if (g->max_subgrid_vis > kMaxSubgridVisLimit) {
    *err = "max_subgrid_vis must be <= " + std::to_string(kMaxSubgridVisLimit) +
           " (a subgrid's visibilities are staged in LDS)";
    return AIDG_E_INVALID;
  }
  if (g->reseed_channels < 0 || g->max_subgrid_vis < 0 || g->workspace_bytes < 0 ||
      !std::isfinite(g->w_step) || !std::isfinite(g->taper_beta) || g->taper_beta < 0) {
    *err = "negative or non-finite numeric parameter";
    return AIDG_E_INVALID;
  }
  o->N = N;
  o->L = L;
  o->K = K;
  o->aterm_interval = g->aterm_interval;
  o->precision = g->precision;
  o->R = g->reseed_channels ? g->reseed_channels : kReseedDefault;
  o->strict = g->strict_range != 0;
  o->max_sg_vis = g->max_subgrid_vis ? g->max_subgrid_vis : kMaxSubgridVisDefault;
  o->dl = g->pixel_scale;
  o->fov = fov;
  o->du = 1.0 / fov;
  o->beta = g->taper_beta > 0 ? g->taper_beta : M_PI * K / 4.0;
  o->workspace = g->workspace_bytes ? g->workspace_bytes : kWorkspaceDefault;
  if (g->center_lattice < 0) {
    *err = "center_lattice must be >= 0";
    return AIDG_E_INVALID;
  }
  if (g->w_fold != 0 && g->w_fold != 1) {
    *err = "w_fold must be 0 or 1";
    return AIDG_E_INVALID;
  }
  o->fold = g->w_fold;
  if (g->aterm_mode != 0 && g->aterm_mode != 1) {
    *err = "aterm_mode must be 0 (adjoint) or 1 (inverse)";
    return AIDG_E_INVALID;
  }
  o->amode = g->aterm_mode;
  if (g->stokes_i != 0 && g->stokes_i != 1) {
    *err = "stokes_i must be 0 or 1";
    return AIDG_E_INVALID;
  }
  o->npol = g->stokes_i ? 1 : 4;
  if (g->degrid_form < AIDG_DEGRID_AUTO || g->degrid_form > AIDG_DEGRID_DIRECT || g->reserved != 0) {
    *err = "degrid_form must be 0 (automatic), 1 (recurrence), 2 (per visibility) or 3 (direct), reserved 0";
    return AIDG_E_INVALID;
  }
  o->degrid_form = g->degrid_form;
  if (g->center_lattice > 0) {
    o->lattice = g->center_lattice;
  } else {
    // largest power of two <= 2 (L - K) / 3: 16, 32, 32 at L = 32, 64, 96 with K = L/4.
    // Coarser steps make larger same-centre groups (fewer subgrid FFTs and grid
    // updates) for a few percent more subgrids; measured best on MWA-like tracks.
    o->lattice = 1;
    while (o->lattice * 2 <= 2 * (L - K) / 3) o->lattice *= 2;
  }
  if (g->w_step > 0) o->w_step = g->w_step;
  else if (g->w_step < 0) o->w_step = 0.0;
  else o->w_step = auto_w_step(*o);
  return AIDG_OK;
}

// w_max (Sec. 2.4 footnote): the w-term's local fringe rate |w - w0| |grad n| must
// stay within the K/4 cells left beside the taper's main lobe, i.e.
// |w - w0| rho FOV <= K/4 with rho the largest |grad n| = r / n on the lattice
// (at its corner).  Layers are spaced by 2 w_max.
double auto_w_step(const Geometry& g) {
  if (g.K == 0) return 0.0;
  const double r = g.fov / std::sqrt(2.0);
  const double rho = r / std::sqrt(1.0 - r * r);
  const double wmax = g.K / (4.0 * g.fov * rho);
  return 2.0 * wmax;
}

namespace {

struct Box {
  double ulo = 1e300, uhi = -1e300, vlo = 1e300, vhi = -1e300;
  void add(double u, double v) {
    ulo = std::min(ulo, u);
    uhi = std::max(uhi, u);
    vlo = std::min(vlo, v);
    vhi = std::max(vhi, v);
  }
};

struct Ctx {
  const Geometry& g;
  int nbl, nt, nc;
  const double* uvw;
  const double* freqs;
  std::vector<Box>* boxes = nullptr;  // scratch of the time extension
  // metres x Hz to grid cells, metres x Hz to wavelengths, wavelengths to layers
  double k_cell = 1.0 / (kSpeedOfLight * g.du), k_w = 1.0 / kSpeedOfLight,
         k_layer = g.w_step > 0 ? 1.0 / g.w_step : 0.0;
  // -1 for a row the fold moves to -uvw (fold mode and w < 0), else +1
  double sign(int bl, int t) const { return g.fold && uvw[3 * ((size_t)bl * nt + t) + 2] < 0 ? -1.0 : 1.0; }
  double cell(int bl, int t, int c, int axis) const {
    return sign(bl, t) * uvw[3 * ((size_t)bl * nt + t) + axis] * freqs[c] * k_cell + g.N / 2;
  }
  double wl(int bl, int t, int c) const {
    return sign(bl, t) * uvw[3 * ((size_t)bl * nt + t) + 2] * freqs[c] * k_w;
  }
  bool inside(double gu, double gv) const {
    const double lo = g.K / 2.0, hi = g.N - g.K / 2.0;
    return gu >= lo && gu <= hi && gv >= lo && gv <= hi && std::isfinite(gu) && std::isfinite(gv);
  }
  bool placeable(int bl, int t, int c) const { return inside(cell(bl, t, c, 0), cell(bl, t, c, 1)); }
  // nearest layer j w_step; with the fold (w >= 0) layers at (j + 1/2) w_step
  int64_t layer(int bl, int t, int c) const {
    if (!(g.w_step > 0)) return 0;
    const double j = wl(bl, t, c) * k_layer;
    return (int64_t)(g.fold ? std::floor(j) : std::nearbyint(j));
  }
};


// Centre cell for a span [lo, hi]: a cell of the lattice N/2 + k * lattice near the
// middle of the span (clamped so that the L-cell window stays on the grid); true
// if every point of the span is then within `half` cells of it.
bool centre(double lo, double hi, double half, int L, int N, int lattice, int* c) {
  const double mid = 0.5 * (lo + hi);
  const double k0 = std::floor((mid - N / 2) / lattice);
  int best = 0;
  double best_d = 1e300;
  for (int dk = -1; dk <= 2; ++dk) {
    int k = N / 2 + (int)(k0 + dk) * lattice;
    k = std::min(std::max(k, L / 2), N - L / 2);
    if (hi - k <= half && k - lo <= half) {
      const double d = std::fabs(k - mid);
      if (d < best_d) {
        best_d = d;
        best = k;
      }
    }
  }
  if (best_d < 1e300) {
    *c = best;
    return true;
  }
  int k = (int)std::floor(mid + 0.5);
  *c = std::min(std::max(k, L / 2), N - L / 2);
  return false;
}

// Along one row (baseline, timestep) u, v and w are one vector scaled by frequency, and
// the channels' frequencies increase: a channel's cell coordinates and layer are
// monotonic in the channel index (with rounding, weakly).  So the channels of a row that
// can be placed form one interval (the placeable region is a box), a channel range's
// bounding box is spanned by its two end channels, and its layers are all equal when
// those of its ends are.  The partitioner below relies on this to look at the ends of
// ranges only.

// First channel in (c, e) for which pred is false, e if none; pred must be true at c
// and, over (c, e), true up to some channel and false after it.
template <typename F>
int first_false(int c, int e, F pred) {
  int lo = c, hi = e;  // pred(lo) true; the answer is in (lo, hi]
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (pred(mid)) lo = mid;
    else hi = mid;
  }
  return hi;
}

// Add row t, channels [c0, c1), to box b; false if the row has another fold state
// than sgn, or a visibility is unplaceable or in another layer.
bool add_row(const Ctx& x, int bl, int t, int c0, int c1, int64_t layer, double sgn, Box* b) {
  if (x.sign(bl, t) != sgn) return false;
  const double u0 = x.cell(bl, t, c0, 0), v0 = x.cell(bl, t, c0, 1);
  const double u1 = x.cell(bl, t, c1 - 1, 0), v1 = x.cell(bl, t, c1 - 1, 1);
  if (!x.inside(u0, v0) || !x.inside(u1, v1)) return false;
  if (x.layer(bl, t, c0) != layer || x.layer(bl, t, c1 - 1) != layer) return false;
  b->add(u0, v0);
  b->add(u1, v1);
  return true;
}

void tile(const Ctx& x, int bl, int ts, int te, int c_lo, int c_hi, PartitionResult* out,
          std::vector<aidg_subgrid>* sgs, const int32_t* baselines) {
  if (ts >= te || c_lo >= c_hi) return;
  const Geometry& g = x.g;
  const double window = g.L - g.K, half = 0.5 * window, comfy = 0.75 * window;
  // Row ts of channels [c_lo, c_hi) is split into runs; every run grows
  // downwards in time, and the rows it leaves below are tiled recursively.
  int c = c_lo;
  while (c < c_hi) {
    if (!x.placeable(bl, ts, c)) {
      int c2 = c;
      while (c2 < c_hi && !x.placeable(bl, ts, c2)) {
        out->excluded.push_back(((int64_t)bl * x.nt + ts) * x.nc + c2);
        ++c2;
      }
      tile(x, bl, ts + 1, te, c, c2, out, sgs, baselines);
      c = c2;
      continue;
    }
    const int64_t lay = x.layer(bl, ts, c);
    // the run [c, e): placeable, one layer, at most max_sg_vis channels, and its box
    // within 3/4 of the window and centred on a lattice cell
    int e_lim = (int)std::min<int64_t>(c_hi, (int64_t)c + g.max_sg_vis);
    e_lim = first_false(c, e_lim, [&](int k) { return x.placeable(bl, ts, k) && x.layer(bl, ts, k) == lay; });
    auto fits = [&](int e) {
      Box q;
      q.add(x.cell(bl, ts, c, 0), x.cell(bl, ts, c, 1));
      q.add(x.cell(bl, ts, e - 1, 0), x.cell(bl, ts, e - 1, 1));
      int cu, cv;
      return q.uhi - q.ulo <= comfy && q.vhi - q.vlo <= comfy && centre(q.ulo, q.uhi, half, g.L, g.N, g.lattice, &cu) &&
             centre(q.vlo, q.vhi, half, g.L, g.N, g.lattice, &cv);
    };
    // largest e in [c + 1, e_lim] that fits (a single channel always does)
    int lo = c + 1, hi = e_lim + 1;
    while (hi - lo > 1) {
      const int mid = lo + (hi - lo) / 2;
      if (fits(mid)) lo = mid;
      else hi = mid;
    }
    const int e = lo;
    Box b;
    b.add(x.cell(bl, ts, c, 0), x.cell(bl, ts, c, 1));
    b.add(x.cell(bl, ts, e - 1, 0), x.cell(bl, ts, e - 1, 1));
    // extend the run over the rows below while they are placeable in the same layer
    // and fold state, the visibilities stay under max_sg_vis and the rows' joint box
    // keeps a lattice centre: prefix boxes of the rows that qualify, then the largest
    // prefix whose box has a centre (binary search; a box that grows keeps none once it
    // has lost it)
    const int t_cap = (int)std::min<int64_t>(te, (int64_t)ts + g.max_sg_vis / (e - c));
    std::vector<Box>& pre = *x.boxes;
    pre.assign(1, b);
    for (int t = ts + 1; t < t_cap; ++t) {
      Box q = pre.back();
      if (!add_row(x, bl, t, c, e, lay, x.sign(bl, ts), &q)) break;
      pre.push_back(q);
    }
    int cu, cv;
    auto has_centre = [&](const Box& q) {
      return centre(q.ulo, q.uhi, half, g.L, g.N, g.lattice, &cu) && centre(q.vlo, q.vhi, half, g.L, g.N, g.lattice, &cv);
    };
    int klo = 0, khi = (int)pre.size();  // prefix klo (rows ts..ts+klo) qualifies
    while (khi - klo > 1) {
      const int mid = klo + (khi - klo) / 2;
      if (has_centre(pre[mid])) klo = mid;
      else khi = mid;
    }
    b = pre[klo];
    const int t1 = ts + 1 + klo;
    int U0, V0;
    centre(b.ulo, b.uhi, half, g.L, g.N, g.lattice, &U0);
    centre(b.vlo, b.vhi, half, g.L, g.N, g.lattice, &V0);
    aidg_subgrid s;
    std::memset(&s, 0, sizeof(s));
    s.bl = bl;
    s.st1 = baselines[2 * bl];
    s.st2 = baselines[2 * bl + 1];
    s.t0 = ts;
    s.nt = t1 - ts;
    s.c0 = c;
    s.nc = e - c;
    s.U0 = U0;
    s.V0 = V0;
    s.wlayer = (int32_t)lay;  // raw layer number, rebased by the caller
    s.aint = ts / g.aterm_interval;
    s.folded = x.sign(bl, ts) < 0;
    s.w0 = g.w_step > 0 ? (lay + (g.fold ? 0.5 : 0.0)) * g.w_step : 0.0;
    s.vis_offset = ((int64_t)bl * x.nt + ts) * x.nc + c;
    sgs->push_back(s);
    tile(x, bl, t1, te, c, e, out, sgs, baselines);
    c = e;
  }
}

}  // namespace

void estimate_shape(const Geometry& g, int nbl, int nt, int nc, const double* uvw, const double* freqs,
                    ShapeEstimate* out) {
  Ctx x{g, nbl, nt, nc, uvw, freqs};
  const double comfy = 0.75 * (g.L - g.K);
  *out = ShapeEstimate{};
  bool any = false;
  int64_t placed = 0;
  // Same-centre groups: the partition centres a run near the middle of its uv span on
  // the lattice N/2 + k lattice (clamped so that the window stays on the grid), so the
  // distinct (layer, nearest lattice cell) pairs of the runs' midpoints count them.
  std::unordered_set<uint64_t> centres;
  auto lattice_cell = [&](double c) {
    const double k = std::nearbyint((c - g.N / 2) / g.lattice);
    const double lo = std::ceil((g.L / 2 - g.N / 2) / (double)g.lattice),
                 hi = std::floor((g.N - g.L / 2 - g.N / 2) / (double)g.lattice);
    return (uint64_t)((int64_t)std::min(std::max(k, lo), hi) + (1 << 19)) & 0xFFFFF;
  };
  auto mark = [&](double cu, double cv, int64_t lay) {
    centres.insert(((uint64_t)(lay + (1 << 23)) & 0xFFFFFF) << 40 | lattice_cell(cu) << 20 | lattice_cell(cv));
  };
  auto take = [&](int64_t lay) {
    out->jmin = any ? std::min(out->jmin, lay) : lay;
    out->jmax = any ? std::max(out->jmax, lay) : lay;
    any = true;
  };
  // One A-term interval of one baseline at a time: a row's channels split into about
  // 1 + extent / (3/4 window) runs, which the partition extends in time until the track
  // has drifted by the quarter window the runs leave free.
  for (int bl = 0; bl < nbl; ++bl)
    for (int ta = 0; ta < nt && nc > 0; ta += g.aterm_interval) {
      const int te = std::min(nt, ta + g.aterm_interval);
      int64_t runs = 0, layers = 0;
      bool whole = true;
      for (int t = ta; t < te && whole; ++t) whole = x.placeable(bl, t, 0) && x.placeable(bl, t, nc - 1);
      if (whole) {
        // Along a row u, v and w scale with frequency: the cells move on a straight
        // line, so all channels of a row whose two ends are placeable are placeable (the
        // placeable region is a box), its extent is that of the ends and its layers run
        // monotonically from one end's to the other's.
        double drift = 0.0;
        const int cm = nc / 2;
        for (int t = ta; t < te; ++t) {
          const int64_t j0 = x.layer(bl, t, 0), j1 = x.layer(bl, t, nc - 1);
          take(j0);
          take(j1);
          const double ext = std::max(std::fabs(x.cell(bl, t, nc - 1, 0) - x.cell(bl, t, 0, 0)),
                                      std::fabs(x.cell(bl, t, nc - 1, 1) - x.cell(bl, t, 0, 1)));
          runs = std::max<int64_t>(runs, 1 + (int64_t)std::floor(ext / comfy));
          layers = std::max<int64_t>(layers, std::llabs(j1 - j0));
          drift = std::max({drift, std::fabs(x.cell(bl, t, cm, 0) - x.cell(bl, ta, cm, 0)),
                            std::fabs(x.cell(bl, t, cm, 1) - x.cell(bl, ta, cm, 1))});
        }
        const int64_t segs = 1 + (int64_t)std::floor(drift / (0.25 * (g.L - g.K)));
        out->n_subgrids += (runs + layers) * segs;
        // the runs' midpoints on the first row of each time segment
        for (int64_t sgm = 0; sgm < segs; ++sgm) {
          const int t = ta + (int)(sgm * (te - ta) / segs);
          const double u0 = x.cell(bl, t, 0, 0), u1 = x.cell(bl, t, nc - 1, 0);
          const double v0 = x.cell(bl, t, 0, 1), v1 = x.cell(bl, t, nc - 1, 1);
          const int64_t j0 = x.layer(bl, t, 0), j1 = x.layer(bl, t, nc - 1);
          for (int64_t i = 0; i < runs; ++i) {
            const double f = (i + 0.5) / runs;
            mark(u0 + f * (u1 - u0), v0 + f * (v1 - v0), std::llround(j0 + f * (double)(j1 - j0)));
          }
        }
        placed += (int64_t)(te - ta) * nc;
        continue;
      }
      for (int t = ta; t < te; ++t) {
      Box b;
      int64_t prev_layer = 0, pieces = 0;
      bool prev_ok = false;
      for (int c = 0; c < nc; ++c) {
        if (!x.placeable(bl, t, c)) {
          ++out->n_excluded;
          prev_ok = false;
          continue;
        }
        const int64_t lay = x.layer(bl, t, c);
        if (!prev_ok || lay != prev_layer) ++pieces;  // a gap or a layer change starts a piece
        prev_ok = true;
        prev_layer = lay;
        b.add(x.cell(bl, t, c, 0), x.cell(bl, t, c, 1));
        take(lay);
        ++placed;
      }
      if (pieces) {
        out->n_subgrids += pieces + (int64_t)std::floor(std::max(b.uhi - b.ulo, b.vhi - b.vlo) / comfy);
        mark(0.5 * (b.ulo + b.uhi), 0.5 * (b.vlo + b.vhi), prev_layer);
      }
      }
    }
  out->n_subgrids += (placed + g.max_sg_vis - 1) / g.max_sg_vis;
  // a quarter more for the groups the size cap splits (at most one in eight) and the
  // centres the midpoint sample misses
  out->n_groups = std::min<int64_t>(((int64_t)centres.size() * 5 + 3) / 4, out->n_subgrids);
}

aidg_status partition(const Geometry& g, int n_st, int nbl, int nt, int nc, const int32_t* baselines,
                      const double* uvw, const double* freqs, PartitionResult* out,
                      std::string* err) {
  if (n_st < 1 || nbl < 0 || nt < 0 || nc < 0 || (nbl && (!baselines || !uvw)) || (nc && !freqs)) {
    *err = "bad observation sizes or NULL host arrays";
    return AIDG_E_INVALID;
  }
  for (int b = 0; b < nbl; ++b) {
    const int p = baselines[2 * b], q = baselines[2 * b + 1];
    if (p < 0 || q < 0 || p >= n_st || q >= n_st) {
      *err = "baseline station index out of range";
      return AIDG_E_INVALID;
    }
  }
  for (int c = 0; c < nc; ++c)
    if (!(freqs[c] > 0) || (c && !(freqs[c] > freqs[c - 1]))) {
      *err = "frequencies must be positive and strictly increasing";
      return AIDG_E_INVALID;
    }
  for (size_t i = 0; i < (size_t)nbl * nt * 3; ++i)
    if (!std::isfinite(uvw[i])) {
      *err = "non-finite uvw";
      return AIDG_E_INVALID;
    }
  Ctx x{g, nbl, nt, nc, uvw, freqs};
  std::vector<Box> boxes;
  x.boxes = &boxes;
  out->table.clear();
  out->excluded.clear();
  out->w_step = g.w_step;
  std::vector<aidg_subgrid> sgs;
  for (int bl = 0; bl < nbl; ++bl)
    for (int ta = 0; ta < nt; ta += g.aterm_interval)
      tile(x, bl, ta, std::min(nt, ta + g.aterm_interval), 0, nc, out, &sgs, baselines);
  int64_t jmin = 0, jmax = 0;
  for (size_t i = 0; i < sgs.size(); ++i) {
    jmin = i ? std::min<int64_t>(jmin, sgs[i].wlayer) : sgs[i].wlayer;
    jmax = i ? std::max<int64_t>(jmax, sgs[i].wlayer) : sgs[i].wlayer;
  }
  for (auto& s : sgs) s.wlayer = (int32_t)(s.wlayer - jmin);
  out->jmin = jmin;
  out->jmax = jmax;
  out->table.swap(sgs);
  std::sort(out->excluded.begin(), out->excluded.end());
  if (g.strict && !out->excluded.empty()) {
    *err = "visibilities outside the grid (strict_range)";
    return AIDG_E_RANGE;
  }
  return AIDG_OK;
}

aidg_status adopt_table(const Geometry& g, int n_st, int nbl, int nt, int nc,
                        const int32_t* baselines, const aidg_subgrid* table, int64_t n_table,
                        PartitionResult* out, std::string* err) {
  out->table.assign(table, table + n_table);
  out->excluded.clear();
  std::vector<uint8_t> cover((size_t)nbl * nt * nc, 0);
  int32_t wmax = -1;
  for (int64_t i = 0; i < n_table; ++i) wmax = std::max(wmax, table[i].wlayer);
  std::vector<double> w0(wmax + 1, NAN);
  for (int64_t i = 0; i < n_table; ++i) {
    const aidg_subgrid& s = table[i];
    char msg[160];
    snprintf(msg, sizeof msg, "subgrid %lld: ", (long long)i);
    if (s.bl < 0 || s.bl >= nbl || s.st1 != baselines[2 * s.bl] || s.st2 != baselines[2 * s.bl + 1] ||
        s.st1 < 0 || s.st1 >= n_st || s.st2 < 0 || s.st2 >= n_st) {
      *err = std::string(msg) + "bad baseline or stations";
      return AIDG_E_INVALID;
    }
    if (s.nt < 1 || s.nc < 1 || s.t0 < 0 || s.c0 < 0 || s.t0 + s.nt > nt || s.c0 + s.nc > nc) {
      *err = std::string(msg) + "sub-table outside the visibility table";
      return AIDG_E_INVALID;
    }
    if (s.t0 / g.aterm_interval != (s.t0 + s.nt - 1) / g.aterm_interval ||
        s.aint != s.t0 / g.aterm_interval) {
      *err = std::string(msg) + "sub-table spans two A-term intervals";
      return AIDG_E_INVALID;
    }
    if (s.U0 - g.L / 2 < 0 || s.U0 + g.L / 2 > g.N || s.V0 - g.L / 2 < 0 || s.V0 + g.L / 2 > g.N) {
      *err = std::string(msg) + "window not on the grid";
      return AIDG_E_INVALID;
    }
    if (s.wlayer < 0 || !std::isfinite(s.w0) ||
        (!std::isnan(w0[s.wlayer]) && w0[s.wlayer] != s.w0)) {
      *err = std::string(msg) + "w-layer index without a single w0";
      return AIDG_E_INVALID;
    }
    w0[s.wlayer] = s.w0;
    if (s.vis_offset != ((int64_t)s.bl * nt + s.t0) * nc + s.c0) {
      *err = std::string(msg) + "vis_offset does not match (bl, t0, c0)";
      return AIDG_E_INVALID;
    }
    if (s.folded != 0 && (s.folded != 1 || !g.fold)) {
      *err = std::string(msg) + "folded sub-table needs a w_fold plan (folded is 0 or 1)";
      return AIDG_E_INVALID;
    }
    for (int t = s.t0; t < s.t0 + s.nt; ++t)
      for (int c = s.c0; c < s.c0 + s.nc; ++c) {
        uint8_t& k = cover[((size_t)s.bl * nt + t) * nc + c];
        if (k) {
          *err = std::string(msg) + "visibility already in another subgrid";
          return AIDG_E_INVALID;
        }
        k = 1;
      }
  }
  for (size_t k = 0; k < cover.size(); ++k)
    if (!cover[k]) out->excluded.push_back((int64_t)k);
  if (g.strict && !out->excluded.empty()) {
    *err = "table leaves visibilities out (strict_range)";
    return AIDG_E_RANGE;
  }
  out->w_step = g.w_step;
  out->jmin = 0;
  out->jmax = wmax;
  return AIDG_OK;
}

// Sub-tables with more than max_vis visibilities are cut into pieces of whole
// rows (or, for a single over-long row, channel ranges) with the same centre and
// layer; the sum over subgrids, and so the grid, is unchanged by this.
std::vector<aidg_subgrid> split_large(const std::vector<aidg_subgrid>& t, int max_vis, int nt_total,
                                      int nc_total) {
  std::vector<aidg_subgrid> out;
  out.reserve(t.size());
  for (const aidg_subgrid& s : t) {
    if ((int64_t)s.nt * s.nc <= max_vis) {
      out.push_back(s);
      continue;
    }
    if (s.nc <= max_vis) {
      const int rows = std::max(1, max_vis / s.nc);
      for (int t = 0; t < s.nt; t += rows) {
        aidg_subgrid p = s;
        p.t0 = s.t0 + t;
        p.nt = std::min(rows, s.nt - t);
        p.vis_offset = ((int64_t)p.bl * nt_total + p.t0) * nc_total + p.c0;
        out.push_back(p);
      }
    } else {
      for (int t = 0; t < s.nt; ++t)
        for (int c = 0; c < s.nc; c += max_vis) {
          aidg_subgrid p = s;
          p.t0 = s.t0 + t;
          p.nt = 1;
          p.c0 = s.c0 + c;
          p.nc = std::min(max_vis, s.nc - c);
          p.vis_offset = ((int64_t)p.bl * nt_total + p.t0) * nc_total + p.c0;
          out.push_back(p);
        }
    }
  }
  return out;
}

// One axis of the Kaiser-Bessel taper sampled at n points: f = (x - n/2) / n,
// t[x] = I0(beta sqrt(1 - (2 f)^2)) / I0(beta).  The subgrid taper takes n = L,
// the image-level correction n = N (the same function at a finer sampling).
void kaiser_bessel_axis(int n, double beta, std::vector<double>* t) {
  t->resize(n);
  const double i0b = std::cyl_bessel_i(0.0, beta);
  for (int x = 0; x < n; ++x) {
    const double f = double(x - n / 2) / n;
    (*t)[x] = std::cyl_bessel_i(0.0, beta * std::sqrt(std::max(0.0, 1.0 - 4.0 * f * f))) / i0b;
  }
}

bool image_radices(int N, int elem_bytes, ImageRadices* out) {
  if (N < 2 || N > kMaxImageN || (int64_t)N * elem_bytes > kMaxImageRowBytes) return false;
  ImageRadices r{};
  int n = N;
  // odd radices first: their lane strides spread the early passes' strided LDS writes
  // over the banks, where a stride of 4 complex values would conflict
  for (int radix : {5, 3, 4, 2}) {
    while (n % radix == 0) {
      if (r.n == kMaxImageRadices) return false;
      r.r[r.n++] = radix;
      n /= radix;
    }
  }
  if (n != 1) return false;
  *out = r;
  return true;
}

void kaiser_bessel_taper(int L, double beta, std::vector<double>* T) {
  std::vector<double> t;
  kaiser_bessel_axis(L, beta, &t);
  T->resize((size_t)L * L);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) (*T)[(size_t)y * L + x] = t[x] * t[y];
}

}  // namespace aidg
