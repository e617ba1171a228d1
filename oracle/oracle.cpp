// FP64 CPU oracle for A-term image-domain gridding (IDG) and degridding.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
// calls this file; only the tests, the smoke check and the bench's CPU-baseline
// leg load it.  It is deliberately plain and slow: every step is a direct sum in
// double precision, in the order the paper states it, with no FFT library and no
// blocking beyond what the equations themselves allow.
//
// Conventions (paper Sec. 2; where the paper is silent, the choice is stated here or at
// the function that makes it):
//   grid of N x N cells, cell (gu, gv) at u = (gu - N/2) du, du = 1 / (N dl)
//   subgrid of L x L cells centred on integer grid cell (U0, V0): u0 = (U0 - N/2) du
//   subgrid image pixel (x, y) at l = (x - L/2) FOV / L, FOV = N dl
//   n1 = sqrt(1 - l^2 - m^2) - 1
//   phase (turns) phi_k(x, y) = (u_k - u0) l + (v_k - v0) m + (w_k - w0) n1
//   u_k = u_metres[bl][t] * f_c / c     (likewise v, w)
//   2x2 Jones / visibilities stored row-major [[XX, XY], [YX, YY]]
//   V_pq = A_p B A_q^H (measurement equation, Sec. 2.1 Eq. 1 in Jones form)
//
// Complex arrays are interleaved (re, im) doubles, i.e. numpy complex128.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cd = std::complex<double>;
constexpr double kSpeedOfLight = 299792458.0;
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

// One subgrid record, as exchanged with the tests through a numpy structured
// array (64 bytes).  bl/st1/st2: baseline and its stations; [t0, t0+nt) x
// [c0, c0+nc): the visibility sub-table; (U0, V0): integer centre cell;
// wlayer/w0: w-layer index and its w value in wavelengths; aint: A-term
// interval; folded: the sub-table is gridded at (-u, -v, -w) by the Hermitian
// symmetry V(-u,-v,-w) = V(u,v,w)^H (Sec. 2.4 footnote): its visibilities enter
// conjugate-transposed and the A-terms of st2 stand on the left; vis_offset: flat
// index of visibility (bl, t0, c0).
struct Subgrid {
  int32_t bl, st1, st2, t0, nt, c0, nc, U0, V0, wlayer, aint, folded;
  double w0;
  int64_t vis_offset;
};
static_assert(sizeof(Subgrid) == 64, "subgrid record is 64 bytes");

struct Mat2 {
  cd a[4];
};

inline Mat2 load_mat(const double* p) {
  Mat2 m;
  for (int i = 0; i < 4; ++i) m.a[i] = cd(p[2 * i], p[2 * i + 1]);
  return m;
}
inline void store_mat(double* p, const Mat2& m) {
  for (int i = 0; i < 4; ++i) {
    p[2 * i] = m.a[i].real();
    p[2 * i + 1] = m.a[i].imag();
  }
}
inline void add_mat(double* p, const Mat2& m) {
  for (int i = 0; i < 4; ++i) {
    p[2 * i] += m.a[i].real();
    p[2 * i + 1] += m.a[i].imag();
  }
}
inline Mat2 mul(const Mat2& x, const Mat2& y) {
  Mat2 r;
  r.a[0] = x.a[0] * y.a[0] + x.a[1] * y.a[2];
  r.a[1] = x.a[0] * y.a[1] + x.a[1] * y.a[3];
  r.a[2] = x.a[2] * y.a[0] + x.a[3] * y.a[2];
  r.a[3] = x.a[2] * y.a[1] + x.a[3] * y.a[3];
  return r;
}
inline Mat2 herm(const Mat2& x) {  // conjugate transpose
  Mat2 r;
  r.a[0] = std::conj(x.a[0]);
  r.a[1] = std::conj(x.a[2]);
  r.a[2] = std::conj(x.a[1]);
  r.a[3] = std::conj(x.a[3]);
  return r;
}
inline Mat2 scale(const Mat2& x, cd s) {
  Mat2 r;
  for (int i = 0; i < 4; ++i) r.a[i] = x.a[i] * s;
  return r;
}
inline Mat2 zero_mat() {
  Mat2 r;
  for (int i = 0; i < 4; ++i) r.a[i] = cd(0.0, 0.0);
  return r;
}
// Inverse of a 2x2 matrix, adj(x) / det(x); the zero matrix when det(x) = 0.
inline Mat2 inverse(const Mat2& x) {
  const cd det = x.a[0] * x.a[3] - x.a[1] * x.a[2];
  if (det == cd(0.0, 0.0)) return zero_mat();
  Mat2 r;
  r.a[0] = x.a[3] / det;
  r.a[1] = -x.a[1] / det;
  r.a[2] = -x.a[2] / det;
  r.a[3] = x.a[0] / det;
  return r;
}
inline double frobenius(const Mat2& x) {
  double s = 0.0;
  for (int i = 0; i < 4; ++i) s += std::norm(x.a[i]);
  return std::sqrt(s);
}

// exp(2 pi i phi) for a phase in turns, reduced to [-1/2, 1/2] first.
inline cd turns_phasor(double phi) {
  const double r = phi - std::nearbyint(phi);
  return cd(std::cos(kTwoPi * r), std::sin(kTwoPi * r));
}

inline double n_minus_one(double l, double m) {
  const double r2 = l * l + m * m;
  return -r2 / (1.0 + std::sqrt(1.0 - r2));
}

// Kaiser-Bessel taper of one axis: I0(beta sqrt(1 - (2f)^2)) / I0(beta),
// f = (x - L/2) / L in [-1/2, 1/2).
inline double kb(int x, int L, double beta) {
  const double f = (x - L / 2) / double(L);
  const double s = std::max(0.0, 1.0 - 4.0 * f * f);
  return std::cyl_bessel_i(0.0, beta * std::sqrt(s)) / std::cyl_bessel_i(0.0, beta);
}

struct Problem {
  int N, L, K;
  int fold;             // fold rows with w < 0 to -uvw (w >= 0 layers at odd multiples)
  int amode;            // gridding A-term: 0 A_p^H . A_q, 1 normalised A_p^-1 . A_q^-H (Sec. 3.3)
  double dl, fov, du, beta;
  int n_st, nbl, nt, nc, aterm_interval, n_int;
  const int32_t* baselines;
  const double* uvw;    // [nbl][nt][3]
  const double* freqs;  // [nc]
  const double* aterms; // complex [n_int][n_st][L][L][4]

  double lpix(int x) const { return (x - L / 2) * (fov / L); }
  const double* aterm(int interval, int st, int x, int y) const {
    return aterms + 2 * 4 * ((((size_t)interval * n_st + st) * L + y) * L + x);
  }
  double taper(int x, int y) const { return kb(x, L, beta) * kb(y, L, beta); }
};

Problem make_problem(int N, int L, int K, double dl, double beta, int n_st, int nbl, int nt, int nc,
                     int aterm_interval, int n_int, const int32_t* baselines, const double* uvw,
                     const double* freqs, const double* aterms) {
  Problem p;
  p.N = N;
  p.L = L;
  p.K = K;
  p.dl = dl;
  p.fov = N * dl;
  p.du = 1.0 / p.fov;
  p.beta = beta > 0 ? beta : M_PI * K / 4.0;
  p.n_st = n_st;
  p.nbl = nbl;
  p.nt = nt;
  p.nc = nc;
  p.aterm_interval = aterm_interval;
  p.n_int = n_int;
  p.baselines = baselines;
  p.uvw = uvw;
  p.freqs = freqs;
  p.aterms = aterms;
  p.fold = 0;
  p.amode = 0;
  return p;
}

// ---------------------------------------------------------------- gridding steps

// Normalisation factor of the inverse A-term mode at one pixel (Sec. 3.3, A-term
// application): 1 / ||A_p^-1 (A_q^-1)^H||_F, and 0 where the product vanishes (a
// singular A-term).
double inverse_norm_factor(const Mat2& Ap, const Mat2& Aq) {
  const double n = frobenius(mul(inverse(Ap), herm(inverse(Aq))));
  return n > 0.0 ? 1.0 / n : 0.0;
}

// G1 + G2 (Sec. 2.4 Eq. withw with the A-term deferred as in Sec. 3.3):
//   S(x,y)  = sum_k V_k exp(+2 pi i phi_k(x,y))
//   S'(x,y) = T(x,y) A_p(x,y)^H S(x,y) A_q(x,y)                       (amode 0)
//   S'(x,y) = T(x,y) f(x,y) A_p(x,y)^-1 S(x,y) A_q(x,y)^-H,
//             f = 1 / ||A_p^-1 A_q^-H||_F                               (amode 1)
// stage 1 returns S, stage 2 returns S'.  out: complex [4][L][L].
void subgrid_image(const Problem& P, const Subgrid& s, const double* vis, int stage, double* out) {
  const int L = P.L;
  const double u0 = (s.U0 - P.N / 2) * P.du, v0 = (s.V0 - P.N / 2) * P.du;
  const double sg = s.folded ? -1.0 : 1.0;  // folded: the visibility enters at -uvw as V^H
  std::vector<Mat2> S((size_t)L * L, zero_mat());
  for (int y = 0; y < L; ++y) {
    const double m = P.lpix(y);
    for (int x = 0; x < L; ++x) {
      const double l = P.lpix(x);
      const double n1 = n_minus_one(l, m);
      Mat2 acc = zero_mat();
      for (int t = s.t0; t < s.t0 + s.nt; ++t) {
        const double* um = P.uvw + 3 * ((size_t)s.bl * P.nt + t);
        for (int c = s.c0; c < s.c0 + s.nc; ++c) {
          const double f = P.freqs[c] / kSpeedOfLight;
          const double phi =
              (sg * um[0] * f - u0) * l + (sg * um[1] * f - v0) * m + (sg * um[2] * f - s.w0) * n1;
          const cd ph = turns_phasor(phi);
          Mat2 V = load_mat(vis + 8 * (((size_t)s.bl * P.nt + t) * P.nc + c));
          if (s.folded) V = herm(V);
          for (int i = 0; i < 4; ++i) acc.a[i] += V.a[i] * ph;
        }
      }
      S[(size_t)y * L + x] = acc;
    }
  }
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      Mat2 r = S[(size_t)y * L + x];
      if (stage >= 2) {
        const Mat2 Ap = load_mat(P.aterm(s.aint, s.folded ? s.st2 : s.st1, x, y));
        const Mat2 Aq = load_mat(P.aterm(s.aint, s.folded ? s.st1 : s.st2, x, y));
        if (P.amode == 1) {
          const double f = inverse_norm_factor(Ap, Aq);
          r = scale(mul(mul(inverse(Ap), r), herm(inverse(Aq))), cd(P.taper(x, y) * f, 0.0));
        } else {
          r = scale(mul(mul(herm(Ap), r), Aq), cd(P.taper(x, y), 0.0));
        }
      }
      for (int pol = 0; pol < 4; ++pol) {
        double* o = out + 2 * (((size_t)pol * L + y) * L + x);
        o[0] = r.a[pol].real();
        o[1] = r.a[pol].imag();
      }
    }
}

// Centred, unnormalised 2-D DFT of one L x L plane, done as two direct 1-D sums
// (over x, then over y):  out(a,b) = sum_{x,y} in(x,y) exp(sign 2 pi i [(a-L/2)(x-L/2) + (b-L/2)(y-L/2)] / L)
void centred_dft2(int L, int sign, const cd* in, cd* out) {
  std::vector<cd> W(L);
  for (int k = 0; k < L; ++k) W[k] = cd(std::cos(kTwoPi * k / L), sign * std::sin(kTwoPi * k / L));
  auto tw = [&](int a, int x) {
    long long e = (long long)(a - L / 2) * (x - L / 2);
    e %= L;
    if (e < 0) e += L;
    return W[(size_t)e];
  };
  std::vector<cd> tmp((size_t)L * L);
  for (int y = 0; y < L; ++y)
    for (int a = 0; a < L; ++a) {
      cd acc(0.0, 0.0);
      for (int x = 0; x < L; ++x) acc += in[(size_t)y * L + x] * tw(a, x);
      tmp[(size_t)y * L + a] = acc;
    }
  for (int b = 0; b < L; ++b)
    for (int a = 0; a < L; ++a) {
      cd acc(0.0, 0.0);
      for (int y = 0; y < L; ++y) acc += tmp[(size_t)y * L + a] * tw(b, y);
      out[(size_t)b * L + a] = acc;
    }
}

// G3 (Sec. 2.5, step 2b): forward (exp -) centred DFT of each polarisation plane.
void subgrid_uv(const Problem& P, const Subgrid& s, const double* vis, double* out) {
  const int L = P.L;
  std::vector<double> img((size_t)4 * L * L * 2);
  subgrid_image(P, s, vis, 2, img.data());
  for (int pol = 0; pol < 4; ++pol) {
    const cd* in = reinterpret_cast<const cd*>(img.data()) + (size_t)pol * L * L;
    cd* o = reinterpret_cast<cd*>(out) + (size_t)pol * L * L;
    centred_dft2(L, -1, in, o);
  }
}

// ---------------------------------------------------------------- partition helpers

struct Cells {
  double gu, gv, w;
};

// -1 for a row that the fold moves to -uvw (fold mode and w < 0), else +1.
inline double row_sign(const Problem& P, int bl, int t) {
  return P.fold && P.uvw[3 * ((size_t)bl * P.nt + t) + 2] < 0 ? -1.0 : 1.0;
}

// Grid cells and w of a visibility, after the fold of its row.
inline Cells cells_of(const Problem& P, int bl, int t, int c) {
  const double* um = P.uvw + 3 * ((size_t)bl * P.nt + t);
  const double f = row_sign(P, bl, t) * P.freqs[c] / kSpeedOfLight;
  return {um[0] * f / P.du + P.N / 2, um[1] * f / P.du + P.N / 2, um[2] * f};
}

// A single visibility can be placed in some subgrid iff it lies at least K/2
// cells inside the grid edge (its subgrid window must lie inside the grid).
inline bool placeable(const Problem& P, const Cells& c) {
  const double lo = P.K / 2.0, hi = P.N - P.K / 2.0;
  return c.gu >= lo && c.gu <= hi && c.gv >= lo && c.gv <= hi;
}

// Layer j of w: nearest j w_step; with the fold (w >= 0) the layers sit at odd
// multiples of w_step / 2 (Sec. 2.4: {w_max, 3 w_max, ...}), j = floor(w / w_step).
inline long long layer_of(double w, double w_step, int fold) {
  if (w_step <= 0) return 0;
  return fold ? (long long)std::floor(w / w_step) : (long long)std::nearbyint(w / w_step);
}
inline double layer_w0(long long j, double w_step, int fold) {
  return w_step > 0 ? (fold ? (j + 0.5) * w_step : j * w_step) : 0.0;
}

// Centre cell for a span [lo, hi]: nearest integer to the middle (ties down),
// clamped so that the L-cell window stays on the grid.
inline int centre_for(double lo, double hi, int L, int N) {
  const double mid = 0.5 * (lo + hi);
  int c = (int)std::floor(mid);
  if (mid - c > 0.5) c += 1;
  return std::min(std::max(c, L / 2), N - L / 2);
}

bool rect_fits(const Problem& P, int bl, int t0, int nt, int c0, int nc, double w_step, int* U0,
               int* V0, long long* layer) {
  double ulo = 1e300, uhi = -1e300, vlo = 1e300, vhi = -1e300;
  long long lay = 0;
  bool first = true;
  for (int t = t0; t < t0 + nt; ++t) {
    if (row_sign(P, bl, t) != row_sign(P, bl, t0)) return false;  // one fold state
    for (int c = c0; c < c0 + nc; ++c) {
      const Cells q = cells_of(P, bl, t, c);
      if (!placeable(P, q)) return false;
      const long long j = layer_of(q.w, w_step, P.fold);
      if (first) lay = j;
      else if (j != lay) return false;
      first = false;
      ulo = std::min(ulo, q.gu);
      uhi = std::max(uhi, q.gu);
      vlo = std::min(vlo, q.gv);
      vhi = std::max(vhi, q.gv);
    }
  }
  const double half = (P.L - P.K) / 2.0;
  const int cu = centre_for(ulo, uhi, P.L, P.N), cv = centre_for(vlo, vhi, P.L, P.N);
  if (std::max(uhi - cu, cu - ulo) > half || std::max(vhi - cv, cv - vlo) > half) return false;
  *U0 = cu;
  *V0 = cv;
  *layer = lay;
  return true;
}

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 1; }

// Separable Kaiser-Bessel taper T[y][x] on the L x L lattice (Sec. 4.2).
void oracle_taper(int L, int K, double beta, double* T) {
  const double b = beta > 0 ? beta : M_PI * K / 4.0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) T[(size_t)y * L + x] = kb(x, L, b) * kb(y, L, b);
}

// Partition every baseline's (time, channel) table into rectangular sub-tables
// that satisfy the subgrid constraints of Sec. 2.2, 2.4 and 3.3: uv within
// (L-K)/2 cells of an integer centre whose window lies on the grid, one w-layer
// (|w - w0| <= w_step/2, w0 = j w_step), one A-term interval.  With fold set,
// rows with w < 0 are taken at -uvw (Sec. 2.4 footnote), a sub-table holds rows of
// one fold state, and the layers sit at w0 = (j + 1/2) w_step for w >= 0.  This is
// the oracle's own, deliberately simple scheme (independent of the library's):
// single-row greedy channel runs, then vertical merging of identical runs while
// the merged rectangle still fits.  Returns the number of subgrids written, or
// -(needed) when cap is too small.  wlayer = j - j_min over the whole table.
int64_t oracle_partition(int N, int L, int K, double dl, int n_st, int nbl, int nt, int nc,
                         int aterm_interval, const int32_t* baselines, const double* uvw,
                         const double* freqs, double w_step, int fold, Subgrid* out, int64_t cap) {
  Problem P = make_problem(N, L, K, dl, 1.0, n_st, nbl, nt, nc, aterm_interval, 1, baselines, uvw,
                           freqs, nullptr);
  P.fold = fold;
  struct Rect {
    int bl, t0, nt, c0, nc, U0, V0;
    long long layer;
  };
  std::vector<Rect> rects;
  for (int bl = 0; bl < nbl; ++bl) {
    for (int ti = 0; ti < nt; ti += aterm_interval) {
      const int te = std::min(nt, ti + aterm_interval);
      std::vector<Rect> open;  // rectangles that end at the previous row
      for (int t = ti; t < te; ++t) {
        std::vector<Rect> runs;
        int c = 0;
        while (c < nc) {
          if (!placeable(P, cells_of(P, bl, t, c))) {
            ++c;
            continue;
          }
          Rect r{bl, t, 1, c, 1, 0, 0, 0};
          if (!rect_fits(P, bl, t, 1, c, 1, w_step, &r.U0, &r.V0, &r.layer)) {
            ++c;  // cannot happen for a placeable visibility when L - K >= 1
            continue;
          }
          int e = c + 1;
          while (e < nc) {
            Rect q = r;
            if (!rect_fits(P, bl, t, 1, c, e - c + 1, w_step, &q.U0, &q.V0, &q.layer)) break;
            r = q;
            r.nc = e - c + 1;
            ++e;
          }
          runs.push_back(r);
          c = e;
        }
        std::vector<Rect> next;
        for (Rect& r : runs) {
          bool merged = false;
          for (Rect& o : open) {
            if (o.nc < 0 || o.c0 != r.c0 || o.nc != r.nc) continue;
            Rect q = o;
            if (rect_fits(P, bl, o.t0, o.nt + 1, o.c0, o.nc, w_step, &q.U0, &q.V0, &q.layer)) {
              q.nt = o.nt + 1;
              next.push_back(q);
              o.nc = -1;  // consumed
              merged = true;
            }
            break;
          }
          if (!merged) next.push_back(r);
        }
        for (Rect& o : open)
          if (o.nc >= 0) rects.push_back(o);
        open.swap(next);
      }
      for (Rect& o : open) rects.push_back(o);
    }
  }
  if ((int64_t)rects.size() > cap) return -(int64_t)rects.size();
  long long jmin = 0;
  bool any = false;
  for (const Rect& r : rects) {
    jmin = any ? std::min(jmin, r.layer) : r.layer;
    any = true;
  }
  for (size_t i = 0; i < rects.size(); ++i) {
    const Rect& r = rects[i];
    Subgrid& s = out[i];
    std::memset(&s, 0, sizeof(s));
    s.bl = r.bl;
    s.st1 = baselines[2 * r.bl];
    s.st2 = baselines[2 * r.bl + 1];
    s.t0 = r.t0;
    s.nt = r.nt;
    s.c0 = r.c0;
    s.nc = r.nc;
    s.U0 = r.U0;
    s.V0 = r.V0;
    s.wlayer = (int32_t)(r.layer - jmin);
    s.aint = r.t0 / aterm_interval;
    s.folded = row_sign(P, r.bl, r.t0) < 0;
    s.w0 = layer_w0(r.layer, w_step, fold);
    s.vis_offset = ((int64_t)r.bl * nt + r.t0) * nc + r.c0;
  }
  return (int64_t)rects.size();
}

// Validity of any partition (whoever made it).  Returns 0 when valid, else an
// error code; *bad receives the offending subgrid (codes 1-6, 9, 10) or flat
// visibility index (codes 7, 8).
//   1 bad baseline/stations   2 sub-table outside the visibility table
//   3 spans two A-term intervals or wrong interval index
//   4 window not on the grid  5 a visibility beyond (L-K)/2 cells of the centre
//   6 a visibility beyond w_step/2 of w0, or w0 not a layer value
//   7 visibility in two subgrids   8 placeable visibility in no subgrid
//   9 one wlayer index with two w0 values   10 wrong vis_offset
//   11 fold flag not the fold state of its rows (w < 0 in fold mode), or set
//      without fold mode
int oracle_check_partition(int N, int L, int K, double dl, int n_st, int nbl, int nt, int nc,
                           int aterm_interval, const int32_t* baselines, const double* uvw,
                           const double* freqs, double w_step, int fold, const Subgrid* sg,
                           int64_t nsg, int64_t* bad) {
  Problem P = make_problem(N, L, K, dl, 1.0, n_st, nbl, nt, nc, aterm_interval, 1, baselines, uvw,
                           freqs, nullptr);
  P.fold = fold;
  const double half = (L - K) / 2.0, tol = 1e-9;
  std::vector<uint8_t> cover((size_t)nbl * nt * nc, 0);
  std::vector<std::pair<int, double>> layer_w;
  for (int64_t i = 0; i < nsg; ++i) {
    const Subgrid& s = sg[i];
    *bad = i;
    if (s.bl < 0 || s.bl >= nbl || s.st1 != baselines[2 * s.bl] || s.st2 != baselines[2 * s.bl + 1])
      return 1;
    if (s.nt < 1 || s.nc < 1 || s.t0 < 0 || s.c0 < 0 || s.t0 + s.nt > nt || s.c0 + s.nc > nc)
      return 2;
    if (s.t0 / aterm_interval != (s.t0 + s.nt - 1) / aterm_interval || s.aint != s.t0 / aterm_interval)
      return 3;
    if (s.U0 - L / 2 < 0 || s.U0 + L / 2 > N || s.V0 - L / 2 < 0 || s.V0 + L / 2 > N) return 4;
    if (w_step > 0) {
      const double j = s.w0 / w_step - (fold ? 0.5 : 0.0);
      if (std::fabs(j - std::nearbyint(j)) > 1e-9) return 6;
    } else if (s.w0 != 0.0) {
      return 6;
    }
    if (s.folded && !fold) return 11;
    bool seen = false;
    for (auto& lw : layer_w)
      if (lw.first == s.wlayer) {
        seen = true;
        if (lw.second != s.w0) return 9;
      }
    if (!seen) layer_w.push_back({s.wlayer, s.w0});
    if (s.vis_offset != ((int64_t)s.bl * nt + s.t0) * nc + s.c0) return 10;
    for (int t = s.t0; t < s.t0 + s.nt; ++t)
      for (int c = s.c0; c < s.c0 + s.nc; ++c) {
        if ((row_sign(P, s.bl, t) < 0) != (s.folded != 0)) return 11;
        const Cells q = cells_of(P, s.bl, t, c);
        if (std::fabs(q.gu - s.U0) > half + tol || std::fabs(q.gv - s.V0) > half + tol) return 5;
        if (w_step > 0 && std::fabs(q.w - s.w0) > 0.5 * w_step * (1 + 1e-12) + 1e-12) return 6;
        const size_t k = ((size_t)s.bl * nt + t) * nc + c;
        if (cover[k]) {
          *bad = (int64_t)k;
          return 7;
        }
        cover[k] = 1;
      }
  }
  for (int bl = 0; bl < nbl; ++bl)
    for (int t = 0; t < nt; ++t)
      for (int c = 0; c < nc; ++c) {
        const size_t k = ((size_t)bl * nt + t) * nc + c;
        if (!cover[k] && placeable(P, cells_of(P, bl, t, c))) {
          *bad = (int64_t)k;
          return 8;
        }
      }
  *bad = -1;
  return 0;
}

// One subgrid's intermediate results: stage 1 = S (G1), 2 = S' (G2),
// 3 = its centred uv subgrid (G3).  out: complex [4][L][L].
int oracle_grid_subgrid(int N, int L, int K, double dl, double beta, int n_st, int nbl, int nt,
                        int nc, int aterm_interval, int n_int, const int32_t* baselines,
                        const double* uvw, const double* freqs, const double* aterms,
                        const double* vis, const Subgrid* s, int stage, int amode, double* out) {
  Problem P = make_problem(N, L, K, dl, beta, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
  P.amode = amode;
  if (stage == 3) subgrid_uv(P, *s, vis, out);
  else subgrid_image(P, *s, vis, stage, out);
  return 0;
}

// IDG gridding, Sec. 2.5 steps 1-2: for each subgrid G1 (direct phasor sum),
// G2 (Jones + taper), G3 (centred forward DFT) and G4 (add at its window of its
// w-layer).  grid: complex [W][4][N][N] (u fastest), ACCUMULATED into.  Subgrid
// images are computed in parallel; the additions run serially in table order.
int oracle_grid(int N, int L, int K, double dl, double beta, int n_st, int nbl, int nt, int nc,
                int aterm_interval, int n_int, const int32_t* baselines, const double* uvw,
                const double* freqs, const double* aterms, const double* vis, const Subgrid* sg,
                int64_t nsg, int W, double* grid, int nthreads, int amode) {
  Problem P = make_problem(N, L, K, dl, beta, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
  P.amode = amode;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  const size_t per = (size_t)4 * L * L * 2;
  const int64_t chunk = 256;
  std::vector<double> buf(per * chunk);
  for (int64_t b0 = 0; b0 < nsg; b0 += chunk) {
    const int64_t b1 = std::min(nsg, b0 + chunk);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = b0; i < b1; ++i) subgrid_uv(P, sg[i], vis, buf.data() + per * (i - b0));
    for (int64_t i = b0; i < b1; ++i) {
      const Subgrid& s = sg[i];
      if (s.wlayer < 0 || s.wlayer >= W) return 1;
      const double* src = buf.data() + per * (i - b0);
      for (int pol = 0; pol < 4; ++pol)
        for (int b = 0; b < L; ++b)
          for (int a = 0; a < L; ++a) {
            const size_t g = (((size_t)s.wlayer * 4 + pol) * N + (s.V0 - L / 2 + b)) * N +
                             (s.U0 - L / 2 + a);
            const size_t q = ((size_t)pol * L + b) * L + a;
            grid[2 * g] += src[2 * q];
            grid[2 * g + 1] += src[2 * q + 1];
          }
    }
  }
  return 0;
}

// Weighted average of the inverse mode's normalisation factor over all subgrids
// (Sec. 3.3, A-term application), each subgrid weighted by its visibility count:
//   M(x,y) = sum_s nvis_s f_s(x,y) / sum_s nvis_s,  f_s = 1 / ||A_p^-1 A_q^-H||_F.
// out: [L][L] (y major), zero when the table holds no visibilities.
int oracle_aterm_norm(int N, int L, double dl, int n_st, int nbl, int nt, int nc,
                      int aterm_interval, int n_int, const int32_t* baselines, const double* uvw,
                      const double* freqs, const double* aterms, const Subgrid* sg, int64_t nsg,
                      double* out) {
  Problem P = make_problem(N, L, 0, dl, 1.0, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
  double total = 0.0;
  for (int64_t i = 0; i < nsg; ++i) total += double(sg[i].nt) * sg[i].nc;
  // each pixel sums over the subgrids in table order (rows of pixels in parallel)
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      double acc = 0.0;
      for (int64_t i = 0; i < nsg; ++i) {
        const Subgrid& s = sg[i];
        const Mat2 Ap = load_mat(P.aterm(s.aint, s.folded ? s.st2 : s.st1, x, y));
        const Mat2 Aq = load_mat(P.aterm(s.aint, s.folded ? s.st1 : s.st2, x, y));
        acc += double(s.nt) * s.nc * inverse_norm_factor(Ap, Aq);
      }
      out[(size_t)y * L + x] = total > 0.0 ? acc / total : 0.0;
    }
  return 0;
}

// IDG degridding, Sec. 2.5 prediction step 3, written as the exact adjoint of
// oracle_grid: D1 copy the window of the subgrid's w-layer, D2 centred inverse
// (exp +) unnormalised DFT, D3 S' = T A_p S A_q^H, D4 V_k = sum_{x,y} S'(x,y)
// exp(-2 pi i phi_k(x,y)).  vis_out: complex [nbl][nt][nc][4], OVERWRITTEN;
// visibilities in no subgrid are set to zero.
int oracle_degrid(int N, int L, int K, double dl, double beta, int n_st, int nbl, int nt, int nc,
                  int aterm_interval, int n_int, const int32_t* baselines, const double* uvw,
                  const double* freqs, const double* aterms, const double* grid, const Subgrid* sg,
                  int64_t nsg, int W, double* vis_out, int nthreads) {
  Problem P = make_problem(N, L, K, dl, beta, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  std::memset(vis_out, 0, sizeof(double) * 8 * (size_t)nbl * nt * nc);
  for (int64_t i = 0; i < nsg; ++i)
    if (sg[i].wlayer < 0 || sg[i].wlayer >= W) return 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nsg; ++i) {
    const Subgrid& s = sg[i];
    std::vector<cd> win((size_t)L * L), img((size_t)4 * L * L);
    for (int pol = 0; pol < 4; ++pol) {
      for (int b = 0; b < L; ++b)
        for (int a = 0; a < L; ++a) {
          const size_t g = (((size_t)s.wlayer * 4 + pol) * N + (s.V0 - L / 2 + b)) * N +
                           (s.U0 - L / 2 + a);
          win[(size_t)b * L + a] = cd(grid[2 * g], grid[2 * g + 1]);
        }
      centred_dft2(L, +1, win.data(), img.data() + (size_t)pol * L * L);
    }
    std::vector<Mat2> Sp((size_t)L * L);
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        Mat2 S;
        for (int pol = 0; pol < 4; ++pol) S.a[pol] = img[((size_t)pol * L + y) * L + x];
        const Mat2 Ap = load_mat(P.aterm(s.aint, s.folded ? s.st2 : s.st1, x, y));
        const Mat2 Aq = load_mat(P.aterm(s.aint, s.folded ? s.st1 : s.st2, x, y));
        Sp[(size_t)y * L + x] = scale(mul(mul(Ap, S), herm(Aq)), cd(P.taper(x, y), 0.0));
      }
    const double u0 = (s.U0 - N / 2) * P.du, v0 = (s.V0 - N / 2) * P.du;
    const double sg = s.folded ? -1.0 : 1.0;  // folded: predicted at -uvw, written as V^H
    for (int t = s.t0; t < s.t0 + s.nt; ++t) {
      const double* um = P.uvw + 3 * ((size_t)s.bl * nt + t);
      for (int c = s.c0; c < s.c0 + s.nc; ++c) {
        const double f = P.freqs[c] / kSpeedOfLight;
        Mat2 acc = zero_mat();
        for (int y = 0; y < L; ++y) {
          const double m = P.lpix(y);
          for (int x = 0; x < L; ++x) {
            const double l = P.lpix(x);
            const double n1 = n_minus_one(l, m);
            const double phi =
                (sg * um[0] * f - u0) * l + (sg * um[1] * f - v0) * m + (sg * um[2] * f - s.w0) * n1;
            const cd ph = std::conj(turns_phasor(phi));
            const Mat2& v = Sp[(size_t)y * L + x];
            for (int q = 0; q < 4; ++q) acc.a[q] += v.a[q] * ph;
          }
        }
        store_mat(vis_out + 8 * (((size_t)s.bl * nt + t) * nc + c), s.folded ? herm(acc) : acc);
      }
    }
  }
  return 0;
}

// Direct A-term imaging (the adjoint of Sec. 2.1 Eq. 1 in Jones form) at
// n_dir directions:  I(l,m) = sum_k A_p^H V_k A_q exp(+2 pi i [u_k l + v_k m + w_k n1]).
// A-terms are taken at lattice pixel (xs, ys) when xs >= 0, otherwise identity.
// Visibilities with mask[k] == 0 are skipped (mask may be null).
void oracle_direct_image(int N, int L, double dl, int n_st, int nbl, int nt, int nc,
                         int aterm_interval, int n_int, const int32_t* baselines, const double* uvw,
                         const double* freqs, const double* aterms, const double* vis,
                         const uint8_t* mask, int n_dir, const double* l, const double* m,
                         const int32_t* xs, const int32_t* ys, double* out, int nthreads) {
  Problem P = make_problem(N, L, 0, dl, 1.0, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int d = 0; d < n_dir; ++d) {
    const double n1 = n_minus_one(l[d], m[d]);
    Mat2 acc = zero_mat();
    for (int bl = 0; bl < nbl; ++bl) {
      const int p = baselines[2 * bl], q = baselines[2 * bl + 1];
      for (int t = 0; t < nt; ++t) {
        const int it = t / aterm_interval;
        Mat2 Ap, Aq;
        if (xs[d] >= 0) {
          Ap = load_mat(P.aterm(it, p, xs[d], ys[d]));
          Aq = load_mat(P.aterm(it, q, xs[d], ys[d]));
        } else {
          Ap = Aq = zero_mat();
          Ap.a[0] = Ap.a[3] = Aq.a[0] = Aq.a[3] = cd(1.0, 0.0);
        }
        const Mat2 ApH = herm(Ap);
        const double* um = uvw + 3 * ((size_t)bl * nt + t);
        for (int c = 0; c < nc; ++c) {
          const size_t k = ((size_t)bl * nt + t) * nc + c;
          if (mask && !mask[k]) continue;
          const double f = freqs[c] / kSpeedOfLight;
          const double phi = um[0] * f * l[d] + um[1] * f * m[d] + um[2] * f * n1;
          const Mat2 V = load_mat(vis + 8 * k);
          const Mat2 r = scale(mul(mul(ApH, V), Aq), turns_phasor(phi));
          for (int i = 0; i < 4; ++i) acc.a[i] += r.a[i];
        }
      }
    }
    store_mat(out + 8 * (size_t)d, acc);
  }
}

// Direct prediction, Sec. 2.1 Eq. 1 in Jones form:
//   V_k = sum_s A_p(s) B_s A_q(s)^H exp(-2 pi i [u_k l_s + v_k m_s + w_k n1_s]).
// A-terms at lattice pixel (xs, ys) when xs >= 0, else identity.
// B: complex [n_src][4]; vis_out: complex [nbl][nt][nc][4], overwritten.
void oracle_direct_predict(int N, int L, double dl, int n_st, int nbl, int nt, int nc,
                           int aterm_interval, int n_int, const int32_t* baselines,
                           const double* uvw, const double* freqs, const double* aterms, int n_src,
                           const double* l, const double* m, const int32_t* xs, const int32_t* ys,
                           const double* B, double* vis_out, int nthreads) {
  Problem P = make_problem(N, L, 0, dl, 1.0, n_st, nbl, nt, nc, aterm_interval, n_int, baselines,
                           uvw, freqs, aterms);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int bl = 0; bl < nbl; ++bl) {
    const int p = baselines[2 * bl], q = baselines[2 * bl + 1];
    for (int t = 0; t < nt; ++t) {
      const int it = t / aterm_interval;
      const double* um = uvw + 3 * ((size_t)bl * nt + t);
      for (int c = 0; c < nc; ++c) {
        const double f = freqs[c] / kSpeedOfLight;
        Mat2 acc = zero_mat();
        for (int s = 0; s < n_src; ++s) {
          Mat2 Ap, Aq;
          if (xs[s] >= 0) {
            Ap = load_mat(P.aterm(it, p, xs[s], ys[s]));
            Aq = load_mat(P.aterm(it, q, xs[s], ys[s]));
          } else {
            Ap = Aq = zero_mat();
            Ap.a[0] = Ap.a[3] = Aq.a[0] = Aq.a[3] = cd(1.0, 0.0);
          }
          const double n1 = n_minus_one(l[s], m[s]);
          const double phi = um[0] * f * l[s] + um[1] * f * m[s] + um[2] * f * n1;
          const Mat2 r = scale(mul(mul(Ap, load_mat(B + 8 * (size_t)s)), herm(Aq)),
                               std::conj(turns_phasor(phi)));
          for (int i = 0; i < 4; ++i) acc.a[i] += r.a[i];
        }
        store_mat(vis_out + 8 * (((size_t)bl * nt + t) * nc + c), acc);
      }
    }
  }
}

// Image of one w-layer grid at arbitrary directions (a non-uniform inverse DFT):
//   I(l,m) = sum_{gu,gv} G[gv][gu] exp(+2 pi i [(gu - N/2) du l + (gv - N/2) du m]).
// G: complex [npol][N][N]; out: complex [n_dir][npol].
void oracle_layer_image_at(const double* G, int npol, int N, double du, int n_dir, const double* l,
                           const double* m, double* out, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int d = 0; d < n_dir; ++d) {
    std::vector<cd> eu(N), ev(N);
    for (int g = 0; g < N; ++g) {
      eu[g] = turns_phasor((g - N / 2) * du * l[d]);
      ev[g] = turns_phasor((g - N / 2) * du * m[d]);
    }
    for (int pol = 0; pol < npol; ++pol) {
      cd acc(0.0, 0.0);
      for (int gv = 0; gv < N; ++gv) {
        const double* row = G + 2 * (((size_t)pol * N + gv) * N);
        cd r(0.0, 0.0);
        for (int gu = 0; gu < N; ++gu) r += cd(row[2 * gu], row[2 * gu + 1]) * eu[gu];
        acc += r * ev[gv];
      }
      out[2 * ((size_t)d * npol + pol)] = acc.real();
      out[2 * ((size_t)d * npol + pol) + 1] = acc.imag();
    }
  }
}

}  // extern "C"
