// HIP kernels for A-term image-domain gridding on gfx950 (CDNA4).
//
// A plan orders its subgrids so that those with the same w-layer and centre form
// consecutive groups; a grouped launch covers subgrid ranges of up to 16 plans,
// with one scratch image slot per group.
//
// Gridding of a batch (Sec. 2.5 imaging, steps 2a-2c):
//   grid_dft   one workgroup per (pixel chunk, group); each lane owns 4 subgrid
//              pixels (2 in FP64) of the chunk.  For every subgrid of the group the
//              visibilities are staged in LDS, paired within each row's recurrence
//              runs of at most R channels (sums and differences of the two channels
//              symmetric about the run's centre), and read by wave broadcast; per run
//              the pairs are weighted by the real and imaginary parts of the phasor
//              steps outward from the centre (4 FMA per polarisation per pair and
//              pixel) and the sum multiplied by the phasor at the centre, seeded from
//              an FP64 phase reduced to a quarter turn (Eq. withw).  The subgrid's
//              T (-1)^(x+y) A_p^H S A_q (Sec. 3.3) is added into the group's image slot.
//   fft_add    one workgroup per (polarisation, group): Stockham FFT of the L x L
//              plane in LDS (radix 4/2/3), then (-1)^(a+b) and an atomic add onto
//              the group's window of its w-layer (Eq. shiftback).
// Degridding (prediction, step 3), the adjoint chain:
//   split_ifft one workgroup per (polarisation, group): copy the window times
//              (-1)^(a+b) into LDS (splitter), inverse FFT, store the group image.
//   degrid_dft one workgroup per subgrid; lanes own P pixels each and apply
//              T (-1)^(x+y) A_p S A_q^H to the group image once per pixel chunk.
//              The plan picks one of three forms per subgrid (Sec. 3.2, Degridder:
//              the design chosen by subgrid occupancy).  Recurrence: per row and
//              run of at most R channels, the image times the run's centre phasor
//              (seeded from FP64) is weighted by the real and imaginary parts of the
//              phasor steps outward from the centre, which gives the two channels
//              symmetric about it at once; direct: every visibility's phasor seeded
//              from FP64 (short rows); in both, for each pair of visibilities every
//              lane forms its pixels' partial sums (16 floats) and a wave-wide
//              transpose-reduction (permlane32/permlane16 swaps, a per-wave LDS area,
//              DPP) leaves each lane with one finished value; the waves' values are
//              staged in LDS and added to the output in wave order (deterministic, no
//              atomics).  Per visibility: lanes own visibilities and walk the
//              corrected image in LDS (Eq. degridder).
// A Stokes-I plan (npol = 1) keeps one grid plane: grid_dft adds (XX + YY) / 2 of the
// corrected image and fft_add transforms that plane only; split_ifft stores the group
// image as I [[1, 0], [0, 1]], which degrid_dft reads like any other.
//
// The centred DFT of Sec. 2.3 relates to a plain FFT by a checkerboard:
//   sum_{x,y} s(x,y) e^{-2 pi i [(a-L/2)(x-L/2) + (b-L/2)(y-L/2)]/L}
//     = (-1)^(a+b) FFT[(-1)^(x+y) s](a,b)     (even L),
// so the (-1)^(x+y) factor is folded into the taper table and (-1)^(a+b) into
// the adder/splitter.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "aidg_internal.h"
#include "device_common.h"

namespace aidg {
namespace {

constexpr int kThreads = 256;
// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin by
// linear workgroup index, so index b runs on XCD b % 8.
constexpr int kXcds = 8;

// Gridder work item of linear workgroup index b: (group slot, pixel chunk) such
// that all chunks of a slot share one XCD (its visibilities are fetched into one
// L2) while consecutive slots, longest first, spread over the XCDs.  The launch
// has ceil(slots / 8) * 8 * chunks workgroups; indices past the last slot exit.
template <int Chunks>
__device__ __forceinline__ void grid_work(int64_t b, int64_t* slot, int* chunk) {
  const int64_t k = b / kXcds;
  *chunk = (int)(k % Chunks);
  *slot = (k / Chunks) * kXcds + b % kXcds;
}

// Degridder subgrid slot of linear workgroup index b < n: within every full tile
// of 64, XCD x takes the 8 consecutive slots 8x..8x+7 (subgrids of one
// same-centre group then mostly share their image in one L2); a last partial
// tile maps one to one.
__device__ __forceinline__ int64_t degrid_slot(int64_t b, int64_t n) {
  return b < (n & ~int64_t(63)) ? ((b & ~int64_t(63)) | ((b & 7) << 3) | ((b >> 3) & 7)) : b;
}
// Gridder tiling: pixels per lane (PIX; a workgroup pass covers kThreads PIX pixels) and
// the waves per SIMD the register allocation aims at (W).
template <typename R> struct GridTune;
template <> struct GridTune<float> { static constexpr int PIX = 4, W = 3; };
template <> struct GridTune<double> { static constexpr int PIX = 2, W = 2; };
// Degridder tiling: NT threads per workgroup (one subgrid), P pixels per lane (NT P
// divides L^2; more pixels amortise the cross-lane reduction per visibility over more
// work) and the waves per SIMD the register allocation aims at (W).
template <int L, typename R> struct DegridTune;
template <> struct DegridTune<32, float> { static constexpr int NT = 256, P = 4, W = 4; };
template <> struct DegridTune<64, float> { static constexpr int NT = 256, P = 8, W = 2; };
template <> struct DegridTune<96, float> { static constexpr int NT = 256, P = 6, W = 3; };
template <int L> struct DegridTune<L, double> { static constexpr int NT = 256, P = 4, W = 2; };

// What a phasor seed needs of a subgrid pixel: its offsets from the centre and n - 1.
struct alignas(16) SeedPixel {
  double n1;     // n - 1
  float dx, dy;  // x - L/2, y - L/2
};

template <int L>
__device__ __forceinline__ SeedPixel pixel_at(int pix, double lstep) {
  const int x = pix % L, y = pix / L;
  const double l = (x - L / 2) * lstep, m = (y - L / 2) * lstep;
  const double r2 = l * l + m * m;
  return {-r2 / (1.0 + sqrt(1.0 - r2)), (float)(x - L / 2), (float)(y - L / 2)};
}

// Values every lane of a wave holds identically, moved to scalar registers word
// by word so that loop bounds and addresses derived from them stay wave-uniform
// (scalar branches, scalar loads of visibilities and uvw).
template <typename T>
__device__ __forceinline__ T uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "word-sized");
  int w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Read-only view of memory no kernel writes while the launch runs: wave-uniform
// loads through it become scalar loads (the scalar data cache broadcasts them).
template <typename T>
using const_view = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ const_view<T> as_const(const T* p) {
  return (const_view<T>)(uintptr_t)p;
}

// A record every lane reads from the same address: scalar loads word by word.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized");
  const_view<int> q = as_const(reinterpret_cast<const int*>(p));
  int w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(q[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Group slot of a grouped launch: the plan's parameters and its subgrid range.
struct GroupSlot {
  KernelArgs a;
  int64_t sb, se;  // subgrids [sb, se) of the group within the job's range
  const void* in;
  void* out;
  int adjoint;
};
__device__ __forceinline__ GroupSlot resolve_group(const Group& g, int64_t slot) {
  int j = 0;
  for (int i = 1; i < g.n; ++i)
    if (slot >= g.job[i].gslot_begin) j = i;
  GroupSlot r;
  r.a = load_uniform(g.job[j].args);
  const int64_t grp = g.job[j].g_first + (slot - g.job[j].gslot_begin);
  const_view<int64_t> gb = as_const(r.a.grp_begin);
  r.sb = max(gb[grp], g.job[j].sg_begin);
  r.se = min(gb[grp + 1], g.job[j].sg_end);
  r.in = uniform(g.job[j].in);
  r.out = uniform(g.job[j].out);
  r.adjoint = uniform(g.job[j].adjoint);
  return r;
}

// Subgrid slot of a grouped launch (degridder): parameters, subgrid and the
// scratch slot holding its group's image.
struct Slot {
  KernelArgs a;
  SubgridDev s;
  int64_t img_slot;
  const void* in;
  void* out;
};
__device__ __forceinline__ Slot resolve(const Group& g, int64_t slot) {
  int j = 0;
  for (int i = 1; i < g.n; ++i)
    if (slot >= g.job[i].slot_begin) j = i;
  Slot r;
  r.a = load_uniform(g.job[j].args);
  r.s = load_uniform(r.a.sg + g.job[j].sg_begin + (slot - g.job[j].slot_begin));
  r.img_slot = g.job[j].gslot_begin + (r.s.group - g.job[j].g_first);
  r.in = uniform(g.job[j].in);
  r.out = uniform(g.job[j].out);
  return r;
}

// ------------------------------------------------------------------ gridder

// Channel runs of the phasor recurrence in a row of nc channels with re-seeding interval
// R.  R = 1 (also what a sub-table without a common channel spacing carries): runs of
// one channel.  Otherwise nr = ceil(nc / R') runs, R' = R rounded down to even, of M
// channels each, M the smallest even length with nr M >= nc (so M <= R'); the last run
// covers the rest.  A run [j0, je) with H = ceil((je - j0) / 2) pairs up its channels
// symmetrically about its centre j0 + H - 1/2: channels j0 + H - 1 - k and j0 + H + k,
// at -(k + 1/2) and +(k + 1/2) channel steps from it; a run of odd length ends on a
// padding channel (j0 + 2 H - 1 = je), which takes no part.
__device__ __forceinline__ int run_length(int nc, int R) {
  if (R <= 1) return 1;
  const int Rs = R & ~1, nr = (nc + Rs - 1) / Rs;
  return 2 * ((nc + 2 * nr - 1) / (2 * nr));
}

// Phasors of the (de)gridder: exp(2 pi i theta) with the phase theta in turns.  A run's
// centre phasor (used once per run of channels) comes from the transcendental unit;
// the half step, which the channel recurrence raises to odd powers up to R - 1, from
// the Taylor form, scaled to unit magnitude: the unit's error varies smoothly with the
// angle, so pixels with nearby step angles share it and k steps add it up coherently
// (measured on the MWA-like workload at R = 32 with the earlier one-sided recurrence:
// 7.9e-7 normwise against 3.0e-7 with Taylor steps), where the Taylor form's FP32
// rounding is uncorrelated between pixels.
__device__ __forceinline__ float2 tphasor(double theta, float) { return phasor_turns(theta); }
__device__ __forceinline__ double2 tphasor(double theta, double) { return phasor(theta, 0.0); }
__device__ __forceinline__ float2 sphasor(double theta, float) { return unit_step(phasor(theta, 0.0f)); }
__device__ __forceinline__ double2 sphasor(double theta, double) { return phasor(theta, 0.0); }

template <int L, typename R>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(GridTune<R>::W)))
void grid_dft(const Group g) {
  using V2 = typename C2<R>::T;
  using V4 = typename C4<R>::T;
  constexpr int kPix = GridTune<R>::PIX, kChunk = kThreads * kPix;
  extern __shared__ unsigned char smem_raw[];
  V4* vlds = reinterpret_cast<V4*>(smem_raw);  // one subgrid's visibilities, 8 values each
  int64_t local;
  int chunk;
  grid_work<(L * L) / kChunk>(blockIdx.x, &local, &chunk);
  if (local >= g.total_grp) return;  // padding of the last XCD round (whole workgroup)
  const GroupSlot gs = resolve_group(g, local);
  const KernelArgs& a = gs.a;
  const R* __restrict__ vis = reinterpret_cast<const R*>(gs.in);
  R* __restrict__ scratch = reinterpret_cast<R*>(g.scratch);
  // Inverse A-term mode: the planes are B = (A^-1)^H, so that B_p^H S B_q is
  // A_p^-1 S A_q^-H, scaled by 1 / ||B_p^H B_q||_F (Sec. 3.3)
  const bool inv = a.ainvh != nullptr;
  const V2* At = reinterpret_cast<const V2*>(inv ? a.ainvh : a.aterms);

  // The group's image, sum over its subgrids of T (-1)^(x+y) A_p^H S A_q, builds up
  // in its scratch slot; each lane owns its pixels there, so it reads back only
  // what it wrote itself (keeping the sum out of registers keeps occupancy).
  const R* taper = reinterpret_cast<const R*>(a.taper);
  V2* out = reinterpret_cast<V2*>(scratch) + local * 4 * L * L;

  for (int64_t si = gs.sb; si < gs.se; ++si) {
    const SubgridDev s = load_uniform(a.sg + si);
    __syncthreads();  // the previous subgrid's visibilities are no longer read
    // Pixel coordinates are recomputed per subgrid from an opaque copy of the lane
    // index: cheaper than holding them (and what derives from them) in registers
    // across the subgrid loop, which would cost occupancy.
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    SeedPixel px[kPix];
#pragma unroll
    for (int p = 0; p < kPix; ++p) px[p] = pixel_at<L>(chunk * kChunk + p * kThreads + lane, a.lstep);

    // Stage the sub-table (rows of nc visibilities, coalesced) in LDS; every lane then
    // reads each staged value by a broadcast LDS load into vector registers, so the
    // accumulation FMAs take only VGPR operands and can dual-issue.  Channels pair up
    // within the recurrence runs (run_length): a pair's low channel holds
    // P = V_hi + V_lo and its high channel Q = i (V_hi - V_lo); the low channel of a run
    // of odd length that has no partner keeps V_lo.
    const int nv = s.nt * s.nc;
    const int M = run_length(s.nc, s.R);
    for (int i = threadIdx.x; i < 2 * nv; i += kThreads) {
      const int k = i >> 1, row = k / s.nc, c = k - row * s.nc;
      // half i & 1 of visibility (row, j): polarisations 2 (i & 1) and 2 (i & 1) + 1
      auto fetch = [&](int j) -> V4 {
        const V4* src = reinterpret_cast<const V4*>(vis) + (s.vis0 + (int64_t)row * a.nc_total + j) * 2;
        if (s.fold) {
          // folded sub-table: stage V^H = [[conj XX, conj YX], [conj XY, conj YY]]
          const V4 h0 = src[0], h1 = src[1];
          return (i & 1) ? V4{h0.z, -h0.w, h1.z, -h1.w} : V4{h0.x, -h0.y, h1.x, -h1.y};
        }
        return src[i & 1];
      };
      const int j0 = c / M * M, je = min(s.nc, j0 + M), Hr = (je - j0 + 1) / 2;
      const int partner = j0 + 2 * Hr - 1 - (c - j0);
      const V4 mine = fetch(c);
      if (partner < je) {
        const V4 other = fetch(partner);
        const bool hi = c - j0 >= Hr;
        const V4 vh = hi ? mine : other, vl = hi ? other : mine;
        vlds[i] = hi ? V4{vl.y - vh.y, vh.x - vl.x, vl.w - vh.w, vh.z - vl.z} : vh + vl;
      } else {
        vlds[i] = mine;
      }
    }
    R acc[kPix][8];
#pragma unroll
    for (int p = 0; p < kPix; ++p)
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[p][i] = 0;
    __syncthreads();

    // Per row and run, with E(x) = exp(2 pi i x), d the per-channel phase step and
    // e_k = E((k + 1/2) d): the run's channels H + k and H - 1 - k add
    // V_hi e_k + V_lo conj(e_k) = P Re e_k + Q Im e_k (real multipliers: 16 FMA per
    // pixel for two visibilities) to H_run, and e_k steps by E(d) outward from the
    // centre in both directions at once (a recurrence along the channels in place of the
    // per-visibility sine and cosine of Sec. 3.2).
    // H_run times E(theta_c), the phasor at the run's centre frequency seeded from FP64,
    // goes into the accumulator.
    const double u0 = (s.U0 - a.N / 2) * a.du, v0 = (s.V0 - a.N / 2) * a.du;
    for (int t = 0; t < s.nt; ++t) {
      const_view<double> uvw = as_const(a.uvw + 3 * (s.uvw0 + t));
      const double um = uvw[0], vm = uvw[1], wm = uvw[2];
      const V4* vrow = vlds + 2 * t * s.nc;
      // the phasors' phases in turns: cu l + cv m + cw n1
      auto seed = [&](V2 (&ph)[kPix], double cu, double cv, double cw, auto step) {
        const double ku = cu * a.lstep, kv = cv * a.lstep;
#pragma unroll
        for (int p = 0; p < kPix; ++p) {
          const double th = fma(ku, (double)px[p].dx, fma(kv, (double)px[p].dy, cw * px[p].n1));
          ph[p] = decltype(step)::value ? sphasor(th, R()) : tphasor(th, R());
        }
      };
      auto load = [&](int j, R (&vv)[8]) {
        const V4 va = vrow[2 * j], vb = vrow[2 * j + 1];
        vv[0] = va.x; vv[1] = va.y; vv[2] = va.z; vv[3] = va.w;
        vv[4] = vb.x; vv[5] = vb.y; vv[6] = vb.z; vv[7] = vb.w;
      };
      V2 hs[kPix], st[kPix];  // E(d / 2) and E(d)
      seed(hs, 0.5 * um * s.dfc, 0.5 * vm * s.dfc, 0.5 * wm * s.dfc, std::true_type());
#pragma unroll
      for (int p = 0; p < kPix; ++p) st[p] = unit_step(cmul<R>(hs[p], hs[p]));
      for (int j0 = 0; j0 < s.nc; j0 += M) {
        // a run of n channels: centre j0 + H - 1/2, n / 2 full pairs and, for odd n, the
        // low channel j0 alone at the last step
        const int n = min(s.nc, j0 + M) - j0, H = (n + 1) / 2, Hf = n / 2;
        V2 h[kPix][4];
        // pair (j0 + H - 1 - k, j0 + H + k) with phasor e_k; `first` starts H_run
        auto pair = [&](auto first, int k, const V2 (&e)[kPix]) {
          R pv[8], qv[8];
          load(j0 + H - 1 - k, pv);
          load(j0 + H + k, qv);
#pragma unroll
          for (int p = 0; p < kPix; ++p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if constexpr (decltype(first)::value) {
                h[p][q].x = pv[2 * q] * e[p].x;
                h[p][q].y = pv[2 * q + 1] * e[p].x;
              } else {
                h[p][q].x = fma(pv[2 * q], e[p].x, h[p][q].x);
                h[p][q].y = fma(pv[2 * q + 1], e[p].x, h[p][q].y);
              }
              h[p][q].x = fma(qv[2 * q], e[p].y, h[p][q].x);
              h[p][q].y = fma(qv[2 * q + 1], e[p].y, h[p][q].y);
            }
          }
        };
        // the low channel j0 of a run of odd length alone: V_lo conj(e_k)
        auto single = [&](auto first, const V2 (&e)[kPix]) {
          R pv[8];
          load(j0, pv);
#pragma unroll
          for (int p = 0; p < kPix; ++p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if constexpr (decltype(first)::value) {
                h[p][q].x = pv[2 * q] * e[p].x;
                h[p][q].y = pv[2 * q + 1] * e[p].x;
              } else {
                h[p][q].x = fma(pv[2 * q], e[p].x, h[p][q].x);
                h[p][q].y = fma(pv[2 * q + 1], e[p].x, h[p][q].y);
              }
              h[p][q].x = fma(pv[2 * q + 1], e[p].y, h[p][q].x);
              h[p][q].y = fma(-pv[2 * q], e[p].y, h[p][q].y);
            }
          }
        };
        if (Hf == 0) {
          single(std::true_type(), hs);
        } else {
          pair(std::true_type(), 0, hs);
          // e_k = e_{k-1} E(d), two steps per iteration (alternating registers)
          V2 e[kPix], f[kPix];
#pragma unroll
          for (int p = 0; p < kPix; ++p) e[p] = cmul<R>(hs[p], st[p]);
          int k = 1;
          for (; k + 1 < Hf; k += 2) {
            pair(std::false_type(), k, e);
#pragma unroll
            for (int p = 0; p < kPix; ++p) f[p] = cmul<R>(e[p], st[p]);
            pair(std::false_type(), k + 1, f);
#pragma unroll
            for (int p = 0; p < kPix; ++p) e[p] = cmul<R>(f[p], st[p]);
          }
          if (k < Hf) {
            pair(std::false_type(), k, e);
            if (n & 1) {
#pragma unroll
              for (int p = 0; p < kPix; ++p) f[p] = cmul<R>(e[p], st[p]);
              single(std::false_type(), f);
            }
          } else if (n & 1) {
            single(std::false_type(), e);
          }
        }
        const double fcc = as_const(a.fc)[s.c0 + j0] + (H - 0.5) * s.dfc;
        V2 ph[kPix];
        seed(ph, um * fcc - u0, vm * fcc - v0, wm * fcc - s.w0, std::false_type());
#pragma unroll
        for (int p = 0; p < kPix; ++p) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[p][2 * q] = fma(h[p][q].x, ph[p].x, acc[p][2 * q]);
            acc[p][2 * q] = fma(-h[p][q].y, ph[p].y, acc[p][2 * q]);
            acc[p][2 * q + 1] = fma(h[p][q].x, ph[p].y, acc[p][2 * q + 1]);
            acc[p][2 * q + 1] = fma(h[p][q].y, ph[p].x, acc[p][2 * q + 1]);
          }
        }
      }
    }

    // Jones correction of this subgrid, A_p^H S A_q, one plane per polarisation,
    // tapered and added to the group's image
#pragma unroll
    for (int p = 0; p < kPix; ++p) {
      const int pix = chunk * kChunk + p * kThreads + lane;
      const V2* Ap = At + ((int64_t)s.ap * L * L + pix) * 4;
      const V2* Aq = At + ((int64_t)s.aq * L * L + pix) * 4;
      V2 a0 = Ap[0], a1 = Ap[1], a2 = Ap[2], a3 = Ap[3];
      a0.y = -a0.y; a1.y = -a1.y; a2.y = -a2.y; a3.y = -a3.y;  // conj
      const V2 b0 = Aq[0], b1 = Aq[1], b2 = Aq[2], b3 = Aq[3];
      const V2 s0 = {acc[p][0], acc[p][1]}, s1 = {acc[p][2], acc[p][3]};
      const V2 s2 = {acc[p][4], acc[p][5]}, s3 = {acc[p][6], acc[p][7]};
      // A_p^H = [[conj a0, conj a2], [conj a1, conj a3]]
      const V2 t0 = cmul<R>(a0, s0) + cmul<R>(a2, s2);
      const V2 t1 = cmul<R>(a0, s1) + cmul<R>(a2, s3);
      const V2 t2 = cmul<R>(a1, s0) + cmul<R>(a3, s2);
      const V2 t3 = cmul<R>(a1, s1) + cmul<R>(a3, s3);
      R w = taper[pix];
      if (inv) {
        // ||B_p^H B_q||_F^2 with B_p^H = [[a0, a2], [a1, a3]] (a already conjugated)
        const V2 m0 = cmul<R>(a0, b0) + cmul<R>(a2, b2), m1 = cmul<R>(a0, b1) + cmul<R>(a2, b3);
        const V2 m2 = cmul<R>(a1, b0) + cmul<R>(a3, b2), m3 = cmul<R>(a1, b1) + cmul<R>(a3, b3);
        const R n2 = m0.x * m0.x + m0.y * m0.y + m1.x * m1.x + m1.y * m1.y + m2.x * m2.x + m2.y * m2.y +
                     m3.x * m3.x + m3.y * m3.y;
        w = n2 > (R)0 ? w / sqrt(n2) : (R)0;
      }
      V2 c[4] = {(cmul<R>(t0, b0) + cmul<R>(t1, b2)) * w, (cmul<R>(t0, b1) + cmul<R>(t1, b3)) * w,
                 (cmul<R>(t2, b0) + cmul<R>(t3, b2)) * w, (cmul<R>(t2, b1) + cmul<R>(t3, b3)) * w};
      if (a.npol == 1) {  // Stokes-I grid: I = (XX + YY) / 2 of the corrected image
        V2 ci = (c[0] + c[3]) * (gs.adjoint ? (R)1 : (R)0.5);
        if (si != gs.sb) ci += out[pix];
        out[pix] = ci;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (si != gs.sb) c[q] += out[q * L * L + pix];
          out[q * L * L + pix] = c[q];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ subgrid FFT

template <int L> struct Radices;
template <> struct Radices<32> { static constexpr int n = 3, r[4] = {4, 4, 2, 1}; };
template <> struct Radices<64> { static constexpr int n = 3, r[4] = {4, 4, 4, 1}; };
template <> struct Radices<96> { static constexpr int n = 4, r[4] = {4, 4, 2, 3}; };

constexpr int pitch(int L) { return L + 1; }

// One Stockham pass (radix R, NS = product of earlier radices) over every line of
// the plane held in LDS; lines are rows (stride 1) or columns (stride L+1).
template <int L, int R, int NS, int DIR, bool ROWS, typename V2>
__device__ __forceinline__ void stockham_pass(V2* buf, const V2* tw) {
  constexpr int NB = L / R, TOTAL = L * NB, PER = (TOTAL + kThreads - 1) / kThreads;
  constexpr int TSTEP = L / (NS * R);
  V2 v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kThreads;
    if (b < TOTAL) {
      const int line = ROWS ? b / NB : b % L, j = ROWS ? b % NB : b / L;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int idx = j + q * NB;
        v[i][q] = buf[ROWS ? line * pitch(L) + idx : idx * pitch(L) + line];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kThreads;
    if (b < TOTAL) {
      const int line = ROWS ? b / NB : b % L, j = ROWS ? b % NB : b / L;
      const int k = j % NS;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        V2 w = tw[(k * q * TSTEP) % L];
        if (DIR > 0) w.y = -w.y;
        v[i][q] = {v[i][q].x * w.x - v[i][q].y * w.y, v[i][q].x * w.y + v[i][q].y * w.x};
      }
      butterfly<V2, R, DIR>(v[i]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int idx = base + q * NS;
        buf[ROWS ? line * pitch(L) + idx : idx * pitch(L) + line] = v[i][q];
      }
    }
  }
  __syncthreads();
}

template <int L, int DIR, bool ROWS, typename V2>
__device__ __forceinline__ void fft_lines(V2* buf, const V2* tw) {
  using Rd = Radices<L>;
  constexpr int r0 = Rd::r[0], r1 = Rd::r[1], r2 = Rd::r[2], r3 = Rd::r[3];
  stockham_pass<L, r0, 1, DIR, ROWS>(buf, tw);
  stockham_pass<L, r1, r0, DIR, ROWS>(buf, tw);
  stockham_pass<L, r2, r0 * r1, DIR, ROWS>(buf, tw);
  if constexpr (Rd::n == 4) stockham_pass<L, r3, r0 * r1 * r2, DIR, ROWS>(buf, tw);
}

template <int L, typename R>
__global__ __launch_bounds__(kThreads) void fft_add(const Group g) {
  using V2 = typename C2<R>::T;
  __shared__ V2 buf[L * pitch(L)];
  __shared__ V2 tw[L];
  const int pol = blockIdx.x;
  const int64_t local = blockIdx.y;
  const GroupSlot gs = resolve_group(g, local);
  const KernelArgs& a = gs.a;
  if (pol >= a.npol) return;  // a Stokes-I plan has one plane (whole workgroup)
  const SubgridDev s = load_uniform(a.sg + gs.sb);  // centre and w-layer of the group
  R* grid = reinterpret_cast<R*>(gs.out);
  const V2* in = reinterpret_cast<const V2*>(g.scratch) + (local * 4 + pol) * L * L;
  for (int e = threadIdx.x; e < L * L; e += kThreads) buf[(e / L) * pitch(L) + e % L] = in[e];
  for (int e = threadIdx.x; e < L; e += kThreads) tw[e] = reinterpret_cast<const V2*>(a.twiddle)[e];
  __syncthreads();
  fft_lines<L, -1, true>(buf, tw);
  fft_lines<L, -1, false>(buf, tw);
  R* win = grid + 2 * ((((int64_t)s.wlayer * a.npol + pol) * a.N + (s.V0 - L / 2)) * a.N + (s.U0 - L / 2));
  for (int e = threadIdx.x; e < L * L; e += kThreads) {
    const int b = e / L, c = e % L;
    V2 val = buf[b * pitch(L) + c];
    if ((b + c) & 1) val = -val;
    R* dst = win + 2 * ((int64_t)b * a.N + c);
    unsafeAtomicAdd(dst, val.x);
    unsafeAtomicAdd(dst + 1, val.y);
  }
}

template <int L, typename R>
__global__ __launch_bounds__(kThreads) void split_ifft(const Group g) {
  using V2 = typename C2<R>::T;
  __shared__ V2 buf[L * pitch(L)];
  __shared__ V2 tw[L];
  const int pol = blockIdx.x;
  const int64_t local = blockIdx.y;
  const GroupSlot gs = resolve_group(g, local);
  const KernelArgs& a = gs.a;
  R* __restrict__ scratch = reinterpret_cast<R*>(g.scratch);
  V2* out = reinterpret_cast<V2*>(scratch) + (local * 4 + pol) * L * L;
  // A Stokes-I plan stores its group image as [[I, 0], [0, I]]: planes 0 and 3 are the
  // transform of the one grid plane, planes 1 and 2 zero (whole workgroups).
  const bool stokes = a.npol == 1;
  if (stokes && (pol == 1 || pol == 2)) {
    for (int e = threadIdx.x; e < L * L; e += kThreads) out[e] = V2{0, 0};
    return;
  }
  const int gp = stokes ? 0 : pol;  // grid plane
  const SubgridDev s = load_uniform(a.sg + gs.sb);  // centre and w-layer of the group
  const R* __restrict__ grid = reinterpret_cast<const R*>(gs.in);
  const V2* win = reinterpret_cast<const V2*>(grid) +
                  (((int64_t)s.wlayer * a.npol + gp) * a.N + (s.V0 - L / 2)) * a.N + (s.U0 - L / 2);
  for (int e = threadIdx.x; e < L * L; e += kThreads) {
    const int b = e / L, c = e % L;
    V2 val = win[(int64_t)b * a.N + c];
    if ((b + c) & 1) val = -val;
    buf[b * pitch(L) + c] = val;
  }
  for (int e = threadIdx.x; e < L; e += kThreads) tw[e] = reinterpret_cast<const V2*>(a.twiddle)[e];
  __syncthreads();
  fft_lines<L, +1, true>(buf, tw);
  fft_lines<L, +1, false>(buf, tw);
  // the adjoint of the Stokes-I reduction (XX + YY) / 2 expands I to diag(I, I) / 2
  const R scale = stokes && gs.adjoint ? (R)0.5 : (R)1;
  for (int e = threadIdx.x; e < L * L; e += kThreads) out[e] = buf[(e / L) * pitch(L) + e % L] * scale;
}

// ------------------------------------------------------------------ degridder

__device__ __forceinline__ void swap32(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ void swap32(double& x, double& y) {
  float xl = __uint_as_float((unsigned)__double_as_longlong(x));
  float xh = __uint_as_float((unsigned)(__double_as_longlong(x) >> 32));
  float yl = __uint_as_float((unsigned)__double_as_longlong(y));
  float yh = __uint_as_float((unsigned)(__double_as_longlong(y) >> 32));
  swap32(xl, yl);
  swap32(xh, yh);
  x = __longlong_as_double(((long long)__float_as_uint(xh) << 32) | __float_as_uint(xl));
  y = __longlong_as_double(((long long)__float_as_uint(yh) << 32) | __float_as_uint(yl));
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  float xl = __uint_as_float((unsigned)__double_as_longlong(x));
  float xh = __uint_as_float((unsigned)(__double_as_longlong(x) >> 32));
  float yl = __uint_as_float((unsigned)__double_as_longlong(y));
  float yh = __uint_as_float((unsigned)(__double_as_longlong(y) >> 32));
  swap16(xl, yl);
  swap16(xh, yh);
  x = __longlong_as_double(((long long)__float_as_uint(xh) << 32) | __float_as_uint(xl));
  y = __longlong_as_double(((long long)__float_as_uint(yh) << 32) | __float_as_uint(yl));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int kDppXor2 = 0x4E, kDppXor1 = 0xB1;  // quad_perm [2,3,0,1] and [1,0,3,2]
constexpr int kDppRowMirror = 0x140;      // lane c of a row of 16 reads lane 15 - c
constexpr int kDppRowHalfMirror = 0x141;  // lane c of a half row of 8 reads lane 7 - c

// Degridder channel blocks: the waves' reduced values of up to kChanBlock channels of a
// row meet in LDS and are added to the output in a fixed order once per block.
constexpr int kChanBlock = 32;
// LDS row pitch (elements) of the reduction area: 68 puts the four rows of 16 lanes on
// different banks for both the 16-byte stores and the strided loads.
constexpr int kRedPitch = 68;


template <int L, typename R>
constexpr size_t degrid_lds_bytes() {
  using D = DegridTune<L, R>;
  return (size_t)D::NT * D::P * sizeof(SeedPixel)               // the lanes' pixels
         + (size_t)(D::NT / 64) * 4 * kRedPitch * sizeof(R)     // per-wave reduction areas
         + (size_t)2 * (D::NT / 64) * kChanBlock * 8 * sizeof(R)  // double-buffered stage
         + (size_t)D::NT * D::P * sizeof(typename C2<R>::T);     // the pixels' half steps
}

// Sum 16 per-lane values over the 64 lanes of a wave.  Two permlane swap levels in
// registers leave lane (r, c) = (ln >> 4, ln & 15) with partials of values 4 r + i,
// i < 4, each over the four lanes c + 16 k.  In FP32 the 16 partials of each value then
// meet in the wave's LDS area (private to the wave, whose LDS operations complete in
// issue order; the wave barriers keep the compiler from moving this call's stores above
// the previous call's loads, or its loads above its stores), four per lane.  In FP64
// two more exchange levels stay in registers (DPP row mirrors: lanes c and 15 - c split
// the row's four values, c < 8 keeping values 0 and 1, then lanes c and 7 - c of each
// half split the pair), which measured 5 % faster there and 5 % slower in FP32.  A quad
// DPP sum finishes.  On return lane ln holds the full sum of value
// 4 (ln >> 4) + ((ln & 15) >> 2) (the four lanes of a quad agree).
template <typename R>
__device__ __forceinline__ R reduce16(R (&a)[16], int ln, R* area) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap32(a[i], a[i + 8]);
    a[i] = a[i] + a[i + 8];  // lanes 0-31: value i, lanes 32-63: value i + 8
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap16(a[i], a[i + 4]);
    a[i] = a[i] + a[i + 4];  // row r of 16 lanes: value i + 4 r
  }
  const int r = ln >> 4, c = ln & 15;
  R v;
  if constexpr (sizeof(R) == 8) {
    const bool lo8 = c < 8, lo4 = (c & 4) == 0;
    const R k0 = lo8 ? a[0] : a[2], s0 = lo8 ? a[2] : a[0];
    const R k1 = lo8 ? a[1] : a[3], s1 = lo8 ? a[3] : a[1];
    const R b0 = k0 + dpp<kDppRowMirror>(s0), b1 = k1 + dpp<kDppRowMirror>(s1);
    v = (lo4 ? b0 : b1) + dpp<kDppRowHalfMirror>(lo4 ? b1 : b0);
  } else {
    __builtin_amdgcn_wave_barrier();
    R* w = area + r * kRedPitch + 4 * c;
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = a[i];
    __builtin_amdgcn_wave_barrier();
    const R* src = area + r * kRedPitch + 16 * (c & 3) + (c >> 2);
    v = (src[0] + src[4]) + (src[8] + src[12]);
  }
  v = v + dpp<kDppXor1>(v);
  return v + dpp<kDppXor2>(v);
}


// The degridder's prologue at one subgrid pixel: S' = T (-1)^(x+y) A_p S A_q^H of the
// group image S (Sec. 3.3, A-term application; the taper table carries the
// checkerboard), and what a phase needs of the pixel (its offsets from the centre and
// n - 1).
template <int L, typename R>
__device__ __forceinline__ void corrected_pixel(const KernelArgs& a, const SubgridDev& s,
                                                const typename C2<R>::T* img, int pix,
                                                typename C2<R>::T (&sp)[4], SeedPixel& px) {
  using V2 = typename C2<R>::T;
  px = pixel_at<L>(pix, a.lstep);
  const V2* At = reinterpret_cast<const V2*>(a.aterms);
  const V2* Ap = At + ((int64_t)s.ap * L * L + pix) * 4;
  const V2* Aq = At + ((int64_t)s.aq * L * L + pix) * 4;
  const V2 a0 = Ap[0], a1 = Ap[1], a2 = Ap[2], a3 = Ap[3];
  V2 b0 = Aq[0], b1 = Aq[1], b2 = Aq[2], b3 = Aq[3];
  b0.y = -b0.y; b1.y = -b1.y; b2.y = -b2.y; b3.y = -b3.y;  // conj
  const V2 s0 = img[0 * L * L + pix], s1 = img[1 * L * L + pix];
  const V2 s2 = img[2 * L * L + pix], s3 = img[3 * L * L + pix];
  const V2 t0 = cmul<R>(a0, s0) + cmul<R>(a1, s2);
  const V2 t1 = cmul<R>(a0, s1) + cmul<R>(a1, s3);
  const V2 t2 = cmul<R>(a2, s0) + cmul<R>(a3, s2);
  const V2 t3 = cmul<R>(a2, s1) + cmul<R>(a3, s3);
  const R w = reinterpret_cast<const R*>(a.taper)[pix];
  // A_q^H = [[conj b0, conj b2], [conj b1, conj b3]]
  sp[0] = (cmul<R>(t0, b0) + cmul<R>(t1, b1)) * w;
  sp[1] = (cmul<R>(t0, b2) + cmul<R>(t1, b3)) * w;
  sp[2] = (cmul<R>(t2, b0) + cmul<R>(t3, b1)) * w;
  sp[3] = (cmul<R>(t2, b2) + cmul<R>(t3, b3)) * w;
}

// Output element i (= 8 x channel offset + component) of a degridded row: a folded
// sub-table returns the conjugate transpose of its prediction at -uvw.
template <typename R>
__device__ __forceinline__ void store_vis(R* vrow, int i, R v, bool fold, bool add) {
  int d = i;
  if (fold) {
    const int comp = i & 7, pol = comp >> 1;
    d = i - comp + (pol == 1 ? 2 : pol == 2 ? 1 : pol) * 2 + (comp & 1);
    if (comp & 1) v = -v;
  }
  vrow[d] = add ? vrow[d] + v : v;
}

// Pixels per LDS chunk of the per-visibility form: the corrected image (4 values) and
// the pixel record of each, within the LDS the cooperative form takes, a multiple of
// the workgroup size.
template <int L, typename R>
constexpr int pervis_chunk() {
  using D = DegridTune<L, R>;
  constexpr int per_pixel = (int)(4 * sizeof(typename C2<R>::T) + sizeof(SeedPixel));
  constexpr int n = (int)(degrid_lds_bytes<L, R>() / per_pixel) / D::NT * D::NT;
  return n < L * L ? n : L * L;
}

// Per-visibility form of the degridder, for sparse subgrids (Sec. 3.2, Degridder: the
// kernel design chosen per subgrid by its occupancy).  The cooperative form below puts
// pixels on lanes, so each row of a sub-table costs two FP64-seeded phasors per pixel
// and each visibility a cross-lane reduction; with a few channels per row those fixed
// costs dominate.  Here lanes own visibilities: the nv = nt nc visibilities of the
// subgrid (nv <= NT, which the plan guarantees for the subgrids it marks) take
// G = floor(NT / nv) lanes each, lane (k, g) summing over the pixels g, g + G, ... of
// every LDS chunk of the corrected image.  Each (visibility, pixel) phase is formed in
// FP64 from the pixel's offsets and n - 1, reduced to a turn and turned into a phasor
// by the transcendental unit (no recurrence, so no seeds).  The G partial sums of a
// visibility meet in LDS and are added in slice order, so the result does not depend
// on timing.
template <int L, typename R>
__device__ __forceinline__ void degrid_pervis(const KernelArgs& a, const SubgridDev& s,
                                              const typename C2<R>::T* img, R* vis,
                                              unsigned char* smem) {
  using V2 = typename C2<R>::T;
  constexpr int NT = DegridTune<L, R>::NT, CHV = pervis_chunk<L, R>();
  static_assert(CHV >= NT && CHV % NT == 0 && (L * L) % NT == 0, "per-visibility chunks");
  static_assert(NT * 8 * sizeof(R) <= degrid_lds_bytes<L, R>(), "partial sums fit the LDS");
  V2* simg = reinterpret_cast<V2*>(smem);                              // [CHV][4]
  SeedPixel* spx = reinterpret_cast<SeedPixel*>(smem + CHV * 4 * sizeof(V2));  // [CHV]
  R* part = reinterpret_cast<R*>(smem);                                // [NT][8], after the chunks
  const int nv = s.nt * s.nc;
  const int G = NT / nv;
  const int k = threadIdx.x / G, gi = threadIdx.x - k * G;
  const bool active = k < nv;
  const int t = active ? k / s.nc : 0, j = active ? k - t * s.nc : 0;
  // phase of exp(-2 pi i phi) in turns: -(c_u dx lstep + c_v dy lstep + c_w n1)
  double ku = 0, kv = 0, kw = 0;
  if (active) {
    const_view<double> uvw = as_const(a.uvw + 3 * (s.uvw0 + t));
    const double fc = as_const(a.fc)[s.c0 + j];
    const double u0 = (s.U0 - a.N / 2) * a.du, v0 = (s.V0 - a.N / 2) * a.du;
    ku = -(uvw[0] * fc - u0) * a.lstep;
    kv = -(uvw[1] * fc - v0) * a.lstep;
    kw = -(uvw[2] * fc - s.w0);
  }
  R acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0;
  for (int c0 = 0; c0 < L * L; c0 += CHV) {
    const int n = min(CHV, L * L - c0);  // a multiple of NT (L^2 and CHV are)
    __syncthreads();  // the previous chunk is no longer read
    // all of a lane's pixels of the chunk at once, so that their loads overlap
#pragma unroll
    for (int r = 0; r < CHV / NT; ++r) {
      const int i = r * NT + threadIdx.x;
      if (r * NT < n) {
        V2 sp[4];
        corrected_pixel<L, R>(a, s, img, c0 + i, sp, spx[i]);
#pragma unroll
        for (int q = 0; q < 4; ++q) simg[4 * i + q] = sp[q];
      }
    }
    __syncthreads();
    if (active) {
      // U pixels per step with independent phase chains; pixels past the chunk take
      // the chunk's last pixel with a zero phasor
      constexpr int U = 4;
      for (int i = gi; i < n; i += U * G) {
        SeedPixel px[U];
        V2 sv[U][4];
        R keep[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int ii = min(i + u * G, n - 1);
          keep[u] = i + u * G < n ? R(1) : R(0);
          px[u] = spx[ii];
#pragma unroll
          for (int q = 0; q < 4; ++q) sv[u][q] = simg[4 * ii + q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          V2 ph = tphasor(fma(ku, (double)px[u].dx, fma(kv, (double)px[u].dy, kw * px[u].n1)), R());
          ph.x *= keep[u];
          ph.y *= keep[u];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const V2 v = sv[u][q];
            acc[2 * q] = fma(v.x, ph.x, acc[2 * q]);
            acc[2 * q] = fma(-v.y, ph.y, acc[2 * q]);
            acc[2 * q + 1] = fma(v.x, ph.y, acc[2 * q + 1]);
            acc[2 * q + 1] = fma(v.y, ph.x, acc[2 * q + 1]);
          }
        }
      }
    }
  }
  __syncthreads();  // the last chunk is no longer read: its LDS takes the partial sums
#pragma unroll
  for (int i = 0; i < 8; ++i) part[threadIdx.x * 8 + i] = acc[i];
  __syncthreads();
  for (int o = threadIdx.x; o < nv * 8; o += NT) {
    const int kk = o >> 3, comp = o & 7;
    R v = part[kk * G * 8 + comp];
    for (int q = 1; q < G; ++q) v = v + part[(kk * G + q) * 8 + comp];
    const int tt = kk / s.nc, jj = kk - tt * s.nc;
    store_vis(vis + (s.vis0 + (int64_t)tt * a.nc_total + jj) * 8, comp, v, s.fold != 0, false);
  }
}

template <int L, typename R>
__global__ __launch_bounds__((DegridTune<L, R>::NT))
__attribute__((amdgpu_waves_per_eu(DegridTune<L, R>::W))) void degrid_dft(const Group g) {
  using V2 = typename C2<R>::T;
  constexpr int NT = DegridTune<L, R>::NT, P = DegridTune<L, R>::P, CH = NT * P, NW = NT / 64;
  static_assert((L * L) % CH == 0, "pixel chunks must tile the subgrid");
  extern __shared__ unsigned char smem_raw[];
  SeedPixel* pxt = reinterpret_cast<SeedPixel*>(smem_raw);           // [CH]
  R* red = reinterpret_cast<R*>(smem_raw + CH * sizeof(SeedPixel));  // [NW][4][kRedPitch]
  R* stage = red + NW * 4 * kRedPitch;                               // [2][NW][kChanBlock][8]
  V2* hst = reinterpret_cast<V2*>(stage + 2 * NW * kChanBlock * 8);  // [P][NT]
  const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
  R* area = red + wave * 4 * kRedPitch;
  const int64_t local = degrid_slot(blockIdx.x, g.total_sg);
  const Slot sl = resolve(g, local);
  const KernelArgs& a = sl.a;
  const SubgridDev& s = sl.s;
  const R* __restrict__ scratch = reinterpret_cast<const R*>(g.scratch);
  R* __restrict__ vis = reinterpret_cast<R*>(sl.out);
  const V2* img = reinterpret_cast<const V2*>(scratch) + sl.img_slot * 4 * L * L;
  if (s.kind == kDegridPerVis) {
    degrid_pervis<L, R>(a, s, img, vis, smem_raw);
    return;
  }
  const double u0 = (s.U0 - a.N / 2) * a.du, v0 = (s.V0 - a.N / 2) * a.du;
  // recurrence runs of the rows (a sub-table without a common channel spacing takes the
  // direct form); the result of a run's padding channel is dropped
  const int M = run_length(s.nc, s.R);
  // the value this lane owns after reduce16, and whether it stores it
  const int vidx = 4 * (ln >> 4) + ((ln & 15) >> 2);
  const bool owner = (ln & 3) == 0;
  int buf = 0;

  for (int chunk = 0; chunk < (L * L) / CH; ++chunk) {
    // the pixels' offsets from the centre and n - 1 go to the lane's own LDS entries
    V2 sp[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int pix = chunk * CH + p * NT + threadIdx.x;
      corrected_pixel<L, R>(a, s, img, pix, sp[p], pxt[p * NT + threadIdx.x]);
    }
    // -(c_u dx lstep + c_v dy lstep + c_w n1): the phase of exp(-2 pi i phi) in turns
    auto seed = [&](V2 (&ph)[P], double cu, double cv, double cw, auto step) {
      const double ku = -cu * a.lstep, kv = -cv * a.lstep, kw = -cw;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        // an opaque index keeps the compiler from hoisting the load and conversions out
        // of the row loop (which would hold 6 registers per pixel across it)
        int e = p * NT + threadIdx.x;
        asm volatile("" : "+v"(e));
        const SeedPixel q = pxt[e];
        const double th = fma(ku, (double)q.dx, fma(kv, (double)q.dy, kw * q.n1));
        ph[p] = decltype(step)::value ? sphasor(th, R()) : tphasor(th, R());
      }
    };
    // Partial sums of two visibilities over the lane's pixels, S'_q ph0 and S'_q ph1
    // (16 values), reduced across the wave: the lane's share of the pair (see reduce16).
    auto pair_value = [&](const V2 (&ph0)[P], const V2 (&ph1)[P]) -> R {
      R part[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        part[2 * q] = sp[0][q].x * ph0[0].x - sp[0][q].y * ph0[0].y;
        part[2 * q + 1] = sp[0][q].x * ph0[0].y + sp[0][q].y * ph0[0].x;
        part[8 + 2 * q] = sp[0][q].x * ph1[0].x - sp[0][q].y * ph1[0].y;
        part[8 + 2 * q + 1] = sp[0][q].x * ph1[0].y + sp[0][q].y * ph1[0].x;
      }
#pragma unroll
      for (int p = 1; p < P; ++p) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          part[2 * q] = fma(sp[p][q].x, ph0[p].x, part[2 * q]);
          part[2 * q] = fma(-sp[p][q].y, ph0[p].y, part[2 * q]);
          part[2 * q + 1] = fma(sp[p][q].x, ph0[p].y, part[2 * q + 1]);
          part[2 * q + 1] = fma(sp[p][q].y, ph0[p].x, part[2 * q + 1]);
          part[8 + 2 * q] = fma(sp[p][q].x, ph1[p].x, part[8 + 2 * q]);
          part[8 + 2 * q] = fma(-sp[p][q].y, ph1[p].y, part[8 + 2 * q]);
          part[8 + 2 * q + 1] = fma(sp[p][q].x, ph1[p].y, part[8 + 2 * q + 1]);
          part[8 + 2 * q + 1] = fma(sp[p][q].y, ph1[p].x, part[8 + 2 * q + 1]);
        }
      }
      return reduce16<R>(part, ln, area);
    };
    // The waves' values of a block of up to kChanBlock visibilities (staged in `stage`),
    // summed in wave order and added to the output (assigned by the first pixel chunk);
    // each output element has one owner thread, the same in every chunk.  out(k) is the
    // output row of the block's visibility k.
    auto flush_block = [&](int n_in_block, auto out) {
      __syncthreads();
      const R* sb = stage + buf * NW * kChanBlock * 8;
      for (int i = threadIdx.x; i < n_in_block * 8; i += NT) {
        R v = sb[i];
#pragma unroll
        for (int w = 1; w < NW; ++w) v = v + sb[w * kChanBlock * 8 + i];
        store_vis(out(i >> 3), i & 7, v, s.fold != 0, chunk != 0);
      }
      buf ^= 1;
    };
    if (s.kind == kDegridDirect) {
      // Direct form (short rows, or channels without a common spacing): the nv = nt nc
      // visibilities in row-major order, two per step, each with its own FP64-seeded
      // phasor: no per-row step seed and no padding of odd rows
      const int nv = s.nt * s.nc;
      auto direct = [&](V2 (&ph)[P], int k) {
        const int t = k / s.nc, j = k - t * s.nc;
        const_view<double> uvw = as_const(a.uvw + 3 * (s.uvw0 + t));
        const double fc = as_const(a.fc)[s.c0 + j];
        seed(ph, uvw[0] * fc - u0, uvw[1] * fc - v0, uvw[2] * fc - s.w0, std::false_type());
      };
      for (int kb0 = 0; kb0 < nv; kb0 += kChanBlock) {
        const int kbn = min(kChanBlock, nv - kb0);
        R* stg = stage + (buf * NW + wave) * kChanBlock * 8;
        for (int k = kb0; k < kb0 + kbn; k += 2) {
          V2 ph0[P], ph1[P];
          direct(ph0, k);
          direct(ph1, min(k + 1, nv - 1));  // an odd last visibility repeats, dropped
          const R val = pair_value(ph0, ph1);
          const int kc = k - kb0 + (vidx >> 3);
          if (owner && k + (vidx >> 3) < nv) stg[kc * 8 + (vidx & 7)] = val;
        }
        flush_block(kbn, [&](int kc) {
          const int k = kb0 + kc, t = k / s.nc, j = k - t * s.nc;
          return vis + (s.vis0 + (int64_t)t * a.nc_total + j) * 8;
        });
      }
      continue;
    }
    // Recurrence form, channels paired about the run centre: with E(x) = exp(2 pi i x),
    // theta_c the phase at the run's centre frequency and d the per-channel phase step,
    // channel H + k of the run sees X E((k + 1/2) d) and channel H - 1 - k sees
    // X E(-(k + 1/2) d), where X = S' E(theta_c).  So with e_k = E((k + 1/2) d), the
    // sums A = sum X Re e_k and B = sum X Im e_k (real multipliers: 16 FMA per pixel for
    // two visibilities) give both, A + iB and A - iB, and e_k steps by E(d) outward from
    // the centre in both directions at once (a recurrence along the channels in place of
    // the per-visibility sine and cosine of Sec. 3.2).  E(theta_c) is seeded from FP64
    // per run, E(d / 2) per row.
    for (int t = 0; t < s.nt; ++t) {
      const_view<double> uvw = as_const(a.uvw + 3 * (s.uvw0 + t));
      const double um = uvw[0], vm = uvw[1], wm = uvw[2];
      V2 st[P];  // E(d)
      {
        V2 hs[P];  // E(d / 2), the first e_k of every run, kept in the lane's LDS entries
        seed(hs, 0.5 * um * s.dfc, 0.5 * vm * s.dfc, 0.5 * wm * s.dfc, std::true_type());
#pragma unroll
        for (int p = 0; p < P; ++p) {
          hst[p * NT + threadIdx.x] = hs[p];
          st[p] = unit_step(cmul<R>(hs[p], hs[p]));
        }
      }
      R* vrow = vis + (s.vis0 + (int64_t)t * a.nc_total) * 8;
      for (int j0 = 0; j0 < s.nc; j0 += M) {
        const int je = min(s.nc, j0 + M), H = (je - j0 + 1) / 2;
        const double fcc = as_const(a.fc)[s.c0 + j0] + (H - 0.5) * s.dfc;
        V2 X[P][4];
        {
          V2 ec[P];
          seed(ec, um * fcc - u0, vm * fcc - v0, wm * fcc - s.w0, std::false_type());
#pragma unroll
          for (int p = 0; p < P; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) X[p][q] = cmul<R>(sp[p][q], ec[p]);
        }
        V2 e[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          int ix = p * NT + threadIdx.x;
          asm volatile("" : "+v"(ix));
          e[p] = hst[ix];
        }
        for (int k0 = 0; k0 < H; k0 += kChanBlock / 2) {
          const int kn = min(kChanBlock / 2, H - k0);
          R* stg = stage + (buf * NW + wave) * kChanBlock * 8;
          // A (values 0-7) and B (8-15) of the lane's pixels for phasors e, reduced
          auto pair_sym = [&](const V2 (&e)[P]) -> R {
            R part[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              part[2 * q] = X[0][q].x * e[0].x;
              part[2 * q + 1] = X[0][q].y * e[0].x;
              part[8 + 2 * q] = X[0][q].x * e[0].y;
              part[8 + 2 * q + 1] = X[0][q].y * e[0].y;
            }
#pragma unroll
            for (int p = 1; p < P; ++p) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                part[2 * q] = fma(X[p][q].x, e[p].x, part[2 * q]);
                part[2 * q + 1] = fma(X[p][q].y, e[p].x, part[2 * q + 1]);
                part[8 + 2 * q] = fma(X[p][q].x, e[p].y, part[8 + 2 * q]);
                part[8 + 2 * q + 1] = fma(X[p][q].y, e[p].y, part[8 + 2 * q + 1]);
              }
            }
            return reduce16<R>(part, ln, area);
          };
          // two pairs per iteration, the phasor steps alternating between e and f
          int k = 0;
          for (; k + 1 < kn; k += 2) {
            V2 f[P];
            const R v0 = pair_sym(e);
#pragma unroll
            for (int p = 0; p < P; ++p) f[p] = cmul<R>(e[p], st[p]);
            const R v1 = pair_sym(f);
#pragma unroll
            for (int p = 0; p < P; ++p) e[p] = cmul<R>(f[p], st[p]);
            if (owner) {
              stg[k * 16 + vidx] = v0;
              stg[(k + 1) * 16 + vidx] = v1;
            }
          }
          if (k < kn) {
            const R v0 = pair_sym(e);
#pragma unroll
            for (int p = 0; p < P; ++p) e[p] = cmul<R>(e[p], st[p]);
            if (owner) stg[k * 16 + vidx] = v0;
          }
          // the waves' A and B of the block's pairs, summed in wave order, combined
          // into the two channels of each pair and added to the output
          __syncthreads();
          const R* sb = stage + buf * NW * kChanBlock * 8;
          for (int i = threadIdx.x; i < kn * 16; i += NT) {
            const int slot = i >> 4, hi = (i >> 3) & 1, comp = i & 7, im = comp & 1;
            const int jj = j0 + (hi ? H + k0 + slot : H - 1 - k0 - slot);
            if (jj >= je) continue;  // padding channel of a run of odd length
            const int ia = slot * 16 + comp, ib = slot * 16 + 8 + (comp ^ 1);
            R va = sb[ia], vb = sb[ib];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
              va = va + sb[w * kChanBlock * 8 + ia];
              vb = vb + sb[w * kChanBlock * 8 + ib];
            }
            // channel H + k: A + iB; channel H - 1 - k: A - iB
            store_vis(vrow + jj * 8, comp, hi == im ? va + vb : va - vb, s.fold != 0, chunk != 0);
          }
          buf ^= 1;
        }
      }
    }
  }
}

template <typename R>
__global__ void zero_vis(const int64_t* __restrict__ idx, int64_t n, R* vis) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * 8) vis[idx[i / 8] * 8 + i % 8] = 0;
}

template <int L, typename R>
int launch_one(KernelClass k, const Group& g, hipStream_t st, int max_nv) {
  const unsigned n = (unsigned)(k == kDegridDft ? g.total_sg : g.total_grp);
  switch (k) {
    case kGridDft:
      hipLaunchKernelGGL((grid_dft<L, R>), dim3((n + kXcds - 1) / kXcds * kXcds * ((L * L) / (kThreads * GridTune<R>::PIX))),
                         dim3(kThreads), (size_t)max_nv * 8 * sizeof(R), st, g);
      break;
    case kFftAdd:
      hipLaunchKernelGGL((fft_add<L, R>), dim3(4, n), dim3(kThreads), 0, st, g);
      break;
    case kSplitIfft:
      hipLaunchKernelGGL((split_ifft<L, R>), dim3(4, n), dim3(kThreads), 0, st, g);
      break;
    case kDegridDft: {
      constexpr int nt = DegridTune<L, R>::NT;
      constexpr size_t lds = degrid_lds_bytes<L, R>();
      hipLaunchKernelGGL((degrid_dft<L, R>), dim3(n), dim3(nt), lds, st, g);
      break;
    }
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace

namespace {
template <typename R>
int degrid_lanes(int L) {
  return L == 32 ? DegridTune<32, R>::NT : L == 64 ? DegridTune<64, R>::NT : DegridTune<96, R>::NT;
}
}  // namespace

int32_t degrid_form(const Geometry& g, int nt, int nc, bool uniform) {
  const int nv = nt * nc;
  const int lanes = g.precision == AIDG_FP32 ? degrid_lanes<float>(g.L) : degrid_lanes<double>(g.L);
  const bool pv_ok = nv >= 1 && nv <= lanes;
  if (!uniform && g.degrid_form != AIDG_DEGRID_PER_VIS) return kDegridDirect;
  switch (g.degrid_form) {
    case AIDG_DEGRID_RECURRENCE: return kDegridRecur;
    case AIDG_DEGRID_DIRECT: return kDegridDirect;
    case AIDG_DEGRID_PER_VIS: return pv_ok ? kDegridPerVis : uniform ? kDegridRecur : kDegridDirect;
    default: break;
  }
  // Automatic: the recurrence or the direct form, whichever has the smaller modelled
  // cost per subgrid pixel: the recurrence pays per visibility of its rows (odd rows
  // padded to even) and a fixed cost per row (kRow visibilities: the row's seeded
  // phasors and block bookkeeping), the direct form kDirect per visibility (one seeded
  // phasor each; an odd sub-table padded).  On the MWA-like observation with every k-th
  // channel kept (k = 1 ... 96, L = 32, 64, 96), fits of the degridder's times put a
  // directly seeded visibility at 3.5 to 4.6 visibilities of the paired recurrence and a
  // run at 4 to 13.  By those fits the constants below choose within 2 % of the best
  // pair on a grid over both, and the automatic choice measured within 1 % of the faster
  // single form, or faster, at every k.  Rows of one to three channels take the direct
  // form.  The per-visibility form measured slower than the direct form at every
  // occupancy and is never chosen automatically.
  constexpr double kRow = 2.0, kDirect = 1.95;
  const double recur = (double)nt * ((nc + (nc & 1)) + kRow);
  const double direct = kDirect * (nv + (nv & 1));
  return direct < recur ? kDegridDirect : kDegridRecur;
}

int launch_group(KernelClass k, int L, int precision, const Group& g, void* stream, int max_nv) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (g.total_sg <= 0) return 0;
  if (g.n < 1 || g.n > kMaxGroup || g.total_grp < 1 || g.total_grp > 65535 || g.total_grp > g.total_sg)
    return (int)hipErrorInvalidValue;
  if (precision == AIDG_FP32) {
    switch (L) {
      case 32: return launch_one<32, float>(k, g, st, max_nv);
      case 64: return launch_one<64, float>(k, g, st, max_nv);
      case 96: return launch_one<96, float>(k, g, st, max_nv);
    }
  } else {
    switch (L) {
      case 32: return launch_one<32, double>(k, g, st, max_nv);
      case 64: return launch_one<64, double>(k, g, st, max_nv);
      case 96: return launch_one<96, double>(k, g, st, max_nv);
    }
  }
  return (int)hipErrorInvalidValue;
}

int launch_zero_vis(int precision, const int64_t* idx, int64_t n, void* vis, void* stream) {
  if (n <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t threads = n * 8;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  if (precision == AIDG_FP32)
    hipLaunchKernelGGL(zero_vis<float>, dim3(blocks), dim3(256), 0, st, idx, n,
                       reinterpret_cast<float*>(vis));
  else
    hipLaunchKernelGGL(zero_vis<double>, dim3(blocks), dim3(256), 0, st, idx, n,
                       reinterpret_cast<double*>(vis));
  return (int)hipGetLastError();
}

}  // namespace aidg
