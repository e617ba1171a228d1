// HIP kernels of the image-level step: w-stacking for imaging (Sec. 2.4, Eq. wstack;
// Sec. 2.5 imaging step 3) and its adjoint for prediction (Eq. wunstack, prediction
// step 2).  A centred N x N transform is two passes of one-dimensional FFTs along
// rows with a tiled transpose between them:
//   image_fft_rows  one workgroup per row: the row times (-1)^x is transformed by
//                   mixed-radix Stockham passes through LDS (radix 4/2/3/5; FP32
//                   twiddles computed, FP64 ones from a table; the last pass writes
//                   global memory) and written back times
//                   (-1)^k.  The prediction variant first multiplies each image
//                   value by exp(-2 pi i w0 n1) / (L^2 T).
//   image_transpose 32 x 32 tiles through LDS.
//   image_wstack    a transposing tile pass that adds one layer's transform times
//                   exp(+2 pi i w0 n1) / (L^2 T) into the image (or stores it, for
//                   the first layer); in the last layer's pass of the inverse A-term
//                   mode, the sum is divided by the normalisation map's bilinear
//                   interpolation.
// For even N, (-1)^k FFT[(-1)^x a](k) is the centred transform times (-1)^(N/2); the
// sign cancels between the two passes of a plane.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "aidg_internal.h"
#include "device_common.h"

namespace aidg {
namespace {

constexpr int kFftThreads = 1024;
constexpr int kTile = 32;

// exp(-2 pi i a / M) for integers 0 <= a < M <= 8192, FP32, without a table (a
// table read would expose a global-memory latency in every pass): the nearest
// quarter turn q comes from an FP32 quotient (a near-tie leaves |t| a hair above
// 1/8, where the polynomials are still accurate), the remainder 4a - qM is exact in
// integers and is scaled once.
__device__ __forceinline__ float2 root_of_unity(int a, int M, float inv_m) {
  const int q = (int)rintf(4.0f * (float)a * inv_m);
  const float2 p = phasor_quarter((float)(4 * a - q * M) * (0.25f * inv_m), q);
  return {p.x, -p.y};
}

// One Stockham pass of radix R over the row held in LDS (Ls = product of the
// earlier radices): butterfly j < N/R reads buf[j + i N/R], multiplies input i by
// exp(DIR 2 pi i k i / (Ls R)) with k = j mod Ls, and writes its outputs to
// buf[(j / Ls) Ls R + k + i Ls].  In place: every read, a barrier, every write.
// The last pass hands its outputs to store(k) instead (coalesced: the last pass has
// j / Ls = 0), which saves the row's separate store pass through LDS and its barrier.
// (Reading the first pass's inputs from global memory as well raised the kernel's
// registers from 53 to over 100, with spills in the prediction variant.)
// FP32 twiddles are computed (root_of_unity for the first, products for its powers);
// FP64 ones come from the table.
template <int R, int DIR, bool LAST, typename V2, typename Store>
__device__ __forceinline__ void row_pass(V2* buf, int N, int Ls, const V2* __restrict__ tw,
                                         const Store& store) {
  using Rt = decltype(V2{}.x);
  constexpr int MAXB = (kMaxImageN / R + kFftThreads - 1) / kFftThreads;
  const int m = N / R, tstep = N / (Ls * R), M = Ls * R;
  const float inv_m = 1.0f / (float)M, inv_ls = 1.0f / (float)Ls;
  V2 y[MAXB][R];
  int kk[MAXB], gg[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * kFftThreads;
    if (j < m) {
      // j / Ls from an FP32 quotient: (j + 1/2) / Ls is at least 1/(2 Ls) away from an
      // integer, far beyond the rounding for j < 8192 (checked exhaustively)
      const int g = (int)(((float)j + 0.5f) * inv_ls), k = j - g * Ls;
      gg[b] = g;
      kk[b] = k;
#pragma unroll
      for (int i = 0; i < R; ++i) y[b][i] = buf[j + i * m];
      if (Ls > 1) {  // the first pass has unit twiddles
        if constexpr (std::is_same_v<Rt, float>) {
          // exp(-2 pi i k / (Ls R)) from the polynomial, its powers i = 2 .. R-1 by
          // complex products (at most R - 2 further roundings)
          V2 w1 = root_of_unity(k, M, inv_m);
          if (DIR > 0) w1.y = -w1.y;
          V2 w = w1;
#pragma unroll
          for (int i = 1; i < R; ++i) {
            if (i > 1) w = cmul<Rt>(w, w1);
            y[b][i] = cmul<Rt>(y[b][i], w);
          }
        } else {
#pragma unroll
          for (int i = 1; i < R; ++i) {
            V2 w = tw[k * i * tstep];  // exp(-2 pi i k i / (Ls R))
            if (DIR > 0) w.y = -w.y;
            y[b][i] = cmul<Rt>(y[b][i], w);
          }
        }
      }
      butterfly<V2, R, DIR>(y[b]);
    }
  }
  // LDS reads before LDS writes (the last pass writes global memory only)
  if constexpr (!LAST) __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = threadIdx.x + b * kFftThreads;
    if (j < m) {
      const int k = kk[b], base = gg[b] * Ls * R + k;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if constexpr (LAST) store(base + i * Ls, y[b][i]);
        else buf[base + i * Ls] = y[b][i];
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
}

template <int R, int DIR, typename V2, typename Store>
__device__ __forceinline__ void row_pass_at(bool last, V2* buf, int N, int Ls, const V2* tw,
                                            const Store& store) {
  if (last) row_pass<R, DIR, true>(buf, N, Ls, tw, store);
  else row_pass<R, DIR, false>(buf, N, Ls, tw, store);
}

// The transform of the row held in LDS; store(k, v) takes output k.
template <int DIR, typename V2, typename Store>
__device__ __forceinline__ void row_fft(V2* buf, const ImageRadices& fr, int N, const V2* tw,
                                        const Store& store) {
  int Ls = 1;
  for (int p = 0; p < fr.n; ++p) {
    const int r = fr.r[p];
    const bool last = p == fr.n - 1;
    if (r == 4) row_pass_at<4, DIR>(last, buf, N, Ls, tw, store);
    else if (r == 2) row_pass_at<2, DIR>(last, buf, N, Ls, tw, store);
    else if (r == 3) row_pass_at<3, DIR>(last, buf, N, Ls, tw, store);
    else row_pass_at<5, DIR>(last, buf, N, Ls, tw, store);
    Ls *= r;
  }
}

// exp(sign 2 pi i w0 n1(X, Y)) / (L^2 T(X, Y)) at image pixel (X, Y), with
// l = (X - N/2) dl, m = (Y - N/2) dl and itaper[X] = 1 / t(X).  FP32 path: n1 = s - 1
// with s = sqrt(1 - l^2 - m^2) from an FP32 square root and one FP64 residual
// correction (s to about 1e-15, so w0 n1 keeps ~1e-12 turns, far below the FP32
// phasor's own rounding).  FP64 path: the cancellation-free -r^2 / (1 + s) in FP64.
template <typename R>
__device__ __forceinline__ typename C2<R>::T wterm(int X, int Y, int N, double dl, double w0,
                                                   const double* __restrict__ itaper, double inv_l2,
                                                   double sign) {
  const R sc = (R)(inv_l2 * itaper[X] * itaper[Y]);
  if (w0 == 0.0) return {sc, (R)0};  // a layer at w = 0: the w-term is exactly 1
  const double l = (X - N / 2) * dl, m = (Y - N / 2) * dl;
  double n1;
  if constexpr (std::is_same_v<R, float>) {
    const double x = fma(-l, l, fma(-m, m, 1.0));
    const float s0 = sqrtf((float)x);
    n1 = (double)s0 + fma(-(double)s0, (double)s0, x) * (double)(0.5f / s0) - 1.0;
  } else {
    const double r2 = l * l + m * m;
    n1 = -r2 / (1.0 + sqrt(1.0 - r2));
  }
  const auto ph = phasor(sign * w0 * n1, R());
  return {ph.x * sc, ph.y * sc};
}

// Row transforms of an N x N plane, src and dst may be the same buffer (each
// workgroup reads its whole row before it writes).  PREDICT: src is an image plane
// [Y][X] and each value is first multiplied by wterm(X, Y) with sign -1.
template <typename R, int DIR, bool PREDICT>
__global__ __launch_bounds__(kFftThreads) void image_fft_rows(const typename C2<R>::T* src,
                                                              typename C2<R>::T* dst, int N,
                                                              ImageRadices fr,
                                                              const typename C2<R>::T* __restrict__ tw,
                                                              const double* __restrict__ itaper,
                                                              double dl, double w0, double inv_l2) {
  using V2 = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  V2* buf = reinterpret_cast<V2*>(smem_raw);
  const int row = blockIdx.x;
  const V2* s = src + (size_t)row * N;
  V2* d = dst + (size_t)row * N;
  for (int x = threadIdx.x; x < N; x += kFftThreads) {
    V2 v = s[x];
    if constexpr (PREDICT) v = cmul<R>(v, wterm<R>(x, row, N, dl, w0, itaper, inv_l2, -1.0));
    buf[x] = (x & 1) ? V2{-v.x, -v.y} : v;
  }
  __syncthreads();
  auto store = [&](int k, V2 v) { d[k] = (k & 1) ? V2{-v.x, -v.y} : v; };
  row_fft<DIR>(buf, fr, N, tw, store);
}

// dst[x][y] = src[y][x] over 32 x 32 tiles (grid ceil(N/32) x ceil(N/32), 256 threads).
template <typename V2>
__global__ __launch_bounds__(256) void image_transpose(const V2* __restrict__ src, V2* __restrict__ dst,
                                                       int N) {
  __shared__ V2 tile[kTile][kTile + 1];
  const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int y = by + j, x = bx + tx;
    if (y < N && x < N) tile[j][tx] = src[(size_t)y * N + x];
  }
  __syncthreads();
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int y = bx + j, x = by + tx;
    if (y < N && x < N) dst[(size_t)y * N + x] = tile[tx][j];
  }
}

// Bilinear interpolation of an L x L lattice map [y][x] at image pixel (X, Y), periodic
// over the field: pixel X sits at lattice coordinate g = (X - N/2) L / N + L/2, i.e.
// g N = (X - N/2) L + (L/2) N, an integer in [0, L N); its quotient by N is the lower
// lattice point (the upper one wraps to 0 past L - 1) and its remainder the weight.
template <typename R>
__device__ __forceinline__ R lattice_bilinear(const double* __restrict__ M, int L, int N, R inv_n, int X, int Y) {
  const int nx = (X - N / 2) * L + (L / 2) * N, ny = (Y - N / 2) * L + (L / 2) * N;
  const int x0 = nx / N, y0 = ny / N;
  const R fx = (R)(nx - x0 * N) * inv_n, fy = (R)(ny - y0 * N) * inv_n;
  const int x1 = x0 + 1 == L ? 0 : x0 + 1, y1 = y0 + 1 == L ? 0 : y0 + 1;
  const R r0 = (R)M[y0 * L + x0] * ((R)1 - fx) + (R)M[y0 * L + x1] * fx;
  const R r1 = (R)M[y1 * L + x0] * ((R)1 - fx) + (R)M[y1 * L + x1] * fx;
  return r0 * ((R)1 - fy) + r1 * fy;
}

// One layer of Eq. wstack: img[Y][X] (+)= B[X][Y] * wterm(X, Y) with sign +1.  B is
// the layer's transform with rows X (the second row pass ran along v); tiles are
// read along Y and written along X.
template <typename R>
__global__ __launch_bounds__(256) void image_wstack(const typename C2<R>::T* __restrict__ B,
                                                    typename C2<R>::T* __restrict__ img, int N,
                                                    const double* __restrict__ itaper, double dl,
                                                    double w0, double inv_l2, int assign,
                                                    const double* __restrict__ nmap, int L) {
  using V2 = typename C2<R>::T;
  __shared__ V2 tile[kTile][kTile + 1];
  const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;  // X and Y ranges
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int X = bx + j, Y = by + tx;
    if (X < N && Y < N) tile[j][tx] = B[(size_t)X * N + Y];
  }
  __syncthreads();
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int Y = by + j, X = bx + tx;
    if (X < N && Y < N) {
      const V2 v = cmul<R>(tile[tx][j], wterm<R>(X, Y, N, dl, w0, itaper, inv_l2, 1.0));
      V2* o = img + (size_t)Y * N + X;
      V2 r = assign ? v : V2{o->x + v.x, o->y + v.y};
      if (nmap) {  // last layer, inverse A-term mode: divide the sum by the normalisation
        const R c = lattice_bilinear<R>(nmap, L, N, (R)1 / (R)N, X, Y);
        const R f = c > (R)0 ? (R)1 / c : (R)0;  // 0 where the map is 0
        r = V2{r.x * f, r.y * f};
      }
      *o = r;
    }
  }
}

template <typename R>
int fft_rows_t(int dir, bool predict, const void* src, void* dst, int N, const ImageRadices& fr,
               const void* tw, const double* itaper, double dl, double w0, double inv_l2,
               hipStream_t st) {
  using V2 = typename C2<R>::T;
  const size_t lds = (size_t)N * sizeof(V2);
  const V2* s = reinterpret_cast<const V2*>(src);
  V2* d = reinterpret_cast<V2*>(dst);
  const V2* t = reinterpret_cast<const V2*>(tw);
  if (predict)
    hipLaunchKernelGGL((image_fft_rows<R, -1, true>), dim3(N), dim3(kFftThreads), lds, st, s, d, N, fr,
                       t, itaper, dl, w0, inv_l2);
  else if (dir > 0)
    hipLaunchKernelGGL((image_fft_rows<R, 1, false>), dim3(N), dim3(kFftThreads), lds, st, s, d, N, fr,
                       t, itaper, dl, w0, inv_l2);
  else
    hipLaunchKernelGGL((image_fft_rows<R, -1, false>), dim3(N), dim3(kFftThreads), lds, st, s, d, N, fr,
                       t, itaper, dl, w0, inv_l2);
  return (int)hipGetLastError();
}

}  // namespace

int launch_image_fft_rows(int precision, int dir, bool predict, const void* src, void* dst, int N,
                          const ImageRadices& fr, const void* tw, const double* itaper, double dl,
                          double w0, double inv_l2, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return precision == AIDG_FP64
             ? fft_rows_t<double>(dir, predict, src, dst, N, fr, tw, itaper, dl, w0, inv_l2, st)
             : fft_rows_t<float>(dir, predict, src, dst, N, fr, tw, itaper, dl, w0, inv_l2, st);
}

int launch_image_transpose(int precision, const void* src, void* dst, int N, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile);
  if (precision == AIDG_FP64)
    hipLaunchKernelGGL((image_transpose<double2>), grid, dim3(256), 0, st,
                       reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), N);
  else
    hipLaunchKernelGGL((image_transpose<float2>), grid, dim3(256), 0, st,
                       reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), N);
  return (int)hipGetLastError();
}

int launch_image_wstack(int precision, const void* B, void* img, int N, const double* itaper, double dl,
                        double w0, double inv_l2, int assign, const double* nmap, int L, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((N + kTile - 1) / kTile, (N + kTile - 1) / kTile);
  if (precision == AIDG_FP64)
    hipLaunchKernelGGL((image_wstack<double>), grid, dim3(256), 0, st,
                       reinterpret_cast<const double2*>(B), reinterpret_cast<double2*>(img), N, itaper,
                       dl, w0, inv_l2, assign, nmap, L);
  else
    hipLaunchKernelGGL((image_wstack<float>), grid, dim3(256), 0, st,
                       reinterpret_cast<const float2*>(B), reinterpret_cast<float2*>(img), N, itaper,
                       dl, w0, inv_l2, assign, nmap, L);
  return (int)hipGetLastError();
}

}  // namespace aidg
