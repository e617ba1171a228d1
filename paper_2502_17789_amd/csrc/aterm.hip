// Inverse A-term mode (Sec. 3.3, A-term application).  The gridder of such a plan
// applies A_p^-1 S A_q^-H scaled by 1 / ||A_p^-1 A_q^-H||_F; it reads the planes
// B = (A^-1)^H, so that its epilogue B_p^H S B_q is the adjoint mode's with B for A.
//   aterm_inverse_h     B = (A^-1)^H = [[conj a3, -conj a2], [-conj a1, conj a0]] / conj(det A)
//                       for every 2x2 of [n_int][n_st][L][L], in FP64; B = 0 where
//                       det A = 0 (such a pixel contributes nothing).
//   aterm_norm_partial  per lattice pixel, over one chunk of the plan's (A_p plane,
//                       A_q plane, visibility count) pairs: sum of count / ||B_p^H B_q||_F
//                       (0 where the product vanishes), one workgroup row per chunk.
//   aterm_norm_reduce   the chunks' sums times 1 / (total count): the weighted average
//                       by which the image is divided.
#include <hip/hip_runtime.h>

#include "aidg_internal.h"
#include "device_common.h"

namespace aidg {
namespace {

constexpr int kThreads = 256;

template <typename R>
__global__ __launch_bounds__(kThreads) void aterm_inverse_h(const typename C2<R>::T* __restrict__ A,
                                                            typename C2<R>::T* __restrict__ B, int64_t n) {
  using V2 = typename C2<R>::T;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const V2* a = A + 4 * i;
  double ar[4], ai[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ar[k] = (double)a[k].x;
    ai[k] = (double)a[k].y;
  }
  // det = a0 a3 - a1 a2
  const double dr = ar[0] * ar[3] - ai[0] * ai[3] - (ar[1] * ar[2] - ai[1] * ai[2]);
  const double di = ar[0] * ai[3] + ai[0] * ar[3] - (ar[1] * ai[2] + ai[1] * ar[2]);
  const double d2 = dr * dr + di * di;
  V2* b = B + 4 * i;
  if (d2 == 0.0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = V2{0, 0};
    return;
  }
  // 1 / conj(det) = det / |det|^2
  const double qr = dr / d2, qi = di / d2;
  // B = [[conj a3, -conj a2], [-conj a1, conj a0]] / conj(det)
  const int src[4] = {3, 2, 1, 0};
  const double sgn[4] = {1.0, -1.0, -1.0, 1.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double cr = sgn[k] * ar[src[k]], ci = -sgn[k] * ai[src[k]];
    b[k] = V2{(R)(cr * qr - ci * qi), (R)(cr * qi + ci * qr)};
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void aterm_norm_partial(const typename C2<R>::T* __restrict__ B,
                                                               const int32_t* __restrict__ pairs,
                                                               const double* __restrict__ count,
                                                               int64_t n_pairs, int64_t chunk_len, int L2,
                                                               double* __restrict__ partial) {
  using V2 = typename C2<R>::T;
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= L2) return;
  const int64_t k0 = (int64_t)blockIdx.y * chunk_len;
  const int64_t k1 = k0 + chunk_len < n_pairs ? k0 + chunk_len : n_pairs;
  double acc = 0.0;
  for (int64_t k = k0; k < k1; ++k) {
    const V2* bp = B + ((int64_t)pairs[2 * k] * L2 + pix) * 4;
    const V2* bq = B + ((int64_t)pairs[2 * k + 1] * L2 + pix) * 4;
    double pr[4], pi[4], qr[4], qi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pr[i] = (double)bp[i].x;
      pi[i] = -(double)bp[i].y;  // conj
      qr[i] = (double)bq[i].x;
      qi[i] = (double)bq[i].y;
    }
    // M = B_p^H B_q, (B_p^H)[r][c] = conj(B_p[c][r]); |M|_F^2
    double n2 = 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int x0 = r, x1 = 2 + r;  // conj(B_p[0][r]), conj(B_p[1][r])
        const int y0 = c, y1 = 2 + c;  // B_q[0][c], B_q[1][c]
        const double mr = pr[x0] * qr[y0] - pi[x0] * qi[y0] + pr[x1] * qr[y1] - pi[x1] * qi[y1];
        const double mi = pr[x0] * qi[y0] + pi[x0] * qr[y0] + pr[x1] * qi[y1] + pi[x1] * qr[y1];
        n2 += mr * mr + mi * mi;
      }
    if (n2 > 0.0) acc += count[k] / sqrt(n2);
  }
  partial[(int64_t)blockIdx.y * L2 + pix] = acc;
}

__global__ __launch_bounds__(kThreads) void aterm_norm_reduce(const double* __restrict__ partial, int n_chunks,
                                                              int L2, double inv_total, double* __restrict__ map) {
  const int pix = blockIdx.x * kThreads + threadIdx.x;
  if (pix >= L2) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += partial[(int64_t)c * L2 + pix];
  map[pix] = s * inv_total;
}

}  // namespace

int launch_aterm_inverse_h(int precision, const void* A, void* B, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  if (precision == AIDG_FP32)
    hipLaunchKernelGGL(aterm_inverse_h<float>, grid, dim3(kThreads), 0, st,
                       reinterpret_cast<const float2*>(A), reinterpret_cast<float2*>(B), n);
  else
    hipLaunchKernelGGL(aterm_inverse_h<double>, grid, dim3(kThreads), 0, st,
                       reinterpret_cast<const double2*>(A), reinterpret_cast<double2*>(B), n);
  return (int)hipGetLastError();
}

int launch_aterm_norm(int precision, const void* B, const int32_t* pairs, const double* count, int64_t n_pairs,
                      int n_chunks, int64_t chunk_len, int L2, double inv_total, double* partial, double* map,
                      void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const unsigned gx = (unsigned)((L2 + kThreads - 1) / kThreads);
  if (precision == AIDG_FP32)
    hipLaunchKernelGGL(aterm_norm_partial<float>, dim3(gx, n_chunks), dim3(kThreads), 0, st,
                       reinterpret_cast<const float2*>(B), pairs, count, n_pairs, chunk_len, L2, partial);
  else
    hipLaunchKernelGGL(aterm_norm_partial<double>, dim3(gx, n_chunks), dim3(kThreads), 0, st,
                       reinterpret_cast<const double2*>(B), pairs, count, n_pairs, chunk_len, L2, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(aterm_norm_reduce, dim3(gx), dim3(kThreads), 0, st, partial, n_chunks, L2, inv_total, map);
  return (int)hipGetLastError();
}

}  // namespace aidg
