// Table preparation kernels: input validation and natural cubic-spline second
// derivatives of every coupling-matrix element along the R grid (the coupling
// tables are tabulated on a grid and interpolated with a cubic spline, paper
// Section III), plus the Monte-Carlo cross-section reduction (end of Section II).
#include "internal.h"

#include <math.h>

namespace mqct {

namespace {

__device__ inline unsigned long long dbits(double x) { return __double_as_longlong(x); }

// Max |M[n][m] - conj(M[m][n])| (stats[0]), max |M| (stats[1]) and the number of
// non-finite entries (stats[2]).  Non-negative doubles order like their bit
// patterns, so the maxima use integer atomics.
__global__ void __launch_bounds__(256)
validate_kernel(const double* __restrict__ M, int N, int K, int ncomp,
                unsigned long long* __restrict__ stats) {
  const int64_t NN = (int64_t)N * N;
  const int64_t total = NN * K;
  double herm = 0.0, amax = 0.0;
  unsigned long long bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / NN;
    const int64_t r = i - k * NN;
    const int64_t n = r / N, m = r - n * N;
    double re = M[i * ncomp], im = ncomp == 2 ? M[i * ncomp + 1] : 0.0;
    if (!isfinite(re) || !isfinite(im)) { ++bad; continue; }
    amax = fmax(amax, sqrt(re * re + im * im));
    if (m > n) {
      const int64_t j = k * NN + m * N + n;
      double tre = M[j * ncomp], tim = ncomp == 2 ? M[j * ncomp + 1] : 0.0;
      double dre = re - tre, dim = im + tim;      // M_nm - conj(M_mn)
      double d = sqrt(dre * dre + dim * dim);
      if (isfinite(d)) herm = fmax(herm, d);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    herm = fmax(herm, __shfl_xor(herm, off, 64));
    amax = fmax(amax, __shfl_xor(amax, off, 64));
    bad += __shfl_xor(bad, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&stats[0], dbits(herm));
    atomicMax(&stats[1], dbits(amax));
    if (bad) atomicAdd(&stats[2], bad);
  }
}

template <typename S> __device__ inline S cast_to(double x) { return (S)x; }

// One thread per real column (stored row m, column n, component).  The
// tridiagonal system of the natural spline,
//   h_{k-1}/6 y2_{k-1} + (h_{k-1}+h_k)/3 y2_k + h_k/6 y2_{k+1}
//       = (y_{k+1}-y_k)/h_k - (y_k-y_{k-1})/h_{k-1},   y2_0 = y2_{K-1} = 0,
// depends on the grid only, so its elimination factors are formed once per
// workgroup in LDS; each thread then runs the forward sweep (into tmp, FP64) and
// back substitution for its column.  Padding columns are written as zeros.
template <typename S>
__global__ void __launch_bounds__(256)
spline_kernel(const double* __restrict__ M_in, const double* __restrict__ R, int N, int K,
              int Npad, int ncomp, int64_t col0, int64_t ncols, S* __restrict__ M_out,
              S* __restrict__ M2_out, double* __restrict__ tmp) {
  extern __shared__ double sh[];
  double* cprime = sh;            // [K]
  double* invden = sh + K;        // [K]
  double* sub = sh + 2 * K;       // [K]
  if (threadIdx.x == 0) {
    double cp = 0.0;
    for (int k = 1; k <= K - 2; ++k) {
      double hl = R[k] - R[k - 1], hr = R[k + 1] - R[k];
      double den = (hl + hr) / 3.0 - (k > 1 ? hl / 6.0 * cp : 0.0);
      cp = hr / 6.0 / den;
      cprime[k] = cp;
      invden[k] = 1.0 / den;
      sub[k] = hl / 6.0;
    }
  }
  __syncthreads();
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int64_t col = col0 + c;                 // column in the output layout
  const int64_t per_row = (int64_t)Npad * ncomp;
  const int64_t m = col / per_row;
  const int64_t rem = col - m * per_row;
  const int64_t n = rem / ncomp, comp = rem - n * ncomp;
  const int64_t out_stride = (int64_t)N * per_row;   // one knot of the output
  if (n >= N) {
    for (int k = 0; k < K; ++k) {
      M_out[k * out_stride + col] = cast_to<S>(0.0);
      M2_out[k * out_stride + col] = cast_to<S>(0.0);
    }
    return;
  }
  const int64_t in_stride = (int64_t)N * N * ncomp;
  const double* y = M_in + (m * N + n) * ncomp + comp;
  double y0 = y[0], y1 = y[in_stride];
  M_out[col] = cast_to<S>(y0);
  double dprev = 0.0;
  for (int k = 1; k <= K - 2; ++k) {
    double y2v = y[(int64_t)(k + 1) * in_stride];
    double hl = R[k] - R[k - 1], hr = R[k + 1] - R[k];
    double rhs = (y2v - y1) / hr - (y1 - y0) / hl;
    double d = (rhs - sub[k] * dprev) * invden[k];
    tmp[(int64_t)k * ncols + c] = d;
    dprev = d;
    M_out[k * out_stride + col] = cast_to<S>(y1);
    y0 = y1;
    y1 = y2v;
  }
  M_out[(int64_t)(K - 1) * out_stride + col] = cast_to<S>(y1);
  M2_out[(int64_t)(K - 1) * out_stride + col] = cast_to<S>(0.0);
  M2_out[col] = cast_to<S>(0.0);
  double nxt = 0.0;
  for (int k = K - 2; k >= 1; --k) {
    double v = tmp[(int64_t)k * ncols + c] - cprime[k] * nxt;
    M2_out[k * out_stride + col] = cast_to<S>(v);
    nxt = v;
  }
}

// level_sums[b][L] = sum over channels n of level L of P[b][n]
__global__ void level_sum_kernel(int64_t B, int N, const double* __restrict__ P,
                                 const int32_t* __restrict__ lev, int n_levels,
                                 double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= B * n_levels) return;
  const int64_t b = i / n_levels;
  const int L = (int)(i - b * n_levels);
  double s = 0.0;
  for (int n = 0; n < N; ++n)
    if (lev[n] == L) s += P[b * N + n];
  out[i] = s;
}

// sigma[L'][L''] = 2 pi b_max / count(L') * sum_{b: init(b) = L'} b_b level_sums[b][L'']
__global__ void xsec_kernel(int64_t B, const double* __restrict__ bpar,
                            const int32_t* __restrict__ init_level, int n_levels, double b_max,
                            const double* __restrict__ level_sums, double* __restrict__ sigma) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_levels * n_levels) return;
  const int L1 = (int)(i / n_levels), L2 = (int)(i % n_levels);
  double s = 0.0, cnt = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    if (init_level[b] != L1) continue;
    cnt += 1.0;
    s += bpar[b] * level_sums[b * n_levels + L2];
  }
  sigma[i] = cnt > 0.0 ? 2.0 * M_PI * b_max / cnt * s : 0.0;
}

// ---- sparse (ELL) layout of the tables ---------------------------------------
//
// An element (m, n) of the stored matrices is kept when its magnitude exceeds
// `thr` at some knot, in either (m, n) or (n, m) (the input is Hermitian to
// rounding; the test is made symmetric so that column n of the stored matrix
// lists the same channels as row n).  Column n's kept rows m, ascending, are
// col[q][n], q < cnt[n]; the values of slot q are the stored element (m, n) of
// M and of its spline curvature, so a kernel that streams "stored row" q reads
// exactly what the dense kernel reads for stored row m = col[q][n].

// amax[m][n] = max over knots of |M_k(m, n)| (FP64 input [K][N][N][ncomp])
__global__ void ell_amax(const double* __restrict__ M, int N, int K, int ncomp,
                         double* __restrict__ amax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t NN = (int64_t)N * N;
  if (i >= NN) return;
  double a = 0.0;
  for (int k = 0; k < K; ++k) {
    const double* e = M + ((int64_t)k * NN + i) * ncomp;
    const double v = ncomp == 2 ? sqrt(e[0] * e[0] + e[1] * e[1]) : fabs(e[0]);
    a = fmax(a, v);
  }
  amax[i] = a;
}

__device__ __forceinline__ bool ell_keep(const double* amax, int N, int m, int n, double thr) {
  return amax[(int64_t)m * N + n] > thr || amax[(int64_t)n * N + m] > thr;
}

__global__ void ell_count(const double* __restrict__ amax, int N, double thr,
                          int* __restrict__ cnt) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int c = 0;
  for (int m = 0; m < N; ++m) c += ell_keep(amax, N, m, n, thr);
  cnt[n] = c;
}

// col[q][n] for q < W and n < Npad; unused slots (and padding columns) point at
// row 0 with zero values
__global__ void ell_fill(const double* __restrict__ amax, int N, int Npad, int W, double thr,
                         int32_t* __restrict__ col) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Npad) return;
  int q = 0;
  if (n < N)
    for (int m = 0; m < N && q < W; ++m)
      if (ell_keep(amax, N, m, n, thr)) col[(int64_t)q++ * Npad + n] = m;
  for (; q < W; ++q) col[(int64_t)q * Npad + n] = 0;
}

// E[k][q][n] = D[k][col[q][n]][n] for kept slots, 0 otherwise (both slices of the
// storage type; ncomp reals per element)
template <typename S>
__global__ void ell_gather(const S* __restrict__ D, const S* __restrict__ D2,
                           const int32_t* __restrict__ col, const int* __restrict__ cnt, int N,
                           int Npad, int K, int W, int ncomp, S* __restrict__ E,
                           S* __restrict__ E2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_knot = (int64_t)W * Npad;
  if (i >= (int64_t)K * per_knot) return;
  const int k = (int)(i / per_knot);
  const int64_t r = i - (int64_t)k * per_knot;
  const int q = (int)(r / Npad), n = (int)(r - (int64_t)q * Npad);
  const bool kept = n < N && q < cnt[n];
  const int64_t src = ((int64_t)k * N * Npad + (int64_t)col[(int64_t)q * Npad + n] * Npad + n) * ncomp;
  for (int c = 0; c < ncomp; ++c) {
    E[i * ncomp + c] = kept ? D[src + c] : (S)0;
    E2[i * ncomp + c] = kept ? D2[src + c] : (S)0;
  }
}

}  // namespace

hipError_t launch_validate(const double* M_in, int N, int K, int ncomp,
                           unsigned long long* stats, hipStream_t s) {
  int64_t total = (int64_t)N * N * K;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  validate_kernel<<<(unsigned)blocks, 256, 0, s>>>(M_in, N, K, ncomp, stats);
  return hipGetLastError();
}

hipError_t launch_spline_prepare(const double* M_in, const double* R, int N, int K, int Npad,
                                 int ncomp, int dtype, void* M_out, void* M2_out, double* tmp,
                                 int64_t tmp_doubles, hipStream_t s) {
  const int64_t total = (int64_t)N * Npad * ncomp;
  const int64_t chunk = tmp_doubles / K;
  const size_t shmem = 3 * (size_t)K * sizeof(double);
  for (int64_t c0 = 0; c0 < total; c0 += chunk) {
    int64_t nc = total - c0 < chunk ? total - c0 : chunk;
    unsigned blocks = (unsigned)((nc + 255) / 256);
    if (dtype_fp32(dtype))
      spline_kernel<float><<<blocks, 256, shmem, s>>>(M_in, R, N, K, Npad, ncomp, c0, nc,
                                                      (float*)M_out, (float*)M2_out, tmp);
    else
      spline_kernel<double><<<blocks, 256, shmem, s>>>(M_in, R, N, K, Npad, ncomp, c0, nc,
                                                       (double*)M_out, (double*)M2_out, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ell_pattern(const double* M_in, int N, int K, int ncomp, double thr,
                              double* amax, int* cnt, hipStream_t s) {
  const int64_t NN = (int64_t)N * N;
  ell_amax<<<(unsigned)((NN + 255) / 256), 256, 0, s>>>(M_in, N, K, ncomp, amax);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ell_count<<<(unsigned)((N + 127) / 128), 128, 0, s>>>(amax, N, thr, cnt);
  return hipGetLastError();
}

hipError_t launch_ell_fill(const double* amax, int N, int Npad, int W, double thr, int32_t* col,
                           hipStream_t s) {
  ell_fill<<<(unsigned)((Npad + 127) / 128), 128, 0, s>>>(amax, N, Npad, W, thr, col);
  return hipGetLastError();
}

hipError_t launch_ell_gather(const void* D, const void* D2, const int32_t* col, const int* cnt,
                             int N, int Npad, int K, int W, int ncomp, int dtype, void* E,
                             void* E2, hipStream_t s) {
  const int64_t total = (int64_t)K * W * Npad;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (dtype_fp32(dtype))
    ell_gather<float><<<blocks, 256, 0, s>>>((const float*)D, (const float*)D2, col, cnt, N, Npad,
                                             K, W, ncomp, (float*)E, (float*)E2);
  else
    ell_gather<double><<<blocks, 256, 0, s>>>((const double*)D, (const double*)D2, col, cnt, N,
                                              Npad, K, W, ncomp, (double*)E, (double*)E2);
  return hipGetLastError();
}

hipError_t launch_xsec(int64_t B, int N, const double* P, const double* b,
                       const int32_t* init_level, const int32_t* level_of_channel, int n_levels,
                       double b_max, double* level_sums, double* sigma, hipStream_t s) {
  int64_t n1 = B * n_levels;
  level_sum_kernel<<<(unsigned)((n1 + 255) / 256), 256, 0, s>>>(B, N, P, level_of_channel,
                                                                 n_levels, level_sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t n2 = (int64_t)n_levels * n_levels;
  xsec_kernel<<<(unsigned)((n2 + 255) / 256), 256, 0, s>>>(B, b, init_level, n_levels, b_max,
                                                           level_sums, sigma);
  return hipGetLastError();
}

}  // namespace mqct
