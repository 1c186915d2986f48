// lbm_spectrum.hip -- power spectrum of a recorded signal, for the shedding
// frequency of the square-cylinder flow (Sec. 4.2: the dominant frequency of
// the last quarter of the velocity recorded at the monitoring point, by the
// discrete Fourier transform).
//
// k_dft_power: one lane per frequency bin k = 0..n/2; the samples are staged
// through LDS in chunks of DFT_CHUNK and read as broadcasts; the twiddle
// e^{-2 pi i j k / n} is advanced by a complex rotation inside a chunk and
// re-seeded exactly (angle 2 pi ((j k) mod n) / n) at every chunk start, so
// its error stays within a few hundred ulps.  Everything is FP64.
// k_dft_peak: one workgroup, the bin k >= 1 of largest power (lowest k on
// ties; NaN powers are never chosen).
#include <hip/hip_runtime.h>

#include "lbm_launch.hpp"

namespace lbm {

constexpr int DFT_TX = 64;
constexpr int DFT_CHUNK = 256;

__global__ __launch_bounds__(DFT_TX) void k_dft_power(const double* __restrict__ x, int64_t n,
                                                      double* __restrict__ power) {
  __shared__ double xs[DFT_CHUNK];
  const int64_t nb = n / 2 + 1;
  const int64_t k = (int64_t)blockIdx.x * DFT_TX + threadIdx.x;
  const int64_t kk = k < nb ? k : 0;
  double sa, ca;  // rotation by 2 pi k / n
  sincospi(2.0 * (double)kk / (double)n, &sa, &ca);
  double re = 0.0, im = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += DFT_CHUNK) {
    const int len = (int)(n - j0 < DFT_CHUNK ? n - j0 : DFT_CHUNK);
    __syncthreads();
    for (int t = threadIdx.x; t < len; t += DFT_TX) xs[t] = x[j0 + t];
    __syncthreads();
    double sn, cs;
    sincospi(2.0 * (double)((j0 * kk) % n) / (double)n, &sn, &cs);
    for (int t = 0; t < len; ++t) {
      const double v = xs[t];
      re = __builtin_fma(v, cs, re);
      im = __builtin_fma(-v, sn, im);
      const double c2 = cs * ca - sn * sa;
      sn = sn * ca + cs * sa;
      cs = c2;
    }
  }
  if (k < nb) power[k] = re * re + im * im;
}

__global__ __launch_bounds__(1024) void k_dft_peak(const double* __restrict__ power, int64_t nb,
                                                   int64_t* __restrict__ peak) {
  __shared__ double bp[1024];
  __shared__ int64_t bk[1024];
  double best = -1.0;
  int64_t bestk = nb > 1 ? 1 : 0;
  for (int64_t k = 1 + threadIdx.x; k < nb; k += 1024) {
    const double p = power[k];
    if (p > best) { best = p; bestk = k; }  // strided ascending: first maximum kept
  }
  bp[threadIdx.x] = best;
  bk[threadIdx.x] = bestk;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double p = bp[threadIdx.x + w];
      const int64_t q = bk[threadIdx.x + w];
      if (p > bp[threadIdx.x] || (p == bp[threadIdx.x] && q < bk[threadIdx.x])) {
        bp[threadIdx.x] = p;
        bk[threadIdx.x] = q;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *peak = bk[0];
}

hipError_t launch_dft_power(const double* x, int64_t n, double* power, int64_t* peak, hipStream_t s) {
  const int64_t nb = n / 2 + 1;
  hipLaunchKernelGGL(k_dft_power, dim3((unsigned)((nb + DFT_TX - 1) / DFT_TX)), dim3(DFT_TX), 0, s, x, n,
                     power);
  if (peak) hipLaunchKernelGGL(k_dft_peak, dim3(1), dim3(1024), 0, s, power, nb, peak);
  return hipGetLastError();
}

}  // namespace lbm
