// Shell-averaged power spectrum of a field on the periodic ng^3 mesh (the
// estimator behind the fractional spectra of Sec. BAO reconstruction):
//
//   delta(k) = H^3 sum_x f(x) exp(-i k . x),  k = 2 pi n / L,  H = L / ng,
//   P(k) = |delta(k)|^2 / L^3,
//
// averaged over shell j (modes with j - 1/2 <= |n| < j + 1/2, n in
// (-ng/2, ng/2]^3), with its mode count and mean |k|; optionally for the
// contrast f / mean(f) - 1 and divided by the squared Fourier window
// prod_a sinc(pi n_a / ng)^(2p) of a mass assignment of order p.
//
// The transform is a plain real-to-complex FFT (hipFFT); the binning is
// ours.  The half spectrum (ng x ng x (ng/2 + 1), last index fastest) holds
// every mode once or, for 0 < n_c < ng/2, together with its conjugate
// partner -n, so those elements count twice.  Binning: one wavefront per
// workgroup takes a contiguous range of rows (a, b) and walks each row in
// chunks of 64 elements.  Along a row |n| grows with n_c, so the shells of a
// chunk are sorted: a segmented scan over the lanes sums each shell's run and
// the run's last lane adds it to the workgroup's histogram in LDS (one writer
// per shell per step, in program order).  The histograms of the workgroups
// are then summed per shell in a fixed order, so the result is the same bits
// on every run.
#include <hipfft/hipfft.h>

#include <climits>
#include <cmath>

#include "../../include/mak.h"
#include "engine.h"
#include "profile.h"

namespace mak {
namespace {

constexpr double kPi = 3.14159265358979323846;

// sinc(pi n / ng)^p
__device__ __forceinline__ double window_factor(int64_t n, int64_t ng, int p) {
  if (n == 0 || p == 0) return 1.0;
  const double x = kPi * double(n) / double(ng);
  const double s = sin(x) / x;
  double w = s;
  for (int k = 1; k < p; ++k) w *= s;
  return w;
}

__global__ __launch_bounds__(64) void k_shell_bin(const double2* __restrict__ spec, int64_t ng,
                                                  int64_t rows_per_wg, int nbins, int window,
                                                  double norm, double kf, int64_t nwg,
                                                  double* __restrict__ part) {
  extern __shared__ double hist[];  // [3][nbins]: power, |k|, modes
  const int lane = threadIdx.x;
  const int64_t wg = blockIdx.x;
  for (int i = lane; i < 3 * nbins; i += 64) hist[i] = 0.0;
  __syncthreads();
  const int64_t nzh = ng / 2 + 1, rows = ng * ng;
  const int64_t r0 = wg * rows_per_wg, r1 = r0 + rows_per_wg < rows ? r0 + rows_per_wg : rows;
  const bool even = (ng & 1) == 0;
  for (int64_t row = r0; row < r1; ++row) {
    const int64_t a = row / ng, b = row % ng;
    const int64_t na = a <= ng / 2 ? a : a - ng, nb = b <= ng / 2 ? b : b - ng;
    const double wab = window_factor(na, ng, window) * window_factor(nb, ng, window);
    const int64_t nab2 = na * na + nb * nb;
    for (int64_t c0 = 0; c0 < nzh; c0 += 64) {
      const int64_t c = c0 + lane;
      const bool act = c < nzh;
      double vp = 0.0, vk = 0.0, vm = 0.0;
      int key = act ? 0 : INT_MAX;
      if (act) {
        const double2 z = spec[row * nzh + c];
        const int64_t n2 = nab2 + c * c;
        const double r = sqrt(double(n2));
        const int j = int(floor(r + 0.5));
        key = j <= nbins ? j : INT_MAX;
        if (j >= 1 && j <= nbins) {
          const double w = (c == 0 || (even && c == ng / 2)) ? 1.0 : 2.0;
          const double W = wab * window_factor(c, ng, window);
          vp = w * norm * (z.x * z.x + z.y * z.y) / (W * W);
          vk = w * kf * r;
          vm = w;
        }
      }
      // segmented inclusive scan over runs of equal keys (keys are sorted)
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double op = __shfl_up(vp, off), ok = __shfl_up(vk, off), om = __shfl_up(vm, off);
        const int okey = __shfl_up(key, off);
        if (lane >= off && okey == key) {
          vp += op;
          vk += ok;
          vm += om;
        }
      }
      const int nkey = __shfl_down(key, 1);
      const bool tail = lane == 63 || nkey != key;
      if (tail && key >= 1 && key <= nbins) {
        hist[key - 1] += vp;
        hist[nbins + key - 1] += vk;
        hist[2 * nbins + key - 1] += vm;
      }
      __syncthreads();
    }
  }
  // partials laid out [3 * nbins][nwg]: one shell's partials are contiguous
  for (int i = lane; i < 3 * nbins; i += 64) part[int64_t(i) * nwg + wg] = hist[i];
}

// One workgroup per (quantity, shell): 256 threads sum strided partials in
// order, then a fixed tree.
__global__ __launch_bounds__(256) void k_shell_reduce(const double* __restrict__ part, int64_t nwg,
                                                      int nbins, double* __restrict__ sums) {
  __shared__ double red[256];
  const int64_t q = blockIdx.x;  // 0 .. 3 * nbins - 1
  double s = 0.0;
  for (int64_t w = threadIdx.x; w < nwg; w += 256) s += part[q * nwg + w];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[q] = red[0];
}

__global__ void k_shell_finish(const double* __restrict__ sums, int nbins, double* __restrict__ k_mean,
                               double* __restrict__ power, int64_t* __restrict__ modes) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nbins) return;
  const double m = sums[2 * nbins + j];
  modes[j] = int64_t(m);
  power[j] = sums[j] / m;  // an empty shell gives NaN
  k_mean[j] = sums[nbins + j] / m;
}

void fft_check(hipfftResult r, const char* what) {
  if (r != HIPFFT_SUCCESS)
    MAK_FAIL(MAK_EHIP, std::string(what) + " failed (hipFFT status " + std::to_string(int(r)) + ")");
}

}  // namespace

void PowerWork::release_plan() {
  if (plan) (void)hipfftDestroy(hipfftHandle(plan));
  plan = 0;
  ng = 0;
}

void power_spectrum(PowerWork& w, const double* field, int64_t ng, double L, int nbins, int window,
                    bool contrast, double* k_mean, double* power, int64_t* modes, hipStream_t st) {
  const int64_t nzh = ng / 2 + 1, rows = ng * ng, n = rows * ng;
  if (w.ng != ng) {
    w.release_plan();
    hipfftHandle h;
    fft_check(hipfftPlan3d(&h, int(ng), int(ng), int(ng), HIPFFT_D2Z), "hipfftPlan3d");
    w.plan = uintptr_t(h);
    w.ng = ng;
  }
  fft_check(hipfftSetStream(hipfftHandle(w.plan), st), "hipfftSetStream");
  double norm = L * L * L / (double(ng) * ng * ng * double(ng) * ng * ng);
  if (contrast) {
    const double mean = dev_reduce_sum(field, n, w.tmp, st) / double(n);
    if (!(mean != 0.0) || !std::isfinite(mean))
      MAK_FAIL(MAK_EINVAL, "contrast needs a field with a finite, nonzero mean");
    norm /= mean * mean;
  }
  w.real.ensure(size_t(n) * sizeof(double));
  w.spec.ensure(size_t(rows) * nzh * sizeof(double2));
  MAK_HIP(hipMemcpyAsync(w.real.p, field, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  {
    ProfScope scope("fft", st, double(n), double(n) * 8 + double(rows * nzh) * 16);
    fft_check(hipfftExecD2Z(hipfftHandle(w.plan), w.real.as<hipfftDoubleReal>(),
                            w.spec.as<hipfftDoubleComplex>()),
              "hipfftExecD2Z");
  }
  int64_t nwg = rows / 16;
  if (nwg < 1) nwg = 1;
  if (nwg > 8192) nwg = 8192;
  const int64_t rpw = ceil_div(rows, nwg);
  nwg = ceil_div(rows, rpw);
  w.part.ensure(size_t(3) * nbins * nwg * sizeof(double));
  w.sums.ensure(size_t(3) * nbins * sizeof(double));
  {
    ProfScope scope("shell_bin", st, double(rows * nzh),
                    double(rows * nzh) * 16 + double(3) * nbins * nwg * 8);
    hipLaunchKernelGGL(k_shell_bin, dim3(unsigned(nwg)), dim3(64), size_t(3) * nbins * sizeof(double), st,
                       w.spec.as<double2>(), ng, rpw, nbins, window, norm, 2.0 * kPi / L, nwg,
                       w.part.as<double>());
    MAK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_shell_reduce, dim3(unsigned(3 * nbins)), dim3(256), 0, st, w.part.as<double>(),
                     nwg, nbins, w.sums.as<double>());
  hipLaunchKernelGGL(k_shell_finish, dim3(unsigned(ceil_div(nbins, 256))), dim3(256), 0, st,
                     w.sums.as<double>(), nbins, k_mean, power, modes);
  MAK_HIP(hipGetLastError());
}

}  // namespace mak
