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
// Transform: the unnormalised forward real-to-complex DFT, separable over
// the three axes, each a batch of one-dimensional transforms of length ng
// done in LDS by one workgroup per tile of lines.  Pass 1 transforms the
// rows of the real field (the last axis) and keeps frequencies
// 0..ng/2 (the rest are their conjugates); passes 2 and 3 transform the
// half spectrum in place along the middle and the first axis, a tile being
// a run of consecutive last-axis indices (coalesced rows).  A
// one-dimensional transform is a self-sorting (Stockham) mixed-radix FFT:
// with ng = R_1 R_2 ... R_s (radix 4 first, then 2, 3, 5, 7 and any other
// prime), stage t reads x[j + r ng / R] (r < R = R_t) for j < ng / R,
// multiplies term r by w^(r k ng / (N_t R)) (k = j mod N_t, N_t = R_1 ...
// R_(t-1), w = exp(-2 pi i / ng)), takes the length-R DFT and writes
// output q to y[(j div N_t) N_t R + k + q N_t]: after the last stage the
// transform sits in natural order.  Twiddles come from a table of w^t,
// t < ng, made once per ng with sincospi (a root of unity to within an ulp
// or two).  Radix 4 and 2 have their own butterflies; another radix forms
// each output as a sum over its R terms with one table twiddle per term.
//
// The half spectrum (ng x ng x (ng/2 + 1), last index fastest) holds
// every mode once or, for 0 < n_c < ng/2, together with its conjugate
// partner -n, so those elements count twice.  Binning: one wavefront per
// workgroup takes a contiguous range of rows (a, b) and walks each row in
// chunks of 64 elements.  Along a row |n| grows with n_c, so the shells of a
// chunk are sorted: a segmented scan over the lanes sums each shell's run and
// the run's last lane adds it to the workgroup's histogram in LDS (one writer
// per shell per step, in program order).  The histograms of the workgroups
// are then summed per shell in a fixed order, so the result is the same bits
// on every run.
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

// ------------------------------------------------------------------ FFT
constexpr int kFftThreads = 256;
constexpr int kFftMaxStages = 24;

struct FftPlan {
  int n;                       // transform length
  int nst;                     // stages
  int radix[kFftMaxStages];    // radix of each stage (product n)
};

__global__ void k_fft_twiddles(double2* __restrict__ w, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s, c;
  sincospi(2.0 * double(t) / double(n), &s, &c);
  w[t] = make_double2(c, -s);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// One-dimensional transforms of nl lines held in LDS (line t at x + t * ls),
// in place as far as the caller sees: returns the buffer holding the result.
__device__ double2* fft_lines_lds(double2* x, double2* y, const double2* __restrict__ W, const FftPlan& P,
                                  int nl, int ls) {
  const int n = P.n;
  int Ns = 1;
  for (int s = 0; s < P.nst; ++s) {
    const int R = P.radix[s];
    const int m = n / R;
    const int tw = n / (Ns * R);  // twiddle stride
    for (int idx = threadIdx.x; idx < nl * m; idx += kFftThreads) {
      const int t = idx / m, j = idx - t * m;
      const double2* xl = x + t * ls;
      double2* yl = y + t * ls;
      const int k = j % Ns;
      const int o = (j / Ns) * Ns * R + k;
      const int ts = k * tw;
      if (R == 4) {
        const double2 v0 = xl[j];
        const double2 v1 = cmul(xl[j + m], W[ts]);
        const double2 v2 = cmul(xl[j + 2 * m], W[2 * ts]);
        const double2 v3 = cmul(xl[j + 3 * m], W[3 * ts]);
        const double2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3);
        const double2 d = csub(v1, v3);
        const double2 a3 = make_double2(d.y, -d.x);  // -i (v1 - v3)
        yl[o] = cadd(a0, a2);
        yl[o + Ns] = cadd(a1, a3);
        yl[o + 2 * Ns] = csub(a0, a2);
        yl[o + 3 * Ns] = csub(a1, a3);
      } else if (R == 2) {
        const double2 a = xl[j];
        const double2 b = cmul(xl[j + m], W[ts]);
        yl[o] = cadd(a, b);
        yl[o + Ns] = csub(a, b);
      } else {
        // output q: sum_r x[j + r m] w^(r (k tw + q m)), exponents mod n
        for (int q = 0; q < R; ++q) {
          const int64_t e = int64_t(ts) + int64_t(q) * m;
          double2 acc = xl[j];
          for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(xl[j + r * m], W[(int64_t(r) * e) % n]));
          yl[o + q * Ns] = acc;
        }
      }
    }
    __syncthreads();
    double2* t = x;
    x = y;
    y = t;
    Ns *= R;
  }
  return x;
}

// LDS of the line kernels (at most 64 KB): two buffers of nl lines of ls
// elements (n + 1 when nl > 1: the padding spreads the lines over the
// banks) and, for n <= 1024, the twiddle table (longer transforms read it
// from global memory).
struct FftShape {
  int nl = 1, ls = 1;
  bool twl = true;
  size_t lds = 0;
};
FftShape fft_shape(int n) {
  FftShape f;
  f.twl = n <= 1024;
  const int budget = 4096 - (f.twl ? n : 0);  // complex doubles in 64 KB
  f.nl = budget / (2 * (n + 1));
  if (f.nl > 16) f.nl = 16;
  if (f.nl >= 2) {
    f.ls = n + 1;
  } else {
    f.nl = 1;
    f.ls = n;
  }
  f.lds = (size_t(2) * f.nl * f.ls + (f.twl ? n : 0)) * sizeof(double2);
  return f;
}

// Pass 1: rows of the real field (ng^2 rows of ng) -> half-spectrum rows
// (frequencies 0..ng/2).  Workgroup g takes rows [g nl, g nl + nl).
template <bool TWL>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_r2c(const double* __restrict__ f,
                                                               double2* __restrict__ spec,
                                                               const double2* __restrict__ tw, FftPlan P,
                                                               int nl, int ls, int64_t nrows) {
  extern __shared__ double2 lds[];
  const int n = P.n, nzh = n / 2 + 1;
  double2* X = lds;
  double2* Y = lds + nl * ls;
  const double2* W = tw;
  if (TWL) {
    double2* Wl = Y + nl * ls;
    for (int i = threadIdx.x; i < n; i += kFftThreads) Wl[i] = tw[i];
    W = Wl;
  }
  const int64_t row0 = int64_t(blockIdx.x) * nl;
  for (int idx = threadIdx.x; idx < nl * n; idx += kFftThreads) {
    const int t = idx / n, i = idx - t * n;
    const int64_t row = row0 + t;
    X[t * ls + i] = make_double2(row < nrows ? f[row * n + i] : 0.0, 0.0);
  }
  __syncthreads();
  const double2* Z = fft_lines_lds(X, Y, W, P, nl, ls);
  for (int idx = threadIdx.x; idx < nl * nzh; idx += kFftThreads) {
    const int t = idx / nzh, i = idx - t * nzh;
    const int64_t row = row0 + t;
    if (row < nrows) spec[row * nzh + i] = Z[t * ls + i];
  }
}

// Passes 2 and 3: in-place transforms of the half spectrum along an axis.
// Workgroup g = (outer, tile): lines c = tile nl + t (t < nl, c < nzh),
// element i of line c at spec[outer ostride + c + i estride].
template <bool TWL>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(double2* __restrict__ spec,
                                                           const double2* __restrict__ tw, FftPlan P,
                                                           int nl, int ls, int64_t ntile, int64_t ostride,
                                                           int64_t estride) {
  extern __shared__ double2 lds[];
  const int n = P.n, nzh = n / 2 + 1;
  double2* X = lds;
  double2* Y = lds + nl * ls;
  const double2* W = tw;
  if (TWL) {
    double2* Wl = Y + nl * ls;
    for (int i = threadIdx.x; i < n; i += kFftThreads) Wl[i] = tw[i];
    W = Wl;
  }
  const int64_t outer = int64_t(blockIdx.x) / ntile;
  const int c0 = int(int64_t(blockIdx.x) - outer * ntile) * nl;
  double2* base = spec + outer * ostride + c0;
  for (int idx = threadIdx.x; idx < nl * n; idx += kFftThreads) {
    const int i = idx / nl, t = idx - i * nl;
    X[t * ls + i] = c0 + t < nzh ? base[int64_t(i) * estride + t] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double2* Z = fft_lines_lds(X, Y, W, P, nl, ls);
  for (int idx = threadIdx.x; idx < nl * n; idx += kFftThreads) {
    const int i = idx / nl, t = idx - i * nl;
    if (c0 + t < nzh) base[int64_t(i) * estride + t] = Z[t * ls + i];
  }
}

FftPlan make_fft_plan(int64_t n) {
  FftPlan P{};
  P.n = int(n);
  int64_t r = n;
  auto take = [&](int f) {
    while (r % f == 0) {
      if (P.nst >= kFftMaxStages) MAK_FAIL(MAK_EINVAL, "FFT length with too many factors");
      P.radix[P.nst++] = f;
      r /= f;
    }
  };
  take(4);
  take(2);
  int f = 3;
  while (r > 1) {
    take(f);
    f += 2;
  }
  return P;
}

template <bool TWL>
void fft_r2c_3d(const double* field, double2* spec, const double2* tw, int64_t ng, const FftShape& F,
                hipStream_t st) {
  const FftPlan P = make_fft_plan(ng);
  const int64_t nzh = ng / 2 + 1, rows = ng * ng;
  hipLaunchKernelGGL(k_fft_rows_r2c<TWL>, dim3(unsigned(ceil_div(rows, F.nl))), dim3(kFftThreads), F.lds, st,
                     field, spec, tw, P, F.nl, F.ls, rows);
  const int64_t ntile = ceil_div(nzh, F.nl);
  // middle axis: lines over b for each (a, c)
  hipLaunchKernelGGL(k_fft_cols<TWL>, dim3(unsigned(ng * ntile)), dim3(kFftThreads), F.lds, st, spec, tw, P,
                     F.nl, F.ls, ntile, ng * nzh, nzh);
  // first axis: lines over a for each (b, c)
  hipLaunchKernelGGL(k_fft_cols<TWL>, dim3(unsigned(ng * ntile)), dim3(kFftThreads), F.lds, st, spec, tw, P,
                     F.nl, F.ls, ntile, nzh, ng * nzh);
  MAK_HIP(hipGetLastError());
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

}  // namespace


void power_spectrum(PowerWork& w, const double* field, int64_t ng, double L, int nbins, int window,
                    bool contrast, double* k_mean, double* power, int64_t* modes, hipStream_t st) {
  const int64_t nzh = ng / 2 + 1, rows = ng * ng, n = rows * ng;
  if (w.ng != ng) {
    w.tw.ensure(size_t(ng) * sizeof(double2));
    hipLaunchKernelGGL(k_fft_twiddles, dim3(unsigned(ceil_div(ng, 256))), dim3(256), 0, st, w.tw.as<double2>(), ng);
    MAK_HIP(hipGetLastError());
    w.ng = ng;
  }
  double norm = L * L * L / (double(ng) * ng * ng * double(ng) * ng * ng);
  if (contrast) {
    const double mean = dev_reduce_sum(field, n, w.tmp, st) / double(n);
    if (!(mean != 0.0) || !std::isfinite(mean))
      MAK_FAIL(MAK_EINVAL, "contrast needs a field with a finite, nonzero mean");
    norm /= mean * mean;
  }
  w.spec.ensure(size_t(rows) * nzh * sizeof(double2));
  {
    ProfScope scope("fft", st, double(n), double(n) * 8 + 5.0 * double(rows * nzh) * 16);
    const FftShape F = fft_shape(int(ng));
    if (F.twl)
      fft_r2c_3d<true>(field, w.spec.as<double2>(), w.tw.as<double2>(), ng, F, st);
    else
      fft_r2c_3d<false>(field, w.spec.as<double2>(), w.tw.as<double2>(), ng, F, st);
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
