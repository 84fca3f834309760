// Device-wide scans and deterministic reductions (fixed grid, fixed tree).
#include <cfloat>

#include "engine.h"

namespace mak {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename TI, typename TO>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile(const TI* in, TO* out, TO* tile_sums,
                                                            int64_t n) {
  __shared__ TO warp_tot[SCAN_THREADS / WAVE];
  const int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_ITEMS;
  TO v[SCAN_ITEMS];
  TO run = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? TO(in[i]) : TO(0);
    run += v[k];
  }
  // inclusive scan of per-thread totals over the block
  TO incl = run;
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const TO t = __shfl_up(incl, o);
    if (l >= o) incl += t;
  }
  const int w = threadIdx.x / WAVE;
  if (l == WAVE - 1) warp_tot[w] = incl;
  __syncthreads();
  TO woff = 0;
  for (int k = 0; k < w; ++k) woff += warp_tot[k];
  TO excl = woff + incl - run;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = excl;
    excl += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1) tile_sums[blockIdx.x] = excl;
}

template <typename TO>
__global__ void k_scan_add(TO* out, const TO* tile_off, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / SCAN_TILE];
}

template <typename TI, typename TO>
__global__ void k_scan_total(const TI* in, TO* out, int64_t n) {
  out[n] = n > 0 ? out[n - 1] + TO(in[n - 1]) : TO(0);
}

// Exclusive scan of n values into out[0..n], out[n] = total.  `tmp` holds the
// tile sums of every recursion level.
template <typename TI, typename TO>
void scan_impl(const TI* in, TO* out, int64_t n, TO* tmp, hipStream_t st) {
  const int64_t tiles = ceil_div(n, SCAN_TILE);
  if (tiles > 0) {
    TO* sums = tmp;
    hipLaunchKernelGGL((k_scan_tile<TI, TO>), dim3(unsigned(tiles)), dim3(SCAN_THREADS), 0, st, in,
                       out, sums, n);
    if (tiles > 1) {
      TO* offs = tmp + tiles + 1;
      scan_impl<TO, TO>(sums, offs, tiles, offs + tiles + 1, st);
      hipLaunchKernelGGL((k_scan_add<TO>), dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st, out,
                         offs, n);
    }
  }
  hipLaunchKernelGGL((k_scan_total<TI, TO>), dim3(1), dim3(1), 0, st, in, out, n);
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t s = 0;
  while (true) {
    const int64_t t = ceil_div(n, SCAN_TILE);
    s += 2 * (t + 1);
    if (t <= 1) break;
    n = t;
  }
  return s + 8;
}

// ---------------------------------------------------------------- reductions
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

struct OpSum {
  __device__ static double id() { return 0.0; }
  __device__ static double f(double a, double b) { return a + b; }
};
struct OpMax {
  __device__ static double id() { return -DBL_MAX; }
  __device__ static double f(double a, double b) { return fmax(a, b); }
};
struct OpMin {
  __device__ static double id() { return DBL_MAX; }
  __device__ static double f(double a, double b) { return fmin(a, b); }
};

template <class Op>
__device__ double block_reduce(double v) {
  __shared__ double sh[RED_THREADS];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] = Op::f(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

template <class Op>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_partial(const double* x, int64_t n,
                                                                double* part) {
  double v = Op::id();
  for (int64_t i = int64_t(blockIdx.x) * RED_THREADS + threadIdx.x; i < n;
       i += int64_t(RED_BLOCKS) * RED_THREADS)
    v = Op::f(v, x[i]);
  v = block_reduce<Op>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

template <class Op>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const double* part, int np,
                                                              double* out) {
  double v = Op::id();
  for (int i = threadIdx.x; i < np; i += RED_THREADS) v = Op::f(v, part[i]);
  v = block_reduce<Op>(v);
  if (threadIdx.x == 0) *out = v;
}

template <class Op>
double reduce_host(const double* x, int64_t n, DevBuf& tmp, hipStream_t st) {
  tmp.ensure((RED_BLOCKS + 8) * sizeof(double));
  double* part = tmp.as<double>();
  hipLaunchKernelGGL((k_reduce_partial<Op>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, x, n,
                     part);
  hipLaunchKernelGGL((k_reduce_final<Op>), dim3(1), dim3(RED_THREADS), 0, st, part, RED_BLOCKS,
                     part + RED_BLOCKS);
  double h = 0;
  MAK_HIP(hipMemcpyAsync(&h, part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  return h;
}

}  // namespace

namespace {
// The scans write n + 1 entries (the total last): refuse an output buffer
// that cannot hold them instead of writing past its end.
void check_scan_out(const DevBuf& out, int64_t n, size_t elem) {
  if (n < 0 || !out.p || out.cap < size_t(n + 1) * elem)
    MAK_FAIL(MAK_EHIP, "exclusive scan of " + std::to_string(n) + " entries: output buffer holds " +
                           std::to_string(out.cap / elem) + " (needs n + 1)");
}
}  // namespace

size_t scan_tmp_bytes_i32(int64_t n) { return size_t(scan_tmp_elems(n)) * sizeof(int32_t); }
size_t reduce_tmp_bytes() { return (RED_BLOCKS + 8) * sizeof(double); }

namespace {
__global__ void k_fill_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
}  // namespace

void fill_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st, p, n);
  MAK_HIP(hipGetLastError());
}

void exclusive_scan_i64(const int64_t* in, DevBuf& out, int64_t n, DevBuf& tmp, hipStream_t st) {
  check_scan_out(out, n, sizeof(int64_t));
  tmp.ensure(size_t(scan_tmp_elems(n)) * sizeof(int64_t));
  scan_impl<int64_t, int64_t>(in, out.as<int64_t>(), n, tmp.as<int64_t>(), st);
  MAK_HIP(hipGetLastError());
}

void exclusive_scan_i32(const int32_t* in, DevBuf& out, int64_t n, DevBuf& tmp, hipStream_t st) {
  check_scan_out(out, n, sizeof(int32_t));
  tmp.ensure(size_t(scan_tmp_elems(n)) * sizeof(int32_t));
  scan_impl<int32_t, int32_t>(in, out.as<int32_t>(), n, tmp.as<int32_t>(), st);
  MAK_HIP(hipGetLastError());
}

double dev_reduce_max(const double* x, int64_t n, DevBuf& tmp, hipStream_t st) {
  return reduce_host<OpMax>(x, n, tmp, st);
}
double dev_reduce_min(const double* x, int64_t n, DevBuf& tmp, hipStream_t st) {
  return reduce_host<OpMin>(x, n, tmp, st);
}
double dev_reduce_sum(const double* x, int64_t n, DevBuf& tmp, hipStream_t st) {
  return reduce_host<OpSum>(x, n, tmp, st);
}

// Device-side max into a device scalar (no host round trip).
void dev_max_to(const double* x, int64_t n, double* out, DevBuf& tmp, hipStream_t st) {
  tmp.ensure((RED_BLOCKS + 8) * sizeof(double));
  double* part = tmp.as<double>();
  hipLaunchKernelGGL((k_reduce_partial<OpMax>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, x, n,
                     part);
  hipLaunchKernelGGL((k_reduce_final<OpMax>), dim3(1), dim3(RED_THREADS), 0, st, part, RED_BLOCKS,
                     out);
  MAK_HIP(hipGetLastError());
}

}  // namespace mak
