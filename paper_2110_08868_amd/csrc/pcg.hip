// Jacobi-preconditioned conjugate gradients for the Newton system J p = g
// (J = dV/dpsi, a graph Laplacian: positive semi-definite with the constants
// as null space; g has zero mean, so CG stays in the range of J), plus the
// elementwise kernels of the Newton driver.  All reductions use a fixed grid
// and a fixed tree, so results are reproducible run to run.
#include <cfloat>

#include "engine.h"
#include "profile.h"

namespace mak {

namespace {

constexpr int TPB = 256;
constexpr int MAXB = 1024;       // blocks of the grid-stride vector kernels
constexpr int SPMV_MAXB = 8192;  // blocks of the SpMV (grid-stride over rows)

// scalar slots (device doubles)
enum { S_GAMMA = 0, S_ALPHA = 1, S_BETA = 2, S_RR = 3, S_BB = 4, S_MEAN = 5, S_TMP = 6, S_DONE = 7, S_ITER = 8 };

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum_d(v);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < TPB / WAVE; ++k) t += sh[k];
  __syncthreads();
  return t;
}

unsigned vec_blocks(int64_t n) {
  const int64_t b = ceil_div(n, TPB);
  return unsigned(b < MAXB ? (b < 1 ? 1 : b) : MAXB);
}

// CSR SpMV (the FP64 path, whose 12-byte slots make the SELL padding cost
// more than it saves): LPR lanes per row, each lane issuing UNR independent
// loads of col / val before the gathers of p (rows hold ~16 nonzeros: one
// unrolled step covers most rows, and the loads of a lane are all in flight
// at once).
constexpr int LPR = 4, UNR = 6;

// A multiple of 8: workgroup b runs on XCD b mod 8 (round-robin dispatch),
// and each XCD takes one contiguous eighth of the rows, so the gathers of p
// by its rows (spatial neighbours in the grid-sorted order) stay in its own
// L2 instead of all eight.
unsigned spmv_blocks(int64_t n) {
  int64_t b = ceil_div(n, TPB / LPR);
  b = b < SPMV_MAXB ? b : SPMV_MAXB;
  return unsigned(ceil_div(b < 1 ? 1 : b, 8) * 8);
}

// q = J p for the Laplacian form (q_i = d_i p_i - sum_j w_ij p_j),
// grid-stride over row groups, and per-block partial of p . q
template <typename W>
__global__ __launch_bounds__(TPB) void k_spmv_dot(const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const W* __restrict__ w,
                                                  const double* __restrict__ diag,
                                                  const double* __restrict__ p, double* __restrict__ q,
                                                  double* __restrict__ part, const double* __restrict__ done,
                                                  int64_t n) {
  __shared__ double sh[TPB / WAVE];
  if (done[0] != 0.0) return;  // CG converged: iterations queued after it do nothing
  const int sub = threadIdx.x & (LPR - 1);
  const int xcd = int(blockIdx.x & 7u);
  const int64_t r0 = n * xcd / 8, r1 = n * (xcd + 1) / 8;
  const int64_t step = int64_t(gridDim.x >> 3) * (TPB / LPR);
  double acc = 0.0;
  for (int64_t row = r0 + int64_t(blockIdx.x >> 3) * (TPB / LPR) + (threadIdx.x / LPR); row < r1;
       row += step) {
    const int64_t b = rp[row], e = rp[row + 1];
    double s = 0.0;
    for (int64_t k = b + sub; k < e; k += UNR * LPR) {
      int32_t c[UNR];
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t kk = k + u * LPR;
        c[u] = kk < e ? col[kk] : -1;
        v[u] = kk < e ? double(w[kk]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) s += c[u] >= 0 ? v[u] * p[c[u]] : 0.0;
    }
#pragma unroll
    for (int o = LPR / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (sub == 0) {
      const double pr = p[row];
      const double qi = diag[row] * pr - s;
      q[row] = qi;
      acc += qi * pr;
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// The same product from the SELL-64 copy (the mixed path's float weights),
// and per-block partials of p . q.  One lane per row: the
// loads of a slice's k-th entries are coalesced across the wavefront and
// independent of one another (no row-pointer chain); on the clustered 128^3
// Hessian this is 21 % faster than CSR with 4 lanes per row, despite 42 %
// padding (sorting rows by length within windows cut the padding but lost
// the gathers' locality: slower).
constexpr int SELL_UNR = 8;
template <typename W>
__global__ __launch_bounds__(TPB) void k_spmv_sell(const int64_t* __restrict__ soff,
                                                   const int32_t* __restrict__ slen,
                                                   const int32_t* __restrict__ col, const W* __restrict__ w,
                                                   const double* __restrict__ diag,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ part, const double* __restrict__ done,
                                                   int64_t n) {
  __shared__ double sh[TPB / WAVE];
  if (done[0] != 0.0) return;  // CG converged: iterations queued after it do nothing
  const int64_t nsl = (n + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int xcd = int(blockIdx.x & 7u);
  const int64_t s0 = nsl * xcd / 8, s1 = nsl * (xcd + 1) / 8;
  const int64_t step = int64_t(gridDim.x >> 3) * (TPB / 64);
  double acc = 0.0;
  for (int64_t sl = s0 + int64_t(blockIdx.x >> 3) * (TPB / 64) + (threadIdx.x / 64); sl < s1; sl += step) {
    const int64_t base = soff[sl] + lane;
    const int len = slen[sl];
    double s = 0.0;
    int k = 0;
    for (; k + SELL_UNR <= len; k += SELL_UNR) {
      int32_t c[SELL_UNR];
      double v[SELL_UNR];
#pragma unroll
      for (int u = 0; u < SELL_UNR; ++u) {
        c[u] = col[base + int64_t(k + u) * 64];
        v[u] = double(w[base + int64_t(k + u) * 64]);
      }
#pragma unroll
      for (int u = 0; u < SELL_UNR; ++u) s += v[u] * p[c[u]];
    }
    for (; k < len; ++k) s += double(w[base + int64_t(k) * 64]) * p[col[base + int64_t(k) * 64]];
    const int64_t row = sl * 64 + lane;
    if (row < n) {
      const double pr = p[row];
      const double qi = diag[row] * pr - s;
      q[row] = qi;
      acc += qi * pr;
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// A multiple of 8: workgroup b runs on XCD b mod 8 (round-robin dispatch),
// and each XCD takes one contiguous eighth of the slices, so the gathers of
// p by its rows (spatial neighbours in the grid-sorted order) stay in its
// own L2 instead of all eight.  Four slices per block per round.
unsigned sell_blocks(int64_t n) {
  int64_t b = ceil_div(ceil_div(n, 64), TPB / 64);
  b = b < SPMV_MAXB ? b : SPMV_MAXB;
  return unsigned(ceil_div(b < 1 ? 1 : b, 8) * 8);
}

// sum of part[0..np) (columns `ncol` interleaved) into scal[dst + c]
__global__ __launch_bounds__(TPB) void k_final(const double* __restrict__ part, int np, int ncol,
                                               double* __restrict__ scal, int dst0, int dst1) {
  __shared__ double sh[TPB / WAVE];
  for (int c = 0; c < ncol; ++c) {
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += TPB) v += part[i * ncol + c];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) scal[c == 0 ? dst0 : dst1] = v;
  }
}

// One step of CG in the Chronopoulos-Gear form (one reduction phase per
// iteration): p = u + beta p, s = w + beta s (s = J p kept by recurrence),
// x += alpha p, r -= alpha s, u = dinv r; partials of r.u and r.r.
__global__ __launch_bounds__(TPB) void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ u, double* __restrict__ p,
                                                   double* __restrict__ s, const double* __restrict__ w,
                                                   const double* __restrict__ dinv,
                                                   const double* __restrict__ scal, double* __restrict__ part,
                                                   int64_t n) {
  __shared__ double sh[TPB / WAVE];
  if (scal[S_DONE] != 0.0) return;  // CG converged
  const double alpha = scal[S_ALPHA], beta = scal[S_BETA];
  double aru = 0.0, arr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
    const double pi = u[i] + beta * p[i];
    const double si = w[i] + beta * s[i];
    p[i] = pi;
    s[i] = si;
    x[i] += alpha * pi;
    const double ri = r[i] - alpha * si;
    r[i] = ri;
    const double ui = dinv[i] * ri;
    u[i] = ui;
    aru += ri * ui;
    arr += ri * ri;
  }
  aru = block_sum(aru, sh);
  arr = block_sum(arr, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = aru;
    part[2 * blockIdx.x + 1] = arr;
  }
}

// gamma' = r.u, rr = r.r (from the update's partials), delta = w.u (from the
// SpMV's); beta = gamma' / gamma, alpha = gamma' / (delta - beta gamma' /
// alpha) (first: beta = 0, alpha = gamma' / delta).  Fixed tree, one block.
// After an iteration (first == 0) it counts it and raises S_DONE once
// rr <= stop: the kernels of the iterations already queued then return at
// once, so the host need not wait for each residual.
constexpr int SCAL_TPB = 1024;
__global__ __launch_bounds__(SCAL_TPB) void k_cg_scalars(const double* __restrict__ pu, int nu,
                                                         const double* __restrict__ ps, int nsp,
                                                         double* __restrict__ scal, int first, double stop) {
  __shared__ double sh[3][SCAL_TPB / WAVE];
  if (scal[S_DONE] != 0.0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nu; i += SCAL_TPB) {
    a += pu[2 * i];
    b += pu[2 * i + 1];
  }
  for (int i = threadIdx.x; i < nsp; i += SCAL_TPB) c += ps[i];
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  c = wave_sum_d(c);
  if (lane_id() == 0) {
    sh[0][threadIdx.x / WAVE] = a;
    sh[1][threadIdx.x / WAVE] = b;
    sh[2][threadIdx.x / WAVE] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = 0.0;
    for (int k = 0; k < SCAL_TPB / WAVE; ++k) {
      a += sh[0][k];
      b += sh[1][k];
      c += sh[2][k];
    }
    const double gn = a;
    double beta = 0.0, den = c;
    if (!first) {
      beta = scal[S_GAMMA] > 0.0 ? gn / scal[S_GAMMA] : 0.0;
      den = c - (scal[S_ALPHA] != 0.0 ? beta * gn / scal[S_ALPHA] : 0.0);
    }
    scal[S_ALPHA] = den > 0.0 ? gn / den : 0.0;
    scal[S_BETA] = beta;
    scal[S_GAMMA] = gn;
    scal[S_RR] = b;
    if (!first) {
      scal[S_ITER] += 1.0;
      if (b <= stop) scal[S_DONE] = 1.0;
    }
  }
}

__global__ void k_diag_inv(const double* __restrict__ diag, double* __restrict__ dinv, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = diag[i];
  dinv[i] = d > 0.0 ? 1.0 / d : 1.0;
}

__global__ __launch_bounds__(TPB) void k_sum_part(const double* __restrict__ x, double* __restrict__ part,
                                                  int64_t n) {
  __shared__ double sh[TPB / WAVE];
  double a = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
    a += x[i];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// r = b - mean (- q = J x when warm; else x = 0); u = dinv r; p = s = 0;
// partials of r.u and r.r
__global__ __launch_bounds__(TPB) void k_cg_init(const double* __restrict__ b, const double* __restrict__ scal,
                                                 const double* __restrict__ q, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ u,
                                                 double* __restrict__ p, double* __restrict__ s,
                                                 const double* __restrict__ dinv, double* __restrict__ part,
                                                 int64_t n) {
  __shared__ double sh[TPB / WAVE];
  const double mean = scal[S_MEAN] / double(n);
  double aru = 0.0, arr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
    double ri = b[i] - mean;
    if (q)
      ri -= q[i];
    else
      x[i] = 0.0;
    r[i] = ri;
    const double ui = dinv[i] * ri;
    u[i] = ui;
    p[i] = 0.0;
    s[i] = 0.0;
    aru += ri * ui;
    arr += ri * ri;
  }
  aru = block_sum(aru, sh);
  arr = block_sum(arr, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = aru;
    part[2 * blockIdx.x + 1] = arr;
  }
}

// partials of |b - mean|^2
__global__ __launch_bounds__(TPB) void k_sq_part(const double* __restrict__ b, const double* __restrict__ scal,
                                                 double* __restrict__ part, int64_t n) {
  __shared__ double sh[TPB / WAVE];
  const double mean = scal[S_MEAN] / double(n);
  double a = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
    const double v = b[i] - mean;
    a += v * v;
  }
  a = block_sum(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ void k_sub_mean(double* __restrict__ x, const double* __restrict__ scal, int slot, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] -= scal[slot] / double(n);
}

}  // namespace

int pcg_solve(const Lap& J, const double* b, double* x, int64_t n, double rtol, int max_iter,
              PcgWork& w, hipStream_t st, bool warm) {
  ProfScope whole("pcg_solve", st, double(n));
  w.r.ensure(size_t(n) * sizeof(double));
  w.z.ensure(size_t(n) * sizeof(double));
  w.p.ensure(size_t(n) * sizeof(double));
  w.q.ensure(size_t(n) * sizeof(double));
  w.s.ensure(size_t(n) * sizeof(double));
  w.dinv.ensure(size_t(n) * sizeof(double));
  const unsigned nbs = J.f32 ? sell_blocks(n) : spmv_blocks(n);
  w.part.ensure(size_t(2 * MAXB + 16) * sizeof(double));
  w.part2.ensure(size_t(nbs + 16) * sizeof(double));
  w.scal.ensure(16 * sizeof(double));
  double* r = w.r.as<double>();
  double* u = w.z.as<double>();   // preconditioned residual
  double* p = w.p.as<double>();
  double* wv = w.q.as<double>();  // J u
  double* sv = w.s.as<double>();  // J p
  double* dinv = w.dinv.as<double>();
  double* part = w.part.as<double>();
  double* part2 = w.part2.as<double>();
  double* scal = w.scal.as<double>();
  const unsigned nb = vec_blocks(n);
  const unsigned nbe = unsigned(ceil_div(n, 256));
  MAK_HIP(hipMemsetAsync(scal + S_DONE, 0, 2 * sizeof(double), st));  // S_DONE, S_ITER

  // q = J v with the partials of q . v in part2
  auto spmv = [&](const double* v, double* qv) {
    // compulsory bytes: row_ptr, diagonal, v (own row), q, and per nonzero
    // col + weight; flops 2 per nonzero + the diagonal and the dot
    const double wb = J.f32 ? 4.0 : 8.0;
    ProfScope ps("spmv", st, double(n), 32.0 * double(n) + (4.0 + wb) * double(J.nnz));
    ps.flops = 2.0 * double(J.nnz) + 4.0 * double(n);
    if (J.f32)
      hipLaunchKernelGGL(k_spmv_sell<float>, dim3(nbs), dim3(TPB), 0, st, J.soff.as<int64_t>(),
                         J.slen.as<int32_t>(), J.scol.as<int32_t>(), J.sw.as<float>(), J.diag.as<double>(), v,
                         qv, part2, scal + S_DONE, n);
    else
      hipLaunchKernelGGL(k_spmv_dot<double>, dim3(nbs), dim3(TPB), 0, st, J.row_ptr.as<int64_t>(),
                         J.col.as<int32_t>(), J.w.as<double>(), J.diag.as<double>(), v, qv, part2,
                         scal + S_DONE, n);
  };
  hipLaunchKernelGGL(k_diag_inv, dim3(nbe), dim3(256), 0, st, J.diag.as<double>(), dinv, n);
  hipLaunchKernelGGL(k_sum_part, dim3(nb), dim3(TPB), 0, st, b, part, n);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, scal, int(S_MEAN), 0);
  hipLaunchKernelGGL(k_sq_part, dim3(nb), dim3(TPB), 0, st, b, scal, part, n);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, scal, int(S_BB), 0);
  double hb[8];
  if (warm) {
    // start from the given x: r0 = b - J x; kept only if |r0| < |b|
    spmv(x, wv);
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(TPB), 0, st, b, scal, wv, x, r, u, p, sv, dinv, part, n);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 2, scal, int(S_TMP), int(S_RR));
    MAK_HIP(hipGetLastError());
    MAK_HIP(hipMemcpyAsync(hb, scal, sizeof(hb), hipMemcpyDeviceToHost, st));
    MAK_HIP(hipStreamSynchronize(st));
    if (!(hb[S_RR] < hb[S_BB])) warm = false;
  }
  if (!warm)
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(TPB), 0, st, b, scal, nullptr, x, r, u, p, sv, dinv, part,
                       n);
  spmv(u, wv);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(SCAL_TPB), 0, st, part, int(nb), part2, int(nbs), scal, 1,
                     -1.0);
  MAK_HIP(hipGetLastError());
  MAK_HIP(hipMemcpyAsync(hb, scal, sizeof(hb), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  const double bb = hb[S_BB];
  if (!(bb > 0.0)) return 0;
  const double stop = rtol * rtol * bb;
  if (hb[S_RR] <= stop) return 0;
  // The loop queues iterations ahead of the device; every 8 iterations it
  // copies the convergence flag to pinned host memory behind an event and
  // looks at the copy queued 8 iterations earlier (waiting for it only when
  // the device is that far behind), so the queue never drains.
  w.ensure_host();
  int slot = 0, pending = -1;
  bool done = false;
  for (int it = 0; it < max_iter && !done; ++it) {
    {
      ProfScope ps("pcg_update", st, double(n), 96.0 * double(n));
      ps.flops = 14.0 * double(n);
      hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(TPB), 0, st, x, r, u, p, sv, wv, dinv, scal, part, n);
    }
    spmv(u, wv);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(SCAL_TPB), 0, st, part, int(nb), part2, int(nbs), scal, 0,
                       stop);
    if ((it & 7) == 7) {
      if (pending >= 0) {
        MAK_HIP(hipEventSynchronize(w.ev[pending]));
        done = w.hflag[pending] != 0.0;
      }
      if (!done) {
        MAK_HIP(hipMemcpyAsync(&w.hflag[slot], scal + S_DONE, sizeof(double), hipMemcpyDeviceToHost, st));
        MAK_HIP(hipEventRecord(w.ev[slot], st));
        pending = slot;
        slot ^= 1;
      }
    }
  }
  double tail[2] = {0.0, 0.0};
  MAK_HIP(hipMemcpyAsync(tail, scal + S_DONE, sizeof(tail), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  const int it = int(tail[1]);
  MAK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_part, dim3(nb), dim3(TPB), 0, st, x, part, n);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, scal, int(S_TMP), 0);
  hipLaunchKernelGGL(k_sub_mean, dim3(nbe), dim3(256), 0, st, x, scal, int(S_TMP), n);
  MAK_HIP(hipGetLastError());
  return it;
}

// ---------------------------------------------------------------- Newton helpers
namespace {

// histogram of floor(log2(V / v0)) + 1 (0 below v0), 64 buckets
__global__ __launch_bounds__(256) void k_vol_hist(const double* __restrict__ vol, double v0,
                                                  unsigned long long* __restrict__ hist, int64_t n) {
  __shared__ unsigned int h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double r = vol[i] / v0;
    int b = r < 1.0 ? 0 : int(floor(log2(r))) + 1;
    b = b > 63 ? 63 : b;
    atomicAdd(&h[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_select_below(const double* __restrict__ vol, double thresh, int32_t* __restrict__ list,
                               unsigned long long* __restrict__ count, int64_t cap, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || !(vol[i] < thresh)) return;
  const unsigned long long k = atomicAdd(count, 1ull);
  if (int64_t(k) < cap) list[k] = int32_t(i);
}

__global__ void k_axpy_into(const double* __restrict__ a, const double* __restrict__ b, double alpha,
                            double* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + alpha * b[i];
}

// target masses: per site (ms, sorted order) or uniform (m when ms is NULL)
__global__ void k_residual(const double* __restrict__ vol, double m, const double* __restrict__ ms,
                           double* __restrict__ g, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) g[i] = (ms ? ms[i] : m) - vol[i];
}

// partials: max |m_i - V_i| / m_i, min V, sum (m_i - V_i)^2
__global__ __launch_bounds__(TPB) void k_res_stats(const double* __restrict__ vol, double m,
                                                   const double* __restrict__ ms,
                                                   double* __restrict__ part, int64_t n) {
  __shared__ double sh[TPB];
  double amax = 0.0, vmin = DBL_MAX, ss = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
    const double mi = ms ? ms[i] : m;
    const double g = mi - vol[i];
    amax = fmax(amax, fabs(g) / mi);
    vmin = fmin(vmin, vol[i]);
    ss += g * g;
  }
  amax = wave_max_d(amax);
  vmin = -wave_max_d(-vmin);
  ss = wave_sum_d(ss);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sh[3 * w] = amax;
    sh[3 * w + 1] = vmin;
    sh[3 * w + 2] = ss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < TPB / WAVE; ++k) {
      sh[0] = fmax(sh[0], sh[3 * k]);
      sh[1] = fmin(sh[1], sh[3 * k + 1]);
      sh[2] += sh[3 * k + 2];
    }
    part[3 * blockIdx.x] = sh[0];
    part[3 * blockIdx.x + 1] = sh[1];
    part[3 * blockIdx.x + 2] = sh[2];
  }
}

__global__ void k_res_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, v = DBL_MAX, s = 0.0;
  for (int k = 0; k < np; ++k) {
    a = fmax(a, part[3 * k]);
    v = fmin(v, part[3 * k + 1]);
    s += part[3 * k + 2];
  }
  out[0] = a;
  out[1] = v;
  out[2] = s;
}

__device__ __forceinline__ double wrap1(double v, double L) {
  v = fmod(v, L);
  if (v < 0) v += L;
  if (!(v < L)) v = 0.0;
  return v;
}

__global__ void k_finalize(const double4* __restrict__ pts, const int32_t* __restrict__ perm,
                           const double* __restrict__ psi_s, const double* __restrict__ mean_slot,
                           const double* __restrict__ vol, const double* __restrict__ mom, double L,
                           double* __restrict__ psi_out, double* __restrict__ cent,
                           double* __restrict__ disp, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t o = perm[p];
  const double4 x = pts[p];
  const double v = vol[p];
  double u0 = 0.0, u1 = 0.0, u2 = 0.0;
  if (v > 0.0) {
    u0 = mom[3 * p] / v;
    u1 = mom[3 * p + 1] / v;
    u2 = mom[3 * p + 2] / v;
  }
  if (psi_out) psi_out[o] = psi_s[p] - mean_slot[0] / double(n);
  cent[3 * o] = wrap1(x.x + u0, L);
  cent[3 * o + 1] = wrap1(x.y + u1, L);
  cent[3 * o + 2] = wrap1(x.z + u2, L);
  if (disp) {
    disp[3 * o] = -u0;
    disp[3 * o + 1] = -u1;
    disp[3 * o + 2] = -u2;
  }
}

__global__ void k_scatter_vol(const int32_t* __restrict__ perm, const double* __restrict__ vs,
                              double* __restrict__ vo, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) vo[perm[p]] = vs[p];
}

__global__ void k_gather(const int32_t* __restrict__ perm, const double* __restrict__ orig,
                         double* __restrict__ sorted, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) sorted[p] = orig[perm[p]];
}

}  // namespace

void axpy_into(const double* a, const double* b, double alpha, double* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_into, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st, a, b, alpha, out, n);
  MAK_HIP(hipGetLastError());
}

void newton_residual(const double* vol, double m, const double* ms, double* g, int64_t n,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st, vol, m, ms, g, n);
  MAK_HIP(hipGetLastError());
}

double residual_stats(const double* vol, double m, const double* ms, int64_t n, DevBuf& tmp,
                      double* max_rel, double* min_vol, hipStream_t st) {
  tmp.ensure(size_t(3 * MAXB + 8) * sizeof(double));
  double* part = tmp.as<double>();
  const unsigned nb = vec_blocks(n);
  hipLaunchKernelGGL(k_res_stats, dim3(nb), dim3(TPB), 0, st, vol, m, ms, part, n);
  hipLaunchKernelGGL(k_res_final, dim3(1), dim3(64), 0, st, part, int(nb), part + 3 * MAXB);
  MAK_HIP(hipGetLastError());
  double h[3];
  MAK_HIP(hipMemcpyAsync(h, part + 3 * MAXB, sizeof(h), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  *max_rel = h[0];
  *min_vol = h[1];
  return std::sqrt(h[2]);
}

void finalize_outputs(const PointSet& ps, const double* psi_sorted, double psi_mean_unused,
                      const double* vol, const double* mom, double* psi_out, double* cent_out,
                      double* disp_out, hipStream_t st) {
  (void)psi_mean_unused;
  const int64_t n = ps.N;
  // mean of psi (device), then the permuted outputs
  DevBuf& tmp = const_cast<PointSet&>(ps).tmp;
  tmp.ensure(size_t(MAXB + 16) * sizeof(double));
  double* part = tmp.as<double>();
  const unsigned nb = vec_blocks(n);
  if (psi_out) {
    hipLaunchKernelGGL(k_sum_part, dim3(nb), dim3(TPB), 0, st, psi_sorted, part, n);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, part + MAXB, 0, 0);
  }
  hipLaunchKernelGGL(k_finalize, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st,
                     ps.pts.as<double4>(), ps.perm.as<int32_t>(), psi_sorted, part + MAXB, vol, mom,
                     ps.g.L, psi_out, cent_out, disp_out, n);
  MAK_HIP(hipGetLastError());
}

void scatter_cells_outputs(const PointSet& ps, const double* vol_s, const double* mom_s,
                           double* vol_out, double* cent_out, hipStream_t st) {
  const int64_t n = ps.N;
  hipLaunchKernelGGL(k_scatter_vol, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st,
                     ps.perm.as<int32_t>(), vol_s, vol_out, n);
  if (cent_out)
    hipLaunchKernelGGL(k_finalize, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st,
                       ps.pts.as<double4>(), ps.perm.as<int32_t>(), nullptr, nullptr, vol_s, mom_s,
                       ps.g.L, nullptr, cent_out, nullptr, n);
  MAK_HIP(hipGetLastError());
}

void gather_sorted(const PointSet& ps, const double* orig, double* sorted, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(unsigned(ceil_div(ps.N, 256))), dim3(256), 0, st,
                     ps.perm.as<int32_t>(), orig, sorted, ps.N);
  MAK_HIP(hipGetLastError());
}

int64_t smallest_cells(const double* vol, double v0, int32_t* list, int64_t cap, int64_t n, DevBuf& tmp,
                       hipStream_t st) {
  tmp.ensure(66 * sizeof(unsigned long long));
  unsigned long long* hist = tmp.as<unsigned long long>();
  MAK_HIP(hipMemsetAsync(hist, 0, 66 * sizeof(unsigned long long), st));
  const unsigned nb = unsigned(std::min<int64_t>(ceil_div(n, 256), 2048));
  hipLaunchKernelGGL(k_vol_hist, dim3(nb), dim3(256), 0, st, vol, v0, hist, n);
  unsigned long long h[64];
  MAK_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  // the largest power-of-two bound below which at most cap cells lie
  int64_t cum = 0;
  int b = 0;
  while (b < 64 && cum + int64_t(h[b]) <= cap) cum += int64_t(h[b++]);
  if (cum == 0) return 0;
  hipLaunchKernelGGL(k_select_below, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st, vol,
                     std::ldexp(v0, b - 1), list, hist + 64, cap, n);
  MAK_HIP(hipGetLastError());
  unsigned long long got = 0;
  MAK_HIP(hipMemcpyAsync(&got, hist + 64, sizeof(got), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  return std::min<int64_t>(int64_t(got), cap);
}

}  // namespace mak
