// Jacobi-preconditioned conjugate gradients for the Newton system J p = g
// (J = dV/dpsi, a graph Laplacian: positive semi-definite with the constants
// as null space; g has zero mean, so CG stays in the range of J), plus the
// elementwise kernels of the Newton driver.  All reductions use a fixed grid
// and a fixed tree, so results are reproducible run to run.
#include <algorithm>
#include <cfloat>

#include "engine.h"
#include "profile.h"

namespace mak {

namespace {

constexpr int TPB = 256;
constexpr int MAXB = 1024;       // blocks of the grid-stride vector kernels
constexpr int SPMV_MAXB = 8192;  // blocks of the SpMV (grid-stride over rows)

// scalar slots (device doubles)
enum { S_GAMMA = 0, S_ALPHA = 1, S_BETA = 2, S_RR = 3, S_BB = 4, S_MEAN = 5, S_TMP = 6, S_DONE = 7, S_ITER = 8,
       S_CDOT = 9 };

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
                                                         double* __restrict__ scal, int first, double stop,
                                                         int coarse) {
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
    const double gn = a + (coarse ? scal[S_CDOT] : 0.0);  // r.u with the coarse levels' part
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

// ---------------------------------------------------------------- three-level preconditioner
// M^-1 r = D^-1 r + P1 D1^-1 P1' r + P1 P2 A2^+ P2' P1' r: point Jacobi, plus
// Jacobi on the aggregates of the neighbour-grid blocks (P1 sums the rows of
// a block; D1 is the diagonal of the Galerkin product P1' J P1, the weight
// leaving the block), plus an exact solve on nd^3 <= 64 aggregates of
// dv^3 blocks (A2 = P2' P1' J P1 P2, a Laplacian, pinned at aggregate 0).
// Every term is symmetric positive semi-definite, so M is a valid CG
// preconditioner.  The sums over a block run in one wavefront in a fixed
// order: the results are the same bits on every run.
constexpr int ML_WPB = TPB / WAVE;  // wavefronts (blocks) per workgroup
constexpr int ML_MAXC = 512;        // aggregates of the exact level (8 per axis)
constexpr int ML_LDSC = 64;         // at most this many: the exact level is inverted in LDS

struct MlGeo {
  const int32_t* cs;  // cell_start: block b rows [cs[64 b], cs[64 b + 64])
  int32_t Gb, dv, nd;
  int64_t nblk;
};

__device__ __forceinline__ int ml_agg(int64_t b, const MlGeo& g) {
  const int bx = int(b / (int64_t(g.Gb) * g.Gb)), by = int((b / g.Gb) % g.Gb), bz = int(b % g.Gb);
  return ((bx / g.dv) * g.nd + by / g.dv) * g.nd + bz / g.dv;
}

__global__ void k_ml_blk_rows(MlGeo g, int32_t* __restrict__ blk_row) {
  const int64_t b = int64_t(blockIdx.x) * ML_WPB + threadIdx.x / WAVE;
  if (b >= g.nblk) return;
  for (int32_t i = g.cs[64 * b] + lane_id(); i < g.cs[64 * b + 64]; i += WAVE) blk_row[i] = int32_t(b);
}

// Per block: 1 / (weight leaving it) and its weights towards the 26
// neighbouring aggregates of the exact level (slot (dx+1) 9 + (dy+1) 3 +
// (dz+1), aggregate offsets wrapped periodically; an edge to an aggregate
// farther than one step is left out of the exact level only).
template <typename W>
__global__ __launch_bounds__(TPB) void k_ml_setup(MlGeo g, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const W* __restrict__ w,
                                                  const int32_t* __restrict__ blk_row,
                                                  double* __restrict__ d1inv, double* __restrict__ a1c) {
  const int64_t b = int64_t(blockIdx.x) * ML_WPB + threadIdx.x / WAVE;
  if (b >= g.nblk) return;
  const int G = g.Gb, nd = g.nd, dv = g.dv;
  const int bx = int(b / (int64_t(G) * G)), by = int((b / G) % G), bz = int(b % G);
  const int cx = bx / dv, cy = by / dv, cz = bz / dv;
  double out = 0.0;
  double acc[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = 0.0;
  for (int32_t i = g.cs[64 * b] + lane_id(); i < g.cs[64 * b + 64]; i += WAVE) {
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t bj = blk_row[col[k]];
      if (bj == b) continue;
      const double wt = double(w[k]);
      out += wt;
      const int jx = int(bj / (G * G)), jy = (bj / G) % G, jz = bj % G;
      auto wrap = [nd](int d) {  // aggregate offset in (-nd/2, nd/2]
        d %= nd;
        if (d < 0) d += nd;
        return 2 * d > nd ? d - nd : d;
      };
      const int dx = wrap(jx / dv - cx), dy = wrap(jy / dv - cy), dz = wrap(jz / dv - cz);
      if ((dx | dy | dz) == 0 || dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) continue;
      const int slot = (dx + 1) * 9 + (dy + 1) * 3 + (dz + 1);
#pragma unroll
      for (int q = 0; q < 27; ++q) acc[q] += q == slot ? wt : 0.0;
    }
  }
  out = wave_sum_d(out);
#pragma unroll
  for (int q = 0; q < 27; ++q) acc[q] = wave_sum_d(acc[q]);
  if (lane_id() == 0) {
    d1inv[b] = out > 0.0 ? 1.0 / out : 0.0;
#pragma unroll
    for (int q = 0; q < 27; ++q) a1c[27 * b + q] = acc[q];
  }
}

// Block b of aggregate c: the li-th block in x-major order of the
// aggregate's dv^3 (fewer at the far end when dv does not divide Gb), or -1.
__device__ __forceinline__ int64_t ml_agg_block(const MlGeo& g, int c, int li) {
  const int nd = g.nd, dv = g.dv;
  const int bx = (c / (nd * nd)) * dv + li / (dv * dv), by = ((c / nd) % nd) * dv + (li / dv) % dv,
            bz = (c % nd) * dv + li % dv;
  if (bx >= g.Gb || by >= g.Gb || bz >= g.Gb) return -1;
  return (int64_t(bx) * g.Gb + by) * g.Gb + bz;
}

// Per aggregate of the exact level (one workgroup each): its blocks' weights
// towards the 26 neighbouring aggregates summed per slot, nine groups of 27
// threads each taking every ninth block, then the groups in a fixed order.
constexpr int ML_AGG_TPB = 256;
__global__ __launch_bounds__(ML_AGG_TPB) void k_ml_aggsum(MlGeo g, const double* __restrict__ a1c,
                                                          double* __restrict__ aggw) {
  __shared__ double part[9][27];
  const int c = blockIdx.x;
  const int t = threadIdx.x, grp = t / 27, q = t % 27;
  const int nblk = g.dv * g.dv * g.dv;
  if (grp < 9) {
    double v = 0.0;
    for (int li = grp; li < nblk; li += 9) {
      const int64_t b = ml_agg_block(g, c, li);
      if (b >= 0) v += a1c[27 * b + q];
    }
    part[grp][q] = v;
  }
  __syncthreads();
  if (t < 27) {
    double v = 0.0;
    for (int k = 0; k < 9; ++k) v += part[k][t];
    aggw[27 * c + t] = v;
  }
}

// The exact level: A2 from the aggregates' neighbour weights, symmetrised,
// its diagonal the row sums, pinned at aggregate 0, inverted in LDS by
// Gauss-Jordan elimination (no pivoting: the pinned Laplacian of a
// connected set of aggregates is positive definite; a zero pivot, from an
// aggregate with no weight to the others, leaves its row and column zero).
__global__ __launch_bounds__(256) void k_ml_dense(MlGeo g, const double* __restrict__ aggw,
                                                   double* __restrict__ ainv) {
  __shared__ double A[ML_LDSC][ML_LDSC];
  __shared__ double rowk[ML_LDSC], fcol[ML_LDSC];
  const int nc = g.nd * g.nd * g.nd;
  const int t = threadIdx.x;
  for (int e = t; e < ML_LDSC * ML_LDSC; e += 256) A[e / ML_LDSC][e % ML_LDSC] = 0.0;
  __syncthreads();
  if (t < nc) {
    const int nd = g.nd;
    const int cx = t / (nd * nd), cy = (t / nd) % nd, cz = t % nd;
    for (int q = 0; q < 27; ++q) {
      const double v = aggw[27 * t + q];
      if (v == 0.0) continue;
      const int ox = (cx + q / 9 - 1 + nd) % nd, oy = (cy + (q / 3) % 3 - 1 + nd) % nd,
                oz = (cz + q % 3 - 1 + nd) % nd;
      const int c2 = (ox * nd + oy) * nd + oz;
      if (c2 != t) A[t][c2] -= v;
    }
  }
  __syncthreads();
  // symmetrise the off-diagonal part (the two sides of a face are computed
  // apart), then the diagonal = minus the off-diagonal row sum
  double sym[ML_LDSC * ML_LDSC / 256];
  for (int e = t, k = 0; e < ML_LDSC * ML_LDSC; e += 256, ++k) {
    const int i = e / ML_LDSC, j = e % ML_LDSC;
    sym[k] = (i < nc && j < nc && i != j) ? 0.5 * (A[i][j] + A[j][i]) : 0.0;
  }
  __syncthreads();
  for (int e = t, k = 0; e < ML_LDSC * ML_LDSC; e += 256, ++k) A[e / ML_LDSC][e % ML_LDSC] = sym[k];
  __syncthreads();
  if (t < nc) {
    double sum = 0.0;
    for (int j = 0; j < nc; ++j) sum += A[t][j];
    fcol[t] = -sum;
  }
  __syncthreads();
  if (t < nc) A[t][t] = fcol[t];
  __syncthreads();
  if (t < nc) {  // pin aggregate 0
    A[0][t] = t == 0 ? 1.0 : 0.0;
    A[t][0] = t == 0 ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < nc; ++k) {
    const double piv = A[k][k];
    const double ip = piv > 0.0 ? 1.0 / piv : 0.0;
    __syncthreads();
    if (t < nc) {
      rowk[t] = (t == k ? 1.0 : A[k][t]) * ip;
      fcol[t] = t == k ? 0.0 : A[t][k];
    }
    __syncthreads();
    for (int e = t; e < nc * nc; e += 256) {
      const int i = e / nc, j = e % nc;
      if (i == k)
        A[i][j] = rowk[j];
      else
        A[i][j] = (j == k ? 0.0 : A[i][j]) - fcol[i] * rowk[j];
    }
    __syncthreads();
  }
  for (int e = t; e < nc * nc; e += 256) ainv[e] = A[e / nc][e % nc];
}

// The same for up to ML_MAXC aggregates (more than fit in LDS): the matrix
// is built and eliminated in global memory (the output buffer) by one
// workgroup; the pivot row and column of each step are staged in LDS.
__global__ __launch_bounds__(1024) void k_ml_dense_big(MlGeo g, const double* __restrict__ aggw,
                                                        double* __restrict__ A) {
  __shared__ double rowk[ML_MAXC], fcol[ML_MAXC];
  const int nc = g.nd * g.nd * g.nd;
  const int t = threadIdx.x;
  constexpr int nt = 1024;
  for (int e = t; e < nc * nc; e += nt) A[e] = 0.0;
  __syncthreads();
  for (int c = t; c < nc; c += nt) {
    const int nd = g.nd;
    const int cx = c / (nd * nd), cy = (c / nd) % nd, cz = c % nd;
    for (int q = 0; q < 27; ++q) {
      const double v = aggw[27 * c + q];
      if (v == 0.0) continue;
      const int ox = (cx + q / 9 - 1 + nd) % nd, oy = (cy + (q / 3) % 3 - 1 + nd) % nd,
                oz = (cz + q % 3 - 1 + nd) % nd;
      const int c2 = (ox * nd + oy) * nd + oz;
      if (c2 != c) A[c * nc + c2] -= v;
    }
  }
  __syncthreads();
  // symmetrise the off-diagonal part (each pair by one thread), the
  // diagonal = minus the off-diagonal row sum, pin aggregate 0
  for (int e = t; e < nc * nc; e += nt) {
    const int i = e / nc, j = e % nc;
    if (i < j) {
      const double v = 0.5 * (A[i * nc + j] + A[j * nc + i]);
      A[i * nc + j] = v;
      A[j * nc + i] = v;
    }
  }
  __syncthreads();
  for (int c = t; c < nc; c += nt) {
    double sum = 0.0;
    for (int j = 0; j < nc; ++j) sum += j == c ? 0.0 : A[c * nc + j];
    fcol[c] = -sum;
  }
  __syncthreads();
  for (int c = t; c < nc; c += nt) A[c * nc + c] = fcol[c];
  __syncthreads();
  for (int c = t; c < nc; c += nt) {
    A[c] = c == 0 ? 1.0 : 0.0;
    A[c * nc] = c == 0 ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < nc; ++k) {
    const double piv = A[k * nc + k];
    const double ip = piv > 0.0 ? 1.0 / piv : 0.0;
    __syncthreads();
    for (int c = t; c < nc; c += nt) {
      rowk[c] = (c == k ? 1.0 : A[k * nc + c]) * ip;
      fcol[c] = c == k ? 0.0 : A[c * nc + k];
    }
    __syncthreads();
    for (int e = t; e < nc * nc; e += nt) {
      const int i = e / nc, j = e % nc;
      if (i == k)
        A[e] = rowk[j];
      else
        A[e] = (j == k ? 0.0 : A[e]) - fcol[i] * rowk[j];
    }
    __syncthreads();
  }
}

// r = b - mean (- q = J x when warm; else x = 0); p = s = 0; per block the
// sum of r; partials of r.(D^-1 r) and r.r.  One wavefront per block.
__global__ __launch_bounds__(TPB) void k_ml_init(MlGeo g, const double* __restrict__ b,
                                                 const double* __restrict__ scal, const double* __restrict__ q,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ p, double* __restrict__ s,
                                                 const double* __restrict__ dinv, double* __restrict__ r1,
                                                 const double* __restrict__ d1inv, double* __restrict__ part,
                                                 int64_t n) {
  __shared__ double sh[TPB / WAVE];
  const double mean = scal[S_MEAN] / double(n);
  double aru = 0.0, arr = 0.0;
  for (int64_t blk = int64_t(blockIdx.x) * ML_WPB + threadIdx.x / WAVE; blk < g.nblk;
       blk += int64_t(gridDim.x) * ML_WPB) {
    double rs = 0.0;
    for (int32_t i = g.cs[64 * blk] + lane_id(); i < g.cs[64 * blk + 64]; i += WAVE) {
      double ri = b[i] - mean;
      if (q)
        ri -= q[i];
      else
        x[i] = 0.0;
      r[i] = ri;
      p[i] = 0.0;
      s[i] = 0.0;
      aru += ri * dinv[i] * ri;
      arr += ri * ri;
      rs += ri;
    }
    rs = wave_sum_d(rs);
    if (lane_id() == 0) {
      r1[blk] = rs;
      aru += rs * d1inv[blk] * rs;  // the block level's part of r.u
    }
  }
  aru = block_sum(aru, sh);
  arr = block_sum(arr, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = aru;
    part[2 * blockIdx.x + 1] = arr;
  }
}

// The CG update of k_cg_update without the preconditioned residual (it
// needs the coarse levels of the new r): p = u + beta p, s = w + beta s,
// x += alpha p, r -= alpha s; per block the sum of r; partials of
// r.(D^-1 r) and r.r.
__global__ __launch_bounds__(TPB) void k_ml_update(MlGeo g, double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ u, double* __restrict__ p,
                                                   double* __restrict__ s, const double* __restrict__ w,
                                                   const double* __restrict__ dinv,
                                                   const double* __restrict__ scal, double* __restrict__ r1,
                                                   const double* __restrict__ d1inv, double* __restrict__ part) {
  __shared__ double sh[TPB / WAVE];
  if (scal[S_DONE] != 0.0) return;
  const double alpha = scal[S_ALPHA], beta = scal[S_BETA];
  double aru = 0.0, arr = 0.0;
  for (int64_t blk = int64_t(blockIdx.x) * ML_WPB + threadIdx.x / WAVE; blk < g.nblk;
       blk += int64_t(gridDim.x) * ML_WPB) {
    double rs = 0.0;
    for (int32_t i = g.cs[64 * blk] + lane_id(); i < g.cs[64 * blk + 64]; i += WAVE) {
      const double pi = u[i] + beta * p[i];
      const double si = w[i] + beta * s[i];
      p[i] = pi;
      s[i] = si;
      x[i] += alpha * pi;
      const double ri = r[i] - alpha * si;
      r[i] = ri;
      aru += ri * dinv[i] * ri;
      arr += ri * ri;
      rs += ri;
    }
    rs = wave_sum_d(rs);
    if (lane_id() == 0) {
      r1[blk] = rs;
      aru += rs * d1inv[blk] * rs;  // the block level's part of r.u
    }
  }
  aru = block_sum(aru, sh);
  arr = block_sum(arr, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = aru;
    part[2 * blockIdx.x + 1] = arr;
  }
}

// The exact level in one workgroup: the aggregates' residuals (tpa threads
// per aggregate, sixteen for up to 64 aggregates, two for 512, each summing
// every tpa-th block, then a fixed tree), the solve e = A2^+ r_agg (tpa
// threads per row), and its part of r.u, sum_agg r_agg e_agg (the
// correction is constant over an aggregate).  The block level's part of r.u
// comes from the update kernel.
constexpr int ML_CTPB = 1024;
__global__ __launch_bounds__(ML_CTPB) void k_ml_coarse(MlGeo g, const double* __restrict__ r1,
                                                       const double* __restrict__ ainv, double* __restrict__ ec,
                                                       double* __restrict__ scal) {
  __shared__ double rc[ML_MAXC], es[ML_MAXC];
  static_assert(ML_CTPB >= 2 * ML_MAXC, "two threads per aggregate at least");
  if (scal[S_DONE] != 0.0) return;
  const int nc = g.nd * g.nd * g.nd;
  int tpa = 16;
  while (tpa * nc > ML_CTPB) tpa >>= 1;
  const int t = threadIdx.x, c = t / tpa, sl = t % tpa;
  const int nblk = g.dv * g.dv * g.dv;
  double v = 0.0;
  if (c < nc) {
#pragma unroll 4
    for (int li = sl; li < nblk; li += tpa) {
      const int64_t b = ml_agg_block(g, c, li);
      if (b >= 0) v += r1[b];
    }
  }
  for (int o = tpa / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (c < nc && sl == 0) rc[c] = c == 0 ? 0.0 : v;  // pinned aggregate
  __syncthreads();
  double e = 0.0;
  if (c < nc)
    for (int j = sl; j < nc; j += tpa) e += ainv[int64_t(c) * nc + j] * rc[j];
  for (int o = tpa / 2; o >= 1; o >>= 1) e += __shfl_xor(e, o);
  if (c < nc && sl == 0) {
    e = c == 0 ? 0.0 : e;
    ec[c] = e;
    es[c] = e;
  }
  __syncthreads();
  if (t == 0) {
    double d = 0.0;
    for (int k = 0; k < nc; ++k) d += rc[k] * es[k];
    scal[S_CDOT] = d;
  }
}

// u = D^-1 r + r1_b / D1_b + e_agg(b), the correction constant over block b
__global__ __launch_bounds__(TPB) void k_ml_apply(MlGeo g, const double* __restrict__ r,
                                                  const double* __restrict__ dinv, const double* __restrict__ r1,
                                                  const double* __restrict__ d1inv, const double* __restrict__ ec,
                                                  double* __restrict__ u, const double* __restrict__ scal) {
  if (scal[S_DONE] != 0.0) return;
  for (int64_t blk = int64_t(blockIdx.x) * ML_WPB + threadIdx.x / WAVE; blk < g.nblk;
       blk += int64_t(gridDim.x) * ML_WPB) {
    const double c = r1[blk] * d1inv[blk] + ec[ml_agg(blk, g)];
    for (int32_t i = g.cs[64 * blk] + lane_id(); i < g.cs[64 * blk + 64]; i += WAVE) u[i] = dinv[i] * r[i] + c;
  }
}

}  // namespace

int pcg_solve(const Lap& J, const double* b, double* x, int64_t n, double rtol, int max_iter,
              PcgWork& w, hipStream_t st, bool warm, const RowBlocks* blocks) {
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
  // three-level preconditioner: geometry, the blocks' weights and the exact
  // level's inverse for this J
  const bool ml = blocks && blocks->cell_start && blocks->Gb >= 1;
  MlGeo geo{};
  unsigned nbm = 1;
  if (ml) {
    geo.cs = blocks->cell_start;
    geo.Gb = blocks->Gb;
    // at most 4 aggregates per axis (inverted in LDS) unless the caller asks
    // for 8 (up to 512 aggregates, eliminated in global memory by one
    // workgroup, ~50 ms per Newton step at 512^3; there it halves the CG
    // iterations per Newton step, 143 -> 73, but is not the default: the
    // solve's damped phase took another path, 11 Newton steps instead of 8)
    const int per_axis = blocks->agg_per_axis > 0 ? blocks->agg_per_axis : 4;
    geo.dv = int32_t(ceil_div(geo.Gb, per_axis));
    geo.nd = int32_t(ceil_div(geo.Gb, geo.dv));
    geo.nblk = int64_t(geo.Gb) * geo.Gb * geo.Gb;
    nbm = unsigned(std::min<int64_t>(ceil_div(geo.nblk, ML_WPB), MAXB));
    w.blk_row.ensure(size_t(n) * sizeof(int32_t));
    w.r1.ensure(size_t(geo.nblk) * sizeof(double));
    w.d1inv.ensure(size_t(geo.nblk) * sizeof(double));
    w.cc.ensure(size_t(ML_MAXC) * sizeof(double));
    w.a1c.ensure(size_t(geo.nblk) * 27 * sizeof(double));
    w.ainv.ensure(size_t(ML_MAXC) * ML_MAXC * sizeof(double));
    w.aggw.ensure(size_t(ML_MAXC) * 27 * sizeof(double));
    const unsigned nbb = unsigned(ceil_div(geo.nblk, ML_WPB));
    ProfScope ps("pcg_setup", st, double(n));
    hipLaunchKernelGGL(k_ml_blk_rows, dim3(nbb), dim3(TPB), 0, st, geo, w.blk_row.as<int32_t>());
    if (J.f32)
      hipLaunchKernelGGL(k_ml_setup<float>, dim3(nbb), dim3(TPB), 0, st, geo, J.row_ptr.as<int64_t>(),
                         J.col.as<int32_t>(), J.w.as<float>(), w.blk_row.as<int32_t>(), w.d1inv.as<double>(),
                         w.a1c.as<double>());
    else
      hipLaunchKernelGGL(k_ml_setup<double>, dim3(nbb), dim3(TPB), 0, st, geo, J.row_ptr.as<int64_t>(),
                         J.col.as<int32_t>(), J.w.as<double>(), w.blk_row.as<int32_t>(), w.d1inv.as<double>(),
                         w.a1c.as<double>());
    const int nc = geo.nd * geo.nd * geo.nd;
    hipLaunchKernelGGL(k_ml_aggsum, dim3(unsigned(nc)), dim3(ML_AGG_TPB), 0, st, geo, w.a1c.as<double>(),
                       w.aggw.as<double>());
    if (nc <= ML_LDSC)
      hipLaunchKernelGGL(k_ml_dense, dim3(1), dim3(256), 0, st, geo, w.aggw.as<double>(), w.ainv.as<double>());
    else
      hipLaunchKernelGGL(k_ml_dense_big, dim3(1), dim3(1024), 0, st, geo, w.aggw.as<double>(),
                         w.ainv.as<double>());
    MAK_HIP(hipGetLastError());
  }
  // u = M^-1 r of the three-level preconditioner, from the blocks' sums r1
  // left by the init / update kernel
  auto ml_apply = [&]() {
    hipLaunchKernelGGL(k_ml_coarse, dim3(1), dim3(ML_CTPB), 0, st, geo, w.r1.as<double>(), w.ainv.as<double>(),
                       w.cc.as<double>(), scal);
    hipLaunchKernelGGL(k_ml_apply, dim3(nbm), dim3(TPB), 0, st, geo, r, dinv, w.r1.as<double>(),
                       w.d1inv.as<double>(), w.cc.as<double>(), u, scal);
  };
  hipLaunchKernelGGL(k_diag_inv, dim3(nbe), dim3(256), 0, st, J.diag.as<double>(), dinv, n);
  hipLaunchKernelGGL(k_sum_part, dim3(nb), dim3(TPB), 0, st, b, part, n);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, scal, int(S_MEAN), 0);
  hipLaunchKernelGGL(k_sq_part, dim3(nb), dim3(TPB), 0, st, b, scal, part, n);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nb), 1, scal, int(S_BB), 0);
  double hb[16];
  // r0 (from b, or with `q` from b - J x), the first preconditioned residual
  // and the partials of r.u and r.r
  const unsigned nbu = ml ? nbm : nb;  // workgroups of the update kernel (its partials)
  auto init = [&](const double* q) {
    if (ml) {
      hipLaunchKernelGGL(k_ml_init, dim3(nbm), dim3(TPB), 0, st, geo, b, scal, q, x, r, p, sv, dinv,
                         w.r1.as<double>(), w.d1inv.as<double>(), part, n);
      ml_apply();
    } else {
      hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(TPB), 0, st, b, scal, q, x, r, u, p, sv, dinv, part, n);
    }
  };
  if (warm) {
    // start from the given x: r0 = b - J x; kept only if |r0| < |b|
    spmv(x, wv);
    init(wv);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(TPB), 0, st, part, int(nbu), 2, scal, int(S_TMP), int(S_RR));
    MAK_HIP(hipGetLastError());
    MAK_HIP(hipMemcpyAsync(hb, scal, sizeof(hb), hipMemcpyDeviceToHost, st));
    MAK_HIP(hipStreamSynchronize(st));
    if (!(hb[S_RR] < hb[S_BB])) warm = false;
  }
  if (!warm) init(nullptr);
  spmv(u, wv);
  hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(SCAL_TPB), 0, st, part, int(nbu), part2, int(nbs), scal, 1,
                     -1.0, ml ? 1 : 0);
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
      // compulsory bytes: the update reads u, w, p, s, x, r and D^-1 and
      // writes p, s, x, r and u (the three-level form writes u in its apply
      // kernel, reading r and D^-1 again)
      ProfScope ps("pcg_update", st, double(n), (ml ? 112.0 : 96.0) * double(n));
      ps.flops = 14.0 * double(n);
      if (ml) {
        hipLaunchKernelGGL(k_ml_update, dim3(nbm), dim3(TPB), 0, st, geo, x, r, u, p, sv, wv, dinv, scal,
                           w.r1.as<double>(), w.d1inv.as<double>(), part);
        ml_apply();
      } else {
        hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(TPB), 0, st, x, r, u, p, sv, wv, dinv, scal, part, n);
      }
    }
    spmv(u, wv);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(SCAL_TPB), 0, st, part, int(nbu), part2, int(nbs), scal, 0,
                       stop, ml ? 1 : 0);
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
