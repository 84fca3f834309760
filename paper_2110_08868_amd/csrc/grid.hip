// Neighbour grid: wrap + validate + counting sort of the sites into
// block-major cell order, and the weight bounds used by the search.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "engine.h"
#include "gridkey.h"
#include "profile.h"

namespace mak {

GridDesc make_grid(int64_t N, double L, double occupancy) {
  GridDesc g;
  if (occupancy <= 0) occupancy = 2.5;
  const double side = std::cbrt(double(N) / occupancy) / BLOCK_SIDE;
  int64_t gb = int64_t(std::llround(side));
  if (gb < 1) gb = 1;
  if (gb > 1024) gb = 1024;
  g.Gb = int32_t(gb);
  g.Gn = int32_t(gb * BLOCK_SIDE);
  g.L = L;
  g.h = L / double(g.Gn);
  return g;
}

namespace {

// Wrap into [0, L), check finiteness, compute the cell key, count the cell.
__global__ void k_stage(const double* __restrict__ points, const double* __restrict__ psi,
                        int64_t n, double L, double h, int Gn, int Gb, double4* __restrict__ xw,
                        int32_t* __restrict__ key, int32_t* __restrict__ rank,
                        int32_t* __restrict__ count, int32_t* __restrict__ status) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double c[3];
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = points[3 * i + a];
    ok = ok && isfinite(v);
    v = fmod(v, L);
    if (v < 0) v += L;
    if (!(v < L) || !(v >= 0)) v = 0.0;
    c[a] = v;
  }
  const double w = psi ? psi[i] : 0.0;
  ok = ok && isfinite(w);
  if (!ok) {
    atomicOr(status, 1);
    c[0] = c[1] = c[2] = 0.0;
  }
  xw[i] = make_double4(c[0], c[1], c[2], ok ? w : 0.0);
  const int cx = cell_coord(c[0], h, Gn), cy = cell_coord(c[1], h, Gn), cz = cell_coord(c[2], h, Gn);
  const int32_t k = int32_t(cell_key(cx, cy, cz, Gb));
  key[i] = k;
  rank[i] = atomicAdd(&count[k], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ key, const int32_t* __restrict__ rank,
                          const int32_t* __restrict__ start, int32_t* __restrict__ perm, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  perm[start[key[i]] + rank[i]] = int32_t(i);
}

// Order the sites of each cell by original index (the atomic ranks above are
// not reproducible; this makes the sorted order deterministic).
__global__ void k_cell_sort(const int32_t* __restrict__ start, int32_t* __restrict__ perm, int64_t G) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int32_t b = start[g], e = start[g + 1];
  for (int32_t k = b + 1; k < e; ++k) {
    const int32_t v = perm[k];
    int32_t m = k - 1;
    while (m >= b && perm[m] > v) {
      perm[m + 1] = perm[m];
      --m;
    }
    perm[m + 1] = v;
  }
}

__global__ void k_gather(const double4* __restrict__ xw, const int32_t* __restrict__ perm,
                         double4* __restrict__ pts, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  pts[p] = xw[perm[p]];
}

__global__ void k_set_psi(const double* __restrict__ psi_sorted, double4* __restrict__ pts, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  pts[p].w = psi_sorted[p];
}

__global__ void k_cell_max(const int32_t* __restrict__ start, const double4* __restrict__ pts,
                           double* __restrict__ cmax, int64_t G) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= G) return;
  double m = -DBL_MAX;
  for (int32_t k = start[g]; k < start[g + 1]; ++k) m = fmax(m, pts[k].w);
  cmax[g] = m;
}

// One wave per block of 64 cells.
__global__ __launch_bounds__(64) void k_block_max(const double* __restrict__ cmax,
                                                  double* __restrict__ bmax, int64_t GB) {
  const int64_t b = blockIdx.x;
  if (b >= GB) return;
  const double v = wave_max_d(cmax[b * 64 + threadIdx.x]);
  if (threadIdx.x == 0) bmax[b] = v;
}

// For every block b and r = 0..SHELL_MAX: the largest weight in the
// (unwrapped, periodic) blocks at Chebyshev block distance exactly r from b.
// One wave per block: the lanes share the (2 SHELL_MAX + 1)^3 offsets and
// reduce per shell.
__global__ __launch_bounds__(64) void k_block_suffix(const double* __restrict__ bmax, double* __restrict__ suf,
                                                     int Gb, int64_t GB) {
  const int64_t b = blockIdx.x;
  if (b >= GB) return;
  const int lane = threadIdx.x;
  const int bx = int(b / (int64_t(Gb) * Gb)), by = int((b / Gb) % Gb), bz = int(b % Gb);
  constexpr int S = 2 * SHELL_MAX + 1;
  double sh[SHELL_MAX + 1];
#pragma unroll
  for (int r = 0; r <= SHELL_MAX; ++r) sh[r] = -DBL_MAX;
  for (int t = lane; t < S * S * S; t += 64) {
    const int ox = t / (S * S) - SHELL_MAX, oy = (t / S) % S - SHELL_MAX, oz = t % S - SHELL_MAX;
    const int r = max(abs(ox), max(abs(oy), abs(oz)));
    const int wx = ((bx + ox) % Gb + Gb) % Gb, wy = ((by + oy) % Gb + Gb) % Gb, wz = ((bz + oz) % Gb + Gb) % Gb;
    const double v = bmax[(int64_t(wx) * Gb + wy) * Gb + wz];
#pragma unroll
    for (int q = 0; q <= SHELL_MAX; ++q)
      if (q == r) sh[q] = fmax(sh[q], v);
  }
#pragma unroll
  for (int r = 0; r <= SHELL_MAX; ++r) {
    const double m = wave_max_d(sh[r]);
    if (lane == 0) suf[b * (SHELL_MAX + 1) + r] = m;
  }
}

// Tilted weight bounds.  For block B with centre x_B take a slope g_B (the
// least-squares fit of psi over the block's sites; any slope gives a valid
// bound) and M = max_j (psi_j - g_B . (x_j - x_B)) over the block's sites,
// and per cell over the cell's sites: every site j of the block satisfies
// psi_j <= M + g_B . (x_j - x_B).  The clip kernel's box tests use these, so
// a linear trend of the weights across a block (converged weights follow the
// displacement field) does not inflate the bound of the whole block.
// One wave per block (its sites are contiguous: block-major keys): the lanes
// share the block's sites for the sums of the normal equations; lane c then
// takes cell c of the block.
__global__ __launch_bounds__(64) void k_block_tilt(const int32_t* __restrict__ start,
                                                   const double4* __restrict__ pts, double bh, int Gb,
                                                   int64_t GB, double* __restrict__ block_g,
                                                   double* __restrict__ block_tmax,
                                                   double* __restrict__ cell_tmax) {
  const int64_t b = blockIdx.x;
  if (b >= GB) return;
  const int lane = threadIdx.x;
  const int bx = int(b / (int64_t(Gb) * Gb)), by = int((b / Gb) % Gb), bz = int(b % Gb);
  const double ox = (bx + 0.5) * bh, oy = (by + 0.5) * bh, oz = (bz + 0.5) * bh;
  const int32_t s0 = start[b * 64], s1 = start[b * 64 + 64];
  const int n = s1 - s0;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (n >= 4) {
    double mx = 0, my = 0, mz = 0, mp = 0;
    for (int32_t k = s0 + lane; k < s1; k += 64) {
      const double4 P = pts[k];
      mx += P.x - ox;
      my += P.y - oy;
      mz += P.z - oz;
      mp += P.w;
    }
    mx = wave_sum_d(mx) / n;
    my = wave_sum_d(my) / n;
    mz = wave_sum_d(mz) / n;
    mp = wave_sum_d(mp) / n;
    double cxx = 0, cxy = 0, cxz = 0, cyy = 0, cyz = 0, czz = 0, vx = 0, vy = 0, vz = 0;
    for (int32_t k = s0 + lane; k < s1; k += 64) {
      const double4 P = pts[k];
      const double ex = P.x - ox - mx, ey = P.y - oy - my, ez = P.z - oz - mz, ep = P.w - mp;
      cxx += ex * ex;
      cxy += ex * ey;
      cxz += ex * ez;
      cyy += ey * ey;
      cyz += ey * ez;
      czz += ez * ez;
      vx += ex * ep;
      vy += ey * ep;
      vz += ez * ep;
    }
    cxx = wave_sum_d(cxx);
    cxy = wave_sum_d(cxy);
    cxz = wave_sum_d(cxz);
    cyy = wave_sum_d(cyy);
    cyz = wave_sum_d(cyz);
    czz = wave_sum_d(czz);
    vx = wave_sum_d(vx);
    vy = wave_sum_d(vy);
    vz = wave_sum_d(vz);
    // adjugate solve of the 3x3 normal equations, skipped when ill-conditioned
    const double a00 = cyy * czz - cyz * cyz, a01 = cxz * cyz - cxy * czz, a02 = cxy * cyz - cxz * cyy;
    const double a11 = cxx * czz - cxz * cxz, a12 = cxy * cxz - cxx * cyz, a22 = cxx * cyy - cxy * cxy;
    const double det = cxx * a00 + cxy * a01 + cxz * a02;
    const double tr = cxx + cyy + czz;
    if (det > 1e-6 * tr * tr * tr) {
      gx = (a00 * vx + a01 * vy + a02 * vz) / det;
      gy = (a01 * vx + a11 * vy + a12 * vz) / det;
      gz = (a02 * vx + a12 * vy + a22 * vz) / det;
    }
  }
  double mc = -DBL_MAX;
  for (int32_t k = start[b * 64 + lane]; k < start[b * 64 + lane + 1]; ++k) {
    const double4 P = pts[k];
    mc = fmax(mc, P.w - (gx * (P.x - ox) + gy * (P.y - oy) + gz * (P.z - oz)));
  }
  cell_tmax[b * 64 + lane] = mc;
  const double M = wave_max_d(mc);
  if (lane == 0) {
    block_tmax[b] = M;
    block_g[3 * b] = gx;
    block_g[3 * b + 1] = gy;
    block_g[3 * b + 2] = gz;
  }
}

}  // namespace

namespace {
size_t up256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

size_t pointset_bytes(int64_t N, const GridDesc& g) {
  const size_t n = size_t(N), G = size_t(g.G()), GB = size_t(g.GB());
  return up256(n * sizeof(double4)) + up256(n * 4) + up256((G + 1) * 4) + 2 * up256(G * 8) +
         up256(GB * 8) * 2 + up256(GB * (SHELL_MAX + 1) * 8) + up256(GB * 3 * 8) + up256(8 * 8) +
         2 * up256(n * 4) + up256(G * 4) + up256(n * sizeof(double4) + 64) +
         up256(std::max(scan_tmp_bytes_i32(int64_t(G)), reduce_tmp_bytes())) + up256(4);
}

void borrow_pointset(PointSet& ps, DevBuf& status, char* base, int64_t N, const GridDesc& g) {
  const size_t n = size_t(N), G = size_t(g.G()), GB = size_t(g.GB());
  size_t off = 0;
  auto take = [&](DevBuf& b, size_t bytes) {
    b.borrow(base + off, bytes);
    off += up256(bytes);
  };
  take(ps.pts, n * sizeof(double4));
  take(ps.perm, n * 4);
  take(ps.cell_start, (G + 1) * 4);
  take(ps.cell_psimax, G * 8);
  take(ps.cell_tmax, G * 8);
  take(ps.block_psimax, GB * 8);
  take(ps.block_tmax, GB * 8);
  take(ps.block_suffix, GB * (SHELL_MAX + 1) * 8);
  take(ps.block_g, GB * 3 * 8);
  take(ps.scal, 8 * 8);
  take(ps.key, n * 4);
  take(ps.rank, n * 4);
  take(ps.count, G * 4);
  take(ps.status, n * sizeof(double4) + 64);
  take(ps.tmp, std::max(scan_tmp_bytes_i32(int64_t(G)), reduce_tmp_bytes()));
  take(status, 4);
}

void build_pointset(PointSet& ps, const double* points, const double* psi, int64_t N, double L,
                    double occupancy, hipStream_t st) {
  ProfScope scope("grid_build", st, double(N));
  ps.N = N;
  ps.g = make_grid(N, L, occupancy);
  const int64_t G = ps.g.G();
  ps.pts.ensure(size_t(N) * sizeof(double4));
  ps.perm.ensure(size_t(N) * sizeof(int32_t));
  ps.cell_start.ensure(size_t(G + 1) * sizeof(int32_t));
  ps.cell_psimax.ensure(size_t(G) * sizeof(double));
  ps.block_psimax.ensure(size_t(ps.g.GB()) * sizeof(double));
  ps.block_suffix.ensure(size_t(ps.g.GB()) * (SHELL_MAX + 1) * sizeof(double));
  ps.block_g.ensure(size_t(ps.g.GB()) * 3 * sizeof(double));
  ps.block_tmax.ensure(size_t(ps.g.GB()) * sizeof(double));
  ps.cell_tmax.ensure(size_t(G) * sizeof(double));
  ps.scal.ensure(8 * sizeof(double));
  ps.key.ensure(size_t(N) * sizeof(int32_t));
  ps.rank.ensure(size_t(N) * sizeof(int32_t));
  ps.count.ensure(size_t(G) * sizeof(int32_t));
  ps.status.ensure(size_t(N) * sizeof(double4) + 64);  // xw staging + status word
  double4* xw = ps.status.as<double4>();
  int32_t* status = reinterpret_cast<int32_t*>(ps.status.as<char>() + size_t(N) * sizeof(double4));

  fill_zero_i32(ps.count.as<int32_t>(), G, st);
  fill_zero_i32(status, 1, st);
  const unsigned nb = unsigned(ceil_div(N, 256));
  hipLaunchKernelGGL(k_stage, dim3(nb), dim3(256), 0, st, points, psi, N, L, ps.g.h, ps.g.Gn,
                     ps.g.Gb, xw, ps.key.as<int32_t>(), ps.rank.as<int32_t>(),
                     ps.count.as<int32_t>(), status);
  exclusive_scan_i32(ps.count.as<int32_t>(), ps.cell_start, G, ps.tmp, st);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, st, ps.key.as<int32_t>(),
                     ps.rank.as<int32_t>(), ps.cell_start.as<int32_t>(), ps.perm.as<int32_t>(), N);
  hipLaunchKernelGGL(k_cell_sort, dim3(unsigned(ceil_div(G, 256))), dim3(256), 0, st,
                     ps.cell_start.as<int32_t>(), ps.perm.as<int32_t>(), G);
  hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, st, xw, ps.perm.as<int32_t>(),
                     ps.pts.as<double4>(), N);
  MAK_HIP(hipGetLastError());
  int32_t hs = 0;
  MAK_HIP(hipMemcpyAsync(&hs, status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  if (hs) MAK_FAIL(MAK_EINVAL, "non-finite coordinate or weight");
  update_psi_bounds(ps, st);
  if (N > (int64_t(1) << 24)) {
    // a large set is built once per solve: give the staging back to the passes
    ps.key.release();
    ps.rank.release();
    ps.count.release();
    ps.status.release();
  }
}

void set_psi_sorted(PointSet& ps, const double* psi_sorted, hipStream_t st) {
  hipLaunchKernelGGL(k_set_psi, dim3(unsigned(ceil_div(ps.N, 256))), dim3(256), 0, st, psi_sorted,
                     ps.pts.as<double4>(), ps.N);
  MAK_HIP(hipGetLastError());
  update_psi_bounds(ps, st);
}

void update_psi_bounds(PointSet& ps, hipStream_t st) {
  const int64_t G = ps.g.G(), GB = ps.g.GB();
  hipLaunchKernelGGL(k_cell_max, dim3(unsigned(ceil_div(G, 256))), dim3(256), 0, st,
                     ps.cell_start.as<int32_t>(), ps.pts.as<double4>(), ps.cell_psimax.as<double>(), G);
  hipLaunchKernelGGL(k_block_max, dim3(unsigned(GB)), dim3(64), 0, st, ps.cell_psimax.as<double>(),
                     ps.block_psimax.as<double>(), GB);
  hipLaunchKernelGGL(k_block_suffix, dim3(unsigned(GB)), dim3(64), 0, st,
                     ps.block_psimax.as<double>(), ps.block_suffix.as<double>(), ps.g.Gb, GB);
  hipLaunchKernelGGL(k_block_tilt, dim3(unsigned(GB)), dim3(64), 0, st,
                     ps.cell_start.as<int32_t>(), ps.pts.as<double4>(), BLOCK_SIDE * ps.g.h, ps.g.Gb,
                     GB, ps.block_g.as<double>(), ps.block_tmax.as<double>(), ps.cell_tmax.as<double>());
  MAK_HIP(hipGetLastError());
  dev_max_to(ps.block_psimax.as<double>(), GB, ps.scal.as<double>(), ps.tmp, st);
}

}  // namespace mak
