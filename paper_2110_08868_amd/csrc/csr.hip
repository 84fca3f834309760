// Hessian assembly: J_ij = -sum over the faces of cell i with images of
// site j of area / |d|,  J_ii = -sum_j J_ij  (derived from Eq. SDK: raising
// psi_j moves the common face towards x_i by dpsi_j / |d|).  Rows are the
// per-cell face lists written by the clip kernel, sorted by column and merged
// over periodic images.
#include "engine.h"
#include "profile.h"

namespace mak {

namespace {

__device__ __forceinline__ FaceRec* face_list(FaceRec* faces, FaceRec* ovf, const int64_t* fbase,
                                              int32_t fslot, int32_t p, int32_t nf) {
  return nf > fslot ? ovf + fbase[p] : faces + int64_t(p) * fslot;
}

// Sort the faces of each cell by (target column, shift); count distinct
// columns (plus one for the diagonal when `diag_entry`).
__global__ void k_sort_count(FaceRec* faces, FaceRec* ovf, const int64_t* fbase, int32_t fslot,
                             const int32_t* __restrict__ nface, const int32_t* __restrict__ perm,
                             int64_t* __restrict__ rowcnt, int64_t* __restrict__ facecnt, int64_t n,
                             int diag_entry) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  FaceRec* f = face_list(faces, ovf, fbase, fslot, int32_t(p), nf);
  auto col = [&](const FaceRec& r) -> int64_t { return perm ? perm[r.j] : r.j; };
  for (int32_t k = 1; k < nf; ++k) {
    const FaceRec v = f[k];
    const int64_t cv = col(v);
    int32_t m = k - 1;
    while (m >= 0) {
      const int64_t cm = col(f[m]);
      if (cm < cv || (cm == cv && f[m].shift <= v.shift)) break;
      f[m + 1] = f[m];
      --m;
    }
    f[m + 1] = v;
  }
  int64_t distinct = 0, prev = -1;
  for (int32_t k = 0; k < nf; ++k) {
    const int64_t c = col(f[k]);
    if (c != prev) ++distinct;
    prev = c;
  }
  const int64_t row = perm ? perm[p] : p;
  rowcnt[row] = distinct + diag_entry;
  if (facecnt) facecnt[row] = nf;
}

__global__ void k_fill(const FaceRec* faces, const FaceRec* ovf, const int64_t* fbase, int32_t fslot,
                       const int32_t* __restrict__ nface, const int32_t* __restrict__ perm,
                       const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                       double* __restrict__ val, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  const FaceRec* f = face_list(const_cast<FaceRec*>(faces), const_cast<FaceRec*>(ovf), fbase, fslot,
                               int32_t(p), nf);
  const int64_t row = perm ? perm[p] : p;
  int64_t o = row_ptr[row];
  // off-diagonal sum first (fixed order), so the diagonal is minus the row sum
  double diag = 0.0;
  for (int32_t k = 0; k < nf; ++k) diag += f[k].w;
  bool diag_done = false;
  int32_t k = 0;
  while (k < nf) {
    const int64_t c = perm ? perm[f[k].j] : f[k].j;
    double w = 0.0;
    while (k < nf && (perm ? perm[f[k].j] : f[k].j) == c) {
      w += f[k].w;
      ++k;
    }
    if (!diag_done && c > row) {
      col[o] = int32_t(row);
      val[o] = diag;
      ++o;
      diag_done = true;
    }
    col[o] = int32_t(c);
    val[o] = -w;
    ++o;
  }
  if (!diag_done) {
    col[o] = int32_t(row);
    val[o] = diag;
  }
}

// The solver's Laplacian rows straight from the face records, without
// sorting them: a row's faces (at most kRegFaces, the face slots of a cell)
// are held in registers; its distinct neighbours are the faces whose column
// does not occur earlier in the list, the rank of a column is the number of
// distinct columns below it, and a column's weight is the sum of its faces'
// weights in list order.  A row kept in the overflow region (more faces than
// slots) is done the same way from memory.  (All loads of a row are issued
// before the arithmetic: a load inside the per-column branch cost a memory
// round trip per face.)
constexpr int kRegFaces = 32;

__device__ int32_t lap_row_mem(const FaceRec* f, int32_t nf, int32_t* col, float* wf, double* wd,
                               double* diag) {
  // first the "first face of its column" flags (rows hold at most 128 faces,
  // the polytope capacity: a 128-bit mask), so the ranks take O(nf^2)
  uint64_t first_lo = 0, first_hi = 0;
  int32_t cnt = 0;
  for (int32_t k = 0; k < nf; ++k) {
    const int32_t jk = f[k].j;
    bool first = true;
    for (int32_t m = 0; m < k && first; ++m) first = f[m].j != jk;
    if (!first) continue;
    ++cnt;
    if (k < 64)
      first_lo |= uint64_t(1) << k;
    else
      first_hi |= uint64_t(1) << (k - 64);
  }
  if (!col) return cnt;
  auto is_first = [&](int32_t m) {
    return m < 64 ? ((first_lo >> m) & 1u) != 0 : ((first_hi >> (m - 64)) & 1u) != 0;
  };
  double d = 0.0;
  for (int32_t k = 0; k < nf; ++k) {
    if (!is_first(k)) continue;
    const int32_t jk = f[k].j;
    int32_t rank = 0;
    double s = 0.0;
    for (int32_t m = 0; m < nf; ++m) {
      const int32_t jm = f[m].j;
      if (jm == jk) s += f[m].w;
      rank += (jm < jk && is_first(m)) ? 1 : 0;
    }
    col[rank] = jk;
    if (wf) {
      wf[rank] = float(s);
      d += double(float(s));
    } else {
      wd[rank] = s;
      d += s;
    }
  }
  if (diag) *diag = d;
  return cnt;
}

__global__ __launch_bounds__(256) void k_lap_count(const FaceRec* faces, const FaceRec* ovf, const int64_t* fbase, int32_t fslot,
                            const int32_t* __restrict__ nface, int64_t* __restrict__ rowcnt, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  const FaceRec* f = face_list(const_cast<FaceRec*>(faces), const_cast<FaceRec*>(ovf), fbase, fslot,
                               int32_t(p), nf);
  if (nf > kRegFaces) {
    rowcnt[p] = lap_row_mem(f, nf, nullptr, nullptr, nullptr, nullptr);
    return;
  }
  int32_t jj[kRegFaces];
#pragma unroll
  for (int k = 0; k < kRegFaces; ++k) jj[k] = k < nf ? f[k].j : -1 - k;
  int32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kRegFaces; ++k) {
    bool first = k < nf;
#pragma unroll
    for (int m = 0; m < k; ++m) first = first && jj[m] != jj[k];
    cnt += first ? 1 : 0;
  }
  rowcnt[p] = cnt;
}

template <typename W>
__global__ __launch_bounds__(256) void k_lap_fill_rows(const FaceRec* faces, const FaceRec* ovf, const int64_t* fbase, int32_t fslot,
                                const int32_t* __restrict__ nface, const int64_t* __restrict__ row_ptr,
                                int32_t* __restrict__ col, W* __restrict__ w, double* __restrict__ diag,
                                int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  const FaceRec* f = face_list(const_cast<FaceRec*>(faces), const_cast<FaceRec*>(ovf), fbase, fslot,
                               int32_t(p), nf);
  const int64_t o = row_ptr[p];
  if (nf > kRegFaces) {
    if (sizeof(W) == 4)
      lap_row_mem(f, nf, col + o, reinterpret_cast<float*>(w + o), nullptr, diag + p);
    else
      lap_row_mem(f, nf, col + o, nullptr, reinterpret_cast<double*>(w + o), diag + p);
    return;
  }
  int32_t jj[kRegFaces];
  double ww[kRegFaces];
#pragma unroll
  for (int k = 0; k < kRegFaces; ++k) {
    jj[k] = k < nf ? f[k].j : -1 - k;
    ww[k] = k < nf ? f[k].w : 0.0;
  }
  uint32_t firsts = 0;
#pragma unroll
  for (int k = 0; k < kRegFaces; ++k) {
    bool first = k < nf;
#pragma unroll
    for (int m = 0; m < k; ++m) first = first && jj[m] != jj[k];
    firsts |= first ? (1u << k) : 0u;
  }
  double d = 0.0;
#pragma unroll
  for (int k = 0; k < kRegFaces; ++k) {
    if (!((firsts >> k) & 1u)) continue;
    int32_t rank = 0;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kRegFaces; ++m) {
      s += jj[m] == jj[k] ? ww[m] : 0.0;  // in list order, as the unsorted sum
      rank += (((firsts >> m) & 1u) && jj[m] < jj[k]) ? 1 : 0;
    }
    const W ws = W(s);
    col[o + rank] = jj[k];
    w[o + rank] = ws;
    d += double(ws);
  }
  diag[p] = d;
}

// SELL-64 copy of the Laplacian rows (one wavefront per slice of 64 rows).
__global__ __launch_bounds__(256) void k_sell_len(const int64_t* __restrict__ rowcnt, int32_t* __restrict__ slen,
                                                  int64_t* __restrict__ slen64, int64_t n, int64_t nsl) {
  const int64_t s = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (s >= nsl) return;  // the same slice for the whole wavefront
  const int64_t r = s * 64 + lane;
  int c = r < n ? int(rowcnt[r]) : 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c = max(c, __shfl_xor(c, o));
  if (lane == 0) {
    slen[s] = c;
    slen64[s] = int64_t(c) * 64;
  }
}

template <typename W>
__global__ __launch_bounds__(256) void k_sell_fill(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const W* __restrict__ w, const int64_t* __restrict__ soff,
                                                   const int32_t* __restrict__ slen, int32_t* __restrict__ scol,
                                                   W* __restrict__ sw, int64_t n, int64_t nsl) {
  const int64_t s = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (s >= nsl) return;
  const int64_t r = s * 64 + lane;
  const int64_t base = soff[s] + lane;
  const int len = slen[s];
  const int64_t o = r < n ? rp[r] : 0;
  const int cnt = r < n ? int(rp[r + 1] - o) : 0;
  const int32_t own = r < n ? int32_t(r) : 0;
  for (int k = 0; k < len; ++k) {
    const bool in = k < cnt;
    scol[base + int64_t(k) * 64] = in ? col[o + k] : own;
    sw[base + int64_t(k) * 64] = in ? w[o + k] : W(0);
  }
}

// Face lists in original order; the area is the stored weight times |d|,
// with d formed as the clip kernel forms it (equal to within rounding).
__global__ void k_face_copy(const FaceRec* faces, const FaceRec* ovf, const int64_t* fbase,
                            int32_t fslot, const int32_t* __restrict__ nface,
                            const int32_t* __restrict__ perm, const double4* __restrict__ pts,
                            double L, const int64_t* __restrict__ fptr, int32_t* __restrict__ fj,
                            int32_t* __restrict__ fs, double* __restrict__ fa, int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  const FaceRec* f = face_list(const_cast<FaceRec*>(faces), const_cast<FaceRec*>(ovf), fbase, fslot,
                               int32_t(p), nf);
  const double4 me = pts[p];
  int64_t o = fptr[perm[p]];
  for (int32_t k = 0; k < nf; ++k, ++o) {
    const int32_t sh = f[k].shift;
    const double4 P = pts[f[k].j];
    const double dx = P.x + unpack_shift(sh, 0) * L - me.x;
    const double dy = P.y + unpack_shift(sh, 1) * L - me.y;
    const double dz = P.z + unpack_shift(sh, 2) * L - me.z;
    fj[o] = perm[f[k].j];
    fs[3 * o] = unpack_shift(sh, 0);
    fs[3 * o + 1] = unpack_shift(sh, 1);
    fs[3 * o + 2] = unpack_shift(sh, 2);
    fa[o] = f[k].w * sqrt(dx * dx + dy * dy + dz * dz);
  }
}

}  // namespace

void build_csr(const PointSet& ps, CellPass& cp, Csr& J, bool original_space, hipStream_t st) {
  const int64_t n = ps.N;
  ProfScope scope("csr_assembly", st, double(n));
  J.n = n;
  // row counts, and (original space, for the face copy) the face counts after them
  J.rowcnt.ensure(size_t(n) * (original_space ? 2 : 1) * sizeof(int64_t));
  J.row_ptr.ensure(size_t(n + 1) * sizeof(int64_t));
  const int32_t* perm = original_space ? ps.perm.as<int32_t>() : nullptr;
  const unsigned nb = unsigned(ceil_div(n, 256));
  const FaceStore& fst = cp.fs();
  hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                     fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                     perm, J.rowcnt.as<int64_t>(), original_space ? J.rowcnt.as<int64_t>() + n : nullptr,
                     n, 1);
  MAK_HIP(hipGetLastError());
  exclusive_scan_i64(J.rowcnt.as<int64_t>(), J.row_ptr, n, cp.scan_tmp, st);
  int64_t nnz = 0;
  MAK_HIP(hipMemcpyAsync(&nnz, J.row_ptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  J.nnz = nnz;
  J.col.ensure(size_t(nnz) * sizeof(int32_t));
  J.val.ensure(size_t(nnz) * sizeof(double));
  hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(), fst.ovf.as<FaceRec>(),
                     fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(), perm,
                     J.row_ptr.as<int64_t>(), J.col.as<int32_t>(), J.val.as<double>(), n);
  MAK_HIP(hipGetLastError());
}

void build_lap(const PointSet& ps, CellPass& cp, Lap& J, bool f32, hipStream_t st) {
  const int64_t n = ps.N;
  ProfScope scope("csr_assembly", st, double(n));
  J.n = n;
  J.f32 = f32;
  J.rowcnt.ensure(size_t(n) * sizeof(int64_t));
  J.row_ptr.ensure(size_t(n + 1) * sizeof(int64_t));
  J.diag.ensure(size_t(n) * sizeof(double));
  const unsigned nb = unsigned(ceil_div(n, 256));
  const FaceStore& fst = cp.fs();
  if (fst.fslot > kRegFaces) MAK_FAIL(MAK_EHIP, "face slots exceed the register rows of the assembly");
  hipLaunchKernelGGL(k_lap_count, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(), fst.ovf.as<FaceRec>(),
                     fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(), J.rowcnt.as<int64_t>(), n);
  MAK_HIP(hipGetLastError());
  exclusive_scan_i64(J.rowcnt.as<int64_t>(), J.row_ptr, n, cp.scan_tmp, st);
  int64_t nnz = 0;
  MAK_HIP(hipMemcpyAsync(&nnz, J.row_ptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  J.nnz = nnz;
  J.col.ensure(size_t(nnz) * sizeof(int32_t));
  J.w.ensure(size_t(nnz) * (f32 ? sizeof(float) : sizeof(double)));
  if (f32)
    hipLaunchKernelGGL(k_lap_fill_rows<float>, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                       fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                       J.row_ptr.as<int64_t>(), J.col.as<int32_t>(), J.w.as<float>(),
                       J.diag.as<double>(), n);
  else
    hipLaunchKernelGGL(k_lap_fill_rows<double>, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                       fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                       J.row_ptr.as<int64_t>(), J.col.as<int32_t>(), J.w.as<double>(),
                       J.diag.as<double>(), n);
  MAK_HIP(hipGetLastError());
  // the SELL-64 copy for the SpMV of the mixed path (float weights)
  if (!f32) {
    J.nsl = J.sell_n = 0;
    return;
  }
  const int64_t nsl = ceil_div(n, 64);
  J.nsl = nsl;
  J.slen.ensure(size_t(nsl) * sizeof(int32_t));
  J.slen64.ensure(size_t(nsl) * sizeof(int64_t));
  J.soff.ensure(size_t(nsl + 1) * sizeof(int64_t));  // the scan writes the total at [nsl]
  const unsigned nbsl = unsigned(ceil_div(nsl, 4));
  hipLaunchKernelGGL(k_sell_len, dim3(nbsl), dim3(256), 0, st, J.rowcnt.as<int64_t>(), J.slen.as<int32_t>(),
                     J.slen64.as<int64_t>(), n, nsl);
  MAK_HIP(hipGetLastError());
  exclusive_scan_i64(J.slen64.as<int64_t>(), J.soff, nsl, cp.scan_tmp, st);
  int64_t total = 0;
  MAK_HIP(hipMemcpyAsync(&total, J.soff.as<int64_t>() + nsl, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  J.sell_n = total;
  J.scol.ensure(size_t(J.sell_n) * sizeof(int32_t));
  J.sw.ensure(size_t(J.sell_n) * sizeof(float));
  hipLaunchKernelGGL(k_sell_fill<float>, dim3(nbsl), dim3(256), 0, st, J.row_ptr.as<int64_t>(),
                     J.col.as<int32_t>(), J.w.as<float>(), J.soff.as<int64_t>(), J.slen.as<int32_t>(),
                     J.scol.as<int32_t>(), J.sw.as<float>(), n, nsl);
  MAK_HIP(hipGetLastError());
}

int64_t count_faces(const PointSet& ps, CellPass& cp, Csr& J, DevBuf& face_ptr, hipStream_t st) {
  // build_csr(original_space) left the per-row face counts after the row counts
  const int64_t n = ps.N;
  face_ptr.ensure(size_t(n + 1) * sizeof(int64_t));
  exclusive_scan_i64(J.rowcnt.as<int64_t>() + n, face_ptr, n, cp.scan_tmp, st);
  int64_t nf = 0;
  MAK_HIP(hipMemcpyAsync(&nf, face_ptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  return nf;
}

void copy_faces(const PointSet& ps, CellPass& cp, const DevBuf& face_ptr, int64_t* out_ptr,
                int32_t* fj, int32_t* fshift, double* farea, hipStream_t st) {
  const int64_t n = ps.N;
  MAK_HIP(hipMemcpyAsync(out_ptr, face_ptr.p, size_t(n + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_face_copy, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, st,
                     cp.fs().faces.as<FaceRec>(), cp.fs().ovf.as<FaceRec>(),
                     cp.fs().fbase.as<int64_t>(), cp.fs().fslot, cp.nface.as<int32_t>(),
                     ps.perm.as<int32_t>(), ps.pts.as<double4>(), ps.g.L, face_ptr.as<int64_t>(), fj,
                     fshift, farea, n);
  MAK_HIP(hipGetLastError());
}

}  // namespace mak
