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

// Laplacian rows (sorted space): one weight per distinct neighbour, summed
// over its images in face order, and the diagonal as the sum of the stored
// (rounded) weights.
template <typename W>
__global__ void k_lap_fill(const FaceRec* faces, const FaceRec* ovf, const int64_t* fbase, int32_t fslot,
                           const int32_t* __restrict__ nface, const int64_t* __restrict__ row_ptr,
                           int32_t* __restrict__ col, W* __restrict__ w, double* __restrict__ diag,
                           int64_t n) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t nf = nface[p];
  const FaceRec* f = face_list(const_cast<FaceRec*>(faces), const_cast<FaceRec*>(ovf), fbase, fslot,
                               int32_t(p), nf);
  int64_t o = row_ptr[p];
  double d = 0.0;
  int32_t k = 0;
  while (k < nf) {
    const int32_t c = f[k].j;
    double s = 0.0;
    while (k < nf && f[k].j == c) {
      s += f[k].w;
      ++k;
    }
    const W ws = W(s);
    col[o] = c;
    w[o] = ws;
    d += double(ws);
    ++o;
  }
  diag[p] = d;
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
  exclusive_scan_i64(J.rowcnt.as<int64_t>(), J.row_ptr.as<int64_t>(), n, cp.scan_tmp, st);
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
  hipLaunchKernelGGL(k_sort_count, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                     fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                     nullptr, J.rowcnt.as<int64_t>(), nullptr, n, 0);
  MAK_HIP(hipGetLastError());
  exclusive_scan_i64(J.rowcnt.as<int64_t>(), J.row_ptr.as<int64_t>(), n, cp.scan_tmp, st);
  int64_t nnz = 0;
  MAK_HIP(hipMemcpyAsync(&nnz, J.row_ptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  J.nnz = nnz;
  J.col.ensure(size_t(nnz) * sizeof(int32_t));
  J.w.ensure(size_t(nnz) * (f32 ? sizeof(float) : sizeof(double)));
  if (f32)
    hipLaunchKernelGGL(k_lap_fill<float>, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                       fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                       J.row_ptr.as<int64_t>(), J.col.as<int32_t>(), J.w.as<float>(),
                       J.diag.as<double>(), n);
  else
    hipLaunchKernelGGL(k_lap_fill<double>, dim3(nb), dim3(256), 0, st, fst.faces.as<FaceRec>(),
                       fst.ovf.as<FaceRec>(), fst.fbase.as<int64_t>(), fst.fslot, cp.nface.as<int32_t>(),
                       J.row_ptr.as<int64_t>(), J.col.as<int32_t>(), J.w.as<double>(),
                       J.diag.as<double>(), n);
  MAK_HIP(hipGetLastError());
}

int64_t count_faces(const PointSet& ps, CellPass& cp, Csr& J, DevBuf& face_ptr, hipStream_t st) {
  // build_csr(original_space) left the per-row face counts after the row counts
  const int64_t n = ps.N;
  face_ptr.ensure(size_t(n + 1) * sizeof(int64_t));
  exclusive_scan_i64(J.rowcnt.as<int64_t>() + n, face_ptr.as<int64_t>(), n, cp.scan_tmp, st);
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
