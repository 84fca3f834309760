// C-ABI entry points (include/mak.h) and the host driver of the damped Newton
// iteration on the semi-discrete Kantorovich dual.
//
// Newton (the paper's method: K concave and C^2, maximised with first and
// second derivatives): g = m - V(psi), solve J p = g by Jacobi-PCG, then the
// Kitagawa-Merigot-Thibert step control: eps0 = 1/2 min(min m, min V(psi^0));
// accept psi + alpha p for the largest alpha in {1, 1/2, ...} with
// min V >= eps0 and ||m - V|| <= (1 - alpha/2) ||g||.  The trial passes are
// full passes (faces included), so an accepted trial's Hessian is reused.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstring>
#include <exception>
#include <string>
#include <utility>

#include "engine.h"
#include "profile.h"

using namespace mak;

namespace mak {

thread_local Profiler* g_prof = nullptr;

void swap_buf(DevBuf& a, DevBuf& b) {
  std::swap(a.p, b.p);
  std::swap(a.cap, b.cap);
}

// Exchange the per-cell results of two passes that share one face store.
void swap_pass(CellPass& a, CellPass& b) {
  swap_buf(a.vol, b.vol);
  swap_buf(a.mom, b.mom);
  swap_buf(a.cflags, b.cflags);
  swap_buf(a.nface, b.nface);
  swap_buf(a.topo_tri, b.topo_tri);
  swap_buf(a.topo_n, b.topo_n);
}

size_t solve_bytes_per_site(int64_t N) {
  // Held for the whole solve (bytes per site):
  //   points: sorted sites 32, perm 4, neighbour grid and weight bounds ~6
  //   two passes (accepted, trial): volume 8, moment 24, flags 4, faces 4,
  //     stage lists 12 -> 2 x 52
  //   one face store: slots fslot x 16, overflow base 8, overflow ~1/8 of a
  //     slot row
  //   J: row_ptr 8, row counts 8, diagonal 8, 16 neighbours per row x 12
  //     (col + float64 weight; 8 with the mixed path's float weights), and
  //     on the mixed path its SELL-64 copy for the SpMV: 24 slots per row
  //     (42 % padding on clustered inputs) x 8, slice tables ~0.3
  //   CG r, u, p, w, s, 1/diag 48;  Newton psi, trial psi, g, step, masses 40
  // The grid build's staging (40 bytes per site) is released before the
  // first pass for sets above 2^24 sites and fits in the pass buffers' share
  // below that.
  const size_t fslot = size_t(face_slots(N));
  const size_t faces = fslot * sizeof(FaceRec) + 8 + 2 * sizeof(FaceRec);
  //   walk certificates (kCertBytesPerSite, with walk_cert on)
  //   combinatorics of the two passes (2 x kTopoBytesPerSite, with topo_reuse on)
  return 42 + 2 * 52 + faces + 24 + 16 * 12 + 24 * 8 + 1 + 48 + 40 + kCertBytesPerSite +
         2 * kTopoBytesPerSite;
}

namespace {

__global__ void k_flag_stats(const int32_t* __restrict__ cf, const int32_t* __restrict__ nface,
                             unsigned long long* out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  unsigned long long e = 0, c = 0, nm = 0, mf = 0;
  if (i < n) {
    e = (cf[i] & CF_EMPTY) ? 1 : 0;
    c = (cf[i] & CF_COINCIDENT) ? 1 : 0;
    nm = (cf[i] & CF_NONMANIFOLD) ? 1 : 0;
    mf = (unsigned long long)nface[i];
  }
  // wave-aggregated atomics
  e = (unsigned long long)wave_sum_i(int(e));
  c = (unsigned long long)wave_sum_i(int(c));
  nm = (unsigned long long)wave_sum_i(int(nm));
  int m = int(mf);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
  if (lane_id() == 0) {
    if (e) atomicAdd(&out[0], e);
    if (c) atomicAdd(&out[1], c);
    if (nm) atomicAdd(&out[2], nm);
    atomicMax(&out[3], (unsigned long long)m);
  }
}

struct FlagStats {
  int64_t empty, coincident, nonmanifold, max_faces;
};

FlagStats flag_stats(const PointSet& ps, const CellPass& cp, DevBuf& tmp, hipStream_t st) {
  tmp.ensure(8 * sizeof(unsigned long long));
  MAK_HIP(hipMemsetAsync(tmp.p, 0, 8 * sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_flag_stats, dim3(unsigned(ceil_div(ps.N, 256))), dim3(256), 0, st,
                     cp.cflags.as<int32_t>(), cp.nface.as<int32_t>(),
                     tmp.as<unsigned long long>(), ps.N);
  MAK_HIP(hipGetLastError());
  unsigned long long h[4];
  MAK_HIP(hipMemcpyAsync(h, tmp.p, sizeof(h), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  return {int64_t(h[0]), int64_t(h[1]), int64_t(h[2]), int64_t(h[3])};
}

}  // namespace
}  // namespace mak

struct mak_ctx {
  int device = 0;
  mak_options opt{};
  std::string err;
  // last mak_laguerre_cells
  PointSet ps;
  CellPass cp;
  Csr J;
  DevBuf face_ptr;
  int64_t nfaces = 0;
  bool cells_valid = false;
  // solver: the accepted pass and the line-search trial share one face store
  PointSet sps;
  FaceStore sfaces;
  CellPass scp, scp_trial;
  Lap sJ;
  PcgWork pw;
  DevBuf psi_s, psi_t, g, pstep, mass_s, tmp;
  DevBuf probe_list, probe_tmp;  // probe cells of a trial: earlier rejecting cells + the smallest
  CertSet scert;                 // walk certificates of the solve
  // Legendre transform / point location
  PointSet lps;
  DevBuf lstatus, dep_acc;
  CellPass dcp;  // cell pass of the exact deposit
  // power spectrum
  PowerWork pk;
  Profiler prof;
  PassRunner* runner = nullptr;  // NULL: passes run on the solve's stream
};

namespace mak {

void set_pass_runner(mak_ctx* ctx, PassRunner* r) { ctx->runner = r; }

}  // namespace mak

namespace {

thread_local std::string g_create_error;

struct ProfBind {
  explicit ProfBind(mak_ctx* c) {
    g_prof = (c && (c->prof.timing || c->prof.counting)) ? &c->prof : nullptr;
  }
  ~ProfBind() { g_prof = nullptr; }
};

template <class F>
mak_status guarded(mak_ctx* ctx, F&& f) {
  ProfBind bind(ctx);
  try {
    f();
    return MAK_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.msg;
    return e.status;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return MAK_EHIP;
  }
}

constexpr int64_t kMaxVoxelsPerCell = int64_t(1) << 22;

void check_args(int64_t N, double L) {
  if (N < 1) MAK_FAIL(MAK_EINVAL, "N must be >= 1");
  if (N >= (int64_t(1) << 31)) MAK_FAIL(MAK_EINVAL, "N must be < 2^31");
  if (!std::isfinite(L) || !(L > 0)) MAK_FAIL(MAK_EINVAL, "L must be finite and > 0");
}

void set_device(const mak_ctx* ctx) { MAK_HIP(hipSetDevice(ctx->device)); }

}  // namespace

extern "C" {

void mak_default_options(mak_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = MAK_FP64;
  opt->max_newton = 60;
  opt->max_cg = 4000;
  opt->max_halvings = 30;
  opt->cg_rtol = 1e-3;
  opt->grid_occupancy = 2.5;
  opt->mem_budget_bytes = 0;
  opt->verbose = 0;
  opt->walk_cert = 1;
  opt->topo_reuse = 1;
}

mak_status mak_create(mak_ctx** out, int device, const mak_options* opt) {
  if (!out) return MAK_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    g_create_error = "no HIP device";
    return MAK_EHIP;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device index out of range";
    return MAK_EINVAL;
  }
  mak_ctx* c = new mak_ctx();
  c->scp.shared = &c->sfaces;
  c->scp_trial.shared = &c->sfaces;
  c->device = device;
  mak_default_options(&c->opt);
  if (opt) c->opt = *opt;
  if (c->opt.precision != MAK_FP64 && c->opt.precision != MAK_MIXED) {
    delete c;
    g_create_error = "unknown precision";
    return MAK_EINVAL;
  }
  const int nstage = c->opt.precision == MAK_MIXED ? 3 : 2;
  if (!(c->opt.cg_rtol > 0) || c->opt.max_newton < 0 || c->opt.max_cg < 1 || c->opt.max_halvings < 0 ||
      c->opt.first_stage < 0 || c->opt.first_stage >= nstage || c->opt.cg_precond < 0 ||
      c->opt.cg_precond > 2 || c->opt.walk_cert < 0 || c->opt.walk_cert > 1 || c->opt.topo_reuse < 0 ||
      c->opt.topo_reuse > 1) {
    delete c;
    g_create_error = "invalid options";
    return MAK_EINVAL;
  }
  // set-up of the no-allocation workspace on this device (once per device,
  // with the device current); a failure only disables mak_legendre_noalloc
  if (hipSetDevice(device) != hipSuccess || !mak::noalloc_setup(device)) (void)hipGetLastError();
  *out = c;
  return MAK_OK;
}

void mak_destroy(mak_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  delete ctx;
}

const char* mak_last_error(const mak_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

mak_status mak_laguerre_cells(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                              double L, double* volumes, double* centroids, mak_csr* hessian,
                              mak_cells_info* info, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points || !psi || !volumes || !centroids) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    ctx->cells_valid = false;
    build_pointset(ctx->ps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    PassOpts po;
    po.precision = ctx->opt.precision;
    po.first_stage = ctx->opt.first_stage;
    ClipStats cs = run_cells(ctx->ps, ctx->cp, po, st);
    FlagStats fs = flag_stats(ctx->ps, ctx->cp, ctx->tmp, st);
    if (fs.coincident > 0) MAK_FAIL(MAK_EDEGENERATE, "coincident sites");
    build_csr(ctx->ps, ctx->cp, ctx->J, true, st);
    ctx->nfaces = count_faces(ctx->ps, ctx->cp, ctx->J, ctx->face_ptr, st);
    scatter_cells_outputs(ctx->ps, ctx->cp.vol.as<double>(), ctx->cp.mom.as<double>(), volumes,
                          centroids, st);
    ctx->cells_valid = true;
    if (hessian) {
      hessian->n_rows = ctx->J.n;
      hessian->nnz = ctx->J.nnz;
      hessian->row_ptr = ctx->J.row_ptr.as<const int64_t>();
      hessian->col = ctx->J.col.as<const int32_t>();
      hessian->val = ctx->J.val.as<const double>();
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->empty_cells = fs.empty;
      info->overflow_cells = cs.retried - cs.fp64_rerun;
      info->fp64_rerun_cells = cs.fp64_rerun;
      info->nnz = ctx->J.nnz;
      info->faces = ctx->nfaces;
      info->max_faces = int32_t(fs.max_faces);
    }
  });
}

mak_status mak_hessian_copy(mak_ctx* ctx, int64_t* row_ptr, int32_t* col, double* val, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    if (!ctx->cells_valid) MAK_FAIL(MAK_EINVAL, "no cell pass to copy from");
    if (!row_ptr || !col || !val) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Csr& J = ctx->J;
    MAK_HIP(hipMemcpyAsync(row_ptr, J.row_ptr.p, size_t(J.n + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, st));
    MAK_HIP(hipMemcpyAsync(col, J.col.p, size_t(J.nnz) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    MAK_HIP(hipMemcpyAsync(val, J.val.p, size_t(J.nnz) * sizeof(double), hipMemcpyDeviceToDevice, st));
  });
}

mak_status mak_faces_copy(mak_ctx* ctx, int64_t* face_ptr, int32_t* face_j, int32_t* face_shift,
                          double* face_area, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    if (!ctx->cells_valid) MAK_FAIL(MAK_EINVAL, "no cell pass to copy from");
    if (!face_ptr || (ctx->nfaces > 0 && (!face_j || !face_shift || !face_area)))
      MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    set_device(ctx);
    copy_faces(ctx->ps, ctx->cp, ctx->face_ptr, face_ptr, face_j, face_shift, face_area,
               static_cast<hipStream_t>(stream));
  });
}

mak_status mak_legendre(mak_ctx* ctx, const double* points, const double* psi, int64_t N, double L,
                        const double* queries, int64_t Q, double* phi, int32_t* idx, double* disp,
                        void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points || (Q > 0 && !queries)) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (Q < 0 || Q >= (int64_t(1) << 40)) MAK_FAIL(MAK_EINVAL, "Q must be in [0, 2^40)");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    build_pointset(ctx->lps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    locate(ctx->lps, queries, Q, 0, 0.0, phi, idx, disp, ctx->lstatus, st);
  });
}

mak_status mak_legendre_noalloc(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                                double L, const double* queries, int64_t Q, double* phi, int32_t* idx,
                                double* disp, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points || (Q > 0 && !queries)) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (Q < 0 || Q >= (int64_t(1) << 40)) MAK_FAIL(MAK_EINVAL, "Q must be in [0, 2^40)");
    const GridDesc g = make_grid(N, L, ctx->opt.grid_occupancy);
    const size_t need = pointset_bytes(N, g);
    if (need > noalloc_capacity())
      MAK_FAIL(MAK_EINVAL, "N = " + std::to_string(N) + " needs " + std::to_string(need) +
                               " bytes of workspace; the no-allocation workspace holds " +
                               std::to_string(noalloc_capacity()) + " bytes");
    set_device(ctx);
    char* base = static_cast<char*>(noalloc_scratch(ctx->device));
    if (!base) MAK_FAIL(MAK_EHIP, "the no-allocation workspace is not available on this device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    PointSet ps;
    DevBuf status;
    borrow_pointset(ps, status, base, N, g);
    build_pointset(ps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    locate(ps, queries, Q, 0, 0.0, phi, idx, disp, status, st);
  });
}

mak_status mak_legendre_mesh(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                             double L, int64_t ng, double offset, double* phi, int32_t* idx,
                             double* disp, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (ng < 1 || ng > 4096) MAK_FAIL(MAK_EINVAL, "ng must be in [1, 4096]");
    if (!std::isfinite(offset)) MAK_FAIL(MAK_EINVAL, "offset must be finite");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    build_pointset(ctx->lps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    locate(ctx->lps, nullptr, 0, ng, offset, phi, idx, disp, ctx->lstatus, st);
  });
}

mak_status mak_za_deposit(mak_ctx* ctx, const double* points, const double* psi, int64_t N, double L,
                          double tau, int64_t n_lag, double lag_offset, int64_t ng, int32_t scheme,
                          double* density, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points || !density) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (!(tau >= 0.0 && tau <= 1.0)) MAK_FAIL(MAK_EINVAL, "tau must be in [0, 1]");
    if (n_lag < 1 || n_lag > 2048) MAK_FAIL(MAK_EINVAL, "n_lag must be in [1, 2048]");
    if (!std::isfinite(lag_offset)) MAK_FAIL(MAK_EINVAL, "lag_offset must be finite");
    if (ng < 1 || ng > 2048) MAK_FAIL(MAK_EINVAL, "ng must be in [1, 2048]");
    if (scheme != 1 && scheme != 2) MAK_FAIL(MAK_EINVAL, "scheme must be 1 (NGP) or 2 (CIC)");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    build_pointset(ctx->lps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    za_deposit(ctx->lps, tau, n_lag, lag_offset, ng, scheme, density, ctx->dep_acc, st);
  });
}

mak_status mak_za_deposit_cells(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                                double L, double tau, int64_t ng, double* density, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    check_args(N, L);
    if (!points || !density) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (!(tau >= 0.0 && tau < 1.0)) MAK_FAIL(MAK_EINVAL, "tau must be in [0, 1)");
    if (ng < 1 || ng > 1024) MAK_FAIL(MAK_EINVAL, "ng must be in [1, 1024]");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    build_pointset(ctx->lps, points, psi, N, L, ctx->opt.grid_occupancy, st);
    PassOpts po;
    po.precision = MAK_FP64;
    // the pass records each cell's combinatorics: the deposit builds the
    // moved cells from them instead of clipping their boxes
    ctx->dcp.topo_tri.ensure(size_t(N) * kTopoTri * sizeof(uint16_t));
    ctx->dcp.topo_n.ensure(size_t(N) * sizeof(int32_t));
    po.topo_out = &ctx->dcp;
    ClipStats cs = run_cells(ctx->lps, ctx->dcp, po, st);
    (void)cs;
    FlagStats fs = flag_stats(ctx->lps, ctx->dcp, ctx->tmp, st);
    if (fs.coincident > 0) MAK_FAIL(MAK_EDEGENERATE, "coincident sites");
    // one wavefront clips all the voxels of a cell: bound that work (a moved
    // cell of volume (1 - tau)^3 V spans at least that many voxel volumes)
    const double vmax = dev_reduce_max(ctx->dcp.vol.as<double>(), N, ctx->tmp, st);
    const double H = L / double(ng), sc = 1.0 - tau;
    if (vmax * sc * sc * sc / (H * H * H) > double(kMaxVoxelsPerCell))
      MAK_FAIL(MAK_EINVAL, "a moved cell spans more than 2^22 voxels: use a coarser mesh (or mak_za_deposit)");
    za_deposit_cells(ctx->lps, ctx->dcp, tau, ng, density, ctx->dep_acc, ctx->lstatus, st);
  });
}

mak_status mak_power_spectrum(mak_ctx* ctx, const double* field, int64_t ng, double L, int32_t nbins,
                              int32_t window, int32_t contrast, double* k_mean, double* power,
                              int64_t* modes, void* stream) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    if (!field || !k_mean || !power || !modes) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    if (ng < 2 || ng > 2048) MAK_FAIL(MAK_EINVAL, "ng must be in [2, 2048]");
    if (!std::isfinite(L) || !(L > 0)) MAK_FAIL(MAK_EINVAL, "L must be finite and > 0");
    if (nbins < 1 || nbins > 2048) MAK_FAIL(MAK_EINVAL, "nbins must be in [1, 2048]");
    if (window < 0 || window > 3) MAK_FAIL(MAK_EINVAL, "window must be 0, 1, 2 or 3");
    set_device(ctx);
    power_spectrum(ctx->pk, field, ng, L, nbins, window, contrast != 0, k_mean, power, modes,
                   static_cast<hipStream_t>(stream));
  });
}

static mak_status solve_impl(mak_ctx* ctx, const double* points, const double* masses, int64_t N,
                             double L, double tol, const double* psi0, double* psi, double* centroids,
                             double* displacements, mak_solve_info* info, void* stream) {
  if (!ctx) return MAK_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  mak_solve_info si{};
  mak_status status = guarded(ctx, [&] {
    check_args(N, L);
    if (!(tol > 0)) MAK_FAIL(MAK_EINVAL, "tol must be > 0");
    if (!points || !psi || !centroids || !displacements) MAK_FAIL(MAK_EINVAL, "NULL pointer argument");
    set_device(ctx);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const mak_options& o = ctx->opt;
    PointSet& ps = ctx->sps;
    build_pointset(ps, points, psi0, N, L, o.grid_occupancy, st);
    ctx->psi_s.ensure(size_t(N) * sizeof(double));
    ctx->psi_t.ensure(size_t(N) * sizeof(double));
    ctx->g.ensure(size_t(N) * sizeof(double));
    ctx->pstep.ensure(size_t(N) * sizeof(double));
    double* psi_s = ctx->psi_s.as<double>();
    if (psi0)
      gather_sorted(ps, psi0, psi_s, st);
    else
      MAK_HIP(hipMemsetAsync(psi_s, 0, size_t(N) * sizeof(double), st));
    const double m = L * L * L / double(N);
    // target masses: uniform L^3 / N, or per site (sorted into the solver's
    // order; positive, summing to L^3)
    const double* ms = nullptr;
    double m_min = m;
    if (masses) {
      ctx->mass_s.ensure(size_t(N) * sizeof(double));
      gather_sorted(ps, masses, ctx->mass_s.as<double>(), st);
      ms = ctx->mass_s.as<double>();
      const double msum = dev_reduce_sum(ms, N, ctx->tmp, st);
      m_min = dev_reduce_min(ms, N, ctx->tmp, st);
      const double total = L * L * L;
      if (!(m_min > 0) || !std::isfinite(msum) || std::fabs(msum - total) > 1e-9 * total)
        MAK_FAIL(MAK_EINVAL, "masses must be positive and sum to L^3");
    }

    // Walk certificates (PassOpts::cert_mode): once the Newton steps are
    // undamped (a full step after a full step), one trial records them;
    // every later pass uses them.  Margin and widening scale with the mean
    // site spacing s: 0.05 s^2 in weight, 0.05 s in space.
    CertSet& ce = ctx->scert;
    ce.valid = false;
    const bool certs = o.walk_cert != 0 && N >= 2 && N <= (int64_t(1) << 27);
    // Combinatorics records of the accepted pass and of the trial (swapped
    // with them on acceptance).
    const bool topo = o.topo_reuse != 0 && N >= 2;
    if (topo) {
      for (CellPass* c : {&ctx->scp, &ctx->scp_trial}) {
        c->topo_tri.ensure(size_t(N) * kTopoTri * sizeof(uint16_t));
        c->topo_n.ensure(size_t(N) * sizeof(int32_t));
      }
    }
    const double spacing = L / std::cbrt(double(N));
    int cur_cert = 0;
    auto pass = [&](CellPass& cp, bool tolerate, double doom_vol, const Lap* warm, int64_t probe_n = 0,
                    const int32_t* probe_list = nullptr) {
      PassOpts po;
      po.precision = o.precision;
      po.cert_mode = cur_cert;
      po.cert = cur_cert ? &ce : nullptr;
      po.tolerate_failure = tolerate;
      po.doom_vol = doom_vol;
      if (warm && warm->n == N) {
        po.warm_rp = warm->row_ptr.as<int64_t>();
        po.warm_col = warm->col.as<int32_t>();
        // J (the warm start) was built from the accepted pass's faces, whose
        // records index its rows
        if (topo) po.topo_in = &ctx->scp;
      }
      if (topo && probe_n <= 0) po.topo_out = &cp;
      po.first_stage = o.first_stage;
      if (probe_n > 0) {
        po.faces = false;
        po.probe_list = probe_list;
        po.probe_n = probe_n;
      }
      return ctx->runner ? ctx->runner->run(ps, cp, po, st) : run_cells(ps, cp, po, st);
    };
    // Probe of a line-search trial: the cells that rejected the earlier
    // trials of the same Newton step are clipped first (the shorter step
    // usually fails on the same cell); one of them below eps0 rejects the
    // trial without the full pass, which would have been rejected for the
    // same cell.  (A linearised volume cannot point at them: the Newton step
    // moves every linearised volume towards its mass.)
    constexpr int kProbeCap = 64;
    const int64_t kSmall = std::min<int64_t>(8192, N);
    ctx->probe_list.ensure(size_t(kProbeCap + kSmall) * sizeof(int32_t));
    std::vector<int32_t> doomed_cells;
    int64_t n_small = 0;
    set_psi_sorted(ps, psi_s, st);
    ClipStats cs = pass(ctx->scp, false, 0.0, nullptr);
    si.cell_passes = 1;
    si.overflow_cells += cs.retried - cs.fp64_rerun;
    si.fp64_rerun_cells += cs.fp64_rerun;
    FlagStats fs = flag_stats(ps, ctx->scp, ctx->tmp, st);
    if (fs.coincident > 0) MAK_FAIL(MAK_EDEGENERATE, "coincident sites");
    build_lap(ps, ctx->scp, ctx->sJ, o.precision == MAK_MIXED, st);
    double err = 0, vmin = 0;
    double gn = residual_stats(ctx->scp.vol.as<double>(), m, ms, N, ctx->tmp, &err, &vmin, st);
    const double eps0 = 0.5 * std::min(m_min, vmin);
    if (o.verbose) fprintf(stderr, "[mak] N=%lld it=0 err=%.3e minV/m=%.3e\n", (long long)N, err, vmin / m);
    std::string noconv;
    double prev_alpha = 1.0;
    for (int it = 0;; ++it) {
      if (err <= tol) break;
      if (it >= o.max_newton) {
        noconv = "Newton iteration limit reached, err=" + std::to_string(err);
        break;
      }
      newton_residual(ctx->scp.vol.as<double>(), m, ms, ctx->g.as<double>(), N, st);
      // After a damped step alpha p the residual is about (1 - alpha) g and J
      // has barely moved, so (1 - alpha) p predicts the next direction: CG
      // starts there (after a full step, from 0).
      const bool warm = it > 0 && prev_alpha < 1.0;
      if (warm)
        axpy_into(ctx->pstep.as<double>(), ctx->pstep.as<double>(), -prev_alpha, ctx->pstep.as<double>(), N, st);
      RowBlocks rb;
      rb.cell_start = ps.cell_start.as<int32_t>();
      rb.Gb = ps.g.Gb;
      rb.agg_per_axis = o.cg_precond == 2 ? 8 : 0;
      const int cgi = pcg_solve(ctx->sJ, ctx->g.as<double>(), ctx->pstep.as<double>(), N, o.cg_rtol,
                                o.max_cg, ctx->pw, st, warm, o.cg_precond != 1 ? &rb : nullptr);
      si.cg_iters_total += cgi;
      doomed_cells.clear();
      // the smallest cells of the accepted pass follow the doomed ones in the list
      n_small = smallest_cells(ctx->scp.vol.as<double>(), eps0, ctx->probe_list.as<int32_t>() + kProbeCap,
                               kSmall, N, ctx->probe_tmp, st);
      double alpha = 1.0;
      bool accepted = false;
      for (int ls = 0; ls <= o.max_halvings; ++ls) {
        axpy_into(ctx->psi_s.as<double>(), ctx->pstep.as<double>(), alpha, ctx->psi_t.as<double>(), N, st);
        set_psi_sorted(ps, ctx->psi_t.as<double>(), st);
        const auto tp0 = std::chrono::steady_clock::now();
        cur_cert = 0;
        if (ce.valid) {
          cert_dmax(ps, ce, st);
          cur_cert = 2;
        }
        const int64_t nd = int64_t(doomed_cells.size());
        if (nd + n_small > 0) {
          // doomed cells fill the slots just before the smallest ones
          int32_t* list = ctx->probe_list.as<int32_t>() + (kProbeCap - nd);
          if (nd > 0)
            MAK_HIP(hipMemcpyAsync(list, doomed_cells.data(), size_t(nd) * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
          const ClipStats pc = pass(ctx->scp_trial, true, eps0, &ctx->sJ, nd + n_small, list);
          if (pc.doomed) {
            si.cell_passes += 1;
            si.ls_trials += 1;
            si.abandoned_trials += 1;
            if (o.verbose >= 2)
              fprintf(stderr, "[mak]   trial alpha=%g probe of %lld cells %.1f ms: a cell below eps0, abandoned\n",
                      alpha, (long long)(nd + n_small),
                      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count());
            alpha *= 0.5;
            continue;
          }
        }
        // a trial with a cell below eps0 is rejected whatever else it gives:
        // the pass stops at the first such cell
        // the accepted pass's neighbours (J) warm-start the trial
        if (certs && !ce.valid && it > 0 && alpha == 1.0 && prev_alpha == 1.0) {
          ce.list.ensure(size_t(N) * kCertCap * sizeof(uint32_t));
          ce.n.ensure(size_t(N) * sizeof(int32_t));
          ce.vtx.ensure(size_t(N) * kCertVtx * sizeof(uint32_t));
          ce.scale.ensure(size_t(N) * sizeof(float));
          ce.psi_ref.ensure(size_t(N) * sizeof(double));
          ce.dmax.ensure(sizeof(unsigned long long));
          ce.margin = 0.05 * spacing * spacing;
          ce.kappa = 0.05 * spacing;
          cert_snapshot(ps, ce, st);
          cur_cert = 1;
        }
        ClipStats ct = pass(ctx->scp_trial, true, eps0, &ctx->sJ);
        if (cur_cert == 1) ce.valid = !ct.doomed && ct.overflow == 0;
        si.cell_passes += 1;
        si.ls_trials += 1;
        if (ct.doomed) {
          si.abandoned_trials += 1;
          if (ct.doom_cell >= 0 && ct.doom_cell < N && int(doomed_cells.size()) < kProbeCap &&
              std::find(doomed_cells.begin(), doomed_cells.end(), int32_t(ct.doom_cell)) == doomed_cells.end())
            doomed_cells.push_back(int32_t(ct.doom_cell));
          if (o.verbose >= 2)
            fprintf(stderr, "[mak]   trial alpha=%g pass %.1f ms: a cell below eps0, abandoned\n", alpha,
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count());
          alpha *= 0.5;
          continue;
        }
        si.overflow_cells += ct.retried - ct.fp64_rerun;
        si.fp64_rerun_cells += ct.fp64_rerun;
        if (ct.overflow > 0) {  // cells beyond the polytope capacity: reject the trial
          if (o.verbose >= 2)
            fprintf(stderr, "[mak]   trial alpha=%g pass %.1f ms: %lld cells over capacity\n", alpha,
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count(),
                    (long long)ct.overflow);
          alpha *= 0.5;
          continue;
        }
        double e2 = 0, v2 = 0;
        const double g2 =
            residual_stats(ctx->scp_trial.vol.as<double>(), m, ms, N, ctx->tmp, &e2, &v2, st);
        if (o.verbose >= 2)
          fprintf(stderr,
                  "[mak]   trial alpha=%g pass %.1f ms retried=%lld cert=%d: err=%.3e |g| %.3e -> %.3e minV/m=%.3e\n",
                  alpha, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count(),
                  (long long)ct.retried, cur_cert, e2, gn, g2, v2 / m);
        if (v2 >= eps0 && g2 <= (1.0 - 0.5 * alpha) * gn) {
          swap_buf(ctx->psi_s, ctx->psi_t);
          swap_pass(ctx->scp, ctx->scp_trial);
          build_lap(ps, ctx->scp, ctx->sJ, o.precision == MAK_MIXED, st);
          err = e2;
          gn = g2;
          vmin = v2;
          accepted = true;
          break;
        }
        alpha *= 0.5;
      }
      if (!accepted) {
        set_psi_sorted(ps, ctx->psi_s.as<double>(), st);
        noconv = "line search failed";
        break;
      }
      si.newton_iters += 1;
      prev_alpha = alpha;
      if (o.verbose)
        fprintf(stderr, "[mak] it=%d err=%.3e alpha=%g cg=%d minV/m=%.3e\n", it + 1, err, alpha, cgi,
                vmin / m);
    }
    si.final_err = err;
    // outputs of the last accepted iterate (also when the limits were hit)
    finalize_outputs(ps, ctx->psi_s.as<double>(), 0.0, ctx->scp.vol.as<double>(),
                     ctx->scp.mom.as<double>(), psi, centroids, displacements, st);
    if (!noconv.empty()) {
      MAK_HIP(hipStreamSynchronize(st));
      MAK_FAIL(MAK_ENOCONV, noconv);
    }
    MAK_HIP(hipStreamSynchronize(st));
  });
  si.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = si;
  return status;
}

mak_status mak_solve(mak_ctx* ctx, const double* points, int64_t N, double L, double tol, double* psi,
                     double* centroids, double* displacements, mak_solve_info* info, void* stream) {
  return solve_impl(ctx, points, nullptr, N, L, tol, nullptr, psi, centroids, displacements, info, stream);
}

mak_status mak_solve_masses(mak_ctx* ctx, const double* points, const double* masses, int64_t N,
                            double L, double tol, double* psi, double* centroids, double* displacements,
                            mak_solve_info* info, void* stream) {
  if (!masses) return MAK_EINVAL;
  return solve_impl(ctx, points, masses, N, L, tol, nullptr, psi, centroids, displacements, info, stream);
}

mak_status mak_solve_from(mak_ctx* ctx, const double* points, int64_t N, double L, double tol,
                          double* psi, double* centroids, double* displacements, mak_solve_info* info,
                          void* stream) {
  if (!psi) return MAK_EINVAL;
  return solve_impl(ctx, points, nullptr, N, L, tol, psi, psi, centroids, displacements, info, stream);
}

mak_status mak_profile_enable(mak_ctx* ctx, int32_t flags) {
  if (!ctx) return MAK_EINVAL;
  return guarded(ctx, [&] {
    set_device(ctx);
    ctx->prof.clear();
    ctx->prof.timing = (flags & 1) != 0;
    ctx->prof.counting = (flags & 2) != 0;
    ctx->prof.cells_only = (flags & 4) != 0;
  });
}

int32_t mak_profile_read(mak_ctx* ctx, mak_kernel_profile* out, int32_t max_entries) {
  if (!ctx) return -1;
  int32_t n = 0;
  const mak_status st = guarded(ctx, [&] {
    set_device(ctx);
    ctx->prof.resolve();
    for (const auto& kv : ctx->prof.acc) {
      if (out && n < max_entries) {
        mak_kernel_profile& o = out[n];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
        o.launches = kv.second.launches;
        o.total_ms = kv.second.ms;
        o.units = kv.second.units;
        o.flops = kv.second.flops;
        o.bytes = kv.second.bytes;
      }
      ++n;
    }
  });
  return st == MAK_OK ? n : -1;
}

mak_status mak_profile_counters(mak_ctx* ctx, double* out) {
  if (!ctx || !out) return MAK_EINVAL;
  for (int k = 0; k < mak::kProfCounters; ++k) out[k] = ctx->prof.counters[k];
  return MAK_OK;
}

size_t mak_solve_memory_estimate(int64_t N, int32_t precision) {
  (void)precision;
  if (N < 1) return 0;
  return size_t(N) * solve_bytes_per_site(N) + (size_t(64) << 20);
}

void mak_device_bytes(size_t* live, size_t* peak, int32_t reset_peak) {
  const int64_t l = mak::g_dev_bytes.live.load();
  if (live) *live = size_t(l > 0 ? l : 0);
  if (peak) {
    const int64_t p = mak::g_dev_bytes.peak.load();
    *peak = size_t(p > 0 ? p : 0);
  }
  if (reset_peak) mak::g_dev_bytes.peak.store(mak::g_dev_bytes.live.load());
}

}  // extern "C"
