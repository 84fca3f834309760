// Host-side engine: device workspace of one point set and the launchers of the
// pass kernels (grid build, clip, CSR assembly, PCG).
#pragma once

#include <atomic>
#include <string>
#include <vector>

#include "common.h"

struct mak_ctx;

namespace mak {

// Device bytes held by all DevBufs of the process (every context and
// server), and the most held at once since the last reset, updated at every
// allocation: what the library really holds, beside the estimates the server
// admits requests by.
struct DevBytes {
  std::atomic<int64_t> live{0}, peak{0};
  void add(int64_t b) {
    const int64_t now = live.fetch_add(b) + b;
    int64_t p = peak.load();
    while (now > p && !peak.compare_exchange_weak(p, now)) {
    }
  }
};
inline DevBytes g_dev_bytes;

// A growable device buffer owned by the engine, or a fixed view of memory
// owned elsewhere (borrow(): never allocated or freed here; a request beyond
// its size fails instead of allocating).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool borrowed = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !borrowed) {
      (void)hipFree(p);
      g_dev_bytes.add(-int64_t(cap));
    }
    p = nullptr;
    cap = 0;
    borrowed = false;
  }
  void borrow(void* q, size_t bytes) {
    release();
    p = q;
    cap = bytes;
    borrowed = true;
  }
  void ensure(size_t bytes) {
    if (bytes <= cap && p) return;
    if (borrowed)
      MAK_FAIL(MAK_ENOMEM, "borrowed workspace of " + std::to_string(cap) + " bytes, " +
                               std::to_string(bytes) + " needed");
    release();
    size_t want = bytes < 256 ? 256 : bytes;
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      MAK_FAIL(MAK_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    cap = want;
    g_dev_bytes.add(int64_t(want));
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// One face of a cell as written by the clip kernel (16 bytes).
struct FaceRec {
  int32_t j;      // other site, sorted index
  int32_t shift;  // packed periodic image of site j
  double w;       // area / |x_j + shift L - x_i|, the Hessian weight of the face
};

// Per-cell flag bits written by the clip kernel.
enum : int32_t {
  CF_EMPTY = 1,
  CF_COINCIDENT = 2,
  CF_CAPACITY = 4,     // polytope capacity exceeded: re-run with the large kernel
  CF_NONMANIFOLD = 8,  // inconsistent cut (rounding): re-run in float64 / reported
  CF_NEARDEG = 16,     // ill-conditioned vertex (mixed precision: re-run in float64)
};

constexpr int BLOCK_SIDE = 4;  // neighbour-grid cells per block side
constexpr int SHELL_MAX = 6;   // block shells covered by the per-block weight bounds

struct GridDesc {
  int32_t Gn = 0;   // cells per axis (multiple of BLOCK_SIDE)
  int32_t Gb = 0;   // blocks per axis
  double h = 0;     // cell side
  double L = 0;
  int64_t G() const { return int64_t(Gn) * Gn * Gn; }
  int64_t GB() const { return int64_t(Gb) * Gb * Gb; }
};

GridDesc make_grid(int64_t N, double L, double occupancy);

// Device state of one point set (sorted by neighbour-grid cell).
struct PointSet {
  int64_t N = 0;
  GridDesc g;
  DevBuf pts;          // double4 [N]: x, y, z (wrapped), psi      (sorted order)
  DevBuf perm;         // int32 [N]: sorted -> original index
  DevBuf cell_start;   // int32 [G + 1]
  DevBuf cell_psimax;  // double [G]
  DevBuf block_psimax; // double [GB]
  DevBuf block_suffix; // double [GB * (SHELL_MAX + 1)]: max weight over the blocks at
                       // Chebyshev block distance exactly r from each block
  DevBuf block_g;      // double [GB * 3]: slope of the tilted bounds
  DevBuf block_tmax;   // double [GB]: max_j psi_j - g . (x_j - x_block centre)
  DevBuf cell_tmax;    // double [G]: the same over the sites of each cell
  DevBuf scal;         // double [8]: [0] global psi max, [1] global psi min
  DevBuf key, rank, count, status, tmp;  // build temporaries (released after the
                                         // build of a large set)
};

// Face records of one cell pass.  A cell with at most `fslot` faces keeps them
// in its own slots; a larger one keeps them all in the overflow region, from
// fbase[cell].  The solver shares one store between the accepted pass and the
// line-search trial: once J is assembled the faces of the accepted pass are
// dead, so a trial may overwrite them.
struct FaceStore {
  DevBuf faces;      // FaceRec [N * fslot]
  DevBuf fbase;      // int64 [N]
  DevBuf ovf;        // FaceRec [ovf_cap]
  int32_t fslot = 0;
  int64_t ovf_cap = 0;
};

// Layout of a pass's device counters (uint64): [0] overflow faces used,
// [1 + s] cells listed by stage s, [4] the doom flag of a line-search trial,
// [5] a cell that raised it, work counters from kCtrStats, the causes of the
// stage re-runs from kCtrCause (three per stage).
constexpr int kCtrStats = 8;
constexpr int kCtrCause = 64;
constexpr int kCtrN = 80;

// Output of one cell pass (sorted order).
struct CellPass {
  DevBuf vol;        // double [N]
  DevBuf mom;        // double [3N] first moment, seed-local
  DevBuf cflags;     // int32 [N]
  DevBuf nface;      // int32 [N]
  DevBuf counters;   // uint64 [kCtrN]: overflow faces used, stage lists, work counters
  DevBuf retry;      // int32 [3N]: cells listed for the next stage
  DevBuf scan_tmp;
  FaceStore own;
  FaceStore* shared = nullptr;  // face storage in use (`own` when NULL)
  FaceStore& fs() { return shared ? *shared : own; }
  const FaceStore& fs() const { return shared ? *shared : own; }
  // Combinatorics of each cell (when the solver asks for them; see PassOpts).
  DevBuf topo_tri;   // uint16 [N][kTopoTri]
  DevBuf topo_n;     // int32 [N]: triangles recorded, or -1
};

// Combinatorics of a cell as a later pass can reuse them: its triangles (the
// dual of its vertices, three 5-bit plane codes in 16 bits) with each plane
// coded as 0..5 (the box of the site's own images) or 6 + r, r the rank of
// the face's site among the cell's face sites in increasing order, which is
// its position in the cell's row of J.  A cell with more than kTopoTri
// triangles or kTopoFaces faces, two faces with the same site, or a triangle
// on a plane that wrote no face (area below the pass's threshold) records
// none.
constexpr int kTopoTri = 48;
constexpr int kTopoFaces = 25;
constexpr size_t kTopoBytesPerSite = 2 * kTopoTri + 4;

// Bytes of device memory per site (and fixed) that one solve holds.
size_t solve_bytes_per_site(int64_t N);

struct Csr {
  int64_t n = 0, nnz = 0;
  DevBuf row_ptr;  // int64 [n + 1]
  DevBuf col;      // int32 [nnz]
  DevBuf val;      // double [nnz]
  DevBuf rowcnt;   // int64 [n]
};

// J in the solver's graph-Laplacian form: off-diagonal weights only,
// w_ij = sum over the faces of cell i with images of site j of A / |d|
// (J_ij = -w_ij), and the diagonal J_ii = sum_j w_ij of the stored weights,
// so the rows sum to zero exactly.  Weights in float on the mixed path (the
// CG vectors, dots and the diagonal stay float64), float64 otherwise.
struct Lap {
  int64_t n = 0, nnz = 0;
  bool f32 = false;
  DevBuf row_ptr;  // int64 [n + 1]
  DevBuf col;      // int32 [nnz], sorted within a row
  DevBuf w;        // float or double [nnz]
  DevBuf diag;     // double [n]
  DevBuf rowcnt;   // int64 [n]
  // Mixed path: the same off-diagonal weights in SELL-64 form for the SpMV
  // (float; not built for FP64 weights): slice s holds
  // rows 64 s .. 64 s + 63 column-major (entry k of row 64 s + l at
  // soff[s] + 64 k + l), padded to the slice's longest row with the row's own
  // column and weight 0.
  int64_t nsl = 0, sell_n = 0;
  DevBuf soff;     // int64 [nsl + 1] (exclusive scan of 64 x slen, total last)
  DevBuf slen;     // int32 [nsl]
  DevBuf slen64;   // int64 [nsl] (scan input)
  DevBuf scol;     // int32 [sell_n]
  DevBuf sw;       // float [sell_n]
};

// --- grid.hip
// Device bytes build_pointset needs for N sites on the grid g, counting each
// buffer rounded up to 256 bytes (the layout borrow_pointset carves).
size_t pointset_bytes(int64_t N, const GridDesc& g);
// Point every buffer of `ps` (and a 4-byte status word) into `base`, which
// holds pointset_bytes(N, g) + 256 bytes; build_pointset then allocates
// nothing.
void borrow_pointset(PointSet& ps, DevBuf& status, char* base, int64_t N, const GridDesc& g);
// Wrap, validate and sort `points` (original order, device) into `ps`; psi may
// be NULL (zeros).  Returns MAK_OK / EINVAL through exceptions.
void build_pointset(PointSet& ps, const double* points, const double* psi, int64_t N, double L,
                    double occupancy, hipStream_t st);
// psi (sorted order, device) -> pts[].w and the per-cell / per-block / global
// maxima used by the search bounds.
void set_psi_sorted(PointSet& ps, const double* psi_sorted, hipStream_t st);
void update_psi_bounds(PointSet& ps, hipStream_t st);

// --- clip.hip
struct ClipStats {
  int64_t retried = 0, overflow = 0, fp64_rerun = 0;
  bool doomed = false;  // a cell ended below doom_vol: the pass was abandoned
  int64_t doom_cell = -1;  // one such cell (sorted index)
};
// Walk certificates.  A recording pass lists, for each cell, every site whose
// bisector, with that site's weight raised by `margin` relative to the
// cell's, could still reach the final polytope P widened by kappa (P + a ball
// of radius kappa); its walk runs with the search bounds widened the same
// way, so every site it does not list can cut no polytope inside P + kappa
// while the weights move by at most `margin`.  It also records P's
// vertices.  A later pass over the same sites whose weights moved by less
// (max_j (psi_j - psi_ref_j) - (psi_i - psi_ref_i) <= margin) clips the
// listed sites only; when every vertex of the result lies within kappa of a
// recorded vertex, the result lies inside P + kappa and the walk is skipped:
// the polytope is the walk's.  Otherwise the cell walks.
constexpr int kCertCap = 48;  // sites a certificate lists
constexpr int kCertVtx = 48;  // vertices it records
struct CertSet {
  DevBuf list;     // uint32 [N][kCertCap]: site << 5 | image code (27 shifts in -1..1)
  DevBuf n;        // int32 [N]: listed sites | vertices << 8, -1 no certificate
  DevBuf vtx;      // uint32 [N][kCertVtx]: vertices, 11/11/10-bit offsets from the site
  DevBuf scale;    // float [N]: scale of those offsets (a bound on the vertex distances)
  DevBuf psi_ref;  // double [N]: the recording pass's weights (sorted order)
  DevBuf dmax;     // uint64 [1]: max_j (psi_j - psi_ref_j) of the current weights (ordered key)
  double margin = 0, kappa = 0;
  bool valid = false;  // a complete recording pass stands behind the arrays
};
// Bytes per site of a CertSet.
constexpr size_t kCertBytesPerSite = 4 * kCertCap + 4 + 4 * kCertVtx + 4 + 8;
// psi_ref <- the weights in ps.pts[].w (at a recording pass).
void cert_snapshot(const PointSet& ps, CertSet& c, hipStream_t st);
// dmax <- max_j (pts[j].w - psi_ref[j]) (before a pass that uses the set).
void cert_dmax(const PointSet& ps, CertSet& c, hipStream_t st);

// How one cell pass runs.
struct PassOpts {
  int precision = MAK_FP64;  // MAK_FP64 or MAK_MIXED
  bool faces = true;         // write the face records (for J)
  // Cells the largest kernel cannot represent are reported in
  // ClipStats::overflow instead of failing the pass (a line-search trial is
  // then rejected).
  bool tolerate_failure = false;
  // > 0 (a line-search trial): the first cell whose volume ends below it (or
  // empty) abandons the pass: ClipStats::doomed, outputs unspecified.
  double doom_vol = 0.0;
  // Neighbour lists of an earlier pass over the same sorted sites (CSR rows;
  // may be NULL): they are clipped first (a warm start; results differ only
  // by rounding).
  const int64_t* warm_rp = nullptr;
  const int32_t* warm_col = nullptr;
  // Stage the pass starts at (0: the first kernel); > 0 runs every cell in
  // the fallback kernels (testing them).
  int first_stage = 0;
  // A probe (probe_n > 0, with doom_vol > 0): only the listed cells (sorted
  // indices, device), only the first stage, no faces; ClipStats::doomed
  // reports whether one of them ended below doom_vol.  Cells the first stage
  // cannot finish are left undecided.  Each listed cell gets the bits the
  // full pass would give it, so a doomed probe means a doomed pass.
  const int32_t* probe_list = nullptr;
  int64_t probe_n = 0;
  // Walk certificates (with a warm start only): 1 records them (full passes
  // only; `cert` sized for N sites, psi_ref snapshotted), 2 uses them (dmax
  // computed for the current weights).
  int cert_mode = 0;
  CertSet* cert = nullptr;
  // Combinatorics reuse (with a warm start only).  topo_in: the records of
  // the pass whose J rows are warm_rp / warm_col; a cell with a record first
  // rebuilds that polytope from its J row's planes at the current weights
  // and keeps it when every vertex lies strictly inside every other plane of
  // the row and the box (then it is exactly the intersection of those
  // half-spaces), instead of clipping the row's planes one by one; the walk
  // follows as usual.  topo_out: where this pass records its cells (full
  // passes only; sized for N sites).
  const CellPass* topo_in = nullptr;
  CellPass* topo_out = nullptr;
};

// Full cell pass at the psi stored in ps.pts[].w.  Throws on failure.
ClipStats run_cells(PointSet& ps, CellPass& out, const PassOpts& o, hipStream_t st);

// Cell passes of several point sets in shared launches (the serving form):
// each job runs its stages like run_cells, but every stage launch carries up
// to kMaxJobs jobs (of one precision).  Errors are reported per job (status
// / err), not thrown.
constexpr int kMaxJobs = 8;
struct PassJob {
  PointSet* ps = nullptr;
  CellPass* out = nullptr;
  PassOpts opt;
  // results
  ClipStats cs;
  mak_status status = MAK_OK;
  std::string err;
  // progress (driver-internal)
  int stage = 0, attempt = 0;
  bool all_cells = true;  // the current stage runs over every cell
  int64_t listed = 0;
  unsigned long long hc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};
void run_cells_batch(PassJob* const* jobs, int njobs, int precision, hipStream_t st);

// Who runs the cell passes of a solve: by default the solve's own stream
// (run_cells); the server substitutes its batcher, which packs the passes of
// concurrent requests into shared launches.
struct PassRunner {
  virtual ~PassRunner() = default;
  virtual ClipStats run(PointSet& ps, CellPass& out, const PassOpts& o, hipStream_t st) = 0;
};
void set_pass_runner(::mak_ctx* ctx, PassRunner* r);

// --- csr.hip
// Assemble J (sorted index space, or original space when perm != NULL).
void build_csr(const PointSet& ps, CellPass& cp, Csr& J, bool original_space, hipStream_t st);
// Assemble the solver's Laplacian form of J (sorted index space).
void build_lap(const PointSet& ps, CellPass& cp, Lap& J, bool f32, hipStream_t st);
// Faces (original space) for mak_faces_copy; returns the face count.
int64_t count_faces(const PointSet& ps, CellPass& cp, Csr& J, DevBuf& face_ptr, hipStream_t st);
void copy_faces(const PointSet& ps, CellPass& cp, const DevBuf& face_ptr, int64_t* out_ptr,
                int32_t* fj, int32_t* fshift, double* farea, hipStream_t st);
// Face slots per cell for a point set of N sites.
int32_t face_slots(int64_t N);

// --- locate.hip
// Legendre transform of the weights stored in ps at query points (queries:
// device (Q, 3), any coordinates) or, when queries is NULL, at the ng^3 mesh
// nodes ((a, b, c) + offset) L / ng (row-major, c fastest): phi, the original
// index of the Laguerre cell holding the point, and x_i + kL - q.  Outputs
// may be NULL.  Throws MAK_EINVAL for a non-finite query coordinate.
void locate(const PointSet& ps, const double* queries, int64_t Q, int64_t ng, double offset,
            double* phi, int32_t* idx, double* disp, DevBuf& status, hipStream_t st);

// Zel'dovich advection and Eulerian deposition: the n_lag^3 mass elements
// at the Lagrangian mesh nodes ((a, b, c) + lag_offset) L / n_lag move to
// q + tau (x_i(q) + kL - q) and are deposited on the ne^3 Eulerian mesh
// (nodes (a, b, c) L / ne; scheme 1 nearest grid point, 2 cloud in cell):
// density (ne^3, mean 1) = deposited mass / cell volume.  acc: scratch of
// ne^3 uint64.
void za_deposit(const PointSet& ps, double tau, int64_t n_lag, double lag_offset, int64_t ne, int scheme,
                double* density, DevBuf& acc, hipStream_t st);

// --- noalloc.hip
// The device array behind mak_legendre_noalloc: noalloc_setup resolves this
// device's copy (call with the device current; false on failure),
// noalloc_scratch returns it (NULL before setup), noalloc_capacity its size.
bool noalloc_setup(int device);
void* noalloc_scratch(int device);
size_t noalloc_capacity();

// --- cells_deposit.hip
// Exact deposit of the cells moved to growth amplitude tau in [0, 1): each
// cell of the pass `cp` (float64, with faces, at the weights in ps) shrunk by
// 1 - tau towards its site, clipped against the voxels of the ng^3 mesh
// (nodes (a, b, c) L / ng); density (ng^3, mean 1) = mass / voxel volume.
// acc: scratch of ng^3 uint64; status: 4 bytes.  Throws MAK_EOVERFLOW when a
// polytope exceeds the kernel's capacity.
void za_deposit_cells(const PointSet& ps, const CellPass& cp, double tau, int64_t ng, double* density,
                      DevBuf& acc, DevBuf& status, hipStream_t st);

// --- power.hip
// Shell-averaged power spectrum of a field on the periodic ng^3 mesh; the
// FFT plan (for the last ng) and the buffers are kept between calls.
struct PowerWork {
  int64_t ng = 0;  // length of the twiddle table in `tw`
  DevBuf tw, spec, part, sums, tmp;
};
void power_spectrum(PowerWork& w, const double* field, int64_t ng, double L, int nbins, int window,
                    bool contrast, double* k_mean, double* power, int64_t* modes, hipStream_t st);

// --- pcg.hip / reductions
double dev_reduce_max(const double* x, int64_t n, DevBuf& tmp, hipStream_t st);
double dev_reduce_min(const double* x, int64_t n, DevBuf& tmp, hipStream_t st);
double dev_reduce_sum(const double* x, int64_t n, DevBuf& tmp, hipStream_t st);
void dev_max_to(const double* x, int64_t n, double* out, DevBuf& tmp, hipStream_t st);
// Exclusive scans into out[0..n] (out[n] = the total); throws when `out` holds
// fewer than n + 1 entries.
void exclusive_scan_i64(const int64_t* in, DevBuf& out, int64_t n, DevBuf& tmp, hipStream_t st);
void exclusive_scan_i32(const int32_t* in, DevBuf& out, int64_t n, DevBuf& tmp, hipStream_t st);
// Bytes of `tmp` the 32-bit scan of n entries and the reductions above use.
size_t scan_tmp_bytes_i32(int64_t n);
size_t reduce_tmp_bytes();
// Zero n 32-bit words on the stream (a fill kernel, not a memset node).
void fill_zero_i32(int32_t* p, int64_t n, hipStream_t st);

struct PcgWork {
  DevBuf r, z, p, q, s, dinv, part, part2, scal;
  // three-level preconditioner: row -> grid block; per block the residual
  // sum, the inverse of the weight leaving it and its weights towards the
  // 26 neighbouring aggregates; per aggregate those weights summed and the
  // exact level's correction; the inverse of the aggregates' Laplacian
  DevBuf blk_row, r1, d1inv, a1c, aggw, cc, ainv;
  // host side of the convergence checks: two pinned flags and their events
  double* hflag = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  PcgWork() = default;
  PcgWork(const PcgWork&) = delete;
  PcgWork& operator=(const PcgWork&) = delete;
  ~PcgWork() {
    if (hflag) (void)hipHostFree(hflag);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void ensure_host() {
    if (!hflag && hipHostMalloc(reinterpret_cast<void**>(&hflag), 2 * sizeof(double), 0) != hipSuccess) {
      hflag = nullptr;
      (void)hipGetLastError();
      MAK_FAIL(MAK_ENOMEM, "pinned host allocation failed");
    }
    for (hipEvent_t& e : ev)
      if (!e) MAK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
};
// The neighbour grid of the rows of J (sites sorted block-major): block b
// holds rows cell_start[64 b] .. cell_start[64 b + 64) of the Gb^3 blocks.
struct RowBlocks {
  const int32_t* cell_start = nullptr;
  int32_t Gb = 0;
  // aggregates per axis of the exact level (at most 8): 0 the default, 4
  int32_t agg_per_axis = 0;
};
// Solve J x = b - mean(b) with preconditioned CG to ||r|| <= rtol ||b -
// mean(b)||; x is overwritten (mean zero on return).  The preconditioner is
// point Jacobi, or with `blocks` the three-level additive one (point Jacobi,
// Jacobi on the grid blocks, an exact solve on at most 64 aggregates of
// blocks).  It starts from 0, or with `warm` from the x given when that
// residual is below ||b - mean(b)||.  Returns the iteration count.
int pcg_solve(const Lap& J, const double* b, double* x, int64_t n, double rtol, int max_iter,
              PcgWork& w, hipStream_t st, bool warm = false, const RowBlocks* blocks = nullptr);

// Elementwise helpers for the Newton driver.
// Target masses: per site (ms, sorted order) or, when ms is NULL, m for all.
void newton_residual(const double* vol, double m, const double* ms, double* g, int64_t n,
                     hipStream_t st);
void axpy_into(const double* psi, const double* p, double alpha, double* out, int64_t n,
               hipStream_t st);
// The cells with the smallest volumes: every cell below v0 2^k for the
// largest k that lists at most `cap` of them (sorted indices into `list`, in
// no particular order); returns how many were listed.
int64_t smallest_cells(const double* vol, double v0, int32_t* list, int64_t cap, int64_t n, DevBuf& tmp,
                       hipStream_t st);

// Returns ||m - V||_2; max_rel = max_i |m_i - V_i| / m_i, min_vol = min_i V_i.
double residual_stats(const double* vol, double m, const double* ms, int64_t n, DevBuf& tmp,
                      double* max_rel, double* min_vol, hipStream_t st);
void finalize_outputs(const PointSet& ps, const double* psi_sorted, double psi_mean,
                      const double* vol, const double* mom, double* psi_out, double* cent_out,
                      double* disp_out, hipStream_t st);
void scatter_cells_outputs(const PointSet& ps, const double* vol_s, const double* mom_s,
                           double* vol_out, double* cent_out, hipStream_t st);
void gather_sorted(const PointSet& ps, const double* orig, double* sorted, hipStream_t st);

}  // namespace mak
