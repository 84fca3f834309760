/*
 * mak.h -- C-ABI of the MI355X semi-discrete optimal transport library.
 *
 * The library computes the hot path of semi-discrete Monge-Ampere-Kantorovich
 * (MAK) reconstruction: the periodic Laguerre (power) diagram of N sites under
 * weights psi (Eq. laguerrecell), the cell integrals that give the gradient
 * and Hessian of the semi-discrete Kantorovich dual K(psi) (Eq. SDK), and the
 * damped Newton maximisation of K (the paper's Newton method on the concave,
 * C^2 functional K; step control of Kitagawa-Merigot-Thibert).
 *
 * Conventions shared by every entry point
 *   - Domain: the flat torus [0, L)^3.  Points outside are wrapped, not
 *     rejected.  Masses are uniform, m_i = L^3 / N (initial density 1).
 *   - Pointers marked DEVICE are HIP device memory on the context's device;
 *     the caller owns them.  Pointers marked HOST are host memory.
 *   - Points are row-major (N, 3) float64 (x, y, z); weights (N,) float64.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = the default stream).
 *     mak_laguerre_cells returns after enqueueing plus one device-to-host
 *     read of the nonzero count; mak_solve blocks until the outputs are
 *     written (Newton control runs on the host).
 *   - Errors are returned as mak_status; nothing throws across the ABI.  The
 *     message of the last failure on a context is at mak_last_error().
 *     After an error the outputs are unspecified.
 *   - A context may be used by one host thread at a time.
 */
#ifndef MAK_H
#define MAK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MAK_OK = 0,
  MAK_EINVAL = 1,       /* N < 1, L not finite or <= 0, tol <= 0, NULL pointer,
                           non-finite coordinate or weight */
  MAK_ENOMEM = 2,       /* device allocation failed / memory budget exceeded */
  MAK_EDEGENERATE = 3,  /* two sites coincide after wrapping */
  MAK_ENOCONV = 4,      /* Newton iteration or line-search limit reached */
  MAK_EOVERFLOW = 5,    /* a cell exceeded the largest polytope capacity */
  MAK_EHIP = 6,         /* HIP runtime error */
  MAK_ENOTFOUND = 7     /* unknown request id (server) */
} mak_status;

typedef enum {
  MAK_FP64 = 0,   /* clipping, integrals and Newton all in float64 */
  MAK_MIXED = 1   /* clipping in float32 seed-local coordinates, integrals
                     accumulated in float64, near-degenerate cells re-run in
                     float64; Newton, line search and CG vectors and dots in
                     float64, the solver's Hessian weights stored in float32 */
} mak_precision;

typedef struct {
  int32_t precision;       /* mak_precision, default MAK_FP64 */
  int32_t max_newton;      /* Newton iteration cap, default 60 */
  int32_t max_cg;          /* CG iterations per Newton step, default 4000 */
  int32_t max_halvings;    /* line-search halvings per step, default 30 */
  double cg_rtol;          /* CG stop: ||r|| <= cg_rtol ||g||, default 1e-3 */
  double grid_occupancy;   /* target sites per neighbour-grid cell, default 2.5 */
  size_t mem_budget_bytes; /* 0 = no limit (server admission uses it) */
  int32_t verbose;         /* 1: one line per Newton iteration on stderr, 2: also per trial */
  int32_t first_stage;     /* cell-pass stage to start at, default 0.  A pass
                              runs every cell in the first kernel and re-runs the
                              cells it cannot finish in the next: float64 path
                              0 = float64, 1 = float64 with the larger polytope
                              and a wider tie tolerance; mixed path 0 = float32
                              (up to 64 vertices), 1 = float64, 2 = the larger
                              float64 kernel.  A later
                              first stage runs all cells in that fallback kernel
                              (for testing it). */
  int32_t batch_window_us; /* server only: after the first cell pass is posted the
                              batcher waits up to this long (microseconds) for the
                              passes of the other solves in flight, so they share
                              launches; default 0 (no wait) */
  int32_t cg_precond;      /* CG preconditioner of the Newton system: 0 (default)
                              three-level additive (point Jacobi, Jacobi on the
                              aggregates of the neighbour-grid blocks, an exact
                              solve on at most 64 aggregates of those), 1 point
                              Jacobi alone, 2 the three-level form with the
                              exact level on up to 512 aggregates (fewer CG
                              iterations on large problems, a costlier set-up
                              per Newton step) */
  int32_t walk_cert;       /* 1 (default): once the Newton steps are undamped,
                              one cell pass records for each cell the sites
                              that can still cut it while the weights move by
                              less than a margin, and later passes within it
                              clip those sites only (same cells, shorter
                              search); 0: every pass searches in full.  Holds
                              about 250 more bytes per site. */
  int32_t topo_reuse;      /* 1 (default): every full cell pass of a solve
                              records each cell's combinatorics (its vertices
                              as triples of faces), and the next pass first
                              rebuilds that polytope from the planes of the
                              cell's J row at the new weights, keeping it when
                              every vertex lies strictly inside every other
                              plane (it is then exactly their intersection)
                              instead of clipping the row plane by plane; the
                              search that follows is unchanged, so the cells
                              are the same to rounding.  0: off.  Holds about
                              200 more bytes per site. */
  int32_t reserved[2];
} mak_options;

/* Fill `opt` with the defaults listed above. */
void mak_default_options(mak_options* opt);

typedef struct {
  int32_t newton_iters;       /* accepted Newton steps */
  int32_t cg_iters_total;     /* CG iterations over all steps */
  int32_t ls_trials;          /* cell passes spent in the line search */
  int32_t cell_passes;        /* all cell passes */
  int64_t fp64_rerun_cells;   /* cells re-run in float64 (mixed precision) */
  int64_t overflow_cells;     /* cells re-run with the large polytope capacity */
  double final_err;           /* max_i |V_i - m_i| / m_i at exit */
  double seconds;             /* wall time of the call */
  int32_t abandoned_trials;   /* line-search passes stopped at the first cell
                                 below eps0 (rejected whatever the rest gives) */
  int32_t reserved;
} mak_solve_info;

typedef struct {
  int64_t empty_cells;        /* cells with zero volume at this psi */
  int64_t fp64_rerun_cells;   /* mixed precision: cells re-run in float64 */
  int64_t overflow_cells;     /* cells re-run with the large polytope capacity */
  int64_t nnz;                /* nonzeros of the Hessian (with diagonal) */
  int64_t faces;              /* reported faces (each (i, j, image) once per side) */
  int32_t max_faces;          /* largest face count of one cell */
  int32_t reserved;
} mak_cells_info;

/* The Hessian of a cell pass in CSR form, as returned by mak_laguerre_cells:
 * library-owned DEVICE arrays, valid until the next mak_laguerre_cells or
 * mak_destroy on the same context; the caller must not write or free them. */
typedef struct {
  int64_t n_rows;          /* N */
  int64_t nnz;             /* nonzeros, diagonal included */
  const int64_t* row_ptr;  /* DEVICE [n_rows + 1] */
  const int32_t* col;      /* DEVICE [nnz], sorted within each row */
  const double* val;       /* DEVICE [nnz] */
} mak_csr;

typedef struct mak_ctx mak_ctx;

/* Create a context on HIP device `device` with options `opt` (NULL = the
 * defaults).  The context owns its device workspace, grown on demand and
 * released by mak_destroy.  *out is set on success. */
mak_status mak_create(mak_ctx** out, int device, const mak_options* opt);
void mak_destroy(mak_ctx* ctx);

/* Message of the last error on `ctx` (or of the last mak_create failure when
 * ctx is NULL).  Valid until the next call on the context. */
const char* mak_last_error(const mak_ctx* ctx);

/* One Laguerre cell pass (Eq. laguerrecell on the torus, integrands of
 * Eq. SDK).
 *   points     DEVICE (N, 3) float64, read only
 *   psi        DEVICE (N,) float64 weights, read only
 *   volumes    DEVICE (N,) float64 out: |V_i| (0 for an empty cell)
 *   centroids  DEVICE (N, 3) float64 out: centroid of V_i wrapped into
 *              [0, L)^3 (x_i for an empty cell)
 *   hessian    HOST, may be NULL: filled with the Hessian of this pass in
 *              CSR form (library-owned, see mak_csr; original site order)
 *   info       HOST, may be NULL: counters of this pass
 * The pass builds the Hessian J = dV/dpsi (= minus the Hessian of K, the
 * derivative of the cell volumes, the gradient of Eq. SDK, in the weights):
 * J_ij = -sum over the faces between cell i and images of site j of
 * area / |x_i - x_j^image|, J_ii = -sum_j J_ij.  Faces of a cell with its own
 * images do not enter J.  mak_hessian_copy copies it into caller memory.
 * Returns after enqueueing plus one device-to-host read of the nonzero count
 * (the outputs are then complete in stream order). */
mak_status mak_laguerre_cells(mak_ctx* ctx, const double* points, const double* psi,
                              int64_t N, double L, double* volumes, double* centroids,
                              mak_csr* hessian, mak_cells_info* info, void* stream);

/* Copy the Hessian of the last mak_laguerre_cells call on `ctx` as CSR with
 * sorted columns (diagonal included):
 *   row_ptr  DEVICE int64 [N + 1]
 *   col      DEVICE int32 [nnz]
 *   val      DEVICE float64 [nnz]
 * nnz is mak_cells_info.nnz of that call. */
mak_status mak_hessian_copy(mak_ctx* ctx, int64_t* row_ptr, int32_t* col, double* val,
                            void* stream);

/* Copy the faces of the last mak_laguerre_cells call (test and diagnostics
 * interface; faces with the site's own images are not reported):
 *   face_ptr   DEVICE int64 [N + 1], faces of cell i at face_ptr[i]..[i+1]
 *   face_j     DEVICE int32 [faces]  other site
 *   face_shift DEVICE int32 [faces, 3] periodic image of site j
 *   face_area  DEVICE float64 [faces]
 * `faces` is mak_cells_info.faces of that call.  Faces are sorted by
 * (j, shift) within a cell. */
mak_status mak_faces_copy(mak_ctx* ctx, int64_t* face_ptr, int32_t* face_j, int32_t* face_shift,
                          double* face_area, void* stream);

/* Damped Newton maximisation of K(psi) from psi = 0 until
 * max_i |V_i - m_i| / m_i <= tol (m_i = L^3 / N).
 * K is the semi-discrete Kantorovich dual of Eq. SDK, maximised under the
 * constraint that no Laguerre cell (Eq. laguerrecell) is empty; Sec. 2's
 * paragraph on the properties of K (concave, C^2) gives the Newton method on
 * its first and second derivatives, with convergence as in the damped scheme
 * of Kitagawa, Merigot and Thibert that it cites.  Each Newton system
 * J p = m - V is solved by preconditioned CG on the Laplacian of the face
 * areas over seed distances (the Hessian of K, as returned by
 * mak_laguerre_cells); the step length alpha = 2^-l is the largest with
 * min_i V_i >= eps0 = 1/2 min(min_i m_i, min_i V_i(0)) and
 * ||m - V||_2 <= (1 - alpha/2) ||m - V(psi)||_2.
 *   points         DEVICE (N, 3) float64, read only
 *   psi            DEVICE (N,) float64 out: the weights, mean zero
 *   centroids      DEVICE (N, 3) float64 out: cell centroids (the
 *                  Lagrangian positions), wrapped into [0, L)^3
 *   displacements  DEVICE (N, 3) float64 out: x_i - centroid_i taken in the
 *                  site's own frame (no wrap ambiguity)
 *   info           HOST, may be NULL
 * Returns MAK_ENOCONV if the Newton or line-search limit is hit (outputs then
 * hold the last accepted iterate). */
mak_status mak_solve(mak_ctx* ctx, const double* points, int64_t N, double L, double tol,
                     double* psi, double* centroids, double* displacements,
                     mak_solve_info* info, void* stream);

/* As mak_solve with a target mass per site instead of L^3 / N (Eq. SDK with
 * weighted sites: sum_i m_i psi_i; each cell must end with volume m_i, e.g.
 * sites standing for haloes of different masses):
 *   masses  DEVICE (N,) float64, read only; every m_i > 0 and sum_i m_i = L^3
 *           (to 1e-9 relative; MAK_EINVAL otherwise, uniform initial density)
 * The stop test is max_i |V_i - m_i| / m_i <= tol and the line search uses
 * eps0 = 1/2 min(min_i m_i, min_i V_i(0)). */
mak_status mak_solve_masses(mak_ctx* ctx, const double* points, const double* masses, int64_t N,
                            double L, double tol, double* psi, double* centroids,
                            double* displacements, mak_solve_info* info, void* stream);

/* As mak_solve, starting from the weights in `psi` (DEVICE, read and
 * overwritten): resumes a solve from a saved psi (the whole solver state). */
mak_status mak_solve_from(mak_ctx* ctx, const double* points, int64_t N, double L, double tol,
                          double* psi, double* centroids, double* displacements,
                          mak_solve_info* info, void* stream);

/* ---- Legendre transform of the weights and point location ----
 * Sec. 2, the equation after Eq. laguerrecell (with Eqs. potpot and
 * Legendre): the initial potential at a Lagrangian point q is
 *   phi(q) = min_i min_k [ 1/2 |q - x_i - k L|^2 - psi_i ]
 * (k over the periodic images), attained at i(q), the Laguerre cell that
 * holds q; x_{i(q)} + k L is where the transport map sends q.
 *   points   DEVICE (N, 3) float64, read only (wrapped like mak_laguerre_cells)
 *   psi      DEVICE (N,) float64, read only; NULL means all zero
 *   queries  DEVICE (Q, 3) float64, read only; any finite coordinates (taken
 *            modulo L); a non-finite one gives MAK_EINVAL (outputs then
 *            unspecified)
 *   phi      DEVICE (Q,) float64 out, or NULL
 *   idx      DEVICE (Q,) int32 out, or NULL: i(q), the original site index
 *   disp     DEVICE (Q, 3) float64 out, or NULL: x_{i(q)} + k L - q for the
 *            minimising image
 * Arithmetic is float64.  Where several sites attain the minimum to within
 * rounding, idx names one of them.  Builds its own copy of the site grid in
 * the context (independent of the last cell pass); synchronises `stream`. */
mak_status mak_legendre(mak_ctx* ctx, const double* points, const double* psi, int64_t N, double L,
                        const double* queries, int64_t Q, double* phi, int32_t* idx, double* disp,
                        void* stream);

/* mak_legendre for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results (bit for bit), but every buffer the
 * grid build and the location need lives in one static device array of
 * 64 MiB that the library holds on each device it runs on until the process
 * ends (its address is resolved by mak_create on that device).  No
 * hipMalloc, hipFree or allocating library routine is called.
 *   - The workspace is about 86 bytes per site (sorted sites, staging, grid
 *     and weight bounds), so N up to roughly 750,000 sites; a larger N gives
 *     MAK_EINVAL with the bytes it would need (the exact bound depends on the
 *     neighbour grid of N and the context's grid_occupancy).
 *   - Every call on one device shares that array: calls that overlap on a
 *     device (other streams or host threads, any context) race and must be
 *     serialised by the caller.  Each call leaves its contents behind; what
 *     must start at zero is cleared by the call's own kernels.
 *   - Like mak_legendre it synchronises `stream` (the non-finite-coordinate
 *     checks read a status word on the host).
 * MAK_EHIP if the array's address could not be resolved on this device. */
mak_status mak_legendre_noalloc(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                                double L, const double* queries, int64_t Q, double* phi, int32_t* idx,
                                double* disp, void* stream);

/* The same at the ng^3 mesh nodes q_abc = ((a, b, c) + offset) L / ng,
 * a, b, c in [0, ng) (1 <= ng <= 4096; offset in mesh spacings, e.g. 0 or
 * 0.5), generated on the device; outputs in row order (a, b, c), c fastest. */
mak_status mak_legendre_mesh(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                             double L, int64_t ng, double offset, double* phi, int32_t* idx,
                             double* disp, void* stream);

/* ---- Zel'dovich advection of the cells and Eulerian deposition ----
 * Sec. 2 (last paragraph) and Fig. 1: each Laguerre cell V_i (at the
 * weights psi) is the Lagrangian region whose mass ends at x_i; at growth
 * amplitude tau (0 initial, 1 final) the Zel'dovich approximation moves the
 * mass element at q to q + tau (x_i(q) - q), and the moved mass is expressed
 * as a density on an Eulerian mesh.  The cells' mass is carried by the
 * n_lag^3 elements at the Lagrangian mesh nodes ((a, b, c) + lag_offset)
 * L / n_lag, each of mass (L / n_lag)^3 (initial density 1), each located in
 * its cell as by mak_legendre_mesh and moved with its cell's image of x_i; as
 * n_lag grows the deposit converges to that of the moved cells.
 *   points, psi  as for mak_legendre (psi NULL: all zero)
 *   tau          in [0, 1]
 *   n_lag        1..2048;  ng 1..2048 (Eulerian nodes (a, b, c) L / ng)
 *   scheme       1: nearest grid point, 2: cloud in cell (trilinear)
 *   density      DEVICE (ng, ng, ng) float64 out, row-major: deposited mass
 *                / (L / ng)^3 (mean 1)
 * Masses are summed in 64-bit fixed point (2^(62 - ceil(log2 n_lag^3)) units
 * per element, at most 2^52; the cloud-in-cell weights are rounded to
 * units with the remainder on the heaviest node), so every element adds
 * exactly its mass and the result is the same bits on every run.  Uses
 * ng^3 x 8 bytes of scratch in the context. */
mak_status mak_za_deposit(mak_ctx* ctx, const double* points, const double* psi, int64_t N, double L,
                          double tau, int64_t n_lag, double lag_offset, int64_t ng, int32_t scheme,
                          double* density, void* stream);

/* The deposit of the moved cells themselves (the limit of mak_za_deposit as
 * n_lag grows): at growth amplitude tau the cell V_i becomes
 * S_i = x_i + (1 - tau)(V_i - x_i), which carries the mass |V_i| at density
 * 1 / (1 - tau)^3; the mass in the voxel [a H - H/2, a H + H/2)^3 of node a
 * (H = L / ng) is the volume of S_i inside it over (1 - tau)^3, found by
 * clipping polytopes in float64 (a cell pass with faces, then each cell
 * clipped against the voxels it reaches).
 *   points, psi  as for mak_legendre (psi NULL: all zero)
 *   tau          in [0, 1)
 *   ng           1..1024
 *   density      DEVICE (ng, ng, ng) float64 out, row-major: mass / H^3 (mean 1)
 * Masses are summed in 64-bit fixed point (unit L^3 2^-60, each cell-voxel
 * part rounded to the nearest unit), so the result is the same bits on every
 * run.  Vertices within 1e-14 L of a cutting plane count as on it (lattice
 * inputs put cell faces on voxel boundaries).  MAK_EDEGENERATE for
 * coincident sites; MAK_EOVERFLOW if a cell has more than 122 faces, a
 * clipped polytope more than 64 faces or 400 face corners in all, or a cut
 * meets more than four points of one face in the plane.  One wavefront
 * clips all the voxels of a cell, so MAK_EINVAL when the largest moved cell
 * spans more than 2^22 voxel volumes ((1 - tau)^3 max V_i / H^3).  Holds the cell pass (about 600 bytes a site)
 * and ng^3 x 8 bytes of scratch in the context. */
mak_status mak_za_deposit_cells(mak_ctx* ctx, const double* points, const double* psi, int64_t N,
                                double L, double tau, int64_t ng, double* density, void* stream);

/* ---- power spectrum of a mesh field ----
 * The estimator behind the fractional spectra of Sec. BAO reconstruction,
 * for a field f on the periodic ng^3 mesh of side L (spacing H = L / ng):
 *   delta(k) = H^3 sum_x f(x) exp(-i k . x), k = 2 pi n / L, n in (-ng/2, ng/2]^3,
 *   P(k) = |delta(k)|^2 / L^3,
 * averaged over shell j = 1..nbins (the modes with j - 1/2 <= |n| < j + 1/2;
 * k = 0 is left out).
 *   field    DEVICE (ng, ng, ng) float64, row-major (last index fastest), read only
 *   ng       2..2048;  nbins 1..2048 (ng / 2 reaches the Nyquist shell)
 *   window   0: none; 1, 2, 3: divide P by W^2, W = prod_a sinc(pi n_a / ng)^p,
 *            the window of nearest-grid-point, cloud-in-cell and
 *            triangular-shaped-cloud assignment (sinc x = sin x / x)
 *   contrast nonzero: the field is a density; use f / mean(f) - 1
 *            (MAK_EINVAL if the mean is zero or not finite)
 *   k_mean, power  DEVICE (nbins,) float64 out: mean |k| and mean P per shell
 *                  (NaN for a shell without modes)
 *   modes          DEVICE (nbins,) int64 out: modes per shell (each n and -n counted)
 * The transform is the library's own real-to-complex FFT (mixed radix, any
 * ng: three passes of one-dimensional transforms in LDS); its twiddle table
 * (for the last ng) and the half spectrum (ng^2 (ng/2 + 1) x 16 bytes) stay
 * in the context.  Deterministic: the same bits on every run. */
mak_status mak_power_spectrum(mak_ctx* ctx, const double* field, int64_t ng, double L, int32_t nbins,
                              int32_t window, int32_t contrast, double* k_mean, double* power,
                              int64_t* modes, void* stream);

/* ---- kernel profile (diagnostics; used by the benchmark) ----
 * When timing is enabled, the library brackets its main kernels with HIP
 * events on the stream each is launched on and accumulates their durations;
 * with work counting it also reads device work counters after every clip
 * launch (this adds a host synchronisation per launch, so time and count in
 * separate runs). */
typedef struct {
  char name[32];       /* "clip", "clip_large", "spmv", "pcg_update", "pcg_setup", "pcg_solve",
                          "csr_assembly", "grid_build", "locate", "deposit", "cells_deposit", "fft", "shell_bin" */
  int64_t launches;
  double total_ms;     /* summed event durations */
  double units;        /* work items processed (cells, rows) */
  double flops;        /* counted arithmetic of the method (work counting only,
                          clip kernels: see mak_profile_counters) */
  double bytes;        /* compulsory HBM bytes of the algorithm */
} mak_kernel_profile;

/* flags: bit 0 = time kernels, bit 1 = count clip work, bit 2 = time only
 * the cell-pass kernels (the events around the others cost ~2 % of a solve).
 * Clears the accumulated profile. */
mak_status mak_profile_enable(mak_ctx* ctx, int32_t flags);
/* Writes up to max_entries entries (HOST array, may be NULL) and returns the
 * number of entries available, or -1 on error.  Waits for pending events. */
int32_t mak_profile_read(mak_ctx* ctx, mak_kernel_profile* out, int32_t max_entries);
/* HOST double[48]: summed clip work counters.
 *   0-9    sites scanned, planes tested, vertex tests, cuts, new vertices,
 *          ball-update vertices, box tests, final vertices, faces, cells;
 *   10-14  shader-clock cycles summed over waves spent in the candidate
 *          search, the serial clipping and the integrals, and within those
 *          in the batch pre-filter (part of the search) and in the cuts that
 *          removed vertices (part of the clipping);
 *   15     the counted flops of the candidate search (site scans, ball
 *          updates, box tests), which the clip kernels' `flops` in
 *          mak_kernel_profile leave out (those count the method's
 *          arithmetic: plane formation, vertex tests, new vertices and the
 *          integrals);
 *   16-19  sites scanned by search phase (warm-start neighbours, the 27
 *          nearest grid cells, the second ring of cells, the cells of the
 *          block shells); 20-23 of those, the sites inside the ball and
 *          bounding-box bounds;
 *   24-27  planes that removed vertices, by the same phases;
 *   28-33  box tests and passes: ring-2 cells, blocks, cells of passing
 *          blocks;
 *   34     the last block shell reached, summed over cells;
 *   35-39  walk certificates of the solver (walk_cert): cells that recorded
 *          one, the sites they list, cells whose list overflowed; cells
 *          whose weights stayed within the margin (they clip the listed
 *          sites first) and, of those, cells whose walk was skipped.
 * Unused entries are zero. */
mak_status mak_profile_counters(mak_ctx* ctx, double* out);

/* ---- serving: many reconstruction requests on one device ----
 * A server owns `max_slots` worker slots, each with its own context (device
 * workspace kept resident between requests) and HIP stream.  The budget is
 * charged with what the slots hold: a slot's workspace, sized for the
 * largest request it has served since it was last emptied (by the memory
 * estimate, mak_solve_memory_estimate), stays charged while the slot is
 * idle.  Requests are admitted first-in first-out when a slot is free and
 * the total held after the head request (that slot's workspace resized for
 * it: kept when the request needs at least half of it, replaced otherwise)
 * fits in `mem_budget_bytes`; when no idle slot can take the head request,
 * idle slots give their workspace back.  Requests submitted while others run
 * start as soon as slots and memory free up (continuous batching).  The cell passes of all requests that need
 * one at the same time are packed into shared clip launches (up to 8 point
 * sets per launch) by the server's pass batcher; the Newton / PCG work of
 * each request runs on its slot's stream and overlaps on the device.
 * Results are bitwise the same as a solo mak_solve of the same input. */
typedef struct mak_server mak_server;

typedef struct {
  int64_t submitted, completed, queued;
  int32_t active, peak_active;          /* requests on the device now / at most */
  int64_t admitted_while_busy;          /* requests started while others ran */
  size_t used_bytes, peak_used_bytes, budget_bytes;
  int64_t pass_batches;                 /* shared cell-pass launches sequences */
  int64_t batched_passes;               /* cell passes run in them */
  int32_t max_batch;                    /* most passes in one of them */
  int32_t reserved;
  int64_t releases;                     /* idle slot workspaces given back to
                                           admit the head request */
} mak_server_info;

/* opt: solver options of every request (NULL = defaults); mem_budget_bytes
 * 0 = unlimited; 1 <= max_slots <= 64. */
mak_status mak_server_create(mak_server** out, int device, const mak_options* opt,
                             size_t mem_budget_bytes, int32_t max_slots);
/* Queue a solve (arguments as mak_solve; all DEVICE pointers stay owned by
 * the caller and must stay valid until the request is done).  The points
 * must be complete on the device when this is called (synchronise the
 * stream that wrote them).  MAK_ENOMEM if the estimate exceeds the budget. */
mak_status mak_server_submit(mak_server* s, const double* points, int64_t N, double L, double tol,
                             double* psi, double* centroids, double* displacements,
                             int64_t* req_id);
/* *done = 1 once the outputs are written; then returns the request's status
 * and fills info.  times (HOST double[3], may be NULL): submit, start, end
 * (seconds, steady clock). */
mak_status mak_server_poll(mak_server* s, int64_t req_id, int32_t* done, mak_solve_info* info,
                           double* times);
/* Block until the request is done; returns its status. */
mak_status mak_server_wait(mak_server* s, int64_t req_id, mak_solve_info* info, double* times);
/* Forget a finished request. */
mak_status mak_server_release(mak_server* s, int64_t req_id);
mak_status mak_server_stats(mak_server* s, mak_server_info* out);
const char* mak_server_last_error(const mak_server* s);
/* Finishes the queued and running requests, then frees the server. */
void mak_server_destroy(mak_server* s);

/* Device memory a solve of N sites needs at most (bytes), for admission. */
size_t mak_solve_memory_estimate(int64_t N, int32_t precision);

/* Device memory the library holds (HOST out pointers, either may be NULL):
 * *live = bytes allocated now by all contexts and servers of the process,
 * *peak = the most held at once since the last reset (updated at every
 * allocation).  reset_peak nonzero: afterwards the peak restarts from the
 * bytes held now.  Measured, not estimated: the sum of the library's own
 * device allocations (torch's or the caller's tensors are not included). */
void mak_device_bytes(size_t* live, size_t* peak, int32_t reset_peak);

#ifdef __cplusplus
}
#endif

#endif /* MAK_H */
