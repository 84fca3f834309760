// Laguerre cell pass: one wavefront per site clips a convex polytope by power
// bisectors (Eq. laguerrecell on the torus) and integrates it (Eq. SDK
// integrands: volume, first moment, face areas -> Hessian rows).
//
// Polytope representation (per wave):
//   planes    LDS  (n, b): u . n <= b inside, u = q - x_i seed-local; planes
//             0..5 are the box [-L/2, L/2]^3 of the site's own images.
//   vertices  one per "triangle" (a, b, c) of plane indices, the dual of the
//             polytope; a simple vertex is the intersection of three planes,
//             stored counter-clockwise seen from outside.  Each lane holds TPL
//             triangle slots in registers (slot = k * 64 + lane) with their
//             coordinates; LDS keeps a staging copy for compaction.
// Cutting by a new plane p:
//   - every lane tests its vertices; a ballot gives the removed set
//     (strictly outside by more than a tolerance eps: a plane that only
//     touches the polytope makes no face);
//   - the removed triangles mark their directed dual edges in an LDS bitmap;
//     a directed edge x->y of a removed triangle whose reverse y->x is not
//     marked lies on the boundary of the removed region and yields the new
//     vertex (x, y, p) (three-plane intersection);
//   - kept and new triangles are compacted through LDS by ballot prefix
//     counts.
// Candidates: the 27 grid cells around the site, then shells of 4x4x4-cell
// blocks.  Blocks, cells and sites are pruned lane-parallel with a bound on
// what a plane can cut from the ball (c, rho) around the polytope, using the
// per-block / per-cell maximum weight; a shell is only visited while its
// distance is below  R + sqrt(R^2 + 2 (psi_max - psi_i)),  R = |c| + rho
// (a bisector at distance t >= that from the site lies beyond the ball).
// Surviving sites of each batch of 64 are sorted by the distance of their
// plane from c (wave bitonic sort) and clipped in that order.
// Integrals: for every triangle T and each of its planes f, the next vertex
// around face f is the other triangle holding planes f and pred_T(f)
// (membership bitmasks in LDS); with v0 a fixed vertex of face f, the
// tetrahedra (site, v0, T, next) give volume and first moment, their face-f
// triangles (v0, T, next) the face areas.
#include <cfloat>

#include "engine.h"
#include "gridkey.h"
#include "profile.h"

// Products and sums in this file may fuse into FMAs (one rounding instead of
// two; fewer instructions).  The tie tolerances and the float32 ambiguity
// band bound the rounding of the unfused forms, so they hold.
#pragma clang fp contract(fast)

namespace mak {

namespace {

struct ClipArgs {
  const double4* pts;
  const int32_t* cell_start;
  const double* block_suffix;
  const double* block_g;     // tilted bounds: slope per block (3 doubles)
  const double* block_tmax;  // max_j psi_j - g . (x_j - block centre) per block
  const double* cell_tmax;   // the same per cell (with its block's slope)
  const double* gmax;
  // Optional warm start: the neighbours of each cell in an earlier pass (CSR
  // rows of J over the same sorted sites).  They are clipped first, so the
  // polytope is near its final shape before the grid walk; the walk then
  // meets them again and skips planes already in the table.
  const int64_t* warm_rp;
  const int32_t* warm_col;
  int32_t Gn, Gb;
  double L, h;
  const int32_t* work;
  int64_t nwork, per_xcd;
  double* vol;
  double* mom;
  int32_t* cflags;
  int32_t* nface;
  FaceRec* faces;
  int64_t* fbase;
  FaceRec* ovf;
  unsigned long long* ovf_used;     // faces placed in the overflow region
  unsigned long long* retry_count;  // cells appended to `retry`
  unsigned long long* cause;        // [0] capacity, [1] inconsistent cut
  int32_t* retry;
  int64_t ovf_cap;
  int32_t fslot;
  int32_t write_faces;
  double area_min;
  double eps_rel;  // float64 tie tolerance (relative to the grid cell side)
  double tol_rel;  // float32 ambiguity band (relative to |v||d| + |b|)
  unsigned long long* stats;  // optional work counters (see CLIP_STATS)
  // Line-search trials: a cell whose volume ends below doom_vol (or empty)
  // rejects the trial; it raises *doom and the workgroups that start after
  // it skip their cell (the host discards the pass).  doom == NULL: off.
  unsigned int* doom;
  unsigned long long* doom_cell;  // a cell that raised *doom (sorted index)
  double doom_vol;
  // Walk certificates (CertSet): 0 off, 1 record, 2 use.
  int32_t cert_mode;
  float cert_kappa;
  double cert_margin;
  uint32_t* cert_list;
  int32_t* cert_n;
  uint32_t* cert_vtx;
  float* cert_scale;
  const double* psi_ref;
  const unsigned long long* cert_dmax;
  // Combinatorics reuse: the records of the warm start's pass (read) and of
  // this pass (written); NULL: off.
  const uint16_t* topo_tri_in;
  const int32_t* topo_n_in;
  uint16_t* topo_tri_out;
  int32_t* topo_n_out;
};

// One launch carries the cell passes of up to kMaxJobs point sets (the
// concurrent requests of the server, or a single pass); job j owns the
// workgroups [blk_start[j], blk_start[j + 1]), 8 per_xcd of them.
struct ClipBatch {
  ClipArgs job[kMaxJobs];
  int64_t blk_start[kMaxJobs + 1];
  int32_t njobs;
};

// Work counters of the clip kernel (optional): sites scanned, planes tested
// against the vertices, vertex tests, cuts, new vertices, ball updates (in
// vertices), box tests, final vertices, reported faces, cells.
// The counting variant also sums shader-clock cycles per wave by phase:
// candidate search (grid walk, site loads, batch filter and sort), serial
// clipping, integrals and output.
// By search phase (w: the warm-start neighbours, n: the 27 nearest cells,
// r: the second ring of cells, b: the cells of the block shells): sites
// scanned, sites inside the ball bound, planes that removed vertices; box
// tests and how many passed (ring-2 cells, blocks, cells of passing blocks);
// the last block shell reached.  Slot 15 is left for the search flops the
// host forms from these counts.  Walk certificates: cells that recorded one,
// the sites they list, cells whose list overflowed; cells that tried one
// (weights within the margin) and cells whose walk it skipped.  Reused
// combinatorics: cells with a record of the warm start's pass, and cells
// that kept the polytope rebuilt from it.
enum { ST_CAND, ST_TEST, ST_VTEST, ST_CUT, ST_NEWV, ST_BALL, ST_BOX, ST_TRI, ST_FACES, ST_CELLS,
       ST_TSEARCH, ST_TCLIP, ST_TINT, ST_TPRE, ST_TCUT, ST_SEARCH_FLOPS,
       ST_SCAN_W, ST_SCAN_N, ST_SCAN_R, ST_SCAN_B, ST_INBALL_W, ST_INBALL_N, ST_INBALL_R, ST_INBALL_B,
       ST_CUT_W, ST_CUT_N, ST_CUT_R, ST_CUT_B, ST_BOXT_R, ST_BOXP_R, ST_BOXT_BLK, ST_BOXP_BLK,
       ST_BOXT_BC, ST_BOXP_BC, ST_SHELL, ST_CERT_REC, ST_CERT_LEN, ST_CERT_OVF, ST_CERT_TRY,
       ST_CERT_OK, ST_TOPO_TRY, ST_TOPO_OK, ST_N };

// Final vertices in float64 (the float32 path recomputes them from their
// three planes before integrating; the float64 path integrates its own).
template <typename R, int N>
struct FinalCoords {
  double x[N], y[N], z[N];
};
template <int N>
struct FinalCoords<double, N> {};

template <int TPL, typename R, bool CERT>
struct ClipLDS {
  // Live planes of a cell are few (faces plus recently cut-away planes): the
  // table holds 64 (128 for the large kernel) and is compacted when full;
  // vertices 64 * TPL.
  static constexpr int PCAP = TPL <= 2 ? 64 : 128;
  static constexpr int TCAP = 64 * TPL;
  double4 pl[PCAP];  // planes in float64 on both paths
  int32_t pj[PCAP];
  int32_t ps[PCAP];
  uint32_t stri[TCAP];
  R sx[TCAP], sy[TCAP], sz[TCAP];
  // the batch of sites being clipped (by lane) while clipping; the float64
  // final vertices and the plane -> vertex membership masks while integrating
  union {
    struct {
      FinalCoords<R, TCAP> fin;
      uint32_t mem[PCAP * TCAP / 32];
    } ints;
    struct {
      double4 cand[64];
      int32_t candj[64];
      int32_t cands[64];
      // the certificate being recorded (sites, image shifts): alive during
      // the search only, beside the batch (within the size of `fin` on the
      // float32 path, so the LDS per wave does not grow)
      uint32_t clist[CERT ? kCertCap : 1];
      int32_t clsh[CERT ? kCertCap : 1];
    } batch;
  } u;
  uint32_t bits[PCAP * PCAP / 32];   // directed dual edges of removed vertices
  uint32_t sbits[PCAP / 32];
  int32_t cstart[64];
  int32_t cpre[64];
  int32_t cshift[64];
};
static_assert(kCertCap <= 64, "a certificate is clipped as one list of 64 lanes");

// Certificate entry: site j and the image shift (each axis in -1..1); 0xffffffff
// when a shift lies outside that range (no certificate then).
__device__ __forceinline__ uint32_t cert_entry(int32_t j, int32_t shv) {
  const int sx = unpack_shift(shv, 0), sy = unpack_shift(shv, 1), sz = unpack_shift(shv, 2);
  if (sx < -1 || sx > 1 || sy < -1 || sy > 1 || sz < -1 || sz > 1) return 0xffffffffu;
  return (uint32_t(j) << 5) | uint32_t((sx + 1) * 9 + (sy + 1) * 3 + (sz + 1));
}
__device__ __forceinline__ int32_t cert_shift(uint32_t e) {
  const int c = int(e & 31u);
  return pack_shift(c / 9 - 1, (c / 3) % 3 - 1, c % 3 - 1);
}
// Order-preserving map of a double onto uint64 (for atomicMax).
__device__ __forceinline__ unsigned long long ordered_key(double v) {
  const unsigned long long b = __double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ordered_value(unsigned long long k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}

__device__ __forceinline__ uint32_t tri_pack(int a, int b, int c) {
  return uint32_t(a) | (uint32_t(b) << 8) | (uint32_t(c) << 16);
}
__device__ __forceinline__ int tri_a(uint32_t t) { return int(t & 255u); }
__device__ __forceinline__ int tri_b(uint32_t t) { return int((t >> 8) & 255u); }
__device__ __forceinline__ int tri_c(uint32_t t) { return int((t >> 16) & 255u); }

// Key of lane ^ J: quad permutes for 1 and 2 (DPP, no LDS round trip),
// swizzles (xor mode within 32 lanes) for 4, 8 and 16, a permute for 32.
template <int J>
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t v) {
  if constexpr (J == 1) return uint32_t(dpp_i<kDppXor1>(int(v)));
  else if constexpr (J == 2) return uint32_t(dpp_i<kDppXor2>(int(v)));
  else if constexpr (J < 32) return uint32_t(__builtin_amdgcn_ds_swizzle(int(v), 0x1F | (J << 10)));
  else return uint32_t(__shfl_xor(int(v), J));
}
template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_stage(uint32_t key, int lane) {
  const uint32_t other = lane_xor_u32<J>(key);
  const bool take_min = ((lane & J) == 0) == ((lane & K) == 0);
  return take_min ? min(key, other) : max(key, other);
}
template <int K>
__device__ __forceinline__ uint32_t bitonic_merge(uint32_t key, int lane) {
  if constexpr (K >= 64) key = bitonic_stage<K, 32>(key, lane);
  if constexpr (K >= 32) key = bitonic_stage<K, 16>(key, lane);
  if constexpr (K >= 16) key = bitonic_stage<K, 8>(key, lane);
  if constexpr (K >= 8) key = bitonic_stage<K, 4>(key, lane);
  if constexpr (K >= 4) key = bitonic_stage<K, 2>(key, lane);
  return bitonic_stage<K, 1>(key, lane);
}
// Ascending bitonic sort of one 32-bit key per lane across the wave.
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t key) {
  const int lane = lane_id();
  key = bitonic_merge<2>(key, lane);
  key = bitonic_merge<4>(key, lane);
  key = bitonic_merge<8>(key, lane);
  key = bitonic_merge<16>(key, lane);
  key = bitonic_merge<32>(key, lane);
  return bitonic_merge<64>(key, lane);
}

// Smallest key of the wave (the DPP reduction of the wave sums).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, uint32_t(dpp_i<kDppXor1>(int(v))));
  v = min(v, uint32_t(dpp_i<kDppXor2>(int(v))));
  v = min(v, uint32_t(dpp_i<kDppHalfMirror>(int(v))));
  v = min(v, uint32_t(dpp_i<kDppMirror>(int(v))));
  v = min(v, uint32_t(bcast_i<kDppBcast15, 0xA>(int(v))));
  v = min(v, uint32_t(bcast_i<kDppBcast31, 0xC>(int(v))));
  return readlane_u(v, 63);
}

// Offset of the t-th block of the Chebyshev shell of radius r (r >= 1).
__host__ __device__ constexpr void shell_offset_calc(int r, int t, int& ox, int& oy, int& oz) {
  if (r == 0) {
    ox = oy = oz = 0;
    return;
  }
  const int S = 2 * r + 1, I = 2 * r - 1;
  if (t < 2 * S * S) {
    const int side = t / (S * S), rem = t % (S * S);
    ox = side ? r : -r;
    oy = rem / S - r;
    oz = rem % S - r;
    return;
  }
  t -= 2 * S * S;
  if (t < 2 * S * I) {
    const int side = t / (S * I), rem = t % (S * I);
    oy = side ? r : -r;
    ox = rem / S - (r - 1);
    oz = rem % S - r;
    return;
  }
  t -= 2 * S * I;
  const int side = t / (I * I), rem = t % (I * I);
  oz = side ? r : -r;
  ox = rem / I - (r - 1);
  oy = rem % I - (r - 1);
}

// The offsets of shells 1..SHELL_MAX in one table (4 bits per axis, biased by
// 8), built at compile time by the function above: the walk reads an entry
// instead of dividing by runtime shell sizes.
constexpr int kShellEntries = (2 * SHELL_MAX + 1) * (2 * SHELL_MAX + 1) * (2 * SHELL_MAX + 1) - 1;
struct ShellTable {
  uint16_t v[kShellEntries];
};
constexpr ShellTable make_shell_table() {
  ShellTable tb{};
  int n = 0;
  for (int r = 1; r <= SHELL_MAX; ++r) {
    const int S = 2 * r + 1, I = 2 * r - 1;
    for (int t = 0; t < S * S * S - I * I * I; ++t) {
      int ox = 0, oy = 0, oz = 0;
      shell_offset_calc(r, t, ox, oy, oz);
      tb.v[n++] = uint16_t((ox + 8) | ((oy + 8) << 4) | ((oz + 8) << 8));
    }
  }
  return tb;
}
static_assert(SHELL_MAX <= 7, "shell offsets are packed in 4 bits");
static_assert(BLOCK_SIDE == 4, "cell -> block uses shifts by 2");
__constant__ ShellTable kShell = make_shell_table();

__device__ __forceinline__ void shell_offset(int r, int t, int& ox, int& oy, int& oz) {
  if (r >= 1 && r <= SHELL_MAX) {
    const int I = 2 * r - 1;
    const uint32_t v = kShell.v[I * I * I - 1 + t];
    ox = int(v & 15u) - 8;
    oy = int((v >> 4) & 15u) - 8;
    oz = int((v >> 8) & 15u) - 8;
    return;
  }
  if (r == 0) {
    ox = oy = oz = 0;
    return;
  }
  shell_offset_calc(r, t, ox, oy, oz);
}

// floor(a / n) for n > 0, without a division in the common case of a within
// one period of [0, n).
__device__ __forceinline__ int period_div(int a, int n) {
  if (a >= 0 && a < n) return 0;
  if (a < 0 && a >= -n) return -1;
  if (a >= n && a < 2 * n) return 1;
  return floor_div(a, n);
}

// Shader clock for the counting variant's phase timers: waits for the
// wave's outstanding memory operations first, so their latency is charged to
// the phase that issued them, and keeps the compiler from moving memory
// operations across the stamp.
__device__ __forceinline__ uint64_t clock_stamp() {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  const uint64_t t = __builtin_amdgcn_s_memtime();
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  return t;
}

// The 27 neighbour cells (code = (ox+1)*9 + (oy+1)*3 + (oz+1)) by distance class.
__constant__ int kNearOrder[27] = {13, 4, 22, 10, 16, 12, 14, 1, 7, 19, 25, 3, 5, 21, 23,
                                   9, 11, 15, 17, 0, 2, 6, 8, 18, 20, 24, 26};

// Occupancy: the kernel is bound by instruction issue and the latency of its
// dependent LDS / memory steps, so more waves per SIMD pay even with some
// registers spilled: 5 waves per SIMD for the float32 first stage (one
// vertex per lane: 96 VGPRs, 7.5 KB of LDS per wave, 20 waves per CU), 4
// for the float64 kernels (128 VGPRs; 10 KB of LDS outside the certificate
// instance), 2 for the large-capacity one.
// CERT: the variant that records or uses walk certificates (the extra live
// state would spill registers in the passes that use neither).
template <int TPL, typename R, bool STATS, bool CERT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TPL == 1 ? 5 : (TPL == 2 ? 4 : 2)))) void k_clip(
    ClipBatch B) {
  constexpr bool kF64 = sizeof(R) == 8;
  constexpr int PCAP = ClipLDS<TPL, R, CERT>::PCAP;
  constexpr int TCAP = ClipLDS<TPL, R, CERT>::TCAP;
  constexpr int TW = TCAP / 32;   // words of one membership mask
  constexpr int PW = PCAP / 32;   // words of one bitmap row
  constexpr int NPC = (PCAP + 63) / 64;  // plane chunks of 64 lanes
  __shared__ ClipLDS<TPL, R, CERT> S;

  const int lane = threadIdx.x;
  // linear workgroup id (2-D grid above 2^16 workgroups; gridDim.x and every
  // job's first workgroup are multiples of 8, so blk & 7 is still the XCD
  // the workgroup runs on)
  const int64_t gblk = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
  if (gblk >= B.blk_start[B.njobs]) return;
  int jb = 0;
  while (jb + 1 < B.njobs && gblk >= B.blk_start[jb + 1]) ++jb;
  const ClipArgs& A = B.job[jb];
  const int64_t blk = gblk - B.blk_start[jb];
  if ((blk >> 3) >= A.per_xcd) return;
  const int64_t item = (blk & 7) * A.per_xcd + (blk >> 3);
  if (item >= A.nwork) return;
  if (A.doom && __hip_atomic_load(A.doom, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int32_t p = A.work ? A.work[item] : int32_t(item);

  const double4 me = A.pts[p];
  const double xi = me.x, yi = me.y, zi = me.z, wi = me.w;
  const double L = A.L, h = A.h;
  const int Gn = A.Gn, Gb = A.Gb;
  const int cx = cell_coord(xi, h, Gn), cy = cell_coord(yi, h, Gn), cz = cell_coord(zi, h, Gn);
  const double gmax = *A.gmax;
  const double mtol = 1e-12 * L * L;

  // Walk certificates (they need the warm start of an earlier pass).
  const int cmode = CERT && A.warm_rp ? A.cert_mode : 0;
  bool use_cert = false;
  if (cmode == 2 && A.cert_n[p] >= 0)  // (the same on every lane: kept in scalar registers)
    use_cert = uniform_i(ordered_value(*A.cert_dmax) - (wi - A.psi_ref[p]) <= A.cert_margin ? 1 : 0) != 0;
  // recording: every pruning test allows the weight margin and bounds the
  // polytope widened by kappa
  const double wslack = cmode == 1 ? A.cert_margin : 0.0;
  const float kap = cmode == 1 ? A.cert_kappa : 0.f;
  int ccount = 0;  // recording: sites listed so far

  int32_t flags = 0;
  bool dead = false;
  // work counters (compiled in only for the counting variant)
  uint32_t c_cand = 0, c_test = 0, c_vt = 0, c_cut = 0, c_newv = 0, c_ball = 0, c_box = 0, c_pre = 0;
  uint32_t c_ph[ST_N - ST_SCAN_W] = {};  // the per-phase counters, from ST_SCAN_W on
  int cur_ph = 0;                        // phase of the list being scanned
#define CPH(idx, v) CNT(c_ph[(idx) - ST_SCAN_W] += uint32_t(v))
  uint64_t t_begin = 0, t_clip = 0, t_search_end = 0, t_pre = 0, t_cut = 0;
  if (STATS) t_begin = clock_stamp();
#define CNT(stmt)  \
  do {             \
    if (STATS) {   \
      stmt;        \
    }              \
  } while (0)

  // ---------------------------------------------------------------- box
  if (lane < 6) {
    const int ax = lane >> 1;
    const double sg = (lane & 1) ? -1.0 : 1.0;
    S.pl[lane] = make_double4(ax == 0 ? sg * L : 0.0, ax == 1 ? sg * L : 0.0,
                              ax == 2 ? sg * L : 0.0, 0.5 * L * L);
    S.pj[lane] = -1;
    const int is = (lane & 1) ? -1 : 1;
    S.ps[lane] = pack_shift(ax == 0 ? is : 0, ax == 1 ? is : 0, ax == 2 ? is : 0);
  }
  uint32_t tri[TPL];
  R vx[TPL], vy[TPL], vz[TPL];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    tri[k] = 0;
    vx[k] = vy[k] = vz[k] = 0.0;
  }
  if (lane < 8) {
    const int px = lane & 1, py = 2 + ((lane >> 1) & 1), pz = 4 + ((lane >> 2) & 1);
    const int sx = (lane & 1) ? -1 : 1, sy = ((lane >> 1) & 1) ? -1 : 1, sz = ((lane >> 2) & 1) ? -1 : 1;
    tri[0] = (sx * sy * sz > 0) ? tri_pack(px, py, pz) : tri_pack(px, pz, py);
    vx[0] = R(sx * 0.5 * L);
    vy[0] = R(sy * 0.5 * L);
    vz[0] = R(sz * 0.5 * L);
    S.stri[lane] = tri[0];
    S.sx[lane] = vx[0];
    S.sy[lane] = vy[0];
    S.sz[lane] = vz[0];
  }
  int nT = 8, nP = 6;
  float bcx = 0.f, bcy = 0.f, bcz = 0.f;
  float brho = float(0.8660254037844386 * L) * 1.0001f;
  if (!A.warm_rp) {
    // Without a warm start the first candidates are ordered by the distance
    // of their planes from the ball's centre: put it at -g, g the slope of
    // the weights over the site's block (a linear trend g . x in the weights
    // moves every cell by -g), so the planes nearest the cell are clipped
    // first and fewer faces are cut only to be cut away again.  The radius
    // grows by |g| so the ball still holds the box.
    const int64_t bk0 = block_key(cx >> 2, cy >> 2, cz >> 2, Gb);
    const float gx = float(A.block_g[3 * bk0]), gy = float(A.block_g[3 * bk0 + 1]),
                gz = float(A.block_g[3 * bk0 + 2]);
    const float gn = __builtin_amdgcn_sqrtf(gx * gx + gy * gy + gz * gz);
    if (gn < 0.5f * float(L)) {
      bcx = -gx;
      bcy = -gy;
      bcz = -gz;
      brho += gn * 1.0001f;
    }
  }
  bool ball_dirty = false;
  float rvert = float(0.8660254037844386 * L) * 1.0001f;  // max vertex distance from x_i
  // axis-aligned bounding box of the vertices (seed-local, widened by far
  // more than the float rounding): with the ball it bounds what a plane can
  // cut, h_P(d) <= sum_a max(d_a hi_a, d_a lo_a)
  float blx = -0.5001f * float(L), bly = blx, blz = blx;
  float bhx = 0.5001f * float(L), bhy = bhx, bhz = bhx;
  // tie tolerance of the vertex-side test: eps = eps_scale |d| (float64); the
  // float32 path uses tol = tol_rel (rvert |d| + |b|) and treats any vertex
  // with |u.d - b| <= tol as ambiguous (the cell is then re-run in float64)
  const double eps_scale = A.eps_rel * h;
  const R tol_rel = R(A.tol_rel);
  for (int w = lane; w < PCAP * PW; w += 64) S.bits[w] = 0u;
  if (lane < PW) S.sbits[lane] = 0u;
  __syncthreads();

  auto setbit = [&](int a, int b) {
    const int idx = a * PCAP + b;
    atomicOr(&S.bits[idx >> 5], 1u << (idx & 31));
  };
  auto getbit = [&](int a, int b) -> bool {
    const int idx = a * PCAP + b;
    return (S.bits[idx >> 5] >> (idx & 31)) & 1u;
  };
  auto clearword = [&](int a, int b) {
    const int idx = a * PCAP + b;
    S.bits[idx >> 5] = 0u;
  };

  auto update_ball = [&]() {
    // the vertices' extent and largest distance from the site first; the
    // ball is centred on the extent's centre (no sums over the vertices)
    float lx = FLT_MAX, ly = FLT_MAX, lz = FLT_MAX, hx = -FLT_MAX, hy = -FLT_MAX, hz = -FLT_MAX;
    float v2 = 0.f;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (k * 64 + lane < nT) {
        const float x = float(vx[k]), y = float(vy[k]), z = float(vz[k]);
        lx = fminf(lx, x);
        ly = fminf(ly, y);
        lz = fminf(lz, z);
        hx = fmaxf(hx, x);
        hy = fmaxf(hy, y);
        hz = fmaxf(hz, z);
        v2 = fmaxf(v2, float(double(vx[k]) * vx[k] + double(vy[k]) * vy[k] + double(vz[k]) * vz[k]));
      }
    }
    // wave-uniform results are moved to scalar registers
    lx = -uniform_f(wave_max_f(-lx));
    ly = -uniform_f(wave_max_f(-ly));
    lz = -uniform_f(wave_max_f(-lz));
    hx = uniform_f(wave_max_f(hx));
    hy = uniform_f(wave_max_f(hy));
    hz = uniform_f(wave_max_f(hz));
    v2 = uniform_f(wave_max_f(v2));
    const float sx = uniform_f(0.5f * (lx + hx)), sy = uniform_f(0.5f * (ly + hy)), sz = uniform_f(0.5f * (lz + hz));
    float r2 = 0.f;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (k * 64 + lane < nT) {
        const float ex = float(vx[k]) - sx, ey = float(vy[k]) - sy, ez = float(vz[k]) - sz;
        r2 = fmaxf(r2, ex * ex + ey * ey + ez * ez);
      }
    }
    r2 = uniform_f(wave_max_f(r2));
    bcx = sx;
    bcy = sy;
    bcz = sz;
    // (hardware roots: their error, about an ulp, is far inside the margins)
    const float cn = __builtin_amdgcn_sqrtf(sx * sx + sy * sy + sz * sz);
    brho = __builtin_amdgcn_sqrtf(r2) * 1.0001f + 1e-6f * (cn + float(h));
    rvert = __builtin_amdgcn_sqrtf(v2) * 1.0001f + 1e-6f * float(h);
    const float slack = 1e-5f * (rvert + float(h));
    blx = lx - slack;
    bly = ly - slack;
    blz = lz - slack;
    bhx = hx + slack;
    bhy = hy + slack;
    bhz = hz + slack;
    if (kap > 0.f) {
      // recording: the bounds cover the polytope widened by kappa
      brho += kap;
      rvert += kap;
      blx -= kap;
      bly -= kap;
      blz -= kap;
      bhx += kap;
      bhy += kap;
      bhz += kap;
    }
  };

  // Drop the planes no vertex refers to any more (cut away by later planes)
  // and renumber the rest; the table fills up when many sites cut the cell
  // in turn (dense clumps).
  auto compact_planes = [&]() {
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (k * 64 + lane < nT) {
        const int a = tri_a(tri[k]), b = tri_b(tri[k]), c = tri_c(tri[k]);
        atomicOr(&S.sbits[a >> 5], 1u << (a & 31));
        atomicOr(&S.sbits[b >> 5], 1u << (b & 31));
        atomicOr(&S.sbits[c >> 5], 1u << (c & 31));
      }
    }
    __syncthreads();
    double4 cpl[NPC];
    int32_t cj[NPC], cs[NPC], cnew[NPC];
    bool calive[NPC];
    int alive_total = 0;
#pragma unroll
    for (int w = 0; w < PW; ++w) alive_total += __popc(S.sbits[w]);
#pragma unroll
    for (int c = 0; c < NPC; ++c) {
      const int f = c * 64 + lane;
      calive[c] = f < nP && ((S.sbits[f >> 5] >> (f & 31)) & 1u);
      int below = 0;
      if (f < nP) {
        below = __popc(S.sbits[f >> 5] & ((1u << (f & 31)) - 1u));
        for (int w = 0; w < (f >> 5); ++w) below += __popc(S.sbits[w]);
      }
      cnew[c] = below;
      if (calive[c]) {
        cpl[c] = S.pl[f];
        cj[c] = S.pj[f];
        cs[c] = S.ps[f];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NPC; ++c) {
      if (calive[c]) {
        const int f = c * 64 + lane;
        S.pl[cnew[c]] = cpl[c];
        S.pj[cnew[c]] = cj[c];
        S.ps[cnew[c]] = cs[c];
        S.bits[f] = uint32_t(cnew[c]);  // old -> new index (bitmap is idle here)
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (k * 64 + lane < nT) {
        const uint32_t t = tri[k];
        tri[k] = tri_pack(int(S.bits[tri_a(t)]), int(S.bits[tri_b(t)]), int(S.bits[tri_c(t)]));
        S.stri[k * 64 + lane] = tri[k];
      }
    }
    __syncthreads();
    for (int w = lane; w < PCAP; w += 64) S.bits[w] = 0u;
    if (lane < PW) S.sbits[lane] = 0u;
    nP = __builtin_amdgcn_readfirstlane(alive_total);
    __syncthreads();
  };

  // Upper bound of max_v v . d over the vertices from their bounding box.
  auto aabb_support = [&](double dx, double dy, double dz) -> double {
    return fmax(dx * double(blx), dx * double(bhx)) + fmax(dy * double(bly), dy * double(bhy)) +
           fmax(dz * double(blz), dz * double(bhz));
  };

  // Clip by u . d <= bb (plane tag jj / ss).
  auto clip_one = [&](double ddx, double ddy, double ddz, double dbb, double dnd, int32_t jj,
                      int32_t ss) {
    if (cmode == 1) {
      // (outside recording, the batch's own ball and bounding-box tests used
      // the same ball and box, which stay fixed until the next batch, with
      // the same threshold and a smaller |d|: there they always pass)
      const double cd = double(bcx) * ddx + double(bcy) * ddy + double(bcz) * ddz;
      if (cd + double(brho) * dnd <= dbb - mtol) return;  // cannot reach the ball
      if (aabb_support(ddx, ddy, ddz) <= dbb - mtol) return;  // nor the bounding box
    }
    if (A.warm_rp && (cur_ph != 0 || use_cert)) {
      // with a warm start the walk meets the warm planes again: a plane
      // already in the table is not applied twice (the warm list itself
      // holds distinct sites and meets only the box planes; a certificate
      // list may follow the reused combinatorics' planes)
      bool same = false;
#pragma unroll
      for (int c = 0; c < NPC; ++c) {
        const int f = c * 64 + lane;
        same = same || (f < nP && S.pj[f] == jj && S.ps[f] == ss);
      }
      if (ballot(same)) return;
    }
    const R dx = R(ddx), dy = R(ddy), dz = R(ddz), bb = R(dbb);
    // float64: out iff s > eps.  float32: out iff s > tol; |s| <= tol is
    // ambiguous at this precision and sends the cell to the float64 kernel.
    const R eps = kF64 ? R(eps_scale * dnd) : tol_rel * (R(rvert) * R(dnd) + fabs(bb));
    CNT(c_test += 1);
    CNT(c_vt += uint32_t(nT));
    uint64_t om[TPL];
    int nout = 0;
    bool amb = false;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      bool out = false;
      if (k == 0 || nT > k * 64) {
        const bool valid = k * 64 + lane < nT;
        const R sv = vx[k] * dx + vy[k] * dy + vz[k] * dz - bb;
        out = valid && sv > eps;
        if (!kF64) amb = amb || (valid && sv > -eps && sv <= eps);
      }
      om[k] = ballot(out);
      nout += __popcll(om[k]);
    }
    if (!kF64 && ballot(amb)) {
      flags |= CF_NEARDEG;
      dead = true;
      return;
    }
    if (nout == 0) return;
    uint64_t tk0 = 0;
    if (STATS) tk0 = clock_stamp();
    if (nout == nT) {
      flags |= CF_EMPTY;
      dead = true;
      return;
    }
    if (nP >= PCAP) {
      compact_planes();
      if (nP >= PCAP) {
        flags |= CF_CAPACITY;
        dead = true;
        return;
      }
    }
    const int pn = nP;
    if (lane == 0) {
      S.pl[pn] = make_double4(ddx, ddy, ddz, dbb);
      S.pj[pn] = jj;
      S.ps[pn] = ss;
    }
    // 1. mark the directed dual edges of the removed triangles
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if ((om[k] >> lane) & 1ull) {
        const int a = tri_a(tri[k]), b = tri_b(tri[k]), c = tri_c(tri[k]);
        setbit(a, b);
        setbit(b, c);
        setbit(c, a);
      }
    }
    __syncthreads();
    // 2. boundary edges: reverse edge not removed
    int bm[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      bm[k] = 0;
      if ((om[k] >> lane) & 1ull) {
        const int a = tri_a(tri[k]), b = tri_b(tri[k]), c = tri_c(tri[k]);
        if (!getbit(b, a)) bm[k] |= 1;
        if (!getbit(c, b)) bm[k] |= 2;
        if (!getbit(a, c)) bm[k] |= 4;
      }
    }
    __syncthreads();
    // 3. clear the marks; each plane may start at most one boundary edge:
    // the starting planes, or-ed into a set, are as many as the edges
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if ((om[k] >> lane) & 1ull) {
        const int a = tri_a(tri[k]), b = tri_b(tri[k]), c = tri_c(tri[k]);
        clearword(a, b);
        clearword(b, c);
        clearword(c, a);
        const int st[3] = {a, b, c};
#pragma unroll
        for (int e = 0; e < 3; ++e)
          if (bm[k] & (1 << e)) atomicOr(&S.sbits[st[e] >> 5], 1u << (st[e] & 31));
      }
    }
    __syncthreads();
    int starts = 0;
#pragma unroll
    for (int w = 0; w < PW; ++w) starts += __popc(uint32_t(__builtin_amdgcn_readfirstlane(int(S.sbits[w]))));
    if (lane < PW) S.sbits[lane] = 0u;  // (after the reads: one wave, in order)
    const int nkept = nT - nout;
    int mynew = 0;
#pragma unroll
    for (int k = 0; k < TPL; ++k) mynew += __popc(bm[k]);
    const int nedge = wave_sum_i(mynew);
    if (starts != nedge) {
      flags |= CF_NONMANIFOLD;
      dead = true;
      return;
    }
    const int nTn = nkept + nedge;
    if (nTn > TCAP) {
      flags |= CF_CAPACITY;
      dead = true;
      return;
    }
    // 4. compaction: kept triangles first (slot order), then the new ones
    const double4 Pn = make_double4(ddx, ddy, ddz, dbb);
    int krun = 0, nrun = 0;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (k > 0 && nT <= k * 64) break;  // no slots in this group (uniform)
      const int slot = k * 64 + lane;
      const bool kept = slot < nT && !((om[k] >> lane) & 1ull);
      const uint64_t km = ballot(kept);
      if (kept) {
        const int dst = krun + lanes_below(km);
        S.stri[dst] = tri[k];
        S.sx[dst] = vx[k];
        S.sy[dst] = vy[k];
        S.sz[dst] = vz[k];
      }
      krun += __popcll(km);
      const int nb = __popc(bm[k]);
      const uint64_t b0 = ballot(nb & 1), b1 = ballot(nb & 2);
      int pos = nkept + nrun + lanes_below(b0) + 2 * lanes_below(b1);
      nrun += __popcll(b0) + 2 * __popcll(b1);
      if (bm[k]) {
        // the new triangles (x, y, p) of this lane's boundary edges; their
        // vertices are computed below, one per lane
        const int st[3] = {tri_a(tri[k]), tri_b(tri[k]), tri_c(tri[k])};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          if (bm[k] & (1 << e)) {
            S.stri[pos] = tri_pack(st[e], st[(e + 1) % 3], pn);
            ++pos;
          }
        }
      }
    }
    __syncthreads();
    // new vertices: intersection of planes x, y, pn (Cramer's rule, float64 on
    // both paths; the float32 path stores the vertex rounded)
    for (int t = nkept + lane; t < nTn; t += 64) {
      const uint32_t tr = S.stri[t];
      const double4 P1 = S.pl[tri_a(tr)], P2 = S.pl[tri_b(tr)];
      const double c23x = P2.y * Pn.z - P2.z * Pn.y, c23y = P2.z * Pn.x - P2.x * Pn.z,
                   c23z = P2.x * Pn.y - P2.y * Pn.x;
      const double c31x = Pn.y * P1.z - Pn.z * P1.y, c31y = Pn.z * P1.x - Pn.x * P1.z,
                   c31z = Pn.x * P1.y - Pn.y * P1.x;
      const double c12x = P1.y * P2.z - P1.z * P2.y, c12y = P1.z * P2.x - P1.x * P2.z,
                   c12z = P1.x * P2.y - P1.y * P2.x;
      const double det = P1.x * c23x + P1.y * c23y + P1.z * c23z;
      const double inv = recip_d(det);
      S.sx[t] = (P1.w * c23x + P2.w * c31x + Pn.w * c12x) * inv;
      S.sy[t] = (P1.w * c23y + P2.w * c31y + Pn.w * c12y) * inv;
      S.sz[t] = (P1.w * c23z + P2.w * c31z + Pn.w * c12z) * inv;
    }
    __syncthreads();
    CNT(c_cut += 1);
    CPH(ST_CUT_W + cur_ph, 1);
    CNT(c_newv += uint32_t(nTn - nkept));
    CNT(c_ball += uint32_t(nTn));
    nT = nTn;
    nP = pn + 1;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const int slot = k * 64 + lane;
      if (k > 0 && nT <= k * 64) {  // no slots in this group (uniform)
        tri[k] = 0;
        continue;
      }
      if (slot < nT) {
        tri[k] = S.stri[slot];
        vx[k] = S.sx[slot];
        vy[k] = S.sy[slot];
        vz[k] = S.sz[slot];
      } else {
        tri[k] = 0;
      }
    }
    ball_dirty = true;  // the ball is refreshed lazily (a stale ball is still a bound)
    if (STATS) t_cut += clock_stamp() - tk0;
  };

  auto refresh_ball = [&]() {
    if (ball_dirty) {
      update_ball();
      ball_dirty = false;
    }
  };

  // Could a site of the seed-local box [lo, hi] cut the ball (c, rho)?  It
  // needs c.d + rho|d| > |d|^2/2 + psi_i - psi_j.  The box lies in block
  // (ubx, uby, ubz) (unwrapped; key bkey) whose sites obey the tilted bound
  // psi_j <= tmax + g . (d - D), D the block centre (seed-local): then a cut
  // needs |d|^2/2 - rho|d| - d.(c + g) < tmax - g.D - psi_i, and the left
  // side is bounded below over the box.
  const double bh = BLOCK_SIDE * h;
  auto box_may_cut = [&](double lx, double ly, double lz, double hx, double hy, double hz,
                         int64_t bkey, int ubx, int uby, int ubz, double tmax) -> bool {
    const double gx = A.block_g[3 * bkey], gy = A.block_g[3 * bkey + 1], gz = A.block_g[3 * bkey + 2];
    const double Dx = (ubx + 0.5) * bh - xi, Dy = (uby + 0.5) * bh - yi, Dz = (ubz + 0.5) * bh - zi;
    const double wmax = tmax - (gx * Dx + gy * Dy + gz * Dz);
    const double mx = lx > 0 ? lx : (hx < 0 ? -hx : 0.0);
    const double my = ly > 0 ? ly : (hy < 0 ? -hy : 0.0);
    const double mz = lz > 0 ? lz : (hz < 0 ? -hz : 0.0);
    // a lower bound of the distance m to the box (a float root, shrunk by
    // far more than its error): f(m) = m^2/2 - r m is increasing for m >= r,
    // so the bound keeps the test conservative
    const double m = double(__builtin_amdgcn_sqrtf(float(mx * mx + my * my + mz * mz))) * (1.0 - 1e-6);
    const double r = double(brho);
    const double f = m >= r ? 0.5 * m * m - r * m : -0.5 * r * r;
    const double ex = double(bcx) + gx, ey = double(bcy) + gy, ez = double(bcz) + gz;
    const double cmax = fmax(ex * lx, ex * hx) + fmax(ey * ly, ey * hy) + fmax(ez * lz, ez * hz);
    const double W = wmax - wi + mtol + wslack;
    if (!(f - cmax < W)) return false;
    // The same with the bounding box of the vertices: with h_P(d) <=
    // sum_a max(d_a hi_a, d_a lo_a) the left side is separable per axis, and
    // on each axis it is the smaller of two parabolas t^2/2 - (g_a + hi_a) t
    // and t^2/2 - (g_a + lo_a) t, whose minima over [l_a, u_a] are at their
    // clamped vertices.
    auto axis_min = [](double l, double u, double g, double lo, double hi) {
      const double a1 = g + hi, a2 = g + lo;
      const double t1 = fmin(fmax(a1, l), u), t2 = fmin(fmax(a2, l), u);
      return fmin(0.5 * t1 * t1 - a1 * t1, 0.5 * t2 * t2 - a2 * t2);
    };
    return axis_min(lx, hx, gx, double(blx), double(bhx)) + axis_min(ly, hy, gy, double(bly), double(bhy)) +
               axis_min(lz, hz, gz, double(blz), double(bhz)) <
           W;
  };

  // Scan the sites of a list of cells (one cell per lane where `act`).
  auto process_list = [&](bool act, int32_t start, int32_t cnt, int32_t sh, int ph) {
    cur_ph = ph;
    const bool has = act && cnt > 0;
    const uint64_t am = ballot(has);
    const int ncl = __popcll(am);
    if (ncl == 0) return;
    const int c_ = has ? cnt : 0;
    const int incl = wave_incl_scan_i(c_);
    const int total = readlane_i(incl, 63);
    if (has) {
      const int idx = lanes_below(am);
      S.cstart[idx] = start;
      S.cpre[idx] = incl - c_;
      S.cshift[idx] = sh;
    }
    __syncthreads();
    for (int base = 0; base < total && !dead; base += 64) {
      const int t = base + lane;
      CNT(c_cand += uint32_t(min(64, total - base)));
      CPH(ST_SCAN_W + ph, min(64, total - base));
      refresh_ball();
      int lo = 0, hi = ncl - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.cpre[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const int q = S.cstart[lo] + (t - S.cpre[lo]);
      const int32_t shv = S.cshift[lo];
      double dx = 0, dy = 0, dz = 0, bb = 0, dn = 0;
      bool may = false, coinc = false;
      uint32_t key = 0xffffffffu;
      if (t < total && q != p) {
        const double4 P = A.pts[q];
        dx = P.x + unpack_shift(shv, 0) * L - xi;
        dy = P.y + unpack_shift(shv, 1) * L - yi;
        dz = P.z + unpack_shift(shv, 2) * L - zi;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 == 0.0) {
          coinc = true;
        } else {
          bb = 0.5 * d2 + wi - P.w;
          // |d| from a float root, enlarged by far more than its error: it
          // only scales the ball test (larger = more conservative), the tie
          // tolerances and the sort key
          dn = double(__builtin_amdgcn_sqrtf(float(d2))) * (1.0 + 1e-6);
          const double cd = double(bcx) * dx + double(bcy) * dy + double(bcz) * dz;
          const double bt = bb - mtol - wslack;
          may = cd + double(brho) * dn > bt && aabb_support(dx, dy, dz) > bt;
          if (may) key = (float_key(float(bb - cd) * __builtin_amdgcn_rcpf(float(dn))) & ~63u) | uint32_t(lane);
        }
      }
      if (ballot(coinc)) flags |= CF_COINCIDENT;
      int ns = __popcll(ballot(may));
      CPH(ST_INBALL_W + ph, ns);
      if (ns == 0) continue;
      // the plane in the working precision (seed-local, so float32 keeps the
      // relative precision of |d|)
      const R rx = R(dx), ry = R(dy), rz = R(dz), rbb = R(bb);
      if (cmode == 1 && ph >= 1) {
        // recording: the exact support of the current vertices (a superset of
        // the final polytope) decides both the cut and the listing: listed is
        // every site whose plane, its weight raised by the margin, reaches
        // the polytope widened by kappa
        const R eps = kF64 ? R(eps_scale * dn) : -tol_rel * (R(rvert) * R(dn) + fabs(rbb));
        R mx = R(-FLT_MAX);
#pragma unroll 1
        for (int v = 0; v < nT; ++v) mx = fmax(mx, S.sx[v] * rx + S.sy[v] * ry + S.sz[v] * rz);
        CNT(c_pre += uint32_t(nT));
        const bool lst = may && mx + R(kap) * R(dn) > rbb - R(wslack) - fabs(eps);
        const uint64_t lm = ballot(lst);
        const int r = ccount + lanes_below(lm);
        if (lst && r < kCertCap) {
          S.u.batch.clist[r] = uint32_t(q);
          S.u.batch.clsh[r] = shv;
        }
        ccount += __popcll(lm);
        may = may && mx - rbb > eps;
        if (!may) key = 0xffffffffu;
        ns = __popcll(ballot(may));
        if (ns == 0) continue;
      } else if (ns > 2) {
        // Exact filter, one candidate per lane against every current vertex
        // (LDS broadcast reads).  A plane that removes no vertex now cannot
        // remove one from any later, smaller polytope.  (float32: planes with
        // a vertex within the ambiguity band are kept for the serial test.)
        const R eps = kF64 ? R(eps_scale * dn) : -tol_rel * (R(rvert) * R(dn) + fabs(rbb));
        bool cut = false;
        uint64_t tp0 = 0;
        if (STATS) tp0 = clock_stamp();
#pragma unroll 1
        for (int v = 0; v < nT; ++v) {
          const R ux = S.sx[v], uy = S.sy[v], uz = S.sz[v];
          cut |= ux * rx + uy * ry + uz * rz - rbb > eps;
        }
        CNT(c_pre += uint32_t(nT));
        if (STATS) t_pre += clock_stamp() - tp0;
        may = may && cut;
        if (!may) key = 0xffffffffu;
        ns = __popcll(ballot(may));
        if (ns == 0) continue;
      }
      if (ns <= 2) {
        // one or two candidates (the common case): their order from wave
        // minima, without the 21 exchange stages of the sort (the keys are
        // distinct, the lane being their low bits)
        const uint32_t k0 = wave_min_u32(key);
        const uint32_t k1 = ns == 2 ? wave_min_u32(key == k0 ? 0xffffffffu : key) : 0xffffffffu;
        key = lane == 0 ? k0 : (lane == 1 ? k1 : 0xffffffffu);
      } else {
        key = wave_sort_u32(key);
      }
      uint64_t tc0 = 0;
      if (STATS) tc0 = clock_stamp();
      // park the batch in LDS (frees its registers during the serial loop)
      S.u.batch.cand[lane] = make_double4(dx, dy, dz, bb);
      S.u.batch.candj[lane] = q;
      S.u.batch.cands[lane] = shv;
      const float dnf = float(dn);
      __syncthreads();
      for (int r = 0; r < ns && !dead; ++r) {
        const int src = int(readlane_u(key, r) & 63u);
        const double4 C = S.u.batch.cand[src];
        clip_one(C.x, C.y, C.z, C.w, double(readlane_f(dnf, src)) * (1.0 + 1e-6), S.u.batch.candj[src],
                 S.u.batch.cands[src]);
      }
      if (STATS) t_clip += clock_stamp() - tc0;
      __syncthreads();
    }
    __syncthreads();
  };

  // ---------------------------------------------------------------- candidates
  // A generator yields lists of neighbour-grid cells (one per lane) to one
  // call site of process_list: first the 27 cells around the site (nearest
  // first), then the 98 cells of the second ring, then the surviving blocks
  // of Chebyshev shells of 4^3-cell blocks (cells already visited skipped),
  // until what is left lies beyond the reach R + sqrt(R^2 + 2 (psi_max - psi_i)).
  {
    const int bx0 = cx >> 2, by0 = cy >> 2, bz0 = cz >> 2;
    double mb = fmin(fmin(xi - bx0 * bh, (bx0 + 1) * bh - xi),
                     fmin(fmin(yi - by0 * bh, (by0 + 1) * bh - yi), fmin(zi - bz0 * bh, (bz0 + 1) * bh - zi)));
    mb = fmax(mb, 0.0);
    const int rb_max = 4 * Gb + 4;
    // distance from the site to the faces of its own grid cell (cell units)
    double mc = fmin(fmin(xi / h - cx, cx + 1 - xi / h),
                     fmin(fmin(yi / h - cy, cy + 1 - yi / h), fmin(zi / h - cz, cz + 1 - zi / h)));
    mc = fmax(mc, 0.0);
    // Reach of the polytope for sites of weight <= w: the bisector with such
    // a site at distance t from x_i lies at distance >= t/2 - (w - psi_i)/t
    // from x_i, beyond every vertex once t >= R + sqrt(R^2 + 2 (w - psi_i)),
    // R = the largest vertex distance from x_i.
    // t >= R + sqrt(R^2 + 2 max(0, w - psi_i)) is tested without the root:
    // for t >= 0 it is equivalent to t (t - 2R) >= 2 max(0, w - psi_i).
    auto out_of_reach = [&](double t, double w) {
      const double Rv = double(rvert);
      return t * (t - 2.0 * Rv) >= 2.0 * fmax(0.0, w + wslack - wi);
    };
    const double* bsuf = A.block_suffix + block_key(bx0, by0, bz0, Gb) * (SHELL_MAX + 1);
    // sites in blocks farther than SHELL_MAX block shells (bounded by the
    // global maximum weight) are out of reach
    auto far_ok = [&]() { return out_of_reach(SHELL_MAX * bh + mb - 1e-12 * L, gmax); };
    // Every site at distance >= t from x_i that lies in a block of shell
    // >= r is out of reach: the sites of shell q are farther than
    // max(t, (q - 1) bh + mb) and weigh at most bsuf[q] (the shell's maximum).
    // (not unrolled: unrolled, the per-shell distances stay live through the
    // whole walk and spill)
    auto beyond = [&](double t, int r) {
#pragma unroll 1
      for (int q = r; q <= SHELL_MAX; ++q) {
        const double dq = fmax(t, q >= 1 ? (q - 1) * bh + mb : 0.0);
        if (!out_of_reach(dq - 1e-12 * L, bsuf[q])) return false;
      }
      return far_ok();
    };
    // Combinatorics of the warm start's pass: the polytope it recorded is
    // rebuilt from the planes of the cell's J row at the current weights
    // (one triangle per lane) and kept when every vertex lies strictly
    // inside every other plane of the row and the box.  A closed set of
    // simple vertices each inside every half-space is the vertex set of their
    // intersection (from each vertex, every edge runs to another vertex of the
    // set and no plane crosses it in between), so the polytope is the one
    // that clipping the row's planes gives; otherwise the row is clipped.
    bool reused = false;
    if (A.topo_n_in && A.warm_rp) {
      const int ntr = A.topo_n_in[p];
      const int64_t wb = A.warm_rp[p];
      const int nw = int(A.warm_rp[p + 1] - wb);
      CPH(ST_TOPO_TRY, ntr > 0 ? 1 : 0);
      if (ntr >= 4 && ntr <= kTopoTri && nw <= kTopoFaces && 6 + nw <= PCAP) {
        const int np = 6 + nw;
        if (lane < nw) {
          // the planes exactly as the warm list forms them (nearest image)
          const int32_t j = A.warm_col[wb + lane];
          const double4 P = A.pts[j];
          const int32_t shw = pack_shift(-int(rint((P.x - xi) / L)), -int(rint((P.y - yi) / L)),
                                         -int(rint((P.z - zi) / L)));
          const double dx = P.x + unpack_shift(shw, 0) * L - xi;
          const double dy = P.y + unpack_shift(shw, 1) * L - yi;
          const double dz = P.z + unpack_shift(shw, 2) * L - zi;
          const double d2 = dx * dx + dy * dy + dz * dz;
          S.pl[6 + lane] = make_double4(dx, dy, dz, 0.5 * d2 + wi - P.w);
          S.pj[6 + lane] = j;
          S.ps[6 + lane] = shw;
        }
        __syncthreads();
        bool bad = false;
        int ta = 0, tb = 0, tc = 0;
        double X = 0.0, Y = 0.0, Z = 0.0;
        if (lane < ntr) {
          const uint32_t code = A.topo_tri_in[int64_t(p) * kTopoTri + lane];
          ta = int(code & 31u);
          tb = int((code >> 5) & 31u);
          tc = int((code >> 10) & 31u);
          bad = ta >= np || tb >= np || tc >= np;
          if (!bad) {
            const double4 P1 = S.pl[ta], P2 = S.pl[tb], P3 = S.pl[tc];
            const double c23x = P2.y * P3.z - P2.z * P3.y, c23y = P2.z * P3.x - P2.x * P3.z,
                         c23z = P2.x * P3.y - P2.y * P3.x;
            const double c31x = P3.y * P1.z - P3.z * P1.y, c31y = P3.z * P1.x - P3.x * P1.z,
                         c31z = P3.x * P1.y - P3.y * P1.x;
            const double c12x = P1.y * P2.z - P1.z * P2.y, c12y = P1.z * P2.x - P1.x * P2.z,
                         c12z = P1.x * P2.y - P1.y * P2.x;
            const double inv = recip_d(P1.x * c23x + P1.y * c23y + P1.z * c23z);
            X = (P1.w * c23x + P2.w * c31x + P3.w * c12x) * inv;
            Y = (P1.w * c23y + P2.w * c31y + P3.w * c12y) * inv;
            Z = (P1.w * c23z + P2.w * c31z + P3.w * c12z) * inv;
            bad = !(isfinite(X) && isfinite(Y) && isfinite(Z));
          }
        }
        // the tie tolerance of each plane (float64: eps = eps_scale |d|;
        // float32: the ambiguity band tol_rel (rvert |d| + |b|) with rvert
        // from these vertices), staged in the idle batch slots
        // (float roots enlarged by far more than their error: the bounds only
        // grow, which keeps the test conservative)
        const double rv =
            double(__builtin_amdgcn_sqrtf(float(wave_max_d(lane < ntr && !bad ? X * X + Y * Y + Z * Z : 0.0)))) *
                1.0001 +
            1e-6 * h;
        if (lane < np) {
          const double4 Q = S.pl[lane];
          const double qn = double(__builtin_amdgcn_sqrtf(float(Q.x * Q.x + Q.y * Q.y + Q.z * Q.z))) * (1.0 + 1e-6);
          S.u.batch.cand[lane].x = kF64 ? eps_scale * qn : double(tol_rel) * (rv * qn + fabs(Q.w));
        }
        __syncthreads();
        int nvt = 0;  // vertex-side tests made (work counters)
        if (lane < ntr && !bad) {
#pragma unroll 1
          for (int f = 0; f < np; ++f) {
            if (f == ta || f == tb || f == tc) continue;
            const double4 Q = S.pl[f];
            CNT(++nvt);
            if (!(X * Q.x + Y * Q.y + Z * Q.z - Q.w < -S.u.batch.cand[f].x)) {
              bad = true;
              break;
            }
          }
        }
        // the rebuilt vertices and their tests are the clipping's arithmetic
        CNT(c_newv += uint32_t(ntr));
        CNT(c_vt += uint32_t(wave_sum_i(nvt)));
        CNT(c_test += uint32_t(nw));
        reused = !ballot(bad);
        if (reused) {
          nT = ntr;
          nP = np;
          tri[0] = lane < ntr ? tri_pack(ta, tb, tc) : 0u;
          vx[0] = R(X);
          vy[0] = R(Y);
          vz[0] = R(Z);
#pragma unroll
          for (int k = 1; k < TPL; ++k) tri[k] = 0;
          if (lane < ntr) {
            S.stri[lane] = tri[0];
            S.sx[lane] = vx[0];
            S.sy[lane] = vy[0];
            S.sz[lane] = vz[0];
          }
          ball_dirty = true;
        }
        CPH(ST_TOPO_OK, reused ? 1 : 0);
        __syncthreads();
      }
    }
    if (use_cert || (A.warm_rp && !reused)) {
      // warm start: the sites of the certificate, or else the earlier
      // neighbours (nearest image); 64 per list, one call site
      const int64_t wb = use_cert ? 0 : A.warm_rp[p];
      const int64_t we = use_cert ? int64_t(A.cert_n[p] & 255) : A.warm_rp[p + 1];
      for (int64_t k0 = wb; k0 < we && !dead; k0 += 64) {
        const int64_t k = k0 + lane;
        int32_t j = -1, shw = 0;
        if (k < we) {
          if (use_cert) {
            const uint32_t e = A.cert_list[int64_t(p) * kCertCap + k];
            j = int32_t(e >> 5);
            shw = cert_shift(e);
          } else {
            j = A.warm_col[k];
          }
        }
        const bool act = j >= 0 && j != p;
        if (act && !use_cert) {
          const double4 P = A.pts[j];
          shw = pack_shift(-int(rint((P.x - xi) / L)), -int(rint((P.y - yi) / L)),
                           -int(rint((P.z - zi) / L)));
        }
        process_list(act, act ? j : 0, 1, shw, 0);
      }
    }
    bool skip_walk = false;
    if (use_cert && uniform_i(dead ? 1 : 0) == 0) {
      // is every vertex within kappa of a recorded vertex?  (Then the
      // polytope lies inside the recorded one widened by kappa, which the
      // recording walk covered.)  The recorded vertices go through LDS.
      const int nv = (A.cert_n[p] >> 8) & 255;
      const float sc = uniform_f(A.cert_scale[p]);
      if (lane < nv) {
        const uint32_t e = A.cert_vtx[int64_t(p) * kCertVtx + lane];
        S.u.batch.cand[lane] = make_double4(double(float(int(e & 2047u) - 1024) * (sc / 1023.f)),
                                            double(float(int((e >> 11) & 2047u) - 1024) * (sc / 1023.f)),
                                            double(float(int(e >> 22) - 512) * (sc / 511.f)), 0.0);
      }
      __syncthreads();
      // kappa less the rounding of the offsets (half a step per axis) and
      // of the float arithmetic
      const float kc = A.cert_kappa - sc * (1.25e-3f + 1e-5f) - 1e-6f * float(h);
      bool outside = !(kc > 0.f);
#pragma unroll
      for (int k = 0; k < TPL; ++k) {
        if (k * 64 + lane < nT) {
          const float ux = float(vx[k]), uy = float(vy[k]), uz = float(vz[k]);
          float dmin = FLT_MAX;
#pragma unroll 1
          for (int t = 0; t < nv; ++t) {
            const double4 U = S.u.batch.cand[t];
            const float ex = ux - float(U.x), ey = uy - float(U.y), ez = uz - float(U.z);
            dmin = fminf(dmin, ex * ex + ey * ey + ez * ez);
          }
          outside = outside || !(dmin <= kc * kc);
        }
      }
      skip_walk = !ballot(outside);
      __syncthreads();
      CPH(ST_CERT_TRY, 1);
      CPH(ST_CERT_OK, skip_walk ? 1 : 0);
    }
    int phase = 0;  // 0: 27 cells, 1 and 2: ring 2 of cells, 3: block shells
    int rb = 0, gbase = 0, gcount = 1;
    uint64_t bmask = 0;
    int ubx = 0, uby = 0, ubz = 0;
    int walk_iter = 0;
    while (!dead && !skip_walk) {
      // a trial another cell has already rejected: stop the walk (the pass is
      // discarded); checked every 16 lists, a long walk of a far cell would
      // otherwise hold the launch open
      if (A.doom && (++walk_iter & 15) == 0 &&
          __hip_atomic_load(A.doom, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        dead = true;
        break;
      }
      bool act = false;
      int32_t st = 0, cnt = 0, shp = 0;
      const int lph = phase == 0 ? 1 : (phase <= 2 ? 2 : 3);
      if (phase == 1 || phase == 2) {
        // ring 2 of grid cells (98 cells, two lists), after a reach check
        if (phase == 1) {
          refresh_ball();
          if (beyond((1.0 + mc) * h, 0)) break;
        }
        const int t = (phase == 1 ? 0 : 64) + lane;
        phase += 1;
        act = t < 98;
        int ox = 0, oy = 0, oz = 0;
        if (act) shell_offset(2, t, ox, oy, oz);
        const int ux = cx + ox, uy = cy + oy, uz = cz + oz;
        const int sx = period_div(ux, Gn), sy = period_div(uy, Gn), sz = period_div(uz, Gn);
        if (act) {
          const int64_t g = cell_key(ux - sx * Gn, uy - sy * Gn, uz - sz * Gn, Gb);
          st = A.cell_start[g];
          cnt = A.cell_start[g + 1] - st;
          act = cnt > 0;
          if (act) {
            const double lx = ux * h - xi - 1e-12 * L, ly = uy * h - yi - 1e-12 * L,
                         lz = uz * h - zi - 1e-12 * L;
            // (arithmetic shifts floor: BLOCK_SIDE is 4)
            const int ubx = ux >> 2, uby = uy >> 2, ubz = uz >> 2;
            const int64_t bk = block_key(ubx - period_div(ubx, Gb) * Gb, uby - period_div(uby, Gb) * Gb,
                                         ubz - period_div(ubz, Gb) * Gb, Gb);
            act = box_may_cut(lx, ly, lz, lx + h + 2e-12 * L, ly + h + 2e-12 * L, lz + h + 2e-12 * L, bk,
                              ubx, uby, ubz, A.cell_tmax[g]);
          }
        }
        CNT(c_box += 64);
        CPH(ST_BOXT_R, __popcll(ballot(t < 98 && cnt > 0)));
        CPH(ST_BOXP_R, __popcll(ballot(act)));
        shp = pack_shift(sx, sy, sz);
      } else if (phase == 0) {
        phase = 1;
        act = lane < 27;
        const int code = act ? kNearOrder[lane] : 13;
        const int ux = cx + code / 9 - 1, uy = cy + (code / 3) % 3 - 1, uz = cz + code % 3 - 1;
        const int sx = period_div(ux, Gn), sy = period_div(uy, Gn), sz = period_div(uz, Gn);
        if (act) {
          const int64_t g = cell_key(ux - sx * Gn, uy - sy * Gn, uz - sz * Gn, Gb);
          st = A.cell_start[g];
          cnt = A.cell_start[g + 1] - st;
        }
        shp = pack_shift(sx, sy, sz);
      } else {
        if (rb == 0 && gbase == 0) {
          refresh_ball();
          if (beyond((2.0 + mc) * h, 0)) break;  // ring 3 out of reach
        }
        // next surviving block (advancing batches and shells as needed)
        bool done = false;
        while (!bmask && !done) {
          refresh_ball();
          if (gbase >= gcount) {
            ++rb;
            if (beyond((rb - 1) * bh + mb, rb)) {
              done = true;
              break;
            }
            if (rb > rb_max) {
              flags |= CF_CAPACITY;
              dead = true;
              done = true;
              break;
            }
            const int S1 = 2 * rb + 1, I1 = 2 * rb - 1;
            gcount = S1 * S1 * S1 - I1 * I1 * I1;
            gbase = 0;
          }
          const int t = gbase + lane;
          CNT(c_box += uint32_t(min(64, gcount - gbase)));
          CPH(ST_BOXT_BLK, min(64, gcount - gbase));
          gbase += 64;
          bool ok = false;
          if (t < gcount) {
            int ox, oy, oz;
            shell_offset(rb, t, ox, oy, oz);
            ubx = bx0 + ox;
            uby = by0 + oy;
            ubz = bz0 + oz;
            const int wbx = ubx - period_div(ubx, Gb) * Gb, wby = uby - period_div(uby, Gb) * Gb,
                      wbz = ubz - period_div(ubz, Gb) * Gb;
            const double lx = ubx * bh - xi - 1e-12 * L, ly = uby * bh - yi - 1e-12 * L,
                         lz = ubz * bh - zi - 1e-12 * L;
            const double hx = lx + bh + 2e-12 * L, hy = ly + bh + 2e-12 * L, hz = lz + bh + 2e-12 * L;
            const int64_t bk = block_key(wbx, wby, wbz, Gb);
            ok = box_may_cut(lx, ly, lz, hx, hy, hz, bk, ubx, uby, ubz, A.block_tmax[bk]);
          }
          bmask = ballot(ok);
          CPH(ST_BOXP_BLK, __popcll(bmask));
        }
        if (done) break;
        refresh_ball();
        const int l = __ffsll((unsigned long long)bmask) - 1;
        bmask &= bmask - 1;
        const int qbx = readlane_i(ubx, l), qby = readlane_i(uby, l), qbz = readlane_i(ubz, l);
        CNT(c_box += 64);
        const int ux = qbx * BLOCK_SIDE + (lane >> 4), uy = qby * BLOCK_SIDE + ((lane >> 2) & 3),
                  uz = qbz * BLOCK_SIDE + (lane & 3);
        const bool inA = abs(ux - cx) <= 2 && abs(uy - cy) <= 2 && abs(uz - cz) <= 2;
        const int sx = period_div(ux, Gn), sy = period_div(uy, Gn), sz = period_div(uz, Gn);
        const int64_t g = cell_key(ux - sx * Gn, uy - sy * Gn, uz - sz * Gn, Gb);
        st = A.cell_start[g];
        cnt = A.cell_start[g + 1] - st;
        act = !inA && cnt > 0;
        CPH(ST_BOXT_BC, __popcll(ballot(act)));
        if (act) {
          const double lx = ux * h - xi - 1e-12 * L, ly = uy * h - yi - 1e-12 * L,
                       lz = uz * h - zi - 1e-12 * L;
          const int64_t bk = block_key(qbx - period_div(qbx, Gb) * Gb, qby - period_div(qby, Gb) * Gb,
                                       qbz - period_div(qbz, Gb) * Gb, Gb);
          act = box_may_cut(lx, ly, lz, lx + h + 2e-12 * L, ly + h + 2e-12 * L, lz + h + 2e-12 * L, bk,
                            qbx, qby, qbz, A.cell_tmax[g]);
        }
        shp = pack_shift(sx, sy, sz);
      }
      if (lph == 3) CPH(ST_BOXP_BC, __popcll(ballot(act && cnt > 0)));
      process_list(act, st, cnt, shp, lph);
    }
    CPH(ST_SHELL, rb);
  }
  bool rec = false;
  if (cmode == 1) {
    // recording: the list now (its LDS is reused below), the vertices with
    // the float64 ones; a cell that dies here is recorded by the stage that
    // finishes it
    uint32_t e = 0;
    if (lane < ccount && lane < kCertCap) e = cert_entry(int32_t(S.u.batch.clist[lane]), S.u.batch.clsh[lane]);
    rec = !dead && ccount <= kCertCap && nT <= kCertVtx && !ballot(e == 0xffffffffu);
    if (lane == 0) A.cert_n[p] = rec ? (ccount | (nT << 8)) : -1;
    if (rec && lane < ccount) A.cert_list[int64_t(p) * kCertCap + lane] = e;
    CPH(ST_CERT_REC, rec ? 1 : 0);
    CPH(ST_CERT_LEN, rec ? ccount : 0);
    CPH(ST_CERT_OVF, (!dead && !rec) ? 1 : 0);
  }

  if (STATS) t_search_end = clock_stamp();
  auto flush_stats = [&](int ntri, int nfaces) {
    if (STATS && A.stats && lane == 0) {
      unsigned long long* st = A.stats;
      const uint64_t t_end = clock_stamp();
      atomicAdd(&st[ST_TSEARCH], (unsigned long long)(t_search_end - t_begin - t_clip));
      atomicAdd(&st[ST_TCLIP], (unsigned long long)t_clip);
      atomicAdd(&st[ST_TINT], (unsigned long long)(t_end - t_search_end));
      atomicAdd(&st[ST_TPRE], (unsigned long long)t_pre);
      atomicAdd(&st[ST_TCUT], (unsigned long long)t_cut);
      atomicAdd(&st[ST_CAND], (unsigned long long)c_cand);
      atomicAdd(&st[ST_TEST], (unsigned long long)c_test);
      atomicAdd(&st[ST_VTEST], (unsigned long long)(c_vt + c_pre));
      atomicAdd(&st[ST_CUT], (unsigned long long)c_cut);
      atomicAdd(&st[ST_NEWV], (unsigned long long)c_newv);
      atomicAdd(&st[ST_BALL], (unsigned long long)c_ball);
      atomicAdd(&st[ST_BOX], (unsigned long long)c_box);
      atomicAdd(&st[ST_TRI], (unsigned long long)ntri);
      atomicAdd(&st[ST_FACES], (unsigned long long)nfaces);
      atomicAdd(&st[ST_CELLS], 1ull);
#pragma unroll
      for (int k = ST_SCAN_W; k < ST_N; ++k) atomicAdd(&st[k], (unsigned long long)c_ph[k - ST_SCAN_W]);
    }
  };

  if (dead) {
    flush_stats(0, 0);
    if (lane == 0) {
      if (A.doom && (flags & CF_EMPTY) &&
          !(flags & (CF_CAPACITY | CF_NONMANIFOLD | CF_NEARDEG))) {
        __hip_atomic_store(A.doom, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(A.doom_cell, (unsigned long long)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (flags & (CF_CAPACITY | CF_NONMANIFOLD | CF_NEARDEG)) {
        atomicAdd(&A.cause[(flags & CF_CAPACITY) ? 0 : ((flags & CF_NONMANIFOLD) ? 1 : 2)], 1ull);
        const unsigned long long r = atomicAdd(A.retry_count, 1ull);
        A.retry[r] = p;
      }
      A.vol[p] = 0.0;
      A.mom[3 * p] = A.mom[3 * p + 1] = A.mom[3 * p + 2] = 0.0;
      A.nface[p] = 0;
      A.cflags[p] = flags;
      if (A.topo_n_out) A.topo_n_out[p] = -1;
    }
    return;
  }

  // ---------------------------------------------------------------- integrals
  auto plane_d = [&](int f) -> double4 { return S.pl[f]; };
  // final vertices in float64
  double fvx[TPL], fvy[TPL], fvz[TPL];
  double* FX;
  double* FY;
  double* FZ;
  if constexpr (kF64) {
    FX = S.sx;
    FY = S.sy;
    FZ = S.sz;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      fvx[k] = vx[k];
      fvy[k] = vy[k];
      fvz[k] = vz[k];
    }
  } else {
    FX = S.u.ints.fin.x;
    FY = S.u.ints.fin.y;
    FZ = S.u.ints.fin.z;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      fvx[k] = fvy[k] = fvz[k] = 0.0;
      const int slot = k * 64 + lane;
      if (slot < nT) {
        const double4 P1 = plane_d(tri_a(tri[k])), P2 = plane_d(tri_b(tri[k])),
                      P3 = plane_d(tri_c(tri[k]));
        const double c23x = P2.y * P3.z - P2.z * P3.y, c23y = P2.z * P3.x - P2.x * P3.z,
                     c23z = P2.x * P3.y - P2.y * P3.x;
        const double c31x = P3.y * P1.z - P3.z * P1.y, c31y = P3.z * P1.x - P3.x * P1.z,
                     c31z = P3.x * P1.y - P3.y * P1.x;
        const double c12x = P1.y * P2.z - P1.z * P2.y, c12y = P1.z * P2.x - P1.x * P2.z,
                     c12z = P1.x * P2.y - P1.y * P2.x;
        const double inv = recip_d(P1.x * c23x + P1.y * c23y + P1.z * c23z);
        fvx[k] = (P1.w * c23x + P2.w * c31x + P3.w * c12x) * inv;
        fvy[k] = (P1.w * c23y + P2.w * c31y + P3.w * c12y) * inv;
        fvz[k] = (P1.w * c23z + P2.w * c31z + P3.w * c12z) * inv;
        FX[slot] = fvx[k];
        FY[slot] = fvy[k];
        FZ[slot] = fvz[k];
      }
    }
  }
  if (rec) {
    // the certificate's vertices: 11/11/10-bit offsets from the site in
    // units of rvert (which bounds every vertex distance)
    const float sc = rvert;
    if (lane < nT) {
      const int qx = min(1023, max(-1023, int(rintf(float(fvx[0]) * (1023.f / sc)))));
      const int qy = min(1023, max(-1023, int(rintf(float(fvy[0]) * (1023.f / sc)))));
      const int qz = min(511, max(-511, int(rintf(float(fvz[0]) * (511.f / sc)))));
      A.cert_vtx[int64_t(p) * kCertVtx + lane] =
          uint32_t(qx + 1024) | (uint32_t(qy + 1024) << 11) | (uint32_t(qz + 512) << 22);
    }
    if (lane == 0) A.cert_scale[p] = sc;
  }
  // membership masks: bit t of mask f is set when triangle t contains plane f
  // (in the LDS the search's batch used: cleared here)
  __syncthreads();
  for (int w = lane; w < PCAP * TW; w += 64) S.u.ints.mem[w] = 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int slot = k * 64 + lane;
    if (slot < nT) {
      const uint32_t bit = 1u << (slot & 31);
      const int w = slot >> 5;
      atomicOr(&S.u.ints.mem[tri_a(tri[k]) * TW + w], bit);
      atomicOr(&S.u.ints.mem[tri_b(tri[k]) * TW + w], bit);
      atomicOr(&S.u.ints.mem[tri_c(tri[k]) * TW + w], bit);
    }
  }
  __syncthreads();
  double v6 = 0, m0 = 0, m1 = 0, m2 = 0;
  double ar[TPL][3];
  bool broken = false;
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    ar[k][0] = ar[k][1] = ar[k][2] = 0.0;
    const int slot = k * 64 + lane;
    if (slot >= nT) continue;
    const int fa[3] = {tri_a(tri[k]), tri_b(tri[k]), tri_c(tri[k])};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int f = fa[e], pr = fa[(e + 2) % 3];
      int tw = -1;
#pragma unroll
      for (int w = 0; w < TW; ++w) {
        uint32_t m = S.u.ints.mem[f * TW + w] & S.u.ints.mem[pr * TW + w];
        if (w == (slot >> 5)) m &= ~(1u << (slot & 31));
        if (m && tw < 0) tw = w * 32 + __ffs(int(m)) - 1;
      }
      if (tw < 0) {
        broken = true;
        continue;
      }
      const double tx = FX[tw], ty = FY[tw], tz = FZ[tw];
      const double4 P = plane_d(f);
      // fan apex: the lowest-slot vertex of face f (on the plane, close to
      // the face, so small faces keep their relative precision)
      int t0 = 0;
#pragma unroll
      for (int w = TW - 1; w >= 0; --w) {
        const uint32_t m = S.u.ints.mem[f * TW + w];
        if (m) t0 = w * 32 + __ffs(int(m)) - 1;
      }
      const double px = FX[t0], py = FY[t0], pz = FZ[t0];
      const double det = px * (fvy[k] * tz - fvz[k] * ty) + py * (fvz[k] * tx - fvx[k] * tz) +
                         pz * (fvx[k] * ty - fvy[k] * tx);
      v6 += det;
      m0 += det * (px + fvx[k] + tx);
      m1 += det * (py + fvy[k] + ty);
      m2 += det * (pz + fvz[k] + tz);
      const double ax = fvx[k] - px, ay = fvy[k] - py, az = fvz[k] - pz;
      const double bx = tx - px, by = ty - py, bz = tz - pz;
      const double crx = ay * bz - az * by, cry = az * bx - ax * bz, crz = ax * by - ay * bx;
      // twice the fan triangle's area times |d| (divided once per face below)
      ar[k][e] = crx * P.x + cry * P.y + crz * P.z;
    }
  }
  v6 = wave_sum_d(v6);
  m0 = wave_sum_d(m0);
  m1 = wave_sum_d(m1);
  m2 = wave_sum_d(m2);
  if (ballot(broken)) flags |= CF_NONMANIFOLD;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int slot = k * 64 + lane;
    if (slot < nT) {
      FX[slot] = ar[k][0];
      FY[slot] = ar[k][1];
      FZ[slot] = ar[k][2];
    }
  }
  __syncthreads();
  // per-face areas: one lane per plane (faces of the own-image box, tagged
  // j < 0, are not faces of J)
  double Af[NPC], Dn[NPC];
  int nf = 0;
#pragma unroll
  for (int c = 0; c < NPC; ++c) {
    const int f = c * 64 + lane;
    double a = 0.0;
    Dn[c] = 1.0;
    const bool real = f < nP && S.pj[f] >= 0;
    if (real) {
#pragma unroll
      for (int w = 0; w < TW; ++w) {
        uint32_t m = S.u.ints.mem[f * TW + w];
        while (m) {
          const int t = w * 32 + __ffs(int(m)) - 1;
          m &= m - 1;
          const uint32_t tr = S.stri[t];
          a += tri_a(tr) == f ? FX[t] : (tri_b(tr) == f ? FY[t] : FZ[t]);
        }
      }
    }
    if (real) {
      const double4 P = plane_d(f);
      Dn[c] = sqrt(P.x * P.x + P.y * P.y + P.z * P.z);
      a = 0.5 * a / Dn[c];
    }
    Af[c] = (real && a > A.area_min) ? a : 0.0;
    nf += __popcll(ballot(Af[c] > 0.0));
  }
  if (A.topo_n_out) {
    // This pass's combinatorics for the next one.  Plane codes: a box plane
    // 2 axis + (side < 0); a written face 6 + the rank of its site among the
    // written faces' sites (its position in the cell's row of J); 31 none.
    // (The cut bitmap is idle now: sites of the written faces, then codes.)
    uint32_t* wj = S.bits;
    uint32_t* pcode = S.bits + PCAP;
#pragma unroll
    for (int c = 0; c < NPC; ++c) {
      const int f = c * 64 + lane;
      if (f < PCAP) wj[f] = (f < nP && Af[c] > 0.0) ? uint32_t(S.pj[f]) : 0xffffffffu;
    }
    __syncthreads();
    bool dup = false;
#pragma unroll
    for (int c = 0; c < NPC; ++c) {
      const int f = c * 64 + lane;
      uint32_t code = 31u;
      if (f < nP && S.pj[f] < 0) {
        const int32_t sh = S.ps[f];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
          if (unpack_shift(sh, ax) != 0) code = uint32_t(2 * ax + (unpack_shift(sh, ax) < 0 ? 1 : 0));
      } else if (f < nP && wj[f] != 0xffffffffu) {
        const uint32_t me = wj[f];
        int rank = 0;
#pragma unroll 1
        for (int g = 0; g < nP; ++g) {
          const uint32_t o = wj[g];
          if (o == 0xffffffffu) continue;
          rank += (o < me) ? 1 : 0;
          dup = dup || (o == me && g != f);
        }
        code = rank < kTopoFaces ? uint32_t(6 + rank) : 31u;
      }
      if (f < PCAP) pcode[f] = code;
    }
    __syncthreads();
    bool miss = false;
    uint32_t rec[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      rec[k] = 0;
      if (k * 64 + lane < nT) {
        const uint32_t ca = pcode[tri_a(tri[k])], cb = pcode[tri_b(tri[k])], cc = pcode[tri_c(tri[k])];
        miss = miss || ca == 31u || cb == 31u || cc == 31u;
        rec[k] = ca | (cb << 5) | (cc << 10);
      }
    }
    const bool ok = nT <= kTopoTri && !ballot(miss || dup);
    if (ok && lane < nT) A.topo_tri_out[int64_t(p) * kTopoTri + lane] = uint16_t(rec[0]);
    if (lane == 0) A.topo_n_out[p] = ok ? nT : -1;
  }
  if (A.write_faces) {
    FaceRec* dst = A.faces + int64_t(p) * A.fslot;
    if (nf > A.fslot) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(A.ovf_used, (unsigned long long)nf);
      base = readlane_u64(base, 0);
      if (int64_t(base) + nf > A.ovf_cap) {
        flags |= CF_CAPACITY;
        dst = nullptr;
      } else {
        dst = A.ovf + base;
        if (lane == 0) A.fbase[p] = int64_t(base);
      }
    }
    int run = 0;
#pragma unroll
    for (int c = 0; c < NPC; ++c) {
      const int f = c * 64 + lane;
      const bool rep = Af[c] > 0.0;
      const uint64_t rm = ballot(rep);
      if (rep && dst) {
        FaceRec fr;
        fr.j = S.pj[f];
        fr.shift = S.ps[f];
        fr.w = Af[c] / Dn[c];
        dst[run + lanes_below(rm)] = fr;
      }
      run += __popcll(rm);
    }
  }
  flush_stats(nT, nf);
  if (lane == 0) {
    if (A.doom && v6 / 6.0 < A.doom_vol) {
      __hip_atomic_store(A.doom, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(A.doom_cell, (unsigned long long)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    A.vol[p] = v6 / 6.0;
    A.mom[3 * p] = m0 / 24.0;
    A.mom[3 * p + 1] = m1 / 24.0;
    A.mom[3 * p + 2] = m2 / 24.0;
    A.nface[p] = nf;
    A.cflags[p] = flags;
  }
}

// Counted arithmetic per work event (float64 ops, FMA = 2).  The method's
// own work, the intersection of the half-spaces of Eq. laguerrecell and the
// integrals of Eq. SDK: forming a candidate plane that reaches the polytope
// 21; one vertex-side test 7; one new vertex (three cross products,
// determinant, solve) 50; integrals per final vertex (three face triangles:
// determinant, moment, area) 135.
double clip_flops(const unsigned long long* c) {
  return 21.0 * c[ST_TEST] + 7.0 * c[ST_VTEST] + 50.0 * c[ST_NEWV] + 135.0 * c[ST_TRI];
}
// The search for the candidates (not the method's arithmetic: a search
// overhead that a tighter bound would remove): scanning a site (image
// offset, |d|^2, plane offset, ball test, sort key) 26; one vertex of a ball
// update 11; one block / cell box test 30.
double clip_search_flops(const unsigned long long* c) {
  return 26.0 * c[ST_CAND] + 11.0 * c[ST_BALL] + 30.0 * c[ST_BOX];
}
// Compulsory HBM bytes: read own site (32), write volume, moment, flags and
// face count (40), write the reported faces (16 each).  Neighbour reads are
// served by the caches.
double clip_bytes(const unsigned long long* c) {
  return 72.0 * c[ST_CELLS] + double(sizeof(FaceRec)) * c[ST_FACES];
}

template <int TPL, typename R>
void launch_clip(ClipBatch& b, CellPass* const* outs, hipStream_t st) {
  Profiler* pr = g_prof;
  const bool counting = pr && pr->counting;
  int64_t items = 0;
  for (int j = 0; j < b.njobs; ++j) {
    items += b.job[j].nwork;
    if (counting) {
      b.job[j].stats = outs[j]->counters.as<unsigned long long>() + kCtrStats;
      MAK_HIP(hipMemsetAsync(b.job[j].stats, 0, ST_N * sizeof(unsigned long long), st));
    }
  }
  const char* name = sizeof(R) == 4 ? "clip_f32" : (TPL == 2 ? "clip" : "clip_large");
  ProfScope ps(name, st, double(items));
  // one 64-lane workgroup per item; the work-items of one grid dimension
  // must stay below 2^32, so launches above 2^16 workgroups use a 2-D grid of
  // rows of 2^16 workgroups
  const int64_t nblk = b.blk_start[b.njobs];
  const int64_t gx = nblk < (int64_t(1) << 16) ? nblk : (int64_t(1) << 16);
  const dim3 grid(unsigned(gx), unsigned(ceil_div(nblk, gx)));
  bool cert = false;
  for (int j = 0; j < b.njobs; ++j) cert = cert || b.job[j].cert_mode != 0;
  if (counting && cert)
    hipLaunchKernelGGL((k_clip<TPL, R, true, true>), grid, dim3(64), 0, st, b);
  else if (counting)
    hipLaunchKernelGGL((k_clip<TPL, R, true, false>), grid, dim3(64), 0, st, b);
  else if (cert)
    hipLaunchKernelGGL((k_clip<TPL, R, false, true>), grid, dim3(64), 0, st, b);
  else
    hipLaunchKernelGGL((k_clip<TPL, R, false, false>), grid, dim3(64), 0, st, b);
  MAK_HIP(hipGetLastError());
  if (counting) {
    double flops = 0, bytes = 0;
    for (int j = 0; j < b.njobs; ++j) {
      unsigned long long c[ST_N];
      MAK_HIP(hipMemcpyAsync(c, b.job[j].stats, sizeof(c), hipMemcpyDeviceToHost, st));
      MAK_HIP(hipStreamSynchronize(st));
      flops += clip_flops(c);
      bytes += clip_bytes(c);
      for (int k = 0; k < ST_N; ++k) pr->counters[k] += double(c[k]);
      pr->counters[ST_SEARCH_FLOPS] += clip_search_flops(c);
      b.job[j].stats = nullptr;
    }
    ps.flops = flops;
    ps.bytes = bytes;
  }
  ps.stop();
}

}  // namespace

namespace {

// Stages: every cell runs in the first kernel; the cells it could not finish
// (capacity, inconsistent cut, float32 ambiguity) go to the next.
//   float64: <2 vertices per lane, f64>  ->  <4, f64, wider tie tolerance>
//   mixed:   <1, f32>  ->  <2, f64>  ->  <4, f64, wider tie tolerance>
// (the float32 stage holds 64 vertices: the few cells that need more, about
// one in 8,000 at psi = 0 on the clustered input, finish in float64)
// counters of a pass: [0] overflow faces used, [1 + s] cells listed by stage
// s, [4] doom flag of a line-search trial, [5] a cell that raised it,
// [kCtrStats ..] work counters,
// [kCtrCause + 3 s ..] causes (capacity, cut, ambiguity)
int num_stages(int precision) { return precision == MAK_MIXED ? 3 : 2; }

void job_begin(PassJob& jb, hipStream_t st) {
  CellPass& out = *jb.out;
  MAK_HIP(hipMemsetAsync(out.counters.p, 0, kCtrN * sizeof(unsigned long long), st));
  jb.stage = jb.opt.first_stage;
  jb.all_cells = jb.opt.probe_n <= 0;
  jb.listed = jb.all_cells ? jb.ps->N : jb.opt.probe_n;
  jb.cs = ClipStats();
}

ClipArgs job_args(PassJob& jb, int stage, int nstage) {
  PointSet& ps = *jb.ps;
  CellPass& out = *jb.out;
  FaceStore& fst = out.fs();
  const int64_t N = ps.N;
  unsigned long long* ctr = out.counters.as<unsigned long long>();
  ClipArgs a{};
  a.pts = ps.pts.as<double4>();
  a.cell_start = ps.cell_start.as<int32_t>();
  a.block_suffix = ps.block_suffix.as<double>();
  a.warm_rp = jb.opt.warm_rp && jb.opt.warm_col ? jb.opt.warm_rp : nullptr;
  a.warm_col = a.warm_rp ? jb.opt.warm_col : nullptr;
  a.block_g = ps.block_g.as<double>();
  a.block_tmax = ps.block_tmax.as<double>();
  a.cell_tmax = ps.cell_tmax.as<double>();
  a.gmax = ps.scal.as<double>();
  a.Gn = ps.g.Gn;
  a.Gb = ps.g.Gb;
  a.L = ps.g.L;
  a.h = ps.g.h;
  a.vol = out.vol.as<double>();
  a.mom = out.mom.as<double>();
  a.cflags = out.cflags.as<int32_t>();
  a.nface = out.nface.as<int32_t>();
  const bool faces = jb.opt.faces;
  a.faces = faces ? fst.faces.as<FaceRec>() : nullptr;
  a.fbase = faces ? fst.fbase.as<int64_t>() : nullptr;
  a.ovf = faces ? fst.ovf.as<FaceRec>() : nullptr;
  a.ovf_used = ctr;
  a.ovf_cap = faces ? fst.ovf_cap : 0;
  a.fslot = fst.fslot;
  a.write_faces = faces ? 1 : 0;
  const double spacing = ps.g.L / std::cbrt(double(N));
  a.area_min = 1e-12 * spacing * spacing;
  a.tol_rel = 1e-6;
  a.stats = nullptr;
  if (jb.opt.probe_n > 0)
    a.work = jb.opt.probe_list;
  else
    a.work = jb.all_cells ? nullptr : out.retry.as<int32_t>() + (stage - 1) * N;
  a.nwork = jb.listed;
  a.per_xcd = ceil_div(jb.listed, 8);
  a.retry = out.retry.as<int32_t>() + stage * N;
  a.retry_count = ctr + 1 + stage;
  a.cause = ctr + kCtrCause + 3 * stage;
  a.eps_rel = stage == nstage - 1 ? 1e-11 : 1e-13;
  a.doom = jb.opt.doom_vol > 0 ? reinterpret_cast<unsigned int*>(ctr + 4) : nullptr;
  a.doom_cell = ctr + 5;
  a.doom_vol = jb.opt.doom_vol;
  CertSet* ce = jb.opt.cert;
  a.cert_mode = ce && a.warm_rp ? jb.opt.cert_mode : 0;
  if (a.cert_mode == 1 && jb.opt.probe_n > 0) a.cert_mode = 0;  // a probe records nothing
  if (a.cert_mode) {
    a.cert_kappa = float(ce->kappa);
    a.cert_margin = ce->margin;
    a.cert_list = ce->list.as<uint32_t>();
    a.cert_n = ce->n.as<int32_t>();
    a.cert_vtx = ce->vtx.as<uint32_t>();
    a.cert_scale = ce->scale.as<float>();
    a.psi_ref = ce->psi_ref.as<double>();
    a.cert_dmax = ce->dmax.as<unsigned long long>();
  }
  const CellPass* ti = jb.opt.topo_in;
  if (ti && a.warm_rp && ti->topo_n.cap >= size_t(N) * sizeof(int32_t) &&
      ti->topo_tri.cap >= size_t(N) * kTopoTri * sizeof(uint16_t)) {
    a.topo_tri_in = ti->topo_tri.as<uint16_t>();
    a.topo_n_in = ti->topo_n.as<int32_t>();
  }
  CellPass* to = jb.opt.topo_out;
  if (to && jb.opt.probe_n <= 0) {  // a probe records nothing
    if (to->topo_n.cap < size_t(N) * sizeof(int32_t) || to->topo_tri.cap < size_t(N) * kTopoTri * sizeof(uint16_t))
      MAK_FAIL(MAK_EHIP, "combinatorics records not sized");
    a.topo_tri_out = to->topo_tri.as<uint16_t>();
    a.topo_n_out = to->topo_n.as<int32_t>();
  }
  return a;
}

// One launch of stage `stage` over jobs[0..n).
void launch_stage(PassJob* const* jobs, int n, int stage, int precision, hipStream_t st) {
  const int nstage = num_stages(precision);
  ClipBatch b{};
  CellPass* outs[kMaxJobs];
  b.njobs = n;
  int64_t nb = 0;
  for (int j = 0; j < n; ++j) {
    b.job[j] = job_args(*jobs[j], stage, nstage);
    outs[j] = jobs[j]->out;
    b.blk_start[j] = nb;
    nb += 8 * b.job[j].per_xcd;
  }
  for (int j = n; j <= kMaxJobs; ++j) b.blk_start[j] = nb;
  const bool mixed = precision == MAK_MIXED;
  if (mixed && stage == 0)
    launch_clip<1, float>(b, outs, st);
  else if (stage < nstage - 1)
    launch_clip<2, double>(b, outs, st);
  else
    launch_clip<4, double>(b, outs, st);
}

}  // namespace

namespace {

__global__ void k_cert_snapshot(const double4* __restrict__ pts, double* __restrict__ ref, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) ref[i] = pts[i].w;
}

__global__ void k_cert_dmax(const double4* __restrict__ pts, const double* __restrict__ ref,
                            unsigned long long* out, int64_t n) {
  double m = -DBL_MAX;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    m = fmax(m, pts[i].w - ref[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane_id() == 0) atomicMax(out, ordered_key(m));
}

}  // namespace

void cert_snapshot(const PointSet& ps, CertSet& c, hipStream_t st) {
  if (c.psi_ref.cap < size_t(ps.N) * sizeof(double)) MAK_FAIL(MAK_EHIP, "certificate weights not sized");
  if (ps.N == 0) return;
  hipLaunchKernelGGL(k_cert_snapshot, dim3(unsigned(ceil_div(ps.N, 256))), dim3(256), 0, st,
                     ps.pts.as<double4>(), c.psi_ref.as<double>(), ps.N);
  MAK_HIP(hipGetLastError());
}

void cert_dmax(const PointSet& ps, CertSet& c, hipStream_t st) {
  if (c.psi_ref.cap < size_t(ps.N) * sizeof(double) || c.dmax.cap < 8)
    MAK_FAIL(MAK_EHIP, "certificate buffers not sized");
  fill_zero_i32(c.dmax.as<int32_t>(), 2, st);  // key 0 lies below every value
  if (ps.N == 0) return;
  const int64_t nb = std::min<int64_t>(2048, ceil_div(ps.N, 256));
  hipLaunchKernelGGL(k_cert_dmax, dim3(unsigned(nb)), dim3(256), 0, st, ps.pts.as<double4>(),
                     c.psi_ref.as<double>(), c.dmax.as<unsigned long long>(), ps.N);
  MAK_HIP(hipGetLastError());
}

int32_t face_slots(int64_t N) { return N <= (int64_t(1) << 24) ? 32 : 20; }

static_assert(kCtrStats + ST_N <= kCtrCause, "work counters overlap the stage causes");
static_assert(ST_N <= kProfCounters, "the profile holds every work counter");

void run_cells_batch(PassJob* const* jobs, int njobs, int precision, hipStream_t st) {
  const int nstage = num_stages(precision);
  const bool mixed = precision == MAK_MIXED;
  std::vector<PassJob*> live;
  for (int j = 0; j < njobs; ++j) {
    PassJob& jb = *jobs[j];
    jb.status = MAK_OK;
    jb.err.clear();
    jb.attempt = 0;
    try {
      const int64_t N = jb.ps->N;
      CellPass& out = *jb.out;
      FaceStore& fst = out.fs();
      fst.fslot = face_slots(N);
      out.vol.ensure(size_t(N) * sizeof(double));
      out.mom.ensure(size_t(N) * 3 * sizeof(double));
      out.cflags.ensure(size_t(N) * sizeof(int32_t));
      out.nface.ensure(size_t(N) * sizeof(int32_t));
      out.retry.ensure(size_t(N) * 3 * sizeof(int32_t));
      out.counters.ensure(kCtrN * sizeof(unsigned long long));
      if (jb.opt.first_stage < 0 || jb.opt.first_stage >= nstage)
        MAK_FAIL(MAK_EINVAL, "first stage out of range");
      if (jb.opt.probe_n > 0 && (!jb.opt.probe_list || jb.opt.probe_n > N || jb.opt.faces ||
                                 !(jb.opt.doom_vol > 0)))
        MAK_FAIL(MAK_EINVAL, "a probe needs a cell list of at most N cells, no faces and doom_vol > 0");
      if (jb.opt.faces) {
        fst.faces.ensure(size_t(N) * fst.fslot * sizeof(FaceRec));
        fst.fbase.ensure(size_t(N) * sizeof(int64_t));
        if (fst.ovf_cap < 4096 + N / 8) fst.ovf_cap = 4096 + N / 8;
        fst.ovf.ensure(size_t(fst.ovf_cap) * sizeof(FaceRec));
      }
      job_begin(jb, st);
      live.push_back(&jb);
    } catch (const Error& e) {
      jb.status = e.status;
      jb.err = e.msg;
    }
  }
  // Rounds: every live job runs its current stage (one launch per stage and
  // up to kMaxJobs jobs), then the stage counters of all of them are read
  // back together and each job advances, finishes or restarts.
  while (!live.empty()) {
    for (int s = 0; s < nstage; ++s) {
      std::vector<PassJob*> grp;
      for (PassJob* jb : live)
        if (jb->stage == s) grp.push_back(jb);
      for (size_t k = 0; k < grp.size(); k += kMaxJobs)
        launch_stage(grp.data() + k, int(std::min<size_t>(kMaxJobs, grp.size() - k)), s, precision, st);
    }
    for (PassJob* jb : live)
      MAK_HIP(hipMemcpyAsync(jb->hc, jb->out->counters.p, sizeof(jb->hc), hipMemcpyDeviceToHost, st));
    MAK_HIP(hipStreamSynchronize(st));
    std::vector<PassJob*> next;
    for (PassJob* jb : live) {
      const int s = jb->stage;
      FaceStore& fst = jb->out->fs();
      try {
        if (jb->opt.faces && int64_t(jb->hc[0]) > fst.ovf_cap) {
          // the overflow region was too small: grow it and run the pass again
          if (++jb->attempt >= 3) MAK_FAIL(MAK_ENOMEM, "face overflow buffer could not be sized");
          fst.ovf_cap = int64_t(jb->hc[0]) + int64_t(jb->hc[0]) / 4 + 4096;
          fst.ovf.ensure(size_t(fst.ovf_cap) * sizeof(FaceRec));
          job_begin(*jb, st);
          next.push_back(jb);
          continue;
        }
        if (jb->hc[4] != 0) {  // a cell below doom_vol: the trial is rejected
          jb->cs.doomed = true;
          jb->cs.doom_cell = int64_t(jb->hc[5]);
          continue;
        }
        if (jb->opt.probe_n > 0) continue;  // a probe stops after its first stage
        const int64_t listed = int64_t(jb->hc[1 + s]);
        if (jb->all_cells) jb->cs.retried = listed;
        if (mixed && s == 0) jb->cs.fp64_rerun = listed;
        if (listed == 0) continue;  // finished
        if (s == nstage - 1) {
          jb->cs.overflow = listed;
          if (jb->opt.tolerate_failure) continue;
          unsigned long long cz[3];
          MAK_HIP(hipMemcpy(cz, jb->out->counters.as<unsigned long long>() + kCtrCause + 3 * s, sizeof(cz),
                            hipMemcpyDeviceToHost));
          MAK_FAIL(MAK_EOVERFLOW, std::to_string(cz[0]) + " cells exceeded the polytope capacity, " +
                                      std::to_string(cz[1]) + " had inconsistent cuts");
        }
        jb->listed = listed;
        jb->stage = s + 1;
        jb->all_cells = false;
        next.push_back(jb);
      } catch (const Error& e) {
        jb->status = e.status;
        jb->err = e.msg;
      }
    }
    live.swap(next);
  }
}

ClipStats run_cells(PointSet& ps, CellPass& out, const PassOpts& o, hipStream_t st) {
  PassJob jb;
  jb.ps = &ps;
  jb.out = &out;
  jb.opt = o;
  PassJob* one = &jb;
  run_cells_batch(&one, 1, o.precision, st);
  if (jb.status != MAK_OK) MAK_FAIL(jb.status, jb.err);
  return jb.cs;
}

}  // namespace mak
