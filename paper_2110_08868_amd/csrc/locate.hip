// Legendre transform of the weights and point location (Sec. 2, the equation
// after Eq. laguerrecell): for a query point q of the torus,
//
//   phi(q) = min over sites i and periodic images k of 1/2 |q - x_i - kL|^2 - psi_i,
//
// attained at i(q), the Laguerre cell that contains q.  With psi at the
// solution of the transport problem phi is the initial potential and
// x_{i(q)} + kL the position that the mass element at q is carried to.
//
// One thread per query.  The weights of converged solutions follow the
// displacement field, so their range spans many h^2 and a bound by the
// largest weight would reach far; the walk therefore prunes with the tilted
// bounds of the site grid (per block B a slope g_B and T_B with
// psi_j <= T_B + g_B . (x_j - c_B) for its sites, per cell the same T over
// the cell's sites).  Over the box of a block or cell the power distance is
// then at least
//   1/2 dist(q + g_B, box)^2 - 1/2 |g_B|^2 - g_B . (q - c_B) - T.
// The thread first scans the 27 cells around q + g of its own block (the
// predicted position of the site), then walks Chebyshev shells of blocks
// around the block of q: a block, and then each of its cells, is skipped when
// its bound cannot beat the best value found.  The walk stops before block
// shell r when every shell s >= r is out of reach by its untilted bound:
// distance >= (s - 1) bh + delta_b (delta_b = distance from q to the faces
// of its block) and weights <= the shell maximum of the block of q (s up to
// SHELL_MAX) or the global maximum (beyond).  Past r = Gb + 2 that distance
// exceeds L > sqrt(3) L / 2, which the global bound alone ends, so every
// thread's walk is finite.
//
// Mesh queries are generated in the kernel, 4 x 4 x 4 nodes per wavefront,
// so a wavefront's lanes walk nearly the same blocks; the bricks are dealt to
// the XCDs in contiguous ranges so neighbouring bricks share an L2.
#include <cfloat>
#include <cmath>

#include "../../include/mak.h"
#include "engine.h"
#include "gridkey.h"
#include "profile.h"

#pragma clang fp contract(fast)

namespace mak {
namespace {

constexpr int kLocBlock = 256;

struct LocArgs {
  const double4* pts;      // sorted sites: x, y, z, psi
  const int32_t* start;    // cell ranges [G + 1]
  const double* bsuf;      // per-block shell maxima [GB * (SHELL_MAX + 1)]
  const double* bg;        // per-block slope of the tilted bounds [GB * 3]
  const double* btmax;     // per-block tilted bound T [GB]
  const double* ctmax;     // per-cell tilted bound T (block's slope) [G]
  const double* scal;      // [0] global weight maximum
  const int32_t* perm;     // sorted -> original index
  const double* q;         // (Q, 3) query points, or NULL for the mesh
  int64_t Q;               // number of queries (mesh: ng^3)
  int64_t ng, nb;          // mesh nodes and 4-node bricks per axis
  int64_t nt;              // tiles of kTile^3 bricks per axis (mesh form)
  double mesh_h, mesh_off; // mesh spacing and node offset (in spacings)
  double L, h;
  int Gn, Gb;
  int64_t per_xcd;         // workgroups per XCD
  double* phi;             // [Q] or NULL
  int32_t* idx;            // [Q] or NULL
  double* disp;            // [Q, 3] or NULL
  int32_t* status;         // set to 1 by a query with a non-finite coordinate
};

__device__ __forceinline__ double wrap_coord(double v, double L) {
  v = fmod(v, L);
  if (v < 0) v += L;
  if (!(v < L) || !(v >= 0)) v = 0.0;
  return v;
}

// Half the squared length of d minus w, with explicit fused operations so
// that every kernel gets the same bits for the same candidate.
__device__ __forceinline__ double power_dist(double dx, double dy, double dz, double w) {
  return 0.5 * __fma_rn(dx, dx, __fma_rn(dy, dy, dz * dz)) - w;
}

// floor(u / n) for a cell or block coordinate u that may lie outside [0, n)
__device__ __forceinline__ int period_floor(int u, int n) { return u >= 0 ? u / n : -((n - 1 - u) / n); }

// The search for one query point (any coordinates): the minimum value, the
// sorted index of the minimising site (-1 only for an empty set) and
// x_site + kL - q.
struct LocHit {
  double best, dx, dy, dz;
  int32_t k;
};

__device__ __forceinline__ LocHit locate_one(const LocArgs& A, double qx, double qy, double qz) {
  const double L = A.L, h = A.h, bh = BLOCK_SIDE * h;
  qx = wrap_coord(qx, L);
  qy = wrap_coord(qy, L);
  qz = wrap_coord(qz, L);
  const int Gn = A.Gn, Gb = A.Gb;
  // rounding slack of the bounds (values are O(L^2))
  const double slack = 1e-12 * L * L;
  const int cx = cell_coord(qx, h, Gn), cy = cell_coord(qy, h, Gn), cz = cell_coord(qz, h, Gn);
  const int bx0 = cx >> 2, by0 = cy >> 2, bz0 = cz >> 2;
  double mb = fmin(fmin(qx - bx0 * bh, (bx0 + 1) * bh - qx),
                   fmin(fmin(qy - by0 * bh, (by0 + 1) * bh - qy), fmin(qz - bz0 * bh, (bz0 + 1) * bh - qz)));
  mb = fmax(mb - 1e-9 * h, 0.0);
  const int64_t b0 = block_key(bx0, by0, bz0, Gb);
  const double* suf = A.bsuf + b0 * (SHELL_MAX + 1);
  const double gmax = A.scal[0];

  double best = INFINITY, bx = 0, by = 0, bz = 0;
  int32_t bk = -1;
  auto scan = [&](int64_t key, double sx, double sy, double sz) {
    const int32_t s0 = A.start[key], s1 = A.start[key + 1];
    for (int32_t k = s0; k < s1; ++k) {
      const double4 p = A.pts[k];
      const double dx = p.x + sx - qx, dy = p.y + sy - qy, dz = p.z + sz - qz;
      const double v = power_dist(dx, dy, dz, p.w);
      if (v < best) {
        best = v;
        bk = k;
        bx = dx;
        by = dy;
        bz = dz;
      }
    }
  };

  // seed: the 27 cells around the predicted site position q + g (unwrapped
  // cell coordinates)
  int ex, ey, ez;
  {
    const double* g0 = A.bg + 3 * b0;
    ex = int(floor((qx + g0[0]) / h));
    ey = int(floor((qy + g0[1]) / h));
    ez = int(floor((qz + g0[2]) / h));
    for (int o = 0; o < 27; ++o) {
      const int ux = ex + o / 9 - 1, uy = ey + (o / 3) % 3 - 1, uz = ez + o % 3 - 1;
      const int sx = period_floor(ux, Gn), sy = period_floor(uy, Gn), sz = period_floor(uz, Gn);
      scan(cell_key(ux - sx * Gn, uy - sy * Gn, uz - sz * Gn, Gb), sx * L, sy * L, sz * L);
    }
  }

  // walk over block shells around the block of q
  for (int r = 0; r <= Gb + 2; ++r) {
    if (r > 0) {
      bool stop = true;
      for (int s = r; s <= SHELL_MAX && stop; ++s) {
        const double t = (s - 1) * bh + mb;
        stop = 0.5 * t * t - suf[s] - slack >= best;
      }
      if (stop) {
        const double t = (max(r, SHELL_MAX + 1) - 1) * bh + mb;
        stop = 0.5 * t * t - gmax - slack >= best;
      }
      if (stop) break;
    }
    for (int ox = -r; ox <= r; ++ox) {
      const bool xe = ox == -r || ox == r;
      for (int oy = -r; oy <= r; ++oy) {
        const bool ye = xe || oy == -r || oy == r;
        const int step = ye ? 1 : 2 * r;
        for (int oz = -r; oz <= r; oz += step) {
          const int ubx = bx0 + ox, uby = by0 + oy, ubz = bz0 + oz;
          const int sx = period_floor(ubx, Gb), sy = period_floor(uby, Gb), sz = period_floor(ubz, Gb);
          const int64_t bkey = block_key(ubx - sx * Gb, uby - sy * Gb, ubz - sz * Gb, Gb);
          const double gx = A.bg[3 * bkey], gy = A.bg[3 * bkey + 1], gz = A.bg[3 * bkey + 2];
          // q + g and the offset term, relative to the unwrapped block
          const double px = qx + gx, py = qy + gy, pz = qz + gz;
          const double lx = ubx * bh, ly = uby * bh, lz = ubz * bh;
          const double base = 0.5 * (gx * gx + gy * gy + gz * gz) +
                              (gx * (qx - lx - 0.5 * bh) + gy * (qy - ly - 0.5 * bh) +
                               gz * (qz - lz - 0.5 * bh)) + slack;
          const double dbx = fmax(fmax(lx - px, px - lx - bh), 0.0);
          const double dby = fmax(fmax(ly - py, py - ly - bh), 0.0);
          const double dbz = fmax(fmax(lz - pz, pz - lz - bh), 0.0);
          if (0.5 * (dbx * dbx + dby * dby + dbz * dbz) - base - A.btmax[bkey] >= best) continue;
          const double Lx = sx * L, Ly = sy * L, Lz = sz * L;
          for (int l = 0; l < 64; ++l) {
            const int ux = 4 * ubx + (l >> 4), uy = 4 * uby + ((l >> 2) & 3), uz = 4 * ubz + (l & 3);
            if (abs(ux - ex) <= 1 && abs(uy - ey) <= 1 && abs(uz - ez) <= 1) continue;  // seeded
            const int64_t key = bkey * 64 + l;
            const double cx0 = ux * h, cy0 = uy * h, cz0 = uz * h;
            const double dcx = fmax(fmax(cx0 - px, px - cx0 - h), 0.0);
            const double dcy = fmax(fmax(cy0 - py, py - cy0 - h), 0.0);
            const double dcz = fmax(fmax(cz0 - pz, pz - cz0 - h), 0.0);
            if (0.5 * (dcx * dcx + dcy * dcy + dcz * dcz) - base - A.ctmax[key] >= best) continue;
            scan(key, Lx, Ly, Lz);
          }
        }
      }
    }
  }
  return LocHit{best, bx, by, bz, bk};
}

// Item -> mesh node (a, b, c): bricks of 4 x 4 x 4 nodes per wavefront.
// False past the mesh.
__device__ __forceinline__ bool mesh_node(int64_t item, int64_t ng, int64_t nb, int64_t& a, int64_t& b,
                                          int64_t& c) {
  const int64_t brick = item >> 6;
  const int l = int(item & 63);
  if (brick >= nb * nb * nb) return false;
  a = 4 * (brick / (nb * nb)) + (l >> 4);
  b = 4 * ((brick / nb) % nb) + ((l >> 2) & 3);
  c = 4 * (brick % nb) + (l & 3);
  return a < ng && b < ng && c < ng;
}

// Workgroup -> item, contiguous ranges per XCD; -1 past the grid.
__device__ __forceinline__ int64_t xcd_item(int64_t per_xcd) {
  const int64_t wg = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
  if ((wg >> 3) >= per_xcd) return -1;
  return ((wg & 7) * per_xcd + (wg >> 3)) * kLocBlock + threadIdx.x;
}

__global__ __launch_bounds__(kLocBlock) void k_locate(LocArgs A) {
  const int64_t item = xcd_item(A.per_xcd);
  if (item < 0) return;
  double qx, qy, qz;
  int64_t out;
  if (A.q) {
    if (item >= A.Q) return;
    out = item;
    qx = A.q[3 * item];
    qy = A.q[3 * item + 1];
    qz = A.q[3 * item + 2];
    if (!(isfinite(qx) && isfinite(qy) && isfinite(qz))) atomicOr(A.status, 1);
  } else {
    int64_t a, b, c;
    if (!mesh_node(item, A.ng, A.nb, a, b, c)) return;
    out = (a * A.ng + b) * A.ng + c;
    qx = (double(a) + A.mesh_off) * A.mesh_h;
    qy = (double(b) + A.mesh_off) * A.mesh_h;
    qz = (double(c) + A.mesh_off) * A.mesh_h;
  }
  const LocHit r = locate_one(A, qx, qy, qz);
  if (A.phi) A.phi[out] = r.best;
  if (A.idx) A.idx[out] = r.k >= 0 ? A.perm[r.k] : -1;
  if (A.disp) {
    A.disp[3 * out] = r.dx;
    A.disp[3 * out + 1] = r.dy;
    A.disp[3 * out + 2] = r.dz;
  }
}

struct DepArgs {
  double tau;                 // growth amplitude of the Zel'dovich step, in [0, 1]
  double H;                   // Eulerian mesh spacing
  int64_t ne;                 // Eulerian nodes per axis
  int scheme;                 // 1: nearest grid point, 2: cloud in cell
  unsigned long long U;       // fixed-point units carried by one mass element
  unsigned long long* acc;    // [ne^3] accumulated units
};

__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t n) {
  i %= n;
  return i < 0 ? i + n : i;
}


// Move the mass element at q by tau (its displacement) and hand its U units
// to `add(node, units)`: all to the nearest node (NGP) or split over the 8
// nodes around y with the trilinear weights (CIC), rounded to units with the
// remainder on the heaviest node so each element adds exactly U.  Integer
// sums are exact and independent of the order of the additions.
template <class Add>
__device__ __forceinline__ void deposit_element(const DepArgs& D, double L, double qx, double qy, double qz,
                                                double dx, double dy, double dz, Add&& add) {
  const double yx = wrap_coord(qx + D.tau * dx, L), yy = wrap_coord(qy + D.tau * dy, L),
               yz = wrap_coord(qz + D.tau * dz, L);
  const double ux = yx / D.H, uy = yy / D.H, uz = yz / D.H;
  const int64_t ne = D.ne;
  if (D.scheme == 1) {
    const int64_t ix = wrap_index(int64_t(floor(ux + 0.5)), ne), iy = wrap_index(int64_t(floor(uy + 0.5)), ne),
                  iz = wrap_index(int64_t(floor(uz + 0.5)), ne);
    add((ix * ne + iy) * ne + iz, D.U);
    return;
  }
  const double fx0 = floor(ux), fy0 = floor(uy), fz0 = floor(uz);
  const double fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
  const int64_t ix = int64_t(fx0), iy = int64_t(fy0), iz = int64_t(fz0);
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
  unsigned long long u[8];
  unsigned long long sum = 0;
  int heavy = 0;
  double wmax = -1.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const double w = wx[t >> 2] * wy[(t >> 1) & 1] * wz[t & 1];
    u[t] = (unsigned long long)(w * double(D.U) + 0.5);
    sum += u[t];
    if (w > wmax) {
      wmax = w;
      heavy = t;
    }
  }
  // the heaviest node takes the remainder (its weight is >= 1/8, far above
  // the rounding of the others)
#pragma unroll
  for (int t = 0; t < 8; ++t)
    if (t == heavy) u[t] = D.U - (sum - u[t]);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (u[t] == 0) continue;
    const int64_t jx = wrap_index(ix + (t >> 2), ne), jy = wrap_index(iy + ((t >> 1) & 1), ne),
                  jz = wrap_index(iz + (t & 1), ne);
    add((jx * ne + jy) * ne + jz, u[t]);
  }
}

// Mesh queries, one wavefront per 4 x 4 x 4 brick of nodes (a lane per
// node): the lanes walk the same blocks together.  Around the box of blocks
// that holds the brick the wave visits shells of blocks; each lane tests a
// block with its own tilted bound, and when some lane needs it the wave
// stages the block's cells that could serve any of the needing lanes (a
// tilted bound over the box of their queries, against the largest of their
// best values) into LDS, kStage sites at a time, and every lane evaluates
// all staged sites.  A lane stops needing blocks at shell r under the same
// test as the per-thread walk (every block at Chebyshev distance >= r from
// its own block is out of reach); the walk ends when all lanes have
// stopped.  The minimum is the same as the per-thread walk's (the same
// candidate values, and a minimum does not depend on the order); only ties
// may pick another site.  DEP: then deposit the element (Zel'dovich step).
constexpr int kStage = 256;
constexpr int64_t kTile = 4;  // bricks per tile side in the mesh form's order
// the deposit's per-brick hash table of node sums (in the site stage)
constexpr int kHashBits = 9;
constexpr int kHashSlots = 1 << kHashBits;
static_assert(kHashSlots >= 8 * 64, "a brick's 64 elements add to at most 512 nodes");
static_assert(kHashSlots * (8 + 8) <= kStage * 32, "the table fits in the site stage");

template <bool DEP>
__global__ __launch_bounds__(64) void k_mesh_coop(LocArgs A, DepArgs D) {
  __shared__ double4 site[kStage];
  __shared__ int32_t sidx[kStage];
  __shared__ int32_t cst[64], cpre[64];
  const int lane = threadIdx.x;
  const int64_t wg = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
  if ((wg >> 3) >= A.per_xcd) return;
  // bricks in tiles of kTile^3 (tiles x-major, bricks x-major within a
  // tile): the bricks an XCD runs at once form a compact region, whose blocks
  // its L2 then serves to the neighbouring bricks
  const int64_t item = (wg & 7) * A.per_xcd + (wg >> 3);
  const int64_t nb = A.nb, nt = A.nt;
  const int64_t tile = item / (kTile * kTile * kTile), in = item % (kTile * kTile * kTile);
  if (tile >= nt * nt * nt) return;
  const int64_t bxi = kTile * (tile / (nt * nt)) + in / (kTile * kTile);
  const int64_t byi = kTile * ((tile / nt) % nt) + (in / kTile) % kTile;
  const int64_t bzi = kTile * (tile % nt) + in % kTile;
  if (bxi >= nb || byi >= nb || bzi >= nb) return;
  const int64_t a = 4 * bxi + (lane >> 4);
  const int64_t b = 4 * byi + ((lane >> 2) & 3);
  const int64_t c = 4 * bzi + (lane & 3);
  const bool valid = a < A.ng && b < A.ng && c < A.ng;
  const double L = A.L, h = A.h, bh = BLOCK_SIDE * h;
  const double q0x = (double(a) + A.mesh_off) * A.mesh_h, q0y = (double(b) + A.mesh_off) * A.mesh_h,
               q0z = (double(c) + A.mesh_off) * A.mesh_h;
  const double qx = wrap_coord(q0x, L), qy = wrap_coord(q0y, L), qz = wrap_coord(q0z, L);
  const int Gn = A.Gn, Gb = A.Gb;
  const double slack = 1e-12 * L * L;
  const int bx0 = cell_coord(qx, h, Gn) >> 2, by0 = cell_coord(qy, h, Gn) >> 2, bz0 = cell_coord(qz, h, Gn) >> 2;
  double mb = fmin(fmin(qx - bx0 * bh, (bx0 + 1) * bh - qx),
                   fmin(fmin(qy - by0 * bh, (by0 + 1) * bh - qy), fmin(qz - bz0 * bh, (bz0 + 1) * bh - qz)));
  mb = fmax(mb - 1e-9 * h, 0.0);
  const double* suf = A.bsuf + block_key(bx0, by0, bz0, Gb) * (SHELL_MAX + 1);
  const double gmax = A.scal[0];
  // the box of blocks of the brick's nodes
  const double big = 1e300;
  const int Bx0 = int(-wave_max_d(valid ? -double(bx0) : -big)), Bx1 = int(wave_max_d(valid ? double(bx0) : -big));
  const int By0 = int(-wave_max_d(valid ? -double(by0) : -big)), By1 = int(wave_max_d(valid ? double(by0) : -big));
  const int Bz0 = int(-wave_max_d(valid ? -double(bz0) : -big)), Bz1 = int(wave_max_d(valid ? double(bz0) : -big));

  double best = INFINITY, bdx = 0, bdy = 0, bdz = 0;
  int32_t bk = -1;
  bool done = !valid;
  for (int r = 0; r <= Gb + 2; ++r) {
    if (r > 0 && !done) {
      bool stop = true;
      for (int s2 = r; s2 <= SHELL_MAX && stop; ++s2) {
        const double t = (s2 - 1) * bh + mb;
        stop = 0.5 * t * t - suf[s2] - slack >= best;
      }
      if (stop) {
        const double t = (max(r, SHELL_MAX + 1) - 1) * bh + mb;
        stop = 0.5 * t * t - gmax - slack >= best;
      }
      done = stop;
    }
    if (ballot(!done) == 0) break;
    const int x0 = Bx0 - r, x1 = Bx1 + r, y0 = By0 - r, y1 = By1 + r, z0 = Bz0 - r, z1 = Bz1 + r;
    for (int ubx = x0; ubx <= x1; ++ubx) {
      const bool xe = r == 0 || ubx == x0 || ubx == x1;
      for (int uby = y0; uby <= y1; ++uby) {
        const bool ye = xe || uby == y0 || uby == y1;
        const int zstep = ye ? 1 : z1 - z0;
        for (int ubz = z0; ubz <= z1; ubz += zstep) {
          const int sx = period_floor(ubx, Gb), sy = period_floor(uby, Gb), sz = period_floor(ubz, Gb);
          const int64_t bkey = block_key(ubx - sx * Gb, uby - sy * Gb, ubz - sz * Gb, Gb);
          const double gx = A.bg[3 * bkey], gy = A.bg[3 * bkey + 1], gz = A.bg[3 * bkey + 2];
          const double lx = ubx * bh, ly = uby * bh, lz = ubz * bh;
          const double cx = lx + 0.5 * bh, cy = ly + 0.5 * bh, cz = lz + 0.5 * bh;
          const double g2 = 0.5 * (gx * gx + gy * gy + gz * gz);
          bool need = false;
          if (!done) {
            const double px = qx + gx, py = qy + gy, pz = qz + gz;
            const double base = g2 + (gx * (qx - cx) + gy * (qy - cy) + gz * (qz - cz)) + slack;
            const double dbx = fmax(fmax(lx - px, px - lx - bh), 0.0);
            const double dby = fmax(fmax(ly - py, py - ly - bh), 0.0);
            const double dbz = fmax(fmax(lz - pz, pz - lz - bh), 0.0);
            need = 0.5 * (dbx * dbx + dby * dby + dbz * dbz) - base - A.btmax[bkey] < best;
          }
          if (ballot(need) == 0) continue;
          // the box of the needing lanes' queries and their largest best
          const double qlx = -wave_max_d(need ? -qx : -big), qhx = wave_max_d(need ? qx : -big);
          const double qly = -wave_max_d(need ? -qy : -big), qhy = wave_max_d(need ? qy : -big);
          const double qlz = -wave_max_d(need ? -qz : -big), qhz = wave_max_d(need ? qz : -big);
          const double bmax = wave_max_d(need ? best : -big);
          // cell `lane` of the block
          const int ux = 4 * ubx + (lane >> 4), uy = 4 * uby + ((lane >> 2) & 3), uz = 4 * ubz + (lane & 3);
          const int64_t key = bkey * 64 + lane;
          const int32_t s0 = A.start[key], cnt = A.start[key + 1] - s0;
          bool has = cnt > 0;
          if (has) {
            const double clx = ux * h, cly = uy * h, clz = uz * h;
            const double gpx = fmax(fmax(clx - (qhx + gx), (qlx + gx) - clx - h), 0.0);
            const double gpy = fmax(fmax(cly - (qhy + gy), (qly + gy) - cly - h), 0.0);
            const double gpz = fmax(fmax(clz - (qhz + gz), (qlz + gz) - clz - h), 0.0);
            const double gq = fmax(gx * (qlx - cx), gx * (qhx - cx)) + fmax(gy * (qly - cy), gy * (qhy - cy)) +
                              fmax(gz * (qlz - cz), gz * (qhz - cz));
            has = 0.5 * (gpx * gpx + gpy * gpy + gpz * gpz) - g2 - gq - A.ctmax[key] - slack < bmax;
          }
          const uint64_t am = ballot(has);
          if (am == 0) continue;
          const int ncl = __popcll(am);
          const int cn = has ? cnt : 0;
          const int incl = wave_incl_scan_i(cn);
          const int total = readlane_i(incl, 63);
          if (has) {
            const int idx = lanes_below(am);
            cst[idx] = s0;
            cpre[idx] = incl - cn;
          }
          __syncthreads();
          const double Lx = sx * L, Ly = sy * L, Lz = sz * L;
          for (int base0 = 0; base0 < total; base0 += kStage) {
            const int m = min(kStage, total - base0);
            for (int t = lane; t < m; t += 64) {
              const int tt = base0 + t;
              int lo = 0, hi = ncl - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (cpre[mid] <= tt) lo = mid; else hi = mid - 1;
              }
              const int32_t k = cst[lo] + (tt - cpre[lo]);
              const double4 P = A.pts[k];
              site[t] = make_double4(P.x + Lx, P.y + Ly, P.z + Lz, P.w);
              sidx[t] = k;
            }
            __syncthreads();
            if (need) {
              for (int t = 0; t < m; ++t) {
                const double4 P = site[t];
                const double dx = P.x - qx, dy = P.y - qy, dz = P.z - qz;
                const double v = power_dist(dx, dy, dz, P.w);
                if (v < best) {
                  best = v;
                  bk = sidx[t];
                  bdx = dx;
                  bdy = dy;
                  bdz = dz;
                }
              }
            }
            __syncthreads();
          }
        }
      }
    }
  }
  if (DEP) {
    // The brick's elements reach few nodes (on the clustered 128^3 solution
    // at tau = 0.5, 137 distinct nodes for its 512 cloud-in-cell shares on
    // average): their units are summed per node in an LDS hash table (the
    // idle site stage: 512 slots, enough for any brick), then each node
    // present gets one global atomic.
    constexpr unsigned long long kEmpty = ~0ull;
    unsigned long long* hkey = reinterpret_cast<unsigned long long*>(site);
    unsigned long long* hval = hkey + kHashSlots;
    __syncthreads();
    for (int i = lane; i < kHashSlots; i += 64) {
      hkey[i] = kEmpty;
      hval[i] = 0ull;
    }
    __syncthreads();
    if (valid)
      deposit_element(D, L, qx, qy, qz, bdx, bdy, bdz, [&](int64_t node, unsigned long long units) {
        const unsigned long long key = (unsigned long long)node;
        uint32_t slot = (uint32_t(key ^ (key >> 32)) * 2654435761u) >> (32 - kHashBits);
        for (;;) {
          const unsigned long long prev = atomicCAS(&hkey[slot], kEmpty, key);
          if (prev == kEmpty || prev == key) {
            atomicAdd(&hval[slot], units);
            break;
          }
          slot = (slot + 1) & (kHashSlots - 1);
        }
      });
    __syncthreads();
    for (int i = lane; i < kHashSlots; i += 64)
      if (hkey[i] != kEmpty && hval[i] != 0ull) atomicAdd(&D.acc[hkey[i]], hval[i]);
    return;
  }
  if (!valid) return;
  {
    const int64_t out = (a * A.ng + b) * A.ng + c;
    if (A.phi) A.phi[out] = best;
    if (A.idx) A.idx[out] = bk >= 0 ? A.perm[bk] : -1;
    if (A.disp) {
      A.disp[3 * out] = bdx;
      A.disp[3 * out + 1] = bdy;
      A.disp[3 * out + 2] = bdz;
    }
  }
}

__global__ void k_units_to_density(const unsigned long long* __restrict__ acc, double scale,
                                   double* __restrict__ rho, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) rho[i] = double(acc[i]) * scale;
}

}  // namespace

namespace {

LocArgs loc_args(const PointSet& ps) {
  LocArgs a{};
  a.pts = ps.pts.as<double4>();
  a.start = ps.cell_start.as<int32_t>();
  a.bsuf = ps.block_suffix.as<double>();
  a.bg = ps.block_g.as<double>();
  a.btmax = ps.block_tmax.as<double>();
  a.ctmax = ps.cell_tmax.as<double>();
  a.scal = ps.scal.as<double>();
  a.perm = ps.perm.as<int32_t>();
  a.L = ps.g.L;
  a.h = ps.g.h;
  a.Gn = ps.g.Gn;
  a.Gb = ps.g.Gb;
  return a;
}

void set_mesh(LocArgs& a, int64_t ng, double offset) {
  a.ng = ng;
  a.nb = ceil_div(ng, 4);
  a.nt = ceil_div(a.nb, kTile);
  a.Q = ng * ng * ng;
  a.mesh_h = a.L / double(ng);
  a.mesh_off = offset;
}

// Grid of one 64-lane workgroup per 4^3-node brick of the mesh (the bricks
// of whole tiles, those past the mesh returning at once), dealt to the XCDs
// in contiguous ranges (2-D above 65536 workgroups).
dim3 brick_grid(LocArgs& a) {
  const int64_t bricks = a.nt * a.nt * a.nt * kTile * kTile * kTile;
  a.per_xcd = ceil_div(bricks, 8);
  const int64_t total = 8 * a.per_xcd;
  const int64_t gx = total < 65536 ? total : 65536;
  const int64_t gy = ceil_div(total, gx);
  if (gy > 65535) MAK_FAIL(MAK_EINVAL, "mesh too large for one launch");
  return dim3(unsigned(gx), unsigned(gy));
}

// Grid of `threads` items in workgroups of kLocBlock, dealt to the XCDs in
// contiguous ranges (2-D above 65536 workgroups).
dim3 xcd_grid(LocArgs& a, int64_t threads) {
  const int64_t wgs = ceil_div(threads, kLocBlock);
  a.per_xcd = ceil_div(wgs, 8);
  const int64_t total = 8 * a.per_xcd;
  const int64_t gx = total < 65536 ? total : 65536;
  const int64_t gy = ceil_div(total, gx);
  if (gy > 65535) MAK_FAIL(MAK_EINVAL, "too many query points for one launch");
  return dim3(unsigned(gx), unsigned(gy));
}

}  // namespace

void locate(const PointSet& ps, const double* queries, int64_t Q, int64_t ng, double offset,
            double* phi, int32_t* idx, double* disp, DevBuf& status, hipStream_t st) {
  LocArgs a = loc_args(ps);
  status.ensure(sizeof(int32_t));
  a.status = status.as<int32_t>();
  a.q = queries;
  a.phi = phi;
  a.idx = idx;
  a.disp = disp;
  int64_t threads;
  if (queries) {
    a.Q = Q;
    threads = Q;
  } else {
    set_mesh(a, ng, offset);
    threads = a.nb * a.nb * a.nb * 64;
  }
  if (a.Q == 0) return;
  if (queries) fill_zero_i32(a.status, 1, st);
  const dim3 grid = queries ? xcd_grid(a, threads) : brick_grid(a);
  ProfScope scope("locate", st, double(a.Q), double(a.Q) * (phi ? 8 : 0) + double(a.Q) * (idx ? 4 : 0) +
                                                 double(a.Q) * (disp ? 24 : 0) +
                                                 double(a.Q) * (queries ? 24 : 0) +
                                                 double(ps.N) * sizeof(double4));
  if (queries)
    hipLaunchKernelGGL(k_locate, grid, dim3(kLocBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_mesh_coop<false>, grid, dim3(64), 0, st, a, DepArgs{});
  MAK_HIP(hipGetLastError());
  scope.stop();
  if (queries) {
    int32_t hs = 0;
    MAK_HIP(hipMemcpyAsync(&hs, a.status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MAK_HIP(hipStreamSynchronize(st));
    if (hs) MAK_FAIL(MAK_EINVAL, "non-finite query coordinate");
  }
}

void za_deposit(const PointSet& ps, double tau, int64_t n_lag, double lag_offset, int64_t ne, int scheme,
                double* density, DevBuf& acc, hipStream_t st) {
  LocArgs a = loc_args(ps);
  set_mesh(a, n_lag, lag_offset);
  const dim3 grid = brick_grid(a);
  const int64_t n_e = ne * ne * ne;
  DepArgs d{};
  d.tau = tau;
  d.H = ps.g.L / double(ne);
  d.ne = ne;
  d.scheme = scheme;
  // units per element: the total over all elements stays below 2^62
  int bits = 0;
  while ((int64_t(1) << bits) < a.Q) ++bits;
  int ub = 62 - bits;
  if (ub > 52) ub = 52;
  d.U = 1ull << ub;
  acc.ensure(size_t(n_e) * sizeof(unsigned long long));
  d.acc = acc.as<unsigned long long>();
  MAK_HIP(hipMemsetAsync(d.acc, 0, size_t(n_e) * sizeof(unsigned long long), st));
  {
    ProfScope scope("deposit", st, double(a.Q), double(ps.N) * sizeof(double4) + double(n_e) * 16);
    hipLaunchKernelGGL(k_mesh_coop<true>, grid, dim3(64), 0, st, a, d);
    MAK_HIP(hipGetLastError());
  }
  // element mass (L / n_lag)^3 over U units, per Eulerian cell volume H^3
  const double m_el = std::pow(ps.g.L / double(n_lag), 3);
  const double scale = m_el / double(d.U) / (d.H * d.H * d.H);
  hipLaunchKernelGGL(k_units_to_density, dim3(unsigned(ceil_div(n_e, 256))), dim3(256), 0, st, d.acc,
                     scale, density, n_e);
  MAK_HIP(hipGetLastError());
}

}  // namespace mak
