// Exact Eulerian deposit of the cells moved by the Zel'dovich step (Sec. 2,
// closing paragraph, and Fig. 1): at growth amplitude tau the mass element at
// q moves to q + tau (x_i - q), so the cell V_i becomes the polytope
// S_i = x_i + (1 - tau)(V_i - x_i), which carries the cell's mass |V_i| at
// density 1 / (1 - tau)^3 (initial density 1).  The mass in the voxel
// [a H - H/2, a H + H/2)^3 of Eulerian node a is the volume of S_i inside it
// over (1 - tau)^3, summed over the cells; 0 <= tau < 1.
//
// One wavefront per cell.  The cell's planes come from the face records of a
// float64 cell pass: u . d <= b with d = x_j + sL - x_i and
// b = |d|^2/2 + psi_i - psi_j (u seed-local), scaled to u . d <= (1 - tau) b,
// plus the box of the site's own images, |u_a| <= (1 - tau) L / 2.  A
// polytope is held in LDS as face polygons, one face per lane, the vertices
// of all faces packed in one pool per polytope.  Clipping by a plane: every
// lane cuts its polygon Sutherland-Hodgman style (the crossing point of an
// edge is evaluated from its inside end and the side tests use explicit
// FMAs, so the two faces sharing an edge produce the same bits; a vertex
// within 1e-14 L of the plane counts as on it, so lattice inputs whose faces
// fall on voxel boundaries cut cleanly), the surviving polygons are
// compacted, the crossing points are gathered (each face's exit point alone
// when no vertex lies on the plane, else all of them, duplicates dropped), and
// the new face is their polygon ordered by angle about their centroid.  S_i is clipped out of its box once; then it is cut
// into the slabs of voxel columns along x, each slab into the columns along
// y, and a column's voxels are the differences of the volumes below the
// successive z boundaries (fans from the first vertex of each face, apex at
// the site).  Masses are summed in 64-bit fixed point (unit L^3 2^-60), so
// every run gives the same bits; the rounding is at most half a unit per
// cell and voxel.
#include <cmath>

#include "../../include/mak.h"
#include "engine.h"
#include "profile.h"

namespace mak {
namespace {

constexpr int kMaxF = 64;        // faces of a polytope (one per lane)
constexpr int kPool = 400;       // face corners of a polytope (Euler: at most 6 F - 12 = 372 for F = 64 faces)
constexpr int kBuf = 4;          // polytopes held: the moved cell, a temporary, a slab, a column
constexpr int kMaxPlanes = 128;  // planes of a cell (faces + 6 box planes)
constexpr int kCap = 4;          // points of one face on a cutting plane
// side values within kSnap L |n| of zero count as on the plane (rounding of
// vertices that lie on it, e.g. lattice sites against voxel boundaries)
constexpr double kSnap = 1e-14;

struct DepCellArgs {
  const double4* pts;
  const FaceRec* faces;
  const FaceRec* ovf;
  const int64_t* fbase;
  int32_t fslot;
  const int32_t* nface;
  const double* vol;        // cell volumes of the pass
  int64_t n;
  double L, tau, H;
  int64_t ng;
  double unit;              // mass of one fixed-point unit
  unsigned long long* acc;  // [ng^3]
  unsigned int* status;     // 1: a cell exceeded the polytope capacity or cut degenerately
  int64_t per_xcd;
};

struct PolyLDS {
  double vx[kBuf][kPool], vy[kBuf][kPool], vz[kBuf][kPool];
  double px[kMaxPlanes], py[kMaxPlanes], pz[kMaxPlanes], pb[kMaxPlanes];
  double cx[kCap * kMaxF], cy[kCap * kMaxF], cz[kCap * kMaxF];  // crossing points, then their angles
  int32_t off[kBuf][kMaxF], nvs[kBuf][kMaxF];          // each face's vertices in the pool
  int32_t nfc[kBuf];                                   // faces of each polytope
};

__device__ __forceinline__ double side(double x, double y, double z, double nx, double ny, double nz,
                                       double b) {
  return fma(x, nx, fma(y, ny, z * nz)) - b;
}

// A strictly increasing function of the angle of (x, y) in [0, 2 pi), with
// values in [0, 4): the position along the unit diamond |x| + |y| = 1 (one
// division instead of an arctangent; only the order is used).
__device__ __forceinline__ double pseudo_angle(double x, double y) {
  const double s = fabs(x) + fabs(y);
  if (!(s > 0.0)) return 0.0;
  const double t = y / s;  // sin-like coordinate in [-1, 1]
  return x >= 0.0 ? (y >= 0.0 ? t : 4.0 + t) : 2.0 - t;
}

// Corners of the six faces of a box, counter-clockwise seen from outside:
// four 3-bit codes (x << 2 | y << 1 | z, 1 = high side) per face.
__device__ __forceinline__ uint32_t box_face_code(int f) {
  switch (f) {
    case 0: return 0x5764u;   // +x
    case 1: return 0x2310u;   // -x
    case 2: return 0x6732u;   // +y
    case 3: return 0x1540u;   // -y
    case 4: return 0x3751u;   // +z
    default: return 0x4620u;  // -z
  }
}

__global__ __launch_bounds__(64) void k_cells_deposit(DepCellArgs A) {
  __shared__ PolyLDS S;
  const int lane = threadIdx.x;
  const int64_t wg = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;
  if ((wg >> 3) >= A.per_xcd) return;
  const int64_t p = (wg & 7) * A.per_xcd + (wg >> 3);
  if (p >= A.n || !(A.vol[p] > 0.0)) return;
  const double L = A.L, sc = 1.0 - A.tau, H = A.H;
  const int64_t ng = A.ng;
  const double4 me = A.pts[p];

  // the cell's planes, scaled to the moved cell (records of the site's own
  // images, if any, are covered by the box planes)
  const int32_t nf = A.nface[p];
  const FaceRec* fr = nf > A.fslot ? A.ovf + A.fbase[p] : A.faces + p * int64_t(A.fslot);
  int npl = 6;
  for (int base = 0; base < nf; base += 64) {
    const int f = base + lane;
    FaceRec r{};
    if (f < nf) r = fr[f];
    const bool use = f < nf && int64_t(r.j) != p;
    const uint64_t m = ballot(use);
    const int slot = npl + __popcll(m & ((uint64_t(1) << lane) - 1));
    if (use && slot < kMaxPlanes) {
      const double4 P = A.pts[r.j];
      const double dx = P.x + unpack_shift(r.shift, 0) * L - me.x;
      const double dy = P.y + unpack_shift(r.shift, 1) * L - me.y;
      const double dz = P.z + unpack_shift(r.shift, 2) * L - me.z;
      S.px[slot] = dx;
      S.py[slot] = dy;
      S.pz[slot] = dz;
      S.pb[slot] = sc * (0.5 * (dx * dx + dy * dy + dz * dz) + me.w - P.w);
    }
    npl += __popcll(m);
  }
  if (npl > kMaxPlanes) {
    if (lane == 0) atomicOr(A.status, 1u);
    return;
  }
  if (lane < 6) {
    const double sgn = (lane & 1) ? -1.0 : 1.0;
    S.px[lane] = (lane >> 1) == 0 ? sgn : 0.0;
    S.py[lane] = (lane >> 1) == 1 ? sgn : 0.0;
    S.pz[lane] = (lane >> 1) == 2 ? sgn : 0.0;
    S.pb[lane] = 0.5 * sc * L;
  }
  __syncthreads();

  bool bad = false;  // capacity exceeded or degenerate cut (wave-uniform after each clip)

  // the box [l, h] (seed-local) as six faces into polytope d
  auto init_box = [&](int d, double lx, double ly, double lz, double hx, double hy, double hz) {
    if (lane < 6) {
      const uint32_t code = box_face_code(lane);
      for (int k = 0; k < 4; ++k) {
        const uint32_t c = (code >> (4 * k)) & 7u;
        S.vx[d][4 * lane + k] = (c & 4u) ? hx : lx;
        S.vy[d][4 * lane + k] = (c & 2u) ? hy : ly;
        S.vz[d][4 * lane + k] = (c & 1u) ? hz : lz;
      }
      S.off[d][lane] = 4 * lane;
      S.nvs[d][lane] = 4;
    }
    if (lane == 0) S.nfc[d] = 6;
    __syncthreads();
  };

  // Polytope src clipped by u . n <= b.  Returns src when nothing of it is
  // outside (unchanged), else d holding the clipped polytope, or -1 when
  // nothing of volume is left.  src != d.
  auto clip = [&](int src, int d, double nx, double ny, double nz, double b) -> int {
    const int nfc = S.nfc[src];
    const int nv = lane < nfc ? S.nvs[src][lane] : 0;
    const int o = lane < nfc ? S.off[src][lane] : 0;
    const double* X = &S.vx[src][o];
    const double* Y = &S.vy[src][o];
    const double* Z = &S.vz[src][o];
    const double tol = kSnap * A.L * sqrt(nx * nx + ny * ny + nz * nz);
    auto sd = [&](double x, double y, double z) {
      const double v = side(x, y, z, nx, ny, nz, b);
      return fabs(v) <= tol ? 0.0 : v;
    };
    // pass 1: how many vertices each face keeps
    int m = 0;
    bool out = false, on_all = nv > 0, zero = false;
    if (nv > 0) {
      const double s0 = sd(X[0], Y[0], Z[0]);
      double sp = s0;
      for (int k = 0; k < nv; ++k) {
        const int k2 = k + 1 < nv ? k + 1 : 0;
        const double sq = k2 ? sd(X[k2], Y[k2], Z[k2]) : s0;
        m += int(sp <= 0.0) + int((sp < 0.0 && sq > 0.0) || (sp > 0.0 && sq < 0.0));
        out = out || sp > 0.0;
        on_all = on_all && sp == 0.0;
        zero = zero || sp == 0.0;
        sp = sq;
      }
    }
    if (ballot(out) == 0) return src;
    // No vertex on the plane: every crossing point is the exit (inside to
    // outside, in traversal order) of exactly one face and the entry of the
    // face across its edge, so the exits alone list the new face's corners
    // once each and need no deduplication.
    const bool generic = ballot(zero) == 0;
    // a face lying in the plane is dropped: the new face replaces it
    const bool live = m >= 3 && !on_all;
    const int dest = wave_incl_scan_i(live ? 1 : 0) - (live ? 1 : 0);
    const int nlive = __popcll(ballot(live));
    const int wincl = wave_incl_scan_i(live ? m : 0);
    const int total = readlane_i(wincl, 63);
    const int wo = wincl - (live ? m : 0);
    const bool fits = total <= kPool;
    if (!fits) bad = true;
    // pass 2: the clipped polygons, compacted, and the crossing points
    int ncap = 0, w = 0;
    double qx[kCap] = {0, 0, 0, 0}, qy[kCap] = {0, 0, 0, 0}, qz[kCap] = {0, 0, 0, 0};
    auto add_cap = [&](double x, double y, double z) {
#pragma unroll
      for (int c = 0; c < kCap; ++c)
        if (c < ncap && x == qx[c] && y == qy[c] && z == qz[c]) return;
#pragma unroll
      for (int c = 0; c < kCap; ++c)
        if (c == ncap) {
          qx[c] = x;
          qy[c] = y;
          qz[c] = z;
        }
      ++ncap;
    };
    auto push = [&](double x, double y, double z) {
      if (live && fits) {
        S.vx[d][wo + w] = x;
        S.vy[d][wo + w] = y;
        S.vz[d][wo + w] = z;
      }
      ++w;
    };
    if (nv > 0 && !on_all) {
      for (int k = 0; k < nv; ++k) {
        const int k2 = k + 1 < nv ? k + 1 : 0;
        const double Px = X[k], Py = Y[k], Pz = Z[k];
        const double Qx = X[k2], Qy = Y[k2], Qz = Z[k2];
        const double sP = sd(Px, Py, Pz), sQ = sd(Qx, Qy, Qz);
        if (sP <= 0.0) {
          push(Px, Py, Pz);
          if (sP == 0.0) add_cap(Px, Py, Pz);
        }
        if (sP < 0.0 && sQ > 0.0) {
          const double t = sP / (sP - sQ);
          const double Xx = fma(Qx - Px, t, Px), Xy = fma(Qy - Py, t, Py), Xz = fma(Qz - Pz, t, Pz);
          push(Xx, Xy, Xz);
          add_cap(Xx, Xy, Xz);
        } else if (sP > 0.0 && sQ < 0.0) {
          const double t = sQ / (sQ - sP);
          const double Xx = fma(Px - Qx, t, Qx), Xy = fma(Py - Qy, t, Qy), Xz = fma(Pz - Qz, t, Qz);
          push(Xx, Xy, Xz);
          if (!generic) add_cap(Xx, Xy, Xz);
        }
      }
    }
    // (a convex face meets a plane in a segment: two points, more only when
    // vertices of the face lie on the plane between them)
    if (ncap > kCap) bad = true;
    if (live) {
      S.off[d][dest] = wo;
      S.nvs[d][dest] = m;
    }
    // gather the crossing points
    const int nc = ncap > kCap ? kCap : ncap;
    const int incl = wave_incl_scan_i(nc);
    const int tot = readlane_i(incl, 63);
#pragma unroll
    for (int c = 0; c < kCap; ++c)
      if (c < nc) {
        S.cx[incl - nc + c] = qx[c];
        S.cy[incl - nc + c] = qy[c];
        S.cz[incl - nc + c] = qz[c];
      }
    __syncthreads();
    // the first occurrence of each point (kCap entries per lane)
    bool keep[kCap] = {false, false, false, false};
    double kx[kCap] = {0, 0, 0, 0}, ky[kCap] = {0, 0, 0, 0}, kz[kCap] = {0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < kCap; ++h) {
      const int t = lane + 64 * h;
      if (t < tot) {
        kx[h] = S.cx[t];
        ky[h] = S.cy[t];
        kz[h] = S.cz[t];
        bool first = true;
        if (!generic)
          for (int u = 0; u < t; ++u)
            first = first && !(S.cx[u] == kx[h] && S.cy[u] == ky[h] && S.cz[u] == kz[h]);
        keep[h] = first;
      }
    }
    int nkeep = 0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int h = 0; h < kCap; ++h)
      if (keep[h]) {
        ++nkeep;
        sx += kx[h];
        sy += ky[h];
        sz += kz[h];
      }
    const int cnt = wave_sum_i(nkeep);
    int nfc_new = nlive;
    const bool cap_fits = nlive < kMaxF && total + cnt <= kPool;
    if (cnt >= 3 && !cap_fits) bad = true;
    if (cnt >= 3 && cap_fits) {
      // centroid and an in-plane basis (e1 normal to n, e2 = n x e1)
      const double gx = wave_sum_d(sx) / cnt;
      const double gy = wave_sum_d(sy) / cnt;
      const double gz = wave_sum_d(sz) / cnt;
      const double inn = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
      const double hx = nx * inn, hy = ny * inn, hz = nz * inn;
      // e1 = t x n with t the x axis, or the y axis when n is close to x
      const bool use_x = fabs(hx) < 0.9;
      double e1x = use_x ? 0.0 : hz, e1y = use_x ? -hz : 0.0, e1z = use_x ? hy : -hx;
      const double ie1 = 1.0 / sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
      e1x *= ie1;
      e1y *= ie1;
      e1z *= ie1;
      const double e2x = hy * e1z - hz * e1y, e2y = hz * e1x - hx * e1z, e2z = hx * e1y - hy * e1x;
      double ang[kCap] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int h = 0; h < kCap; ++h) {
        const double rx = kx[h] - gx, ry = ky[h] - gy, rz = kz[h] - gz;
        ang[h] = pseudo_angle(rx * e1x + ry * e1y + rz * e1z, rx * e2x + ry * e2y + rz * e2z);
      }
      __syncthreads();  // the crossing points are read; their slots now take the angles
#pragma unroll
      for (int h = 0; h < kCap; ++h) {
        const int t = lane + 64 * h;
        S.cx[t] = (t < tot && keep[h]) ? ang[h] : INFINITY;
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < kCap; ++h) {
        const int t = lane + 64 * h;
        if (t < tot && keep[h]) {
          int rank = 0;
          for (int u = 0; u < tot; ++u) {
            const double au = S.cx[u];
            rank += (au < ang[h] || (au == ang[h] && u < t)) ? 1 : 0;
          }
          S.vx[d][total + rank] = kx[h];
          S.vy[d][total + rank] = ky[h];
          S.vz[d][total + rank] = kz[h];
        }
      }
      if (lane == 0) {
        S.off[d][nlive] = total;
        S.nvs[d][nlive] = cnt;
      }
      nfc_new = nlive + 1;
    }
    bad = ballot(bad) != 0;
    // a solid has at least four faces; fewer means nothing of volume is left
    if (nfc_new < 4) nfc_new = 0;
    if (lane == 0) S.nfc[d] = nfc_new;
    __syncthreads();
    return nfc_new > 0 ? d : -1;
  };

  // polytope src copied into d (same pool layout)
  auto copy = [&](int src, int d) {
    const int nfc = S.nfc[src];
    if (lane < nfc) {
      const int nv = S.nvs[src][lane], o = S.off[src][lane];
      for (int k = 0; k < nv; ++k) {
        S.vx[d][o + k] = S.vx[src][o + k];
        S.vy[d][o + k] = S.vy[src][o + k];
        S.vz[d][o + k] = S.vz[src][o + k];
      }
      S.off[d][lane] = o;
      S.nvs[d][lane] = nv;
    }
    if (lane == 0) S.nfc[d] = nfc;
    __syncthreads();
  };

  // polytope volume: fans from each face's first vertex, apex at the site
  auto volume = [&](int src) -> double {
    const int nfc = S.nfc[src];
    double v = 0.0;
    if (lane < nfc) {
      const int nv = S.nvs[src][lane], o = S.off[src][lane];
      const double* X = &S.vx[src][o];
      const double* Y = &S.vy[src][o];
      const double* Z = &S.vz[src][o];
      for (int k = 1; k + 1 < nv; ++k)
        v += X[0] * (Y[k] * Z[k + 1] - Z[k] * Y[k + 1]) + Y[0] * (Z[k] * X[k + 1] - X[k] * Z[k + 1]) +
             Z[0] * (X[k] * Y[k + 1] - Y[k] * X[k + 1]);
    }
    return wave_sum_d(v) / 6.0;
  };

  // voxel index range of polytope src along axis ax (0 x, 1 y, 2 z), within
  // the moved cell's box
  const double hb = 0.5 * sc * L;
  auto vrange = [&](int src, int ax, int64_t& v0, int64_t& v1) {
    const int nfc = S.nfc[src];
    double lo = INFINITY, hi = -INFINITY;
    if (lane < nfc) {
      const int nv = S.nvs[src][lane], o = S.off[src][lane];
      const double* C = ax == 0 ? &S.vx[src][o] : (ax == 1 ? &S.vy[src][o] : &S.vz[src][o]);
      for (int k = 0; k < nv; ++k) {
        lo = fmin(lo, C[k]);
        hi = fmax(hi, C[k]);
      }
    }
    const double org = ax == 0 ? me.x : (ax == 1 ? me.y : me.z);
    const double l = fmax(-wave_max_d(-lo), -hb), h = fmin(wave_max_d(hi), hb);
    v0 = int64_t(floor((org + l) / H + 0.5));
    v1 = l <= h ? int64_t(floor((org + h) / H + 0.5)) : v0 - 1;
  };

  // the moved cell, built by clipping its box (ping-pong between 0 and 1)
  int cur = 0, tmp = 1;
  init_box(cur, -hb, -hb, -hb, hb, hb, hb);
  for (int k = 0; k < npl; ++k) {
    const int r = clip(cur, tmp, S.px[k], S.py[k], S.pz[k], S.pb[k]);
    if (bad || r < 0) {
      if (bad && lane == 0) atomicOr(A.status, 1u);
      return;
    }
    if (r == tmp) {
      tmp = cur;
      cur = r;
    }
  }
  if (cur != 0) copy(cur, 0);
  // polytopes: 0 the moved cell, 1 a temporary, 2 an x slab, 3 a y column of it
  const double inv3 = 1.0 / (sc * sc * sc);
  int64_t a0, a1;
  vrange(0, 0, a0, a1);
  for (int64_t a = a0; a <= a1; ++a) {
    const double xl = (double(a) - 0.5) * H - me.x, xh = (double(a) + 0.5) * H - me.x;
    int xs = clip(0, 1, -1.0, 0.0, 0.0, -xl);
    if (xs >= 0) xs = clip(xs, 2, 1.0, 0.0, 0.0, xh);
    if (bad) break;
    if (xs < 0) continue;
    if (xs == 1) {
      copy(1, 2);
      xs = 2;
    }
    int64_t b0, b1;
    vrange(xs, 1, b0, b1);
    for (int64_t bb = b0; bb <= b1; ++bb) {
      const double yl = (double(bb) - 0.5) * H - me.y, yh = (double(bb) + 0.5) * H - me.y;
      int ys = clip(xs, 1, 0.0, -1.0, 0.0, -yl);
      if (ys >= 0) ys = clip(ys, 3, 0.0, 1.0, 0.0, yh);
      if (bad) break;
      if (ys < 0) continue;
      if (ys == 1) {
        copy(1, 3);
        ys = 3;
      }
      int64_t c0, c1;
      vrange(ys, 2, c0, c1);
      // the column's voxels: differences of the volumes below the z boundaries
      double below = 0.0;
      for (int64_t c = c0; c <= c1; ++c) {
        const double zh = (double(c) + 0.5) * H - me.z;
        const int zs = clip(ys, 1, 0.0, 0.0, 1.0, zh);
        if (bad) break;
        const double vz = zs < 0 ? 0.0 : volume(zs);
        const double part = vz - below;
        below = vz;
        if (lane == 0 && part > 0.0) {
          const unsigned long long u = (unsigned long long)llrint(part * inv3 / A.unit);
          const int64_t wa = ((a % ng) + ng) % ng, wb = ((bb % ng) + ng) % ng, wc = ((c % ng) + ng) % ng;
          if (u) atomicAdd(&A.acc[(wa * ng + wb) * ng + wc], u);
        }
      }
      if (bad) break;
    }
    if (bad) break;
  }
  if (bad && lane == 0) atomicOr(A.status, 1u);
}

__global__ void k_units_to_rho(const unsigned long long* __restrict__ acc, double scale,
                               double* __restrict__ rho, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) rho[i] = double(acc[i]) * scale;
}

}  // namespace

void za_deposit_cells(const PointSet& ps, const CellPass& cp, double tau, int64_t ng, double* density,
                      DevBuf& acc, DevBuf& status, hipStream_t st) {
  const int64_t n = ps.N, nv = ng * ng * ng;
  if (!(tau >= 0.0 && tau < 1.0)) MAK_FAIL(MAK_EINVAL, "tau must be in [0, 1)");
  const FaceStore& fs = cp.fs();
  DepCellArgs a{};
  a.pts = ps.pts.as<double4>();
  a.faces = fs.faces.as<FaceRec>();
  a.ovf = fs.ovf.as<FaceRec>();
  a.fbase = fs.fbase.as<int64_t>();
  a.fslot = fs.fslot;
  a.nface = cp.nface.as<int32_t>();
  a.vol = cp.vol.as<double>();
  a.n = n;
  a.L = ps.g.L;
  a.tau = tau;
  a.H = ps.g.L / double(ng);
  a.ng = ng;
  a.unit = ps.g.L * ps.g.L * ps.g.L * std::ldexp(1.0, -60);
  acc.ensure(size_t(nv) * sizeof(unsigned long long));
  status.ensure(sizeof(unsigned int));
  a.acc = acc.as<unsigned long long>();
  a.status = status.as<unsigned int>();
  MAK_HIP(hipMemsetAsync(a.acc, 0, size_t(nv) * sizeof(unsigned long long), st));
  MAK_HIP(hipMemsetAsync(a.status, 0, sizeof(unsigned int), st));
  a.per_xcd = ceil_div(n, 8);
  const int64_t total = 8 * a.per_xcd;
  const int64_t gx = total < 65536 ? total : 65536;
  const int64_t gy = ceil_div(total, gx);
  if (gy > 65535) MAK_FAIL(MAK_EINVAL, "too many cells for one launch");
  {
    ProfScope scope("cells_deposit", st, double(n), double(n) * 32.0 + double(nv) * 16.0);
    hipLaunchKernelGGL(k_cells_deposit, dim3(unsigned(gx), unsigned(gy)), dim3(64), 0, st, a);
    MAK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_units_to_rho, dim3(unsigned(ceil_div(nv, 256))), dim3(256), 0, st, a.acc,
                     a.unit / (a.H * a.H * a.H), density, nv);
  MAK_HIP(hipGetLastError());
  unsigned int hs = 0;
  MAK_HIP(hipMemcpyAsync(&hs, a.status, sizeof(hs), hipMemcpyDeviceToHost, st));
  MAK_HIP(hipStreamSynchronize(st));
  if (hs) MAK_FAIL(MAK_EOVERFLOW, "a moved cell exceeded the polytope capacity of the exact deposit");
}

}  // namespace mak
