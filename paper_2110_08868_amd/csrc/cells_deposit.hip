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
// the new face is their polygon ordered by angle about their centroid.
// S_i itself is built from the combinatorics the cell pass recorded (its
// triangles: the homothety keeps them, so each vertex solves its three
// scaled planes and each face's polygon is the cycle of triangles around
// it), or, for a cell without a record, clipped out of its box.  It is then
// cut into the slabs of voxel columns along x and each slab into the columns
// along y; a column's voxels are the differences of the volumes below the
// successive z boundaries, each summed face by face over the polygons
// clipped on the fly and fanned from a point of the boundary plane (the cap
// in that plane adds nothing, so the clipped polytope is never built).
// Masses are summed in 64-bit fixed point (unit L^3 2^-60), so every run
// gives the same bits; the rounding is at most half a unit per cell and
// voxel.
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
  // combinatorics recorded by the cell pass (NULL: build every moved cell by
  // clipping its box)
  const uint16_t* topo_tri;
  const int32_t* topo_n;
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
  // images, if any, are covered by the box planes).  With a record of the
  // cell's combinatorics a face's plane goes to slot 6 + the rank of its
  // site among the face sites (the record's plane codes).
  const int32_t nf = A.nface[p];
  const FaceRec* fr = nf > A.fslot ? A.ovf + A.fbase[p] : A.faces + p * int64_t(A.fslot);
  const int ntr = A.topo_n ? A.topo_n[p] : -1;
  const bool ranked = ntr >= 4 && ntr <= kTopoTri && nf <= kTopoFaces;
  int npl = 6;
  for (int base = 0; base < nf; base += 64) {
    const int f = base + lane;
    FaceRec r{};
    if (f < nf) r = fr[f];
    const bool use = f < nf && int64_t(r.j) != p;
    const uint64_t m = ballot(use);
    int slot = npl + __popcll(m & ((uint64_t(1) << lane) - 1));
    if (ranked) {
      // (one list of at most kTopoFaces faces, distinct sites)
      int rank = 0;
      for (int g = 0; g < nf; ++g) rank += __shfl(r.j, g) < r.j ? 1 : 0;
      slot = 6 + rank;
    }
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

  // volume of the part of polytope src below z = zh (seed-local), without
  // building it: each face's polygon is clipped on the fly (the side tests
  // and crossing points of `clip`) and fanned from a point of the plane, so
  // the cap face, which lies in the plane, adds nothing
  auto volume_below_z = [&](int src, double zh) -> double {
    const int nfc = S.nfc[src];
    double v = 0.0;
    if (lane < nfc) {
      const int nv = S.nvs[src][lane], o = S.off[src][lane];
      const double* X = &S.vx[src][o];
      const double* Y = &S.vy[src][o];
      const double* Z = &S.vz[src][o];
      const double tol = kSnap * A.L;
      auto sd = [&](double x, double y, double z) {
        const double t = side(x, y, z, 0.0, 0.0, 1.0, zh);
        return fabs(t) <= tol ? 0.0 : t;
      };
      int ne = 0;
      double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
      auto emit = [&](double x, double y, double z) {
        const double rz = z - zh;
        if (ne >= 2)
          v += ax * (by * rz - bz * y) + ay * (bz * x - bx * rz) + az * (bx * y - by * x);
        if (ne == 0) {
          ax = x;
          ay = y;
          az = rz;
        } else {
          bx = x;
          by = y;
          bz = rz;
        }
        ++ne;
      };
      for (int k = 0; k < nv; ++k) {
        const int k2 = k + 1 < nv ? k + 1 : 0;
        const double Px = X[k], Py = Y[k], Pz = Z[k];
        const double Qx = X[k2], Qy = Y[k2], Qz = Z[k2];
        const double sP = sd(Px, Py, Pz), sQ = sd(Qx, Qy, Qz);
        if (sP <= 0.0) emit(Px, Py, Pz);
        if (sP < 0.0 && sQ > 0.0) {
          const double t = sP / (sP - sQ);
          emit(fma(Qx - Px, t, Px), fma(Qy - Py, t, Py), fma(Qz - Pz, t, Pz));
        } else if (sP > 0.0 && sQ < 0.0) {
          const double t = sQ / (sQ - sP);
          emit(fma(Px - Qx, t, Qx), fma(Py - Qy, t, Qy), fma(Pz - Qz, t, Qz));
        }
      }
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

  // The moved cell from the recorded combinatorics: the homothety maps the
  // cell's polytope onto it with the same triangles (vertex t solves its
  // three scaled planes), and face f's polygon runs counter-clockwise seen
  // from outside through the triangles around f: after (f, x, y) comes the
  // triangle holding f followed by y, i.e. (f, y, z).  Each vertex is
  // computed once, so the faces sharing it hold the same bits.
  bool built = false;
  if (ranked) {
    bool fail = false;
    int ta = 0, tb = 0, tc = 0;
    if (lane < ntr) {
      const uint32_t code = A.topo_tri[p * kTopoTri + lane];
      ta = int(code & 31u);
      tb = int((code >> 5) & 31u);
      tc = int((code >> 10) & 31u);
      fail = ta >= npl || tb >= npl || tc >= npl;
      if (!fail) {
        const double ax = S.px[ta], ay = S.py[ta], az = S.pz[ta], ab = S.pb[ta];
        const double bx = S.px[tb], by = S.py[tb], bz = S.pz[tb], bbv = S.pb[tb];
        const double cx = S.px[tc], cy = S.py[tc], cz = S.pz[tc], cb = S.pb[tc];
        const double c23x = by * cz - bz * cy, c23y = bz * cx - bx * cz, c23z = bx * cy - by * cx;
        const double c31x = cy * az - cz * ay, c31y = cz * ax - cx * az, c31z = cx * ay - cy * ax;
        const double c12x = ay * bz - az * by, c12y = az * bx - ax * bz, c12z = ax * by - ay * bx;
        const double det = ax * c23x + ay * c23y + az * c23z;
        const double X = (ab * c23x + bbv * c31x + cb * c12x) / det;
        const double Y = (ab * c23y + bbv * c31y + cb * c12y) / det;
        const double Z = (ab * c23z + bbv * c31z + cb * c12z) / det;
        fail = !(isfinite(X) && isfinite(Y) && isfinite(Z));
        S.cx[lane] = X;
        S.cy[lane] = Y;
        S.cz[lane] = Z;
        S.off[3][lane] = ta | (tb << 8) | (tc << 16);
      }
    }
    fail = ballot(fail) != 0;
    __syncthreads();
    if (!fail) {
      // faces: one plane per lane; degree = triangles holding it
      int deg = 0, t0 = -1;
      if (lane < npl) {
        for (int t = 0; t < ntr; ++t) {
          const int c = S.off[3][t];
          if ((c & 255) == lane || ((c >> 8) & 255) == lane || ((c >> 16) & 255) == lane) {
            ++deg;
            if (t0 < 0) t0 = t;
          }
        }
      }
      const bool live = deg >= 3;
      const int dest = wave_incl_scan_i(live ? 1 : 0) - (live ? 1 : 0);
      const int nlive = __popcll(ballot(live));
      const int wincl = wave_incl_scan_i(live ? deg : 0);
      const int wo = wincl - (live ? deg : 0);
      if (deg == 1 || deg == 2 || readlane_i(wincl, 63) > kPool || nlive > kMaxF) fail = true;
      if (live && !fail) {
        // (f, x, y) of the first triangle, rotated to start at f
        const int c0 = S.off[3][t0];
        const int a0 = c0 & 255, b0 = (c0 >> 8) & 255, e0 = (c0 >> 16) & 255;
        int y = a0 == lane ? e0 : (b0 == lane ? a0 : b0);
        int t = t0;
        for (int k = 0; k < deg; ++k) {
          S.vx[0][wo + k] = S.cx[t];
          S.vy[0][wo + k] = S.cy[t];
          S.vz[0][wo + k] = S.cz[t];
          if (k + 1 == deg) break;
          // the triangle holding f followed by y
          int nt = -1, ny = 0;
          for (int u = 0; u < ntr && nt < 0; ++u) {
            const int c = S.off[3][u];
            const int a = c & 255, b = (c >> 8) & 255, e = (c >> 16) & 255;
            if (a == lane && b == y) { nt = u; ny = e; }
            else if (b == lane && e == y) { nt = u; ny = a; }
            else if (e == lane && a == y) { nt = u; ny = b; }
          }
          if (nt < 0) {
            fail = true;
            break;
          }
          t = nt;
          y = ny;
        }
        S.off[0][dest] = wo;
        S.nvs[0][dest] = deg;
      }
      fail = ballot(fail) != 0;
      if (!fail && nlive >= 4) {
        if (lane == 0) S.nfc[0] = nlive;
        built = true;
      }
    }
    __syncthreads();
  }
  // otherwise built by clipping its box (ping-pong between 0 and 1)
  if (!built) {
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
  }
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
        const double vz = volume_below_z(ys, zh);
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
  if (cp.topo_n.cap >= size_t(n) * sizeof(int32_t) && cp.topo_tri.cap >= size_t(n) * kTopoTri * sizeof(uint16_t)) {
    a.topo_tri = cp.topo_tri.as<uint16_t>();
    a.topo_n = cp.topo_n.as<int32_t>();
  }
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
