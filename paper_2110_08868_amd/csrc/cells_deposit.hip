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
// polytope is held in LDS as face polygons, one face per lane (vertices
// double-buffered, vertex-major so that the lanes' accesses do not collide).
// Clipping by a plane: every lane cuts its polygon Sutherland-Hodgman style
// (the crossing point of an edge is evaluated from its inside end and the
// side tests use explicit FMAs, so the two faces sharing an edge produce the
// same bits), the surviving polygons are compacted, the crossing points are
// gathered and duplicates dropped, and the new face is their polygon ordered
// by angle about their centroid.  The moved cell is clipped out of its box
// first, to find the voxels it can reach; then each of those voxels (as a
// box) is clipped by the same planes, and the volume of what remains (fans
// from the first vertex of each face, apex at the site) goes to the voxel.
// Masses are summed in 64-bit fixed point (unit L^3 2^-60), so every run
// gives the same bits; the rounding is at most half a unit per cell and
// voxel.
#include <cmath>

#include "../../include/mak.h"
#include "engine.h"
#include "profile.h"

namespace mak {
namespace {

constexpr int kMaxF = 64;        // face slots of a polytope (one per lane)
constexpr int kMaxV = 16;        // vertices of a face polygon
constexpr int kMaxPlanes = 128;  // planes of a cell (faces + 6 box planes)

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
  double vx[2][kMaxV][kMaxF], vy[2][kMaxV][kMaxF], vz[2][kMaxV][kMaxF];
  double px[kMaxPlanes], py[kMaxPlanes], pz[kMaxPlanes], pb[kMaxPlanes];
  double cx[2 * kMaxF], cy[2 * kMaxF], cz[2 * kMaxF];  // crossing points, then their angles
  int32_t nvs[kMaxF];                                  // vertex counts of the face slots
};

__device__ __forceinline__ double side(double x, double y, double z, double nx, double ny, double nz,
                                       double b) {
  return fma(x, nx, fma(y, ny, z * nz)) - b;
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

  int buf = 0;       // vertex buffer holding the current polygons
  int nfc = 0;       // face slots in use (wave-uniform)
  int nv = 0;        // vertex count of this lane's face slot
  bool bad = false;  // capacity exceeded or degenerate cut (wave-uniform after each clip)

  auto init_box = [&](double lx, double ly, double lz, double hx, double hy, double hz) {
    buf = 0;
    nfc = 6;
    nv = lane < 6 ? 4 : 0;
    if (lane < 6) {
      const uint32_t code = box_face_code(lane);
      for (int k = 0; k < 4; ++k) {
        const uint32_t c = (code >> (4 * k)) & 7u;
        S.vx[0][k][lane] = (c & 4u) ? hx : lx;
        S.vy[0][k][lane] = (c & 2u) ? hy : ly;
        S.vz[0][k][lane] = (c & 1u) ? hz : lz;
      }
    }
    __syncthreads();
  };

  // Clip the polytope by u . n <= b; false when nothing of volume is left.
  auto clip = [&](double nx, double ny, double nz, double b) -> bool {
    const double* X = &S.vx[buf][0][lane];
    const double* Y = &S.vy[buf][0][lane];
    const double* Z = &S.vz[buf][0][lane];
    // pass 1: how many vertices each face keeps
    int m = 0;
    bool out = false, on_all = nv > 0;
    if (lane < nfc && nv > 0) {
      const double s0 = side(X[0], Y[0], Z[0], nx, ny, nz, b);
      double sp = s0;
      for (int k = 0; k < nv; ++k) {
        const int k2 = k + 1 < nv ? k + 1 : 0;
        const double sq = k2 ? side(X[k2 * kMaxF], Y[k2 * kMaxF], Z[k2 * kMaxF], nx, ny, nz, b) : s0;
        m += int(sp <= 0.0) + int((sp < 0.0 && sq > 0.0) || (sp > 0.0 && sq < 0.0));
        out = out || sp > 0.0;
        on_all = on_all && sp == 0.0;
        sp = sq;
      }
    }
    if (ballot(out) == 0) return true;
    // a face lying in the plane is dropped: the new face replaces it
    if (m > kMaxV) bad = true;
    const bool live = m >= 3 && m <= kMaxV && !on_all;
    const int dest = wave_incl_scan_i(live ? 1 : 0) - (live ? 1 : 0);
    const int nlive = __popcll(ballot(live));
    const int ob = buf ^ 1;
    // pass 2: the clipped polygons, compacted, and the crossing points
    int ncap = 0, w = 0;
    double c0x = 0, c0y = 0, c0z = 0, c1x = 0, c1y = 0, c1z = 0;
    auto add_cap = [&](double x, double y, double z) {
      if (ncap > 0 && x == c0x && y == c0y && z == c0z) return;
      if (ncap > 1 && x == c1x && y == c1y && z == c1z) return;
      if (ncap == 0) {
        c0x = x;
        c0y = y;
        c0z = z;
      } else if (ncap == 1) {
        c1x = x;
        c1y = y;
        c1z = z;
      }
      ++ncap;
    };
    auto push = [&](double x, double y, double z) {
      if (live) {
        S.vx[ob][w][dest] = x;
        S.vy[ob][w][dest] = y;
        S.vz[ob][w][dest] = z;
      }
      ++w;
    };
    if (lane < nfc && nv > 0 && !on_all) {
      for (int k = 0; k < nv; ++k) {
        const int k2 = k + 1 < nv ? k + 1 : 0;
        const double Px = X[k * kMaxF], Py = Y[k * kMaxF], Pz = Z[k * kMaxF];
        const double Qx = X[k2 * kMaxF], Qy = Y[k2 * kMaxF], Qz = Z[k2 * kMaxF];
        const double sP = side(Px, Py, Pz, nx, ny, nz, b), sQ = side(Qx, Qy, Qz, nx, ny, nz, b);
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
          add_cap(Xx, Xy, Xz);
        }
      }
    }
    if (ncap > 2) bad = true;
    if (live) S.nvs[dest] = m;
    // gather the crossing points (at most two per face)
    const int nc = ncap > 2 ? 2 : ncap;
    const int incl = wave_incl_scan_i(nc);
    const int tot = readlane_i(incl, 63);
    if (nc > 0) {
      S.cx[incl - nc] = c0x;
      S.cy[incl - nc] = c0y;
      S.cz[incl - nc] = c0z;
      if (nc > 1) {
        S.cx[incl - 1] = c1x;
        S.cy[incl - 1] = c1y;
        S.cz[incl - 1] = c1z;
      }
    }
    __syncthreads();
    // the first occurrence of each point (two entries per lane)
    bool keep[2] = {false, false};
    double kx[2] = {0, 0}, ky[2] = {0, 0}, kz[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
      const int t = lane + 64 * h;
      if (t < tot) {
        kx[h] = S.cx[t];
        ky[h] = S.cy[t];
        kz[h] = S.cz[t];
        bool first = true;
        for (int u = 0; u < t; ++u)
          first = first && !(S.cx[u] == kx[h] && S.cy[u] == ky[h] && S.cz[u] == kz[h]);
        keep[h] = first;
      }
    }
    const int cnt = wave_sum_i(int(keep[0]) + int(keep[1]));
    int nfc_new = nlive;
    if (cnt > kMaxV || (cnt >= 3 && nlive >= kMaxF)) bad = true;
    if (cnt >= 3 && cnt <= kMaxV && nlive < kMaxF) {
      // centroid and an in-plane basis (e1 normal to n, e2 = n x e1)
      const double gx = wave_sum_d((keep[0] ? kx[0] : 0.0) + (keep[1] ? kx[1] : 0.0)) / cnt;
      const double gy = wave_sum_d((keep[0] ? ky[0] : 0.0) + (keep[1] ? ky[1] : 0.0)) / cnt;
      const double gz = wave_sum_d((keep[0] ? kz[0] : 0.0) + (keep[1] ? kz[1] : 0.0)) / cnt;
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
      double ang[2] = {0.0, 0.0};
      for (int h = 0; h < 2; ++h) {
        const double rx = kx[h] - gx, ry = ky[h] - gy, rz = kz[h] - gz;
        ang[h] = atan2(rx * e2x + ry * e2y + rz * e2z, rx * e1x + ry * e1y + rz * e1z);
      }
      __syncthreads();  // the crossing points are read; their slots now take the angles
      for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        S.cx[t] = (t < tot && keep[h]) ? ang[h] : INFINITY;
      }
      __syncthreads();
      for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        if (t < tot && keep[h]) {
          int rank = 0;
          for (int u = 0; u < tot; ++u) {
            const double au = S.cx[u];
            rank += (au < ang[h] || (au == ang[h] && u < t)) ? 1 : 0;
          }
          S.vx[ob][rank][nlive] = kx[h];
          S.vy[ob][rank][nlive] = ky[h];
          S.vz[ob][rank][nlive] = kz[h];
        }
      }
      if (lane == 0) S.nvs[nlive] = cnt;
      nfc_new = nlive + 1;
    }
    buf = ob;
    bad = ballot(bad) != 0;
    // a solid has at least four faces; fewer means nothing of volume is left
    nfc = nfc_new >= 4 ? nfc_new : 0;
    __syncthreads();
    nv = lane < nfc ? S.nvs[lane] : 0;
    return nfc > 0;
  };

  // polytope volume: fans from each face's first vertex, apex at the site
  auto volume = [&]() -> double {
    double v = 0.0;
    if (lane < nfc && nv >= 3) {
      const double ax = S.vx[buf][0][lane], ay = S.vy[buf][0][lane], az = S.vz[buf][0][lane];
      for (int k = 1; k + 1 < nv; ++k) {
        const double bx = S.vx[buf][k][lane], by = S.vy[buf][k][lane], bz = S.vz[buf][k][lane];
        const double qx = S.vx[buf][k + 1][lane], qy = S.vy[buf][k + 1][lane], qz = S.vz[buf][k + 1][lane];
        v += ax * (by * qz - bz * qy) + ay * (bz * qx - bx * qz) + az * (bx * qy - by * qx);
      }
    }
    return wave_sum_d(v) / 6.0;
  };

  auto clip_all = [&]() -> bool {
    for (int k = 0; k < npl; ++k) {
      const bool left = clip(S.px[k], S.py[k], S.pz[k], S.pb[k]);
      if (bad || !left) return false;
    }
    return true;
  };

  // the moved cell, for the voxels it can reach
  const double hb = 0.5 * sc * L;
  init_box(-hb, -hb, -hb, hb, hb, hb);
  if (!clip_all()) {
    if (bad && lane == 0) atomicOr(A.status, 1u);
    return;
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (lane < nfc)
    for (int k = 0; k < nv; ++k) {
      lo[0] = fmin(lo[0], S.vx[buf][k][lane]);
      lo[1] = fmin(lo[1], S.vy[buf][k][lane]);
      lo[2] = fmin(lo[2], S.vz[buf][k][lane]);
      hi[0] = fmax(hi[0], S.vx[buf][k][lane]);
      hi[1] = fmax(hi[1], S.vy[buf][k][lane]);
      hi[2] = fmax(hi[2], S.vz[buf][k][lane]);
    }
  // the moved cell lies in its box: clamping to it bounds the voxel loops
  // (at most ng + 2 voxels an axis)
  const double org[3] = {me.x, me.y, me.z};
  int64_t v0[3], v1[3];
  for (int a = 0; a < 3; ++a) {
    const double l = fmax(-wave_max_d(-lo[a]), -hb), h = fmin(wave_max_d(hi[a]), hb);
    v0[a] = int64_t(floor((org[a] + l) / H + 0.5));
    v1[a] = l <= h ? int64_t(floor((org[a] + h) / H + 0.5)) : v0[a] - 1;
  }
  __syncthreads();
  const double inv3 = 1.0 / (sc * sc * sc);
  for (int64_t a = v0[0]; a <= v1[0]; ++a)
    for (int64_t b = v0[1]; b <= v1[1]; ++b)
      for (int64_t c = v0[2]; c <= v1[2]; ++c) {
        const double lx = a * H - 0.5 * H - me.x, ly = b * H - 0.5 * H - me.y, lz = c * H - 0.5 * H - me.z;
        init_box(lx, ly, lz, lx + H, ly + H, lz + H);
        const bool left = clip_all();
        if (bad) {
          if (lane == 0) atomicOr(A.status, 1u);
          return;
        }
        if (!left) continue;
        const double vol = volume();
        __syncthreads();  // the next box overwrites the polygons
        if (lane == 0 && vol > 0.0) {
          const unsigned long long u = (unsigned long long)llrint(vol * inv3 / A.unit);
          const int64_t wa = ((a % ng) + ng) % ng, wb = ((b % ng) + ng) % ng, wc = ((c % ng) + ng) % ng;
          if (u) atomicAdd(&A.acc[(wa * ng + wb) * ng + wc], u);
        }
      }
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
