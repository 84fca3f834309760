/*
 * Plain FP64 oracle for the periodic Laguerre (power) cell pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP implementation.
 *
 * What it computes (the definition, written out):
 *
 *   Laguerre cell (Eq. laguerrecell):  V_i = { q : 1/2|x_i - q|^2 - psi_i
 *                                               < 1/2|x_j - q|^2 - psi_j, j != i }
 *   on the flat torus [0, L)^3, i.e. against every site j and every periodic
 *   image x_j + s L.  In seed-local coordinates u = q - x_i the condition
 *   against (j, s) is the half-space   u . d <= b,
 *       d = x_j + s L - x_i,   b = 1/2 |d|^2 + psi_i - psi_j.
 *
 * Algorithm (no grid, no ordering, no security radius):
 *   1. Start from the box [-L/2, L/2]^3: the bisectors with the site's own
 *      images (equal weights, so plain mid-planes at L/2).
 *   2. For every j != i and every shift s in {-K..K}^3, clip the polytope by
 *      the half-space (the 64 nearest minimum-image sites first: the
 *      intersection does not depend on the order, this only lets the skip
 *      test reject far planes early).  Tie rule: a vertex is removed iff u.d - b > 0
 *      strictly, so a plane that only touches the polytope makes no face (the
 *      cells of Eq. laguerrecell are open sets).  Each face polygon is clipped
 *      Sutherland-Hodgman style; the new face is the polygon of the points
 *      that now lie on the plane, ordered by angle.
 *      Exact shortcut: a plane whose distance b/|d| from the site is at least
 *      the largest vertex norm R cannot remove any vertex and is skipped.
 *   3. Integrals by fan triangulation of each face, tetrahedra with apex at
 *      the site:  volume, first moment int u, second moment int |u|^2 (the
 *      integrand of Eq. SDK), and per-face area.
 *   4. Image range check: any image left out lies at distance >= K L from the
 *      site; it cannot cut a polytope of vertex radius R when
 *      R + sqrt(R^2 + 2 max(0, psi_max - psi_i)) <= K L.  If that fails the
 *      cell is recomputed with K + 1.
 *
 * Also: the exact deposit of the cells moved by the Zel'dovich step onto an
 * Eulerian mesh (each cell shrunk towards its site, clipped against the
 * voxels it overlaps; oracle_deposit_exact).
 *
 * Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC (oracle/build.py).
 */
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct Face {
  std::vector<V3> poly;  // counter-clockwise seen from outside the cell
  int32_t j;             // other site (== i for the box faces)
  int32_t s[3];          // periodic image of site j
  V3 n;                  // plane normal d (not normalised)
  double b;              // plane offset: u . n <= b inside
};

struct CellOut {
  double V = 0, M[3] = {0, 0, 0}, S = 0, R = 0;
  int32_t flags = 0;  // 1 empty, 2 coincident site, 4 image range insufficient
  std::vector<Face> faces;
};

constexpr int32_t FLAG_EMPTY = 1, FLAG_COINCIDENT = 2, FLAG_RANGE = 4;

void init_box(std::vector<Face>& faces, double L, int32_t i) {
  const double h = 0.5 * L;
  // Vertex of the box with sign pattern (sx, sy, sz).
  auto P = [h](int sx, int sy, int sz) { return V3{sx * h, sy * h, sz * h}; };
  faces.clear();
  auto add = [&](std::vector<V3> poly, int ax, int sg) {
    Face f;
    f.poly = std::move(poly);
    f.j = i;
    f.s[0] = f.s[1] = f.s[2] = 0;
    f.s[ax] = sg;
    V3 n{0, 0, 0};
    if (ax == 0) n.x = sg * L;
    if (ax == 1) n.y = sg * L;
    if (ax == 2) n.z = sg * L;
    f.n = n;
    f.b = 0.5 * L * L;
    faces.push_back(std::move(f));
  };
  // Each polygon is counter-clockwise when seen from outside (right-hand rule
  // about the outward normal).
  add({P(1, -1, -1), P(1, 1, -1), P(1, 1, 1), P(1, -1, 1)}, 0, +1);
  add({P(-1, -1, -1), P(-1, -1, 1), P(-1, 1, 1), P(-1, 1, -1)}, 0, -1);
  add({P(-1, 1, -1), P(-1, 1, 1), P(1, 1, 1), P(1, 1, -1)}, 1, +1);
  add({P(-1, -1, -1), P(1, -1, -1), P(1, -1, 1), P(-1, -1, 1)}, 1, -1);
  add({P(-1, -1, 1), P(1, -1, 1), P(1, 1, 1), P(-1, 1, 1)}, 2, +1);
  add({P(-1, -1, -1), P(-1, 1, -1), P(1, 1, -1), P(1, -1, -1)}, 2, -1);
}

// Point where the edge from an inside vertex (s_in < 0) to an outside vertex
// (s_out > 0) crosses the plane.  Always evaluated from the inside vertex, so
// the two faces sharing the edge produce bit-identical points.
inline V3 edge_point(V3 pin, double sin_, V3 pout, double sout) {
  const double t = sin_ / (sin_ - sout);
  return pin + (pout - pin) * t;
}

bool lex_less(const V3& a, const V3& b) {
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  return a.z < b.z;
}
bool same(const V3& a, const V3& b) { return a.x == b.x && a.y == b.y && a.z == b.z; }

// Clip by  u . n <= b.  Returns true if the polytope changed.
bool clip(std::vector<Face>& faces, V3 n, double b, int32_t j, const int32_t s[3]) {
  bool any_out = false;
  for (const Face& f : faces) {
    for (const V3& v : f.poly) {
      if (dot(v, n) - b > 0) {
        any_out = true;
        break;
      }
    }
    if (any_out) break;
  }
  if (!any_out) return false;

  std::vector<V3> cap;
  std::vector<Face> kept;
  kept.reserve(faces.size() + 1);
  for (Face& f : faces) {
    const size_t m = f.poly.size();
    std::vector<V3> np;
    np.reserve(m + 2);
    for (size_t k = 0; k < m; ++k) {
      const V3 P = f.poly[k], Q = f.poly[(k + 1) % m];
      const double sP = dot(P, n) - b, sQ = dot(Q, n) - b;
      if (sP <= 0) {
        np.push_back(P);
        if (sP == 0) cap.push_back(P);
      }
      if (sP < 0 && sQ > 0) {
        V3 X = edge_point(P, sP, Q, sQ);
        np.push_back(X);
        cap.push_back(X);
      } else if (sP > 0 && sQ < 0) {
        V3 X = edge_point(Q, sQ, P, sP);
        np.push_back(X);
        cap.push_back(X);
      }
    }
    if (np.size() >= 3) {
      f.poly = std::move(np);
      kept.push_back(std::move(f));
    }
  }
  faces = std::move(kept);

  std::sort(cap.begin(), cap.end(), lex_less);
  cap.erase(std::unique(cap.begin(), cap.end(), same), cap.end());
  if (cap.size() >= 3) {
    V3 c{0, 0, 0};
    for (const V3& p : cap) c = c + p;
    c = c * (1.0 / double(cap.size()));
    const V3 nh = n * (1.0 / norm(n));
    // e1: any unit vector orthogonal to nh; e2 = nh x e1 (so e1, e2, nh is
    // right-handed and increasing angle is counter-clockwise about nh).
    V3 t = std::fabs(nh.x) < 0.9 ? V3{1, 0, 0} : V3{0, 1, 0};
    V3 e1 = cross(t, nh);
    e1 = e1 * (1.0 / norm(e1));
    V3 e2 = cross(nh, e1);
    std::vector<std::pair<double, V3>> ang;
    ang.reserve(cap.size());
    for (const V3& p : cap) {
      V3 r = p - c;
      ang.push_back({std::atan2(dot(r, e2), dot(r, e1)), p});
    }
    std::sort(ang.begin(), ang.end(), [](const std::pair<double, V3>& a,
                                         const std::pair<double, V3>& b2) {
      if (a.first != b2.first) return a.first < b2.first;
      return lex_less(a.second, b2.second);
    });
    Face f;
    for (auto& a : ang) f.poly.push_back(a.second);
    f.j = j;
    f.s[0] = s[0];
    f.s[1] = s[1];
    f.s[2] = s[2];
    f.n = n;
    f.b = b;
    faces.push_back(std::move(f));
  }
  return true;
}

double max_vertex_norm(const std::vector<Face>& faces) {
  double r2 = 0;
  for (const Face& f : faces)
    for (const V3& v : f.poly) r2 = std::max(r2, dot(v, v));
  return std::sqrt(r2);
}

void integrate(CellOut& out) {
  out.V = 0;
  out.M[0] = out.M[1] = out.M[2] = 0;
  out.S = 0;
  for (const Face& f : out.faces) {
    const size_t m = f.poly.size();
    const V3 a = f.poly[0];
    for (size_t t = 1; t + 1 < m; ++t) {
      const V3 b = f.poly[t], c = f.poly[t + 1];
      const double vol = dot(a, cross(b, c)) / 6.0;
      out.V += vol;
      const V3 g = (a + b + c) * (vol / 4.0);
      out.M[0] += g.x;
      out.M[1] += g.y;
      out.M[2] += g.z;
      out.S += vol / 10.0 *
               (dot(a, a) + dot(b, b) + dot(c, c) + dot(a, b) + dot(b, c) + dot(c, a));
    }
  }
}

double polygon_area(const Face& f) {
  V3 acc{0, 0, 0};
  const size_t m = f.poly.size();
  const V3 a = f.poly[0];
  for (size_t t = 1; t + 1 < m; ++t) acc = acc + cross(f.poly[t] - a, f.poly[t + 1] - a);
  return 0.5 * norm(acc);
}

void compute_cell(const double* x, const double* psi, int64_t n, double L, double psi_max,
                  int64_t i, CellOut& out) {
  const V3 xi{x[3 * i], x[3 * i + 1], x[3 * i + 2]};

  // Warm start.  The cell is the intersection of all half-spaces, whatever
  // the order in which they are applied; applying the bisectors of the
  // nearest sites first only makes the exact skip test below reject the far
  // ones early.  Nearest = smallest minimum-image distance, ties by index.
  struct Cand {
    double d2;
    int64_t j;
    int32_t s[3];
  };
  std::vector<Cand> near;
  near.reserve(size_t(n));
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    Cand c;
    c.j = j;
    double d2 = 0;
    for (int a = 0; a < 3; ++a) {
      const double da = x[3 * j + a] - x[3 * i + a];
      c.s[a] = da > 0.5 * L ? -1 : (da < -0.5 * L ? 1 : 0);
      const double e = da + c.s[a] * L;
      d2 += e * e;
    }
    c.d2 = d2;
    near.push_back(c);
  }
  const size_t nwarm = std::min<size_t>(64, near.size());
  auto closer = [](const Cand& a, const Cand& b) {
    return a.d2 != b.d2 ? a.d2 < b.d2 : a.j < b.j;
  };
  std::partial_sort(near.begin(), near.begin() + nwarm, near.end(), closer);
  near.resize(nwarm);
  auto is_warm = [&](int64_t j, int sx, int sy, int sz) {
    for (const Cand& c : near)
      if (c.j == j && c.s[0] == sx && c.s[1] == sy && c.s[2] == sz) return true;
    return false;
  };

  for (int K = 1; K <= 4; ++K) {
    out = CellOut();
    init_box(out.faces, L, int32_t(i));
    double R = max_vertex_norm(out.faces);
    bool empty = false;
    for (const Cand& c : near) {
      if (empty) break;
      const V3 d = V3{x[3 * c.j], x[3 * c.j + 1], x[3 * c.j + 2]} +
                   V3{c.s[0] * L, c.s[1] * L, c.s[2] * L} - xi;
      const double dn = norm(d);
      if (dn == 0) {
        out.flags |= FLAG_COINCIDENT;
        continue;
      }
      const double b = 0.5 * dot(d, d) + psi[i] - psi[c.j];
      if (b / dn >= R) continue;
      if (clip(out.faces, d, b, int32_t(c.j), c.s)) {
        if (out.faces.empty())
          empty = true;
        else
          R = max_vertex_norm(out.faces);
      }
    }
    for (int64_t j = 0; j < n && !empty; ++j) {
      if (j == i) continue;
      const V3 xj{x[3 * j], x[3 * j + 1], x[3 * j + 2]};
      for (int sx = -K; sx <= K && !empty; ++sx)
        for (int sy = -K; sy <= K && !empty; ++sy)
          for (int sz = -K; sz <= K && !empty; ++sz) {
            const V3 d = xj + V3{sx * L, sy * L, sz * L} - xi;
            const double dn = norm(d);
            if (dn == 0) {
              out.flags |= FLAG_COINCIDENT;
              continue;
            }
            const double b = 0.5 * dot(d, d) + psi[i] - psi[j];
            if (b / dn >= R) continue;  // cannot remove any vertex
            if (is_warm(j, sx, sy, sz)) continue;  // already applied
            const int32_t s[3] = {sx, sy, sz};
            if (clip(out.faces, d, b, int32_t(j), s)) {
              if (out.faces.empty()) {
                empty = true;
              } else {
                R = max_vertex_norm(out.faces);
              }
            }
          }
    }
    if (out.faces.empty()) {
      out.flags |= FLAG_EMPTY;
      out.R = 0;
      return;
    }
    integrate(out);
    out.R = R;
    const double dpsi = std::max(0.0, psi_max - psi[i]);
    if (R + std::sqrt(R * R + 2.0 * dpsi) <= K * L) return;
    if (K == 4) out.flags |= FLAG_RANGE;
  }
}

// Exact deposit of one moved cell (Zel'dovich step of the cell at growth
// amplitude tau: the cell shrunk by 1 - tau towards its site, carrying the
// cell's mass at density 1 / (1 - tau)^3) onto the voxels of the Eulerian
// nodes a H (voxel [a H - H/2, a H + H/2) per axis): the shrunk polytope is
// clipped against the six planes of every voxel its box overlaps.
void deposit_cell(const CellOut& c, V3 xi, double L, double tau, int64_t ng, double* rho) {
  if (c.faces.empty()) return;
  const double sc = 1.0 - tau;
  std::vector<Face> f0 = c.faces;
  V3 lo{INFINITY, INFINITY, INFINITY}, hi{-INFINITY, -INFINITY, -INFINITY};
  for (Face& f : f0) {
    for (V3& v : f.poly) {
      v = v * sc;
      lo = V3{std::min(lo.x, v.x), std::min(lo.y, v.y), std::min(lo.z, v.z)};
      hi = V3{std::max(hi.x, v.x), std::max(hi.y, v.y), std::max(hi.z, v.z)};
    }
    f.b *= sc;
  }
  const double H = L / double(ng);
  const double w = 1.0 / (sc * sc * sc * H * H * H);
  auto first = [H](double u) { return int64_t(std::floor((u + 0.5 * H) / H)); };
  const int64_t a0 = first(xi.x + lo.x), a1 = first(xi.x + hi.x);
  const int64_t b0 = first(xi.y + lo.y), b1 = first(xi.y + hi.y);
  const int64_t c0 = first(xi.z + lo.z), c1 = first(xi.z + hi.z);
  const int32_t s0[3] = {0, 0, 0};
  auto wrap = [ng](int64_t k) { return ((k % ng) + ng) % ng; };
  for (int64_t a = a0; a <= a1; ++a)
    for (int64_t b = b0; b <= b1; ++b)
      for (int64_t cc = c0; cc <= c1; ++cc) {
        std::vector<Face> f = f0;
        const V3 vl{a * H - 0.5 * H - xi.x, b * H - 0.5 * H - xi.y, cc * H - 0.5 * H - xi.z};
        const V3 vh = vl + V3{H, H, H};
        clip(f, V3{1, 0, 0}, vh.x, -1, s0);
        if (!f.empty()) clip(f, V3{-1, 0, 0}, -vl.x, -1, s0);
        if (!f.empty()) clip(f, V3{0, 1, 0}, vh.y, -1, s0);
        if (!f.empty()) clip(f, V3{0, -1, 0}, -vl.y, -1, s0);
        if (!f.empty()) clip(f, V3{0, 0, 1}, vh.z, -1, s0);
        if (!f.empty()) clip(f, V3{0, 0, -1}, -vl.z, -1, s0);
        if (f.empty()) continue;
        CellOut t;
        t.faces = std::move(f);
        integrate(t);
        rho[(wrap(a) * ng + wrap(b)) * ng + wrap(cc)] += t.V * w;
      }
}

}  // namespace

struct OracleResult {
  std::vector<CellOut> cells;
};

extern "C" {

OracleResult* oracle_cells(const double* x, const double* psi, int64_t n, double L,
                           const int64_t* idx, int64_t nidx, int nthreads) {
  OracleResult* r = new OracleResult();
  r->cells.resize(size_t(nidx));
  double psi_max = -INFINITY;
  for (int64_t k = 0; k < n; ++k) psi_max = std::max(psi_max, psi[k]);
  if (nthreads <= 0) nthreads = int(std::max(1u, std::thread::hardware_concurrency()));
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (;;) {
      const int64_t k = next.fetch_add(1);
      if (k >= nidx) break;
      compute_cell(x, psi, n, L, psi_max, idx[k], r->cells[size_t(k)]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  return r;
}

int64_t oracle_nfaces(const OracleResult* r) {
  int64_t s = 0;
  for (const CellOut& c : r->cells) s += int64_t(c.faces.size());
  return s;
}

// Per cell: V, first moment M (seed-local), second moment S, max vertex norm
// R, flags.  Faces in CSR-like layout: face_ptr[k]..face_ptr[k+1] for cell k,
// each with the other site j, its image shift, area, |d| and offset b.
void oracle_fetch(const OracleResult* r, double* V, double* M, double* S, double* R,
                  int32_t* flags, int64_t* face_ptr, int32_t* face_j, int32_t* face_shift,
                  double* face_area, double* face_dist, double* face_b) {
  int64_t f = 0;
  for (size_t k = 0; k < r->cells.size(); ++k) {
    const CellOut& c = r->cells[k];
    V[k] = c.V;
    M[3 * k] = c.M[0];
    M[3 * k + 1] = c.M[1];
    M[3 * k + 2] = c.M[2];
    S[k] = c.S;
    R[k] = c.R;
    flags[k] = c.flags;
    face_ptr[k] = f;
    for (const Face& fc : c.faces) {
      face_j[f] = fc.j;
      face_shift[3 * f] = fc.s[0];
      face_shift[3 * f + 1] = fc.s[1];
      face_shift[3 * f + 2] = fc.s[2];
      face_area[f] = polygon_area(fc);
      face_dist[f] = norm(fc.n);
      face_b[f] = fc.b;
      ++f;
    }
  }
  face_ptr[r->cells.size()] = f;
}

void oracle_free(OracleResult* r) { delete r; }

// Exact Eulerian deposit of the cells moved to growth amplitude tau < 1:
// rho (ng^3, row-major) = mass per voxel / voxel volume, over every cell, or
// over the cells idx[0..nidx) when idx is not NULL.
void oracle_deposit_exact(const double* x, const double* psi, int64_t n, double L, double tau, int64_t ng,
                          const int64_t* idx, int64_t nidx, double* rho, int nthreads) {
  const int64_t ncell = idx ? nidx : n;
  double psi_max = -INFINITY;
  for (int64_t k = 0; k < n; ++k) psi_max = std::max(psi_max, psi[k]);
  if (nthreads <= 0) nthreads = int(std::max(1u, std::thread::hardware_concurrency()));
  const size_t nv = size_t(ng * ng * ng);
  std::vector<std::vector<double>> acc(size_t(nthreads), std::vector<double>(nv, 0.0));
  std::atomic<int64_t> next{0};
  auto work = [&](int t) {
    for (;;) {
      const int64_t k = next.fetch_add(1);
      if (k >= ncell) break;
      const int64_t i = idx ? idx[k] : k;
      CellOut c;
      compute_cell(x, psi, n, L, psi_max, i, c);
      deposit_cell(c, V3{x[3 * i], x[3 * i + 1], x[3 * i + 2]}, L, tau, ng, acc[size_t(t)].data());
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  for (size_t v = 0; v < nv; ++v) {
    double sum = 0.0;
    for (int t = 0; t < nthreads; ++t) sum += acc[size_t(t)][v];
    rho[v] = sum;
  }
}

}  // extern "C"
