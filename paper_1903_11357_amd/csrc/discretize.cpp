// Host-side SIPG assembly and coarse transfer for libasdg.
//
// SIPG form (Sec. 2, eqs. (Ah), (lifting), (Sigma)): with rho constant per
// cell the lifting terms become face integrals of the weighted average
// {rho grad u}_w, w = rho^-/(rho^+ + rho^-), which equals
// (<rho>/2)(grad u^+ + grad u^-) with <rho> the harmonic average. Per face F
// with unit normal n (outward from the plus cell) and sides t, s in {+,-}
// (eps_+ = 1, eps_- = -1) the block coupling test side t and trial side s is
//   int_F -(g/2) eps_t phi^t_a (grad phi^s_b . n) - (g/2) eps_s (grad phi^t_a . n) phi^s_b
//         + sigma eps_t eps_s phi^t_a phi^s_b,
// g = <rho>_F, sigma = C_sigma g p^2 / <h>_F (harmonic mean of diameters);
// on a boundary face g = rho_K, <h> = h_K and the 1/2 factors are absent.
//
// Quadrature: every cell is split into triangles (area centroid, v_k, v_k+1),
// each integrated by a collapsed tensor Gauss-Legendre rule with m = p + 2
// points per direction (exact to total degree 2m - 2); faces use m-point
// Gauss-Legendre. All bilinear forms are therefore integrated exactly.
//
// Coarse transfer (Sec. 3, eq. (R0T)): block of fine cell K and coarse cell D
// is M_K^{-1} int_{K cap D} phi^K psi^D; nested coarse cells contain whole
// fine cells (Remark 3.2: the result is the injection), non-nested convex
// coarse cells are intersected with each fine cell by polygon clipping.
// A_0 = P_0^T A P_0 (eq. (A0)).
#include "discretize.h"

#include "asdg.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <atomic>
#include <memory>
#include <thread>
#include <unordered_map>

namespace asdg {

namespace {
thread_local int tl_thread_cap = 0;
}

HostThreadCap::HostThreadCap(int n) : prev_(tl_thread_cap) { tl_thread_cap = n; }
HostThreadCap::~HostThreadCap() { tl_thread_cap = prev_; }

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn) {
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 16));
  if (tl_thread_cap > 0) nt = std::min<int64_t>(nt, tl_thread_cap);
  if (n < 2048 || nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&fn, a, b] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

namespace {

struct QuadPoint {
  double x, y, w;
};

// Collapsed rule on triangle (a, b, c): x = (1-s)a + s((1-t)b + t c),
// weight 2|T| s ws wt.
void triangle_points(const double* a, const double* b, const double* c, const std::vector<double>& g,
                     const std::vector<double>& wg, std::vector<QuadPoint>& out) {
  double e1x = b[0] - a[0], e1y = b[1] - a[1];
  double e2x = c[0] - a[0], e2y = c[1] - a[1];
  double area = 0.5 * std::fabs(e1x * e2y - e1y * e2x);
  int m = (int)g.size();
  for (int i = 0; i < m; ++i) {
    double s = g[i];
    for (int j = 0; j < m; ++j) {
      double t = g[j];
      double px = (1.0 - s) * a[0] + s * ((1.0 - t) * b[0] + t * c[0]);
      double py = (1.0 - s) * a[1] + s * ((1.0 - t) * b[1] + t * c[1]);
      out.push_back({px, py, 2.0 * area * s * wg[i] * wg[j]});
    }
  }
}

double polygon_area_centroid(const std::vector<double>& P, double& cx, double& cy) {
  size_t k = P.size() / 2;
  double a = 0.0, sx = 0.0, sy = 0.0;
  for (size_t i = 0; i < k; ++i) {
    size_t j = (i + 1) % k;
    double cr = P[2 * i] * P[2 * j + 1] - P[2 * j] * P[2 * i + 1];
    a += cr;
    sx += (P[2 * i] + P[2 * j]) * cr;
    sy += (P[2 * i + 1] + P[2 * j + 1]) * cr;
  }
  a *= 0.5;
  cx = sx / (6.0 * a);
  cy = sy / (6.0 * a);
  return a;
}

// Centroid-fan rule over a polygon given as flat xy list.
void polygon_points(const std::vector<double>& P, const std::vector<double>& g,
                    const std::vector<double>& wg, std::vector<QuadPoint>& out) {
  double cx, cy;
  polygon_area_centroid(P, cx, cy);
  double c[2] = {cx, cy};
  size_t k = P.size() / 2;
  for (size_t i = 0; i < k; ++i) {
    size_t j = (i + 1) % k;
    triangle_points(c, &P[2 * i], &P[2 * j], g, wg, out);
  }
}

// Sutherland-Hodgman: subject polygon clipped by convex CCW clipper.
std::vector<double> clip_polygon(const std::vector<double>& subject, const std::vector<double>& clipper) {
  std::vector<double> out = subject, in;
  size_t k = clipper.size() / 2;
  for (size_t i = 0; i < k && !out.empty(); ++i) {
    double ax = clipper[2 * i], ay = clipper[2 * i + 1];
    size_t i1 = (i + 1) % k;
    double ex = clipper[2 * i1] - ax, ey = clipper[2 * i1 + 1] - ay;
    in.swap(out);
    out.clear();
    size_t n = in.size() / 2;
    for (size_t j = 0; j < n; ++j) {
      size_t j1 = (j + 1) % n;
      double Px = in[2 * j], Py = in[2 * j + 1], Qx = in[2 * j1], Qy = in[2 * j1 + 1];
      double sP = ex * (Py - ay) - ey * (Px - ax);
      double sQ = ex * (Qy - ay) - ey * (Qx - ax);
      if (sP >= 0.0) {
        out.push_back(Px);
        out.push_back(Py);
        if (sQ < 0.0) {
          double t = sP / (sP - sQ);
          out.push_back(Px + (Qx - Px) * t);
          out.push_back(Py + (Qy - Py) * t);
        }
      } else if (sQ >= 0.0) {
        double t = sP / (sP - sQ);
        out.push_back(Px + (Qx - Px) * t);
        out.push_back(Py + (Qy - Py) * t);
      }
    }
  }
  if (out.size() < 6) out.clear();
  return out;
}

// Small dense SPD solve (Cholesky), matrix n x n row-major, rhs n x k.
}  // namespace

bool spd_solve(int n, std::vector<double> M, double* B, int k) {
  for (int j = 0; j < n; ++j) {
    double d = M[j * n + j];
    for (int l = 0; l < j; ++l) d -= M[j * n + l] * M[j * n + l];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    M[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = M[i * n + j];
      for (int l = 0; l < j; ++l) s -= M[i * n + l] * M[j * n + l];
      M[i * n + j] = s / d;
    }
  }
  for (int c = 0; c < k; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = B[i * k + c];
      for (int l = 0; l < i; ++l) s -= M[i * n + l] * B[l * k + c];
      B[i * k + c] = s / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = B[i * k + c];
      for (int l = i + 1; l < n; ++l) s -= M[l * n + i] * B[l * k + c];
      B[i * k + c] = s / M[i * n + i];
    }
  }
  return true;
}

namespace {

bool on_boundary_side(double ax, double ay, double bx, double by) {
  const double tol = 1e-12;
  for (double s : {0.0, 1.0}) {
    if (std::fabs(ax - s) < tol && std::fabs(bx - s) < tol) return true;
    if (std::fabs(ay - s) < tol && std::fabs(by - s) < tol) return true;
  }
  return false;
}

std::string geometry(const MeshView& m, CellGeom& g, bool require_ccw) {
  int32_t N = m.n_cells;
  g.area.assign(N, 0.0);
  g.cx.assign(N, 0.0);
  g.cy.assign(N, 0.0);
  g.diam.assign(N, 0.0);
  g.box.assign(N, Box{0, 0, 0, 0});
  for (int32_t c = 0; c < N; ++c) {
    int32_t a = m.ptr[c], b = m.ptr[c + 1];
    if (b - a < 3) return "cell " + std::to_string(c) + " has fewer than 3 vertices";
    for (int32_t k = a; k < b; ++k)
      if (m.verts[k] < 0 || m.verts[k] >= m.n_vertices) return "vertex id out of range";
  }
  std::vector<int> bad(N, 0);
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    std::vector<double> P;
    for (int64_t c = lo; c < hi; ++c) {
      int32_t a = m.ptr[c], b = m.ptr[c + 1];
      P.clear();
      for (int32_t k = a; k < b; ++k) {
        P.push_back(m.xy[2 * m.verts[k]]);
        P.push_back(m.xy[2 * m.verts[k] + 1]);
      }
      double cx, cy;
      double ar = polygon_area_centroid(P, cx, cy);
      if (!(ar > 0.0) && require_ccw) {
        bad[c] = 1;
        continue;
      }
      g.area[c] = ar;
      g.cx[c] = cx;
      g.cy[c] = cy;
      size_t k = P.size() / 2;
      double d2 = 0.0;
      Box B{P[0], P[0], P[1], P[1]};
      for (size_t i = 0; i < k; ++i) {
        B.x0 = std::min(B.x0, P[2 * i]);
        B.x1 = std::max(B.x1, P[2 * i]);
        B.y0 = std::min(B.y0, P[2 * i + 1]);
        B.y1 = std::max(B.y1, P[2 * i + 1]);
        for (size_t j = i + 1; j < k; ++j) {
          double dx = P[2 * i] - P[2 * j], dy = P[2 * i + 1] - P[2 * j + 1];
          d2 = std::max(d2, dx * dx + dy * dy);
        }
      }
      g.diam[c] = std::sqrt(d2);
      g.box[c] = B;
    }
  });
  for (int32_t c = 0; c < N; ++c)
    if (bad[c]) return "cell " + std::to_string(c) + " is clockwise or degenerate";
  return "";
}

void cell_polygon(const MeshView& m, int32_t c, std::vector<double>& P) {
  P.clear();
  for (int32_t k = m.ptr[c]; k < m.ptr[c + 1]; ++k) {
    P.push_back(m.xy[2 * m.verts[k]]);
    P.push_back(m.xy[2 * m.verts[k] + 1]);
  }
}

// Quadrature points of a cell's centroid fan (order fixed by vertex order).
void cell_points(const MeshView& m, const CellGeom& g, int32_t c, const std::vector<double>& gq,
                 const std::vector<double>& wq, std::vector<QuadPoint>& out) {
  out.clear();
  double C[2] = {g.cx[c], g.cy[c]};
  int32_t a = m.ptr[c], b = m.ptr[c + 1];
  for (int32_t k = a; k < b; ++k) {
    int32_t k1 = (k + 1 < b) ? k + 1 : a;
    triangle_points(C, &m.xy[2 * m.verts[k]], &m.xy[2 * m.verts[k1]], gq, wq, out);
  }
}

}  // namespace

void gauss_legendre01(int m, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on P_m using the three-term recurrence; nodes are the
  // roots of P_m on [-1, 1], weights 2 / ((1 - t^2) P_m'(t)^2), then mapped.
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < m; ++i) {
    double t = std::cos(pi * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 1; k < m; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (m == 1) {
        p1 = t;
        p0 = 1.0;
      }
      dp = m * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < m; ++k) {
      double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    if (m == 1) p0 = 1.0;
    dp = m * (t * p1 - p0) / (t * t - 1.0);
    x[i] = 0.5 * (t + 1.0);
    w[i] = 0.5 * 2.0 / ((1.0 - t * t) * dp * dp);
  }
  // ascending order
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(m), ws(m);
  for (int i = 0; i < m; ++i) {
    xs[i] = x[idx[i]];
    ws[i] = w[idx[i]];
  }
  x.swap(xs);
  w.swap(ws);
}

int n_basis(int p) { return (p + 1) * (p + 2) / 2; }

void basis_prepare(int p, const Box& B, BasisBox& bb) {
  bb.p = p;
  bb.dx = B.x1 - B.x0;
  bb.dy = B.y1 - B.y0;
  bb.cx = 0.5 * (B.x0 + B.x1);
  bb.cy = 0.5 * (B.y0 + B.y1);
  bb.sx = 2.0 / bb.dx;
  bb.sy = 2.0 / bb.dy;
  int a = 0;
  for (int d = 0; d <= p; ++d)
    for (int j = 0; j <= d; ++j, ++a) {
      const int i = d - j;
      bb.s[a] = std::sqrt((2.0 * i + 1.0) * (2.0 * j + 1.0) / (bb.dx * bb.dy));
    }
}

void basis_eval(const BasisBox& bb, double x, double y, double* val, double* gx, double* gy) {
  const int p = bb.p;
  double xi = 2.0 * (x - bb.cx) / bb.dx;
  double eta = 2.0 * (y - bb.cy) / bb.dy;
  double Lx[16], dLx[16], Ly[16], dLy[16];
  Lx[0] = 1.0;
  dLx[0] = 0.0;
  Ly[0] = 1.0;
  dLy[0] = 0.0;
  if (p >= 1) {
    Lx[1] = xi;
    dLx[1] = 1.0;
    Ly[1] = eta;
    dLy[1] = 1.0;
  }
  for (int k = 1; k < p; ++k) {
    Lx[k + 1] = ((2 * k + 1) * xi * Lx[k] - k * Lx[k - 1]) / (k + 1);
    Ly[k + 1] = ((2 * k + 1) * eta * Ly[k] - k * Ly[k - 1]) / (k + 1);
    dLx[k + 1] = dLx[k - 1] + (2 * k + 1) * Lx[k];
    dLy[k + 1] = dLy[k - 1] + (2 * k + 1) * Ly[k];
  }
  int a = 0;
  for (int d = 0; d <= p; ++d) {
    for (int j = 0; j <= d; ++j, ++a) {
      int i = d - j;
      const double s = bb.s[a];
      val[a] = s * Lx[i] * Ly[j];
      if (gx) gx[a] = s * dLx[i] * bb.sx * Ly[j];
      if (gy) gy[a] = s * Lx[i] * dLy[j] * bb.sy;
    }
  }
}

// Subdomain-major permutation (stable), BSR structure and rows of the SIPG
// system from per-cell volume blocks vol [N][np*np] and loads rhs_c [N][np]
// (caller order) and per-face blocks fblk [F][4][np*np] of the faces
// pm = (plus, minus) (minus < 0: boundary face, block 0 only). Rows add the
// volume block, then the cell's faces in face-index order (deterministic).
std::string finish_assembly(Assembled& A, const int32_t* subdomain, const std::vector<std::pair<int32_t, int32_t>>& pm,
                            const double* vol, const double* rhs_c, const double* fblk) {
  const int32_t N = A.n_cells;
  const int np = A.np;
  // subdomains and subdomain-major permutation (stable)
  int32_t nsub = 0;
  for (int32_t c = 0; c < N; ++c) {
    if (subdomain[c] < 0) return "negative subdomain id";
    nsub = std::max(nsub, subdomain[c] + 1);
  }
  A.n_sub = nsub;
  A.sub_ptr.assign(nsub + 1, 0);
  for (int32_t c = 0; c < N; ++c) A.sub_ptr[subdomain[c] + 1]++;
  for (int32_t i = 0; i < nsub; ++i) {
    if (A.sub_ptr[i + 1] == 0) return "subdomain id " + std::to_string(i) + " is unused";
    A.sub_ptr[i + 1] += A.sub_ptr[i];
  }
  A.perm.assign(N, 0);
  A.iperm.assign(N, 0);
  {
    std::vector<int32_t> fill(A.sub_ptr.begin(), A.sub_ptr.end() - 1);
    for (int32_t c = 0; c < N; ++c) {
      int32_t r = fill[subdomain[c]]++;
      A.perm[r] = c;
      A.iperm[c] = r;
    }
  }

  // per-cell face lists (caller order), in face-index order
  std::vector<int32_t> cf_ptr(N + 1, 0);
  for (const auto& F : pm) {
    cf_ptr[F.first + 1]++;
    if (F.second >= 0) cf_ptr[F.second + 1]++;
  }
  for (int32_t c = 0; c < N; ++c) cf_ptr[c + 1] += cf_ptr[c];
  std::vector<int32_t> cf(cf_ptr[N]);
  {
    std::vector<int32_t> fill(cf_ptr.begin(), cf_ptr.end() - 1);
    for (int32_t fidx = 0; fidx < (int32_t)pm.size(); ++fidx) {
      const auto& F = pm[fidx];
      cf[fill[F.first]++] = 2 * fidx;  // side +
      if (F.second >= 0) cf[fill[F.second]++] = 2 * fidx + 1;  // side -
    }
  }

  // BSR structure, internal order
  A.row_ptr.assign(N + 1, 0);
  std::vector<std::vector<int32_t>> cols(N);
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      int32_t c = A.perm[r];
      auto& cl = cols[r];
      cl.push_back((int32_t)r);
      for (int32_t k = cf_ptr[c]; k < cf_ptr[c + 1]; ++k) {
        const auto& F = pm[cf[k] >> 1];
        if (F.second < 0) continue;
        int32_t other = (cf[k] & 1) ? F.first : F.second;
        cl.push_back(A.iperm[other]);
      }
      std::sort(cl.begin(), cl.end());
      cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
    }
  });
  for (int32_t r = 0; r < N; ++r) A.row_ptr[r + 1] = A.row_ptr[r] + (int32_t)cols[r].size();
  A.col_idx.resize(A.row_ptr[N]);
  for (int32_t r = 0; r < N; ++r) std::copy(cols[r].begin(), cols[r].end(), A.col_idx.begin() + A.row_ptr[r]);
  cols.clear();
  cols.shrink_to_fit();

  // accumulate rows (internal order), deterministic order: volume, then the
  // cell's faces in face-index order
  // (the blocks are left uninitialised and zeroed row by row in parallel:
  // a serial fill of the whole array cost as much as the accumulation)
  A.blocks.clear();
  A.blocks.resize((size_t)A.row_ptr[N] * np * np);
  A.rhs.assign((size_t)N * np, 0.0);
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      int32_t c = A.perm[r];
      int32_t rs = A.row_ptr[r], re = A.row_ptr[r + 1];
      std::fill(A.blocks.begin() + (size_t)rs * np * np, A.blocks.begin() + (size_t)re * np * np, 0.0);
      auto slot = [&](int32_t col) {
        int32_t k = (int32_t)(std::lower_bound(A.col_idx.begin() + rs, A.col_idx.begin() + re, col) -
                              A.col_idx.begin());
        return &A.blocks[(size_t)k * np * np];
      };
      // the per-cell (symmetric) and per-face blocks are row-major, as the
      // operator's blocks (the device layout)
      const int nn = np * np;
      auto add = [nn](double* dst, const double* src) {
        for (int e = 0; e < nn; ++e) dst[e] += src[e];
      };
      double* D = slot((int32_t)r);
      add(D, &vol[(size_t)c * np * np]);
      for (int32_t k = cf_ptr[c]; k < cf_ptr[c + 1]; ++k) {
        int32_t fi = cf[k] >> 1;
        int t = cf[k] & 1;
        const auto& F = pm[fi];
        const double* Bk = &fblk[(size_t)fi * 4 * np * np];
        if (F.second < 0) {
          add(D, Bk);
          continue;
        }
        add(D, Bk + (t * 2 + t) * np * np);
        int32_t other = t ? F.first : F.second;
        add(slot(A.iperm[other]), Bk + (t * 2 + (1 - t)) * np * np);
      }
      for (int a = 0; a < np; ++a) A.rhs[(size_t)r * np + a] = rhs_c[(size_t)c * np + a];
    }
  });
  return "";
}

namespace {

// basis_eval with the degree fixed at compile time (same arithmetic, fully
// unrolled loops)
template <int P>
inline void basis_eval_p(const BasisBox& bb, double x, double y, double* val, double* gx, double* gy) {
  double xi = 2.0 * (x - bb.cx) / bb.dx;
  double eta = 2.0 * (y - bb.cy) / bb.dy;
  double Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
  Lx[0] = 1.0;
  dLx[0] = 0.0;
  Ly[0] = 1.0;
  dLy[0] = 0.0;
  Lx[1] = xi;
  dLx[1] = 1.0;
  Ly[1] = eta;
  dLy[1] = 1.0;
#pragma GCC unroll 4
  for (int k = 1; k < P; ++k) {
    Lx[k + 1] = ((2 * k + 1) * xi * Lx[k] - k * Lx[k - 1]) / (k + 1);
    Ly[k + 1] = ((2 * k + 1) * eta * Ly[k] - k * Ly[k - 1]) / (k + 1);
    dLx[k + 1] = dLx[k - 1] + (2 * k + 1) * Lx[k];
    dLy[k + 1] = dLy[k - 1] + (2 * k + 1) * Ly[k];
  }
  int a = 0;
#pragma GCC unroll 5
  for (int d = 0; d <= P; ++d) {
#pragma GCC unroll 5
    for (int j = 0; j <= d; ++j, ++a) {
      int i = d - j;
      const double s = bb.s[a];
      val[a] = s * Lx[i] * Ly[j];
      gx[a] = s * dLx[i] * bb.sx * Ly[j];
      gy[a] = s * Lx[i] * dLy[j] * bb.sy;
    }
  }
}

// Basis values only (the same arithmetic as basis_eval's values).
template <int P>
inline void basis_val_p(const BasisBox& bb, double x, double y, double* val) {
  double xi = 2.0 * (x - bb.cx) / bb.dx;
  double eta = 2.0 * (y - bb.cy) / bb.dy;
  double Lx[P + 1], Ly[P + 1];
  Lx[0] = 1.0;
  Ly[0] = 1.0;
  Lx[1] = xi;
  Ly[1] = eta;
#pragma GCC unroll 4
  for (int k = 1; k < P; ++k) {
    Lx[k + 1] = ((2 * k + 1) * xi * Lx[k] - k * Lx[k - 1]) / (k + 1);
    Ly[k + 1] = ((2 * k + 1) * eta * Ly[k] - k * Ly[k - 1]) / (k + 1);
  }
  int a = 0;
#pragma GCC unroll 5
  for (int d = 0; d <= P; ++d)
#pragma GCC unroll 5
    for (int j = 0; j <= d; ++j, ++a) val[a] = bb.s[a] * Lx[d - j] * Ly[j];
}

// Volume blocks (rho grad v . grad u) and loads (f v) of cells c0 + [lo, hi),
// points of cell c0 + cc at [pptr[cc], pptr[cc + 1]).
template <int P>
void volume_range(int64_t c0, int64_t lo, int64_t hi, const int64_t* pptr, const double* pts, const double* wts,
                  const double* fv, const CellGeom& G, const double* rho, double* vol, double* rhs_c) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  double v[NP], gx[NP], gy[NP];
  BasisBox bb;
  for (int64_t cc = lo; cc < hi; ++cc) {
    const int64_t c = c0 + cc;
    double* K = vol + (size_t)c * NP * NP;
    double* bl = rhs_c + (size_t)c * NP;
    std::fill(K, K + NP * NP, 0.0);
    std::fill(bl, bl + NP, 0.0);
    basis_prepare(P, G.box[c], bb);
    for (int64_t k = pptr[cc]; k < pptr[cc + 1]; ++k) {
      basis_eval_p<P>(bb, pts[2 * k], pts[2 * k + 1], v, gx, gy);
      const double w = wts[k];
      const double wr = w * rho[c];
      // the (a, b) and (b, a) terms are the same products: one triangle, mirrored below
#pragma GCC unroll 15
      for (int b = 0; b < NP; ++b)
#pragma GCC unroll 15
        for (int a = b; a < NP; ++a) K[b * NP + a] += wr * (gx[a] * gx[b] + gy[a] * gy[b]);
      const double wf = w * fv[k];
#pragma GCC unroll 15
      for (int a = 0; a < NP; ++a) bl[a] += wf * v[a];
    }
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < b; ++a) K[b * NP + a] = K[a * NP + b];
  }
}

struct FaceCtx {
  const MeshView* mesh;
  const CellGeom* G;
  const std::vector<Face>* faces;
  const double* rho;
  double c_sigma, pp;
  int m;
  const double* gq;
  const double* wq;
  double* fblk;
};

// Face blocks of faces [lo, hi): interior faces the four blocks (++, +-, -+,
// --), boundary faces block 0; block (t, s) element (a, b) at a*np + b.
template <int P>
void face_range(const FaceCtx& X, int64_t lo, int64_t hi) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  double vp[NP], gxp[NP], gyp[NP], vm[NP], gxm[NP], gym[NP], gnp[NP], gnm[NP];
  BasisBox bp, bm;
  const MeshView& mesh = *X.mesh;
  const CellGeom& G = *X.G;
  for (int64_t fi = lo; fi < hi; ++fi) {
    const Face& F = (*X.faces)[fi];
    double ax = mesh.xy[2 * F.v0], ay = mesh.xy[2 * F.v0 + 1];
    double bx = mesh.xy[2 * F.v1], by = mesh.xy[2 * F.v1 + 1];
    double dx = bx - ax, dy = by - ay;
    double L = std::sqrt(dx * dx + dy * dy);
    double nx = dy / L, ny = -dx / L;
    double* Bk = X.fblk + (size_t)fi * 4 * NP * NP;
    std::fill(Bk, Bk + 4 * NP * NP, 0.0);
    basis_prepare(P, G.box[F.plus], bp);
    if (F.minus >= 0) {
      basis_prepare(P, G.box[F.minus], bm);
      double rp = X.rho[F.plus], rm = X.rho[F.minus];
      double g = 2.0 * rp * rm / (rp + rm);
      double hp = G.diam[F.plus], hm = G.diam[F.minus];
      double hF = 2.0 * hp * hm / (hp + hm);
      double sigma = X.c_sigma * g * X.pp / hF;
      for (int q = 0; q < X.m; ++q) {
        double x = ax + X.gq[q] * dx, y = ay + X.gq[q] * dy, w = L * X.wq[q];
        basis_eval_p<P>(bp, x, y, vp, gxp, gyp);
        basis_eval_p<P>(bm, x, y, vm, gxm, gym);
        for (int a = 0; a < NP; ++a) {
          gnp[a] = gxp[a] * nx + gyp[a] * ny;
          gnm[a] = gxm[a] * nx + gym[a] * ny;
        }
        const double* V[2] = {vp, vm};
        const double* GN[2] = {gnp, gnm};
        const double eps[2] = {1.0, -1.0};
        for (int t = 0; t < 2; ++t)
          for (int s = 0; s < 2; ++s) {
            double* blk = Bk + (t * 2 + s) * NP * NP;
            double c1 = -0.5 * g * eps[t] * w, c2 = -0.5 * g * eps[s] * w;
            double c3 = sigma * eps[t] * eps[s] * w;
            const double* Vt = V[t];
            const double* Vs = V[s];
            const double* Gt = GN[t];
            const double* Gs = GN[s];
#pragma GCC unroll 15
            for (int a = 0; a < NP; ++a)
#pragma GCC unroll 15
              for (int b = 0; b < NP; ++b)
                blk[a * NP + b] += c1 * Vt[a] * Gs[b] + c2 * Gt[a] * Vs[b] + c3 * Vt[a] * Vs[b];
          }
      }
    } else {
      double r = X.rho[F.plus];
      double sigma = X.c_sigma * r * X.pp / G.diam[F.plus];
      for (int q = 0; q < X.m; ++q) {
        double x = ax + X.gq[q] * dx, y = ay + X.gq[q] * dy, w = L * X.wq[q];
        basis_eval_p<P>(bp, x, y, vp, gxp, gyp);
        for (int a = 0; a < NP; ++a) gnp[a] = gxp[a] * nx + gyp[a] * ny;
#pragma GCC unroll 15
        for (int a = 0; a < NP; ++a)
#pragma GCC unroll 15
          for (int b = 0; b < NP; ++b)
            Bk[a * NP + b] += w * (-r * vp[a] * gnp[b] - r * gnp[a] * vp[b] + sigma * vp[a] * vp[b]);
      }
    }
  }
}

}  // namespace

// Faces of a polygon mesh by edge matching: one face per edge of a cell,
// shared by the two cells whose edges join the same two vertices (in
// opposite directions). Faces are numbered in the order in which their
// first edge appears (cells in order, edges in each cell's vertex order);
// plus = that edge's cell, minus = the other one (-1 on the boundary).
// Edges are bucketed by their smaller vertex id, so each edge finds its
// partner among the few edges at that vertex.
static std::string match_faces(const MeshView& mesh, std::vector<Face>& faces) {
  const int32_t N = mesh.n_cells;
  const int64_t E = mesh.ptr[N];
  std::vector<int32_t> cell(E), other(E), lo(E), hi(E), partner(E, -1);
  std::atomic<int32_t> bad_cell{INT32_MAX};
  parallel_for(N, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      const int32_t a = mesh.ptr[c], b = mesh.ptr[c + 1];
      for (int32_t k = a; k < b; ++k) {
        const int32_t v0 = mesh.verts[k], v1 = mesh.verts[(k + 1 < b) ? k + 1 : a];
        if (v0 == v1) {
          int32_t cur = bad_cell.load();
          while ((int32_t)c < cur && !bad_cell.compare_exchange_weak(cur, (int32_t)c)) {
          }
        }
        cell[k] = (int32_t)c;
        other[k] = v1;
        lo[k] = std::min(v0, v1);
        hi[k] = std::max(v0, v1);
      }
    }
  });
  if (bad_cell.load() != INT32_MAX) return "repeated vertex in cell " + std::to_string(bad_cell.load());
  // edges bucketed by their smaller vertex, in edge order within a bucket
  std::vector<int64_t> bptr((size_t)mesh.n_vertices + 1, 0);
  for (int64_t k = 0; k < E; ++k) {
    if (lo[k] < 0 || hi[k] >= mesh.n_vertices) return "vertex id out of range";
    bptr[lo[k] + 1]++;
  }
  for (int32_t v = 0; v < mesh.n_vertices; ++v) bptr[v + 1] += bptr[v];
  std::vector<int64_t> bucket(E);
  {
    std::vector<int64_t> fill(bptr.begin(), bptr.end() - 1);
    for (int64_t k = 0; k < E; ++k) bucket[fill[lo[k]]++] = k;
  }
  std::atomic<int> shared3{0};
  parallel_for(E, [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      int found = 0;
      for (int64_t i = bptr[lo[k]]; i < bptr[lo[k] + 1]; ++i) {
        const int64_t j = bucket[i];
        if (j != k && hi[j] == hi[k]) {
          partner[k] = (int32_t)j;
          ++found;
        }
      }
      if (found > 1) shared3 = 1;
    }
  });
  if (shared3) return "edge shared by more than two cells";
  // a face per edge without a partner or whose partner comes later
  std::vector<int32_t> face_of(E, -1);
  faces.clear();
  for (int64_t k = 0; k < E; ++k) {
    if (partner[k] < 0 || partner[k] > k) {
      const int32_t v0 = mesh.verts[k];
      face_of[k] = (int32_t)faces.size();
      faces.push_back({cell[k], -1, v0, other[k]});
    }
  }
  for (int64_t k = 0; k < E; ++k) {
    if (partner[k] < 0 || partner[k] > k) continue;
    Face& F = faces[face_of[partner[k]]];
    const int32_t v0 = mesh.verts[k], v1 = other[k];
    if (!(F.v0 == v1 && F.v1 == v0)) return "inconsistent orientation across an edge";
    F.minus = cell[k];
  }
  return "";
}

std::string assemble_sipg(const MeshView& mesh, int p, double c_sigma, const double* rho,
                          const int32_t* subdomain,
                          void (*f)(int64_t, const double*, double*, void*), void* f_user,
                          Assembled& A) {
  if (p < 1 || p > kMaxDegree2D) return "p must be in 1.." + std::to_string(kMaxDegree2D);
  if (!(c_sigma > 0.0)) return "c_sigma must be positive";
  const int32_t N = mesh.n_cells;
  if (N < 1) return "empty mesh";
  for (int32_t c = 0; c < N; ++c)
    if (!(rho[c] > 0.0) || !std::isfinite(rho[c])) return "rho must be positive and finite";
  A.dim = 2;
  A.box3.clear();
  A.diam3.clear();
  A.p = p;
  A.np = n_basis(p);
  A.c_sigma = c_sigma;
  A.n_cells = N;
  const int np = A.np;
  std::string err = geometry(mesh, A.geom, true);
  if (!err.empty()) return err;
  const CellGeom& G = A.geom;

  // faces by edge matching
  {
    std::string e = match_faces(mesh, A.faces);
    if (!e.empty()) return e;
  }
  for (const Face& F : A.faces) {
    if (F.minus < 0 &&
        !on_boundary_side(mesh.xy[2 * F.v0], mesh.xy[2 * F.v0 + 1], mesh.xy[2 * F.v1], mesh.xy[2 * F.v1 + 1]))
      return "non-conforming mesh: unmatched edge inside the domain";
  }

  const int m = p + 2;
  std::vector<double> gq, wq;
  gauss_legendre01(m, gq, wq);
  const double pp = (double)p * (double)p;

  // volume blocks and load vector, caller order (zeroed per cell by volume_range)
  std::vector<double, DefaultInit<double>> vol((size_t)N * np * np), rhs_c((size_t)N * np);
  {
    const int64_t chunk = 8192;
    // point buffers of one chunk, reused by every chunk and not
    // value-initialised: each chunk writes every entry it reads (a zero fill
    // of fresh buffers per chunk cost as much as the volume integrals)
    int64_t max_pts = 0;
    for (int64_t c0 = 0; c0 < N; c0 += chunk) {
      const int64_t c1 = std::min<int64_t>(N, c0 + chunk);
      max_pts = std::max<int64_t>(max_pts, (int64_t)(mesh.ptr[c1] - mesh.ptr[c0]) * m * m);
    }
    std::vector<double, DefaultInit<double>> pts(2 * max_pts), wts(max_pts), fv(max_pts);
    if (!f)
      parallel_for(max_pts, [&](int64_t lo, int64_t hi) { std::fill(fv.begin() + lo, fv.begin() + hi, 0.0); });
    std::vector<int64_t> pptr(chunk + 1, 0);
    for (int64_t c0 = 0; c0 < N; c0 += chunk) {
      int64_t c1 = std::min<int64_t>(N, c0 + chunk);
      // points of this chunk, in cell order
      for (int64_t c = c0; c < c1; ++c)
        pptr[c - c0 + 1] = pptr[c - c0] + (int64_t)(mesh.ptr[c + 1] - mesh.ptr[c]) * m * m;
      parallel_for(c1 - c0, [&](int64_t lo, int64_t hi) {
        std::vector<QuadPoint> qp;
        for (int64_t cc = lo; cc < hi; ++cc) {
          cell_points(mesh, G, (int32_t)(c0 + cc), gq, wq, qp);
          int64_t o = pptr[cc];
          for (size_t k = 0; k < qp.size(); ++k) {
            pts[2 * (o + k)] = qp[k].x;
            pts[2 * (o + k) + 1] = qp[k].y;
            wts[o + k] = qp[k].w;
          }
        }
      });
      if (f) f(pptr[c1 - c0], pts.data(), fv.data(), f_user);
      parallel_for(c1 - c0, [&](int64_t lo, int64_t hi) {
        const int64_t* pp_ = pptr.data();
        switch (p) {
          case 1: volume_range<1>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 2: volume_range<2>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 3: volume_range<3>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 4: volume_range<4>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 5: volume_range<5>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 6: volume_range<6>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 7: volume_range<7>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          case 8: volume_range<8>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
          default: volume_range<9>(c0, lo, hi, pp_, pts.data(), wts.data(), fv.data(), G, rho, vol.data(), rhs_c.data()); break;
        }
      });
    }
  }

  // face blocks: interior faces 4 blocks (++, +-, -+, --), boundary 1 block;
  // block (t, s) element (a, b) stored at a*np + b (a: test on t, b: trial on s;
  // row-major, the operator's layout)
  const int64_t NF = (int64_t)A.faces.size();
  // not value-initialised: face_range zeroes each face's blocks in its own
  // thread (a serial fill of this buffer cost as much as computing it)
  std::vector<double, DefaultInit<double>> fblk((size_t)NF * 4 * np * np);
  const FaceCtx X{&mesh, &G, &A.faces, rho, c_sigma, pp, m, gq.data(), wq.data(), fblk.data()};
  parallel_for(NF, [&](int64_t lo, int64_t hi) {
    switch (p) {
      case 1: face_range<1>(X, lo, hi); break;
      case 2: face_range<2>(X, lo, hi); break;
      case 3: face_range<3>(X, lo, hi); break;
      case 4: face_range<4>(X, lo, hi); break;
      case 5: face_range<5>(X, lo, hi); break;
      case 6: face_range<6>(X, lo, hi); break;
      case 7: face_range<7>(X, lo, hi); break;
      case 8: face_range<8>(X, lo, hi); break;
      default: face_range<9>(X, lo, hi); break;
    }
  });

  std::vector<std::pair<int32_t, int32_t>> pm(A.faces.size());
  for (size_t fi = 0; fi < A.faces.size(); ++fi) pm[fi] = {A.faces[fi].plus, A.faces[fi].minus};
  return finish_assembly(A, subdomain, pm, vol.data(), rhs_c.data(), fblk.data());
}

// P_0 as CSR by internal fine cell from per-caller-cell block lists
// (coarse cells bcol[c], np x nq blocks bval[c]), its transposed lists, and
// the Galerkin A_0 = P_0^T A P_0 (dense). C.q, C.nq, C.n_coarse are set.
void finish_coarse(const Assembled& A, const std::vector<std::vector<int32_t>>& bcol,
                   const std::vector<std::vector<double>>& bval, Coarse& C) {
  const int32_t N = A.n_cells;
  const int np = A.np, nq = C.nq;
  // CSR by internal fine cell
  C.ptr.assign(N + 1, 0);
  for (int32_t r = 0; r < N; ++r) C.ptr[r + 1] = C.ptr[r] + (int32_t)bcol[A.perm[r]].size();
  C.col.resize(C.ptr[N]);
  C.val.resize((size_t)C.ptr[N] * np * nq);
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      const int32_t c = A.perm[r];
      std::copy(bcol[c].begin(), bcol[c].end(), C.col.begin() + C.ptr[r]);
      std::copy(bval[c].begin(), bval[c].end(), C.val.begin() + (size_t)C.ptr[r] * np * nq);
    }
  });
  // transposed lists (coarse cell -> entries in increasing fine order)
  const int32_t nc = C.n_coarse;
  C.tptr.assign(nc + 1, 0);
  for (int32_t e = 0; e < C.ptr[N]; ++e) C.tptr[C.col[e] + 1]++;
  for (int32_t j = 0; j < nc; ++j) C.tptr[j + 1] += C.tptr[j];
  C.tcell.resize(C.ptr[N]);
  C.tblk.resize(C.ptr[N]);
  {
    std::vector<int32_t> fill(C.tptr.begin(), C.tptr.end() - 1);
    for (int32_t r = 0; r < N; ++r)
      for (int32_t e = C.ptr[r]; e < C.ptr[r + 1]; ++e) {
        int32_t k = fill[C.col[e]]++;
        C.tcell[k] = r;
        C.tblk[k] = e;
      }
  }

  // Galerkin A_0 = P_0^T A P_0. W_r = sum over row blocks A[r, s] P_0[s, :]
  // (per fine row, sparse over coarse cells), then rows of A_0 per coarse cell.
  std::vector<std::vector<int32_t>> wcol(N);
  std::vector<std::vector<double>> wval(N);
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      auto& wc = wcol[r];
      auto& wv = wval[r];
      for (int32_t k = A.row_ptr[r]; k < A.row_ptr[r + 1]; ++k) {
        int32_t s = A.col_idx[k];
        const double* Ab = &A.blocks[(size_t)k * np * np];
        for (int32_t e = C.ptr[s]; e < C.ptr[s + 1]; ++e) {
          int32_t J = C.col[e];
          size_t pos = std::find(wc.begin(), wc.end(), J) - wc.begin();
          if (pos == wc.size()) {
            wc.push_back(J);
            wv.resize(wv.size() + (size_t)np * nq, 0.0);
          }
          double* W = &wv[pos * np * nq];
          const double* Pb = &C.val[(size_t)e * np * nq];
          for (int a = 0; a < np; ++a)
            for (int d = 0; d < nq; ++d) {
              double acc = 0.0;
              for (int b = 0; b < np; ++b) acc += Ab[a * np + b] * Pb[b * nq + d];
              W[a * nq + d] += acc;
            }
        }
      }
    }
  });
  const int64_t n0 = (int64_t)nc * nq;
  C.a0.clear();
  C.a0.resize((size_t)(n0 * n0));  // uninitialised, zeroed in parallel (rows of n0)
  parallel_for(n0, [&](int64_t lo, int64_t hi) {
    std::fill(C.a0.begin() + lo * n0, C.a0.begin() + hi * n0, 0.0);
  });
  parallel_for(nc, [&](int64_t lo, int64_t hi) {
    for (int64_t J = lo; J < hi; ++J) {
      for (int32_t k = C.tptr[J]; k < C.tptr[J + 1]; ++k) {
        int32_t r = C.tcell[k];
        const double* Pb = &C.val[(size_t)C.tblk[k] * np * nq];
        for (size_t t = 0; t < wcol[r].size(); ++t) {
          int32_t K = wcol[r][t];
          const double* W = &wval[r][t * np * nq];
          for (int c = 0; c < nq; ++c)
            for (int d = 0; d < nq; ++d) {
              double acc = 0.0;
              for (int a = 0; a < np; ++a) acc += Pb[a * nq + c] * W[a * nq + d];
              C.a0[(size_t)(J * nq + c) * n0 + (size_t)K * nq + d] += acc;
            }
        }
      }
    }
  });
}

namespace {

// Nested coarse transfer of fine cells [lo, hi) without quadrature over the
// cell. Inside a fine cell the coarse basis function psi_(i,j) of its coarse
// element (degree q <= p) is a polynomial of the fine space, so its L2
// projection (M^{-1} B above) is psi itself written in the fine basis
// (Remark 3.2: the injection). Both bases are products of 1D scaled
// Legendre polynomials, orthonormal on their boxes, so the coefficients are
// products of 1D ones: psi_(i,j) = sum_(i',j') Tx[i][i'] Ty[j][j'] phi_(i',j')
// with Tx[i][i'] = int over the fine box's x-interval of the coarse 1D factor
// of degree i times the fine 1D factor of degree i' (zero for i' > i), by
// Gauss-Legendre with p + 1 points (exact for degree i + i' <= 2p).
void nested_exact_range(int p, int q, const CellGeom& G, const int32_t* coarse_of_cell, const std::vector<Box>& cbox,
                        int64_t lo, int64_t hi, std::vector<std::vector<int32_t>>& bcol,
                        std::vector<std::vector<double>>& bval) {
  const int np = n_basis(p), nq = n_basis(q), m = p + 1;
  std::vector<double> gx, gw;
  gauss_legendre01(m, gx, gw);
  // 1D normalised Legendre factors sqrt((2k+1)/len) L_k(2(t - c)/len), k <= kmax
  auto leg = [](double t, double c, double len, int kmax, double* out) {
    const double xi = 2.0 * (t - c) / len;
    double l0 = 1.0, l1 = xi;
    out[0] = 1.0;
    if (kmax >= 1) out[1] = xi;
    for (int k = 1; k < kmax; ++k) {
      const double l2 = ((2 * k + 1) * xi * l1 - k * l0) / (k + 1);
      l0 = l1;
      l1 = l2;
      out[k + 1] = l2;
    }
    for (int k = 0; k <= kmax; ++k) out[k] *= std::sqrt((2.0 * k + 1.0) / len);
  };
  auto transfer = [&](double f0, double f1, double c0, double c1, double* T /* [q+1][p+1] */) {
    const double lf = f1 - f0, lc = c1 - c0, cf = 0.5 * (f0 + f1), cc = 0.5 * (c0 + c1);
    std::fill(T, T + (q + 1) * (p + 1), 0.0);
    double vf[kMaxDegree2D + 1], vc[kMaxDegree2D + 1];
    for (int k = 0; k < m; ++k) {
      const double t = f0 + lf * gx[k], w = lf * gw[k];
      leg(t, cf, lf, p, vf);
      leg(t, cc, lc, q, vc);
      for (int i = 0; i <= q; ++i)
        for (int i2 = 0; i2 <= i; ++i2) T[i * (p + 1) + i2] += w * vc[i] * vf[i2];
    }
  };
  std::vector<double> Tx((q + 1) * (p + 1)), Ty((q + 1) * (p + 1)), B(np * nq);
  for (int64_t c = lo; c < hi; ++c) {
    const int32_t j = coarse_of_cell[c];
    const Box& F = G.box[c];
    const Box& D = cbox[j];
    transfer(F.x0, F.x1, D.x0, D.x1, Tx.data());
    transfer(F.y0, F.y1, D.y0, D.y1, Ty.data());
    // degree-graded order: for d = 0..deg, for jj = 0..d: (d - jj, jj)
    int a = 0;
    for (int d = 0; d <= p; ++d)
      for (int ja = 0; ja <= d; ++ja, ++a) {
        const int ia = d - ja;
        int bb = 0;
        for (int e = 0; e <= q; ++e)
          for (int jb = 0; jb <= e; ++jb, ++bb) {
            const int ib = e - jb;
            B[a * nq + bb] = (ia <= ib && ja <= jb) ? Tx[ib * (p + 1) + ia] * Ty[jb * (p + 1) + ja] : 0.0;
          }
      }
    bcol[c] = {j};
    bval[c].assign(B.begin(), B.end());
  }
}

}  // namespace

std::string build_coarse(const MeshView& fine, const Assembled& A, int q, const int32_t* coarse_of_cell,
                         const MeshView* cmesh, Coarse& C) {
  if (q < 1 || q > A.p) return "coarse degree q must satisfy 1 <= q <= p";
  const int np = A.np, nq = n_basis(q);
  const int32_t N = A.n_cells;
  C.q = q;
  C.nq = nq;
  const int m = A.p + 2;
  std::vector<double> gq, wq;
  gauss_legendre01(m, gq, wq);
  std::vector<std::vector<int32_t>> bcol(N);
  std::vector<std::vector<double>> bval(N);
  std::vector<Box> cbox;
  const CellGeom& G = A.geom;

  // mass matrix of a fine cell (caller index c)
  auto mass = [&](int32_t c, std::vector<QuadPoint>& qp, std::vector<double>& M) {
    double v[kMaxBasis2D];
    cell_points(fine, G, c, gq, wq, qp);
    M.assign(np * np, 0.0);
    BasisBox fbb;
    basis_prepare(A.p, G.box[c], fbb);
    for (auto& P : qp) {
      basis_eval(fbb, P.x, P.y, v, nullptr, nullptr);
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) M[a * np + b] += P.w * v[a] * v[b];
    }
  };

  if (cmesh == nullptr) {
    if (!coarse_of_cell) return "need coarse_of_cell or coarse_mesh";
    int32_t nc = 0;
    for (int32_t c = 0; c < N; ++c) {
      if (coarse_of_cell[c] < 0) return "negative coarse id";
      nc = std::max(nc, coarse_of_cell[c] + 1);
    }
    std::vector<int> used(nc, 0);
    cbox.assign(nc, Box{1e300, -1e300, 1e300, -1e300});
    for (int32_t c = 0; c < N; ++c) {
      int32_t j = coarse_of_cell[c];
      used[j] = 1;
      Box& B = cbox[j];
      B.x0 = std::min(B.x0, G.box[c].x0);
      B.x1 = std::max(B.x1, G.box[c].x1);
      B.y0 = std::min(B.y0, G.box[c].y0);
      B.y1 = std::max(B.y1, G.box[c].y1);
    }
    for (int32_t j = 0; j < nc; ++j)
      if (!used[j]) return "coarse id " + std::to_string(j) + " is unused";
    C.n_coarse = nc;
    parallel_for(N, [&](int64_t lo, int64_t hi) {
      nested_exact_range(A.p, q, G, coarse_of_cell, cbox, lo, hi, bcol, bval);
    });
  } else {
    CellGeom CG;
    std::string err = geometry(*cmesh, CG, true);
    if (!err.empty()) return "coarse mesh: " + err;
    int32_t nc = cmesh->n_cells;
    C.n_coarse = nc;
    cbox = CG.box;
    std::vector<std::vector<double>> cpoly(nc);
    for (int32_t j = 0; j < nc; ++j) cell_polygon(*cmesh, j, cpoly[j]);
    std::atomic<bool> fail{false};
    parallel_for(N, [&](int64_t lo, int64_t hi) {
      std::vector<QuadPoint> qp, cq;
      std::vector<double> M, B(np * nq), P;
      double v[kMaxBasis2D], psi[kMaxBasis2D];
      for (int64_t c = lo; c < hi; ++c) {
        mass((int32_t)c, qp, M);
        cell_polygon(fine, (int32_t)c, P);
        const Box& fb = G.box[c];
        for (int32_t j = 0; j < nc; ++j) {
          const Box& cb = cbox[j];
          if (cb.x0 > fb.x1 || cb.x1 < fb.x0 || cb.y0 > fb.y1 || cb.y1 < fb.y0) continue;
          std::vector<double> Q = clip_polygon(P, cpoly[j]);
          if (Q.empty()) continue;
          double qx, qy;
          double ar = polygon_area_centroid(Q, qx, qy);
          if (!(ar > 0.0)) continue;
          cq.clear();
          polygon_points(Q, gq, wq, cq);
          std::fill(B.begin(), B.end(), 0.0);
          BasisBox fbb, cbb;
          basis_prepare(A.p, fb, fbb);
          basis_prepare(q, cb, cbb);
          for (auto& X : cq) {
            basis_eval(fbb, X.x, X.y, v, nullptr, nullptr);
            basis_eval(cbb, X.x, X.y, psi, nullptr, nullptr);
            for (int a = 0; a < np; ++a)
              for (int b = 0; b < nq; ++b) B[a * nq + b] += X.w * v[a] * psi[b];
          }
          if (!spd_solve(np, M, B.data(), nq)) fail = true;
          bcol[c].push_back(j);
          bval[c].insert(bval[c].end(), B.begin(), B.end());
        }
      }
    });
    if (fail) return "singular fine-cell mass matrix";
    for (int32_t c = 0; c < N; ++c)
      if (bcol[c].empty()) return "fine cell " + std::to_string(c) + " not covered by the coarse mesh";
  }

  finish_coarse(A, bcol, bval, C);
  return "";
}

}  // namespace asdg

namespace {

// sin(pi t) and cos(pi t) for a block of points, written so that the loop
// over points vectorises (no library calls, no branches). Reduction: with
// k the integer nearest t (by the 1.5 * 2^52 rounding trick, exact for
// |t| < 2^51) and r = t - k in [-1/2, 1/2] (exact), sin(pi t) = (-1)^k
// sin(pi r) and cos(pi t) = (-1)^k cos(pi r); for |x| = |pi r| <= pi/2 the
// Taylor series of sin to x^21 and of cos to x^22 leave remainders below
// 2e-18, so the results are within a few ulps of the exact values.
void sincospi_block(const double* t, int64_t stride, int m, double* s, double* c) {
  constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
  constexpr double kPi = 3.141592653589793238462643383279502884;
  // 1 / n! for the odd (sine) and even (cosine) terms
  constexpr double s3 = -1.0 / 6, s5 = 1.0 / 120, s7 = -1.0 / 5040, s9 = 1.0 / 362880, s11 = -1.0 / 39916800,
                   s13 = 1.0 / 6227020800.0, s15 = -1.0 / 1307674368000.0, s17 = 1.0 / 355687428096000.0,
                   s19 = -1.0 / 121645100408832000.0, s21 = 1.0 / 51090942171709440000.0;
  constexpr double c2 = -1.0 / 2, c4 = 1.0 / 24, c6 = -1.0 / 720, c8 = 1.0 / 40320, c10 = -1.0 / 3628800,
                   c12 = 1.0 / 479001600.0, c14 = -1.0 / 87178291200.0, c16 = 1.0 / 20922789888000.0,
                   c18 = -1.0 / 6402373705728000.0, c20 = 1.0 / 2432902008176640000.0,
                   c22 = -1.0 / 1124000727777607680000.0;
  for (int i = 0; i < m; ++i) {
    const double ti = t[(int64_t)i * stride];
    const double k = (ti + kRound) - kRound;
    const double half = (0.5 * k + kRound) - kRound;  // k / 2 rounded: k odd <=> k - 2 half = +-1
    const double sign = 1.0 - 2.0 * std::fabs(k - 2.0 * half);
    const double x = kPi * (ti - k), x2 = x * x;
    const double ps = s3 + x2 * (s5 + x2 * (s7 + x2 * (s9 + x2 * (s11 + x2 * (s13 + x2 * (s15 + x2 * (s17 + x2 * (s19 + x2 * s21))))))));
    const double pc = c2 + x2 * (c4 + x2 * (c6 + x2 * (c8 + x2 * (c10 + x2 * (c12 + x2 * (c14 + x2 * (c16 + x2 * (c18 + x2 * (c20 + x2 * c22)))))))));
    s[i] = sign * (x + x * x2 * ps);
    c[i] = sign * (1.0 + x2 * pc);
  }
}

}  // namespace

// Double sine series load (asdg_field_sine_series): per point one sine and
// one cosine per direction (sincospi_block), the higher frequencies by the
// recurrence sin((k+1)a) = 2 cos(a) sin(ka) - sin((k-1)a); blocks of points
// split over the host threads of the calling assembly, each step a loop over
// the block's points.
extern "C" void asdg_field_sine_series(int64_t n, const double* xy, double* out, void* user) {
  const asdg_sine_series* S = static_cast<const asdg_sine_series*>(user);
  if (!S || !S->coef || S->kx < 1 || S->ky < 1) {
    for (int64_t i = 0; i < n; ++i) out[i] = std::nan("");
    return;
  }
  const int kx = S->kx, ky = S->ky;
  const double* c = S->coef;
  constexpr int B = 64;  // points per block
  asdg::parallel_for(n, [&](int64_t lo, int64_t hi) {
    std::vector<double> sx((size_t)kx * B), sy((size_t)ky * B), cx(B), cy(B), t(B), v(B);
    for (int64_t i0 = lo; i0 < hi; i0 += B) {
      const int m = (int)std::min<int64_t>(B, hi - i0);
      sincospi_block(xy + 2 * i0, 2, m, sx.data(), cx.data());
      sincospi_block(xy + 2 * i0 + 1, 2, m, sy.data(), cy.data());
      for (int i = 0; i < m; ++i) {
        cx[i] *= 2.0;
        cy[i] *= 2.0;
      }
      if (kx > 1)
        for (int i = 0; i < m; ++i) sx[B + i] = cx[i] * sx[i];
      for (int k = 2; k < kx; ++k)
        for (int i = 0; i < m; ++i) sx[k * B + i] = cx[i] * sx[(k - 1) * B + i] - sx[(k - 2) * B + i];
      if (ky > 1)
        for (int i = 0; i < m; ++i) sy[B + i] = cy[i] * sy[i];
      for (int l = 2; l < ky; ++l)
        for (int i = 0; i < m; ++i) sy[l * B + i] = cy[i] * sy[(l - 1) * B + i] - sy[(l - 2) * B + i];
      for (int i = 0; i < m; ++i) v[i] = 0.0;
      for (int k = 0; k < kx; ++k) {
        for (int i = 0; i < m; ++i) t[i] = 0.0;
        for (int l = 0; l < ky; ++l) {
          const double ckl = c[k * ky + l];
          for (int i = 0; i < m; ++i) t[i] += ckl * sy[l * B + i];
        }
        for (int i = 0; i < m; ++i) v[i] += t[i] * sx[k * B + i];
      }
      for (int i = 0; i < m; ++i) out[i0 + i] = v[i];
    }
  });
}
