// Host-side discretisation for tetrahedral meshes: the SIPG system of
// Sec. 2 (eq. (Ah) in flux form, penalty eq. (Sigma) with h the cell
// diameter) and the nested L2 coarse transfer of Sec. 3 (eq. (R0T)), for
// d = 3. Same conventions as the 2D builder (discretize.cpp): scaled
// Legendre basis on the cell's bounding box, m = p + 2 Gauss-Legendre points
// per direction; cells are integrated by the collapsed map of the unit cube
// onto the tetrahedron (exact to total degree 2m - 3) and faces by the
// collapsed triangle rule (exact to 2m - 2).
#include <algorithm>
#include <memory>
#include <cmath>
#include <unordered_map>

#include "discretize.h"

namespace asdg {

namespace {

constexpr int MAXB = 64;  // basis scratch (n_p <= 20 for p <= 3)

struct QP3 {
  double x, y, z, w;
};

double det3(const double* a, const double* b, const double* c, const double* d) {
  const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
  return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) + u[2] * (v[0] * w[1] - v[1] * w[0]);
}

// Points of the tetrahedron (a, b, c, d): X = (1-s) a + s((1-t) b + t((1-u) c + u d)),
// weight 6|T| s^2 t ws wt wu.
void tet_points(const double* a, const double* b, const double* c, const double* d, const std::vector<double>& g,
                const std::vector<double>& wg, std::vector<QP3>& out) {
  const double vol6 = std::fabs(det3(a, b, c, d));
  const int m = (int)g.size();
  out.clear();
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < m; ++k) {
        const double s = g[i], t = g[j], u = g[k];
        QP3 q;
        double X[3];
        for (int e = 0; e < 3; ++e) X[e] = (1.0 - s) * a[e] + s * ((1.0 - t) * b[e] + t * ((1.0 - u) * c[e] + u * d[e]));
        q.x = X[0];
        q.y = X[1];
        q.z = X[2];
        q.w = vol6 * wg[i] * wg[j] * wg[k] * s * s * t;
        out.push_back(q);
      }
}

// Points of the triangle (a, b, c) in space: X = (1-s) a + s((1-t) b + t c), weight 2|T| s ws wt.
void tri_points(const double* a, const double* b, const double* c, const std::vector<double>& g,
                const std::vector<double>& wg, std::vector<QP3>& out) {
  const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  const double area2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  const int m = (int)g.size();
  out.clear();
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double s = g[i], t = g[j];
      QP3 q;
      q.x = (1.0 - s) * a[0] + s * ((1.0 - t) * b[0] + t * c[0]);
      q.y = (1.0 - s) * a[1] + s * ((1.0 - t) * b[1] + t * c[1]);
      q.z = (1.0 - s) * a[2] + s * ((1.0 - t) * b[2] + t * c[2]);
      q.w = area2 * wg[i] * wg[j] * s;
      out.push_back(q);
    }
}

const double* vtx(const TetView& m, int32_t v) { return m.xyz + 3 * (size_t)v; }

}  // namespace

int n_basis3(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

void basis_prepare3(int p, const Box3& B, BasisBox3& bb) {
  bb.p = p;
  bb.d[0] = B.x1 - B.x0;
  bb.d[1] = B.y1 - B.y0;
  bb.d[2] = B.z1 - B.z0;
  bb.c[0] = 0.5 * (B.x0 + B.x1);
  bb.c[1] = 0.5 * (B.y0 + B.y1);
  bb.c[2] = 0.5 * (B.z0 + B.z1);
  for (int e = 0; e < 3; ++e) bb.sc[e] = 2.0 / bb.d[e];
  const double vol = bb.d[0] * bb.d[1] * bb.d[2];
  int a = 0;
  for (int dg = 0; dg <= p; ++dg)
    for (int k = 0; k <= dg; ++k)
      for (int j = 0; j <= dg - k; ++j, ++a) {
        const int i = dg - j - k;
        bb.s[a] = std::sqrt((2.0 * i + 1.0) * (2.0 * j + 1.0) * (2.0 * k + 1.0) / vol);
      }
}

void basis_eval3(const BasisBox3& bb, double x, double y, double z, double* val, double* gx, double* gy,
                 double* gz) {
  const int p = bb.p;
  const double t[3] = {2.0 * (x - bb.c[0]) / bb.d[0], 2.0 * (y - bb.c[1]) / bb.d[1], 2.0 * (z - bb.c[2]) / bb.d[2]};
  double L[3][8], dL[3][8];
  for (int e = 0; e < 3; ++e) {
    L[e][0] = 1.0;
    dL[e][0] = 0.0;
    if (p >= 1) {
      L[e][1] = t[e];
      dL[e][1] = 1.0;
    }
    for (int k = 1; k < p; ++k) {
      L[e][k + 1] = ((2 * k + 1) * t[e] * L[e][k] - k * L[e][k - 1]) / (k + 1);
      dL[e][k + 1] = dL[e][k - 1] + (2 * k + 1) * L[e][k];
    }
  }
  int a = 0;
  for (int dg = 0; dg <= p; ++dg)
    for (int k = 0; k <= dg; ++k)
      for (int j = 0; j <= dg - k; ++j, ++a) {
        const int i = dg - j - k;
        const double s = bb.s[a];
        val[a] = s * L[0][i] * L[1][j] * L[2][k];
        if (gx) gx[a] = s * dL[0][i] * bb.sc[0] * L[1][j] * L[2][k];
        if (gy) gy[a] = s * L[0][i] * dL[1][j] * bb.sc[1] * L[2][k];
        if (gz) gz[a] = s * L[0][i] * L[1][j] * dL[2][k] * bb.sc[2];
      }
}

std::string assemble_sipg_tet(const TetView& mesh, int p, double c_sigma, const double* rho,
                              const int32_t* subdomain,
                              void (*f)(int64_t, const double*, double*, void*), void* f_user, Assembled& A) {
  if (p < 1 || p > 3) return "p must be in 1..3 for tetrahedral meshes";
  if (!(c_sigma > 0.0)) return "c_sigma must be positive";
  const int32_t N = mesh.n_cells;
  if (N < 1) return "empty mesh";
  for (int32_t c = 0; c < N; ++c)
    if (!(rho[c] > 0.0) || !std::isfinite(rho[c])) return "rho must be positive and finite";
  for (int64_t e = 0; e < 4 * (int64_t)N; ++e)
    if (mesh.tets[e] < 0 || mesh.tets[e] >= mesh.n_vertices) return "vertex id out of range";
  A.dim = 3;
  A.p = p;
  A.np = n_basis3(p);
  A.c_sigma = c_sigma;
  A.n_cells = N;
  const int np = A.np;
  A.geom = CellGeom{};
  A.faces.clear();

  // geometry
  A.box3.resize(N);
  A.diam3.resize(N);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v = 0; v < mesh.n_vertices; ++v)
    for (int e = 0; e < 3; ++e) {
      lo[e] = std::min(lo[e], mesh.xyz[3 * (size_t)v + e]);
      hi[e] = std::max(hi[e], mesh.xyz[3 * (size_t)v + e]);
    }
  for (int32_t c = 0; c < N; ++c) {
    const int32_t* T = mesh.tets + 4 * (size_t)c;
    if (!(std::fabs(det3(vtx(mesh, T[0]), vtx(mesh, T[1]), vtx(mesh, T[2]), vtx(mesh, T[3]))) > 0.0))
      return "degenerate tetrahedron " + std::to_string(c);
    Box3 B{1e300, -1e300, 1e300, -1e300, 1e300, -1e300};
    double dm = 0.0;
    for (int i = 0; i < 4; ++i) {
      const double* P = vtx(mesh, T[i]);
      B.x0 = std::min(B.x0, P[0]);
      B.x1 = std::max(B.x1, P[0]);
      B.y0 = std::min(B.y0, P[1]);
      B.y1 = std::max(B.y1, P[1]);
      B.z0 = std::min(B.z0, P[2]);
      B.z1 = std::max(B.z1, P[2]);
      for (int j = 0; j < i; ++j) {
        const double* Q = vtx(mesh, T[j]);
        dm = std::max(dm, std::sqrt((P[0] - Q[0]) * (P[0] - Q[0]) + (P[1] - Q[1]) * (P[1] - Q[1]) +
                                    (P[2] - Q[2]) * (P[2] - Q[2])));
      }
    }
    A.box3[c] = B;
    A.diam3[c] = dm;
  }

  // faces by vertex-triple matching: plus = first cell, triangle and the plus cell's opposite vertex
  struct F3 {
    int32_t plus, minus, v[3], opp;
  };
  std::vector<F3> faces;
  faces.reserve((size_t)N * 2 + 16);
  {
    std::unordered_map<uint64_t, int32_t> open;
    open.reserve((size_t)N * 4);
    const uint64_t V = (uint64_t)mesh.n_vertices;
    if (V >= (1ull << 21)) return "too many vertices for face matching (at most 2^21)";
    static const int loc[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int32_t c = 0; c < N; ++c) {
      const int32_t* T = mesh.tets + 4 * (size_t)c;
      for (int o = 0; o < 4; ++o) {
        int32_t t3[3] = {T[loc[o][0]], T[loc[o][1]], T[loc[o][2]]};
        int32_t s3[3] = {t3[0], t3[1], t3[2]};
        std::sort(s3, s3 + 3);
        if (s3[0] == s3[1] || s3[1] == s3[2]) return "repeated vertex in cell " + std::to_string(c);
        const uint64_t key = ((uint64_t)s3[0] << 42) | ((uint64_t)s3[1] << 21) | (uint64_t)s3[2];
        auto it = open.find(key);
        if (it == open.end()) {
          open.emplace(key, (int32_t)faces.size());
          faces.push_back({c, -1, {t3[0], t3[1], t3[2]}, T[o]});
        } else {
          F3& F = faces[it->second];
          if (F.minus >= 0) return "face shared by more than two cells";
          F.minus = c;
          open.erase(it);
        }
      }
    }
  }
  for (const F3& F : faces) {
    if (F.minus >= 0) continue;
    bool side = false;
    for (int e = 0; e < 3 && !side; ++e)
      for (double b : {lo[e], hi[e]}) {
        bool all = true;
        for (int i = 0; i < 3; ++i) all = all && std::fabs(vtx(mesh, F.v[i])[e] - b) <= 1e-12 * (hi[e] - lo[e]);
        side = side || all;
      }
    if (!side) return "non-conforming mesh: unmatched face inside the domain";
  }

  const int m = p + 2;
  std::vector<double> gq, wq;
  gauss_legendre01(m, gq, wq);
  const double pp = (double)p * (double)p;

  // volume blocks and load vector, caller order (each cell's zeroed by its thread)
  std::unique_ptr<double[]> vol(new double[(size_t)N * np * np]);
  std::unique_ptr<double[]> rhs_c(new double[(size_t)N * np]);
  {
    const int64_t chunk = 8192, per = (int64_t)m * m * m;
    for (int64_t c0 = 0; c0 < N; c0 += chunk) {
      const int64_t c1 = std::min<int64_t>(N, c0 + chunk);
      std::vector<double> pts(3 * (c1 - c0) * per), wts((c1 - c0) * per), fv((c1 - c0) * per, 0.0);
      parallel_for(c1 - c0, [&](int64_t lo_, int64_t hi_) {
        std::vector<QP3> qp;
        for (int64_t cc = lo_; cc < hi_; ++cc) {
          const int32_t* T = mesh.tets + 4 * (size_t)(c0 + cc);
          tet_points(vtx(mesh, T[0]), vtx(mesh, T[1]), vtx(mesh, T[2]), vtx(mesh, T[3]), gq, wq, qp);
          for (int64_t k = 0; k < per; ++k) {
            pts[3 * (cc * per + k)] = qp[k].x;
            pts[3 * (cc * per + k) + 1] = qp[k].y;
            pts[3 * (cc * per + k) + 2] = qp[k].z;
            wts[cc * per + k] = qp[k].w;
          }
        }
      });
      if (f) f((c1 - c0) * per, pts.data(), fv.data(), f_user);
      parallel_for(c1 - c0, [&](int64_t lo_, int64_t hi_) {
        double v[MAXB], gx[MAXB], gy[MAXB], gz[MAXB];
        BasisBox3 bb;
        for (int64_t cc = lo_; cc < hi_; ++cc) {
          const int64_t c = c0 + cc;
          double* K = &vol[(size_t)c * np * np];
          double* bl = &rhs_c[(size_t)c * np];
          std::fill(K, K + np * np, 0.0);
          std::fill(bl, bl + np, 0.0);
          basis_prepare3(p, A.box3[c], bb);
          for (int64_t k = cc * per; k < (cc + 1) * per; ++k) {
            basis_eval3(bb, pts[3 * k], pts[3 * k + 1], pts[3 * k + 2], v, gx, gy, gz);
            const double w = wts[k], wr = w * rho[c];
            // the (a, b) and (b, a) terms are the same products: one triangle, mirrored below
            for (int b = 0; b < np; ++b)
              for (int a = b; a < np; ++a) K[b * np + a] += wr * (gx[a] * gx[b] + gy[a] * gy[b] + gz[a] * gz[b]);
            const double wf = w * fv[k];
            for (int a = 0; a < np; ++a) bl[a] += wf * v[a];
          }
          for (int b = 0; b < np; ++b)
            for (int a = 0; a < b; ++a) K[b * np + a] = K[a * np + b];
        }
      });
    }
  }

  // face blocks (same layout as 2D: interior ++, +-, -+, --; boundary one block)
  const int64_t NF = (int64_t)faces.size();
  // not value-initialised: each face's four blocks are zeroed by its thread
  std::unique_ptr<double[]> fblk(new double[(size_t)NF * 4 * np * np]);
  parallel_for(NF, [&](int64_t lo_, int64_t hi_) {
    double vp[MAXB], gxp[MAXB], gyp[MAXB], gzp[MAXB], vm[MAXB], gxm[MAXB], gym[MAXB], gzm[MAXB];
    double gnp[MAXB], gnm[MAXB];
    std::vector<QP3> qp;
    BasisBox3 bp, bm;
    for (int64_t fi = lo_; fi < hi_; ++fi) {
      const F3& F = faces[fi];
      const double *a = vtx(mesh, F.v[0]), *b = vtx(mesh, F.v[1]), *c = vtx(mesh, F.v[2]);
      const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double w3[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double n[3] = {u[1] * w3[2] - u[2] * w3[1], u[2] * w3[0] - u[0] * w3[2], u[0] * w3[1] - u[1] * w3[0]};
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      const double* o = vtx(mesh, F.opp);
      const double side = n[0] * (o[0] - a[0]) + n[1] * (o[1] - a[1]) + n[2] * (o[2] - a[2]);
      for (int e = 0; e < 3; ++e) n[e] = (side > 0 ? -n[e] : n[e]) / nn;  // outward from the plus cell
      tri_points(a, b, c, gq, wq, qp);
      double* Bk = &fblk[(size_t)fi * 4 * np * np];
      std::fill(Bk, Bk + 4 * np * np, 0.0);
      basis_prepare3(p, A.box3[F.plus], bp);
      if (F.minus >= 0) {
        basis_prepare3(p, A.box3[F.minus], bm);
        const double rp = rho[F.plus], rm = rho[F.minus];
        const double g = 2.0 * rp * rm / (rp + rm);
        const double hp = A.diam3[F.plus], hm = A.diam3[F.minus];
        const double hF = 2.0 * hp * hm / (hp + hm);
        const double sigma = c_sigma * g * pp / hF;
        for (const QP3& q : qp) {
          basis_eval3(bp, q.x, q.y, q.z, vp, gxp, gyp, gzp);
          basis_eval3(bm, q.x, q.y, q.z, vm, gxm, gym, gzm);
          for (int k = 0; k < np; ++k) {
            gnp[k] = gxp[k] * n[0] + gyp[k] * n[1] + gzp[k] * n[2];
            gnm[k] = gxm[k] * n[0] + gym[k] * n[1] + gzm[k] * n[2];
          }
          const double* V[2] = {vp, vm};
          const double* GN[2] = {gnp, gnm};
          const double eps[2] = {1.0, -1.0};
          for (int t = 0; t < 2; ++t)
            for (int s = 0; s < 2; ++s) {
              double* blk = Bk + (t * 2 + s) * np * np;
              const double c1 = -0.5 * g * eps[t] * q.w, c2 = -0.5 * g * eps[s] * q.w;
              const double c3 = sigma * eps[t] * eps[s] * q.w;
              for (int aa = 0; aa < np; ++aa)
                for (int bb = 0; bb < np; ++bb)
                  blk[aa * np + bb] +=
                      c1 * V[t][aa] * GN[s][bb] + c2 * GN[t][aa] * V[s][bb] + c3 * V[t][aa] * V[s][bb];
            }
        }
      } else {
        const double r = rho[F.plus];
        const double sigma = c_sigma * r * pp / A.diam3[F.plus];
        for (const QP3& q : qp) {
          basis_eval3(bp, q.x, q.y, q.z, vp, gxp, gyp, gzp);
          for (int k = 0; k < np; ++k) gnp[k] = gxp[k] * n[0] + gyp[k] * n[1] + gzp[k] * n[2];
          for (int aa = 0; aa < np; ++aa)
            for (int bb = 0; bb < np; ++bb)
              Bk[aa * np + bb] += q.w * (-r * vp[aa] * gnp[bb] - r * gnp[aa] * vp[bb] + sigma * vp[aa] * vp[bb]);
        }
      }
    }
  });
  std::vector<std::pair<int32_t, int32_t>> pm(faces.size());
  for (size_t fi = 0; fi < faces.size(); ++fi) pm[fi] = {faces[fi].plus, faces[fi].minus};
  return finish_assembly(A, subdomain, pm, vol.get(), rhs_c.get(), fblk.get());
}

std::string build_coarse_tet(const TetView& fine, const Assembled& A, int q, const int32_t* coarse_of_cell,
                             Coarse& C) {
  if (A.dim != 3) return "not a tetrahedral system";
  if (q < 1 || q > A.p) return "coarse degree q must satisfy 1 <= q <= p";
  if (!coarse_of_cell) return "tetrahedral meshes need coarse_of_cell (nested agglomerates)";
  const int np = A.np, nq = n_basis3(q);
  const int32_t N = A.n_cells;
  C.q = q;
  C.nq = nq;
  int32_t nc = 0;
  for (int32_t c = 0; c < N; ++c) {
    if (coarse_of_cell[c] < 0) return "negative coarse id";
    nc = std::max(nc, coarse_of_cell[c] + 1);
  }
  std::vector<int> used(nc, 0);
  std::vector<Box3> cbox(nc, Box3{1e300, -1e300, 1e300, -1e300, 1e300, -1e300});
  for (int32_t c = 0; c < N; ++c) {
    const int32_t j = coarse_of_cell[c];
    used[j] = 1;
    Box3& B = cbox[j];
    const Box3& b = A.box3[c];
    B.x0 = std::min(B.x0, b.x0);
    B.x1 = std::max(B.x1, b.x1);
    B.y0 = std::min(B.y0, b.y0);
    B.y1 = std::max(B.y1, b.y1);
    B.z0 = std::min(B.z0, b.z0);
    B.z1 = std::max(B.z1, b.z1);
  }
  for (int32_t j = 0; j < nc; ++j)
    if (!used[j]) return "coarse id " + std::to_string(j) + " is unused";
  C.n_coarse = nc;
  std::vector<double> gq, wq;
  gauss_legendre01(A.p + 2, gq, wq);
  std::vector<std::vector<int32_t>> bcol(N);
  std::vector<std::vector<double>> bval(N);
  bool fail = false;
  parallel_for(N, [&](int64_t lo, int64_t hi) {
    std::vector<QP3> qp;
    std::vector<double> M, B(np * nq);
    double v[MAXB], psi[MAXB];
    for (int64_t c = lo; c < hi; ++c) {
      const int32_t* T = fine.tets + 4 * (size_t)c;
      tet_points(vtx(fine, T[0]), vtx(fine, T[1]), vtx(fine, T[2]), vtx(fine, T[3]), gq, wq, qp);
      const int32_t j = coarse_of_cell[c];
      M.assign((size_t)np * np, 0.0);
      std::fill(B.begin(), B.end(), 0.0);
      BasisBox3 fbb, cbb;
      basis_prepare3(A.p, A.box3[c], fbb);
      basis_prepare3(q, cbox[j], cbb);
      for (const QP3& P : qp) {
        basis_eval3(fbb, P.x, P.y, P.z, v, nullptr, nullptr, nullptr);
        basis_eval3(cbb, P.x, P.y, P.z, psi, nullptr, nullptr, nullptr);
        for (int a = 0; a < np; ++a) {
          for (int b = 0; b < np; ++b) M[a * np + b] += P.w * v[a] * v[b];
          for (int b = 0; b < nq; ++b) B[a * nq + b] += P.w * v[a] * psi[b];
        }
      }
      if (!spd_solve(np, M, B.data(), nq)) fail = true;
      bcol[c] = {j};
      bval[c] = B;
    }
  });
  if (fail) return "singular fine-cell mass matrix";
  finish_coarse(A, bcol, bval, C);
  return "";
}

}  // namespace asdg
