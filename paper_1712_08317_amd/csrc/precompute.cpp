// FP64 precompute of the per-cell coefficients (host).
//
// Paper: Sec. 2 (face length, outer normal and the two Gauss points of eq.
// (quadrature)), Sec. 3.1 (the zero-mean quadratic basis of eq. (base), the
// constraint matrix A_jk = E_j <p^k>_{Omega_ij}, the regularised least
// squares of eq. (quadratic-2), the point-value coefficients eta of eq.
// (polynomial-eta), the candidate linear polynomials on the sub-stencils,
// the matrix B and the linear weights of eq. (linearweight-matrix)),
// Sec. 3.2 (the same for triangles), Sec. 3.3 (the optimisation weights d_j
// and the re-solved weights).
//
// Choices where the paper is silent:
// * every target cell works in its scaled frame xi = (x - centroid)/sqrt|Omega|,
//   so zeta acts on dimensionless matrices;
// * (zeta I + M^T M)^{-1} M^T is evaluated through a one-sided Jacobi SVD
//   as sum_i v_i (M v_i)^T / (s_i^2 + zeta), dropping singular values below
//   1e-12 of the largest (rounding noise of an exactly rank-deficient
//   matrix);
// * the candidate fit keeps the zero-mean form W_i0 + g.(p^1, p^2) and
//   solves the two remaining constraints for g (a 2x2 regularised solve);
// * the optimisation weights d come from each Gauss point's own unoptimised
//   weights (or the largest over the cell's points), one pass.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "uw_host.h"

namespace uw {

namespace {

const double kGA = (3.0 + std::sqrt(3.0)) / 6.0;
const double kGB = (3.0 - std::sqrt(3.0)) / 6.0;
constexpr double kRankTol = 1e-12;

struct Poly {
  double p[4][2];
  int nf;
};

// Exact integrals of 1, x, y, x^2, y^2, xy over a counter-clockwise polygon:
// signed fan from vertex 0, the three-edge-midpoint rule on each triangle.
void moments(const Poly& P, double mom[6]) {
  for (int q = 0; q < 6; ++q) mom[q] = 0.0;
  for (int k = 1; k + 1 < P.nf; ++k) {
    const double* a = P.p[0];
    const double* b = P.p[k];
    const double* c = P.p[k + 1];
    double t = 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]));
    double f[6] = {0, 0, 0, 0, 0, 0};
    const double mids[3][2] = {{0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1])},
                               {0.5 * (b[0] + c[0]), 0.5 * (b[1] + c[1])},
                               {0.5 * (c[0] + a[0]), 0.5 * (c[1] + a[1])}};
    for (const auto& m : mids) {
      double x = m[0], y = m[1];
      f[0] += 1.0;
      f[1] += x;
      f[2] += y;
      f[3] += x * x;
      f[4] += y * y;
      f[5] += x * y;
    }
    for (int q = 0; q < 6; ++q) mom[q] += (t / 3.0) * f[q];
  }
}

}  // namespace

int tikhonov(const double* Mat, int m, int n, double zeta, double* X) {
  // columns padded to 16 rows
  alignas(64) double a[12][16];
  alignas(64) double v[12][12];
  double nrm[12];
  for (int j = 0; j < n; ++j) {
    for (int r = 0; r < 16; ++r) a[j][r] = r < m ? Mat[r * n + j] : 0.0;
    for (int r = 0; r < 12; ++r) v[j][r] = (r == j) ? 1.0 : 0.0;
  }
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int r = 0; r < 16; ++r) s += a[j][r] * a[j][r];
    nrm[j] = s;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    // columns below 1e-13 of the largest are dropped as rank noise at the
    // end, so they need not be orthogonalised (rotating noise never converges)
    double big = 0.0;
    for (int j = 0; j < n; ++j) big = std::max(big, nrm[j]);
    const double tiny = 1e-26 * big;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double al = nrm[p], be = nrm[q];
        if (al <= tiny || be <= tiny) continue;
        double g = 0.0;
        for (int r = 0; r < 16; ++r) g += a[p][r] * a[q][r];
        if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(al * be)) continue;
        rotated = true;
        const double z = (be - al) / (2.0 * g);
        const double t = (z >= 0.0 ? 1.0 : -1.0) / (std::fabs(z) + std::sqrt(1.0 + z * z));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        double np = 0.0, nq = 0.0;
        for (int r = 0; r < 16; ++r) {
          const double x = a[p][r], y = a[q][r];
          const double xp = c * x - s * y, yq = s * x + c * y;
          a[p][r] = xp;
          a[q][r] = yq;
          np += xp * xp;
          nq += yq * yq;
        }
        nrm[p] = np;
        nrm[q] = nq;
        for (int r = 0; r < 12; ++r) {
          const double x = v[p][r], y = v[q][r];
          v[p][r] = c * x - s * y;
          v[q][r] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  double smax = 0.0;
  for (int j = 0; j < n; ++j) smax = std::max(smax, std::sqrt(nrm[j]));
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < m; ++r) X[c * m + r] = 0.0;
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double sj = std::sqrt(nrm[j]);
    if (!(sj > kRankTol * smax)) continue;
    ++rank;
    const double f = 1.0 / (nrm[j] + zeta);
    for (int c = 0; c < n; ++c) {
      const double vc = v[j][c] * f;
      for (int r = 0; r < m; ++r) X[c * m + r] += vc * a[j][r];
    }
  }
  return rank;
}

namespace {

struct CellOut {
  double Y[12][4];
  double off[8][2];
  double gam[8][12];
  double gam_raw[8][12];
  double eta[8][13];
  double area;
  double normal[4][2];
  double length[4];
  double max_raw, max_opt, resid, sumdev;
  int absent;
  bool rank_def;
};

void cell_polygon(const HostMesh& m, int64_t c, const double* shift, Poly& P) {
  P.nf = m.nf[c];
  for (int k = 0; k < P.nf; ++k) {
    const int32_t v = m.cell_nodes[4 * c + k];
    P.p[k][0] = m.xy[2 * v] + (shift ? shift[0] : 0.0);
    P.p[k][1] = m.xy[2 * v + 1] + (shift ? shift[1] : 0.0);
  }
}

void precompute_cell(const HostMesh& m, const SchemeParams& sp, int64_t i, CellOut& o) {
  const TypeConst& T = type_const(m.nf[i]);
  const int n = T.n, S = T.S, M = T.M, G = 2 * n;
  std::memset(&o, 0, sizeof(o));

  // target polygon, area and centroid (moments relative to vertex 0)
  Poly P0;
  cell_polygon(m, i, nullptr, P0);
  Poly rel = P0;
  for (int k = 0; k < n; ++k) {
    rel.p[k][0] -= P0.p[0][0];
    rel.p[k][1] -= P0.p[0][1];
  }
  double mom[6];
  moments(rel, mom);
  const double area = mom[0];
  const double cx = P0.p[0][0] + mom[1] / mom[0], cy = P0.p[0][1] + mom[2] / mom[0];
  const double h0 = std::sqrt(area);
  o.area = area;
  auto to_xi = [&](double x, double y, double* out) {
    out[0] = (x - cx) / h0;
    out[1] = (y - cy) / h0;
  };
  Poly X0;
  X0.nf = n;
  for (int k = 0; k < n; ++k) to_xi(P0.p[k][0], P0.p[k][1], X0.p[k]);

  // cell averages of xi, eta, xi^2, eta^2, xi eta over every present slot
  const int32_t* st_cell = &m.st_cell[kMaxS * i];
  const double* st_shift = &m.st_shift[2 * kMaxS * i];
  const int8_t* st_ghost = &m.st_ghost[kMaxS * i];
  const int8_t* st_res = &m.st_res[kMaxS * i];
  const uint8_t* present = &m.st_present[kMaxS * i];
  double avg[kMaxS][5];
  for (int j = 0; j < S; ++j) {
    for (int q = 0; q < 5; ++q) avg[j][q] = 0.0;
    if (!present[j]) {
      o.absent++;
      continue;
    }
    Poly Q;
    if (j > 0 && st_ghost[j] >= 0) {
      // mirror image of the target across the boundary face
      const int k = st_ghost[j];
      const double* a = X0.p[k];
      const double* b = X0.p[(k + 1) % n];
      double nx = b[1] - a[1], ny = -(b[0] - a[0]);
      const double ln = std::sqrt(nx * nx + ny * ny);
      nx /= ln;
      ny /= ln;
      Poly R;
      R.nf = n;
      for (int q = 0; q < n; ++q) {
        const double s = (X0.p[q][0] - a[0]) * nx + (X0.p[q][1] - a[1]) * ny;
        R.p[q][0] = X0.p[q][0] - 2.0 * s * nx;
        R.p[q][1] = X0.p[q][1] - 2.0 * s * ny;
      }
      Q.nf = n;
      Q.p[0][0] = R.p[0][0];
      Q.p[0][1] = R.p[0][1];
      for (int q = 1; q < n; ++q) {  // reverse the order: counter-clockwise again
        Q.p[q][0] = R.p[n - q][0];
        Q.p[q][1] = R.p[n - q][1];
      }
    } else {
      Poly raw;
      cell_polygon(m, st_cell[j], st_shift + 2 * j, raw);
      Q.nf = raw.nf;
      for (int k = 0; k < raw.nf; ++k) to_xi(raw.p[k][0], raw.p[k][1], Q.p[k]);
    }
    double mo[6];
    moments(Q, mo);
    for (int q = 0; q < 5; ++q) avg[j][q] = mo[q + 1] / mo[0];
  }
  double mean0[5];
  for (int q = 0; q < 5; ++q) mean0[q] = avg[0][q];
  double basis[kMaxS][5];  // cell averages of the zero-mean basis functions
  for (int j = 0; j < S; ++j)
    for (int q = 0; q < 5; ++q) basis[j][q] = present[j] ? avg[j][q] - mean0[q] : 0.0;

  // A (S-1) x 5, row-major; E mask
  double A[12 * 5], E[12];
  for (int j = 1; j < S; ++j) {
    E[j - 1] = present[j] ? 1.0 : 0.0;
    for (int q = 0; q < 5; ++q) A[(j - 1) * 5 + q] = basis[j][q];
  }

  // faces and Gauss points
  double pG[8][5];
  for (int k = 0; k < n; ++k) {
    const double* a = P0.p[k];
    const double* b = P0.p[(k + 1) % n];
    const double ex = b[0] - a[0], ey = b[1] - a[1];
    const double ln = std::sqrt(ex * ex + ey * ey);
    o.length[k] = ln;
    o.normal[k][0] = ey / ln;
    o.normal[k][1] = -ex / ln;
    for (int q = 0; q < 2; ++q) {
      const double wa = q == 0 ? kGA : kGB, wb = q == 0 ? kGB : kGA;
      double xi[2];
      to_xi(wa * a[0] + wb * b[0], wa * a[1] + wb * b[1], xi);
      double* p = pG[2 * k + q];
      p[0] = xi[0] - mean0[0];
      p[1] = xi[1] - mean0[1];
      p[2] = xi[0] * xi[0] - mean0[2];
      p[3] = xi[1] * xi[1] - mean0[3];
      p[4] = xi[0] * xi[1] - mean0[4];
      o.off[2 * k + q][0] = p[0];
      o.off[2 * k + q][1] = p[1];
    }
  }

  // eta with row weights D (all ones for the unoptimised pass)
  auto eta_at = [&](const double* D, const double* p, double* eta_out) {
    double DA[12 * 5], X[5 * 12];
    for (int j = 0; j < S - 1; ++j)
      for (int q = 0; q < 5; ++q) DA[j * 5 + q] = D[j] * A[j * 5 + q];
    tikhonov(DA, S - 1, 5, sp.zeta, X);
    double s = 0.0;
    for (int j = 0; j < S - 1; ++j) {
      double e = 0.0;
      for (int q = 0; q < 5; ++q) e += p[q] * X[q * (S - 1) + j];
      e *= D[j] * E[j];
      eta_out[j + 1] = e;
      s += e;
    }
    eta_out[0] = 1.0 - s;
  };
  // the unoptimised operator is shared by all Gauss points
  double eta_raw[8][13];
  {
    double X[5 * 12];
    int rk = tikhonov(A, S - 1, 5, sp.zeta, X);
    o.rank_def = rk < 5;
    for (int g = 0; g < G; ++g) {
      double s = 0.0;
      for (int j = 0; j < S - 1; ++j) {
        double e = 0.0;
        for (int q = 0; q < 5; ++q) e += pG[g][q] * X[q * (S - 1) + j];
        e *= E[j];
        eta_raw[g][j + 1] = e;
        s += e;
      }
      eta_raw[g][0] = 1.0 - s;
    }
  }

  // candidate operators Y_j: g = Y_j (dW_a, dW_b)
  for (int j = 0; j < M; ++j) {
    const int sa = T.sub_a[j], sb = st_res[T.sub_b[j]];
    double Mj[4] = {basis[sa][0], basis[sa][1], basis[sb][0], basis[sb][1]};
    double Xj[4];
    tikhonov(Mj, 2, 2, sp.zeta, Xj);
    for (int e = 0; e < 4; ++e) o.Y[j][e] = Xj[e];  // [c][r]: Y00 Y01 Y10 Y11
  }

  // per Gauss point: B (shared by both passes), gamma before the optimisation
  double B[8][13 * 12], PB[8][12 * 13];
  for (int g = 0; g < G; ++g) {
    double* Bg = B[g];
    for (int e = 0; e < S * M; ++e) Bg[e] = 0.0;
    const double ox = pG[g][0], oy = pG[g][1];
    for (int j = 0; j < M; ++j) {
      const double ba = ox * o.Y[j][0] + oy * o.Y[j][2];
      const double bb = ox * o.Y[j][1] + oy * o.Y[j][3];
      const int sa = T.sub_a[j], sb = st_res[T.sub_b[j]];
      Bg[0 * M + j] += 1.0 - ba - bb;
      Bg[sa * M + j] += ba;
      Bg[sb * M + j] += bb;
    }
    tikhonov(Bg, S, M, sp.zeta, PB[g]);
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int r = 0; r < S; ++r) s += PB[g][j * S + r] * eta_raw[g][r];
      o.gam_raw[g][j] = s;
      o.gam[g][j] = s;
    }
    for (int r = 0; r < S; ++r) o.eta[g][r] = eta_raw[g][r];
  }
  // optimisation: row weights d from |gamma|, weighted least squares, re-solve
  if (sp.optimize) {
    double cellmax[12];
    for (int j = 0; j < M; ++j) {
      cellmax[j] = 0.0;
      for (int g = 0; g < G; ++g) cellmax[j] = std::max(cellmax[j], std::fabs(o.gam_raw[g][j]));
    }
    for (int g = 0; g < G; ++g) {
      double D[12];
      for (int s = 1; s < S; ++s) {
        double big = 1.0;
        const int c0 = T.d_c0[s], c1 = T.d_c1[s];
        auto mag = [&](int c) {
          return sp.d_scope == 1 ? cellmax[c - 1] : std::fabs(o.gam_raw[g][c - 1]);
        };
        if (c0) big = std::max(big, mag(c0));
        if (c1) big = std::max(big, mag(c1));
        D[s - 1] = 1.0 / big;
      }
      eta_at(D, pG[g], o.eta[g]);
      for (int j = 0; j < M; ++j) {
        double s = 0.0;
        for (int r = 0; r < S; ++r) s += PB[g][j * S + r] * o.eta[g][r];
        o.gam[g][j] = s;
      }
    }
  }
  // diagnostics: ||B gamma - eta||_inf and |sum gamma - 1|
  for (int g = 0; g < G; ++g) {
    double sg = 0.0;
    for (int r = 0; r < S; ++r) {
      double s = 0.0;
      for (int j = 0; j < M; ++j) s += B[g][r * M + j] * o.gam[g][j];
      o.resid = std::max(o.resid, std::fabs(s - o.eta[g][r]));
    }
    for (int j = 0; j < M; ++j) sg += o.gam[g][j];
    o.sumdev = std::max(o.sumdev, std::fabs(sg - 1.0));
  }
  for (int g = 0; g < G; ++g)
    for (int j = 0; j < M; ++j) {
      o.max_raw = std::max(o.max_raw, std::fabs(o.gam_raw[g][j]));
      o.max_opt = std::max(o.max_opt, std::fabs(o.gam[g][j]));
    }
}

}  // namespace

void precompute_tables(const HostMesh& m, const SchemeParams& sp, HostTables& t, int threads) {
  const int64_t N = m.N, Nq = m.Nq, Nt = N - Nq;
  t.quad.Nt = Nq;
  t.quad.first = 0;
  t.tri.Nt = Nt;
  t.tri.first = Nq;
  const bool linear = sp.mode == 1;
  for (TypeTables* tt : {&t.quad, &t.tri}) {
    const TypeConst& T = (tt == &t.quad) ? kQuad : kTri;
    const int64_t n = tt->Nt;
    tt->sid.assign((T.S - 1) * n, 0);
    tt->Y.assign(T.M * 4 * n, 0.0);
    tt->off.assign(2 * T.n * 2 * n, 0.0);
    tt->gam.assign(2 * T.n * T.M * n, 0.0);
    tt->eta.assign(linear ? 2 * T.n * (T.S - 1) * n : 0, 0.0);
  }
  t.area.assign(N, 0.0);
  t.debug = N <= 4000000;
  if (t.debug) {
    t.dbg_gamma.assign(N * 96, 0.0);
    t.dbg_gamma_raw.assign(N * 96, 0.0);
    t.dbg_eta.assign(N * 104, 0.0);
    t.dbg_Y.assign(N * 48, 0.0);
    t.dbg_off.assign(N * 16, 0.0);
    t.dbg_face.assign(N * 12, 0.0);
  }
  std::vector<double> normal(8 * N), length(4 * N);
  std::atomic<int64_t> absent{0}, rankdef{0};
  struct Acc {
    double a = 0, b = 0, c = 0, d = 0;
  };
  std::vector<Acc> acc(N ? (N + 1023) / 1024 : 1);

  parallel_for(N, threads, [&](int64_t s, int64_t e) {
    CellOut o;
    Acc local;
    int64_t la = 0, lr = 0;
    for (int64_t i = s; i < e; ++i) {
      precompute_cell(m, sp, i, o);
      const TypeConst& T = type_const(m.nf[i]);
      const bool q = i < Nq;
      TypeTables& tt = q ? t.quad : t.tri;
      const int64_t r = i - tt.first, n = tt.Nt;
      const int32_t* cell = &m.st_cell[kMaxS * i];
      const int8_t* res = &m.st_res[kMaxS * i];
      for (int s2 = 1; s2 < T.S; ++s2) tt.sid[(s2 - 1) * n + r] = cell[res[s2]];
      for (int j = 0; j < T.M; ++j)
        for (int c = 0; c < 4; ++c) tt.Y[(j * 4 + c) * n + r] = o.Y[j][c];
      for (int g = 0; g < 2 * T.n; ++g) {
        tt.off[(g * 2) * n + r] = o.off[g][0];
        tt.off[(g * 2 + 1) * n + r] = o.off[g][1];
        for (int j = 0; j < T.M; ++j) tt.gam[(g * T.M + j) * n + r] = o.gam[g][j];
        if (linear)
          for (int s2 = 1; s2 < T.S; ++s2) tt.eta[(g * (T.S - 1) + s2 - 1) * n + r] = o.eta[g][s2];
      }
      t.area[i] = o.area;
      for (int k = 0; k < 4; ++k) {
        normal[8 * i + 2 * k] = o.normal[k][0];
        normal[8 * i + 2 * k + 1] = o.normal[k][1];
        length[4 * i + k] = o.length[k];
      }
      if (t.debug) {
        for (int g = 0; g < 8; ++g) {
          for (int j = 0; j < 12; ++j) {
            t.dbg_gamma[i * 96 + g * 12 + j] = o.gam[g][j];
            t.dbg_gamma_raw[i * 96 + g * 12 + j] = o.gam_raw[g][j];
          }
          for (int s2 = 0; s2 < 13; ++s2) t.dbg_eta[i * 104 + g * 13 + s2] = o.eta[g][s2];
          t.dbg_off[i * 16 + 2 * g] = o.off[g][0];
          t.dbg_off[i * 16 + 2 * g + 1] = o.off[g][1];
        }
        for (int j = 0; j < 12; ++j)
          for (int c = 0; c < 4; ++c) t.dbg_Y[i * 48 + j * 4 + c] = o.Y[j][c];
      }
      local.a = std::max(local.a, o.max_raw);
      local.b = std::max(local.b, o.max_opt);
      local.c = std::max(local.c, o.resid);
      local.d = std::max(local.d, o.sumdev);
      la += o.absent;
      lr += o.rank_def ? 1 : 0;
    }
    acc[s / 1024] = local;
    absent += la;
    rankdef += lr;
  });
  for (const Acc& a : acc) {
    t.max_abs_gamma_raw = std::max(t.max_abs_gamma_raw, a.a);
    t.max_abs_gamma_opt = std::max(t.max_abs_gamma_opt, a.b);
    t.resid_opt = std::max(t.resid_opt, a.c);
    t.sum_dev = std::max(t.sum_dev, a.d);
  }
  t.n_absent = absent;
  t.n_rank_def = rankdef;

  // LDS staging lists of every tile of kTile consecutive cells
  for (TypeTables* tt : {&t.quad, &t.tri}) {
    const TypeConst& T = (tt == &t.quad) ? kQuad : kTri;
    const int64_t n = tt->Nt, nt = (n + kTile - 1) / kTile;
    std::vector<std::vector<int32_t>> lists(nt);
    tt->lidx.assign((size_t)T.S * n, 0);
    parallel_for(nt, threads, [&](int64_t s0, int64_t e0) {
      std::vector<int32_t> ids;
      for (int64_t tile = s0; tile < e0; ++tile) {
        const int64_t r0 = tile * kTile, r1 = std::min(n, r0 + kTile);
        ids.clear();
        for (int64_t r = r0; r < r1; ++r) {
          ids.push_back((int32_t)(tt->first + r));
          for (int s2 = 1; s2 < T.S; ++s2) ids.push_back(tt->sid[(s2 - 1) * n + r]);
        }
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        for (int64_t r = r0; r < r1; ++r)
          for (int s2 = 0; s2 < T.S; ++s2) {
            const int32_t id = s2 == 0 ? (int32_t)(tt->first + r) : tt->sid[(s2 - 1) * n + r];
            tt->lidx[s2 * n + r] =
                (uint16_t)(std::lower_bound(ids.begin(), ids.end(), id) - ids.begin());
          }
        lists[tile] = ids;
      }
    });
    tt->tile_off.assign(nt + 1, 0);
    tt->max_tile_len = 0;
    for (int64_t k = 0; k < nt; ++k) {
      tt->tile_off[k + 1] = tt->tile_off[k] + (int32_t)lists[k].size();
      tt->max_tile_len = std::max<int32_t>(tt->max_tile_len, (int32_t)lists[k].size());
    }
    tt->tile_ids.resize(tt->tile_off[nt]);
    for (int64_t k = 0; k < nt; ++k)
      std::copy(lists[k].begin(), lists[k].end(), tt->tile_ids.begin() + tt->tile_off[k]);
  }

  // face tables: the canonical normal and length are the left cell's
  t.fnb.assign(4 * N, -1);
  t.fgeo.assign(12 * N, 0.0);
  parallel_for(N, threads, [&](int64_t s, int64_t e) {
    for (int64_t i = s; i < e; ++i) {
      for (int k = 0; k < m.nf[i]; ++k) {
        const int32_t nb = m.nbr[4 * i + k];
        const bool left = m.left[4 * i + k] != 0;
        double nx, ny, ln;
        if (nb < 0 || left) {
          nx = normal[8 * i + 2 * k];
          ny = normal[8 * i + 2 * k + 1];
          ln = length[4 * i + k];
        } else {
          const int kp = m.nbr_face[4 * i + k];
          nx = normal[8 * nb + 2 * kp];
          ny = normal[8 * nb + 2 * kp + 1];
          ln = length[4 * nb + kp];
        }
        if (nb >= 0)
          t.fnb[k * N + i] = (nb << 3) | (m.nbr_face[4 * i + k] << 1) | (left ? 1 : 0);
        const double coef = ln / (2.0 * t.area[i]);
        t.fgeo[(k * 3 + 0) * N + i] = nx;
        t.fgeo[(k * 3 + 1) * N + i] = ny;
        t.fgeo[(k * 3 + 2) * N + i] = coef;
        if (t.debug) {
          t.dbg_face[i * 12 + k * 3 + 0] = nx;
          t.dbg_face[i * 12 + k * 3 + 1] = ny;
          t.dbg_face[i * 12 + k * 3 + 2] = coef;
        }
      }
    }
  });
}

}  // namespace uw
