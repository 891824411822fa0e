// Per-cell FP64 precompute shared by the host (threads) and the device (one
// GPU thread per cell): the same source, compiled by g++ and by hipcc.
//
// Paper: Sec. 2 (face length, outer normal, the two Gauss points of eq.
// (quadrature)), Sec. 3.1 (the zero-mean quadratic basis of eq. (base), the
// constraint matrix A_jk = E_j <p^k>_{Omega_ij}, the regularised least
// squares of eq. (quadratic-2), the point-value coefficients eta of eq.
// (polynomial-eta), the candidate polynomials on the sub-stencils, the
// matrix B and the linear weights of eq. (linearweight-matrix)), Sec. 3.2
// (the same for triangles), Sec. 3.3 (the weights d_j and the optimised
// linear weights).
//
// Choices where the paper is silent:
// * every target cell works in its scaled frame xi = (x - centroid)/sqrt|Omega|,
//   so zeta acts on dimensionless matrices;
// * (zeta I + M^T M)^{-1} M^T is evaluated through a one-sided Jacobi SVD as
//   sum_i v_i (M v_i)^T / (s_i^2 + zeta), dropping singular values below
//   1e-12 of the largest (rounding noise of an exactly rank-deficient matrix);
// * the candidate fit keeps the zero-mean form W_i0 + g.(p^1, p^2) and solves
//   the two remaining constraints for g (a 2x2 regularised solve);
// * the optimisation weights d come from each Gauss point's own unoptimised
//   weights (or the largest over the cell's points), one pass;
// * optimised weights below 1e-10 in magnitude are zero: they are rounding
//   residue of O(1) terms (degenerate candidates next to boundaries), and a
//   rounding-level weight on a candidate with a zero smoothness indicator
//   would outweigh every other candidate in the nonlinear weights.
#pragma once

#include <cmath>
#include <cstdint>

#ifdef __HIPCC__
#define UW_HD __host__ __device__
#else
#define UW_HD
#endif

namespace uw {
namespace geom {

constexpr double kRankTol = 1e-12;
constexpr double kGammaZero = 1e-10;
// Gauss points of eq. (quadrature): (3 +- sqrt3)/6
constexpr double kGA = 0.78867513459481288225457439025097872782380087563506;
constexpr double kGB = 0.21132486540518711774542560974902127217619912436494;

// Stencil type constants (see TypeConst in uw_host.h), passed by value.
struct TypeC {
  int n, S, M;
  int sub_a[12], sub_b[12];
  int d_c0[13], d_c1[13];
};

// Read-only views of one mesh (internal numbering).
struct CellIn {
  const int32_t* nf;          // [N]
  const int32_t* cell_nodes;  // [N*4]
  const double* xy;           // [n_nodes*2]
  const int32_t* st_cell;     // [N*13]
  const double* st_shift;     // [N*13*2]
  const int8_t* st_ghost;     // [N*13]
  const int8_t* st_res;       // [N*13]
  const uint8_t* st_present;  // [N*13]
  int64_t Nq;                 // cells [0, Nq) are quadrilaterals
};

// Where the results of one cell type go (structure of arrays [k][n]).
struct TypeOut {
  double* Y;     // [M*4][n]
  double* off;   // [2n*2][n]
  double* gam;   // [2n*M][n] gamma_j / (2 sigma+) per Gauss point (split form)
  double* sig;   // [2n*3][n] sigma+, sigma-, sigma+ / sigma- per Gauss point
  double* eta;   // [2n*(S-1)][n] or null
  int32_t* sid;  // [S-1][n]
  int64_t n;
};

struct CellOut {
  TypeOut quad, tri;
  double* area;     // [N]
  double* normal;   // [N][4][2] own outer normals
  double* length;   // [N][4]
  double* diag;     // [N][4]: max|gamma| raw, max|gamma| opt, ||B gamma - eta||_inf, |sum gamma - 1|
  int32_t* counts;  // [N][2]: absent slots, rank(A) < 5
  // full per-cell copies, host only (null on the device)
  double* dbg_gamma;      // [N][8][12]
  double* dbg_gamma_raw;  // [N][8][12]
  double* dbg_eta;        // [N][8][13]
  double* dbg_Y;          // [N][12][4]
  double* dbg_off;        // [N][8][2]
};

struct Params {
  double zeta, theta;
  int optimize, d_scope, linear;
};

struct Poly {
  double p[4][2];
  int nf;
};

// Exact integrals of 1, x, y, x^2, y^2, xy over a counter-clockwise polygon:
// signed fan from vertex 0, the three-edge-midpoint rule on each triangle.
UW_HD inline void moments(const Poly& P, double mom[6]) {
  for (int q = 0; q < 6; ++q) mom[q] = 0.0;
  for (int k = 1; k + 1 < P.nf; ++k) {
    const double* a = P.p[0];
    const double* b = P.p[k];
    const double* c = P.p[k + 1];
    const double t = 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]));
    double f[6] = {0, 0, 0, 0, 0, 0};
    const double mids[3][2] = {{0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1])},
                               {0.5 * (b[0] + c[0]), 0.5 * (b[1] + c[1])},
                               {0.5 * (c[0] + a[0]), 0.5 * (c[1] + a[1])}};
    for (int m = 0; m < 3; ++m) {
      const double x = mids[m][0], y = mids[m][1];
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

// X = (zeta I + M^T M)^{-1} M^T for an m x n matrix (m >= n, row-major,
// m <= 13, n <= 12), X row-major n x m.  Returns the numerical rank.
UW_HD inline int tikhonov(const double* Mat, int m, int n, double zeta, double* X) {
  double a[12][16];
  double v[12][12];
  double nrm[12];
  for (int j = 0; j < n; ++j) {
    for (int r = 0; r < 16; ++r) a[j][r] = r < m ? Mat[r * n + j] : 0.0;
    for (int r = 0; r < 12; ++r) v[j][r] = (r == j) ? 1.0 : 0.0;
  }
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int r = 0; r < m; ++r) s += a[j][r] * a[j][r];
    nrm[j] = s;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    // columns below 1e-13 of the largest are dropped as rank noise at the
    // end, so they need not be orthogonalised (rotating noise never converges)
    double big = 0.0;
    for (int j = 0; j < n; ++j) big = big > nrm[j] ? big : nrm[j];
    const double tiny = 1e-26 * big;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double al = nrm[p], be = nrm[q];
        if (al <= tiny || be <= tiny) continue;
        double g = 0.0;
        for (int r = 0; r < m; ++r) g += a[p][r] * a[q][r];
        if (g == 0.0 || fabs(g) <= 1e-15 * sqrt(al * be)) continue;
        rotated = true;
        const double z = (be - al) / (2.0 * g);
        const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        double np = 0.0, nq = 0.0;
        for (int r = 0; r < m; ++r) {
          const double x = a[p][r], y = a[q][r];
          const double xp = c * x - s * y, yq = s * x + c * y;
          a[p][r] = xp;
          a[q][r] = yq;
          np += xp * xp;
          nq += yq * yq;
        }
        nrm[p] = np;
        nrm[q] = nq;
        for (int r = 0; r < n; ++r) {
          const double x = v[p][r], y = v[q][r];
          v[p][r] = c * x - s * y;
          v[q][r] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  double smax = 0.0;
  for (int j = 0; j < n; ++j) {
    const double sj = sqrt(nrm[j]);
    smax = smax > sj ? smax : sj;
  }
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < m; ++r) X[c * m + r] = 0.0;
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    if (!(sqrt(nrm[j]) > kRankTol * smax)) continue;
    ++rank;
    const double f = 1.0 / (nrm[j] + zeta);
    for (int c = 0; c < n; ++c) {
      const double vc = v[j][c] * f;
      for (int r = 0; r < m; ++r) X[c * m + r] += vc * a[j][r];
    }
  }
  return rank;
}

UW_HD inline void cell_polygon(const CellIn& in, int64_t c, const double* shift, Poly& P) {
  P.nf = in.nf[c];
  for (int k = 0; k < P.nf; ++k) {
    const int32_t v = in.cell_nodes[4 * c + k];
    P.p[k][0] = in.xy[2 * v] + (shift ? shift[0] : 0.0);
    P.p[k][1] = in.xy[2 * v + 1] + (shift ? shift[1] : 0.0);
  }
}

// B at one Gauss point (row = stencil slot, column = candidate), then its
// regularised pseudo-inverse PB (M x S).
UW_HD inline void weight_matrix(const TypeC& T, const int8_t* st_res, const double Y[12][4],
                                const double* pg, double* B, double* PB, double zeta) {
  const int S = T.S, M = T.M;
  for (int e = 0; e < S * M; ++e) B[e] = 0.0;
  for (int j = 0; j < M; ++j) {
    const double ba = pg[0] * Y[j][0] + pg[1] * Y[j][2];
    const double bb = pg[0] * Y[j][1] + pg[1] * Y[j][3];
    const int sa = T.sub_a[j], sb = st_res[T.sub_b[j]];
    B[0 * M + j] += 1.0 - ba - bb;
    B[sa * M + j] += ba;
    B[sb * M + j] += bb;
  }
  tikhonov(B, S, M, zeta, PB);
}

// eta at one Gauss point from the operator X = (zeta I + (DA)^T DA)^{-1} (DA)^T
// of row weights D (null = all ones).
UW_HD inline void eta_from(const TypeC& T, const double* X, const double* E, const double* D,
                           const double* pg, double* eta) {
  const int S = T.S;
  double s = 0.0;
  for (int j = 0; j < S - 1; ++j) {
    double e = 0.0;
    for (int q = 0; q < 5; ++q) e += pg[q] * X[q * (S - 1) + j];
    e *= (D ? D[j] : 1.0) * E[j];
    eta[j + 1] = e;
    s += e;
  }
  eta[0] = 1.0 - s;
}

// eta at one Gauss point with row weights D.
UW_HD inline void eta_at(const TypeC& T, const double* A, const double* E, const double* D,
                         const double* pg, double zeta, double* eta) {
  const int S = T.S;
  double DA[12 * 5], X[5 * 12];
  for (int j = 0; j < S - 1; ++j)
    for (int q = 0; q < 5; ++q) DA[j * 5 + q] = D[j] * A[j * 5 + q];
  tikhonov(DA, S - 1, 5, zeta, X);
  eta_from(T, X, E, D, pg, eta);
}

UW_HD inline void precompute_cell(const CellIn& in, const TypeC& TQ, const TypeC& TT,
                                  const Params& sp, int64_t i, const CellOut& out) {
  const bool isq = i < in.Nq;
  const TypeC& T = isq ? TQ : TT;
  const TypeOut& to = isq ? out.quad : out.tri;
  const int64_t r = isq ? i : i - in.Nq, nrow = to.n;
  const int n = T.n, S = T.S, M = T.M, G = 2 * n;

  // target polygon, area and centroid (moments relative to vertex 0)
  Poly P0;
  cell_polygon(in, i, nullptr, P0);
  Poly rel = P0;
  for (int k = 0; k < n; ++k) {
    rel.p[k][0] -= P0.p[0][0];
    rel.p[k][1] -= P0.p[0][1];
  }
  double mom[6];
  moments(rel, mom);
  const double area = mom[0];
  const double cx = P0.p[0][0] + mom[1] / mom[0], cy = P0.p[0][1] + mom[2] / mom[0];
  const double h0 = sqrt(area);
  Poly X0;
  X0.nf = n;
  for (int k = 0; k < n; ++k) {
    X0.p[k][0] = (P0.p[k][0] - cx) / h0;
    X0.p[k][1] = (P0.p[k][1] - cy) / h0;
  }

  // cell averages of xi, eta, xi^2, eta^2, xi eta over every present slot
  const int32_t* st_cell = in.st_cell + 13 * i;
  const double* st_shift = in.st_shift + 26 * i;
  const int8_t* st_ghost = in.st_ghost + 13 * i;
  const int8_t* st_res = in.st_res + 13 * i;
  const uint8_t* present = in.st_present + 13 * i;
  double basis[13][5];
  double mean0[5] = {0, 0, 0, 0, 0};
  int absent = 0;
  for (int j = 0; j < S; ++j) {
    for (int q = 0; q < 5; ++q) basis[j][q] = 0.0;
    if (!present[j]) {
      ++absent;
      continue;
    }
    Poly Q;
    if (j > 0 && st_ghost[j] >= 0) {
      // mirror image of the target across the boundary face, re-ordered
      // counter-clockwise
      const int k = st_ghost[j];
      const double* a = X0.p[k];
      const double* b = X0.p[(k + 1) % n];
      double nx = b[1] - a[1], ny = -(b[0] - a[0]);
      const double ln = sqrt(nx * nx + ny * ny);
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
      for (int q = 1; q < n; ++q) {
        Q.p[q][0] = R.p[n - q][0];
        Q.p[q][1] = R.p[n - q][1];
      }
    } else {
      Poly raw;
      cell_polygon(in, st_cell[j], st_shift + 2 * j, raw);
      Q.nf = raw.nf;
      for (int k = 0; k < raw.nf; ++k) {
        Q.p[k][0] = (raw.p[k][0] - cx) / h0;
        Q.p[k][1] = (raw.p[k][1] - cy) / h0;
      }
    }
    double mo[6];
    moments(Q, mo);
    for (int q = 0; q < 5; ++q) basis[j][q] = mo[q + 1] / mo[0];
    if (j == 0)
      for (int q = 0; q < 5; ++q) mean0[q] = basis[0][q];
  }
  // averages of the zero-mean basis functions p^k - <p^k>_{i0}
  for (int j = 0; j < S; ++j)
    if (present[j])
      for (int q = 0; q < 5; ++q) basis[j][q] -= mean0[q];

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
    const double ln = sqrt(ex * ex + ey * ey);
    out.length[4 * i + k] = ln;
    out.normal[8 * i + 2 * k] = ey / ln;
    out.normal[8 * i + 2 * k + 1] = -ex / ln;
    for (int q = 0; q < 2; ++q) {
      const double wa = q == 0 ? kGA : kGB, wb = q == 0 ? kGB : kGA;
      const double xi = (wa * a[0] + wb * b[0] - cx) / h0;
      const double et = (wa * a[1] + wb * b[1] - cy) / h0;
      double* p = pG[2 * k + q];
      p[0] = xi - mean0[0];
      p[1] = et - mean0[1];
      p[2] = xi * xi - mean0[2];
      p[3] = et * et - mean0[3];
      p[4] = xi * et - mean0[4];
    }
  }
  for (int k = n; k < 4; ++k) {
    out.length[4 * i + k] = 0.0;
    out.normal[8 * i + 2 * k] = 0.0;
    out.normal[8 * i + 2 * k + 1] = 0.0;
  }
  out.area[i] = area;

  // candidate operators Y_j: g = Y_j (dW_a, dW_b)
  double Y[12][4];
  for (int j = 0; j < M; ++j) {
    const int sa = T.sub_a[j], sb = st_res[T.sub_b[j]];
    const double Mj[4] = {basis[sa][0], basis[sa][1], basis[sb][0], basis[sb][1]};
    double Xj[4];
    tikhonov(Mj, 2, 2, sp.zeta, Xj);
    for (int e = 0; e < 4; ++e) Y[j][e] = Xj[e];
  }

  // the unweighted operator is shared by all Gauss points
  double XA[5 * 12];
  const int rankA = tikhonov(A, S - 1, 5, sp.zeta, XA);
  double max_raw = 0.0, max_opt = 0.0, resid = 0.0, sumdev = 0.0;
  // largest |gamma_j| over the cell's points (only for d_scope = per cell)
  double cellmax[12];
  for (int j = 0; j < 12; ++j) cellmax[j] = 0.0;
  double B[13 * 12], PB[12 * 13], eta_raw[13], eta[13], graw[12], gam[12];
  if (sp.optimize && sp.d_scope == 1) {
    for (int g = 0; g < G; ++g) {
      eta_from(T, XA, E, nullptr, pG[g], eta_raw);
      weight_matrix(T, st_res, Y, pG[g], B, PB, sp.zeta);
      for (int j = 0; j < M; ++j) {
        double s = 0.0;
        for (int q = 0; q < S; ++q) s += PB[j * S + q] * eta_raw[q];
        cellmax[j] = cellmax[j] > fabs(s) ? cellmax[j] : fabs(s);
      }
    }
  }
  for (int g = 0; g < G; ++g) {
    eta_from(T, XA, E, nullptr, pG[g], eta_raw);
    weight_matrix(T, st_res, Y, pG[g], B, PB, sp.zeta);
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int q = 0; q < S; ++q) s += PB[j * S + q] * eta_raw[q];
      graw[j] = s;
      gam[j] = s;
    }
    for (int q = 0; q < S; ++q) eta[q] = eta_raw[q];
    if (sp.optimize) {
      // Sec. 3.3: d_j = 1 / max(1, |gamma| of the candidates that use slot j)
      double D[12];
      for (int s = 1; s < S; ++s) {
        double big = 1.0;
        const int c0 = T.d_c0[s], c1 = T.d_c1[s];
        if (c0) {
          const double v0 = sp.d_scope == 1 ? cellmax[c0 - 1] : fabs(graw[c0 - 1]);
          big = big > v0 ? big : v0;
        }
        if (c1) {
          const double v1 = sp.d_scope == 1 ? cellmax[c1 - 1] : fabs(graw[c1 - 1]);
          big = big > v1 ? big : v1;
        }
        D[s - 1] = 1.0 / big;
      }
      eta_at(T, A, E, D, pG[g], sp.zeta, eta);
      for (int j = 0; j < M; ++j) {
        double s = 0.0;
        for (int q = 0; q < S; ++q) s += PB[j * S + q] * eta[q];
        gam[j] = s;
      }
    }
    for (int j = 0; j < M; ++j)
      if (fabs(gam[j]) < kGammaZero) gam[j] = 0.0;
    // diagnostics
    double sg = 0.0;
    for (int q = 0; q < S; ++q) {
      double s = 0.0;
      for (int j = 0; j < M; ++j) s += B[q * M + j] * gam[j];
      const double d = fabs(s - eta[q]);
      resid = resid > d ? resid : d;
    }
    for (int j = 0; j < M; ++j) {
      sg += gam[j];
      max_raw = max_raw > fabs(graw[j]) ? max_raw : fabs(graw[j]);
      max_opt = max_opt > fabs(gam[j]) ? max_opt : fabs(gam[j]);
    }
    sumdev = sumdev > fabs(sg - 1.0) ? sumdev : fabs(sg - 1.0);
    // outputs of this Gauss point
    to.off[(2 * g) * nrow + r] = pG[g][0];
    to.off[(2 * g + 1) * nrow + r] = pG[g][1];
    // the split of Sec. 3.4 in the form the reconstruction uses: with
    // h_j = gamma_j / (2 sigma+), the normalised weights are
    // gamma+_j = h_j + theta |h_j| and gamma-_j = (sigma+/sigma-)(gamma+_j - 2 h_j)
    double sgp = 0.0, sgm = 0.0;
    for (int j = 0; j < M; ++j) {
      const double tp = 0.5 * (gam[j] + sp.theta * fabs(gam[j]));
      sgp += tp;
      sgm += tp - gam[j];
    }
    for (int j = 0; j < M; ++j) to.gam[(g * M + j) * nrow + r] = gam[j] / (2.0 * sgp);
    to.sig[(3 * g) * nrow + r] = sgp;
    to.sig[(3 * g + 1) * nrow + r] = sgm;
    to.sig[(3 * g + 2) * nrow + r] = sgp / sgm;
    if (to.eta)
      for (int q = 1; q < S; ++q) to.eta[(g * (S - 1) + q - 1) * nrow + r] = eta[q];
    if (out.dbg_gamma) {
      for (int j = 0; j < 12; ++j) {
        out.dbg_gamma[i * 96 + g * 12 + j] = j < M ? gam[j] : 0.0;
        out.dbg_gamma_raw[i * 96 + g * 12 + j] = j < M ? graw[j] : 0.0;
      }
      for (int q = 0; q < 13; ++q) out.dbg_eta[i * 104 + g * 13 + q] = q < S ? eta[q] : 0.0;
      out.dbg_off[i * 16 + 2 * g] = pG[g][0];
      out.dbg_off[i * 16 + 2 * g + 1] = pG[g][1];
    }
  }
  if (out.dbg_gamma) {
    for (int g = G; g < 8; ++g) {
      for (int j = 0; j < 12; ++j) {
        out.dbg_gamma[i * 96 + g * 12 + j] = 0.0;
        out.dbg_gamma_raw[i * 96 + g * 12 + j] = 0.0;
      }
      for (int q = 0; q < 13; ++q) out.dbg_eta[i * 104 + g * 13 + q] = 0.0;
      out.dbg_off[i * 16 + 2 * g] = 0.0;
      out.dbg_off[i * 16 + 2 * g + 1] = 0.0;
    }
    for (int j = 0; j < 12; ++j)
      for (int c = 0; c < 4; ++c) out.dbg_Y[i * 48 + j * 4 + c] = j < M ? Y[j][c] : 0.0;
  }
  for (int j = 0; j < M; ++j)
    for (int c = 0; c < 4; ++c) to.Y[(j * 4 + c) * nrow + r] = Y[j][c];
  for (int q = 1; q < S; ++q) to.sid[(q - 1) * nrow + r] = st_cell[st_res[q]];
  out.diag[4 * i + 0] = max_raw;
  out.diag[4 * i + 1] = max_opt;
  out.diag[4 * i + 2] = resid;
  out.diag[4 * i + 3] = sumdev;
  out.counts[2 * i + 0] = absent;
  out.counts[2 * i + 1] = rankA < 5 ? 1 : 0;
}

}  // namespace geom
}  // namespace uw
