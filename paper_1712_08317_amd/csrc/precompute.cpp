// FP64 precompute of the per-cell coefficients: host driver, LDS tile
// lists and face tables.  The per-cell arithmetic lives in cellgeom.h and is
// shared with the device driver (precompute_dev.hip).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cellgeom.h"
#include "uw_host.h"

namespace uw {

int tikhonov(const double* Mat, int m, int n, double zeta, double* X) {
  return geom::tikhonov(Mat, m, n, zeta, X);
}

geom::TypeC type_c(const TypeConst& T) {
  geom::TypeC c;
  c.n = T.n;
  c.S = T.S;
  c.M = T.M;
  for (int j = 0; j < 12; ++j) {
    c.sub_a[j] = T.sub_a[j];
    c.sub_b[j] = T.sub_b[j];
  }
  for (int j = 0; j < 13; ++j) {
    c.d_c0[j] = T.d_c0[j];
    c.d_c1[j] = T.d_c1[j];
  }
  return c;
}

void alloc_tables(const HostMesh& m, const SchemeParams& sp, HostTables& t) {
  const int64_t N = m.N, Nq = m.Nq;
  t.quad.Nt = Nq;
  t.quad.first = 0;
  t.tri.Nt = N - Nq;
  t.tri.first = Nq;
  const bool linear = sp.mode == 1;
  for (TypeTables* tt : {&t.quad, &t.tri}) {
    const TypeConst& T = (tt == &t.quad) ? kQuad : kTri;
    const int64_t n = tt->Nt;
    tt->sid.assign((T.S - 1) * n, 0);
    tt->Y.assign(T.M * 4 * n, 0.0);
    tt->off.assign(2 * T.n * 2 * n, 0.0);
    tt->gam.assign(2 * T.n * T.M * n, 0.0);
    tt->sig.assign(2 * T.n * 3 * n, 0.0);
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
}

void reduce_diag(const std::vector<double>& diag, const std::vector<int32_t>& counts,
                 HostTables& t) {
  const int64_t N = (int64_t)diag.size() / 4;
  t.max_abs_gamma_raw = t.max_abs_gamma_opt = t.resid_opt = t.sum_dev = 0.0;
  t.n_absent = t.n_rank_def = 0;
  for (int64_t i = 0; i < N; ++i) {
    t.max_abs_gamma_raw = std::max(t.max_abs_gamma_raw, diag[4 * i]);
    t.max_abs_gamma_opt = std::max(t.max_abs_gamma_opt, diag[4 * i + 1]);
    t.resid_opt = std::max(t.resid_opt, diag[4 * i + 2]);
    t.sum_dev = std::max(t.sum_dev, diag[4 * i + 3]);
    t.n_absent += counts[2 * i];
    t.n_rank_def += counts[2 * i + 1];
  }
}

void precompute_tables(const HostMesh& m, const SchemeParams& sp, HostTables& t, int threads) {
  const int64_t N = m.N;
  alloc_tables(m, sp, t);
  std::vector<double> normal(8 * N), length(4 * N), diag(4 * N);
  std::vector<int32_t> counts(2 * N);
  geom::CellIn in{m.nf.data(),       m.cell_nodes.data(), m.xy.data(),
                  m.st_cell.data(),  m.st_shift.data(),   m.st_ghost.data(),
                  m.st_res.data(),   m.st_present.data(), m.Nq};
  geom::CellOut out;
  out.quad = geom::TypeOut{t.quad.Y.data(), t.quad.off.data(), t.quad.gam.data(),
                           t.quad.sig.data(), t.quad.eta.empty() ? nullptr : t.quad.eta.data(),
                           t.quad.sid.data(), t.quad.Nt};
  out.tri = geom::TypeOut{t.tri.Y.data(), t.tri.off.data(), t.tri.gam.data(), t.tri.sig.data(),
                          t.tri.eta.empty() ? nullptr : t.tri.eta.data(), t.tri.sid.data(),
                          t.tri.Nt};
  out.area = t.area.data();
  out.normal = normal.data();
  out.length = length.data();
  out.diag = diag.data();
  out.counts = counts.data();
  out.dbg_gamma = t.debug ? t.dbg_gamma.data() : nullptr;
  out.dbg_gamma_raw = t.debug ? t.dbg_gamma_raw.data() : nullptr;
  out.dbg_eta = t.debug ? t.dbg_eta.data() : nullptr;
  out.dbg_Y = t.debug ? t.dbg_Y.data() : nullptr;
  out.dbg_off = t.debug ? t.dbg_off.data() : nullptr;
  const geom::TypeC tq = type_c(kQuad), tt = type_c(kTri);
  const geom::Params gp{sp.zeta, sp.theta, sp.optimize, sp.d_scope, sp.mode == 1};
  parallel_for(N, threads, [&](int64_t s, int64_t e) {
    for (int64_t i = s; i < e; ++i) geom::precompute_cell(in, tq, tt, gp, i, out);
  });
  reduce_diag(diag, counts, t);
  finish_tables(m, t, normal, length, threads);
}

void build_tile_lists(const int32_t* sid, int64_t stride, int64_t row0, int64_t n, int64_t first,
                      int S, int tile, int threads, uint16_t* lidx,
                      std::vector<std::vector<int32_t>>& lists) {
  const int64_t nt = (n + tile - 1) / tile;
  lists.assign(nt, {});
  parallel_for(nt, threads, [&](int64_t s0, int64_t e0) {
    std::vector<int32_t> ids;
    for (int64_t k = s0; k < e0; ++k) {
      const int64_t r0 = k * tile, r1 = std::min(n, r0 + tile);
      ids.clear();
      for (int64_t r = r0; r < r1; ++r) {
        ids.push_back((int32_t)(first + r));
        for (int s2 = 1; s2 < S; ++s2) ids.push_back(sid[(s2 - 1) * stride + row0 + r]);
      }
      std::sort(ids.begin(), ids.end());
      ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
      for (int64_t r = r0; r < r1; ++r)
        for (int s2 = 0; s2 < S; ++s2) {
          const int32_t id =
              s2 == 0 ? (int32_t)(first + r) : sid[(s2 - 1) * stride + row0 + r];
          lidx[s2 * stride + row0 + r] =
              (uint16_t)(std::lower_bound(ids.begin(), ids.end(), id) - ids.begin());
        }
      lists[k] = ids;
    }
  });
}

void finish_tables(const HostMesh& m, HostTables& t, const std::vector<double>& normal,
                   const std::vector<double>& length, int threads) {
  const int64_t N = m.N;
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
        else
          t.fnb[k * N + i] = -m.bkind[4 * i + k];   // boundary: minus its kind
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
