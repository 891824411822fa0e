// Mesh validation, face connectivity, Hilbert renumbering and big-stencil
// selection (host, integer work; bit-exact by construction).
//
// Paper: Sec. 2 (polygon cells bounded by straight faces), Sec. 3.1 (the
// quadrilateral stencil i0..i12, presence flags E_j, substitutions
// i_j -> i0 for j = 5..8 and i_j -> i_{j-4} for j = 9..12, the twelve
// sub-stencils), Sec. 3.2 (the triangular stencil i0..i9, substitutions
// i_j -> i0 for j = 4..6 and i_j -> i_{j-3} for j = 7..9, nine sub-stencils).
//
// The stencil figures of the paper are not reproduced in its text; the
// outer slots are defined here as: slot(c, v) = the cell across the face of
// face neighbour c that contains vertex v of i0 and is not the face c shares
// with i0.  With the slot table below every substitution falls back to a
// cell at the same vertex.  A slot is absent if there is no such cell, if it
// is i0 or a face neighbour, or if it repeats an earlier present slot (cells
// compared with their periodic image).  Transmissive boundary faces have a
// ghost face neighbour (the mirror image of i0, carrying i0's value); slots
// reached through a ghost are absent.
//
// This file must be compiled without floating-point contraction: the
// Hilbert quantisation below is specified operation by operation.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "uw_host.h"

namespace uw {

const TypeConst kQuad = {
    4, 13, 12,
    {0, 0, 2, 2, 3, 1, 1, 3}, {0, 1, 0, 1, 1, 0, 1, 0}, {0, 0, 0, 0, 5, 6, 7, 8},
    {1, 2, 3, 4, 1, 1, 3, 3, 4, 2, 2, 4}, {2, 3, 4, 1, 5, 6, 7, 8, 9, 10, 11, 12},
    {0, 0, 0, 0, 0, 5, 6, 7, 8, 9, 10, 11, 12}, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
};

const TypeConst kTri = {
    3, 10, 9,
    {0, 1, 2, 2, 0, 1, 0, 0}, {0, 0, 0, 1, 1, 1, 0, 0}, {0, 0, 0, 4, 5, 6, 0, 0},
    {1, 2, 3, 1, 2, 3, 3, 1, 2, 0, 0, 0}, {2, 3, 1, 4, 5, 6, 7, 8, 9, 0, 0, 0},
    {0, 0, 0, 0, 4, 5, 6, 7, 8, 9, 0, 0, 0}, {0, 0, 0, 0, 8, 9, 7, 6, 4, 5, 0, 0, 0},
};

int default_threads() {
  unsigned hc = std::thread::hardware_concurrency();
  int t = hc ? (int)hc : 4;
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    int v = std::atoi(e);
    if (v > 0) t = v;
  }
  return std::max(1, std::min(t, 64));
}

// Stable LSD radix sort of indices by 64-bit keys (16-bit digits).
static void radix_sort(const std::vector<uint64_t>& key, std::vector<int64_t>& idx) {
  const int64_t n = (int64_t)key.size();
  idx.resize(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  uint64_t mx = 0;
  for (uint64_t k : key) mx = std::max(mx, k);
  std::vector<int64_t> tmp(n);
  std::vector<int64_t> cnt(65537);
  for (int shift = 0; shift < 64 && (shift == 0 || (mx >> shift) != 0); shift += 16) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = 0; i < n; ++i) cnt[((key[idx[i]] >> shift) & 0xFFFF) + 1]++;
    for (int d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
    for (int64_t i = 0; i < n; ++i) tmp[cnt[(key[idx[i]] >> shift) & 0xFFFF]++] = idx[i];
    idx.swap(tmp);
  }
}

// Order-16 Hilbert index: quadrants visited (0,0),(0,1),(1,1),(1,0); the
// lower-left sub-curve is transposed, the lower-right anti-transposed.
static uint32_t hilbert16(uint32_t x, uint32_t y) {
  uint32_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    x &= s - 1;
    y &= s - 1;
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - x;
        y = s - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

static double shoelace(const double* xy, const int32_t* c, int nf) {
  double a = 0.0;
  for (int k = 0; k < nf; ++k) {
    const double* p = xy + 2 * c[k];
    const double* q = xy + 2 * c[(k + 1) % nf];
    a += p[0] * q[1] - q[0] * p[1];
  }
  return 0.5 * a;
}

bool build_mesh(int64_t n_nodes, const double* xy, int64_t n_cells, const int32_t* cells,
                const int32_t* node_id, int bc, const int32_t* face_bc, int32_t n_inflow,
                const double* inflow_W, int32_t n_fronts, const double* fronts, HostMesh& m,
                Error& err) {
  const int threads = default_threads();
  m.n_nodes = n_nodes;
  m.N = n_cells;
  m.periodic = (bc == 0);
  m.xy.assign(xy, xy + 2 * n_nodes);
  m.inflow.assign(inflow_W ? inflow_W : xy, inflow_W ? inflow_W + 4 * (int64_t)n_inflow : xy);
  m.fronts.assign(fronts ? fronts : xy, fronts ? fronts + 12 * (int64_t)n_fronts : xy);

  // ---- validation
  std::vector<int32_t> nf0(n_cells);
  std::atomic<int64_t> bad{-1};
  std::atomic<int> bad_kind{0};
  parallel_for(n_cells, threads, [&](int64_t s, int64_t e) {
    for (int64_t c = s; c < e; ++c) {
      const int32_t* cn = cells + 4 * c;
      int nf = cn[3] < 0 ? 3 : 4;
      nf0[c] = nf;
      int kind = 0;
      for (int k = 0; k < 3; ++k)
        if (cn[k] < 0) kind = 1;
      if (cn[3] < -1) kind = 1;
      for (int k = 0; k < nf && !kind; ++k)
        if (cn[k] >= n_nodes) kind = 1;
      for (int a = 0; a < nf && !kind; ++a)
        for (int b = a + 1; b < nf; ++b)
          if (cn[a] == cn[b]) kind = 2;
      if (!kind && !(shoelace(xy, cn, nf) > 0.0)) kind = 3;
      if (kind) {
        int64_t expect = -1;
        if (bad.compare_exchange_strong(expect, c)) bad_kind = kind;
      }
    }
  });
  if (bad >= 0) {
    static const char* what[] = {"", "invalid node index", "repeated node in a cell",
                                 "non-positive signed area (cell not counter-clockwise)"};
    err = {2, std::string("cell ") + std::to_string((long long)bad.load()) + ": " + what[bad_kind]};
    return false;
  }
  std::vector<int64_t> canon(n_nodes);
  for (int64_t v = 0; v < n_nodes; ++v) {
    canon[v] = node_id ? node_id[v] : v;
    if (canon[v] < 0) {
      err = {2, "negative canonical node id"};
      return false;
    }
  }
  int64_t mc = 0;
  for (int64_t v = 0; v < n_nodes; ++v) mc = std::max(mc, canon[v] + 1);

  // ---- half-edges, sorted by canonical edge key
  std::vector<int64_t> he_start(n_cells + 1, 0);
  for (int64_t c = 0; c < n_cells; ++c) he_start[c + 1] = he_start[c] + nf0[c];
  const int64_t H = he_start[n_cells];
  std::vector<uint64_t> key(H);
  std::vector<int32_t> he_cell(H);
  std::vector<int8_t> he_k(H);
  for (int64_t c = 0; c < n_cells; ++c) {
    for (int k = 0; k < nf0[c]; ++k) {
      int64_t h = he_start[c] + k;
      int64_t a = canon[cells[4 * c + k]], b = canon[cells[4 * c + (k + 1) % nf0[c]]];
      if (a == b) {
        err = {2, "cell " + std::to_string((long long)c) + ": degenerate edge"};
        return false;
      }
      int64_t lo = std::min(a, b), hi = std::max(a, b);
      key[h] = (uint64_t)lo * (uint64_t)mc + (uint64_t)hi;
      he_cell[h] = (int32_t)c;
      he_k[h] = (int8_t)k;
    }
  }
  std::vector<int64_t> order;
  radix_sort(key, order);
  std::vector<int32_t> nbr0(4 * n_cells, -1);
  std::vector<int8_t> nface0(4 * n_cells, -1);
  std::vector<int32_t> bkind0(4 * n_cells, 0);
  std::vector<double> shift0(8 * n_cells, 0.0);
  int64_t interior = 0;
  for (int64_t p = 0; p < H;) {
    int64_t q = p + 1;
    while (q < H && key[order[q]] == key[order[p]]) ++q;
    if (q - p > 2) {
      err = {2, "edge shared by more than two cells"};
      return false;
    }
    if (q - p == 2) {
      int64_t h1 = order[p], h2 = order[p + 1];
      int32_t c1 = he_cell[h1], c2 = he_cell[h2];
      int k1 = he_k[h1], k2 = he_k[h2];
      int32_t a1 = cells[4 * c1 + k1], b1 = cells[4 * c1 + (k1 + 1) % nf0[c1]];
      int32_t a2 = cells[4 * c2 + k2], b2 = cells[4 * c2 + (k2 + 1) % nf0[c2]];
      if (canon[a1] != canon[b2] || canon[b1] != canon[a2]) {
        err = {2, "edge traversed in the same direction by both owners"};
        return false;
      }
      nbr0[4 * c1 + k1] = c2;
      nface0[4 * c1 + k1] = (int8_t)k2;
      shift0[8 * c1 + 2 * k1] = xy[2 * a1] - xy[2 * b2];
      shift0[8 * c1 + 2 * k1 + 1] = xy[2 * a1 + 1] - xy[2 * b2 + 1];
      nbr0[4 * c2 + k2] = c1;
      nface0[4 * c2 + k2] = (int8_t)k1;
      shift0[8 * c2 + 2 * k2] = xy[2 * a2] - xy[2 * b1];
      shift0[8 * c2 + 2 * k2 + 1] = xy[2 * a2 + 1] - xy[2 * b1 + 1];
      ++interior;
    } else {
      // an unmatched face: its boundary kind
      const int64_t h = order[p];
      const int32_t c = he_cell[h];
      const int k = he_k[h];
      int kind = face_bc ? face_bc[4 * c + k] : 0;
      if (kind == 0) kind = m.periodic ? 0 : 1;
      if (kind == 0) {
        err = {2, "unmatched face on a periodic mesh"};
        return false;
      }
      const bool front = kind >= kFrontKind && kind - kFrontKind < n_fronts;
      if (kind < 0 || (kind > 2 + n_inflow && !front)) {
        err = {1, "face_bc: unknown kind, prescribed state or front index"};
        return false;
      }
      bkind0[4 * c + k] = kind;
    }
    p = q;
  }
  m.n_interior_faces = interior;

  // ---- renumbering: quadrilaterals first, then triangles, by Hilbert index
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  for (int64_t v = 0; v < n_nodes; ++v)
    for (int d = 0; d < 2; ++d) {
      lo[d] = std::min(lo[d], xy[2 * v + d]);
      hi[d] = std::max(hi[d], xy[2 * v + d]);
    }
  std::vector<uint64_t> skey(n_cells);
  parallel_for(n_cells, threads, [&](int64_t s, int64_t e) {
    for (int64_t c = s; c < e; ++c) {
      const int32_t* cn = cells + 4 * c;
      uint32_t q[2];
      for (int d = 0; d < 2; ++d) {
        double sum = xy[2 * cn[0] + d] + xy[2 * cn[1] + d];
        sum = sum + xy[2 * cn[2] + d];
        if (nf0[c] == 4) sum = sum + xy[2 * cn[3] + d];
        double cc = sum / (double)nf0[c];
        double t = std::floor(65536.0 * (cc - lo[d]) / (hi[d] - lo[d]));
        q[d] = (uint32_t)std::min(65535.0, t);
      }
      skey[c] = ((uint64_t)(nf0[c] == 3 ? 1 : 0) << 32) | hilbert16(q[0], q[1]);
    }
  });
  std::vector<int64_t> perm;
  radix_sort(skey, perm);
  m.old_of_new.resize(n_cells);
  m.new_of_old.resize(n_cells);
  m.Nq = 0;
  for (int64_t i = 0; i < n_cells; ++i) {
    m.old_of_new[i] = (int32_t)perm[i];
    m.new_of_old[perm[i]] = (int32_t)i;
    if (nf0[perm[i]] == 4) m.Nq++;
  }

  // ---- connectivity in internal numbering
  m.nf.resize(n_cells);
  m.cell_nodes.resize(4 * n_cells);
  m.nbr.assign(4 * n_cells, -1);
  m.nbr_face.assign(4 * n_cells, -1);
  m.shift.assign(8 * n_cells, 0.0);
  m.left.assign(4 * n_cells, 0);
  m.bkind.assign(4 * n_cells, 0);
  parallel_for(n_cells, threads, [&](int64_t s, int64_t e) {
    for (int64_t i = s; i < e; ++i) {
      int64_t o = m.old_of_new[i];
      m.nf[i] = nf0[o];
      for (int k = 0; k < 4; ++k) {
        m.cell_nodes[4 * i + k] = cells[4 * o + k];
        int32_t nb = nbr0[4 * o + k];
        if (k < nf0[o]) {
          if (nb >= 0) {
            m.nbr[4 * i + k] = m.new_of_old[nb];
            m.nbr_face[4 * i + k] = nface0[4 * o + k];
            m.shift[8 * i + 2 * k] = shift0[8 * o + 2 * k];
            m.shift[8 * i + 2 * k + 1] = shift0[8 * o + 2 * k + 1];
            m.left[4 * i + k] = (o < nb) ? 1 : 0;
          } else {
            m.left[4 * i + k] = 1;
            m.bkind[4 * i + k] = bkind0[4 * o + k];
          }
        }
      }
    }
  });
  // faces on moving fronts: the side of the front is decided on e.m, m the
  // midpoint of the face's two nodes as given
  m.ff_face.clear();
  m.ff_front.clear();
  m.ff_proj.clear();
  for (int64_t i = 0; i < n_cells; ++i)
    for (int k = 0; k < m.nf[i]; ++k) {
      const int32_t kind = m.bkind[4 * i + k];
      if (kind < kFrontKind) continue;
      const int32_t f = kind - kFrontKind;
      const int32_t a = m.cell_nodes[4 * i + k], b = m.cell_nodes[4 * i + (k + 1) % m.nf[i]];
      const double mx = 0.5 * (xy[2 * a] + xy[2 * b]);
      const double my = 0.5 * (xy[2 * a + 1] + xy[2 * b + 1]);
      const double px = m.fronts[12 * f] * mx;
      const double py = m.fronts[12 * f + 1] * my;
      m.ff_face.push_back((int32_t)(4 * i + k));
      m.ff_front.push_back(f);
      m.ff_proj.push_back(px + py);
    }

  // ---- stencils (Sec. 3.1 / 3.2 selection procedures)
  m.st_cell.assign(kMaxS * n_cells, -1);
  m.st_shift.assign(2 * kMaxS * n_cells, 0.0);
  m.st_ghost.assign(kMaxS * n_cells, -1);
  m.st_res.assign(kMaxS * n_cells, 0);
  m.st_present.assign(kMaxS * n_cells, 0);
  parallel_for(n_cells, threads, [&](int64_t s, int64_t e) {
    for (int64_t i = s; i < e; ++i) {
      const TypeConst& T = type_const(m.nf[i]);
      int32_t* cell = &m.st_cell[kMaxS * i];
      double* sh = &m.st_shift[2 * kMaxS * i];
      int8_t* gh = &m.st_ghost[kMaxS * i];
      int8_t* res = &m.st_res[kMaxS * i];
      uint8_t* pr = &m.st_present[kMaxS * i];
      for (int j = 0; j < kMaxS; ++j) res[j] = (int8_t)j;
      cell[0] = (int32_t)i;
      pr[0] = 1;
      for (int k = 0; k < T.n; ++k) {
        int32_t nb = m.nbr[4 * i + k];
        pr[k + 1] = 1;
        if (nb < 0) {
          cell[k + 1] = (int32_t)i;
          gh[k + 1] = (int8_t)k;
        } else {
          cell[k + 1] = nb;
          sh[2 * (k + 1)] = m.shift[8 * i + 2 * k];
          sh[2 * (k + 1) + 1] = m.shift[8 * i + 2 * k + 1];
        }
      }
      for (int o = 0; o < T.S - T.n - 1; ++o) {
        const int j = T.n + 1 + o, k = T.outer_face[o];
        bool ok = gh[k + 1] < 0;
        int32_t cand = -1;
        double cs[2] = {0.0, 0.0};
        if (ok) {
          int32_t c = cell[k + 1];
          int kp = m.nbr_face[4 * i + k], nfc = m.nf[c];
          int other = T.outer_end[o] == 0 ? (kp + 1) % nfc : (kp + nfc - 1) % nfc;
          cand = m.nbr[4 * c + other];
          ok = cand >= 0;
          if (ok) {
            cs[0] = sh[2 * (k + 1)] + m.shift[8 * c + 2 * other];
            cs[1] = sh[2 * (k + 1) + 1] + m.shift[8 * c + 2 * other + 1];
          }
        }
        if (ok && cand == (int32_t)i && cs[0] == 0.0 && cs[1] == 0.0) ok = false;
        for (int f = 1; ok && f <= T.n; ++f)
          if (gh[f] < 0 && cell[f] == cand && sh[2 * f] == cs[0] && sh[2 * f + 1] == cs[1]) ok = false;
        for (int q = T.n + 1; ok && q < j; ++q)
          if (pr[q] && cell[q] == cand && sh[2 * q] == cs[0] && sh[2 * q + 1] == cs[1]) ok = false;
        if (ok) {
          cell[j] = cand;
          sh[2 * j] = cs[0];
          sh[2 * j + 1] = cs[1];
          pr[j] = 1;
        } else {
          res[j] = res[T.outer_repl[o]];
        }
      }
    }
  });
  return true;
}

}  // namespace uw
