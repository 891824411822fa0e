// Host-side data structures of the uweno library (internal).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

namespace uw {

// Stencil type constants (paper Sec. 3.1 quadrilateral, Sec. 3.2 triangle).
// Slots 0..S-1: i0, the n face neighbours, the outer slots.  Outer slot
// n+1+o is reached from face neighbour across face OUTER_FACE[o], at the
// first (0) or second (1) vertex of that face; when absent it takes the cell
// of slot OUTER_REPL[o].  Sub-stencil j = {i0, SUB_A[j], SUB_B[j]}.
struct TypeConst {
  int n, S, M;
  int outer_face[8], outer_end[8], outer_repl[8];
  int sub_a[12], sub_b[12];
  // optimisation: the weight of slot s uses |gamma| of candidates d_c0[s], d_c1[s] (1-based, 0 = none)
  int d_c0[13], d_c1[13];
};

extern const TypeConst kQuad;
extern const TypeConst kTri;
inline const TypeConst& type_const(int nf) { return nf == 4 ? kQuad : kTri; }

constexpr int kMaxS = 13, kMaxM = 12, kMaxG = 8;
constexpr int kTile = 256;   // default cells per tile (= threads per stage block)
inline bool tile_size_ok(int t) { return t == 256 || t == 512; }

// face kind of the first moving front (kinds 3 .. kFrontKind - 1 are
// prescribed states)
constexpr int32_t kFrontKind = 1 << 16;

struct Error {
  int code;
  std::string msg;
};

// Connectivity and stencils of one mesh in the library's internal numbering.
struct HostMesh {
  int64_t n_nodes = 0, N = 0, Nq = 0;
  bool periodic = true;
  std::vector<double> xy;            // [n_nodes*2]
  std::vector<int32_t> cell_nodes;   // [N*4], internal numbering of cells
  std::vector<int32_t> nf;           // [N]
  std::vector<int32_t> new_of_old;   // [N]
  std::vector<int32_t> old_of_new;   // [N]
  std::vector<int32_t> nbr;          // [N*4] internal id, -1 = boundary/unused
  std::vector<int8_t> nbr_face;      // [N*4]
  std::vector<double> shift;         // [N*4*2]
  std::vector<uint8_t> left;         // [N*4] 1: this cell is the canonical left state
  // boundary kind of each unmatched face: 1 transmissive, 2 reflective,
  // 3 + s prescribed state s, kFrontKind + f moving front f; 0 for matched
  // and unused faces
  std::vector<int32_t> bkind;        // [N*4]
  std::vector<double> inflow;        // [n_inflow*4] prescribed conserved states
  std::vector<double> fronts;        // [n_fronts*12] (ex, ey, c0, s, A[4], B[4])
  // faces on moving fronts, by internal cell and face: 4*i + k, the front,
  // and e.m of the face midpoint m (FP64, no fused multiply-add)
  std::vector<int32_t> ff_face, ff_front;
  std::vector<double> ff_proj;
  // stencils
  std::vector<int32_t> st_cell;      // [N*13] slot cell (ghost: self; absent: -1)
  std::vector<double> st_shift;      // [N*13*2]
  std::vector<int8_t> st_ghost;      // [N*13] ghost face index or -1
  std::vector<int8_t> st_res;        // [N*13] resolved slot after substitution
  std::vector<uint8_t> st_present;   // [N*13]
  int64_t n_interior_faces = 0;
};

// Builds connectivity, renumbering and stencils.  Returns false and fills
// err on an invalid mesh.
bool build_mesh(int64_t n_nodes, const double* xy, int64_t n_cells, const int32_t* cells,
                const int32_t* node_id, int bc, const int32_t* face_bc, int32_t n_inflow,
                const double* inflow_W, int32_t n_fronts, const double* fronts, HostMesh& m,
                Error& err);

struct SchemeParams {
  double zeta = 1e-14, theta = 3.0, eps = 1e-3;
  int optimize = 1, d_scope = 0, mode = 0;
};

// FP64 device-layout tables of one cell type, structure of arrays [k][Nt]
// (row r = internal cell index - first).
struct TypeTables {
  int64_t Nt = 0, first = 0;
  std::vector<int32_t> sid;     // [S-1][Nt] cell read by slot s = 1..S-1 (after substitution)
  std::vector<double> Y;        // [M*4][Nt] candidate operators (Y00, Y01, Y10, Y11)
  std::vector<double> off;      // [2n*2][Nt] (p^1, p^2) at each Gauss point
  std::vector<double> gam;      // [2n*M][Nt] optimised linear weights / (2 sigma+)
  std::vector<double> sig;      // [2n*3][Nt] sigma+, sigma-, sigma+/sigma- of the split
  std::vector<double> eta;      // [2n*(S-1)][Nt] point-value coefficients of P^2 (linear mode)
};

struct HostTables {
  TypeTables quad, tri;
  std::vector<int32_t> fnb;     // [4][N] (nbr << 3) | (nbr_face << 1) | left; boundary: -kind
  std::vector<double> fgeo;     // [4*3][N] canonical normal nx, ny and |l|/(2|Omega_i|)
  std::vector<double> area;     // [N]
  // full per-cell copies for inspection (kept for small meshes only)
  bool debug = false;
  std::vector<double> dbg_gamma, dbg_gamma_raw, dbg_eta, dbg_Y, dbg_off, dbg_face;
  double max_abs_gamma_raw = 0, max_abs_gamma_opt = 0, resid_opt = 0, sum_dev = 0;
  int64_t n_absent = 0, n_rank_def = 0;
};

// LDS staging for tiles of `tile` consecutive rows [row0, row0 + n) of one
// cell type (cells first .. first + n - 1): for every tile, the sorted
// distinct cells its stencils read (lists), and for every slot of every row
// its position in that list (lidx [S][stride]).  sid: [S-1][stride] the cell
// each slot s >= 1 reads.
void build_tile_lists(const int32_t* sid, int64_t stride, int64_t row0, int64_t n, int64_t first,
                      int S, int tile, int threads, uint16_t* lidx,
                      std::vector<std::vector<int32_t>>& lists);

// Host precompute (threads).
void precompute_tables(const HostMesh& m, const SchemeParams& sp, HostTables& t, int threads);
// The same on HIP device `device` (one thread per cell); false and a message
// on a HIP error.
bool precompute_tables_device(const HostMesh& m, const SchemeParams& sp, HostTables& t, int device,
                              int threads, std::string& err, int& hip_code);
// shared steps of both drivers
void alloc_tables(const HostMesh& m, const SchemeParams& sp, HostTables& t);
void reduce_diag(const std::vector<double>& diag, const std::vector<int32_t>& counts,
                 HostTables& t);
void finish_tables(const HostMesh& m, HostTables& t, const std::vector<double>& normal,
                   const std::vector<double>& length, int threads);

// Tikhonov-regularised least squares operator X = (zeta I + M^T M)^{-1} M^T
// for an m x n matrix (m >= n, row-major), through a one-sided Jacobi SVD;
// singular values below 1e-12 of the largest are dropped.  X is n x m.
// Returns the numerical rank.
int tikhonov(const double* Mat, int m, int n, double zeta, double* X);

int default_threads();

// Runs f(begin, end) over [0, n) in chunks on a pool of threads.
template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  if (n <= 0) return;
  const int64_t chunk = 1024;
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (n + chunk - 1) / chunk));
  if (threads == 1) {
    f((int64_t)0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (;;) {
        int64_t s = next.fetch_add(chunk);
        if (s >= n) break;
        f(s, std::min(n, s + chunk));
      }
    });
  for (auto& th : pool) th.join();
}

}  // namespace uw
