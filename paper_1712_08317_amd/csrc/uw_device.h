// Device-side table views and kernel launchers of the uweno library (internal).
//
// Work is organised in tiles: runs of up to `tile` (256 or 512) consecutive
// cells of one cell type and one mesh instance (a single mesh is a batch of
// one); a reconstruction or flux block of `tile` threads works on one tile
// at a time.
// Quadrilateral tiles come first, then triangle tiles; within each type the
// tiles are ordered by instance.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace uw {

struct Tile {
  int32_t first;   // first cell (state index) of the tile
  int32_t row0;    // its row in the tables of its cell type
  int32_t count;   // cells in the tile (<= the tile size)
  int32_t inst;    // mesh instance
};

// Per-cell tables of one cell type.  A table of K columns ([K][Nt] below)
// is stored in chunks of kTableChunk rows: column c of row r at
// ((r / kTableChunk) K + c) kTableChunk + r % kTableChunk.  A lane forms
// its row's address once (table_row) and reads column c at the constant
// offset c kTableChunk, which the loads take as an immediate, instead of
// one base address per column.
constexpr int kTableChunk = 64;

template <typename T>
struct TypeDev {
  int64_t Nt = 0;
  const uint16_t* lidx = nullptr;   // [S][Nt] LDS position of each stencil slot (0 = the cell)
  const T* Y = nullptr;             // [M*4][Nt] candidate operators
  const T* off = nullptr;           // [2n*2][Nt] Gauss-point offsets (p^1, p^2)
  const T* gam = nullptr;           // [2n*M][Nt] optimised linear weights / (2 sigma+)
  const T* sig = nullptr;           // [2n*3][Nt] sigma+, sigma-, sigma+/sigma- of the split
  const T* eta = nullptr;           // [2n*(S-1)][Nt] point-value coefficients (linear mode)
};

// A lane's row of the tables: its wave's chunk (the same for every lane of
// the wave) and its place in the chunk.
struct RowRef {
  int64_t chunk;
  uint32_t lane;
};

// Column 0 of a lane's row of a chunked table of K columns: the chunk's
// start is wave-uniform (scalar registers), the lane adds a 32-bit offset.
template <int K, typename P>
__device__ inline P* table_row(P* base, RowRef r) {
  return (base + r.chunk * (int64_t)(K * kTableChunk)) + r.lane;
}

// Boundary codes of face tables (fnb): -1 transmissive, -2 reflective,
// -3 - s prescribed state s, kFrontCode - j front face j.
constexpr int32_t kFrontCode = -(1 << 24);

// Time at which an evaluation sees its boundary data: t[inst] (or t0 when
// t is null) plus c dt[inst] (none when dt is null).  The stages of a
// Runge-Kutta step from t take c = 0, 1 and 1/2.
struct StageTime {
  const double* t = nullptr;
  const double* dt = nullptr;
  double c = 0.0, t0 = 0.0;
};

template <typename T>
struct MeshDev {
  int64_t N = 0;                    // cells of all instances
  int32_t n_inst = 1;
  int32_t tile = 256;               // cells per tile
  int32_t n_tq = 0, n_tt = 0;       // quadrilateral and triangle tiles
  const Tile* tiles = nullptr;      // [n_tq + n_tt]
  const int32_t* tile_off = nullptr;   // [n_tq + n_tt + 1] LDS staging list offsets
  const int32_t* tile_ids = nullptr;   // cells staged by each tile, sorted
  int32_t max_len_q = 0, max_len_t = 0;
  const int32_t* inst_tiles = nullptr; // [2][n_inst + 1] quad / triangle tile ranges per instance
  TypeDev<T> quad, tri;
  const int32_t* fnb = nullptr;     // [4][N] (nbr << 3) | (nbr_face << 1) | left; boundary:
                                    // the codes above
  const double* inflow = nullptr;   // [n_states][4] prescribed states (conserved)
  const double* fronts = nullptr;   // [n_fronts][12] (ex, ey, c0, s, A[4], B[4])
  const int32_t* front_inst = nullptr; // [n_fronts] instance of each front
  const int32_t* ff_front = nullptr;   // [n_front_faces] front of each front face
  const double* ff_proj = nullptr;     // [n_front_faces] e.m of its midpoint m
  int32_t special = 0;              // 1 if any face is a wall, prescribed state or front
  StageTime tm;                     // set per launch
  const T* fnrm = nullptr;          // [4*2][N] canonical unit normal of each face
  const double* fcoef = nullptr;    // [4][N] |l| / (2 |Omega_i|), closed for the stored normals
};

struct PhysDev {
  int equation;   // 0 advection, 1 Euler
  double ax, ay, gamma;
};

struct SchemeDev {
  double eps, theta;
  int mode;       // 0 WENO, 1 linear
  int vars;       // 0 conserved, 1 characteristic variables (Euler)
};

// Launch shape: number of persistent blocks of each kernel (0 = one block
// per tile); recon_t = -1: both cell types in one reconstruction launch of
// recon_q blocks.
struct Schedule {
  int recon_q = 0, recon_t = 0, flux = 0;
};

// Dynamic LDS bytes of a reconstruction block.
template <typename T>
size_t recon_lds(int maxlen, int nvar, int tile);

// Face states at the Gauss points, face-major: Gauss point q of face k of
// cell i, variable v, at FS[((k*N + i)*2 + q)*V + v] (4 N V pairs).
template <typename T>
hipError_t launch_recon(const MeshDev<T>& m, const SchemeDev& s, const PhysDev& p,
                        const Schedule& sch, int nvar, const double* W, T* FS,
                        const StageTime& tm, hipStream_t st);

// Flux, residual gather and RK stage.  mode 0: W_out = L(W_in); mode 1..3:
// the three stages of the TVD Runge-Kutta scheme from W_in, Wn and dt[inst].
// partial (nullable, mode 3): each tile's time-step bound of the states
// written, for launch_cfl of the next step with have_partial.
template <typename T>
hipError_t launch_flux(const MeshDev<T>& m, const PhysDev& p, const Schedule& sch, int nvar,
                       int mode, const T* FS, const double* W_in, const double* Wn, double* W_out,
                       const double* dt, int* flag, const StageTime& tm, hipStream_t st,
                       double* partial = nullptr);

// Per instance k: dt[k] = min(cfl * min_i 1 / sum_p coef_p (|u.n_p| + c),
// t_end - t[k]) (or min(dt_fixed, t_end - t[k]) if dt_fixed > 0); t may be
// null (then t = 0).  partial: [n_tq + n_tt] per-tile bounds, formed here
// from W unless have_partial (a flux launch formed them from W already).
template <typename T>
hipError_t launch_cfl(const MeshDev<T>& m, const PhysDev& p, int nvar, const double* W, double cfl,
                      double dt_fixed, double t_end, const double* t, double* partial,
                      double* dt, hipStream_t st, bool have_partial = false);

// t[k] += dt[k] for every instance.
hipError_t launch_advance(int n_inst, double* t, const double* dt, hipStream_t st);

}  // namespace uw
