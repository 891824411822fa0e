// Device-side table views and kernel launchers of the uweno library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace uw {

// Tables of one cell type, structure of arrays [k][Nt].
constexpr int kReconBlock = 256;   // cells per reconstruction tile (one block)

template <typename T>
struct TypeDev {
  int64_t Nt = 0, first = 0;
  const int32_t* tile_off = nullptr;   // [n_tiles + 1]
  const int32_t* tile_ids = nullptr;   // cells staged in LDS by each tile
  const uint16_t* lidx = nullptr;      // [S][Nt] LDS position of each slot (0 = self)
  int32_t max_tile_len = 0;
  const T* Y = nullptr;           // [M*4][Nt]
  const T* off = nullptr;         // [2n*2][Nt]
  const T* gam = nullptr;         // [2n*M][Nt]
  const T* eta = nullptr;         // [2n*(S-1)][Nt]
};

template <typename T>
struct MeshDev {
  int64_t N = 0, Nq = 0;
  TypeDev<T> quad, tri;
  const int32_t* fnb = nullptr;   // [4][N]
  const T* fgeo = nullptr;        // [4*3][N]
};

struct PhysDev {
  int equation;   // 0 advection, 1 Euler
  double ax, ay, gamma;
};

struct SchemeDev {
  double eps, theta;
  int mode;       // 0 WENO, 1 linear
};

// Face states at the Gauss points: FS[(i*8 + g)*V + v].  One block of
// kReconBlock threads per tile.
template <typename T>
hipError_t launch_recon(const MeshDev<T>& m, const SchemeDev& s, int nvar, const double* W, T* FS,
                        hipStream_t st);

// Flux, residual gather and RK stage.  mode 0: L = L(W_in); mode 1..3: the
// three stages of the TVD Runge-Kutta scheme, W_out from W_in, Wn and *dt.
template <typename T>
hipError_t launch_flux(const MeshDev<T>& m, const PhysDev& p, int nvar, int mode, const T* FS,
                       const double* W_in, const double* Wn, double* W_out, const double* dt,
                       double* t, int* flag, int block, hipStream_t st);

// dt = min(cfl * min_i 1 / sum_k coef_k (|u.n_k| + c), t_end - *t) (or
// min(dt_fixed, t_end - *t) if dt_fixed > 0), written to *dt.
template <typename T>
hipError_t launch_cfl(const MeshDev<T>& m, const PhysDev& p, int nvar, const double* W, double cfl,
                      double dt_fixed, double t_end, const double* t, double* partial,
                      double* dt, hipStream_t st);

constexpr int kCflBlock = 256;
inline int64_t cfl_partials(int64_t N) { return (N + kCflBlock - 1) / kCflBlock; }

}  // namespace uw
