// HIP kernels of the per-stage operator (gfx950).
//
// Paper: Sec. 3.4 (split of the linear weights, new smoothness indicator,
// nonlinear weights, split reconstruction), Sec. 2 (Gauss-point fluxes of
// eq. (quadrature), rotation of eq. (transform), HLLC, the residual of eq.
// (semidiscrete)), Sec. 4 (three-stage TVD Runge-Kutta).
//
// One thread per cell.  The reconstruction kernel reads the cell averages of
// the big stencil, forms the candidate gradients g_j = Y_j (dW_a, dW_b) and
// smoothness indicators beta_j = |g_j|^2 once per cell, then for every
// Gauss point splits the linear weights, forms the nonlinear weights and
// writes R(x_G) = W_i0 + sigma+ sum(a+ d)/sum(a+) - sigma- sum(a- d)/sum(a-),
// d_j = P_j(x_G) - W_i0.  Differences W_ij - W_i0 are formed in FP64 before
// any conversion to the compute precision.
//
// The flux kernel evaluates each face flux in a canonical orientation (left
// state = the cell with the lower original id, normal = that cell's outer
// normal), so the two cells of a face compute bit-identical fluxes and the
// gather is cell-centric, without atomics.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "uw_device.h"

namespace uw {
namespace {

template <int NF>
struct Layout;
template <>
struct Layout<4> {
  static constexpr int S = 13, M = 12;
  __device__ static constexpr int a(int j) {
    constexpr int t[12] = {1, 2, 3, 4, 1, 1, 3, 3, 4, 2, 2, 4};
    return t[j];
  }
  __device__ static constexpr int b(int j) {
    constexpr int t[12] = {2, 3, 4, 1, 5, 6, 7, 8, 9, 10, 11, 12};
    return t[j];
  }
};
template <>
struct Layout<3> {
  static constexpr int S = 10, M = 9;
  __device__ static constexpr int a(int j) {
    constexpr int t[9] = {1, 2, 3, 1, 2, 3, 3, 1, 2};
    return t[j];
  }
  __device__ static constexpr int b(int j) {
    constexpr int t[9] = {2, 3, 1, 4, 5, 6, 7, 8, 9};
    return t[j];
  }
};

// Reciprocal without the IEEE division sequence: v_rcp_f32 (1 ulp) in FP32;
// in FP64 v_rcp_f64 refined by one Newton step.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
}

// Unnormalised weights of both signs of one candidate in FP64 (Sec. 3.4):
// alpha+- = gamma+- / q+-^2, q = beta (1 + t + t^2) + eps with t = gamma
// beta, written q = beta (t + t^2) + (beta + eps).  v_rcp_f64 occupies its
// SIMD four times as long as an FMA and takes a Newton step, so both signs
// share the reciprocal of the product q+^2 q-^2 (three more
// multiplications; the product stays far inside the FP64 range).
__device__ inline void alphas_fp64(double gp, double gm, double b, double bpe, double& ap,
                                   double& am) {
  double t = gp * b;
  const double qp = fma(b, fma(t, t, t), bpe);
  t = gm * b;
  const double qm = fma(b, fma(t, t, t), bpe);
  const double Qp = qp * qp, Qm = qm * qm;
  const double r = rcp(Qp * Qm);
  ap = gp * (Qm * r);
  am = gm * (Qp * r);
}

// a / b and sqrt(x) in the flux: FP32 takes the hardware reciprocal and
// square root (1 ulp; the correctly rounded sequences made the flux kernel 8%
// slower once its face states came from LDS), FP64 the correctly rounded
// operations.
__device__ inline float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double fdiv(double a, double b) { return a / b; }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fsqrt(double x) { return sqrt(x); }

template <typename T, int V>
__device__ inline void store_state(T* p, const T* x) {
#pragma unroll
  for (int v = 0; v < V; ++v) p[v] = x[v];
}
template <>
__device__ inline void store_state<float, 4>(float* p, const float* x) {
  *reinterpret_cast<float4*>(p) = make_float4(x[0], x[1], x[2], x[3]);
}
template <>
__device__ inline void store_state<double, 4>(double* p, const double* x) {
  reinterpret_cast<double2*>(p)[0] = make_double2(x[0], x[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(x[2], x[3]);
}

template <typename T, int V>
__device__ inline void load_state(const T* p, T* x) {
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = p[v];
}
template <>
__device__ inline void load_state<float, 4>(const float* p, float* x) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  x[0] = a.x;
  x[1] = a.y;
  x[2] = a.z;
  x[3] = a.w;
}
template <>
__device__ inline void load_state<double, 4>(const double* p, double* x) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  x[0] = a.x;
  x[1] = a.y;
  x[2] = b.x;
  x[3] = b.y;
}

// Stages the cell averages read by one tile's stencils into LDS (FP64),
// then synchronises the block.  Returns the staged list length.
template <int V>
__device__ inline int stage_tile(const double* __restrict__ W, int64_t N, const int32_t* tile_off,
                                 const int32_t* __restrict__ tile_ids, int tile, double* lds) {
  const int beg = tile_off[tile], len = tile_off[tile + 1] - beg;
  for (int k = threadIdx.x; k < len; k += blockDim.x) {
    const int64_t id = tile_ids[beg + k];
#pragma unroll
    for (int v = 0; v < V; ++v) lds[v * len + k] = W[v * N + id];
  }
  __syncthreads();
  return len;
}

// Time at which instance `inst` sees its boundary data.
__device__ inline double stage_time(const StageTime& tm, int inst) {
  double t = tm.t ? tm.t[inst] : tm.t0;
  if (tm.dt) t = t + tm.c * tm.dt[inst];   // c dt is exact for c = 0, 1, 1/2
  return t;
}

// Position c0 + s t of a moving front, rounded as two separate operations.
__device__ inline double front_position(double c0, double s, double t) {
#pragma clang fp contract(off)
  return c0 + s * t;
}

// State outside a boundary face with code pk < 0 and outward unit normal
// (nx, ny), from the inner state w: -1 transmissive (w itself), -2 slip
// wall (w with its normal momentum reversed; transmissive for a scalar),
// -3 - s prescribed state s, kFrontCode - j front face j (state A of its
// front where the face lies behind the front's position at the stage time
// of the front's instance, else state B; everything is looked up here, so
// that the common faces keep no extra registers live).  FRONTS = false
// compiles the front case out, for meshes without front faces.
template <typename U, int V, typename T, bool FRONTS = true>
__device__ inline void outside_state(int32_t pk, const U* w, U nx, U ny, const MeshDev<T>& m,
                                     U* g) {
#pragma unroll
  for (int v = 0; v < V; ++v) g[v] = w[v];
  if (pk == -2) {
    if constexpr (V == 4) {
      const U mn = w[1] * nx + w[2] * ny;
      g[1] = w[1] - U(2) * mn * nx;
      g[2] = w[2] - U(2) * mn * ny;
    }
  } else if (FRONTS && pk <= kFrontCode) {
    const int32_t j = kFrontCode - pk;
    const int32_t fi = m.ff_front[j];
    const double* f = m.fronts + 12 * fi;
    const double tnow = stage_time(m.tm, m.front_inst[fi]);
    const double* st = f + (m.ff_proj[j] < front_position(f[2], f[3], tnow) ? 4 : 8);
#pragma unroll
    for (int v = 0; v < V; ++v) g[v] = (U)st[v];
  } else if (pk <= -3) {
    const double* st = m.inflow + 4 * (-3 - pk);
#pragma unroll
    for (int v = 0; v < V; ++v) g[v] = (U)st[v];
  }
}

// Ghost face neighbours of a wall, inflow or front face carry that face's
// outside state (a transmissive ghost reads the cell itself, as staged):
// replace the difference of slot k + 1, the neighbour across face k.
template <typename T, int NF, int V>
__device__ inline void ghost_differences(const MeshDev<T>& m, int64_t i, const double* w0,
                                         T (&dW)[Layout<NF>::S - 1][V]) {
  if (!m.special) return;   // only open and periodic boundaries: nothing to replace
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int32_t pk = m.fnb[k * m.N + i];
    if (pk <= -2) {
      double g[V];
      outside_state<double, V>(pk, w0, (double)m.fnrm[(k * 2 + 0) * m.N + i],
                               (double)m.fnrm[(k * 2 + 1) * m.N + i], m, g);
#pragma unroll
      for (int v = 0; v < V; ++v) dW[k][v] = (T)(g[v] - w0[v]);
    }
  }
}

// Per-cell inputs of the WENO reconstruction that do not depend on the
// state.  Latency hiding (measured on gfx950): the triangle kernel reads the
// stencil positions and candidate operators before the tile's staging
// barrier, so that their latency overlaps the staging loads; the
// quadrilateral kernel, whose candidate state already fills the registers of
// two waves per SIMD, reads them when needed (held across the barrier they
// spill about 270 bytes per lane).
template <int NF>
constexpr bool kPrefetch = NF == 3;

template <typename T, int NF>
struct WenoIn {
  int li[Layout<NF>::S];       // LDS positions of the stencil cells
  T Y[Layout<NF>::M][4];       // candidate operators
};

template <typename T, int NF>
__device__ inline void weno_load(const TypeDev<T>& td, RowRef r, WenoIn<T, NF>& in) {
  using L = Layout<NF>;
  const uint16_t* lr = table_row<L::S>(td.lidx, r);
  const T* yr = table_row<L::M * 4>(td.Y, r);
#pragma unroll
  for (int s = 0; s < L::S; ++s) in.li[s] = lr[s * kTableChunk];
#pragma unroll
  for (int j = 0; j < L::M; ++j)
#pragma unroll
    for (int k = 0; k < 4; ++k) in.Y[j][k] = yr[(j * 4 + k) * kTableChunk];
}

// Normalised split weights of one Gauss point (Sec. 3.4) from the stored
// h_j = gamma_j / (2 sigma+) and sigma+/sigma-: gamma~+_j = (gamma_j +
// theta |gamma_j|)/2 gives gamma+_j = gamma~+_j / sigma+ = h_j + theta |h_j|,
// and gamma~-_j = gamma~+_j - gamma_j gives gamma-_j = (sigma+/sigma-)
// (gamma+_j - 2 h_j).
template <typename T, int M>
__device__ inline void split_weights(const T (&h)[M], T theta, T ratio, T (&gp)[M], T (&gm)[M]) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    gp[j] = fma(theta, fabs(h[j]), h[j]);
    gm[j] = ratio * fma(T(-2), h[j], gp[j]);
  }
}

// WENO point values of one cell at its 2n Gauss points (paper Sec. 3.4).
template <typename T, int NF, int V>
__device__ inline void weno_cell(const TypeDev<T>& td, RowRef r, const WenoIn<T, NF>& in,
                                 const double* lds, int len, const MeshDev<T>& m, int64_t i,
                                 T* fs, T eps, T theta) {
  using L = Layout<NF>;
  constexpr int S = L::S, M = L::M, G = 2 * NF, C = kTableChunk;
  const uint16_t* lr = table_row<S>(td.lidx, r);
  const T* yr = table_row<M * 4>(td.Y, r);
  const T* offr = table_row<2 * G>(td.off, r);
  const T* sigr = table_row<3 * G>(td.sig, r);
  const T* gamr = table_row<G * M>(td.gam, r);
  // Each Gauss point's offsets and weights are fetched one point ahead.
  // Measured on gfx950: the quadrilateral kernels then spill a few values
  // (24 bytes per lane in FP32, 12 in FP64) and still run 4% (FP32) and 30%
  // (FP64) faster than with the loads at the point itself, where the FP64
  // kernel, at one wave per SIMD, waited for each weight's load in turn.
  T ga_n[M], ox_n = offr[0], oy_n = offr[C];
  T s0_n = sigr[0], s1_n = sigr[C], s2_n = sigr[2 * C];
#pragma unroll
  for (int j = 0; j < M; ++j) ga_n[j] = gamr[j * C];
  // per-cell inputs: prefetched, or read here
  auto li = [&](int s) { return kPrefetch<NF> ? in.li[s] : (int)lr[s * C]; };
  auto Y = [&](int j, int k) { return kPrefetch<NF> ? in.Y[j][k] : yr[(j * 4 + k) * C]; };
  double w0[V];
  const int l0 = li(0);
#pragma unroll
  for (int v = 0; v < V; ++v) w0[v] = lds[v * len + l0];
  // differences to the stencil cells, formed in FP64
  T dW[S - 1][V];
#pragma unroll
  for (int s = 0; s < S - 1; ++s) {
    const int l = li(s + 1);
#pragma unroll
    for (int v = 0; v < V; ++v) dW[s][v] = (T)(lds[v * len + l] - w0[v]);
  }
  ghost_differences<T, NF, V>(m, i, w0, dW);
  // candidate gradients g_j = Y_j (dW_a, dW_b) and indicators beta_j = |g_j|^2
  T gx[M][V], gy[M][V], be[M][V], bpe[M][V];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int a = L::a(j) - 1, b = L::b(j) - 1;
    const T y00 = Y(j, 0), y01 = Y(j, 1), y10 = Y(j, 2), y11 = Y(j, 3);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      gx[j][v] = y00 * dW[a][v] + y01 * dW[b][v];
      gy[j][v] = y10 * dW[a][v] + y11 * dW[b][v];
      be[j][v] = gx[j][v] * gx[j][v] + gy[j][v] * gy[j][v];
      bpe[j][v] = be[j][v] + eps;
    }
  }
#pragma unroll 1
  for (int g = 0; g < G; ++g) {
    const T ox = ox_n, oy = oy_n, sp = s0_n, sm = s1_n, ratio = s2_n;
    T ga[M];
#pragma unroll
    for (int j = 0; j < M; ++j) ga[j] = ga_n[j];
    if (g + 1 < G) {
      ox_n = offr[(2 * g + 2) * C];
      oy_n = offr[(2 * g + 3) * C];
      s0_n = sigr[(3 * g + 3) * C];
      s1_n = sigr[(3 * g + 4) * C];
      s2_n = sigr[(3 * g + 5) * C];
#pragma unroll
      for (int j = 0; j < M; ++j) ga_n[j] = gamr[((g + 1) * M + j) * C];
    }
    T gp[M], gm[M];
    split_weights<T, M>(ga, theta, ratio, gp, gm);
    T R[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      // alpha = gamma / (beta (1 + gamma beta + (gamma beta)^2) + eps)^2
      T Np = 0, Dp = 0, Nm = 0, Dm = 0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const T d = fma(ox, gx[j][v], oy * gy[j][v]);
        const T b = be[j][v];
        if constexpr (sizeof(T) == 8) {
          T ap, am;
          alphas_fp64(gp[j], gm[j], b, bpe[j][v], ap, am);
          Dp += ap;
          Np = fma(ap, d, Np);
          Dm += am;
          Nm = fma(am, d, Nm);
        } else {
          // q = beta u + (beta + eps) with u = t + t^2, t = gamma beta
          T t = gp[j] * b;
          T q = fma(b, fma(t, t, t), bpe[j][v]);
          T al = gp[j] * rcp(q * q);
          Dp += al;
          Np = fma(al, d, Np);
          t = gm[j] * b;
          q = fma(b, fma(t, t, t), bpe[j][v]);
          al = gm[j] * rcp(q * q);
          Dm += al;
          Nm = fma(al, d, Nm);
        }
      }
      R[v] = (T)w0[v] + (sp * (Np * rcp(Dp)) - sm * (Nm * rcp(Dm)));
    }
    store_state<T, V>(fs + g * V, R);
  }
}

// Eigenvectors of Roe's mean matrix n_x dF/dW + n_y dG/dW (Euler, Sec. 4) for
// the mean of WA and WB: right eigenvectors as columns of Rm, left ones as
// rows of Lm, fields ordered u.n - c, u.n (entropy), u.n (shear), u.n + c.
template <typename T>
__device__ inline void roe_eigen(const T* WA, const T* WB, T nx, T ny, T gam, T (&Rm)[4][4],
                                 T (&Lm)[4][4]) {
  const T sA = sqrt(WA[0]), sB = sqrt(WB[0]);
  const T iA = T(1) / WA[0], iB = T(1) / WB[0];
  const T uA = WA[1] * iA, vA = WA[2] * iA, uB = WB[1] * iB, vB = WB[2] * iB;
  const T pA = (gam - T(1)) * (WA[3] - T(0.5) * WA[0] * (uA * uA + vA * vA));
  const T pB = (gam - T(1)) * (WB[3] - T(0.5) * WB[0] * (uB * uB + vB * vB));
  const T HA = (WA[3] + pA) * iA, HB = (WB[3] + pB) * iB;
  const T iw = T(1) / (sA + sB);
  const T u = (sA * uA + sB * uB) * iw, v = (sA * vA + sB * vB) * iw;
  const T H = (sA * HA + sB * HB) * iw;
  const T q2 = T(0.5) * (u * u + v * v);
  const T c = sqrt((gam - T(1)) * (H - q2)), ic = T(1) / c;
  const T un = u * nx + v * ny, ut = -u * ny + v * nx;
  const T b1 = (gam - T(1)) * ic * ic, b2 = q2 * b1;
  Rm[0][0] = 1;          Rm[0][1] = 1; Rm[0][2] = 0;   Rm[0][3] = 1;
  Rm[1][0] = u - c * nx; Rm[1][1] = u; Rm[1][2] = -ny; Rm[1][3] = u + c * nx;
  Rm[2][0] = v - c * ny; Rm[2][1] = v; Rm[2][2] = nx;  Rm[2][3] = v + c * ny;
  Rm[3][0] = H - c * un; Rm[3][1] = q2; Rm[3][2] = ut; Rm[3][3] = H + c * un;
  Lm[0][0] = T(0.5) * (b2 + un * ic);
  Lm[0][1] = T(0.5) * (-b1 * u - nx * ic);
  Lm[0][2] = T(0.5) * (-b1 * v - ny * ic);
  Lm[0][3] = T(0.5) * b1;
  Lm[1][0] = T(1) - b2; Lm[1][1] = b1 * u; Lm[1][2] = b1 * v; Lm[1][3] = -b1;
  Lm[2][0] = -ut;       Lm[2][1] = -ny;    Lm[2][2] = nx;     Lm[2][3] = 0;
  Lm[3][0] = T(0.5) * (b2 - un * ic);
  Lm[3][1] = T(0.5) * (-b1 * u + nx * ic);
  Lm[3][2] = T(0.5) * (-b1 * v + ny * ic);
  Lm[3][3] = T(0.5) * b1;
}

// WENO point values of one cell reconstructed in characteristic variables
// (Sec. 4, Euler): per face, the projection of Roe's mean matrix between the
// cell and the face neighbour, with the cell's outward normal; the stencil
// differences are projected one field at a time, the candidate gradients,
// indicators and nonlinear weights are formed per field, and the two Gauss
// points of the face are projected back.
template <typename T, int NF>
__device__ inline void weno_cell_char(const TypeDev<T>& td, RowRef r, const WenoIn<T, NF>& in,
                                      const double* lds, int len, const MeshDev<T>& m,
                                      int64_t i, T* fs, T eps, T theta, T gam) {
  using L = Layout<NF>;
  constexpr int S = L::S, M = L::M, V = 4, G = 2 * NF, C = kTableChunk;
  const uint16_t* lr = table_row<S>(td.lidx, r);
  const T* yr = table_row<M * 4>(td.Y, r);
  const T* offr = table_row<2 * G>(td.off, r);
  const T* sigr = table_row<3 * G>(td.sig, r);
  const T* gamr = table_row<G * M>(td.gam, r);
  auto li = [&](int s) { return kPrefetch<NF> ? in.li[s] : (int)lr[s * C]; };
  auto Y = [&](int j, int k) { return kPrefetch<NF> ? in.Y[j][k] : yr[(j * 4 + k) * C]; };
  double w0[V];
  const int l0 = li(0);
#pragma unroll
  for (int v = 0; v < V; ++v) w0[v] = lds[v * len + l0];
  T W0[V];
#pragma unroll
  for (int v = 0; v < V; ++v) W0[v] = (T)w0[v];
  T dW[S - 1][V];
#pragma unroll
  for (int s = 0; s < S - 1; ++s) {
    const int l = li(s + 1);
#pragma unroll
    for (int v = 0; v < V; ++v) dW[s][v] = (T)(lds[v * len + l] - w0[v]);
  }
  ghost_differences<T, NF, V>(m, i, w0, dW);
#pragma unroll 1
  for (int k = 0; k < NF; ++k) {
    // Roe mean of the cell and the neighbour across face k (slot k + 1)
    T Rm[4][4], Lm[4][4], Wk[V];
    // the cell's outward normal: the stored canonical normal, reversed where
    // the neighbour is the left cell of the face
    const int32_t pk = m.fnb[k * m.N + i];
    const T sg = (pk < 0 || (pk & 1)) ? T(1) : T(-1);
    const T nxk = sg * m.fnrm[(k * 2 + 0) * m.N + i], nyk = sg * m.fnrm[(k * 2 + 1) * m.N + i];
    if (pk <= -2) {
      // a wall or inflow face: its outside state is the ghost neighbour
      double g[V];
      outside_state<double, V>(pk, w0, (double)nxk, (double)nyk, m, g);
#pragma unroll
      for (int v = 0; v < V; ++v) Wk[v] = (T)g[v];
    } else {
      // face neighbour: slot k + 1 (read again per face: indexing the
      // prefetched slot list with the loop counter would place it in
      // private memory)
      const int l = lr[(k + 1) * C];
#pragma unroll
      for (int v = 0; v < V; ++v) Wk[v] = (T)lds[v * len + l];
    }
    roe_eigen<T>(W0, Wk, nxk, nyk, gam, Rm, Lm);
    // split linear weights of the face's two Gauss points
    T gp[2][M], gm[2][M], sp[2], sm[2], ox[2], oy[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int g = 2 * k + q;
      ox[q] = offr[(2 * g) * C];
      oy[q] = offr[(2 * g + 1) * C];
      sp[q] = sigr[(3 * g) * C];
      sm[q] = sigr[(3 * g + 1) * C];
      T h[M];
#pragma unroll
      for (int j = 0; j < M; ++j) h[j] = gamr[(g * M + j) * C];
      split_weights<T, M>(h, theta, sigr[(3 * g + 2) * C], gp[q], gm[q]);
    }
    T inc[2][V];   // reconstructed increments per field at the two points
#pragma unroll
    for (int c = 0; c < V; ++c) {
      // field c of the stencil differences, then its candidate gradients
      T dc[S - 1];
#pragma unroll
      for (int s = 0; s < S - 1; ++s)
        dc[s] = Lm[c][0] * dW[s][0] + Lm[c][1] * dW[s][1] + Lm[c][2] * dW[s][2] +
                Lm[c][3] * dW[s][3];
      T gx[M], gy[M], be[M], bpe[M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int a = L::a(j) - 1, b = L::b(j) - 1;
        gx[j] = Y(j, 0) * dc[a] + Y(j, 1) * dc[b];
        gy[j] = Y(j, 2) * dc[a] + Y(j, 3) * dc[b];
        be[j] = gx[j] * gx[j] + gy[j] * gy[j];
        bpe[j] = be[j] + eps;
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        T Np = 0, Dp = 0, Nm = 0, Dm = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const T d = fma(ox[q], gx[j], oy[q] * gy[j]);
          const T b = be[j];
          if constexpr (sizeof(T) == 8) {
            T ap, am;
            alphas_fp64(gp[q][j], gm[q][j], b, bpe[j], ap, am);
            Dp += ap;
            Np = fma(ap, d, Np);
            Dm += am;
            Nm = fma(am, d, Nm);
          } else {
            T t = gp[q][j] * b;
            T qq = fma(b, fma(t, t, t), bpe[j]);
            T al = gp[q][j] * rcp(qq * qq);
            Dp += al;
            Np = fma(al, d, Np);
            t = gm[q][j] * b;
            qq = fma(b, fma(t, t, t), bpe[j]);
            al = gm[q][j] * rcp(qq * qq);
            Dm += al;
            Nm = fma(al, d, Nm);
          }
        }
        inc[q][c] = sp[q] * (Np * rcp(Dp)) - sm[q] * (Nm * rcp(Dm));
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      T R[V];
#pragma unroll
      for (int v = 0; v < V; ++v)
        R[v] = W0[v] + (Rm[v][0] * inc[q][0] + Rm[v][1] * inc[q][1] + Rm[v][2] * inc[q][2] +
                        Rm[v][3] * inc[q][3]);
      store_state<T, V>(fs + (2 * k + q) * V, R);
    }
  }
}

// Point values of the quadratic P^2 (eq. (polynomial-eta)): the linear scheme.
template <typename T, int NF, int V>
__device__ inline void linear_cell(const TypeDev<T>& td, RowRef r, const double* lds, int len,
                                   const MeshDev<T>& m, int64_t i, T* fs) {
  using L = Layout<NF>;
  constexpr int S = L::S, G = 2 * NF, C = kTableChunk;
  const uint16_t* lr = table_row<S>(td.lidx, r);
  const T* etar = table_row<G * (S - 1)>(td.eta, r);
  double w0[V];
  const int l0 = lr[0];
#pragma unroll
  for (int v = 0; v < V; ++v) w0[v] = lds[v * len + l0];
  T dW[S - 1][V];
#pragma unroll
  for (int s = 0; s < S - 1; ++s) {
    const int l = lr[(s + 1) * C];
#pragma unroll
    for (int v = 0; v < V; ++v) dW[s][v] = (T)(lds[v * len + l] - w0[v]);
  }
  ghost_differences<T, NF, V>(m, i, w0, dW);
#pragma unroll 1
  for (int g = 0; g < G; ++g) {
    T acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0;
#pragma unroll
    for (int s = 0; s < S - 1; ++s) {
      const T e = etar[(g * (S - 1) + s) * C];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] += e * dW[s][v];
    }
    T R[V];
#pragma unroll
    for (int v = 0; v < V; ++v) R[v] = (T)w0[v] + acc[v];
    store_state<T, V>(fs + g * V, R);
  }
}

// Persistent reconstruction over the tiles of one cell type.  Dynamic LDS:
// the staged cell averages (FP64, padded to 16 bytes), then the tile's face
// states, written out in one coalesced block per tile.
// KIND: 0 WENO on the conserved variables, 1 the linear scheme, 2 WENO on
// the characteristic variables (Euler).
// Occupancy measured on gfx950 (FP32): the WENO kernels run fastest with 2
// waves per SIMD forced (256 VGPRs each; the quadrilateral ones then spill a
// few values: the characteristic kernel runs 39% faster than at 1 wave, the
// conserved one, which reads its weights one point ahead, 4% faster than
// without that prefetch, when it fitted 2 waves unspilled).  The FP32 linear
// kernels and every FP64 kernel keep the whole register file.  Blocks of
// TILE threads: 2 waves per SIMD are 512 / TILE blocks per compute unit.
template <typename T, int NF, int KIND, int TILE>
constexpr int kReconBlocksPerCu = (sizeof(T) == 4 && (NF == 3 || KIND != 1) ? 2 : 1) * 256 / TILE;

// Face states in FS, face-major: the two Gauss-point states of face k of
// cell i at fs_index(N, k, i), V values each (FS holds 4 N such pairs).
// Consecutive cells' records of one face are adjacent, so that a wavefront
// reading the neighbours across a tile edge (often consecutive cells of the
// other tile, seen through the same face) shares cache lines.
template <int V>
__device__ inline int64_t fs_index(int64_t N, int k, int64_t i) {
  return ((int64_t)k * N + i) * (2 * V);
}
// Copy unit of the records: 16 bytes, or 8 for the 8-byte FP32 scalar pair.
template <typename T, int V>
using FsUnit = typename std::conditional<(2 * V * sizeof(T) >= 16), int4, int2>::type;

// One tile of cell type NF: stage its stencil values, reconstruct each
// cell's Gauss-point states into LDS, write the tile's records out.
template <typename T, int NF, int V, int KIND>
__device__ inline void recon_tile(const double* __restrict__ W, const MeshDev<T>& m,
                                  T* __restrict__ FS, T eps, T theta, T gam, int tile, int wave,
                                  double* lds) {
  const TypeDev<T>& td = NF == 4 ? m.quad : m.tri;
  const int maxlen = NF == 4 ? m.max_len_q : m.max_len_t;
  T* fs_lds = reinterpret_cast<T*>(lds + ((maxlen * V + 1) & ~1));
  constexpr int REC = 8 * V;              // face-state values per cell
  constexpr int PER = 16 / sizeof(T);     // values per 16-byte unit
  constexpr int STRIDE = REC + PER;       // LDS row per cell, padded against bank conflicts
  const Tile tl = m.tiles[tile];
  const bool act = (int)threadIdx.x < tl.count;
  // rows of a tile start at a multiple of kTableChunk: each wave reads
  // whole chunks of the tables
  const RowRef r{tl.row0 / kTableChunk + wave, threadIdx.x % kTableChunk};
  WenoIn<T, NF> in;
  if (KIND != 1 && kPrefetch<NF> && act) weno_load<T, NF>(td, r, in);
  const int len = stage_tile<V>(W, m.N, m.tile_off, m.tile_ids, tile, lds);
  if (act) {
    T* fs = fs_lds + threadIdx.x * STRIDE;
    if constexpr (KIND == 1) {
      linear_cell<T, NF, V>(td, r, lds, len, m, tl.first + threadIdx.x, fs);
    } else if constexpr (KIND == 2 && V == 4) {
      weno_cell_char<T, NF>(td, r, in, lds, len, m, tl.first + threadIdx.x, fs, eps, theta, gam);
    } else {
      weno_cell<T, NF, V>(td, r, in, lds, len, m, tl.first + threadIdx.x, fs, eps, theta);
    }
  }
  __syncthreads();
  // FS is face-major: face k of the tile's cells is one contiguous block,
  // copied in units of 16 bytes (8 for FP32 scalar records)
  using Unit = FsUnit<T, V>;
  constexpr int PU = sizeof(Unit) / sizeof(T);   // values per unit
  constexpr int FU = 2 * V / PU;                 // units per cell and face
  const int n = tl.count * FU;
  for (int k = 0; k < NF; ++k) {
    Unit* dst = reinterpret_cast<Unit*>(FS + fs_index<V>(m.N, k, tl.first));
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
      const int c = q / FU, u = q - c * FU;
      dst[q] = *reinterpret_cast<const Unit*>(fs_lds + c * STRIDE + (2 * k * V + u * PU));
    }
  }
  __syncthreads();   // the next tile overwrites both LDS regions
}

template <typename T, int NF, int V, int KIND, int TILE>
__global__ __launch_bounds__(TILE, (kReconBlocksPerCu<T, NF, KIND, TILE>)) void k_recon(
    const double* __restrict__ W, MeshDev<T> m, T* __restrict__ FS, T eps, T theta, T gam) {
  extern __shared__ double lds[];
  const int t0 = NF == 4 ? 0 : m.n_tq, nt = NF == 4 ? m.n_tq : m.n_tt;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) / kTableChunk;
  for (int k = blockIdx.x; k < nt; k += gridDim.x)
    recon_tile<T, NF, V, KIND>(W, m, FS, eps, theta, gam, t0 + k, wave, lds);
}

// Both cell types in one launch: block b takes tiles b, b + gridDim.x, ...
// of the quadrilateral tiles followed by the triangle ones (for kinds whose
// two kernels share their launch bounds).
template <typename T, int V, int KIND, int TILE>
__global__ __launch_bounds__(TILE, (kReconBlocksPerCu<T, 4, KIND, TILE>)) void k_recon_both(
    const double* __restrict__ W, MeshDev<T> m, T* __restrict__ FS, T eps, T theta, T gam) {
  static_assert(kReconBlocksPerCu<T, 4, KIND, TILE> == kReconBlocksPerCu<T, 3, KIND, TILE>);
  extern __shared__ double lds[];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) / kTableChunk;
  const int nt = m.n_tq + m.n_tt;
  for (int k = blockIdx.x; k < nt; k += gridDim.x) {
    if (k < m.n_tq)
      recon_tile<T, 4, V, KIND>(W, m, FS, eps, theta, gam, k, wave, lds);
    else
      recon_tile<T, 3, V, KIND>(W, m, FS, eps, theta, gam, k, wave, lds);
  }
}

// HLLC flux through a face with unit normal (nx, ny), left state WL, right
// state WR: rotate into the face frame, Toro's HLLC with Davis wave speeds.
// Returns the flux in the face frame (mass, normal momentum, tangential
// momentum, energy); the caller rotates it back in FP64.
template <typename T>
__device__ inline void hllc(const T* WL, const T* WR, T nx, T ny, T gam, T* f) {
  const T rL = WL[0], rR = WR[0];
  const T irL = fdiv(T(1), rL), irR = fdiv(T(1), rR);
  const T uL = (WL[1] * nx + WL[2] * ny) * irL, vL = (-WL[1] * ny + WL[2] * nx) * irL;
  const T uR = (WR[1] * nx + WR[2] * ny) * irR, vR = (-WR[1] * ny + WR[2] * nx) * irR;
  const T EL = WL[3], ER = WR[3];
  const T pL = (gam - T(1)) * (EL - T(0.5) * rL * (uL * uL + vL * vL));
  const T pR = (gam - T(1)) * (ER - T(0.5) * rR * (uR * uR + vR * vR));
  const T aL = fsqrt(gam * pL * irL), aR = fsqrt(gam * pR * irR);
  const T SL = fmin(uL - aL, uR - aR), SR = fmax(uL + aL, uR + aR);
  const T Ss = fdiv(pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR),
                    rL * (SL - uL) - rR * (SR - uR));
  if (T(0) <= SL) {
    f[0] = rL * uL;
    f[1] = rL * uL * uL + pL;
    f[2] = rL * uL * vL;
    f[3] = (EL + pL) * uL;
  } else if (T(0) <= Ss) {
    // F*_L = F_L + S_L (U*_L - U_L), with U*_L - U_L written in terms of
    // d = S* - u_L so that it vanishes exactly for equal states
    const T d = Ss - uL;
    const T cm = fdiv(rL * d, SL - Ss);   // rho*_L - rho_L
    f[0] = rL * uL + SL * cm;
    f[1] = rL * uL * uL + pL + SL * (cm * Ss + rL * d);
    f[2] = rL * uL * vL + SL * (cm * vL);
    f[3] = (EL + pL) * uL +
           SL * (EL * irL * cm + (rL + cm) * d * (Ss + fdiv(pL, rL * (SL - uL))));
  } else if (T(0) < SR) {
    const T d = Ss - uR;
    const T cm = fdiv(rR * d, SR - Ss);   // rho*_R - rho_R
    f[0] = rR * uR + SR * cm;
    f[1] = rR * uR * uR + pR + SR * (cm * Ss + rR * d);
    f[2] = rR * uR * vR + SR * (cm * vR);
    f[3] = (ER + pR) * uR +
           SR * (ER * irR * cm + (rR + cm) * d * (Ss + fdiv(pR, rR * (SR - uR))));
  } else {
    f[0] = rR * uR;
    f[1] = rR * uR * uR + pR;
    f[2] = rR * uR * vR;
    f[3] = (ER + pR) * uR;
  }
}

// Numerical flux through a face in the lab frame, in FP64: the HLLC flux is
// evaluated in the compute precision in the face frame and rotated back with
// the stored normal in FP64, so that a uniform state, whose face fluxes are
// then exactly p n (and 0), leaves a residual of FP64 size only.
template <typename T, int V>
__device__ inline void face_flux(const T* WL, const T* WR, T nx, T ny, const PhysDev& p,
                                 double* F) {
  if constexpr (V == 4) {
    T f[4];
    hllc<T>(WL, WR, nx, ny, (T)p.gamma, f);
    const double x = nx, y = ny, f1 = f[1], f2 = f[2];
    F[0] = f[0];
    F[1] = f1 * x - f2 * y;
    F[2] = f1 * y + f2 * x;
    F[3] = f[3];
  } else {
    const double an = p.ax * (double)nx + p.ay * (double)ny;
    F[0] = an * (double)(an >= 0.0 ? WL[0] : WR[0]);
  }
}

__device__ inline double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}

// Local time-step bound 1 / sum_p (|l_p| / (2 |Omega|)) (|u.n_p| + c) of
// cell i with state w, written out without contractions so that every
// kernel that forms it (k_cfl from a state, k_flux from the state it has
// just written) gets the same bits.
template <typename T, int V>
__device__ inline double cell_dt_bound(const MeshDev<T>& m, const PhysDev& p, int nf, int64_t i,
                                       const double (&w)[V]) {
#pragma clang fp contract(off)
  const int64_t N = m.N;
  double u, v, c;
  if constexpr (V == 4) {
    const double rho = w[0], mu = w[1], mv = w[2], E = w[3];
    u = mu / rho;
    v = mv / rho;
    const double pr = (p.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    c = sqrt(p.gamma * pr / rho);
  } else {
    u = p.ax;
    v = p.ay;
    c = 0.0;
  }
  double s = 0.0;
  for (int k = 0; k < nf; ++k) {
    const double nx = m.fnrm[(k * 2 + 0) * N + i], ny = m.fnrm[(k * 2 + 1) * N + i];
    const double coef = m.fcoef[k * N + i];
    s += coef * (fabs(u * nx + v * ny) + c);
  }
  return 1.0 / s;
}

// FRONTS: the mesh has moving-front faces.  Measured on gfx950: the flux
// kernel runs 8% slower on meshes without such faces when the front case is
// compiled in, although it never executes, so it has an instantiation
// without it.
//
// In FP32 each tile first copies its cells' face-state records (contiguous in
// FS) to LDS in 16-byte units: a thread's own record and every neighbour
// inside the tile are then read from LDS, and only neighbours in other tiles
// from FS.  Measured on gfx950: reading each face's states from FS instead
// took 18% longer (the lines of a wave's 64 records, 32 bytes used per face,
// were fetched again for later faces).  The FP64 kernel reads FS directly:
// its 256-byte records would fill 68 KB of LDS per block, and at two blocks
// per CU it ran 25% slower.
// partial (nullable): the time-step bound of the next step, each tile's
// minimum of cell_dt_bound over the states this launch writes (the last
// stage of a step), so that the next step needs no time-step pass of its
// own.
template <typename T, int V, int MODE, bool FRONTS, int TILE>
__global__ __launch_bounds__(TILE) void k_flux(MeshDev<T> m, PhysDev p,
                                                     const T* __restrict__ FS, const double* W_in,
                                                     const double* Wn, double* W_out,
                                                     const double* __restrict__ dtp, int* flag,
                                                     double* __restrict__ partial) {
  extern __shared__ double lds[];
  __shared__ double red[TILE / 64];
  T* rec = reinterpret_cast<T*>(lds);
  constexpr int REC = 8 * V;              // face-state values per cell
  constexpr int PER = 16 / sizeof(T);     // values per 16-byte unit
  constexpr int STRIDE = REC + PER;       // LDS row per cell, padded against bank conflicts
  constexpr bool STAGE = sizeof(T) == 4;  // records staged in LDS
  const int64_t N = m.N;
  const int ntiles = m.n_tq + m.n_tt;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const Tile tl = m.tiles[tile];
    const int nf = tile < m.n_tq ? 4 : 3;
    if (STAGE) {
      // the tile's records, face by face, into one padded LDS row per cell
      using Unit = FsUnit<T, V>;
      constexpr int PU = sizeof(Unit) / sizeof(T);
      constexpr int FU = 2 * V / PU;
      const int n = tl.count * FU;
      for (int k = 0; k < nf; ++k) {
        const Unit* src = reinterpret_cast<const Unit*>(FS + fs_index<V>(N, k, tl.first));
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
          const int c = q / FU, u = q - c * FU;
          *reinterpret_cast<Unit*>(rec + c * STRIDE + (2 * k * V + u * PU)) = src[q];
        }
      }
    }
    __syncthreads();
    double bound = INFINITY;
    if ((int)threadIdx.x < tl.count) {
      const int64_t i = tl.first + threadIdx.x;
      double acc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = 0.0;
      bool bad = false;
      for (int k = 0; k < nf; ++k) {
        const int32_t pk = m.fnb[k * N + i];
        const T nx = m.fnrm[(k * 2 + 0) * N + i];
        const T ny = m.fnrm[(k * 2 + 1) * N + i];
        const double coef = m.fcoef[k * N + i];
        T o0[V], o1[V], t0[V], t1[V];
        const T* own = STAGE ? rec + threadIdx.x * STRIDE + 2 * k * V : FS + fs_index<V>(N, k, i);
        load_state<T, V>(own, o0);
        load_state<T, V>(own + V, o1);
        bool left = true;
        if (pk < 0) {
          // boundary face: the outside states (the stored normal is the cell's)
          outside_state<T, V, T, FRONTS>(pk, o0, nx, ny, m, t0);
          outside_state<T, V, T, FRONTS>(pk, o1, nx, ny, m, t1);
        } else {
          const int64_t c = pk >> 3;
          const int kp = (pk >> 1) & 3;
          left = (pk & 1) != 0;
          // the neighbour's Gauss points run the other way along the face
          const int64_t lc = c - tl.first;
          const T* nb = STAGE && (uint64_t)lc < (uint64_t)tl.count
                            ? rec + lc * STRIDE + 2 * kp * V
                            : FS + fs_index<V>(N, kp, c);
          load_state<T, V>(nb + V, t0);
          load_state<T, V>(nb, t1);
        }
        if constexpr (V == 4) {
          // an inadmissible reconstruction (the scheme is not positivity
          // preserving): density or pressure not positive at a Gauss point
          // (p > 0 with rho > 0 is 2 rho E > |m|^2, as gamma > 1)
          const T e0 = T(2) * o0[0] * o0[3] - (o0[1] * o0[1] + o0[2] * o0[2]);
          const T e1 = T(2) * o1[0] * o1[3] - (o1[1] * o1[1] + o1[2] * o1[2]);
          bad |= !(o0[0] > T(0)) || !(o1[0] > T(0)) || !(e0 > T(0)) || !(e1 > T(0));
        }
        double F0[V], F1[V];
        if (left) {
          face_flux<T, V>(o0, t0, nx, ny, p, F0);
          face_flux<T, V>(o1, t1, nx, ny, p, F1);
        } else {
          face_flux<T, V>(t0, o0, nx, ny, p, F0);
          face_flux<T, V>(t1, o1, nx, ny, p, F1);
        }
        const double sc = left ? coef : -coef;
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += sc * (F0[v] + F1[v]);
      }
      double dt = 0.0;
      if (MODE != 0) dt = dtp[tl.inst];
      double outs[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double Lv = -acc[v];
        double out;
        if (MODE == 0) {
          out = Lv;
        } else if (MODE == 1) {
          out = W_in[v * N + i] + dt * Lv;
        } else if (MODE == 2) {
          out = 0.75 * Wn[v * N + i] + 0.25 * (W_in[v * N + i] + dt * Lv);
        } else {
          out = Wn[v * N + i] * (1.0 / 3.0) + 2.0 / 3.0 * (W_in[v * N + i] + dt * Lv);
        }
        bad |= !isfinite(out);
        W_out[v * N + i] = out;
        outs[v] = out;
      }
      if (bad && flag) *flag = 1;
      if (partial) bound = cell_dt_bound<T, V>(m, p, nf, i, outs);
    }
    if (partial) {   // uniform: every thread of the block takes this branch
      bound = wave_min(bound);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bound;
      __syncthreads();
      if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < TILE / 64; ++w) b = fmin(b, red[w]);
        partial[tile] = b;
      }
    }
    __syncthreads();   // the next tile overwrites the records
  }
}

// Local time-step bound of every cell of one tile, reduced to the tile's
// minimum (wavefront then block); one 256-thread block per tile of any size.
constexpr int kCflBlock = 256;
template <typename T, int V>
__global__ __launch_bounds__(kCflBlock) void k_cfl(MeshDev<T> m, PhysDev p,
                                                   const double* __restrict__ W,
                                                   double* __restrict__ partial) {
  __shared__ double red[kCflBlock / 64];
  const int tile = blockIdx.x;
  const Tile tl = m.tiles[tile];
  const int64_t N = m.N;
  const int nf = tile < m.n_tq ? 4 : 3;
  double x = INFINITY;
  for (int j = threadIdx.x; j < tl.count; j += kCflBlock) {
    const int64_t i = tl.first + j;
    double w[V];
#pragma unroll
    for (int v = 0; v < V; ++v) w[v] = W[v * N + i];
    x = fmin(x, cell_dt_bound<T, V>(m, p, nf, i, w));
  }
  x = wave_min(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < kCflBlock / 64; ++w) b = fmin(b, red[w]);
    partial[tile] = b;
  }
}

// One block per instance: the minimum over the instance's tiles.
constexpr int kCflFinal = 1024;
template <typename T>
__global__ __launch_bounds__(kCflFinal) void k_cfl_final(MeshDev<T> m,
                                                         const double* __restrict__ partial,
                                                         double cfl, double dt_fixed, double t_end,
                                                         const double* t, double* dt) {
  __shared__ double red[kCflFinal / 64];
  const int k = blockIdx.x;
  double x = INFINITY;
  if (dt_fixed <= 0.0) {
    const int q0 = m.inst_tiles[k], q1 = m.inst_tiles[k + 1];
    const int s0 = m.n_tq + m.inst_tiles[m.n_inst + 1 + k];
    const int s1 = m.n_tq + m.inst_tiles[m.n_inst + 1 + k + 1];
    for (int j = q0 + threadIdx.x; j < q1; j += kCflFinal) x = fmin(x, partial[j]);
    for (int j = s0 + threadIdx.x; j < s1; j += kCflFinal) x = fmin(x, partial[j]);
  }
  x = wave_min(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCflFinal / 64; ++w) x = fmin(x, red[w]);
    double d = dt_fixed > 0.0 ? dt_fixed : cfl * x;
    const double rest = t_end - (t ? t[k] : 0.0);
    d = fmin(d, rest);
    dt[k] = d > 0.0 ? d : 0.0;
  }
}

__global__ void k_advance(int n, double* t, const double* dt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) t[k] += dt[k];
}

}  // namespace

// LDS a block may allocate on the current device (queried once per device).
size_t lds_limit() {
  static int cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev >= 64) {
    int v = 0;
    return hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess
               ? (size_t)v : 0;
  }
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return 0;
    cache[dev] = v;
  }
  return (size_t)cache[dev];
}

template <typename T>
size_t recon_lds(int maxlen, int nvar, int tile) {
  return (size_t)((maxlen * nvar + 1) & ~1) * sizeof(double) +
         (size_t)tile * (8 * nvar * sizeof(T) + 16);
}

// 512-cell tiles exist for the FP32 WENO kernels on the conserved variables;
// everything else runs 256-cell tiles.
template <typename T>
hipError_t launch_recon(const MeshDev<T>& m0, const SchemeDev& s, const PhysDev& p,
                        const Schedule& sch, int nvar, const double* W, T* FS,
                        const StageTime& tm, hipStream_t st) {
  MeshDev<T> m = m0;
  m.tm = tm;
  const int kind = s.mode == 1 ? 1 : (s.vars == 1 && nvar == 4 ? 2 : 0);
  const T eps = (T)s.eps, th = (T)s.theta, gam = (T)p.gamma;
  if (m.tile != 256 && !(m.tile == 512 && sizeof(T) == 4 && kind == 0))
    return hipErrorInvalidValue;
  auto one = [&](int ntiles, int maxlen, int want, auto nf_tag) -> hipError_t {
    constexpr int NF = decltype(nf_tag)::value;
    if (ntiles <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(want > 0 && want < ntiles ? want : ntiles);
    const size_t shm = recon_lds<T>(maxlen, nvar, m.tile);
    if (shm > lds_limit()) return hipErrorInvalidConfiguration;
    auto go = [&](auto v_tag, auto kind_tag, auto tile_tag) {
      constexpr int V = decltype(v_tag)::value, K = decltype(kind_tag)::value;
      constexpr int TL = decltype(tile_tag)::value;
      k_recon<T, NF, V, K, TL><<<grid, TL, shm, st>>>(W, m, FS, eps, th, gam);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I4 = std::integral_constant<int, 4>;
    using T256 = std::integral_constant<int, 256>;
    if (kind == 1) {
      if (nvar == 4) go(I4{}, I1{}, T256{});
      else go(I1{}, I1{}, T256{});
    } else if (kind == 2) {
      go(I4{}, std::integral_constant<int, 2>{}, T256{});
    } else {
      auto by_tile = [&](auto v_tag) {
        if constexpr (sizeof(T) == 4) {
          if (m.tile == 512) return go(v_tag, I0{}, std::integral_constant<int, 512>{});
        }
        go(v_tag, I0{}, T256{});
      };
      if (nvar == 4) by_tile(I4{});
      else by_tile(I1{});
    }
    return hipGetLastError();
  };
  // recon_t < 0: both types in one launch of recon_q blocks, where the two
  // kernels share their launch bounds (every kind but the FP32 linear one)
  if (sch.recon_t < 0 && m.n_tq > 0 && m.n_tt > 0 && (sizeof(T) == 8 || kind != 1)) {
    const int ntiles = m.n_tq + m.n_tt;
    const unsigned grid = (unsigned)(sch.recon_q > 0 && sch.recon_q < ntiles ? sch.recon_q : ntiles);
    const size_t shm = std::max(recon_lds<T>(m.max_len_q, nvar, m.tile),
                                recon_lds<T>(m.max_len_t, nvar, m.tile));
    if (shm > lds_limit()) return hipErrorInvalidConfiguration;
    auto go = [&](auto v_tag, auto kind_tag, auto tile_tag) {
      constexpr int V = decltype(v_tag)::value, K = decltype(kind_tag)::value;
      constexpr int TL = decltype(tile_tag)::value;
      if constexpr (sizeof(T) == 8 || K != 1)
        k_recon_both<T, V, K, TL><<<grid, TL, shm, st>>>(W, m, FS, eps, th, gam);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I4 = std::integral_constant<int, 4>;
    using T256 = std::integral_constant<int, 256>;
    if (kind == 1) {
      if (nvar == 4) go(I4{}, I1{}, T256{});
      else go(I1{}, I1{}, T256{});
    } else if (kind == 2) {
      go(I4{}, std::integral_constant<int, 2>{}, T256{});
    } else {
      auto by_tile = [&](auto v_tag) {
        if constexpr (sizeof(T) == 4) {
          if (m.tile == 512) return go(v_tag, I0{}, std::integral_constant<int, 512>{});
        }
        go(v_tag, I0{}, T256{});
      };
      if (nvar == 4) by_tile(I4{});
      else by_tile(I1{});
    }
    return hipGetLastError();
  }
  hipError_t e = one(m.n_tq, m.max_len_q, sch.recon_q, std::integral_constant<int, 4>{});
  if (e != hipSuccess) return e;
  return one(m.n_tt, m.max_len_t, sch.recon_t, std::integral_constant<int, 3>{});
}

template <typename T>
hipError_t launch_flux(const MeshDev<T>& m0, const PhysDev& p, const Schedule& sch, int nvar,
                       int mode, const T* FS, const double* W_in, const double* Wn, double* W_out,
                       const double* dt, int* flag, const StageTime& tm, hipStream_t st,
                       double* partial) {
  MeshDev<T> m = m0;
  m.tm = tm;
  const int ntiles = m.n_tq + m.n_tt;
  if (ntiles <= 0) return hipSuccess;
  const unsigned grid = (unsigned)(sch.flux > 0 && sch.flux < ntiles ? sch.flux : ntiles);
  if (m.tile != 256 && !(m.tile == 512 && sizeof(T) == 4)) return hipErrorInvalidValue;
  // one padded record row per cell of a tile (FP32)
  const size_t shm = sizeof(T) == 4 ? (size_t)m.tile * (8 * nvar * sizeof(T) + 16) : 0;
  if (shm > lds_limit()) return hipErrorInvalidConfiguration;
  // meshes without front faces get the instantiation without the front case
  auto go2 = [&](auto v_tag, auto mode_tag, auto tile_tag) {
    constexpr int V = decltype(v_tag)::value, MD = decltype(mode_tag)::value;
    constexpr int TL = decltype(tile_tag)::value;
    if (m.fronts)
      k_flux<T, V, MD, true, TL><<<grid, TL, shm, st>>>(m, p, FS, W_in, Wn, W_out, dt, flag,
                                                        partial);
    else
      k_flux<T, V, MD, false, TL><<<grid, TL, shm, st>>>(m, p, FS, W_in, Wn, W_out, dt, flag,
                                                         partial);
  };
  auto go = [&](auto v_tag, auto mode_tag) {
    if constexpr (sizeof(T) == 4) {
      if (m.tile == 512) return go2(v_tag, mode_tag, std::integral_constant<int, 512>{});
    }
    go2(v_tag, mode_tag, std::integral_constant<int, 256>{});
  };
  auto by_mode = [&](auto v_tag) {
    switch (mode) {
      case 0: go(v_tag, std::integral_constant<int, 0>{}); break;
      case 1: go(v_tag, std::integral_constant<int, 1>{}); break;
      case 2: go(v_tag, std::integral_constant<int, 2>{}); break;
      default: go(v_tag, std::integral_constant<int, 3>{}); break;
    }
  };
  if (nvar == 4)
    by_mode(std::integral_constant<int, 4>{});
  else
    by_mode(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl(const MeshDev<T>& m, const PhysDev& p, int nvar, const double* W, double cfl,
                      double dt_fixed, double t_end, const double* t, double* partial,
                      double* dt, hipStream_t st, bool have_partial) {
  const int ntiles = m.n_tq + m.n_tt;
  if (dt_fixed <= 0.0 && ntiles > 0 && !have_partial) {
    if (nvar == 4)
      k_cfl<T, 4><<<(unsigned)ntiles, kCflBlock, 0, st>>>(m, p, W, partial);
    else
      k_cfl<T, 1><<<(unsigned)ntiles, kCflBlock, 0, st>>>(m, p, W, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  k_cfl_final<T><<<(unsigned)m.n_inst, kCflFinal, 0, st>>>(m, partial, cfl, dt_fixed, t_end, t, dt);
  return hipGetLastError();
}

hipError_t launch_advance(int n_inst, double* t, const double* dt, hipStream_t st) {
  k_advance<<<(unsigned)((n_inst + 255) / 256), 256, 0, st>>>(n_inst, t, dt);
  return hipGetLastError();
}

template size_t recon_lds<double>(int, int, int);
template size_t recon_lds<float>(int, int, int);
template hipError_t launch_recon<double>(const MeshDev<double>&, const SchemeDev&, const PhysDev&,
                                         const Schedule&, int, const double*, double*,
                                         const StageTime&, hipStream_t);
template hipError_t launch_recon<float>(const MeshDev<float>&, const SchemeDev&, const PhysDev&,
                                        const Schedule&, int, const double*, float*,
                                        const StageTime&, hipStream_t);
template hipError_t launch_flux<double>(const MeshDev<double>&, const PhysDev&, const Schedule&,
                                        int, int, const double*, const double*, const double*,
                                        double*, const double*, int*, const StageTime&,
                                        hipStream_t, double*);
template hipError_t launch_flux<float>(const MeshDev<float>&, const PhysDev&, const Schedule&, int,
                                       int, const float*, const double*, const double*, double*,
                                       const double*, int*, const StageTime&, hipStream_t,
                                       double*);
template hipError_t launch_cfl<double>(const MeshDev<double>&, const PhysDev&, int, const double*,
                                       double, double, double, const double*, double*, double*,
                                       hipStream_t, bool);
template hipError_t launch_cfl<float>(const MeshDev<float>&, const PhysDev&, int, const double*,
                                      double, double, double, const double*, double*, double*,
                                      hipStream_t, bool);

}  // namespace uw
