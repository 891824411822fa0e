// C-ABI of the uweno library: mesh upload, FP64 precompute, residual,
// SSP-RK3 steps (single meshes and batches), CFL time step, launch
// schedule tuning, launch timing and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "uweno.h"
#include "uw_device.h"
#include "uw_host.h"


namespace {

thread_local std::string g_err;

uw_status fail(uw_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

uw_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? UW_ENOMEM : UW_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define UW_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

#define UW_TRY(call)            \
  do {                          \
    uw_status s_ = (call);      \
    if (s_ != UW_OK) return s_; \
  } while (0)

// Device buffer owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <class T>
  hipError_t upload(const std::vector<T>& v) {
    hipError_t e = ensure(v.size() * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// A cell type's [K][R] table (structure of arrays, R rows) in the device
// layout: rows in chunks of kTableChunk, column c of row r at
// ((r / kTableChunk) K + c) kTableChunk + r % kTableChunk, converted to T.
// A lane then reads all columns of its row at constant offsets from one
// address.  The tail of the last chunk is zero.
template <class T, class U>
std::vector<T> chunked(const std::vector<U>& in, int64_t R) {
  if (R <= 0 || in.empty()) return {};
  const int64_t C = uw::kTableChunk, K = (int64_t)in.size() / R, nch = (R + C - 1) / C;
  std::vector<T> out((size_t)(nch * K * C), T(0));
  uw::parallel_for(nch, uw::default_threads(), [&](int64_t b, int64_t e) {
    for (int64_t ch = b; ch < e; ++ch) {
      const int64_t rows = std::min(C, R - ch * C);
      for (int64_t c = 0; c < K; ++c) {
        const U* src = in.data() + c * R + ch * C;
        T* dst = out.data() + (ch * K + c) * C;
        for (int64_t l = 0; l < rows; ++l) dst[l] = (T)src[l];
      }
    }
  });
  return out;
}

// Face tables of the flux kernel from the FP64 face table fgeo [4*3][N]
// (canonical normal, |l|/(2|Omega_i|)) and the pairing fnb: the normals in
// the compute precision, [4*2][N], and the gather factors in FP64, [4][N].
// In FP32 the rounded normals no longer close (sum_k s_k c_k n_k != 0, s_k
// the orientation sign), which would leave a residual of FP32 size in a
// uniform state; the factors are therefore moved by the least-norm
// correction that restores closure for the stored normals.  In FP64 they
// are used as computed.
template <class T>
void face_tables(const std::vector<double>& fgeo, const std::vector<int32_t>& fnb, int64_t N,
                 std::vector<T>& nrm, std::vector<double>& coef) {
  nrm.assign((size_t)8 * N, T(0));
  coef.assign((size_t)4 * N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    double n[4][2], c[4], sg[4];
    double rx = 0.0, ry = 0.0, axx = 0.0, axy = 0.0, ayy = 0.0;
    for (int k = 0; k < 4; ++k) {
      const T nx = (T)fgeo[(k * 3 + 0) * N + i], ny = (T)fgeo[(k * 3 + 1) * N + i];
      nrm[(k * 2 + 0) * N + i] = nx;
      nrm[(k * 2 + 1) * N + i] = ny;
      n[k][0] = (double)nx;
      n[k][1] = (double)ny;
      c[k] = fgeo[(k * 3 + 2) * N + i];
      const int32_t pk = fnb[k * N + i];
      sg[k] = (pk < 0 || (pk & 1)) ? 1.0 : -1.0;
      rx += sg[k] * c[k] * n[k][0];
      ry += sg[k] * c[k] * n[k][1];
      axx += n[k][0] * n[k][0];
      axy += n[k][0] * n[k][1];
      ayy += n[k][1] * n[k][1];
    }
    if constexpr (!std::is_same<T, double>::value) {
      const double det = axx * ayy - axy * axy;
      if (det > 0.0) {
        const double lx = (ayy * rx - axy * ry) / det, ly = (axx * ry - axy * rx) / det;
        for (int k = 0; k < 4; ++k) c[k] -= sg[k] * (n[k][0] * lx + n[k][1] * ly);
      }
    }
    for (int k = 0; k < 4; ++k) coef[k * N + i] = c[k];
  }
}

// Host copy of the device layout of one or more meshes (a batch), FP64.
struct Staged {
  int64_t N = 0;
  int32_t n_inst = 0, n_tq = 0, n_tt = 0, max_len_q = 0, max_len_t = 0;
  int32_t tile = uw::kTile;     // cells per tile of the lists below
  // per type: the cell each stencil slot s >= 1 reads ([S-1][rows], batch
  // ids), and per instance its first row and first cell of that type
  std::vector<int32_t> q_sid, t_sid;
  // rows of each type: instance k's rows start at row0[k] (a multiple of
  // kTableChunk, so that every wave of a tile reads whole table chunks) and
  // number nrow[k]
  std::vector<int64_t> q_row0, t_row0, q_nrow, t_nrow, q_first, t_first;
  std::vector<uw::Tile> tiles;
  std::vector<int32_t> tile_off, tile_ids, inst_tiles, fnb;
  std::vector<double> inflow;   // [n_states][4] prescribed states of all instances
  std::vector<double> fronts;   // [n_fronts][12] moving fronts of all instances
  std::vector<int32_t> front_inst;   // [n_fronts] their instances
  std::vector<int32_t> ff_front;   // [n_front_faces] front of each front face
  std::vector<double> ff_proj;     // [n_front_faces] e.m of its midpoint
  int32_t special = 0;          // any wall, prescribed-state or front face
  int64_t rows_q = 0, rows_t = 0;
  std::vector<uint16_t> q_lidx, t_lidx;
  std::vector<double> q_Y, q_off, q_gam, q_sig, q_eta, t_Y, t_off, t_gam, t_sig, t_eta, fgeo;
};

template <class V, class Get>
void cat_type(const std::vector<const uw::HostTables*>& ts, bool quad, Get get, int64_t rows_total,
              const std::vector<int64_t>& row_off, V& out) {
  size_t K = 0;
  for (const uw::HostTables* t : ts) {
    const uw::TypeTables& tt = quad ? t->quad : t->tri;
    if (tt.Nt > 0) K = get(tt).size() / tt.Nt;
  }
  out.assign(K * rows_total, 0);
  for (size_t k = 0; k < ts.size(); ++k) {
    const uw::TypeTables& tt = quad ? ts[k]->quad : ts[k]->tri;
    if (tt.Nt <= 0) continue;
    const auto& in = get(tt);
    for (size_t c = 0; c < K; ++c)
      std::copy(in.begin() + c * tt.Nt, in.begin() + (c + 1) * tt.Nt,
                out.begin() + c * rows_total + row_off[k]);
  }
}

// Tiles of `tile` consecutive cells of one type and one instance (all
// quadrilateral tiles, then all triangle tiles, each by instance), their LDS
// staging lists and slot positions.  Needs the sid tables and instance
// ranges of S.
void retile(Staged& S, int tile) {
  const int n = S.n_inst;
  const int threads = uw::default_threads();
  S.tile = tile;
  S.tiles.clear();
  S.tile_ids.clear();
  S.tile_off.assign(1, 0);
  S.inst_tiles.assign(2 * (n + 1), 0);
  S.max_len_q = S.max_len_t = 0;
  for (int type = 0; type < 2; ++type) {
    const bool q = type == 0;
    const int Sn = q ? uw::kQuad.S : uw::kTri.S;
    const int64_t R = q ? S.rows_q : S.rows_t;
    std::vector<uint16_t>& lidx = q ? S.q_lidx : S.t_lidx;
    lidx.assign((size_t)Sn * R, 0);
    const std::vector<int32_t>& sid = q ? S.q_sid : S.t_sid;
    int32_t count = 0;
    std::vector<std::vector<int32_t>> lists;
    for (int k = 0; k < n; ++k) {
      const int64_t r0 = (q ? S.q_row0 : S.t_row0)[k];
      const int64_t nk = (q ? S.q_nrow : S.t_nrow)[k];
      const int64_t first = (q ? S.q_first : S.t_first)[k];
      if (nk > 0)
        uw::build_tile_lists(sid.data(), R, r0, nk, first, Sn, tile, threads, lidx.data(), lists);
      else
        lists.clear();
      for (size_t j = 0; j < lists.size(); ++j) {
        uw::Tile tl;
        tl.first = (int32_t)(first + (int64_t)j * tile);
        tl.row0 = (int32_t)(r0 + (int64_t)j * tile);
        tl.count = (int32_t)std::min<int64_t>(tile, nk - (int64_t)j * tile);
        tl.inst = k;
        S.tiles.push_back(tl);
        S.tile_ids.insert(S.tile_ids.end(), lists[j].begin(), lists[j].end());
        S.tile_off.push_back((int32_t)S.tile_ids.size());
        int32_t& mx = q ? S.max_len_q : S.max_len_t;
        mx = std::max(mx, (int32_t)lists[j].size());
      }
      count += (int32_t)lists.size();
      S.inst_tiles[type * (n + 1) + k + 1] = count;
    }
    (q ? S.n_tq : S.n_tt) = count;
  }
}

// Concatenates per-mesh tables into the batch layout: cells of instance k
// occupy [off_k, off_k + n_k); each type's table rows are concatenated by
// instance; neighbour and staging ids are rebased.
void assemble(const std::vector<const uw::HostMesh*>& ms, const std::vector<const uw::HostTables*>& ts,
              bool linear, int tile, Staged& S) {
  const int n = (int)ms.size();
  S = Staged();
  S.n_inst = n;
  std::vector<int64_t> off(n + 1, 0), qrow(n + 1, 0), trow(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    off[k + 1] = off[k] + ms[k]->N;
    const int64_t C = uw::kTableChunk;
    qrow[k + 1] = (qrow[k] + ts[k]->quad.Nt + C - 1) / C * C;
    trow[k + 1] = (trow[k] + ts[k]->tri.Nt + C - 1) / C * C;
  }
  S.N = off[n];
  S.rows_q = qrow[n];
  S.rows_t = trow[n];
  // stencil slot cells per type (batch ids) and the instances' ranges
  S.q_row0.assign(qrow.begin(), qrow.end());
  S.t_row0.assign(trow.begin(), trow.end());
  S.q_first.resize(n);
  S.t_first.resize(n);
  S.q_nrow.resize(n);
  S.t_nrow.resize(n);
  for (int k = 0; k < n; ++k) {
    S.q_nrow[k] = ts[k]->quad.Nt;
    S.t_nrow[k] = ts[k]->tri.Nt;
    S.q_first[k] = off[k] + ts[k]->quad.first;
    S.t_first[k] = off[k] + ts[k]->tri.first;
  }
  for (int type = 0; type < 2; ++type) {
    const bool q = type == 0;
    const int64_t R = q ? S.rows_q : S.rows_t;
    const int Sn = q ? uw::kQuad.S : uw::kTri.S;
    std::vector<int32_t>& out = q ? S.q_sid : S.t_sid;
    out.assign((size_t)(Sn - 1) * R, 0);
    for (int k = 0; k < n; ++k) {
      const uw::TypeTables& tt = q ? ts[k]->quad : ts[k]->tri;
      const int64_t r0 = q ? qrow[k] : trow[k];
      for (int s2 = 0; s2 < Sn - 1; ++s2)
        for (int64_t r = 0; r < tt.Nt; ++r)
          out[(size_t)s2 * R + r0 + r] = (int32_t)(tt.sid[(size_t)s2 * tt.Nt + r] + off[k]);
    }
  }
  retile(S, tile);
  // per-type tables, structure of arrays with the batch row count
  for (int type = 0; type < 2; ++type) {
    const bool q = type == 0;
    const int64_t R = q ? S.rows_q : S.rows_t;
    const std::vector<int64_t>& ro = q ? qrow : trow;
    cat_type(ts, q, [](const uw::TypeTables& t) -> const std::vector<double>& { return t.Y; }, R,
             ro, q ? S.q_Y : S.t_Y);
    cat_type(ts, q, [](const uw::TypeTables& t) -> const std::vector<double>& { return t.off; }, R,
             ro, q ? S.q_off : S.t_off);
    cat_type(ts, q, [](const uw::TypeTables& t) -> const std::vector<double>& { return t.gam; }, R,
             ro, q ? S.q_gam : S.t_gam);
    cat_type(ts, q, [](const uw::TypeTables& t) -> const std::vector<double>& { return t.sig; }, R,
             ro, q ? S.q_sig : S.t_sig);
    if (linear)
      cat_type(ts, q, [](const uw::TypeTables& t) -> const std::vector<double>& { return t.eta; },
               R, ro, q ? S.q_eta : S.t_eta);
  }
  // face tables; prescribed states, fronts and front faces of all
  // instances in one table each
  S.fnb.assign(4 * S.N, -1);
  S.fgeo.assign(12 * S.N, 0.0);
  for (int k = 0; k < n; ++k) {
    const int64_t Nk = ms[k]->N;
    const int32_t soff = (int32_t)(S.inflow.size() / 4);
    const int32_t foff = (int32_t)(S.fronts.size() / 12);
    const int32_t joff = (int32_t)S.ff_front.size();
    S.inflow.insert(S.inflow.end(), ms[k]->inflow.begin(), ms[k]->inflow.end());
    S.fronts.insert(S.fronts.end(), ms[k]->fronts.begin(), ms[k]->fronts.end());
    S.front_inst.resize(S.fronts.size() / 12, k);
    for (int c = 0; c < 4; ++c)
      for (int64_t i = 0; i < Nk; ++i) {
        const int32_t p = ts[k]->fnb[c * Nk + i];
        S.fnb[c * S.N + off[k] + i] =
            p <= -3 ? p - soff
                    : p < 0 ? p : (int32_t)((((int64_t)(p >> 3) + off[k]) << 3) | (p & 7));
        if (p <= -2) S.special = 1;
      }
    for (size_t j = 0; j < ms[k]->ff_face.size(); ++j) {
      const int64_t i = ms[k]->ff_face[j] / 4, c = ms[k]->ff_face[j] % 4;
      S.fnb[c * S.N + off[k] + i] = uw::kFrontCode - (joff + (int32_t)j);
      S.ff_front.push_back(ms[k]->ff_front[j] + foff);
      S.ff_proj.push_back(ms[k]->ff_proj[j]);
    }
    for (int c = 0; c < 12; ++c)
      std::copy(ts[k]->fgeo.begin() + c * Nk, ts[k]->fgeo.begin() + (c + 1) * Nk,
                S.fgeo.begin() + c * S.N + off[k]);
  }
}

template <class T>
struct DevTables {
  bool ready = false;
  DevBuf tiles, tile_off, tile_ids, inst_tiles, q_li, q_Y, q_off, q_gam, q_sig, q_eta, t_li, t_Y,
      t_off, t_gam, t_sig, t_eta, fnb, fnrm, fcoef, inflow, fronts, front_inst, ff_front, ff_proj;
  uw::MeshDev<T> view;
  void reset() {
    for (DevBuf* b : {&tiles, &tile_off, &tile_ids, &inst_tiles, &q_li, &q_Y, &q_off, &q_gam,
                      &q_sig, &q_eta, &t_li, &t_Y, &t_off, &t_gam, &t_sig, &t_eta, &fnb, &fnrm, &fcoef,
                      &inflow, &fronts, &front_inst, &ff_front, &ff_proj})
      b->release();
    view = uw::MeshDev<T>();
    ready = false;
  }
};

// Device state shared by a mesh and a batch: tables in both precisions
// (uploaded on first use), work buffers, launch schedule and timing.
struct Engine {
  int device = 0;
  uw::SchemeDev scheme{1e-3, 3.0, 0, 0};
  Staged staged;
  bool staged_ready = false;
  DevTables<double> d64;
  DevTables<float> d32;
  DevBuf FS, Wtmp, dt, partial, flag;
  int tile = uw::kTile;   // tile size asked for (the staged tables follow it)
  uw::Schedule sched;
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  // captured multi-step graphs, keyed by their arguments, with the serial
  // number of their last use; at most kMaxGraphs are kept (least recently
  // used evicted), so callers that vary the arguments do not accumulate them
  static constexpr size_t kMaxGraphs = 8;
  std::map<std::tuple<const void*, const void*, int, double, double, double, int, double, double,
                      double>,
           std::pair<hipGraphExec_t, uint64_t>>
      graphs;
  uint64_t graph_uses = 0;
  // graphs cannot be captured on the null stream: calls made on it capture
  // and replay on this blocking stream, which orders itself with the null one
  hipStream_t own_stream = nullptr;
  void reset_device() {
    d64.reset();
    d32.reset();
    clear_graphs();
  }
  void clear_graphs() {
    // a graph may still be running: let the device finish before destroying
    if (!graphs.empty() && device >= 0) {
      (void)hipSetDevice(device);
      (void)hipDeviceSynchronize();
    }
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second.first);
    graphs.clear();
  }
  ~Engine() {
    // queued launches and graphs may still use the buffers freed below
    if (device >= 0 && (d64.ready || d32.ready || FS.p)) {
      (void)hipSetDevice(device);
      (void)hipDeviceSynchronize();
    }
    clear_graphs();
    if (own_stream) (void)hipStreamDestroy(own_stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& u : ev_used) {
      (void)hipEventDestroy(u.second.first);
      (void)hipEventDestroy(u.second.second);
    }
  }
};

template <class T>
DevTables<T>& tables_of(Engine& e);
template <>
DevTables<double>& tables_of<double>(Engine& e) {
  return e.d64;
}
template <>
DevTables<float>& tables_of<float>(Engine& e) {
  return e.d32;
}

template <class T>
uw_status ensure_tables(Engine& E) {
  DevTables<T>& d = tables_of<T>(E);
  if (d.ready) return UW_OK;
  UW_HIP(hipSetDevice(E.device));
  const Staged& S = E.staged;
  hipError_t e = hipSuccess;
  auto up = [&](DevBuf& b, const auto& v) {
    if (e == hipSuccess) e = b.upload(v);
  };
  up(d.tiles, S.tiles);
  up(d.tile_off, S.tile_off);
  up(d.tile_ids, S.tile_ids);
  up(d.inst_tiles, S.inst_tiles);
  const int64_t Rq = S.rows_q, Rt = S.rows_t;
  up(d.q_li, chunked<uint16_t>(S.q_lidx, Rq));
  up(d.q_Y, chunked<T>(S.q_Y, Rq));
  up(d.q_off, chunked<T>(S.q_off, Rq));
  up(d.q_gam, chunked<T>(S.q_gam, Rq));
  up(d.q_sig, chunked<T>(S.q_sig, Rq));
  up(d.q_eta, chunked<T>(S.q_eta, Rq));
  up(d.t_li, chunked<uint16_t>(S.t_lidx, Rt));
  up(d.t_Y, chunked<T>(S.t_Y, Rt));
  up(d.t_off, chunked<T>(S.t_off, Rt));
  up(d.t_gam, chunked<T>(S.t_gam, Rt));
  up(d.t_sig, chunked<T>(S.t_sig, Rt));
  up(d.t_eta, chunked<T>(S.t_eta, Rt));
  up(d.fnb, S.fnb);
  if (!S.inflow.empty()) up(d.inflow, S.inflow);
  if (!S.ff_front.empty()) {
    up(d.fronts, S.fronts);
    up(d.front_inst, S.front_inst);
    up(d.ff_front, S.ff_front);
    up(d.ff_proj, S.ff_proj);
  }
  {
    std::vector<T> nrm;
    std::vector<double> coef;
    face_tables<T>(S.fgeo, S.fnb, S.N, nrm, coef);
    up(d.fnrm, nrm);
    up(d.fcoef, coef);
  }
  if (e == hipErrorOutOfMemory) return fail(UW_ENOMEM, "device tables: out of memory");
  if (e != hipSuccess) return hip_fail(e, "device tables upload");
  uw::MeshDev<T>& v = d.view;
  v.N = S.N;
  v.n_inst = S.n_inst;
  v.tile = S.tile;
  v.n_tq = S.n_tq;
  v.n_tt = S.n_tt;
  v.tiles = d.tiles.template as<uw::Tile>();
  v.tile_off = d.tile_off.template as<int32_t>();
  v.tile_ids = d.tile_ids.template as<int32_t>();
  v.max_len_q = S.max_len_q;
  v.max_len_t = S.max_len_t;
  v.inst_tiles = d.inst_tiles.template as<int32_t>();
  v.quad.Nt = S.rows_q;
  v.quad.lidx = d.q_li.template as<uint16_t>();
  v.quad.Y = d.q_Y.template as<T>();
  v.quad.off = d.q_off.template as<T>();
  v.quad.gam = d.q_gam.template as<T>();
  v.quad.sig = d.q_sig.template as<T>();
  v.quad.eta = d.q_eta.template as<T>();
  v.tri.Nt = S.rows_t;
  v.tri.lidx = d.t_li.template as<uint16_t>();
  v.tri.Y = d.t_Y.template as<T>();
  v.tri.off = d.t_off.template as<T>();
  v.tri.gam = d.t_gam.template as<T>();
  v.tri.sig = d.t_sig.template as<T>();
  v.tri.eta = d.t_eta.template as<T>();
  v.fnb = d.fnb.template as<int32_t>();
  v.inflow = S.inflow.empty() ? nullptr : d.inflow.template as<double>();
  // fronts is the kernels' test for front faces: null when there are none
  const bool ff = !S.ff_front.empty();
  v.fronts = ff ? d.fronts.template as<double>() : nullptr;
  v.front_inst = ff ? d.front_inst.template as<int32_t>() : nullptr;
  v.ff_front = ff ? d.ff_front.template as<int32_t>() : nullptr;
  v.ff_proj = ff ? d.ff_proj.template as<double>() : nullptr;
  v.special = S.special;
  v.fnrm = d.fnrm.template as<T>();
  v.fcoef = d.fcoef.template as<double>();
  d.ready = true;
  return UW_OK;
}

uw_status ensure_work(Engine& E, int nvar, size_t fs_elem) {
  const int64_t N = E.staged.N;
  const int64_t ntiles = (int64_t)E.staged.n_tq + E.staged.n_tt;
  const size_t fs_bytes = (size_t)N * 8 * nvar * fs_elem;
  const size_t w_bytes = (size_t)N * nvar * sizeof(double);
  // a buffer about to be replaced may still be read by queued launches or
  // graphs: let the device finish first
  if ((E.FS.p && fs_bytes > E.FS.bytes) || (E.Wtmp.p && w_bytes > E.Wtmp.bytes))
    UW_HIP(hipDeviceSynchronize());
  const void* before[4] = {E.FS.p, E.Wtmp.p, E.dt.p, E.partial.p};
  UW_HIP(E.FS.ensure(fs_bytes));
  UW_HIP(E.Wtmp.ensure(w_bytes));
  UW_HIP(E.dt.ensure((size_t)E.staged.n_inst * sizeof(double)));
  UW_HIP(E.partial.ensure((size_t)std::max<int64_t>(ntiles, 1) * sizeof(double)));
  // captured graphs hold the work buffers' addresses: a buffer that moved
  // (a larger one for more variables or a wider precision) retires them
  const void* after[4] = {E.FS.p, E.Wtmp.p, E.dt.p, E.partial.p};
  for (int k = 0; k < 4; ++k)
    if (before[k] && before[k] != after[k]) E.clear_graphs();
  if (!E.flag.p) {
    UW_HIP(E.flag.ensure(sizeof(int)));
    UW_HIP(hipMemset(E.flag.p, 0, sizeof(int)));
  }
  return UW_OK;
}

uw_status check_physics(const uw_physics* p) {
  if (!p) return fail(UW_EINVAL, "physics is NULL");
  if (p->equation != UW_ADVECTION && p->equation != UW_EULER)
    return fail(UW_EINVAL, "physics.equation must be UW_ADVECTION or UW_EULER");
  if (p->precision != UW_FP64 && p->precision != UW_FP32)
    return fail(UW_EINVAL, "physics.precision must be UW_FP64 or UW_FP32");
  if (p->equation == UW_EULER && !(p->gamma > 1.0))
    return fail(UW_EINVAL, "physics.gamma must exceed 1");
  return UW_OK;
}

int nvar_of(const uw_physics* p) { return p->equation == UW_EULER ? 4 : 1; }

uw::PhysDev phys_dev(const uw_physics* p) {
  return uw::PhysDev{p->equation, p->ax, p->ay, p->gamma};
}

hipError_t ev_begin(Engine& E, hipStream_t st, hipEvent_t* a, hipEvent_t* b) {
  for (hipEvent_t* e : {a, b}) {
    if (!E.ev_pool.empty()) {
      *e = E.ev_pool.back();
      E.ev_pool.pop_back();
    } else {
      hipError_t r = hipEventCreate(e);
      if (r != hipSuccess) return r;
    }
  }
  return hipEventRecord(*a, st);
}

// One residual evaluation (mode 0) or RK stage (modes 1..3), with the face
// states in FS (the engine's buffer unless given).
template <class T>
uw_status stage(Engine& E, const uw_physics* p, int mode, const double* W_in, const double* Wn,
                double* W_out, const uw::StageTime& tm, hipStream_t st, bool timed,
                T* FS = nullptr, double* partial = nullptr) {
  const int nvar = nvar_of(p);
  DevTables<T>& d = tables_of<T>(E);
  if (!FS) FS = E.FS.template as<T>();
  if (E.staged.tile != 256 &&
      (sizeof(T) == 8 || E.scheme.mode == 1 || (E.scheme.vars == 1 && nvar == 4)))
    return fail(UW_EINVAL, "512-cell tiles serve FP32 WENO on the conserved variables only; "
                           "set the tile size to 256 (uw_tile_size)");
  const bool prof = timed && E.profiling;
  hipEvent_t a = nullptr, b = nullptr;
  if (prof) UW_HIP(ev_begin(E, st, &a, &b));
  hipError_t e =
      uw::launch_recon<T>(d.view, E.scheme, phys_dev(p), E.sched, nvar, W_in, FS, tm, st);
  if (e != hipSuccess) return hip_fail(e, "reconstruction launch");
  if (prof) {
    UW_HIP(hipEventRecord(b, st));
    E.ev_used.push_back({0, {a, b}});
    UW_HIP(ev_begin(E, st, &a, &b));
  }
  e = uw::launch_flux<T>(d.view, phys_dev(p), E.sched, nvar, mode, FS, W_in, Wn, W_out,
                         E.dt.as<double>(), E.flag.as<int>(), tm, st, partial);
  if (e != hipSuccess) return hip_fail(e, "flux launch");
  if (prof) {
    UW_HIP(hipEventRecord(b, st));
    E.ev_used.push_back({1, {a, b}});
  }
  return UW_OK;
}

template <class T>
uw_status prepare(Engine& E, const uw_physics* p) {
  UW_TRY(ensure_tables<T>(E));
  return ensure_work(E, nvar_of(p), sizeof(T));
}

// One SSP-RK3 step of every instance (time step on the device).  Inside a
// run of steps the last stage's flux launch forms the next step's per-tile
// time-step bounds (make_partial), and the next step then only reduces them
// (have_partial): the same bounds, from the same states and formula, as a
// separate pass over W.
template <class T>
uw_status rk3(Engine& E, const uw_physics* p, double* W, double cfl, double dt_fixed,
              double t_end, double* t_dev, hipStream_t st, bool timed,
              bool have_partial = false, bool make_partial = false) {
  DevTables<T>& d = tables_of<T>(E);
  hipError_t e = uw::launch_cfl<T>(d.view, phys_dev(p), nvar_of(p), W, cfl, dt_fixed, t_end,
                                   t_dev, E.partial.as<double>(), E.dt.as<double>(), st,
                                   have_partial && dt_fixed <= 0.0);
  if (e != hipSuccess) return hip_fail(e, "time-step launch");
  double* W1 = E.Wtmp.as<double>();
  // the stages see the boundary data at t, t + dt and t + dt/2
  const double* dtp = E.dt.as<double>();
  UW_TRY(stage<T>(E, p, 1, W, W, W1, uw::StageTime{t_dev, dtp, 0.0, 0.0}, st, timed));
  UW_TRY(stage<T>(E, p, 2, W1, W, W1, uw::StageTime{t_dev, dtp, 1.0, 0.0}, st, timed));
  UW_TRY(stage<T>(E, p, 3, W1, W, W, uw::StageTime{t_dev, dtp, 0.5, 0.0}, st, timed, nullptr,
                  make_partial && dt_fixed <= 0.0 ? E.partial.as<double>() : nullptr));
  e = uw::launch_advance(E.staged.n_inst, t_dev, E.dt.as<double>(), st);
  if (e != hipSuccess) return hip_fail(e, "time advance launch");
  return UW_OK;
}

template <class T>
uw_status rk3_steps(Engine& E, const uw_physics* p, double* W, double cfl, double dt_fixed,
                    double t_end, int n_steps, double* t_dev, hipStream_t st, bool graph) {
  UW_TRY(prepare<T>(E, p));
  if (!graph || n_steps <= 0) {
    for (int k = 0; k < n_steps; ++k)
      UW_TRY(rk3<T>(E, p, W, cfl, dt_fixed, t_end, t_dev, st, true, k > 0, k + 1 < n_steps));
    return UW_OK;
  }
  if (!st) {
    if (!E.own_stream) UW_HIP(hipStreamCreate(&E.own_stream));
    st = E.own_stream;
  }
  auto key = std::make_tuple((const void*)W, (const void*)t_dev, n_steps, cfl, dt_fixed, t_end,
                             p->precision * 16 + p->equation, p->gamma, p->ax, p->ay);
  auto it = E.graphs.find(key);
  if (it == E.graphs.end()) {
    if (E.graphs.size() >= Engine::kMaxGraphs) {
      // evict the least recently used graph, after the device has finished
      // anything it may still be running
      auto lru = E.graphs.begin();
      for (auto g = E.graphs.begin(); g != E.graphs.end(); ++g)
        if (g->second.second < lru->second.second) lru = g;
      UW_HIP(hipDeviceSynchronize());
      (void)hipGraphExecDestroy(lru->second.first);
      E.graphs.erase(lru);
    }
    UW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    uw_status s = UW_OK;
    for (int k = 0; k < n_steps && s == UW_OK; ++k)
      s = rk3<T>(E, p, W, cfl, dt_fixed, t_end, t_dev, st, false, k > 0, k + 1 < n_steps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != UW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    it = E.graphs.emplace(key, std::make_pair(ex, uint64_t{0})).first;
  }
  it->second.second = ++E.graph_uses;
  UW_HIP(hipGraphLaunch(it->second.first, st));
  return UW_OK;
}

// Face states of uw_residual_noalloc: one fixed array per device, never
// allocated or freed by the library.  In host code `scratch` names a host
// stand-in; its device address on each GPU comes from hipGetSymbolAddress,
// taken once per device with that device current and kept in scratch_dev.
constexpr size_t kNoAllocScratch = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};

// Device address of `scratch` on `device`, which must be the current device.
uw_status scratch_on(int device, void** out) {
  if (device < 0 || device >= 64) return fail(UW_EINVAL, "device index out of range (0..63)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(UW_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return UW_OK;
}

template <class T>
uw_status residual_noalloc(Engine& E, const uw_physics* p, const double* W, double* L,
                           hipStream_t st) {
  if (!tables_of<T>(E).ready || !E.flag.p)
    return fail(UW_ESTATE,
                "uw_residual_noalloc: the mesh's device tables in this precision do not exist "
                "yet; call uw_residual (or uw_rk3_step, uw_cfl_dt, uw_autotune) once in this "
                "precision first");
  const int64_t N = E.staged.N;
  const size_t need = (size_t)N * 8 * (size_t)nvar_of(p) * sizeof(T);
  if (need > kNoAllocScratch)
    return fail(UW_EINVAL, "uw_residual_noalloc: " + std::to_string(N) + " cells need " +
                               std::to_string(need) + " bytes of face-state scratch; the limit "
                               "is " + std::to_string(kNoAllocScratch) + " bytes");
  void* ptr = nullptr;
  UW_TRY(scratch_on(E.device, &ptr));
  return stage<T>(E, p, 0, W, W, L, uw::StageTime{nullptr, nullptr, 0.0, 0.0}, st, false,
                  static_cast<T*>(ptr));
}

// Re-tiles a mesh's or batch's staged tables for `tile` cells per tile:
// device tables are dropped (uploaded again on first use) after the device
// has finished queued work, and captured steps are retired.
uw_status set_tile(Engine& E, int tile) {
  if (!uw::tile_size_ok(tile)) return fail(UW_EINVAL, "tile size must be 256 or 512");
  if (tile == E.tile && (!E.staged_ready || E.staged.tile == tile)) return UW_OK;
  if (E.device >= 0 && (E.d64.ready || E.d32.ready)) {
    UW_HIP(hipSetDevice(E.device));
    UW_HIP(hipDeviceSynchronize());
  }
  E.tile = tile;
  E.reset_device();
  if (E.staged_ready) {
    try {
      retile(E.staged, tile);
    } catch (const std::bad_alloc&) {
      E.staged_ready = false;
      return fail(UW_ENOMEM, "host allocation while re-tiling");
    }
  }
  return UW_OK;
}
uw_status check_scheme(const uw_scheme* sc) {
  if (!sc) return fail(UW_EINVAL, "scheme is NULL");
  if (!(sc->zeta >= 0.0) || !(sc->eps > 0.0) || !(sc->theta > 1.0) || !std::isfinite(sc->theta))
    return fail(UW_EINVAL, "scheme needs zeta >= 0, eps > 0, theta > 1");
  if (sc->mode != UW_WENO && sc->mode != UW_LINEAR) return fail(UW_EINVAL, "scheme.mode");
  if (sc->variables != UW_CONSERVED && sc->variables != UW_CHARACTERISTIC)
    return fail(UW_EINVAL, "scheme.variables");
  if (sc->d_scope != UW_D_PER_GP && sc->d_scope != UW_D_PER_CELL)
    return fail(UW_EINVAL, "scheme.d_scope");
  return UW_OK;
}

}  // namespace

struct uw_mesh {
  uw::HostMesh host;
  uw::HostTables tables;
  uw::SchemeParams scheme;
  bool precomputed = false;
  Engine eng;
};

struct uw_batch {
  std::vector<uw_mesh*> meshes;
  uw_physics physics;
  std::vector<int64_t> offsets;
  Engine eng;
};

namespace {

uw_status mesh_ready(uw_mesh* m) {
  if (!m->precomputed) return fail(UW_ESTATE, "call uw_precompute_geometry first");
  if (m->eng.device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
  if (!m->eng.staged_ready) {
    try {
      assemble({&m->host}, {&m->tables}, m->scheme.mode == 1, m->eng.tile, m->eng.staged);
    } catch (const std::bad_alloc&) {
      return fail(UW_ENOMEM, "host allocation while staging tables");
    }
    m->eng.staged_ready = true;
  }
  UW_HIP(hipSetDevice(m->eng.device));
  return UW_OK;
}

}  // namespace

extern "C" {

const char* uw_last_error(void) { return g_err.c_str(); }

uw_status uw_mesh_upload(const uw_mesh_desc* desc, int device, uw_mesh** out) {
  g_err.clear();
  if (!desc || !out) return fail(UW_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  if (!desc->node_xy || !desc->cell_nodes || desc->n_nodes < 3 || desc->n_cells < 1)
    return fail(UW_EINVAL, "mesh needs node_xy, cell_nodes, >= 3 nodes and >= 1 cell");
  if (desc->bc != UW_BC_PERIODIC && desc->bc != UW_BC_TRANSMISSIVE)
    return fail(UW_EINVAL, "bc must be UW_BC_PERIODIC or UW_BC_TRANSMISSIVE");
  if (desc->n_cells > (int64_t(1) << 28)) return fail(UW_EINVAL, "at most 2^28 cells");
  if (desc->n_inflow < 0 || desc->n_inflow > UW_BC_FRONT - UW_BC_INFLOW ||
      (desc->n_inflow > 0 && !desc->inflow_W))
    return fail(UW_EINVAL, "n_inflow must be in [0, 65533] with inflow_W given");
  if (desc->n_fronts < 0 || desc->n_fronts > (1 << 20) || (desc->n_fronts > 0 && !desc->fronts))
    return fail(UW_EINVAL, "n_fronts must be in [0, 2^20] with fronts given");
  for (int64_t q = 0; q < 12 * (int64_t)desc->n_fronts; ++q)
    if (!std::isfinite(desc->fronts[q])) return fail(UW_EINVAL, "fronts must be finite");
  uw_mesh* m = new (std::nothrow) uw_mesh();
  if (!m) return fail(UW_ENOMEM, "host allocation");
  m->eng.device = device;
  uw::Error err;
  try {
    if (!uw::build_mesh(desc->n_nodes, desc->node_xy, desc->n_cells, desc->cell_nodes,
                        desc->node_id, desc->bc, desc->face_bc, desc->n_inflow, desc->inflow_W,
                        desc->n_fronts, desc->fronts, m->host, err)) {
      delete m;
      return fail((uw_status)err.code, err.msg);
    }
  } catch (const std::bad_alloc&) {
    delete m;
    return fail(UW_ENOMEM, "host allocation while building the mesh");
  }
  if (device >= 0) {
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || device >= ndev) {
      delete m;
      return fail(UW_EDEVICE, "no such HIP device");
    }
  }
  *out = m;
  return UW_OK;
}

uw_status uw_mesh_info(const uw_mesh* m, int64_t* n_cells, int64_t* n_quads,
                       int64_t* n_interior_faces, int32_t* new_of_old) {
  g_err.clear();
  if (!m) return fail(UW_EINVAL, "mesh is NULL");
  if (n_cells) *n_cells = m->host.N;
  if (n_quads) *n_quads = m->host.Nq;
  if (n_interior_faces) *n_interior_faces = m->host.n_interior_faces;
  if (new_of_old)
    std::memcpy(new_of_old, m->host.new_of_old.data(), sizeof(int32_t) * m->host.N);
  return UW_OK;
}

uw_status uw_mesh_export(const uw_mesh* m, int32_t* slots, uint8_t* present, int32_t* nbr) {
  g_err.clear();
  if (!m) return fail(UW_EINVAL, "mesh is NULL");
  const int64_t N = m->host.N;
  for (int64_t i = 0; i < N; ++i) {
    const int S = m->host.nf[i] == 4 ? 13 : 10;
    for (int j = 0; j < 13; ++j) {
      const int64_t k = 13 * i + j;
      if (slots) slots[k] = j < S ? m->host.st_cell[13 * i + m->host.st_res[k]] : -1;
      if (present) present[k] = j < S ? m->host.st_present[k] : 0;
    }
    if (nbr)
      for (int k = 0; k < 4; ++k) nbr[4 * i + k] = m->host.nbr[4 * i + k];
  }
  return UW_OK;
}

uw_status uw_precompute_geometry(uw_mesh* m, const uw_scheme* sc, uw_diag* diag) {
  g_err.clear();
  if (!m) return fail(UW_EINVAL, "mesh is NULL");
  UW_TRY(check_scheme(sc));
  m->scheme.zeta = sc->zeta;
  m->scheme.theta = sc->theta;
  m->scheme.eps = sc->eps;
  m->scheme.optimize = sc->optimize;
  m->scheme.d_scope = sc->d_scope;
  m->scheme.mode = sc->mode;
  // queued launches and graphs may still read the tables about to be freed
  if (m->eng.device >= 0 && (m->eng.d64.ready || m->eng.d32.ready)) {
    UW_HIP(hipSetDevice(m->eng.device));
    UW_HIP(hipDeviceSynchronize());
  }
  m->eng.reset_device();
  m->eng.staged = Staged();
  m->eng.staged_ready = false;
  m->eng.scheme = uw::SchemeDev{sc->eps, sc->theta, sc->mode, sc->variables};
  // on the mesh's GPU (one thread per cell) when it has one, else on host threads
  try {
    m->tables = uw::HostTables();
    if (m->eng.device >= 0) {
      std::string msg;
      int code = 0;
      if (!uw::precompute_tables_device(m->host, m->scheme, m->tables, m->eng.device,
                                        uw::default_threads(), msg, code)) {
        m->tables = uw::HostTables();
        return fail(code == (int)hipErrorOutOfMemory ? UW_ENOMEM : UW_EDEVICE, msg);
      }
    } else {
      uw::precompute_tables(m->host, m->scheme, m->tables, uw::default_threads());
    }
  } catch (const std::bad_alloc&) {
    return fail(UW_ENOMEM, "host allocation in precompute");
  }
  m->precomputed = true;
  if (diag) {
    diag->max_abs_gamma_raw = m->tables.max_abs_gamma_raw;
    diag->max_abs_gamma_opt = m->tables.max_abs_gamma_opt;
    diag->resid_opt = m->tables.resid_opt;
    diag->sum_dev = m->tables.sum_dev;
    diag->n_absent_slots = m->tables.n_absent;
    diag->n_rank_deficient = m->tables.n_rank_def;
  }
  return UW_OK;
}

uw_status uw_mesh_table(const uw_mesh* m, int32_t which, double* out) {
  g_err.clear();
  if (!m || !out) return fail(UW_EINVAL, "mesh and out must not be NULL");
  if (!m->precomputed) return fail(UW_ESTATE, "no precompute yet");
  const uw::HostTables& t = m->tables;
  if (!t.debug) return fail(UW_ESTATE, "per-cell tables are kept for meshes up to 4M cells only");
  const std::vector<double>* src = nullptr;
  switch (which) {
    case 0: src = &t.dbg_gamma; break;
    case 1: src = &t.dbg_eta; break;
    case 2: src = &t.dbg_Y; break;
    case 3: src = &t.dbg_off; break;
    case 4: src = &t.dbg_face; break;
    case 5: src = &t.dbg_gamma_raw; break;
    default: return fail(UW_EINVAL, "which must be 0..5");
  }
  std::memcpy(out, src->data(), src->size() * sizeof(double));
  return UW_OK;
}

uw_status uw_residual_at(uw_mesh* m, const uw_physics* p, const double* W, double* L, double t,
                         void* stream) {
  g_err.clear();
  if (!m || !W || !L) return fail(UW_EINVAL, "mesh, W and L must not be NULL");
  if (!std::isfinite(t)) return fail(UW_EINVAL, "t must be finite");
  UW_TRY(check_physics(p));
  UW_TRY(mesh_ready(m));
  hipStream_t st = (hipStream_t)stream;
  const uw::StageTime tm{nullptr, nullptr, 0.0, t};
  if (p->precision == UW_FP64) {
    UW_TRY(prepare<double>(m->eng, p));
    return stage<double>(m->eng, p, 0, W, W, L, tm, st, true);
  }
  UW_TRY(prepare<float>(m->eng, p));
  return stage<float>(m->eng, p, 0, W, W, L, tm, st, true);
}

uw_status uw_residual(uw_mesh* m, const uw_physics* p, const double* W, double* L, void* stream) {
  return uw_residual_at(m, p, W, L, 0.0, stream);
}

uw_status uw_residual_noalloc(uw_mesh* m, const uw_physics* p, const double* W, double* L,
                              void* stream) {
  g_err.clear();
  if (!m || !W || !L) return fail(UW_EINVAL, "mesh, W and L must not be NULL");
  UW_TRY(check_physics(p));
  if (!m->precomputed) return fail(UW_ESTATE, "call uw_precompute_geometry first");
  if (m->eng.device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
  if (!m->eng.staged_ready)
    return fail(UW_ESTATE, "uw_residual_noalloc: the mesh's device tables do not exist yet; call "
                           "uw_residual once in this precision first");
  UW_HIP(hipSetDevice(m->eng.device));
  hipStream_t st = (hipStream_t)stream;
  if (p->precision == UW_FP64) return residual_noalloc<double>(m->eng, p, W, L, st);
  return residual_noalloc<float>(m->eng, p, W, L, st);
}

uw_status uw_rk3_steps(uw_mesh* m, const uw_physics* p, double* W, double cfl, double dt_fixed,
                       double t_end, int32_t n_steps, double* t_dev, void* stream) {
  g_err.clear();
  if (!m || !W || !t_dev) return fail(UW_EINVAL, "mesh, W and t_dev must not be NULL");
  if (n_steps < 0) return fail(UW_EINVAL, "n_steps must be >= 0");
  UW_TRY(check_physics(p));
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(UW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  UW_TRY(mesh_ready(m));
  hipStream_t st = (hipStream_t)stream;
  // replay a captured graph of the steps (one launch instead of about a
  // dozen per step) unless per-kernel timing is on, which records events
  // between launches
  const bool graph = !m->eng.profiling;
  if (p->precision == UW_FP64)
    return rk3_steps<double>(m->eng, p, W, cfl, dt_fixed, t_end, n_steps, t_dev, st, graph);
  return rk3_steps<float>(m->eng, p, W, cfl, dt_fixed, t_end, n_steps, t_dev, st, graph);
}

uw_status uw_rk3_step(uw_mesh* m, const uw_physics* p, double* W, double cfl, double dt_fixed,
                      double t_end, double* t_dev, void* stream) {
  return uw_rk3_steps(m, p, W, cfl, dt_fixed, t_end, 1, t_dev, stream);
}

uw_status uw_cfl_dt(uw_mesh* m, const uw_physics* p, const double* W, double cfl, double* dt_dev,
                    void* stream) {
  g_err.clear();
  if (!m || !W || !dt_dev) return fail(UW_EINVAL, "mesh, W and dt_dev must not be NULL");
  UW_TRY(check_physics(p));
  if (!(cfl > 0.0)) return fail(UW_EINVAL, "cfl must be > 0");
  UW_TRY(mesh_ready(m));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (p->precision == UW_FP64) {
    UW_TRY(prepare<double>(m->eng, p));
    e = uw::launch_cfl<double>(m->eng.d64.view, phys_dev(p), nvar_of(p), W, cfl, 0.0, INFINITY,
                               nullptr, m->eng.partial.as<double>(), dt_dev, st);
  } else {
    UW_TRY(prepare<float>(m->eng, p));
    e = uw::launch_cfl<float>(m->eng.d32.view, phys_dev(p), nvar_of(p), W, cfl, 0.0, INFINITY,
                              nullptr, m->eng.partial.as<double>(), dt_dev, st);
  }
  if (e != hipSuccess) return hip_fail(e, "time-step launch");
  return UW_OK;
}

uw_status uw_batch_create(uw_mesh* const* meshes, int32_t n, const uw_physics* p, uw_batch** out) {
  g_err.clear();
  if (!meshes || !out || n < 1) return fail(UW_EINVAL, "need meshes, out and n >= 1");
  *out = nullptr;
  UW_TRY(check_physics(p));
  std::vector<const uw::HostMesh*> hm;
  std::vector<const uw::HostTables*> ht;
  int64_t total = 0, states = 0, ffaces = 0;
  for (int32_t k = 0; k < n; ++k) {
    uw_mesh* m = meshes[k];
    if (!m || !m->precomputed) return fail(UW_ESTATE, "every batch mesh must be precomputed");
    if (m->eng.device < 0 || m->eng.device != meshes[0]->eng.device)
      return fail(UW_EINVAL, "batch meshes must live on one device");
    if (m->scheme.mode != meshes[0]->scheme.mode || m->scheme.eps != meshes[0]->scheme.eps ||
        m->scheme.theta != meshes[0]->scheme.theta ||
        m->eng.scheme.vars != meshes[0]->eng.scheme.vars)
      return fail(UW_EINVAL, "batch meshes must share one scheme");
    hm.push_back(&m->host);
    ht.push_back(&m->tables);
    total += m->host.N;
    states += (int64_t)m->host.inflow.size() / 4;
    ffaces += (int64_t)m->host.ff_face.size();
  }
  if (total > (int64_t(1) << 28)) return fail(UW_EINVAL, "at most 2^28 cells in a batch");
  // boundary codes: -3 - s for state s must stay above the front codes
  if (states > -uw::kFrontCode - 4)
    return fail(UW_EINVAL, "at most 2^24 - 4 prescribed states in a batch");
  if (ffaces > (int64_t(1) << 30)) return fail(UW_EINVAL, "at most 2^30 front faces in a batch");
  uw_batch* b = new (std::nothrow) uw_batch();
  if (!b) return fail(UW_ENOMEM, "host allocation");
  b->physics = *p;
  b->offsets.push_back(0);
  for (int32_t k = 0; k < n; ++k) {
    b->meshes.push_back(meshes[k]);
    b->offsets.push_back(b->offsets.back() + meshes[k]->host.N);
  }
  b->eng.device = meshes[0]->eng.device;
  b->eng.scheme = meshes[0]->eng.scheme;
  try {
    assemble(hm, ht, meshes[0]->scheme.mode == 1, b->eng.tile, b->eng.staged);
  } catch (const std::bad_alloc&) {
    delete b;
    return fail(UW_ENOMEM, "host allocation while staging the batch");
  }
  b->eng.staged_ready = true;
  *out = b;
  return UW_OK;
}

uw_status uw_batch_offsets(const uw_batch* b, int64_t* cell_offsets) {
  g_err.clear();
  if (!b || !cell_offsets) return fail(UW_EINVAL, "batch and cell_offsets must not be NULL");
  std::memcpy(cell_offsets, b->offsets.data(), sizeof(int64_t) * b->offsets.size());
  return UW_OK;
}

uw_status uw_batch_rk3_step(uw_batch* b, double* W, double cfl, double dt_fixed, double t_end,
                            int32_t n_steps, double* t_dev, void* stream) {
  g_err.clear();
  if (!b || !W || !t_dev || n_steps < 0) return fail(UW_EINVAL, "batch, W, t_dev, n_steps >= 0");
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(UW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  UW_HIP(hipSetDevice(b->eng.device));
  hipStream_t st = (hipStream_t)stream;
  if (b->physics.precision == UW_FP64)
    return rk3_steps<double>(b->eng, &b->physics, W, cfl, dt_fixed, t_end, n_steps, t_dev, st,
                             true);
  return rk3_steps<float>(b->eng, &b->physics, W, cfl, dt_fixed, t_end, n_steps, t_dev, st,
                          true);
}

uw_status uw_autotune(uw_mesh* m, uw_batch* b, const uw_physics* p, const char* cache_path,
                      void* stream) {
  g_err.clear();
  if ((!m) == (!b)) return fail(UW_EINVAL, "give exactly one of a mesh or a batch");
  UW_TRY(check_physics(p));
  if (m) UW_TRY(mesh_ready(m));
  Engine& E = m ? m->eng : b->eng;
  UW_HIP(hipSetDevice(E.device));
  hipStream_t st = (hipStream_t)stream;
  const int nvar = nvar_of(p);
  char key[200];
  // the workload's shape, independent of the tile size the tuning may change
  std::snprintf(key, sizeof(key), "%lld %d %lld %lld %d %d %d", (long long)E.staged.N,
                E.staged.n_inst, (long long)E.staged.rows_q, (long long)E.staged.rows_t, nvar,
                p->precision, E.scheme.mode + 2 * E.scheme.vars);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[320];
      bool found = false;
      int tile_found = uw::kTile;
      while (std::fgets(line, sizeof(line), f)) {
        long long a, c2, c3;
        int c1, c4, c5, c6, rq, rt, fl, tl;
        if (std::sscanf(line, "%lld %d %lld %lld %d %d %d %d %d %d %d", &a, &c1, &c2, &c3, &c4,
                        &c5, &c6, &rq, &rt, &fl, &tl) == 11) {
          char k2[200];
          std::snprintf(k2, sizeof(k2), "%lld %d %lld %lld %d %d %d", a, c1, c2, c3, c4, c5, c6);
          if (std::strcmp(k2, key) == 0 && rq >= 0 && rt >= -1 && fl >= 0 &&
              uw::tile_size_ok(tl)) {
            E.sched = uw::Schedule{rq, rt, fl};
            tile_found = tl;
            found = true;
          }
        }
      }
      std::fclose(f);
      if (found) {
        UW_TRY(set_tile(E, tile_found));
        E.clear_graphs();
        return UW_OK;
      }
    }
  }
  // a uniform admissible state to time the kernels on
  const int64_t N = E.staged.N;
  std::vector<double> h((size_t)nvar * N);
  for (int64_t i = 0; i < N; ++i) {
    if (nvar == 4) {
      h[i] = 1.0;
      h[N + i] = 0.5;
      h[2 * N + i] = 0.25;
      h[3 * N + i] = 2.5;
    } else {
      h[i] = 1.0;
    }
  }
  DevBuf Wt, Lt;
  UW_HIP(Wt.upload(h));
  UW_HIP(Lt.ensure(h.size() * sizeof(double)));
  int cus = 256;
  UW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, E.device));
  hipEvent_t e0, e1;
  UW_HIP(hipEventCreate(&e0));
  UW_HIP(hipEventCreate(&e1));
  uw_status s = UW_OK;
  // time of one residual evaluation (mean of three after a warm-up run)
  auto time_residual = [&](float* out) -> uw_status {
    float tot = 0.0f;
    for (int rep = 0; rep < 4; ++rep) {
      UW_HIP(hipEventRecord(e0, st));
      UW_TRY(p->precision == UW_FP64
                 ? stage<double>(E, p, 0, Wt.as<double>(), Wt.as<double>(), Lt.as<double>(),
                                 uw::StageTime{}, st, false)
                 : stage<float>(E, p, 0, Wt.as<double>(), Wt.as<double>(), Lt.as<double>(),
                                uw::StageTime{}, st, false));
      UW_HIP(hipEventRecord(e1, st));
      UW_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      UW_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tot += ms;
    }
    *out = tot / 3.0f;
    return UW_OK;
  };
  // tile sizes: 512 only where the kernels exist for it (FP32, WENO on the
  // conserved variables) and its LDS fits
  std::vector<int> tiles = {256};
  if (p->precision == UW_FP32 && E.scheme.mode == 0 && !(E.scheme.vars == 1 && nvar == 4))
    tiles.push_back(512);
  // candidate launch shapes: one block per tile (0) or k persistent blocks per CU
  const int mult[5] = {0, 1, 2, 4, 8};
  float best_all = 1e30f;
  int best_tile = E.tile;
  uw::Schedule best_sched = E.sched;
  for (int tile : tiles) {
    s = set_tile(E, tile);
    if (s == UW_OK) s = p->precision == UW_FP64 ? prepare<double>(E, p) : prepare<float>(E, p);
    if (s != UW_OK) break;
    if (tile != 256) {
      const size_t need =
          std::max(p->precision == UW_FP64
                       ? uw::recon_lds<double>(std::max(E.staged.max_len_q, E.staged.max_len_t),
                                               nvar, tile)
                       : uw::recon_lds<float>(std::max(E.staged.max_len_q, E.staged.max_len_t),
                                              nvar, tile),
                   (size_t)0);
      int lim = 0;
      UW_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, E.device));
      if (need > (size_t)lim) continue;
    }
    if (E.sched.recon_t < 0) E.sched.recon_t = 0;   // separate launches first
    for (int knob = 0; knob < 3 && s == UW_OK; ++knob) {
      int* val = knob == 0 ? &E.sched.recon_q : knob == 1 ? &E.sched.recon_t : &E.sched.flux;
      int best_v = *val;
      float best = 1e30f;
      for (int c : mult) {
        *val = c * cus;
        float ms = 0.0f;
        s = time_residual(&ms);
        if (s != UW_OK) break;
        if (ms < best) {
          best = ms;
          best_v = *val;
        }
      }
      *val = best_v;
    }
    float ms = 0.0f;
    if (s == UW_OK) s = time_residual(&ms);
    if (s != UW_OK) break;
    // both cell types in one reconstruction launch (recon_t = -1), where
    // both types are present and the two kernels share launch bounds
    const bool mergeable = E.staged.n_tq > 0 && E.staged.n_tt > 0 &&
                           (p->precision == UW_FP64 || E.scheme.mode != 1);
    if (mergeable) {
      const uw::Schedule sep = E.sched;
      float best_m = ms;
      uw::Schedule best_ms = sep;
      for (int c : mult) {
        E.sched = uw::Schedule{c * cus, -1, sep.flux};
        float mm = 0.0f;
        s = time_residual(&mm);
        if (s != UW_OK) break;
        if (mm < best_m) {
          best_m = mm;
          best_ms = E.sched;
        }
      }
      if (s != UW_OK) break;
      E.sched = best_ms;
      ms = best_m;
    }
    if (ms < best_all) {
      best_all = ms;
      best_tile = tile;
      best_sched = E.sched;
    }
  }
  if (s == UW_OK) {
    s = set_tile(E, best_tile);
    E.sched = best_sched;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != UW_OK) return s;
  E.clear_graphs();
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %d %d %d %d\n", key, E.sched.recon_q, E.sched.recon_t, E.sched.flux,
                   E.tile);
      std::fclose(f);
    }
  }
  return UW_OK;
}

uw_status uw_tile_size(uw_mesh* m, uw_batch* b, int32_t set, int32_t* get) {
  g_err.clear();
  if ((!m) == (!b)) return fail(UW_EINVAL, "give exactly one of a mesh or a batch");
  Engine& E = m ? m->eng : b->eng;
  if (set != 0) UW_TRY(set_tile(E, set));
  if (get) *get = E.tile;
  return UW_OK;
}

uw_status uw_schedule(uw_mesh* m, uw_batch* b, int32_t* get, const int32_t* set) {
  g_err.clear();
  if ((!m) == (!b)) return fail(UW_EINVAL, "give exactly one of a mesh or a batch");
  Engine& E = m ? m->eng : b->eng;
  if (set) {
    if (set[0] < 0 || set[1] < -1 || set[2] < 0)
      return fail(UW_EINVAL, "schedule entries must be >= 0 (the second >= -1)");
    E.sched = uw::Schedule{set[0], set[1], set[2]};
    E.clear_graphs();
  }
  if (get) {
    get[0] = E.sched.recon_q;
    get[1] = E.sched.recon_t;
    get[2] = E.sched.flux;
  }
  return UW_OK;
}

uw_status uw_check(uw_mesh* m, uw_batch* b, void* stream) {
  g_err.clear();
  hipStream_t st = (hipStream_t)stream;
  UW_HIP(hipStreamSynchronize(st));
  bool bad = false;
  for (Engine* E : {m ? &m->eng : nullptr, b ? &b->eng : nullptr}) {
    if (!E || !E->flag.p) continue;
    int h = 0;
    UW_HIP(hipMemcpy(&h, E->flag.p, sizeof(int), hipMemcpyDeviceToHost));
    if (h) {
      bad = true;
      UW_HIP(hipMemset(E->flag.p, 0, sizeof(int)));
    }
  }
  if (bad) return fail(UW_ENONFINITE, "non-finite value or non-positive density in a step");
  return UW_OK;
}

uw_status uw_profile(uw_mesh* m, int32_t enable, double* ms, int64_t* count) {
  g_err.clear();
  if (!m) return fail(UW_EINVAL, "mesh is NULL");
  Engine& E = m->eng;
  if (ms || count) {
    for (int k = 0; k < 2; ++k) {
      if (ms) ms[k] = 0.0;
      if (count) count[k] = 0;
    }
    for (auto& u : E.ev_used) {
      UW_HIP(hipEventSynchronize(u.second.second));
      float t = 0.0f;
      UW_HIP(hipEventElapsedTime(&t, u.second.first, u.second.second));
      if (ms) ms[u.first] += t;
      if (count) count[u.first] += 1;
    }
  }
  for (auto& u : E.ev_used) {
    E.ev_pool.push_back(u.second.first);
    E.ev_pool.push_back(u.second.second);
  }
  E.ev_used.clear();
  if (enable >= 0) E.profiling = enable != 0;
  return UW_OK;
}

void uw_mesh_destroy(uw_mesh* m) { delete m; }

void uw_batch_destroy(uw_batch* b) { delete b; }

}  // extern "C"
