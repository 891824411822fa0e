// C-ABI of the uweno library: mesh upload, FP64 precompute, residual,
// SSP-RK3 steps, CFL time step, batches, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/uweno.h"
#include "uw_device.h"
#include "uw_host.h"

static_assert(uw::kTile == uw::kReconBlock, "tile size and reconstruction block differ");

namespace {

thread_local std::string g_err;

uw_status fail(uw_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

uw_status hip_fail(hipError_t e, const char* what) {
  return fail(UW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define UW_HIP(call)                                         \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail(e_, #call);        \
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

template <class T>
std::vector<T> convert(const std::vector<double>& v) {
  if constexpr (std::is_same<T, double>::value) {
    return v;
  } else {
    std::vector<T> o(v.size());
    for (size_t k = 0; k < v.size(); ++k) o[k] = (T)v[k];
    return o;
  }
}

template <class T>
struct DevTables {
  bool ready = false;
  DevBuf q_to, q_ti, q_li, q_Y, q_off, q_gam, q_eta, t_to, t_ti, t_li, t_Y, t_off, t_gam, t_eta,
      fnb, fgeo;
  uw::MeshDev<T> view;
  void reset() {
    for (DevBuf* b : {&q_to, &q_ti, &q_li, &q_Y, &q_off, &q_gam, &q_eta, &t_to, &t_ti, &t_li,
                      &t_Y, &t_off, &t_gam, &t_eta, &fnb, &fgeo})
      b->release();
    view = uw::MeshDev<T>();
    ready = false;
  }
};

}  // namespace

struct uw_mesh {
  int device = 0;
  uw::HostMesh host;
  uw::HostTables tables;
  uw::SchemeParams scheme;
  bool precomputed = false;
  DevTables<double> d64;
  DevTables<float> d32;
  DevBuf FS, Wtmp, dt, partial, flag;
  int block_recon = 256, block_flux = 256;
  // optional timing of every launch with HIP events on the caller's stream
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;  // kind, (start, stop)
  ~uw_mesh() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& u : ev_used) {
      (void)hipEventDestroy(u.second.first);
      (void)hipEventDestroy(u.second.second);
    }
  }
};

struct uw_batch {
  std::vector<uw_mesh*> meshes;
  uw_physics physics;
  std::vector<int64_t> offsets;
};

namespace {

template <class T>
DevTables<T>& tables_of(uw_mesh* m);
template <>
DevTables<double>& tables_of<double>(uw_mesh* m) {
  return m->d64;
}
template <>
DevTables<float>& tables_of<float>(uw_mesh* m) {
  return m->d32;
}

template <class T>
uw_status ensure_tables(uw_mesh* m) {
  DevTables<T>& d = tables_of<T>(m);
  if (d.ready) return UW_OK;
  UW_HIP(hipSetDevice(m->device));
  const uw::HostTables& t = m->tables;
  auto up_type = [&](const uw::TypeTables& tt, DevBuf& to, DevBuf& ti, DevBuf& li, DevBuf& Y,
                     DevBuf& off, DevBuf& gam, DevBuf& eta, uw::TypeDev<T>& view) -> hipError_t {
    hipError_t e;
    if ((e = to.upload(tt.tile_off)) != hipSuccess) return e;
    if ((e = ti.upload(tt.tile_ids)) != hipSuccess) return e;
    if ((e = li.upload(tt.lidx)) != hipSuccess) return e;
    if ((e = Y.upload(convert<T>(tt.Y))) != hipSuccess) return e;
    if ((e = off.upload(convert<T>(tt.off))) != hipSuccess) return e;
    if ((e = gam.upload(convert<T>(tt.gam))) != hipSuccess) return e;
    if ((e = eta.upload(convert<T>(tt.eta))) != hipSuccess) return e;
    view.Nt = tt.Nt;
    view.first = tt.first;
    view.tile_off = to.template as<int32_t>();
    view.tile_ids = ti.template as<int32_t>();
    view.lidx = li.template as<uint16_t>();
    view.max_tile_len = tt.max_tile_len;
    view.Y = Y.template as<T>();
    view.off = off.template as<T>();
    view.gam = gam.template as<T>();
    view.eta = eta.template as<T>();
    return hipSuccess;
  };
  hipError_t e =
      up_type(t.quad, d.q_to, d.q_ti, d.q_li, d.q_Y, d.q_off, d.q_gam, d.q_eta, d.view.quad);
  if (e == hipSuccess)
    e = up_type(t.tri, d.t_to, d.t_ti, d.t_li, d.t_Y, d.t_off, d.t_gam, d.t_eta, d.view.tri);
  if (e == hipSuccess) e = d.fnb.upload(t.fnb);
  if (e == hipSuccess) e = d.fgeo.upload(convert<T>(t.fgeo));
  if (e == hipErrorOutOfMemory) return fail(UW_ENOMEM, "device tables: out of memory");
  if (e != hipSuccess) return hip_fail(e, "device tables upload");
  d.view.N = m->host.N;
  d.view.Nq = m->host.Nq;
  d.view.fnb = d.fnb.template as<int32_t>();
  d.view.fgeo = d.fgeo.template as<T>();
  d.ready = true;
  return UW_OK;
}

uw_status ensure_work(uw_mesh* m, int nvar, size_t fs_elem) {
  const int64_t N = m->host.N;
  UW_HIP(m->FS.ensure((size_t)N * 8 * nvar * fs_elem));
  UW_HIP(m->Wtmp.ensure((size_t)N * nvar * sizeof(double)));
  UW_HIP(m->dt.ensure(sizeof(double)));
  UW_HIP(m->partial.ensure((size_t)uw::cfl_partials(N) * sizeof(double)));
  if (!m->flag.p) {
    UW_HIP(m->flag.ensure(sizeof(int)));
    UW_HIP(hipMemset(m->flag.p, 0, sizeof(int)));
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

uw::PhysDev phys_dev(const uw_physics* p) {
  return uw::PhysDev{p->equation, p->ax, p->ay, p->gamma};
}

uw::SchemeDev scheme_dev(const uw_mesh* m) {
  return uw::SchemeDev{m->scheme.eps, m->scheme.theta, m->scheme.mode};
}

hipError_t ev_begin(uw_mesh* m, hipStream_t st, hipEvent_t* a, hipEvent_t* b) {
  for (hipEvent_t* e : {a, b}) {
    if (!m->ev_pool.empty()) {
      *e = m->ev_pool.back();
      m->ev_pool.pop_back();
    } else {
      hipError_t r = hipEventCreate(e);
      if (r != hipSuccess) return r;
    }
  }
  return hipEventRecord(*a, st);
}

// One residual evaluation or RK stage on the given state.
template <class T>
uw_status stage(uw_mesh* m, const uw_physics* p, int mode, const double* W_in, const double* Wn,
                double* W_out, double* t, hipStream_t st) {
  const int nvar = p->equation == UW_EULER ? 4 : 1;
  DevTables<T>& d = tables_of<T>(m);
  T* FS = m->FS.template as<T>();
  hipEvent_t a = nullptr, b = nullptr;
  if (m->profiling) UW_HIP(ev_begin(m, st, &a, &b));
  hipError_t e = uw::launch_recon<T>(d.view, scheme_dev(m), nvar, W_in, FS, st);
  if (e != hipSuccess) return hip_fail(e, "reconstruction launch");
  if (m->profiling) {
    UW_HIP(hipEventRecord(b, st));
    m->ev_used.push_back({0, {a, b}});
    UW_HIP(ev_begin(m, st, &a, &b));
  }
  e = uw::launch_flux<T>(d.view, phys_dev(p), nvar, mode, FS, W_in, Wn, W_out,
                         m->dt.as<double>(), t, m->flag.as<int>(), m->block_flux, st);
  if (e != hipSuccess) return hip_fail(e, "flux launch");
  if (m->profiling) {
    UW_HIP(hipEventRecord(b, st));
    m->ev_used.push_back({1, {a, b}});
  }
  return UW_OK;
}

template <class T>
uw_status prepare(uw_mesh* m, const uw_physics* p) {
  uw_status s = ensure_tables<T>(m);
  if (s != UW_OK) return s;
  return ensure_work(m, p->equation == UW_EULER ? 4 : 1, sizeof(T));
}

template <class T>
uw_status rk3(uw_mesh* m, const uw_physics* p, double* W, double cfl, double dt_fixed,
              double t_end, double* t_dev, hipStream_t st) {
  uw_status s = prepare<T>(m, p);
  if (s != UW_OK) return s;
  const int nvar = p->equation == UW_EULER ? 4 : 1;
  DevTables<T>& d = tables_of<T>(m);
  hipError_t e = uw::launch_cfl<T>(d.view, phys_dev(p), nvar, W, cfl, dt_fixed, t_end, t_dev,
                                   m->partial.as<double>(), m->dt.as<double>(), st);
  if (e != hipSuccess) return hip_fail(e, "time-step launch");
  double* W1 = m->Wtmp.as<double>();
  if ((s = stage<T>(m, p, 1, W, W, W1, nullptr, st)) != UW_OK) return s;
  if ((s = stage<T>(m, p, 2, W1, W, W1, nullptr, st)) != UW_OK) return s;
  return stage<T>(m, p, 3, W1, W, W, t_dev, st);
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
  uw_mesh* m = new (std::nothrow) uw_mesh();
  if (!m) return fail(UW_ENOMEM, "host allocation");
  m->device = device;
  uw::Error err;
  try {
    if (!uw::build_mesh(desc->n_nodes, desc->node_xy, desc->n_cells, desc->cell_nodes,
                        desc->node_id, desc->bc, m->host, err)) {
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
  if (!m || !sc) return fail(UW_EINVAL, "mesh and scheme must not be NULL");
  if (!(sc->zeta >= 0.0) || !(sc->eps > 0.0) || !(sc->theta >= 1.0))
    return fail(UW_EINVAL, "scheme needs zeta >= 0, eps > 0, theta >= 1");
  if (sc->mode != UW_WENO && sc->mode != UW_LINEAR) return fail(UW_EINVAL, "scheme.mode");
  if (sc->d_scope != UW_D_PER_GP && sc->d_scope != UW_D_PER_CELL)
    return fail(UW_EINVAL, "scheme.d_scope");
  m->scheme.zeta = sc->zeta;
  m->scheme.theta = sc->theta;
  m->scheme.eps = sc->eps;
  m->scheme.optimize = sc->optimize;
  m->scheme.d_scope = sc->d_scope;
  m->scheme.mode = sc->mode;
  m->d64.reset();
  m->d32.reset();
  try {
    m->tables = uw::HostTables();
    uw::precompute_tables(m->host, m->scheme, m->tables, uw::default_threads());
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

uw_status uw_residual(uw_mesh* m, const uw_physics* p, const double* W, double* L, void* stream) {
  g_err.clear();
  if (!m || !W || !L) return fail(UW_EINVAL, "mesh, W and L must not be NULL");
  uw_status s = check_physics(p);
  if (s != UW_OK) return s;
  if (!m->precomputed) return fail(UW_ESTATE, "uw_residual before uw_precompute_geometry");
  if (m->device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
  hipStream_t st = (hipStream_t)stream;
  UW_HIP(hipSetDevice(m->device));
  if (p->precision == UW_FP64) {
    if ((s = prepare<double>(m, p)) != UW_OK) return s;
    return stage<double>(m, p, 0, W, W, L, nullptr, st);
  }
  if ((s = prepare<float>(m, p)) != UW_OK) return s;
  return stage<float>(m, p, 0, W, W, L, nullptr, st);
}

uw_status uw_rk3_step(uw_mesh* m, const uw_physics* p, double* W, double cfl, double dt_fixed,
                      double t_end, double* t_dev, void* stream) {
  g_err.clear();
  if (!m || !W || !t_dev) return fail(UW_EINVAL, "mesh, W and t_dev must not be NULL");
  uw_status s = check_physics(p);
  if (s != UW_OK) return s;
  if (!m->precomputed) return fail(UW_ESTATE, "uw_rk3_step before uw_precompute_geometry");
  if (m->device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(UW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  hipStream_t st = (hipStream_t)stream;
  UW_HIP(hipSetDevice(m->device));
  if (p->precision == UW_FP64) return rk3<double>(m, p, W, cfl, dt_fixed, t_end, t_dev, st);
  return rk3<float>(m, p, W, cfl, dt_fixed, t_end, t_dev, st);
}

uw_status uw_cfl_dt(uw_mesh* m, const uw_physics* p, const double* W, double cfl, double* dt_dev,
                    void* stream) {
  g_err.clear();
  if (!m || !W || !dt_dev) return fail(UW_EINVAL, "mesh, W and dt_dev must not be NULL");
  uw_status s = check_physics(p);
  if (s != UW_OK) return s;
  if (!m->precomputed) return fail(UW_ESTATE, "uw_cfl_dt before uw_precompute_geometry");
  if (m->device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
  if (!(cfl > 0.0)) return fail(UW_EINVAL, "cfl must be > 0");
  hipStream_t st = (hipStream_t)stream;
  UW_HIP(hipSetDevice(m->device));
  const int nvar = p->equation == UW_EULER ? 4 : 1;
  hipError_t e;
  if (p->precision == UW_FP64) {
    if ((s = prepare<double>(m, p)) != UW_OK) return s;
    e = uw::launch_cfl<double>(m->d64.view, phys_dev(p), nvar, W, cfl, 0.0, INFINITY, nullptr,
                               m->partial.as<double>(), dt_dev, st);
  } else {
    if ((s = prepare<float>(m, p)) != UW_OK) return s;
    e = uw::launch_cfl<float>(m->d32.view, phys_dev(p), nvar, W, cfl, 0.0, INFINITY, nullptr,
                              m->partial.as<double>(), dt_dev, st);
  }
  if (e != hipSuccess) return hip_fail(e, "time-step launch");
  return UW_OK;
}

uw_status uw_check(uw_mesh* m, uw_batch* b, void* stream) {
  g_err.clear();
  hipStream_t st = (hipStream_t)stream;
  UW_HIP(hipStreamSynchronize(st));
  std::vector<uw_mesh*> ms;
  if (m) ms.push_back(m);
  if (b) ms.insert(ms.end(), b->meshes.begin(), b->meshes.end());
  bool bad = false;
  for (uw_mesh* x : ms) {
    if (!x->flag.p) continue;
    int h = 0;
    UW_HIP(hipMemcpy(&h, x->flag.p, sizeof(int), hipMemcpyDeviceToHost));
    if (h) {
      bad = true;
      UW_HIP(hipMemset(x->flag.p, 0, sizeof(int)));
    }
  }
  if (bad) return fail(UW_ENONFINITE, "non-finite value or non-positive density in a step");
  return UW_OK;
}

uw_status uw_batch_create(uw_mesh* const* meshes, int32_t n, const uw_physics* p, uw_batch** out) {
  g_err.clear();
  if (!meshes || !out || n < 1) return fail(UW_EINVAL, "need meshes, out and n >= 1");
  *out = nullptr;
  uw_status s = check_physics(p);
  if (s != UW_OK) return s;
  uw_batch* b = new (std::nothrow) uw_batch();
  if (!b) return fail(UW_ENOMEM, "host allocation");
  b->physics = *p;
  b->offsets.push_back(0);
  for (int32_t k = 0; k < n; ++k) {
    uw_mesh* m = meshes[k];
    if (!m || !m->precomputed) {
      delete b;
      return fail(UW_ESTATE, "every batch mesh must be precomputed");
    }
    if (m->device != meshes[0]->device) {
      delete b;
      return fail(UW_EINVAL, "batch meshes must live on one device");
    }
    b->meshes.push_back(m);
    b->offsets.push_back(b->offsets.back() + m->host.N);
  }
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
  const int nvar = b->physics.equation == UW_EULER ? 4 : 1;
  for (int32_t step = 0; step < n_steps; ++step)
    for (size_t k = 0; k < b->meshes.size(); ++k) {
      uw_status s = uw_rk3_step(b->meshes[k], &b->physics, W + nvar * b->offsets[k], cfl, dt_fixed,
                                t_end, t_dev + k, stream);
      if (s != UW_OK) return s;
    }
  return UW_OK;
}

uw_status uw_autotune(uw_mesh* m, uw_batch* b, const uw_physics* p, const char* cache_path,
                      void* stream) {
  g_err.clear();
  if (!m && !b) return fail(UW_EINVAL, "need a mesh or a batch");
  uw_status s = check_physics(p);
  if (s != UW_OK) return s;
  std::vector<uw_mesh*> ms;
  if (m) ms.push_back(m);
  if (b) ms.insert(ms.end(), b->meshes.begin(), b->meshes.end());
  hipStream_t st = (hipStream_t)stream;
  const int nvar = p->equation == UW_EULER ? 4 : 1;
  for (uw_mesh* x : ms) {
    if (!x->precomputed) return fail(UW_ESTATE, "autotune before precompute");
    if (x->device < 0) return fail(UW_ESTATE, "mesh was uploaded host-only (device -1)");
    char key[160];
    std::snprintf(key, sizeof(key), "%lld %lld %d %d %d", (long long)x->host.N,
                  (long long)x->host.Nq, nvar, p->precision, x->scheme.mode);
    bool found = false;
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "r")) {
        char line[256];
        while (std::fgets(line, sizeof(line), f)) {
          long long a, bq;
          int c, d, e, br, bf;
          if (std::sscanf(line, "%lld %lld %d %d %d %d %d", &a, &bq, &c, &d, &e, &br, &bf) == 7) {
            char k2[160];
            std::snprintf(k2, sizeof(k2), "%lld %lld %d %d %d", a, bq, c, d, e);
            if (std::strcmp(k2, key) == 0 && br > 0 && br <= 256 && bf > 0 && bf <= 256) {
              x->block_recon = br;
              x->block_flux = bf;
              found = true;
            }
          }
        }
        std::fclose(f);
      }
    }
    if (found) continue;
    UW_HIP(hipSetDevice(x->device));
    s = p->precision == UW_FP64 ? prepare<double>(x, p) : prepare<float>(x, p);
    if (s != UW_OK) return s;
    // a uniform admissible state to time the kernels on
    std::vector<double> h((size_t)nvar * x->host.N);
    for (int64_t i = 0; i < x->host.N; ++i) {
      if (nvar == 4) {
        h[i] = 1.0;
        h[x->host.N + i] = 0.5;
        h[2 * x->host.N + i] = 0.25;
        h[3 * x->host.N + i] = 2.5;
      } else {
        h[i] = 1.0;
      }
    }
    DevBuf Wt, Lt;
    UW_HIP(Wt.upload(h));
    UW_HIP(Lt.ensure(h.size() * sizeof(double)));
    hipEvent_t e0, e1;
    UW_HIP(hipEventCreate(&e0));
    UW_HIP(hipEventCreate(&e1));
    const int cands[3] = {64, 128, 256};
    for (int which = 1; which < 2; ++which) {
      int* knob = &x->block_flux;
      int best_c = *knob;
      float best = 1e30f;
      for (int c : cands) {
        *knob = c;
        float tot = 0.0f;
        for (int rep = 0; rep < 4; ++rep) {
          UW_HIP(hipEventRecord(e0, st));
          s = p->precision == UW_FP64
                  ? stage<double>(x, p, 0, Wt.as<double>(), Wt.as<double>(), Lt.as<double>(), nullptr, st)
                  : stage<float>(x, p, 0, Wt.as<double>(), Wt.as<double>(), Lt.as<double>(), nullptr, st);
          if (s != UW_OK) return s;
          UW_HIP(hipEventRecord(e1, st));
          UW_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          UW_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) tot += ms;
        }
        if (tot < best) {
          best = tot;
          best_c = c;
        }
      }
      *knob = best_c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %d %d\n", key, x->block_recon, x->block_flux);
        std::fclose(f);
      }
    }
  }
  return UW_OK;
}

uw_status uw_profile(uw_mesh* m, int32_t enable, double* ms, int64_t* count) {
  g_err.clear();
  if (!m) return fail(UW_EINVAL, "mesh is NULL");
  if (ms || count) {
    for (int k = 0; k < 2; ++k) {
      if (ms) ms[k] = 0.0;
      if (count) count[k] = 0;
    }
    for (auto& u : m->ev_used) {
      UW_HIP(hipEventSynchronize(u.second.second));
      float t = 0.0f;
      UW_HIP(hipEventElapsedTime(&t, u.second.first, u.second.second));
      if (ms) ms[u.first] += t;
      if (count) count[u.first] += 1;
    }
  }
  for (auto& u : m->ev_used) {
    m->ev_pool.push_back(u.second.first);
    m->ev_pool.push_back(u.second.second);
  }
  m->ev_used.clear();
  if (enable >= 0) m->profiling = enable != 0;
  return UW_OK;
}

void uw_mesh_destroy(uw_mesh* m) { delete m; }

void uw_batch_destroy(uw_batch* b) { delete b; }

}  // extern "C"
