// FP64 precompute on the GPU: one thread per cell runs the same per-cell
// routine as the host driver (cellgeom.h); results are copied back into the
// host tables, which then receive their tile lists and face tables.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cellgeom.h"
#include "uw_host.h"

namespace uw {

geom::TypeC type_c(const TypeConst& T);

namespace {

__global__ __launch_bounds__(64) void k_precompute(geom::CellIn in, geom::TypeC tq, geom::TypeC tt,
                                                   geom::Params p, geom::CellOut out, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) geom::precompute_cell(in, tq, tt, p, i, out);
}

struct Buf {
  void* p = nullptr;
  size_t n = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

bool precompute_tables_device(const HostMesh& m, const SchemeParams& sp, HostTables& t, int device,
                              int threads, std::string& err, int& hip_code) {
  const int64_t N = m.N;
  alloc_tables(m, sp, t);
  std::vector<double> normal(8 * N), length(4 * N), diag(4 * N);
  std::vector<int32_t> counts(2 * N);
  std::vector<Buf> bufs(40);
  int nb = 0;
  hipError_t e = hipSetDevice(device);
  auto dev = [&](const auto& v) -> void* {
    if (e != hipSuccess || v.empty()) return nullptr;
    Buf& b = bufs[nb++];
    b.n = v.size() * sizeof(v[0]);
    e = hipMalloc(&b.p, b.n);
    if (e == hipSuccess) e = hipMemcpy(b.p, v.data(), b.n, hipMemcpyHostToDevice);
    return b.p;
  };
  geom::CellIn in;
  in.nf = (const int32_t*)dev(m.nf);
  in.cell_nodes = (const int32_t*)dev(m.cell_nodes);
  in.xy = (const double*)dev(m.xy);
  in.st_cell = (const int32_t*)dev(m.st_cell);
  in.st_shift = (const double*)dev(m.st_shift);
  in.st_ghost = (const int8_t*)dev(m.st_ghost);
  in.st_res = (const int8_t*)dev(m.st_res);
  in.st_present = (const uint8_t*)dev(m.st_present);
  in.Nq = m.Nq;
  // outputs: device copies of the host arrays (uploaded zeros)
  struct Pair {
    void* dev;
    void* host;
    size_t bytes;
  };
  std::vector<Pair> back;
  auto out_of = [&](auto& v) -> decltype(v.data()) {
    void* d = dev(v);
    if (d) back.push_back(Pair{d, v.data(), v.size() * sizeof(v[0])});
    return (decltype(v.data()))d;
  };
  geom::CellOut out;
  auto type_out = [&](TypeTables& tt) {
    geom::TypeOut o;
    o.Y = out_of(tt.Y);
    o.off = out_of(tt.off);
    o.gam = out_of(tt.gam);
    o.sig = out_of(tt.sig);
    o.eta = out_of(tt.eta);
    o.sid = out_of(tt.sid);
    o.n = tt.Nt;
    return o;
  };
  out.quad = type_out(t.quad);
  out.tri = type_out(t.tri);
  out.area = out_of(t.area);
  out.normal = out_of(normal);
  out.length = out_of(length);
  out.diag = out_of(diag);
  out.counts = out_of(counts);
  out.dbg_gamma = t.debug ? out_of(t.dbg_gamma) : nullptr;
  out.dbg_gamma_raw = t.debug ? out_of(t.dbg_gamma_raw) : nullptr;
  out.dbg_eta = t.debug ? out_of(t.dbg_eta) : nullptr;
  out.dbg_Y = t.debug ? out_of(t.dbg_Y) : nullptr;
  out.dbg_off = t.debug ? out_of(t.dbg_off) : nullptr;
  if (e == hipSuccess && N > 0) {
    const geom::TypeC tq = type_c(kQuad), tt = type_c(kTri);
    const geom::Params gp{sp.zeta, sp.theta, sp.optimize, sp.d_scope, sp.mode == 1};
    k_precompute<<<(unsigned)((N + 63) / 64), 64>>>(in, tq, tt, gp, out, N);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  for (const Pair& pr : back)
    if (e == hipSuccess) e = hipMemcpy(pr.host, pr.dev, pr.bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    hip_code = (int)e;
    err = std::string("device precompute: ") + hipGetErrorString(e);
    return false;
  }
  bufs.clear();
  reduce_diag(diag, counts, t);
  finish_tables(m, t, normal, length, threads);
  return true;
}

}  // namespace uw
