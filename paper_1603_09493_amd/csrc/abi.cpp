// C ABI of the batched FE-LLG island solver: context, mesh groups, instances, runs, results.
// The declarations and their contracts are in include/bpm_llg.h.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <tuple>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <type_traits>
#include <string>
#include <vector>

#include "bpm_internal.h"
#include "field_eval.h"
#include "mlp_internal.h"
#include "heun_internal.h"

namespace bpm {

std::string hip_err_string(hipError_t e) { return hipGetErrorString(e); }

void to_float_device(size_t cnt, const double* a, float* b, hipStream_t stream);
void pack_tiles_device(int n, int ldS, const double* S, float* T, hipStream_t stream);
hipError_t absmax_device(size_t cnt, const double* a, float* out, hipStream_t stream);
void pack_tiles16_device(int n, int ldS, const double* S, double scale, uint16_t* T, hipStream_t stream);
hipError_t extract_m_device(int precision, long n, long rstride, long offset, const void* src, double* dst,
                            hipStream_t stream);
void symmetrize_device(int n, int ldS, double* S, hipStream_t stream);
hipError_t gp_ei_device(const GpArgs& a, long m, double* cand, uint64_t seed, double* yhat, double* sd, double* ei,
                        hipStream_t stream);
int argmax_blocks(long m);
hipError_t argmax_device(const double* v, long m, double* bv, long* bi, int64_t* out, hipStream_t stream);
hipError_t string_reparam_device(int precision, long n, int P, const StringImages& im, double* d_dist,
                                 double* d_out, hipStream_t stream);

template <typename real>
size_t dp5_lds_bytes(const LdsPlan&);
template <typename real>
hipError_t launch_dp5(const GroupView<real>*, const RunParams&, int, int, const LdsPlan&, bool, bool, hipStream_t, int);
template <typename real>
hipError_t max_coresident(const LdsPlan&, bool, int, bool, int*, int*);
template <typename real>
hipError_t launch_energy(const GroupView<real>*, const int2*, int, const RunParams&, double*, int, hipStream_t);

// device copies of the assembled quantities, in one precision
template <typename real>
struct DevGeom {
  int32_t *rowptr = nullptr, *col = nullptr, *colx = nullptr, *layer = nullptr, *partner = nullptr;
  real *K = nullptr, *D = nullptr, *DT = nullptr, *V = nullptr, *aif = nullptr;
  double *x = nullptr, *y = nullptr, *z = nullptr;
};

struct DeviceMesh {
  DevGeom<double> g64;
  DevGeom<float> g32;
};

// one device allocation list, freed together
struct Arena {
  std::vector<void*> ptrs;
  ~Arena() { clear(); }
  void clear() {
    for (void* p : ptrs) hipFree(p);
    ptrs.clear();
  }
  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

}  // namespace bpm

using namespace bpm;

struct bpm_ctx {
  int device = 0;
  std::string err;
  hipStream_t own_stream = nullptr;
  std::vector<std::unique_ptr<MeshGroup>> meshes;
  std::vector<std::unique_ptr<DeviceMesh>> dmeshes;
  std::vector<std::unique_ptr<Arena>> mesh_arena;
  std::vector<Instance> insts;
  // last run
  Arena run;
  hipStream_t run_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool run_pending = false, have_results = false;
  int run_precision = 64, run_traj_cap = 0, run_grid = 0, run_G = 0;
  int run_ninst = 0, run_nsys = 0;
  bool run_rfast = false;                  // state layout [3][N][R] (Heun path)
  int run_csr_cap = 0;                     // CSR entries staged in LDS per workgroup (0 = none)
  LdsPlan run_plan{};                      // LDS plan of the last stepping launch
  int run_bs = 0, run_RB = 0;
  std::vector<int32_t> slot_R;             // run slot -> R of its group (Heun path)
  hipGraphExec_t graph_exec = nullptr;
  std::vector<int32_t> inst_order;         // run slot -> instance id
  std::vector<int32_t> slot_of;            // instance id -> run slot
  std::vector<int32_t> slot_group;         // run slot -> mesh id
  std::vector<int32_t> slot_local;         // run slot -> local index in its group
  std::vector<int32_t> group_inst0;        // mesh id -> first slot (or -1)
  std::vector<int32_t> sys_of_slot;
  SysOut* d_sys_out = nullptr;
  InstOut* d_inst_out = nullptr;
  double* d_traj = nullptr;
  double* d_energy = nullptr;
  void* d_state_m[2] = {nullptr, nullptr};  // unused placeholder
  std::vector<void*> group_m;               // per mesh id: device m of the run (precision-typed)
  std::vector<SysOut> h_sys_out;
  std::vector<InstOut> h_inst_out;
  std::vector<double> h_energy;
  float kernel_ms = 0.f;
  double* heun_obs = nullptr;
  long long heun_nsteps = 0;
  double heun_dt = 0.0, heun_t_end = 0.0;
  // launch of the last stepping run, kept so that a run with BPM_FLAG_CONTINUE can resume it
  bool run_resumable = false;
  int64_t inst_version = 0, run_version = -1;   // bumped by every change of the instance set
  int run_integrator = -1, run_flags = 0;
  bool run_fixed = false, run_coop = false;
  double run_t_end = 0.0, run_dt_fixed = 0.0;
  RunParams run_P{};
  void* run_d_groups = nullptr;
  int2* run_d_imap = nullptr;
  int run_nmax = 0, run_ng = 0;
  double *run_d_err = nullptr, *run_d_obs = nullptr, *run_d_mom = nullptr;
  unsigned long long* run_d_bar = nullptr;
  int2* run_d_map = nullptr;                 // blockIdx -> (group, local workgroup)
  std::vector<int> run_group_G, run_group_n, run_group_sys0, run_group_nsys;
  std::vector<int64_t> run_att_start;       // attempts of each system when the last launch began
  std::vector<int2> run_wmap;               // host copy of a reordered map (kept until the copy ran)
  // field grids of BPM_FIELD_GRID instances, one device copy per distinct content
  struct FieldGrid {
    float* dev = nullptr;
    std::shared_ptr<const std::vector<float>> host;
    int32_t n[3] = {0, 0, 0};
  };
  std::map<uint64_t, FieldGrid> grids;
  // autotuned workgroups per mesh group, keyed by (log2 bucket of N, instances, precision)
  std::map<std::tuple<int, int, int>, int> tune;
  std::string tune_path;
};

static std::tuple<int, int, int> tune_key(int nmax, int rtot, int precision) {
  int b = 0;
  while ((1 << b) < nmax) ++b;
  return std::make_tuple(b, rtot, precision);
}

static int fail(bpm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                            \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) return fail(ctx, BPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

extern "C" {

int bpm_create(bpm_ctx** out, int device, const char* tune_cache) {
  if (!out) return BPM_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BPM_EHIP;
  if (hipSetDevice(device) != hipSuccess) return BPM_EHIP;
  bpm_ctx* c = new bpm_ctx();
  c->device = device;
  if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return BPM_EHIP;
  }
  // device address of this GPU's scratch area of the allocation-free top-k (a failure here is
  // retried, and reported, by bpm_topk_noalloc)
  (void)topk_scratch_init(device);
  const char* cache = tune_cache ? tune_cache : std::getenv("BPM_TUNE_CACHE");
  if (cache && *cache) {
    const char* p = cache;
    c->tune_path = p;
    std::ifstream f(p);
    int b, r, pr, g;
    while (f >> b >> r >> pr >> g) c->tune[std::make_tuple(b, r, pr)] = g;
  }
  *out = c;
  return BPM_OK;
}

void bpm_destroy(bpm_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->run_pending && c->run_stream) hipStreamSynchronize(c->run_stream);
  c->run.clear();
  for (auto& m : c->meshes) {
    if (m->dS64) hipFree(m->dS64);
    if (m->dS32) hipFree(m->dS32);
    if (m->dS32t) hipFree(m->dS32t);
    if (m->dS16t) hipFree(m->dS16t);
  }
  c->mesh_arena.clear();
  for (auto& kv : c->grids) hipFree(kv.second.dev);
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  delete c;
}

const char* bpm_last_error(const bpm_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

template <typename real>
static int upload_geom(bpm_ctx* c, const MeshGroup& g, DevGeom<real>& d, Arena& A) {
  // the CSR arrays carry kCsrPad zero entries past the last row (column 0, coefficient 0), so
  // that a row's entries can be read in fixed-size batches without a clamp
  const size_t nz = (size_t)g.nnz + kCsrPad;
  std::vector<real> K(g.K.begin(), g.K.end()), D(g.D.begin(), g.D.end()), DT(g.DT.begin(), g.DT.end());
  K.resize(nz, (real)0);
  D.resize(3 * nz, (real)0);
  DT.resize(3 * nz, (real)0);
  std::vector<int32_t> col(g.col.begin(), g.col.end());
  col.resize(nz, 0);
  std::vector<real> V(g.V.begin(), g.V.end()), aif(g.aif.begin(), g.aif.end());
  HIPCHK(c, A.alloc(&d.rowptr, g.n + 1));
  HIPCHK(c, A.alloc(&d.col, nz));
  HIPCHK(c, A.alloc(&d.colx, nz));
  HIPCHK(c, A.alloc(&d.layer, g.n));
  HIPCHK(c, A.alloc(&d.partner, g.n));
  HIPCHK(c, A.alloc(&d.K, nz));
  HIPCHK(c, A.alloc(&d.D, 3 * nz));
  HIPCHK(c, A.alloc(&d.DT, 3 * nz));
  HIPCHK(c, A.alloc(&d.V, g.n));
  HIPCHK(c, A.alloc(&d.aif, g.n));
  HIPCHK(c, A.alloc(&d.x, g.n));
  HIPCHK(c, A.alloc(&d.y, g.n));
  HIPCHK(c, A.alloc(&d.z, g.n));
  HIPCHK(c, hipMemcpy(d.rowptr, g.rowptr.data(), sizeof(int32_t) * (g.n + 1), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.col, col.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
  {
    std::vector<int32_t> colx(nz, 0);
    for (int q = 0; q < g.nnz; ++q) colx[q] = g.col[q] | (g.layer[g.col[q]] << 16);
    HIPCHK(c, hipMemcpy(d.colx, colx.data(), sizeof(int32_t) * nz, hipMemcpyHostToDevice));
  }
  HIPCHK(c, hipMemcpy(d.layer, g.layer.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.partner, g.partner.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.K, K.data(), sizeof(real) * nz, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.D, D.data(), sizeof(real) * 3 * nz, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.DT, DT.data(), sizeof(real) * 3 * nz, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.V, V.data(), sizeof(real) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.aif, aif.data(), sizeof(real) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.x, g.x.data(), sizeof(double) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.y, g.y.data(), sizeof(double) * g.n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.z, g.z.data(), sizeof(double) * g.n, hipMemcpyHostToDevice));
  return BPM_OK;
}

extern "C" {

int bpm_mesh_add(bpm_ctx* c, const bpm_mesh* mesh, const double* S_host, double demag_beta, int32_t* mesh_id) {
  return bpm_mesh_add_ex(c, mesh, S_host, demag_beta, BPM_KEEP_S64 | BPM_KEEP_S32, mesh_id);
}

int bpm_mesh_add_ex(bpm_ctx* c, const bpm_mesh* mesh, const double* S_host, double demag_beta, int32_t flags,
                    int32_t* mesh_id) {
  if (c && !(flags & (BPM_KEEP_S64 | BPM_KEEP_S32 | BPM_KEEP_S32_TILES | BPM_KEEP_S16_TILES)))
    return fail(c, BPM_EINVAL, "bpm_mesh_add_ex: keep at least one copy of S");
  if (!c) return BPM_EINVAL;
  if (!mesh || !mesh_id || !mesh->xyz || !mesh->tet || !mesh->node_layer)
    return fail(c, BPM_EINVAL, "bpm_mesh_add: null argument");
  if (mesh->n_nodes <= 0 || mesh->n_tets <= 0 || mesh->n_iface < 0 || (mesh->n_iface > 0 && !mesh->iface))
    return fail(c, BPM_EINVAL, "bpm_mesh_add: empty mesh or bad sizes");
  if (mesh->n_nodes > 65535) return fail(c, BPM_EINVAL, "bpm_mesh_add: more than 65535 nodes per island");
  hipSetDevice(c->device);
  auto g = std::make_unique<MeshGroup>();
  const int n = mesh->n_nodes;
  g->n = n;
  g->ntet = mesh->n_tets;
  g->nif = mesh->n_iface;
  g->x.assign(mesh->xyz, mesh->xyz + n);
  g->y.assign(mesh->xyz + n, mesh->xyz + 2 * n);
  g->z.assign(mesh->xyz + 2 * n, mesh->xyz + 3 * n);
  g->tet.assign(mesh->tet, mesh->tet + 4 * (size_t)mesh->n_tets);
  for (int32_t v : g->tet)
    if (v < 0 || v >= n) return fail(c, BPM_EINVAL, "bpm_mesh_add: tet index out of range");
  g->layer.assign(mesh->node_layer, mesh->node_layer + n);
  for (int32_t v : g->layer)
    if (v != 0 && v != 1) return fail(c, BPM_EINVAL, "bpm_mesh_add: node_layer must be 0 or 1");
  if (g->nif) g->iface.assign(mesh->iface, mesh->iface + 2 * (size_t)g->nif);
  std::string err;
  int rc = assemble_mesh(*g, err);
  if (rc) return fail(c, rc, "bpm_mesh_add: " + err);
  auto dm = std::make_unique<DeviceMesh>();
  auto arena = std::make_unique<Arena>();
  if ((rc = upload_geom<double>(c, *g, dm->g64, *arena))) return rc;
  if ((rc = upload_geom<float>(c, *g, dm->g32, *arena))) return rc;
  const int ldS = (n + 15) / 16 * 16;
  if (S_host) {
    HIPCHK(c, hipMalloc(&g->dS64, sizeof(double) * (size_t)n * ldS));
    HIPCHK(c, hipMemset(g->dS64, 0, sizeof(double) * (size_t)n * ldS));
    HIPCHK(c, hipMemcpy2D(g->dS64, sizeof(double) * ldS, S_host, sizeof(double) * n, sizeof(double) * n, n,
                          hipMemcpyHostToDevice));
  } else {
    double beta = demag_beta > 0.0 ? demag_beta : 5.0 / (6.0 * std::sqrt(kPi)) * std::cbrt(3.0 / (4.0 * kPi));
    rc = demag_assemble_device(*g, beta, c->own_stream, err);
    if (rc) return fail(c, rc, "bpm_mesh_add: " + err);
  }
  symmetrize_device(n, ldS, g->dS64, c->own_stream);
  HIPCHK(c, hipGetLastError());
  if (flags & BPM_KEEP_S32) {
    HIPCHK(c, hipMalloc(&g->dS32, sizeof(float) * (size_t)n * ldS));
    to_float_device((size_t)n * ldS, g->dS64, g->dS32, c->own_stream);
  }
  if (flags & BPM_KEEP_S32_TILES) {
    HIPCHK(c, hipMalloc(&g->dS32t, sizeof(float) * (size_t)tile_count(n) * kTile * kTile));
    pack_tiles_device(n, ldS, g->dS64, g->dS32t, c->own_stream);
  }
  if (flags & BPM_KEEP_S16_TILES) {
    // a power-of-two scale keeps the products exact and puts max |S| in [2^13, 2^14)
    float* d_max = nullptr;
    HIPCHK(c, hipMalloc(&d_max, sizeof(float)));
    hipError_t e = absmax_device((size_t)n * ldS, g->dS64, d_max, c->own_stream);
    float mx = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&mx, d_max, sizeof(float), hipMemcpyDeviceToHost, c->own_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->own_stream);
    hipFree(d_max);
    HIPCHK(c, e);
    if (!std::isfinite(mx)) return fail(c, BPM_EINVAL, "bpm_mesh_add: demag operator is not finite");
    g->s16_scale = mx > 0.f ? std::ldexp(1.0, 13 - std::ilogb((double)mx)) : 1.0;
    HIPCHK(c, hipMalloc(&g->dS16t, sizeof(uint16_t) * (size_t)tile_count(n) * kTile * kTile));
    pack_tiles16_device(n, ldS, g->dS64, g->s16_scale, g->dS16t, c->own_stream);
  }
  HIPCHK(c, hipStreamSynchronize(c->own_stream));
  if (!(flags & BPM_KEEP_S64)) {
    HIPCHK(c, hipFree(g->dS64));
    g->dS64 = nullptr;
  }
  g->S_ready = true;
  *mesh_id = (int32_t)c->meshes.size();
  c->meshes.push_back(std::move(g));
  c->dmeshes.push_back(std::move(dm));
  c->mesh_arena.push_back(std::move(arena));
  return BPM_OK;
}

int bpm_mesh_get_S(bpm_ctx* c, int32_t id, double* S_out) {
  if (!c || !S_out || id < 0 || id >= (int)c->meshes.size()) return fail(c, BPM_EINVAL, "bpm_mesh_get_S: bad argument");
  hipSetDevice(c->device);
  const MeshGroup& g = *c->meshes[id];
  const int ldS = (g.n + 15) / 16 * 16;
  if (g.dS64) {
    HIPCHK(c, hipMemcpy2D(S_out, sizeof(double) * g.n, g.dS64, sizeof(double) * ldS, sizeof(double) * g.n, g.n,
                          hipMemcpyDeviceToHost));
  } else if (!g.dS32 && !g.dS32t) {
    // only the packed FP16 tiles: unpack both triangles and undo the scale
    const int nb = (g.n + kTile - 1) / kTile;
    std::vector<_Float16> tmp((size_t)tile_count(g.n) * kTile * kTile);
    HIPCHK(c, hipMemcpy(tmp.data(), g.dS16t, sizeof(uint16_t) * tmp.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < g.n; ++k)
      for (int l = 0; l < g.n; ++l) {
        const int a = std::min(k, l), b = std::max(k, l);
        const size_t f = (size_t)tile_index(nb, a / kTile, b / kTile);
        S_out[(size_t)k * g.n + l] = (double)tmp[f * kTile * kTile + tile16_offset(a % kTile, b % kTile)] / g.s16_scale;
      }
  } else if (!g.dS32) {
    // only the packed FP32 tiles: unpack both triangles
    const int nb = (g.n + kTile - 1) / kTile;
    std::vector<float> tmp((size_t)tile_count(g.n) * kTile * kTile);
    HIPCHK(c, hipMemcpy(tmp.data(), g.dS32t, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < g.n; ++k)
      for (int l = 0; l < g.n; ++l) {
        const int a = std::min(k, l), b = std::max(k, l);
        const size_t f = (size_t)tile_index(nb, a / kTile, b / kTile);
        S_out[(size_t)k * g.n + l] = tmp[f * kTile * kTile + tile_offset(a % kTile, b % kTile)];
      }
  } else {
    std::vector<float> tmp((size_t)g.n * ldS);
    HIPCHK(c, hipMemcpy(tmp.data(), g.dS32, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < g.n; ++k)
      for (int l = 0; l < g.n; ++l) S_out[(size_t)k * g.n + l] = tmp[(size_t)k * ldS + l];
  }
  return BPM_OK;
}

int bpm_mesh_get_assembly(bpm_ctx* c, int32_t id, int32_t* nnz, double* V, int32_t* rowptr, int32_t* col,
                          double* K, double* D, double* aif) {
  if (!c || id < 0 || id >= (int)c->meshes.size()) return fail(c, BPM_EINVAL, "bpm_mesh_get_assembly: bad mesh id");
  const MeshGroup& g = *c->meshes[id];
  if (nnz) *nnz = g.nnz;
  if (V) std::copy(g.V.begin(), g.V.end(), V);
  if (rowptr) std::copy(g.rowptr.begin(), g.rowptr.end(), rowptr);
  if (col) std::copy(g.col.begin(), g.col.end(), col);
  if (K) std::copy(g.K.begin(), g.K.end(), K);
  if (D) std::copy(g.D.begin(), g.D.end(), D);
  if (aif) std::copy(g.aif.begin(), g.aif.end(), aif);
  return BPM_OK;
}

int bpm_instance_add(bpm_ctx* c, int32_t mesh_id, const bpm_material* mat, const bpm_field* f,
                     const double* offset, const double* m0, uint64_t seed, int32_t* inst_id) {
  if (!c) return BPM_EINVAL;
  if (!mat || !f || !inst_id) return fail(c, BPM_EINVAL, "bpm_instance_add: null argument");
  if (mesh_id < 0 || mesh_id >= (int)c->meshes.size()) return fail(c, BPM_EINVAL, "bpm_instance_add: bad mesh id");
  if (f->kind != BPM_FIELD_UNIFORM && f->kind != BPM_FIELD_POLE && f->kind != BPM_FIELD_GRID)
    return fail(c, BPM_EINVAL, "bpm_instance_add: bad field kind");
  if (f->kind == BPM_FIELD_GRID &&
      (!f->grid || f->nx < 2 || f->ny < 2 || f->nz < 2 || !(f->g_h > 0.0) ||
       (double)f->nx * f->ny * f->nz * 3 > 1.0e9))
    return fail(c, BPM_EINVAL, "bpm_instance_add: a field grid needs data, nx, ny, nz >= 2 and g_h > 0");
  for (int L = 0; L < 2; ++L)
    if (!(mat->Ms[L] > 0.0)) return fail(c, BPM_EINVAL, "bpm_instance_add: Ms must be positive");
  if (!(mat->delta_int > 0.0) || !(mat->alpha >= 0.0)) return fail(c, BPM_EINVAL, "bpm_instance_add: delta_int > 0 and alpha >= 0 required");
  if (f->kind == BPM_FIELD_POLE && !(f->L_grad > 0.0)) return fail(c, BPM_EINVAL, "bpm_instance_add: L_grad must be positive");
  const MeshGroup& g = *c->meshes[mesh_id];
  Instance I;
  I.mesh = mesh_id;
  InstConst& k = I.c;
  for (int L = 0; L < 2; ++L) {
    k.Ms[L] = mat->Ms[L];
    k.cex[L] = 2.0 * mat->A[L] / mat->Ms[L];
    k.can[L] = 2.0 * mat->K[L] / mat->Ms[L];
    double nrm = std::sqrt(mat->axis[L][0] * mat->axis[L][0] + mat->axis[L][1] * mat->axis[L][1] + mat->axis[L][2] * mat->axis[L][2]);
    if (!(nrm > 0.0)) return fail(c, BPM_EINVAL, "bpm_instance_add: zero anisotropy axis");
    for (int d = 0; d < 3; ++d) k.axis[L][d] = mat->axis[L][d] / nrm;
    k.cint[L] = mat->A_int / mat->delta_int / mat->Ms[L];
    k.A[L] = mat->A[L];
    k.K[L] = mat->K[L];
  }
  k.Jint = mat->A_int / mat->delta_int;
  k.alpha = mat->alpha;
  k.gp = kGammaE / (1.0 + mat->alpha * mat->alpha);
  k.fkind = f->kind;
  k.B_peak = f->B_peak;
  k.t_rise = f->t_rise;
  k.L_grad = f->L_grad;
  k.W_pole = f->W_pole;
  for (int d = 0; d < 3; ++d) {
    k.dir[d] = f->dir[d];
    k.v[d] = f->v[d];
    k.x_off[d] = f->x_off[d];
    k.B_ext[d] = f->B_ext[d];
    k.off[d] = offset ? offset[d] : 0.0;
  }
  k.key[0] = (uint32_t)seed;
  k.key[1] = (uint32_t)(seed >> 32);
  k.grid = nullptr;
  if (f->kind == BPM_FIELD_GRID) {
    const size_t cnt = (size_t)3 * f->nx * f->ny * f->nz;
    // FNV-1a over the dimensions and the bytes: instances given equal grids share one device copy
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&hsh](const void* p, size_t bytes) {
      const unsigned char* b = static_cast<const unsigned char*>(p);
      for (size_t q = 0; q < bytes; ++q) hsh = (hsh ^ b[q]) * 1099511628211ull;
    };
    const int32_t dims[3] = {f->nx, f->ny, f->nz};
    mix(dims, sizeof(dims));
    mix(f->grid, cnt * sizeof(float));
    auto it = c->grids.find(hsh);
    if (it == c->grids.end() || it->second.n[0] != f->nx || it->second.n[1] != f->ny || it->second.n[2] != f->nz ||
        std::memcmp(it->second.host->data(), f->grid, cnt * sizeof(float)) != 0) {
      bpm_ctx::FieldGrid fg;
      auto host = std::make_shared<std::vector<float>>(f->grid, f->grid + cnt);
      HIPCHK(c, hipSetDevice(c->device));
      HIPCHK(c, hipMalloc(&fg.dev, sizeof(float) * cnt));
      HIPCHK(c, hipMemcpy(fg.dev, host->data(), sizeof(float) * cnt, hipMemcpyHostToDevice));
      fg.host = host;
      fg.n[0] = f->nx; fg.n[1] = f->ny; fg.n[2] = f->nz;
      while (c->grids.count(hsh)) ++hsh;   // a hash collision keeps both grids
      it = c->grids.emplace(hsh, fg).first;
    }
    k.grid = it->second.dev;
    I.grid_host = it->second.host;
    for (int d = 0; d < 3; ++d) { k.gorig[d] = f->g_origin[d]; k.gn[d] = it->second.n[d]; }
    k.gh = f->g_h;
  }
  if (m0) I.m0.resize(3 * (size_t)g.n);   // no vector kept for the default state (+z everywhere)
  for (int i = 0; m0 && i < g.n; ++i) {
    double a = m0[i], b = m0[g.n + i], d = m0[2 * g.n + i];
    double l = std::sqrt(a * a + b * b + d * d);
    if (!(l > 0.0) || !std::isfinite(l)) {
      // a non-finite or zero initial vector is kept as is: the run reports BPM_ENONFINITE
      l = 1.0;
    }
    I.m0[i] = a / l;
    I.m0[g.n + i] = b / l;
    I.m0[2 * g.n + i] = d / l;
  }
  *inst_id = (int32_t)c->insts.size();
  c->insts.push_back(std::move(I));
  c->have_results = false;
  c->inst_version++;
  return BPM_OK;
}

int bpm_couple_dipoles(bpm_ctx* c, int32_t n, const int32_t* ids) {
  if (!c) return BPM_EINVAL;
  if (n < 2 || !ids) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: need at least two instances");
  if (n > kMaxInstPerGroup) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: too many instances");
  int mesh = -1;
  for (int i = 0; i < n; ++i) {
    if (ids[i] < 0 || ids[i] >= (int)c->insts.size()) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: bad instance id");
    if (c->insts[ids[i]].coupled) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: instance already coupled");
    if (mesh < 0) mesh = c->insts[ids[i]].mesh;
    if (c->insts[ids[i]].mesh != mesh) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: instances on different meshes");
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double* a = c->insts[ids[i]].c.off;
      const double* b = c->insts[ids[j]].c.off;
      if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) return fail(c, BPM_EINVAL, "bpm_couple_dipoles: two islands at one position");
    }
  for (int i = 0; i < n; ++i) {
    c->insts[ids[i]].coupled = true;
    c->insts[ids[i]].sys = ids[0];
  }
  c->have_results = false;
  c->inst_version++;
  return BPM_OK;
}

int bpm_clear_instances(bpm_ctx* c) {
  if (!c) return BPM_EINVAL;
  if (c->run_pending) return fail(c, BPM_ESTATE, "bpm_clear_instances: a run is pending; call bpm_sync first");
  c->insts.clear();
  c->have_results = false;
  c->inst_version++;
  return BPM_OK;
}

}  // extern "C"

// Relative cost of one field evaluation of an n-node island in a batch: the bytes of its demag
// tiles plus a per-node term for the gather-bound exchange and field phases (on the 4096-island
// batch those phases take about 0.43 of the demag stream's time, i.e. about 1.2 KB of stream per
// node).
static double island_eval_cost(int n) {
  return (double)tile_count(n) * kTile * kTile * sizeof(float) + 1200.0 * n;
}

template <typename real>
static int run_typed(bpm_ctx* c, const bpm_run_opts* o, hipStream_t stream) {
  Arena& A = c->run;
  A.clear();
  const int nm = (int)c->meshes.size();
  // order instances by mesh group, coupled sets contiguous (system root order)
  std::vector<std::vector<int32_t>> by_mesh(nm);
  for (int32_t i = 0; i < (int32_t)c->insts.size(); ++i) by_mesh[c->insts[i].mesh].push_back(i);
  c->inst_order.clear();
  c->slot_of.assign(c->insts.size(), -1);
  c->slot_group.clear();
  c->slot_local.clear();
  c->group_inst0.assign(nm, -1);
  std::vector<int32_t> group_ids;
  std::vector<SysView> sysv;
  std::vector<InstConst> ic;
  std::vector<int32_t> group_sys0, group_nsys;
  for (int mi = 0; mi < nm; ++mi) {
    auto& v = by_mesh[mi];
    if (v.empty()) continue;
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      int ra = c->insts[a].coupled ? c->insts[a].sys : a, rb = c->insts[b].coupled ? c->insts[b].sys : b;
      return ra < rb;
    });
    if ((int)v.size() > kMaxInstPerGroup)
      return fail(c, BPM_EINVAL, "bpm_run: more than 64 instances on one mesh group");
    group_ids.push_back(mi);
    c->group_inst0[mi] = (int32_t)c->inst_order.size();
    group_sys0.push_back((int32_t)sysv.size());
    int local = 0;
    int last_root = -1;
    for (int32_t id : v) {
      const int root = c->insts[id].coupled ? c->insts[id].sys : id;
      if (root != last_root) {
        SysView sv{(int32_t)c->inst_order.size(), 0, c->insts[id].coupled ? 1 : 0, 0};
        sysv.push_back(sv);
        last_root = root;
      }
      sysv.back().count++;
      c->slot_of[id] = (int32_t)c->inst_order.size();
      c->inst_order.push_back(id);
      c->slot_group.push_back(mi);
      c->slot_local.push_back(local++);
      InstConst k = c->insts[id].c;
      k.group = (int32_t)group_ids.size() - 1;
      k.sys = (int32_t)sysv.size() - 1;
      k.local = local - 1;
      ic.push_back(k);
    }
    group_nsys.push_back((int32_t)sysv.size() - group_sys0.back());
  }
  const int ng = (int)group_ids.size();
  const int ninst = (int)ic.size(), nsys = (int)sysv.size();
  c->sys_of_slot.resize(ninst);
  for (int s = 0; s < ninst; ++s) c->sys_of_slot[s] = ic[s].sys;
  if (ng == 0) return fail(c, BPM_ESTATE, "bpm_run: no instances");

  // launch shape
  const bool fixed = o->integrator == BPM_DP5_FIXED;
  int ldS_max = 16, Rmax = 1, nmax = 1;
  for (int gi = 0; gi < ng; ++gi) {
    const MeshGroup& g = *c->meshes[group_ids[gi]];
    ldS_max = std::max(ldS_max, (g.n + 15) / 16 * 16);
    nmax = std::max(nmax, g.n);
    Rmax = std::max(Rmax, (int)by_mesh[group_ids[gi]].size());
  }
  const bool sym = (o->flags & BPM_FLAG_SYMMETRIC_DEMAG) && sizeof(real) == 4;
  int tuned_wg = 0;
  if (o->wg_per_group <= 0) {
    auto it = c->tune.find(tune_key(nmax, ninst, (int)sizeof(real) * 8));
    if (it != c->tune.end()) tuned_wg = it->second;
  }
  // 512-thread workgroups: when asked for, when the tuner chose them, and by default for untuned
  // launches of several mesh groups (twice the waves per island); BPM_FLAG_WG256 forces 256
  const bool want512 = (o->flags & BPM_FLAG_WG512) || tuned_wg < 0 ||
                       (ng > 1 && o->wg_per_group <= 0 && tuned_wg == 0);
  const int bs = (want512 && !(o->flags & BPM_FLAG_WG256)) ? 512 : 256;
  const size_t lds_budget = sym ? 48 * 1024 : 96 * 1024;
  int RB = (int)std::max<size_t>(1, std::min<size_t>(16, lds_budget / (sizeof(real) * (size_t)ldS_max)));
  RB = std::min(RB, Rmax);
  if ((size_t)RB * ldS_max * sizeof(real) > 120 * 1024)
    return fail(c, BPM_EINVAL, "bpm_run: island too large for the LDS staging of the demag product");
  // dipole pair geometry of coupled instances staged in LDS for groups of up to 16 instances
  bool any_coupled = false;
  for (const auto& I : c->insts) any_coupled = any_coupled || I.coupled;
  const int dip = (any_coupled && Rmax <= 16) ? Rmax : 0;
  // rows longer than one round of the demag product keep per-wave round sums after the staged b
  const int part = ldS_max > 12 * 64 * (int)(16 / sizeof(real)) ? (bs / 64) * 4 * 16 : 0;
  LdsPlan L{Rmax, (sym ? 2 : 1) * RB * ldS_max + part, 0, 0, 0, ldS_max, dip};
  int per_cu = 0, cus = 0;
  {
    hipError_t e = max_coresident<real>(L, fixed, bs, true, &per_cu, &cus);
    if (e != hipSuccess) return fail(c, BPM_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
    if (per_cu <= 0) return fail(c, BPM_EINVAL, "bpm_run: the stepping kernel does not fit a compute unit with this island size");
  }
  const int cap = std::max(1, per_cu * cus);
  std::vector<int> G(ng, 1);
  bool coop = false;
  int wg_req = o->wg_per_group > 0 ? o->wg_per_group : (tuned_wg < 0 ? -tuned_wg : tuned_wg);
  if (wg_req > 0) {
    for (int gi = 0; gi < ng; ++gi) G[gi] = std::max(1, std::min(wg_req, c->meshes[group_ids[gi]]->n / 8));
  } else if (ng < cap) {
    // share the resident workgroups among the groups in proportion to their demag work
    std::vector<double> w(ng);
    double tot = 0.0;
    for (int gi = 0; gi < ng; ++gi) {
      const MeshGroup& g = *c->meshes[group_ids[gi]];
      w[gi] = (double)g.n * g.n * by_mesh[group_ids[gi]].size();
      tot += w[gi];
    }
    for (int gi = 0; gi < ng; ++gi) {
      const int nmaxwg = std::max(1, c->meshes[group_ids[gi]]->n / 16);
      G[gi] = std::max(1, std::min(nmaxwg, (int)std::floor(cap * 0.5 * w[gi] / tot)));
    }
  }
  int grid = 0;
  for (int gi = 0; gi < ng; ++gi) {
    grid += G[gi];
    if (G[gi] > 1) coop = true;
  }
  if (coop && grid > cap) return fail(c, BPM_EINVAL, "bpm_run: workgroups per group exceed the resident capacity");
  // Cooperative runs keep the CSR rows and node data of the owned nodes in LDS and, when they fit
  // with every workgroup still resident, the owned rows of S (with the largest RB that fits).
  if (coop) {
    int own_max = 0, nnz_max = 0;
    for (int gi = 0; gi < ng; ++gi) {
      const MeshGroup& g = *c->meshes[group_ids[gi]];
      for (int w = 0; w < G[gi]; ++w) {
        const int a = (int)((long long)g.n * w / G[gi]), b = (int)((long long)g.n * (w + 1) / G[gi]);
        own_max = std::max(own_max, b - a);
        nnz_max = std::max(nnz_max, g.rowptr[b] - g.rowptr[a]);
      }
    }
    auto fits = [&](const LdsPlan& T) {
      if (dp5_lds_bytes<real>(T) > 160 * 1024) return false;
      int pc = 0, cu = 0;
      return max_coresident<real>(T, fixed, bs, true, &pc, &cu) == hipSuccess && pc * cu >= grid;
    };
    bool found = false;
    if (!(o->flags & BPM_FLAG_STREAM_S) && !sym) {
      for (int rb = std::min(Rmax, 16); rb >= 1 && !found; --rb) {
        LdsPlan T{Rmax, rb * ldS_max + part, nnz_max + 64, own_max, own_max, ldS_max, dip};
        if (fits(T)) { L = T; RB = rb; found = true; }
      }
    }
    if (!found) {
      LdsPlan T = L;
      T.csr_cap = nnz_max + 64;
      T.own_cap = own_max;
      if (fits(T)) L = T;
    }
  }
  const int csr_cap = L.csr_cap;
  c->run_plan = L;
  c->run_bs = bs;
  c->run_RB = RB;
  c->run_csr_cap = csr_cap;
  c->run_grid = grid;
  c->run_G = *std::max_element(G.begin(), G.end());

  // device buffers
  InstConst* d_ic;
  SysView* d_sys;
  int2* d_map;
  int2* d_imap;
  double *d_err, *d_obs, *d_mom;
  unsigned long long* d_bar;
  GroupView<real>* d_groups;
  HIPCHK(c, A.alloc(&d_ic, ninst));
  HIPCHK(c, A.alloc(&d_sys, nsys));
  HIPCHK(c, A.alloc(&d_map, grid));
  HIPCHK(c, A.alloc(&d_imap, ninst));
  HIPCHK(c, A.alloc(&d_err, (size_t)nsys * 3));
  HIPCHK(c, A.alloc(&d_obs, (size_t)ninst * 3 * 6));
  HIPCHK(c, A.alloc(&d_mom, (size_t)ninst * 3 * 3));
  HIPCHK(c, A.alloc(&d_bar, ng));
  HIPCHK(c, A.alloc(&d_groups, ng));
  HIPCHK(c, A.alloc(&c->d_sys_out, nsys));
  HIPCHK(c, A.alloc(&c->d_inst_out, ninst));
  HIPCHK(c, A.alloc(&c->d_energy, ninst));
  const int tcap = std::max(0, o->traj_cap);
  HIPCHK(c, A.alloc(&c->d_traj, (size_t)ninst * std::max(1, tcap) * kTrajW));

  std::vector<GroupView<real>> gv(ng);
  std::vector<int2> wmap;
  std::vector<int2> imap(ninst);
  c->group_m.assign(nm, nullptr);
  int wg = 0;
  for (int gi = 0; gi < ng; ++gi) {
    const int mi = group_ids[gi];
    const MeshGroup& g = *c->meshes[mi];
    const DevGeom<real>& d = std::is_same<real, double>::value
                                 ? *reinterpret_cast<const DevGeom<real>*>(&c->dmeshes[mi]->g64)
                                 : *reinterpret_cast<const DevGeom<real>*>(&c->dmeshes[mi]->g32);
    GroupView<real>& v = gv[gi];
    const int R = (int)by_mesh[mi].size();
    v.n = g.n; v.nnz = g.nnz; v.R = R; v.nsys = group_nsys[gi];
    v.ldS = (g.n + 15) / 16 * 16;
    v.wg0 = wg; v.G = G[gi];
    v.inst0 = c->group_inst0[mi]; v.sys0 = group_sys0[gi];
    v.rowptr = d.rowptr; v.col = d.col; v.colx = d.colx; v.K = d.K; v.D = d.D; v.DT = d.DT;
    v.S = std::is_same<real, double>::value ? reinterpret_cast<const real*>(g.dS64) : reinterpret_cast<const real*>(g.dS32);
    v.St = std::is_same<real, float>::value ? g.dS32t : nullptr;
    v.St16 = std::is_same<real, float>::value && !g.dS32t ? g.dS16t : nullptr;
    v.s16_inv = (float)(1.0 / g.s16_scale);
    // the packed tiles serve only the upper-triangle product of single-workgroup groups
    if (!v.S && !((v.St || v.St16) && sym && G[gi] == 1 && !coop))
      return fail(c, BPM_EINVAL, (v.St || v.St16) ? "bpm_run: a group keeping only the packed tiles of S needs "
                                        "BPM_FLAG_SYMMETRIC_DEMAG and one workgroup per group"
                                      : "bpm_run: a mesh group does not keep S in the run precision");
    v.V = d.V; v.layer = d.layer; v.partner = d.partner; v.aif = d.aif;
    v.x = d.x; v.y = d.y; v.z = d.z;
    for (int k = 0; k < 3; ++k) v.cen[k] = g.centroid[k];
    v.Vsoft = g.vol_layer[0]; v.Vhard = g.vol_layer[1];
    const size_t st3 = (size_t)3 * g.n;
    HIPCHK(c, A.alloc(&v.m, R * st3));
    HIPCHK(c, A.alloc(&v.ys, 2 * R * st3));
    HIPCHK(c, A.alloc(&v.k, 7 * R * st3));
    HIPCHK(c, A.alloc(&v.yex, R * st3));
    HIPCHK(c, A.alloc(&v.b, (size_t)R * v.ldS));
    HIPCHK(c, A.alloc(&v.u, (size_t)R * v.ldS));
    HIPCHK(c, hipMemsetAsync(v.k, 0, sizeof(real) * 7 * R * st3, stream));
    HIPCHK(c, hipMemsetAsync(v.b, 0, sizeof(real) * R * v.ldS, stream));   // padding stays zero
    HIPCHK(c, hipMemsetAsync(v.u, 0, sizeof(real) * R * v.ldS, stream));
    v.bar = d_bar + gi;
    c->group_m[mi] = v.m;
    std::vector<real> m0(R * st3);
    for (int r = 0; r < R; ++r) {
      const auto& src = c->insts[by_mesh[mi][r]].m0;
      for (size_t q = 0; q < st3; ++q) m0[r * st3 + q] = src.empty() ? (real)(q >= 2 * (size_t)g.n) : (real)src[q];
      imap[v.inst0 + r] = make_int2(gi, r);
    }
    HIPCHK(c, hipMemcpyAsync(v.m, m0.data(), sizeof(real) * m0.size(), hipMemcpyHostToDevice, stream));
    wg += G[gi];
  }
  // Workgroups are dispatched in map order and, past the resident capacity, start as earlier ones
  // finish: the groups with the most work per workgroup go first, so that long islands do not
  // start last and set the length of the launch.  Work of a group = its demag bytes per evaluation
  // (N^2 R / G) times the evaluations it will need, which the exchange-limited step makes
  // proportional to the largest exchange field scale 2 A / Ms over its layers and instances.
  {
    std::vector<double> cost(ng);
    for (int gi = 0; gi < ng; ++gi) {
      double stiff = 0.0;
      for (int r = 0; r < gv[gi].R; ++r) {
        const InstConst& k = ic[gv[gi].inst0 + r];
        stiff = std::max({stiff, k.cex[0], k.cex[1]});
      }
      cost[gi] = island_eval_cost(gv[gi].n) * gv[gi].R / G[gi] * stiff;
    }
    std::vector<int> order(ng);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int gi : order) {
      gv[gi].wg0 = (int)wmap.size();
      for (int w = 0; w < G[gi]; ++w) wmap.push_back(make_int2(gi, w));
    }
  }
  HIPCHK(c, hipMemcpyAsync(d_groups, gv.data(), sizeof(GroupView<real>) * ng, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_ic, ic.data(), sizeof(InstConst) * ninst, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_sys, sysv.data(), sizeof(SysView) * nsys, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_map, wmap.data(), sizeof(int2) * grid, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_imap, imap.data(), sizeof(int2) * ninst, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemsetAsync(d_err, 0, sizeof(double) * nsys * 3, stream));
  HIPCHK(c, hipMemsetAsync(d_obs, 0, sizeof(double) * ninst * 18, stream));
  HIPCHK(c, hipMemsetAsync(d_mom, 0, sizeof(double) * ninst * 9, stream));
  HIPCHK(c, hipMemsetAsync(d_bar, 0, sizeof(unsigned long long) * ng, stream));
  HIPCHK(c, hipMemsetAsync(c->d_sys_out, 0, sizeof(SysOut) * nsys, stream));
  HIPCHK(c, hipMemsetAsync(c->d_inst_out, 0, sizeof(InstOut) * ninst, stream));

  RunParams P{};
  P.ngroups = ng; P.ninst = ninst; P.nsys = nsys; P.integrator = o->integrator;
  P.t_end = o->t_end; P.dt0 = o->dt0; P.dt_fixed = o->dt_fixed; P.rtol = o->rtol; P.atol = o->atol;
  P.dt_min = o->dt_min; P.temperature = o->temperature; P.max_steps = o->max_steps;
  P.save_every = o->save_every; P.traj_cap = tcap;
  P.flags = o->flags & ~BPM_FLAG_CONTINUE;
  P.resume = 0;
  P.inst = d_ic; P.sys = d_sys; P.sys_out = c->d_sys_out; P.inst_out = c->d_inst_out; P.traj = c->d_traj;
  P.err_acc = d_err; P.obs_acc = d_obs; P.mom_acc = d_mom; P.wg_map = d_map;

  HIPCHK(c, hipEventRecord(c->ev0, stream));
  {
    hipError_t e = launch_dp5<real>(d_groups, P, grid, RB, L, fixed, coop, stream, bs);
    if (e != hipSuccess) return fail(c, BPM_EHIP, std::string("stepping kernel launch: ") + hipGetErrorString(e));
  }
  HIPCHK(c, hipEventRecord(c->ev1, stream));
  {
    hipError_t e = launch_energy<real>(d_groups, d_imap, ninst, P, c->d_energy, nmax, stream);
    if (e != hipSuccess) return fail(c, BPM_EHIP, std::string("energy kernel launch: ") + hipGetErrorString(e));
  }
  c->run_ninst = ninst;
  c->run_nsys = nsys;
  c->run_traj_cap = tcap;
  c->run_precision = sizeof(real) == 8 ? 64 : 32;
  c->run_stream = stream;
  c->run_pending = true;
  c->have_results = false;
  c->run_resumable = true;
  c->run_version = c->inst_version;
  c->run_integrator = o->integrator;
  c->run_flags = o->flags & ~BPM_FLAG_CONTINUE;
  c->run_fixed = fixed;
  c->run_coop = coop;
  c->run_t_end = o->t_end;
  c->run_dt_fixed = o->dt_fixed;
  c->run_P = P;
  c->run_d_groups = d_groups;
  c->run_d_imap = d_imap;
  c->run_nmax = nmax;
  c->run_ng = ng;
  c->run_d_err = d_err;
  c->run_d_obs = d_obs;
  c->run_d_mom = d_mom;
  c->run_d_bar = d_bar;
  c->run_d_map = d_map;
  c->run_group_G = G;
  c->run_group_n.resize(ng);
  c->run_group_sys0 = group_sys0;
  c->run_group_nsys = group_nsys;
  for (int gi = 0; gi < ng; ++gi) c->run_group_n[gi] = gv[gi].n;
  c->run_att_start.assign(nsys, 0);
  return BPM_OK;
}

// Continues the last stepping run up to the new t_end: same instances, buffers and launch shape;
// the kernel starts from the state, controller and crossing data the previous launch stored.
template <typename real>
static int resume_typed(bpm_ctx* c, const bpm_run_opts* o, hipStream_t stream) {
  RunParams P = c->run_P;
  P.t_end = o->t_end;
  P.rtol = o->rtol;
  P.atol = o->atol;
  P.dt_min = o->dt_min;
  P.max_steps = o->max_steps;
  P.save_every = o->save_every;
  P.resume = 1;
  // the step-control, observable and moment accumulators and the barrier counters restart at zero
  HIPCHK(c, hipMemsetAsync(c->run_d_err, 0, sizeof(double) * c->run_nsys * 3, stream));
  HIPCHK(c, hipMemsetAsync(c->run_d_obs, 0, sizeof(double) * c->run_ninst * 18, stream));
  HIPCHK(c, hipMemsetAsync(c->run_d_mom, 0, sizeof(double) * c->run_ninst * 9, stream));
  HIPCHK(c, hipMemsetAsync(c->run_d_bar, 0, sizeof(unsigned long long) * c->run_ng, stream));
  // Single-workgroup groups are dispatched by the work they took in the previous launch (its
  // attempts times their demag bytes), largest first: step counts differ by several times between
  // islands, and the longest ones must not start last.
  const int ng = (int)c->run_group_n.size();
  bool all_single = true;
  for (int gi = 0; gi < ng; ++gi) all_single = all_single && c->run_group_G[gi] == 1;
  if (all_single && (int)c->h_sys_out.size() == c->run_nsys) {
    std::vector<double> cost(ng, 0.0);
    std::vector<int64_t> att_now(c->run_nsys);
    for (int sl = 0; sl < c->run_nsys; ++sl) att_now[sl] = c->h_sys_out[sl].n_accept + c->h_sys_out[sl].n_reject;
    for (int gi = 0; gi < ng; ++gi) {
      int64_t att = 0;
      for (int sl = c->run_group_sys0[gi]; sl < c->run_group_sys0[gi] + c->run_group_nsys[gi]; ++sl) {
        const bool live = c->h_sys_out[sl].status == BPM_OK && c->h_sys_out[sl].t_reached < o->t_end;
        if (live) att = std::max<int64_t>(att, std::max<int64_t>(1, att_now[sl] - c->run_att_start[sl]));
      }
      cost[gi] = island_eval_cost(c->run_group_n[gi]) * (double)att;
    }
    std::vector<int> order(ng);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    c->run_wmap.resize(ng);
    for (int q = 0; q < ng; ++q) c->run_wmap[q] = make_int2(order[q], 0);
    HIPCHK(c, hipMemcpyAsync(c->run_d_map, c->run_wmap.data(), sizeof(int2) * ng, hipMemcpyHostToDevice, stream));
    c->run_att_start = att_now;
  }
  const GroupView<real>* d_groups = reinterpret_cast<const GroupView<real>*>(c->run_d_groups);
  HIPCHK(c, hipEventRecord(c->ev0, stream));
  {
    hipError_t e = launch_dp5<real>(d_groups, P, c->run_grid, c->run_RB, c->run_plan, c->run_fixed, c->run_coop,
                                    stream, c->run_bs);
    if (e != hipSuccess) return fail(c, BPM_EHIP, std::string("stepping kernel launch: ") + hipGetErrorString(e));
  }
  HIPCHK(c, hipEventRecord(c->ev1, stream));
  {
    hipError_t e = launch_energy<real>(d_groups, c->run_d_imap, c->run_ninst, P, c->d_energy, c->run_nmax, stream);
    if (e != hipSuccess) return fail(c, BPM_EHIP, std::string("energy kernel launch: ") + hipGetErrorString(e));
  }
  c->run_t_end = o->t_end;
  c->run_P.t_end = o->t_end;
  c->run_stream = stream;
  c->run_pending = true;
  c->have_results = false;
  return BPM_OK;
}


template <typename real>
static int run_heun_typed(bpm_ctx* c, const bpm_run_opts* o, hipStream_t stream) {
  Arena& A = c->run;
  A.clear();
  const int nm = (int)c->meshes.size();
  std::vector<std::vector<int32_t>> by_mesh(nm);
  for (int32_t i = 0; i < (int32_t)c->insts.size(); ++i) {
    if (c->insts[i].coupled) return fail(c, BPM_EINVAL, "bpm_run: dipole coupling is not available with BPM_HEUN");
    by_mesh[c->insts[i].mesh].push_back(i);
  }
  c->inst_order.clear();
  c->slot_of.assign(c->insts.size(), -1);
  c->slot_group.clear(); c->slot_local.clear(); c->slot_R.clear();
  c->group_inst0.assign(nm, -1);
  c->group_m.assign(nm, nullptr);
  std::vector<InstConst> ic;
  std::vector<HeunGroup<real>> hg;
  std::vector<int2> bmap;
  std::vector<int4> tmap;
  std::vector<uint2> keys;
  std::vector<size_t> key_off;
  int Rmax = 1;
  for (int mi = 0; mi < nm; ++mi) {
    auto& v = by_mesh[mi];
    if (v.empty()) continue;
    const MeshGroup& g = *c->meshes[mi];
    const DevGeom<real>& d = std::is_same<real, double>::value
                                 ? *reinterpret_cast<const DevGeom<real>*>(&c->dmeshes[mi]->g64)
                                 : *reinterpret_cast<const DevGeom<real>*>(&c->dmeshes[mi]->g32);
    const int R = (int)v.size();
    Rmax = std::max(Rmax, R);
    HeunGroup<real> h{};
    key_off.push_back(keys.size());   // this group's realizations' keys start here
    h.n = g.n; h.R = R; h.ldS = (g.n + 15) / 16 * 16; h.inst0 = (int)ic.size(); h.ldR = (R + 3) / 4 * 4;
    h.rowptr = d.rowptr; h.col = d.col; h.colx = d.colx; h.K = d.K; h.D = d.D; h.DT = d.DT;
    h.S = std::is_same<real, double>::value ? reinterpret_cast<const real*>(g.dS64) : reinterpret_cast<const real*>(g.dS32);
    if (!h.S) return fail(c, BPM_EINVAL, "bpm_run: BPM_HEUN needs the row-major S in the run precision (BPM_KEEP_S64 / BPM_KEEP_S32)");
    h.V = d.V; h.layer = d.layer; h.partner = d.partner; h.aif = d.aif; h.x = d.x; h.y = d.y; h.z = d.z;
    h.Vsoft = g.vol_layer[0]; h.Vhard = g.vol_layer[1];
    const size_t cs = (size_t)g.n * R;
    HIPCHK(c, A.alloc(&h.m, 3 * cs));
    HIPCHK(c, A.alloc(&h.yt, 3 * cs));
    HIPCHK(c, A.alloc(&h.k1, 3 * cs));
    HIPCHK(c, A.alloc(&h.mnext, 3 * cs));
    HIPCHK(c, A.alloc(&h.b, (size_t)g.n * h.ldR));
    HIPCHK(c, A.alloc(&h.u, (size_t)g.n * h.ldR));
    HIPCHK(c, hipMemsetAsync(h.b, 0, sizeof(real) * g.n * h.ldR, stream));   // padding columns stay zero
    // [3][n][R] initial state; realizations in the default state (+z) need no transposition
    std::vector<real> m0(3 * cs, (real)0);
    std::fill(m0.begin() + 2 * cs, m0.end(), (real)1);
    for (int r0 = 0; r0 < R; r0 += 32)
      for (int comp = 0; comp < 3; ++comp)
        for (int i0 = 0; i0 < g.n; i0 += 32)
          for (int r = r0; r < std::min(R, r0 + 32); ++r) {
            const auto& src = c->insts[v[r]].m0;
            if (src.empty()) continue;
            for (int i = i0; i < std::min(g.n, i0 + 32); ++i)
              m0[comp * cs + (size_t)i * R + r] = (real)src[(size_t)comp * g.n + i];
          }
    c->group_inst0[mi] = (int32_t)c->inst_order.size();
    for (int r = 0; r < R; ++r) {
      const int id = v[r];
      c->slot_of[id] = (int32_t)c->inst_order.size();
      c->inst_order.push_back(id);
      c->slot_group.push_back(mi);
      c->slot_local.push_back(r);
      c->slot_R.push_back(R);
      InstConst k = c->insts[id].c;
      k.group = (int32_t)hg.size(); k.sys = (int32_t)ic.size(); k.local = r;
      ic.push_back(k);
      keys.push_back(make_uint2(k.key[0], k.key[1]));
    }
    // realizations that differ only in their noise key share one constant block on the device
    h.uniform = 1;
    for (int r = 1; r < R && h.uniform; ++r)
      if (std::memcmp(&ic[h.inst0], &ic[h.inst0 + r], offsetof(InstConst, key)) != 0) h.uniform = 0;
    HIPCHK(c, hipMemcpyAsync(h.m, m0.data(), sizeof(real) * m0.size(), hipMemcpyHostToDevice, stream));
    c->group_m[mi] = h.m;
    const int gi = (int)hg.size();
    const long nb = ((long)g.n * R + 255) / 256;
    for (long b = 0; b < nb; ++b) bmap.push_back(make_int2(gi, (int)b));   // node-major: contiguous runs share neighbours
    constexpr int T = heun_tile<real>();
    for (int m0r = 0; m0r < g.n; m0r += T)
      for (int n0 = 0; n0 < R; n0 += T) tmap.push_back(make_int4(gi, m0r, n0, 0));
    hg.push_back(h);
  }
  const int ng = (int)hg.size(), ninst = (int)ic.size();
  if (ng == 0) return fail(c, BPM_ESTATE, "bpm_run: no instances");
  while (tmap.size() % 8) tmap.push_back(make_int4(-1, 0, 0, 0));   // whole rounds over the eight XCDs
  while (bmap.size() % 8) bmap.push_back(make_int2(-1, 0));
  if (bmap.size() > 0x7fffffffu || tmap.size() > 0x7fffffffu) return fail(c, BPM_EINVAL, "bpm_run: batch too large");
  HeunGroup<real>* d_groups;
  HeunGroup<real>* d_groups_odd;
  int2* d_bmap;
  int4* d_tmap;
  InstConst* d_ic;
  unsigned long long* d_step;
  double* d_obs;
  HIPCHK(c, A.alloc(&d_groups, ng));
  HIPCHK(c, A.alloc(&d_groups_odd, ng));
  HIPCHK(c, A.alloc(&d_bmap, bmap.size()));
  HIPCHK(c, A.alloc(&d_tmap, tmap.size()));
  HIPCHK(c, A.alloc(&d_ic, ninst));
  HIPCHK(c, A.alloc(&d_step, 1));
  HIPCHK(c, A.alloc(&d_obs, 2 * (size_t)ninst));
  HIPCHK(c, A.alloc(&c->d_energy, ninst));
  uint2* d_keys;
  HIPCHK(c, A.alloc(&d_keys, keys.size()));
  for (int gi = 0; gi < ng; ++gi) hg[gi].keys = d_keys + key_off[gi];
  // two group tables with m and mnext swapped: steps alternate between them (no copy-back);
  // built once every device pointer of the even table is final
  std::vector<HeunGroup<real>> hg_odd(hg);
  for (auto& h : hg_odd) std::swap(h.m, h.mnext);
  for (int gi = 0; gi < ng; ++gi)
    for (const HeunGroup<real>* h : {&hg[gi], &hg_odd[gi]})
      if (h->keys < d_keys || h->keys + h->R > d_keys + keys.size() || !h->m || !h->mnext || h->m == h->mnext)
        return fail(c, BPM_ESTATE, "bpm_run: inconsistent Heun group table (internal error)");
  HIPCHK(c, hipMemcpyAsync(d_keys, keys.data(), sizeof(uint2) * keys.size(), hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_groups, hg.data(), sizeof(HeunGroup<real>) * ng, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_groups_odd, hg_odd.data(), sizeof(HeunGroup<real>) * ng, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_bmap, bmap.data(), sizeof(int2) * bmap.size(), hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_tmap, tmap.data(), sizeof(int4) * tmap.size(), hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemcpyAsync(d_ic, ic.data(), sizeof(InstConst) * ninst, hipMemcpyHostToDevice, stream));
  HIPCHK(c, hipMemsetAsync(d_step, 0, sizeof(unsigned long long), stream));
  HeunLaunch<real> L{d_groups, d_bmap, d_tmap, d_ic, (int)bmap.size(), (int)tmap.size(),
                     HeunParams{o->dt_fixed, o->dt_fixed, o->temperature, d_step}, true, true};
  for (const auto& h : hg) {
    L.all_uniform = L.all_uniform && h.uniform;
    L.all_wave = L.all_wave && (h.R % 64 == 0);
  }
  const long long nsteps = (long long)std::ceil(o->t_end / o->dt_fixed - 1e-9);
  const double h_last = o->t_end - (double)(nsteps - 1) * o->dt_fixed;
  const bool clip = nsteps > 0 && std::fabs(h_last - o->dt_fixed) > 1e-12 * o->dt_fixed;
  const long long nfull = clip ? nsteps - 1 : nsteps;
  HeunLaunch<real> Lodd = L;
  Lodd.groups = d_groups_odd;
  HIPCHK(c, hipEventRecord(c->ev0, stream));
  if (nfull >= 2) {
    // two regular steps (even table, then odd table) captured once, replayed nfull / 2 times
    hipGraph_t graph = nullptr;
    if (c->graph_exec) {
      hipGraphExecDestroy(c->graph_exec);
      c->graph_exec = nullptr;
    }
    HIPCHK(c, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    hipError_t ce = heun_step<real>(L, stream);
    if (ce == hipSuccess) ce = heun_step<real>(Lodd, stream);
    hipError_t ee = hipStreamEndCapture(stream, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(c, BPM_EHIP, std::string("Heun graph capture: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(c, BPM_EHIP, std::string("Heun graph instantiate: ") + hipGetErrorString(ie));
    for (long long st = 0; st + 1 < nfull; st += 2) HIPCHK(c, hipGraphLaunch(c->graph_exec, stream));
  }
  if (nfull % 2) HIPCHK(c, heun_step<real>(L, stream));
  if (clip) {
    HeunLaunch<real> Ll = (nfull % 2) ? Lodd : L;
    Ll.params.h = h_last;
    HIPCHK(c, heun_step<real>(Ll, stream));
  }
  HIPCHK(c, hipEventRecord(c->ev1, stream));
  // the final state is in the m of the even table after an even number of steps, else of the odd one
  const bool odd = nsteps % 2;
  HIPCHK(c, heun_observe_launch<real>(odd ? Lodd : L, ng, Rmax, d_obs, stream));
  for (int mi = 0, gi = 0; mi < nm; ++mi)
    if (c->group_m[mi]) c->group_m[mi] = (odd ? hg_odd : hg)[gi++].m;
  // results in the same shapes as the DP5 path (one system per instance)
  c->run_ninst = ninst;
  c->run_nsys = ninst;
  c->sys_of_slot.resize(ninst);
  for (int s2 = 0; s2 < ninst; ++s2) c->sys_of_slot[s2] = s2;
  c->h_sys_out.assign(ninst, SysOut{});
  c->h_inst_out.assign(ninst, InstOut{});
  c->h_energy.assign(ninst, NAN);
  c->heun_obs = d_obs;
  c->heun_nsteps = nsteps;
  c->heun_dt = o->dt_fixed;
  c->heun_t_end = o->t_end;
  c->run_traj_cap = 0;
  c->run_precision = sizeof(real) == 8 ? 64 : 32;
  c->run_stream = stream;
  c->run_rfast = true;
  c->run_pending = true;
  c->have_results = false;
  c->run_grid = L.nblk;
  c->run_G = 1;
  return BPM_OK;
}

extern "C" {

int bpm_run(bpm_ctx* c, const bpm_run_opts* o, void* hip_stream) {
  if (!c) return BPM_EINVAL;
  if (!o) return fail(c, BPM_EINVAL, "bpm_run: null options");
  if (c->run_pending) return fail(c, BPM_ESTATE, "bpm_run: previous run not synchronised");
  if (o->precision != 32 && o->precision != 64) return fail(c, BPM_EINVAL, "bpm_run: precision must be 32 or 64");
  if (o->integrator != BPM_DP45 && o->integrator != BPM_DP5_FIXED && o->integrator != BPM_HEUN)
    return fail(c, BPM_EINVAL, "bpm_run: unknown integrator");
  if (o->integrator == BPM_HEUN && (!(o->dt_fixed > 0.0) || !(o->temperature >= 0.0)))
    return fail(c, BPM_EINVAL, "bpm_run: BPM_HEUN needs dt_fixed > 0 and temperature >= 0");
  if (!(o->t_end >= 0.0) || !std::isfinite(o->t_end)) return fail(c, BPM_EINVAL, "bpm_run: t_end must be finite and >= 0");
  if (o->integrator == BPM_DP5_FIXED && !(o->dt_fixed > 0.0)) return fail(c, BPM_EINVAL, "bpm_run: dt_fixed must be > 0");
  if (o->integrator == BPM_DP45 && (!(o->dt0 > 0.0) || !(o->rtol > 0.0) || !(o->atol > 0.0)))
    return fail(c, BPM_EINVAL, "bpm_run: dt0, rtol, atol must be > 0");
  if (o->traj_cap < 0) return fail(c, BPM_EINVAL, "bpm_run: traj_cap must be >= 0");
  if (c->insts.empty()) return fail(c, BPM_ESTATE, "bpm_run: no instances");
  hipSetDevice(c->device);
  hipStream_t s = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->own_stream;
  if (o->flags & BPM_FLAG_CONTINUE) {
    if (!c->run_resumable || c->run_version != c->inst_version)
      return fail(c, BPM_ESTATE, "bpm_run: BPM_FLAG_CONTINUE needs a previous DP5 run of the same instances");
    if (o->integrator != c->run_integrator || o->precision != c->run_precision)
      return fail(c, BPM_EINVAL, "bpm_run: a continued run keeps the integrator and precision of the run it continues");
    if (o->t_end < c->run_t_end) return fail(c, BPM_EINVAL, "bpm_run: a continued run cannot end before the run it continues");
    if (o->integrator == BPM_DP5_FIXED) {
      const double q = c->run_t_end / c->run_dt_fixed;
      if (o->dt_fixed != c->run_dt_fixed || std::fabs(q - std::round(q)) > 1e-9 * std::max(1.0, q))
        return fail(c, BPM_EINVAL, "bpm_run: a continued fixed-step run needs the same dt_fixed and a previous end on its grid");
    }
    return o->precision == 64 ? resume_typed<double>(c, o, s) : resume_typed<float>(c, o, s);
  }
  c->run_resumable = false;
  c->run_rfast = false;
  if (o->integrator == BPM_HEUN) return o->precision == 64 ? run_heun_typed<double>(c, o, s) : run_heun_typed<float>(c, o, s);
  return o->precision == 64 ? run_typed<double>(c, o, s) : run_typed<float>(c, o, s);
}

int bpm_autotune(bpm_ctx* c, const bpm_run_opts* o, int32_t n_cand, const int32_t* cand, int64_t probe_attempts,
                 int32_t* best, double* ms_per_attempt) {
  if (!c) return BPM_EINVAL;
  if (!o || n_cand <= 0 || !cand || probe_attempts <= 0 || !best)
    return fail(c, BPM_EINVAL, "bpm_autotune: bad argument");
  if (o->integrator == BPM_HEUN) return fail(c, BPM_EINVAL, "bpm_autotune: tunes the DP5 kernels only");
  if (c->insts.empty()) return fail(c, BPM_ESTATE, "bpm_autotune: no instances");
  int nmax = 1;
  for (auto& I : c->insts) nmax = std::max(nmax, c->meshes[I.mesh]->n);
  double best_t = INFINITY;
  int best_g = 0;
  for (int q = 0; q < n_cand; ++q) {
    bpm_run_opts p = *o;
    p.wg_per_group = cand[q] > 0 ? cand[q] : -cand[q];
    p.flags = cand[q] > 0 ? ((o->flags & ~BPM_FLAG_WG512) | BPM_FLAG_WG256) : ((o->flags | BPM_FLAG_WG512) & ~BPM_FLAG_WG256);
    p.max_steps = probe_attempts;
    p.traj_cap = 0;
    int rc = bpm_run(c, &p, nullptr);
    if (rc == BPM_OK) rc = bpm_sync(c);
    double t = INFINITY;
    if (rc == BPM_OK) {
      // time per attempt of the longest-running system (every system gets the same budget)
      int64_t att = 1;
      for (const SysOut& so : c->h_sys_out) att = std::max<int64_t>(att, so.n_accept + so.n_reject);
      t = c->kernel_ms / (double)att;
    } else if (rc != BPM_EINVAL) {
      return rc;
    }
    if (ms_per_attempt) ms_per_attempt[q] = t;
    if (t < best_t) {
      best_t = t;
      best_g = cand[q] > 0 ? c->run_G : -c->run_G;
    }
  }
  // a winning 512-thread candidate is reported negative, so test the time, not the sign
  if (!std::isfinite(best_t) || best_g == 0) return fail(c, BPM_EINVAL, "bpm_autotune: no candidate could run");
  *best = best_g;
  const auto key = tune_key(nmax, (int)c->insts.size(), o->precision);
  c->tune[key] = best_g;
  if (!c->tune_path.empty()) {
    std::ofstream f(c->tune_path, std::ios::app);
    f << std::get<0>(key) << " " << std::get<1>(key) << " " << std::get<2>(key) << " " << best_g << "\n";
  }
  c->have_results = false;
  return BPM_OK;
}

int bpm_sync(bpm_ctx* c) {
  if (!c) return BPM_EINVAL;
  if (!c->run_pending) return c->have_results ? BPM_OK : fail(c, BPM_ESTATE, "bpm_sync: no run queued");
  hipSetDevice(c->device);
  c->run_pending = false;
  HIPCHK(c, hipStreamSynchronize(c->run_stream));
  HIPCHK(c, hipEventElapsedTime(&c->kernel_ms, c->ev0, c->ev1));
  if (c->run_rfast) {
    std::vector<double> obs(2 * (size_t)c->run_ninst);
    HIPCHK(c, hipMemcpy(obs.data(), c->heun_obs, sizeof(double) * obs.size(), hipMemcpyDeviceToHost));
    for (int s2 = 0; s2 < c->run_ninst; ++s2) {
      SysOut& so = c->h_sys_out[s2];
      InstOut& io = c->h_inst_out[s2];
      const bool finite = std::isfinite(obs[2 * s2]) && std::isfinite(obs[2 * s2 + 1]);
      so.status = finite ? BPM_OK : BPM_ENONFINITE;
      so.t_reached = c->heun_t_end;
      so.n_accept = c->heun_nsteps;
      so.n_reject = 0;
      so.dt_min_used = so.dt_max_used = c->heun_dt;
      so.max_norm_dev = 0.0;
      io.crossed = 0;
      io.t_sw = NAN;
      io.mz_soft = obs[2 * s2];
      io.mz_hard = obs[2 * s2 + 1];
      io.switched = io.mz_hard < 0.0;
      io.n_traj = 0;
    }
    c->have_results = true;
    return BPM_OK;
  }
  c->h_sys_out.resize(c->run_nsys);
  c->h_inst_out.resize(c->run_ninst);
  c->h_energy.resize(c->run_ninst);
  HIPCHK(c, hipMemcpy(c->h_sys_out.data(), c->d_sys_out, sizeof(SysOut) * c->run_nsys, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(c->h_inst_out.data(), c->d_inst_out, sizeof(InstOut) * c->run_ninst, hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(c->h_energy.data(), c->d_energy, sizeof(double) * c->run_ninst, hipMemcpyDeviceToHost));
  c->have_results = true;
  return BPM_OK;
}

// |B_applied| at the island centroid at time t (host evaluation; grids from the host copy)
static double applied_mag(const Instance& I, const MeshGroup& g, double t) {
  InstConst k = I.c;
  if (I.grid_host) k.grid = I.grid_host->data();
  double b[3];
  applied_field_at(k, t, g.centroid[0] + k.off[0], g.centroid[1] + k.off[1], g.centroid[2] + k.off[2], b[0], b[1], b[2]);
  return std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
}

int bpm_get_results(bpm_ctx* c, int32_t n, const int32_t* ids, bpm_result* out) {
  if (!c) return BPM_EINVAL;
  if (n < 0 || (n > 0 && (!ids || !out))) return fail(c, BPM_EINVAL, "bpm_get_results: bad argument");
  if (!c->have_results) return fail(c, BPM_ESTATE, "bpm_get_results: no synchronised run");
  for (int q = 0; q < n; ++q) {
    const int id = ids[q];
    if (id < 0 || id >= (int)c->slot_of.size() || c->slot_of[id] < 0) return fail(c, BPM_EINVAL, "bpm_get_results: bad instance id");
    const int s = c->slot_of[id];
    const SysOut& so = c->h_sys_out[c->sys_of_slot[s]];
    const InstOut& io = c->h_inst_out[s];
    bpm_result& r = out[q];
    r.status = so.status;
    r.switched = io.switched;
    r.t_sw = io.crossed ? io.t_sw : NAN;
    r.B_sw = io.crossed ? applied_mag(c->insts[id], *c->meshes[c->insts[id].mesh], io.t_sw) : NAN;
    r.mz_soft = io.mz_soft;
    r.mz_hard = io.mz_hard;
    r.t_reached = so.t_reached;
    r.energy = c->h_energy[s];
    r.n_accept = so.n_accept;
    r.n_reject = so.n_reject;
    r.dt_min_used = so.dt_min_used;
    r.dt_max_used = so.dt_max_used;
    r.max_norm_dev = so.max_norm_dev;
  }
  return BPM_OK;
}

int bpm_get_trajectory(bpm_ctx* c, int32_t id, double* out, int64_t cap, int64_t* n_written) {
  if (!c) return BPM_EINVAL;
  if (!out || !n_written || cap < 0) return fail(c, BPM_EINVAL, "bpm_get_trajectory: bad argument");
  if (!c->have_results) return fail(c, BPM_ESTATE, "bpm_get_trajectory: no synchronised run");
  if (id < 0 || id >= (int)c->slot_of.size() || c->slot_of[id] < 0) return fail(c, BPM_EINVAL, "bpm_get_trajectory: bad instance id");
  const int s = c->slot_of[id];
  const int64_t nt = std::min<int64_t>({c->h_inst_out[s].n_traj, cap, (int64_t)c->run_traj_cap});
  if (nt > 0)
    HIPCHK(c, hipMemcpy(out, c->d_traj + (size_t)s * c->run_traj_cap * kTrajW, sizeof(double) * nt * kTrajW,
                        hipMemcpyDeviceToHost));
  *n_written = nt;
  return BPM_OK;
}

int bpm_get_m(bpm_ctx* c, int32_t id, void* dst, int32_t dst_is_device) {
  if (!c) return BPM_EINVAL;
  if (!dst) return fail(c, BPM_EINVAL, "bpm_get_m: null output");
  if (!c->have_results) return fail(c, BPM_ESTATE, "bpm_get_m: no synchronised run");
  if (id < 0 || id >= (int)c->slot_of.size() || c->slot_of[id] < 0) return fail(c, BPM_EINVAL, "bpm_get_m: bad instance id");
  HIPCHK(c, hipSetDevice(c->device));
  const int s = c->slot_of[id];
  const int mi = c->slot_group[s];
  const long n = c->meshes[mi]->n;
  // [3][n][R] for thermal runs, [R][3][n] for stepping runs
  const long rstride = c->run_rfast ? c->slot_R[s] : 1;
  const long offset = c->run_rfast ? c->slot_local[s] : (long)c->slot_local[s] * 3 * n;
  if (dst_is_device) {
    HIPCHK(c, extract_m_device(c->run_precision, n, rstride, offset, c->group_m[mi], static_cast<double*>(dst),
                               c->own_stream));
    HIPCHK(c, hipStreamSynchronize(c->own_stream));
    return BPM_OK;
  }
  double* m_out = static_cast<double*>(dst);
  const size_t cnt = c->run_rfast ? 3 * (size_t)n * rstride : 3 * (size_t)n;
  const size_t first = c->run_rfast ? 0 : (size_t)offset;
  std::vector<double> all(cnt);
  if (c->run_precision == 64) {
    HIPCHK(c, hipMemcpy(all.data(), reinterpret_cast<double*>(c->group_m[mi]) + first, sizeof(double) * cnt,
                        hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(cnt);
    HIPCHK(c, hipMemcpy(tmp.data(), reinterpret_cast<float*>(c->group_m[mi]) + first, sizeof(float) * cnt,
                        hipMemcpyDeviceToHost));
    for (size_t q = 0; q < cnt; ++q) all[q] = tmp[q];
  }
  for (long comp = 0; comp < 3; ++comp)
    for (long i = 0; i < n; ++i)
      m_out[comp * n + i] = c->run_rfast ? all[(size_t)(comp * n + i) * rstride + offset] : all[(size_t)(comp * n + i)];
  return BPM_OK;
}

int bpm_string_reparam(bpm_ctx* c, int32_t P, const int32_t* ids, double* arclen) {
  if (!c) return BPM_EINVAL;
  if (!ids || P < 3 || P > kStringMaxImages)
    return fail(c, BPM_EINVAL, "bpm_string_reparam: need 3..64 image ids");
  if (!c->have_results || c->run_rfast || c->run_version != c->inst_version)
    return fail(c, BPM_ESTATE, "bpm_string_reparam: the last synchronised run must be a DP5 run of the current instances");
  int mi = -1;
  StringImages im{};
  for (int k = 0; k < P; ++k) {
    const int id = ids[k];
    if (id < 0 || id >= (int)c->slot_of.size() || c->slot_of[id] < 0)
      return fail(c, BPM_EINVAL, "bpm_string_reparam: bad instance id");
    for (int l = 0; l < k; ++l)
      if (ids[l] == id) return fail(c, BPM_EINVAL, "bpm_string_reparam: an image appears twice");
    const int s = c->slot_of[id];
    if (mi >= 0 && c->slot_group[s] != mi)
      return fail(c, BPM_EINVAL, "bpm_string_reparam: the images must share one mesh group");
    mi = c->slot_group[s];
    const size_t off = (size_t)c->slot_local[s] * 3 * c->meshes[mi]->n;
    im.p[k] = c->run_precision == 64 ? (const void*)(reinterpret_cast<const double*>(c->group_m[mi]) + off)
                                     : (const void*)(reinterpret_cast<const float*>(c->group_m[mi]) + off);
  }
  const long n = c->meshes[mi]->n;
  HIPCHK(c, hipSetDevice(c->device));
  double *d_dist = nullptr, *d_out = nullptr;
  HIPCHK(c, hipMalloc(&d_dist, sizeof(double) * P));
  hipError_t e = hipMalloc(&d_out, sizeof(double) * 3 * n * P);
  if (e == hipSuccess) e = string_reparam_device(c->run_precision, n, P, im, d_dist, d_out, c->own_stream);
  std::vector<double> h_out, h_d(P - 1);
  if (e == hipSuccess) {
    h_out.resize((size_t)3 * n * P);
    e = hipMemcpyAsync(h_out.data(), d_out, sizeof(double) * h_out.size(), hipMemcpyDeviceToHost, c->own_stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_d.data(), d_dist, sizeof(double) * (P - 1), hipMemcpyDeviceToHost, c->own_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->own_stream);
  hipFree(d_dist);
  if (d_out) hipFree(d_out);
  HIPCHK(c, e);
  for (int k = 0; k < P; ++k) {
    Instance& I = c->insts[ids[k]];
    I.m0.assign(h_out.begin() + (size_t)k * 3 * n, h_out.begin() + (size_t)(k + 1) * 3 * n);
  }
  if (arclen) {
    arclen[0] = 0.0;
    for (int k = 1; k < P; ++k) arclen[k] = arclen[k - 1] + h_d[k - 1];
  }
  return BPM_OK;
}

int bpm_gp_ei(bpm_ctx* c, const bpm_gp* gp, int64_t m, double* cand, uint64_t seed, double* yhat, double* s,
              double* ei, void* hip_stream) {
  if (!c) return BPM_EINVAL;
  if (!gp || !ei || !cand || m < 0) return fail(c, BPM_EINVAL, "bpm_gp_ei: null argument or negative count");
  if (gp->d < 1 || gp->d > kMaxGpDim || gp->n < 1 || !gp->X || !gp->theta || !gp->G)
    return fail(c, BPM_EINVAL, "bpm_gp_ei: need 1 <= d <= 16, n >= 1 and the model arrays");
  if (!(gp->c > 0.0) || !(gp->sigma2 >= 0.0) || !std::isfinite(gp->mu) || !std::isfinite(gp->f_min))
    return fail(c, BPM_EINVAL, "bpm_gp_ei: need c > 0, sigma2 >= 0 and finite mu, f_min");
  HIPCHK(c, hipSetDevice(c->device));
  GpArgs a{gp->n, gp->d, gp->mu, gp->sigma2, gp->c, gp->f_min, gp->X, gp->theta, gp->G};
  hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->own_stream;
  HIPCHK(c, gp_ei_device(a, (long)m, cand, seed, yhat, s, ei, st));
  return BPM_OK;
}

int bpm_argmax(bpm_ctx* c, const double* v, int64_t m, int64_t* idx, void* hip_stream) {
  if (!c) return BPM_EINVAL;
  if (!v || !idx || m < 1) return fail(c, BPM_EINVAL, "bpm_argmax: need m >= 1 and device arrays");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->own_stream;
  const int nb = argmax_blocks((long)m);
  double* bv = nullptr;
  long* bi = nullptr;
  HIPCHK(c, hipMallocAsync(reinterpret_cast<void**>(&bv), sizeof(double) * nb, st));
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&bi), sizeof(long) * nb, st);
  if (e == hipSuccess) e = argmax_device(v, (long)m, bv, bi, idx, st);
  hipFreeAsync(bv, st);
  if (bi) hipFreeAsync(bi, st);
  HIPCHK(c, e);
  return BPM_OK;
}

int bpm_last_run_info(bpm_ctx* c, double* kernel_ms, int32_t* grid, int32_t* wg_per_group) {
  if (!c) return BPM_EINVAL;
  if (kernel_ms) *kernel_ms = c->kernel_ms;
  if (grid) *grid = c->run_grid;
  if (wg_per_group) *wg_per_group = c->run_G;
  return BPM_OK;
}

int bpm_last_run_layout(bpm_ctx* c, int32_t* threads_per_wg, int32_t* s_rows_lds, int32_t* csr_cap_lds,
                        int32_t* rhs_block, int64_t* lds_bytes) {
  if (!c) return BPM_EINVAL;
  if (threads_per_wg) *threads_per_wg = c->run_bs;
  if (s_rows_lds) *s_rows_lds = c->run_plan.s_rows;
  if (csr_cap_lds) *csr_cap_lds = c->run_plan.csr_cap;
  if (rhs_block) *rhs_block = c->run_RB;
  if (lds_bytes) *lds_bytes = c->run_precision == 64 ? (int64_t)dp5_lds_bytes<double>(c->run_plan)
                                                     : (int64_t)dp5_lds_bytes<float>(c->run_plan);
  return BPM_OK;
}

}  // extern "C"

// ===========================================================================================
// Surrogate MLP and screening
// ===========================================================================================
struct bpm_mlp {
  bpm_ctx* ctx = nullptr;
  bpm::Mlp net;
  bpm::ScreenScratch sc;
  bpm::Arena arena;
};

extern "C" {

int bpm_mlp_num_params(void) { return (int)kMlpParams; }

int bpm_mlp_create(bpm_ctx* c, int32_t max_batch, const float* theta, bpm_mlp** out) {
  if (!c) return BPM_EINVAL;
  if (!out || max_batch <= 0) return fail(c, BPM_EINVAL, "bpm_mlp_create: bad argument");
  hipSetDevice(c->device);
  auto* M = new bpm_mlp();
  M->ctx = c;
  Mlp& n = M->net;
  n.max_batch = max_batch;
  Arena& A = M->arena;
  const long B = max_batch;
  hipError_t e = hipSuccess;
  auto al = [&](auto** p, size_t cnt) {
    if (e == hipSuccess) e = A.alloc(p, cnt);
  };
  al(&n.theta, kMlpParams); al(&n.m, kMlpParams); al(&n.v, kMlpParams); al(&n.grad, kMlpParams);
  for (int l = 0; l < 5; ++l) al(&n.Z[l], B * mlp_size(l + 1));
  for (int l = 0; l < 4; ++l) al(&n.Aout[l], B * kMlpHidden);
  al(&n.dZ, B * kMlpOut); al(&n.dA, B * kMlpHidden); al(&n.dZh, B * kMlpHidden); al(&n.dZh2, B * kMlpHidden);
  al(&n.d_loss, 1);
  const int kp[5] = {32, 256, 256, 256, 256}, op[5] = {256, 256, 256, 256, 16};
  for (int l = 0; l < 5; ++l) {
    al(&n.dev.w[l], (size_t)kp[l] * op[l]);
    al(&n.dev.b[l], (size_t)op[l]);
  }
  if (e != hipSuccess) {
    delete M;
    return fail(c, BPM_ENOMEM, std::string("bpm_mlp_create: ") + hipGetErrorString(e));
  }
  hipMemset(n.m, 0, sizeof(float) * kMlpParams);
  hipMemset(n.v, 0, sizeof(float) * kMlpParams);
  if (theta) hipMemcpy(n.theta, theta, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
  else hipMemset(n.theta, 0, sizeof(float) * kMlpParams);
  mlp_pack(n, c->own_stream);
  if ((e = hipStreamSynchronize(c->own_stream)) != hipSuccess) {
    delete M;
    return fail(c, BPM_EHIP, std::string("bpm_mlp_create: ") + hipGetErrorString(e));
  }
  *out = M;
  return BPM_OK;
}

void bpm_mlp_destroy(bpm_mlp* M) {
  if (!M) return;
  hipSetDevice(M->ctx->device);
  hipDeviceSynchronize();
  if (M->sc.hist) hipFree(M->sc.hist);
  if (M->sc.state) hipFree(M->sc.state);
  if (M->sc.cand) hipFree(M->sc.cand);
  if (M->sc.blk) hipFree(M->sc.blk);
  delete M;
}

int bpm_mlp_set_params(bpm_mlp* M, const float* theta) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!theta) return fail(c, BPM_EINVAL, "bpm_mlp_set_params: null");
  hipSetDevice(c->device);
  HIPCHK(c, hipMemcpy(M->net.theta, theta, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(M->net.m, 0, sizeof(float) * kMlpParams));
  HIPCHK(c, hipMemset(M->net.v, 0, sizeof(float) * kMlpParams));
  M->net.step = 0;
  HIPCHK(c, mlp_pack(M->net, c->own_stream));
  HIPCHK(c, hipStreamSynchronize(c->own_stream));
  return BPM_OK;
}

int bpm_mlp_get_params(bpm_mlp* M, float* theta) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!theta) return fail(c, BPM_EINVAL, "bpm_mlp_get_params: null");
  hipSetDevice(c->device);
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, hipMemcpy(theta, M->net.theta, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return BPM_OK;
}

int bpm_mlp_predict(bpm_mlp* M, const float* X, float* Y, int64_t n, void* stream) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (n < 0 || (n > 0 && (!X || !Y))) return fail(c, BPM_EINVAL, "bpm_mlp_predict: bad argument");
  hipSetDevice(c->device);
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, mlp_predict(M->net, X, Y, (long)n, s));
  return BPM_OK;
}

int bpm_mlp_grads(bpm_mlp* M, const float* X, const float* T, const uint8_t* mask, int32_t batch, float* loss,
                  float* grads) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!X || !T || !mask || batch <= 0 || batch > M->net.max_batch) return fail(c, BPM_EINVAL, "bpm_mlp_grads: bad argument");
  hipSetDevice(c->device);
  HIPCHK(c, mlp_forward_backward(M->net, X, T, mask, batch, c->own_stream));
  HIPCHK(c, hipStreamSynchronize(c->own_stream));
  if (loss) {
    double l = 0;
    HIPCHK(c, hipMemcpy(&l, M->net.d_loss, sizeof(double), hipMemcpyDeviceToHost));
    *loss = (float)l;
  }
  if (grads) HIPCHK(c, hipMemcpy(grads, M->net.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return BPM_OK;
}

int bpm_mlp_train_step(bpm_mlp* M, const float* X, const float* T, const uint8_t* mask, int32_t batch, float lr,
                       float* loss, void* stream) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!X || !T || !mask || batch <= 0 || batch > M->net.max_batch || !(lr > 0.f))
    return fail(c, BPM_EINVAL, "bpm_mlp_train_step: bad argument");
  hipSetDevice(c->device);
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, mlp_forward_backward(M->net, X, T, mask, batch, s));
  HIPCHK(c, mlp_adam(M->net, lr, s));
  if (loss) {
    double l = 0;
    HIPCHK(c, hipMemcpyAsync(&l, M->net.d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *loss = (float)l;
  }
  return BPM_OK;
}

int bpm_sample_designs(bpm_ctx* c, uint64_t seed, int64_t n, float* X, void* stream) {
  if (!c) return BPM_EINVAL;
  if (n < 0 || (n > 0 && !X)) return fail(c, BPM_EINVAL, "bpm_sample_designs: bad argument");
  hipSetDevice(c->device);
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, sample_designs(seed, (long)n, X, s));
  return BPM_OK;
}

int bpm_topk(bpm_mlp* M, const float* score, int64_t n, int64_t k, int64_t* idx, void* stream) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!score || !idx || n <= 0 || n > 0x7fffffffLL || k <= 0 || k > n || k > kTopkMax)
    return fail(c, BPM_EINVAL, "bpm_topk: need 0 < k <= min(n, 16384), n < 2^31");
  hipSetDevice(c->device);
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, topk_select(score, (long)n, (long)k, idx, M->sc, s));
  return BPM_OK;
}

int bpm_topk_noalloc(bpm_ctx* c, const float* score, int64_t n, int64_t k, int64_t* idx, void* stream) {
  if (!c) return BPM_EINVAL;
  if (!score || !idx || n <= 0 || k <= 0 || k > n || k > kTopkMax)
    return fail(c, BPM_EINVAL, "bpm_topk_noalloc: need 0 < k <= min(n, 16384)");
  if (n > kTopkNoAllocMaxN)
    return fail(c, BPM_EINVAL, "bpm_topk_noalloc: n exceeds the " + std::to_string(kTopkNoAllocMaxN) +
                                   " scores its fixed scratch area holds (use bpm_topk)");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, topk_select_noalloc(score, (long)n, (long)k, idx, c->device, s));
  return BPM_OK;
}

int bpm_screen(bpm_mlp* M, uint64_t seed, int64_t n, int64_t k, const double* lo, const double* hi,
               double min_stability, float* X, float* Y, float* score, int64_t* idx, void* stream) {
  if (!M) return BPM_EINVAL;
  bpm_ctx* c = M->ctx;
  if (!lo || !hi || !X || !Y || !score || !idx || n <= 0 || n > 0x7fffffffLL || k <= 0 || k > n || k > kTopkMax)
    return fail(c, BPM_EINVAL, "bpm_screen: bad argument");
  for (int f = 0; f < 12; ++f)
    if (!(hi[f] > lo[f]) || !std::isfinite(lo[f]) || !std::isfinite(hi[f]))
      return fail(c, BPM_EINVAL, "bpm_screen: every range needs finite lo < hi");
  hipSetDevice(c->device);
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : c->own_stream;
  HIPCHK(c, sample_designs(seed, (long)n, X, s));
  HIPCHK(c, design_features(X, (long)n, lo, hi, s));
  HIPCHK(c, mlp_predict(M->net, X, Y, (long)n, s));
  HIPCHK(c, screen_score(X, Y, (long)n, lo, hi, min_stability, score, s));
  HIPCHK(c, topk_select(score, (long)n, (long)k, idx, M->sc, s));
  return BPM_OK;
}

}  // extern "C"
