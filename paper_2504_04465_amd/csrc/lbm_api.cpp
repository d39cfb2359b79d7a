// lbm_api.cpp -- the C-ABI of liblbm.so: context, grid upload, the level
// scheduler of Sec. 4.5 (asynchronous time stepping, coarsest level first,
// coupling before collide-and-stream) and the synchronous read-backs.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "grid_builder.h"
#include "grid_device.h"
#include "lattice.h"
#include "layout.h"
#include "lbm.h"
#include "mlp_ops.h"
#include "ops.h"

#include <random>

#include "remesh.h"

using namespace lbm;

struct ProfSlot {
  hipEvent_t a, b;
  int level;
};

struct lbm_ctx {
  lbm_params p{};
  std::string err;
  hipStream_t stream = nullptr;
  lbm_dev_alloc_fn dalloc = nullptr;
  lbm_dev_free_fn dfree = nullptr;
  void *actx = nullptr;
  LatticeInfo lat{};
  Ops ops{};
  bool ddf = false, lamf = false;
  // grid
  bool have_grid = false;
  bool device_build = true;  // build grids and layouts on the GPU (not for host-only contexts)
  int32_t *d_gslot = nullptr;  // in place: slot -> staging slot (see stage)
  int32_t *d_bc_row = nullptr; // in place: exception row of each boundary-layer cell
  DeviceGridArrays dg;         // canonical tables kept on the device by the device grid build
  std::vector<int32_t> stage;  // in place: slot -> staging slot (coarse ghosts, boundary sources), or -1
  // the last device build's inputs: the canonical neighbour list is not
  // kept on the device (the bulk pulls do not use it); an export of it
  // builds the grid again
  struct BuildInputs {
    int dim = 0, L = 0;
    int32_t ext[3] = {1, 1, 1};
    std::vector<std::vector<uint8_t>> rdata, sdata;
    std::vector<MaskView> rv, sv;
    bool has_solid = false;
    FaceSpec fs[6];
    bool periodic[3] = {false, false, false};
  } bi;
  HostGrid g;
  DeviceLayout lay;
  lbm_face_bc face[6]{};
  int dim = 0, L = 0;
  double tau[8]{};
  double bpu[8]{};  // algorithmic bytes per cell update of the collide kernel, per level
  int64_t N = 0, NS = 0, Ng = 0, stride = 0;  // cells, slots, coarse ghosts, slots per population buffer
  // device
  std::vector<void *> allocs;
  void *f[2]{}, *gb[2]{};
  int32_t *d_nbrick = nullptr, *d_xbase = nullptr, *d_xnbr = nullptr;
  double *d_xdu = nullptr;  // xi_i . inflow noise per explicit row [Q-1][xstride], or null
  uint64_t *d_xmask = nullptr, *d_xreg = nullptr;
  int32_t *d_cell_of = nullptr, *d_slot_of = nullptr, *d_crow = nullptr;
  uint8_t *d_flags = nullptr;
  double *d_sigma = nullptr, *d_rhoinf = nullptr;
  double *d_sums_static = nullptr;     // this GPU's static partials array
  hipError_t sums_static_err = hipSuccess;  // its address lookup at creation
  void *d_lam = nullptr;   // multipliers: FP64 with FP64 storage, else FP32
  int lam_bytes = 4;
  int32_t *d_ghost = nullptr, *d_child = nullptr;
  uint64_t *d_unknown = nullptr;
  int32_t *d_bc_cell = nullptr, *d_bc_src = nullptr;
  int8_t *d_bc_face = nullptr;
  unsigned long long *d_counters = nullptr;
  double *d_scratch = nullptr;
  size_t scratch_bytes = 0;
  int parity[8]{};
  bool pre[8]{};
  bool have_state = false;
  int64_t updates[8]{};
  int64_t coarse_steps = 0;
  // multiplier surrogate
  float *d_mlp_w = nullptr, *d_mlp_m = nullptr, *d_mlp_v = nullptr, *d_mlp_g = nullptr;
  void *d_mlp_ops = nullptr;
  float *d_mlp_loss = nullptr;
  bool have_mlp = false;
  // graph replay of two coarse steps (launch-bound grids)
  bool use_graphs = false;
  // one collide launch for all levels active at a substep (on by default
  // where the model has it)
  bool fuse_levels = true;
  hipGraphExec_t gexec = nullptr;
  int gparity[8]{};
  // profiling
  bool prof = false;
  std::vector<ProfSlot> slots;
  std::vector<hipEvent_t> pool;
  int64_t prof_launches[8]{};
  double prof_ms[8]{};
};

namespace {

lbm_status set_err(lbm_ctx *c, lbm_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                               \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_err(ctx, LBM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

void *dev_alloc(lbm_ctx *c, size_t bytes) {
  void *p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (c->dalloc) {
    p = c->dalloc(bytes, c->actx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}

void drop_graph(lbm_ctx *c) {
  if (c->gexec) {
    hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
}

void free_device(lbm_ctx *c) {
  if (c->p.host_only) return;
  drop_graph(c);
  if (!c->allocs.empty()) hipStreamSynchronize(c->stream);
  for (void *p : c->allocs) {
    if (c->dfree) c->dfree(p, c->actx);
    else hipFree(p);
  }
  c->allocs.clear();
  c->f[0] = c->f[1] = c->gb[0] = c->gb[1] = nullptr;
  c->d_nbrick = c->d_xbase = c->d_xnbr = nullptr;
  c->d_xdu = nullptr;
  c->d_xmask = c->d_xreg = nullptr;
  c->d_cell_of = c->d_slot_of = c->d_crow = nullptr;
  c->d_flags = nullptr;
  c->d_gslot = nullptr;
  c->d_bc_row = nullptr;
  c->dg = DeviceGridArrays();
  c->d_sigma = c->d_rhoinf = nullptr;
  c->d_lam = nullptr;
  c->d_ghost = c->d_child = nullptr;
  c->d_unknown = nullptr;
  c->d_bc_cell = c->d_bc_src = nullptr;
  c->d_bc_face = nullptr;
  c->d_counters = nullptr;
  c->d_scratch = nullptr;
  c->scratch_bytes = 0;
  c->d_mlp_w = c->d_mlp_m = c->d_mlp_v = c->d_mlp_g = c->d_mlp_loss = nullptr;
  c->d_mlp_ops = nullptr;
  c->have_mlp = false;
}

void dev_release(lbm_ctx *c, void *p) {
  if (!p) return;
  hipStreamSynchronize(c->stream);
  for (size_t k = 0; k < c->allocs.size(); ++k)
    if (c->allocs[k] == p) {
      c->allocs.erase(c->allocs.begin() + k);
      break;
    }
  if (c->dfree) c->dfree(p, c->actx);
  else hipFree(p);
}

// Device buffers of one call: every buffer taken through take() is released
// when the call returns, on its error paths as on success.
struct CallBuffers {
  lbm_ctx *c;
  std::vector<void *> held;
  explicit CallBuffers(lbm_ctx *ctx) : c(ctx) {}
  CallBuffers(const CallBuffers &) = delete;
  CallBuffers &operator=(const CallBuffers &) = delete;
  void *take(size_t bytes) {
    void *p = dev_alloc(c, bytes);
    if (p) held.push_back(p);
    return p;
  }
  ~CallBuffers() {
    for (void *p : held) dev_release(c, p);
  }
};

template <class T>
lbm_status upload(lbm_ctx *c, T **dst, const T *src, size_t count) {
  *dst = (T *)dev_alloc(c, count * sizeof(T));
  if (!*dst) return set_err(c, LBM_E_NOMEM, "device allocation failed");
  if (count) HIP_TRY(c, hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return LBM_OK;
}

PhysArgs phys(const lbm_ctx *c, int l) {
  PhysArgs ph{};
  ph.tau = c->tau[l];
  ph.omega = 1.0 / c->tau[l];
  ph.krr = 1.0 - 1.0 / c->tau[l];
  ph.cs2w = c->ddf ? c->p.T0 : c->lat.cs2;
  for (int k = 0; k < 6; ++k)
    for (int d = 0; d < 3; ++d)
      ph.uw[k][d] = c->face[k].kind == LBM_BC_MOVING_WALL ? c->face[k].u[d] : 0.0;
  ph.Cv = 1.0 / (c->p.gamma - 1.0);
  ph.sensor_A = c->p.sensor_A;
  ph.sensor_on = c->p.sensor_on;
  ph.trace_eq = c->p.trace_equilibration;
  ph.newton_tol = c->p.newton_tol;
  ph.fallback_tol = c->p.fallback_tol;
  ph.newton_max_it = c->p.newton_max_it;
  ph.warm = c->p.lambda_warm_start;
  ph.mlp = c->d_mlp_ops;
  return ph;
}

const void *fbuf(const lbm_ctx *c, int l) { return c->f[c->parity[l]]; }
const void *gbuf(const lbm_ctx *c, int l) { return c->gb[c->parity[l]]; }

Topo topo(const lbm_ctx *c) {
  Topo t{};
  t.nbrick = c->d_nbrick;
  t.xmask = c->d_xmask;
  t.xbase = c->d_xbase;
  t.xnbr = c->d_xnbr;
  t.xreg = c->d_xreg;
  t.xstride = c->lay.xstride;
  t.xdu = c->d_xdu;
  t.off32 = (double)c->ops.sizeof_storage * c->lat.Q * (double)c->stride < 4294967296.0;
  return t;
}

bool read_pre(const lbm_ctx *c, int l);

void launch_coalesce(lbm_ctx *c, int l) {
  const int64_t cnt = c->g.goff[l + 1] - c->g.goff[l];
  if (cnt <= 0) return;
  CArgs a{};
  a.fin_child = fbuf(c, l + 1);
  a.gin_child = gbuf(c, l + 1);
  a.fout_coarse = const_cast<void *>(fbuf(c, l));
  a.gout_coarse = const_cast<void *>(gbuf(c, l));
  a.lam = c->d_lam;
  a.stride = c->stride;
  a.vbase = c->NS;
  a.xnbr = c->d_xnbr;
  a.xstride = c->lay.xstride;
  a.xdu = c->d_xdu;
  a.child = c->d_child;
  a.crow = c->d_crow;
  a.unknown = c->d_unknown;
  a.ghost_cell = c->d_ghost;
  a.g0 = c->g.goff[l];
  a.count = cnt;
  PhysArgs ph = phys(c, l);
  a.cs2w = ph.cs2w;
  memcpy(a.uw, ph.uw, sizeof a.uw);
  a.aa = c->p.in_place && c->parity[l + 1] == 1 ? 2 : 0;
  a.swap = c->p.in_place && c->parity[l] == 1 ? 1 : 0;
  c->ops.coalesce(a, read_pre(c, l + 1), c->stream);
}

void launch_explode(lbm_ctx *c, int l) {
  const int64_t cnt = c->g.goff[l + 1] - c->g.goff[l];
  if (cnt <= 0) return;
  EArgs a{};
  a.fin_coarse = fbuf(c, l);
  a.fout_fine = const_cast<void *>(fbuf(c, l + 1));
  a.gin_coarse = gbuf(c, l);
  a.gout_fine = const_cast<void *>(gbuf(c, l + 1));
  a.lam = c->d_lam;
  a.stride = c->stride;
  a.child = c->d_child;
  a.ghost_cell = c->d_ghost;
  a.g0 = c->g.goff[l];
  a.count = cnt;
  if (c->p.in_place) {
    // the fine level has just stepped: odd phase, rows swapped
    a.mode = c->parity[l + 1] == 1 ? 1 : 2;
    a.vbase = c->NS;
    a.xnbr = c->d_xnbr;
    a.xstride = c->lay.xstride;
    a.crow = c->d_crow;
    const PhysArgs ph = phys(c, l + 1);
    a.cs2w = ph.cs2w;
    memcpy(a.uw, ph.uw, sizeof a.uw);
  }
  c->ops.explode(a, c->stream);
}

FaceVals face_vals(const lbm_ctx *c) {
  FaceVals fv{};
  for (int k = 0; k < 6; ++k) {
    fv.rho[k] = c->face[k].rho;
    fv.T[k] = c->face[k].T;
    for (int d = 0; d < 3; ++d) fv.u[k][d] = c->face[k].u[d];
    fv.extrap[k] = c->face[k].kind == LBM_BC_EQUILIBRIUM ? (c->face[k].extrapolate_rho ? 1 : 0) : -1;
  }
  return fv;
}

void launch_bcfill(lbm_ctx *c, int l) {
  const int64_t cnt = c->g.boff[l + 1] - c->g.boff[l];
  if (cnt <= 0) return;
  BArgs a{};
  a.f = const_cast<void *>(fbuf(c, l));
  a.g = const_cast<void *>(gbuf(c, l));
  a.lam = c->d_lam;
  a.stride = c->stride;
  a.bc_cell = c->d_bc_cell;
  a.bc_src = c->d_bc_src;
  a.bc_face = c->d_bc_face;
  a.b0 = c->g.boff[l];
  a.count = cnt;
  a.fv = face_vals(c);
  a.ph = phys(c, l);
  a.counters = c->d_counters;
  if (c->p.in_place) {
    // the level has just stepped: odd phase, rows swapped
    a.mode = c->parity[l] == 1 ? 1 : 2;
    a.stage = c->d_gslot;
    a.bc_row = c->d_bc_row;
    a.xnbr = c->d_xnbr;
    a.xstride = c->lay.xstride;
  }
  c->ops.bcfill(a, c->stream);
}

hipEvent_t take_event(lbm_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// argument block of level l's collide reading buffer par
KArgs collide_args(lbm_ctx *c, int l, int par) {
  KArgs a{};
  a.fin = c->f[par];
  a.fout = c->f[1 - par];
  a.gin = c->gb[par];
  a.gout = c->gb[1 - par];
  a.stride = c->stride;
  a.vbase = c->NS;
  a.topo = topo(c);
  a.flags = c->d_flags;
  a.sigma = c->d_sigma;
  a.rho_inf = c->d_rhoinf;
  a.lam = c->d_lam;
  a.begin = c->lay.soff[l];
  a.count = c->lay.soff[l + 1] - c->lay.soff[l];
  a.ph = phys(c, l);
  a.counters = c->d_counters;
  a.gslot = c->d_gslot;
  return a;
}

void launch_collide(lbm_ctx *c, int l) {
  const int64_t cnt = c->lay.soff[l + 1] - c->lay.soff[l];
  if (cnt > 0) {
    KArgs a = collide_args(c, l, c->parity[l]);
    ProfSlot slot{};
    if (c->prof) {
      slot.a = take_event(c);
      slot.b = take_event(c);
      slot.level = l;
      hipEventRecord(slot.a, c->stream);
    }
    // in place, a level's phase is the parity of its step count: even, its
    // own rows hold the streamed populations; odd, the post-collision ones
    // sit swapped in the rows of their opposites
    if (c->p.in_place) a.aa = c->parity[l] == 0 ? 1 : 2;
    c->ops.collide(a, c->pre[l], c->stream);
    if (c->prof) {
      hipEventRecord(slot.b, c->stream);
      c->slots.push_back(slot);
    }
    c->updates[l] += c->g.off[l + 1] - c->g.off[l];
  }
  c->parity[l] ^= 1;
  c->pre[l] = false;
}

lbm_status check_launch(lbm_ctx *c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, LBM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return LBM_OK;
}

// the counters, summed over their copies
lbm_status read_counters(lbm_ctx *c, unsigned long long *out) {
  std::vector<unsigned long long> h((size_t)CNT_COUNT * CNT_COPIES);
  HIP_TRY(c, hipMemcpyAsync(h.data(), c->d_counters, h.size() * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < CNT_COUNT; ++k) out[k] = 0;
  for (size_t j = 0; j < h.size(); ++j) out[j % CNT_COUNT] += h[j];
  return LBM_OK;
}

lbm_status numeric_check(lbm_ctx *c) {
  unsigned long long cnt[CNT_COUNT];
  lbm_status s = read_counters(c, cnt);
  if (s != LBM_OK) return s;
  if (cnt[CNT_NEWTON_FAIL] || cnt[CNT_NONFINITE]) {
    char buf[160];
    snprintf(buf, sizeof buf, "numerical failure: %llu Newton failures, %llu non-finite cells",
             cnt[CNT_NEWTON_FAIL], cnt[CNT_NONFINITE]);
    return set_err(c, LBM_E_NUMERIC, buf);
  }
  return LBM_OK;
}

double *scratch(lbm_ctx *c, size_t bytes) {
  if (c->scratch_bytes < bytes) {
    // the old buffer goes back to the allocator before the larger one is taken
    dev_release(c, c->d_scratch);
    c->d_scratch = nullptr;
    c->scratch_bytes = 0;
    c->d_scratch = (double *)dev_alloc(c, bytes);
    c->scratch_bytes = c->d_scratch ? bytes : 0;
  }
  return c->d_scratch;
}

// coalesced slots of every coarse ghost, for read-backs of the sync state
void coalesce_all(lbm_ctx *c) {
  for (int l = 0; l + 1 < c->L; ++l) launch_coalesce(c, l);
}

// readers of the synchronisation-point state: own rows (pre-collision at
// start, or the in-place buffer after an odd step), or swapped pulls
bool read_pre(const lbm_ctx *c, int l) { return c->pre[l] || (c->p.in_place && c->parity[l] == 0); }

MArgs gather_args(lbm_ctx *c, int l, int mode) {
  MArgs a{};
  a.aa = c->p.in_place && c->parity[l] == 1 ? 2 : 0;
  a.fin = fbuf(c, l);
  a.gin = gbuf(c, l);
  a.lam = c->d_lam;
  a.stride = c->stride;
  a.vbase = c->NS;
  a.topo = topo(c);
  a.flags = c->d_flags;
  a.cell_of = c->d_cell_of;
  a.begin = c->lay.soff[l];
  a.count = c->lay.soff[l + 1] - c->lay.soff[l];
  PhysArgs ph = phys(c, l);
  a.cs2w = ph.cs2w;
  memcpy(a.uw, ph.uw, sizeof a.uw);
  a.Cv = ph.Cv;
  a.mode = mode;
  a.n = c->N;
  a.vol = std::ldexp(1.0, -c->dim * l);
  return a;
}

int n_mom(const lbm_ctx *c) { return 1 + c->lat.D + (c->ddf ? 1 : 0); }

lbm_status need_state(lbm_ctx *c) {
  if (!c) return LBM_E_ARG;
  if (c->p.host_only) return set_err(c, LBM_E_STATE, "context is host-only");
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  if (!c->have_state) return set_err(c, LBM_E_STATE, "not initialised");
  return LBM_OK;
}

lbm_status mlp_ensure(lbm_ctx *c) {
  if (c->p.host_only) return set_err(c, LBM_E_STATE, "context is host-only");
  if (c->lat.kind != LAT_D2Q21) return set_err(c, LBM_E_ARG, "the multiplier surrogate needs a D2Q21 context");
  if (c->d_mlp_w) return LBM_OK;
  c->d_mlp_w = (float *)dev_alloc(c, sizeof(float) * MLP_PARAMS);
  c->d_mlp_m = (float *)dev_alloc(c, sizeof(float) * MLP_PARAMS);
  c->d_mlp_v = (float *)dev_alloc(c, sizeof(float) * MLP_PARAMS);
  c->d_mlp_g = (float *)dev_alloc(c, sizeof(float) * MLP_PARAMS);
  c->d_mlp_loss = (float *)dev_alloc(c, sizeof(float) * 64);
  c->d_mlp_ops = dev_alloc(c, mlp_operands_bytes());
  if (!c->d_mlp_w || !c->d_mlp_m || !c->d_mlp_v || !c->d_mlp_g || !c->d_mlp_ops || !c->d_mlp_loss)
    return set_err(c, LBM_E_NOMEM, "surrogate allocation failed");
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_ops, 0, mlp_operands_bytes(), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_m, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_v, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_g, 0, sizeof(float) * MLP_PARAMS, c->stream));
  return LBM_OK;
}

lbm_status mlp_upload_weights(lbm_ctx *c, const float *w) {
  HIP_TRY(c, hipMemcpyAsync(c->d_mlp_w, w, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, c->stream));
  mlp_operands(c->d_mlp_w, c->d_mlp_ops, c->stream);
  lbm_status s = check_launch(c);
  if (s != LBM_OK) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->have_mlp = true;
  return LBM_OK;
}

// temporaries of the device grid build, through the context's allocator
void *build_alloc(size_t bytes, void *ctx) { return dev_alloc((lbm_ctx *)ctx, bytes); }
void build_release(void *p, void *ctx) { dev_release((lbm_ctx *)ctx, p); }

}  // namespace

extern "C" {

lbm_status lbm_create(const lbm_params *params, lbm_dev_alloc_fn dev_alloc_fn,
                      lbm_dev_free_fn dev_free_fn, void *alloc_ctx, void *hip_stream,
                      lbm_ctx **out) {
  if (!params || !out) return LBM_E_ARG;
  *out = nullptr;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_E_NOMEM;
  c->p = *params;
  c->stream = (hipStream_t)hip_stream;
  c->dalloc = dev_alloc_fn;
  c->dfree = dev_free_fn;
  c->actx = alloc_ctx;
  const int lat = params->lattice, coll = params->collision, sto = params->storage;
  if (!get_lattice_info(lat, &c->lat) || coll < 0 || coll > 5 || sto < 0 || sto > 2) {
    delete c;
    return LBM_E_ARG;
  }
  bool ok = false;
  switch (lat) {
    case LBM_D2Q9: ok = get_ops_d2q9(coll, sto, &c->ops); break;
    case LBM_D3Q27: ok = get_ops_d3q27(coll, sto, &c->ops); break;
    case LBM_D2Q21: ok = get_ops_d2q21(coll, sto, &c->ops); break;
    case LBM_D2Q37: ok = get_ops_d2q37(coll, sto, &c->ops); break;
    case LBM_D2Q13: ok = get_ops_d2q13(coll, sto, &c->ops); break;
  }
  if (!ok) {
    delete c;
    return LBM_E_UNSUPPORTED;
  }
  if (coll >= LBM_DDF_POLY && !(params->gamma > 1.0)) {
    delete c;
    return LBM_E_ARG;
  }
  c->ddf = coll >= LBM_DDF_POLY;
  c->lamf = coll >= LBM_DDF_NEWTON;
  c->lam_bytes = c->p.storage == LBM_FP64 ? 8 : 4;
  // address of the current GPU's static partials array (allocation-free sums)
  if (!c->p.host_only) c->sums_static_err = sums_scratch(&c->d_sums_static);
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  free_device(c);
  for (auto &s : c->slots) {
    hipEventDestroy(s.a);
    hipEventDestroy(s.b);
  }
  for (auto e : c->pool) hipEventDestroy(e);
  delete c;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

lbm_status lbm_set_device_build(lbm_ctx *c, int on) {
  if (!c) return LBM_E_ARG;
  c->device_build = on != 0;
  return LBM_OK;
}

lbm_status lbm_grid_build(lbm_ctx *c, int dim, const int32_t ext[3], int n_levels,
                          const lbm_mask *refine, const lbm_mask *solid,
                          const lbm_face_bc faces[6]) {
  if (!c || !ext || !faces || n_levels < 1 || n_levels > 8) return set_err(c, LBM_E_ARG, "bad arguments");
  if (n_levels > 1 && !refine) return set_err(c, LBM_E_ARG, "refine masks missing");
  free_device(c);
  c->have_grid = false;
  c->have_state = false;
  std::vector<MaskView> rv(std::max(1, n_levels - 1)), sv(n_levels);
  for (int l = 0; l + 1 < n_levels; ++l) {
    rv[l].data = refine[l].data;
    for (int a = 0; a < 3; ++a) {
      rv[l].lo[a] = refine[l].lo[a];
      rv[l].n[a] = a < dim ? refine[l].n[a] : (refine[l].data ? 1 : 0);
    }
  }
  for (int l = 0; solid && l < n_levels; ++l) {
    sv[l].data = solid[l].data;
    for (int a = 0; a < 3; ++a) {
      sv[l].lo[a] = solid[l].lo[a];
      sv[l].n[a] = a < dim ? solid[l].n[a] : (solid[l].data ? 1 : 0);
    }
  }
  FaceSpec fs[6];
  for (int k = 0; k < 6; ++k) {
    c->face[k] = faces[k];
    fs[k].kind = faces[k].kind;
    fs[k].rho = faces[k].rho;
    for (int d = 0; d < 3; ++d) fs[k].u[d] = faces[k].u[d];
    fs[k].T = faces[k].T;
    fs[k].extrapolate_rho = faces[k].extrapolate_rho;
    fs[k].sponge_sigma_max = faces[k].sponge_sigma_max;
    fs[k].sponge_width = faces[k].sponge_width;
  }
  std::string err;
  bool periodic[3];
  for (int a = 0; a < 3; ++a)
    periodic[a] = a < dim && faces[2 * a].kind == LBM_BC_PERIODIC && faces[2 * a + 1].kind == LBM_BC_PERIODIC;
  const bool on_device = c->device_build && !c->p.host_only;
  if (on_device) {
    // the tree and its layout built on the GPU, copied into c->g / c->lay
    auto &bi = c->bi;
    bi.dim = dim;
    bi.L = n_levels;
    for (int a = 0; a < 3; ++a) bi.ext[a] = ext[a];
    bi.rdata.assign(rv.size(), {});
    bi.sdata.assign(sv.size(), {});
    bi.rv = rv;
    bi.sv = sv;
    bi.has_solid = solid != nullptr;
    for (size_t l = 0; l < rv.size(); ++l)
      if (rv[l].data) {
        bi.rdata[l].assign(rv[l].data, rv[l].data + (size_t)rv[l].n[0] * rv[l].n[1] * rv[l].n[2]);
        bi.rv[l].data = bi.rdata[l].data();
      }
    for (size_t l = 0; l < sv.size(); ++l)
      if (sv[l].data) {
        bi.sdata[l].assign(sv[l].data, sv[l].data + (size_t)sv[l].n[0] * sv[l].n[1] * sv[l].n[2]);
        bi.sv[l].data = bi.sdata[l].data();
      }
    for (int k = 0; k < 6; ++k) bi.fs[k] = fs[k];
    for (int a = 0; a < 3; ++a) bi.periodic[a] = periodic[a];
    DevAlloc da{&build_alloc, &build_release, c};
    const int rc = build_grid_device(c->lat, dim, ext, n_levels, rv.data(), solid ? sv.data() : nullptr, fs,
                                     periodic, da, c->stream, &c->g, &c->lay, &c->dg, &err);
    if (rc != 0) return set_err(c, rc == -2 ? LBM_E_MASK : (rc == -3 ? LBM_E_DEVICE : LBM_E_ARG), err);
  } else {
    const int rc = build_grid(c->lat, dim, ext, n_levels, rv.data(), solid ? sv.data() : nullptr, fs, &c->g, &err);
    if (rc != 0) return set_err(c, rc == -2 ? LBM_E_MASK : LBM_E_ARG, err);
  }
  c->dim = dim;
  c->L = n_levels;
  // relaxation time per level, nu_l = nu_finest / 2^(L-1-l) (acoustic scaling)
  const double cs2e = c->ddf ? c->p.T0 : c->lat.cs2;
  for (int l = 0; l < n_levels; ++l)
    c->tau[l] = c->p.nu_finest <= 0.0 ? 0.5 : c->p.nu_finest / std::ldexp(1.0, n_levels - 1 - l) / cs2e + 0.5;
  c->N = c->g.n;
  c->Ng = c->g.goff[n_levels];
  if (!on_device && build_layout(c->g, c->lat, periodic, &c->lay, &err) != 0) return set_err(c, LBM_E_ARG, err);
  c->NS = c->lay.nslot;
  // in place, every coarse ghost and every boundary-layer source cell gets
  // a staging slot for its post-collision populations (explosion, boundary
  // fill): the ghosts their coalesced slot, the sources slots of their own
  // after those
  c->stage.clear();
  int64_t nstage = 0;
  if (c->p.in_place && (c->Ng > 0 || !c->g.bc_src.empty())) {
    c->stage.assign((size_t)c->NS, -1);
    for (int64_t k = 0; k < c->Ng; ++k) c->stage[c->lay.slot_of[c->g.ghost_cell[k]]] = (int32_t)(c->NS + k);
    for (size_t k = 0; k < c->g.bc_src.size(); ++k) {
      const int32_t ss = c->lay.slot_of[c->g.bc_src[k]];
      if (c->stage[ss] < 0) c->stage[ss] = (int32_t)(c->NS + c->Ng + nstage++);
    }
  }
  c->stride = ((c->NS + c->Ng + nstage + PCH - 1) / PCH) * PCH;  // whole population chunks
  {
    // bytes one update of level l must move at least: its populations in
    // and out (and multipliers), plus the level's share of the flag, brick
    // and exception tables and of the sponge fields
    const int Q = c->lat.Q;
    const double pops = 2.0 * Q * c->ops.sizeof_storage * (c->ddf ? 2 : 1) + (c->lamf ? 2.0 * NLAM * c->lam_bytes : 0.0);
    for (int l = 0; l < n_levels; ++l) {
      const int64_t ncell = c->g.off[l + 1] - c->g.off[l];
      const int64_t nsl = c->lay.soff[l + 1] - c->lay.soff[l];
      int64_t nx = 0, nsp = 0;
      for (int64_t k = c->g.off[l]; k < c->g.off[l + 1]; ++k) {
        nx += c->lay.xrow_of[k] >= 0;
        nsp += (c->g.flag[k] & F_SPONGE) != 0;
      }
      const double tables = nsl * (1.0 + (c->lay.nbp * 4.0 + 12.0) / 64.0) + nx * 4.0 * (Q - 1) + nsp * 16.0;
      c->bpu[l] = ncell > 0 ? pops + tables / (double)ncell : pops;
    }
  }
  if (c->p.in_place && !(c->lat.kind >= 0 && c->p.collision <= LBM_DDF_NEWTON))
    return set_err(c, LBM_E_UNSUPPORTED, "in-place streaming: not with the surrogate");
  c->have_grid = true;
  if (c->p.host_only) return LBM_OK;
  // ---- device upload ----------------------------------------------------
  const int Q = c->lat.Q, Qm = Q - 1, NCH = 1 << dim;
  const size_t ssz = (size_t)c->ops.sizeof_storage;
  const DeviceLayout &y = c->lay;
  const int64_t N = c->N, NS = c->NS;
  // bulk gathers stage each brick's offset in units of 64 values in 32 bits
  if ((double)c->stride / 64.0 * Q >= 4294967296.0) return set_err(c, LBM_E_ARG, "grid too large for 32-bit brick offsets");
  for (int b = 0; b < 2; ++b) {
    if (b == 1 && c->p.in_place) {
      c->f[1] = c->f[0];
      c->gb[1] = c->gb[0];
      break;
    }
    c->f[b] = dev_alloc(c, ssz * Q * c->stride);
    if (!c->f[b]) return set_err(c, LBM_E_NOMEM, "population allocation failed");
    if (c->ddf) {
      c->gb[b] = dev_alloc(c, ssz * Q * c->stride);
      if (!c->gb[b]) return set_err(c, LBM_E_NOMEM, "population allocation failed");
    }
  }
  lbm_status s;
  if ((s = upload(c, &c->d_nbrick, y.nbrick.data(), y.nbrick.size())) != LBM_OK) return s;
  if ((s = upload(c, &c->d_xmask, y.xmask.data(), y.xmask.size())) != LBM_OK) return s;
  if ((s = upload(c, &c->d_xbase, y.xbase.data(), y.xbase.size())) != LBM_OK) return s;
  if ((s = upload(c, &c->d_xnbr, y.xnbr.data(), y.xnbr.size())) != LBM_OK) return s;
  {
    std::vector<uint64_t> xreg;
    regular_pulls(y, c->lat, &xreg);
    if ((s = upload(c, &c->d_xreg, xreg.data(), xreg.size())) != LBM_OK) return s;
  }
  if ((s = upload(c, &c->d_cell_of, y.cell_of.data(), y.cell_of.size())) != LBM_OK) return s;
  if (c->dg.slot_of) c->d_slot_of = c->dg.slot_of;
  else if ((s = upload(c, &c->d_slot_of, y.slot_of.data(), y.slot_of.size())) != LBM_OK) return s;
  if (c->dg.nbr) {
    c->d_flags = (uint8_t *)dev_alloc(c, std::max<int64_t>(NS, 1));
    if (!c->d_flags) return set_err(c, LBM_E_NOMEM, "flag allocation failed");
    launch_slot_flags(c->dg, NS, c->d_flags, c->stream);
    if ((s = check_launch(c)) != LBM_OK) return s;
    dev_release(c, c->dg.nbr);  // (Q-1) x 4 B per cell the update never reads
    c->dg.nbr = nullptr;
  } else {
    // device flags per slot: the canonical ones, F_MOVING where a population
    // is pulled from a moving wall, F_HOLE for slots without a cell
    std::vector<uint8_t> fl(NS, (uint8_t)F_HOLE);
#pragma omp parallel for schedule(static)
    for (int64_t cc = 0; cc < N; ++cc) {
      uint8_t v = c->g.flag[cc];
      for (int i = 0; i < Qm; ++i)
        if (c->g.nbr[(size_t)i * N + cc] <= -3) v |= F_MOVING;
      fl[y.slot_of[cc]] = v;
    }
    if ((s = upload(c, &c->d_flags, fl.data(), fl.size())) != LBM_OK) return s;
  }
  if (!c->g.sigma.empty()) {
    std::vector<double> sg(NS, 0.0), ri(NS, 0.0);
    for (int64_t cc = 0; cc < N; ++cc) {
      sg[y.slot_of[cc]] = c->g.sigma[cc];
      ri[y.slot_of[cc]] = c->g.rho_inf[cc];
    }
    if ((s = upload(c, &c->d_sigma, sg.data(), sg.size())) != LBM_OK) return s;
    if ((s = upload(c, &c->d_rhoinf, ri.data(), ri.size())) != LBM_OK) return s;
  }
  if (c->lamf) {
    c->d_lam = dev_alloc(c, (size_t)c->lam_bytes * NLAM * c->stride);
    if (!c->d_lam) return set_err(c, LBM_E_NOMEM, "multiplier allocation failed");
  }
  {
    // ghost, child and boundary lists over slots; every child of a coarse
    // ghost has an exception row, which the coalescence pulls through
    std::vector<int32_t> gs(c->g.ghost_cell.size()), ch(c->g.child.size()), cr(c->g.child.size(), 0);
    for (size_t k = 0; k < gs.size(); ++k) gs[k] = y.slot_of[c->g.ghost_cell[k]];
    for (size_t k = 0; k < ch.size(); ++k) {
      const int32_t v = c->g.child[k];
      ch[k] = v < 0 ? -1 : y.slot_of[v];
      if (v >= 0) {
        cr[k] = y.xrow_of[v];
        if (cr[k] < 0) return set_err(c, LBM_E_ARG, "internal: child of a coarse ghost without an exception row");
      }
    }
    std::vector<int32_t> bcc(c->g.bc_cell.size()), bcs(c->g.bc_src.size());
    for (size_t k = 0; k < bcc.size(); ++k) bcc[k] = y.slot_of[c->g.bc_cell[k]];
    for (size_t k = 0; k < bcs.size(); ++k) bcs[k] = y.slot_of[c->g.bc_src[k]];
    if ((s = upload(c, &c->d_ghost, gs.data(), gs.size())) != LBM_OK) return s;
    if ((s = upload(c, &c->d_child, ch.data(), ch.size())) != LBM_OK) return s;
    if ((s = upload(c, &c->d_crow, cr.data(), cr.size())) != LBM_OK) return s;
    if ((s = upload(c, &c->d_bc_cell, bcc.data(), bcc.size())) != LBM_OK) return s;
    if ((s = upload(c, &c->d_bc_src, bcs.data(), bcs.size())) != LBM_OK) return s;
  }
  if ((s = upload(c, &c->d_unknown, c->g.unknown.data(), c->Ng)) != LBM_OK) return s;
  if ((s = upload(c, &c->d_bc_face, c->g.bc_face.data(), c->g.bc_face.size())) != LBM_OK) return s;
  if (!c->stage.empty()) {
    // where coarse ghosts and boundary-layer sources leave their
    // post-collision populations when streaming in place
    if ((s = upload(c, &c->d_gslot, c->stage.data(), c->stage.size())) != LBM_OK) return s;
    // exception row of each boundary-layer cell (its pushes go through it)
    std::vector<int32_t> br(c->g.bc_cell.size());
    for (size_t k = 0; k < br.size(); ++k) {
      br[k] = y.xrow_of[c->g.bc_cell[k]];
      if (br[k] < 0) return set_err(c, LBM_E_ARG, "internal: boundary cell without an exception row");
    }
    if ((s = upload(c, &c->d_bc_row, br.data(), br.size())) != LBM_OK) return s;
  }
  (void)NCH;
  c->d_counters = (unsigned long long *)dev_alloc(c, sizeof(unsigned long long) * CNT_COUNT * CNT_COPIES);
  if (!c->d_counters) return set_err(c, LBM_E_NOMEM, "counter allocation failed");
  HIP_TRY(c, hipMemset(c->d_counters, 0, sizeof(unsigned long long) * CNT_COUNT * CNT_COPIES));
  return LBM_OK;
}

lbm_status lbm_grid_info(lbm_ctx *c, int64_t *n_cells, int64_t *n_per_level, int64_t *n_ghosts,
                         double *eq_fine) {
  if (!c) return LBM_E_ARG;
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  if (n_cells) *n_cells = c->N;
  if (n_ghosts) *n_ghosts = c->Ng;
  double e = 0.0;
  for (int l = 0; l < c->L; ++l) {
    const int64_t k = c->g.off[l + 1] - c->g.off[l];
    if (n_per_level) n_per_level[l] = k;
    e += (double)k / std::ldexp(1.0, c->L - 1 - l);
  }
  if (eq_fine) *eq_fine = e;
  return LBM_OK;
}

lbm_status lbm_layout_export(lbm_ctx *c, int32_t *slot_of, int32_t *xrow_of, int32_t *nbrick, uint64_t *xmask,
                             int32_t *xnbr) {
  if (!c) return LBM_E_ARG;
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  const DeviceLayout &y = c->lay;
  const int64_t n = c->g.n, nb = y.nslot / 64, Qm = c->lat.Q - 1;
  if (slot_of) std::copy(y.slot_of.begin(), y.slot_of.end(), slot_of);
  if (xrow_of) std::copy(y.xrow_of.begin(), y.xrow_of.end(), xrow_of);
  if (nbrick) std::copy(y.nbrick.begin(), y.nbrick.begin() + nb * y.nbp, nbrick);
  if (xmask) std::copy(y.xmask.begin(), y.xmask.begin() + nb, xmask);
  if (xnbr)
    for (int64_t i = 0; i < Qm; ++i)
      std::copy(y.xnbr.begin() + i * y.xstride, y.xnbr.begin() + i * y.xstride + y.nx, xnbr + i * y.nx);
  (void)n;
  return LBM_OK;
}

lbm_status lbm_layout_info(lbm_ctx *c, int64_t *n_slots, int64_t *n_rows, int64_t *slots_per_level,
                           int64_t *rows_per_level) {
  if (!c) return LBM_E_ARG;
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  if (n_slots) *n_slots = c->lay.nslot;
  if (n_rows) *n_rows = c->lay.nx;
  for (int l = 0; l < c->L; ++l) {
    if (slots_per_level) slots_per_level[l] = c->lay.soff[l + 1] - c->lay.soff[l];
    if (rows_per_level) {
      int64_t k = 0;
      for (int64_t q = c->g.off[l]; q < c->g.off[l + 1]; ++q) k += c->lay.xrow_of[q] >= 0;
      rows_per_level[l] = k;
    }
  }
  return LBM_OK;
}

lbm_status lbm_grid_export(lbm_ctx *c, int32_t *coords, int8_t *level, uint8_t *flags, int32_t *nbr,
                           int32_t *child, int32_t *bc_src) {
  if (!c) return LBM_E_ARG;
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  const int64_t n = c->N;
  const int Qm = c->lat.Q - 1;
  if (coords || nbr) {
    // a device-built grid keeps its coordinates on the device, and not its
    // canonical neighbour list: that comes from building the grid again
    std::string err;
    if (fetch_host_mirror(c->dg, &c->g, c->stream, &err) != 0) return set_err(c, LBM_E_DEVICE, err);
    if (nbr && c->g.nbr.empty()) {
      const auto &bi = c->bi;
      HostGrid tg;
      DeviceLayout ty;
      DevAlloc da{&build_alloc, &build_release, c};
      if (build_grid_device(c->lat, bi.dim, bi.ext, bi.L, bi.rv.data(), bi.has_solid ? bi.sv.data() : nullptr, bi.fs,
                            bi.periodic, da, c->stream, &tg, &ty, nullptr, &err) != 0 ||
          tg.n != c->g.n)
        return set_err(c, LBM_E_DEVICE, "neighbour list rebuild: " + err);
      c->g.nbr = std::move(tg.nbr);
    }
  }
  if (coords) memcpy(coords, c->g.xyz.data(), sizeof(int32_t) * 3 * n);
  if (level) memcpy(level, c->g.lev.data(), n);
  if (flags) memcpy(flags, c->g.flag.data(), n);
  if (nbr) {
#pragma omp parallel for schedule(static)
    for (int64_t cc = 0; cc < n; ++cc)
      for (int i = 0; i < Qm; ++i) nbr[cc * Qm + i] = c->g.nbr[(size_t)i * n + cc];
  }
  if (child) memcpy(child, c->g.child.data(), sizeof(int32_t) * c->g.child.size());
  if (bc_src) memcpy(bc_src, c->g.bc_src_all.data(), sizeof(int32_t) * n);
  return LBM_OK;
}

// mode 0: moments, 1: populations (and multipliers); the sources are host
// arrays, or device arrays when on_device (then used in place)
static lbm_status init_common(lbm_ctx *c, const double *src, const double *src_g, const double *src_lam,
                              int mode, bool on_device = false) {
  if (!c) return LBM_E_ARG;
  if (c->p.host_only) return set_err(c, LBM_E_STATE, "context is host-only");
  if (!c->have_grid) return set_err(c, LBM_E_STATE, "no grid");
  const int64_t n = c->N;
  const size_t rows = mode == 0 ? (size_t)n_mom(c) : (size_t)c->lat.Q;
  double *d = nullptr, *dg = nullptr, *dl = nullptr;
  if (on_device) {
    d = (double *)src;
    dg = mode == 1 && c->ddf ? (double *)src_g : nullptr;
    dl = mode == 1 && c->lamf ? (double *)src_lam : nullptr;
  } else {
    const size_t need = rows * n + (mode == 1 && c->ddf ? rows * n : 0) + (mode == 1 && src_lam ? NLAM * n : 0);
    d = scratch(c, sizeof(double) * std::max<size_t>(need, 1));
    if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
    HIP_TRY(c, hipMemcpyAsync(d, src, sizeof(double) * rows * n, hipMemcpyHostToDevice, c->stream));
    if (mode == 1 && c->ddf) {
      dg = d + rows * n;
      HIP_TRY(c, hipMemcpyAsync(dg, src_g, sizeof(double) * rows * n, hipMemcpyHostToDevice, c->stream));
    }
    if (mode == 1 && src_lam && c->lamf) {
      dl = d + rows * n * (c->ddf ? 2 : 1);
      HIP_TRY(c, hipMemcpyAsync(dl, src_lam, sizeof(double) * NLAM * n, hipMemcpyHostToDevice, c->stream));
    }
  }
  HIP_TRY(c, hipMemsetAsync(c->d_counters, 0, sizeof(unsigned long long) * CNT_COUNT * CNT_COPIES, c->stream));
  IArgs a{};
  a.f = c->f[0];
  a.g = c->gb[0];
  a.lam = c->d_lam;
  a.stride = c->stride;
  a.n = n;
  a.slot_of = c->d_slot_of;
  a.src = d;
  a.src_g = dg;
  a.src_lam = dl;
  a.mode = mode;
  a.ph = phys(c, c->L - 1);
  a.counters = c->d_counters;
  c->ops.init(a, c->stream);
  lbm_status s = check_launch(c);
  if (s != LBM_OK) return s;
  for (int l = 0; l < c->L; ++l) {
    c->parity[l] = 0;
    c->pre[l] = true;
    c->updates[l] = 0;
  }
  c->coarse_steps = 0;
  c->have_state = true;
  s = numeric_check(c);
  if (s != LBM_OK) return s;
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx *c, const double *moments) {
  if (!moments) return set_err(c, LBM_E_ARG, "null moments");
  return init_common(c, moments, nullptr, nullptr, 0);
}

lbm_status lbm_set_state(lbm_ctx *c, const double *f, const double *g, const double *lambda) {
  if (!f) return set_err(c, LBM_E_ARG, "null populations");
  if (c && c->ddf && !g) return set_err(c, LBM_E_ARG, "DDF state needs g");
  return init_common(c, f, g, lambda, 1);
}

lbm_status lbm_sensor(lbm_ctx *c, double *eps) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (!eps) return set_err(c, LBM_E_ARG, "null output");
  double *d = scratch(c, sizeof(double) * (size_t)std::max<int64_t>(c->N, 1));
  if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  coalesce_all(c);
  for (int l = 0; l < c->L; ++l) {
    MArgs a = gather_args(c, l, 0);
    a.out = d;
    c->ops.sensor(a, phys(c, l), read_pre(c, l), c->stream);
  }
  if ((s = check_launch(c)) != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(eps, d, sizeof(double) * c->N, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_remesh(lbm_ctx *c, const lbm_mask *refine, const lbm_mask *solid) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (c->p.in_place) return set_err(c, LBM_E_UNSUPPORTED, "remeshing keeps two population buffers (no in-place streaming)");
  if (c->L > 1 && !refine) return set_err(c, LBM_E_ARG, "refine masks missing");
  std::vector<float> mlpw;
  if (c->have_mlp) {
    mlpw.resize(MLP_PARAMS);
    HIP_TRY(c, hipMemcpy(mlpw.data(), c->d_mlp_w, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost));
  }
  // 1. the old tree's synchronisation-point state, canonical [rows][n_old],
  //    in a buffer of its own (the new grid releases the context's memory)
  const int Q = c->lat.Q;
  const int pop_rows = Q * (c->ddf ? 2 : 1);
  const int rows = pop_rows + (c->lamf ? NLAM : 0);
  const int64_t n_old = c->N;
  double *old = nullptr;
  {
    const size_t bytes = sizeof(double) * (size_t)rows * (size_t)std::max<int64_t>(n_old, 1);
    if (c->dalloc) old = (double *)c->dalloc(bytes, c->actx);
    else if (hipMalloc((void **)&old, bytes) != hipSuccess) old = nullptr;
    if (!old) return set_err(c, LBM_E_NOMEM, "remesh: state buffer allocation failed");
  }
  auto release_old = [&]() {
    hipStreamSynchronize(c->stream);
    if (c->dfree) c->dfree(old, c->actx);
    else hipFree(old);
  };
  coalesce_all(c);
  for (int l = 0; l < c->L; ++l) {
    MArgs a = gather_args(c, l, 1);
    a.out = old;
    a.lam_out = c->lamf ? old + (size_t)pop_rows * n_old : nullptr;
    c->ops.gather(a, read_pre(c, l), c->stream);
  }
  if ((s = check_launch(c)) != LBM_OK) {
    release_old();
    return s;
  }
  // 2. the new tree: same extent, levels and faces.  The old tree's device
  // tables (a device-built grid) are taken out of the context's allocations
  // so that the new build leaves them for the source lists.
  DeviceGridArrays old_dg = c->dg;
  for (void *p : {(void *)old_dg.xyz, (void *)old_dg.lev, (void *)old_dg.flag, (void *)old_dg.nbr,
                  (void *)old_dg.slot_of})
    for (size_t k = 0; p && k < c->allocs.size(); ++k)
      if (c->allocs[k] == p) {
        c->allocs.erase(c->allocs.begin() + k);
        break;
      }
  if (c->d_slot_of == old_dg.slot_of) c->d_slot_of = nullptr;
  auto release_old_dg = [&]() {
    for (void *p : {(void *)old_dg.xyz, (void *)old_dg.lev, (void *)old_dg.flag, (void *)old_dg.nbr,
                    (void *)old_dg.slot_of})
      if (p) {
        hipStreamSynchronize(c->stream);
        if (c->dfree) c->dfree(p, c->actx);
        else hipFree(p);
      }
    old_dg = DeviceGridArrays();
  };
  HostGrid prev = std::move(c->g);
  lbm_face_bc faces[6];
  for (int k = 0; k < 6; ++k) faces[k] = c->face[k];
  const int64_t steps = c->coarse_steps;
  int64_t upd[8];
  memcpy(upd, c->updates, sizeof upd);
  s = lbm_grid_build(c, prev.D, prev.ext, prev.L, refine, solid, faces);
  if (s != LBM_OK) {
    release_old();
    release_old_dg();
    return s;
  }
  // 3. where every new cell takes its state from
  int64_t *d_off = nullptr;
  int32_t *d_src = nullptr;
  double *d_wt = nullptr;
  auto release_all = [&]() {
    release_old();
    release_old_dg();
    dev_release(c, d_off);
    dev_release(c, d_src);
    dev_release(c, d_wt);
  };
  std::string err;
  if (old_dg.xyz && c->dg.xyz) {
    // on the device, from the two trees' coordinates, levels and flags
    DevAlloc da{&build_alloc, &build_release, c};
    const int rc = remesh_sources_device(prev, old_dg, c->g, c->dg, da, c->stream, &d_off, &d_src, &d_wt, &err);
    if (rc != 0) {
      release_all();
      if (rc != -1) return set_err(c, LBM_E_DEVICE, err);
      c->have_state = false;
      return set_err(c, LBM_E_MASK, err);
    }
  } else {
    std::vector<int64_t> off;
    std::vector<int32_t> src;
    std::vector<double> wt;
    // host lists need both trees' coordinates on the host
    if (fetch_host_mirror(old_dg, &prev, c->stream, &err) != 0 ||
        fetch_host_mirror(c->dg, &c->g, c->stream, &err) != 0) {
      release_all();
      return set_err(c, LBM_E_DEVICE, err);
    }
    if (remesh_sources(prev, c->g, &off, &src, &wt, &err) != 0) {
      release_all();
      c->have_state = false;
      return set_err(c, LBM_E_MASK, err);
    }
    if ((s = upload(c, &d_off, off.data(), off.size())) != LBM_OK ||
        (s = upload(c, &d_src, src.data(), src.size())) != LBM_OK ||
        (s = upload(c, &d_wt, wt.data(), wt.size())) != LBM_OK) {
      release_all();
      return s;
    }
  }
  // 4. move it across on the device and start the new tree from it
  const int64_t n_new = c->N;
  double *nw = scratch(c, sizeof(double) * (size_t)rows * (size_t)std::max<int64_t>(n_new, 1));
  if (!nw) {
    release_all();
    return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  }
  launch_remap(old, n_old, nw, n_new, rows, d_off, d_src, d_wt, c->stream);
  if ((s = check_launch(c)) != LBM_OK) {
    release_all();
    return s;
  }
  s = init_common(c, nw, c->ddf ? nw + (size_t)Q * n_new : nullptr,
                  c->lamf ? nw + (size_t)pop_rows * n_new : nullptr, 1, true);
  release_all();
  if (s != LBM_OK) return s;
  c->coarse_steps = steps;
  memcpy(c->updates, upd, sizeof upd);
  if (!mlpw.empty()) {
    if ((s = mlp_ensure(c)) != LBM_OK) return s;
    return mlp_upload_weights(c, mlpw.data());
  }
  return LBM_OK;
}

}  // extern "C"

namespace {

// one coarse step: 2^(L-1) finest substeps, active levels coarsest first
// whether a substep's collides can go in one launch: the model has the
// fused kernel, the argument blocks are on the device, the levels read
// post-collision input from two buffers, and no launch is being timed
bool fused_ok(const lbm_ctx *c, int t) {
  if (!c->fuse_levels || !c->ops.collide_multi || c->prof || c->p.in_place) return false;
  int n = 0;
  for (int l = 0; l < c->L; ++l) {
    if (t % (1 << (c->L - 1 - l)) != 0) continue;
    if (c->pre[l]) return false;
    ++n;
  }
  return n >= 2;
}

// the collides of the active levels of substep t in one launch; buffer
// parities, update counts and pre-collision flags as launch_collide leaves them
void launch_collide_fused(lbm_ctx *c, int t) {
  int lv[MAX_LEVELS], n = 0;
  for (int l = 0; l < c->L; ++l)
    if (t % (1 << (c->L - 1 - l)) == 0) lv[n++] = l;
  KArgs a = collide_args(c, lv[0], c->parity[lv[0]]);
  MultiTable &m = a.multi;
  for (int p = 0; p < 2; ++p) {
    m.f[p] = c->f[p];
    m.g[p] = c->gb[p];
  }
  int64_t nb = 0;
  const int cb = c->ops.collide_block;
  for (int k = 0; k < n; ++k) {
    const int l = lv[k];
    m.parity[k] = c->parity[l];
    m.begin[k] = c->lay.soff[l];
    m.count[k] = c->lay.soff[l + 1] - c->lay.soff[l];
    m.tau[k] = c->tau[l];
    m.omega[k] = 1.0 / c->tau[l];
    m.krr[k] = 1.0 - 1.0 / c->tau[l];
    m.block0[k] = nb;
    nb += ((m.count[k] + cb - 1) / cb + 7) / 8 * 8;  // a multiple of 8 blocks per level
  }
  m.block0[n] = nb;
  m.n = n;
  c->ops.collide_multi(a, c->stream);
  for (int k = 0; k < n; ++k) {
    const int l = lv[k];
    c->updates[l] += c->g.off[l + 1] - c->g.off[l];
    c->parity[l] ^= 1;
    c->pre[l] = false;
  }
}

void coarse_step(lbm_ctx *c) {
  const int L = c->L;
  for (int t = 0; t < (1 << (L - 1)); ++t) {
    if (fused_ok(c, t)) {
      // coalescences (each reads the finer level's state of the previous
      // substep), the collides of all active levels at once, then the
      // boundary fills and explosions in the per-level order
      for (int l = 0; l + 1 < L; ++l)
        if (t % (1 << (L - 1 - l)) == 0) launch_coalesce(c, l);
      launch_collide_fused(c, t);
      for (int l = 0; l < L; ++l) {
        if (t % (1 << (L - 1 - l)) != 0) continue;
        launch_bcfill(c, l);
        if (l > 0 && t % (1 << (L - l)) == 0) launch_explode(c, l - 1);
      }
      continue;
    }
    for (int l = 0; l < L; ++l) {
      if (t % (1 << (L - 1 - l)) != 0) continue;
      if (l + 1 < L) launch_coalesce(c, l);
      launch_collide(c, l);
      launch_bcfill(c, l);
      if (l > 0 && t % (1 << (L - l)) == 0) launch_explode(c, l - 1);
    }
  }
  c->coarse_steps++;
}



// Two coarse steps as one HIP graph: after two steps every level's buffer
// parity is back where it was (level l flips 2^(l+1) times), so the
// captured launches replay unchanged as long as the parities, the face
// values and the context's buffers are those of the capture.
bool graph_ready(lbm_ctx *c) {
  for (int l = 0; l < c->L; ++l)
    if (c->pre[l]) return false;
  if (c->gexec) {
    bool same = true;
    for (int l = 0; l < c->L; ++l) same = same && c->gparity[l] == c->parity[l];
    if (same) return true;
    drop_graph(c);
  }
  int par[8];
  int64_t upd[8], cs = c->coarse_steps;
  for (int l = 0; l < 8; ++l) {
    par[l] = c->parity[l];
    upd[l] = c->updates[l];
  }
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  coarse_step(c);
  coarse_step(c);
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  for (int l = 0; l < 8; ++l) {
    c->parity[l] = par[l];
    c->updates[l] = upd[l];
  }
  c->coarse_steps = cs;
  if (e != hipSuccess || !g) {
    hipGetLastError();
    return false;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ei != hipSuccess) {
    hipGetLastError();
    return false;
  }
  c->gexec = x;
  for (int l = 0; l < c->L; ++l) c->gparity[l] = c->parity[l];
  return true;
}

}  // namespace

extern "C" {

lbm_status lbm_step(lbm_ctx *c, int64_t n) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (n < 0) return set_err(c, LBM_E_ARG, "negative step count");
  if (c->p.collision >= LBM_DDF_MLP && !c->have_mlp) return set_err(c, LBM_E_STATE, "surrogate weights not set");
  while (n > 0) {
    if (c->use_graphs && n >= 2 && !c->prof && graph_ready(c)) {
      HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
      for (int l = 0; l < c->L; ++l) c->updates[l] += 2 * (c->g.off[l + 1] - c->g.off[l]) << l;
      c->coarse_steps += 2;
      n -= 2;
      continue;
    }
    coarse_step(c);
    n -= 1;
  }
  return check_launch(c);
}

lbm_status lbm_set_graphs(lbm_ctx *c, int on) {
  if (!c) return LBM_E_ARG;
  c->use_graphs = on != 0;
  if (!c->use_graphs) drop_graph(c);
  return LBM_OK;
}

lbm_status lbm_set_inflow_noise(lbm_ctx *c, const double *du) {
  if (!c) return LBM_E_ARG;
  if (c->p.host_only || !c->have_grid) return set_err(c, LBM_E_STATE, "no grid on the device");
  if (du && (c->p.in_place || c->p.collision >= LBM_DDF_NEWTON))
    return set_err(c, LBM_E_UNSUPPORTED, "inflow noise: not with in-place streaming or the numerical equilibria");
  drop_graph(c);  // the graph holds the table's address
  if (!du) {
    dev_release(c, c->d_xdu);
    c->d_xdu = nullptr;
    return LBM_OK;
  }
  // the perturbation of every cell projected on each velocity, moved to the
  // cell's explicit row (a cell with a moving-wall link always has one)
  const int64_t xs = c->lay.xstride, n = c->N;
  const int Q = c->lat.Q;
  std::vector<double> h((size_t)(Q - 1) * xs, 0.0);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t r = c->lay.xrow_of[k];
    if (r < 0) continue;
    double v[3];
    for (int d = 0; d < 3; ++d) {
      v[d] = du[(size_t)d * n + k];
      if (!std::isfinite(v[d])) return set_err(c, LBM_E_ARG, "non-finite inflow noise");
    }
    for (int i = 1; i < Q; ++i)
      h[(size_t)(i - 1) * xs + r] = c->lat.c[i][0] * v[0] + c->lat.c[i][1] * v[1] + c->lat.c[i][2] * v[2];
  }
  if (!c->d_xdu) {
    c->d_xdu = (double *)dev_alloc(c, sizeof(double) * h.size());
    if (!c->d_xdu) return set_err(c, LBM_E_NOMEM, "inflow noise allocation failed");
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_xdu, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_level_fusion(lbm_ctx *c, int on) {
  if (!c) return LBM_E_ARG;
  if ((on != 0) != c->fuse_levels) drop_graph(c);
  c->fuse_levels = on != 0;
  return LBM_OK;
}

lbm_status lbm_set_face_bc(lbm_ctx *c, int face, const lbm_face_bc *bc) {
  if (!c || !bc || face < 0 || face > 5) return set_err(c, LBM_E_ARG, "bad face");
  if (c->have_grid && bc->kind != c->face[face].kind) return set_err(c, LBM_E_ARG, "face kind cannot change");
  if (memcmp(&c->face[face], bc, sizeof *bc) != 0) drop_graph(c);  // the graph holds the face values
  c->face[face] = *bc;
  return LBM_OK;
}

lbm_status lbm_moments_device(lbm_ctx *c, double *out_dev) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  coalesce_all(c);
  for (int l = 0; l < c->L; ++l) {
    MArgs a = gather_args(c, l, 0);
    a.out = out_dev;
    c->ops.gather(a, read_pre(c, l), c->stream);
  }
  return check_launch(c);
}

lbm_status lbm_moments(lbm_ctx *c, double *out) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (!out) return set_err(c, LBM_E_ARG, "null output");
  const size_t bytes = sizeof(double) * n_mom(c) * c->N;
  double *d = scratch(c, bytes);
  if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  if ((s = lbm_moments_device(c, d)) != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, c->stream));
  return numeric_check(c);
}

lbm_status lbm_get_state(lbm_ctx *c, double *f, double *g, double *lambda) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (!f || (c->ddf && !g)) return set_err(c, LBM_E_ARG, "null output");
  const int Q = c->lat.Q;
  const size_t rows = (size_t)Q * (c->ddf ? 2 : 1);
  const size_t need = rows * c->N + (c->lamf ? NLAM * c->N : 0);
  double *d = scratch(c, sizeof(double) * need);
  if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  coalesce_all(c);
  for (int l = 0; l < c->L; ++l) {
    MArgs a = gather_args(c, l, 1);
    a.out = d;
    a.lam_out = c->lamf ? d + rows * c->N : nullptr;
    c->ops.gather(a, read_pre(c, l), c->stream);
  }
  if ((s = check_launch(c)) != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(f, d, sizeof(double) * Q * c->N, hipMemcpyDeviceToHost, c->stream));
  if (c->ddf)
    HIP_TRY(c, hipMemcpyAsync(g, d + (size_t)Q * c->N, sizeof(double) * Q * c->N, hipMemcpyDeviceToHost,
                              c->stream));
  if (c->lamf && lambda)
    HIP_TRY(c, hipMemcpyAsync(lambda, d + rows * c->N, sizeof(double) * NLAM * c->N, hipMemcpyDeviceToHost,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_get_cells(lbm_ctx *c, const int64_t *cells, int64_t n, double *f, double *g, double *lambda) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (n < 0 || (n > 0 && (!cells || !f || (c->ddf && !g)))) return set_err(c, LBM_E_ARG, "bad arguments");
  if (n == 0) return LBM_OK;
  const int Q = c->lat.Q;
  // group the request by level (stable), keeping each entry's position
  std::vector<int64_t> order(n);
  std::vector<int32_t> lst(n);
  std::vector<int64_t> lbeg(c->L + 1, 0);
  std::vector<int> lev(n);
  for (int64_t k = 0; k < n; ++k) {
    if (cells[k] < 0 || cells[k] >= c->N) return set_err(c, LBM_E_ARG, "cell index out of range");
    lev[k] = c->g.lev[cells[k]];
    lbeg[lev[k] + 1]++;
  }
  for (int l = 0; l < c->L; ++l) lbeg[l + 1] += lbeg[l];
  {
    std::vector<int64_t> pos(lbeg.begin(), lbeg.end() - 1);
    for (int64_t k = 0; k < n; ++k) {
      const int64_t q = pos[lev[k]]++;
      order[q] = k;
      lst[q] = (int32_t)cells[k];
    }
  }
  const size_t rows = (size_t)Q * (c->ddf ? 2 : 1);
  const size_t need = rows * n + (c->lamf ? NLAM * n : 0) + (n + 1) / 2;
  double *d = scratch(c, sizeof(double) * need);
  if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  int32_t *dl = (int32_t *)(d + rows * n + (c->lamf ? NLAM * n : 0));
  HIP_TRY(c, hipMemcpyAsync(dl, lst.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
  coalesce_all(c);
  for (int l = 0; l < c->L; ++l) {
    if (lbeg[l + 1] == lbeg[l]) continue;
    MArgs a = gather_args(c, l, 3);
    a.cells_list = dl;
    a.slot_of = c->d_slot_of;
    a.list_begin = lbeg[l];
    a.count = lbeg[l + 1] - lbeg[l];
    a.n = n;
    a.out = d;
    a.lam_out = c->lamf ? d + rows * n : nullptr;
    c->ops.gather(a, read_pre(c, l), c->stream);
  }
  if ((s = check_launch(c)) != LBM_OK) return s;
  std::vector<double> h(need - (n + 1) / 2);
  HIP_TRY(c, hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int64_t q = 0; q < n; ++q) {
    const int64_t k = order[q];
    for (int i = 0; i < Q; ++i) {
      f[(size_t)i * n + k] = h[(size_t)i * n + q];
      if (c->ddf) g[(size_t)i * n + k] = h[(size_t)(Q + i) * n + q];
    }
    if (c->lamf && lambda)
      for (int a = 0; a < NLAM; ++a) lambda[(size_t)a * n + k] = h[rows * n + (size_t)a * n + q];
  }
  return LBM_OK;
}

// The conserved sums of the synchronisation-point state into out[6] (mass,
// momentum x / y / z, total energy, kinetic energy), enqueued on the
// context stream: coalescence of every interface, one k_sums launch per
// level into partials [SUM_LEVELS][SUM_BLOCKS][6], and the fixed-order final
// reduction.  The caller provides both device buffers.
static lbm_status enqueue_sums(lbm_ctx *c, double *partials, double *out) {
  if (c->L > SUM_LEVELS) return set_err(c, LBM_E_ARG, "conserved sums: more than 8 levels");
  coalesce_all(c);
  int nb[SUM_LEVELS] = {0};
  for (int l = 0; l < c->L; ++l) {
    MArgs a = gather_args(c, l, 2);
    a.partials = partials + (size_t)l * SUM_BLOCKS * SUM_Q;
    nb[l] = a.count > 0 ? sum_blocks(a.count) : 0;
    c->ops.sums(a, read_pre(c, l), c->stream);
  }
  launch_sum_partials(partials, nb, c->L, out, c->stream);
  return check_launch(c);
}

lbm_status lbm_sums_device(lbm_ctx *c, double *out_dev) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (!out_dev) return set_err(c, LBM_E_ARG, "null output");
  if (c->L > SUM_LEVELS)
    return set_err(c, LBM_E_ARG, "lbm_sums_device: grids of at most 8 levels (the static partials hold 8 x 1024 x 6)");
  if (c->sums_static_err != hipSuccess || !c->d_sums_static)
    return set_err(c, LBM_E_DEVICE, std::string("lbm_sums_device: no address for the static partials: ") +
                                        hipGetErrorString(c->sums_static_err));
  // partials in the static array, the result straight into the caller's buffer
  return enqueue_sums(c, c->d_sums_static, out_dev);
}

lbm_status lbm_stats_get(lbm_ctx *c, lbm_stats *out) {
  lbm_status s = need_state(c);
  if (s != LBM_OK) return s;
  if (!out) return set_err(c, LBM_E_ARG, "null output");
  memset(out, 0, sizeof *out);
  double *d = scratch(c, sizeof(double) * (SUM_PARTIALS + SUM_Q));
  if (!d) return set_err(c, LBM_E_NOMEM, "scratch allocation failed");
  if ((s = enqueue_sums(c, d, d + SUM_PARTIALS)) != LBM_OK) return s;
  double acc[SUM_Q];
  HIP_TRY(c, hipMemcpyAsync(acc, d + SUM_PARTIALS, sizeof acc, hipMemcpyDeviceToHost, c->stream));
  unsigned long long cnt[CNT_COUNT];
  if ((s = read_counters(c, cnt)) != LBM_OK) return s;
  out->mass = acc[0];
  for (int d2 = 0; d2 < 3; ++d2) out->momentum[d2] = acc[1 + d2];
  out->energy = acc[4];
  out->kinetic_energy = acc[5];
  for (int k = 0; k < NHIST; ++k) out->newton_hist[k] = (int64_t)cnt[CNT_HIST0 + k];
  for (int l = 0; l < c->L; ++l) out->updates[l] = c->updates[l];
  out->newton_calls = (int64_t)cnt[CNT_NEWTON_CALLS];
  out->newton_iterations = (int64_t)cnt[CNT_NEWTON_ITERS];
  out->newton_failures = (int64_t)cnt[CNT_NEWTON_FAIL];
  out->mlp_fallbacks = (int64_t)cnt[CNT_MLP_FALLBACK];
  out->nonfinite_cells = (int64_t)cnt[CNT_NONFINITE];
  out->coarse_steps = c->coarse_steps;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx *c) {
  if (!c) return LBM_E_ARG;
  if (c->p.host_only || !c->have_grid) return LBM_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return numeric_check(c);
}

lbm_status lbm_profile_enable(lbm_ctx *c, int on) {
  if (!c) return LBM_E_ARG;
  drop_graph(c);
  c->prof = on != 0;
  if (c->prof)
    for (int l = 0; l < 8; ++l) {
      c->prof_launches[l] = 0;
      c->prof_ms[l] = 0.0;
    }
  return LBM_OK;
}

lbm_status lbm_mlp_set_weights(lbm_ctx *c, const float *w, int64_t n) {
  if (!c || !w) return LBM_E_ARG;
  if (n != MLP_PARAMS) return set_err(c, LBM_E_ARG, "expected 9176 packed parameters");
  lbm_status s = mlp_ensure(c);
  if (s != LBM_OK) return s;
  return mlp_upload_weights(c, w);
}

lbm_status lbm_mlp_get_weights(lbm_ctx *c, float *w, int64_t n) {
  if (!c || !w) return LBM_E_ARG;
  if (n != MLP_PARAMS) return set_err(c, LBM_E_ARG, "expected 9176 packed parameters");
  if (!c->have_mlp) return set_err(c, LBM_E_STATE, "surrogate weights not set");
  HIP_TRY(c, hipMemcpyAsync(w, c->d_mlp_w, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_label(lbm_ctx *c, const double *x, int64_t n, double *lambda, uint8_t *ok, int32_t *iters) {
  if (!c || !x || !lambda || !ok || n < 0) return LBM_E_ARG;
  lbm_status s = mlp_ensure(c);
  if (s != LBM_OK) return s;
  if (n == 0) return LBM_OK;
  CallBuffers tmp(c);
  double *dx = (double *)tmp.take(sizeof(double) * 4 * n);
  double *dl = (double *)tmp.take(sizeof(double) * 8 * n);
  uint8_t *dok = (uint8_t *)tmp.take(n);
  int *dit = (int *)tmp.take(sizeof(int) * n);
  if (!dx || !dl || !dok || !dit) return set_err(c, LBM_E_NOMEM, "label allocation failed");
  HIP_TRY(c, hipMemcpyAsync(dx, x, sizeof(double) * 4 * n, hipMemcpyHostToDevice, c->stream));
  mlp_label(dx, n, c->p.newton_tol, c->p.newton_max_it, dl, dok, dit, c->stream);
  if ((s = check_launch(c)) != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(lambda, dl, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(ok, dok, n, hipMemcpyDeviceToHost, c->stream));
  if (iters) HIP_TRY(c, hipMemcpyAsync(iters, dit, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_predict(lbm_ctx *c, const double *x, int64_t n, double *lambda) {
  if (!c || !x || !lambda || n < 0) return LBM_E_ARG;
  if (!c->have_mlp) return set_err(c, LBM_E_STATE, "surrogate weights not set");
  if (n == 0) return LBM_OK;
  CallBuffers tmp(c);
  double *dx = (double *)tmp.take(sizeof(double) * 4 * n);
  double *dl = (double *)tmp.take(sizeof(double) * 8 * n);
  if (!dx || !dl) return set_err(c, LBM_E_NOMEM, "prediction allocation failed");
  HIP_TRY(c, hipMemcpyAsync(dx, x, sizeof(double) * 4 * n, hipMemcpyHostToDevice, c->stream));
  mlp_predict(c->d_mlp_ops, dx, n, dl, c->stream);
  lbm_status s = check_launch(c);
  if (s != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(lambda, dl, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_grad(lbm_ctx *c, const float *xh, const float *th, int64_t n, double *loss, float *grad) {
  if (!c || !xh || !th || !grad || n <= 0 || n % 32) return set_err(c, LBM_E_ARG, "bad batch");
  if (!c->have_mlp) return set_err(c, LBM_E_STATE, "surrogate weights not set");
  CallBuffers tmp(c);
  float *dx = (float *)tmp.take(sizeof(float) * 4 * n);
  float *dt = (float *)tmp.take(sizeof(float) * 8 * n);
  int32_t *dp = (int32_t *)tmp.take(sizeof(int32_t) * n);
  float *gp = (float *)tmp.take(mlp_partials_bytes(n));
  if (!dx || !dt || !dp || !gp) return set_err(c, LBM_E_NOMEM, "gradient allocation failed");
  std::vector<int32_t> perm(n);
  for (int64_t k = 0; k < n; ++k) perm[k] = (int32_t)k;
  HIP_TRY(c, hipMemcpyAsync(dx, xh, sizeof(float) * 4 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(dt, th, sizeof(float) * 8 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(dp, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_g, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_loss, 0, sizeof(float), c->stream));
  mlp_train_batch(c->d_mlp_ops, dx, dt, dp, 0, n, gp, c->d_mlp_g, c->d_mlp_loss, c->stream);
  lbm_status s = check_launch(c);
  if (s != LBM_OK) return s;
  float lh = 0.0f;
  HIP_TRY(c, hipMemcpyAsync(grad, c->d_mlp_g, sizeof(float) * MLP_TRAINABLE, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&lh, c->d_mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_g, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = lh;
  return LBM_OK;
}

lbm_status lbm_mlp_train(lbm_ctx *c, const double *x, const double *lambda, int64_t n, int epochs, int batch,
                         double lr, uint64_t seed, double *epoch_loss) {
  if (!c || !x || !lambda || n <= 0 || epochs < 0 || batch <= 0 || batch % 32 || n < batch)
    return set_err(c, LBM_E_ARG, "bad training arguments");
  lbm_status s = mlp_ensure(c);
  if (s != LBM_OK) return s;
  std::mt19937_64 rng(seed);
  std::vector<float> w(MLP_PARAMS, 0.0f);
  if (c->have_mlp) {
    HIP_TRY(c, hipMemcpy(w.data(), c->d_mlp_w, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost));
  } else {
    // uniform initialisation scaled by the fan-in; biases zero
    const int offs[4] = {0, 320, 4480, 8640}, fan[4] = {4, 64, 64, 64}, cnt[4] = {256, 4096, 4096, 512};
    for (int k = 0; k < 4; ++k) {
      std::uniform_real_distribution<double> U(-1.0, 1.0);
      const double lim = 0.5 * std::sqrt(6.0 / fan[k]);
      for (int q = 0; q < cnt[k]; ++q) w[offs[k] + q] = (float)(lim * U(rng));
    }
  }
  // the network learns the canonical octant u_x >= u_y >= 0 (reflection
  // symmetry of the lattice); map every sample and its label there
  std::vector<double> xc(x, x + 4 * n), lc(lambda, lambda + 8 * n);
  for (int64_t i = 0; i < n; ++i) {
    double *xi = &xc[4 * i], *li = &lc[8 * i];
    if (xi[1] < 0.0) { xi[1] = -xi[1]; li[1] = -li[1]; li[4] = -li[4]; li[6] = -li[6]; }
    if (xi[2] < 0.0) { xi[2] = -xi[2]; li[2] = -li[2]; li[4] = -li[4]; li[7] = -li[7]; }
    if (xi[2] > xi[1]) {
      std::swap(xi[1], xi[2]);
      std::swap(li[1], li[2]);
      std::swap(li[3], li[5]);
      std::swap(li[6], li[7]);
    }
  }
  x = xc.data();
  lambda = lc.data();
  // output normalisation from the labels
  double mu[8] = {0}, sg[8] = {0};
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 8; ++k) mu[k] += lambda[i * 8 + k];
  for (int k = 0; k < 8; ++k) mu[k] /= (double)n;
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 8; ++k) sg[k] += (lambda[i * 8 + k] - mu[k]) * (lambda[i * 8 + k] - mu[k]);
  for (int k = 0; k < 8; ++k) {
    sg[k] = std::sqrt(sg[k] / (double)n);
    if (!(sg[k] > 1e-12)) sg[k] = 1.0;
    w[9160 + k] = (float)mu[k];
    w[9168 + k] = (float)sg[k];
  }
  if ((s = mlp_upload_weights(c, w.data())) != LBM_OK) return s;
  std::vector<float> xh(4 * n), th(8 * n);
  for (int64_t i = 0; i < n; ++i) {
    xh[4 * i] = (float)((x[4 * i] - 2.6) / 2.4);
    xh[4 * i + 1] = (float)(x[4 * i + 1] / 2.5);
    xh[4 * i + 2] = (float)(x[4 * i + 2] / 2.5);
    xh[4 * i + 3] = (float)((x[4 * i + 3] - 1.75) / 1.25);
    for (int k = 0; k < 8; ++k) th[8 * i + k] = (float)((lambda[8 * i + k] - mu[k]) / sg[k]);
  }
  CallBuffers tmp(c);
  float *dx = (float *)tmp.take(sizeof(float) * 4 * n);
  float *dt = (float *)tmp.take(sizeof(float) * 8 * n);
  int32_t *dp = (int32_t *)tmp.take(sizeof(int32_t) * n);
  float *gp = (float *)tmp.take(mlp_partials_bytes(batch));
  if (!dx || !dt || !dp || !gp) return set_err(c, LBM_E_NOMEM, "training allocation failed");
  HIP_TRY(c, hipMemcpyAsync(dx, xh.data(), sizeof(float) * 4 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(dt, th.data(), sizeof(float) * 8 * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_m, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_v, 0, sizeof(float) * MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_mlp_g, 0, sizeof(float) * MLP_PARAMS, c->stream));
  const int64_t nb = n / batch;
  const int64_t total = nb * epochs;
  std::vector<int32_t> perm(n);
  int t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t k = 0; k < n; ++k) perm[k] = (int32_t)k;
    for (int64_t k = n - 1; k > 0; --k) {
      std::uniform_int_distribution<int64_t> D(0, k);
      std::swap(perm[k], perm[D(rng)]);
    }
    HIP_TRY(c, hipMemcpyAsync(dp, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_mlp_loss, 0, sizeof(float), c->stream));
    for (int64_t b = 0; b < nb; ++b) {
      ++t;
      const double frac = (double)(t - 1) / (double)std::max<int64_t>(total, 1);
      const float lr_t = (float)(lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(3.14159265358979323846 * frac))));
      mlp_train_batch(c->d_mlp_ops, dx, dt, dp, b * batch, batch, gp, c->d_mlp_g, c->d_mlp_loss, c->stream);
      mlp_adam(c->d_mlp_w, c->d_mlp_m, c->d_mlp_v, c->d_mlp_g, c->d_mlp_ops, lr_t, t, c->stream);
    }
    if ((s = check_launch(c)) != LBM_OK) return s;
    float lh = 0.0f;
    HIP_TRY(c, hipMemcpyAsync(&lh, c->d_mlp_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (epoch_loss) epoch_loss[e] = lh / (double)nb;
  }
  return LBM_OK;
}

lbm_status lbm_profile_read(lbm_ctx *c, int level, int64_t *launches, double *total_ms,
                            double *bytes_per_update) {
  if (!c) return LBM_E_ARG;
  if (level < 0 || level >= 8) return set_err(c, LBM_E_ARG, "bad level");
  if (!c->p.host_only && !c->slots.empty()) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto &sl : c->slots) {
      float ms = 0.0f;
      HIP_TRY(c, hipEventElapsedTime(&ms, sl.a, sl.b));
      c->prof_ms[sl.level] += ms;
      c->prof_launches[sl.level] += 1;
      c->pool.push_back(sl.a);
      c->pool.push_back(sl.b);
    }
    c->slots.clear();
  }
  if (launches) *launches = c->prof_launches[level];
  if (total_ms) *total_ms = c->prof_ms[level];
  if (bytes_per_update) *bytes_per_update = c->bpu[level];
  return LBM_OK;
}

}  // extern "C"
