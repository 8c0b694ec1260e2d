// fish.hip -- the C interface of include/fish.h over the host engine
// (engine.h): argument validation, the single-box context (an engine holding
// one box) and the batch of many boxes.  No arithmetic of the scheme runs
// here.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <link.h>

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fish.h"
#include "batch.h"
#include "capi.h"
#include "engine.h"

using fish::check_common;
using fish::check_runtime;
using fish::Engine;
using fish::EngineConfig;
using fish::Scalars;

struct fish_ctx {
  fish_params p{};
  Engine e;
  int slot = 0;
};


namespace fish {

int check_common(double gamma, int limiter, double alpha, int precision, int gravity, int hse) {
  if (!(gamma > 1.0) || !std::isfinite(gamma)) return FISH_ERR_ARG;
  if (limiter != FISH_MINMOD && limiter != FISH_VANLEER && limiter != FISH_MACH_SWITCH) return FISH_ERR_ARG;
  if (!(alpha >= 0.0) || alpha > 1.0) return FISH_ERR_ARG;
  if (precision != FISH_FP64 && precision != FISH_FP32) return FISH_ERR_ARG;
  if (gravity < 0 || gravity > 2 || (hse != 0 && hse != 1)) return FISH_ERR_ARG;
  if (hse && !gravity) return FISH_ERR_ARG;
  return FISH_OK;
}

}  // namespace fish

namespace {

double cmax_of(const Scalars& s) {
  double v;
  std::memcpy(&v, &s.cmax_bits, sizeof v);
  return v;
}

}  // namespace

namespace {
// message of the last failed fish_create / fish_batch_create on this thread
thread_local std::string g_create_err;

// ------------------------------------------------ which HIP runtime
// A process can hold two copies of the HIP runtime (libamdhip64): PyTorch
// wheels ship their own, found through their RPATH under the unversioned
// name libamdhip64.so, while this library asks for the SONAME
// libamdhip64.so.7.  The dynamic linker reuses a loaded copy whose SONAME
// matches, so the library binds to PyTorch's runtime when PyTorch is loaded
// first; loaded before PyTorch it binds to the system runtime, and PyTorch
// then maps its own copy next to it.  Streams and device memory belong to
// the runtime that made them, so a stream or allocator callback from the
// other copy cannot work here.
std::string resolved(const char* name) {
  char buf[PATH_MAX];
  return realpath(name, buf) ? std::string(buf) : std::string(name);
}

int collect_runtime(struct dl_phdr_info* info, size_t, void* data) {
  auto* v = static_cast<std::vector<std::string>*>(data);
  const char* name = info->dlpi_name;
  if (!name || !*name || !std::strstr(name, "libamdhip64")) return 0;
  const std::string path = resolved(name);
  for (const auto& s : *v)
    if (s == path) return 0;
  v->push_back(path);
  return 0;
}

}  // namespace

namespace fish {

void set_thread_error(const std::string& msg) { g_create_err = msg; }

// Checked before any HIP call; streams, allocators and device memory of the
// caller are all made by the runtime that made them.
int check_runtime(const void* stream, bool caller_memory, std::string* msg) {
  if (!stream && !caller_memory) return FISH_OK;  // everything is made by this library's runtime
  std::vector<std::string> loaded;
  dl_iterate_phdr(collect_runtime, &loaded);
  if (loaded.size() <= 1) return FISH_OK;
  Dl_info di;
  std::string own = "?";
  if (dladdr(reinterpret_cast<void*>(&hipGetDeviceCount), &di) && di.dli_fname) own = resolved(di.dli_fname);
  std::string others;
  for (const auto& s : loaded)
    if (s != own) others += (others.empty() ? "" : ", ") + s;
  *msg = "this library uses the HIP runtime " + own + ", but the process has also loaded " + others +
         "; a stream or allocator of that runtime cannot be used here.  Load this library after the runtime "
         "that owns them (with PyTorch: import torch first), or pass stream = NULL and alloc = NULL";
  return FISH_ERR_DEVICE;
}

}  // namespace fish

extern "C" {

// ------------------------------------------------------------ single box

int fish_create(const fish_params* p, fish_ctx** out) {
  if (!out) return FISH_ERR_ARG;
  *out = nullptr;
  if (!p) return FISH_ERR_ARG;
  const int n[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->dx, p->dy, p->dz};
  const int bc[3] = {p->bc[0], p->bc[1], p->bc[2]};
  if (Engine::validate_box(n, h, bc, p->cfl)) return FISH_ERR_ARG;
  if (check_common(p->gamma, p->limiter, p->predictor_alpha, p->precision, p->gravity, p->hse)) return FISH_ERR_ARG;
  if ((p->alloc == nullptr) != (p->free == nullptr)) return FISH_ERR_ARG;
  if (check_runtime(p->stream, p->alloc != nullptr, &g_create_err)) return FISH_ERR_DEVICE;
  const long long cells = (long long)n[0] * n[1] * n[2];
  if (cells > (1ll << 34)) return FISH_ERR_ARG;
  const size_t esize = p->precision == FISH_FP64 ? 8 : 4;
  const long long ne = (long long)(n[0] + bc[0]) * (n[1] + bc[1]) * (n[2] + bc[2]);
  if ((unsigned long long)ne * esize >= (1ull << 32)) return FISH_ERR_UNSUPPORTED;

  fish_ctx* c = new (std::nothrow) fish_ctx();
  if (!c) return FISH_ERR_NOMEM;
  c->p = *p;
  EngineConfig cfg;
  cfg.precision = p->precision;
  cfg.gamma = p->gamma;
  cfg.alpha = p->predictor_alpha;
  cfg.limiter = p->limiter;
  cfg.gravity = p->gravity;
  cfg.hse = p->hse;
  cfg.device = p->device;
  cfg.stream = static_cast<hipStream_t>(p->stream);
  cfg.alloc = p->alloc;
  cfg.free = p->free;
  cfg.alloc_user = p->alloc_user;
  int rc = c->e.init(cfg, ne, 1);
  if (!rc) rc = c->e.add_box(n, h, bc, p->cfl, &c->slot);
  if (rc) {
    g_create_err = c->e.err;
    delete c;
    return rc;
  }
  *out = c;
  return FISH_OK;
}

void fish_destroy(fish_ctx* c) { delete c; }

const char* fish_last_error(const fish_ctx* c) {
  if (c) return c->e.err.c_str();
  return g_create_err.empty() ? "null context" : g_create_err.c_str();
}

size_t fish_device_bytes(const fish_ctx* c) { return c ? c->e.device_bytes : 0; }

int fish_set_state(fish_ctx* c, const double* cell5, const double* bx, const double* by, const double* bz,
                   const double* phi) {
  if (!c) return FISH_ERR_ARG;
  if (!cell5 || !bx || !by || !bz) return c->e.fail(FISH_ERR_ARG, "null state pointer");
  if (c->p.gravity && !phi) return c->e.fail(FISH_ERR_ARG, "gravity needs phi");
  int rc = c->e.upload(c->slot, cell5, bx, by, bz, phi);
  if (rc) return rc;
  if ((rc = c->e.check_cfl_all())) return rc;
  Scalars s;
  if ((rc = c->e.read_scalars(c->slot, &s))) return rc;
  if (s.status) return c->e.fail(FISH_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  return FISH_OK;
}

int fish_get_state(fish_ctx* c, double* cell5, double* bx, double* by, double* bz, double* t_out) {
  if (!c) return FISH_ERR_ARG;
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  int rc = c->e.set_device();
  if (rc) return rc;
  if ((rc = c->e.check_cfl_all())) return rc;
  if ((rc = c->e.download(c->slot, cell5, bx, by, bz))) return rc;
  Scalars s;
  if ((rc = c->e.read_scalars(c->slot, &s))) return rc;
  if (t_out) *t_out = s.t;
  if (s.status) return c->e.fail(FISH_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  return FISH_OK;
}

int fish_cfl_dt(fish_ctx* c, double* dt_out) {
  if (!c || !dt_out) return c ? c->e.fail(FISH_ERR_ARG, "null dt_out") : FISH_ERR_ARG;
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  int rc = c->e.set_device();
  if (rc) return rc;
  if (!c->e.boxes[c->slot].cfl_fresh && (rc = c->e.check_cfl_all())) return rc;
  Scalars s;
  if ((rc = c->e.read_scalars(c->slot, &s))) return rc;
  if (s.status) return c->e.fail(FISH_ERR_STATE, "CFL found rho <= 0, p <= 0 or a non-finite value");
  const double cmax = cmax_of(s);
  if (!(cmax > 0.0) || !std::isfinite(cmax)) return c->e.fail(FISH_ERR_STATE, "CFL speed is zero or non-finite");
  *dt_out = c->p.cfl / cmax;
  return FISH_OK;
}

int fish_sweep(fish_ctx* c, int op, int dir, double dt) {
  if (!c) return FISH_ERR_ARG;
  if ((op != 0 && op != 1) || dir < 0 || dir > 2 || !(dt > 0.0) || !std::isfinite(dt))
    return c->e.fail(FISH_ERR_ARG, "bad sweep arguments");
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  return c->e.sweep(c->slot, op, dir, dt);
}

int fish_strang_step(fish_ctx* c, double dt) {
  if (!c) return FISH_ERR_ARG;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return c->e.fail(FISH_ERR_ARG, "dt must be >= 0 and finite");
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  return c->e.strang_step(dt);
}

int fish_advance_to(fish_ctx* c, double t_end, int max_steps, int* steps_taken, double* t_out) {
  if (!c) return FISH_ERR_ARG;
  if (!std::isfinite(t_end) || max_steps < 0) return c->e.fail(FISH_ERR_ARG, "t_end must be finite, max_steps >= 0");
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  return c->e.advance_to(c->slot, t_end, max_steps, steps_taken, t_out);
}

int fish_diagnostics(fish_ctx* c, double* out10) {
  if (!c || !out10) return c ? c->e.fail(FISH_ERR_ARG, "null output") : FISH_ERR_ARG;
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  return c->e.diagnostics(c->slot, out10);
}

int fish_set_spacing(fish_ctx* c, int axis, const double* widths) {
  if (!c) return FISH_ERR_ARG;
  if (axis < 0 || axis > 2 || !widths) return c->e.fail(FISH_ERR_ARG, "bad axis or widths");
  const int n = c->e.boxes[c->slot].n[axis];
  for (int i = 0; i < n; ++i)
    if (!(widths[i] > 0.0) || !std::isfinite(widths[i])) return c->e.fail(FISH_ERR_ARG, "widths must be finite and > 0");
  return c->e.set_spacing(c->slot, axis, widths);
}

int fish_autotune(fish_ctx* c, int reps, int32_t* targets_out) {
  if (!c) return FISH_ERR_ARG;
  if (reps < 1 || reps > 100) return c->e.fail(FISH_ERR_ARG, "reps must be in [1, 100]");
  if (!c->e.boxes[c->slot].have_state) return c->e.fail(FISH_ERR_ARG, "no state");
  int chosen[fish::K_NUM] = {};
  int rc = c->e.autotune(reps, chosen);
  if (!rc && targets_out)
    for (int k = 0; k < FISH_NUM_KINDS; ++k) targets_out[k] = chosen[k];
  return rc;
}

int fish_set_shape(fish_ctx* c, int kind, int32_t value) {
  if (!c) return FISH_ERR_ARG;
  return c->e.set_shape(kind, value);
}

static int timing_enable(Engine& e, int mask, int max_launches) {
  if (mask < 0 || max_launches < 0 || max_launches > (1 << 20)) return e.fail(FISH_ERR_ARG, "bad timing arguments");
  int rc = e.set_device();
  if (rc) return rc;
  if (hipStreamSynchronize(e.cfg.stream) != hipSuccess) return e.fail(FISH_ERR_DEVICE, "hipStreamSynchronize");
  e.timing_mask = 0;
  e.ev_used = 0;
  while ((int)e.ev_start.size() < max_launches) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return e.fail(FISH_ERR_DEVICE, "hipEventCreate");
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return e.fail(FISH_ERR_DEVICE, "hipEventCreate");
    }
    e.ev_start.push_back(a);
    e.ev_stop.push_back(b);
  }
  e.timing_max = max_launches;
  e.timing_mask = mask;
  return FISH_OK;
}

static int timing_read(Engine& e, int* launches, double* total_ms) {
  int rc = e.set_device();
  if (rc) return rc;
  if (hipStreamSynchronize(e.cfg.stream) != hipSuccess) return e.fail(FISH_ERR_DEVICE, "hipStreamSynchronize");
  double sum = 0.0;
  for (int i = 0; i < e.ev_used; ++i) {
    float ms = 0.0f;
    hipError_t er = hipEventElapsedTime(&ms, e.ev_start[i], e.ev_stop[i]);
    if (er != hipSuccess) return e.fail(FISH_ERR_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(er));
    sum += ms;
  }
  *launches = e.ev_used;
  *total_ms = sum;
  e.ev_used = 0;
  return FISH_OK;
}

int fish_timing_enable(fish_ctx* c, int mask, int max_launches) {
  if (!c) return FISH_ERR_ARG;
  return timing_enable(c->e, mask, max_launches);
}

int fish_timing_read(fish_ctx* c, int* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return c ? c->e.fail(FISH_ERR_ARG, "null output") : FISH_ERR_ARG;
  return timing_read(c->e, launches, total_ms);
}

int fish_selftest_lane_shift(int device, float* out128) {
  if (!out128) return FISH_ERR_ARG;
  return fish::selftest_lane_shift(device, out128);
}

int fish_selftest_math(int device, int n, const double* x, double* rcp_out, double* sqrt_out) {
  if (!x || !rcp_out || !sqrt_out || n < 1 || n > (1 << 24)) return FISH_ERR_ARG;
  return fish::selftest_math(device, n, x, rcp_out, sqrt_out);
}

// ------------------------------------------------------------ batch
size_t fish_box_pool_bytes(const fish_box* b, int precision, int gravity) {
  if (!b) return 0;
  const size_t esize = precision == FISH_FP64 ? 8 : 4;
  const long long ne = (long long)(b->nx + (b->bc[0] == FISH_OUTFLOW)) * (b->ny + (b->bc[1] == FISH_OUTFLOW)) *
                       (b->nz + (b->bc[2] == FISH_OUTFLOW));
  const long long reserved = (ne + 63) / 64 * 64;
  return (size_t)reserved * esize * (16 + (gravity ? 1 : 0));
}

int fish_batch_create(const fish_batch_params* p, fish_batch** out) {
  if (!out) return FISH_ERR_ARG;
  *out = nullptr;
  if (!p) return FISH_ERR_ARG;
  if (check_common(p->gamma, p->limiter, p->predictor_alpha, p->precision, p->gravity, p->hse)) return FISH_ERR_ARG;
  if ((p->alloc == nullptr) != (p->free == nullptr)) return FISH_ERR_ARG;
  if (p->max_boxes < 1 || p->max_boxes > (1 << 20)) return FISH_ERR_ARG;
  if (check_runtime(p->stream, p->alloc != nullptr, &g_create_err)) return FISH_ERR_DEVICE;
  const size_t esize = p->precision == FISH_FP64 ? 8 : 4;
  const size_t per_elem = esize * (16 + (p->gravity ? 1 : 0));
  const long long cap = (long long)(p->pool_bytes / per_elem);
  if (cap < 64) return FISH_ERR_ARG;
  fish_batch* b = new (std::nothrow) fish_batch();
  if (!b) return FISH_ERR_NOMEM;
  b->p = *p;
  EngineConfig cfg;
  cfg.precision = p->precision;
  cfg.gamma = p->gamma;
  cfg.alpha = p->predictor_alpha;
  cfg.limiter = p->limiter;
  cfg.gravity = p->gravity;
  cfg.hse = p->hse;
  cfg.device = p->device;
  cfg.stream = static_cast<hipStream_t>(p->stream);
  cfg.alloc = p->alloc;
  cfg.free = p->free;
  cfg.alloc_user = p->alloc_user;
  if (!cfg.stream) {
    // graph capture needs a stream other than the null stream
    if (hipSetDevice(p->device) != hipSuccess ||
        hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking) != hipSuccess) {
      g_create_err = "stream creation failed";
      delete b;
      return FISH_ERR_DEVICE;
    }
    cfg.stream = b->own_stream;
  }
  int rc = b->e.init(cfg, cap, p->max_boxes);
  if (rc) {
    g_create_err = b->e.err;
    fish_batch_destroy(b);
    return rc;
  }
  *out = b;
  return FISH_OK;
}

void fish_batch_destroy(fish_batch* b) {
  if (!b) return;
  b->e.release();
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
}

const char* fish_batch_last_error(const fish_batch* b) { return b ? b->e.err.c_str() : "null batch"; }

size_t fish_batch_device_bytes(const fish_batch* b) { return b ? b->e.device_bytes : 0; }

size_t fish_batch_free_bytes(const fish_batch* b) {
  if (!b) return 0;
  return (size_t)b->e.free_elems() * b->e.esize * (16 + (b->p.gravity ? 1 : 0));
}

int fish_batch_count(const fish_batch* b) { return b ? b->e.count() : 0; }

int fish_batch_add(fish_batch* b, const fish_box* box, const double* cell5, const double* bx, const double* by,
                   const double* bz, const double* phi, int* id_out) {
  if (!b) return FISH_ERR_ARG;
  if (!box || !id_out || !cell5 || !bx || !by || !bz) return b->e.fail(FISH_ERR_ARG, "null argument");
  if (b->p.gravity && !phi) return b->e.fail(FISH_ERR_ARG, "gravity needs phi");
  *id_out = -1;
  const int n[3] = {box->nx, box->ny, box->nz};
  const double h[3] = {box->dx, box->dy, box->dz};
  const int bc[3] = {box->bc[0], box->bc[1], box->bc[2]};
  int slot = -1;
  int rc = b->e.add_box(n, h, bc, box->cfl, &slot);
  if (rc) return rc;
  if ((rc = b->e.upload(slot, cell5, bx, by, bz, phi)) || (rc = b->e.check_cfl_all())) {
    (void)b->e.remove_box(slot);
    return rc;
  }
  Scalars s;
  if ((rc = b->e.read_scalars(slot, &s))) {
    (void)b->e.remove_box(slot);
    return rc;
  }
  if (s.status) {
    (void)b->e.remove_box(slot);
    return b->e.fail(FISH_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  }
  *id_out = slot;
  return FISH_OK;
}

int fish_batch_remove(fish_batch* b, int id) {
  if (!b) return FISH_ERR_ARG;
  return b->e.remove_box(id);
}

int fish_batch_set_spacing(fish_batch* b, int id, int axis, const double* widths) {
  if (!b) return FISH_ERR_ARG;
  if (id < 0 || id >= (int)b->e.boxes.size() || !b->e.boxes[id].used) return b->e.fail(FISH_ERR_ARG, "no such box");
  if (axis < 0 || axis > 2 || !widths) return b->e.fail(FISH_ERR_ARG, "bad axis or widths");
  const int n = b->e.boxes[id].n[axis];
  for (int i = 0; i < n; ++i)
    if (!(widths[i] > 0.0) || !std::isfinite(widths[i])) return b->e.fail(FISH_ERR_ARG, "widths must be finite and > 0");
  return b->e.set_spacing(id, axis, widths);
}

int fish_batch_get(fish_batch* b, int id, double* cell5, double* bx, double* by, double* bz, double* t_out) {
  if (!b) return FISH_ERR_ARG;
  if (id < 0 || id >= (int)b->e.boxes.size() || !b->e.boxes[id].used) return b->e.fail(FISH_ERR_ARG, "no such box");
  int rc = b->e.download(id, cell5, bx, by, bz);
  if (rc) return rc;
  Scalars s;
  if ((rc = b->e.read_scalars(id, &s))) return rc;
  if (t_out) *t_out = s.t;
  if (s.status) return b->e.fail(FISH_ERR_STATE, "box state has rho <= 0, p <= 0 or a non-finite value");
  return FISH_OK;
}

int fish_batch_box_info(fish_batch* b, int id, double* t_out, double* dt_out, int* bad_out) {
  if (!b) return FISH_ERR_ARG;
  if (id < 0 || id >= (int)b->e.boxes.size() || !b->e.boxes[id].used) return b->e.fail(FISH_ERR_ARG, "no such box");
  Scalars s;
  int rc = b->e.set_device();
  if (rc || (rc = b->e.read_scalars(id, &s))) return rc;
  if (t_out) *t_out = s.t;
  if (dt_out) *dt_out = s.dt;
  if (bad_out) *bad_out = s.status;
  return FISH_OK;
}

int fish_batch_box_steps(fish_batch* b, int id, int* steps_out) {
  if (!b || !steps_out) return b ? b->e.fail(FISH_ERR_ARG, "null steps_out") : FISH_ERR_ARG;
  if (id < 0 || id >= (int)b->e.boxes.size() || !b->e.boxes[id].used) return b->e.fail(FISH_ERR_ARG, "no such box");
  Scalars s;
  int rc = b->e.set_device();
  if (rc || (rc = b->e.read_scalars(id, &s))) return rc;
  *steps_out = s.taken;
  return FISH_OK;
}

int fish_batch_step(fish_batch* b, int nsteps) {
  if (!b) return FISH_ERR_ARG;
  if (nsteps < 0) return b->e.fail(FISH_ERR_ARG, "nsteps must be >= 0");
  return b->e.steps(nsteps);
}

int fish_batch_use_graph(fish_batch* b, int on) {
  if (!b) return FISH_ERR_ARG;
  return b->e.set_graph(on != 0);
}

int fish_batch_autotune(fish_batch* b, int reps, int32_t* targets_out) {
  if (!b) return FISH_ERR_ARG;
  if (reps < 1 || reps > 100) return b->e.fail(FISH_ERR_ARG, "reps must be in [1, 100]");
  int chosen[fish::K_NUM] = {};
  int rc = b->e.autotune(reps, chosen);
  if (!rc && targets_out)
    for (int k = 0; k < FISH_NUM_KINDS; ++k) targets_out[k] = chosen[k];
  return rc;
}

int fish_batch_set_shape(fish_batch* b, int kind, int32_t value) {
  if (!b) return FISH_ERR_ARG;
  return b->e.set_shape(kind, value);
}

int fish_batch_sync(fish_batch* b) {
  if (!b) return FISH_ERR_ARG;
  int rc = b->e.set_device();
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(b->e.cfg.stream);
  if (e != hipSuccess) return b->e.fail(FISH_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return FISH_OK;
}

int fish_batch_timing_enable(fish_batch* b, int mask, int max_launches) {
  if (!b) return FISH_ERR_ARG;
  return timing_enable(b->e, mask, max_launches);
}

int fish_batch_timing_read(fish_batch* b, int* launches, double* total_ms) {
  if (!b || !launches || !total_ms) return b ? b->e.fail(FISH_ERR_ARG, "null output") : FISH_ERR_ARG;
  return timing_read(b->e, launches, total_ms);
}

}  // extern "C"
