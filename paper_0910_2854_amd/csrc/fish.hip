// fish.hip -- host context and C interface (include/fish.h) of the FISH
// split MHD step on gfx950.  The host side validates, owns the device
// arena and sequences the sub-operators on one stream; every step of the
// arithmetic runs in the kernels of sweeps.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fish.h"
#include "sweeps.h"

using fish::Geo;
using fish::Scalars;

namespace {

constexpr int kBlock = 256;

struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct fish_ctx {
  fish_params p{};
  int prec = FISH_FP64;
  size_t esize = 8;
  int n[3]{};
  int o[3]{};          // extra layer on outflow axes
  long long ext[3]{};  // allocated extents
  long long st[3]{};   // strides
  size_t nelem = 0;    // elements per array
  hipStream_t stream = nullptr;
  // state: [buffer][field] with fields rho, mx, my, mz, E, bx, by, bz
  DeviceBuf fields[2][8];
  int cur[8]{};        // current buffer of each field
  DeviceBuf phi, scal, partial, diag_out;
  int npartial = 0;
  int seg[3]{};        // segment length of the streaming sweeps per axis
  bool have_state = false;
  bool cfl_fresh = false;  // Scalars::cmax_bits holds the CFL speed of the current state
  bool last_fluid_cfl = false;  // the next x fluid sweep also reduces the CFL speed
  std::string err;
  size_t device_bytes = 0;
  // measurement hook: event pairs around launches of the selected classes
  int timing_mask = 0;
  int timing_max = 0;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
};

namespace {

int fail(fish_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(c, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((c), FISH_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int dev_alloc(fish_ctx* c, DeviceBuf& b, size_t bytes) {
  b.bytes = bytes;
  if (bytes == 0) {
    b.ptr = nullptr;
    return FISH_OK;
  }
  if (c->p.alloc) {
    b.ptr = c->p.alloc(bytes, c->p.stream, c->p.alloc_user);
    if (!b.ptr) return fail(c, FISH_ERR_NOMEM, "allocator callback returned NULL");
  } else {
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return fail(c, FISH_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  c->device_bytes += bytes;
  return FISH_OK;
}

void dev_free(fish_ctx* c, DeviceBuf& b) {
  if (!b.ptr) return;
  if (c->p.alloc) {
    if (c->p.free) c->p.free(b.ptr, b.bytes, c->p.stream, c->p.alloc_user);
  } else {
    (void)hipFree(b.ptr);
  }
  c->device_bytes -= b.bytes;
  b.ptr = nullptr;
  b.bytes = 0;
}

Geo make_geo(const fish_ctx* c) {
  Geo g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = c->n[a];
    g.bc[a] = c->p.bc[a];
    g.st[a] = c->st[a];
  }
  g.h[0] = c->p.dx;
  g.h[1] = c->p.dy;
  g.h[2] = c->p.dz;
  return g;
}

template <typename T>
T* field(fish_ctx* c, int f, int buf) {
  return static_cast<T*>(c->fields[buf][f].ptr);
}
template <typename T>
T* cur(fish_ctx* c, int f) {
  return field<T>(c, f, c->cur[f]);
}
template <typename T>
T* nxt(fish_ctx* c, int f) {
  return field<T>(c, f, 1 - c->cur[f]);
}

Scalars* scal(fish_ctx* c) { return static_cast<Scalars*>(c->scal.ptr); }

unsigned grid_for(long long threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

// Bracket one kernel launch with events when its class is being timed.
struct TimedLaunch {
  fish_ctx* c;
  int idx = -1;
  TimedLaunch(fish_ctx* ctx, int cls) : c(ctx) {
    if ((c->timing_mask & cls) && c->ev_used < c->timing_max) {
      idx = c->ev_used++;
      (void)hipEventRecord(c->ev_start[idx], c->stream);
    }
  }
  ~TimedLaunch() {
    if (idx >= 0) (void)hipEventRecord(c->ev_stop[idx], c->stream);
  }
};

int launch_check(fish_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FISH_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return FISH_OK;
}

// ------------------------------------------------------------ sub-operators
// Whole rows per wave for the x sweeps (lanes policy): about 12 iterations of
// 64 positions per wave.
int rows_per_wave(int nx, int halo) { return std::max(1, 768 / (nx + 2 * halo)); }

template <typename T, int D, bool GRAV, bool HSE, int LIM>
void launch_fluid(fish_ctx* c) {
  fish::FluidArgs<T> a;
  for (int k = 0; k < 5; ++k) {
    a.u[k] = cur<T>(c, k);
    a.uo[k] = nxt<T>(c, k);
  }
  for (int k = 0; k < 3; ++k) a.b[k] = cur<T>(c, 5 + k);
  a.phi = static_cast<const T*>(c->phi.ptr);
  a.g = make_geo(c);
  a.gamma = c->p.gamma;
  a.alpha = c->p.predictor_alpha;
  a.seg = c->seg[D];
  a.nseg = (c->n[D] + a.seg - 1) / a.seg;
  a.rows_per_wave = rows_per_wave(c->n[0], 3);
  a.sc = scal(c);
  TimedLaunch tl(c, FISH_KERNEL_FLUID);
  if (D == 0) {
    const long long nrows = (long long)c->n[1] * c->n[2];
    const long long waves = (nrows + a.rows_per_wave - 1) / a.rows_per_wave;
    if (c->last_fluid_cfl)
      hipLaunchKernelGGL((fish::fluid_lanes_kernel<T, GRAV, HSE, LIM, true>), dim3(grid_for(waves * 64)),
                         dim3(kBlock), 0, c->stream, a);
    else
      hipLaunchKernelGGL((fish::fluid_lanes_kernel<T, GRAV, HSE, LIM, false>), dim3(grid_for(waves * 64)),
                         dim3(kBlock), 0, c->stream, a);
  } else {
    constexpr int DD = D == 0 ? 1 : D;
    const long long pencils = (long long)c->n[0] * c->n[3 - DD];
    const long long threads = (pencils + 63) / 64 * 64 * a.nseg;
    hipLaunchKernelGGL((fish::fluid_strided_kernel<T, DD, GRAV, HSE, LIM>), dim3(grid_for(threads)), dim3(kBlock),
                       0, c->stream, a);
  }
}

template <typename T, int D, int LIM>
void fluid_dispatch_lim(fish_ctx* c) {
  if (!c->p.gravity)
    launch_fluid<T, D, false, false, LIM>(c);
  else if (!c->p.hse)
    launch_fluid<T, D, true, false, LIM>(c);
  else
    launch_fluid<T, D, true, true, LIM>(c);
}

template <typename T, int D>
int fluid_dispatch(fish_ctx* c) {
  if (c->p.limiter == FISH_MINMOD)
    fluid_dispatch_lim<T, D, 0>(c);
  else
    fluid_dispatch_lim<T, D, 1>(c);
  for (int k = 0; k < 5; ++k) c->cur[k] = 1 - c->cur[k];
  return launch_check(c);
}

template <typename T, int D, int LIM>
int field_sweep_lim(fish_ctx* c) {
  const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  fish::FieldArgs<T> a;
  a.rho = cur<T>(c, 0);
  a.md = cur<T>(c, 1 + D);
  a.bt[0] = cur<T>(c, 5 + t1);
  a.bt[1] = cur<T>(c, 5 + t2);
  a.bd = cur<T>(c, 5 + D);
  a.bto[0] = nxt<T>(c, 5 + t1);
  a.bto[1] = nxt<T>(c, 5 + t2);
  a.bdo = nxt<T>(c, 5 + D);
  a.g = make_geo(c);
  a.seg = c->seg[D];
  a.nseg = (c->n[D] + a.seg - 1) / a.seg;
  a.rows_per_wave = rows_per_wave(c->n[0], 4);
  a.sc = scal(c);
  {
    TimedLaunch tl(c, FISH_KERNEL_FIELD);
    if (D == 0) {
      const long long rows = (long long)(c->n[1] + c->o[1]) * (c->n[2] + c->o[2]);
      const long long waves = (rows + a.rows_per_wave - 1) / a.rows_per_wave;
      hipLaunchKernelGGL((fish::field_lanes_kernel<T, LIM>), dim3(grid_for(waves * 64)), dim3(kBlock), 0, c->stream,
                         a);
    } else {
      constexpr int DD = D == 0 ? 1 : D;
      const long long rows = (long long)(c->n[0] + c->o[0]) * (c->n[3 - DD] + c->o[3 - DD]);
      const long long threads = (rows + 63) / 64 * 64 * a.nseg;
      hipLaunchKernelGGL((fish::field_strided_kernel<T, DD, LIM>), dim3(grid_for(threads)), dim3(kBlock), 0,
                         c->stream, a);
    }
  }
  for (int f = 5; f < 8; ++f) c->cur[f] = 1 - c->cur[f];
  return launch_check(c);
}

template <typename T, int D>
int field_sweep(fish_ctx* c) {
  return c->p.limiter == FISH_MINMOD ? field_sweep_lim<T, D, 0>(c) : field_sweep_lim<T, D, 1>(c);
}

template <typename T>
int sub_operator(fish_ctx* c, int op, int d) {
  if (op == 0) {
    switch (d) {
      case 0: return fluid_dispatch<T, 0>(c);
      case 1: return fluid_dispatch<T, 1>(c);
      default: return fluid_dispatch<T, 2>(c);
    }
  }
  switch (d) {
    case 0: return field_sweep<T, 0>(c);
    case 1: return field_sweep<T, 1>(c);
    default: return field_sweep<T, 2>(c);
  }
}

int run_sub(fish_ctx* c, int op, int d) {
  return c->prec == FISH_FP64 ? sub_operator<double>(c, op, d) : sub_operator<float>(c, op, d);
}

template <typename T>
int launch_check_cfl(fish_ctx* c) {
  fish::CheckArgs<T> a;
  for (int k = 0; k < 5; ++k) a.u[k] = cur<T>(c, k);
  for (int k = 0; k < 3; ++k) a.b[k] = cur<T>(c, 5 + k);
  a.g = make_geo(c);
  a.gamma = c->p.gamma;
  a.sc = scal(c);
  const long long ncell = (long long)c->n[0] * c->n[1] * c->n[2];
  const unsigned grid = (unsigned)std::min<long long>(grid_for(ncell), 4096);
  hipLaunchKernelGGL(fish::reset_cmax_kernel, dim3(1), dim3(1), 0, c->stream, scal(c));
  {
    TimedLaunch tl(c, FISH_KERNEL_CHECK);
    hipLaunchKernelGGL((fish::check_cfl_kernel<T>), dim3(grid), dim3(kBlock), 0, c->stream, a);
  }
  return launch_check(c);
}

int check_cfl(fish_ctx* c) {
  int rc = c->prec == FISH_FP64 ? launch_check_cfl<double>(c) : launch_check_cfl<float>(c);
  if (rc == FISH_OK) c->cfl_fresh = true;
  return rc;
}

template <typename T>
int launch_diag(fish_ctx* c) {
  fish::DiagArgs<T> a;
  for (int k = 0; k < 5; ++k) a.u[k] = cur<T>(c, k);
  for (int k = 0; k < 3; ++k) a.b[k] = cur<T>(c, 5 + k);
  a.g = make_geo(c);
  a.partial = static_cast<double*>(c->partial.ptr);
  const long long ncell = (long long)c->n[0] * c->n[1] * c->n[2];
  const long long per_block = (ncell + c->npartial - 1) / c->npartial;
  hipLaunchKernelGGL((fish::diag_partial_kernel<T>), dim3(c->npartial), dim3(kBlock), 0, c->stream, a, per_block);
  const double vol = c->p.dx * c->p.dy * c->p.dz;
  hipLaunchKernelGGL(fish::diag_final_kernel, dim3(1), dim3(1), 0, c->stream,
                     static_cast<const double*>(c->partial.ptr), c->npartial, static_cast<double*>(c->diag_out.ptr),
                     vol, c->p.dy * c->p.dz, c->p.dx * c->p.dz, c->p.dx * c->p.dy);
  return launch_check(c);
}

// Host-side repacking between the interface layout and the device layout.
// Face array `a` (0 = x) along its own normal: the interface carries n+1 faces;
// the device stores n (periodic) or n+1 (outflow).
template <typename T>
void pack_cell(const fish_ctx* c, const double* src, std::vector<T>& dst) {
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        dst[i + c->st[1] * j + c->st[2] * k] = (T)src[(size_t)i + (size_t)nx * (j + (size_t)ny * k)];
}

template <typename T>
void pack_face(const fish_ctx* c, int a, const double* src, std::vector<T>& dst) {
  int m[3] = {c->n[0], c->n[1], c->n[2]};  // input extents
  m[a] += 1;
  int keep[3] = {c->n[0], c->n[1], c->n[2]};  // stored faces
  keep[a] += c->o[a];
  for (int k = 0; k < keep[2]; ++k)
    for (int j = 0; j < keep[1]; ++j)
      for (int i = 0; i < keep[0]; ++i)
        dst[i + c->st[1] * j + c->st[2] * k] = (T)src[(size_t)i + (size_t)m[0] * (j + (size_t)m[1] * k)];
}

template <typename T>
void unpack_cell(const fish_ctx* c, const std::vector<T>& src, double* dst, size_t field_off) {
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        dst[field_off + (size_t)i + (size_t)nx * (j + (size_t)ny * k)] = (double)src[i + c->st[1] * j + c->st[2] * k];
}

template <typename T>
void unpack_face(const fish_ctx* c, int a, const std::vector<T>& src, double* dst) {
  int m[3] = {c->n[0], c->n[1], c->n[2]};
  m[a] += 1;
  for (int k = 0; k < m[2]; ++k)
    for (int j = 0; j < m[1]; ++j)
      for (int i = 0; i < m[0]; ++i) {
        int q[3] = {i, j, k};
        if (c->p.bc[a] == FISH_PERIODIC && q[a] == c->n[a]) q[a] = 0;  // face n is face 0
        dst[(size_t)i + (size_t)m[0] * (j + (size_t)m[1] * k)] = (double)src[q[0] + c->st[1] * q[1] + c->st[2] * q[2]];
      }
}

template <typename T>
int upload(fish_ctx* c, const double* cell5, const double* bx, const double* by, const double* bz,
           const double* phi) {
  std::vector<T> h(c->nelem, T(0));
  const size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  for (int f = 0; f < 5; ++f) {
    std::fill(h.begin(), h.end(), T(0));
    pack_cell<T>(c, cell5 + f * nc, h);
    HIP_TRY(c, hipMemcpyAsync(field<T>(c, f, 0), h.data(), c->nelem * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->cur[f] = 0;
  }
  const double* bsrc[3] = {bx, by, bz};
  for (int a = 0; a < 3; ++a) {
    std::fill(h.begin(), h.end(), T(0));
    pack_face<T>(c, a, bsrc[a], h);
    HIP_TRY(c, hipMemcpyAsync(field<T>(c, 5 + a, 0), h.data(), c->nelem * sizeof(T), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->cur[5 + a] = 0;
  }
  if (c->p.gravity) {
    std::fill(h.begin(), h.end(), T(0));
    pack_cell<T>(c, phi, h);
    HIP_TRY(c, hipMemcpyAsync(c->phi.ptr, h.data(), c->nelem * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return FISH_OK;
}

template <typename T>
int download(fish_ctx* c, double* cell5, double* bx, double* by, double* bz) {
  std::vector<T> h(c->nelem);
  const size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  if (cell5)
    for (int f = 0; f < 5; ++f) {
      HIP_TRY(c, hipMemcpyAsync(h.data(), cur<T>(c, f), c->nelem * sizeof(T), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      unpack_cell<T>(c, h, cell5, f * nc);
    }
  double* bdst[3] = {bx, by, bz};
  for (int a = 0; a < 3; ++a) {
    if (!bdst[a]) continue;
    HIP_TRY(c, hipMemcpyAsync(h.data(), cur<T>(c, 5 + a), c->nelem * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unpack_face<T>(c, a, h, bdst[a]);
  }
  return FISH_OK;
}

int read_scalars(fish_ctx* c, Scalars* out) {
  HIP_TRY(c, hipMemcpyAsync(out, c->scal.ptr, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FISH_OK;
}

int set_device(fish_ctx* c) {
  HIP_TRY(c, hipSetDevice(c->p.device));
  return FISH_OK;
}

}  // namespace

extern "C" {

int fish_create(const fish_params* p, fish_ctx** out) {
  if (!out) return FISH_ERR_ARG;
  *out = nullptr;
  if (!p) return FISH_ERR_ARG;
  const int n[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->dx, p->dy, p->dz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > (1 << 20)) return FISH_ERR_ARG;
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) return FISH_ERR_ARG;
    if (p->bc[a] != FISH_PERIODIC && p->bc[a] != FISH_OUTFLOW) return FISH_ERR_ARG;
  }
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return FISH_ERR_ARG;
  if (!(p->cfl > 0.0) || p->cfl > 1.0) return FISH_ERR_ARG;
  if (p->limiter != FISH_MINMOD && p->limiter != FISH_VANLEER) return FISH_ERR_ARG;
  if (!(p->predictor_alpha >= 0.0) || p->predictor_alpha > 1.0) return FISH_ERR_ARG;
  if (p->precision != FISH_FP64 && p->precision != FISH_FP32) return FISH_ERR_ARG;
  if ((p->gravity != 0 && p->gravity != 1) || (p->hse != 0 && p->hse != 1)) return FISH_ERR_ARG;
  if (p->hse && !p->gravity) return FISH_ERR_ARG;
  if ((p->alloc == nullptr) != (p->free == nullptr)) return FISH_ERR_ARG;
  const long long cells = (long long)n[0] * n[1] * n[2];
  if (cells > (1ll << 34)) return FISH_ERR_ARG;

  fish_ctx* c = new (std::nothrow) fish_ctx();
  if (!c) return FISH_ERR_NOMEM;
  c->p = *p;
  c->prec = p->precision;
  c->esize = p->precision == FISH_FP64 ? 8 : 4;
  c->stream = static_cast<hipStream_t>(p->stream);
  for (int a = 0; a < 3; ++a) {
    c->n[a] = n[a];
    c->o[a] = p->bc[a] == FISH_OUTFLOW ? 1 : 0;
    c->ext[a] = n[a] + c->o[a];
    c->seg[a] = std::min(n[a], 64);
  }
  c->st[0] = 1;
  c->st[1] = c->ext[0];
  c->st[2] = c->ext[0] * c->ext[1];
  c->nelem = (size_t)(c->ext[0] * c->ext[1] * c->ext[2]);
  if (c->nelem * c->esize >= (1ull << 32)) {
    // the kernels address each array with 32-bit byte offsets
    delete c;
    return FISH_ERR_UNSUPPORTED;
  }
  int rc = set_device(c);
  if (rc) {
    delete c;
    return rc;
  }
  const size_t bytes = c->nelem * c->esize;
  for (int b = 0; b < 2 && rc == FISH_OK; ++b)
    for (int f = 0; f < 8 && rc == FISH_OK; ++f) rc = dev_alloc(c, c->fields[b][f], bytes);
  if (rc == FISH_OK && p->gravity) rc = dev_alloc(c, c->phi, bytes);
  if (rc == FISH_OK) rc = dev_alloc(c, c->scal, sizeof(Scalars));
  c->npartial = (int)std::min<long long>(1024, std::max<long long>(1, cells / 4096));
  if (rc == FISH_OK) rc = dev_alloc(c, c->partial, (size_t)c->npartial * 10 * sizeof(double));
  if (rc == FISH_OK) rc = dev_alloc(c, c->diag_out, 16 * sizeof(double));
  if (rc != FISH_OK) {
    fish_destroy(c);
    return rc;
  }
  hipLaunchKernelGGL(fish::set_scalars_kernel, dim3(1), dim3(1), 0, c->stream, scal(c), 0.0, 0);
  rc = launch_check(c);
  if (rc == FISH_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = FISH_ERR_DEVICE;
  }
  if (rc != FISH_OK) {
    fish_destroy(c);
    return rc;
  }
  *out = c;
  return FISH_OK;
}

void fish_destroy(fish_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->p.device);
  (void)hipStreamSynchronize(c->stream);
  for (auto e : c->ev_start) (void)hipEventDestroy(e);
  for (auto e : c->ev_stop) (void)hipEventDestroy(e);
  for (int b = 0; b < 2; ++b)
    for (int f = 0; f < 8; ++f) dev_free(c, c->fields[b][f]);
  dev_free(c, c->phi);
  dev_free(c, c->scal);
  dev_free(c, c->partial);
  dev_free(c, c->diag_out);
  delete c;
}

const char* fish_last_error(const fish_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t fish_device_bytes(const fish_ctx* c) { return c ? c->device_bytes : 0; }

int fish_set_state(fish_ctx* c, const double* cell5, const double* bx, const double* by, const double* bz,
                   const double* phi) {
  if (!c) return FISH_ERR_ARG;
  if (!cell5 || !bx || !by || !bz) return fail(c, FISH_ERR_ARG, "null state pointer");
  if (c->p.gravity && !phi) return fail(c, FISH_ERR_ARG, "gravity needs phi");
  int rc = set_device(c);
  if (rc) return rc;
  rc = c->prec == FISH_FP64 ? upload<double>(c, cell5, bx, by, bz, phi) : upload<float>(c, cell5, bx, by, bz, phi);
  if (rc) return rc;
  hipLaunchKernelGGL(fish::set_scalars_kernel, dim3(1), dim3(1), 0, c->stream, scal(c), 0.0, 0);
  if ((rc = launch_check(c))) return rc;
  c->have_state = true;
  if ((rc = check_cfl(c))) return rc;
  Scalars s;
  if ((rc = read_scalars(c, &s))) return rc;
  if (s.status) return fail(c, FISH_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  return FISH_OK;
}

int fish_get_state(fish_ctx* c, double* cell5, double* bx, double* by, double* bz, double* t_out) {
  if (!c) return FISH_ERR_ARG;
  if (!c->have_state) return fail(c, FISH_ERR_ARG, "no state");
  int rc = set_device(c);
  if (rc) return rc;
  if ((rc = check_cfl(c))) return rc;
  rc = c->prec == FISH_FP64 ? download<double>(c, cell5, bx, by, bz) : download<float>(c, cell5, bx, by, bz);
  if (rc) return rc;
  Scalars s;
  if ((rc = read_scalars(c, &s))) return rc;
  if (t_out) *t_out = s.t;
  if (s.status) return fail(c, FISH_ERR_STATE, "state has rho <= 0, p <= 0 or a non-finite value");
  return FISH_OK;
}

int fish_cfl_dt(fish_ctx* c, double* dt_out) {
  if (!c || !dt_out) return c ? fail(c, FISH_ERR_ARG, "null dt_out") : FISH_ERR_ARG;
  if (!c->have_state) return fail(c, FISH_ERR_ARG, "no state");
  int rc = set_device(c);
  if (rc) return rc;
  if (!c->cfl_fresh && (rc = check_cfl(c))) return rc;
  c->cfl_fresh = true;
  Scalars s;
  if ((rc = read_scalars(c, &s))) return rc;
  if (s.status) return fail(c, FISH_ERR_STATE, "CFL found rho <= 0, p <= 0 or a non-finite value");
  const double cmax = [&] {
    double v;
    std::memcpy(&v, &s.cmax_bits, sizeof v);
    return v;
  }();
  if (!(cmax > 0.0) || !std::isfinite(cmax)) return fail(c, FISH_ERR_STATE, "CFL speed is zero or non-finite");
  *dt_out = c->p.cfl / cmax;
  return FISH_OK;
}

int fish_sweep(fish_ctx* c, int op, int dir, double dt) {
  if (!c) return FISH_ERR_ARG;
  if ((op != 0 && op != 1) || dir < 0 || dir > 2 || !(dt > 0.0) || !std::isfinite(dt))
    return fail(c, FISH_ERR_ARG, "bad sweep arguments");
  if (!c->have_state) return fail(c, FISH_ERR_ARG, "no state");
  int rc = set_device(c);
  if (rc) return rc;
  hipLaunchKernelGGL(fish::set_dt_kernel, dim3(1), dim3(1), 0, c->stream, scal(c), dt);
  if ((rc = launch_check(c))) return rc;
  c->cfl_fresh = false;
  return run_sub(c, op, dir);
}

int fish_strang_step(fish_ctx* c, double dt) {
  if (!c) return FISH_ERR_ARG;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(c, FISH_ERR_ARG, "dt must be >= 0 and finite");
  if (!c->have_state) return fail(c, FISH_ERR_ARG, "no state");
  int rc = set_device(c);
  if (rc) return rc;
  if (dt == 0.0) {
    // the CFL speed of the current state is left by the previous step's last
    // sweep (or by set_state); otherwise reduce it now
    if (!c->cfl_fresh && (rc = check_cfl(c))) return rc;
    hipLaunchKernelGGL(fish::finalize_dt_kernel, dim3(1), dim3(1), 0, c->stream, scal(c), c->p.cfl);
  } else {
    hipLaunchKernelGGL(fish::set_dt_kernel, dim3(1), dim3(1), 0, c->stream, scal(c), dt);
  }
  if ((rc = launch_check(c))) return rc;
  c->cfl_fresh = false;
  // Eqs. (12)-(13), symmetric order
  for (int d = 0; d < 3; ++d) {
    if ((rc = run_sub(c, 0, d))) return rc;
    if ((rc = run_sub(c, 1, d))) return rc;
  }
  for (int d = 2; d >= 1; --d) {
    if ((rc = run_sub(c, 1, d))) return rc;
    if ((rc = run_sub(c, 0, d))) return rc;
  }
  if ((rc = run_sub(c, 1, 0))) return rc;
  // the last sub-operator also reduces the CFL speed of the new state
  hipLaunchKernelGGL(fish::reset_cmax_kernel, dim3(1), dim3(1), 0, c->stream, scal(c));
  c->last_fluid_cfl = true;
  rc = run_sub(c, 0, 0);
  c->last_fluid_cfl = false;
  if (rc) return rc;
  hipLaunchKernelGGL(fish::advance_time_kernel, dim3(1), dim3(1), 0, c->stream, scal(c));
  if ((rc = launch_check(c))) return rc;
  c->cfl_fresh = true;
  return FISH_OK;
}

int fish_diagnostics(fish_ctx* c, double* out10) {
  if (!c || !out10) return c ? fail(c, FISH_ERR_ARG, "null output") : FISH_ERR_ARG;
  if (!c->have_state) return fail(c, FISH_ERR_ARG, "no state");
  int rc = set_device(c);
  if (rc) return rc;
  rc = c->prec == FISH_FP64 ? launch_diag<double>(c) : launch_diag<float>(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(out10, c->diag_out.ptr, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FISH_OK;
}

int fish_timing_enable(fish_ctx* c, int mask, int max_launches) {
  if (!c) return FISH_ERR_ARG;
  if (mask < 0 || max_launches < 0 || max_launches > (1 << 20)) return fail(c, FISH_ERR_ARG, "bad timing arguments");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timing_mask = 0;
  c->ev_used = 0;
  while ((int)c->ev_start.size() < max_launches) {
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
      (void)hipEventDestroy(a);
      return fail(c, FISH_ERR_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    c->ev_start.push_back(a);
    c->ev_stop.push_back(b);
  }
  c->timing_max = max_launches;
  c->timing_mask = mask;
  return FISH_OK;
}

int fish_timing_read(fish_ctx* c, int* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return c ? fail(c, FISH_ERR_ARG, "null output") : FISH_ERR_ARG;
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double sum = 0.0;
  for (int i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]));
    sum += ms;
  }
  *launches = c->ev_used;
  *total_ms = sum;
  c->ev_used = 0;
  return FISH_OK;
}

int fish_selftest_lane_shift(int device, float* out128) {
  if (!out128) return FISH_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return FISH_ERR_DEVICE;
  float* d = nullptr;
  if (hipMalloc(&d, 128 * sizeof(float)) != hipSuccess) return FISH_ERR_NOMEM;
  hipLaunchKernelGGL(fish::lane_shift_selftest_kernel, dim3(1), dim3(64), 0, nullptr, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(out128, d, 128 * sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? FISH_OK : FISH_ERR_DEVICE;
}

}  // extern "C"
