// noalloc.hip -- the double step of Eqs. (12)-(13) on a box whose state the
// caller holds in device memory, with no context and no device allocation:
// the box table, the step scalars and the work lists live in one static
// device array per GPU (`scratch`), and the sweeps ping-pong between the
// caller's state and work arrays.  The kernels are the engine's (launch_api.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/fish.h"
#include "capi.h"
#include "engine.h"
#include "launch_api.h"

namespace fish {
namespace {

// scratch: [0, 1 KiB) the box's BoxDesc, [1 KiB, 2 KiB) its Scalars, then the
// work list shared by every kind (all zeros: every wave belongs to box 0).
constexpr size_t kTableOff = 0;
constexpr size_t kScalOff = 1024;
constexpr size_t kListOff = 2048;
constexpr size_t kScratchBytes = kListOff + sizeof(int) * (size_t)FISH_NOALLOC_MAX_WAVES;
static_assert(sizeof(BoxDesc) <= kScalOff - kTableOff, "BoxDesc outgrows its scratch slot");
static_assert(sizeof(Scalars) <= kListOff - kScalOff, "Scalars outgrow their scratch slot");
static_assert(kScratchBytes == FISH_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header's");

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address: the device address of each GPU's
// copy comes from hipGetSymbolAddress (scratch_on).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current;
// looked up once per device.
int scratch_on(int device, void** out, std::string* msg) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return FISH_ERR_DEVICE;
    }
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return FISH_OK;
}

// The box's table entry and step scalars, and zeros over the first nzero
// entries of the work list (the previous call may have used fewer).
__global__ __launch_bounds__(256) void noalloc_setup_kernel(BoxDesc desc, BoxDesc* table, Scalars* sc, int* list,
                                                            int nzero) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *table = desc;
    Scalars s;
    s.dt = s.t = s.t_end = 0.0;
    s.cmax_bits = 0ull;
    s.status = s.has_end = s.taken = s.pad = 0;
    for (int d = 0; d < 3; ++d) s.kh[d] = s.kf[d] = 0.0;
    *sc = s;
  }
  for (int w = i; w < nzero; w += gridDim.x * blockDim.x) list[w] = 0;
}

// The step size taken, the CFL step of the new state (Eq. 14; the CFL speed
// was reduced by the last sweep) and the state flag.
__global__ void noalloc_report_kernel(const BoxDesc* table, const Scalars* sc, fish_step_report* r) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double cmax = __longlong_as_double((long long)sc->cmax_bits);
  const bool bad = sc->status != 0 || !(cmax > 0.0) || !isfinite(cmax);
  fish_step_report out;
  out.dt = sc->dt;
  out.dt_next = bad ? 0.0 : table->cfl / cmax;
  out.status = bad ? FISH_ERR_STATE : FISH_OK;
  out.pad = 0;
  *r = out;
}

template <typename T>
struct Step {
  T* buf[2][8];  // [0] the caller's state, [1] its work arrays
  int cur[8] = {};
  const T* phi = nullptr;
  double gamma = 0.0, alpha = 0.0;
  const BoxDesc* table = nullptr;
  Scalars* sc = nullptr;
  const int* list = nullptr;
  long long waves[K_NUM] = {};
  int n[3] = {};
  SweepSel sel;

  WorkList wl(int kind) const {
    WorkList w;
    w.boxes = table;
    w.wave_box = list;
    w.nwaves = (int)waves[kind];
    w.xcd_remap = 0;
    w.row_groups = 0;
    return w;
  }

  template <int D>
  void fluid(bool cfl) {
    // y or z with one cell: the identity, left out as the context does
    if (D != 0 && n[D] == 1) return;
    FluidLaunch<T> L;
    for (int k = 0; k < 5; ++k) {
      L.u[k] = buf[cur[k]][k];
      L.uo[k] = buf[1 - cur[k]][k];
    }
    for (int k = 0; k < 3; ++k) L.b[k] = buf[cur[5 + k]][5 + k];
    L.phi = phi;
    for (int k = 0; k < 3; ++k) L.wid[k] = nullptr;
    L.gamma = gamma;
    L.alpha = alpha;
    L.wl = wl(K_FLUID_X + D);
    L.sc = sc;
    launch_fluid_sweep<T, D>(sel, L, cfl);
    for (int k = 0; k < 5; ++k) cur[k] = 1 - cur[k];
  }

  template <int D>
  void field() {
    const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    FieldLaunch<T> L;
    L.rho = buf[cur[0]][0];
    L.md = buf[cur[1 + D]][1 + D];
    L.bt[0] = buf[cur[5 + t1]][5 + t1];
    L.bt[1] = buf[cur[5 + t2]][5 + t2];
    L.bd = buf[cur[5 + D]][5 + D];
    L.bto[0] = buf[1 - cur[5 + t1]][5 + t1];
    L.bto[1] = buf[1 - cur[5 + t2]][5 + t2];
    L.bdo = buf[1 - cur[5 + D]][5 + D];
    for (int k = 0; k < 3; ++k) L.wid[k] = nullptr;
    L.wl = wl(K_FIELD_X + D);
    L.sc = sc;
    launch_field_sweep<T, D>(sel, L);
    for (int f = 5; f < 8; ++f) cur[f] = 1 - cur[f];
  }

  void check() {
    CheckLaunch<T> L;
    for (int k = 0; k < 5; ++k) L.u[k] = buf[cur[k]][k];
    for (int k = 0; k < 3; ++k) L.b[k] = buf[cur[5 + k]][5 + k];
    for (int k = 0; k < 3; ++k) L.wid[k] = nullptr;
    L.gamma = gamma;
    L.wl = wl(K_CHECK);
    L.sc = sc;
    launch_check<T>(L, sel.stream);
  }
};

// hipSuccess, or the first launch error since the last check.
#define LAUNCHED()                                                                     \
  do {                                                                                 \
    const hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) {                                                            \
      *msg = std::string("kernel launch: ") + hipGetErrorString(e_);                   \
      return FISH_ERR_DEVICE;                                                          \
    }                                                                                  \
  } while (0)

// The launches of one double step: the step size (given, or the CFL step of
// the state: its CFL speed reduced by the check kernel, then dt = k / C, with
// the maximum cleared for the last sweep), the twelve sub-operators in
// symmetric order with the CFL speed of the new state reduced by the last
// one, and the report.
template <typename T>
int enqueue(Step<T>& s, double dt, fish_step_report* report, std::string* msg) {
  if (dt == 0.0) {
    s.check();
    LAUNCHED();
  }
  launch_begin_step(s.table, 1, s.sc, dt, s.sel.stream);
  LAUNCHED();
  s.template fluid<0>(false);
  LAUNCHED();
  s.template field<0>();
  LAUNCHED();
  s.template fluid<1>(false);
  LAUNCHED();
  s.template field<1>();
  LAUNCHED();
  s.template fluid<2>(false);
  LAUNCHED();
  s.template field<2>();
  LAUNCHED();
  s.template field<2>();
  LAUNCHED();
  s.template fluid<2>(false);
  LAUNCHED();
  s.template field<1>();
  LAUNCHED();
  s.template fluid<1>(false);
  LAUNCHED();
  s.template field<0>();
  LAUNCHED();
  s.template fluid<0>(true);
  LAUNCHED();
  if (report) {
    hipLaunchKernelGGL(noalloc_report_kernel, dim3(1), dim3(64), 0, s.sel.stream, s.table, s.sc, report);
    LAUNCHED();
  }
  return FISH_OK;
}

// The checks and launches; *msg gets the reason of a failure.
int step_noalloc(const fish_params* p, void* const state[8], void* const work[8], const void* phi, double dt,
                 fish_step_report* report, std::string* msg) {
  if (!p || !state || !work) {
    *msg = "null params, state or work";
    return FISH_ERR_ARG;
  }
  const int n[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->dx, p->dy, p->dz};
  const int bc[3] = {p->bc[0], p->bc[1], p->bc[2]};
  if (Engine::validate_box(n, h, bc, p->cfl) ||
      check_common(p->gamma, p->limiter, p->predictor_alpha, p->precision, p->gravity, p->hse)) {
    *msg = "invalid box geometry or scheme setting";
    return FISH_ERR_ARG;
  }
  if (!(dt >= 0.0) || !std::isfinite(dt)) {
    *msg = "dt must be >= 0 and finite";
    return FISH_ERR_ARG;
  }
  for (int f = 0; f < 8; ++f)
    if (!state[f] || !work[f] || state[f] == work[f]) {
      *msg = "every state and work array must be given, and distinct";
      return FISH_ERR_ARG;
    }
  if (p->gravity && !phi) {
    *msg = "gravity needs phi";
    return FISH_ERR_ARG;
  }
  const size_t esize = p->precision == FISH_FP64 ? 8 : 4;
  const long long ne = (long long)(n[0] + bc[0]) * (n[1] + bc[1]) * (n[2] + bc[2]);
  if ((unsigned long long)ne * esize >= (1ull << 32)) {
    *msg = "each array must stay below 4 GiB (32-bit byte offsets)";
    return FISH_ERR_UNSUPPORTED;
  }
  BoxDesc d{};
  long long waves[K_NUM];
  plan_single_box(n, bc, d.par, d.nseg, waves);
  long long most = 0;
  for (int k = 0; k < K_NUM; ++k) most = waves[k] > most ? waves[k] : most;
  if (most > FISH_NOALLOC_MAX_WAVES) {
    *msg = "the box needs " + std::to_string(most) + " wavefronts in one launch; the scratch holds " +
           std::to_string(FISH_NOALLOC_MAX_WAVES);
    return FISH_ERR_UNSUPPORTED;
  }
  if (check_runtime(p->stream, true, msg)) return FISH_ERR_DEVICE;

  int count = 0, prev = -1;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    *msg = "hipGetDeviceCount failed (no HIP device?)";
    return FISH_ERR_DEVICE;
  }
  if (p->device < 0 || p->device >= count || p->device >= kMaxDevices) {
    *msg = "no such HIP device";
    return FISH_ERR_ARG;
  }
  if (hipGetDevice(&prev) != hipSuccess || (prev != p->device && hipSetDevice(p->device) != hipSuccess)) {
    *msg = "hipSetDevice failed";
    return FISH_ERR_DEVICE;
  }
  int rc = FISH_OK;
  void* base = nullptr;
  (void)hipGetLastError();  // an earlier failure of the caller is not this call's
  if (!(rc = scratch_on(p->device, &base, msg))) {
    unsigned char* s8 = static_cast<unsigned char*>(base);
    for (int a = 0; a < 3; ++a) {
      d.g.n[a] = n[a];
      d.g.bc[a] = bc[a];
      d.g.h[a] = h[a];
      d.ih[a] = 1.0 / h[a];
      d.i2h[a] = 1.0 / (2.0 * h[a]);
      d.woff[a] = 0;
    }
    d.g.st[0] = 1;
    d.g.st[1] = n[0] + bc[0];
    d.g.st[2] = d.g.st[1] * (n[1] + bc[1]);
    d.off = 0;
    d.cfl = p->cfl;
    d.slot = 0;
    for (int k = 0; k < K_NUM; ++k) d.wave0[k] = 0;
    const hipStream_t stream = static_cast<hipStream_t>(p->stream);
    BoxDesc* table = reinterpret_cast<BoxDesc*>(s8 + kTableOff);
    Scalars* sc = reinterpret_cast<Scalars*>(s8 + kScalOff);
    int* list = reinterpret_cast<int*>(s8 + kListOff);
    const int nzero = (int)most;
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>(1024, (most + 255) / 256));
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(blocks), dim3(256), 0, stream, d, table, sc, list, nzero);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      *msg = std::string("kernel launch: ") + hipGetErrorString(e);
      rc = FISH_ERR_DEVICE;
    } else if (p->precision == FISH_FP64) {
      Step<double> st;
      for (int f = 0; f < 8; ++f) {
        st.buf[0][f] = static_cast<double*>(state[f]);
        st.buf[1][f] = static_cast<double*>(work[f]);
      }
      st.phi = p->gravity ? static_cast<const double*>(phi) : nullptr;
      st.gamma = p->gamma;
      st.alpha = p->predictor_alpha;
      st.table = table;
      st.sc = sc;
      st.list = list;
      for (int k = 0; k < K_NUM; ++k) st.waves[k] = waves[k];
      for (int a = 0; a < 3; ++a) st.n[a] = n[a];
      st.sel.limiter = p->limiter;
      st.sel.gravity = p->gravity;
      st.sel.hse = p->hse;
      st.sel.stream = stream;
      rc = enqueue(st, dt, report, msg);
    } else {
      Step<float> st;
      for (int f = 0; f < 8; ++f) {
        st.buf[0][f] = static_cast<float*>(state[f]);
        st.buf[1][f] = static_cast<float*>(work[f]);
      }
      st.phi = p->gravity ? static_cast<const float*>(phi) : nullptr;
      st.gamma = p->gamma;
      st.alpha = p->predictor_alpha;
      st.table = table;
      st.sc = sc;
      st.list = list;
      for (int k = 0; k < K_NUM; ++k) st.waves[k] = waves[k];
      for (int a = 0; a < 3; ++a) st.n[a] = n[a];
      st.sel.limiter = p->limiter;
      st.sel.gravity = p->gravity;
      st.sel.hse = p->hse;
      st.sel.stream = stream;
      rc = enqueue(st, dt, report, msg);
    }
  }
  if (prev != p->device) (void)hipSetDevice(prev);
  return rc;
}

}  // namespace
}  // namespace fish

extern "C" int fish_strang_step_noalloc(const fish_params* p, void* const state[8], void* const work[8],
                                        const void* phi, double dt, fish_step_report* report) {
  std::string msg;
  const int rc = fish::step_noalloc(p, state, work, phi, dt, report, &msg);
  if (rc) fish::set_thread_error(msg);
  return rc;
}
