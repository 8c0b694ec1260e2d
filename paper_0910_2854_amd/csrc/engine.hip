// engine.hip -- the host engine of engine.h: device pools and their offset
// allocator, box upload/download, the box table and work lists, the
// sequencing of the symmetric double step of Eqs. (12)-(13), its capture in
// a HIP graph, and the autotuner of the work-list shapes.
#include "engine.h"

#include "launch.h"
#include "launch_api.h"
#include "step_kernels.h"
#include "sweeps.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

namespace fish {

namespace {

constexpr long long kAlign = 64;  // box offsets in elements (256 B in FP32)

}  // namespace

Tuning default_tuning() {
  Tuning t;
  t.target[K_FLUID_X] = 768;
  t.target[K_FIELD_X] = 768;
  t.target[K_FLUID_Y] = t.target[K_FLUID_Z] = 64;
  t.target[K_FIELD_Y] = t.target[K_FIELD_Z] = 64;
  t.target[K_CHECK] = 16;
  for (int k = 0; k < K_NUM; ++k) t.remap[k] = t.groups[k] = 0;
  return t;
}


Engine::~Engine() { release(); }

int Engine::fail(int code, const std::string& msg) {
  err = msg;
  return code;
}

int Engine::set_device() {
  HIP_TRY(hipSetDevice(cfg.device));
  return 0;
}

int Engine::dev_alloc(DeviceBuf& b, size_t bytes) {
  b.bytes = bytes;
  if (bytes == 0) {
    b.ptr = nullptr;
    return 0;
  }
  if (cfg.alloc) {
    b.ptr = cfg.alloc(bytes, cfg.stream, cfg.alloc_user);
    if (!b.ptr) return fail(2, "allocator callback returned NULL");
  } else {
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return fail(2, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  device_bytes += bytes;
  return 0;
}

void Engine::dev_free(DeviceBuf& b) {
  if (!b.ptr) return;
  if (cfg.alloc) {
    if (cfg.free) cfg.free(b.ptr, b.bytes, cfg.stream, cfg.alloc_user);
  } else {
    (void)hipFree(b.ptr);
  }
  device_bytes -= b.bytes;
  b.ptr = nullptr;
  b.bytes = 0;
}

int Engine::launch_check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(3, std::string("kernel launch: ") + hipGetErrorString(e));
  return 0;
}

int Engine::init(const EngineConfig& c, long long cap_elems, int max_boxes) {
  cfg = c;
  live = true;
  esize = cfg.precision == 0 ? 8 : 4;
  cap = (cap_elems + kAlign - 1) / kAlign * kAlign;
  int rc = set_device();
  if (rc) return rc;
  const size_t bytes = (size_t)cap * esize;
  for (int b = 0; b < 2 && !rc; ++b)
    for (int f = 0; f < 8 && !rc; ++f) rc = dev_alloc(pool[b][f], bytes);
  if (!rc && cfg.gravity) rc = dev_alloc(phi, bytes);
  if (!rc) rc = dev_alloc(scal, sizeof(Scalars) * (size_t)max_boxes);
  if (!rc) rc = dev_alloc(table, sizeof(BoxDesc) * (size_t)max_boxes);
  if (!rc) rc = dev_alloc(spare.table, sizeof(BoxDesc) * (size_t)max_boxes);
  if (!rc) rc = dev_alloc(partial, (size_t)npartial * 10 * sizeof(double));
  if (!rc) rc = dev_alloc(diag_out, 16 * sizeof(double));
  if (rc) return rc;
  HIP_TRY(hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&list_done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&spare.done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&copy_ev, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&compute_ev, hipEventDisableTiming));
  for (int b = 0; b < 2; ++b) HIP_TRY(hipEventCreateWithFlags(&stage_ev[b], hipEventDisableTiming));
  boxes.assign(max_boxes, HostBox());
  free_list.clear();
  free_list[0] = cap;
  for (int s = 0; s < max_boxes; ++s) {
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(1), 0, cfg.stream, (Scalars*)scal.ptr + s, 0.0, 0);
  }
  if ((rc = launch_check())) return rc;
  HIP_TRY(hipStreamSynchronize(cfg.stream));
  return 0;
}

void Engine::release() {
  if (!live) return;
  live = false;
  (void)hipSetDevice(cfg.device);
  (void)hipStreamSynchronize(cfg.stream);
  if (copy_stream) (void)hipStreamSynchronize(copy_stream);
  invalidate_graph();
  drop_retired_graphs();
  for (int b = 0; b < 2; ++b) {
    if (stage[b]) (void)hipHostFree(stage[b]);
    stage[b] = nullptr;
    if (stage_ev[b]) (void)hipEventDestroy(stage_ev[b]);
    stage_ev[b] = nullptr;
  }
  stage_bytes = 0;
  if (copy_ev) (void)hipEventDestroy(copy_ev);
  if (compute_ev) (void)hipEventDestroy(compute_ev);
  copy_ev = compute_ev = nullptr;
  if (copy_stream) (void)hipStreamDestroy(copy_stream);
  copy_stream = nullptr;
  for (auto e : ev_start) (void)hipEventDestroy(e);
  for (auto e : ev_stop) (void)hipEventDestroy(e);
  ev_start.clear();
  ev_stop.clear();
  for (int b = 0; b < 2; ++b)
    for (int f = 0; f < 8; ++f) dev_free(pool[b][f]);
  dev_free(phi);
  for (int k = 0; k < 3; ++k) dev_free(wid[k]);
  nonuniform = false;
  dev_free(scal);
  dev_free(table);
  for (int k = 0; k < K_NUM; ++k) dev_free(lists[k]);
  dev_free(spare.table);
  for (int k = 0; k < K_NUM; ++k) dev_free(spare.lists[k]);
  for (void* h : {list_host, spare.host})
    if (h) (void)hipHostFree(h);
  list_host = spare.host = nullptr;
  for (hipEvent_t ev : {list_done, spare.done})
    if (ev) (void)hipEventDestroy(ev);
  list_done = spare.done = nullptr;
  for (auto& b : boxes)
    if (b.ready) {
      (void)hipEventDestroy(b.ready);
      b.ready = nullptr;
    }
  dev_free(partial);
  dev_free(diag_out);
}

// A graph may still be executing when the set of boxes changes: it is
// destroyed once an event recorded behind its launches has completed.
void Engine::invalidate_graph() {
  if (gexec || graph) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev, cfg.stream) != hipSuccess) {
      (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    retired_graphs.push_back({graph, gexec, ev});
  }
  gexec = nullptr;
  graph = nullptr;
  graph_ok = false;
}

void Engine::drop_retired_graphs() {
  std::vector<RetiredGraph> keep;
  for (auto& g : retired_graphs) {
    if (live && g.after && hipEventQuery(g.after) != hipSuccess) {
      keep.push_back(g);
      continue;
    }
    if (!g.after) (void)hipStreamSynchronize(cfg.stream);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.after) (void)hipEventDestroy(g.after);
  }
  retired_graphs.swap(keep);
}

// ------------------------------------------------------------ boxes
int Engine::validate_box(const int n[3], const double h[3], const int bc[3], double cfl) {
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > (1 << 20)) return 1;
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) return 1;
    if (bc[a] != 0 && bc[a] != 1) return 1;
  }
  if (!(cfl > 0.0) || cfl > 1.0) return 1;
  return 0;
}

long long Engine::box_elems(const int n[3], const int bc[3]) const {
  return (long long)(n[0] + bc[0]) * (n[1] + bc[1]) * (n[2] + bc[2]);
}

int Engine::count() const {
  int c = 0;
  for (const auto& b : boxes) c += b.used ? 1 : 0;
  return c;
}

long long Engine::free_elems() const {
  long long f = 0;
  for (const auto& kv : free_list) f += kv.second;
  return f;
}

int Engine::add_box(const int n[3], const double h[3], const int bc[3], double cfl, int* slot_out) {
  if (validate_box(n, h, bc, cfl)) return fail(1, "invalid box geometry");
  const long long ne = box_elems(n, bc);
  if ((unsigned long long)ne * esize >= (1ull << 32))
    return fail(5, "each array of a box must stay below 4 GiB (32-bit byte offsets)");
  int slot = -1;
  for (int s = 0; s < (int)boxes.size(); ++s)
    if (!boxes[s].used) {
      slot = s;
      break;
    }
  if (slot < 0) return fail(2, "no free box slot");
  const long long need = (ne + kAlign - 1) / kAlign * kAlign;
  // first fit over the free ranges
  auto it = free_list.begin();
  for (; it != free_list.end(); ++it)
    if (it->second >= need) break;
  if (it == free_list.end()) return fail(2, "pool has no free range large enough for the box");
  const long long off = it->first, len = it->second;
  free_list.erase(it);
  if (len > need) free_list[off + need] = len - need;
  HostBox& b = boxes[slot];
  b = HostBox();
  b.used = true;
  for (int a = 0; a < 3; ++a) {
    b.n[a] = n[a];
    b.bc[a] = bc[a];
    b.o[a] = bc[a] == 1 ? 1 : 0;
    b.h[a] = h[a];
  }
  b.cfl = cfl;
  b.st[0] = 1;
  b.st[1] = n[0] + b.o[0];
  b.st[2] = b.st[1] * (n[1] + b.o[1]);
  b.nelem = ne;
  b.off = off;
  b.reserved = need;
  dirty = true;
  invalidate_graph();
  *slot_out = slot;
  return 0;
}

int Engine::remove_box(int slot) {
  if (slot < 0 || slot >= (int)boxes.size() || !boxes[slot].used) return fail(1, "no such box");
  int rc = set_device();
  if (rc) return rc;
  HostBox& b = boxes[slot];
  if (b.ready) {
    // a parked box: every launch that touched it is behind its event
    HIP_TRY(hipEventSynchronize(b.ready));
    HIP_TRY(hipStreamSynchronize(copy_stream));
    (void)hipEventDestroy(b.ready);
    b.ready = nullptr;
  } else {
    HIP_TRY(hipStreamSynchronize(cfg.stream));  // no launch in flight reads its range
  }
  drop_retired_graphs();
  long long off = b.off, len = b.reserved;
  // return the range and merge with its neighbours
  auto nx = free_list.lower_bound(off);
  if (nx != free_list.end() && nx->first == off + len) {
    len += nx->second;
    free_list.erase(nx);
  }
  auto pv = free_list.lower_bound(off);
  if (pv != free_list.begin()) {
    --pv;
    if (pv->first + pv->second == off) {
      off = pv->first;
      len += pv->second;
      free_list.erase(pv);
    }
  }
  free_list[off] = len;
  const bool was_listed = !b.parked;
  b = HostBox();
  if (was_listed) {
    dirty = true;
    invalidate_graph();
  }
  return 0;
}

// Take a box out of the launches but keep its state readable: its event is
// recorded behind every launch enqueued so far.
int Engine::park(int slot) {
  if (slot < 0 || slot >= (int)boxes.size() || !boxes[slot].used) return fail(1, "no such box");
  int rc = set_device();
  if (rc) return rc;
  HostBox& b = boxes[slot];
  if (!b.ready) HIP_TRY(hipEventCreateWithFlags(&b.ready, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(b.ready, cfg.stream));
  b.parked = true;
  dirty = true;
  invalidate_graph();
  return 0;
}

// ------------------------------------------------------------ host transfers
// Host arrays (the interface layout, FP64) are repacked into the device layout
// and precision in pinned staging buffers, several threads at a time, and
// cross PCIe on the copy stream: two staging buffers alternate, so the host
// packs one chunk (whole z-planes of the device layout) while the previous
// one is copied.  The compute stream waits for an upload through an event;
// a download waits for the compute stream the same way.

// Run f(a, b) over [0, n) split across up to 16 threads.
static void parallel_for(long long n, const std::function<void(long long, long long)>& f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const long long nt = std::min<long long>(std::min<long long>(hw, 16), n);
  if (nt <= 1 || n < 8) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve((size_t)nt);
  for (long long t = 0; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt);
  for (auto& x : th) x.join();
}

// Array a of a box: 0-4 cell fields, 5-7 face fields along x, y, z, 8 phi.
// Interface extents m (n, with n+1 along its own normal for a face array);
// stored extents keep (n, with n+o along its own normal); device extents
// ext = n + o on every axis.
struct ArrayShape {
  int m[3], keep[3], ext[3];
  long long st1, st2;
};

static ArrayShape array_shape(const HostBox& c, int a) {
  ArrayShape s;
  for (int x = 0; x < 3; ++x) {
    s.m[x] = c.n[x];
    s.keep[x] = c.n[x];
    s.ext[x] = c.n[x] + c.o[x];
  }
  if (a >= 5 && a <= 7) {
    const int ax = a - 5;
    s.m[ax] += 1;
    s.keep[ax] += c.o[ax];
  }
  s.st1 = c.st[1];
  s.st2 = c.st[2];
  return s;
}

// Device planes [k0, k1) of array a from the interface array src into dst
// (zero outside the stored region).
template <typename T>
static void pack_planes(const HostBox& c, int a, const double* src, T* dst, int k0, int k1) {
  const ArrayShape s = array_shape(c, a);
  const long long rows = (long long)(k1 - k0) * s.ext[1];
  parallel_for(rows, [&](long long r0, long long r1) {
    for (long long r = r0; r < r1; ++r) {
      const int k = k0 + (int)(r / s.ext[1]);
      const int j = (int)(r % s.ext[1]);
      T* d = dst + (long long)(k - k0) * s.st2 + (long long)j * s.st1;
      if (k >= s.keep[2] || j >= s.keep[1]) {
        for (int i = 0; i < s.ext[0]; ++i) d[i] = T(0);
        continue;
      }
      const double* q = src + (size_t)s.m[0] * ((size_t)j + (size_t)s.m[1] * k);
      for (int i = 0; i < s.keep[0]; ++i) d[i] = (T)q[i];
      for (int i = s.keep[0]; i < s.ext[0]; ++i) d[i] = T(0);
    }
  });
}

// Interface planes of array a whose device plane lies in [k0, k1), from the
// device planes in src.  On a periodic axis face n is written equal to face 0.
template <typename T>
static void unpack_planes(const HostBox& c, int a, const T* src, double* dst, int k0, int k1) {
  const ArrayShape s = array_shape(c, a);
  const int ax = (a >= 5 && a <= 7) ? a - 5 : -1;
  // interface planes to fill: k in [k0, k1) within m[2], plus plane n of a
  // periodic z-face array when device plane 0 is in the chunk
  std::vector<std::pair<int, int>> planes;  // (interface k, device k)
  for (int k = k0; k < k1 && k < s.m[2]; ++k) planes.push_back({k, k});
  if (ax == 2 && c.bc[2] == 0 && k0 == 0) planes.push_back({c.n[2], 0});
  if (ax == 2 && c.bc[2] == 0) {
    // interface plane n maps to device plane 0, never to device plane n
    planes.erase(std::remove_if(planes.begin(), planes.end(),
                                [&](const std::pair<int, int>& p) { return p.first == c.n[2] && p.second != 0; }),
                 planes.end());
  }
  const long long rows = (long long)planes.size() * s.m[1];
  parallel_for(rows, [&](long long r0, long long r1) {
    for (long long r = r0; r < r1; ++r) {
      const auto& pk = planes[(size_t)(r / s.m[1])];
      int j = (int)(r % s.m[1]);
      double* d = dst + (size_t)s.m[0] * ((size_t)j + (size_t)s.m[1] * pk.first);
      if (ax == 1 && c.bc[1] == 0 && j == c.n[1]) j = 0;  // face n is face 0
      const T* q = src + (long long)(pk.second - k0) * s.st2 + (long long)j * s.st1;
      if (ax == 0 && c.bc[0] == 0) {
        for (int i = 0; i < c.n[0]; ++i) d[i] = (double)q[i];
        d[c.n[0]] = (double)q[0];
      } else {
        for (int i = 0; i < s.m[0]; ++i) d[i] = (double)q[i];
      }
    }
  });
}

int Engine::ensure_stage(size_t bytes) {
  bytes = std::max(bytes, kStageBytes);
  if (stage_bytes >= bytes) return 0;
  for (int b = 0; b < 2; ++b) {
    if (stage[b]) (void)hipHostFree(stage[b]);
    stage[b] = nullptr;
  }
  stage_bytes = 0;
  for (int b = 0; b < 2; ++b) HIP_TRY(hipHostMalloc(&stage[b], bytes, hipHostMallocDefault));
  stage_bytes = bytes;
  return 0;
}

template <typename T>
int Engine::upload_t(int slot, const double* cell5, const double* bx, const double* by, const double* bz,
                     const double* phi_in) {
  const HostBox& c = boxes[slot];
  const size_t nc = (size_t)c.n[0] * c.n[1] * c.n[2];
  const size_t plane = (size_t)c.st[2] * sizeof(T);
  int rc = ensure_stage(plane);
  if (rc) return rc;
  const int ppc = (int)std::max<size_t>(1, stage_bytes / plane);
  const int nz = c.n[2] + c.o[2];
  if (c.have_state) {
    // the box's range may still be read by launches already enqueued
    HIP_TRY(hipEventRecord(compute_ev, cfg.stream));
    HIP_TRY(hipStreamWaitEvent(copy_stream, compute_ev, 0));
  }
  int idx = 0;
  for (int a = 0; a < 9; ++a) {
    if (a == 8 && !cfg.gravity) break;
    const double* src = a < 5 ? cell5 + a * nc : a == 5 ? bx : a == 6 ? by : a == 7 ? bz : phi_in;
    T* dev = (a < 8 ? (T*)pool[cur[a]][a].ptr : (T*)phi.ptr) + c.off;
    for (int k0 = 0; k0 < nz; k0 += ppc) {
      const int k1 = std::min(nz, k0 + ppc);
      HIP_TRY(hipEventSynchronize(stage_ev[idx]));  // the buffer's previous copy is done
      pack_planes<T>(c, a, src, (T*)stage[idx], k0, k1);
      HIP_TRY(hipMemcpyAsync(dev + (long long)k0 * c.st[2], stage[idx], (size_t)(k1 - k0) * plane,
                             hipMemcpyHostToDevice, copy_stream));
      HIP_TRY(hipEventRecord(stage_ev[idx], copy_stream));
      idx ^= 1;
    }
  }
  HIP_TRY(hipEventRecord(copy_ev, copy_stream));
  HIP_TRY(hipStreamWaitEvent(cfg.stream, copy_ev, 0));
  return 0;
}

int Engine::upload(int slot, const double* cell5, const double* bx, const double* by, const double* bz,
                   const double* phi_in) {
  if (slot < 0 || slot >= (int)boxes.size() || !boxes[slot].used) return fail(1, "no such box");
  int rc = set_device();
  if (rc) return rc;
  rc = esize == 8 ? upload_t<double>(slot, cell5, bx, by, bz, phi_in) : upload_t<float>(slot, cell5, bx, by, bz, phi_in);
  if (rc) return rc;
  hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(1), 0, cfg.stream, (Scalars*)scal.ptr + slot, 0.0, 0);
  if ((rc = launch_check())) return rc;
  boxes[slot].have_state = true;
  boxes[slot].cfl_fresh = false;
  boxes[slot].parked = false;
  if (!dirty && !table_slots.empty()) {
    // the table lists only boxes with a state
    bool listed = std::find(table_slots.begin(), table_slots.end(), slot) != table_slots.end();
    if (!listed) dirty = true;
  } else {
    dirty = true;
  }
  return 0;
}

template <typename T>
int Engine::download_t(int slot, double* cell5, double* bx, double* by, double* bz) {
  const HostBox& c = boxes[slot];
  const size_t nc = (size_t)c.n[0] * c.n[1] * c.n[2];
  const size_t plane = (size_t)c.st[2] * sizeof(T);
  int rc = ensure_stage(plane);
  if (rc) return rc;
  const int ppc = (int)std::max<size_t>(1, stage_bytes / plane);
  const int nz = c.n[2] + c.o[2];
  if (c.parked && c.ready) {
    HIP_TRY(hipStreamWaitEvent(copy_stream, c.ready, 0));  // not the launches enqueued since
  } else {
    HIP_TRY(hipEventRecord(compute_ev, cfg.stream));
    HIP_TRY(hipStreamWaitEvent(copy_stream, compute_ev, 0));
  }
  // chunks in order; chunk i is unpacked while chunk i+1 is copied
  struct Pending {
    int a, k0, k1, idx;
    double* dst;
  };
  std::vector<Pending> pend;
  int idx = 0;
  auto drain = [&](const Pending& q) -> int {
    HIP_TRY(hipEventSynchronize(stage_ev[q.idx]));
    unpack_planes<T>(c, q.a, (const T*)stage[q.idx], q.dst, q.k0, q.k1);
    return 0;
  };
  for (int a = 0; a < 8; ++a) {
    double* dst = a < 5 ? (cell5 ? cell5 + a * nc : nullptr) : a == 5 ? bx : a == 6 ? by : bz;
    if (!dst) continue;
    const T* dev = (const T*)pool[cur[a]][a].ptr + c.off;
    for (int k0 = 0; k0 < nz; k0 += ppc) {
      const int k1 = std::min(nz, k0 + ppc);
      // the buffer is free once its previous chunk has been unpacked
      if (!pend.empty() && pend.front().idx == idx) {
        if ((rc = drain(pend.front()))) return rc;
        pend.erase(pend.begin());
      }
      HIP_TRY(hipMemcpyAsync(stage[idx], dev + (long long)k0 * c.st[2], (size_t)(k1 - k0) * plane,
                             hipMemcpyDeviceToHost, copy_stream));
      HIP_TRY(hipEventRecord(stage_ev[idx], copy_stream));
      pend.push_back({a, k0, k1, idx, dst});
      idx ^= 1;
    }
  }
  for (const auto& q : pend)
    if ((rc = drain(q))) return rc;
  return 0;
}

int Engine::download(int slot, double* cell5, double* bx, double* by, double* bz) {
  if (slot < 0 || slot >= (int)boxes.size() || !boxes[slot].used) return fail(1, "no such box");
  int rc = set_device();
  if (rc) return rc;
  return esize == 8 ? download_t<double>(slot, cell5, bx, by, bz) : download_t<float>(slot, cell5, bx, by, bz);
}

// A parked box's scalars, read on the copy stream behind its event (not
// behind the launches enqueued since).
int Engine::read_scalars_parked(int slot, Scalars* out) {
  const HostBox& b = boxes[slot];
  if (!b.parked || !b.ready) return read_scalars(slot, out);
  HIP_TRY(hipStreamWaitEvent(copy_stream, b.ready, 0));
  HIP_TRY(hipMemcpyAsync(out, (Scalars*)scal.ptr + slot, sizeof(Scalars), hipMemcpyDeviceToHost, copy_stream));
  HIP_TRY(hipStreamSynchronize(copy_stream));
  return 0;
}

int Engine::read_scalars(int slot, Scalars* out) {
  HIP_TRY(hipMemcpyAsync(out, (Scalars*)scal.ptr + slot, sizeof(Scalars), hipMemcpyDeviceToHost, cfg.stream));
  HIP_TRY(hipStreamSynchronize(cfg.stream));
  return 0;
}

// ------------------------------------------------------------ work lists
static long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// Waves of one box in the list of one kind, and the per-box parameter.
// Pencil waves of one segment of a y/z kind (strided_map's two orders).
static long long strided_waves(long long nA, long long nO, int groups) {
  if (groups && nA >= 64) return ceil_div(nA, 64) * ceil_div(nO, 4) * 4;
  return ceil_div(nA * nO, 64);
}

static long long kind_waves(const HostBox& b, int kind, int target, int groups, int* par) {
  switch (kind) {
    case K_FLUID_X: {
      if (groups) {  // the strided policy along x: lanes along y, segments of the rows
        const int seg = std::max(1, std::min(target, b.n[0]));
        *par = seg;
        return strided_waves(b.n[1], b.n[2], groups) * ceil_div(b.n[0], seg);
      }
      const int rpw = std::max(1, target / (b.n[0] + 6));
      *par = rpw;
      return ceil_div((long long)b.n[1] * b.n[2], rpw);
    }
    case K_FIELD_X: {
      const int rpw = std::max(1, target / (b.n[0] + 8));
      *par = rpw;
      return ceil_div((long long)(b.n[1] + b.o[1]) * (b.n[2] + b.o[2]), rpw);
    }
    case K_FLUID_Y:
    case K_FLUID_Z: {
      const int D = kind - K_FLUID_X;
      const int seg = std::max(1, std::min(target, b.n[D]));
      *par = seg;
      return strided_waves(b.n[0], b.n[3 - D], groups) * ceil_div(b.n[D], seg);
    }
    case K_FIELD_Y:
    case K_FIELD_Z: {
      const int D = kind - K_FIELD_X;
      const int seg = std::max(1, std::min(target, b.n[D]));
      *par = seg;
      return strided_waves(b.n[0] + b.o[0], b.n[3 - D] + b.o[3 - D], groups) * ceil_div(b.n[D], seg);
    }
    default: {
      const int cpl = std::max(1, target);
      *par = cpl;
      return ceil_div((long long)b.n[0] * b.n[1] * b.n[2], 64ll * cpl);
    }
  }
}

// A box alone in its engine at a default work shape: halve the shape while
// the box fills fewer than 2048 waves (8 per CU), down to one row per wave
// (x kinds), 8-cell segments (y/z kinds) or 64 cells per wave (check).  The
// default suits a 256^3 box; a small box alone would leave most of the chip
// idle.  A batch fills the chip with its many boxes, and a shape set by
// fish_set_shape or the autotuner is used as set.
static int single_box_target(const HostBox& b, int kind, int target, int groups) {
  int lo = 1;
  if (kind == K_FLUID_X) lo = groups ? 8 : b.n[0] + 6;
  if (kind == K_FIELD_X) lo = b.n[0] + 8;
  if (kind == K_FLUID_Y || kind == K_FLUID_Z || kind == K_FIELD_Y || kind == K_FIELD_Z) lo = 8;
  int par = 1;
  while (target / 2 >= lo && kind_waves(b, kind, target, groups, &par) < 2048) target /= 2;
  return target;
}

// Segments per pencil of a y/z kind, ceil(n_d / segment length); 0 for the
// other kinds.
static int kind_segments(const HostBox& b, int kind, int par) {
  if (kind == K_FLUID_X) return (b.n[0] + par - 1) / par;  // read by the strided layout only
  if (kind == K_FLUID_Y || kind == K_FIELD_Y) return (b.n[1] + par - 1) / par;
  if (kind == K_FLUID_Z || kind == K_FIELD_Z) return (b.n[2] + par - 1) / par;
  return 0;
}

void plan_single_box(const int n[3], const int bc[3], int par[K_NUM], int nseg[K_NUM], long long waves[K_NUM]) {
  HostBox b;
  for (int a = 0; a < 3; ++a) {
    b.n[a] = n[a];
    b.bc[a] = bc[a];
    b.o[a] = bc[a] == 1 ? 1 : 0;
  }
  const Tuning t = default_tuning();
  for (int k = 0; k < K_NUM; ++k) {
    const int target = single_box_target(b, k, t.target[k], t.groups[k]);
    waves[k] = kind_waves(b, k, target, t.groups[k], &par[k]);
    nseg[k] = kind_segments(b, k, par[k]);
  }
}

int Engine::build_lists() {
  std::vector<int> slots;
  for (int s = 0; s < (int)boxes.size(); ++s)
    if (boxes[s].used && boxes[s].have_state && !boxes[s].parked) slots.push_back(s);
  const int nb = (int)slots.size();
  std::vector<BoxDesc> desc(nb);
  std::vector<int> list[K_NUM];
  // irregular meshes: width offsets of every table box when any has widths
  bool anynu = false;
  long long wtotal[3] = {0, 0, 0};
  for (int s : slots)
    for (int a = 0; a < 3; ++a) anynu = anynu || !boxes[s].widths[a].empty();
  for (int s : slots)
    for (int a = 0; a < 3; ++a) {
      boxes[s].woff[a] = anynu ? wtotal[a] : 0;
      if (anynu) wtotal[a] += boxes[s].n[a];
    }
  for (int t = 0; t < nb; ++t) {
    const HostBox& b = boxes[slots[t]];
    BoxDesc& d = desc[t];
    std::memset(&d, 0, sizeof d);
    for (int a = 0; a < 3; ++a) {
      d.g.n[a] = b.n[a];
      d.g.bc[a] = b.bc[a];
      d.g.st[a] = b.st[a];
      d.g.h[a] = b.h[a];
    }
    d.off = b.off;
    d.cfl = b.cfl;
    for (int a = 0; a < 3; ++a) {
      d.ih[a] = 1.0 / b.h[a];
      d.i2h[a] = 1.0 / (2.0 * b.h[a]);
    }
    d.slot = slots[t];
    for (int a = 0; a < 3; ++a) d.woff[a] = b.woff[a];
    const Tuning defaults = default_tuning();
    for (int k = 0; k < K_NUM; ++k) {
      int par = 1;
      int target = tuning.target[k];
      if (nb == 1 && target == defaults.target[k]) target = single_box_target(b, k, target, tuning.groups[k]);
      const long long w = kind_waves(b, k, target, tuning.groups[k], &par);
      if ((long long)list[k].size() + w >= (1ll << 31) / 64)
        return fail(5, "work list exceeds the launch size");
      d.wave0[k] = (int)list[k].size();
      d.par[k] = par;
      d.nseg[k] = kind_segments(b, k, par);
      list[k].insert(list[k].end(), (size_t)w, t);
    }
  }
  int rc = set_device();
  if (rc) return rc;
  if (anynu && (rc = esize == 8 ? upload_widths<double>(slots, wtotal) : upload_widths<float>(slots, wtotal)))
    return rc;
  nonuniform = anynu;
  for (int a = 0; a < 3; ++a) {
    flat[a] = nb > 0;
    for (int s : slots) flat[a] = flat[a] && boxes[s].n[a] == 1;
  }
  // the spare set is written once every launch that read it has completed
  HIP_TRY(hipEventSynchronize(spare.done));
  drop_retired_graphs();
  size_t total = sizeof(BoxDesc) * (size_t)nb;
  for (int k = 0; k < K_NUM; ++k) total += list[k].size() * sizeof(int);
  if (spare.host_bytes < total) {
    if (spare.host) (void)hipHostFree(spare.host);
    spare.host = nullptr;
    spare.host_bytes = 0;
    const size_t want = total + total / 4 + 4096;
    HIP_TRY(hipHostMalloc(&spare.host, want, hipHostMallocDefault));
    spare.host_bytes = want;
  }
  char* h = static_cast<char*>(spare.host);
  if (nb > 0) {
    std::memcpy(h, desc.data(), sizeof(BoxDesc) * nb);
    HIP_TRY(hipMemcpyAsync(spare.table.ptr, h, sizeof(BoxDesc) * nb, hipMemcpyHostToDevice, cfg.stream));
  }
  h += sizeof(BoxDesc) * nb;
  for (int k = 0; k < K_NUM; ++k) {
    const size_t bytes = list[k].size() * sizeof(int);
    if (spare.lists[k].bytes < bytes) {
      dev_free(spare.lists[k]);
      if ((rc = dev_alloc(spare.lists[k], bytes + bytes / 4))) return rc;
    }
    if (bytes) {
      std::memcpy(h, list[k].data(), bytes);
      HIP_TRY(hipMemcpyAsync(spare.lists[k].ptr, h, bytes, hipMemcpyHostToDevice, cfg.stream));
    }
    h += bytes;
    spare.nwaves[k] = (int)list[k].size();
  }
  spare.slots.swap(slots);
  // the current set stops being current behind everything enqueued so far
  HIP_TRY(hipEventRecord(list_done, cfg.stream));
  std::swap(table, spare.table);
  for (int k = 0; k < K_NUM; ++k) {
    std::swap(lists[k], spare.lists[k]);
    std::swap(nwaves[k], spare.nwaves[k]);
  }
  table_slots.swap(spare.slots);
  std::swap(list_host, spare.host);
  std::swap(list_host_bytes, spare.host_bytes);
  std::swap(list_done, spare.done);
  dirty = false;
  invalidate_graph();
  return 0;
}

int Engine::ensure_table() { return dirty ? build_lists() : 0; }


template <typename T>
int Engine::sub_operator(int op, int d) {
  if (op == 0) {
    switch (d) {
      case 0: return fluid_dispatch<T, 0>();
      case 1: return fluid_dispatch<T, 1>();
      default: return fluid_dispatch<T, 2>();
    }
  }
  switch (d) {
    case 0: return field_sweep<T, 0>();
    case 1: return field_sweep<T, 1>();
    default: return field_sweep<T, 2>();
  }
}

int Engine::run_sub(int op, int d) { return esize == 8 ? sub_operator<double>(op, d) : sub_operator<float>(op, d); }

template <typename T>
int Engine::launch_check_cfl() {
  CheckLaunch<T> L;
  for (int k = 0; k < 5; ++k) L.u[k] = (const T*)pool[cur[k]][k].ptr;
  for (int k = 0; k < 3; ++k) L.b[k] = (const T*)pool[cur[5 + k]][5 + k].ptr;
  for (int k = 0; k < 3; ++k) L.wid[k] = nonuniform ? (const T*)wid[k].ptr : nullptr;
  L.gamma = cfg.gamma;
  L.wl = make_wl(this, K_CHECK);
  L.sc = (Scalars*)scal.ptr;
  const int nb = (int)table_slots.size();
  if (nb == 0) return 0;
  hipLaunchKernelGGL(reset_cmax_kernel, dim3(grid_for(nb)), dim3(kBlock), 0, cfg.stream,
                     (const BoxDesc*)table.ptr, nb, (Scalars*)scal.ptr);
  if (L.wl.nwaves > 0) {
    TimedLaunch tl(this, 8);
    hipLaunchKernelGGL((check_cfl_kernel<T>), dim3(grid_for((long long)L.wl.nwaves * 64)), dim3(kBlock), 0,
                       cfg.stream, L);
  }
  return launch_check();
}

// Width arrays of the table's boxes (build_lists): box t's widths along axis
// a at woff[a]; a box without widths on an axis gets its uniform spacing.
// Launches still in flight may read the old arrays, so the stream is drained
// first (only when the set of boxes changes on an irregular mesh).
template <typename T>
int Engine::upload_widths(const std::vector<int>& slots, const long long* total) {
  HIP_TRY(hipStreamSynchronize(cfg.stream));
  for (int a = 0; a < 3; ++a) {
    std::vector<T> w((size_t)total[a]);
    for (int s : slots) {
      const HostBox& b = boxes[s];
      for (int i = 0; i < b.n[a]; ++i)
        w[(size_t)(b.woff[a] + i)] = (T)(b.widths[a].empty() ? b.h[a] : b.widths[a][i]);
    }
    const size_t bytes = w.size() * sizeof(T);
    if (wid[a].bytes < bytes) {
      dev_free(wid[a]);
      int rc = dev_alloc(wid[a], bytes);
      if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(wid[a].ptr, w.data(), bytes, hipMemcpyHostToDevice, cfg.stream));
    HIP_TRY(hipStreamSynchronize(cfg.stream));
  }
  return 0;
}

// Irregular mesh (Sect. 2.5) of one box along axis: kept on the host and
// converted to the storage precision when the table is rebuilt; the other
// axes keep their uniform width until they are set too.
int Engine::set_spacing(int slot, int axis, const double* widths) {
  if (slot < 0 || slot >= (int)boxes.size() || !boxes[slot].used) return fail(1, "no box");
  HostBox& b = boxes[slot];
  b.widths[axis].assign(widths, widths + b.n[axis]);
  b.cfl_fresh = false;  // its CFL speed depends on the widths
  dirty = true;         // the width arrays are rebuilt with the table
  invalidate_graph();
  return 0;
}

// The CFL speed of boxes just added (their step scalars start at zero): the
// check kernel over the table without the reset; a box already fresh gets
// its own value again (the same function of the same state).
int Engine::check_new() {
  int rc = ensure_table();
  if (rc) return rc;
  if (table_slots.empty()) return 0;
  if (esize == 8) {
    CheckLaunch<double> L;
    for (int k = 0; k < 5; ++k) L.u[k] = (const double*)pool[cur[k]][k].ptr;
    for (int k = 0; k < 3; ++k) L.b[k] = (const double*)pool[cur[5 + k]][5 + k].ptr;
    for (int k = 0; k < 3; ++k) L.wid[k] = nonuniform ? (const double*)wid[k].ptr : nullptr;
    L.gamma = cfg.gamma;
    L.wl = make_wl(this, K_CHECK);
    L.sc = (Scalars*)scal.ptr;
    if (L.wl.nwaves > 0)
      hipLaunchKernelGGL((check_cfl_kernel<double>), dim3(grid_for((long long)L.wl.nwaves * 64)), dim3(kBlock), 0,
                         cfg.stream, L);
  } else {
    CheckLaunch<float> L;
    for (int k = 0; k < 5; ++k) L.u[k] = (const float*)pool[cur[k]][k].ptr;
    for (int k = 0; k < 3; ++k) L.b[k] = (const float*)pool[cur[5 + k]][5 + k].ptr;
    for (int k = 0; k < 3; ++k) L.wid[k] = nonuniform ? (const float*)wid[k].ptr : nullptr;
    L.gamma = cfg.gamma;
    L.wl = make_wl(this, K_CHECK);
    L.sc = (Scalars*)scal.ptr;
    if (L.wl.nwaves > 0)
      hipLaunchKernelGGL((check_cfl_kernel<float>), dim3(grid_for((long long)L.wl.nwaves * 64)), dim3(kBlock), 0,
                         cfg.stream, L);
  }
  if ((rc = launch_check())) return rc;
  for (int s : table_slots) boxes[s].cfl_fresh = true;
  return 0;
}

int Engine::check_cfl_all() {
  int rc = ensure_table();
  if (rc) return rc;
  rc = esize == 8 ? launch_check_cfl<double>() : launch_check_cfl<float>();
  if (rc) return rc;
  for (int s : table_slots) boxes[s].cfl_fresh = true;
  return 0;
}

// The launches of one double step with every box's CFL step: dt from the
// CFL speed of the current state (with t += 2 dt and the maximum cleared in
// the same kernel), the twelve sub-operators of Eqs. (12)-(13) in symmetric
// order, the CFL speed of the new state reduced by the last sweep.
int Engine::enqueue_step_cfl() {
  const int nb = (int)table_slots.size();
  const BoxDesc* tb = (const BoxDesc*)table.ptr;
  Scalars* sc = (Scalars*)scal.ptr;
  int rc;
  hipLaunchKernelGGL(begin_step_kernel, dim3(grid_for(nb)), dim3(kBlock), 0, cfg.stream, tb, nb, sc, 0.0);
  if ((rc = launch_check())) return rc;
  for (int d = 0; d < 3; ++d) {
    if ((rc = run_sub(0, d))) return rc;
    if ((rc = run_sub(1, d))) return rc;
  }
  for (int d = 2; d >= 1; --d) {
    if ((rc = run_sub(1, d))) return rc;
    if ((rc = run_sub(0, d))) return rc;
  }
  if ((rc = run_sub(1, 0))) return rc;
  return last_sweep_and_cfl();
}

// The last L_x of a step and the CFL speed of the state it leaves: reduced by
// the sweep itself, or by the check kernel after it (tuning choice; the same
// per-cell function, so the same value either way).
int Engine::last_sweep_and_cfl() {
  int rc;
  // the strided x layout has no fused reduction: the check kernel follows it
  if (tuning.groups[K_CHECK] || tuning.groups[K_FLUID_X]) {
    if ((rc = run_sub(0, 0))) return rc;
    return esize == 8 ? launch_check_cfl<double>() : launch_check_cfl<float>();  // resets cmax first
  }
  last_fluid_cfl = true;  // the step's begin_step_kernel cleared the maximum
  rc = run_sub(0, 0);
  last_fluid_cfl = false;
  return rc;
}

int Engine::strang_step(double dt) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;
  if (table_slots.empty()) return 0;
  bool fresh = true;
  for (int s : table_slots) fresh = fresh && boxes[s].cfl_fresh;
  if (dt == 0.0) {
    if (!fresh && (rc = check_cfl_all())) return rc;
    if ((rc = enqueue_step_cfl())) return rc;
  } else {
    // a given step size (one box): every sub-operator of size dt
    hipLaunchKernelGGL(begin_step_kernel, dim3(grid_for((long long)table_slots.size())), dim3(kBlock), 0, cfg.stream,
                       (const BoxDesc*)table.ptr, (int)table_slots.size(), (Scalars*)scal.ptr, dt);
    if ((rc = launch_check())) return rc;
    for (int d = 0; d < 3; ++d) {
      if ((rc = run_sub(0, d))) return rc;
      if ((rc = run_sub(1, d))) return rc;
    }
    for (int d = 2; d >= 1; --d) {
      if ((rc = run_sub(1, d))) return rc;
      if ((rc = run_sub(0, d))) return rc;
    }
    if ((rc = run_sub(1, 0))) return rc;
    if ((rc = last_sweep_and_cfl())) return rc;
  }
  for (int s : table_slots) boxes[s].cfl_fresh = true;
  return 0;
}

// One kind's work shape in the autotuner's encoding: the shape (positions
// per wave, segment length or cells per lane) in bits 0-15, the XCD-grouped
// block order in bit 16, the alternative layout in bit 17.
int Engine::set_shape(int kind, int value) {
  if (kind < 0 || kind >= K_NUM) return fail(1, "no such kernel kind");
  const int target = value & 0xFFFF, remap = (value >> 16) & 1, alt = (value >> 17) & 1;
  if (target < 1 || (value >> 18) != 0) return fail(1, "bad shape value");
  tuning.target[kind] = target;
  tuning.remap[kind] = remap;
  tuning.groups[kind] = alt;
  dirty = true;
  invalidate_graph();
  return 0;
}

int Engine::set_graph(bool on) {
  use_graph = on;
  if (!on) invalidate_graph();
  return 0;
}

// nsteps CFL-stepped double steps of every box.  With graphs on, the launches
// of one step are captured once per table and replayed.
int Engine::steps(int nsteps) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;
  if (table_slots.empty() || nsteps <= 0) return 0;
  bool fresh = true;
  for (int s : table_slots) fresh = fresh && boxes[s].cfl_fresh;
  if (!fresh && (rc = check_cfl_all())) return rc;
  if (!use_graph || timing_mask) {
    for (int i = 0; i < nsteps; ++i)
      if ((rc = enqueue_step_cfl())) return rc;
    return 0;
  }
  if (!graph_ok) {
    // the buffer parity of every field is the same after a whole step, so
    // one captured step can be replayed any number of times
    int saved[8];
    std::memcpy(saved, cur, sizeof cur);
    HIP_TRY(hipStreamBeginCapture(cfg.stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_step_cfl();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cfg.stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      std::memcpy(cur, saved, sizeof cur);
      return rc;
    }
    if (e != hipSuccess) return fail(3, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    for (int f = 0; f < 8; ++f)
      if (cur[f] != saved[f]) {
        (void)hipGraphDestroy(g);
        return fail(3, "a captured step must return every field to its buffer");
      }
    graph = g;
    e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      invalidate_graph();
      return fail(3, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    graph_ok = true;
  }
  for (int i = 0; i < nsteps; ++i) HIP_TRY(hipGraphLaunch(gexec, cfg.stream));
  return 0;
}

// CFL-stepped double steps of one box (an engine with one box) until its time
// reaches t_end: the device clamps each step so that the last lands on t_end
// and later ones take dt = 0 (exact no-ops).  Steps run in chunks sized from
// the current CFL step, as captured replays on a stream of the caller's (the
// null stream cannot be captured: eager launches there); the host reads the
// step scalars once per chunk.
int Engine::advance_to(int slot, double t_end, int max_steps, int* taken, double* t_out) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;
  if (table_slots.size() != 1) return fail(5, "advance_to takes an engine with one box");
  if (!boxes[slot].cfl_fresh && (rc = check_cfl_all())) return rc;
  Scalars s;
  if ((rc = read_scalars(slot, &s))) return rc;
  const int taken0 = s.taken;
  hipLaunchKernelGGL(set_end_kernel, dim3(1), dim3(1), 0, cfg.stream, (Scalars*)scal.ptr + slot, t_end, 1);
  if ((rc = launch_check())) return rc;
  const bool graph_was = use_graph;
  use_graph = timing_mask == 0 && cfg.stream != nullptr;  // the null stream cannot be captured
  int done = 0;
  while (done < max_steps && !s.status && s.t < t_end) {
    // remaining double steps at the current CFL step, plus one for the landing
    double cm;
    std::memcpy(&cm, &s.cmax_bits, sizeof cm);
    const double dt = cm > 0.0 ? boxes[slot].cfl / cm : 0.0;
    double est = dt > 0.0 ? (t_end - s.t) / (2.0 * dt) + 1.0 : 1.0;
    const int k = (int)std::min<double>({est, 64.0, (double)(max_steps - done)});
    if ((rc = steps(std::max(1, k)))) break;
    done += std::max(1, k);
    if ((rc = read_scalars(slot, &s))) break;
  }
  use_graph = graph_was;
  if (!graph_was) invalidate_graph();
  hipLaunchKernelGGL(set_end_kernel, dim3(1), dim3(1), 0, cfg.stream, (Scalars*)scal.ptr + slot, 0.0, 0);
  int rc2 = launch_check();
  if (!rc && !rc2) rc2 = read_scalars(slot, &s);
  if (rc) return rc;
  if (rc2) return rc2;
  if (taken) *taken = s.taken - taken0;
  if (t_out) *t_out = s.t;
  if (s.status) return fail(4, "the state went bad (rho <= 0, p <= 0 or a non-finite value)");
  return 0;
}

int Engine::sweep(int slot, int op, int dir, double dt) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;
  // the sub-operator of one box: its step factors from its table entry
  const auto it = std::find(table_slots.begin(), table_slots.end(), slot);
  if (it == table_slots.end()) return fail(1, "the box has no state");
  hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(1), 0, cfg.stream,
                     (const BoxDesc*)table.ptr + (it - table_slots.begin()), 1, (Scalars*)scal.ptr, dt);
  if ((rc = launch_check())) return rc;
  for (int s : table_slots) boxes[s].cfl_fresh = false;
  return run_sub(op, dir);
}

template <typename T>
int Engine::launch_diag(int slot) {
  const HostBox& b = boxes[slot];
  DiagArgs<T> a;
  for (int k = 0; k < 5; ++k) a.u[k] = (const T*)pool[cur[k]][k].ptr + b.off;
  for (int k = 0; k < 3; ++k) a.b[k] = (const T*)pool[cur[5 + k]][5 + k].ptr + b.off;
  for (int k = 0; k < 3; ++k) a.wid[k] = nonuniform ? (const T*)wid[k].ptr + b.woff[k] : nullptr;
  for (int x = 0; x < 3; ++x) {
    a.g.n[x] = b.n[x];
    a.g.bc[x] = b.bc[x];
    a.g.st[x] = b.st[x];
    a.g.h[x] = b.h[x];
  }
  a.partial = static_cast<double*>(partial.ptr);
  const long long ncell = (long long)b.n[0] * b.n[1] * b.n[2];
  const int nblk = (int)std::min<long long>(npartial, std::max<long long>(1, ncell / 4096));
  const long long per_block = (ncell + nblk - 1) / nblk;
  hipLaunchKernelGGL((diag_partial_kernel<T>), dim3(nblk), dim3(kBlock), 0, cfg.stream, a, per_block);
  // irregular mesh: every cell and face already carries its own volume or area
  const double vol = nonuniform ? 1.0 : b.h[0] * b.h[1] * b.h[2];
  const double ax = nonuniform ? 1.0 : b.h[1] * b.h[2], ay = nonuniform ? 1.0 : b.h[0] * b.h[2],
               az = nonuniform ? 1.0 : b.h[0] * b.h[1];
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(1), 0, cfg.stream, static_cast<const double*>(partial.ptr),
                     nblk, static_cast<double*>(diag_out.ptr), vol, ax, ay, az);
  return launch_check();
}

int Engine::diagnostics(int slot, double* out10) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;  // the width arrays follow the table
  if (nonuniform && std::find(table_slots.begin(), table_slots.end(), slot) == table_slots.end())
    return fail(5, "diagnostics of a box outside the launches on an irregular mesh");
  rc = esize == 8 ? launch_diag<double>(slot) : launch_diag<float>(slot);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(out10, diag_out.ptr, 10 * sizeof(double), hipMemcpyDeviceToHost, cfg.stream));
  HIP_TRY(hipStreamSynchronize(cfg.stream));
  return 0;
}

// Autotuner: for each sweep kind, time its kernel over the current table for
// every candidate shape and keep the fastest.  The timed launches write the
// idle buffers only (no buffer flips), so the state is unchanged.
int Engine::autotune(int reps, int* chosen) {
  int rc = set_device();
  if (rc) return rc;
  if ((rc = ensure_table())) return rc;
  if (table_slots.empty()) return fail(1, "no box with a state to tune on");
  bool fresh = true;
  for (int s : table_slots) fresh = fresh && boxes[s].cfl_fresh;
  if (!fresh && (rc = check_cfl_all())) return rc;
  // a valid dt in every box for the timed sweeps
  const int nb = (int)table_slots.size();
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(grid_for(nb)), dim3(kBlock), 0, cfg.stream, (const BoxDesc*)table.ptr,
                     nb, (Scalars*)scal.ptr);
  if ((rc = launch_check())) return rc;
  static const int lanes_c[] = {256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144};
  static const int seg_c[] = {8, 16, 24, 32, 48, 64, 96, 128, 192, 256};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int saved_mask = timing_mask;
  timing_mask = 0;
  for (int kind = K_FLUID_X; kind <= K_FIELD_Z; ++kind) {
    const bool lanes = kind == K_FLUID_X || kind == K_FIELD_X;
    const int* cand = lanes ? lanes_c : seg_c;
    const int ncand = lanes ? (int)(sizeof lanes_c / sizeof(int)) : (int)(sizeof seg_c / sizeof(int));
    // second knob: the pencil order of the y/z kinds, two positions per lane
    // for the x field sweep
    const int nord = (lanes && kind != K_FIELD_X) ? 1 : 2;
    const int op = kind >= K_FIELD_X ? 1 : 0;
    const int d = op ? kind - K_FIELD_X : kind - K_FLUID_X;
    float best = 1e30f;
    int best_t = tuning.target[kind], best_r = tuning.remap[kind], best_g = tuning.groups[kind];
    std::vector<long long> seen;
    for (int cj = 0; cj < ncand * 2 * nord && !rc; ++cj) {
      const int ci = cj / (2 * nord), r = cj % 2, g = (cj / 2) % nord;
      tuning.target[kind] = cand[ci];
      tuning.remap[kind] = r;
      tuning.groups[kind] = g;
      // skip variants that give every box a shape already timed
      long long sig = 0;
      for (int s : table_slots) {
        int par = 0;
        const long long w = kind_waves(boxes[s], kind, cand[ci], g, &par);
        sig = sig * 1000003 + par * 7919 + w;
      }
      sig = sig * 4 + r * 2 + g;
      if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
      seen.push_back(sig);
      if ((rc = build_lists())) break;
      int saved[8];
      std::memcpy(saved, cur, sizeof cur);
      // the x fluid kind runs twice per step, once with the fused CFL
      // reduction (fewer waves per SIMD): a shape is timed on both
      auto one = [&]() {
        int r1 = run_sub(op, d);
        std::memcpy(cur, saved, sizeof cur);
        if (!r1 && kind == K_FLUID_X) {
          last_fluid_cfl = true;
          r1 = run_sub(op, d);
          last_fluid_cfl = false;
          std::memcpy(cur, saved, sizeof cur);
        }
        return r1;
      };
      if ((rc = one())) break;  // warm-up
      (void)hipEventRecord(e0, cfg.stream);
      for (int rr = 0; rr < reps && !rc; ++rr) rc = one();
      (void)hipEventRecord(e1, cfg.stream);
      if (rc) break;
      hipError_t e = hipEventSynchronize(e1);
      if (e != hipSuccess) {
        rc = fail(3, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_t = cand[ci];
        best_r = r;
        best_g = g;
      }
    }
    tuning.target[kind] = best_t;
    tuning.remap[kind] = best_r;
    tuning.groups[kind] = best_g;
    if (chosen) chosen[kind] = best_t | (best_r << 16) | (best_g << 17);
    if (rc) break;
  }
  // the CFL speed of a step's new state: fused into the last x sweep, or the
  // check kernel after a plain one (both time the x sweep too)
  if (!rc) {
    if ((rc = build_lists())) goto done;
    float tbest = 1e30f;
    int gbest = tuning.groups[K_CHECK];
    for (int gsel = 0; gsel < 2 && !rc; ++gsel) {
      tuning.groups[K_CHECK] = gsel;
      int saved[8];
      std::memcpy(saved, cur, sizeof cur);
      if ((rc = last_sweep_and_cfl())) break;  // warm-up
      std::memcpy(cur, saved, sizeof cur);
      (void)hipEventRecord(e0, cfg.stream);
      for (int rr = 0; rr < reps && !rc; ++rr) {
        rc = last_sweep_and_cfl();
        std::memcpy(cur, saved, sizeof cur);
      }
      (void)hipEventRecord(e1, cfg.stream);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(3, "hipEventSynchronize failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < tbest) {
        tbest = ms;
        gbest = gsel;
      }
    }
    tuning.groups[K_CHECK] = gbest;
  }
done:
  timing_mask = saved_mask;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (chosen) chosen[K_CHECK] = tuning.target[K_CHECK] | (tuning.groups[K_CHECK] << 17);
  dirty = true;
  int rc2 = ensure_table();
  // the timed sweeps left the CFL speeds of other states: reduce the current one again
  if (!rc && !rc2) rc2 = check_cfl_all();
  return rc ? rc : rc2;
}

// ------------------------------------------------------------ launches (launch_api.h)
template <typename T>
void launch_check(const CheckLaunch<T>& L, hipStream_t stream) {
  if (L.wl.nwaves > 0)
    hipLaunchKernelGGL((check_cfl_kernel<T>), dim3(grid_for((long long)L.wl.nwaves * 64)), dim3(kBlock), 0, stream, L);
}
template void launch_check<float>(const CheckLaunch<float>&, hipStream_t);
template void launch_check<double>(const CheckLaunch<double>&, hipStream_t);

void launch_begin_step(const BoxDesc* boxes, int nb, Scalars* sc, double dt, hipStream_t stream) {
  hipLaunchKernelGGL(begin_step_kernel, dim3(grid_for(nb)), dim3(kBlock), 0, stream, boxes, nb, sc, dt);
}

int selftest_lane_shift(int device, float* out128) {
  if (hipSetDevice(device) != hipSuccess) return 3;
  float* d = nullptr;
  if (hipMalloc(&d, 128 * sizeof(float)) != hipSuccess) return 2;
  hipLaunchKernelGGL(lane_shift_selftest_kernel, dim3(1), dim3(64), 0, nullptr, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(out128, d, 128 * sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? 0 : 3;
}

int selftest_math(int device, int n, const double* x, double* rcp_out, double* sqrt_out) {
  if (hipSetDevice(device) != hipSuccess) return 3;
  const size_t bytes = (size_t)n * sizeof(double);
  double* d = nullptr;
  if (hipMalloc(&d, 3 * bytes) != hipSuccess) return 2;
  hipError_t e = hipMemcpy(d, x, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(math_selftest_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, nullptr, d, d + n,
                       d + 2 * (size_t)n, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(rcp_out, d + n, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(sqrt_out, d + 2 * (size_t)n, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? 0 : 3;
}

}  // namespace fish
