// engine.h -- host engine of the FISH split MHD step on gfx950: one stream,
// one pool per field (two buffers each), any number of boxes at element
// offsets of the pools, a device box table and per-kernel work lists, and
// the sequencing of the sub-operators.  The single-box context and the batch
// of the C interface are both an Engine; every step of the arithmetic runs in
// the kernels of sweeps.h.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "layout.h"

namespace fish {

struct SweepSel;

struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// One box of the engine (host side).
struct HostBox {
  bool used = false;
  bool have_state = false;
  bool cfl_fresh = false;   // its Scalars::cmax_bits holds the CFL speed of its state
  int n[3]{};
  int o[3]{};               // extra layer on outflow axes
  int bc[3]{};
  double h[3]{};
  double cfl = 0.5;
  long long st[3]{};        // element strides (1, sy, sz)
  long long nelem = 0;      // elements per array
  long long off = 0;        // element offset in every pool
  long long reserved = 0;   // elements reserved in the pools (aligned)
  bool parked = false;      // kept (state readable) but out of the launches
  hipEvent_t ready = nullptr;  // parked: completes after the last launch that touched the box
  std::vector<double> widths[3];  // irregular mesh (Sect. 2.5): cell widths per axis, empty = uniform
  long long woff[3]{};            // offset of the box's widths in the engine's width arrays (table boxes)
};

struct EngineConfig {
  int precision = 0;        // 0 FP64, 1 FP32
  double gamma = 5.0 / 3.0;
  double alpha = 1.0;
  int limiter = 1;
  int gravity = 0;
  int hse = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free)(void*, size_t, void*, void*) = nullptr;
  void* alloc_user = nullptr;
};

// Tuning targets per kernel kind: stream positions per wave for the x kinds
// (whole rows of the box fill it), the segment length along the sweep for
// the y/z kinds, cells per lane for the CFL check.
struct Tuning {
  int target[K_NUM];
  int remap[K_NUM];   // XCD-aware block order per kind (0/1)
  int groups[K_NUM];  // y/z kinds: waves of a block on consecutive rows; x field kind: two
                      // stream positions per lane; check kind: the step's CFL reduction in
                      // the check kernel instead of the last x sweep (0/1)
};
Tuning default_tuning();

class Engine {
 public:
  EngineConfig cfg;
  bool live = false;        // init ran; release() frees once
  size_t esize = 8;
  std::string err;
  size_t device_bytes = 0;

  // pools: [buffer][field] with fields rho, m_x, m_y, m_z, E, b_x, b_y, b_z
  long long cap = 0;  // elements per pool
  DeviceBuf pool[2][8];
  DeviceBuf phi;
  // irregular meshes (Sect. 2.5): when a box of the table has cell widths,
  // the widths of every table box per axis in the storage precision (the
  // uniform boxes' filled with their spacing), at BoxDesc::woff, and every
  // sweep takes per-cell widths
  DeviceBuf wid[3];
  bool nonuniform = false;
  // axes along which every table box has one cell: the fluid sweep there is
  // the identity (every ghost is the cell itself, so every flux difference
  // and every potential difference is zero) and is not launched
  bool flat[3] = {false, false, false};
  int cur[8]{};
  std::map<long long, long long> free_list;  // offset -> length (elements)

  std::vector<HostBox> boxes;  // slots
  DeviceBuf scal;              // Scalars per slot
  DeviceBuf partial, diag_out;
  int npartial = 1024;

  // device table and work lists (rebuilt when the set of boxes changes); two
  // sets alternate, so that a rebuild never waits for launches still reading
  // the current one
  DeviceBuf table;
  DeviceBuf lists[K_NUM];
  int nwaves[K_NUM]{};
  std::vector<int> table_slots;
  void* list_host = nullptr;       // pinned staging of the uploads into this set
  size_t list_host_bytes = 0;
  hipEvent_t list_done = nullptr;  // recorded when this set stops being current
  struct ListSet {
    DeviceBuf table;
    DeviceBuf lists[K_NUM];
    int nwaves[K_NUM]{};
    std::vector<int> slots;
    void* host = nullptr;
    size_t host_bytes = 0;
    hipEvent_t done = nullptr;
  } spare;
  bool dirty = true;
  Tuning tuning = default_tuning();

  // graph of one CFL-stepped double step for the current table
  bool use_graph = false;
  bool graph_ok = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct RetiredGraph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t after;  // completes after every launch of the graph
  };
  std::vector<RetiredGraph> retired_graphs;

  bool last_fluid_cfl = false;

  // host transfers: pinned staging pair on the copy stream
  static constexpr size_t kStageBytes = 32u << 20;
  hipStream_t copy_stream = nullptr;
  hipEvent_t copy_ev = nullptr, compute_ev = nullptr;
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  void* stage[2] = {nullptr, nullptr};
  size_t stage_bytes = 0;

  // measurement hook
  int timing_mask = 0;
  int timing_max = 0;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;

  ~Engine();
  int fail(int code, const std::string& msg);
  int init(const EngineConfig& c, long long cap_elems, int max_boxes);
  void release();
  int set_device();

  // boxes
  static int validate_box(const int n[3], const double h[3], const int bc[3], double cfl);
  long long box_elems(const int n[3], const int bc[3]) const;
  int add_box(const int n[3], const double h[3], const int bc[3], double cfl, int* slot);
  int remove_box(int slot);
  int park(int slot);
  int upload(int slot, const double* cell5, const double* bx, const double* by, const double* bz,
             const double* phi_in);
  int download(int slot, double* cell5, double* bx, double* by, double* bz);
  int read_scalars(int slot, Scalars* out);
  int read_scalars_parked(int slot, Scalars* out);
  int count() const;
  long long free_elems() const;

  // stepping
  int ensure_table();
  int check_cfl_all();
  int check_new();
  int strang_step(double dt);               // every box of the table
  int steps(int nsteps);                    // CFL-stepped double steps, graph when enabled
  int advance_to(int slot, double t_end, int max_steps, int* taken, double* t_out);
  int sweep(int slot, int op, int dir, double dt);
  int diagnostics(int slot, double* out10);
  int autotune(int reps, int* chosen);
  int set_shape(int kind, int value);
  int set_graph(bool on);
  int set_spacing(int slot, int axis, const double* widths);  // irregular mesh along axis

 private:
  int ensure_stage(size_t bytes);
  int dev_alloc(DeviceBuf& b, size_t bytes);
  void dev_free(DeviceBuf& b);
  int launch_check();
  int run_sub(int op, int d);
  int enqueue_step_cfl();                   // the launches of one CFL-stepped double step
  int last_sweep_and_cfl();
  void invalidate_graph();
  template <typename T>
  int upload_widths(const std::vector<int>& slots, const long long* total);
  void drop_retired_graphs();
  int build_lists();
  template <typename T>
  int sub_operator(int op, int d);
  SweepSel sweep_sel() const;               // the kernel selection of the sweeps
  template <typename T, int D>
  int fluid_dispatch();
  template <typename T, int D>
  int field_sweep();
  template <typename T>
  int launch_check_cfl();
  template <typename T>
  int launch_diag(int slot);
  template <typename T>
  int upload_t(int slot, const double* cell5, const double* bx, const double* by, const double* bz,
               const double* phi_in);
  template <typename T>
  int download_t(int slot, double* cell5, double* bx, double* by, double* bz);
  friend struct TimedLaunch;
};

// Run the lane-shift self-test kernel on `device` (out128: host, 128 values).
int selftest_lane_shift(int device, float* out128);

// Run the FP64 reciprocal/square-root self-test kernel on `device` (host
// arrays of n values, 1 <= n <= 2^24).
int selftest_math(int device, int n, const double* x, double* rcp_out, double* sqrt_out);

}  // namespace fish
