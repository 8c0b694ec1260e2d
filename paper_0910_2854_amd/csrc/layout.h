// layout.h -- data structures shared by the host engine and the kernels:
// box geometry, per-box step scalars, the box table and the work lists.
#pragma once

namespace fish {

struct Geo {
  int n[3];
  int bc[3];          // 0 periodic, 1 outflow
  long long st[3];    // element strides, st[0] = 1
  double h[3];
};

// Device-resident step scalars.
struct Scalars {
  double dt;                    // step size of every sub-operator
  double t;                     // simulation time
  double t_end;                 // with has_end: the CFL step is clamped to land on t_end
  unsigned long long cmax_bits; // max CFL speed (FP64 bits; all values >= 0)
  int status;                   // sticky: 1 = bad state seen
  int has_end;
  int taken;                    // double steps taken with dt > 0
  int pad;
  double kh[3], kf[3];          // dt / (2 h_d) and dt / h_d per axis, set with dt
};

// ------------------------------------------------------------ work lists
// A launch covers every box of a batch.  Boxes live at element offset `off`
// of one pool per field; each kernel kind has a list giving the box of every
// wave, and the box gives the wave's position within it.  The box, its
// geometry and its offset are wave-uniform (scalar registers).
enum Kind { K_FLUID_X = 0, K_FLUID_Y, K_FLUID_Z, K_FIELD_X, K_FIELD_Y, K_FIELD_Z, K_CHECK, K_NUM };

struct BoxDesc {
  Geo g;
  long long off;      // element offset of the box in every pool
  double cfl;         // Courant number of Eq. (14)
  int slot;           // index of the box's Scalars
  int wave0[K_NUM];   // first wave of the box in each kind's list
  int par[K_NUM];     // rows per wave (x kinds), segment length (y/z kinds), cells per lane (check)
  int nseg[K_NUM];    // y/z kinds: segments per pencil, ceil(n_d / par)
  long long woff[3];  // irregular meshes: element offset of the box's cell widths in each axis's width array
  double ih[3], i2h[3];  // 1 / h_d and 1 / (2 h_d)
};

struct WorkList {
  const BoxDesc* boxes;
  const int* wave_box;  // table index of the box of every wave
  int nwaves;
  int xcd_remap;        // 1: consecutive blocks of the list run on one XCD (see work_item)
  int row_groups;       // y/z kinds: 1 = a block's waves on consecutive rows (see strided_map)
};

}  // namespace fish
