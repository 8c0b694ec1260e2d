/*
 * fish.h -- C interface of the MI355X (gfx950) implementation of the FISH
 * operator-split ideal-MHD step (Kaeppeli, Whitehouse, Scheidegger, Pen &
 * Liebendoerfer, "FISH: A 3D parallel MHD code for astrophysical
 * applications", Sect. 2).
 *
 * One context advances one Cartesian box of cells.  The cell state is
 * u = (rho, m_x, m_y, m_z, E) (cell averages, Eq. 8) and the magnetic field
 * lives on the faces (face averages, Eqs. 9-11).  A double step applies the
 * symmetric product of fluid sweeps L_d (Sect. 2.2, with the unsplit gravity
 * of Sect. 2.3 and the hydrostatic-gradient subtraction of Eqs. 51-57) and
 * constrained-transport field sweeps B_d (Sect. 2.4), Eqs. (12)-(13).
 *
 * Conventions shared by every call:
 *  - Host arrays are FP64, C order, owned by the caller and copied on every
 *    call; the library never keeps a host pointer.
 *      cell5 : [5][nz][ny][nx]   rho, m_x, m_y, m_z, E
 *      bx    : [nz][ny][nx+1]    entry f is the face between cells f-1 and f
 *      by    : [nz][ny+1][nx]
 *      bz    : [nz+1][ny][nx]
 *      phi   : [nz][ny][nx]      fixed gravitational potential (G = 1)
 *    On a periodic axis face n duplicates face 0: it is ignored on input and
 *    written equal to face 0 on output.  On an outflow axis it is real.
 *  - Device memory is owned by the context (allocated through the callbacks
 *    of fish_params, or hipMalloc) and released by fish_destroy.
 *  - Work is enqueued on the stream of fish_params (NULL = the default
 *    stream).  fish_strang_step and fish_sweep return without waiting; the
 *    other calls synchronise the stream.
 *  - Every call returns a fish_status; no C++ exception crosses the
 *    interface.  fish_last_error gives a message for the last failure.
 *  - A state error found on the device (rho <= 0, p <= 0 or a non-finite
 *    value; there are no floors, a run stops on negative internal energy,
 *    Sect. 4.4) is sticky: fish_cfl_dt and fish_get_state report it until the
 *    next fish_set_state.
 *  - A context is not thread safe; distinct contexts on distinct streams may
 *    run concurrently.
 */
#ifndef FISH_H
#define FISH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fish_status {
  FISH_OK = 0,
  FISH_ERR_ARG = 1,         /* invalid argument or shape                    */
  FISH_ERR_NOMEM = 2,       /* device or host allocation failed             */
  FISH_ERR_DEVICE = 3,      /* a HIP runtime call or kernel launch failed   */
  FISH_ERR_STATE = 4,       /* rho <= 0, p <= 0 or a non-finite value       */
  FISH_ERR_UNSUPPORTED = 5  /* valid request this build does not implement  */
} fish_status;

enum { FISH_PERIODIC = 0, FISH_OUTFLOW = 1 };
enum { FISH_MINMOD = 0, FISH_VANLEER = 1 };
enum { FISH_FP64 = 0, FISH_FP32 = 1 };

typedef struct fish_params {
  int32_t nx, ny, nz;        /* interior cells per axis, >= 1 (1 = inactive axis)      */
  double dx, dy, dz;         /* uniform spacing > 0 (Sect. 2.1)                         */
  double gamma;              /* ratio of specific heats > 1, Eq. (5)                    */
  double cfl;                /* Courant number k of Eq. (14), 0 < k <= 1                */
  int32_t limiter;           /* FISH_MINMOD Eq. (29) or FISH_VANLEER Eq. (30)           */
  double predictor_alpha;    /* predictor dissipation scale in [0, 1] (Sect. 2.2)       */
  int32_t bc[3];             /* per axis FISH_PERIODIC or FISH_OUTFLOW (Sect. 4, 4.6)   */
  int32_t precision;         /* FISH_FP64, or FISH_FP32 storage and arithmetic with FP64
                                pressure recovery, CFL reduction and totals            */
  int32_t gravity;           /* 0 none, 1 fixed potential, unsplit Eqs. (41)-(43)       */
  int32_t hse;               /* 0/1 hydrostatic-gradient subtraction (needs gravity)    */
  int32_t device;            /* HIP device ordinal                                      */
  void* stream;              /* hipStream_t to enqueue on, NULL = default stream        */
  /* Device allocator.  NULL alloc uses hipMalloc/hipFree.  alloc returns NULL on
   * failure; free receives the pointer, its size and the same stream/user. */
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* alloc_user;
} fish_params;

typedef struct fish_ctx fish_ctx;

/* Create a context for one box.  *out is NULL on failure.  Validates every
 * field of *p (FISH_ERR_ARG) and allocates the device state (FISH_ERR_NOMEM).
 * Each state array must stay below 4 GiB ((nx+o)(ny+o)(nz+o) elements of 4 or
 * 8 bytes, o = 1 on outflow axes), else FISH_ERR_UNSUPPORTED. */
int fish_create(const fish_params* p, fish_ctx** out);

/* Release the context and all its device memory.  NULL is a no-op. */
void fish_destroy(fish_ctx* ctx);

/* Message describing the last failure on ctx (never NULL). */
const char* fish_last_error(const fish_ctx* ctx);

/* Upload a state (layouts above).  phi is required when gravity is on and
 * ignored otherwise.  Values are converted to the storage precision.  Checks
 * the state and returns FISH_ERR_STATE (state kept, flag set) if a cell has
 * rho <= 0, p <= 0 or a non-finite value.  Resets the simulation time to 0
 * and clears the sticky state flag first.  Synchronises the stream. */
int fish_set_state(fish_ctx* ctx, const double* cell5, const double* bx, const double* by,
                   const double* bz, const double* phi);

/* Download the state (any pointer may be NULL to skip it) and the simulation
 * time.  Returns FISH_ERR_STATE if the state flag is set or the state fails
 * the check; the arrays are filled either way.  Synchronises the stream. */
int fish_get_state(fish_ctx* ctx, double* cell5, double* bx, double* by, double* bz,
                   double* t_out);

/* CFL step of the current state, Eq. (14) with Eq. (15):
 * dt = k / max over cells and active axes of (|v_d| + c_F,d)/dx_d, reduced in
 * FP64 on the device.  Synchronises the stream. */
int fish_cfl_dt(fish_ctx* ctx, double* dt_out);

/* One symmetric double step, Eqs. (12)-(13): the twelve sub-operators
 *   L_x B_x L_y B_y L_z B_z B_z L_z B_y L_y B_x L_x
 * each of size dt, then t += 2 dt.  dt > 0 is used as given; dt == 0 takes
 * the CFL step of the current state on the device (no host round trip).
 * Asynchronous. */
int fish_strang_step(fish_ctx* ctx, double dt);

/* One sub-operator for testing: op 0 = fluid L_dir, op 1 = field B_dir,
 * dir 0/1/2 = x/y/z, of size dt > 0.  Asynchronous. */
int fish_sweep(fish_ctx* ctx, int op, int dir, double dt);

/* Diagnostics of the current state, Eq. (18) and Eq. (62), reduced in FP64 in
 * a fixed order: out[0..4] = sums of rho, m_x, m_y, m_z, E times the cell
 * volume; out[5..7] = sums of bx, by, bz over the real faces times the face
 * area; out[8] = max |div b|; out[9] = max |b| over faces.  Synchronises. */
int fish_diagnostics(fish_ctx* ctx, double* out10);

/* Bytes of device memory the context holds (state, double buffers, scratch). */
size_t fish_device_bytes(const fish_ctx* ctx);

/* Kernel classes for the timing hook below. */
enum {
  FISH_KERNEL_FLUID = 1,       /* fluid sweep L_d                          */
  FISH_KERNEL_FIELD = 2,       /* field sweep B_d (advection + constraint) */
  FISH_KERNEL_CHECK = 8        /* CFL reduction and state check            */
};

/* Measurement hook (not part of the scheme): while enabled, every launch of a
 * kernel class in `mask` is bracketed by two hipEvents recorded on the
 * context's stream (at most max_launches launches are recorded).  mask == 0
 * disables it.  fish_timing_read synchronises the stream, returns the number
 * of recorded launches and their summed duration in milliseconds, and clears
 * the record. */
int fish_timing_enable(fish_ctx* ctx, int mask, int max_launches);
int fish_timing_read(fish_ctx* ctx, int* launches, double* total_ms);

/* Self-test of the wavefront lane-shift primitive the x sweeps stream with
 * (no context): one wave of 64 lanes runs two iterations with lane values
 * v = 100*it + lane; out128[64*it + lane] receives the value one stream
 * position back (lane-1 of the same iteration, lane 63 of the previous one
 * for lane 0; -1 before the first).  Synchronous; the caller owns out128. */
int fish_selftest_lane_shift(int device, float* out128);

#ifdef __cplusplus
}
#endif

#endif /* FISH_H */
