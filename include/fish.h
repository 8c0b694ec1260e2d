/*
 * fish.h -- C interface of the MI355X (gfx950) implementation of the FISH
 * operator-split ideal-MHD step (Kaeppeli, Whitehouse, Scheidegger, Pen &
 * Liebendoerfer, "FISH: A 3D parallel MHD code for astrophysical
 * applications", Sect. 2).
 *
 * One context advances one Cartesian box of cells.  The cell state is
 * u = (rho, m_x, m_y, m_z, E) (cell averages, Eq. 8) and the magnetic field
 * lives on the faces (face averages, Eqs. 9-11).  A double step applies the
 * symmetric product of fluid sweeps L_d (Sect. 2.2, with the unsplit or split
 * gravity of Sect. 2.3 and the hydrostatic-gradient subtraction of Eqs. 51-57) and
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
  FISH_ERR_UNSUPPORTED = 5  /* valid request the library does not implement */
} fish_status;

enum { FISH_PERIODIC = 0, FISH_OUTFLOW = 1 };
enum { FISH_MINMOD = 0, FISH_VANLEER = 1, FISH_MACH_SWITCH = 2 };
enum { FISH_FP64 = 0, FISH_FP32 = 1 };

typedef struct fish_params {
  int32_t nx, ny, nz;        /* interior cells per axis, >= 1 (1 = inactive axis)      */
  double dx, dy, dz;         /* uniform spacing > 0 (Sect. 2.1)                         */
  double gamma;              /* ratio of specific heats > 1, Eq. (5)                    */
  double cfl;                /* Courant number k of Eq. (14), 0 < k <= 1                */
  int32_t limiter;           /* FISH_MINMOD Eq. (29), FISH_VANLEER Eq. (30), or
                                FISH_MACH_SWITCH: van Leer where a cell's half-step
                                state has |v| <= c_S, minmod where |v| > c_S, in the
                                fluid sweeps (Sect. 2.2); the field advection then
                                keeps van Leer                                        */
  double predictor_alpha;    /* predictor dissipation scale in [0, 1] (Sect. 2.2)       */
  int32_t bc[3];             /* per axis FISH_PERIODIC or FISH_OUTFLOW (Sect. 4, 4.6)   */
  int32_t precision;         /* FISH_FP64, or FISH_FP32 storage and arithmetic with FP64
                                pressure recovery, CFL reduction and totals            */
  int32_t gravity;           /* 0 none; with a fixed potential phi: 1 unsplit, the
                                source in the predictor and corrector, Eqs. (41)-(43);
                                2 split, each L_d replaced by G_d(dt/2) L_d G_d(dt/2),
                                Eqs. (38)-(40): G_d changes m_d by -rho dphi/dx dt and
                                holds rho and the internal energy                      */
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

/* Message describing the last failure on ctx (never NULL).  With ctx NULL:
 * the message of the last fish_create, fish_batch_create or
 * fish_strang_step_noalloc that failed on the calling thread. */
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

/* CFL-stepped double steps until the box's time reaches t_end, with no host
 * round trip per step: the device clamps each step, dt = min(k/C, (t_end -
 * t)/2), so that the last one lands on t_end exactly (the steps a host loop
 * of fish_cfl_dt and fish_strang_step with that clamp would take, bitwise),
 * and takes dt = 0 once t_end is reached.  The steps run in chunks sized
 * from the current CFL step, as captured graph replays when the context has a
 * stream of its own (eager launches on the null stream); the host reads the
 * step scalars once per chunk.  At most max_steps double steps are enqueued.
 * *steps_taken (may be NULL) gets the double steps taken with dt > 0, *t_out
 * (may be NULL) the time reached.  FISH_ERR_STATE if the state went bad on
 * the way (the box stops, as in fish_strang_step).  Synchronises. */
int fish_advance_to(fish_ctx* ctx, double t_end, int max_steps, int* steps_taken, double* t_out);

/* One sub-operator for testing: op 0 = fluid L_dir, op 1 = field B_dir,
 * dir 0/1/2 = x/y/z, of size dt > 0.  Asynchronous. */
int fish_sweep(fish_ctx* ctx, int op, int dir, double dt);

/* Diagnostics of the current state, Eq. (18) and Eq. (62), reduced in FP64 in
 * a fixed order: out[0..4] = sums of rho, m_x, m_y, m_z, E times the cell
 * volume; out[5..7] = sums of bx, by, bz over the real faces times the face
 * area; out[8] = max |div b|; out[9] = max |b| over faces.  On an irregular
 * mesh (fish_set_spacing) each cell carries its own volume, each face its own
 * area and each divergence term its cell's width (Sect. 2.5).  Synchronises. */
int fish_diagnostics(fish_ctx* ctx, double* out10);

/* Irregular Cartesian mesh (Sect. 2.5): the widths of the n cells along axis
 * (0/1/2), host FP64 array of n values, all finite and > 0, copied.  From
 * then on every sweep and the CFL step use per-cell widths: the flux
 * differences of a cell divide by its own width (Eq. 69), the second-order
 * slopes divide each difference by the distance of its two cell centres and
 * are carried half a cell width to the interface, the gravity gradient spans
 * the two neighbouring centres, the face velocity of Eq. (65) interpolates
 * linearly between the two cell centres, the constraint update (Eq. 64) uses
 * the widths of the face's cell, and the CFL step takes each cell's widths
 * (Eq. 70).  Ghost cells take the width of the cell they map to.  Axes not
 * set keep the uniform width of fish_params.  The widths reach the device
 * at the next call that steps, after the stream has drained.
 * FISH_ERR_ARG for a bad axis, a null array or a width that is not finite
 * and positive. */
int fish_set_spacing(fish_ctx* ctx, int axis, const double* widths);

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

/* Kernel kinds of the sweeps, for the autotuner: the fluid sweeps along x, y,
 * z, the field sweeps along x, y, z, and the CFL check. */
enum {
  FISH_KIND_FLUID_X = 0, FISH_KIND_FLUID_Y, FISH_KIND_FLUID_Z,
  FISH_KIND_FIELD_X, FISH_KIND_FIELD_Y, FISH_KIND_FIELD_Z,
  FISH_KIND_CHECK, FISH_NUM_KINDS
};

/* Autotuner (not part of the scheme): times every candidate work shape of
 * each sweep kind on the current state, reps launches each, and keeps the
 * fastest; the state is unchanged.  Shapes: stream positions per wavefront
 * for the x kinds (whole rows), segment length along the sweep for the y/z
 * kinds, each with the plain or the XCD-grouped block order (consecutive
 * blocks of a launch on one XCD, sharing its L2), and with an alternative
 * layout: for the y/z kinds the four waves of a block on four consecutive
 * rows instead of contiguous pencils, for the x field kind two stream
 * positions per lane instead of one, for the check kind the CFL speed of a
 * step's new state reduced by the check kernel after the last x sweep
 * instead of inside it (the same value either way).  The x fluid kind has
 * an alternative layout too, the strided policy with the lanes along y and
 * the shape as its segment length; the autotuner does not try it (set it
 * with fish_set_shape), and with it the check kernel reduces the CFL speed.  targets_out (may be NULL) receives
 * FISH_NUM_KINDS chosen values: the shape in bits 0-15, the block order
 * (1 = XCD-grouped) in bit 16, the alternative layout in bit 17.
 * Results do not depend on the shapes (each cell is computed by the same
 * operations whatever wave computes it).  Synchronises the stream. */
int fish_autotune(fish_ctx* ctx, int reps, int32_t* targets_out);

/* Set one kind's work shape directly, in the encoding fish_autotune returns
 * (for reproducing a tuned configuration).  FISH_ERR_ARG for an unknown kind
 * or a value outside the encoding. */
int fish_set_shape(fish_ctx* ctx, int kind, int32_t value);

/* Self-test of the wavefront lane-shift primitive the x sweeps stream with
 * (no context): one wave of 64 lanes runs two iterations with lane values
 * v = 100*it + lane; out128[64*it + lane] receives the value one stream
 * position back, i.e. lane - 1's of the same iteration, and 0 in lane 0 (the
 * x sweeps make their first lanes a halo, so nothing crosses iterations).
 * Synchronous; the caller owns out128. */
int fish_selftest_lane_shift(int device, float* out128);

/* Self-test of the FP64 reciprocal and square root the FP64 sweeps compute
 * with (no context): hardware estimates refined by Newton steps (1/x) and
 * Goldschmidt steps (sqrt x), in place of the IEEE division and square-root
 * sequences.  For the n host values x: rcp_out[i] = 1/x[i] and sqrt_out[i] =
 * sqrt(x[i]) as the kernels form them.  1 <= n <= 2^24, else FISH_ERR_ARG;
 * synchronous; the caller owns the three host arrays. */
int fish_selftest_math(int device, int n, const double* x, double* rcp_out, double* sqrt_out);

/* ------------------------------------------------------------------------
 * Allocation-free double step, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The double step of fish_strang_step on one box whose
 * state the caller keeps in device memory, with no context: the library
 * allocates nothing, neither device nor pinned memory.
 *
 * Arrays (device memory of p->device, owned by the caller, storage precision
 * of p->precision: double for FISH_FP64, float for FISH_FP32):
 *   state[8] : rho, m_x, m_y, m_z, E, b_x, b_y, b_z, each of
 *              (nx+ox)(ny+oy)(nz+oz) elements, o_d = 1 on an outflow axis
 *              and 0 on a periodic one; entry (i, j, k) at
 *              i + (nx+ox) (j + (ny+oy) k).  Cell arrays hold cell (i, j, k)
 *              for i < nx, j < ny, k < nz; b_x holds face i (between cells
 *              i-1 and i) for i < nx+ox, and likewise b_y along y and b_z
 *              along z (on a periodic axis face n is face 0 and is not
 *              stored).  Entries outside these ranges are not read.
 *              Read and overwritten with the state after the step.
 *   work[8]  : eight more arrays of the same size, distinct from state;
 *              overwritten (the sub-operators alternate between the two sets,
 *              an even number of times per field).
 *   phi      : with gravity, the potential in the cell layout; else ignored.
 * dt > 0 is used as given; dt == 0 takes the CFL step of the state (Eq. 14),
 * computed on the device.  report: NULL, or device memory for one
 * fish_step_report, written after the step.  p->alloc and p->free are
 * ignored; p->stream is the stream the work is enqueued on (NULL = default).
 * Asynchronous.  Irregular meshes are not available here.
 *
 * Scratch: the step's box table, step scalars and work lists live in one
 * static device array of FISH_NOALLOC_SCRATCH_BYTES on each GPU the call
 * runs on, held until the process ends and found at the first call on that
 * GPU.  Every call on a GPU uses the same array, and each call rewrites what
 * it reads: calls in stream order are independent, calls that overlap on one
 * GPU (two host threads, two streams) race and give wrong results.  A box
 * that needs more than FISH_NOALLOC_MAX_WAVES wavefronts in one sweep is
 * refused (FISH_ERR_UNSUPPORTED): every box up to 1024^3 cells fits, a flat
 * box such as 16384 x 1 x 16384 does not.
 *
 * Returns FISH_ERR_ARG for an invalid setting, a null or repeated array, or
 * a missing phi; FISH_ERR_UNSUPPORTED beyond the limits (also an array of
 * 4 GiB or more); FISH_ERR_DEVICE when a HIP call or launch fails.  The
 * message is fish_last_error(NULL).  A bad state (rho <= 0, p <= 0 or a
 * non-finite value, before or after the step) is reported in the report,
 * not by the return value.  The caller's current device is restored. */
#define FISH_NOALLOC_MAX_WAVES (1 << 20)
#define FISH_NOALLOC_SCRATCH_BYTES (2048 + 4 * FISH_NOALLOC_MAX_WAVES)

typedef struct fish_step_report {
  double dt;       /* the step size of every sub-operator (0 for a state refused before the step) */
  double dt_next;  /* CFL step of the new state, Eq. (14) (0 when it is bad)                      */
  int32_t status;  /* FISH_OK, or FISH_ERR_STATE for a bad state before or after the step          */
  int32_t pad;
} fish_step_report;

int fish_strang_step_noalloc(const fish_params* p, void* const state[8], void* const work[8], const void* phi,
                             double dt, fish_step_report* report);

/* ------------------------------------------------------------------------
 * Batches: many independent boxes of different shapes advanced together.
 *
 * A batch owns one device pool per field (two buffers each, plus phi with
 * gravity) of pool_bytes in total and places each box at an offset of the
 * pools (first fit; a removed box's range is returned and merged).  Every
 * launch of a step covers all boxes of the batch: a device table lists the
 * boxes and, per kernel kind, the box of every wavefront.  Each box takes its
 * own CFL step (Eq. 14) every double step; boxes never interact, so a box's
 * result is the same alone or in any mix (bitwise, same precision).
 * The scheme settings (gamma, limiter, predictor alpha, precision, gravity,
 * HSE) are per batch; the geometry and Courant number per box.
 * ------------------------------------------------------------------------ */
typedef struct fish_batch fish_batch;

typedef struct fish_batch_params {
  double gamma;
  int32_t limiter;
  double predictor_alpha;
  int32_t precision;
  int32_t gravity;           /* as in fish_params */
  int32_t hse;
  int32_t device;
  void* stream;              /* NULL: the batch creates its own (graphs cannot
                                capture the null stream)                   */
  size_t pool_bytes;         /* device bytes for box state (see fish_box_pool_bytes) */
  int32_t max_boxes;         /* box slots, >= 1                             */
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* alloc_user;
} fish_batch_params;

typedef struct fish_box {
  int32_t nx, ny, nz;        /* interior cells per axis, >= 1              */
  double dx, dy, dz;         /* spacing > 0                                 */
  double cfl;                /* Courant number, 0 < k <= 1                  */
  int32_t bc[3];             /* FISH_PERIODIC / FISH_OUTFLOW per axis       */
} fish_box;

/* Pool bytes one box takes in a batch of the given precision and gravity
 * (its arrays, both buffers, padded to 64 elements): the admission test of a
 * caller that budgets device memory.  0 for NULL. */
size_t fish_box_pool_bytes(const fish_box* box, int precision, int gravity);

/* Create / destroy a batch (fish_params conventions: FISH_ERR_ARG on a bad
 * field, FISH_ERR_NOMEM when the pools cannot be allocated). */
int fish_batch_create(const fish_batch_params* p, fish_batch** out);
void fish_batch_destroy(fish_batch* b);
const char* fish_batch_last_error(const fish_batch* b);
size_t fish_batch_device_bytes(const fish_batch* b);
/* Pool bytes not held by any box (possibly fragmented). */
size_t fish_batch_free_bytes(const fish_batch* b);
/* Boxes in the batch. */
int fish_batch_count(const fish_batch* b);

/* Add a box with its state (layouts of fish_set_state).  *id_out receives
 * its id (>= 0).  FISH_ERR_NOMEM when no slot or pool range is free (the
 * batch is unchanged), FISH_ERR_STATE when the state fails the check (the box
 * is not added).  Synchronises the stream. */
int fish_batch_add(fish_batch* b, const fish_box* box, const double* cell5, const double* bx,
                   const double* by, const double* bz, const double* phi, int* id_out);

/* Remove a box and return its pool range.  Synchronises the stream. */
int fish_batch_remove(fish_batch* b, int id);

/* Irregular Cartesian mesh (Sect. 2.5) of one box of the batch along axis
 * (0/1/2): the widths of its n cells, as for fish_set_spacing, applied from
 * the next step on (its CFL speed is taken again).  While any box of the
 * batch has widths, every box's sweeps take per-cell widths: a uniform box
 * then runs the irregular formulas with its own spacing, equal to its result
 * alone to rounding, and a box on an irregular mesh gives bitwise its result
 * alone.  The widths are copied to the device when the set of boxes changes,
 * after the stream has drained.  FISH_ERR_ARG for a bad id or axis, a null
 * array or a width that is not finite and positive. */
int fish_batch_set_spacing(fish_batch* b, int id, int axis, const double* widths);

/* Download one box's state and time (fish_get_state layouts; NULL skips an
 * array).  FISH_ERR_STATE if the box's sticky state flag is set (a box with a
 * bad state stops: its later steps have dt = 0).  Synchronises the stream. */
int fish_batch_get(fish_batch* b, int id, double* cell5, double* bx, double* by, double* bz,
                   double* t_out);

/* Time, last dt and the sticky state flag of one box.  Synchronises. */
int fish_batch_box_info(fish_batch* b, int id, double* t_out, double* dt_out, int* bad_out);

/* Double steps taken with dt > 0 by one box since its state was set (a box
 * whose state went bad, or one that reached its end time, stops counting):
 * the work a throughput figure may credit to the box.  Synchronises. */
int fish_batch_box_steps(fish_batch* b, int id, int* steps_out);

/* nsteps double steps of every box, each with its own CFL step.
 * Asynchronous. */
int fish_batch_step(fish_batch* b, int nsteps);

/* With on != 0 the launches of one double step are captured once into a HIP
 * graph (per set of boxes) and replayed by fish_batch_step. */
int fish_batch_use_graph(fish_batch* b, int on);

/* The autotuner of fish_autotune over all boxes of the batch. */
int fish_batch_autotune(fish_batch* b, int reps, int32_t* targets_out);

/* fish_set_shape for a batch. */
int fish_batch_set_shape(fish_batch* b, int kind, int32_t value);

/* Wait for the batch's stream. */
int fish_batch_sync(fish_batch* b);

/* The measurement hook of fish_timing_enable / fish_timing_read (eager
 * launches only: fish_batch_step does not replay a graph while it is on). */
int fish_batch_timing_enable(fish_batch* b, int mask, int max_launches);
int fish_batch_timing_read(fish_batch* b, int* launches, double* total_ms);

/* ------------------------------------------------------------------------
 * Serving: a request loop over a batch.
 *
 * Requests (a box, its state and a number of double steps) wait in a FIFO
 * queue.  Each fish_server_pump call
 *   1. enqueues k = min(chunk, fewest steps left) double steps of every
 *      resident box in the same launches (each box with its own CFL step),
 *   2. while they run, admits queued requests in arrival order while the head
 *      fits in the batch's pool (the HBM budget; a request never overtakes the
 *      head); their host repacking and copies overlap the steps, and they
 *      take their first step in the next call, and
 *   3. retires the boxes that are done: their state is written to the
 *      request's output arrays and their pool range is freed.
 * A request's result is the same as stepping its box alone (bitwise).
 * ------------------------------------------------------------------------ */
typedef struct fish_server fish_server;

typedef struct fish_request {
  fish_box box;
  int32_t nsteps;                    /* double steps, >= 1                          */
  const double *cell5, *bx, *by, *bz, *phi;  /* input state (fish_set_state layouts),
                                        read at admission; phi only with gravity */
  double *out_cell5, *out_bx, *out_by, *out_bz;  /* final state, written at
                                        retirement (any may be NULL)             */
  int64_t tag;                       /* returned by fish_server_pump on completion  */
  const double* widths[3];           /* irregular mesh (Sect. 2.5): the cell widths
                                        along each axis (n values, finite and > 0,
                                        as for fish_set_spacing), or NULL for the
                                        uniform spacing of box; read at admission */
} fish_request;

/* Create a server whose batch has the given parameters; chunk_steps >= 1 is
 * the most steps advanced between admissions. */
int fish_server_create(const fish_batch_params* p, int chunk_steps, fish_server** out);
void fish_server_destroy(fish_server* s);
const char* fish_server_last_error(const fish_server* s);
/* The server's batch (owned by the server; for autotuning or graphs). */
fish_batch* fish_server_batch(fish_server* s);

/* Queue a request.  The request record is copied; its arrays are owned by the
 * caller and must stay valid until the request completes.  FISH_ERR_NOMEM if
 * the box can never fit the pool. */
int fish_server_submit(fish_server* s, const fish_request* r);

/* One scheduling round (above).  Completed requests: *ndone tags in
 * done_tags[0..max_done) with their status in done_status (FISH_OK, or
 * FISH_ERR_STATE when the box's state went bad; may be NULL).  Synchronises
 * the stream. */
int fish_server_pump(fish_server* s, int64_t* done_tags, int32_t* done_status, int max_done, int* ndone);

/* Queue length, resident boxes, free pool bytes and cells x double steps
 * enqueued so far, counting a box whose state went bad (it stops with dt = 0)
 * until it retires (any pointer may be NULL). */
int fish_server_stats(const fish_server* s, int* queued, int* resident, size_t* pool_free,
                      int64_t* cell_steps);

#ifdef __cplusplus
}
#endif

#endif /* FISH_H */
