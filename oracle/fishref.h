/*
 * fishref.h -- plain FP64 CPU oracle of the FISH operator-split ideal-MHD step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library
 * against a slow, obviously correct implementation written from the paper
 * (Kaeppeli, Whitehouse, Scheidegger, Pen & Liebendoerfer, "FISH: A 3D
 * parallel MHD code for astrophysical applications", Sect. 2).  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or constant with the HIP library.
 *
 * Array conventions (all host, FP64, C order, caller-owned, copied on every
 * call):
 *   cell5 : [5][nz][ny][nx]  rho, m_x, m_y, m_z, E     (cell averages, Eq. 8)
 *   bx    : [nz][ny][nx+1]   face averages, Eq. (9);  entry f is the face
 *   by    : [nz][ny+1][nx]   between cells f-1 and f along the normal
 *   bz    : [nz+1][ny][nx]   (Eqs. 10, 11)
 *   phi   : [nz][ny][nx]     fixed gravitational potential, may be NULL
 * On a periodic axis face n duplicates face 0: it is ignored on input and
 * written equal to face 0 on output.  On an outflow axis it is a real face.
 */
#ifndef FISHREF_H
#define FISHREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FISHREF_OK = 0,
  FISHREF_ERR_ARG = 1,
  FISHREF_ERR_NOMEM = 2,
  FISHREF_ERR_STATE = 4, /* rho <= 0, p <= 0 or a non-finite value */
  FISHREF_ERR_UNSUPPORTED = 5
};

typedef struct fishref_params {
  int32_t nx, ny, nz;     /* interior cells per axis, >= 1 (1 = inactive axis)  */
  double dx, dy, dz;      /* uniform spacing > 0 (Sect. 2.1)                     */
  double gamma;           /* ratio of specific heats > 1, Eq. (5)                */
  double cfl;             /* Courant number k of Eq. (14), 0 < k <= 1            */
  int32_t limiter;        /* 0 minmod Eq. (29), 1 van Leer Eq. (30), 2 van Leer   */
                          /* where |v| <= c_S, minmod where |v| > c_S (fluid)   */
  double predictor_alpha; /* predictor freezing-speed scale in [0, 1] (Sect. 2.2)*/
  int32_t bc[3];          /* per axis: 0 periodic, 1 outflow (zeroth order)      */
  int32_t gravity;        /* 0 none; fixed potential: 1 unsplit Eqs. (41)-(43),  */
                          /* 2 split G(dt/2) L G(dt/2), Eqs. (38)-(40)          */
  int32_t hse;            /* 0/1 hydrostatic-gradient subtraction Eqs. (51)-(57) */
  int32_t nthreads;       /* OpenMP threads, 0 = runtime default                 */
} fishref_params;

typedef struct fishref_ctx fishref_ctx;

int fishref_create(const fishref_params* p, fishref_ctx** out);
void fishref_destroy(fishref_ctx* c);
const char* fishref_last_error(const fishref_ctx* c);

int fishref_set_state(fishref_ctx* c, const double* cell5, const double* bx,
                      const double* by, const double* bz, const double* phi);
int fishref_get_state(fishref_ctx* c, double* cell5, double* bx, double* by,
                      double* bz, double* t_out);

/* Eq. (14): dt = k / max over cells and active axes of (|v_d| + c_F,d)/dx_d. */
int fishref_cfl_dt(fishref_ctx* c, double* dt_out);

/* One symmetric double step, Eqs. (12)-(13): twelve sub-operators of size dt,
 * t += 2 dt.  dt == 0 takes the CFL step of the current state. */
int fishref_strang_step(fishref_ctx* c, double dt);

/* One sub-operator: op 0 = fluid L_d (Sect. 2.2/2.3), op 1 = field B_d
 * (Sect. 2.4); dir 0/1/2 = x/y/z. */
int fishref_apply(fishref_ctx* c, int op, int dir, double dt);

/* Irregular Cartesian mesh (Sect. 2.5): the widths of the n cells along axis
 * (0/1/2), all > 0.  From then on every sweep, the CFL step and the
 * diagnostics use per-cell widths (the other axes keep theirs). */
int fishref_set_spacing(fishref_ctx* c, int axis, const double* widths);

/* out[0..4]  = sums of rho, m_x, m_y, m_z, E times the cell volume,
 * out[5..7]  = sums of bx, by, bz over the real faces times the face area,
 * out[8]     = max |div b| over cells, Eq. (62),
 * out[9]     = max |b| over faces. */
int fishref_diagnostics(fishref_ctx* c, double* out);

#ifdef __cplusplus
}
#endif

#endif /* FISHREF_H */
