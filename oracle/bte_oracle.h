/*
 * CPU FP64 oracle for the phonon BTE time step -- TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain, slow, obviously correct reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it.  It shares no
 * code, header or table with the HIP library.
 *
 * What it computes (paper Sec. 3.1, Eq. eq-bte and Eq. eq-bte-fv, with the
 * boundary ghosts of Eq. eq-bdry):
 *   dI_{d,b}/dt + v_b s_d . grad I_{d,b} = (I0_b(T) - I_{d,b}) / tau_b
 * on a uniform Cartesian finite-volume mesh with first-order upwind face values
 * (Sec. 2.1, the upwind operator), stepped either
 *   - implicitly (backward Euler) with point-Jacobi inner iterations coupled to
 *     a per-cell Newton inversion for T after every sweep, stopped on the
 *     step-relative increment norm, or
 *   - explicitly with forward Euler (Sec. 2.1, Eq. eq-conservation-discrete),
 *     the temperature being updated once after the step (Sec. 3.2,
 *     postStepFunction).
 *
 * Storage: I[P][d][b] (cell outermost), P = x + nx*(y + ny*z).
 * Wall order -x,+x,-y,+y,-z,+z; wall-face arrays run over the two other axes,
 * lower axis fastest.  In 2D (dim = 2) nz must be 1, faces normal to z do not
 * exist and s_z is ignored.
 */
#ifndef BTE_ORACLE_H
#define BTE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVAL (-1)
#define ORACLE_E_NOMEM (-2)
#define ORACLE_E_NUMERIC (-4)

#define ORACLE_WALL_ISOTHERMAL 0
#define ORACLE_WALL_SPECULAR 1
#define ORACLE_WALL_SYMMETRY 2
#define ORACLE_WALL_DIFFUSE 3 /* adiabatic, re-emits the outgoing flux isotropically */

#define ORACLE_IMPLICIT 0
#define ORACLE_EXPLICIT 1

#define ORACLE_T_TAU_WEIGHTED 0
#define ORACLE_T_ENERGY 1

typedef struct oracle_bte oracle_bte;

typedef struct {
  int inner;            /* inner sweeps taken in the step (1 in explicit mode) */
  double res;           /* last step-relative increment norm */
  int newton_max;       /* largest Newton iteration count over cells and sweeps */
  double energy;        /* sum_P V * E_P after the step */
} oracle_stats;

/* Copies every input array.  On failure returns NULL and writes a message into
 * err (if err != NULL).  wall_T is an array of 6 pointers (NULL unless that wall
 * is isothermal).  Band inputs: omega, domega, group speed vg, relaxation time
 * tau (at temperature tau_T0), density of states per polarisation dos,
 * degeneracy deg, and (nullable: all zero) the exponents tau_exp of
 * tau_b(T) = tau_b (tau_T0 / T)^tau_exp_b; tau_T0 <= 0 means 300 K. */
oracle_bte* oracle_create(int dim, const int* n, const double* h, const int* wall,
                          const double* const* wall_T, const double* T_init,
                          int nd, const double* s, const double* w,
                          int nb, const double* omega, const double* domega,
                          const double* vg, const double* tau, const double* dos,
                          const double* deg, const double* tau_exp, double tau_T0,
                          double dt, double tol, int max_inner, int scheme,
                          int t_definition, char* err, int errlen);
void oracle_destroy(oracle_bte* o);

/* One time step.  fixed_inner > 0 takes exactly that many inner sweeps
 * (replaying another solver's schedule); 0 stops on tol / max_inner. */
int oracle_step(oracle_bte* o, int fixed_inner, oracle_stats* st);

/* One implicit time step seeded with a starting temperature T0 [N_c] (a
 * warm start of the inner iteration): the first sweep takes T^(0) = T0 and
 * I0_b(T0); with shift != 0 its starting iterate is also moved by the
 * isotropic equilibrium difference I0_b(T0) - I0_b(T_n).  The iteration and its
 * stopping rule are those of oracle_step, so only the route to the fixed point
 * changes. */
int oracle_step_warm(oracle_bte* o, int fixed_inner, const double* T0, int shift,
                     oracle_stats* st);

void oracle_get_T(const oracle_bte* o, double* T);          /* [N_c] */
void oracle_get_I(const oracle_bte* o, double* I);          /* [N_c][N_d][N_b] */
void oracle_get_E(const oracle_bte* o, double* E, double* G); /* [N_c] each, may be NULL */
int oracle_set_state(oracle_bte* o, const double* I, const double* T);
int oracle_failed_cell(const oracle_bte* o);                /* last numeric failure, -1 if none */
/* New face temperatures [faces] of an isothermal wall, for the next steps. */
int oracle_set_wall_temperature(oracle_bte* o, int side, const double* T_face);
void oracle_set_threads(int n);
int oracle_get_threads(void);

/* Stand-alone pieces, exposed for the pin tests. */
double oracle_equilibrium(const oracle_bte* o, int b, double T);
/* Newton inversion of F(T) = G from T_start; returns status, writes T and the
 * iteration count. */
int oracle_invert_temperature(const oracle_bte* o, double G, double T_start,
                              double* T_out, int* iters);
/* Temperature from per-band direction sums e[b] = sum_d w_d I_{d,b} with
 * temperature-dependent relaxation times: Newton on
 * sum_b (W I0_b(T) - e_b) / tau_b(T) = 0 from T_start. */
int oracle_invert_temperature_bands(const oracle_bte* o, const double* e, double T_start,
                                    double* T_out, int* iters);
/* Mirror map across the given axis (0, 1, 2); -1 entries when not closed. */
void oracle_mirror_map(const oracle_bte* o, int axis, int* map);

#ifdef __cplusplus
}
#endif
#endif
