/*
 * CPU FP64 oracle for the phonon BTE time step -- TEST INFRASTRUCTURE ONLY.
 * Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
 * never by the product path.  Shares no code with the HIP library.
 *
 * Plain loops, FP64, no FMA contraction (built with -ffp-contract=off), sums in
 * a fixed order so the result does not depend on the OpenMP thread count.
 *
 * Readings of the paper used here (the paper defers the physics of I0 and of
 * the temperature relation to outside references):
 *   - Equilibrium intensity of band b (Bose-Einstein, per steradian):
 *       I0_b(T) = C_b / (exp(hbar omega_b / (k_B T)) - 1),
 *       C_b = g_b hbar omega_b D_b domega_b / (4 pi).
 *   - Temperature from the intensity (Sec. 2.2: integrate over directions and
 *     bands, first law): the relaxation-time-weighted form
 *       F(T) = W sum_b I0_b(T) / tau_b  =  G = sum_b (1/tau_b) sum_d w_d I_{d,b},
 *     W = sum_d w_d, which makes the relaxation term conserve energy exactly
 *     when tau_b differs between bands.  The plain energy form
 *       W sum_b I0_b(T) = E = sum_b sum_d w_d I_{d,b}
 *     is available as an option; both agree for a single relaxation time.
 *   - Implicit step: backward Euler of Eq. eq-bte-fv solved by point-Jacobi in
 *     defect form, the temperature re-inverted after every sweep, stopped when
 *     ||I^{k+1}-I^k|| <= tol ||I^{k+1}-I^n|| (||x||^2 = sum_P V sum_{d,b} w_d x^2).
 *   - Walls (Eq. eq-bdry): on an inflow wall face the ghost intensity is
 *     I0_b(T_wall) (isothermal) or the cell's own intensity in the mirrored
 *     direction (specular / symmetry; identical on axis-aligned walls).
 */
/*
 *   - Diffuse walls (the paper's walls are isothermal or symmetric; a diffuse
 *     adiabatic wall is the common third kind of phonon boundary): a wall face
 *     re-emits the energy flux that leaves the cell through it, isotropically:
 *     the ghost of every inflow direction is the outgoing flux-weighted mean
 *     sum_{s.n > 0} w_d (s.n) I_{d,b} / sum_{s.n > 0} w_d (s.n) of the cell.
 *   - Relaxation times that depend on temperature (Sec. 2.2: I0 and tau both
 *     depend on T; the paper gives no law): tau_b(T) = tau_b (T0 / T)^p_b per
 *     band entry, i.e. a scattering rate growing as T^p_b.  The sweep takes
 *     tau at the cell's current temperature; the relaxation-time-weighted
 *     temperature then solves H(T) = sum_b (W I0_b(T) - e_b) / tau_b(T) = 0
 *     with e_b = sum_d w_d I_{d,b}, the condition for the relaxation term to
 *     conserve energy.  All p_b = 0 is the constant-tau path, bit for bit.
 */
#include "bte_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 exact / recommended values. */
static const double HBAR = 1.054571817e-34; /* J s */
static const double KB = 1.380649e-23;      /* J / K */
static const double PI = 3.14159265358979323846;

#define NEWTON_MAX_ITERS 50
#define NEWTON_ACCEPT_REL 1e-14
#define NEWTON_STEP_REL 1e-13
#define MIRROR_TOL 1e-12

struct oracle_bte {
  int dim, n[3], nc, nd, nb;
  double h[3], vol;
  int wall[6];
  double* wall_I0[6]; /* [face][b] equilibrium intensity of an isothermal wall */
  double *s, *w, W;
  double *omega, *vg, *tau, *C;
  double *tau_p, tau_T0; /* tau_b(T) = tau_b (T0 / T)^p_b */
  int tauT;              /* some p_b != 0 */
  double dt, tol;
  int max_inner, scheme, tdef;
  int* mirror[3]; /* [d] -> mirrored direction across each axis, -1 if none */
  double *In, *Ik, *Inew; /* [P][d][b] */
  double *Tn, *Tk, *Tnew, *Tprev;
  double *cell_num, *cell_den;
  int* cell_newton;
  int* cell_fail;
  int failed_cell;
};

static void set_err(char* err, int errlen, const char* msg) {
  if (err && errlen > 0) {
    strncpy(err, msg, (size_t)errlen - 1);
    err[errlen - 1] = 0;
  }
}

/* ---------------------------------------------------------------- physics */

double oracle_equilibrium(const oracle_bte* o, int b, double T) {
  double x = HBAR * o->omega[b] / (KB * T);
  return o->C[b] / expm1(x);
}

/* d I0_b / dT */
static double equilibrium_dT(const oracle_bte* o, int b, double T) {
  double x = HBAR * o->omega[b] / (KB * T);
  double em1 = expm1(x);
  return o->C[b] * (x / T) * (em1 + 1.0) / (em1 * em1);
}

static double band_weight(const oracle_bte* o, int b) {
  return o->tdef == ORACLE_T_TAU_WEIGHTED ? 1.0 / o->tau[b] : 1.0;
}

/* Relaxation time of band b at temperature T. */
static double tau_at(const oracle_bte* o, int b, double T) {
  return o->tau[b] * pow(o->tau_T0 / T, o->tau_p[b]);
}

/* Temperature from per-band direction sums e_b when the weights 1/tau_b(T)
 * depend on T.  The root of sum_b (W I0_b(T) - e_b) / tau_b(T) = 0 is the
 * root of K(T) = N(T) / D(T) - 1 with N = W sum_b I0_b(T) / tau_b(T) and
 * D = sum_b e_b / tau_b(T) (D > 0); Newton runs on K, whose ratio form keeps
 * the steps in check far from the root (for one band K = W I0(T) / e - 1,
 * whatever the law), and which for constant tau takes the steps of the
 * constant-tau inversion.  d/dT (1/tau_b(T)) = p_b / (T tau_b(T)).  Same
 * accept-first test and stopping rule as the constant-tau inversion. */
int oracle_invert_temperature_bands(const oracle_bte* o, const double* e, double T_start,
                                    double* T_out, int* iters) {
  *iters = 0;
  *T_out = T_start;
  if (!(T_start > 0.0)) return ORACLE_E_NUMERIC;
  double T = T_start;
  for (int it = 0;; ++it) {
    double N = 0.0, dN = 0.0, D = 0.0, dD = 0.0;
    for (int b = 0; b < o->nb; ++b) {
      double r = 1.0 / tau_at(o, b, T);
      double dr = o->tau_p[b] / T * r;
      double i0 = oracle_equilibrium(o, b, T);
      N += r * o->W * i0;
      dN += dr * o->W * i0 + r * o->W * equilibrium_dT(o, b, T);
      D += r * e[b];
      dD += dr * e[b];
    }
    if (!(D > 0.0) || !isfinite(D)) return ORACLE_E_NUMERIC;
    double K = N / D - 1.0;
    if (it == 0 && fabs(K) <= NEWTON_ACCEPT_REL) { /* already consistent: keep T */
      *T_out = T;
      return ORACLE_OK;
    }
    if (it == NEWTON_MAX_ITERS) return ORACLE_E_NUMERIC;
    double dK = (dN * D - N * dD) / (D * D);
    double dT = K / dK;
    T = T - dT;
    *iters = it + 1;
    if (!isfinite(T) || !(T > 0.0)) return ORACLE_E_NUMERIC;
    if (fabs(dT) <= NEWTON_STEP_REL * T) {
      *T_out = T;
      return ORACLE_OK;
    }
  }
}

/* F(T) = W sum_b weight_b I0_b(T) */
static double F_of_T(const oracle_bte* o, double T) {
  double sum = 0.0;
  for (int b = 0; b < o->nb; ++b) sum += band_weight(o, b) * oracle_equilibrium(o, b, T);
  return o->W * sum;
}

static double dF_of_T(const oracle_bte* o, double T) {
  double sum = 0.0;
  for (int b = 0; b < o->nb; ++b) sum += band_weight(o, b) * equilibrium_dT(o, b, T);
  return o->W * sum;
}

int oracle_invert_temperature(const oracle_bte* o, double G, double T_start, double* T_out,
                              int* iters) {
  *iters = 0;
  *T_out = T_start;
  if (!(G > 0.0) || !isfinite(G) || !(T_start > 0.0)) return ORACLE_E_NUMERIC;
  double T = T_start;
  double F = F_of_T(o, T);
  if (fabs(F - G) <= NEWTON_ACCEPT_REL * G) { /* already consistent: keep T */
    *T_out = T;
    return ORACLE_OK;
  }
  for (int it = 1; it <= NEWTON_MAX_ITERS; ++it) {
    double dT = (F - G) / dF_of_T(o, T);
    T = T - dT;
    *iters = it;
    if (!isfinite(T) || !(T > 0.0)) return ORACLE_E_NUMERIC;
    if (fabs(dT) <= NEWTON_STEP_REL * T) {
      *T_out = T;
      return ORACLE_OK;
    }
    F = F_of_T(o, T);
  }
  return ORACLE_E_NUMERIC;
}

/* ---------------------------------------------------------------- geometry */

static int wall_face_index(const oracle_bte* o, int side, int x, int y, int z) {
  int axis = side / 2;
  if (axis == 0) return y + o->n[1] * z;
  if (axis == 1) return x + o->n[0] * z;
  return x + o->n[0] * y;
}

void oracle_mirror_map(const oracle_bte* o, int axis, int* map) {
  for (int d = 0; d < o->nd; ++d) {
    double t[3] = {o->s[3 * d], o->s[3 * d + 1], o->s[3 * d + 2]};
    t[axis] = -t[axis];
    map[d] = -1;
    for (int e = 0; e < o->nd; ++e) {
      const double* u = o->s + 3 * e;
      if (fabs(u[0] - t[0]) <= MIRROR_TOL && fabs(u[1] - t[1]) <= MIRROR_TOL &&
          fabs(u[2] - t[2]) <= MIRROR_TOL) {
        map[d] = e;
        break;
      }
    }
  }
}

static size_t idx(const oracle_bte* o, int P, int d, int b) {
  return ((size_t)P * o->nd + d) * o->nb + b;
}

/* ---------------------------------------------------------------- create */

static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

oracle_bte* oracle_create(int dim, const int* n, const double* h, const int* wall,
                          const double* const* wall_T, const double* T_init, int nd,
                          const double* s, const double* w, int nb, const double* omega,
                          const double* domega, const double* vg, const double* tau,
                          const double* dos, const double* deg, const double* tau_exp,
                          double tau_T0, double dt, double tol, int max_inner, int scheme,
                          int t_definition, char* err, int errlen) {
  if (dim != 2 && dim != 3) { set_err(err, errlen, "dim must be 2 or 3"); return NULL; }
  if (n[0] < 1 || n[1] < 1 || n[2] < 1 || (dim == 2 && n[2] != 1)) {
    set_err(err, errlen, "bad mesh size"); return NULL;
  }
  if (nd < 1 || nb < 1) { set_err(err, errlen, "need at least one direction and band"); return NULL; }
  if (!(dt > 0.0)) { set_err(err, errlen, "dt must be positive"); return NULL; }
  if (scheme != ORACLE_IMPLICIT && scheme != ORACLE_EXPLICIT) {
    set_err(err, errlen, "unknown scheme"); return NULL;
  }
  if (t_definition != ORACLE_T_TAU_WEIGHTED && t_definition != ORACLE_T_ENERGY) {
    set_err(err, errlen, "unknown temperature definition"); return NULL;
  }
  oracle_bte* o = (oracle_bte*)xcalloc(1, sizeof(oracle_bte));
  if (!o) { set_err(err, errlen, "out of memory"); return NULL; }
  o->dim = dim;
  o->nc = n[0] * n[1] * n[2];
  o->nd = nd;
  o->nb = nb;
  o->vol = 1.0;
  for (int a = 0; a < 3; ++a) {
    o->n[a] = n[a];
    o->h[a] = (dim == 2 && a == 2) ? 1.0 : h[a];
    o->vol *= o->h[a];
  }
  o->dt = dt;
  o->tol = tol;
  o->max_inner = max_inner > 0 ? max_inner : 200;
  o->scheme = scheme;
  o->tdef = t_definition;
  o->failed_cell = -1;
  o->tau_T0 = tau_T0 > 0.0 ? tau_T0 : 300.0;

  o->s = (double*)xcalloc((size_t)3 * nd, sizeof(double));
  o->w = (double*)xcalloc(nd, sizeof(double));
  o->omega = (double*)xcalloc(nb, sizeof(double));
  o->vg = (double*)xcalloc(nb, sizeof(double));
  o->tau = (double*)xcalloc(nb, sizeof(double));
  o->tau_p = (double*)xcalloc(nb, sizeof(double));
  o->C = (double*)xcalloc(nb, sizeof(double));
  size_t ndof = (size_t)o->nc * nd * nb;
  o->In = (double*)xcalloc(ndof, sizeof(double));
  o->Ik = (double*)xcalloc(ndof, sizeof(double));
  o->Inew = (double*)xcalloc(ndof, sizeof(double));
  o->Tn = (double*)xcalloc(o->nc, sizeof(double));
  o->Tk = (double*)xcalloc(o->nc, sizeof(double));
  o->Tnew = (double*)xcalloc(o->nc, sizeof(double));
  o->Tprev = (double*)xcalloc(o->nc, sizeof(double));
  o->cell_num = (double*)xcalloc(o->nc, sizeof(double));
  o->cell_den = (double*)xcalloc(o->nc, sizeof(double));
  o->cell_newton = (int*)xcalloc(o->nc, sizeof(int));
  o->cell_fail = (int*)xcalloc(o->nc, sizeof(int));
  for (int a = 0; a < 3; ++a) o->mirror[a] = (int*)xcalloc(nd, sizeof(int));
  if (!o->s || !o->w || !o->omega || !o->vg || !o->tau || !o->tau_p || !o->C || !o->In || !o->Ik ||
      !o->Inew || !o->Tn || !o->Tk || !o->Tnew || !o->Tprev || !o->cell_num ||
      !o->cell_den || !o->cell_newton || !o->cell_fail || !o->mirror[0] || !o->mirror[1] ||
      !o->mirror[2]) {
    set_err(err, errlen, "out of memory");
    oracle_destroy(o);
    return NULL;
  }

  memcpy(o->s, s, sizeof(double) * 3 * nd);
  memcpy(o->w, w, sizeof(double) * nd);
  if (dim == 2)
    for (int d = 0; d < nd; ++d) o->s[3 * d + 2] = 0.0; /* z component plays no part */
  o->W = 0.0;
  for (int d = 0; d < nd; ++d) o->W += o->w[d];
  for (int b = 0; b < nb; ++b) {
    if (!(omega[b] > 0.0) || !(domega[b] > 0.0) || !(vg[b] > 0.0) || !(tau[b] > 0.0) ||
        !(dos[b] > 0.0) || !(deg[b] > 0.0)) {
      set_err(err, errlen, "band tables must be positive");
      oracle_destroy(o);
      return NULL;
    }
    o->omega[b] = omega[b];
    o->vg[b] = vg[b];
    o->tau[b] = tau[b];
    o->tau_p[b] = tau_exp ? tau_exp[b] : 0.0;
    if (!isfinite(o->tau_p[b])) {
      set_err(err, errlen, "relaxation-time exponents must be finite");
      oracle_destroy(o);
      return NULL;
    }
    if (o->tau_p[b] != 0.0) o->tauT = 1;
    o->C[b] = deg[b] * HBAR * omega[b] * dos[b] * domega[b] / (4.0 * PI);
  }

  for (int a = 0; a < 3; ++a) oracle_mirror_map(o, a, o->mirror[a]);
  for (int side = 0; side < 2 * dim; ++side) {
    int kind = wall[side];
    o->wall[side] = kind;
    if (kind == ORACLE_WALL_ISOTHERMAL) {
      if (!wall_T || !wall_T[side]) {
        set_err(err, errlen, "isothermal wall needs a temperature array");
        oracle_destroy(o);
        return NULL;
      }
      int axis = side / 2;
      int nf = o->nc / o->n[axis];
      o->wall_I0[side] = (double*)xcalloc((size_t)nf * nb, sizeof(double));
      if (!o->wall_I0[side]) { set_err(err, errlen, "out of memory"); oracle_destroy(o); return NULL; }
      for (int f = 0; f < nf; ++f) {
        if (!(wall_T[side][f] > 0.0)) {
          set_err(err, errlen, "wall temperature must be positive");
          oracle_destroy(o);
          return NULL;
        }
        for (int b = 0; b < nb; ++b)
          o->wall_I0[side][(size_t)f * nb + b] = oracle_equilibrium(o, b, wall_T[side][f]);
      }
    } else if (kind == ORACLE_WALL_DIFFUSE) {
      /* nothing to precompute: the ghost follows the cell's own intensity */
    } else if (kind == ORACLE_WALL_SPECULAR || kind == ORACLE_WALL_SYMMETRY) {
      int axis = side / 2;
      for (int d = 0; d < nd; ++d)
        if (o->mirror[axis][d] < 0) {
          set_err(err, errlen, "direction set is not closed under the wall's mirror");
          oracle_destroy(o);
          return NULL;
        }
    } else {
      set_err(err, errlen, "unknown wall kind");
      oracle_destroy(o);
      return NULL;
    }
  }

  /* Initial condition: equilibrium at the initial temperature, every direction. */
  for (int P = 0; P < o->nc; ++P) {
    if (!(T_init[P] > 0.0)) {
      set_err(err, errlen, "initial temperature must be positive");
      oracle_destroy(o);
      return NULL;
    }
    o->Tn[P] = T_init[P];
    o->Tprev[P] = T_init[P];
    for (int d = 0; d < nd; ++d)
      for (int b = 0; b < nb; ++b) o->In[idx(o, P, d, b)] = oracle_equilibrium(o, b, T_init[P]);
  }
  return o;
}

void oracle_destroy(oracle_bte* o) {
  if (!o) return;
  for (int a = 0; a < 6; ++a) free(o->wall_I0[a]);
  for (int a = 0; a < 3; ++a) free(o->mirror[a]);
  free(o->s); free(o->w); free(o->omega); free(o->vg); free(o->tau); free(o->tau_p); free(o->C);
  free(o->In); free(o->Ik); free(o->Inew);
  free(o->Tn); free(o->Tk); free(o->Tnew); free(o->Tprev);
  free(o->cell_num); free(o->cell_den); free(o->cell_newton); free(o->cell_fail);
  free(o);
}

/* ---------------------------------------------------------------- sweep */

/*
 * Residual of the finite-volume balance of Eq. eq-bte-fv for DOF (P, d, b),
 * divided by the cell volume, evaluated with intensities I (current iterate)
 * and equilibrium I0P of cell P:
 *   R = (I0 - I_P)/tau + sum over faces with s.n < 0 of c_f (I_in - I_P),
 *   c_f = v_b A_f |s.n| / V.
 * Outflow faces carry the cell's own value, so after using the closed-cell
 * identity (sum of A_f s.n over the faces of a cell is zero) only inflow faces
 * remain.  Also returns the outflow coefficient sum via *c_out.
 */
static double balance(const oracle_bte* o, const double* I, int P, int x, int y, int z, int d,
                      int b, double I0P, double tauP, double* c_out) {
  const double* sd = o->s + 3 * d;
  int coord[3] = {x, y, z};
  int stride[3] = {1, o->n[0], o->n[0] * o->n[1]};
  double IP = I[idx(o, P, d, b)];
  double r = (I0P - IP) / tauP;
  double cout = 0.0;
  for (int f = 0; f < 2 * o->dim; ++f) {
    int axis = f / 2;
    double normal = (f % 2) ? 1.0 : -1.0; /* outward normal component along axis */
    double mu = sd[axis] * normal;
    double c = o->vg[b] * fabs(mu) / o->h[axis]; /* A_f / V = 1 / h_axis */
    if (mu > 0.0) {
      cout += c;
    } else if (mu < 0.0) {
      double Iin;
      int on_wall = (f % 2) ? (coord[axis] == o->n[axis] - 1) : (coord[axis] == 0);
      if (!on_wall) {
        int Q = P + ((f % 2) ? stride[axis] : -stride[axis]);
        Iin = I[idx(o, Q, d, b)];
      } else if (o->wall[f] == ORACLE_WALL_DIFFUSE) {
        /* re-emission of the outgoing flux through this face (outward normal
           component of direction d' along axis: sd'[axis] * normal > 0) */
        double num = 0.0, den = 0.0;
        for (int e = 0; e < o->nd; ++e) {
          double mu_e = o->s[3 * e + axis] * normal;
          if (mu_e > 0.0) {
            num += o->w[e] * mu_e * I[idx(o, P, e, b)];
            den += o->w[e] * mu_e;
          }
        }
        Iin = num / den;
      } else if (o->wall[f] == ORACLE_WALL_ISOTHERMAL) {
        int fi = wall_face_index(o, f, x, y, z);
        Iin = o->wall_I0[f][(size_t)fi * o->nb + b];
      } else {
        Iin = I[idx(o, P, o->mirror[axis][d], b)];
      }
      r += c * (Iin - IP);
    }
  }
  *c_out = cout;
  return r;
}

/* One point-Jacobi sweep (implicit) or one forward-Euler update (explicit),
 * followed by the per-cell temperature inversion and the per-cell pieces of the
 * increment norms.  Reads Ik, In, Tk; writes Inew, Tnew. */
static int sweep_and_temperature(oracle_bte* o) {
  const int nx = o->n[0], ny = o->n[1];
  int nfail = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfail)
  for (int P = 0; P < o->nc; ++P) {
    int x = P % nx, y = (P / nx) % ny, z = P / (nx * ny);
    double* I0P = (double*)malloc(sizeof(double) * 3 * o->nb);
    double* tauP = I0P + o->nb; /* relaxation time at the cell's current temperature */
    double* eP = I0P + 2 * o->nb;
    for (int b = 0; b < o->nb; ++b) {
      I0P[b] = oracle_equilibrium(o, b, o->Tk[P]);
      tauP[b] = tau_at(o, b, o->Tk[P]);
    }
    for (int d = 0; d < o->nd; ++d) {
      for (int b = 0; b < o->nb; ++b) {
        size_t i = idx(o, P, d, b);
        double cout;
        double r = balance(o, o->Ik, P, x, y, z, d, b, I0P[b], tauP[b], &cout);
        if (o->scheme == ORACLE_EXPLICIT) {
          o->Inew[i] = o->In[i] + o->dt * r;
        } else {
          r += (o->In[i] - o->Ik[i]) / o->dt;
          double a = 1.0 / o->dt + 1.0 / tauP[b] + cout;
          o->Inew[i] = o->Ik[i] + r / a;
        }
      }
    }
    /* energy sums: band outer, direction inner */
    double G = 0.0;
    for (int b = 0; b < o->nb; ++b) {
      double Sb = 0.0;
      for (int d = 0; d < o->nd; ++d) Sb += o->w[d] * o->Inew[idx(o, P, d, b)];
      eP[b] = Sb;
      G += band_weight(o, b) * Sb;
    }
    int it = 0;
    int st = (o->tauT && o->tdef == ORACLE_T_TAU_WEIGHTED)
                 ? oracle_invert_temperature_bands(o, eP, o->Tk[P], &o->Tnew[P], &it)
                 : oracle_invert_temperature(o, G, o->Tk[P], &o->Tnew[P], &it);
    free(I0P);
    o->cell_newton[P] = it;
    o->cell_fail[P] = (st != ORACLE_OK);
    nfail += (st != ORACLE_OK);
    double num = 0.0, den = 0.0;
    for (int d = 0; d < o->nd; ++d)
      for (int b = 0; b < o->nb; ++b) {
        size_t i = idx(o, P, d, b);
        double a = o->Inew[i] - o->Ik[i];
        double c = o->Inew[i] - o->In[i];
        num += o->vol * o->w[d] * a * a;
        den += o->vol * o->w[d] * c * c;
      }
    o->cell_num[P] = num;
    o->cell_den[P] = den;
  }
  if (nfail) {
    for (int P = 0; P < o->nc; ++P)
      if (o->cell_fail[P]) { o->failed_cell = P; break; }
    return ORACLE_E_NUMERIC;
  }
  return ORACLE_OK;
}

static void swap_ptr(double** a, double** b) {
  double* t = *a;
  *a = *b;
  *b = t;
}

static double total_energy(const oracle_bte* o) {
  double tot = 0.0;
  for (int P = 0; P < o->nc; ++P) {
    double E = 0.0;
    for (int b = 0; b < o->nb; ++b)
      for (int d = 0; d < o->nd; ++d) E += o->w[d] * o->In[idx(o, P, d, b)];
    tot += o->vol * E;
  }
  return tot;
}

/* One time step from the starting temperature T0 (NULL: T_n).  With shift,
 * the starting iterate is I^n + I0_b(T0) - I0_b(T_n) (an isotropic shift of
 * every direction); the increment norm's denominator still uses I^n. */
static int step_from(oracle_bte* o, int fixed_inner, const double* T0, int shift,
                     oracle_stats* st) {
  size_t ndof = (size_t)o->nc * o->nd * o->nb;
  memcpy(o->Ik, o->In, sizeof(double) * ndof);
  memcpy(o->Tk, T0 ? T0 : o->Tn, sizeof(double) * o->nc);
  if (T0 && shift) {
    for (int P = 0; P < o->nc; ++P)
      for (int b = 0; b < o->nb; ++b) {
        double dI = oracle_equilibrium(o, b, T0[P]) - oracle_equilibrium(o, b, o->Tn[P]);
        for (int d = 0; d < o->nd; ++d) o->Ik[idx(o, P, d, b)] += dI;
      }
  }
  o->failed_cell = -1;
  int k = 0, newton_max = 0;
  double res = 0.0;
  for (;;) {
    int rc = sweep_and_temperature(o);
    if (rc != ORACLE_OK) return rc;
    double num = 0.0, den = 0.0;
    for (int P = 0; P < o->nc; ++P) {
      num += o->cell_num[P];
      den += o->cell_den[P];
      if (o->cell_newton[P] > newton_max) newton_max = o->cell_newton[P];
    }
    if (num == 0.0) res = 0.0;
    else if (den == 0.0) res = INFINITY;
    else res = sqrt(num / den);
    swap_ptr(&o->Ik, &o->Inew);
    swap_ptr(&o->Tk, &o->Tnew);
    ++k;
    if (o->scheme == ORACLE_EXPLICIT) break;
    if (fixed_inner > 0) {
      if (k >= fixed_inner) break;
    } else if (res <= o->tol || k >= o->max_inner) {
      break;
    }
  }
  swap_ptr(&o->In, &o->Ik);
  memcpy(o->Tprev, o->Tn, sizeof(double) * o->nc);
  memcpy(o->Tn, o->Tk, sizeof(double) * o->nc);
  if (st) {
    st->inner = k;
    st->res = res;
    st->newton_max = newton_max;
    st->energy = total_energy(o);
  }
  return ORACLE_OK;
}

/* ---------------------------------------------------------------- access */

void oracle_get_T(const oracle_bte* o, double* T) { memcpy(T, o->Tn, sizeof(double) * o->nc); }

void oracle_get_I(const oracle_bte* o, double* I) {
  memcpy(I, o->In, sizeof(double) * (size_t)o->nc * o->nd * o->nb);
}

void oracle_get_E(const oracle_bte* o, double* E, double* G) {
  for (int P = 0; P < o->nc; ++P) {
    double e = 0.0, g = 0.0;
    for (int b = 0; b < o->nb; ++b) {
      double Sb = 0.0;
      for (int d = 0; d < o->nd; ++d) Sb += o->w[d] * o->In[idx(o, P, d, b)];
      e += Sb;
      g += Sb / o->tau[b];
    }
    if (E) E[P] = e;
    if (G) G[P] = g;
  }
}

int oracle_step(oracle_bte* o, int fixed_inner, oracle_stats* st) {
  return step_from(o, fixed_inner, NULL, 0, st);
}

int oracle_step_warm(oracle_bte* o, int fixed_inner, const double* T0, int shift,
                     oracle_stats* st) {
  if (!T0) return ORACLE_E_INVAL;
  for (int P = 0; P < o->nc; ++P)
    if (!(T0[P] > 0.0)) return ORACLE_E_INVAL;
  return step_from(o, fixed_inner, T0, shift, st);
}

int oracle_set_state(oracle_bte* o, const double* I, const double* T) {
  for (int P = 0; P < o->nc; ++P)
    if (!(T[P] > 0.0)) return ORACLE_E_INVAL;
  memcpy(o->In, I, sizeof(double) * (size_t)o->nc * o->nd * o->nb);
  memcpy(o->Tn, T, sizeof(double) * o->nc);
  memcpy(o->Tprev, T, sizeof(double) * o->nc);
  return ORACLE_OK;
}

int oracle_set_wall_temperature(oracle_bte* o, int side, const double* T_face) {
  if (side < 0 || side >= 2 * o->dim || o->wall[side] != ORACLE_WALL_ISOTHERMAL || !T_face)
    return ORACLE_E_INVAL;
  int nf = o->nc / o->n[side / 2];
  for (int f = 0; f < nf; ++f)
    if (!(T_face[f] > 0.0)) return ORACLE_E_INVAL;
  for (int f = 0; f < nf; ++f)
    for (int b = 0; b < o->nb; ++b)
      o->wall_I0[side][(size_t)f * o->nb + b] = oracle_equilibrium(o, b, T_face[f]);
  return ORACLE_OK;
}

int oracle_failed_cell(const oracle_bte* o) { return o->failed_cell; }

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
