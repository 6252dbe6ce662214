/*
 * bte.h -- C ABI of the MI355X (gfx950) phonon Boltzmann transport time step.
 *
 * The library advances the non-gray, discrete-ordinates, finite-volume phonon
 * BTE under the single-relaxation-time approximation (paper Sec. 3.1,
 * Eq. eq-bte and its finite-volume form Eq. eq-bte-fv):
 *
 *   dI_{d,b}/dt + v_b s_d . grad I_{d,b} = (I0_b(T) - I_{d,b}) / tau_b
 *
 * for every cell P, direction d and band entry b of a uniform Cartesian mesh,
 * with first-order upwind face values (Sec. 2.1, the upwind operator),
 * isothermal and specular/symmetry walls through ghost intensities
 * (Eq. eq-bdry), and the per-cell temperature recovered from the intensity by
 * integrating over directions and bands (Sec. 2.2, "first law").  Every step of
 * that path runs in HIP kernels on the caller's stream; the host only validates,
 * launches and reads back small control words.
 *
 * Conventions shared by every call:
 *   - cell index P = x + nx*(y + ny*z)   (x fastest); 2D meshes have nz = 1,
 *     hz is ignored (quantities per unit depth) and s_z is ignored;
 *   - wall order -x, +x, -y, +y, -z, +z;
 *   - a wall-face array runs over the two other axes, lower axis fastest:
 *     +-x walls: y + ny*z;  +-y walls: x + nx*z;  +-z walls: x + nx*y;
 *   - intensity on the device and in bte_intensity(): [band][direction][cell];
 *   - every host pointer argument is read during the call only and may be freed
 *     on return; device memory is owned by the caller (see bte_options).
 *
 * Errors: every call returns BTE_OK or a negative status and never aborts.
 * bte_last_error() gives a thread-local message for the last failure.
 * Validation failures (BTE_E_INVAL) leave the context untouched.  After
 * BTE_E_DEVICE only bte_destroy() is valid.  BTE_E_NUMERIC (a cell whose energy
 * is not positive and finite, or whose temperature inversion fails) names the
 * cell in the message; the step's results are then not meaningful.
 * Threading: one context may be used by one thread at a time; distinct
 * contexts are independent.
 */
#ifndef BTE_H
#define BTE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bte_ctx bte_ctx;

enum bte_status {
  BTE_OK = 0,
  BTE_E_INVAL = -1,   /* bad argument or inconsistent input */
  BTE_E_NOMEM = -2,   /* workspace missing or too small */
  BTE_E_DEVICE = -3,  /* HIP runtime error; context is poisoned */
  BTE_E_NUMERIC = -4, /* non-physical state in a cell (message names it) */
  BTE_E_NOTCONV = -5, /* a step hit max_inner (only if fail_on_notconv) */
  BTE_E_STATE = -6    /* state buffer of the wrong size */
};

/* Wall kinds (Eq. eq-bdry).  Specular and symmetry give the same ghost on
 * axis-aligned walls: the cell's own intensity in the mirrored direction.
 * DIFFUSE (adiabatic, not among the paper's kinds): the wall re-emits the
 * energy flux leaving the cell through it isotropically; the ghost of every
 * inflow direction is sum_{s.n > 0} w_d (s.n) I_{d,b} / sum_{s.n > 0} w_d (s.n)
 * of the cell at the current iterate. */
enum bte_wall {
  BTE_WALL_ISOTHERMAL = 0,
  BTE_WALL_SPECULAR = 1,
  BTE_WALL_SYMMETRY = 2,
  BTE_WALL_DIFFUSE = 3
};

/* Time discretisation.  IMPLICIT_JACOBI: backward Euler, point-Jacobi inner
 * sweeps, temperature re-inverted after every sweep.  EXPLICIT_EULER: the
 * paper's forward Euler (Sec. 2.1, Eq. eq-conservation-discrete), temperature
 * updated once after the step (Sec. 3.2, postStepFunction). */
enum bte_scheme { BTE_IMPLICIT_JACOBI = 0, BTE_EXPLICIT_EULER = 1 };

/* Storage / arithmetic of the intensity sweep.  FP32_MIXED stores each
 * intensity as its FP32 deviation from I0_b at the coldest input temperature; the
 * sweep computes the update in FP64 and rounds it once to storage, and the
 * energy reduction, temperature inversion and residual norms are FP64. */
enum bte_precision { BTE_FP64 = 0, BTE_FP32_MIXED = 1 };

/* Temperature definition.  TAU_WEIGHTED: W sum_b I0_b(T)/tau_b =
 * sum_b (1/tau_b) sum_d w_d I_{d,b} (energy-conserving relaxation when tau
 * varies by band).  ENERGY: W sum_b I0_b(T) = sum_b sum_d w_d I_{d,b}. */
enum bte_tdef { BTE_T_TAU_WEIGHTED = 0, BTE_T_ENERGY = 1 };

/* Mesh, walls and initial temperature (host arrays). */
typedef struct {
  int dim;                  /* 2 or 3 */
  int n[3];                 /* cells per axis; n[2] = 1 in 2D; N_c = n[0] n[1] n[2].  The
                               padded count -- 2D: n[0] rounded up to 32 cells (16 with
                               FP64 storage) times n[1]; 3D: N_c rounded up to 64 -- is at
                               most 268435424 (an FP64 slab stays within 32-bit byte
                               offsets); BTE_E_INVAL above */
  double h[3];              /* cell size per axis [m]; h[2] ignored in 2D */
  int wall[6];              /* bte_wall per side; z sides ignored in 2D */
  const double* wall_T[6];  /* per-face temperature [K] of isothermal walls, else NULL */
  const double* T_init;     /* [N_c] initial temperature [K]; I starts at I0_b(T_init) */
} bte_mesh;

/* Discrete directions (host arrays): unit vectors s[3*d + axis] and solid-angle
 * weights w[d] [sr].  Specular/symmetry walls need the set to be closed under
 * the wall's mirror (checked at create). */
typedef struct {
  int n;
  const double* s;
  const double* w;
} bte_dirs;

/* Band entries (host arrays): angular frequency omega[b] and band width
 * domega[b] [rad/s]. */
typedef struct {
  int n;
  const double* omega;
  const double* domega;
} bte_bands;

/* Per-band material data (host arrays of length bands->n): group speed vg [m/s],
 * relaxation time tau [s], density of states per polarisation dos [s/m^3] and
 * polarisation degeneracy deg.  The equilibrium intensity per steradian is
 * I0_b(T) = C_b / (exp(hbar omega_b / k_B T) - 1), C_b = deg hbar omega dos domega / (4 pi).
 *
 * Relaxation times may depend on temperature (Sec. 2.2: I0 and tau both do):
 * tau_b(T) = tau[b] (tau_T0 / T)^tau_exp[b], a scattering rate that grows as
 * T^tau_exp[b].  Every relaxation term then takes tau at its cell's current
 * temperature, and the relaxation-time-weighted temperature solves
 * sum_b (W I0_b(T) - sum_d w_d I_{d,b}) / tau_b(T) = 0 (the relaxation term
 * conserves energy).  tau_exp NULL (or all zero) keeps tau constant; tau_T0
 * <= 0 means 300 K.  Batches take constant relaxation times only. */
typedef struct {
  const double* vg;
  const double* tau;
  const double* dos;
  const double* deg;
  const double* tau_exp;  /* nullable */
  double tau_T0;          /* [K] */
} bte_dispersion;

typedef struct {
  double dt;            /* time step [s] > 0; with EXPLICIT_EULER at most
                           1 / (1/tau_b + sum_a v_b |s_{d,a}| / h_a) for every band and
                           direction (the step then keeps intensities positive and
                           bounded; bte_create rejects a larger one with BTE_E_INVAL) */
  double tol;           /* inner stop: ||I^{k+1}-I^k|| <= tol ||I^{k+1}-I^n|| */
  int max_inner;        /* cap on inner sweeps per step (<= 0: 200) */
  int scheme;           /* bte_scheme */
  int precision;        /* bte_precision */
  int t_definition;     /* bte_tdef */
  int fail_on_notconv;  /* nonzero: a step that hits max_inner returns BTE_E_NOTCONV */
  int timing;           /* nonzero: time every sweep kernel with HIP events */
  void* stream;         /* hipStream_t the work is enqueued on (NULL = null stream) */
  void* workspace;      /* device memory of >= bte_workspace_size() bytes, 256-B aligned,
                           owned by the caller and kept alive until bte_destroy() */
  size_t workspace_bytes;
  /* Learned warm start of the next temperature (not in the paper; a
     perceptron on bf16 matrix cores, trained on the device from the solver's
     own steps).  The inner iteration still runs to the same tolerance and
     judges the guess; an implausible guess in a cell falls back to T_n. */
  int warm_start;       /* BTE_WARM_NONE / BTE_WARM_T / BTE_WARM_T_SHIFT */
  int nn_train_steps;   /* plain steps recorded before training (<= 0: 20) */
  int nn_epochs;        /* passes over the recorded samples (<= 0: at least 2 passes
                           and at least 300 minibatch updates) */
  float nn_lr;          /* Adam learning rate (<= 0: 1e-3) */
  unsigned long long nn_seed;  /* initial-weight seed (SplitMix64 counter stream) */
  int nn_guard;         /* the plain iteration judges the guess: whenever nn_guard
                           consecutive warm-started steps take more inner sweeps in
                           total than the last nn_guard plain steps recorded before
                           training, the guess is switched off for the rest of the run
                           (0: 4; < 0: never) */
} bte_options;

/* Warm-start modes.  T: the first sweep of a step uses I0 at the guessed
 * temperature.  T_SHIFT: additionally starts the intensity from
 * I^n + I0_b(T_guess) - I0_b(T_n) (an isotropic shift), fused into the first
 * sweep.
 *
 * The rules of the learned warm start (not in the paper):
 *   - recording: each of the first nn_train_steps steps records, in FP32,
 *     T_n, T_{n-1}, E_n at its start and T_{n+1} at its end (T_{n-1} = T_n
 *     for the first step after create);
 *   - normalisation, from every recorded sample: mu_T and s_T the mean and
 *     population standard deviation of the T_n channel, mu_E and s_E those of
 *     E_n, s_D the root mean square of T_{n+1} - T_n.  A non-positive variance
 *     gives a scale of 1; a T or E scale at or below 1e-6 |mean| becomes
 *     1e-6 |mean| + 1e-30; a zero s_D becomes 1;
 *   - training order: N = nn_train_steps x N_c samples, sample i = step
 *     i / N_c, cell i % N_c.  Position p of epoch e takes sample
 *     (a p + c_e) mod N with a = floor(0.6180339887 N) | 1, raised by 2 until
 *     gcd(a, N) = 1, and c_e = 7919 e mod N; minibatches are 8192 consecutive
 *     positions (the last one of an epoch shorter);
 *   - loss: mean over the minibatch of (y - (T_{n+1} - T_n)/s_D)^2;
 *   - Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, FP32 masters and
 *     moments) on every weight and bias; the zero-padded feature columns of W1
 *     stay zero;
 *   - use: guess = T_n + s_D y per cell; it is rejected (the cell starts from
 *     T_n and counts as a fallback) unless s_D y is finite, at most
 *     10 max(s_D, |T_n - T_{n-1}|) in size, and the guess is positive. */
enum bte_warm { BTE_WARM_NONE = 0, BTE_WARM_T = 1, BTE_WARM_T_SHIFT = 2 };

typedef struct {
  int inner;       /* inner sweeps taken (1 in explicit mode) */
  int converged;   /* 1 if the tolerance (or the requested fixed count) was met */
  int newton_max;  /* most Newton iterations any cell needed in the step */
  int warm;        /* 1 if the step started from the network's guess */
  double res;      /* final step-relative increment norm */
  int fallbacks;   /* cells whose guess was rejected in this step */
  int trained;     /* 1 if the network was trained at the end of this step */
  double nn_loss;  /* last training minibatch loss (normalised units), if trained */
} bte_step_stats;

/* Bytes of device workspace that bte_create() needs for these inputs. */
int bte_workspace_size(const bte_mesh* mesh, const bte_dirs* dirs, const bte_bands* bands,
                       const bte_options* opt, size_t* bytes);

/* Validates and copies every input, derives the mirror maps and the per-(d,b)
 * coefficients, binds the workspace and stream, and enqueues the initial state
 * I_{d,b,P} = I0_b(T_init(P)) (Sec. 3.2, initial condition).  On success *out
 * receives the context. */
int bte_create(const bte_mesh* mesh, const bte_dirs* dirs, const bte_bands* bands,
               const bte_dispersion* disp, const bte_options* opt, bte_ctx** out);

/* Advances nsteps time steps.  fixed_inner (nullable, [nsteps]): if non-NULL and
 * fixed_inner[i] > 0, step i takes exactly that many inner sweeps (replays
 * another solver's schedule); otherwise it stops on tol / max_inner.  stats
 * (nullable, [nsteps]) receives one record per step.  Returns when the work is
 * complete on the stream. */
int bte_step(bte_ctx* ctx, int nsteps, const int* fixed_inner, bte_step_stats* stats);

/* Copies the cell temperatures [N_c] to host memory T_out (n_cells entries). */
int bte_temperature(bte_ctx* ctx, double* T_out, size_t n_cells);

/* Copies the intensity at the current time level to host memory, FP64,
 * layout [band][direction][cell]; n = N_b * N_d * N_c. */
int bte_intensity(bte_ctx* ctx, double* I_out, size_t n);

/* Copies the per-cell energy density E_P = sum_b sum_d w_d I_{d,b,P} [N_c]. */
int bte_energy(bte_ctx* ctx, double* E_out, size_t n_cells);

/* Replaces the intensity (host, FP64, [band][direction][cell]) and the
 * temperature [N_c] (each > 0) of the current time level; the energy density
 * is recomputed from the intensity and the previous time level's temperature
 * is set to the given one.  The temperature must be consistent with the
 * intensity for the result to be meaningful (it seeds the next inversion).
 * To resume a run exactly, use bte_get_state / bte_set_state. */
int bte_set_fields(bte_ctx* ctx, const double* I, size_t n, const double* T, size_t n_cells);

/* Checkpoint of everything the next steps depend on: the intensity of the
 * current time level in storage format, T_n, T_{n-1}, the energy density, the
 * equilibrium intensities, the storage reference, the sweep layout, the step
 * count, and with a learned warm start its recorded training history, the
 * sweeps of the recorded steps, its parameters, Adam moments and step count,
 * and the guard counters.  A context created from the same inputs and
 * options that restores it continues bit for bit as the saved context would
 * have (the sweep layout is restored with it where the context can hold it;
 * otherwise results agree to rounding).
 *
 * Layout of the state bytes: this header, then the sections at the byte
 * offsets off[] (each 256-byte aligned; 0 = absent):
 *   off[0] intensity [band][direction][cell], FP64 (BTE_FP64) or the FP32
 *          deviation from the storage reference (BTE_FP32_MIXED);
 *   off[1] T_n, off[2] T_{n-1}, off[3] E_n: FP64 [N_c] each;
 *   off[4] I0_b(T_n): FP64 [band][cell];  off[5] storage reference: FP64 [band];
 *   off[6] inner sweeps of each recorded plain step: int32 [nn_rec];
 *   off[7] parameters, off[8] Adam first moments, off[9] Adam second
 *          moments: FP32 [nn_params] each;
 *   off[10] recorded history: FP32 [nn_rec][4][N_c], channels T_n, T_{n-1},
 *          E_n, T_{n+1} (the first nn_recorded steps are valid). */
typedef struct {
  char magic[8];       /* "BTESTAT1" */
  int version;         /* 1 */
  int header_bytes;    /* sizeof(bte_state_header) */
  int dim, n[3], nd, nb;
  int precision, scheme, warm_start, nn_rec;
  int layout[4];       /* sweep layout: kind, rows, planes, direction groups */
  long long steps;     /* time steps taken since create */
  int nn_recorded;     /* plain steps recorded for training */
  int nn_trained;      /* network trained (or parameters set) */
  int nn_off;          /* guess switched off by the guard */
  int nn_warm_steps, nn_warm_sweeps;  /* guard window so far */
  int nn_adam_t;       /* Adam updates taken */
  int nn_last_batch;   /* samples of the last minibatch */
  int nn_params;       /* parameter count (0 without a warm start) */
  unsigned long long off[11];
  unsigned long long total;  /* bytes of the whole state */
} bte_state_header;

/* Bytes of the state of this context. */
int bte_state_size(bte_ctx* ctx, size_t* bytes);
/* Writes the state into host memory buf of at least bte_state_size() bytes
 * (waits for the context's stream). */
int bte_get_state(bte_ctx* ctx, void* buf, size_t bytes);
/* Restores a state written by bte_get_state.  BTE_E_STATE if it was taken
 * from a context of another shape, precision, scheme, warm-start mode,
 * recording length or storage reference, or is truncated; the context is
 * then untouched. */
int bte_set_state(bte_ctx* ctx, const void* buf, size_t bytes);

/* New face temperatures of an isothermal wall (side 0..5, n = that side's
 * face count, each > 0) for the steps that follow: the boundary of the paper's
 * boundary callbacks that changes in time, set from the host between steps
 * (Sec. 3.2, boundary conditions as callbacks).  BTE_E_INVAL if the side is
 * not isothermal. */
int bte_set_wall_temperature(bte_ctx* ctx, int side, const double* T_face, size_t n);

/* Sum and count of the sweep-kernel durations measured since the last call
 * (options.timing must be set); resets the accumulators. */
int bte_sweep_time(bte_ctx* ctx, double* total_ms, int* count);

/* The sweep layout in use (all nullable): kernel family (0 one cell per
 * thread, 1 2D column walk, 2 3D column walk, 3 3D flattened (x, y) plane),
 * rows walked per wave (0 for the flattened plane), planes held per wave
 * (1 in 2D) and direction groups.  Chosen at create (BTE_SWEEP_* variables
 * override it) or by bte_autotune. */
int bte_sweep_layout(bte_ctx* ctx, int* kind, int* ry, int* rz, int* ndg);

/* Learned warm start.  The parameter vector (FP32) is, in order:
 * W1[128][KP] | b1[128] | W2[128][128] | b2[128] | w3[128] | b3, 3 zeros |
 * mu_T, s_T, mu_E, s_E, s_D, 3 zeros
 * with KP = 32 (2D) or 96 (3D) input features (27 or 81 used, the rest zero).
 * Inputs of cell P: the 3^dim neighbourhood (replicate padding at the mesh
 * edge) of (T_n - mu_T)/s_T, (T_{n-1} - mu_T)/s_T, (E_n - mu_E)/s_E, ordered
 * [channel][dz][dy][dx]; output y, guess T_{n+1} = T_n + s_D y.
 * These calls need options.warm_start != BTE_WARM_NONE. */
int bte_nn_param_count(bte_ctx* ctx, size_t* n);
int bte_nn_params(bte_ctx* ctx, float* out, size_t n);
/* Replaces the parameters (and normalisation) and marks the network trained. */
int bte_nn_set_params(bte_ctx* ctx, const float* in, size_t n);
/* The network's guess of T_{n+1} (host, [N_c]) from the current state, before
 * any plausibility check. */
int bte_nn_predict(bte_ctx* ctx, double* T_guess, size_t n_cells);
/* Mean squared error of the current network (normalised units) and its
 * gradient with respect to the parameter vector, over every cell of one
 * sample (T_n, T_{n-1}, E_n -> T_{n+1}) given on the host; needs
 * N_c <= 8192.  y_out (nullable, [N_c]) receives the network outputs.  The
 * parameters are not changed. */
int bte_nn_gradient(bte_ctx* ctx, const double* T_n, const double* T_prev, const double* E_n,
                    const double* T_next, size_t n_cells, float* grad, size_t n, double* loss,
                    float* y_out);

/* Sweep layout tuning.  Times the candidate layouts of this context's shape on
 * the device and keeps the fastest, or takes the layout recorded for the same
 * shape in the text file cache_path (appended to after a measurement; NULL =
 * no cache).  2D layouts: 4 or 8 rows walked per wave x 1-16 direction
 * groups; 3D layouts: 2x2, 1x4 or 2x4 (rows x planes held per wave), or 4 or
 * 2 planes of the flattened (x, y) plane (reported as 0 rows), x 1-4
 * direction groups.  *ry and *rz are in/out: a positive value on entry
 * restricts the search to that row / plane count, and *ry = -1 tunes for a
 * batch: one direction group, 4 rows in 2D, and in 3D 4 planes per wave of
 * the family create picks by idle lanes (the flattened plane where 64-column
 * tiles leave more than an eighth of the lanes idle, else the 1x4 walk).  In
 * a batch the geometries fill the device together, so layouts that spread
 * one sweep wider only add bytes; batch choices are cached apart from
 * single-geometry ones.  The choice is returned in *ry, *rz, *ndg and its sweep time (measured now
 * or recorded in the cache) in *sweep_ms (all nullable; -1 for
 * shapes with a single layout).  BTE_E_INVAL if the restriction matches no
 * layout. */
int bte_autotune(bte_ctx* ctx, const char* cache_path, int* ry, int* rz, int* ndg,
                 double* sweep_ms);

/* Batched stepping of independent contexts (geometries of any size, 2D or
 * 3D, one precision, sharing one stream): every inner iteration of all of them
 * runs as persistent sweeps over work lists of (geometry, tile, band,
 * direction group) items -- one list per kernel family, largest geometry
 * first, converged geometries skipped -- followed by batched temperature and
 * convergence kernels.  With use_graph (and a non-null stream) that iteration
 * is captured once as a HIP graph and replayed until every geometry has
 * converged.  Networks of the learned warm start that fall due in the same
 * step train together.  Each context gives exactly the results it gives when
 * stepped alone.  Batches need a layout bte_autotune's *ry = -1 search
 * allows (4 rows in 2D; 2x2, 1x4 or the flattened plane in 3D), the implicit
 * scheme, and warm start NONE or T.  The batch holds small device arrays of
 * its own (descriptors, work lists, training schedules). */
typedef struct bte_batch bte_batch;
int bte_batch_create(int n, bte_ctx* const* ctxs, int use_graph, bte_batch** out);
/* stats (nullable): [nsteps][n] */
int bte_batch_step(bte_batch* batch, int nsteps, bte_step_stats* stats);
int bte_batch_destroy(bte_batch* batch);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the batched step of
 * bte_batch_step without a batch object, allocating nothing.  Its geometry
 * descriptors, work lists (kept as per-geometry item ranges) and counters
 * live in a fixed device array of the library, one per GPU (219 KB,
 * held until the process ends), filled afresh by every call; the host stages
 * them in a fixed block under a lock, so calls from several threads take
 * turns, and calls that overlap on one GPU through other means race.  Same
 * rules as bte_batch_create for the contexts, plus: at most 256 contexts, and
 * no context may still have to record or train its warm-start network (train
 * it first by stepping it alone or in a bte_batch).  No graph is captured;
 * the host waits for each inner iteration.  Results equal bte_batch_step's.
 * stats (nullable): [nsteps][n]. */
int bte_batch_step_static(int n, bte_ctx* const* ctxs, int nsteps, bte_step_stats* stats);

/* Releases host-side resources (not the caller's workspace). */
int bte_destroy(bte_ctx* ctx);

/* Message of the calling thread's last failure ("" if none). */
const char* bte_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BTE_H */
