// Internal declarations shared by the kernels and the C-ABI host code of the
// BTE library.  Not installed; the public interface is include/bte.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace bte {

// CODATA 2018 values.
constexpr double kHbar = 1.054571817e-34;  // J s
constexpr double kBoltzmann = 1.380649e-23;  // J / K
constexpr double kPi = 3.14159265358979323846;

constexpr int kNewtonMaxIters = 50;
constexpr double kNewtonAcceptRel = 1e-14;
constexpr double kNewtonStepRel = 1e-13;

constexpr int kSweepBlock = 256;     // threads per sweep workgroup (4 waves)
constexpr int kCellBlock = 64;       // threads per per-cell kernel workgroup (one wave)
constexpr int kReduceBlock = 256;    // threads of the single-workgroup reductions
constexpr int kSlabAlign = 64;       // cells per slab rounded up to this
// Sweep workgroups that fill a 256-CU device (about 32 per compute unit); the
// default direction-group count of a sweep plan aims at this many.
constexpr long long kSweepFillWorkgroups = 8192;
// Temperature inversion: lanes per cell (each owns every lanes-th band entry)
// and cells per 256-thread workgroup.  Four lanes where there are at most 32
// band entries, eight above (measured: 2.5 % faster batches of 8-40 entries
// with four, 17 % slower inversion at 55 entries).
__host__ __device__ inline int temp_lanes(int nb) { return nb <= 32 ? 4 : 8; }
__host__ __device__ inline int temp_cells_per_block(int nb) { return 256 / temp_lanes(nb); }

// Control words of the inner iteration, written by the device, mirrored to the host.
struct Control {
  int converged;   // inner loop finished (later kernels of the step are no-ops)
  int k;           // sweeps completed in the current step
  int newton_max;  // most Newton iterations in any cell this step
  int err_cell;    // smallest failing cell index, INT_MAX if none
  double res;      // last step-relative increment norm
  double num;      // last ||I^{k+1} - I^k||^2
  double den;      // last ||I^{k+1} - I^n||^2
};

// Per (band, direction): c_a = v_b |s_{d,a}| / h_a; scale = 1 / (1/dt + 1/tau_b +
// sum_a c_a) (backward Euler) or dt (forward Euler); q = the coefficient of
// I^n in the direct form of the FP32-storage update: 1/dt, or
// 1/dt - 1/tau_b - sum_a c_a under forward Euler.
struct Coef {
  double c[3];
  double scale;
  double q;
};
static_assert(sizeof(Coef) == 5 * sizeof(double), "Coef is read as five contiguous doubles");

// Direction flags: bit a set if s_{d,a} > 0, bit (4 + a) set if s_{d,a} < 0.
__host__ __device__ inline bool dir_pos(int flags, int a) { return (flags >> a) & 1; }
__host__ __device__ inline bool dir_neg(int flags, int a) { return (flags >> (4 + a)) & 1; }

// Cell P = x + nx (y + ny z).  Per-cell arrays ([b][P]) hold nc values in
// rows of ncp; an intensity slab ([b][d][.]) holds cell P at x + px (y + ny z):
// on 2D meshes px is nx rounded up to a 128-byte line of stored values, so
// every row of a slab starts on a line (rows that straddle lines cost the
// column walk 20-40 %), and ncp = px ny; on 3D meshes px = nx and ncp is nc
// rounded up to kSlabAlign.
struct Geometry {
  int dim;
  int nx, ny, nz;
  int nc;    // cells
  int ncp;   // cells per slab, padding included
  int px;    // intensity row pitch in cells
  int nd, nb;
  int ndg;   // direction groups of the energy partials S[ndg][nb][ncp]
  double vol;
};

// Position of cell P in an intensity slab.
__host__ __device__ inline size_t ipos(const Geometry& g, size_t P) {
  return g.px == g.nx ? P : (P / g.nx) * g.px + P % g.nx;
}

// How a sweep is laid out on the device.
enum SweepKind {
  kSweepCellPerThread = 0,
  kSweepColumnWalk2D = 1,
  kSweepColumnWalk3D = 2,
  kSweepFlat3D = 3,  // 3D, lanes over the flattened (x, y) plane
};

struct SweepPlan {
  int kind;
  int ry;        // rows walked per wave (column-walk kernels)
  int rz;        // planes held per wave (3D column walk)
  int ntx, nty;  // tiles along x (64 lanes each) and along y (4 waves x ry rows each)
  int ntz;       // tiles along z (rz planes each; 1 in 2D)
  int ndg, dgs;  // direction groups and directions per group
  int ntiles;    // workgroups per (band, direction group)
  int nparts;    // norm partials written per sweep (one per workgroup)
};

// Chooses the sweep layout for a mesh; ry / rz / ndg <= 0 and kind < 0 pick
// defaults.
SweepPlan make_sweep_plan(int dim, int nx, int ny, int nz, int nd, int nb, int ry, int rz,
                          int ndg, int kind);

struct Tables {
  const Coef* coef;          // [nb][nd]
  const int* dflags;         // [nd]
  const int* mirror;         // [3][nd]
  const double* w;           // [nd]
  const double* Cb;          // [nb] equilibrium prefactor
  const double* xfac;        // [nb] hbar omega / k_B
  const double* inv_tau;     // [nb]
  const double* fweight;     // [nb] band weight of the temperature relation
  const double* Iref;        // [nb] storage reference: stored value = I - Iref[b]
                             // (zero in FP64 mode, I0_b(T_ref) in FP32 mode)
  // Temperature-dependent relaxation (null / zero when tau is constant):
  // 1/tau_b(T) = inv_tau[b] (T / tau_T0)^tau_p[b]; relax[b][cell] holds it at
  // each cell's current temperature, refreshed with I0.
  const double* tau_p;       // [nb] exponents
  double* relax;             // [nb][ncp]
  double tau_T0;
  int tau_weighted;          // temperature definition weights bands by 1/tau_b(T)
  int explicit_scheme;       // forward Euler (the update scale is dt)
  double W;                  // sum of the direction weights
  int wall[6];
  const double* wall_I0[6];  // [nb][nfaces] for isothermal walls, else null
  const void* wall_S[6];     // the same in intensity storage format (Real, minus Iref)
  int wall_nf[6];
};

// Scattering rate 1/tau_b(T) of a temperature-dependent relaxation time
// tau_b(T) = tau_b (T0 / T)^p_b (Sec. 2.2: I0 and tau both depend on T).
__device__ __forceinline__ double relax_rate(double inv_tau, double p, double T, double T0) {
  return inv_tau * pow(T / T0, p);
}

// Everything one sweep launch reads: mesh, tables, the three intensity
// fields of the iteration (current iterate, step start, new iterate), the
// equilibrium at the current temperature, the outputs.
template <typename Real>
struct SweepParams {
  Geometry g;
  Tables t;
  const Real* __restrict__ Ik;
  const Real* __restrict__ In;
  Real* __restrict__ Iout;
  const double* __restrict__ I0;
  double* __restrict__ S;
  double* __restrict__ part;
  const Control* ctl;
  double inv_dt;
  // first sweep of a warm-started step: I^(0) = I^n + shift[b][P] (isotropic
  // equilibrium shift at the guessed temperature); null otherwise
  const double* __restrict__ shift;
};

// Launchers (bte_kernels.hip).  All enqueue on `stream` and return the launch status.
template <typename Real>
hipError_t launch_sweep(hipStream_t stream, const Geometry& g, const Tables& t,
                        const SweepPlan& plan, double inv_dt, const Real* Ik, const Real* In,
                        Real* Iout, const double* I0, double* S, double* part,
                        const Control* ctl, const double* shift);

hipError_t launch_temperature(hipStream_t stream, const Geometry& g, const Tables& t,
                              double* S, double* T, double* I0, double* E, Control* ctl);

hipError_t launch_control(hipStream_t stream, int nparts, const double* part, double vol,
                          int fixed_k, int max_inner, double tol, int explicit_mode,
                          Control* ctl);

hipError_t launch_reset(hipStream_t stream, Control* ctl);

// ---------------------------------------------------------------- batches
// One geometry of a batched step as the batched kernels see it.  The three
// intensity fields F[] and in_idx (which one holds I^n) let the kernels pick
// each inner iteration's source and destination from the device iteration
// count, so one captured launch sequence serves every iteration.
struct BatchCtx {
  SweepParams<double> sp64;  // sweep parameters (the one matching the storage is used);
  SweepParams<float> sp32;   // Ik / Iout are rewritten on the device every iteration
  SweepPlan plan;
  int precision;  // 0 FP64, 1 FP32 storage
  int in_idx;
  void* F[3];
  double* I0;
  double* S;
  double* part;
  double* T;
  double* E;
  Control* ctl;
  double tol;
  int max_inner, fixed_k;
  int cell_block0, cell_blocks;  // blocks of the batched temperature kernel
};

struct BatchItem {
  int ctx, bx, by, bz;
};

struct BatchControl {
  int next_item;     // persistent-sweep work counter (2D list)
  int iteration;     // batched iterations completed
  int active;        // geometries not yet converged after the last iteration
  int next_item3d;   // persistent-sweep work counter (3D list)
  int next_item_f4;  // persistent-sweep work counter (3D flattened-plane 4-plane list)
  int pad[3];
};

// Work lists of a batch, one persistent launch each: 2D column walks; 3D
// column walks and the flattened plane with 2 planes; the flattened plane
// with 4 planes (a kernel of its own, since it needs more registers).
enum BatchList { kList2D = 0, kList3D = 1, kListFlat4 = 2, kBatchLists = 3 };

// A work list described by its geometries' item ranges instead of stored
// items: geometry ctx[j] owns items [start[j], start[j + 1]) of the list,
// ordered direction group, band, tile (tile fastest).
struct BatchRanges {
  int n;             // geometries in the list
  const int* ctx;    // [n] context index
  const int* start;  // [n + 1] first item of each geometry, then the item count
};

// One inner iteration of every geometry: persistent sweep over the work list,
// temperature inversion, per-geometry control, active count (+ reset of the
// work counter for the next iteration).
// items holds the lists back to back; counts[l] and sweep_blocks[l] per BatchList.
hipError_t launch_batch_iteration(hipStream_t stream, int precision, BatchCtx* ctxs,
                                  int nctx, const BatchItem* items,
                                  const int counts[kBatchLists], BatchControl* bc,
                                  const int sweep_blocks[kBatchLists], int temp_blocks);
// The same iteration with the work lists given as geometry ranges (no stored
// items).
hipError_t launch_batch_iteration_ranges(hipStream_t stream, int precision, BatchCtx* ctxs,
                                         int nctx, const BatchRanges ranges[kBatchLists],
                                         const int counts[kBatchLists], BatchControl* bc,
                                         const int sweep_blocks[kBatchLists], int temp_blocks);
hipError_t launch_batch_reset(hipStream_t stream, BatchCtx* ctxs, int nctx, BatchControl* bc);
// Resident workgroups per compute unit of one list's persistent sweep kernel.
int batch_sweep_occupancy(int precision, int list);

// I0[b][P] = I0_b(T_P) (and t.relax at T_P if the relaxation times depend on
// T); E_P = W sum_b I0_b(T_P) if E is given.
hipError_t launch_equilibrium(hipStream_t stream, const Geometry& g, const Tables& t,
                              const double* T, double* I0, double* E);

hipError_t launch_wall_table(hipStream_t stream, int nb, int nf, const double* Cb,
                             const double* xfac, const double* wallT, double* out);

// The isothermal wall table in intensity storage format: out[i] = in[i] - Iref[i / nf]
// as Real (identity for FP64).
template <typename Real>
hipError_t launch_wall_storage(hipStream_t stream, int nb, int nf, const double* in,
                               const double* Iref, Real* out);

// The ghost table of a diffuse wall side from the current iterate I:
// wall_I0[b][face] = sum_d wts[d] I_{d,b,P(face)} (+ the isotropic first-sweep
// shift of P, if given), wts the side's normalised outgoing-flux weights, and
// wall_S the same in storage format.
template <typename Real>
hipError_t launch_diffuse_wall(hipStream_t stream, const Geometry& g, const Tables& t, int side,
                               const double* wts, const Real* I, const double* shift,
                               double* wall_I0, Real* wall_S);

// Iref[b] = I0_b(T_ref) if T_ref > 0, else 0.
hipError_t launch_reference(hipStream_t stream, int nb, const double* Cb, const double* xfac,
                            double T_ref, double* Iref);

template <typename Real>
hipError_t launch_broadcast(hipStream_t stream, const Geometry& g, const Tables& t,
                            const double* I0, Real* I);

template <typename Real>
hipError_t launch_energy(hipStream_t stream, const Geometry& g, const Tables& t, const Real* I,
                         double* E);

}  // namespace bte
