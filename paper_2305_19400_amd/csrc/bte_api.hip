// C ABI of the phonon BTE library (declared in include/bte.h): input
// validation, workspace layout, per-(direction, band) coefficient tables,
// mirror maps, and the time-step driver that enqueues the HIP kernels of
// bte_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"
#include "bte_nn.h"

using namespace bte;

namespace bte {

// Launch layout of a sweep: kernel family, tile shape, tile counts and
// direction groups for a mesh (host logic; the kernels take the plan as is).
SweepPlan make_sweep_plan(int dim, int nx, int ny, int nz, int nd, int nb, int ry, int rz,
                          int ndg, int kind) {
  SweepPlan pl{};
  pl.rz = 1;
  pl.ntz = 1;
  if (dim == 2 && kind != kSweepCellPerThread) {
    pl.kind = kSweepColumnWalk2D;
    if (ry != 4 && ry != 8 && ry != 16) ry = 4;
    pl.ry = ry;
    pl.ntx = (nx + 63) / 64;
    pl.nty = (ny + 4 * ry - 1) / (4 * ry);
    pl.ntiles = pl.ntx * pl.nty;
  } else if (dim == 3 && kind == kSweepFlat3D) {
    pl.kind = kSweepFlat3D;
    // 256 plane cells (4 waves x 64 lanes) x rz planes per workgroup
    if (rz != 2 && rz != 4) rz = 4;
    pl.ry = 0;
    pl.rz = rz;
    pl.ntx = (nx * ny + 255) / 256;
    pl.nty = 1;
    pl.ntz = (nz + rz - 1) / rz;
    pl.ntiles = pl.ntx * pl.ntz;
  } else if (dim == 3 && kind != kSweepCellPerThread) {
    pl.kind = kSweepColumnWalk3D;
    // (rows, planes) per wave: 2 x 2 (default), 1 x 4 or 2 x 4
    if (!((ry == 2 && rz == 2) || (ry == 1 && rz == 4) || (ry == 2 && rz == 4))) {
      ry = 2;
      rz = 2;
    }
    pl.ry = ry;
    pl.rz = rz;
    pl.ntx = (nx + 63) / 64;
    pl.nty = (ny + 4 * ry - 1) / (4 * ry);
    pl.ntz = (nz + rz - 1) / rz;
    pl.ntiles = pl.ntx * pl.nty * pl.ntz;
  } else {
    pl.kind = kSweepCellPerThread;
    pl.ry = 1;
    pl.ntx = (nx * ny * nz + kSweepBlock - 1) / kSweepBlock;
    pl.nty = 1;
    pl.ntiles = pl.ntx;
    ndg = 1;
  }
  if (ndg <= 0) {
    // aim for about 32 workgroups per compute unit of a 256-CU device, so the
    // last partial round of workgroups is a small fraction of the sweep ...
    const long long wg = (long long)pl.ntiles * nb;
    const long long fill = std::max<long long>(1, (kSweepFillWorkgroups + wg - 1) / wg);
    // ... but each direction group writes an 8-byte energy partial per (band,
    // cell), which the temperature kernel reads back: keep that within 1/25 of
    // the sweep's intensity bytes (3 x 4 bytes per direction in FP32 storage,
    // twice that in FP64), unless the launch would drop below 4 workgroups
    // per compute unit (a small sweep is bound by latency, not bytes)
    const long long by_bytes = std::max<long long>(1, (3LL * nd * 4) / (8 * 25));
    const long long quarter = std::max<long long>(1, (1024 + wg - 1) / wg);
    ndg = (int)std::min<long long>(nd, std::min(fill, std::max(by_bytes, quarter)));
  }
  ndg = std::max(1, std::min(ndg, nd));
  pl.dgs = (nd + ndg - 1) / ndg;
  pl.ndg = (nd + pl.dgs - 1) / pl.dgs;
  pl.nparts = pl.ntiles * nb * pl.ndg;
  return pl;
}

}  // namespace bte

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

constexpr size_t kAlign = 256;
constexpr int kRing = 4;         // pinned control snapshots in flight
constexpr int kDeferSteps = 64;  // steps queued before the host reads their control words
constexpr int kMaxStepGraphs = 24;
constexpr double kMirrorTol = 1e-12;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t ctl, coef, dflags, mirror, w, Cb, xfac, inv_tau, fweight, Iref;
  size_t wallT[6], wallI0[6], wallS[6], dwt;
  size_t T, Tprev, E, I0, S, part, relax, tau_p;
  // learned warm start (present if warm_start != 0)
  size_t nn_params, nn_grad, nn_m, nn_v, nn_W1b, nn_W2b, nn_W2Tb, nn_y, nn_hist, nn_loss,
      nn_fallbacks, nn_XT, nn_H1T, nn_dZ1T, nn_dZ2T, nn_part, nn_shift, nn_guess;
  size_t In, Ia, Ib;
  size_t total;
};

struct Shape {
  int dim, nx, ny, nz, nc, ncp, px, nd, nb;  // as in Geometry
  int nf[6];
  bool iso[6];   // isothermal: face temperatures given
  bool diff[6];  // diffuse: ghost table recomputed every iteration
  size_t real_size;
  SweepPlan plan;
  int ndg_cap, nparts_cap;  // room for any layout the autotuner may pick
  int warm;       // bte_warm
  int nn_rec;     // recorded steps before training
};

// 3D: whether 64-column tiles would leave more than an eighth of the lanes
// idle (a narrow mesh or a ragged last tile), where the flattened (x, y)
// plane is the default family.
bool flat_by_lanes(int nx) {
  const double lanes_used = (double)nx / (64.0 * ((nx + 63) / 64));
  return lanes_used < 0.875;
}

// The layouts a batched persistent sweep compiles: 4 rows per wave in 2D;
// in 3D 2 rows x 2 planes or 1 row x 4 planes per wave, or the flattened
// (x, y) plane with 2 or 4 planes per wave.
bool batch_layout(int kind, int ry, int rz) {
  if (kind == kSweepColumnWalk2D) return ry == 4;
  if (kind == kSweepColumnWalk3D) return (ry == 2 && rz == 2) || (ry == 1 && rz == 4);
  if (kind == kSweepFlat3D) return rz == 2 || rz == 4;
  return false;
}

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return (v && *v) ? atoi(v) : dflt;
}

Layout make_layout(const Shape& s) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.ctl = take(sizeof(Control));
  L.coef = take(sizeof(Coef) * (size_t)s.nb * s.nd);
  L.dflags = take(sizeof(int) * (size_t)s.nd);
  L.mirror = take(sizeof(int) * 3 * (size_t)s.nd);
  L.w = take(sizeof(double) * (size_t)s.nd);
  L.Cb = take(sizeof(double) * (size_t)s.nb);
  L.xfac = take(sizeof(double) * (size_t)s.nb);
  L.inv_tau = take(sizeof(double) * (size_t)s.nb);
  L.fweight = take(sizeof(double) * (size_t)s.nb);
  L.Iref = take(sizeof(double) * (size_t)s.nb);
  for (int f = 0; f < 6; ++f) {
    const bool table = s.iso[f] || s.diff[f];
    L.wallT[f] = s.iso[f] ? take(sizeof(double) * (size_t)s.nf[f]) : 0;
    L.wallI0[f] = table ? take(sizeof(double) * (size_t)s.nf[f] * s.nb) : 0;
    L.wallS[f] = table ? take(s.real_size * (size_t)s.nf[f] * s.nb) : 0;
  }
  L.dwt = take(sizeof(double) * 6 * (size_t)s.nd);
  L.T = take(sizeof(double) * (size_t)s.ncp);
  L.Tprev = take(sizeof(double) * (size_t)s.ncp);
  L.E = take(sizeof(double) * (size_t)s.ncp);
  L.I0 = take(sizeof(double) * (size_t)s.nb * s.ncp);
  L.S = take(sizeof(double) * (size_t)s.ndg_cap * s.nb * s.ncp);
  L.part = take(sizeof(double) * 2 * (size_t)s.nparts_cap);
  // scattering rates at the cells' temperatures, used if the relaxation
  // times depend on temperature (the dispersion is not known when sizing)
  L.relax = take(sizeof(double) * (size_t)s.nb * s.ncp);
  L.tau_p = take(sizeof(double) * (size_t)s.nb);
  if (s.warm) {
    const NnLayout N = make_nn_layout(s.dim);
    const size_t P = (size_t)N.total;
    L.nn_params = take(sizeof(float) * P);
    L.nn_grad = take(sizeof(float) * P);
    L.nn_m = take(sizeof(float) * P);
    L.nn_v = take(sizeof(float) * P);
    L.nn_W1b = take(2 * (size_t)kNnHidden * N.KP);
    L.nn_W2b = take(2 * (size_t)kNnHidden * kNnHidden);
    L.nn_W2Tb = take(2 * (size_t)kNnHidden * kNnHidden);
    L.nn_y = take(sizeof(float) * (size_t)s.nc);
    // one extra slot for bte_nn_gradient's sample
    L.nn_hist = take(sizeof(float) * 4 * (size_t)(s.nn_rec + 1) * s.nc);
    L.nn_loss = take(sizeof(float));
    L.nn_fallbacks = take(sizeof(int));
    L.nn_XT = take(2 * (size_t)N.KP * kNnBatch);
    L.nn_H1T = take(2 * (size_t)kNnHidden * kNnBatch);
    L.nn_dZ1T = take(2 * (size_t)kNnHidden * kNnBatch);
    L.nn_dZ2T = take(2 * (size_t)kNnHidden * kNnBatch);
    L.nn_part = take(sizeof(float) * (size_t)(kNnBatch / 64) * kNnPartWidth);
    L.nn_shift = take(sizeof(double) * (size_t)s.nb * s.ncp);
    L.nn_guess = take(sizeof(double) * (size_t)s.nc);
  }
  const size_t field = s.real_size * (size_t)s.nb * s.nd * s.ncp;
  L.In = take(field);
  L.Ia = take(field);
  L.Ib = take(field);
  L.total = off + 65536;  // tail slack: no kernel access may reach past the last array
  return L;
}

constexpr long long kMaxCells = (INT_MAX - 255) / 8;  // slab bytes fit a signed 32-bit offset

int validate(const bte_mesh* m, const bte_dirs* d, const bte_bands* b, const bte_options* o,
             Shape* out) {
  if (!m || !d || !b || !o) return fail(BTE_E_INVAL, "null argument");
  if (m->dim != 2 && m->dim != 3) return fail(BTE_E_INVAL, "dim must be 2 or 3, got %d", m->dim);
  for (int a = 0; a < 3; ++a)
    if (m->n[a] < 1) return fail(BTE_E_INVAL, "n[%d] must be >= 1", a);
  if (m->dim == 2 && m->n[2] != 1) return fail(BTE_E_INVAL, "2D mesh needs n[2] == 1");
  for (int a = 0; a < m->dim; ++a)
    if (!(m->h[a] > 0.0) || !std::isfinite(m->h[a])) return fail(BTE_E_INVAL, "h[%d] must be positive", a);
  const long long nc = (long long)m->n[0] * m->n[1] * m->n[2];
  // the sweeps address one (band, direction) slab of FP64 values with 32-bit
  // byte offsets
  if (nc > kMaxCells)
    return fail(BTE_E_INVAL, "too many cells (%lld; at most %lld)", nc, (long long)kMaxCells);
  if (d->n < 1 || !d->s || !d->w) return fail(BTE_E_INVAL, "need at least one direction");
  if (d->n > 65535) return fail(BTE_E_INVAL, "at most 65535 directions");
  if (b->n < 1 || !b->omega || !b->domega) return fail(BTE_E_INVAL, "need at least one band");
  if (b->n > 65535) return fail(BTE_E_INVAL, "at most 65535 band entries");
  {
    // a side's wall table [band entry][face] is addressed with 32-bit byte offsets too
    const long long nx = m->n[0], ny = m->n[1], nz = m->n[2];
    const long long faces =
        m->dim == 3 ? std::max(ny * nz, std::max(nx * nz, nx * ny)) : std::max(nx, ny);
    if ((long long)b->n * faces > kMaxCells)
      return fail(BTE_E_INVAL, "band entries x wall faces too large (%lld x %lld)",
                  (long long)b->n, faces);
  }
  if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(BTE_E_INVAL, "dt must be positive");
  if (o->scheme != BTE_IMPLICIT_JACOBI && o->scheme != BTE_EXPLICIT_EULER)
    return fail(BTE_E_INVAL, "unknown scheme %d", o->scheme);
  if (o->precision != BTE_FP64 && o->precision != BTE_FP32_MIXED)
    return fail(BTE_E_INVAL, "unknown precision %d", o->precision);
  if (o->t_definition != BTE_T_TAU_WEIGHTED && o->t_definition != BTE_T_ENERGY)
    return fail(BTE_E_INVAL, "unknown temperature definition %d", o->t_definition);
  if (!m->T_init) return fail(BTE_E_INVAL, "T_init is required");
  if (o->warm_start < BTE_WARM_NONE || o->warm_start > BTE_WARM_T_SHIFT)
    return fail(BTE_E_INVAL, "unknown warm_start %d", o->warm_start);
  if (o->warm_start != BTE_WARM_NONE && o->scheme != BTE_IMPLICIT_JACOBI)
    return fail(BTE_E_INVAL, "the learned warm start seeds the implicit inner iteration only");
  Shape s{};
  s.dim = m->dim;
  s.nx = m->n[0];
  s.ny = m->n[1];
  s.nz = m->n[2];
  s.nc = (int)nc;
  {
    // 2D: intensity rows padded to a 128-byte line of stored values
    const long long line = o->precision == BTE_FP64 ? 16 : 32;
    const long long px = s.dim == 2 ? (s.nx + line - 1) / line * line : s.nx;
    const long long ncp =
        s.dim == 2 ? px * s.ny : (nc + kSlabAlign - 1) / kSlabAlign * kSlabAlign;
    if (ncp > kMaxCells)
      return fail(BTE_E_INVAL, "too many cells with padding (%lld; at most %lld)", ncp,
                  (long long)kMaxCells);
    s.px = (int)px;
    s.ncp = (int)ncp;
  }
  s.nd = d->n;
  s.nb = b->n;
  // Launch layout of the sweep; BTE_SWEEP_RY / BTE_SWEEP_RZ / BTE_SWEEP_NDG /
  // BTE_SWEEP_KIND override the rows and planes per wave, the number of
  // direction groups and the kernel family (tuning knobs).  3D defaults: when
  // 64-column tiles would leave more than an eighth of the lanes idle (a
  // narrow mesh or a ragged last tile), the flattened (x, y) plane, with 4
  // planes per wave for FP32 storage; with FP64 storage 4 planes once the
  // 4-plane launch fills the device with a single direction group (4-5 %
  // faster there) and 2 below that (whose registers allow more waves, and the
  // extra tiles fewer direction groups); otherwise 2 rows x 2 planes per wave
  // with FP64 storage and 1 row x 4 planes with FP32 storage (the faster at
  // 64^3).
  const bool fp32 = o->precision != BTE_FP64;
  int ry_dflt = 0, rz_dflt = 0, kind_dflt = -1;
  if (s.dim == 3) {
    if (flat_by_lanes(s.nx)) {
      kind_dflt = kSweepFlat3D;
      const long long tiles4 =
          ((long long)s.nx * s.ny + 255) / 256 * ((s.nz + 3) / 4) * (long long)s.nb;
      rz_dflt = (fp32 || tiles4 >= kSweepFillWorkgroups) ? 4 : 2;
    } else if (fp32) {
      ry_dflt = 1;
      rz_dflt = 4;
    }
  }
  s.plan = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, env_int("BTE_SWEEP_RY", ry_dflt),
                           env_int("BTE_SWEEP_RZ", rz_dflt), env_int("BTE_SWEEP_NDG", 0),
                           env_int("BTE_SWEEP_KIND", kind_dflt));
  s.ndg_cap = s.plan.ndg;
  s.nparts_cap = s.plan.nparts;
  if (s.plan.kind == kSweepColumnWalk2D) {
    // the 4-row layout has the most tiles; up to 16 direction groups
    const SweepPlan widest = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, 4, 1,
                                             std::min(s.nd, 16), kSweepColumnWalk2D);
    s.ndg_cap = std::max(s.ndg_cap, widest.ndg);
    s.nparts_cap = std::max(s.nparts_cap, widest.ntiles * s.nb * s.ndg_cap);
  } else if (s.plan.kind == kSweepColumnWalk3D || s.plan.kind == kSweepFlat3D) {
    // 2 x 2, 1 x 4 (rows x planes) and the flattened 2-plane layout have the
    // most tiles; up to 4 direction groups
    const SweepPlan a = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, 2, 2,
                                        std::min(s.nd, 4), kSweepColumnWalk3D);
    const SweepPlan c = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, 1, 4,
                                        std::min(s.nd, 4), kSweepColumnWalk3D);
    const SweepPlan fp = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, 0, 2,
                                         std::min(s.nd, 4), kSweepFlat3D);
    s.ndg_cap = std::max(s.ndg_cap, std::max(std::max(a.ndg, c.ndg), fp.ndg));
    s.nparts_cap = std::max(s.nparts_cap, std::max(std::max(a.ntiles, c.ntiles), fp.ntiles) *
                                              s.nb * s.ndg_cap);
  }
  s.real_size = o->precision == BTE_FP64 ? sizeof(double) : sizeof(float);
  s.warm = o->warm_start;
  s.nn_rec = o->nn_train_steps > 0 ? o->nn_train_steps : 20;
  const int nfaces[3] = {s.ny * s.nz, s.nx * s.nz, s.nx * s.ny};
  for (int f = 0; f < 6; ++f) {
    s.nf[f] = nfaces[f / 2];
    s.iso[f] = false;
    s.diff[f] = false;
    if (f >= 2 * s.dim) continue;
    const int kind = m->wall[f];
    if (kind == BTE_WALL_ISOTHERMAL) {
      if (!m->wall_T[f]) return fail(BTE_E_INVAL, "isothermal wall %d needs wall_T", f);
      s.iso[f] = true;
    } else if (kind == BTE_WALL_DIFFUSE) {
      s.diff[f] = true;
    } else if (kind != BTE_WALL_SPECULAR && kind != BTE_WALL_SYMMETRY) {
      return fail(BTE_E_INVAL, "unknown wall kind %d on side %d", kind, f);
    }
  }
  *out = s;
  return BTE_OK;
}

}  // namespace

struct bte_ctx {
  Shape s;
  Layout L;
  Geometry g;
  Tables t;
  bte_options opt;
  hipStream_t stream;
  char* ws;
  Control* ctl;
  Control* host_ring;  // pinned
  hipEvent_t ring_ev[kRing];
  Control* host_steps;  // pinned, one per step queued without a host wait
  // captured chunks of inner iterations of free-running steps, one per
  // arrangement of the three intensity fields (see enqueue_chunk)
  struct StepGraph {
    const void* In;
    const void* Ia;
    const void* Ib;
    const double* shift;
    int first;
    SweepPlan plan;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<StepGraph> step_graphs;
  std::vector<hipEvent_t> t_start, t_stop;
  double timing_ms;
  int timing_count;
  void* In;
  void* Ia;
  void* Ib;
  double* T;
  double* Tprev;
  double* E;
  double* I0;
  double* S;
  double* part;
  const double* first_shift;  // shift of the first sweep of the current step (or null)
  std::vector<double> Iref;  // host copy of the storage reference per band
  // learned warm start
  NnLayout nnL;
  NnBuffers nnB;
  double* nn_shift;
  double* nn_guess;
  int nn_nrec;      // steps recorded so far
  int nn_ready;     // network trained (or parameters set)
  int nn_off;       // guess switched off: it did not save sweeps
  int nn_warm_steps, nn_warm_sweeps;  // warm-started steps so far and their sweeps
  std::vector<int> nn_plain_sweeps;   // sweeps of the recorded plain steps
  int nn_adam_t;    // Adam steps taken
  // Set by a batch step: a training that falls due is queued here and run,
  // together with the other geometries' trainings, by the batch (null: train
  // at once).
  std::vector<bte_ctx*>* train_queue = nullptr;
  bool nn_loss_pending = false;     // trained; loss not read yet
  int nn_last_batch = 1;            // samples of the last minibatch
  long long steps_taken = 0;        // time steps completed since create
  double* dwt = nullptr;            // [6][nd] diffuse walls' outgoing-flux weights
  bool any_diffuse = false;
  bool poisoned;
};

namespace {

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      if (ctx) ctx->poisoned = true;                                                          \
      return fail(BTE_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));               \
    }                                                                                         \
  } while (0)

template <typename T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

void find_mirrors(const bte_dirs* d, int dim, std::vector<int>& mirror) {
  mirror.assign(3 * (size_t)d->n, -1);
  for (int a = 0; a < 3; ++a) {
    for (int i = 0; i < d->n; ++i) {
      double t[3] = {d->s[3 * i], d->s[3 * i + 1], d->s[3 * i + 2]};
      t[a] = -t[a];
      for (int j = 0; j < d->n; ++j) {
        const double* u = d->s + 3 * (size_t)j;
        if (std::fabs(u[0] - t[0]) <= kMirrorTol && std::fabs(u[1] - t[1]) <= kMirrorTol &&
            std::fabs(u[2] - t[2]) <= kMirrorTol) {
          mirror[(size_t)a * d->n + i] = j;
          break;
        }
      }
    }
  }
  (void)dim;
}

template <typename Real>
int enqueue_sweep(bte_ctx* ctx, const void* src, void* dst, const double* shift) {
  HIP_TRY(launch_sweep<Real>(ctx->stream, ctx->g, ctx->t, ctx->s.plan, 1.0 / ctx->opt.dt,
                             static_cast<const Real*>(src), static_cast<const Real*>(ctx->In),
                             static_cast<Real*>(dst), ctx->I0, ctx->S, ctx->part, ctx->ctl,
                             shift));
  return BTE_OK;
}

int enqueue_iteration(bte_ctx* ctx, int j, int fixed_k) {
  const void* src = (j == 0) ? ctx->In : ((j & 1) ? ctx->Ia : ctx->Ib);
  void* dst = (j & 1) ? ctx->Ib : ctx->Ia;
  const bool timing = ctx->opt.timing != 0;
  if (timing) {
    while ((int)ctx->t_start.size() <= j) {
      hipEvent_t a, b;
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      ctx->t_start.push_back(a);
      ctx->t_stop.push_back(b);
    }
    HIP_TRY(hipEventRecord(ctx->t_start[j], ctx->stream));
  }
  const double* shift = (j == 0) ? ctx->first_shift : nullptr;
  if (ctx->any_diffuse) {
    // diffuse walls' ghosts from the iterate this sweep reads
    for (int f = 0; f < 2 * ctx->s.dim; ++f) {
      if (!ctx->s.diff[f]) continue;
      double* w0 = const_cast<double*>(ctx->t.wall_I0[f]);
      void* wsr = const_cast<void*>(ctx->t.wall_S[f]);
      if (ctx->opt.precision == BTE_FP64)
        HIP_TRY(launch_diffuse_wall<double>(ctx->stream, ctx->g, ctx->t, f,
                                            ctx->dwt + (size_t)f * ctx->s.nd,
                                            static_cast<const double*>(src), shift, w0,
                                            static_cast<double*>(wsr)));
      else
        HIP_TRY(launch_diffuse_wall<float>(ctx->stream, ctx->g, ctx->t, f,
                                           ctx->dwt + (size_t)f * ctx->s.nd,
                                           static_cast<const float*>(src), shift, w0,
                                           static_cast<float*>(wsr)));
    }
  }
  int rc = ctx->opt.precision == BTE_FP64 ? enqueue_sweep<double>(ctx, src, dst, shift)
                                          : enqueue_sweep<float>(ctx, src, dst, shift);
  if (rc != BTE_OK) return rc;
  if (timing) HIP_TRY(hipEventRecord(ctx->t_stop[j], ctx->stream));
  HIP_TRY(launch_temperature(ctx->stream, ctx->g, ctx->t, ctx->S, ctx->T, ctx->I0, ctx->E,
                             ctx->ctl));
  HIP_TRY(launch_control(ctx->stream, ctx->s.plan.nparts, ctx->part, ctx->g.vol, fixed_k,
                         ctx->opt.max_inner, ctx->opt.tol,
                         ctx->opt.scheme == BTE_EXPLICIT_EULER, ctx->ctl));
  return BTE_OK;
}

long long gcd_ll(long long a, long long b) {
  while (b) {
    const long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Mean loss over the last minibatch of the last training (waits for it).
int nn_read_loss(bte_ctx* ctx, double* last_loss) {
  float loss = 0.f;
  HIP_TRY(hipMemcpyAsync(&loss, ctx->nnB.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (last_loss) *last_loss = (double)loss / (double)ctx->nn_last_batch;
  ctx->nn_loss_pending = false;
  return BTE_OK;
}

// The minibatch schedule of a training: Adam over minibatches in a
// pseudo-random sample order (affine permutation i -> (a i + c_e) mod N with
// gcd(a, N) = 1, c_e per epoch), at least two passes and 300 updates unless
// nn_epochs is given.
struct TrainSchedule {
  long long N, a;
  float lr;
  struct Update {
    long long b0, c;
    int batch;
  };
  std::vector<Update> updates;
};

TrainSchedule nn_schedule(const bte_ctx* ctx) {
  TrainSchedule ts;
  ts.N = (long long)ctx->nn_nrec * ctx->s.nc;
  const long long N = ts.N;
  ts.a = (long long)(0.6180339887 * (double)N) | 1;
  while (gcd_ll(ts.a, N) != 1) ts.a += 2;
  const long long per_epoch = (N + kNnBatch - 1) / kNnBatch;
  int epochs = ctx->opt.nn_epochs;
  if (epochs <= 0) epochs = (int)std::max<long long>(2, (300 + per_epoch - 1) / per_epoch);
  ts.lr = ctx->opt.nn_lr > 0.f ? ctx->opt.nn_lr : 1e-3f;
  for (int e = 0; e < epochs; ++e) {
    const long long c = ((long long)e * 7919) % N;
    for (long long b0 = 0; b0 < N; b0 += kNnBatch)
      ts.updates.push_back({b0, c, (int)std::min<long long>(kNnBatch, N - b0)});
  }
  return ts;
}

// Trains the network on the recorded steps: normalisation constants, then the
// minibatch schedule above (or queues the context for its batch to train).
int nn_train(bte_ctx* ctx, double* last_loss) {
  if (ctx->train_queue) {  // the batch trains it with the others
    ctx->train_queue->push_back(ctx);
    if (last_loss) *last_loss = 0.0;
    return BTE_OK;
  }
  HIP_TRY(nn_stats(ctx->stream, ctx->nnL, ctx->nnB, ctx->nn_nrec, ctx->s.nc));
  const TrainSchedule ts = nn_schedule(ctx);
  for (const auto& u : ts.updates) {
    ctx->nn_adam_t += 1;
    HIP_TRY(nn_train_batch(ctx->stream, ctx->g, ctx->nnL, ctx->nnB, ts.N, ts.a, u.c, u.b0,
                           u.batch, ts.lr, ctx->nn_adam_t, true));
  }
  ctx->nn_last_batch = ts.updates.back().batch;
  ctx->nn_ready = 1;
  return nn_read_loss(ctx, last_loss);
}

// What one time step decided before its inner loop.
struct StepState {
  bool explicit_mode, check, warm, record;
  int fixed, limit;
  float* slot;
};

// Everything before the inner loop: record the network's training inputs,
// or apply its guess of T_{n+1} (which also moves T_n into T_prev); otherwise
// T_prev <- T_n.
int step_begin(bte_ctx* ctx, int fixed, StepState* ss) {
  const int nc = ctx->s.nc;
  ss->explicit_mode = ctx->opt.scheme == BTE_EXPLICIT_EULER;
  ss->fixed = fixed;
  ss->limit = ss->explicit_mode ? 1 : (fixed > 0 ? fixed : ctx->opt.max_inner);
  ss->check = !ss->explicit_mode && fixed <= 0;
  ss->warm = ctx->s.warm && ctx->nn_ready && !ctx->nn_off;
  ss->record = ctx->s.warm && !ctx->nn_ready && ctx->nn_nrec < ctx->s.nn_rec;
  ss->slot = ctx->s.warm ? ctx->nnB.hist + (size_t)ctx->nn_nrec * 4 * nc : nullptr;
  if (ss->record) HIP_TRY(nn_record(ctx->stream, nc, ctx->T, ctx->Tprev, ctx->E, ss->slot, 0));
  double* shift = nullptr;
  if (ss->warm) {
    HIP_TRY(hipMemsetAsync(ctx->nnB.fallbacks, 0, sizeof(int), ctx->stream));
    HIP_TRY(nn_predict(ctx->stream, ctx->g, ctx->nnL, ctx->nnB, ctx->T, ctx->Tprev, ctx->E));
    shift = ctx->s.warm == BTE_WARM_T_SHIFT ? ctx->nn_shift : nullptr;
    HIP_TRY(nn_apply_guess(ctx->stream, ctx->g, ctx->t, ctx->nnL, ctx->nnB, ctx->Tprev, ctx->T,
                           ctx->I0, shift, 10.0f));
  } else {
    HIP_TRY(hipMemcpyAsync(ctx->Tprev, ctx->T, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                           ctx->stream));
  }
  ctx->first_shift = shift;
  return BTE_OK;
}

// Everything after the inner loop, given the final control words: error
// report, sweep timing, I^{n+1} <- newest iterate, the network's training
// target and training, statistics.
int step_finish(bte_ctx* ctx, const StepState& ss, const Control& fin, bte_step_stats* st,
                bool swapped = false) {
  const int nc = ctx->s.nc;
  if (fin.err_cell != INT_MAX) {
    const int P = fin.err_cell;
    const int x = P % ctx->s.nx, y = (P / ctx->s.nx) % ctx->s.ny, z = P / (ctx->s.nx * ctx->s.ny);
    return fail(BTE_E_NUMERIC,
                "temperature inversion failed in cell %d (x=%d y=%d z=%d): energy not positive "
                "and finite, or Newton did not converge",
                P, x, y, z);
  }
  if (ctx->opt.timing) {
    for (int j = 0; j < fin.k && j < (int)ctx->t_start.size(); ++j) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->t_start[j], ctx->t_stop[j]));
      ctx->timing_ms += ms;
      ctx->timing_count += 1;
    }
  }
  // the newest iterate becomes I^{n+1}
  if (!swapped) {
    void*& last = ((fin.k - 1) & 1) ? ctx->Ib : ctx->Ia;
    std::swap(ctx->In, last);
  }
  ctx->steps_taken += 1;
  int trained = 0, fallbacks = 0;
  double loss = 0.0;
  if (ss.warm) {
    HIP_TRY(hipMemcpyAsync(&fallbacks, ctx->nnB.fallbacks, sizeof(int), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  if (ss.record) {
    HIP_TRY(nn_record(ctx->stream, nc, ctx->T, ctx->Tprev, ctx->E, ss.slot, 1));
    ctx->nn_plain_sweeps.push_back(fin.k);
    ctx->nn_nrec += 1;
    if (ctx->nn_nrec == ctx->s.nn_rec) {
      int rc = nn_train(ctx, &loss);
      if (rc != BTE_OK) return rc;
      trained = 1;
    }
  }
  if (ss.warm) {
    // The plain iteration judges the guess: every `guard` warm steps, their
    // sweeps are compared with the last `guard` plain steps recorded before
    // training, and a guess that costs sweeps is switched off for good.
    const int guard = ctx->opt.nn_guard == 0 ? 4 : ctx->opt.nn_guard;
    ctx->nn_warm_steps += 1;
    ctx->nn_warm_sweeps += fin.k;
    const int nplain = (int)ctx->nn_plain_sweeps.size();
    if (guard > 0 && ctx->nn_warm_steps == guard && nplain >= guard) {
      int plain = 0;
      for (int i = nplain - guard; i < nplain; ++i) plain += ctx->nn_plain_sweeps[i];
      if (ctx->nn_warm_sweeps > plain) ctx->nn_off = 1;
      ctx->nn_warm_steps = 0;  // next window
      ctx->nn_warm_sweeps = 0;
    }
  }
  if (st) {
    st->inner = fin.k;
    st->newton_max = fin.newton_max;
    st->res = fin.res;
    st->converged =
        ss.explicit_mode || (ss.fixed > 0 ? fin.k >= ss.fixed : fin.res <= ctx->opt.tol);
    st->warm = ss.warm ? 1 : 0;
    st->fallbacks = fallbacks;
    st->trained = trained;
    st->nn_loss = loss;
  }
  if (!ss.explicit_mode && ss.fixed <= 0 && fin.res > ctx->opt.tol && ctx->opt.fail_on_notconv)
    return fail(BTE_E_NOTCONV, "inner iteration hit max_inner=%d with res=%g > tol=%g",
                ctx->opt.max_inner, fin.res, ctx->opt.tol);
  return BTE_OK;
}

// Inner iterations per captured chunk of a free-running step (BTE_GRAPH_CHUNK
// overrides; 0 turns the graphs off).
int graph_chunk() {
  static const int c = env_int("BTE_GRAPH_CHUNK", 4);
  return c;
}

void drop_step_graphs(bte_ctx* ctx) {
  for (auto& g : ctx->step_graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  ctx->step_graphs.clear();
}

bool same_plan(const SweepPlan& a, const SweepPlan& b) {
  return a.kind == b.kind && a.ry == b.ry && a.rz == b.rz && a.ndg == b.ndg &&
         a.ntiles == b.ntiles && a.nparts == b.nparts;
}

// Enqueues iterations [j0, j0 + chunk) of a free-running step as one graph
// launch.  Which field an iteration reads and writes depends only on whether it
// is the step's first (it reads I^n) and on its parity, so with an even chunk
// every chunk after the first replays the same launches; the graphs are kept
// per arrangement of the three fields (the field that holds I^n changes from
// step to step), built on first use.  Surplus iterations after convergence
// return at once (device flag).
int enqueue_chunk(bte_ctx* ctx, int j0, int chunk) {
  const int first = j0 == 0;
  const double* shift = first ? ctx->first_shift : nullptr;
  ctx->first_shift = first ? ctx->first_shift : nullptr;
  for (const auto& g : ctx->step_graphs)
    if (g.In == ctx->In && g.Ia == ctx->Ia && g.Ib == ctx->Ib && g.shift == shift &&
        g.first == first && same_plan(g.plan, ctx->s.plan)) {
      HIP_TRY(hipGraphLaunch(g.exec, ctx->stream));
      return BTE_OK;
    }
  if ((int)ctx->step_graphs.size() >= kMaxStepGraphs) drop_step_graphs(ctx);
  bte_ctx::StepGraph g{ctx->In, ctx->Ia, ctx->Ib, shift, first, ctx->s.plan, nullptr, nullptr};
  HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  int rc = BTE_OK;
  const double* saved = ctx->first_shift;
  for (int jj = 0; jj < chunk && rc == BTE_OK; ++jj) {
    // iteration j0 + jj, with j0 = 0 or any even j0 >= 2
    const int j = first ? jj : 2 + jj;
    ctx->first_shift = shift;
    rc = enqueue_iteration(ctx, j, 0);
  }
  ctx->first_shift = saved;
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(ctx->stream, &graph);
  if (rc != BTE_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  HIP_TRY(e_end);
  g.graph = graph;
  const hipError_t e_inst = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (e_inst != hipSuccess) {
    (void)hipGraphDestroy(graph);
    HIP_TRY(e_inst);
  }
  ctx->step_graphs.push_back(g);
  HIP_TRY(hipGraphLaunch(g.exec, ctx->stream));
  return BTE_OK;
}

int one_step(bte_ctx* ctx, int fixed, bte_step_stats* st) {
  StepState ss;
  int rc = step_begin(ctx, fixed, &ss);
  if (rc != BTE_OK) return rc;
  HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
  const int chunk = graph_chunk() & ~1;
  if (ss.check && chunk > 0 && !ctx->opt.timing && ctx->stream != nullptr) {
    // Free-running: captured chunks of iterations, one chunk queued ahead of
    // the convergence test.
    for (int m = 0; m * chunk < ss.limit; ++m) {
      rc = enqueue_chunk(ctx, m * chunk, chunk);
      if (rc != BTE_OK) return rc;
      HIP_TRY(hipMemcpyAsync(&ctx->host_ring[m % kRing], ctx->ctl, sizeof(Control),
                             hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(hipEventRecord(ctx->ring_ev[m % kRing], ctx->stream));
      if (m >= 1) {
        HIP_TRY(hipEventSynchronize(ctx->ring_ev[(m - 1) % kRing]));
        if (ctx->host_ring[(m - 1) % kRing].converged) break;
      }
    }
  } else {
    for (int j = 0; j < ss.limit; ++j) {
      rc = enqueue_iteration(ctx, j, ss.check ? 0 : fixed);
      if (rc != BTE_OK) return rc;
      if (ss.check) {
        // Keep one iteration queued ahead of the convergence test so the device
        // never waits for the host; a surplus iteration is a no-op on the device.
        HIP_TRY(hipMemcpyAsync(&ctx->host_ring[j % kRing], ctx->ctl, sizeof(Control),
                               hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipEventRecord(ctx->ring_ev[j % kRing], ctx->stream));
        if (j >= 1) {
          HIP_TRY(hipEventSynchronize(ctx->ring_ev[(j - 1) % kRing]));
          if (ctx->host_ring[(j - 1) % kRing].converged) break;
        }
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(&ctx->host_ring[0], ctx->ctl, sizeof(Control), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const Control fin = ctx->host_ring[0];
  return step_finish(ctx, ss, fin, st);
}

// Steps whose sweep count the host knows beforehand (forward Euler: one; a
// replayed schedule: the given count) are queued back to back: the field
// swap at the end of each is known, so the host reads their control words
// only every kDeferSteps steps.  Contexts with a learned warm start step one
// at a time (the guess, the recording and the guard read device results).
bool steps_known(const bte_ctx* ctx, const int* fixed_inner, int nsteps) {
  if (ctx->s.warm || ctx->opt.timing) return false;
  if (ctx->opt.scheme == BTE_EXPLICIT_EULER) return true;
  if (!fixed_inner) return false;
  for (int i = 0; i < nsteps; ++i)
    if (fixed_inner[i] <= 0) return false;
  return true;
}

int run_known_steps(bte_ctx* ctx, int nsteps, const int* fixed_inner, bte_step_stats* stats) {
  StepState ss[kDeferSteps];
  for (int i0 = 0; i0 < nsteps; i0 += kDeferSteps) {
    const int n = std::min(kDeferSteps, nsteps - i0);
    for (int q = 0; q < n; ++q) {
      const int fixed = fixed_inner ? fixed_inner[i0 + q] : 0;
      int rc = step_begin(ctx, fixed, &ss[q]);
      if (rc != BTE_OK) return rc;
      HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
      for (int j = 0; j < ss[q].limit; ++j) {
        rc = enqueue_iteration(ctx, j, fixed);
        if (rc != BTE_OK) return rc;
      }
      HIP_TRY(hipMemcpyAsync(&ctx->host_steps[q], ctx->ctl, sizeof(Control),
                             hipMemcpyDeviceToHost, ctx->stream));
      void*& last = ((ss[q].limit - 1) & 1) ? ctx->Ib : ctx->Ia;
      std::swap(ctx->In, last);
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < n; ++q) {
      const int rc = step_finish(ctx, ss[q], ctx->host_steps[q],
                                 stats ? &stats[i0 + q] : nullptr, true);
      if (rc != BTE_OK) return rc;
    }
  }
  return BTE_OK;
}

}  // namespace

extern "C" {

int bte_workspace_size(const bte_mesh* mesh, const bte_dirs* dirs, const bte_bands* bands,
                       const bte_options* opt, size_t* bytes) {
  if (!bytes) return fail(BTE_E_INVAL, "bytes is null");
  Shape s;
  int rc = validate(mesh, dirs, bands, opt, &s);
  if (rc != BTE_OK) return rc;
  *bytes = make_layout(s).total;
  return BTE_OK;
}

int bte_create(const bte_mesh* mesh, const bte_dirs* dirs, const bte_bands* bands,
               const bte_dispersion* disp, const bte_options* opt, bte_ctx** out) {
  bte_ctx* ctx = nullptr;
  if (!out) return fail(BTE_E_INVAL, "out is null");
  *out = nullptr;
  Shape s;
  int rc = validate(mesh, dirs, bands, opt, &s);
  if (rc != BTE_OK) return rc;
  if (!disp || !disp->vg || !disp->tau || !disp->dos || !disp->deg)
    return fail(BTE_E_INVAL, "dispersion tables are required");
  const Layout L = make_layout(s);
  if (!opt->workspace) return fail(BTE_E_NOMEM, "no workspace given (need %zu bytes)", L.total);
  if (opt->workspace_bytes < L.total)
    return fail(BTE_E_NOMEM, "workspace has %zu bytes, need %zu", opt->workspace_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(opt->workspace) % kAlign)
    return fail(BTE_E_INVAL, "workspace must be %zu-byte aligned", kAlign);

  // ---- host-side tables
  const int nd = s.nd, nb = s.nb;
  bool tauT = false;
  for (int b = 0; b < nb; ++b) {
    const double vals[6] = {bands->omega[b], bands->domega[b], disp->vg[b], disp->tau[b],
                            disp->dos[b], disp->deg[b]};
    for (double v : vals)
      if (!(v > 0.0) || !std::isfinite(v))
        return fail(BTE_E_INVAL, "band %d: omega, domega, vg, tau, dos, deg must be positive", b);
    if (disp->tau_exp) {
      if (!std::isfinite(disp->tau_exp[b]))
        return fail(BTE_E_INVAL, "band %d: relaxation-time exponent must be finite", b);
      tauT |= disp->tau_exp[b] != 0.0;
    }
  }
  if (tauT && !(disp->tau_T0 <= 0.0 || std::isfinite(disp->tau_T0)))
    return fail(BTE_E_INVAL, "tau_T0 must be finite");
  for (int i = 0; i < nd; ++i)
    if (!(dirs->w[i] > 0.0) || !std::isfinite(dirs->w[i]))
      return fail(BTE_E_INVAL, "direction %d has a non-positive weight", i);
  for (int P = 0; P < s.nc; ++P)
    if (!(mesh->T_init[P] > 0.0) || !std::isfinite(mesh->T_init[P]))
      return fail(BTE_E_INVAL, "T_init[%d] must be positive", P);
  for (int f = 0; f < 6; ++f)
    if (s.iso[f])
      for (int i = 0; i < s.nf[f]; ++i)
        if (!(mesh->wall_T[f][i] > 0.0) || !std::isfinite(mesh->wall_T[f][i]))
          return fail(BTE_E_INVAL, "wall %d face %d temperature must be positive", f, i);

  std::vector<int> mirror;
  find_mirrors(dirs, s.dim, mirror);
  for (int f = 0; f < 2 * s.dim; ++f) {
    if (s.iso[f] || s.diff[f]) continue;
    const int a = f / 2;
    for (int i = 0; i < nd; ++i)
      if (mirror[(size_t)a * nd + i] < 0)
        return fail(BTE_E_INVAL,
                    "direction set is not closed under the mirror of wall %d (direction %d)", f, i);
  }
  double h[3] = {mesh->h[0], mesh->h[1], s.dim == 3 ? mesh->h[2] : 1.0};
  std::vector<Coef> coef((size_t)nb * nd);
  std::vector<int> dflags(nd, 0);
  std::vector<double> Cb(nb), xfac(nb), inv_tau(nb), fweight(nb);
  double W = 0.0;
  for (int i = 0; i < nd; ++i) {
    W += dirs->w[i];
    int fl = 0;
    for (int a = 0; a < s.dim; ++a) {
      const double c = dirs->s[3 * (size_t)i + a];
      if (c > 0.0) fl |= 1 << a;
      if (c < 0.0) fl |= 1 << (4 + a);
    }
    dflags[i] = fl;
  }
  // Forward Euler keeps every intensity a convex combination of old values
  // (positive, bounded) only if dt (1/tau_b + sum_a c_a) <= 1 everywhere.
  double max_rate = 0.0;
  int worst_b = 0, worst_d = 0;
  for (int b = 0; b < nb; ++b) {
    Cb[b] = disp->deg[b] * kHbar * bands->omega[b] * disp->dos[b] * bands->domega[b] / (4.0 * kPi);
    xfac[b] = kHbar * bands->omega[b] / kBoltzmann;
    inv_tau[b] = 1.0 / disp->tau[b];
    fweight[b] = opt->t_definition == BTE_T_TAU_WEIGHTED ? inv_tau[b] : 1.0;
    for (int i = 0; i < nd; ++i) {
      Coef& cf = coef[(size_t)b * nd + i];
      double diag = 1.0 / opt->dt + inv_tau[b];
      for (int a = 0; a < 3; ++a) {
        cf.c[a] = (a < s.dim) ? disp->vg[b] * std::fabs(dirs->s[3 * (size_t)i + a]) / h[a] : 0.0;
        diag += cf.c[a];
      }
      cf.scale = opt->scheme == BTE_EXPLICIT_EULER ? opt->dt : 1.0 / diag;
      cf.q = opt->scheme == BTE_EXPLICIT_EULER
                 ? 1.0 / opt->dt - (((inv_tau[b] + cf.c[0]) + cf.c[1]) + cf.c[2])
                 : 1.0 / opt->dt;
      const double rate = inv_tau[b] + cf.c[0] + cf.c[1] + cf.c[2];
      if (rate > max_rate) {
        max_rate = rate;
        worst_b = b;
        worst_d = i;
      }
    }
  }
  if (opt->scheme == BTE_EXPLICIT_EULER && opt->dt * max_rate > 1.0 + 1e-12)
    return fail(BTE_E_INVAL,
                "explicit step too large: dt (1/tau + sum v|s_a|/h_a) = %.6g > 1 for band %d, "
                "direction %d (largest stable dt %.6g s)",
                opt->dt * max_rate, worst_b, worst_d, 1.0 / max_rate);

  ctx = new (std::nothrow) bte_ctx();
  if (!ctx) return fail(BTE_E_NOMEM, "out of host memory");
  ctx->s = s;
  ctx->L = L;
  ctx->opt = *opt;
  if (ctx->opt.max_inner <= 0) ctx->opt.max_inner = 200;
  ctx->stream = static_cast<hipStream_t>(opt->stream);
  ctx->ws = static_cast<char*>(opt->workspace);
  ctx->poisoned = false;
  ctx->host_ring = nullptr;
  ctx->host_steps = nullptr;
  for (auto& e : ctx->ring_ev) e = nullptr;
  char* ws = ctx->ws;
  ctx->ctl = at<Control>(ws, L.ctl);
  ctx->T = at<double>(ws, L.T);
  ctx->Tprev = at<double>(ws, L.Tprev);
  ctx->E = at<double>(ws, L.E);
  ctx->I0 = at<double>(ws, L.I0);
  ctx->S = at<double>(ws, L.S);
  ctx->part = at<double>(ws, L.part);
  ctx->In = ws + L.In;
  ctx->Ia = ws + L.Ia;
  ctx->Ib = ws + L.Ib;
  ctx->timing_ms = 0.0;
  ctx->timing_count = 0;
  ctx->first_shift = nullptr;
  ctx->nn_shift = nullptr;
  ctx->nn_guess = nullptr;
  ctx->nn_nrec = 0;
  ctx->nn_ready = 0;
  ctx->nn_off = 0;
  ctx->nn_warm_steps = 0;
  ctx->nn_warm_sweeps = 0;
  ctx->nn_adam_t = 0;
  ctx->nnB = NnBuffers{};
  if (s.warm) {
    ctx->nnL = make_nn_layout(s.dim);
    NnBuffers& B = ctx->nnB;
    B.params = at<float>(ws, L.nn_params);
    B.grad = at<float>(ws, L.nn_grad);
    B.adam_m = at<float>(ws, L.nn_m);
    B.adam_v = at<float>(ws, L.nn_v);
    B.W1b = at<unsigned short>(ws, L.nn_W1b);
    B.W2b = at<unsigned short>(ws, L.nn_W2b);
    B.W2Tb = at<unsigned short>(ws, L.nn_W2Tb);
    B.y = at<float>(ws, L.nn_y);
    B.hist = at<float>(ws, L.nn_hist);
    B.loss = at<float>(ws, L.nn_loss);
    B.fallbacks = at<int>(ws, L.nn_fallbacks);
    B.scr = NnScratch{at<unsigned short>(ws, L.nn_XT), at<unsigned short>(ws, L.nn_H1T),
                      at<unsigned short>(ws, L.nn_dZ1T), at<unsigned short>(ws, L.nn_dZ2T),
                      at<float>(ws, L.nn_part), kNnBatch};
    ctx->nn_shift = at<double>(ws, L.nn_shift);
    ctx->nn_guess = at<double>(ws, L.nn_guess);
  }

  Geometry& g = ctx->g;
  g.dim = s.dim;
  g.nx = s.nx;
  g.ny = s.ny;
  g.nz = s.nz;
  g.nc = s.nc;
  g.ncp = s.ncp;
  g.px = s.px;
  g.nd = nd;
  g.nb = nb;
  g.ndg = s.plan.ndg;
  g.vol = h[0] * h[1] * h[2];
  Tables& t = ctx->t;
  t.coef = at<Coef>(ws, L.coef);
  t.dflags = at<int>(ws, L.dflags);
  t.mirror = at<int>(ws, L.mirror);
  t.w = at<double>(ws, L.w);
  t.Cb = at<double>(ws, L.Cb);
  t.xfac = at<double>(ws, L.xfac);
  t.inv_tau = at<double>(ws, L.inv_tau);
  t.fweight = at<double>(ws, L.fweight);
  t.Iref = at<double>(ws, L.Iref);
  t.tau_p = at<double>(ws, L.tau_p);
  t.relax = tauT ? at<double>(ws, L.relax) : nullptr;
  t.tau_T0 = disp->tau_T0 > 0.0 ? disp->tau_T0 : 300.0;
  t.tau_weighted = opt->t_definition == BTE_T_TAU_WEIGHTED;
  t.explicit_scheme = opt->scheme == BTE_EXPLICIT_EULER;
  t.W = W;
  for (int f = 0; f < 6; ++f) {
    // the sweeps read a diffuse wall's ghosts from its table, as an isothermal one's
    t.wall[f] = (f < 2 * s.dim) ? (s.diff[f] ? (int)BTE_WALL_ISOTHERMAL : mesh->wall[f])
                                : BTE_WALL_SPECULAR;
    t.wall_nf[f] = s.nf[f];
    const bool table = s.iso[f] || s.diff[f];
    t.wall_I0[f] = table ? at<double>(ws, L.wallI0[f]) : nullptr;
    t.wall_S[f] = table ? static_cast<const void*>(ws + L.wallS[f]) : nullptr;
  }
  ctx->dwt = at<double>(ws, L.dwt);
  ctx->any_diffuse = false;
  for (int f = 0; f < 6; ++f) ctx->any_diffuse |= s.diff[f];

  auto cleanup_fail = [&](int code) {
    bte_destroy(ctx);
    return code;
  };
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, ctx->stream);
  };
#define CREATE_TRY(expr)                                                               \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      fail(BTE_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
      return cleanup_fail(BTE_E_DEVICE);                                               \
    }                                                                                  \
  } while (0)
  CREATE_TRY(hipHostMalloc((void**)&ctx->host_ring, sizeof(Control) * kRing));
  CREATE_TRY(hipHostMalloc((void**)&ctx->host_steps, sizeof(Control) * kDeferSteps));
  for (auto& e : ctx->ring_ev) CREATE_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  CREATE_TRY(up(L.coef, coef.data(), sizeof(Coef) * coef.size()));
  CREATE_TRY(up(L.dflags, dflags.data(), sizeof(int) * dflags.size()));
  CREATE_TRY(up(L.mirror, mirror.data(), sizeof(int) * mirror.size()));
  CREATE_TRY(up(L.w, dirs->w, sizeof(double) * nd));
  CREATE_TRY(up(L.Cb, Cb.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.xfac, xfac.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.inv_tau, inv_tau.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.fweight, fweight.data(), sizeof(double) * nb));
  {
    std::vector<double> tau_p(nb, 0.0);
    if (disp->tau_exp) tau_p.assign(disp->tau_exp, disp->tau_exp + nb);
    CREATE_TRY(up(L.tau_p, tau_p.data(), sizeof(double) * nb));
    CREATE_TRY(hipStreamSynchronize(ctx->stream));  // the vector goes out of scope
  }
  {
    // per side: normalised outgoing-flux weights w_d (s_d . n) of the
    // directions leaving through it (zero for the others)
    std::vector<double> dwt(6 * (size_t)nd, 0.0);
    for (int f = 0; f < 2 * s.dim; ++f) {
      if (!s.diff[f]) continue;
      const double n_out = (f % 2) ? 1.0 : -1.0;
      double sum = 0.0;
      for (int i = 0; i < nd; ++i) {
        const double mu = dirs->s[3 * (size_t)i + f / 2] * n_out;
        if (mu > 0.0) {
          dwt[(size_t)f * nd + i] = dirs->w[i] * mu;
          sum += dwt[(size_t)f * nd + i];
        }
      }
      if (!(sum > 0.0)) {
        fail(BTE_E_INVAL, "no direction leaves through diffuse wall %d", f);
        return cleanup_fail(BTE_E_INVAL);
      }
      for (int i = 0; i < nd; ++i) dwt[(size_t)f * nd + i] /= sum;
    }
    CREATE_TRY(up(L.dwt, dwt.data(), sizeof(double) * dwt.size()));
    CREATE_TRY(hipStreamSynchronize(ctx->stream));  // the vector goes out of scope
  }
  CREATE_TRY(up(L.T, mesh->T_init, sizeof(double) * s.nc));
  for (int f = 0; f < 6; ++f) {
    if (!s.iso[f]) continue;
    CREATE_TRY(up(L.wallT[f], mesh->wall_T[f], sizeof(double) * s.nf[f]));
    CREATE_TRY(launch_wall_table(ctx->stream, nb, s.nf[f], t.Cb, t.xfac,
                                 at<double>(ws, L.wallT[f]), at<double>(ws, L.wallI0[f])));
  }
  // FP32 storage keeps I - I0_b(T_ref) with T_ref the coldest input temperature.
  double T_ref = 0.0;
  if (opt->precision == BTE_FP32_MIXED) {
    T_ref = mesh->T_init[0];
    for (int P = 1; P < s.nc; ++P) T_ref = std::min(T_ref, mesh->T_init[P]);
    for (int f = 0; f < 6; ++f)
      if (s.iso[f])
        for (int i = 0; i < s.nf[f]; ++i) T_ref = std::min(T_ref, mesh->wall_T[f][i]);
  }
  CREATE_TRY(launch_reference(ctx->stream, nb, t.Cb, t.xfac, T_ref, at<double>(ws, L.Iref)));
  for (int f = 0; f < 6; ++f) {
    if (!s.iso[f]) continue;
    if (opt->precision == BTE_FP64)
      CREATE_TRY(launch_wall_storage<double>(ctx->stream, nb, s.nf[f], t.wall_I0[f], t.Iref,
                                             at<double>(ws, L.wallS[f])));
    else
      CREATE_TRY(launch_wall_storage<float>(ctx->stream, nb, s.nf[f], t.wall_I0[f], t.Iref,
                                            at<float>(ws, L.wallS[f])));
  }
  ctx->Iref.assign(nb, 0.0);
  CREATE_TRY(hipMemcpyAsync(ctx->Iref.data(), at<double>(ws, L.Iref), sizeof(double) * nb,
                            hipMemcpyDeviceToHost, ctx->stream));
  CREATE_TRY(launch_reset(ctx->stream, ctx->ctl));
  CREATE_TRY(launch_equilibrium(ctx->stream, g, t, ctx->T, ctx->I0, ctx->E));
  CREATE_TRY(hipMemcpyAsync(ctx->Tprev, ctx->T, sizeof(double) * s.nc, hipMemcpyDeviceToDevice,
                            ctx->stream));
  if (opt->precision == BTE_FP64) {
    CREATE_TRY(launch_broadcast<double>(ctx->stream, g, t, ctx->I0, static_cast<double*>(ctx->In)));
    CREATE_TRY(launch_broadcast<double>(ctx->stream, g, t, ctx->I0, static_cast<double*>(ctx->Ia)));
    CREATE_TRY(launch_broadcast<double>(ctx->stream, g, t, ctx->I0, static_cast<double*>(ctx->Ib)));
  } else {
    CREATE_TRY(launch_broadcast<float>(ctx->stream, g, t, ctx->I0, static_cast<float*>(ctx->In)));
    CREATE_TRY(launch_broadcast<float>(ctx->stream, g, t, ctx->I0, static_cast<float*>(ctx->Ia)));
    CREATE_TRY(launch_broadcast<float>(ctx->stream, g, t, ctx->I0, static_cast<float*>(ctx->Ib)));
  }
  if (s.warm) {
    CREATE_TRY(nn_init(ctx->stream, ctx->nnL, ctx->nnB, opt->nn_seed));
    CREATE_TRY(hipMemsetAsync(ctx->nnB.fallbacks, 0, sizeof(int), ctx->stream));
    CREATE_TRY(hipMemsetAsync(ctx->nnB.loss, 0, sizeof(float), ctx->stream));
  }
  CREATE_TRY(hipStreamSynchronize(ctx->stream));
#undef CREATE_TRY
  *out = ctx;
  return BTE_OK;
}

int bte_step(bte_ctx* ctx, int nsteps, const int* fixed_inner, bte_step_stats* stats) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned by an earlier device error");
  if (nsteps < 0) return fail(BTE_E_INVAL, "nsteps must be >= 0");
  if (steps_known(ctx, fixed_inner, nsteps)) return run_known_steps(ctx, nsteps, fixed_inner, stats);
  for (int i = 0; i < nsteps; ++i) {
    const int fixed = fixed_inner ? fixed_inner[i] : 0;
    int rc = one_step(ctx, fixed, stats ? &stats[i] : nullptr);
    if (rc != BTE_OK) return rc;
  }
  return BTE_OK;
}

// Copies the intensity field between a dense [b][d][P] array of stored
// values and the device slabs (ncp cells apart; on 2D meshes with padded rows,
// rows of nx cells px apart, and ncp = px ny).
static hipError_t copy_intensity(void* dst, const void* src, const Shape& s, hipMemcpyKind kind,
                                 hipStream_t stream) {
  const size_t sz = s.real_size, slabs = (size_t)s.nb * s.nd;
  const bool rows = s.px != s.nx;
  const size_t width = rows ? (size_t)s.nx : (size_t)s.nc;
  const size_t pitch = rows ? (size_t)s.px : (size_t)s.ncp;
  const size_t height = rows ? slabs * s.ny : slabs;
  const bool to_device = kind == hipMemcpyHostToDevice;
  return hipMemcpy2DAsync(dst, sz * (to_device ? pitch : width), src,
                          sz * (to_device ? width : pitch), sz * width, height, kind, stream);
}

static int copy_cells(bte_ctx* ctx, const double* src, double* dst, size_t n) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!dst) return fail(BTE_E_INVAL, "null output");
  if (n != (size_t)ctx->s.nc) return fail(BTE_E_INVAL, "expected %d cells, got %zu", ctx->s.nc, n);
  HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

int bte_temperature(bte_ctx* ctx, double* T_out, size_t n_cells) {
  return copy_cells(ctx, ctx ? ctx->T : nullptr, T_out, n_cells);
}

int bte_energy(bte_ctx* ctx, double* E_out, size_t n_cells) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (ctx->opt.precision == BTE_FP64)
    HIP_TRY(launch_energy<double>(ctx->stream, ctx->g, ctx->t, static_cast<double*>(ctx->In), ctx->E));
  else
    HIP_TRY(launch_energy<float>(ctx->stream, ctx->g, ctx->t, static_cast<float*>(ctx->In), ctx->E));
  return copy_cells(ctx, ctx->E, E_out, n_cells);
}

int bte_intensity(bte_ctx* ctx, double* I_out, size_t n) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!I_out) return fail(BTE_E_INVAL, "null output");
  const size_t rows = (size_t)ctx->s.nb * ctx->s.nd;
  if (n != rows * ctx->s.nc)
    return fail(BTE_E_INVAL, "expected %zu intensities, got %zu", rows * ctx->s.nc, n);
  if (ctx->opt.precision == BTE_FP64) {
    HIP_TRY(copy_intensity(I_out, ctx->In, ctx->s, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  } else {
    std::vector<float> tmp;
    try {
      tmp.resize(n);
    } catch (...) {
      return fail(BTE_E_NOMEM, "out of host memory");
    }
    HIP_TRY(copy_intensity(tmp.data(), ctx->In, ctx->s, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const size_t nc = ctx->s.nc;
    for (size_t i = 0; i < n; ++i) I_out[i] = ctx->Iref[i / (nc * ctx->s.nd)] + (double)tmp[i];
  }
  return BTE_OK;
}

int bte_set_fields(bte_ctx* ctx, const double* I, size_t n, const double* T, size_t n_cells) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!I || !T) return fail(BTE_E_INVAL, "null state");
  const size_t rows = (size_t)ctx->s.nb * ctx->s.nd;
  if (n != rows * ctx->s.nc || n_cells != (size_t)ctx->s.nc)
    return fail(BTE_E_STATE, "state has the wrong size");
  for (size_t P = 0; P < n_cells; ++P)
    if (!(T[P] > 0.0) || !std::isfinite(T[P]))
      return fail(BTE_E_INVAL, "T[%zu] must be positive", P);
  if (ctx->opt.precision == BTE_FP64) {
    HIP_TRY(copy_intensity(ctx->In, I, ctx->s, hipMemcpyHostToDevice, ctx->stream));
  } else {
    std::vector<float> tmp;
    try {
      tmp.resize(n);
    } catch (...) {
      return fail(BTE_E_NOMEM, "out of host memory");
    }
    const size_t nc = ctx->s.nc;
    for (size_t i = 0; i < n; ++i)
      tmp[i] = static_cast<float>(I[i] - ctx->Iref[i / (nc * ctx->s.nd)]);
    HIP_TRY(copy_intensity(ctx->In, tmp.data(), ctx->s, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  HIP_TRY(hipMemcpyAsync(ctx->T, T, sizeof(double) * n_cells, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->Tprev, T, sizeof(double) * n_cells, hipMemcpyHostToDevice,
                         ctx->stream));
  HIP_TRY(launch_equilibrium(ctx->stream, ctx->g, ctx->t, ctx->T, ctx->I0, nullptr));
  // the energy density of the new intensity (the warm start's next input)
  if (ctx->opt.precision == BTE_FP64)
    HIP_TRY(launch_energy<double>(ctx->stream, ctx->g, ctx->t, static_cast<double*>(ctx->In),
                                  ctx->E));
  else
    HIP_TRY(launch_energy<float>(ctx->stream, ctx->g, ctx->t, static_cast<float*>(ctx->In),
                                 ctx->E));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

// ---------------------------------------------------------------- checkpoint
namespace {

enum StateSection {
  kSecI = 0, kSecT, kSecTprev, kSecE, kSecI0, kSecIref, kSecPlain, kSecParams, kSecM, kSecV,
  kSecHist, kStateSections
};
static_assert(kStateSections == 11, "bte_state_header.off has 11 sections");
constexpr char kStateMagic[8] = {'B', 'T', 'E', 'S', 'T', 'A', 'T', '1'};

// Header (shape, counters) and section offsets of this context's state.
bte_state_header state_header(const bte_ctx* ctx) {
  bte_state_header h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kStateMagic, 8);
  h.version = 1;
  h.header_bytes = (int)sizeof(bte_state_header);
  const Shape& s = ctx->s;
  h.dim = s.dim;
  h.n[0] = s.nx;
  h.n[1] = s.ny;
  h.n[2] = s.nz;
  h.nd = s.nd;
  h.nb = s.nb;
  h.precision = ctx->opt.precision;
  h.scheme = ctx->opt.scheme;
  h.warm_start = s.warm;
  h.nn_rec = s.warm ? s.nn_rec : 0;
  h.layout[0] = s.plan.kind;
  h.layout[1] = s.plan.ry;
  h.layout[2] = s.plan.rz;
  h.layout[3] = s.plan.ndg;
  h.steps = ctx->steps_taken;
  h.nn_recorded = ctx->nn_nrec;
  h.nn_trained = ctx->nn_ready;
  h.nn_off = ctx->nn_off;
  h.nn_warm_steps = ctx->nn_warm_steps;
  h.nn_warm_sweeps = ctx->nn_warm_sweeps;
  h.nn_adam_t = ctx->nn_adam_t;
  h.nn_last_batch = ctx->nn_last_batch;
  h.nn_params = s.warm ? ctx->nnL.total : 0;
  const size_t nc = s.nc;
  size_t off = align_up(sizeof(bte_state_header));
  auto take = [&](int sec, size_t bytes) {
    h.off[sec] = off;
    off = align_up(off + bytes);
  };
  take(kSecI, s.real_size * (size_t)s.nb * s.nd * nc);
  take(kSecT, sizeof(double) * nc);
  take(kSecTprev, sizeof(double) * nc);
  take(kSecE, sizeof(double) * nc);
  take(kSecI0, sizeof(double) * (size_t)s.nb * nc);
  take(kSecIref, sizeof(double) * (size_t)s.nb);
  if (s.warm) {
    const size_t P = (size_t)ctx->nnL.total;
    take(kSecPlain, sizeof(int) * (size_t)s.nn_rec);
    take(kSecParams, sizeof(float) * P);
    take(kSecM, sizeof(float) * P);
    take(kSecV, sizeof(float) * P);
    take(kSecHist, sizeof(float) * 4 * (size_t)s.nn_rec * nc);
  }
  h.total = off;
  return h;
}

}  // namespace

int bte_state_size(bte_ctx* ctx, size_t* bytes) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (!bytes) return fail(BTE_E_INVAL, "bytes is null");
  *bytes = (size_t)state_header(ctx).total;
  return BTE_OK;
}

int bte_get_state(bte_ctx* ctx, void* buf, size_t bytes) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!buf) return fail(BTE_E_INVAL, "null buffer");
  const bte_state_header h = state_header(ctx);
  if (bytes < h.total)
    return fail(BTE_E_STATE, "state needs %llu bytes, buffer has %zu", h.total, bytes);
  char* out = static_cast<char*>(buf);
  memcpy(out, &h, sizeof h);
  const Shape& s = ctx->s;
  const size_t nc = s.nc;
  auto d2h = [&](int sec, const void* src, size_t n) {
    return hipMemcpyAsync(out + h.off[sec], src, n, hipMemcpyDeviceToHost, ctx->stream);
  };
  HIP_TRY(copy_intensity(out + h.off[kSecI], ctx->In, s, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(d2h(kSecT, ctx->T, sizeof(double) * nc));
  HIP_TRY(d2h(kSecTprev, ctx->Tprev, sizeof(double) * nc));
  HIP_TRY(d2h(kSecE, ctx->E, sizeof(double) * nc));
  HIP_TRY(hipMemcpy2DAsync(out + h.off[kSecI0], sizeof(double) * nc, ctx->I0,
                           sizeof(double) * s.ncp, sizeof(double) * nc, (size_t)s.nb,
                           hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(d2h(kSecIref, ctx->t.Iref, sizeof(double) * s.nb));
  if (s.warm) {
    int* plain = reinterpret_cast<int*>(out + h.off[kSecPlain]);
    for (int i = 0; i < s.nn_rec; ++i)
      plain[i] = i < (int)ctx->nn_plain_sweeps.size() ? ctx->nn_plain_sweeps[i] : 0;
    const size_t P = (size_t)ctx->nnL.total;
    HIP_TRY(d2h(kSecParams, ctx->nnB.params, sizeof(float) * P));
    HIP_TRY(d2h(kSecM, ctx->nnB.adam_m, sizeof(float) * P));
    HIP_TRY(d2h(kSecV, ctx->nnB.adam_v, sizeof(float) * P));
    HIP_TRY(d2h(kSecHist, ctx->nnB.hist, sizeof(float) * 4 * (size_t)s.nn_rec * nc));
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

int bte_set_state(bte_ctx* ctx, const void* buf, size_t bytes) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!buf) return fail(BTE_E_INVAL, "null buffer");
  if (bytes < sizeof(bte_state_header)) return fail(BTE_E_STATE, "state is truncated");
  bte_state_header h;
  memcpy(&h, buf, sizeof h);
  const bte_state_header mine = state_header(ctx);
  if (memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 1 ||
      h.header_bytes != (int)sizeof(bte_state_header))
    return fail(BTE_E_STATE, "not a state written by bte_get_state (version 1)");
  if (h.dim != mine.dim || h.n[0] != mine.n[0] || h.n[1] != mine.n[1] || h.n[2] != mine.n[2] ||
      h.nd != mine.nd || h.nb != mine.nb)
    return fail(BTE_E_STATE, "state of a %dD %dx%dx%d mesh with %d directions and %d band "
                "entries, context has %dD %dx%dx%d, %d, %d", h.dim, h.n[0], h.n[1], h.n[2], h.nd,
                h.nb, mine.dim, mine.n[0], mine.n[1], mine.n[2], mine.nd, mine.nb);
  if (h.precision != mine.precision || h.scheme != mine.scheme ||
      h.warm_start != mine.warm_start || h.nn_rec != mine.nn_rec ||
      h.nn_params != mine.nn_params)
    return fail(BTE_E_STATE, "state has another precision, scheme, warm-start mode or "
                "recording length than the context");
  if (bytes < mine.total || h.total != mine.total)
    return fail(BTE_E_STATE, "state has %zu bytes, expected %llu", bytes, mine.total);
  for (int i = 0; i < kStateSections; ++i)
    if (h.off[i] != mine.off[i]) return fail(BTE_E_STATE, "state section %d is misplaced", i);
  const Shape& s = ctx->s;
  const char* in = static_cast<const char*>(buf);
  if (memcmp(in + h.off[kSecIref], ctx->Iref.data(), sizeof(double) * s.nb) != 0)
    return fail(BTE_E_STATE, "the state's storage reference differs from the context's "
                "(another coldest input temperature)");
  if (h.nn_recorded < 0 || h.nn_recorded > h.nn_rec || h.nn_adam_t < 0 || h.steps < 0)
    return fail(BTE_E_STATE, "state counters out of range");
  const size_t nc = s.nc;
  auto h2d = [&](void* dst, int sec, size_t n) {
    return hipMemcpyAsync(dst, in + h.off[sec], n, hipMemcpyHostToDevice, ctx->stream);
  };
  HIP_TRY(copy_intensity(ctx->In, in + h.off[kSecI], s, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(h2d(ctx->T, kSecT, sizeof(double) * nc));
  HIP_TRY(h2d(ctx->Tprev, kSecTprev, sizeof(double) * nc));
  HIP_TRY(h2d(ctx->E, kSecE, sizeof(double) * nc));
  HIP_TRY(hipMemcpy2DAsync(ctx->I0, sizeof(double) * s.ncp, in + h.off[kSecI0],
                           sizeof(double) * nc, sizeof(double) * nc, (size_t)s.nb,
                           hipMemcpyHostToDevice, ctx->stream));
  if (s.warm) {
    const size_t P = (size_t)ctx->nnL.total;
    HIP_TRY(h2d(ctx->nnB.params, kSecParams, sizeof(float) * P));
    HIP_TRY(h2d(ctx->nnB.adam_m, kSecM, sizeof(float) * P));
    HIP_TRY(h2d(ctx->nnB.adam_v, kSecV, sizeof(float) * P));
    HIP_TRY(h2d(ctx->nnB.hist, kSecHist, sizeof(float) * 4 * (size_t)s.nn_rec * nc));
    HIP_TRY(nn_refresh(ctx->stream, ctx->nnL, ctx->nnB));
  }
  // scattering rates at the restored temperatures (the formula of the
  // temperature inversion, so the same bits)
  if (ctx->t.relax) HIP_TRY(launch_equilibrium(ctx->stream, ctx->g, ctx->t, ctx->T, ctx->I0, nullptr));
  HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  // host-side counters, and the layout the saved context swept with if this
  // one can hold it (direction groups change the energy sum's grouping)
  ctx->steps_taken = h.steps;
  if (s.warm) {
    const int* plain = reinterpret_cast<const int*>(in + h.off[kSecPlain]);
    ctx->nn_plain_sweeps.assign(plain, plain + h.nn_recorded);
    ctx->nn_nrec = h.nn_recorded;
    ctx->nn_ready = h.nn_trained;
    ctx->nn_off = h.nn_off;
    ctx->nn_warm_steps = h.nn_warm_steps;
    ctx->nn_warm_sweeps = h.nn_warm_sweeps;
    ctx->nn_adam_t = h.nn_adam_t;
    ctx->nn_last_batch = h.nn_last_batch > 0 ? h.nn_last_batch : 1;
    ctx->nn_loss_pending = false;
  }
  auto family = [](int kind) { return kind == kSweepFlat3D ? (int)kSweepColumnWalk3D : kind; };
  if (family(h.layout[0]) == family(s.plan.kind) &&
      (h.layout[0] != s.plan.kind || h.layout[1] != s.plan.ry || h.layout[2] != s.plan.rz ||
       h.layout[3] != s.plan.ndg)) {
    const SweepPlan pl = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, h.layout[1],
                                         h.layout[2], h.layout[3], h.layout[0]);
    if (pl.kind == h.layout[0] && pl.ry == h.layout[1] && pl.rz == h.layout[2] &&
        pl.ndg == h.layout[3] && pl.ndg <= s.ndg_cap && pl.nparts <= s.nparts_cap) {
      ctx->s.plan = pl;
      ctx->g.ndg = pl.ndg;
    }
  }
  return BTE_OK;
}


static int nn_check(bte_ctx* ctx) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (!ctx->s.warm) return fail(BTE_E_INVAL, "the context was created without a warm start");
  return BTE_OK;
}

int bte_nn_param_count(bte_ctx* ctx, size_t* n) {
  int rc = nn_check(ctx);
  if (rc != BTE_OK) return rc;
  if (!n) return fail(BTE_E_INVAL, "null output");
  *n = (size_t)ctx->nnL.total;
  return BTE_OK;
}

int bte_nn_params(bte_ctx* ctx, float* out, size_t n) {
  int rc = nn_check(ctx);
  if (rc != BTE_OK) return rc;
  if (!out || n != (size_t)ctx->nnL.total)
    return fail(BTE_E_INVAL, "expected %d parameters", ctx->nnL.total);
  HIP_TRY(hipMemcpyAsync(out, ctx->nnB.params, sizeof(float) * n, hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

int bte_nn_set_params(bte_ctx* ctx, const float* in, size_t n) {
  int rc = nn_check(ctx);
  if (rc != BTE_OK) return rc;
  if (!in || n != (size_t)ctx->nnL.total)
    return fail(BTE_E_INVAL, "expected %d parameters", ctx->nnL.total);
  const float* nm = in + ctx->nnL.o_norm;
  if (!(nm[1] > 0.f) || !(nm[3] > 0.f) || !(nm[4] > 0.f))
    return fail(BTE_E_INVAL, "normalisation scales s_T, s_E, s_D must be positive");
  HIP_TRY(hipMemcpyAsync(ctx->nnB.params, in, sizeof(float) * n, hipMemcpyHostToDevice,
                         ctx->stream));
  HIP_TRY(nn_refresh(ctx->stream, ctx->nnL, ctx->nnB));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->nn_ready = 1;
  ctx->nn_off = 0;
  ctx->nn_warm_steps = 0;
  ctx->nn_warm_sweeps = 0;
  return BTE_OK;
}

int bte_nn_predict(bte_ctx* ctx, double* T_guess, size_t n_cells) {
  int rc = nn_check(ctx);
  if (rc != BTE_OK) return rc;
  if (!T_guess || n_cells != (size_t)ctx->s.nc)
    return fail(BTE_E_INVAL, "expected %d cells", ctx->s.nc);
  HIP_TRY(nn_predict(ctx->stream, ctx->g, ctx->nnL, ctx->nnB, ctx->T, ctx->Tprev, ctx->E));
  HIP_TRY(nn_guess_out(ctx->stream, ctx->s.nc, ctx->nnL, ctx->nnB, ctx->T, ctx->nn_guess));
  HIP_TRY(hipMemcpyAsync(T_guess, ctx->nn_guess, sizeof(double) * n_cells, hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

int bte_nn_gradient(bte_ctx* ctx, const double* T_n, const double* T_prev, const double* E_n,
                    const double* T_next, size_t n_cells, float* grad, size_t n, double* loss,
                    float* y_out) {
  int rc = nn_check(ctx);
  if (rc != BTE_OK) return rc;
  const int nc = ctx->s.nc;
  if (!T_n || !T_prev || !E_n || !T_next || !grad || n_cells != (size_t)nc ||
      n != (size_t)ctx->nnL.total)
    return fail(BTE_E_INVAL, "bad arguments (expected %d cells, %d parameters)", nc,
                ctx->nnL.total);
  if (nc > kNnBatch) return fail(BTE_E_INVAL, "at most %d cells", kNnBatch);
  std::vector<float> sample(4 * (size_t)nc);
  for (int P = 0; P < nc; ++P) {
    sample[P] = (float)T_n[P];
    sample[(size_t)nc + P] = (float)T_prev[P];
    sample[2 * (size_t)nc + P] = (float)E_n[P];
    sample[3 * (size_t)nc + P] = (float)T_next[P];
  }
  // the extra history slot after the recording slots
  NnBuffers B = ctx->nnB;
  B.hist = ctx->nnB.hist + (size_t)ctx->s.nn_rec * 4 * nc;
  HIP_TRY(hipMemcpyAsync(B.hist, sample.data(), sizeof(float) * sample.size(),
                         hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(nn_train_batch(ctx->stream, ctx->g, ctx->nnL, B, nc, 1, 0, 0, nc, 0.f, 1, false,
                         y_out ? B.y : nullptr));
  float l = 0.f;
  if (y_out)
    HIP_TRY(hipMemcpyAsync(y_out, B.y, sizeof(float) * nc, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipMemcpyAsync(grad, B.grad, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipMemcpyAsync(&l, B.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (loss) *loss = (double)l / (double)nc;
  return BTE_OK;
}

int bte_set_wall_temperature(bte_ctx* ctx, int side, const double* T_face, size_t n) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  if (side < 0 || side >= 2 * ctx->s.dim || !ctx->s.iso[side])
    return fail(BTE_E_INVAL, "side %d is not an isothermal wall", side);
  if (!T_face || n != (size_t)ctx->s.nf[side])
    return fail(BTE_E_INVAL, "side %d has %d faces, got %zu temperatures", side,
                ctx->s.nf[side], n);
  for (size_t i = 0; i < n; ++i)
    if (!(T_face[i] > 0.0) || !std::isfinite(T_face[i]))
      return fail(BTE_E_INVAL, "wall %d face %zu temperature must be positive", side, i);
  const Layout& L = ctx->L;
  double* wT = at<double>(ctx->ws, L.wallT[side]);
  double* w0 = at<double>(ctx->ws, L.wallI0[side]);
  HIP_TRY(hipMemcpyAsync(wT, T_face, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(launch_wall_table(ctx->stream, ctx->s.nb, (int)n, ctx->t.Cb, ctx->t.xfac, wT, w0));
  if (ctx->opt.precision == BTE_FP64)
    HIP_TRY(launch_wall_storage<double>(ctx->stream, ctx->s.nb, (int)n, w0, ctx->t.Iref,
                                        at<double>(ctx->ws, L.wallS[side])));
  else
    HIP_TRY(launch_wall_storage<float>(ctx->stream, ctx->s.nb, (int)n, w0, ctx->t.Iref,
                                       at<float>(ctx->ws, L.wallS[side])));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BTE_OK;
}

int bte_sweep_time(bte_ctx* ctx, double* total_ms, int* count) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (total_ms) *total_ms = ctx->timing_ms;
  if (count) *count = ctx->timing_count;
  ctx->timing_ms = 0.0;
  ctx->timing_count = 0;
  return BTE_OK;
}

int bte_sweep_layout(bte_ctx* ctx, int* kind, int* ry, int* rz, int* ndg) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  const SweepPlan& pl = ctx->s.plan;
  if (kind) *kind = pl.kind;
  if (ry) *ry = pl.ry;
  if (rz) *rz = pl.rz;
  if (ndg) *ndg = pl.ndg;
  return BTE_OK;
}

int bte_destroy(bte_ctx* ctx) {
  if (!ctx) return BTE_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto e : ctx->t_start) (void)hipEventDestroy(e);
  for (auto e : ctx->t_stop) (void)hipEventDestroy(e);
  if (ctx->host_ring) (void)hipHostFree(ctx->host_ring);
  if (ctx->host_steps) (void)hipHostFree(ctx->host_steps);
  drop_step_graphs(ctx);
  delete ctx;
  return BTE_OK;
}

const char* bte_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------- autotuner
static std::string tune_key(const bte_ctx* ctx) {
  char buf[160];
  snprintf(buf, sizeof buf, "sweep dim=%d n=%dx%dx%d dirs=%d bands=%d prec=%d", ctx->s.dim,
           ctx->s.nx, ctx->s.ny, ctx->s.nz, ctx->s.nd, ctx->s.nb, ctx->opt.precision);
  return buf;
}

static void apply_plan(bte_ctx* ctx, const SweepPlan& pl) {
  ctx->s.plan = pl;
  ctx->g.ndg = pl.ndg;
}

int bte_autotune(bte_ctx* ctx, const char* cache_path, int* ry_out, int* rz_out, int* ndg_out,
                 double* ms_out) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned");
  const int kind = ctx->s.plan.kind;
  const bool family3d = kind == kSweepColumnWalk3D || kind == kSweepFlat3D;
  // candidate (rows, planes) per wave and direction-group counts of this kernel
  // family; in 3D, 0 rows stands for the flattened (x, y) plane
  std::vector<std::pair<int, int>> shapes;
  std::vector<int> groups;
  if (kind == kSweepColumnWalk2D) {
    shapes = {{4, 1}, {8, 1}};
    groups = {1, 2, 4, 8, 16};
  } else if (family3d) {
    shapes = {{2, 2}, {1, 4}, {2, 4}, {0, 4}, {0, 2}};
    groups = {1, 2, 4};
  }
  auto kind_of = [&](int ry) {
    return family3d ? (ry == 0 ? kSweepFlat3D : kSweepColumnWalk3D) : kind;
  };
  const int ry_only = ry_out ? *ry_out : 0;
  const int rz_only = rz_out ? *rz_out : 0;
  // In a batch the geometries fill the device together, and a geometry timed
  // alone is a poor guide: it favours layouts that spread a small sweep over
  // more workgroups (more direction groups, 2 planes per wave instead of 4),
  // which in a batch only cost bytes (energy partials for the temperature
  // kernel to read back, tile faces).  A batch tune therefore takes one
  // direction group, 4 rows in 2D, and in 3D the family that create picks by
  // idle lanes (the flattened plane where 64-column tiles would leave more
  // than an eighth of the lanes idle, else the column walk) with 4 planes
  // per wave.  Measured on the 64-geometry draw, 4 steps: 3.49 s with the
  // layouts that time fastest alone, 3.31 s timing the two 4-plane families
  // at one group, 3.19-3.22 s with this choice.
  if (ry_only == -1) {
    groups = {1};
    if (family3d)
      shapes = {flat_by_lanes(ctx->s.nx) ? std::make_pair(0, 4) : std::make_pair(1, 4)};
  }
  auto listed_groups = [&](int ndg) {
    return std::find(groups.begin(), groups.end(), ndg) != groups.end();
  };
  auto allowed = [&](int ry, int rz) {
    bool listed = false;
    for (const auto& sh : shapes) listed |= (sh.first == ry && sh.second == rz);
    if (ry_only == -1) return listed && batch_layout(kind_of(ry), ry, rz);
    return listed && (ry_only <= 0 || ry == ry_only) && (rz_only <= 0 || rz == rz_only);
  };
  auto plan_for = [&](int ry, int rz, int ndg) {
    return make_sweep_plan(ctx->s.dim, ctx->s.nx, ctx->s.ny, ctx->s.nz, ctx->s.nd, ctx->s.nb, ry,
                           rz, ndg, kind_of(ry));
  };
  auto fits = [&](const SweepPlan& pl) {
    return pl.ndg <= ctx->s.ndg_cap && pl.nparts <= ctx->s.nparts_cap;
  };
  const std::string key = tune_key(ctx) + (ry_only == -1 ? " batch" : "");
  SweepPlan best = ctx->s.plan;
  double best_ms = -1.0;
  bool found = shapes.empty();  // a single-layout family needs no search
  if (!found && cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[256];
      while (fgets(line, sizeof line, f)) {
        const char* sep = strstr(line, " -> ");
        if (!sep || std::string(line, sep - line) != key) continue;
        int ry = 0, rz = 0, ndg = 0;
        double ms = 0.0;
        if (sscanf(sep + 4, "ry=%d rz=%d ndg=%d ms=%lf", &ry, &rz, &ndg, &ms) == 4 &&
            allowed(ry, rz) && listed_groups(ndg)) {
          const SweepPlan pl = plan_for(ry, rz, ndg);
          if (fits(pl)) {
            best = pl;
            best_ms = ms;
            found = true;
          }
        }
      }
      fclose(f);
    }
  }
  if (!found) {
    // Time every candidate layout on this context's own state: the sweeps read
    // one ping-pong iterate and I^n and write the other iterate and the
    // partials, so the state is untouched.  The iterate read must not be I^n
    // itself, or half of the reads would hit in cache and flatter every layout.
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (const auto& sh : shapes) {
      if (!allowed(sh.first, sh.second)) continue;
      for (int nd_try : groups) {
        const SweepPlan pl = plan_for(sh.first, sh.second, nd_try);
        if (pl.ndg != nd_try || !fits(pl)) continue;
        apply_plan(ctx, pl);
        HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
        ctx->first_shift = nullptr;
        int rc = BTE_OK;
        for (int r = 0; r < 4 && rc == BTE_OK; ++r) {
          if (r == 1) HIP_TRY(hipEventRecord(e0, ctx->stream));  // first launch warms up
          rc = ctx->opt.precision == BTE_FP64
                   ? enqueue_sweep<double>(ctx, ctx->Ib, ctx->Ia, nullptr)
                   : enqueue_sweep<float>(ctx, ctx->Ib, ctx->Ia, nullptr);
        }
        if (rc != BTE_OK) return rc;
        HIP_TRY(hipEventRecord(e1, ctx->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms /= 3.f;
        if (best_ms < 0.0 || ms < best_ms) {
          best_ms = ms;
          best = pl;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_ms < 0.0) return fail(BTE_E_INVAL, "no layout matches the requested rows/planes");
    if (cache_path) {
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "%s -> ry=%d rz=%d ndg=%d ms=%.6f\n", key.c_str(), best.ry, best.rz, best.ndg,
                best_ms);
        fclose(f);
      }
    }
  }
  apply_plan(ctx, best);
  HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ry_out) *ry_out = best.ry;
  if (rz_out) *rz_out = best.rz;
  if (ndg_out) *ndg_out = best.ndg;
  if (ms_out) *ms_out = best_ms;
  return BTE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
struct bte_batch {
  std::vector<bte_ctx*> ctx;
  hipStream_t stream;
  int precision;
  BatchCtx* d_ctx;
  BatchCtx* h_ctx;  // pinned staging
  BatchItem* d_items;
  int counts[kBatchLists];  // items per work list, stored back to back
  BatchControl* d_bc;
  BatchControl* h_bc;  // pinned
  Control* h_ctl;      // pinned, one per geometry
  int sweep_blocks[kBatchLists];
  // trainings of several geometries run together: jobs and per-iteration
  // minibatches in device memory (grown on demand)
  NnTrainJob* d_jobs;
  NnTrainStep* d_steps;
  size_t jobs_cap, steps_cap;
  int temp_blocks;
  int max_inner;
  bool use_graph;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t ev[kRing];
  // each context's sweep layout when the work lists were built: the lists,
  // tile counts and partial indices hold only for these
  std::vector<SweepPlan> plans;
};

namespace {

// The device descriptor of one geometry for the next step of a batch.
void fill_batch_ctx(BatchCtx& d, const bte_ctx* ctx, int cell_block0) {
  memset(&d, 0, sizeof d);
  d.sp64.g = ctx->g;
  d.sp64.t = ctx->t;
  d.sp64.In = static_cast<const double*>(ctx->In);
  d.sp64.I0 = ctx->I0;
  d.sp64.S = ctx->S;
  d.sp64.part = ctx->part;
  d.sp64.ctl = ctx->ctl;
  d.sp64.inv_dt = 1.0 / ctx->opt.dt;
  d.sp64.shift = nullptr;
  d.sp32.g = ctx->g;
  d.sp32.t = ctx->t;
  d.sp32.In = static_cast<const float*>(ctx->In);
  d.sp32.I0 = ctx->I0;
  d.sp32.S = ctx->S;
  d.sp32.part = ctx->part;
  d.sp32.ctl = ctx->ctl;
  d.sp32.inv_dt = 1.0 / ctx->opt.dt;
  d.sp32.shift = nullptr;
  d.plan = ctx->s.plan;
  d.precision = ctx->opt.precision;
  d.in_idx = 0;
  d.F[0] = ctx->In;
  d.F[1] = ctx->Ia;
  d.F[2] = ctx->Ib;
  d.I0 = ctx->I0;
  d.S = ctx->S;
  d.part = ctx->part;
  d.T = ctx->T;
  d.E = ctx->E;
  d.ctl = ctx->ctl;
  d.tol = ctx->opt.tol;
  d.max_inner = ctx->opt.max_inner;
  d.fixed_k = 0;
  d.cell_block0 = cell_block0;
  d.cell_blocks =
      (ctx->s.nc + temp_cells_per_block(ctx->s.nb) - 1) / temp_cells_per_block(ctx->s.nb);
}

// The checks every batch applies to its contexts.
int check_batch_members(int n, bte_ctx* const* ctxs) {
  for (int i = 0; i < n; ++i) {
    const bte_ctx* c = ctxs[i];
    if (!c || c->poisoned) return fail(BTE_E_INVAL, "context %d is null or poisoned", i);
    if (c->stream != ctxs[0]->stream) return fail(BTE_E_INVAL, "contexts must share one stream");
    if (c->opt.precision != ctxs[0]->opt.precision)
      return fail(BTE_E_INVAL, "contexts must share one precision");
    if (c->opt.scheme != BTE_IMPLICIT_JACOBI)
      return fail(BTE_E_INVAL, "batches run the implicit scheme");
    if (c->s.warm == BTE_WARM_T_SHIFT)
      return fail(BTE_E_INVAL, "batches seed warm starts through the temperature only");
    const SweepPlan& pl = c->s.plan;
    if (!batch_layout(pl.kind, pl.ry, pl.rz))
      return fail(BTE_E_INVAL,
                  "batches need the 4-row 2D, the 2x2 or 1x4 3D column-walk or the "
                  "flattened-plane layout (context %d)", i);
    if (c->opt.timing) return fail(BTE_E_INVAL, "per-sweep timing is not available in batches");
    if (c->any_diffuse)
      return fail(BTE_E_INVAL, "batches take isothermal, specular and symmetry walls "
                  "(context %d has a diffuse wall)", i);
    if (c->t.relax)
      return fail(BTE_E_INVAL,
                  "batches take constant relaxation times (context %d has a temperature law)", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(BTE_E_INVAL, "context %d appears twice", i);
  }
  return BTE_OK;
}

// Which work list a context's layout belongs to.
int batch_list_of(const SweepPlan& pl) {
  if (pl.kind == kSweepColumnWalk2D) return kList2D;
  if (pl.kind == kSweepFlat3D && pl.rz == 4) return kListFlat4;
  return kList3D;
}

int batch_fail_free(bte_batch* b, int code) {
  bte_batch_destroy(b);
  return code;
}

// One iteration of every geometry, as eager launches or as the captured graph.
int batch_enqueue_iteration(bte_batch* b) {
  bte_ctx* ctx = nullptr;
  if (b->use_graph) {
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  } else {
    HIP_TRY(launch_batch_iteration(b->stream, b->precision, b->d_ctx, (int)b->ctx.size(),
                                   b->d_items, b->counts, b->d_bc, b->sweep_blocks,
                                   b->temp_blocks));
    HIP_TRY(hipMemcpyAsync(b->h_bc, b->d_bc, sizeof(BatchControl), hipMemcpyDeviceToHost,
                           b->stream));
  }
  return BTE_OK;
}

}  // namespace

extern "C" {

int bte_batch_create(int n, bte_ctx* const* ctxs, int use_graph, bte_batch** out) {
  bte_ctx* ctx = nullptr;
  if (!out || n < 1 || !ctxs) return fail(BTE_E_INVAL, "need at least one context");
  *out = nullptr;
  {
    const int rc = check_batch_members(n, ctxs);
    if (rc != BTE_OK) return rc;
  }
  bte_batch* b = new (std::nothrow) bte_batch();
  if (!b) return fail(BTE_E_NOMEM, "out of host memory");
  b->ctx.assign(ctxs, ctxs + n);
  for (int i = 0; i < n; ++i) b->plans.push_back(ctxs[i]->s.plan);
  b->stream = ctxs[0]->stream;
  b->precision = ctxs[0]->opt.precision;
  b->use_graph = use_graph != 0 && b->stream != nullptr;
  b->graph = nullptr;
  b->exec = nullptr;
  for (auto& e : b->ev) e = nullptr;
  b->d_jobs = nullptr;
  b->d_steps = nullptr;
  b->jobs_cap = b->steps_cap = 0;
  b->max_inner = 0;
  // work lists (2D; 3D; 3D flattened plane with 4 planes), each ordered
  // largest geometry first
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    const double wa = (double)ctxs[a]->s.nc * ctxs[a]->s.nd * ctxs[a]->s.nb;
    const double wc = (double)ctxs[c]->s.nc * ctxs[c]->s.nd * ctxs[c]->s.nb;
    return wa > wc;
  });
  std::vector<BatchItem> lists[kBatchLists];
  for (int i : order) {
    const SweepPlan& pl = ctxs[i]->s.plan;
    auto& dst = lists[batch_list_of(pl)];
    const int nz = pl.ndg;  // direction groups
    for (int bz = 0; bz < nz; ++bz)
      for (int by = 0; by < ctxs[i]->s.nb; ++by)
        for (int bx = 0; bx < pl.ntiles; ++bx) dst.push_back(BatchItem{i, bx, by, bz});
    b->max_inner = std::max(b->max_inner, ctxs[i]->opt.max_inner);
  }
  std::vector<BatchItem> items;
  for (int l = 0; l < kBatchLists; ++l) {
    b->counts[l] = (int)lists[l].size();
    items.insert(items.end(), lists[l].begin(), lists[l].end());
  }
  int cus = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  for (int l = 0; l < kBatchLists; ++l)
    b->sweep_blocks[l] = cus * batch_sweep_occupancy(b->precision, l);
  int blocks = 0;
  for (int i = 0; i < n; ++i)
    blocks += (ctxs[i]->s.nc + temp_cells_per_block(ctxs[i]->s.nb) - 1) /
              temp_cells_per_block(ctxs[i]->s.nb);
  b->temp_blocks = blocks;
#define BATCH_TRY(expr)                                                               \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      fail(BTE_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));             \
      return batch_fail_free(b, BTE_E_DEVICE);                                        \
    }                                                                                 \
  } while (0)
  b->d_ctx = nullptr;
  b->h_ctx = nullptr;
  b->d_items = nullptr;
  b->d_bc = nullptr;
  b->h_bc = nullptr;
  b->h_ctl = nullptr;
  BATCH_TRY(hipMalloc((void**)&b->d_ctx, sizeof(BatchCtx) * n));
  BATCH_TRY(hipHostMalloc((void**)&b->h_ctx, sizeof(BatchCtx) * n));
  BATCH_TRY(hipMalloc((void**)&b->d_items, sizeof(BatchItem) * std::max<size_t>(1, items.size())));
  BATCH_TRY(hipMalloc((void**)&b->d_bc, sizeof(BatchControl)));
  BATCH_TRY(hipHostMalloc((void**)&b->h_bc, sizeof(BatchControl)));
  BATCH_TRY(hipHostMalloc((void**)&b->h_ctl, sizeof(Control) * n));
  for (auto& e : b->ev) BATCH_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (!items.empty())
    BATCH_TRY(hipMemcpyAsync(b->d_items, items.data(), sizeof(BatchItem) * items.size(),
                             hipMemcpyHostToDevice, b->stream));
  BATCH_TRY(hipStreamSynchronize(b->stream));
  if (b->use_graph) {
    BATCH_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e1 = launch_batch_iteration(b->stream, b->precision, b->d_ctx, n, b->d_items,
                                                 b->counts, b->d_bc, b->sweep_blocks,
                                                 b->temp_blocks);
    const hipError_t e2 = hipMemcpyAsync(b->h_bc, b->d_bc, sizeof(BatchControl),
                                         hipMemcpyDeviceToHost, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e3 = hipStreamEndCapture(b->stream, &g);
    b->graph = g;
    BATCH_TRY(e1);
    BATCH_TRY(e2);
    BATCH_TRY(e3);
    BATCH_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
#undef BATCH_TRY
  *out = b;
  (void)ctx;
  return BTE_OK;
}

// Trains the networks of the queued geometries together: normalisation
// constants of each, then one launch per kernel and iteration for all of
// them, each following its own minibatch schedule.
static int batch_train(bte_batch* b, const std::vector<bte_ctx*>& due) {
  bte_ctx* ctx = due.front();
  const int nj = (int)due.size();
  std::vector<TrainSchedule> ts(nj);
  std::vector<NnTrainJob> jobs(nj);
  size_t niters = 0;
  int max_kp = 0;
  for (int j = 0; j < nj; ++j) {
    bte_ctx* c = due[j];
    HIP_TRY(nn_stats(b->stream, c->nnL, c->nnB, c->nn_nrec, c->s.nc));
    ts[j] = nn_schedule(c);
    jobs[j] = NnTrainJob{c->g, c->nnL, c->nnB, ts[j].N, ts[j].a, ts[j].lr};
    niters = std::max(niters, ts[j].updates.size());
    max_kp = std::max(max_kp, c->nnL.KP);
  }
  std::vector<NnTrainStep> steps(niters * nj, NnTrainStep{0, 0, 0, 0, 1.f, 1.f});
  for (int j = 0; j < nj; ++j)
    for (size_t it = 0; it < ts[j].updates.size(); ++it) {
      const auto& u = ts[j].updates[it];
      const int t = due[j]->nn_adam_t + (int)it + 1;  // Adam step number of this update
      steps[it * nj + j] = NnTrainStep{u.b0, u.c, u.batch, 1, 1.f - powf(0.9f, (float)t),
                                       1.f - powf(0.999f, (float)t)};
    }
  if (jobs.size() > b->jobs_cap) {
    if (b->d_jobs) HIP_TRY(hipFree(b->d_jobs));
    b->d_jobs = nullptr;
    HIP_TRY(hipMalloc((void**)&b->d_jobs, sizeof(NnTrainJob) * jobs.size()));
    b->jobs_cap = jobs.size();
  }
  if (steps.size() > b->steps_cap) {
    if (b->d_steps) HIP_TRY(hipFree(b->d_steps));
    b->d_steps = nullptr;
    HIP_TRY(hipMalloc((void**)&b->d_steps, sizeof(NnTrainStep) * steps.size()));
    b->steps_cap = steps.size();
  }
  HIP_TRY(hipMemcpyAsync(b->d_jobs, jobs.data(), sizeof(NnTrainJob) * jobs.size(),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_steps, steps.data(), sizeof(NnTrainStep) * steps.size(),
                         hipMemcpyHostToDevice, b->stream));
  for (size_t it = 0; it < niters; ++it)
    HIP_TRY(nn_train_many(b->stream, b->d_jobs, b->d_steps, nj, (int)it, max_kp));
  // the host vectors are read by the copies above: wait before they go
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int j = 0; j < nj; ++j) {
    bte_ctx* c = due[j];
    c->nn_adam_t += (int)ts[j].updates.size();
    c->nn_last_batch = ts[j].updates.back().batch;
    c->nn_ready = 1;
    c->nn_loss_pending = true;
  }
  (void)ctx;
  return BTE_OK;
}

int bte_batch_step(bte_batch* b, int nsteps, bte_step_stats* stats) {
  bte_ctx* ctx = nullptr;
  if (!b) return fail(BTE_E_INVAL, "null batch");
  if (nsteps < 0) return fail(BTE_E_INVAL, "nsteps must be >= 0");
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i) {
    const SweepPlan& p = b->ctx[i]->s.plan;
    const SweepPlan& q = b->plans[i];
    if (p.kind != q.kind || p.ry != q.ry || p.rz != q.rz || p.ndg != q.ndg ||
        p.ntiles != q.ntiles || p.nparts != q.nparts)
      return fail(BTE_E_INVAL,
                  "context %d changed its sweep layout after joining the batch (the batch's "
                  "work lists are built for the old one): create the batch again", i);
  }
  std::vector<StepState> ss(n);
  for (int step = 0; step < nsteps; ++step) {
    for (int i = 0; i < n; ++i) {
      ctx = b->ctx[i];
      if (ctx->poisoned) return fail(BTE_E_DEVICE, "context %d is poisoned", i);
      int rc = step_begin(ctx, 0, &ss[i]);
      if (rc != BTE_OK) return rc;
      fill_batch_ctx(b->h_ctx[i], ctx,
                     (i == 0) ? 0 : b->h_ctx[i - 1].cell_block0 + b->h_ctx[i - 1].cell_blocks);
    }
    ctx = nullptr;
    HIP_TRY(hipMemcpyAsync(b->d_ctx, b->h_ctx, sizeof(BatchCtx) * n, hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(launch_batch_reset(b->stream, b->d_ctx, n, b->d_bc));
    for (int j = 0; j < b->max_inner; ++j) {
      int rc = batch_enqueue_iteration(b);
      if (rc != BTE_OK) return rc;
      HIP_TRY(hipEventRecord(b->ev[j % kRing], b->stream));
      if (j >= 1) {
        // the device runs one iteration ahead; the active count only falls
        HIP_TRY(hipEventSynchronize(b->ev[(j - 1) % kRing]));
        if (b->h_bc->active == 0) break;
      }
    }
    for (int i = 0; i < n; ++i)
      HIP_TRY(hipMemcpyAsync(&b->h_ctl[i], b->ctx[i]->ctl, sizeof(Control), hipMemcpyDeviceToHost,
                             b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    // The geometries whose training falls due in this step are queued and
    // trained together (each on its own samples, in its own order, so the
    // results are those of training it alone).
    std::vector<bte_ctx*> due;
    for (int i = 0; i < n; ++i) b->ctx[i]->train_queue = &due;
    int rc = BTE_OK;
    for (int i = 0; i < n && rc == BTE_OK; ++i) {
      const Control fin = b->h_ctl[i];
      rc = step_finish(b->ctx[i], ss[i], fin, stats ? &stats[(size_t)step * n + i] : nullptr);
    }
    for (int i = 0; i < n; ++i) b->ctx[i]->train_queue = nullptr;
    if (rc != BTE_OK) return rc;
    if (!due.empty()) {
      rc = batch_train(b, due);
      if (rc != BTE_OK) return rc;
    }
    for (int i = 0; i < n; ++i)
      if (b->ctx[i]->nn_loss_pending) {
        double loss = 0.0;
        const int lrc = nn_read_loss(b->ctx[i], &loss);
        if (lrc != BTE_OK) return lrc;
        if (stats) stats[(size_t)step * n + i].nn_loss = loss;
      }
  }
  return BTE_OK;
}

int bte_batch_destroy(bte_batch* b) {
  if (!b) return BTE_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_steps) (void)hipFree(b->d_steps);
  if (b->d_ctx) (void)hipFree(b->d_ctx);
  if (b->h_ctx) (void)hipHostFree(b->h_ctx);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_bc) (void)hipFree(b->d_bc);
  if (b->h_bc) (void)hipHostFree(b->h_bc);
  if (b->h_ctl) (void)hipHostFree(b->h_ctl);
  delete b;
  return BTE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batch step that allocates nothing
// For callers that cannot allocate (graph capture, tight serving loops):
// bte_batch_step_static runs the batched step of bte_batch_step without a
// batch object.  The geometry descriptors, the work lists (kept as per-
// geometry item ranges, decoded by the persistent sweeps) and the counters
// live in the file-scope device array `scratch`, one copy per GPU; the host
// side stages them in a file-scope host block under a mutex.  No graph is
// captured (instantiating one allocates).
namespace {

constexpr int kStaticBatchMax = 256;  // contexts per call

struct StaticBatch {
  BatchCtx ctx[kStaticBatchMax];
  BatchControl bc;
  int list_ctx[kBatchLists][kStaticBatchMax];
  int list_start[kBatchLists][kStaticBatchMax + 1];
};

// host staging: descriptors and lists on the way in, control words on the way out
struct StaticBatchHost {
  StaticBatch dev;  // mirror of the device block
  Control ctl[kStaticBatchMax];
  StepState ss[kStaticBatchMax];
  int order[kStaticBatchMax];
};

}  // namespace

static __device__ __align__(256) char scratch[sizeof(StaticBatch)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;                       // guards the host staging and the table below
StaticBatchHost g_static_host;                // file-scope: nothing allocated per call
StaticBatch* g_static_dev[kMaxDevices] = {};  // device address of `scratch` on each GPU

// The device address of `scratch` on the current GPU (looked up once per
// GPU; the array's name is not a device address in host code).  Called with
// g_static_mu held.
int static_scratch(StaticBatch** out) {
  int dev = 0;
  bte_ctx* ctx = nullptr;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BTE_E_DEVICE, "device %d out of range", dev);
  if (!g_static_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_static_dev[dev] = static_cast<StaticBatch*>(p);
  }
  *out = g_static_dev[dev];
  return BTE_OK;
}

}  // namespace

extern "C" {

int bte_batch_step_static(int n, bte_ctx* const* ctxs, int nsteps, bte_step_stats* stats) {
  bte_ctx* ctx = nullptr;
  if (n < 1 || !ctxs) return fail(BTE_E_INVAL, "need at least one context");
  if (n > kStaticBatchMax)
    return fail(BTE_E_INVAL, "at most %d contexts per call (got %d)", kStaticBatchMax, n);
  if (nsteps < 0) return fail(BTE_E_INVAL, "nsteps must be >= 0");
  {
    const int rc = check_batch_members(n, ctxs);
    if (rc != BTE_OK) return rc;
  }
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->s.warm && !ctxs[i]->nn_ready)
      return fail(BTE_E_INVAL,
                  "context %d would record and train its warm-start network in these steps "
                  "(training allocates): step it with bte_batch_step or alone until trained", i);
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticBatch* d = nullptr;
  {
    const int rc = static_scratch(&d);
    if (rc != BTE_OK) return rc;
  }
  StaticBatchHost& H = g_static_host;
  const hipStream_t stream = ctxs[0]->stream;
  const int precision = ctxs[0]->opt.precision;
  // work lists, largest geometry first (as bte_batch_create orders them)
  for (int i = 0; i < n; ++i) H.order[i] = i;
  std::stable_sort(H.order, H.order + n, [&](int a, int c) {
    const double wa = (double)ctxs[a]->s.nc * ctxs[a]->s.nd * ctxs[a]->s.nb;
    const double wc = (double)ctxs[c]->s.nc * ctxs[c]->s.nd * ctxs[c]->s.nb;
    return wa > wc;
  });
  int counts[kBatchLists] = {0, 0, 0};
  int ngeo[kBatchLists] = {0, 0, 0};
  int max_inner = 0;
  for (int k = 0; k < n; ++k) {
    const int i = H.order[k];
    const SweepPlan& pl = ctxs[i]->s.plan;
    const int l = batch_list_of(pl);
    const long long items = (long long)pl.ndg * ctxs[i]->s.nb * pl.ntiles;
    if ((long long)counts[l] + items > INT_MAX)
      return fail(BTE_E_INVAL, "work list %d exceeds 2^31 items", l);
    H.dev.list_ctx[l][ngeo[l]] = i;
    H.dev.list_start[l][ngeo[l]] = counts[l];
    ngeo[l] += 1;
    counts[l] += (int)items;
    max_inner = std::max(max_inner, ctxs[i]->opt.max_inner);
  }
  for (int l = 0; l < kBatchLists; ++l) H.dev.list_start[l][ngeo[l]] = counts[l];
  BatchRanges ranges[kBatchLists];
  for (int l = 0; l < kBatchLists; ++l)
    ranges[l] = BatchRanges{ngeo[l], d->list_ctx[l], d->list_start[l]};
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  int sweep_blocks[kBatchLists];
  for (int l = 0; l < kBatchLists; ++l) sweep_blocks[l] = cus * batch_sweep_occupancy(precision, l);
  int temp_blocks = 0;
  for (int i = 0; i < n; ++i)
    temp_blocks += (ctxs[i]->s.nc + temp_cells_per_block(ctxs[i]->s.nb) - 1) /
                   temp_cells_per_block(ctxs[i]->s.nb);
  HIP_TRY(hipMemcpyAsync(d->list_ctx, H.dev.list_ctx, sizeof(H.dev.list_ctx),
                         hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(d->list_start, H.dev.list_start, sizeof(H.dev.list_start),
                         hipMemcpyHostToDevice, stream));
  for (int step = 0; step < nsteps; ++step) {
    int block0 = 0;
    for (int i = 0; i < n; ++i) {
      ctx = ctxs[i];
      if (ctx->poisoned) return fail(BTE_E_DEVICE, "context %d is poisoned", i);
      int rc = step_begin(ctx, 0, &H.ss[i]);
      if (rc != BTE_OK) return rc;
      fill_batch_ctx(H.dev.ctx[i], ctx, block0);
      block0 += H.dev.ctx[i].cell_blocks;
    }
    ctx = nullptr;
    HIP_TRY(hipMemcpyAsync(d->ctx, H.dev.ctx, sizeof(BatchCtx) * n, hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(launch_batch_reset(stream, d->ctx, n, &d->bc));
    for (int j = 0; j < max_inner; ++j) {
      HIP_TRY(launch_batch_iteration_ranges(stream, precision, d->ctx, n, ranges, counts, &d->bc,
                                            sweep_blocks, temp_blocks));
      HIP_TRY(hipMemcpyAsync(&H.dev.bc, &d->bc, sizeof(BatchControl), hipMemcpyDeviceToHost,
                             stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (H.dev.bc.active == 0) break;
    }
    for (int i = 0; i < n; ++i)
      HIP_TRY(hipMemcpyAsync(&H.ctl[i], ctxs[i]->ctl, sizeof(Control), hipMemcpyDeviceToHost,
                             stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (int i = 0; i < n; ++i) {
      const int rc = step_finish(ctxs[i], H.ss[i], H.ctl[i],
                                 stats ? &stats[(size_t)step * n + i] : nullptr);
      if (rc != BTE_OK) return rc;
    }
  }
  return BTE_OK;
}

}  // extern "C"
