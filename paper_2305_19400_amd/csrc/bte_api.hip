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
#include <new>
#include <string>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"

using namespace bte;

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
constexpr double kMirrorTol = 1e-12;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t ctl, coef, dflags, mirror, w, Cb, xfac, inv_tau, fweight, Iref;
  size_t wallT[6], wallI0[6];
  size_t T, Tprev, E, I0, S, part;
  size_t In, Ia, Ib;
  size_t total;
};

struct Shape {
  int dim, nx, ny, nz, nc, ncp, nd, nb;
  int nf[6];
  bool iso[6];
  size_t real_size;
  SweepPlan plan;
};

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
    L.wallT[f] = s.iso[f] ? take(sizeof(double) * (size_t)s.nf[f]) : 0;
    L.wallI0[f] = s.iso[f] ? take(sizeof(double) * (size_t)s.nf[f] * s.nb) : 0;
  }
  L.T = take(sizeof(double) * (size_t)s.ncp);
  L.Tprev = take(sizeof(double) * (size_t)s.ncp);
  L.E = take(sizeof(double) * (size_t)s.ncp);
  L.I0 = take(sizeof(double) * (size_t)s.nb * s.ncp);
  L.S = take(sizeof(double) * (size_t)s.plan.ndg * s.nb * s.ncp);
  L.part = take(sizeof(double) * 2 * (size_t)s.plan.nparts);
  const size_t field = s.real_size * (size_t)s.nb * s.nd * s.ncp;
  L.In = take(field);
  L.Ia = take(field);
  L.Ib = take(field);
  L.total = off + 65536;  // tail slack: no kernel access may reach past the last array
  return L;
}

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
  if (nc > INT_MAX / 2) return fail(BTE_E_INVAL, "too many cells (%lld)", nc);
  if (d->n < 1 || !d->s || !d->w) return fail(BTE_E_INVAL, "need at least one direction");
  if (d->n > 65535) return fail(BTE_E_INVAL, "at most 65535 directions");
  if (b->n < 1 || !b->omega || !b->domega) return fail(BTE_E_INVAL, "need at least one band");
  if (b->n > 65535) return fail(BTE_E_INVAL, "at most 65535 band entries");
  if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(BTE_E_INVAL, "dt must be positive");
  if (o->scheme != BTE_IMPLICIT_JACOBI && o->scheme != BTE_EXPLICIT_EULER)
    return fail(BTE_E_INVAL, "unknown scheme %d", o->scheme);
  if (o->precision != BTE_FP64 && o->precision != BTE_FP32_MIXED)
    return fail(BTE_E_INVAL, "unknown precision %d", o->precision);
  if (o->t_definition != BTE_T_TAU_WEIGHTED && o->t_definition != BTE_T_ENERGY)
    return fail(BTE_E_INVAL, "unknown temperature definition %d", o->t_definition);
  if (!m->T_init) return fail(BTE_E_INVAL, "T_init is required");
  Shape s{};
  s.dim = m->dim;
  s.nx = m->n[0];
  s.ny = m->n[1];
  s.nz = m->n[2];
  s.nc = (int)nc;
  s.ncp = (int)((nc + kSlabAlign - 1) / kSlabAlign * kSlabAlign);
  s.nd = d->n;
  s.nb = b->n;
  // Launch layout of the sweep; BTE_SWEEP_RY / BTE_SWEEP_NDG / BTE_SWEEP_KIND
  // override the rows per wave, the number of direction groups and the kernel
  // family (tuning knobs).
  s.plan = make_sweep_plan(s.dim, s.nx, s.ny, s.nz, s.nd, s.nb, env_int("BTE_SWEEP_RY", 0),
                           env_int("BTE_SWEEP_NDG", 0), env_int("BTE_SWEEP_KIND", -1));
  s.real_size = o->precision == BTE_FP64 ? sizeof(double) : sizeof(float);
  const int nfaces[3] = {s.ny * s.nz, s.nx * s.nz, s.nx * s.ny};
  for (int f = 0; f < 6; ++f) {
    s.nf[f] = nfaces[f / 2];
    s.iso[f] = false;
    if (f >= 2 * s.dim) continue;
    const int kind = m->wall[f];
    if (kind == BTE_WALL_ISOTHERMAL) {
      if (!m->wall_T[f]) return fail(BTE_E_INVAL, "isothermal wall %d needs wall_T", f);
      s.iso[f] = true;
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
  std::vector<double> Iref;  // host copy of the storage reference per band
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
int enqueue_sweep(bte_ctx* ctx, const void* src, void* dst) {
  HIP_TRY(launch_sweep<Real>(ctx->stream, ctx->g, ctx->t, ctx->s.plan, 1.0 / ctx->opt.dt,
                             static_cast<const Real*>(src), static_cast<const Real*>(ctx->In),
                             static_cast<Real*>(dst), ctx->I0, ctx->S, ctx->part, ctx->ctl));
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
  int rc = ctx->opt.precision == BTE_FP64 ? enqueue_sweep<double>(ctx, src, dst)
                                          : enqueue_sweep<float>(ctx, src, dst);
  if (rc != BTE_OK) return rc;
  if (timing) HIP_TRY(hipEventRecord(ctx->t_stop[j], ctx->stream));
  HIP_TRY(launch_temperature(ctx->stream, ctx->g, ctx->t, ctx->S, ctx->T, ctx->I0, ctx->E,
                             ctx->ctl));
  HIP_TRY(launch_control(ctx->stream, ctx->s.plan.nparts, ctx->part, ctx->g.vol, fixed_k,
                         ctx->opt.max_inner, ctx->opt.tol,
                         ctx->opt.scheme == BTE_EXPLICIT_EULER, ctx->ctl));
  return BTE_OK;
}

int one_step(bte_ctx* ctx, int fixed, bte_step_stats* st) {
  const bool explicit_mode = ctx->opt.scheme == BTE_EXPLICIT_EULER;
  const int limit = explicit_mode ? 1 : (fixed > 0 ? fixed : ctx->opt.max_inner);
  const bool check = !explicit_mode && fixed <= 0;
  HIP_TRY(hipMemcpyAsync(ctx->Tprev, ctx->T, sizeof(double) * ctx->s.nc, hipMemcpyDeviceToDevice,
                         ctx->stream));
  HIP_TRY(launch_reset(ctx->stream, ctx->ctl));
  for (int j = 0; j < limit; ++j) {
    int rc = enqueue_iteration(ctx, j, check ? 0 : fixed);
    if (rc != BTE_OK) return rc;
    if (check) {
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
  Control fin;
  HIP_TRY(hipMemcpyAsync(&ctx->host_ring[0], ctx->ctl, sizeof(Control), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  fin = ctx->host_ring[0];
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
  void*& last = ((fin.k - 1) & 1) ? ctx->Ib : ctx->Ia;
  std::swap(ctx->In, last);
  if (st) {
    st->inner = fin.k;
    st->newton_max = fin.newton_max;
    st->res = fin.res;
    st->converged = explicit_mode || (fixed > 0 ? fin.k >= fixed : fin.res <= ctx->opt.tol);
    st->reserved = 0;
  }
  if (!explicit_mode && fixed <= 0 && fin.res > ctx->opt.tol && ctx->opt.fail_on_notconv)
    return fail(BTE_E_NOTCONV, "inner iteration hit max_inner=%d with res=%g > tol=%g",
                ctx->opt.max_inner, fin.res, ctx->opt.tol);
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
  for (int b = 0; b < nb; ++b) {
    const double vals[6] = {bands->omega[b], bands->domega[b], disp->vg[b], disp->tau[b],
                            disp->dos[b], disp->deg[b]};
    for (double v : vals)
      if (!(v > 0.0) || !std::isfinite(v))
        return fail(BTE_E_INVAL, "band %d: omega, domega, vg, tau, dos, deg must be positive", b);
  }
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
    if (s.iso[f]) continue;
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
    }
  }

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

  Geometry& g = ctx->g;
  g.dim = s.dim;
  g.nx = s.nx;
  g.ny = s.ny;
  g.nz = s.nz;
  g.nc = s.nc;
  g.ncp = s.ncp;
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
  t.W = W;
  for (int f = 0; f < 6; ++f) {
    t.wall[f] = (f < 2 * s.dim) ? mesh->wall[f] : BTE_WALL_SPECULAR;
    t.wall_nf[f] = s.nf[f];
    t.wall_I0[f] = s.iso[f] ? at<double>(ws, L.wallI0[f]) : nullptr;
  }

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
  for (auto& e : ctx->ring_ev) CREATE_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  CREATE_TRY(up(L.coef, coef.data(), sizeof(Coef) * coef.size()));
  CREATE_TRY(up(L.dflags, dflags.data(), sizeof(int) * dflags.size()));
  CREATE_TRY(up(L.mirror, mirror.data(), sizeof(int) * mirror.size()));
  CREATE_TRY(up(L.w, dirs->w, sizeof(double) * nd));
  CREATE_TRY(up(L.Cb, Cb.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.xfac, xfac.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.inv_tau, inv_tau.data(), sizeof(double) * nb));
  CREATE_TRY(up(L.fweight, fweight.data(), sizeof(double) * nb));
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
  CREATE_TRY(hipStreamSynchronize(ctx->stream));
#undef CREATE_TRY
  *out = ctx;
  return BTE_OK;
}

int bte_step(bte_ctx* ctx, int nsteps, const int* fixed_inner, bte_step_stats* stats) {
  if (!ctx) return fail(BTE_E_INVAL, "null context");
  if (ctx->poisoned) return fail(BTE_E_DEVICE, "context is poisoned by an earlier device error");
  if (nsteps < 0) return fail(BTE_E_INVAL, "nsteps must be >= 0");
  for (int i = 0; i < nsteps; ++i) {
    const int fixed = fixed_inner ? fixed_inner[i] : 0;
    int rc = one_step(ctx, fixed, stats ? &stats[i] : nullptr);
    if (rc != BTE_OK) return rc;
  }
  return BTE_OK;
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
    HIP_TRY(hipMemcpy2DAsync(I_out, sizeof(double) * ctx->s.nc, ctx->In,
                             sizeof(double) * ctx->s.ncp, sizeof(double) * ctx->s.nc, rows,
                             hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  } else {
    std::vector<float> tmp;
    try {
      tmp.resize(n);
    } catch (...) {
      return fail(BTE_E_NOMEM, "out of host memory");
    }
    HIP_TRY(hipMemcpy2DAsync(tmp.data(), sizeof(float) * ctx->s.nc, ctx->In,
                             sizeof(float) * ctx->s.ncp, sizeof(float) * ctx->s.nc, rows,
                             hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const size_t nc = ctx->s.nc;
    for (size_t i = 0; i < n; ++i) I_out[i] = ctx->Iref[i / (nc * ctx->s.nd)] + (double)tmp[i];
  }
  return BTE_OK;
}

int bte_set_state(bte_ctx* ctx, const double* I, size_t n, const double* T, size_t n_cells) {
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
    HIP_TRY(hipMemcpy2DAsync(ctx->In, sizeof(double) * ctx->s.ncp, I, sizeof(double) * ctx->s.nc,
                             sizeof(double) * ctx->s.nc, rows, hipMemcpyHostToDevice, ctx->stream));
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
    HIP_TRY(hipMemcpy2DAsync(ctx->In, sizeof(float) * ctx->s.ncp, tmp.data(),
                             sizeof(float) * ctx->s.nc, sizeof(float) * ctx->s.nc, rows,
                             hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  HIP_TRY(hipMemcpyAsync(ctx->T, T, sizeof(double) * n_cells, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->Tprev, T, sizeof(double) * n_cells, hipMemcpyHostToDevice,
                         ctx->stream));
  HIP_TRY(launch_equilibrium(ctx->stream, ctx->g, ctx->t, ctx->T, ctx->I0, nullptr));
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

int bte_destroy(bte_ctx* ctx) {
  if (!ctx) return BTE_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto e : ctx->t_start) (void)hipEventDestroy(e);
  for (auto e : ctx->t_stop) (void)hipEventDestroy(e);
  if (ctx->host_ring) (void)hipHostFree(ctx->host_ring);
  delete ctx;
  return BTE_OK;
}

const char* bte_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
