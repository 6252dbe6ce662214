// HIP kernels of the phonon BTE time step for gfx950 (CDNA4, wave64).
//
// Data layout in HBM: intensity I[b][d][P] with P = x + nx*(y + ny*z) and each
// (b, d) slab padded to a multiple of 64 cells, so a wavefront streams 64
// consecutive cells of one slab (coalesced 512-B FP64 / 256-B FP32 accesses).
// Per-(b, d) coefficients are wave-uniform and live in scalar registers.
#include <algorithm>
#include <climits>
#include <cmath>

#include "bte_internal.h"

namespace bte {

// ---------------------------------------------------------------- equilibrium
// Bose-Einstein equilibrium intensity of one band at temperature T:
// I0 = C / (exp(hbar omega / k_B T) - 1), with C and hbar omega / k_B given.
__device__ __forceinline__ double equilibrium(double C, double xf, double T) {
  return C / expm1(xf / T);
}

// ---------------------------------------------------------------- control flags
// The control word is read through a generic pointer, which the compiler must
// treat as possibly divergent.  Every branch that decides whether a workgroup
// reaches a barrier reads it through this helper: readfirstlane makes the
// value (and so the branch) wave-uniform, which keeps __syncthreads() in
// uniform control flow.  Without it the structurizer may nest a persistent
// loop so that most lanes circle the barrier while the lane that advances the
// work counter waits outside the inner loop.
__device__ __forceinline__ bool step_done(const Control* ctl) {
  return __builtin_amdgcn_readfirstlane(ctl->converged) != 0;
}

// The sweep, temperature and control bodies are inlined into both the
// per-geometry kernels and the batched persistent kernels.  They set
// "fp contract(on)": a multiply is fused into an add only inside one source
// expression, never across statements at the compiler's discretion, so every
// kernel that inlines a body rounds exactly alike and batched results equal
// single-geometry results bit for bit.

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  // Butterfly over the 64 lanes; the order is fixed, so results are reproducible.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Neumaier-compensated accumulation (used where FP32-stored values are summed).
struct CompSum {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double v) {
    const double t = s + v;
    c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

// Stored intensities: FP64 holds I itself; FP32 holds the deviation from a
// per-band reference, I - Iref[b], which keeps the FP32 rounding relative to
// the (small) departure from equilibrium rather than to I.
template <typename Real>
struct Storage;
template <>
struct Storage<double> {
  static constexpr bool kDeviation = false;
  using Arith = double;
};
template <>
struct Storage<float> {
  static constexpr bool kDeviation = true;
  using Arith = double;
};

// Arithmetic of the column-walk sweeps: FP64 on the intensities (FP64
// storage) or on the deviations I - Iref_b (FP32 storage).  Every term of the
// point-Jacobi update is a difference of two intensities of one band
// (I^n - I, I0 - I, I_upwind - I), so Iref_b cancels, and the update is
// rounded once, to the stored value.  (The update computed in FP32 leaves
// rounding noise of an ulp in every increment: a converged iterate keeps
// flickering and the increment norm stalls far above tight tolerances.)
template <typename Real>
using Arith = typename Storage<Real>::Arith;
// Arithmetic value of an FP64 intensity (cell equilibrium, warm-start shift).
template <typename Real>
__device__ __forceinline__ Arith<Real> to_arith(double iref, double I) {
  if constexpr (Storage<Real>::kDeviation) return I - iref;
  else return I;
}

// Intensity from a stored value (exact identity for FP64 storage).
template <typename Real>
__device__ __forceinline__ double decode(double iref, Real v) {
  if constexpr (Storage<Real>::kDeviation) return iref + static_cast<double>(v);
  else return static_cast<double>(v);
}
// Stored value of an intensity.
template <typename Real>
__device__ __forceinline__ Real encode(double iref, double I) {
  if constexpr (Storage<Real>::kDeviation) return static_cast<Real>(I - iref);
  else return static_cast<Real>(I);
}

// ---------------------------------------------------------------- sweep

// Energy sum over a direction group of one (band, cell): sum_d w_d I.  With
// FP64 storage a plain FP64 sum of the intensities; with FP32 storage a
// compensated (Kahan) FP64 sum of the deviations w_d (I - Iref_b), to which
// Iref_b sum_d w_d is added once at the end.  Sc carries the negated rounding
// error of the running sum.
template <typename Real>
__device__ __forceinline__ void accumulate_energy(double& S, double& Sc, double w, double v) {
  if constexpr (Storage<Real>::kDeviation) {
    const double y = w * v - Sc;
    const double t = S + y;
    Sc = (t - S) - y;
    S = t;
  } else {
    S += w * v;
  }
}
template <typename Real>
__device__ __forceinline__ double energy_partial(double S, double Sc, double iref, double wsum) {
  if constexpr (Storage<Real>::kDeviation) return iref * wsum + (S - Sc);
  else return S;
}

// The point-Jacobi update of one cell, I_new = I + R / a with
// R = (I^n - I)/dt + (I0 - I)/tau + sum_in c (I_up - I) and a = 1/dt + 1/tau +
// sum c.  With FP64 storage it is evaluated in this defect form, which leaves
// a uniform equilibrium state bit for bit unchanged.  With FP32 storage the
// equal direct form I_new = (q I^n + I0/tau + sum_in c I_up) / a with q = 1/dt
// is used on the deviations (fewer operations); its FP64 rounding is far
// below the single rounding to the stored value.  Under forward Euler the
// sweep reads I = I^n and 1/a = dt, and the same direct form is the explicit
// update with q = 1/dt - 1/tau - sum_in c (the defect form needs no q).  Each
// helper is one expression, so FMA contraction is the same wherever it is
// inlined.
template <typename Real, typename A>
__device__ __forceinline__ A update_start(A in, A i0, A v, A q, A inv_dt, A inv_tau) {
#pragma clang fp contract(on)
  if constexpr (Storage<Real>::kDeviation) return in * q + i0 * inv_tau;
  else return (in - v) * inv_dt + (i0 - v) * inv_tau;
}
template <typename Real, typename A>
__device__ __forceinline__ A update_add(A acc, A c, A up, A v) {
#pragma clang fp contract(on)
  if constexpr (Storage<Real>::kDeviation) return acc + c * up;
  else return acc + c * (up - v);
}
template <typename Real, typename A>
__device__ __forceinline__ Real update_finish(A acc, A v, A scale) {
#pragma clang fp contract(on)
  if constexpr (Storage<Real>::kDeviation) return static_cast<Real>(acc * scale);
  else return static_cast<Real>(v + acc * scale);
}

// The update scale of a cell whose relaxation rate depends on its
// temperature: 1 / (1/dt + rate + sum_axis c_axis), summed in the order of the
// per-(direction, band) table's constant-rate diagonal; dt for forward Euler.
__device__ __forceinline__ double cell_scale(const Coef& cf, double inv_dt, double rate,
                                             int explicit_scheme) {
  if (explicit_scheme) return cf.scale;
  return 1.0 / ((((inv_dt + rate) + cf.c[0]) + cf.c[1]) + cf.c[2]);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float read_lane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Raw buffer access to one (band, direction) slab: the base address and the
// row offset are wave-uniform (scalar registers), the lane offset is one vector
// register shared by every row; reads past the slab's valid cells return 0.
constexpr int kBufferWord3 = 0x00020000;  // gfx9-family buffer resource flags
// A byte offset past the end of every slab (create limits a slab to
// 2^31 - 256 bytes): a raw buffer access there reads 0 or is dropped, without
// a memory access.
constexpr int kPastEnd = 0x7ffffff0;

// Cache-policy bits of the slab loads and stores (0: default, 2: non-temporal).
// The new iterate is not read again within the sweep, so it is streamed out
// non-temporally; measured ~3 % faster than default stores on the 2D sweep.
#ifndef BTE_SLAB_LOAD_AUX
#define BTE_SLAB_LOAD_AUX 0
#endif
#ifndef BTE_SLAB_STORE_AUX
#define BTE_SLAB_STORE_AUX 2
#endif
// The step-start field I^n is read once per sweep, each value by its own
// cell's lane, so its loads are non-temporal too: they then do not displace
// the current iterate's rows, which neighbouring tiles re-read as halos
// (measured on 400 directions x 55 band entries: 64^3 sweeps 6 % faster in
// FP32 and 2 % in FP64, 128 x 128 FP32 1 %, 96^3 FP32 0.6 %; making the
// iterate's own loads non-temporal as well was 9-11 % slower).
#ifndef BTE_STEP_LOAD_AUX
#define BTE_STEP_LOAD_AUX 2
#endif

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufferWord3);
}

// Read-only table entry through the constant address space: with a
// wave-uniform index the compiler emits a scalar load, which neither waits for
// nor delays the vector loads of the intensity slabs.
template <typename T>
__device__ __forceinline__ T cld(const T* base, size_t i) {
  return ((const __attribute__((address_space(4))) T*)base)[i];
}
__device__ __forceinline__ Coef cld_coef(const Coef* base, size_t i) {
  const double* c = base[i].c;  // c[0], c[1], c[2], scale, q are contiguous doubles
  Coef r;
  r.c[0] = cld(c, 0);
  r.c[1] = cld(c, 1);
  r.c[2] = cld(c, 2);
  r.scale = cld(c, 3);
  r.q = cld(c, 4);
  return r;
}

template <typename Real>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, BTE_SLAB_LOAD_AUX);
  return __longlong_as_double(((long long)v[1] << 32) | (unsigned int)v[0]);
}
template <>
__device__ __forceinline__ double buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, BTE_SLAB_LOAD_AUX));
}

// The stored value itself (no conversion), so that a load issued inside a
// branch is not waited for inside it.
template <typename Real>
__device__ __forceinline__ Real buf_load_raw(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ double buf_load_raw<double>(__amdgpu_buffer_rsrc_t r, int voff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, BTE_SLAB_LOAD_AUX);
  return __longlong_as_double(((long long)v[1] << 32) | (unsigned int)v[0]);
}
template <>
__device__ __forceinline__ float buf_load_raw<float>(__amdgpu_buffer_rsrc_t r, int voff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, BTE_SLAB_LOAD_AUX));
}

// A value of the step-start field I^n (non-temporal load).
template <typename Real>
__device__ __forceinline__ Real buf_load_step(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ double buf_load_step<double>(__amdgpu_buffer_rsrc_t r, int voff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, BTE_STEP_LOAD_AUX);
  return __longlong_as_double(((long long)v[1] << 32) | (unsigned int)v[0]);
}
template <>
__device__ __forceinline__ float buf_load_step<float>(__amdgpu_buffer_rsrc_t r, int voff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, BTE_STEP_LOAD_AUX));
}

template <typename Real>
__device__ __forceinline__ void buf_store(Real v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff,
                                                 int soff) {
  const long long bits = __double_as_longlong(v);
  __attribute__((ext_vector_type(2))) unsigned int u;
  u[0] = (unsigned int)(bits & 0xffffffffll);
  u[1] = (unsigned int)(bits >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(u, r, voff, soff, BTE_SLAB_STORE_AUX);
}
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int voff,
                                                int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, BTE_SLAB_STORE_AUX);
}

// One point-Jacobi sweep (or forward-Euler update) over every direction of one
// band for a tile of kSweepBlock cells, fused with the per-(band, cell) energy
// partial sum_d w_d I^{k+1} and the per-block pieces of the increment norms.
//
// For DOF (P, d, b) with current iterate I^k, step-start value I^n and
// equilibrium I0 = I0_b(T_P^k) (Eq. eq-bte-fv, backward Euler, upwind faces):
//   R = (I^n - I^k)/dt + (I0 - I^k)/tau_b + sum_axis c_axis (I_up,axis - I^k)
//   I^{k+1} = I^k + R * scale,   scale = 1/(1/dt + 1/tau_b + sum_axis c_axis)
// Forward Euler passes I^k = I^n and scale = dt, which is Eq.
// eq-conservation-discrete with the same upwind fluxes.
template <typename Real, int DIM, bool SHIFT, bool TAUT>
__device__ __forceinline__ void sweep_body(const SweepParams<Real>& p, const int bx, const int by,
                                           const int gx) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  const int b = by;
  const int P = bx * kSweepBlock + threadIdx.x;
  const Geometry& g = p.g;
  const bool active = P < g.nc;
  const int Pc = active ? P : g.nc - 1;  // every lane addresses a valid cell
  const int cx = Pc % g.nx;
  const int cy = (Pc / g.nx) % g.ny;
  const int cz = Pc / (g.nx * g.ny);
  const size_t ncp = (size_t)g.ncp;
  const size_t band_off = (size_t)b * g.nd * ncp;
  const Real* __restrict__ Ikb = p.Ik + band_off;
  const Real* __restrict__ Inb = p.In + band_off;
  Real* __restrict__ Iob = p.Iout + band_off;
  const double I0P = p.I0[(size_t)b * ncp + Pc];
  const double inv_tau = TAUT ? p.t.relax[(size_t)b * ncp + Pc] : cld(p.t.inv_tau, (size_t)b);
  const double iref = Storage<Real>::kDeviation ? cld(p.t.Iref, (size_t)b) : 0.0;
  const int slab_bytes = g.px * g.ny * g.nz * (int)sizeof(Real);
  const int Qc = (int)ipos(g, Pc);  // this cell's position in a slab
  const int voff = Qc * (int)sizeof(Real);
  // Per axis: coordinate, extent, cell stride (per-cell arrays, slabs) and
  // wall-face index of this cell.
  const int co[3] = {cx, cy, cz};
  const int ext[3] = {g.nx, g.ny, g.nz};
  const int str[3] = {1, g.nx, g.nx * g.ny};
  const int istr[3] = {1, g.px, g.px * g.ny};
  const int face[3] = {cy + g.ny * cz, cx + g.nx * cz, cx + g.nx * cy};
  double sh0 = 0.0, shn[DIM][2];  // warm-start shift of this cell and its neighbours
  if constexpr (SHIFT) {
    const double* __restrict__ sb = p.shift + (size_t)b * ncp;
    sh0 = sb[Pc];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      shn[a][0] = co[a] > 0 ? sb[Pc - str[a]] : sh0;
      shn[a][1] = co[a] < ext[a] - 1 ? sb[Pc + str[a]] : sh0;
    }
  }

  CompSum S;
  double Splain = 0.0, num = 0.0, den = 0.0;
  for (int d = 0; d < g.nd; ++d) {
    const Coef cf = cld_coef(p.t.coef, (size_t)b * g.nd + d);
    const int fl = cld(p.t.dflags, (size_t)d);
    const double wd = cld(p.t.w, (size_t)d);
    const Real* __restrict__ slab = Ikb + (size_t)d * ncp;
    const Real ik_r = buf_load_raw<Real>(slab_rsrc(slab, slab_bytes), voff);
    const Real in_r = buf_load_raw<Real>(slab_rsrc(Inb + (size_t)d * ncp, slab_bytes), voff);
    // Upwind value along each axis: the inflow neighbour, or on a wall face
    // the ghost (Eq. eq-bdry) -- the isothermal wall's equilibrium, or this
    // cell's own intensity in the mirrored direction.  Both candidates are
    // loaded for every lane from valid addresses, before any is waited for.
    Real nb_r[DIM];
    double wt[DIM];
    bool inside[DIM], iso[DIM], flows[DIM], minus[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      flows[a] = dir_pos(fl, a) || dir_neg(fl, a);
      minus[a] = dir_pos(fl, a);  // inflow from the minus side
      inside[a] = minus[a] ? co[a] > 0 : co[a] < ext[a] - 1;
      const int side = 2 * a + (minus[a] ? 0 : 1);
      iso[a] = p.t.wall[side] == 0;
      const int r = iso[a] ? d : cld(p.t.mirror, (size_t)a * g.nd + d);
      const Real* src = inside[a] ? slab + (minus[a] ? Qc - istr[a] : Qc + istr[a])
                                  : Ikb + (size_t)r * ncp + Qc;
      nb_r[a] = *src;
      const double* __restrict__ wtab = iso[a] ? p.t.wall_I0[side] : p.t.w;
      wt[a] = wtab[iso[a] ? (size_t)b * p.t.wall_nf[side] + face[a] : 0];
    }
    const double ik = decode(iref, ik_r) + (SHIFT ? sh0 : 0.0);
    const double in = decode(iref, in_r);
    double acc = (in - ik) * p.inv_dt + (I0P - ik) * inv_tau;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      if (!flows[a]) continue;
      double up;
      if (!inside[a] && iso[a]) {
        up = wt[a];
      } else {
        up = decode(iref, nb_r[a]);
        if constexpr (SHIFT) up += inside[a] ? shn[a][minus[a] ? 0 : 1] : sh0;
      }
      acc += cf.c[a] * (up - ik);
    }
    const double scale = TAUT ? cell_scale(cf, p.inv_dt, inv_tau, p.t.explicit_scheme) : cf.scale;
    const Real inew_r = encode<Real>(iref, ik + acc * scale);
    if (active) buf_store<Real>(inew_r, slab_rsrc(Iob + (size_t)d * ncp, slab_bytes), voff, 0);
    const double inew = decode(iref, inew_r);
    const double da = inew - ik;
    const double dn = inew - in;
    if (active) {
      if constexpr (Storage<Real>::kDeviation) S.add(wd * inew);
      else Splain += wd * inew;
      num += wd * da * da;
      den += wd * dn * dn;
    }
  }
  if (active) p.S[(size_t)b * ncp + P] = Storage<Real>::kDeviation ? S.value() : Splain;

  __shared__ double red[2][kSweepBlock / 64];
  num = wave_sum(num);
  den = wave_sum(den);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = num;
    red[1][wave] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kSweepBlock / 64; ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    const size_t blk = (size_t)by * gx + bx;
    p.part[2 * blk] = a;
    p.part[2 * blk + 1] = c;
  }
}

template <typename Real, int DIM, bool SHIFT, bool TAUT>
__global__ __launch_bounds__(kSweepBlock) void sweep_kernel(const SweepParams<Real> p) {
  if (step_done(p.ctl)) return;
  sweep_body<Real, DIM, SHIFT, TAUT>(p, blockIdx.x, blockIdx.y, gridDim.x);
}

// ---------------------------------------------------------------- 2D column walk

// The same update as sweep_kernel for 2D meshes, organised for reuse: a
// workgroup owns a tile of 64 columns x (4 * RY) rows of one band and a group of
// directions.  Lane = column, each wave walks RY consecutive rows, so the
// y-upwind neighbour is the lane's previous/next row held in registers and the
// x-upwind neighbour comes from the adjacent lane by a cross-lane shuffle; only
// tile edges read halo values (the x halo column is fetched by RY lanes in one
// load and broadcast with readlane).  The per-(direction group, band, cell)
// energy partials and per-workgroup norm partials are fused as in sweep_kernel.
template <typename Real, int RY, bool SHIFT, bool TAUT>
__device__ __forceinline__ void walk2d_body(const SweepParams<Real>& p, const int ntx,
                                            const int dgs, const int bx, const int by,
                                            const int bz, const int gx, const int gy) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  const Geometry& g = p.g;
  const int nx = g.nx, ny = g.ny;
  const int tx = bx % ntx;
  const int ty = bx / ntx;
  const int b = by;
  const int dg = bz;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * 64;
  const int x = x0 + lane;
  const int y0 = ty * (4 * RY) + wave * RY;
  const int nrows = max(0, min(RY, ny - y0));
  const bool colok = x < nx;
  const int d_begin = dg * dgs;
  const int d_end = min(g.nd, d_begin + dgs);
  const size_t ncp = (size_t)g.ncp;
  const size_t band_off = (size_t)b * g.nd * ncp;
  const Real* __restrict__ Ikb = p.Ik + band_off;
  const Real* __restrict__ Inb = p.In + band_off;
  Real* __restrict__ Iob = p.Iout + band_off;
  const double inv_tau = p.t.inv_tau[b];
  const double iref = Storage<Real>::kDeviation ? p.t.Iref[b] : 0.0;
  const int px = g.px;  // slab row pitch (rows start on a 128-byte line)
  const int slab_bytes = px * ny * (int)sizeof(Real);
  // Every lane and row addresses a valid cell: lanes past the mesh edge reuse
  // column x0 and rows past the mesh reuse this wave's first row (their values
  // are never used), so no access leaves the slab's valid cells.
  const int voff = (colok ? lane : 0) * (int)sizeof(Real);
  const int y0c = min(y0, ny - 1);
  const int row0 = (y0c * px + x0) * (int)sizeof(Real);  // byte offset of (x0, y0)
  const int rowb = px * (int)sizeof(Real);
  int rowoff[RY];  // byte offset of (x0, row j) in a slab
  int vrow[RY];    // this lane's byte offset in row j (offsets live in VGPRs, so the
                   // slab loads never need a uniform register for them)
  int celloff[RY];  // byte offset of (x0, row j) in a per-cell FP64 array
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    rowoff[j] = row0 + (j < nrows ? j : 0) * rowb;
    vrow[j] = voff + rowoff[j];
    celloff[j] = ((y0c + (j < nrows ? j : 0)) * nx + x0) * 8;
  }

  using A = Arith<Real>;
  A I0r[RY], sh[RY], rate[RY];
  double S[RY], Sc[RY];
  {
    const auto r0 = slab_rsrc(p.I0 + (size_t)b * ncp, g.nc * 8);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(r0, (colok ? lane : 0) * 8,
                                                          celloff[j], 0);
      I0r[j] = to_arith<Real>(iref,
                              __longlong_as_double(((long long)v[1] << 32) | (unsigned int)v[0]));
      rate[j] = inv_tau;
      if constexpr (TAUT) {
        const auto r2 = slab_rsrc(p.t.relax + (size_t)b * ncp, g.nc * 8);
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r2, (colok ? lane : 0) * 8,
                                                            celloff[j], 0);
        rate[j] = __longlong_as_double(((long long)u[1] << 32) | (unsigned int)u[0]);
      }
      S[j] = 0.0;
      Sc[j] = 0.0;
      sh[j] = 0;
      if constexpr (SHIFT) {
        const auto r1 = slab_rsrc(p.shift + (size_t)b * ncp, g.nc * 8);
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r1, (colok ? lane : 0) * 8,
                                                            celloff[j], 0);
        sh[j] = static_cast<A>(__longlong_as_double(((long long)u[1] << 32) | (unsigned int)u[0]));
      }
    }
  }
  const A a_inv_dt = static_cast<A>(p.inv_dt), a_inv_tau = static_cast<A>(inv_tau);
  // 1 under forward Euler, where the table's q holds the band's constant
  // rate, which a temperature-dependent one replaces
  const A a_expl = p.t.explicit_scheme ? A(1) : A(0);
  double num = 0.0, den = 0.0, wsum = 0.0;

  // Tile edges.  Lane j fetches the x-inflow value of row y0 + j (the
  // neighbouring tile's column, or the wall ghost at the mesh edge); every lane
  // fetches the y-inflow value of its column (the row just outside this wave's
  // rows, or the wall ghost).  Which source applies is wave-uniform for a
  // direction, so each edge is one load, issued with the slab loads before any
  // of them is waited for.  Indices are clamped to valid cells.
  const int jl = min(lane, max(nrows - 1, 0));
  const int ye = min(y0 + jl, ny - 1);          // row whose x edge this lane fetches
  const int xcol = colok ? x : x0;              // a valid column for every lane
  const int last = min(63, nx - 1 - x0);        // last lane holding a mesh column
  const bool wall_l = x0 == 0;                  // -x inflow of lane 0 is the wall
  const bool wall_r = x0 + last == nx - 1;      // +x inflow of lane `last` is the wall
  const int col_l = wall_l ? 0 : x0 - 1;
  const int col_r = wall_r ? nx - 1 : x0 + 64;
  const bool wall_p = y0 == 0;                  // +y-moving inflow through the -y wall
  const bool wall_n = y0 + nrows >= ny;         // -y-moving inflow through the +y wall
  const int row_p = wall_p ? 0 : min(y0 - 1, ny - 1);
  const int row_n = wall_n ? ny - 1 : y0 + nrows;
  A shx_l = 0, shx_r = 0, shy_p = 0, shy_n = 0;
  if constexpr (SHIFT) {
    const double* __restrict__ sb = p.shift + (size_t)b * ncp;
    shx_l = static_cast<A>(sb[ye * nx + col_l]);
    shx_r = static_cast<A>(sb[ye * nx + col_r]);
    shy_p = static_cast<A>(sb[row_p * nx + xcol]);
    shy_n = static_cast<A>(sb[row_n * nx + xcol]);
  }

  // With FP32 storage the slab rows of direction d + 1 are requested (after
  // direction d's edge loads) before direction d is computed, so they stay in
  // flight during the arithmetic (measured 5 % faster); with FP64 storage this
  // measured neutral and each direction loads its own rows.
  constexpr bool kPrefetch = Storage<Real>::kDeviation;
  Real rk_v[RY], rn_v[RY];
  // The first sweep of a step (and every forward-Euler update) reads I^n as
  // its iterate: then I^n is loaded once (measured: forward-Euler sweeps of
  // 120 x 120 cells, 20 directions x 55 band entries, 4.6 % faster; 128 x 128
  // cells, 400 x 55 over whole steps 0.4 % in FP64 and 0.9 % in FP32).
  const bool same = Inb == Ikb;
  auto load_rows = [same](const Real* slab_k, const Real* slab_n, int bytes,
                          const int (&vr)[RY], Real (&k)[RY], Real (&n)[RY]) {
    const auto rk = slab_rsrc(slab_k, bytes);
    const auto rn = slab_rsrc(slab_n, bytes);
#pragma unroll
    for (int j = 0; j < RY; ++j) k[j] = buf_load_raw<Real>(rk, vr[j]);
    if (!same)
#pragma unroll
      for (int j = 0; j < RY; ++j) n[j] = buf_load_step<Real>(rn, vr[j]);
  };
  if constexpr (kPrefetch)
    if (nrows > 0 && d_begin < d_end)
      load_rows(Ikb + (size_t)d_begin * ncp, Inb + (size_t)d_begin * ncp, slab_bytes, vrow, rk_v,
                rn_v);
  for (int d = d_begin; d < d_end && nrows > 0; ++d) {
    const Coef cf = cld_coef(p.t.coef, (size_t)b * g.nd + d);
    const int fl = cld(p.t.dflags, d);
    const double wd = cld(p.t.w, d);
    const bool xpos = dir_pos(fl, 0), xneg = dir_neg(fl, 0);
    const bool ypos = dir_pos(fl, 1), yneg = dir_neg(fl, 1);
    const auto ro = slab_rsrc(Iob + (size_t)d * ncp, slab_bytes);
    if constexpr (!kPrefetch)
      load_rows(Ikb + (size_t)d * ncp, Inb + (size_t)d * ncp, slab_bytes, vrow, rk_v, rn_v);
    // Edges: both candidate sources are loaded without branching (the slab
    // value -- neighbouring tile or, through a specular/symmetry wall, the wall
    // cell in the mirrored direction -- and the isothermal wall's equilibrium
    // in storage format, read from a valid placeholder address when the side
    // is not isothermal),
    // and wave-uniform selects pick one after every load of this direction has
    // been issued.  (One load from a wave-uniformly chosen buffer, as in the 3D
    // walk, measured slower here: it left waits between the stores.)
    const bool wx = xpos ? wall_l : wall_r;  // x inflow through a wall
    const int sx = xpos ? 0 : 1;
    const bool iso_x = wx && p.t.wall[sx] == 0;
    const int dx_src = (wx && !iso_x) ? cld(p.t.mirror, (size_t)d) : d;
    const Real ex_r = buf_load_raw<Real>(slab_rsrc(Ikb + (size_t)dx_src * ncp, slab_bytes),
                                         (ye * px + (xpos ? col_l : col_r)) * (int)sizeof(Real));
    const Real* __restrict__ wbx =  // valid either way
        iso_x ? static_cast<const Real*>(p.t.wall_S[sx]) : reinterpret_cast<const Real*>(p.t.w);
    const Real ex_w = wbx[iso_x ? (size_t)b * p.t.wall_nf[sx] + ye : 0];
    const bool wy = ypos ? wall_p : wall_n;  // y inflow through a wall
    const int sy = ypos ? 2 : 3;
    const bool iso_y = wy && p.t.wall[sy] == 0;
    const int dy_src = (wy && !iso_y) ? cld(p.t.mirror, (size_t)g.nd + d) : d;
    const Real ey_r = buf_load_raw<Real>(slab_rsrc(Ikb + (size_t)dy_src * ncp, slab_bytes),
                                         ((ypos ? row_p : row_n) * px + xcol) * (int)sizeof(Real));
    const Real* __restrict__ wby =
        iso_y ? static_cast<const Real*>(p.t.wall_S[sy]) : reinterpret_cast<const Real*>(p.t.w);
    const Real ey_w = wby[iso_y ? (size_t)b * p.t.wall_nf[sy] + xcol : 0];
    Real nk_v[RY], nn_v[RY];  // direction d + 1 (clamped: the group's last re-reads d)
    if constexpr (kPrefetch) {
      const int dn = min(d + 1, d_end - 1);
      load_rows(Ikb + (size_t)dn * ncp, Inb + (size_t)dn * ncp, slab_bytes, vrow, nk_v, nn_v);
    }
    A ex = iso_x ? ex_w : ex_r;
    A ey = iso_y ? ey_w : ey_r;
    if constexpr (SHIFT) {
      if (!iso_x) ex += xpos ? shx_l : shx_r;
      if (!iso_y) ey += ypos ? shy_p : shy_n;
    }
    A ik[RY], in[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      ik[j] = rk_v[j];
      in[j] = same ? rk_v[j] : rn_v[j];
      if constexpr (SHIFT) ik[j] += sh[j];
    }
    const A c0 = static_cast<A>(cf.c[0]), c1 = static_cast<A>(cf.c[1]);
    const A scale = static_cast<A>(cf.scale);
    wsum += wd;
    // lane holding the x-upwind neighbour (direction sign is wave-uniform)
    const int src_lane = xpos ? max(lane - 1, 0) : min(lane + 1, 63);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const A nbr = __shfl(ik[j], src_lane, 64);
      const A exj = read_lane(ex, j);
      if (colok && j < nrows) {
        const A v = ik[j];
        const A rt = TAUT ? rate[j] : a_inv_tau;
        const A q = TAUT ? static_cast<A>(cf.q) + a_expl * (a_inv_tau - rt) : static_cast<A>(cf.q);
        A acc = update_start<Real>(in[j], I0r[j], v, q, a_inv_dt, rt);
        if (xpos) {
          const A up = lane == 0 ? exj : nbr;
          acc = update_add<Real>(acc, c0, up, v);
        } else if (xneg) {
          const A up = lane == last ? exj : nbr;
          acc = update_add<Real>(acc, c0, up, v);
        }
        if (ypos) {
          const A up = (j == 0) ? ey : ik[j > 0 ? j - 1 : 0];
          acc = update_add<Real>(acc, c1, up, v);
        } else if (yneg) {
          const A up = (j == nrows - 1) ? ey : ik[j + 1 < RY ? j + 1 : RY - 1];
          acc = update_add<Real>(acc, c1, up, v);
        }
        // the stored value drives the norms and the energy: once the
        // iterate stops changing in storage precision its increment is zero
        const A sc = TAUT ? cell_scale(cf, p.inv_dt, rate[j], p.t.explicit_scheme) : scale;
        const Real inew_r = update_finish<Real>(acc, v, sc);
        buf_store<Real>(inew_r, ro, vrow[j], 0);
        const A inew = inew_r;
        const double da = static_cast<double>(inew - v);
        const double dn = static_cast<double>(inew - in[j]);
        accumulate_energy<Real>(S[j], Sc[j], wd, static_cast<double>(inew));
        num += wd * da * da;
        den += wd * dn * dn;
      }
    }
    if constexpr (kPrefetch) {
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        rk_v[j] = nk_v[j];
        rn_v[j] = nn_v[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RY; ++j)
    if (colok && j < nrows)
      p.S[((size_t)dg * g.nb + b) * ncp + (size_t)(y0 + j) * nx + x] =
          energy_partial<Real>(S[j], Sc[j], iref, wsum);

  __shared__ double red[2][kSweepBlock / 64];
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) {
    red[0][wave] = num;
    red[1][wave] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kSweepBlock / 64; ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    const size_t blk = ((size_t)bz * gy + by) * gx + bx;
    p.part[2 * blk] = a;
    p.part[2 * blk + 1] = c;
  }
}

template <typename Real, int RY, bool SHIFT, bool TAUT>
__global__ __launch_bounds__(kSweepBlock) void sweep2d_walk_kernel(const SweepParams<Real> p,
                                                                   const int ntx, const int dgs) {
  if (step_done(p.ctl)) return;
  walk2d_body<Real, RY, SHIFT, TAUT>(p, ntx, dgs, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x,
                               gridDim.y);
}

// ---------------------------------------------------------------- 3D column walk
// The 3D counterpart of walk2d_body.  A workgroup owns 64 columns x (4 * RY)
// rows x RZ planes of one band and a group of directions; each wave holds RY
// rows x RZ planes of its 64 columns in registers.  The y- and z-upwind
// neighbours inside the block come from registers, the x-upwind neighbour
// from the adjacent lane; per direction one load per block face row fetches
// the inflow values outside the block -- the neighbouring block, or on a wall
// the ghost: the isothermal wall's equilibrium (kept in storage format, so it
// is one load from a wave-uniformly chosen buffer like any slab value) or the
// wall cell's own intensity in the mirrored direction.  Every load of a
// direction is issued before the first wait.
template <typename Real, int RY, int RZ, bool SHIFT, bool TAUT>
__device__ __forceinline__ void walk3d_body(const SweepParams<Real>& p, const int ntx,
                                            const int nty, const int dgs, const int bx,
                                            const int by, const int bz, const int gx,
                                            const int gy) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  constexpr int sz = (int)sizeof(Real);
  const Geometry& g = p.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int tx = bx % ntx;
  const int ty = (bx / ntx) % nty;
  const int tz = bx / (ntx * nty);
  const int b = by;
  const int dg = bz;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * 64;
  const int x = x0 + lane;
  const int y0 = ty * (4 * RY) + wave * RY;
  const int z0 = tz * RZ;
  const int nrows = max(0, min(RY, ny - y0));
  const int nplanes = max(0, min(RZ, nz - z0));
  const bool live = nrows > 0 && nplanes > 0;
  const bool colok = x < nx;
  const int xcol = colok ? x : x0;  // a valid column for every lane
  const int d_begin = dg * dgs;
  const int d_end = min(g.nd, d_begin + dgs);
  const size_t ncp = (size_t)g.ncp;
  const size_t band_off = (size_t)b * g.nd * ncp;
  const Real* __restrict__ Ikb = p.Ik + band_off;
  const Real* __restrict__ Inb = p.In + band_off;
  Real* __restrict__ Iob = p.Iout + band_off;
  const double inv_tau = cld(p.t.inv_tau, (size_t)b);
  const double iref = Storage<Real>::kDeviation ? cld(p.t.Iref, (size_t)b) : 0.0;
  const int slab_bytes = g.nc * sz;  // 3D slabs have no row padding (px = nx)
  // Register cell (j, k) is row y0 + j of plane z0 + k; rows and planes past
  // the mesh reuse the last valid one (their values are never used), so every
  // access stays on valid cells.
  int yr[RY], zp[RZ];
#pragma unroll
  for (int j = 0; j < RY; ++j) yr[j] = min(y0 + min(j, max(nrows - 1, 0)), ny - 1);
#pragma unroll
  for (int k = 0; k < RZ; ++k) zp[k] = min(z0 + min(k, max(nplanes - 1, 0)), nz - 1);
  int vc[RY][RZ];  // byte offset of this lane's cell (j, k) in a slab
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int k = 0; k < RZ; ++k) vc[j][k] = ((zp[k] * ny + yr[j]) * nx + xcol) * sz;

  using A = Arith<Real>;
  A I0r[RY][RZ], sh[RY][RZ], rate[RY][RZ];
  double S[RY][RZ], Sc[RY][RZ];
  {
    const auto r0 = slab_rsrc(p.I0 + (size_t)b * ncp, g.nc * 8);
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        I0r[j][k] = to_arith<Real>(iref, buf_load_raw<double>(r0, vc[j][k] / sz * 8));
        rate[j][k] = inv_tau;
        if constexpr (TAUT)
          rate[j][k] = buf_load_raw<double>(slab_rsrc(p.t.relax + (size_t)b * ncp, g.nc * 8),
                                            vc[j][k] / sz * 8);
        S[j][k] = 0.0;
        Sc[j][k] = 0.0;
        sh[j][k] = 0;
        if constexpr (SHIFT) sh[j][k] = static_cast<A>(p.shift[(size_t)b * ncp + vc[j][k] / sz]);
      }
  }
  const A a_inv_dt = static_cast<A>(p.inv_dt), a_inv_tau = static_cast<A>(inv_tau);
  // 1 under forward Euler, where the table's q holds the band's constant
  // rate, which a temperature-dependent one replaces
  const A a_expl = p.t.explicit_scheme ? A(1) : A(0);
  // Block faces.  x: lane l fetches the x-inflow value of register row
  // (l % RY, l / RY); y: one value per plane; z: one value per row.
  const int jl = min(lane % RY, max(nrows - 1, 0));
  const int kl = min((lane / RY) % RZ, max(nplanes - 1, 0));
  const int yel = min(y0 + jl, ny - 1);  // row and plane of the x edge this lane fetches
  const int ze = min(z0 + kl, nz - 1);
  const int last = min(63, nx - 1 - x0);   // last lane holding a mesh column
  const bool wall_l = x0 == 0;
  const bool wall_r = x0 + last == nx - 1;
  const int col_l = wall_l ? 0 : x0 - 1;
  const int col_r = wall_r ? nx - 1 : x0 + 64;
  const bool wall_yp = y0 == 0;
  const bool wall_yn = y0 + nrows >= ny;
  const int row_p = wall_yp ? 0 : min(y0 - 1, ny - 1);
  const int row_n = wall_yn ? ny - 1 : y0 + nrows;
  const bool wall_zp = z0 == 0;
  const bool wall_zn = z0 + nplanes >= nz;
  const int pl_p = wall_zp ? 0 : min(z0 - 1, nz - 1);
  const int pl_n = wall_zn ? nz - 1 : z0 + nplanes;
  const size_t sb = (size_t)b * ncp;
  A shx_l = 0, shx_r = 0, shy_p[RZ], shy_n[RZ], shz_p[RY], shz_n[RY];
#pragma unroll
  for (int k = 0; k < RZ; ++k) shy_p[k] = shy_n[k] = 0;
#pragma unroll
  for (int j = 0; j < RY; ++j) shz_p[j] = shz_n[j] = 0;
  if constexpr (SHIFT) {
    shx_l = static_cast<A>(p.shift[sb + ((size_t)ze * ny + yel) * nx + col_l]);
    shx_r = static_cast<A>(p.shift[sb + ((size_t)ze * ny + yel) * nx + col_r]);
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      shy_p[k] = static_cast<A>(p.shift[sb + ((size_t)zp[k] * ny + row_p) * nx + xcol]);
      shy_n[k] = static_cast<A>(p.shift[sb + ((size_t)zp[k] * ny + row_n) * nx + xcol]);
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      shz_p[j] = static_cast<A>(p.shift[sb + ((size_t)pl_p * ny + yr[j]) * nx + xcol]);
      shz_n[j] = static_cast<A>(p.shift[sb + ((size_t)pl_n * ny + yr[j]) * nx + xcol]);
    }
  }
  double num = 0.0, den = 0.0, wsum = 0.0;

  // With FP64 storage the slab values of direction d + 1 are requested (after
  // direction d's face loads) before direction d is computed (measured ~3 %
  // faster); with FP32 storage this measured slower, and each direction loads
  // its own values.
  constexpr bool kPrefetch = !Storage<Real>::kDeviation;
  Real rk_v[RY][RZ], rn_v[RY][RZ];
  auto load_block = [](const Real* slab_k, const Real* slab_n, int bytes,
                       const int (&off)[RY][RZ], Real (&k)[RY][RZ], Real (&n)[RY][RZ]) {
    const auto rk = slab_rsrc(slab_k, bytes);
    const auto rn = slab_rsrc(slab_n, bytes);
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int q = 0; q < RZ; ++q) {
        k[j][q] = buf_load_raw<Real>(rk, off[j][q]);
        n[j][q] = buf_load_step<Real>(rn, off[j][q]);
      }
  };
  if constexpr (kPrefetch)
    if (live && d_begin < d_end)
      load_block(Ikb + (size_t)d_begin * ncp, Inb + (size_t)d_begin * ncp, slab_bytes, vc, rk_v,
                 rn_v);
  for (int d = d_begin; d < d_end && live; ++d) {
    const Coef cf = cld_coef(p.t.coef, (size_t)b * g.nd + d);
    const int fl = cld(p.t.dflags, (size_t)d);
    const double wd = cld(p.t.w, (size_t)d);
    const bool xpos = dir_pos(fl, 0), xneg = dir_neg(fl, 0);
    const bool ypos = dir_pos(fl, 1), yneg = dir_neg(fl, 1);
    const bool zpos = dir_pos(fl, 2), zneg = dir_neg(fl, 2);
    const auto ro = slab_rsrc(Iob + (size_t)d * ncp, slab_bytes);
    if constexpr (!kPrefetch)
      load_block(Ikb + (size_t)d * ncp, Inb + (size_t)d * ncp, slab_bytes, vc, rk_v, rn_v);
    // x face
    const bool wx = xpos ? wall_l : wall_r;
    const int sx = xpos ? 0 : 1;
    const bool isox = wx && p.t.wall[sx] == 0;
    const int dxs = (wx && !isox) ? cld(p.t.mirror, (size_t)d) : d;
    const auto rxs = isox ? slab_rsrc(p.t.wall_S[sx], g.nb * p.t.wall_nf[sx] * sz)
                          : slab_rsrc(Ikb + (size_t)dxs * ncp, slab_bytes);
    const Real ex_r = buf_load_raw<Real>(
        rxs, isox ? (b * p.t.wall_nf[sx] + yel + ny * ze) * sz
                  : ((ze * ny + yel) * nx + (xpos ? col_l : col_r)) * sz);
    // y faces
    const bool wy = ypos ? wall_yp : wall_yn;
    const int sy = ypos ? 2 : 3;
    const bool isoy = wy && p.t.wall[sy] == 0;
    const int dys = (wy && !isoy) ? cld(p.t.mirror, (size_t)g.nd + d) : d;
    const auto rys = isoy ? slab_rsrc(p.t.wall_S[sy], g.nb * p.t.wall_nf[sy] * sz)
                          : slab_rsrc(Ikb + (size_t)dys * ncp, slab_bytes);
    const int row = ypos ? row_p : row_n;
    Real ey_r[RZ];
#pragma unroll
    for (int k = 0; k < RZ; ++k)
      ey_r[k] = buf_load_raw<Real>(rys, isoy ? (b * p.t.wall_nf[sy] + xcol + nx * zp[k]) * sz
                                             : ((zp[k] * ny + row) * nx + xcol) * sz);
    // z faces
    const bool wz = zpos ? wall_zp : wall_zn;
    const int sz_side = zpos ? 4 : 5;
    const bool isoz = wz && p.t.wall[sz_side] == 0;
    const int dzs = (wz && !isoz) ? cld(p.t.mirror, (size_t)2 * g.nd + d) : d;
    const auto rzs = isoz ? slab_rsrc(p.t.wall_S[sz_side], g.nb * p.t.wall_nf[sz_side] * sz)
                          : slab_rsrc(Ikb + (size_t)dzs * ncp, slab_bytes);
    const int plane = zpos ? pl_p : pl_n;
    Real ez_r[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j)
      ez_r[j] = buf_load_raw<Real>(rzs, isoz ? (b * p.t.wall_nf[sz_side] + xcol + nx * yr[j]) * sz
                                             : ((plane * ny + yr[j]) * nx + xcol) * sz);
    Real nk_v[RY][RZ], nn_v[RY][RZ];  // direction d + 1 (clamped)
    if constexpr (kPrefetch) {
      const int dn = min(d + 1, d_end - 1);
      load_block(Ikb + (size_t)dn * ncp, Inb + (size_t)dn * ncp, slab_bytes, vc, nk_v, nn_v);
    }
    A ex = ex_r;
    A ey[RZ], ez[RY];
#pragma unroll
    for (int k = 0; k < RZ; ++k) ey[k] = ey_r[k];
#pragma unroll
    for (int j = 0; j < RY; ++j) ez[j] = ez_r[j];
    if constexpr (SHIFT) {
      if (!isox) ex += xpos ? shx_l : shx_r;
#pragma unroll
      for (int k = 0; k < RZ; ++k)
        if (!isoy) ey[k] += ypos ? shy_p[k] : shy_n[k];
#pragma unroll
      for (int j = 0; j < RY; ++j)
        if (!isoz) ez[j] += zpos ? shz_p[j] : shz_n[j];
    }
    A ik[RY][RZ], in[RY][RZ];
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        ik[j][k] = rk_v[j][k];
        in[j][k] = rn_v[j][k];
        if constexpr (SHIFT) ik[j][k] += sh[j][k];
      }
    const A c0 = static_cast<A>(cf.c[0]), c1 = static_cast<A>(cf.c[1]);
    const A c2 = static_cast<A>(cf.c[2]), scale = static_cast<A>(cf.scale);
    wsum += wd;
    const int src_lane = xpos ? max(lane - 1, 0) : min(lane + 1, 63);
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        const A nbr = __shfl(ik[j][k], src_lane, 64);
        const A exjk = read_lane(ex, j + RY * k);
        if (colok && j < nrows && k < nplanes) {
          const A v = ik[j][k];
          const A rt = TAUT ? rate[j][k] : a_inv_tau;
          const A q =
              TAUT ? static_cast<A>(cf.q) + a_expl * (a_inv_tau - rt) : static_cast<A>(cf.q);
          A acc = update_start<Real>(in[j][k], I0r[j][k], v, q, a_inv_dt, rt);
          if (xpos) {
            const A up = lane == 0 ? exjk : nbr;
            acc = update_add<Real>(acc, c0, up, v);
          } else if (xneg) {
            const A up = lane == last ? exjk : nbr;
            acc = update_add<Real>(acc, c0, up, v);
          }
          if (ypos) {
            const A up = (j == 0) ? ey[k] : ik[j > 0 ? j - 1 : 0][k];
            acc = update_add<Real>(acc, c1, up, v);
          } else if (yneg) {
            const A up = (j == nrows - 1) ? ey[k] : ik[j + 1 < RY ? j + 1 : RY - 1][k];
            acc = update_add<Real>(acc, c1, up, v);
          }
          if (zpos) {
            const A up = (k == 0) ? ez[j] : ik[j][k > 0 ? k - 1 : 0];
            acc = update_add<Real>(acc, c2, up, v);
          } else if (zneg) {
            const A up = (k == nplanes - 1) ? ez[j] : ik[j][k + 1 < RZ ? k + 1 : RZ - 1];
            acc = update_add<Real>(acc, c2, up, v);
          }
          // the stored value drives the norms and the energy: once the
          // iterate stops changing in storage precision its increment is zero
          const A sc =
              TAUT ? cell_scale(cf, p.inv_dt, rate[j][k], p.t.explicit_scheme) : scale;
          const Real inew_r = update_finish<Real>(acc, v, sc);
          buf_store<Real>(inew_r, ro, vc[j][k], 0);
          const A inew = inew_r;
          const double da = static_cast<double>(inew - v);
          const double dn = static_cast<double>(inew - in[j][k]);
          accumulate_energy<Real>(S[j][k], Sc[j][k], wd, static_cast<double>(inew));
          num += wd * da * da;
          den += wd * dn * dn;
        }
      }
    if constexpr (kPrefetch) {
#pragma unroll
      for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int k = 0; k < RZ; ++k) {
          rk_v[j][k] = nk_v[j][k];
          rn_v[j][k] = nn_v[j][k];
        }
    }
  }
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int k = 0; k < RZ; ++k)
      if (colok && j < nrows && k < nplanes)
        p.S[((size_t)dg * g.nb + b) * ncp + vc[j][k] / sz] =
            energy_partial<Real>(S[j][k], Sc[j][k], iref, wsum);

  __shared__ double red[2][kSweepBlock / 64];
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) {
    red[0][wave] = num;
    red[1][wave] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kSweepBlock / 64; ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    const size_t blk = ((size_t)bz * gy + by) * gx + bx;
    p.part[2 * blk] = a;
    p.part[2 * blk + 1] = c;
  }
}

template <typename Real, int RY, int RZ, bool SHIFT, bool TAUT>
__global__ __launch_bounds__(kSweepBlock) void sweep3d_walk_kernel(const SweepParams<Real> p,
                                                                   const int ntx, const int nty,
                                                                   const int dgs) {
  if (step_done(p.ctl)) return;
  walk3d_body<Real, RY, RZ, SHIFT, TAUT>(p, ntx, nty, dgs, blockIdx.x, blockIdx.y, blockIdx.z,
                                   gridDim.x, gridDim.y);
}

// ---------------------------------------------------------------- 3D flattened walk
// For meshes whose x extent leaves many lanes of a 64-column tile idle (a
// narrow mesh, or a ragged last tile), the 256 lanes of a workgroup take 256
// consecutive cells f = x + nx y of the (x, y) plane instead, and each lane
// holds RZ planes of its cell in registers.  The z-upwind neighbour comes from
// registers (one load per block face plane).  For the x- and y-upwind
// neighbours the workgroup stages its tile's source values in LDS for every
// direction (two buffers alternating by direction, one barrier per
// direction): a neighbour inside the tile is read from there, and only the
// tile's halo (the row before its first or after its last cell, and the cell
// beyond either end) is loaded from memory.  Without the staging every wave
// loaded rows and edge cells that its neighbour waves load too; with no
// barrier between them the waves drift apart by several directions, and the
// second reads missed L2.  Lanes on an x or y wall take the ghost (isothermal
// equilibrium in storage format, or the cell's own intensity in the mirrored
// direction) from a load masked to them.
template <typename Real, int RZ, bool SHIFT, bool TAUT>
__device__ __forceinline__ void flat3d_body(const SweepParams<Real>& p, const int nft,
                                            const int dgs, const int bx, const int by,
                                            const int bz, const int gx, const int gy) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  using A = Arith<Real>;
  // staged in the arithmetic type (with the cell's shift, if any), so that a
  // neighbour needs no conversion
  using L = A;
  constexpr int sz = (int)sizeof(Real);
  constexpr int kTile = kSweepBlock;
  __shared__ L stage[2][RZ][kTile];
  const Geometry& g = p.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int nxy = nx * ny;
  const int tf = bx % nft;
  const int tz = bx / nft;
  const int b = by;
  const int dg = bz;
  const int li = threadIdx.x;            // the cell's place in the plane tile
  const int wave = __builtin_amdgcn_readfirstlane(li >> 6);
  const int t0 = tf * kTile;             // first plane cell of the tile
  const int f = t0 + li;
  const bool fok = f < nxy;
  const int fc = fok ? f : nxy - 1;      // a valid cell for every lane
  const int x = fc % nx;
  const int y = fc / nx;
  const int z0 = tz * RZ;
  const int nplanes = max(0, min(RZ, nz - z0));
  // the whole workgroup runs the direction loop (it holds the barriers);
  // waves whose cells all lie past the plane skip loads and updates
  const bool block_live = t0 < nxy && nplanes > 0;
  const bool live = t0 + wave * 64 < nxy && nplanes > 0;
  const int d_begin = dg * dgs;
  const int d_end = min(g.nd, d_begin + dgs);
  const size_t ncp = (size_t)g.ncp;
  const size_t band_off = (size_t)b * g.nd * ncp;
  const Real* __restrict__ Ikb = p.Ik + band_off;
  const Real* __restrict__ Inb = p.In + band_off;
  Real* __restrict__ Iob = p.Iout + band_off;
  const double inv_tau = cld(p.t.inv_tau, (size_t)b);
  const double iref = Storage<Real>::kDeviation ? cld(p.t.Iref, (size_t)b) : 0.0;
  const int slab_bytes = g.nc * sz;  // 3D slabs have no row padding (px = nx)
  // planes past the mesh reuse the last valid one (their values are never used)
  int zp[RZ], vc[RZ];
#pragma unroll
  for (int k = 0; k < RZ; ++k) {
    zp[k] = min(z0 + min(k, max(nplanes - 1, 0)), nz - 1);
    vc[k] = (zp[k] * nxy + fc) * sz;
  }
  // neighbour cells in the plane (clamped to the cell itself on a wall), and
  // whether they lie in this tile
  const int fy_p = y > 0 ? fc - nx : fc;
  const int fy_n = y < ny - 1 ? fc + nx : fc;
  const bool yin_p = fy_p >= t0;
  const bool yin_n = fy_n < t0 + kTile;
  // the tile's x ends: lane 0 takes the cell before the tile, lane 255 the
  // cell after it (the other lanes' value is never used)
  const int fe = li == 0 ? max(t0 - 1, 0) : min(t0 + kTile, nxy - 1);
  const bool xin_p = li > 0;
  const bool xin_n = li < kTile - 1;
  // z block faces
  const bool wall_zp = z0 == 0;
  const bool wall_zn = z0 + nplanes >= nz;
  const int pl_p = wall_zp ? 0 : z0 - 1;
  const int pl_n = wall_zn ? nz - 1 : z0 + nplanes;

  A I0r[RZ], sh[RZ], rate[RZ];
  double S[RZ], Sc[RZ];
  A shy_p[RZ], shy_n[RZ], shx[RZ];
  A shz_p = 0, shz_n = 0;
  {
    const auto r0 = slab_rsrc(p.I0 + (size_t)b * ncp, g.nc * 8);
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      I0r[k] = to_arith<Real>(iref, buf_load_raw<double>(r0, vc[k] / sz * 8));
      rate[k] = inv_tau;
      if constexpr (TAUT)
        rate[k] = buf_load_raw<double>(slab_rsrc(p.t.relax + (size_t)b * ncp, g.nc * 8),
                                       vc[k] / sz * 8);
      S[k] = 0.0;
      Sc[k] = 0.0;
      sh[k] = 0;
      shy_p[k] = 0;
      shy_n[k] = 0;
      shx[k] = 0;
    }
  }
  if constexpr (SHIFT) {
    const double* __restrict__ sb = p.shift + (size_t)b * ncp;
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      sh[k] = static_cast<A>(sb[(size_t)zp[k] * nxy + fc]);
      shy_p[k] = static_cast<A>(sb[(size_t)zp[k] * nxy + fy_p]);
      shy_n[k] = static_cast<A>(sb[(size_t)zp[k] * nxy + fy_n]);
      shx[k] = static_cast<A>(sb[(size_t)zp[k] * nxy + fe]);
    }
    shz_p = static_cast<A>(sb[(size_t)pl_p * nxy + fc]);
    shz_n = static_cast<A>(sb[(size_t)pl_n * nxy + fc]);
  }
  const A a_inv_dt = static_cast<A>(p.inv_dt), a_inv_tau = static_cast<A>(inv_tau);
  // 1 under forward Euler, where the table's q holds the band's constant
  // rate, which a temperature-dependent one replaces
  const A a_expl = p.t.explicit_scheme ? A(1) : A(0);
  double num = 0.0, den = 0.0, wsum = 0.0;

  for (int d = d_begin; d < d_end && block_live; ++d) {
    const Coef cf = cld_coef(p.t.coef, (size_t)b * g.nd + d);
    const int fl = cld(p.t.dflags, (size_t)d);
    const double wd = cld(p.t.w, (size_t)d);
    const bool xpos = dir_pos(fl, 0), xneg = dir_neg(fl, 0);
    const bool ypos = dir_pos(fl, 1), yneg = dir_neg(fl, 1);
    const bool zpos = dir_pos(fl, 2), zneg = dir_neg(fl, 2);
    const bool xw = (xpos && x == 0) || (xneg && x == nx - 1);
    const bool yw = (ypos && y == 0) || (yneg && y == ny - 1);
    const bool xin = xpos ? xin_p : xin_n;
    const bool yin = ypos ? yin_p : yin_n;
    const int fy = ypos ? fy_p : fy_n;
    L (&st)[RZ][kTile] = stage[d & 1];
    Real rk_v[RZ], rn_v[RZ], ey_r[RZ], ex_r[RZ];
    A xg[RZ], yg[RZ], ik[RZ], in[RZ];
    Real ez_r = 0;
    bool isoz = false;
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      ey_r[k] = ex_r[k] = 0;
      xg[k] = yg[k] = 0;
    }
    if (live) {
      const auto rk = slab_rsrc(Ikb + (size_t)d * ncp, slab_bytes);
      const auto rn = slab_rsrc(Inb + (size_t)d * ncp, slab_bytes);
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        rk_v[k] = buf_load_raw<Real>(rk, vc[k]);
        rn_v[k] = buf_load_step<Real>(rn, vc[k]);
      }
      // the halo: upwind cells outside the tile (masked to the lanes that
      // need them)
      if ((xpos || xneg) && !xin && !xw)
#pragma unroll
        for (int k = 0; k < RZ; ++k) ex_r[k] = buf_load_raw<Real>(rk, (zp[k] * nxy + fe) * sz);
      if ((ypos || yneg) && !yin && !yw)
#pragma unroll
        for (int k = 0; k < RZ; ++k) ey_r[k] = buf_load_raw<Real>(rk, (zp[k] * nxy + fy) * sz);
      // z face: the neighbouring block's plane, or on a wall (wave-uniform)
      // the isothermal equilibrium or this plane's cell in the mirrored
      // direction
      const bool wz = zpos ? wall_zp : wall_zn;
      const int fz = zpos ? 4 : 5;
      isoz = wz && p.t.wall[fz] == 0;
      const int dzs = (wz && !isoz) ? cld(p.t.mirror, (size_t)2 * g.nd + d) : d;
      const auto rzs = isoz ? slab_rsrc(p.t.wall_S[fz], g.nb * p.t.wall_nf[fz] * sz)
                            : slab_rsrc(Ikb + (size_t)dzs * ncp, slab_bytes);
      ez_r = buf_load_raw<Real>(rzs, isoz ? (b * p.t.wall_nf[fz] + fc) * sz
                                          : ((zpos ? pl_p : pl_n) * nxy + fc) * sz);
      // x and y walls: lanes on a wall load their ghosts (masked to them)
      if (xw) {
        const int fx = xpos ? 0 : 1;
        const bool iso = p.t.wall[fx] == 0;
        const auto r = iso ? slab_rsrc(p.t.wall_S[fx], g.nb * p.t.wall_nf[fx] * sz)
                           : slab_rsrc(Ikb + (size_t)cld(p.t.mirror, (size_t)d) * ncp, slab_bytes);
#pragma unroll
        for (int k = 0; k < RZ; ++k)
          xg[k] = buf_load_raw<Real>(r, iso ? (b * p.t.wall_nf[fx] + y + ny * zp[k]) * sz : vc[k]);
        if constexpr (SHIFT)
          if (!iso)
#pragma unroll
            for (int k = 0; k < RZ; ++k) xg[k] += sh[k];
      }
      if (yw) {
        const int fyw = ypos ? 2 : 3;
        const bool iso = p.t.wall[fyw] == 0;
        const auto r = iso ? slab_rsrc(p.t.wall_S[fyw], g.nb * p.t.wall_nf[fyw] * sz)
                           : slab_rsrc(Ikb + (size_t)cld(p.t.mirror, (size_t)g.nd + d) * ncp,
                                       slab_bytes);
#pragma unroll
        for (int k = 0; k < RZ; ++k)
          yg[k] = buf_load_raw<Real>(r, iso ? (b * p.t.wall_nf[fyw] + x + nx * zp[k]) * sz : vc[k]);
        if constexpr (SHIFT)
          if (!iso)
#pragma unroll
            for (int k = 0; k < RZ; ++k) yg[k] += sh[k];
      }
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        ik[k] = rk_v[k];
        in[k] = rn_v[k];
        if constexpr (SHIFT) ik[k] += sh[k];
        st[k][li] = ik[k];
      }
    }
    // the buffer written here was last read two directions ago, before every
    // wave passed the previous direction's barrier.  The marker names this
    // barrier in the assembly, where a static check allows it (alone) one
    // loop level deeper than the kernel's other barriers.
    asm volatile("; bte: direction-loop barrier" ::: "memory");
    __syncthreads();
    if (!live) continue;
    A ez = ez_r;
    if constexpr (SHIFT)
      if (!isoz) ez += zpos ? shz_p : shz_n;
    const A c0 = static_cast<A>(cf.c[0]), c1 = static_cast<A>(cf.c[1]);
    const A c2 = static_cast<A>(cf.c[2]), scale = static_cast<A>(cf.scale);
    wsum += wd;
    const int lx = xpos ? li - 1 : li + 1;
    const int ly = fy - t0;
    const auto ro = slab_rsrc(Iob + (size_t)d * ncp, slab_bytes);
    // lanes past the plane run the update on a valid cell's values too; their
    // store goes past the end of the slab (dropped) and their weight is 0
    const double wf = fok ? wd : 0.0;
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      if (k < nplanes) {
        const A v = ik[k];
        const A rt = TAUT ? rate[k] : a_inv_tau;
        const A q = TAUT ? static_cast<A>(cf.q) + a_expl * (a_inv_tau - rt) : static_cast<A>(cf.q);
        A acc = update_start<Real>(in[k], I0r[k], v, q, a_inv_dt, rt);
        if (xpos || xneg) {
          A up;
          if (xw) {
            up = xg[k];
          } else if (xin) {
            up = st[k][lx];
          } else {
            up = ex_r[k];
            if constexpr (SHIFT) up += shx[k];
          }
          acc = update_add<Real>(acc, c0, up, v);
        }
        if (ypos || yneg) {
          A up;
          if (yw) {
            up = yg[k];
          } else if (yin) {
            up = st[k][ly];
          } else {
            up = ey_r[k];
            if constexpr (SHIFT) up += ypos ? shy_p[k] : shy_n[k];
          }
          acc = update_add<Real>(acc, c1, up, v);
        }
        if (zpos) {
          const A up = (k == 0) ? ez : ik[k > 0 ? k - 1 : 0];
          acc = update_add<Real>(acc, c2, up, v);
        } else if (zneg) {
          const A up = (k == nplanes - 1) ? ez : ik[k + 1 < RZ ? k + 1 : RZ - 1];
          acc = update_add<Real>(acc, c2, up, v);
        }
        // the stored value drives the norms and the energy: once the
        // iterate stops changing in storage precision its increment is zero
        const A sc = TAUT ? cell_scale(cf, p.inv_dt, rate[k], p.t.explicit_scheme) : scale;
        const Real inew_r = update_finish<Real>(acc, v, sc);
        buf_store<Real>(inew_r, ro, fok ? vc[k] : kPastEnd, 0);
        const A inew = inew_r;
        const double da = static_cast<double>(inew - v);
        const double dn = static_cast<double>(inew - in[k]);
        accumulate_energy<Real>(S[k], Sc[k], wf, static_cast<double>(inew));
        num += wf * da * da;
        den += wf * dn * dn;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RZ; ++k)
    if (live && fok && k < nplanes)
      p.S[((size_t)dg * g.nb + b) * ncp + vc[k] / sz] =
          energy_partial<Real>(S[k], Sc[k], iref, wsum);

  const int lane = li & 63;
  __shared__ double red[2][kSweepBlock / 64];
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) {
    red[0][wave] = num;
    red[1][wave] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < kSweepBlock / 64; ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    const size_t blk = ((size_t)bz * gy + by) * gx + bx;
    p.part[2 * blk] = a;
    p.part[2 * blk + 1] = c;
  }
}

template <typename Real, int RZ, bool SHIFT, bool TAUT>
__global__ __launch_bounds__(kSweepBlock) void sweep3d_flat_kernel(const SweepParams<Real> p,
                                                                   const int nft, const int dgs) {
  if (step_done(p.ctl)) return;
  // Workgroups go to the eight XCDs in turn, and each XCD has its own L2.  A
  // plane tile reads the row before its first and after its last cell from
  // the neighbouring tiles, so when the tile count divides by eight, each XCD
  // is given a contiguous range of tiles (neighbours then share an L2).  The
  // partials stay indexed by tile, so results do not change.
  int bx = blockIdx.x;
  if ((gridDim.x & 7) == 0) {
    const int per_xcd = gridDim.x >> 3;
    bx = (bx & 7) * per_xcd + (bx >> 3);
  }
  flat3d_body<Real, RZ, SHIFT, TAUT>(p, nft, dgs, bx, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y);
}

template <typename Real, bool SHIFT, bool TAUT>
static void launch_sweep_t(hipStream_t stream, const SweepPlan& plan, const SweepParams<Real>& p) {
  const Geometry& g = p.g;
  if (plan.kind == kSweepColumnWalk2D) {
    const dim3 grid(plan.ntiles, g.nb, plan.ndg);
    switch (plan.ry) {
      case 4:
        hipLaunchKernelGGL((sweep2d_walk_kernel<Real, 4, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                           stream, p, plan.ntx, plan.dgs);
        break;
      case 8:
        hipLaunchKernelGGL((sweep2d_walk_kernel<Real, 8, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                           stream, p, plan.ntx, plan.dgs);
        break;
      default:
        hipLaunchKernelGGL((sweep2d_walk_kernel<Real, 16, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                           stream, p, plan.ntx, plan.dgs);
        break;
    }
    return;
  }
  if (plan.kind == kSweepFlat3D) {
    const dim3 grid(plan.ntiles, g.nb, plan.ndg);
    if (plan.rz == 2)
      hipLaunchKernelGGL((sweep3d_flat_kernel<Real, 2, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                         stream, p, plan.ntx, plan.dgs);
    else
      hipLaunchKernelGGL((sweep3d_flat_kernel<Real, 4, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                         stream, p, plan.ntx, plan.dgs);
    return;
  }
  if (plan.kind == kSweepColumnWalk3D) {
    const dim3 grid(plan.ntiles, g.nb, plan.ndg);
    if (plan.rz == 4 && plan.ry == 1)
      hipLaunchKernelGGL((sweep3d_walk_kernel<Real, 1, 4, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                         stream, p, plan.ntx, plan.nty, plan.dgs);
    else if (plan.rz == 4)
      hipLaunchKernelGGL((sweep3d_walk_kernel<Real, 2, 4, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                         stream, p, plan.ntx, plan.nty, plan.dgs);
    else
      hipLaunchKernelGGL((sweep3d_walk_kernel<Real, 2, 2, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0,
                         stream, p, plan.ntx, plan.nty, plan.dgs);
    return;
  }
  const dim3 grid(plan.ntiles, g.nb);
  if (g.dim == 3)
    hipLaunchKernelGGL((sweep_kernel<Real, 3, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0, stream, p);
  else
    hipLaunchKernelGGL((sweep_kernel<Real, 2, SHIFT, TAUT>), grid, dim3(kSweepBlock), 0, stream, p);
}

template <typename Real>
hipError_t launch_sweep(hipStream_t stream, const Geometry& g, const Tables& t,
                        const SweepPlan& plan, double inv_dt, const Real* Ik, const Real* In,
                        Real* Iout, const double* I0, double* S, double* part,
                        const Control* ctl, const double* shift) {
  const SweepParams<Real> p{g, t, Ik, In, Iout, I0, S, part, ctl, inv_dt, shift};
  if (t.relax) {
    if (shift) launch_sweep_t<Real, true, true>(stream, plan, p);
    else launch_sweep_t<Real, false, true>(stream, plan, p);
  } else {
    if (shift) launch_sweep_t<Real, true, false>(stream, plan, p);
    else launch_sweep_t<Real, false, false>(stream, plan, p);
  }
  return hipGetLastError();
}

template hipError_t launch_sweep<double>(hipStream_t, const Geometry&, const Tables&,
                                         const SweepPlan&, double, const double*, const double*,
                                         double*, const double*, double*, double*,
                                         const Control*, const double*);
template hipError_t launch_sweep<float>(hipStream_t, const Geometry&, const Tables&,
                                        const SweepPlan&, double, const float*, const float*,
                                        float*, const double*, double*, double*, const Control*,
                                        const double*);

// ---------------------------------------------------------------- temperature
// Each cell is handled by LANES lanes of one wavefront (temp_lanes); lane l of a
// cell owns the bands b = l, l + L, l + 2L, ...  Sums over bands are completed
// with an xor butterfly inside the lane group and the group's first lane's
// total is then broadcast, so every lane of the group holds bit-identical
// values (whatever the compiler fuses into the butterfly) and the group's
// Newton iterations stay in lockstep.
template <int LANES>
__device__ __forceinline__ double group_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int m = 1; m < LANES; m <<= 1) v += __shfl_xor(v, m, 64);
  if (LANES > 1) {
    const int lane = threadIdx.x & 63;
    v = __shfl(v, lane & ~(LANES - 1), 64);
  }
  return v;
}

// Partial F(T) = W sum_b f_b I0_b(T) and dF/dT over this lane's bands; f_b is
// 1/tau_b (relaxation-time weighted) or 1 (plain energy).
template <int LANES>
__device__ __forceinline__ void relation_part(const Tables& t, int nb, int l, double T, double& F,
                                              double& dF) {
#pragma clang fp contract(off)
  double f = 0.0, df = 0.0;
  // unrolled by 2, not 4: with constant relaxation times the inversion then
  // fits 94 VGPRs, 5 waves per SIMD instead of 4 (the batched inversion of
  // the 64-geometry draw measured 18 % less time)
#pragma unroll 2
  for (int b = l; b < nb; b += LANES) {
    const double x = t.xfac[b] / T;
    const double em1 = expm1(x);
    const double i0 = t.Cb[b] / em1;
    f += t.fweight[b] * i0;
    df += t.fweight[b] * i0 * (x / T) * (em1 + 1.0) / em1;
  }
  F = t.W * f;
  dF = t.W * df;
}

// With temperature-dependent relaxation times: partial sums over this lane's
// bands of N(T) = W sum_b I0_b(T) / tau_b(T), D(T) = sum_b e_b / tau_b(T)
// and their T-derivatives (d/dT 1/tau_b(T) = p_b / (T tau_b(T))); e_b is read
// from E0[b * stride].
template <int LANES>
__device__ __forceinline__ void relation_part_tau(const Tables& t, int nb, int l, double T,
                                                  const double* E0, size_t stride, double& N,
                                                  double& dN, double& D, double& dD) {
#pragma clang fp contract(off)
  double n = 0.0, dn = 0.0, d = 0.0, dd = 0.0;
  for (int b = l; b < nb; b += LANES) {
    const double r = relax_rate(t.inv_tau[b], t.tau_p[b], T, t.tau_T0);
    const double dr = t.tau_p[b] / T * r;
    const double x = t.xfac[b] / T;
    const double em1 = expm1(x);
    const double i0 = t.Cb[b] / em1;
    const double di0 = i0 * (x / T) * (em1 + 1.0) / em1;
    const double e = E0[(size_t)b * stride];
    n += r * i0;
    dn += dr * i0 + r * di0;
    d += r * e;
    dd += dr * e;
  }
  N = t.W * n;
  dN = t.W * dn;
  D = d;
  dD = dd;
}

// Per cell: finalise the energy sums from the per-(direction group, band)
// partials, invert the temperature relation by Newton from the current T
// (accept-first, quadratic convergence; Sec. 2.2 and Sec. 3.2 temperature
// update), then refresh the equilibrium intensities I0[b][P] for the next sweep.
// TAUT: relaxation times depend on T (their Newton relation and rate refresh
// take registers that would cost the constant-tau kernel a wave per SIMD).
template <int LANES, bool TAUT>
__device__ __forceinline__ void temperature_body(const Geometry& g, const Tables& t,
                                                 double* __restrict__ S,
                                                 double* __restrict__ T, double* __restrict__ I0,
                                                 double* __restrict__ E, Control* ctl,
                                                 const int bx) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  const int l = threadIdx.x % LANES;
  const int P = bx * (256 / LANES) + threadIdx.x / LANES;
  const bool active = P < g.nc;
  const int Pc = active ? P : 0;
  const size_t ncp = (size_t)g.ncp;
  const bool tau_newton = TAUT && t.tau_weighted;
  CompSum Gs, Es;
  if (active) {
    // The partials of up to kChunk of this lane's bands are requested
    // together for each direction group, so their loads are in flight at
    // once; each band still sums its groups in order, and the bands enter
    // G and E in order.
    constexpr int kChunk = 4;
    const size_t qstride = (size_t)g.nb * ncp;
    for (int b0 = l; b0 < g.nb; b0 += LANES * kChunk) {
      CompSum s[kChunk];
      for (int q = 0; q < g.ndg; ++q) {
        double v[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
          const int b = b0 + i * LANES;
          v[i] = b < g.nb ? S[(size_t)q * qstride + (size_t)b * ncp + Pc] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kChunk; ++i) s[i].add(v[i]);
      }
#pragma unroll
      for (int i = 0; i < kChunk; ++i) {
        const int b = b0 + i * LANES;
        if (b < g.nb) {
          Gs.add(t.fweight[b] * s[i].value());
          Es.add(s[i].value());
          // temperature-dependent weights: the Newton iterations below re-read
          // each band's sum, kept in the first group's partial (the next
          // sweep rewrites it)
          if (tau_newton) S[(size_t)b * ncp + Pc] = s[i].value();
        }
      }
    }
  }
  const double Gp = Gs.value(), Ep = Es.value();
  const double G = group_sum<LANES>(Gp);
  const double En = group_sum<LANES>(Ep);
  double Tc = T[Pc];
  int it = 0;
  bool ok = (G > 0.0) && isfinite(G) && (Tc > 0.0);
  if (tau_newton) {
    // The relaxation-time-weighted temperature with tau_b(T): the root of
    // K(T) = N(T) / D(T) - 1 (Newton, accept-first, same stopping rule).
    ok = Tc > 0.0;
    const double* E0 = S + Pc;
    for (int k = 0; ok; ++k) {
      double Np, dNp, Dp, dDp;
      relation_part_tau<LANES>(t, g.nb, l, Tc, E0, ncp, Np, dNp, Dp, dDp);
      const double N = group_sum<LANES>(Np), dN = group_sum<LANES>(dNp);
      const double D = group_sum<LANES>(Dp), dD = group_sum<LANES>(dDp);
      if (!(D > 0.0) || !isfinite(D)) {
        ok = false;
        break;
      }
      const double K = N / D - 1.0;
      if (k == 0 && fabs(K) <= kNewtonAcceptRel) break;
      if (k == kNewtonMaxIters) {
        ok = false;
        break;
      }
      const double dT = K / ((dN * D - N * dD) / (D * D));
      Tc -= dT;
      it = k + 1;
      if (!isfinite(Tc) || !(Tc > 0.0)) {
        ok = false;
        break;
      }
      if (fabs(dT) <= kNewtonStepRel * Tc) break;
    }
  } else if (ok) {
    double Fp, dFp;
    relation_part<LANES>(t, g.nb, l, Tc, Fp, dFp);
    double F = group_sum<LANES>(Fp), dF = group_sum<LANES>(dFp);
    if (fabs(F - G) > kNewtonAcceptRel * G) {
      ok = false;
      for (it = 1; it <= kNewtonMaxIters; ++it) {
        const double dT = (F - G) / dF;
        Tc -= dT;
        if (!isfinite(Tc) || !(Tc > 0.0)) break;
        if (fabs(dT) <= kNewtonStepRel * Tc) {
          ok = true;
          break;
        }
        relation_part<LANES>(t, g.nb, l, Tc, Fp, dFp);
        F = group_sum<LANES>(Fp);
        dF = group_sum<LANES>(dFp);
      }
    }
  }
  // The step's largest Newton count, one atomic per wave: one per cell put
  // millions of atomics on one address per iteration and doubled the
  // batched inversion's time once the warm start made every cell iterate.
  // Every lane of the wave is active here.
  int itw = (active && ok) ? it : 0;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) itw = max(itw, __shfl_xor(itw, m, 64));
  if ((threadIdx.x & 63) == 0 && itw > 0) atomicMax(&ctl->newton_max, itw);
  if (!active) return;
  if (!ok) {
    if (l == 0) atomicMin(&ctl->err_cell, P);
    return;
  }
#pragma unroll 2
  for (int b = l; b < g.nb; b += LANES)
    I0[(size_t)b * ncp + P] = equilibrium(t.Cb[b], t.xfac[b], Tc);
  if constexpr (TAUT)
    for (int b = l; b < g.nb; b += LANES)
      t.relax[(size_t)b * ncp + P] = relax_rate(t.inv_tau[b], t.tau_p[b], Tc, t.tau_T0);
  if (l == 0) {
    T[P] = Tc;
    E[P] = En;
  }
}

template <int LANES, bool TAUT>
__global__ __launch_bounds__(256) void temperature_kernel(Geometry g, Tables t,
                                                          double* __restrict__ S,
                                                          double* __restrict__ T,
                                                          double* __restrict__ I0,
                                                          double* __restrict__ E, Control* ctl) {
  if (step_done(ctl)) return;
  temperature_body<LANES, TAUT>(g, t, S, T, I0, E, ctl, blockIdx.x);
}

hipError_t launch_temperature(hipStream_t stream, const Geometry& g, const Tables& t,
                              double* S, double* T, double* I0, double* E, Control* ctl) {
  const int cells_per_block = temp_cells_per_block(g.nb);
  const dim3 grid((g.nc + cells_per_block - 1) / cells_per_block);
  const bool four = temp_lanes(g.nb) == 4;
  if (t.relax)
    hipLaunchKernelGGL((four ? temperature_kernel<4, true> : temperature_kernel<8, true>), grid,
                       dim3(256), 0, stream, g, t, S, T, I0, E, ctl);
  else
    hipLaunchKernelGGL((four ? temperature_kernel<4, false> : temperature_kernel<8, false>), grid,
                       dim3(256), 0, stream, g, t, S, T, I0, E, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- control
// Sums the per-block norm partials in a fixed order, forms the step-relative
// increment norm res = ||I^{k+1}-I^k|| / ||I^{k+1}-I^n|| (0/0 -> 0) and decides
// whether the inner loop is finished; later kernels of the step then return
// immediately.
__device__ __forceinline__ void control_body(int nparts, const double* __restrict__ part,
                                             double vol, int fixed_k, int max_inner, double tol,
                                             int explicit_mode, Control* ctl) {
#pragma clang fp contract(on)  // fuse a*b+c only within one expression
  __shared__ double sn[kReduceBlock];
  __shared__ double sd[kReduceBlock];
  double n = 0.0, d = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kReduceBlock) {
    n += part[2 * i];
    d += part[2 * i + 1];
  }
  sn[threadIdx.x] = n;
  sd[threadIdx.x] = d;
  __syncthreads();
  for (int s = kReduceBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sn[threadIdx.x] += sn[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double num = sn[0] * vol;
    const double den = sd[0] * vol;
    const double res = (num == 0.0) ? 0.0 : (den == 0.0 ? INFINITY : sqrt(num / den));
    const int k = ctl->k + 1;
    int done;
    if (explicit_mode) done = 1;
    else if (fixed_k > 0) done = (k >= fixed_k);
    else done = (res <= tol) || (k >= max_inner);
    if (ctl->err_cell != INT_MAX) done = 1;
    ctl->k = k;
    ctl->res = res;
    ctl->num = num;
    ctl->den = den;
    ctl->converged = done;
  }
}

__global__ __launch_bounds__(kReduceBlock) void control_kernel(int nparts,
                                                               const double* __restrict__ part,
                                                               double vol, int fixed_k,
                                                               int max_inner, double tol,
                                                               int explicit_mode, Control* ctl) {
  if (step_done(ctl)) return;
  control_body(nparts, part, vol, fixed_k, max_inner, tol, explicit_mode, ctl);
}

hipError_t launch_control(hipStream_t stream, int nparts, const double* part, double vol,
                          int fixed_k, int max_inner, double tol, int explicit_mode,
                          Control* ctl) {
  hipLaunchKernelGGL(control_kernel, dim3(1), dim3(kReduceBlock), 0, stream, nparts, part, vol,
                     fixed_k, max_inner, tol, explicit_mode, ctl);
  return hipGetLastError();
}

__global__ void reset_kernel(Control* ctl) {
  if (threadIdx.x == 0) {
    ctl->converged = 0;
    ctl->k = 0;
    ctl->newton_max = 0;
    ctl->err_cell = INT_MAX;
    ctl->res = 0.0;
    ctl->num = 0.0;
    ctl->den = 0.0;
  }
}

hipError_t launch_reset(hipStream_t stream, Control* ctl) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- set-up kernels
// I0[b][P] = I0_b(T_P) and E_P = W sum_b I0_b(T_P) (an equilibrium state).
__global__ __launch_bounds__(kCellBlock) void equilibrium_kernel(Geometry g, Tables t,
                                                                 const double* __restrict__ T,
                                                                 double* __restrict__ I0,
                                                                 double* __restrict__ E) {
  const int P = blockIdx.x * kCellBlock + threadIdx.x;
  if (P >= g.nc) return;
  const double Tc = T[P];
  double sum = 0.0;
  for (int b = 0; b < g.nb; ++b) {
    const double v = equilibrium(t.Cb[b], t.xfac[b], Tc);
    I0[(size_t)b * g.ncp + P] = v;
    sum += v;
    if (t.relax) t.relax[(size_t)b * g.ncp + P] = relax_rate(t.inv_tau[b], t.tau_p[b], Tc, t.tau_T0);
  }
  if (E) E[P] = t.W * sum;
}

hipError_t launch_equilibrium(hipStream_t stream, const Geometry& g, const Tables& t,
                              const double* T, double* I0, double* E) {
  const dim3 grid((g.nc + kCellBlock - 1) / kCellBlock);
  hipLaunchKernelGGL(equilibrium_kernel, grid, dim3(kCellBlock), 0, stream, g, t, T, I0, E);
  return hipGetLastError();
}

// Diffuse wall: per (face, band), the outgoing flux-weighted mean of the wall
// cell's intensities at the current iterate, as a ghost table in FP64 and in
// storage format (the sweeps read it like an isothermal wall's).  FP32
// storage sums the deviations, so the reference is added once.
template <typename Real>
__global__ void diffuse_wall_kernel(Geometry g, Tables t, int side, const double* __restrict__ wts,
                                    const Real* __restrict__ I, const double* __restrict__ shift,
                                    double* __restrict__ wall_I0, Real* __restrict__ wall_S) {
  const int nf = t.wall_nf[side];
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (f >= nf) return;
  const int axis = side / 2, plus = side % 2;
  int x, y, z;
  if (axis == 0) {
    x = plus ? g.nx - 1 : 0;
    y = f % g.ny;
    z = f / g.ny;
  } else if (axis == 1) {
    y = plus ? g.ny - 1 : 0;
    x = f % g.nx;
    z = f / g.nx;
  } else {
    z = plus ? g.nz - 1 : 0;
    x = f % g.nx;
    y = f / g.nx;
  }
  const size_t P = (size_t)x + (size_t)g.nx * (y + (size_t)g.ny * z);
  const size_t ncp = (size_t)g.ncp;
  const double ref = Storage<Real>::kDeviation ? t.Iref[b] : 0.0;
  double dev = 0.0;
  for (int d = 0; d < g.nd; ++d) {
    const double wd = wts[d];
    if (wd > 0.0) dev += wd * static_cast<double>(I[((size_t)b * g.nd + d) * ncp + ipos(g, P)]);
  }
  if (shift) dev += shift[(size_t)b * ncp + P];
  wall_I0[(size_t)b * nf + f] = ref + dev;
  wall_S[(size_t)b * nf + f] = Storage<Real>::kDeviation ? static_cast<Real>(dev)
                                                         : static_cast<Real>(ref + dev);
}

template <typename Real>
hipError_t launch_diffuse_wall(hipStream_t stream, const Geometry& g, const Tables& t, int side,
                               const double* wts, const Real* I, const double* shift,
                               double* wall_I0, Real* wall_S) {
  const dim3 grid((t.wall_nf[side] + 63) / 64, g.nb);
  hipLaunchKernelGGL((diffuse_wall_kernel<Real>), grid, dim3(64), 0, stream, g, t, side, wts, I,
                     shift, wall_I0, wall_S);
  return hipGetLastError();
}
template hipError_t launch_diffuse_wall<double>(hipStream_t, const Geometry&, const Tables&, int,
                                                const double*, const double*, const double*,
                                                double*, double*);
template hipError_t launch_diffuse_wall<float>(hipStream_t, const Geometry&, const Tables&, int,
                                               const double*, const float*, const double*,
                                               double*, float*);

// Equilibrium intensity of every face of an isothermal wall, [b][face].
__global__ void wall_table_kernel(int nb, int nf, const double* __restrict__ Cb,
                                  const double* __restrict__ xfac,
                                  const double* __restrict__ wallT, double* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double Tw = wallT[f];
  for (int b = 0; b < nb; ++b) out[(size_t)b * nf + f] = equilibrium(Cb[b], xfac[b], Tw);
}

hipError_t launch_wall_table(hipStream_t stream, int nb, int nf, const double* Cb,
                             const double* xfac, const double* wallT, double* out) {
  hipLaunchKernelGGL(wall_table_kernel, dim3((nf + 255) / 256), dim3(256), 0, stream, nb, nf, Cb,
                     xfac, wallT, out);
  return hipGetLastError();
}

template <typename Real>
__global__ void wall_storage_kernel(int n, int nf, const double* __restrict__ in,
                                    const double* __restrict__ Iref, Real* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = encode<Real>(Storage<Real>::kDeviation ? Iref[i / nf] : 0.0, in[i]);
}

template <typename Real>
hipError_t launch_wall_storage(hipStream_t stream, int nb, int nf, const double* in,
                               const double* Iref, Real* out) {
  const int n = nb * nf;
  hipLaunchKernelGGL((wall_storage_kernel<Real>), dim3((n + 255) / 256), dim3(256), 0, stream, n,
                     nf, in, Iref, out);
  return hipGetLastError();
}
template hipError_t launch_wall_storage<double>(hipStream_t, int, int, const double*,
                                                const double*, double*);
template hipError_t launch_wall_storage<float>(hipStream_t, int, int, const double*,
                                               const double*, float*);

// I[b][d][P] = I0[b][P] for every direction (isotropic equilibrium); padding zeroed.
template <typename Real>
__global__ __launch_bounds__(256) void broadcast_kernel(Geometry g, const double* __restrict__ I0,
                                                        const double* __restrict__ Iref,
                                                        Real* __restrict__ I) {
  const int Q = blockIdx.x * 256 + threadIdx.x;  // position in the slab
  const int d = blockIdx.y;
  const int b = blockIdx.z;
  if (Q >= g.ncp) return;
  const int x = Q % g.px, r = Q / g.px;  // column and row (y + ny z)
  const bool cell = x < g.nx && r < g.ny * g.nz;
  const double ref = Storage<Real>::kDeviation ? Iref[b] : 0.0;
  I[((size_t)b * g.nd + d) * g.ncp + Q] =
      cell ? encode<Real>(ref, I0[(size_t)b * g.ncp + (size_t)r * g.nx + x])
           : static_cast<Real>(0);
}

template <typename Real>
hipError_t launch_broadcast(hipStream_t stream, const Geometry& g, const Tables& t,
                            const double* I0, Real* I) {
  const dim3 grid((g.ncp + 255) / 256, g.nd, g.nb);
  hipLaunchKernelGGL((broadcast_kernel<Real>), grid, dim3(256), 0, stream, g, I0, t.Iref, I);
  return hipGetLastError();
}

template hipError_t launch_broadcast<double>(hipStream_t, const Geometry&, const Tables&,
                                             const double*, double*);
template hipError_t launch_broadcast<float>(hipStream_t, const Geometry&, const Tables&,
                                            const double*, float*);

__global__ void reference_kernel(int nb, const double* __restrict__ Cb,
                                 const double* __restrict__ xfac, double T_ref,
                                 double* __restrict__ Iref) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  Iref[b] = (T_ref > 0.0) ? equilibrium(Cb[b], xfac[b], T_ref) : 0.0;
}

hipError_t launch_reference(hipStream_t stream, int nb, const double* Cb, const double* xfac,
                            double T_ref, double* Iref) {
  hipLaunchKernelGGL(reference_kernel, dim3((nb + 63) / 64), dim3(64), 0, stream, nb, Cb, xfac,
                     T_ref, Iref);
  return hipGetLastError();
}

// E_P = sum_b sum_d w_d I[b][d][P] (band outer, direction inner).
template <typename Real>
__global__ __launch_bounds__(kCellBlock) void energy_kernel(Geometry g, Tables t,
                                                            const Real* __restrict__ I,
                                                            double* __restrict__ E) {
  const int P = blockIdx.x * kCellBlock + threadIdx.x;
  if (P >= g.nc) return;
  const size_t Q = ipos(g, P);
  CompSum e;
  for (int b = 0; b < g.nb; ++b) {
    const double ref = Storage<Real>::kDeviation ? t.Iref[b] : 0.0;
    CompSum s;
    for (int d = 0; d < g.nd; ++d)
      s.add(t.w[d] * decode(ref, I[((size_t)b * g.nd + d) * g.ncp + Q]));
    e.add(s.value());
  }
  E[P] = e.value();
}

template <typename Real>
hipError_t launch_energy(hipStream_t stream, const Geometry& g, const Tables& t, const Real* I,
                         double* E) {
  const dim3 grid((g.nc + kCellBlock - 1) / kCellBlock);
  hipLaunchKernelGGL((energy_kernel<Real>), grid, dim3(kCellBlock), 0, stream, g, t, I, E);
  return hipGetLastError();
}

template hipError_t launch_energy<double>(hipStream_t, const Geometry&, const Tables&,
                                          const double*, double*);
template hipError_t launch_energy<float>(hipStream_t, const Geometry&, const Tables&,
                                         const float*, double*);

}  // namespace bte

namespace bte {

// ---------------------------------------------------------------- batched
template <typename Real>
__device__ __forceinline__ const SweepParams<Real>& batch_params(const BatchCtx& c);
template <>
__device__ __forceinline__ const SweepParams<double>& batch_params<double>(const BatchCtx& c) {
  return c.sp64;
}
template <>
__device__ __forceinline__ const SweepParams<float>& batch_params<float>(const BatchCtx& c) {
  return c.sp32;
}

// One work item of a batched sweep.  The geometry's parameters live in device
// memory (the source / destination iterates are rewritten there after every
// iteration), and batches seed warm starts through the temperature only (no
// intensity shift).  LIST is the work list: 2D with 4 rows per wave; 3D with
// 2 rows x 2 planes or 1 row x 4 planes per wave or the flattened (x, y)
// plane with 2 planes per wave, chosen per geometry (none of them raises the
// kernel's register count above the 2 x 2 walk's); or the flattened plane
// with 4 planes per wave.
template <typename Real, int LIST>
__device__ __forceinline__ void batch_item(const BatchCtx& c, const BatchItem& w) {
  const SweepParams<Real>& p = batch_params<Real>(c);
  const SweepPlan& pl = c.plan;
  if constexpr (LIST == kList2D)
    walk2d_body<Real, 4, false, false>(p, pl.ntx, pl.dgs, w.bx, w.by, w.bz, pl.ntiles, p.g.nb);
  else if constexpr (LIST == kListFlat4)
    flat3d_body<Real, 4, false, false>(p, pl.ntx, pl.dgs, w.bx, w.by, w.bz, pl.ntiles, p.g.nb);
  else if (__builtin_amdgcn_readfirstlane(pl.kind) == kSweepFlat3D)
    flat3d_body<Real, 2, false, false>(p, pl.ntx, pl.dgs, w.bx, w.by, w.bz, pl.ntiles, p.g.nb);
  else if (__builtin_amdgcn_readfirstlane(pl.ry) == 1)
    walk3d_body<Real, 1, 4, false, false>(p, pl.ntx, pl.nty, pl.dgs, w.bx, w.by, w.bz, pl.ntiles,
                                   p.g.nb);
  else
    walk3d_body<Real, 2, 2, false, false>(p, pl.ntx, pl.nty, pl.dgs, w.bx, w.by, w.bz, pl.ntiles,
                                   p.g.nb);
}

// Persistent sweep: each workgroup takes work items (geometry, tile, band,
// direction group) from a shared counter until the list is exhausted; items of
// geometries that have already converged are skipped.  The list is ordered
// largest geometry first.
//
// The loop header is the barrier that publishes the claimed item, and thread 0
// claims the next item at the end of an iteration.  With the claim at the top
// of the loop instead, the compiler threads the "thread 0" condition of the
// item's own final reduction into the next claim across the back-edge, which
// makes the loop's continuation divergent: lanes other than thread 0 then
// circle the barrier re-reading a stale item while thread 0 waits outside the
// inner loop, and the kernel never finishes.
//
// The items come from a stored list, or (decoded) from the list's geometry
// ranges: geometry j of the list owns items [start[j], start[j + 1]), ordered
// direction group, band, tile (tile fastest), as the stored lists are.
template <typename Real, int LIST, bool DECODE>
__global__ __launch_bounds__(kSweepBlock) void batch_sweep_kernel(const BatchCtx* __restrict__ ctxs,
                                                                  const BatchItem* __restrict__ items,
                                                                  const BatchRanges ranges,
                                                                  int nitems, int* next_item) {
  __shared__ int item_s;
  if (threadIdx.x == 0) item_s = atomicAdd(next_item, 1);
  for (;;) {
    __syncthreads();  // the claimed item is visible to every lane
    // the item and everything derived from it are wave-uniform (scalar registers)
    const int it = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();  // every lane has read it before thread 0 claims the next one
    if (it >= nitems) break;
    BatchItem w;
    if constexpr (DECODE) {
      // the list's geometry holding item it: how many ranges start at or
      // before it, less one (starts ascend), 64 at a time by a ballot
      int j = -1;
      for (int g0 = 0; g0 < ranges.n; g0 += 64) {
        const int q = g0 + (int)(threadIdx.x & 63);
        const unsigned long long m = __ballot(q < ranges.n && ranges.start[q] <= it);
        j += __popcll(m);
        if (m != ~0ull) break;
      }
      j = __builtin_amdgcn_readfirstlane(max(j, 0));
      w.ctx = __builtin_amdgcn_readfirstlane(ranges.ctx[j]);
      const int r = it - __builtin_amdgcn_readfirstlane(ranges.start[j]);
      const int ntiles = __builtin_amdgcn_readfirstlane(ctxs[w.ctx].plan.ntiles);
      const int nb = __builtin_amdgcn_readfirstlane(ctxs[w.ctx].sp64.g.nb);
      w.bx = r % ntiles;
      w.by = (r / ntiles) % nb;
      w.bz = r / (ntiles * nb);
    } else {
      w.ctx = __builtin_amdgcn_readfirstlane(items[it].ctx);
      w.bx = __builtin_amdgcn_readfirstlane(items[it].bx);
      w.by = __builtin_amdgcn_readfirstlane(items[it].by);
      w.bz = __builtin_amdgcn_readfirstlane(items[it].bz);
    }
    const BatchCtx& c = ctxs[w.ctx];
    if (!step_done(c.ctl)) batch_item<Real, LIST>(c, w);
    if (threadIdx.x == 0) item_s = atomicAdd(next_item, 1);
  }
}

__global__ __launch_bounds__(256) void batch_temperature_kernel(const BatchCtx* __restrict__ ctxs,
                                                                int nctx) {
  const int blk = blockIdx.x;
  // the context of this block: the number of contexts whose first block is
  // at or before it, less one (first blocks ascend), counted 64 at a time
  // by a ballot over the lanes instead of a chain of dependent loads
  int ci = -1;
  for (int c0 = 0; c0 < nctx; c0 += 64) {
    const int j = c0 + (int)(threadIdx.x & 63);
    const unsigned long long m = __ballot(j < nctx && ctxs[j].cell_block0 <= blk);
    ci += __popcll(m);
    if (m != ~0ull) break;
  }
  ci = __builtin_amdgcn_readfirstlane(max(ci, 0));
  const BatchCtx& c = ctxs[ci];
  if (blk - c.cell_block0 >= c.cell_blocks || step_done(c.ctl)) return;
  // geometry and tables by value: read once, since the kernel's own stores
  // could otherwise alias the context array and force them to be reloaded
  const Geometry g = c.sp64.g;
  const Tables t = c.sp64.t;
  // a batch takes constant relaxation times only (bte_batch_create refuses a
  // temperature law)
  if (temp_lanes(g.nb) == 4)
    temperature_body<4, false>(g, t, c.S, c.T, c.I0, c.E, c.ctl, blk - c.cell_block0);
  else
    temperature_body<8, false>(g, t, c.S, c.T, c.I0, c.E, c.ctl, blk - c.cell_block0);
}

__global__ __launch_bounds__(kReduceBlock) void batch_control_kernel(BatchCtx* ctxs) {
  BatchCtx& c = ctxs[blockIdx.x];
  if (step_done(c.ctl)) return;
  control_body(c.plan.nparts, c.part, c.sp64.g.vol, c.fixed_k, c.max_inner, c.tol, 0, c.ctl);
  if (threadIdx.x == 0) {
    // next iteration reads the iterate just written and writes the other one
    const int k = c.ctl->k;
    const int ia = (c.in_idx + 1) % 3, ib = (c.in_idx + 2) % 3;
    void* written = c.F[((k - 1) & 1) ? ib : ia];
    void* other = c.F[((k - 1) & 1) ? ia : ib];
    c.sp64.Ik = static_cast<const double*>(written);
    c.sp64.Iout = static_cast<double*>(other);
    c.sp32.Ik = static_cast<const float*>(written);
    c.sp32.Iout = static_cast<float*>(other);
  }
}

__global__ void batch_count_kernel(const BatchCtx* __restrict__ ctxs, int nctx, BatchControl* bc) {
  if (threadIdx.x != 0) return;
  int active = 0;
  for (int i = 0; i < nctx; ++i) active += ctxs[i].ctl->converged ? 0 : 1;
  bc->active = active;
  bc->iteration += 1;
  bc->next_item = 0;
  bc->next_item3d = 0;
  bc->next_item_f4 = 0;
}

__global__ void batch_reset_kernel(BatchCtx* ctxs, int nctx, BatchControl* bc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nctx) {
    BatchCtx& c = ctxs[i];
    const int ia = (c.in_idx + 1) % 3;
    c.sp64.Ik = static_cast<const double*>(c.F[c.in_idx]);
    c.sp64.Iout = static_cast<double*>(c.F[ia]);
    c.sp32.Ik = static_cast<const float*>(c.F[c.in_idx]);
    c.sp32.Iout = static_cast<float*>(c.F[ia]);
    Control* ctl = c.ctl;
    ctl->converged = 0;
    ctl->k = 0;
    ctl->newton_max = 0;
    ctl->err_cell = INT_MAX;
    ctl->res = 0.0;
    ctl->num = 0.0;
    ctl->den = 0.0;
  }
  if (i == 0) {
    bc->next_item = 0;
    bc->iteration = 0;
    bc->active = nctx;
    bc->next_item3d = 0;
    bc->next_item_f4 = 0;
  }
}

template <typename Real, bool DECODE>
static void launch_batch_sweeps(hipStream_t stream, const BatchCtx* ctxs, const BatchItem* items,
                                const BatchRanges* ranges, const int counts[kBatchLists],
                                BatchControl* bc, const int blocks[kBatchLists]) {
  // each work list is consumed by its own persistent launch, compiled for
  // that list's layouts only, so no list pays another's registers
  const BatchItem* list = items;
  const BatchRanges none{0, nullptr, nullptr};
  if (counts[kList2D] > 0)
    hipLaunchKernelGGL((batch_sweep_kernel<Real, kList2D, DECODE>), dim3(blocks[kList2D]),
                       dim3(kSweepBlock), 0, stream, ctxs, list,
                       DECODE ? ranges[kList2D] : none, counts[kList2D], &bc->next_item);
  if (!DECODE) list += counts[kList2D];
  if (counts[kList3D] > 0)
    hipLaunchKernelGGL((batch_sweep_kernel<Real, kList3D, DECODE>), dim3(blocks[kList3D]),
                       dim3(kSweepBlock), 0, stream, ctxs, list,
                       DECODE ? ranges[kList3D] : none, counts[kList3D], &bc->next_item3d);
  if (!DECODE) list += counts[kList3D];
  if (counts[kListFlat4] > 0)
    hipLaunchKernelGGL((batch_sweep_kernel<Real, kListFlat4, DECODE>), dim3(blocks[kListFlat4]),
                       dim3(kSweepBlock), 0, stream, ctxs, list,
                       DECODE ? ranges[kListFlat4] : none, counts[kListFlat4],
                       &bc->next_item_f4);
}

static void launch_batch_rest(hipStream_t stream, BatchCtx* ctxs, int nctx, BatchControl* bc,
                              int temp_blocks) {
  hipLaunchKernelGGL(batch_temperature_kernel, dim3(temp_blocks), dim3(256), 0, stream, ctxs, nctx);
  hipLaunchKernelGGL(batch_control_kernel, dim3(nctx), dim3(kReduceBlock), 0, stream, ctxs);
  hipLaunchKernelGGL(batch_count_kernel, dim3(1), dim3(64), 0, stream, ctxs, nctx, bc);
}

hipError_t launch_batch_iteration(hipStream_t stream, int precision, BatchCtx* ctxs,
                                  int nctx, const BatchItem* items,
                                  const int counts[kBatchLists], BatchControl* bc,
                                  const int sweep_blocks[kBatchLists], int temp_blocks) {
  if (precision == 0)
    launch_batch_sweeps<double, false>(stream, ctxs, items, nullptr, counts, bc, sweep_blocks);
  else
    launch_batch_sweeps<float, false>(stream, ctxs, items, nullptr, counts, bc, sweep_blocks);
  launch_batch_rest(stream, ctxs, nctx, bc, temp_blocks);
  return hipGetLastError();
}

hipError_t launch_batch_iteration_ranges(hipStream_t stream, int precision, BatchCtx* ctxs,
                                         int nctx, const BatchRanges ranges[kBatchLists],
                                         const int counts[kBatchLists], BatchControl* bc,
                                         const int sweep_blocks[kBatchLists], int temp_blocks) {
  if (precision == 0)
    launch_batch_sweeps<double, true>(stream, ctxs, nullptr, ranges, counts, bc, sweep_blocks);
  else
    launch_batch_sweeps<float, true>(stream, ctxs, nullptr, ranges, counts, bc, sweep_blocks);
  launch_batch_rest(stream, ctxs, nctx, bc, temp_blocks);
  return hipGetLastError();
}

hipError_t launch_batch_reset(hipStream_t stream, BatchCtx* ctxs, int nctx, BatchControl* bc) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((nctx + 63) / 64), dim3(64), 0, stream, ctxs, nctx, bc);
  return hipGetLastError();
}

template <typename Real>
static hipError_t list_occupancy(int* n, int list) {
  switch (list) {
    case kList2D:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, batch_sweep_kernel<Real, kList2D, false>, kSweepBlock, 0);
    case kList3D:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, batch_sweep_kernel<Real, kList3D, false>, kSweepBlock, 0);
    default:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, batch_sweep_kernel<Real, kListFlat4, false>, kSweepBlock, 0);
  }
}

int batch_sweep_occupancy(int precision, int list) {
  int n = 0;
  const hipError_t e =
      precision == 0 ? list_occupancy<double>(&n, list) : list_occupancy<float>(&n, list);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace bte
