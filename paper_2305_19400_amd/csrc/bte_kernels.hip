// HIP kernels of the phonon BTE time step for gfx950 (CDNA4, wave64).
//
// Data layout in HBM: intensity I[b][d][P] with P = x + nx*(y + ny*z) and each
// (b, d) slab padded to a multiple of 64 cells, so a wavefront streams 64
// consecutive cells of one slab (coalesced 512-B FP64 / 256-B FP32 accesses).
// Per-(b, d) coefficients are wave-uniform and live in scalar registers.
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

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  // Butterfly over the 64 lanes; the order is fixed, so results are reproducible.
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------- sweep
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
};

// Upwind value along one axis for a cell with coordinate `coord` along it:
// the neighbour on the inflow side, or the wall ghost (Eq. eq-bdry) when the
// inflow face is a wall face.
template <typename Real>
__device__ __forceinline__ double upwind_value(const SweepParams<Real>& p, const Real* slab,
                                               const Real* band_base, int P, int b, int d,
                                               int axis, bool from_minus, int coord, int n,
                                               int stride, int face) {
  if (from_minus) {
    if (coord > 0) return static_cast<double>(slab[P - stride]);
  } else {
    if (coord < n - 1) return static_cast<double>(slab[P + stride]);
  }
  const int side = 2 * axis + (from_minus ? 0 : 1);
  if (p.t.wall[side] == 0) {  // isothermal: equilibrium at the wall temperature
    return p.t.wall_I0[side][(size_t)b * p.t.wall_nf[side] + face];
  }
  // specular / symmetry: the cell's own intensity in the mirrored direction
  const int r = p.t.mirror[axis * p.g.nd + d];
  return static_cast<double>(band_base[(size_t)r * p.g.ncp + P]);
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
template <typename Real, int DIM>
__global__ __launch_bounds__(kSweepBlock) void sweep_kernel(const SweepParams<Real> p) {
  if (p.ctl->converged) return;
  const int b = blockIdx.y;
  const int P = blockIdx.x * kSweepBlock + threadIdx.x;
  const Geometry& g = p.g;
  const bool active = P < g.nc;
  int x = 0, y = 0, z = 0;
  if (active) {
    x = P % g.nx;
    const int r = P / g.nx;
    y = r % g.ny;
    z = r / g.ny;
  }
  const size_t ncp = (size_t)g.ncp;
  const size_t band_off = (size_t)b * g.nd * ncp;
  const Real* __restrict__ Ikb = p.Ik + band_off;
  const Real* __restrict__ Inb = p.In + band_off;
  Real* __restrict__ Iob = p.Iout + band_off;
  const double I0P = active ? p.I0[(size_t)b * ncp + P] : 0.0;
  const double inv_tau = p.t.inv_tau[b];
  const Coef* __restrict__ coef = p.t.coef + (size_t)b * g.nd;
  const int face_x = y + g.ny * z;
  const int face_y = x + g.nx * z;
  const int face_z = x + g.nx * y;
  const int sy = g.nx;
  const int sz = g.nx * g.ny;

  double S = 0.0, num = 0.0, den = 0.0;
  for (int d = 0; d < g.nd; ++d) {
    const Coef cf = coef[d];
    const int fl = p.t.dflags[d];
    const double wd = p.t.w[d];
    if (active) {
      const Real* slab = Ikb + (size_t)d * ncp;
      const double ik = static_cast<double>(slab[P]);
      const double in = static_cast<double>(Inb[(size_t)d * ncp + P]);
      double acc = (in - ik) * p.inv_dt + (I0P - ik) * inv_tau;
      if (dir_pos(fl, 0) || dir_neg(fl, 0)) {
        const double up = upwind_value(p, slab, Ikb, P, b, d, 0, dir_pos(fl, 0), x, g.nx, 1, face_x);
        acc += cf.c[0] * (up - ik);
      }
      if (dir_pos(fl, 1) || dir_neg(fl, 1)) {
        const double up = upwind_value(p, slab, Ikb, P, b, d, 1, dir_pos(fl, 1), y, g.ny, sy, face_y);
        acc += cf.c[1] * (up - ik);
      }
      if (DIM == 3 && (dir_pos(fl, 2) || dir_neg(fl, 2))) {
        const double up = upwind_value(p, slab, Ikb, P, b, d, 2, dir_pos(fl, 2), z, g.nz, sz, face_z);
        acc += cf.c[2] * (up - ik);
      }
      const Real inew_r = static_cast<Real>(ik + acc * cf.scale);
      Iob[(size_t)d * ncp + P] = inew_r;
      const double inew = static_cast<double>(inew_r);
      const double da = inew - ik;
      const double dn = inew - in;
      S += wd * inew;
      num += wd * da * da;
      den += wd * dn * dn;
    }
  }
  if (active) p.S[(size_t)b * ncp + P] = S;

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
    const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    p.part[2 * blk] = a;
    p.part[2 * blk + 1] = c;
  }
}

template <typename Real>
hipError_t launch_sweep(hipStream_t stream, const Geometry& g, const Tables& t, double inv_dt,
                        const Real* Ik, const Real* In, Real* Iout, const double* I0, double* S,
                        double* part, const Control* ctl) {
  const SweepParams<Real> p{g, t, Ik, In, Iout, I0, S, part, ctl, inv_dt};
  const dim3 grid((g.nc + kSweepBlock - 1) / kSweepBlock, g.nb);
  if (g.dim == 3)
    hipLaunchKernelGGL((sweep_kernel<Real, 3>), grid, dim3(kSweepBlock), 0, stream, p);
  else
    hipLaunchKernelGGL((sweep_kernel<Real, 2>), grid, dim3(kSweepBlock), 0, stream, p);
  return hipGetLastError();
}

template hipError_t launch_sweep<double>(hipStream_t, const Geometry&, const Tables&, double,
                                         const double*, const double*, double*, const double*,
                                         double*, double*, const Control*);
template hipError_t launch_sweep<float>(hipStream_t, const Geometry&, const Tables&, double,
                                        const float*, const float*, float*, const double*,
                                        double*, double*, const Control*);

// ---------------------------------------------------------------- temperature
// F(T) = W sum_b f_b I0_b(T) and dF/dT for the temperature relation; f_b is
// 1/tau_b (relaxation-time weighted) or 1 (plain energy).
__device__ __forceinline__ void relation(const Tables& t, int nb, double T, double& F,
                                         double& dF) {
  double f = 0.0, df = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double x = t.xfac[b] / T;
    const double em1 = expm1(x);
    const double i0 = t.Cb[b] / em1;
    f += t.fweight[b] * i0;
    df += t.fweight[b] * i0 * (x / T) * (em1 + 1.0) / em1;
  }
  F = t.W * f;
  dF = t.W * df;
}

// Per cell: finalise the energy sums from the per-band partials (band order
// fixed), invert the temperature relation by Newton from the current T
// (accept-first, quadratic convergence; Sec. 2.2 and Sec. 3.2 temperature
// update), then refresh the equilibrium intensities I0[b][P] for the next sweep.
__global__ __launch_bounds__(kCellBlock) void temperature_kernel(Geometry g, Tables t,
                                                                 const double* __restrict__ S,
                                                                 double* __restrict__ T,
                                                                 double* __restrict__ I0,
                                                                 double* __restrict__ E,
                                                                 Control* ctl) {
  if (ctl->converged) return;
  const int P = blockIdx.x * kCellBlock + threadIdx.x;
  if (P >= g.nc) return;
  const size_t ncp = (size_t)g.ncp;
  double G = 0.0, En = 0.0;
  for (int b = 0; b < g.nb; ++b) {
    const double s = S[(size_t)b * ncp + P];
    G += t.fweight[b] * s;
    En += s;
  }
  double Tc = T[P];
  int it = 0;
  bool ok = (G > 0.0) && isfinite(G) && (Tc > 0.0);
  if (ok) {
    double F, dF;
    relation(t, g.nb, Tc, F, dF);
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
        relation(t, g.nb, Tc, F, dF);
      }
    }
  }
  if (!ok) {
    atomicMin(&ctl->err_cell, P);
    return;
  }
  T[P] = Tc;
  E[P] = En;
  for (int b = 0; b < g.nb; ++b) I0[(size_t)b * ncp + P] = equilibrium(t.Cb[b], t.xfac[b], Tc);
  if (it > 0) atomicMax(&ctl->newton_max, it);
}

hipError_t launch_temperature(hipStream_t stream, const Geometry& g, const Tables& t,
                              const double* S, double* T, double* I0, double* E, Control* ctl) {
  const dim3 grid((g.nc + kCellBlock - 1) / kCellBlock);
  hipLaunchKernelGGL(temperature_kernel, grid, dim3(kCellBlock), 0, stream, g, t, S, T, I0, E,
                     ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- control
// Sums the per-block norm partials in a fixed order, forms the step-relative
// increment norm res = ||I^{k+1}-I^k|| / ||I^{k+1}-I^n|| (0/0 -> 0) and decides
// whether the inner loop is finished; later kernels of the step then return
// immediately.
__global__ __launch_bounds__(kReduceBlock) void control_kernel(int nparts,
                                                               const double* __restrict__ part,
                                                               double vol, int fixed_k,
                                                               int max_inner, double tol,
                                                               int explicit_mode, Control* ctl) {
  __shared__ double sn[kReduceBlock];
  __shared__ double sd[kReduceBlock];
  if (ctl->converged) return;
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
  }
  if (E) E[P] = t.W * sum;
}

hipError_t launch_equilibrium(hipStream_t stream, const Geometry& g, const Tables& t,
                              const double* T, double* I0, double* E) {
  const dim3 grid((g.nc + kCellBlock - 1) / kCellBlock);
  hipLaunchKernelGGL(equilibrium_kernel, grid, dim3(kCellBlock), 0, stream, g, t, T, I0, E);
  return hipGetLastError();
}

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

// I[b][d][P] = I0[b][P] for every direction (isotropic equilibrium); padding zeroed.
template <typename Real>
__global__ __launch_bounds__(256) void broadcast_kernel(Geometry g, const double* __restrict__ I0,
                                                        Real* __restrict__ I) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  const int b = blockIdx.z;
  if (P >= g.ncp) return;
  const double v = (P < g.nc) ? I0[(size_t)b * g.ncp + P] : 0.0;
  I[((size_t)b * g.nd + d) * g.ncp + P] = static_cast<Real>(v);
}

template <typename Real>
hipError_t launch_broadcast(hipStream_t stream, const Geometry& g, const double* I0, Real* I) {
  const dim3 grid((g.ncp + 255) / 256, g.nd, g.nb);
  hipLaunchKernelGGL((broadcast_kernel<Real>), grid, dim3(256), 0, stream, g, I0, I);
  return hipGetLastError();
}

template hipError_t launch_broadcast<double>(hipStream_t, const Geometry&, const double*, double*);
template hipError_t launch_broadcast<float>(hipStream_t, const Geometry&, const double*, float*);

// E_P = sum_b sum_d w_d I[b][d][P] (band outer, direction inner).
template <typename Real>
__global__ __launch_bounds__(kCellBlock) void energy_kernel(Geometry g, Tables t,
                                                            const Real* __restrict__ I,
                                                            double* __restrict__ E) {
  const int P = blockIdx.x * kCellBlock + threadIdx.x;
  if (P >= g.nc) return;
  double e = 0.0;
  for (int b = 0; b < g.nb; ++b) {
    double s = 0.0;
    for (int d = 0; d < g.nd; ++d)
      s += t.w[d] * static_cast<double>(I[((size_t)b * g.nd + d) * g.ncp + P]);
    e += s;
  }
  E[P] = e;
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
