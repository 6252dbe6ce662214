// Learned warm start of the per-cell temperature for the next time step: a
// 3-layer perceptron (features -> 128 -> 128 -> 1, ReLU) evaluated and trained
// on the device with bf16 matrix-core (MFMA 16x16x32) products and FP32
// accumulation, FP32 master weights and an Adam optimiser.
//
// Features of cell P for the step n -> n+1: the 3^dim neighbourhood of P
// (replicate padding at mesh edges) of (T_n - mu_T)/s_T, (T_{n-1} - mu_T)/s_T
// and (E_n - mu_E)/s_E, ordered [channel][dz][dy][dx] and zero-padded to a
// multiple of 32.  Output y: predicted (T_{n+1} - T_n)/s_D.
//
// MFMA 16x16x32 bf16 operand layout (lane l, i = 0..7):
//   A[m][k]: lane holds A[l % 16][8 (l / 16) + i]
//   B[k][n]: lane holds B[8 (l / 16) + i][l % 16]
//   D[m][n]: lane holds D[4 (l / 16) + i][l % 16], i = 0..3
// so a row-major matrix with contiguous k gives each lane one 16-byte load.
#include <climits>
#include <cmath>

#include "bte_internal.h"
#include "bte_nn.h"

namespace bte {

typedef __attribute__((ext_vector_type(8))) short bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u)  // inf / nan: keep class
    return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float((unsigned int)h << 16);
}
__device__ __forceinline__ bf16x8 load8(const unsigned short* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Sum over the 16 lanes that share l / 16 (they hold one row's columns).
__device__ __forceinline__ float row_sum16(float v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}
// Sum over the 4 lane groups l / 16 (they hold different rows of one column).
__device__ __forceinline__ float col_sum4(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

struct Norm {
  float muT, sT, muE, sE, sD;
};

__device__ __forceinline__ Norm read_norm(const float* params, const NnLayout& L) {
  const float* q = params + L.o_norm;
  return Norm{q[0], q[1], q[2], q[3], q[4]};
}

// Where the three input fields of a sample come from.
struct FieldSource {
  // live fields (inference), FP64 [N_c]
  const double* T;
  const double* Tp;
  const double* E;
  // recorded history (training): hist[s][channel][N_c], channels T_n, T_{n-1}, E_n, T_{n+1}
  const float* hist;
  long long nsamples;  // recorded samples (steps x cells)
  long long perm_a, perm_c;  // minibatch sample order: i -> (a i + c) mod nsamples
  long long batch0;    // first permuted position of this minibatch
  int batch;           // samples in this minibatch
};

__device__ __forceinline__ double field_value(const FieldSource& src, int ch, long long step,
                                              int Q, int nc, bool train) {
  if (train) return (double)src.hist[((size_t)step * 4 + ch) * nc + Q];
  return ch == 0 ? src.T[Q] : (ch == 1 ? src.Tp[Q] : src.E[Q]);
}

// One workgroup (number bx) = 4 waves x 16 samples.  TRAIN also
// back-propagates and writes the transposed activations / pre-activation
// gradients of its samples for the weight-gradient products, plus
// per-workgroup partial sums of the bias and output-weight gradients and of
// the loss.
template <bool TRAIN>
__device__ __forceinline__ void mlp_body(const Geometry& g, const NnLayout& L,
                                         const float* params, const unsigned short* W1b,
                                         const unsigned short* W2b, const unsigned short* W2Tb,
                                         const FieldSource& src, float* yout,
                                         const NnScratch& scr, const int bx) {
  __shared__ __attribute__((aligned(16))) unsigned short xs[4][16][kNnMaxK + 8];
  __shared__ __attribute__((aligned(16))) unsigned short hs[4][16][kNnHidden + 8];
  __shared__ __attribute__((aligned(16))) unsigned short ds[4][16][kNnHidden + 8];
  __shared__ float red[4][3][kNnHidden];
  __shared__ float red_s[4][2];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int K = L.K, KP = L.KP;
  const int nc = g.nc;
  const int r0 = (bx * 4 + w) * 16;  // first sample (minibatch position) of this wave
  const int nsamp = TRAIN ? src.batch : nc;
  const Norm nm = read_norm(params, L);
  const int S = (g.dim == 3) ? 27 : 9;

  // ---- gather features of the wave's 16 samples into LDS (bf16, row-major)
  for (int e = lane; e < 16 * KP; e += 64) {
    const int m = e / KP, k = e % KP;
    const int r = r0 + m;
    float v = 0.f;
    if (k < K && r < nsamp) {
      long long step = 0;
      int P = r;
      if (TRAIN) {
        const long long i = (src.perm_a * (src.batch0 + r) + src.perm_c) % src.nsamples;
        step = i / nc;
        P = (int)(i % nc);
      }
      const int ch = k / S, st = k % S;
      const int dx = st % 3 - 1, dy = (st / 3) % 3 - 1, dz = (g.dim == 3) ? st / 9 - 1 : 0;
      const int x = P % g.nx, y = (P / g.nx) % g.ny, z = P / (g.nx * g.ny);
      const int qx = min(max(x + dx, 0), g.nx - 1);
      const int qy = min(max(y + dy, 0), g.ny - 1);
      const int qz = min(max(z + dz, 0), g.nz - 1);
      const int Q = qx + g.nx * (qy + g.ny * qz);
      const double fv = field_value(src, ch, step, Q, nc, TRAIN);
      v = (ch < 2) ? (float)((fv - nm.muT) / nm.sT) : (float)((fv - nm.muE) / nm.sE);
    }
    const unsigned short hv = to_bf16(v);
    xs[w][m][k] = hv;
    if (TRAIN && r0 + m < scr.M) scr.XT[(size_t)k * scr.M + r0 + m] = hv;
  }
  __syncthreads();

  const int col = lane & 15;   // n within a 16-column tile / row of an A fragment
  const int grp = lane >> 4;   // lane group: k slice 8*grp (operands), rows 4*grp (result)

  // ---- layer 1: z1 = X W1^T + b1
  f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < KP; kc += 32) {
    const bf16x8 a = load8(&xs[w][col][kc + 8 * grp]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bf16x8 b = load8(W1b + (size_t)(16 * t + col) * KP + kc + 8 * grp);
      acc[t] = mfma(a, b, acc[t]);
    }
  }
  const float* b1 = params + L.o_b1;
  const float* b2 = params + L.o_b2;
  const float* w3 = params + L.o_w3;
  const float b3 = params[L.o_b3];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int n = 16 * t + col;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 4 * grp + i;
      const float h = fmaxf(acc[t][i] + b1[n], 0.f);
      const unsigned short hb = to_bf16(h);
      hs[w][m][n] = hb;
      if (TRAIN && r0 + m < scr.M) scr.H1T[(size_t)n * scr.M + r0 + m] = hb;
    }
  }
  __syncthreads();

  // ---- layer 2: z2 = H1 W2^T + b2
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < kNnHidden; kc += 32) {
    const bf16x8 a = load8(&hs[w][col][kc + 8 * grp]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bf16x8 b = load8(W2b + (size_t)(16 * t + col) * kNnHidden + kc + 8 * grp);
      acc[t] = mfma(a, b, acc[t]);
    }
  }
  // ---- output: y = w3 . relu(z2) + b3 (rows 4 grp + i)
  float ysum[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float p = 0.f;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 16 * t + col;
      p += fmaxf(acc[t][i] + b2[n], 0.f) * w3[n];
    }
    ysum[i] = row_sum16(p) + b3;
  }
  if (yout && col == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + 4 * grp + i;
      if (r < nsamp) yout[r] = ysum[i];
    }
  }
  if (!TRAIN) return;

  // ---- backward (mean squared error over the minibatch)
  float dy[4];
  float loss = 0.f, db3 = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + 4 * grp + i;
    dy[i] = 0.f;
    if (r < nsamp) {
      const long long idx = (src.perm_a * (src.batch0 + r) + src.perm_c) % src.nsamples;
      const long long step = idx / nc;
      const int P = (int)(idx % nc);
      const float tn = src.hist[((size_t)step * 4 + 0) * nc + P];
      const float t1 = src.hist[((size_t)step * 4 + 3) * nc + P];
      const float target = (float)(((double)t1 - (double)tn) / nm.sD);
      const float e = ysum[i] - target;
      dy[i] = 2.f * e / (float)src.batch;
      if (col == 0) {
        loss += e * e;
        db3 += dy[i];
      }
    }
  }
  // dz2 = dy w3 (relu'), partials of db2 and dw3 per column
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int n = 16 * t + col;
    float pdb2 = 0.f, pdw3 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 4 * grp + i;
      const float z2 = acc[t][i] + b2[n];
      const float d = (z2 > 0.f) ? dy[i] * w3[n] : 0.f;
      pdb2 += d;
      pdw3 += dy[i] * fmaxf(z2, 0.f);
      const unsigned short db = to_bf16(d);
      ds[w][m][n] = db;
      if (r0 + m < scr.M) scr.dZ2T[(size_t)n * scr.M + r0 + m] = db;
    }
    pdb2 = col_sum4(pdb2);
    pdw3 = col_sum4(pdw3);
    if (grp == 0) {
      red[w][1][n] = pdb2;
      red[w][2][n] = pdw3;
    }
  }
  loss = row_sum16(loss);
  db3 = row_sum16(db3);
  loss = col_sum4(loss);
  db3 = col_sum4(db3);
  if (lane == 0) {
    red_s[w][0] = db3;
    red_s[w][1] = loss;
  }
  __syncthreads();
  // dh1 = dz2 W2 ; dz1 = dh1 relu'(z1)
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < kNnHidden; kc += 32) {
    const bf16x8 a = load8(&ds[w][col][kc + 8 * grp]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bf16x8 b = load8(W2Tb + (size_t)(16 * t + col) * kNnHidden + kc + 8 * grp);
      acc[t] = mfma(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int n = 16 * t + col;
    float pdb1 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 4 * grp + i;
      const float d = (from_bf16(hs[w][m][n]) > 0.f) ? acc[t][i] : 0.f;
      pdb1 += d;
      if (r0 + m < scr.M) scr.dZ1T[(size_t)n * scr.M + r0 + m] = to_bf16(d);
    }
    pdb1 = col_sum4(pdb1);
    if (grp == 0) red[w][0][n] = pdb1;
  }
  __syncthreads();
  // per-workgroup partials, waves summed in a fixed order
  float* part = scr.part + (size_t)bx * kNnPartWidth;
  if (threadIdx.x < kNnHidden) {
    const int n = threadIdx.x;
    for (int q = 0; q < 3; ++q) {
      float s = 0.f;
      for (int v = 0; v < 4; ++v) s += red[v][q][n];
      part[q * kNnHidden + n] = s;
    }
  } else if (threadIdx.x == kNnHidden) {
    float a = 0.f, b = 0.f;
    for (int v = 0; v < 4; ++v) {
      a += red_s[v][0];
      b += red_s[v][1];
    }
    part[3 * kNnHidden] = a;
    part[3 * kNnHidden + 1] = b;
  }
}

template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_kernel(Geometry g, NnLayout L, const float* params,
                                                  const unsigned short* W1b,
                                                  const unsigned short* W2b,
                                                  const unsigned short* W2Tb, FieldSource src,
                                                  float* yout, NnScratch scr) {
  mlp_body<TRAIN>(g, L, params, W1b, W2b, W2Tb, src, yout, scr, blockIdx.x);
}

// dW = dZ^T A over the minibatch: one wave per 16x16 tile of dW1 (128 x KP) or
// dW2 (128 x 128), samples in a fixed order.
__device__ __forceinline__ int wgrad_tiles(const NnLayout& L) { return 8 * (L.KP / 16) + 64; }
__device__ __forceinline__ void wgrad_body(const NnLayout& L, const NnScratch& scr, float* grad,
                                           int tile) {
  const int lane = threadIdx.x;
  const int col = lane & 15, grp = lane >> 4;
  const int t1 = 8 * (L.KP / 16);
  const unsigned short* dZT;
  const unsigned short* AT;
  int kdim;
  size_t base;
  if (tile < t1) {
    dZT = scr.dZ1T;
    AT = scr.XT;
    kdim = L.KP;
    base = L.o_W1;
  } else {
    tile -= t1;
    dZT = scr.dZ2T;
    AT = scr.H1T;
    kdim = kNnHidden;
    base = L.o_W2;
  }
  const int tn = tile / (kdim / 16), tk = tile % (kdim / 16);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int s0 = 0; s0 < scr.M; s0 += 32) {
    const bf16x8 a = load8(dZT + (size_t)(16 * tn + col) * scr.M + s0 + 8 * grp);
    const bf16x8 b = load8(AT + (size_t)(16 * tk + col) * scr.M + s0 + 8 * grp);
    acc = mfma(a, b, acc);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    grad[base + (size_t)(16 * tn + 4 * grp + i) * kdim + 16 * tk + col] = acc[i];
}
__global__ __launch_bounds__(64) void wgrad_kernel(NnLayout L, NnScratch scr, float* grad) {
  wgrad_body(L, scr, grad, blockIdx.x);
}

// Bias / output-weight gradients and the loss: partials of all workgroups
// summed in a fixed order.
__device__ __forceinline__ void bias_grad_body(const NnLayout& L, const NnScratch& scr, int nwg,
                                               float* grad, float* loss) {
  const int j = threadIdx.x;
  if (j >= kNnPartWidth) return;
  float s = 0.f;
  for (int q = 0; q < nwg; ++q) s += scr.part[(size_t)q * kNnPartWidth + j];
  if (j < kNnHidden) grad[L.o_b1 + j] = s;
  else if (j < 2 * kNnHidden) grad[L.o_b2 + j - kNnHidden] = s;
  else if (j < 3 * kNnHidden) grad[L.o_w3 + j - 2 * kNnHidden] = s;
  else if (j == 3 * kNnHidden) grad[L.o_b3] = s;
  else if (j == 3 * kNnHidden + 1 && loss) *loss = s;
}
__global__ void bias_grad_kernel(NnLayout L, NnScratch scr, int nwg, float* grad, float* loss) {
  bias_grad_body(L, scr, nwg, grad, loss);
}

// Adam step on every trainable parameter (padded feature columns stay zero),
// then refresh the bf16 operand copies.
__device__ __forceinline__ void adam_body(const NnLayout& L, float* params, const float* grad,
                                          float* m, float* v, float lr, float b1c, float b2c,
                                          unsigned short* W1b, unsigned short* W2b,
                                          unsigned short* W2Tb, int bx) {
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= L.o_norm) return;
  const bool pad_col = (i < L.o_b1) && ((i % L.KP) >= L.K);
  const bool b3pad = (i > L.o_b3 && i < L.o_b3 + 4);
  if (!pad_col && !b3pad) {
    const float gr = grad[i];
    const float mi = 0.9f * m[i] + 0.1f * gr;
    const float vi = 0.999f * v[i] + 0.001f * gr * gr;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / b1c) / (sqrtf(vi / b2c) + 1e-8f);
  }
  const float p = params[i];
  if (i < L.o_b1) {
    W1b[i] = to_bf16(p);
  } else if (i >= L.o_W2 && i < L.o_b2) {
    const int j = i - L.o_W2;
    W2b[j] = to_bf16(p);
    W2Tb[(j % kNnHidden) * kNnHidden + j / kNnHidden] = to_bf16(p);
  }
}
__global__ void adam_kernel(NnLayout L, float* params, const float* grad, float* m, float* v,
                            float lr, float b1c, float b2c, unsigned short* W1b,
                            unsigned short* W2b, unsigned short* W2Tb) {
  adam_body(L, params, grad, m, v, lr, b1c, b2c, W1b, W2b, W2Tb, blockIdx.x);
}

__global__ void refresh_bf16_kernel(NnLayout L, const float* params, unsigned short* W1b,
                                    unsigned short* W2b, unsigned short* W2Tb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L.o_b1) W1b[i] = to_bf16(params[i]);
  if (i >= L.o_W2 && i < L.o_b2) {
    const int j = i - L.o_W2;
    const unsigned short h = to_bf16(params[i]);
    W2b[j] = h;
    W2Tb[(j % kNnHidden) * kNnHidden + j / kNnHidden] = h;
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): counter-based initial weights.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// He-uniform initial weights, zero biases, zero Adam moments.
__global__ void init_params_kernel(NnLayout L, float* params, float* m, float* v, float* grad,
                                   unsigned long long seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.total) return;
  grad[i] = 0.f;
  if (i >= L.o_norm) {  // normalisation: identity until trained or set
    params[i] = (i == L.o_norm + 1 || i == L.o_norm + 3 || i == L.o_norm + 4) ? 1.f : 0.f;
    m[i] = 0.f;
    v[i] = 0.f;
    return;
  }
  const double u = (double)(splitmix64(seed * 0x100000001B3ull + (unsigned long long)i) >> 11) *
                   (1.0 / 9007199254740992.0);
  float p = 0.f;
  if (i < L.o_b1) {
    if ((i % L.KP) < L.K) p = (float)((2.0 * u - 1.0) * sqrt(6.0 / L.K));
  } else if (i >= L.o_W2 && i < L.o_b2) {
    p = (float)((2.0 * u - 1.0) * sqrt(6.0 / kNnHidden));
  } else if (i >= L.o_w3 && i < L.o_b3) {
    p = (float)((2.0 * u - 1.0) * sqrt(6.0 / kNnHidden));
  }
  params[i] = p;
  m[i] = 0.f;
  v[i] = 0.f;
}

// Copy the step's input fields (or the target) into the history ring.
__global__ void record_kernel(int nc, const double* T, const double* Tp, const double* E,
                              float* slot, int which) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= nc) return;
  if (which == 0) {
    slot[P] = (float)T[P];
    slot[(size_t)nc + P] = (float)Tp[P];
    slot[2 * (size_t)nc + P] = (float)E[P];
  } else {
    slot[3 * (size_t)nc + P] = (float)T[P];
  }
}

// Normalisation constants from the recorded history (single workgroup, fixed
// order): mean / std of T (both T channels), of E, and RMS of T_{n+1} - T_n.
__global__ __launch_bounds__(256) void stats_kernel(const float* hist, long long nrec, int nc,
                                                    float* norm) {
  __shared__ double sh[5][256];
  double s[5] = {0, 0, 0, 0, 0};
  const long long n = nrec * nc;
  for (long long i = threadIdx.x; i < n; i += 256) {
    const long long st = i / nc;
    const int P = (int)(i % nc);
    const double t = hist[(st * 4 + 0) * nc + P];
    const double e = hist[(st * 4 + 2) * nc + P];
    const double d = (double)hist[(st * 4 + 3) * nc + P] - t;
    s[0] += t;
    s[1] += t * t;
    s[2] += e;
    s[3] += e * e;
    s[4] += d * d;
  }
  for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double inv = 1.0 / (double)n;
    const double muT = sh[0][0] * inv, muE = sh[2][0] * inv;
    const double vT = sh[1][0] * inv - muT * muT, vE = sh[3][0] * inv - muE * muE;
    const double sD = sqrt(sh[4][0] * inv);
    norm[0] = (float)muT;
    norm[1] = (float)(vT > 0 ? sqrt(vT) : 1.0);
    norm[2] = (float)muE;
    norm[3] = (float)(vE > 0 ? sqrt(vE) * 1.0 : 1.0);
    norm[4] = (float)(sD > 0 ? sD : 1.0);
    if (!(norm[1] > 1e-6f * fabsf(norm[0]))) norm[1] = 1e-6f * fabsf(norm[0]) + 1e-30f;
    if (!(norm[3] > 1e-6f * fabsf(norm[2]))) norm[3] = 1e-6f * fabsf(norm[2]) + 1e-30f;
    norm[5] = norm[6] = norm[7] = 0.f;
  }
}

// Apply the prediction: T^(0) = T_n + s_D y where plausible, else T_n
// (counted); refresh I0 at T^(0) and, optionally, the isotropic shift
// I0(T^(0)) - I0(T_n) that seeds the first sweep's intensity.
__global__ __launch_bounds__(64) void apply_guess_kernel(Geometry g, Tables t, const float* y,
                                                         const float* params, NnLayout L,
                                                         double* Tp, double* T, double* I0,
                                                         double* shift, float max_step,
                                                         int* fallbacks) {
  const int P = blockIdx.x * 64 + threadIdx.x;
  if (P >= g.nc) return;
  const float sD = params[L.o_norm + 4];
  const double Tn = T[P];
  const double dT = (double)sD * (double)y[P];
  const double lim = max_step * fmax((double)sD, fabs(Tn - Tp[P]));
  Tp[P] = Tn;  // T_{n-1} of the next step
  double T0 = Tn + dT;
  if (!isfinite(dT) || fabs(dT) > lim || !(T0 > 0.0)) {
    T0 = Tn;
    atomicAdd(fallbacks, 1);
  }
  T[P] = T0;
  for (int b = 0; b < g.nb; ++b) {
    const double old = I0[(size_t)b * g.ncp + P];
    const double nw = t.Cb[b] / expm1(t.xfac[b] / T0);
    I0[(size_t)b * g.ncp + P] = nw;
    if (t.relax) t.relax[(size_t)b * g.ncp + P] = relax_rate(t.inv_tau[b], t.tau_p[b], T0, t.tau_T0);
    if (shift) shift[(size_t)b * g.ncp + P] = nw - old;
  }
}

// Zero the scratch columns [from, M) of every transposed array (workgroup bx
// of gx, grid-stride).
__device__ __forceinline__ void zero_tail_body(const NnLayout& L, const NnScratch& scr, int from,
                                               int bx, int gx) {
  const int width = scr.M - from;
  const long long total = (long long)(L.KP + 3 * kNnHidden) * width;
  for (long long e = bx * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gx * blockDim.x) {
    const int row = (int)(e / width);
    const int c = from + (int)(e % width);
    if (row < L.KP) scr.XT[(size_t)row * scr.M + c] = 0;
    else if (row < L.KP + kNnHidden) scr.H1T[(size_t)(row - L.KP) * scr.M + c] = 0;
    else if (row < L.KP + 2 * kNnHidden) scr.dZ1T[(size_t)(row - L.KP - kNnHidden) * scr.M + c] = 0;
    else scr.dZ2T[(size_t)(row - L.KP - 2 * kNnHidden) * scr.M + c] = 0;
  }
}

__global__ void zero_tail_kernel(NnLayout L, NnScratch scr, int from) {
  zero_tail_body(L, scr, from, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- several networks
// One training iteration of several networks (one per geometry of a batch) in
// one launch per kernel: blockIdx.y selects the network, steps[it * njobs +
// job] its minibatch of iteration it, and a network whose schedule has ended
// (or whose minibatch needs fewer workgroups) skips.  Each network runs the
// same kernels on the same data in the same order as when trained alone.
__device__ __forceinline__ const NnTrainStep& train_step(const NnTrainStep* steps, int njobs,
                                                         int it) {
  return steps[(size_t)it * njobs + blockIdx.y];
}

__global__ void zero_tail_many_kernel(const NnTrainJob* jobs, const NnTrainStep* steps, int njobs,
                                      int it) {
  const NnTrainStep st = train_step(steps, njobs, it);
  const NnTrainJob& J = jobs[blockIdx.y];
  const int from = (st.batch + 63) / 64 * 64;
  if (!st.active || from >= J.B.scr.M) return;
  zero_tail_body(J.L, J.B.scr, from, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void mlp_train_many_kernel(const NnTrainJob* jobs,
                                                             const NnTrainStep* steps, int njobs,
                                                             int it) {
  const NnTrainStep st = train_step(steps, njobs, it);
  if (!st.active || (int)blockIdx.x >= (st.batch + 63) / 64) return;
  const NnTrainJob& J = jobs[blockIdx.y];
  const FieldSource src{nullptr, nullptr, nullptr, J.B.hist, J.nsamples, J.perm_a,
                        st.perm_c, st.batch0, st.batch};
  mlp_body<true>(J.g, J.L, J.B.params, J.B.W1b, J.B.W2b, J.B.W2Tb, src, nullptr, J.B.scr,
                 blockIdx.x);
}

__global__ __launch_bounds__(64) void wgrad_many_kernel(const NnTrainJob* jobs,
                                                        const NnTrainStep* steps, int njobs,
                                                        int it) {
  const NnTrainStep st = train_step(steps, njobs, it);
  const NnTrainJob& J = jobs[blockIdx.y];
  if (!st.active || (int)blockIdx.x >= wgrad_tiles(J.L)) return;
  wgrad_body(J.L, J.B.scr, J.B.grad, blockIdx.x);
}

__global__ void bias_grad_many_kernel(const NnTrainJob* jobs, const NnTrainStep* steps, int njobs,
                                      int it) {
  const NnTrainStep st = train_step(steps, njobs, it);
  if (!st.active) return;
  const NnTrainJob& J = jobs[blockIdx.y];
  bias_grad_body(J.L, J.B.scr, (st.batch + 63) / 64, J.B.grad, J.B.loss);
}

__global__ void adam_many_kernel(const NnTrainJob* jobs, const NnTrainStep* steps, int njobs,
                                 int it) {
  const NnTrainStep st = train_step(steps, njobs, it);
  if (!st.active) return;
  const NnTrainJob& J = jobs[blockIdx.y];
  adam_body(J.L, J.B.params, J.B.grad, J.B.adam_m, J.B.adam_v, J.lr, st.b1c, st.b2c, J.B.W1b,
            J.B.W2b, J.B.W2Tb, blockIdx.x);
}

// out[P] = T_n[P] + s_D y[P] (the raw guess, for reporting).
__global__ void guess_out_kernel(int nc, NnLayout L, const float* params, const double* T,
                                 const float* y, double* out) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= nc) return;
  out[P] = T[P] + (double)params[L.o_norm + 4] * (double)y[P];
}

// ---------------------------------------------------------------- launchers
hipError_t nn_guess_out(hipStream_t s, int nc, const NnLayout& L, const NnBuffers& B,
                        const double* T, double* out) {
  hipLaunchKernelGGL(guess_out_kernel, dim3((nc + 255) / 256), dim3(256), 0, s, nc, L, B.params, T,
                     B.y, out);
  return hipGetLastError();
}

hipError_t nn_predict(hipStream_t s, const Geometry& g, const NnLayout& L, const NnBuffers& B,
                      const double* T, const double* Tp, const double* E) {
  FieldSource src{T, Tp, E, nullptr, 0, 1, 0, 0, 0};
  const int nwg = (g.nc + 63) / 64;
  NnScratch none = B.scr;
  hipLaunchKernelGGL((mlp_kernel<false>), dim3(nwg), dim3(256), 0, s, g, L, B.params, B.W1b,
                     B.W2b, B.W2Tb, src, B.y, none);
  return hipGetLastError();
}

hipError_t nn_apply_guess(hipStream_t s, const Geometry& g, const Tables& t, const NnLayout& L,
                          const NnBuffers& B, double* Tp, double* T, double* I0,
                          double* shift, float max_step) {
  hipLaunchKernelGGL(apply_guess_kernel, dim3((g.nc + 63) / 64), dim3(64), 0, s, g, t, B.y,
                     B.params, L, Tp, T, I0, shift, max_step, B.fallbacks);
  return hipGetLastError();
}

hipError_t nn_train_batch(hipStream_t s, const Geometry& g, const NnLayout& L, const NnBuffers& B,
                          long long nsamples, long long perm_a, long long perm_c,
                          long long batch0, int batch, float lr, int adam_t, bool update,
                          float* yout) {
  FieldSource src{nullptr, nullptr, nullptr, B.hist, nsamples, perm_a, perm_c, batch0, batch};
  const int nwg = (batch + 63) / 64;
  // the weight-gradient products read every column of the scratch: columns past
  // this minibatch must hold zeros
  if (nwg * 64 < B.scr.M) {
    hipLaunchKernelGGL(zero_tail_kernel, dim3(256), dim3(256), 0, s, L, B.scr, nwg * 64);
  }
  hipLaunchKernelGGL((mlp_kernel<true>), dim3(nwg), dim3(256), 0, s, g, L, B.params, B.W1b,
                     B.W2b, B.W2Tb, src, yout, B.scr);
  const int ntiles = 8 * (L.KP / 16) + 64;
  hipLaunchKernelGGL(wgrad_kernel, dim3(ntiles), dim3(64), 0, s, L, B.scr, B.grad);
  hipLaunchKernelGGL(bias_grad_kernel, dim3(1), dim3(512), 0, s, L, B.scr, nwg, B.grad, B.loss);
  if (update) {
    const float b1c = 1.f - powf(0.9f, (float)adam_t);
    const float b2c = 1.f - powf(0.999f, (float)adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3((L.o_norm + 255) / 256), dim3(256), 0, s, L, B.params,
                       B.grad, B.adam_m, B.adam_v, lr, b1c, b2c, B.W1b, B.W2b, B.W2Tb);
  }
  return hipGetLastError();
}

hipError_t nn_train_many(hipStream_t s, const NnTrainJob* jobs, const NnTrainStep* steps,
                         int njobs, int it, int max_kp) {
  if (njobs <= 0) return hipSuccess;
  const dim3 per(1, njobs);
  const int nwg = (kNnBatch + 63) / 64;
  const int tiles = 8 * (max_kp / 16) + 64;
  const int adam_blocks = (kNnHidden * max_kp + kNnHidden * kNnHidden + 4 * kNnHidden + 255) / 256;
  hipLaunchKernelGGL(zero_tail_many_kernel, dim3(256, njobs), dim3(256), 0, s, jobs, steps, njobs,
                     it);
  hipLaunchKernelGGL(mlp_train_many_kernel, dim3(nwg, njobs), dim3(256), 0, s, jobs, steps, njobs,
                     it);
  hipLaunchKernelGGL(wgrad_many_kernel, dim3(tiles, njobs), dim3(64), 0, s, jobs, steps, njobs, it);
  hipLaunchKernelGGL(bias_grad_many_kernel, per, dim3(512), 0, s, jobs, steps, njobs, it);
  hipLaunchKernelGGL(adam_many_kernel, dim3(adam_blocks, njobs), dim3(256), 0, s, jobs, steps,
                     njobs, it);
  return hipGetLastError();
}

hipError_t nn_init(hipStream_t s, const NnLayout& L, const NnBuffers& B, unsigned long long seed) {
  hipLaunchKernelGGL(init_params_kernel, dim3((L.total + 255) / 256), dim3(256), 0, s, L,
                     B.params, B.adam_m, B.adam_v, B.grad, seed);
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((L.o_norm + 255) / 256), dim3(256), 0, s, L,
                     B.params, B.W1b, B.W2b, B.W2Tb);
  return hipGetLastError();
}

hipError_t nn_refresh(hipStream_t s, const NnLayout& L, const NnBuffers& B) {
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((L.o_norm + 255) / 256), dim3(256), 0, s, L,
                     B.params, B.W1b, B.W2b, B.W2Tb);
  return hipGetLastError();
}

hipError_t nn_record(hipStream_t s, int nc, const double* T, const double* Tp, const double* E,
                     float* slot, int which) {
  hipLaunchKernelGGL(record_kernel, dim3((nc + 255) / 256), dim3(256), 0, s, nc, T, Tp, E, slot,
                     which);
  return hipGetLastError();
}

hipError_t nn_stats(hipStream_t s, const NnLayout& L, const NnBuffers& B, long long nrec, int nc) {
  hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(256), 0, s, B.hist, nrec, nc,
                     B.params + L.o_norm);
  return hipGetLastError();
}

}  // namespace bte
