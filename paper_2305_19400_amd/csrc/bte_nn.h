// Internal declarations of the learned warm start (bte_nn.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bte_internal.h"

namespace bte {

constexpr int kNnHidden = 128;
constexpr int kNnMaxK = 96;                      // 3 channels x 27 neighbours, padded to 32
constexpr int kNnPartWidth = 3 * kNnHidden + 2;  // db1, db2, dw3, db3, loss per workgroup
constexpr int kNnBatch = 8192;                   // minibatch size (multiple of 64)

// Offsets (in floats) of the parameter vector:
// W1[128][KP] | b1[128] | W2[128][128] | b2[128] | w3[128] | b3 (+3 pad) | norm[8]
// norm = mu_T, s_T, mu_E, s_E, s_D (output scale of T_{n+1} - T_n), 3 spare.
struct NnLayout {
  int K, KP;
  int o_W1, o_b1, o_W2, o_b2, o_w3, o_b3, o_norm, total;
};

inline NnLayout make_nn_layout(int dim) {
  NnLayout L{};
  L.K = 3 * (dim == 3 ? 27 : 9);
  L.KP = (L.K + 31) / 32 * 32;
  L.o_W1 = 0;
  L.o_b1 = kNnHidden * L.KP;
  L.o_W2 = L.o_b1 + kNnHidden;
  L.o_b2 = L.o_W2 + kNnHidden * kNnHidden;
  L.o_w3 = L.o_b2 + kNnHidden;
  L.o_b3 = L.o_w3 + kNnHidden;
  L.o_norm = L.o_b3 + 4;
  L.total = L.o_norm + 8;
  return L;
}

// Training scratch: transposed bf16 activations [feature][M] of one minibatch
// and per-workgroup partials.
struct NnScratch {
  unsigned short* XT;
  unsigned short* H1T;
  unsigned short* dZ1T;
  unsigned short* dZ2T;
  float* part;
  int M;
};

struct NnBuffers {
  float* params;   // FP32 master parameters [L.total]
  float* grad;     // [L.total]
  float* adam_m;
  float* adam_v;
  unsigned short* W1b;   // [128][KP]
  unsigned short* W2b;   // [128][128]
  unsigned short* W2Tb;  // [128][128], W2 transposed
  float* y;        // [N_c] network outputs of the last prediction
  float* hist;     // [n_rec][4][N_c]: T_n, T_{n-1}, E_n, T_{n+1}
  float* loss;     // last minibatch loss
  int* fallbacks;  // cells whose guess was rejected (accumulates)
  NnScratch scr;
};

// Training of several networks at once (the geometries of a batch).
struct NnTrainJob {
  Geometry g;
  NnLayout L;
  NnBuffers B;
  long long nsamples, perm_a;  // recorded samples and the sample-order multiplier
  float lr;
};
// One network's minibatch of one iteration (active = 0: its schedule has ended).
struct NnTrainStep {
  long long batch0, perm_c;
  int batch, active;
  float b1c, b2c;  // Adam bias corrections of this update
};
// Iteration it of every job (jobs and steps in device memory, steps[it][job]);
// max_kp bounds the jobs' padded feature counts.
hipError_t nn_train_many(hipStream_t s, const NnTrainJob* jobs, const NnTrainStep* steps,
                         int njobs, int it, int max_kp);

hipError_t nn_init(hipStream_t s, const NnLayout& L, const NnBuffers& B, unsigned long long seed);
hipError_t nn_refresh(hipStream_t s, const NnLayout& L, const NnBuffers& B);
hipError_t nn_record(hipStream_t s, int nc, const double* T, const double* Tp, const double* E,
                     float* slot, int which);
hipError_t nn_stats(hipStream_t s, const NnLayout& L, const NnBuffers& B, long long nrec, int nc);
hipError_t nn_train_batch(hipStream_t s, const Geometry& g, const NnLayout& L, const NnBuffers& B,
                          long long nsamples, long long perm_a, long long perm_c,
                          long long batch0, int batch, float lr, int adam_t, bool update,
                          float* yout = nullptr);
hipError_t nn_predict(hipStream_t s, const Geometry& g, const NnLayout& L, const NnBuffers& B,
                      const double* T, const double* Tp, const double* E);
// T^(0) from the prediction (per-cell fallback to T_n), T_prev <- T_n, I0 at
// T^(0), and (if shift != null) shift = I0(T^(0)) - I0(T_n).
hipError_t nn_apply_guess(hipStream_t s, const Geometry& g, const Tables& t, const NnLayout& L,
                          const NnBuffers& B, double* Tp, double* T, double* I0,
                          double* shift, float max_step);
hipError_t nn_guess_out(hipStream_t s, int nc, const NnLayout& L, const NnBuffers& B,
                        const double* T, double* out);

}  // namespace bte
