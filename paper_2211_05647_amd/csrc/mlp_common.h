// mlp_common.h -- sizes, parameter layout and device structs of the learned closure.
#pragma once
#include <stdint.h>

namespace fdtdp {

constexpr int kHist = 16;                 // past E samples per feature row
constexpr int kNIn = kHist + 2;           // + omega_p dt and log10(nu dt), both scaled
constexpr int kNH = 128;                  // hidden width (two layers)
constexpr int kK1 = 32;                   // first-layer K padded to the MFMA K granule
constexpr int kK1P = kK1 + 8;             // LDS/global row pitch of W1 and of feature tiles
constexpr int kK2P = kNH + 8;             // row pitch of W2 and of activation tiles
// FP32 master parameter vector: W1[128][18], b1[128], W2[128][128], b2[128], w3[128], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNH * kNIn;
constexpr int kOffW2 = kOffB1 + kNH;
constexpr int kOffB2 = kOffW2 + kNH * kNH;
constexpr int kOffW3 = kOffB2 + kNH;
constexpr int kOffB3 = kOffW3 + kNH;
constexpr int kNParam = kOffB3 + 1;       // 19073
constexpr int kReplayNv = 32;             // 2V replay grid (the 2D workloads' grid)
constexpr int kReplayHalf = kReplayNv * kReplayNv / 2;

// Device copies the GEMM kernels read (bf16 weights, padded rows; FP32 biases).
struct MlpWeights {
  uint16_t* W1;    // [128][kK1P]
  uint16_t* W2;    // [128][kK2P]
  uint16_t* W2T;   // [128][kK2P], W2 transposed
  float* b1;
  float* b2;
  float* w3q;      // w3 rounded to bf16, held as float
  float* b3;
};

struct ReplayCell {
  float tau;       // dt * nu_mean
  float dens;      // electron density
};

// Closure cells of a 2D run.
struct MlpCells2D {
  const int32_t* idx;   // [n] grid index j * nx + i of each closure cell
  const float* coef;    // [n][4] alpha, beta, q1, q2
  float* ring;          // [n][2][kHist] cell-centre E history of (x, y), slot = step % kHist
  int n;
};

struct PairSeries {
  float alpha, beta;   // single-pole recurrence of the cell's current
  float q1, q2;        // scaled omega_p dt and log10(nu_mean dt)
};

}  // namespace fdtdp
