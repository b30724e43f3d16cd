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
  uint16_t* W2P;   // [128][kK2P], W2 with its columns in the inference kernels' k order
                   // (mlp_w2p_col: the 16x16x32 B-operand order of the layer-1 output)
  float* b1;
  float* b2;
  float* w3q;      // w3 rounded to bf16, held as float
  float* b3;
};

// Column of W2 held at column k of W2P.  The inference kernels compute each layer
// transposed (Z^T = W X^T) with 16x16x32 MFMAs, so the layer-1 output of hidden tile t
// lands in lane (r, q) as units 16 t + 4 q + e, e < 4 (the D layout); the B operand of a
// 32-deep k block of layer 2 takes 8 consecutive k per lane, k = 32 kk + 8 q + e.  Joining
// the D registers of tiles 2 kk and 2 kk + 1 gives exactly that operand if k stands for
// hidden unit 32 kk + 16 (e / 4) + 4 q + (e % 4) -- a fixed permutation of the sum's terms.
constexpr int mlp_w2p_col(int k) {
  const int kk = k >> 5, q = (k >> 3) & 3, e = k & 7;
  return 32 * kk + 16 * (e >> 2) + 4 * q + (e & 3);
}

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
