// closure_static.hip -- the closure network's gradient without any device allocation:
// the variant of fdtd_closure_grad for callers that cannot allocate (code under HIP graph
// capture, tight serving loops).  Its kernels are those of fdtd_closure_grad (bf16 packing
// of the FP32 parameters, forward + backward of 64-row blocks with per-block partial
// gradients, the fixed-order reduction); their scratch buffers -- the bf16 weight copies
// (the packing writes all of them, the inference layout included) and the per-block
// partials -- live in one file-scope device array of fixed size.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fdtd_closure.h"
#include "host_internal.h"
#include "mlp_common.h"

namespace fdtdp {

hipError_t mlp_launch_grad(const MlpWeights& W, const float* X, const float* T, int n, float* P,
                           float* lossp, float* G, float* loss, hipStream_t st);
hipError_t mlp_launch_pack(const float* master, const MlpWeights& W, hipStream_t st);

namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// layout of the scratch array (byte offsets)
constexpr size_t kScrW1 = 0;
constexpr size_t kScrW2 = kScrW1 + align256((size_t)kNH * kK1P * 2);
constexpr size_t kScrW2T = kScrW2 + align256((size_t)kNH * kK2P * 2);
constexpr size_t kScrW2P = kScrW2T + align256((size_t)kNH * kK2P * 2);
constexpr size_t kScrB1 = kScrW2P + align256((size_t)kNH * kK2P * 2);
constexpr size_t kScrB2 = kScrB1 + align256(kNH * 4);
constexpr size_t kScrW3 = kScrB2 + align256(kNH * 4);
constexpr size_t kScrB3 = kScrW3 + align256(kNH * 4);
constexpr size_t kScrP = kScrB3 + 256;
constexpr int kMaxBlocks = (FDTD_CLOSURE_STATIC_MAX_ROWS + 63) / 64;
constexpr size_t kScrLossP = kScrP + align256((size_t)kMaxBlocks * kNParam * 4);
constexpr size_t kScratchBytes = kScrLossP + align256((size_t)kMaxBlocks * 4);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), looked up once.
int scratch_ptr(int device, char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(FDTD_EDEVICE, "no device address for the closure scratch array");
    g_ptr[device] = static_cast<char*>(p);
  }
  *out = g_ptr[device];
  return FDTD_OK;
}

}  // namespace
}  // namespace fdtdp

using namespace fdtdp;

extern "C" int fdtd_closure_grad_static(int32_t device, void* hip_stream, const float* params_dev,
                                        const float* x_dev, const float* t_dev, int32_t n,
                                        float* grad_dev, float* loss_dev) {
  if (!params_dev || !x_dev || !t_dev || !grad_dev || !loss_dev)
    return fail(FDTD_EINVAL, "null device pointer");
  if (n < 1 || n > FDTD_CLOSURE_STATIC_MAX_ROWS)
    return fail(FDTD_ERANGE, "row count %d outside [1, %d]", n, FDTD_CLOSURE_STATIC_MAX_ROWS);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e || ndev <= 0) return fail(FDTD_EDEVICE, "no HIP device");
  if (device < 0 || device >= ndev || device >= kMaxDevices)
    return fail(FDTD_EINVAL, "device %d out of range", device);
  e = hipSetDevice(device);
  if (e) return hip_fail(e, "hipSetDevice");
  char* base = nullptr;
  int rc = scratch_ptr(device, &base);
  if (rc) return rc;
  MlpWeights W{};
  W.W1 = reinterpret_cast<uint16_t*>(base + kScrW1);
  W.W2 = reinterpret_cast<uint16_t*>(base + kScrW2);
  W.W2T = reinterpret_cast<uint16_t*>(base + kScrW2T);
  W.W2P = reinterpret_cast<uint16_t*>(base + kScrW2P);
  W.b1 = reinterpret_cast<float*>(base + kScrB1);
  W.b2 = reinterpret_cast<float*>(base + kScrB2);
  W.w3q = reinterpret_cast<float*>(base + kScrW3);
  W.b3 = reinterpret_cast<float*>(base + kScrB3);
  float* P = reinterpret_cast<float*>(base + kScrP);
  float* lossp = reinterpret_cast<float*>(base + kScrLossP);
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // every byte the gradient kernels read is written first in this call (the packed
  // weights by the pack kernel, every partial and loss slot of the n / 64 blocks by the
  // gradient kernel), so nothing is cleared
  e = mlp_launch_pack(params_dev, W, st);
  if (!e) e = mlp_launch_grad(W, x_dev, t_dev, n, P, lossp, grad_dev, loss_dev, st);
  return e ? hip_fail(e, "closure gradient (static scratch)") : FDTD_OK;
}
