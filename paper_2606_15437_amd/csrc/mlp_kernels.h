// Pair-scoring MLP: sizes, parameter layout and device state.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kripke {

constexpr uint32_t kSigWords = 64;  // 4,096-bit signatures
constexpr uint32_t kIn = 8192, kH1 = 512, kH2 = 256;
// FP32 parameter vector: W1 [512][8192], b1 [512], W2 [256][512], b2 [256], w3 [256], b3
constexpr uint64_t kOffW1 = 0;
constexpr uint64_t kOffB1 = kOffW1 + (uint64_t)kH1 * kIn;
constexpr uint64_t kOffW2 = kOffB1 + kH1;
constexpr uint64_t kOffB2 = kOffW2 + (uint64_t)kH2 * kH1;
constexpr uint64_t kOffW3 = kOffB2 + kH2;
constexpr uint64_t kOffB3 = kOffW3 + kH2;
constexpr uint64_t kParams = kOffB3 + 1;  // 4,326,401

struct MlpState {
  uint32_t max_batch = 0;
  int64_t step = 0;
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t *w1b = nullptr, *w2b = nullptr, *w2tb = nullptr;  // bf16 working copies
  uint16_t *a1 = nullptr, *a1t = nullptr, *a2b = nullptr;    // activations (bf16)
  float *a2 = nullptr, *logit = nullptr, *dz = nullptr, *lossv = nullptr;
  float *dh2f = nullptr, *dh1f = nullptr;
  uint16_t *dh2 = nullptr, *dh2t = nullptr, *dh1t = nullptr;
};

hipError_t mlp_refresh(MlpState& S, hipStream_t s);
hipError_t mlp_forward(MlpState& S, const uint64_t* sig, const uint64_t* pairs, uint32_t M,
                       float* logit, bool train, hipStream_t s);
hipError_t mlp_backward(MlpState& S, const uint64_t* sig, const uint64_t* pairs,
                        const float* label, uint32_t M, float pos_weight, float* loss,
                        hipStream_t s);
hipError_t mlp_adam(MlpState& S, float lr, float b1, float b2, float eps, hipStream_t s);

}  // namespace kripke
