// Surrogate MLP: fixed architecture 12 -> 256 -> 256 -> 256 -> 256 -> 3.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bpm {

constexpr int kMlpIn = 12, kMlpHidden = 256, kMlpOut = 3, kMlpLayers = 5;
constexpr long kMlpParams = 12L * 256 + 256 + 3L * (256 * 256 + 256) + 256L * 3 + 3;   // 201475

__host__ __device__ constexpr int mlp_size(int i) {
  return i == 0 ? kMlpIn : (i == kMlpLayers ? kMlpOut : kMlpHidden);
}
#define kMlpSizes_(i) ::bpm::mlp_size(i)

struct MlpDevParams {
  __bf16* w[5];     // packed bf16 weights [out_padded][in_padded]: [256][32], 3 x [256][256], [16][256]
  float* b[5];      // biases padded to the same output count
};

struct Mlp {
  int max_batch = 0;
  long step = 0;
  float* theta = nullptr;   // FP32 master parameters, flat: per layer W [out][in] then b [out]
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* Z[5] = {};         // pre-activations [B][out]
  float* Aout[4] = {};      // GELU outputs of the hidden layers
  float* dZ = nullptr;      // [B][3]
  float* dA = nullptr;      // [B][256]
  float* dZh = nullptr;
  float* dZh2 = nullptr;
  double* d_loss = nullptr;
  MlpDevParams dev{};
};

hipError_t mlp_pack(Mlp& net, hipStream_t s);
hipError_t mlp_predict(Mlp& net, const float* X, float* Y, long n, hipStream_t s);
hipError_t mlp_forward_backward(Mlp& net, const float* X, const float* T, const uint8_t* mask, int B, hipStream_t s);
hipError_t mlp_adam(Mlp& net, float lr, hipStream_t s);

// screening (screen.hip)
struct ScreenScratch {
  uint32_t* hist = nullptr;        // [256]
  uint32_t* state = nullptr;       // [8]: prefix, mask, k_rem, count_gt, ...
  uint32_t* blk = nullptr;         // per-block tie counts / offsets
  unsigned long long* cand = nullptr;  // [16384]
  long blk_cap = 0;
};
constexpr long kTopkMax = 16384;
constexpr long kTopkNoAllocMaxN = 1L << 26;          // scores per allocation-free selection
constexpr size_t kTopkNoAllocScratchBytes = 394496;  // its scratch area per GPU
constexpr int kMaxDevices = 64;
hipError_t topk_scratch_init(int device);            // the calling thread's current device
hipError_t topk_select_noalloc(const float* score, long n, long k, int64_t* idx, int device, hipStream_t s);
hipError_t sample_designs(uint64_t seed, long n, float* X, hipStream_t s);
hipError_t design_features(float* X, long n, const double* lo, const double* hi, hipStream_t s);
hipError_t topk_select(const float* score, long n, long k, int64_t* idx, ScreenScratch& sc, hipStream_t s);
hipError_t screen_score(const float* X, const float* Y, long n, const double* lo, const double* hi, double min_stability,
                        float* score, hipStream_t s);

}  // namespace bpm
