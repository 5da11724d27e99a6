// Internal interface of the learned-start network (kernels in pm_net.hip,
// C ABI in pm_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {
namespace net {

typedef __bf16 bf16;

// brick groups of a weight-gradient launch (each writes one partial sum): at
// most kWgradGroups, and no more than kWgradPartialFloats / (27 cin cout)
constexpr int kWgradGroups = 2048;
constexpr int64_t kWgradPartialFloats = 64LL << 20;   // 256 MB of FP32 partial sums
constexpr int kWgradSlices = 64;                       // first-stage slices of their reduction

// Layers in parameter order; weights [taps][cin][cout] FP32 then bias [cout].
enum Layer { E1A, E1B, E2A, E2B, B3A, B3B, D2A, D2B, D1A, D1B, OUT, NLAYER };
struct LayerShape {
  int cin;    // input channels of the parameter tensor
  int cout;
  int taps;   // 27 or 1
  int cin_p;  // input channels as stored on the device (padded to 16)
};
extern const LayerShape kLayers[NLAYER];
int64_t param_count();
int64_t weight_offset(int layer);  // offset of the layer's weights in the flat parameter vector
int64_t bias_offset(int layer);

// Device buffers of one network (owned by the C ABI's pm_net).
struct Buffers {
  int n = 0;          // voxels per axis at level 1 (half or a quarter of the FFT box)
  int max_batch = 0;
  float* params = nullptr;   // FP32 master parameters [P]
  float* grads = nullptr;    // [P]
  float* adam_m = nullptr;   // [P]
  float* adam_v = nullptr;   // [P]
  bf16* wf[NLAYER] = {};     // forward weights [cout][taps][cin_p]
  bf16* wb[NLAYER] = {};     // backward-data weights [cin_p][taps][cout], taps mirrored
  // activations, batch-major, channels last
  bf16 *x = nullptr, *a1 = nullptr, *s1 = nullptr, *p1 = nullptr, *a2 = nullptr, *s2 = nullptr, *p2 = nullptr,
       *a3 = nullptr, *b3 = nullptr, *a4 = nullptr, *d2 = nullptr, *a5 = nullptr, *d1 = nullptr;
  // gradient scratch
  bf16 *g16a = nullptr, *g16b = nullptr, *gc1 = nullptr, *g32a = nullptr, *g32b = nullptr, *gc2 = nullptr,
       *g64a = nullptr, *g64b = nullptr, *gp1 = nullptr, *gp2 = nullptr;
  float* yhat = nullptr;     // [batch][3][n^3]
  float* target = nullptr;   // [batch][3][n^3]
  double* rms = nullptr;     // [max_batch] scale of each slot
  double* sums = nullptr;    // [max_batch + 4] FP64 reduction results
  float* partial = nullptr;  // weight-gradient partial sums
  float* partial2 = nullptr; // [kWgradSlices][27 cin cout] first-stage sums
  int64_t partial_floats = 0;
  double* dpartial = nullptr;  // FP64 block partials
  int64_t dpartial_count = 0;
};

// Sizes in bytes of each buffer group, for allocation.
int64_t level_voxels(int n, int level);  // (n >> level)^3

hipError_t pack_weights(const Buffers& b, hipStream_t st);
hipError_t forward(const Buffers& b, int batch, hipStream_t st);
// loss (FP64 sum of squares / count) lands in b.sums[max_batch]
hipError_t loss_backward(const Buffers& b, int batch, hipStream_t st);
hipError_t adam(const Buffers& b, float lr, float beta1, float beta2, float eps, int step, hipStream_t st);

// The network works on the periodic FFT box of N = 2 n cells per axis at half
// resolution (n^3 voxels, each the mean of a 2 x 2 x 2 block of cells).
// Input of one slot from the Newton potential phiN [N^3]: g_N = -D phi_N
// (central differences), its block means g_c, rms = sqrt(mean |g_c|^2), and
// the channels [g_c / rms, log10(|g_c| / a0 + 1e-30)].
// fb: box cells per network voxel along an axis (n_pad / n), 2 or 4
hipError_t features(const Buffers& b, int slot, const float* phiN, double inv_2s, double a0, int fb, hipStream_t st);
// The slot's block means g_c ([3][n^3] floats, kept in its part of a gradient
// scratch buffer), and the slot's input from block means already written
// there (the scale rms and the channels, as features forms them).
float* feature_means(const Buffers& b, int slot);
hipError_t features_from_means(const Buffers& b, int slot, double a0, hipStream_t st);
// Training target of one slot: block mean of (F - g_N) / rms (F: [3][N^3]).
hipError_t target_from_field(const Buffers& b, int slot, const float* phiN, const float* F, double inv_2s, int fb,
                             hipStream_t st);
// H0 [3][N^3]: rms * yhat of slot 0 repeated over each fb x fb x fb block.
hipError_t start_field(const Buffers& b, float* H0, int fb, hipStream_t st);
// Test helpers: FP32 [4][n^3] (device) -> input channels of a slot.
hipError_t set_input(const Buffers& b, int slot, const float* x4, hipStream_t st);
// and back: the 4 input channels of a slot as FP32 [4][n^3] (device).
hipError_t get_input(const Buffers& b, int slot, float* x4, hipStream_t st);
// A stored activation or gradient tensor of a slot as FP32 channels first
// (device [C][voxels of its level]); which: 0..12 the activations x, a1, s1,
// p1, a2, s2, p2, a3, b3, a4, d2, a5, d1; 13..22 the gradient buffers g16a,
// g16b, gc1, g32a, g32b, gc2, g64a, g64b, gp1, gp2 (their last contents).
hipError_t get_tensor(const Buffers& b, int which, int slot, float* out, hipStream_t st);
// Text naming the step that failed in the last failing call (then cleared).
const char* last_failure();

}  // namespace net
}  // namespace pm
