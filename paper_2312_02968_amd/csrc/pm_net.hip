// Learned starting guess for the AQUAL iteration (Sect. 2.1 allows any
// divergence-free start; the paper starts from zero): a 3-level
// encoder-decoder of 3x3x3 convolutions on the physical n^3 region.
//
// 3x3x3 convolutions are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation).  Activations
// are BF16, channels last ([batch][z][y][x][C]); weights are packed to BF16
// from FP32 master copies after every optimiser step.  The concatenation of a
// skip tensor with the upsampled coarser tensor is never materialised: the
// consuming convolution reads the skip channels at v and the coarse channels
// at v / 2.
#include <math.h>

#include "pm_net.h"

namespace pm {
namespace net {

const LayerShape kLayers[NLAYER] = {
    {4, 16, 27, 16},  {16, 16, 27, 16}, {16, 32, 27, 16}, {32, 32, 27, 32},
    {32, 64, 27, 32}, {64, 64, 27, 64}, {96, 32, 27, 96}, {32, 32, 27, 32},
    {48, 16, 27, 48}, {16, 16, 27, 16}, {16, 3, 1, 16}};

int64_t weight_offset(int layer) {
  int64_t o = 0;
  for (int l = 0; l < layer; ++l)
    o += (int64_t)kLayers[l].taps * kLayers[l].cin * kLayers[l].cout + kLayers[l].cout;
  return o;
}
int64_t bias_offset(int layer) {
  return weight_offset(layer) + (int64_t)kLayers[layer].taps * kLayers[layer].cin * kLayers[layer].cout;
}
int64_t param_count() { return weight_offset(NLAYER); }
int64_t level_voxels(int n, int level) {
  const int64_t m = n >> level;
  return m * m * m;
}

namespace {

thread_local const char* g_where = nullptr;   // first failing step of the last call

hipError_t launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess && !g_where) g_where = what;
  return e;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;
#ifndef PM_CONV_PAD
#define PM_CONV_PAD 0
#endif
#ifndef PM_CONV_BY
#define PM_CONV_BY 4
#endif
// forward / backward-data brick: 16 x 4 x 4 voxels, one z plane per wave
constexpr int BX = 16, BY = PM_CONV_BY, BZ = 4;
constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;
constexpr int HSLOTS = HX * HY * HZ;
// weight-gradient brick: 16 x 4 x 2 voxels
constexpr int WBX = 16, WBY = 4, WBZ = 2;
constexpr int WROWS = (WBY + 2) * (WBZ + 2);
constexpr int WXS = 3 * WROWS * WBX + 8;   // LDS stride of one input channel (3 x-shifted copies)
constexpr int WGROUPS = kWgradGroups;
constexpr int RGROUPS = 1024;              // blocks of the reductions over voxels

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float bf(bf16 v) { return (float)v; }

// One 16-byte group of 8 input channels of voxel (gx, gy, gz), taken modulo n
// (the grids are periodic, like the FFT box they sample): channels below C0
// from src0 (resolution n), the rest from src1 at half resolution (the
// nearest-neighbour upsampled coarse tensor).  n is a power of two.
template <int CIN, int C0>
__device__ __forceinline__ uint4 load_in8(const bf16* src0, const bf16* src1, int n, int b, int gx, int gy, int gz,
                                          int c) {
  uint4 v;
  gx &= n - 1;
  gy &= n - 1;
  gz &= n - 1;
  if (c < C0) {
    const int64_t idx = (((int64_t)b * n + gz) * n + gy) * n + gx;
    v = *reinterpret_cast<const uint4*>(src0 + idx * C0 + c);
  } else {
    const int nh = n >> 1;
    const int64_t idx = (((int64_t)b * nh + (gz >> 1)) * nh + (gy >> 1)) * nh + (gx >> 1);
    v = *reinterpret_cast<const uint4*>(src1 + idx * (CIN - C0) + (c - C0));
  }
  return v;
}

struct ConvArgs {
  const bf16* src0;   // [batch][n^3][C0]
  const bf16* src1;   // [batch][(n/2)^3][CIN - C0] (upsampled), or null when C0 == CIN
  const bf16* w;      // [COUT][27][CIN]
  const float* bias;  // [COUT] or null
  const bf16* mask;   // [batch][n^3][COUT] or null: outputs where mask <= 0 are zeroed
  bf16* out;          // [batch][n^3][COUT]
  int n;
};

// out[v][o] = bias[o] + sum over taps t and channels c of in[v + tap_t][c] w[o][t][c],
// then ReLU and the mask.  A block owns a 16 x 4 x 4 brick; wave w computes
// its z plane w as 4 rows (M tiles of 16 voxels along x) times COUT / 16
// N tiles.  The input halo brick is staged in LDS in chunks of CC channels;
// a k step of 32 covers 32 / CC taps of one chunk.
template <int CIN, int COUT, int C0, bool RELU>
__global__ __launch_bounds__(NT) void k_conv(ConvArgs a) {
  constexpr int CC = (CIN % 32 == 0) ? 32 : 16;
  constexpr int CS = CC + PM_CONV_PAD;   // voxel slot stride in LDS (bf16); padding measured no faster
  constexpr int NCH = CIN / CC;
  constexpr int KS = (27 * CC + 31) / 32;
  constexpr int NTL = COUT / 16;
  __shared__ uint4 tile4[HSLOTS * CS / 8];

  const int n = a.n;
  const int nbx = (n + BX - 1) / BX, nby = (n + BY - 1) / BY, nbz = (n + BZ - 1) / BZ;
  int bid = blockIdx.x;
  const int bx = bid % nbx;
  bid /= nbx;
  const int by = bid % nby;
  bid /= nby;
  const int bz = bid % nbz;
  const int b = bid / nbz;
  const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;

  f32x4 acc[BY][NTL];
#pragma unroll
  for (int i = 0; i < BY; ++i)
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int ch = 0; ch < NCH; ++ch) {
    if (ch) __syncthreads();
    for (int u = tid; u < HSLOTS * (CC / 8); u += NT) {
      const int slot = u / (CC / 8), cg = u % (CC / 8);
      const int sx = slot % HX, sy = (slot / HX) % HY, sz = slot / (HX * HY);
      tile4[(slot * CS + cg * 8) / 8] =
          load_in8<CIN, C0>(a.src0, a.src1, n, b, x0 - 1 + sx, y0 - 1 + sy, z0 - 1 + sz, ch * CC + cg * 8);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = ks * 32 + 8 * g;
      const int tap = k0 / CC, c = k0 % CC;
      const bool valid = tap < 27;
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
      bf16x8 bw[NTL];
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        uint4 wv = make_uint4(0u, 0u, 0u, 0u);
        if (valid) wv = *reinterpret_cast<const uint4*>(a.w + ((int64_t)(16 * t + m) * 27 + tap) * CIN + ch * CC + c);
        bw[t] = as_bf16x8(wv);
      }
#pragma unroll
      for (int i = 0; i < BY; ++i) {
        uint4 av = make_uint4(0u, 0u, 0u, 0u);
        if (valid) {
          const int slot = ((wave + 1 + dz) * HY + (i + 1 + dy)) * HX + (m + 1 + dx);
          av = tile4[(slot * CS + c) / 8];
        }
        const bf16x8 af = as_bf16x8(av);
#pragma unroll
        for (int t = 0; t < NTL; ++t) acc[i][t] = mfma(af, bw[t], acc[i][t]);
      }
    }
  }

  // lane holds voxel x = 4 g + j of row i, channel o = 16 t + m
  const int gz = z0 + wave;
#pragma unroll
  for (int i = 0; i < BY; ++i) {
    const int gy = y0 + i;
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      const int o = 16 * t + m;
      const float bo = a.bias ? a.bias[o] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gx = x0 + 4 * g + j;
        if (gx < n && gy < n && gz < n) {
          const int64_t idx = (((int64_t)b * n + gz) * n + gy) * n + gx;
          float v = acc[i][t][j] + bo;
          if (RELU) v = fmaxf(v, 0.0f);
          if (a.mask && !(bf(a.mask[idx * COUT + o]) > 0.0f)) v = 0.0f;
          a.out[idx * COUT + o] = (bf16)v;
        }
      }
    }
  }
}

struct WgradArgs {
  const bf16* src0;
  const bf16* src1;
  const bf16* gz;     // [batch][n^3][COUT]
  float* partial;     // [G][27][CIN][COUT]
  int n, batch, G;
};

// Weight gradient gw[t][c][o] = sum_v in[v + tap_t][c] gz[v][o] as a GEMM
// with the voxels as the reduction axis: A = gz^T (16 output channels x 32
// voxels), B = the shifted input (32 voxels x 16 input channels of one tap).
// Block (G, CIN / 16): brick group blockIdx.x, channel chunk blockIdx.y.  Both
// operands are staged transposed in LDS (voxels contiguous), the input in
// three copies shifted by dx = -1, 0, 1 so that every 8-voxel read is aligned.
// Wave w owns output tile mt = w mod (COUT / 16) and the taps t = q, q + WPM,
// ... with q = w / (COUT / 16).
template <int CIN, int COUT, int C0>
__global__ __launch_bounds__(NT) void k_wgrad(WgradArgs a) {
  constexpr int MT = COUT / 16;
  constexpr int WPM = 4 / MT;
  constexpr int NTAP = (27 + WPM - 1) / WPM;
  constexpr int GS = WBX * WBY * WBZ + 8;
  __shared__ bf16 xin[16 * WXS];
  __shared__ bf16 gzT[COUT * GS];

  const int ch = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
  const int mt = wave % MT, q = wave / MT;
  const int n = a.n;
  const int nbx = (n + WBX - 1) / WBX, nby = (n + WBY - 1) / WBY, nbz = (n + WBZ - 1) / WBZ;
  const int nbricks = nbx * nby * nbz * a.batch;

  f32x4 acc[NTAP];
#pragma unroll
  for (int i = 0; i < NTAP; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int br = blockIdx.x; br < nbricks; br += a.G) {
    int r_ = br;
    const int bx = r_ % nbx;
    r_ /= nbx;
    const int by = r_ % nby;
    r_ /= nby;
    const int bz = r_ % nbz;
    const int b = r_ / nbz;
    const int x0 = bx * WBX, y0 = by * WBY, z0 = bz * WBZ;
    __syncthreads();
    for (int u = tid; u < WBX * WBY * WBZ * (COUT / 8); u += NT) {
      const int v = u / (COUT / 8), og = u % (COUT / 8);
      const int x = v % WBX, y = (v / WBX) % WBY, z = v / (WBX * WBY);
      const int gx = x0 + x, gy = y0 + y, gzz = z0 + z;
      uint4 val = make_uint4(0u, 0u, 0u, 0u);
      if (gx < n && gy < n && gzz < n) {
        const int64_t idx = (((int64_t)b * n + gzz) * n + gy) * n + gx;
        val = *reinterpret_cast<const uint4*>(a.gz + idx * COUT + og * 8);
      }
      const bf16* e = reinterpret_cast<const bf16*>(&val);
#pragma unroll
      for (int i = 0; i < 8; ++i) gzT[(og * 8 + i) * GS + v] = e[i];
    }
    for (int u = tid; u < WROWS * (WBX + 2) * 2; u += NT) {
      const int half = u & 1, rest = u >> 1;
      const int hx = rest % (WBX + 2), row = rest / (WBX + 2);
      const int sy = row % (WBY + 2), sz = row / (WBY + 2);
      const uint4 val = load_in8<CIN, C0>(a.src0, a.src1, n, b, x0 - 1 + hx, y0 - 1 + sy, z0 - 1 + sz,
                                          ch * 16 + half * 8);
      const bf16* e = reinterpret_cast<const bf16*>(&val);
#pragma unroll
      for (int dxs = 0; dxs < 3; ++dxs) {
        const int xx = hx - dxs;
        if (xx >= 0 && xx < WBX) {
#pragma unroll
          for (int i = 0; i < 8; ++i) xin[(half * 8 + i) * WXS + (row * 3 + dxs) * WBX + xx] = e[i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < (WBX * WBY * WBZ) / 32; ++ks) {
      const int r = 2 * ks + (g >> 1), xg = 8 * (g & 1);
      const int y = r % WBY, z = r / WBY;
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(gzT + (16 * mt + m) * GS + 32 * ks + 8 * g);
#pragma unroll
      for (int i = 0; i < NTAP; ++i) {
        const int t = q + i * WPM;
        if (t < 27) {
          const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
          const int row = (z + 1 + dz) * (WBY + 2) + (y + 1 + dy);
          const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(xin + m * WXS + (row * 3 + dx + 1) * WBX + xg);
          acc[i] = mfma(af, bfr, acc[i]);
        }
      }
    }
  }
  // lane holds D[o = 16 mt + 4 g + j][c = m]
  float* P = a.partial + (int64_t)blockIdx.x * 27 * CIN * COUT;
#pragma unroll
  for (int i = 0; i < NTAP; ++i) {
    const int t = q + i * WPM;
    if (t < 27) {
#pragma unroll
      for (int j = 0; j < 4; ++j) P[((int64_t)t * CIN + ch * 16 + m) * COUT + 16 * mt + 4 * g + j] = acc[i][j];
    }
  }
}

// Two-stage sum over the brick groups.  Stage 1: part2[s][i] = sum over the
// groups of slice s (blockIdx.y) of partial[g][t][c][o], with
// i = (t cin_real + c) COUT + o and c < cin_real.
__global__ __launch_bounds__(NT) void k_reduce_wgrad1(const float* __restrict__ partial, int G, int S, int CIN,
                                                      int COUT, int cin_real, float* __restrict__ part2) {
  const int64_t count = 27LL * cin_real * COUT;
  const int64_t stride = 27LL * CIN * COUT;
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= count) return;
  const int o = (int)(i % COUT);
  const int64_t tc = i / COUT;
  const int c = (int)(tc % cin_real), t = (int)(tc / cin_real);
  const int64_t src = ((int64_t)t * CIN + c) * COUT + o;
  const int s = blockIdx.y;
  const int g0 = (int)((int64_t)G * s / S), g1 = (int)((int64_t)G * (s + 1) / S);
  float acc = 0.0f;
  for (int gi = g0; gi < g1; ++gi) acc += partial[gi * stride + src];
  part2[s * count + i] = acc;
}

// Stage 2: out[i] = sum over slices of part2[s][i].
__global__ __launch_bounds__(NT) void k_reduce_wgrad2(const float* __restrict__ part2, int S, int64_t count,
                                                      float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= count) return;
  float acc = 0.0f;
  for (int s = 0; s < S; ++s) acc += part2[s * count + i];
  out[i] = acc;
}

// partial[block][c] = sum over this block's voxels of g[v][c]; a thread reads
// 8 channels (16 bytes) at a time (C a multiple of 8 dividing 256)
__global__ __launch_bounds__(NT) void k_colsum(const bf16* __restrict__ g, int64_t nvox, int C, float* partial) {
  __shared__ float red[NT * 8];
  const int groups = C / 8, cg = threadIdx.x % groups, lanes = NT / groups, l = threadIdx.x / groups;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t v = blockIdx.x * (int64_t)lanes + l; v < nvox; v += (int64_t)gridDim.x * lanes) {
    const uint4 u = *reinterpret_cast<const uint4*>(g + v * C + cg * 8);
    const bf16* e = reinterpret_cast<const bf16*>(&u);
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] += bf(e[i]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) red[threadIdx.x * 8 + i] = s[i];
  __syncthreads();
  if (threadIdx.x < C) {
    const int c = threadIdx.x, g8 = c / 8, i = c % 8;
    float t = 0.0f;
    for (int k = 0; k < lanes; ++k) t += red[(k * groups + g8) * 8 + i];
    partial[blockIdx.x * C + c] = t;
  }
}

// out[c] = sum over k of partial[k * C + c]; one block, C divides 256
__global__ __launch_bounds__(NT) void k_reduce_cols(const float* __restrict__ partial, int nblk, int C, float* out) {
  __shared__ float red[NT];
  const int c = threadIdx.x % C, lanes = NT / C;
  float s = 0.0f;
  for (int k = threadIdx.x / C; k < nblk; k += lanes) s += partial[k * C + c];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < C) {
    float t = 0.0f;
    for (int l = 0; l < lanes; ++l) t += red[l * C + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// 2 x 2 x 2 average pooling: out at level size nh = n / 2
template <int C>
__global__ __launch_bounds__(NT) void k_pool(const bf16* __restrict__ in, bf16* __restrict__ out, int n, int batch) {
  const int nh = n >> 1;
  const int64_t units = (int64_t)batch * nh * nh * nh * (C / 8);
  for (int64_t u = blockIdx.x * (int64_t)NT + threadIdx.x; u < units; u += (int64_t)gridDim.x * NT) {
    const int cg = (int)(u % (C / 8));
    int64_t v = u / (C / 8);
    const int x = (int)(v % nh);
    v /= nh;
    const int y = (int)(v % nh);
    v /= nh;
    const int z = (int)(v % nh);
    const int b = (int)(v / nh);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t idx = (((int64_t)b * n + 2 * z + (k >> 2)) * n + 2 * y + ((k >> 1) & 1)) * n + 2 * x + (k & 1);
      const uint4 val = *reinterpret_cast<const uint4*>(in + idx * C + cg * 8);
      const bf16* e = reinterpret_cast<const bf16*>(&val);
#pragma unroll
      for (int i = 0; i < 8; ++i) s[i] += bf(e[i]);
    }
    uint4 o;
    bf16* oe = reinterpret_cast<bf16*>(&o);
#pragma unroll
    for (int i = 0; i < 8; ++i) oe[i] = (bf16)(s[i] * 0.125f);
    const int64_t oidx = (((int64_t)b * nh + z) * nh + y) * nh + x;
    *reinterpret_cast<uint4*>(out + oidx * C + cg * 8) = o;
  }
}

// Gradient of the upsampled branch: out[v'][c] = sum over the 8 children of
// gcat[child][COFF + c], zeroed where act[v'][c] <= 0 (ReLU of the coarse layer).
template <int CCAT, int COFF, int C>
__global__ __launch_bounds__(NT) void k_upgrad(const bf16* __restrict__ gcat, const bf16* __restrict__ act,
                                               bf16* __restrict__ out, int n, int batch) {
  const int nh = n >> 1;
  const int64_t units = (int64_t)batch * nh * nh * nh * (C / 8);
  for (int64_t u = blockIdx.x * (int64_t)NT + threadIdx.x; u < units; u += (int64_t)gridDim.x * NT) {
    const int cg = (int)(u % (C / 8));
    int64_t v = u / (C / 8);
    const int64_t vc = v;
    const int x = (int)(v % nh);
    v /= nh;
    const int y = (int)(v % nh);
    v /= nh;
    const int z = (int)(v % nh);
    const int b = (int)(v / nh);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t idx = (((int64_t)b * n + 2 * z + (k >> 2)) * n + 2 * y + ((k >> 1) & 1)) * n + 2 * x + (k & 1);
      const uint4 val = *reinterpret_cast<const uint4*>(gcat + idx * CCAT + COFF + cg * 8);
      const bf16* e = reinterpret_cast<const bf16*>(&val);
#pragma unroll
      for (int i = 0; i < 8; ++i) s[i] += bf(e[i]);
    }
    const uint4 av = *reinterpret_cast<const uint4*>(act + vc * C + cg * 8);
    const bf16* ae = reinterpret_cast<const bf16*>(&av);
    uint4 o;
    bf16* oe = reinterpret_cast<bf16*>(&o);
#pragma unroll
    for (int i = 0; i < 8; ++i) oe[i] = (bf16)(bf(ae[i]) > 0.0f ? s[i] : 0.0f);
    *reinterpret_cast<uint4*>(out + vc * C + cg * 8) = o;
  }
}

// Gradient of a skip tensor: out[v][c] = gcat[v][c] + gpool[parent(v)][c] / 8,
// zeroed where act[v][c] <= 0.
template <int CCAT, int C>
__global__ __launch_bounds__(NT) void k_poolgrad(const bf16* __restrict__ gcat, const bf16* __restrict__ gpool,
                                                 const bf16* __restrict__ act, bf16* __restrict__ out, int n,
                                                 int batch) {
  const int nh = n >> 1;
  const int64_t units = (int64_t)batch * n * n * n * (C / 8);
  for (int64_t u = blockIdx.x * (int64_t)NT + threadIdx.x; u < units; u += (int64_t)gridDim.x * NT) {
    const int cg = (int)(u % (C / 8));
    int64_t v = u / (C / 8);
    const int64_t vf = v;
    const int x = (int)(v % n);
    v /= n;
    const int y = (int)(v % n);
    v /= n;
    const int z = (int)(v % n);
    const int b = (int)(v / n);
    const int64_t pidx = (((int64_t)b * nh + (z >> 1)) * nh + (y >> 1)) * nh + (x >> 1);
    const uint4 gv = *reinterpret_cast<const uint4*>(gcat + vf * CCAT + cg * 8);
    const uint4 pv = *reinterpret_cast<const uint4*>(gpool + pidx * C + cg * 8);
    const uint4 av = *reinterpret_cast<const uint4*>(act + vf * C + cg * 8);
    const bf16* ge = reinterpret_cast<const bf16*>(&gv);
    const bf16* pe = reinterpret_cast<const bf16*>(&pv);
    const bf16* ae = reinterpret_cast<const bf16*>(&av);
    uint4 o;
    bf16* oe = reinterpret_cast<bf16*>(&o);
#pragma unroll
    for (int i = 0; i < 8; ++i) oe[i] = (bf16)(bf(ae[i]) > 0.0f ? bf(ge[i]) + 0.125f * bf(pe[i]) : 0.0f);
    *reinterpret_cast<uint4*>(out + vf * C + cg * 8) = o;
  }
}

// Block reduction of NV doubles per thread into part[blockIdx.x * NV + k].
template <int NV>
__device__ void block_reduce_store(double (&v)[NV], double* part) {
  __shared__ double red[NT / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += NT) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w][k];
    part[blockIdx.x * NV + k] = s;
  }
}

// out[k] = sum over blocks of part[b * nv + k] (FP64); one block, all threads
// share every k
__global__ __launch_bounds__(NT) void k_reduce_d(const double* __restrict__ part, int nblk, int nv, double* out) {
  __shared__ double red[NT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) s += part[b * nv + k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red[w];
      out[k] = t;
    }
    __syncthreads();
  }
}

// 1x1x1 head: y[c] = sum_k w[c][k] d1[k] + bias[c] (w: [3][1][16] BF16).
// MODE 0 stores yhat; MODE 1 also forms the loss, its gradient and the head
// gradients: e = y - t, gy = 2 e / count, gz[k] = (d1[k] > 0) sum_c w[c][k] gy[c].
template <int MODE>
__global__ __launch_bounds__(NT) void k_head(const bf16* __restrict__ d1, const bf16* __restrict__ w,
                                             const float* __restrict__ bias, float* __restrict__ yhat,
                                             const float* __restrict__ target, bf16* __restrict__ gz, int64_t nvox,
                                             int batch, double inv_count, double* part) {
  float wf[3][16];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < 16; ++k) wf[c][k] = bf(w[c * 16 + k]);
  const float b0 = bias[0], b1 = bias[1], b2 = bias[2];
  constexpr int NV = (MODE == 1) ? 52 : 1;
  double accv[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) accv[k] = 0.0;
  const int64_t total = nvox * batch;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
    const int b = (int)(i / nvox);
    const int64_t v = i % nvox;
    uint4 u0 = *reinterpret_cast<const uint4*>(d1 + i * 16);
    uint4 u1 = *reinterpret_cast<const uint4*>(d1 + i * 16 + 8);
    float h[16];
    const bf16* e0 = reinterpret_cast<const bf16*>(&u0);
    const bf16* e1 = reinterpret_cast<const bf16*>(&u1);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      h[k] = bf(e0[k]);
      h[k + 8] = bf(e1[k]);
    }
    float y[3] = {b0, b1, b2};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 16; ++k) y[c] = fmaf(wf[c][k], h[k], y[c]);
    float* yb = yhat + (int64_t)b * 3 * nvox + v;
    yb[0] = y[0];
    yb[nvox] = y[1];
    yb[2 * nvox] = y[2];
    if constexpr (MODE == 1) {
      const float* tb = target + (int64_t)b * 3 * nvox + v;
      float gy[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double e = (double)y[c] - (double)tb[c * nvox];
        accv[51] += e * e;
        gy[c] = (float)(2.0 * e * inv_count);
        accv[48 + c] += gy[c];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) accv[k * 3 + c] += (double)h[k] * gy[c];
      uint4 o0, o1;
      bf16* oe0 = reinterpret_cast<bf16*>(&o0);
      bf16* oe1 = reinterpret_cast<bf16*>(&o1);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const float s = wf[0][k] * gy[0] + wf[1][k] * gy[1] + wf[2][k] * gy[2];
        const bf16 r = (bf16)(h[k] > 0.0f ? s : 0.0f);
        if (k < 8) oe0[k] = r; else oe1[k - 8] = r;
      }
      *reinterpret_cast<uint4*>(gz + i * 16) = o0;
      *reinterpret_cast<uint4*>(gz + i * 16 + 8) = o1;
    }
  }
  if constexpr (MODE == 1) block_reduce_store<NV>(accv, part);
}

// Head gradients from the reduced sums: sums[k * 3 + c] = dL/dw[k][c],
// sums[48 + c] = dL/db[c], sums[51] = sum of squared errors.
__global__ void k_head_grads(const double* __restrict__ sums, float* gw, float* gb, double* loss, double inv_count) {
  const int t = threadIdx.x;
  if (t < 48) gw[t] = (float)sums[t];
  if (t < 3) gb[t] = (float)sums[48 + t];
  if (t == 0) *loss = sums[51] * inv_count;
}

// Central-difference gradient D phi at box cell (x, y, z) (periodic).
__device__ __forceinline__ void dphi(const float* __restrict__ phi, int x, int y, int z, int N, float inv_2s,
                                     float* d) {
  const int m = N - 1;
  const int64_t NN = (int64_t)N * N;
  const int64_t zr = (int64_t)z * NN, yr = (int64_t)y * N;
  d[0] = (phi[zr + yr + ((x + 1) & m)] - phi[zr + yr + ((x - 1) & m)]) * inv_2s;
  d[1] = (phi[zr + (int64_t)((y + 1) & m) * N + x] - phi[zr + (int64_t)((y - 1) & m) * N + x]) * inv_2s;
  d[2] = (phi[(int64_t)((z + 1) & m) * NN + yr + x] - phi[(int64_t)((z - 1) & m) * NN + yr + x]) * inv_2s;
}

// Block mean of g_N = -D phi_N over the FB^3 cells of coarse voxel (X, Y, Z)
// (FB = N / n: 2, or 4 for the quarter-resolution network).
template <int FB>
__device__ __forceinline__ void coarse_gN(const float* __restrict__ phi, int X, int Y, int Z, int N, float inv_2s,
                                          float* g) {
  g[0] = g[1] = g[2] = 0.0f;
#pragma unroll
  for (int k = 0; k < FB * FB * FB; ++k) {
    float d[3];
    dphi(phi, FB * X + k % FB, FB * Y + (k / FB) % FB, FB * Z + k / (FB * FB), N, inv_2s, d);
    g[0] -= d[0];
    g[1] -= d[1];
    g[2] -= d[2];
  }
  constexpr float w = 1.0f / (FB * FB * FB);
  g[0] *= w;
  g[1] *= w;
  g[2] *= w;
}

// coarse voxel index v of an n^3 grid (n = N / FB) -> (X, Y, Z)
__device__ __forceinline__ void coarse_xyz(int64_t v, int n, int& X, int& Y, int& Z) {
  X = (int)(v % n);
  Y = (int)((v / n) % n);
  Z = (int)(v / ((int64_t)n * n));
}

template <int FB>
__global__ __launch_bounds__(NT) void k_feat_g(const float* __restrict__ phi, int n, float inv_2s, float* __restrict__ g3,
                                               double* part) {
  // the block means g_c of every voxel, kept as g3[c][v] for k_feat_write,
  // and the FP64 partial sums of |g_c|^2 for the scale
  double acc[1] = {0.0};
  const int N = FB * n;
  const int64_t nvox = (int64_t)n * n * n;
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
    int X, Y, Z;
    coarse_xyz(v, n, X, Y, Z);
    float g[3];
    coarse_gN<FB>(phi, X, Y, Z, N, inv_2s, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) g3[c * nvox + v] = g[c];
    acc[0] += (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
  }
  block_reduce_store<1>(acc, part);
}

// x[v] = [g_c / rms, log10(|g_c| / a0 + 1e-30), 0 ...] from the block means
// k_feat_g kept, so the full-resolution potential is read once
__global__ __launch_bounds__(NT) void k_feat_write(const float* __restrict__ g3, int64_t nvox, float inv_a0,
                                                   const double* __restrict__ sumsq, double* rms_out,
                                                   bf16* __restrict__ x) {
  const double rms = sqrt(*sumsq / (double)nvox);
  const float scale = rms > 0.0 ? (float)(1.0 / rms) : 0.0f;
  if (blockIdx.x == 0 && threadIdx.x == 0) *rms_out = rms;
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
    const float g[3] = {g3[v], g3[nvox + v], g3[2 * nvox + v]};
    const float mag = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    uint4 o0 = make_uint4(0u, 0u, 0u, 0u), o1 = make_uint4(0u, 0u, 0u, 0u);
    bf16* e = reinterpret_cast<bf16*>(&o0);
    e[0] = (bf16)(g[0] * scale);
    e[1] = (bf16)(g[1] * scale);
    e[2] = (bf16)(g[2] * scale);
    e[3] = (bf16)log10f(mag * inv_a0 + 1e-30f);
    *reinterpret_cast<uint4*>(x + v * 16) = o0;
    *reinterpret_cast<uint4*>(x + v * 16 + 8) = o1;
  }
}

// FP64 partial sums of |g_c|^2 over the block means g3[c][v]
__global__ __launch_bounds__(NT) void k_sumsq3(const float* __restrict__ g3, int64_t nvox, double* part) {
  double acc[1] = {0.0};
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
    const float g0 = g3[v], g1 = g3[nvox + v], g2 = g3[2 * nvox + v];
    acc[0] += (double)g0 * g0 + (double)g1 * g1 + (double)g2 * g2;
  }
  block_reduce_store<1>(acc, part);
}

// target[c][v] = block mean of (F[c] - g_N[c]) = (F[c] + D_c phi_N), over rms
template <int FB>
__global__ __launch_bounds__(NT) void k_target(const float* __restrict__ phi, const float* __restrict__ F, int n,
                                               float inv_2s, const double* __restrict__ rms, float* __restrict__ t) {
  const int N = FB * n;
  const int64_t nvox = (int64_t)n * n * n, cs = (int64_t)N * N * N;
  const double r = *rms;
  const float inv = r > 0.0 ? (float)(1.0 / (FB * FB * FB * r)) : 0.0f;
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
    int X, Y, Z;
    coarse_xyz(v, n, X, Y, Z);
    float h[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < FB * FB * FB; ++k) {
      const int x = FB * X + k % FB, y = FB * Y + (k / FB) % FB, z = FB * Z + k / (FB * FB);
      float d[3];
      dphi(phi, x, y, z, N, inv_2s, d);
      const int64_t j = ((int64_t)z * N + y) * N + x;
#pragma unroll
      for (int c = 0; c < 3; ++c) h[c] += F[c * cs + j] + d[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c * nvox + v] = h[c] * inv;
  }
}

// H0[c][j] = rms * yhat[c][parent(j)] for every cell j of the N^3 box
template <int FB>
__global__ __launch_bounds__(NT) void k_start(const float* __restrict__ yhat, const double* __restrict__ rms, int n,
                                              float* __restrict__ H0) {
  const int N = FB * n;
  const int64_t nvox = (int64_t)n * n * n, cs = (int64_t)N * N * N;
  const float r = (float)*rms;
  for (int64_t j = blockIdx.x * (int64_t)NT + threadIdx.x; j < cs; j += (int64_t)gridDim.x * NT) {
    const int x = (int)(j % N), y = (int)((j / N) % N), z = (int)(j / ((int64_t)N * N));
    const int64_t v = ((int64_t)(z / FB) * n + (y / FB)) * n + (x / FB);
#pragma unroll
    for (int c = 0; c < 3; ++c) H0[c * cs + j] = r * yhat[c * nvox + v];
  }
}

__global__ __launch_bounds__(NT) void k_set_input(const float* __restrict__ x4, int64_t nvox, bf16* __restrict__ x) {
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
    uint4 o0 = make_uint4(0u, 0u, 0u, 0u), o1 = make_uint4(0u, 0u, 0u, 0u);
    bf16* e = reinterpret_cast<bf16*>(&o0);
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = (bf16)x4[c * nvox + v];
    *reinterpret_cast<uint4*>(x + v * 16) = o0;
    *reinterpret_cast<uint4*>(x + v * 16 + 8) = o1;
  }
}

__global__ __launch_bounds__(NT) void k_get_input(const bf16* __restrict__ x, int64_t nvox, float* __restrict__ x4) {
  for (int64_t v = blockIdx.x * (int64_t)NT + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * NT) {
#pragma unroll
    for (int c = 0; c < 4; ++c) x4[c * nvox + v] = bf(x[v * 16 + c]);
  }
}

// out[c][v] = t[v][cs + c] for c < C (a stored tensor, channels last with
// pitch CP, as FP32 channels first)
__global__ __launch_bounds__(NT) void k_get_tensor(const bf16* __restrict__ t, int64_t nvox, int CP, int C,
                                                   float* __restrict__ out) {
  const int64_t total = nvox * C;
  for (int64_t j = blockIdx.x * (int64_t)NT + threadIdx.x; j < total; j += (int64_t)gridDim.x * NT) {
    const int c = (int)(j / nvox);
    const int64_t v = j % nvox;
    out[j] = bf(t[v * CP + c]);
  }
}

// wf[o][t][c] = w[t][c][o] (zero for c >= cin); wb[c][t][o] = w[taps - 1 - t][c][o]
__global__ __launch_bounds__(NT) void k_pack(const float* __restrict__ w, int taps, int cin, int cin_p, int cout,
                                             bf16* __restrict__ wf, bf16* __restrict__ wb) {
  const int64_t count = (int64_t)taps * cin_p * cout;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < count; i += (int64_t)gridDim.x * NT) {
    const int c = (int)(i % cin_p);
    const int64_t ot = i / cin_p;
    const int t = (int)(ot % taps), o = (int)(ot / taps);
    wf[i] = (bf16)(c < cin ? w[((int64_t)t * cin + c) * cout + o] : 0.0f);
    // same element count, other order: i = (c taps + t) cout + o
    const int o2 = (int)(i % cout);
    const int64_t ct = i / cout;
    const int t2 = (int)(ct % taps), c2 = (int)(ct / taps);
    wb[i] = (bf16)(c2 < cin ? w[((int64_t)(taps - 1 - t2) * cin + c2) * cout + o2] : 0.0f);
  }
}

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= lr (m c1) / (sqrt(v c2) + eps), c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ __launch_bounds__(NT) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                             float* __restrict__ v, int64_t count, float lr, float b1, float b2,
                                             float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < count; i += (int64_t)gridDim.x * NT) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

int grid_for(int64_t units) {
  const int64_t b = (units + NT - 1) / NT;
  return (int)(b < RGROUPS ? (b < 1 ? 1 : b) : RGROUPS);
}

int conv_blocks(int n, int batch) {
  return ((n + BX - 1) / BX) * ((n + BY - 1) / BY) * ((n + BZ - 1) / BZ) * batch;
}

template <int CIN, int COUT, int C0, bool RELU>
hipError_t conv(const bf16* s0, const bf16* s1, const bf16* w, const float* bias, const bf16* mask, bf16* out, int n,
                int batch, hipStream_t st) {
  ConvArgs a{s0, s1, w, bias, mask, out, n};
  hipLaunchKernelGGL((k_conv<CIN, COUT, C0, RELU>), dim3(conv_blocks(n, batch)), dim3(NT), 0, st, a);
  return launched("k_conv");
}

#define NETCHK(call)                         \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) {                  \
      if (!g_where) g_where = #call;         \
      return e_;                             \
    }                                        \
  } while (0)

template <int CIN, int COUT, int C0>
hipError_t wgrad(const Buffers& B, int layer, const bf16* s0, const bf16* s1, const bf16* gz, int n, int batch,
                 hipStream_t st) {
  // as many brick groups as the partial-sum buffer holds (up to 2048), so that
  // even the 16-channel layers put several blocks on every CU
  const int nbricks = ((n + WBX - 1) / WBX) * ((n + WBY - 1) / WBY) * ((n + WBZ - 1) / WBZ) * batch;
  int64_t gmax = B.partial_floats / (27LL * CIN * COUT);
  if (gmax > WGROUPS) gmax = WGROUPS;
  const int G = nbricks < gmax ? nbricks : (int)gmax;
  if (G < 1 || (int64_t)G * 27 * CIN * COUT > B.partial_floats) {
    g_where = "weight-gradient partial buffer too small";
    return hipErrorInvalidValue;
  }
  WgradArgs a{s0, s1, gz, B.partial, n, batch, G};
  hipLaunchKernelGGL((k_wgrad<CIN, COUT, C0>), dim3(G, CIN / 16), dim3(NT), 0, st, a);
  NETCHK(launched("k_wgrad"));
  const int cin_real = kLayers[layer].cin;
  const int64_t cnt = 27LL * cin_real * COUT;
  const int S = G < kWgradSlices ? G : kWgradSlices;
  const int nbx = (int)((cnt + NT - 1) / NT);
  hipLaunchKernelGGL(k_reduce_wgrad1, dim3(nbx, S), dim3(NT), 0, st, B.partial, G, S, CIN, COUT, cin_real,
                     B.partial2);
  NETCHK(launched("k_reduce_wgrad1"));
  hipLaunchKernelGGL(k_reduce_wgrad2, dim3(nbx), dim3(NT), 0, st, B.partial2, S, cnt,
                     B.grads + weight_offset(layer));
  NETCHK(launched("k_reduce_wgrad2"));
  const int64_t nvox = level_voxels(n, 0) * batch;
  const int nb = grid_for(nvox / (NT / (COUT / 8)) + 1);
  hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(NT), 0, st, gz, nvox, COUT, B.partial);
  NETCHK(launched("k_colsum"));
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(NT), 0, st, B.partial, nb, COUT, B.grads + bias_offset(layer));
  return launched("k_reduce_cols");
}

template <int C>
hipError_t pool(const bf16* in, bf16* out, int n, int batch, hipStream_t st) {
  const int nh = n >> 1;
  hipLaunchKernelGGL((k_pool<C>), dim3(grid_for((int64_t)batch * nh * nh * nh * (C / 8))), dim3(NT), 0, st, in, out,
                     n, batch);
  return launched("k_pool");
}

}  // namespace

const char* last_failure() {
  const char* w = g_where;
  g_where = nullptr;
  return w ? w : "";
}

hipError_t pack_weights(const Buffers& b, hipStream_t st) {
  for (int l = 0; l < NLAYER; ++l) {
    const LayerShape& L = kLayers[l];
    const int64_t cnt = (int64_t)L.taps * L.cin_p * L.cout;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(cnt)), dim3(NT), 0, st, b.params + weight_offset(l), L.taps, L.cin,
                       L.cin_p, L.cout, b.wf[l], b.wb[l]);
    NETCHK(launched("k_pack"));
  }
  return hipSuccess;
}

hipError_t forward(const Buffers& B, int batch, hipStream_t st) {
  const int n = B.n, n2 = n >> 1, n4 = n >> 2;
  auto bias = [&](int l) { return B.params + bias_offset(l); };
  NETCHK((conv<16, 16, 16, true>(B.x, nullptr, B.wf[E1A], bias(E1A), nullptr, B.a1, n, batch, st)));
  NETCHK((conv<16, 16, 16, true>(B.a1, nullptr, B.wf[E1B], bias(E1B), nullptr, B.s1, n, batch, st)));
  NETCHK(pool<16>(B.s1, B.p1, n, batch, st));
  NETCHK((conv<16, 32, 16, true>(B.p1, nullptr, B.wf[E2A], bias(E2A), nullptr, B.a2, n2, batch, st)));
  NETCHK((conv<32, 32, 32, true>(B.a2, nullptr, B.wf[E2B], bias(E2B), nullptr, B.s2, n2, batch, st)));
  NETCHK(pool<32>(B.s2, B.p2, n2, batch, st));
  NETCHK((conv<32, 64, 32, true>(B.p2, nullptr, B.wf[B3A], bias(B3A), nullptr, B.a3, n4, batch, st)));
  NETCHK((conv<64, 64, 64, true>(B.a3, nullptr, B.wf[B3B], bias(B3B), nullptr, B.b3, n4, batch, st)));
  NETCHK((conv<96, 32, 32, true>(B.s2, B.b3, B.wf[D2A], bias(D2A), nullptr, B.a4, n2, batch, st)));
  NETCHK((conv<32, 32, 32, true>(B.a4, nullptr, B.wf[D2B], bias(D2B), nullptr, B.d2, n2, batch, st)));
  NETCHK((conv<48, 16, 16, true>(B.s1, B.d2, B.wf[D1A], bias(D1A), nullptr, B.a5, n, batch, st)));
  NETCHK((conv<16, 16, 16, true>(B.a5, nullptr, B.wf[D1B], bias(D1B), nullptr, B.d1, n, batch, st)));
  const int64_t nvox = level_voxels(n, 0);
  hipLaunchKernelGGL((k_head<0>), dim3(grid_for(nvox * batch)), dim3(NT), 0, st, B.d1, B.wf[OUT], bias(OUT), B.yhat,
                     nullptr, nullptr, nvox, batch, 0.0, nullptr);
  return launched("k_head");
}

hipError_t loss_backward(const Buffers& B, int batch, hipStream_t st) {
  const int n = B.n, n2 = n >> 1, n4 = n >> 2;
  const int64_t nvox = level_voxels(n, 0);
  const double inv_count = 1.0 / (3.0 * (double)nvox * batch);
  const int nb = grid_for(nvox * batch);
  if ((int64_t)nb * 52 > B.dpartial_count) {
    g_where = "head partial buffer too small";
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((k_head<1>), dim3(nb), dim3(NT), 0, st, B.d1, B.wf[OUT], B.params + bias_offset(OUT), B.yhat,
                     B.target, B.g16a, nvox, batch, inv_count, B.dpartial);
  NETCHK(launched("k_head"));
  double* hs = B.sums + B.max_batch + 1;   // 52 head sums
  hipLaunchKernelGGL(k_reduce_d, dim3(1), dim3(NT), 0, st, B.dpartial, nb, 52, hs);
  NETCHK(launched("k_reduce_d"));
  hipLaunchKernelGGL(k_head_grads, dim3(1), dim3(64), 0, st, hs, B.grads + weight_offset(OUT),
                     B.grads + bias_offset(OUT), B.sums + B.max_batch, inv_count);
  NETCHK(launched("k_head_grads"));
  // decoder level 1
  NETCHK((wgrad<16, 16, 16>(B, D1B, B.a5, nullptr, B.g16a, n, batch, st)));
  NETCHK((conv<16, 16, 16, false>(B.g16a, nullptr, B.wb[D1B], nullptr, B.a5, B.g16b, n, batch, st)));
  NETCHK((wgrad<48, 16, 16>(B, D1A, B.s1, B.d2, B.g16b, n, batch, st)));
  NETCHK((conv<16, 48, 16, false>(B.g16b, nullptr, B.wb[D1A], nullptr, nullptr, B.gc1, n, batch, st)));
  hipLaunchKernelGGL((k_upgrad<48, 16, 32>), dim3(grid_for(level_voxels(n, 1) * batch * 4)), dim3(NT), 0, st, B.gc1,
                     B.d2, B.g32a, n, batch);
  NETCHK(launched("k_upgrad"));
  // decoder level 2
  NETCHK((wgrad<32, 32, 32>(B, D2B, B.a4, nullptr, B.g32a, n2, batch, st)));
  NETCHK((conv<32, 32, 32, false>(B.g32a, nullptr, B.wb[D2B], nullptr, B.a4, B.g32b, n2, batch, st)));
  NETCHK((wgrad<96, 32, 32>(B, D2A, B.s2, B.b3, B.g32b, n2, batch, st)));
  NETCHK((conv<32, 96, 32, false>(B.g32b, nullptr, B.wb[D2A], nullptr, nullptr, B.gc2, n2, batch, st)));
  hipLaunchKernelGGL((k_upgrad<96, 32, 64>), dim3(grid_for(level_voxels(n, 2) * batch * 8)), dim3(NT), 0, st, B.gc2,
                     B.b3, B.g64a, n2, batch);
  NETCHK(launched("k_upgrad"));
  // bottleneck
  NETCHK((wgrad<64, 64, 64>(B, B3B, B.a3, nullptr, B.g64a, n4, batch, st)));
  NETCHK((conv<64, 64, 64, false>(B.g64a, nullptr, B.wb[B3B], nullptr, B.a3, B.g64b, n4, batch, st)));
  NETCHK((wgrad<32, 64, 32>(B, B3A, B.p2, nullptr, B.g64b, n4, batch, st)));
  NETCHK((conv<64, 32, 64, false>(B.g64b, nullptr, B.wb[B3A], nullptr, nullptr, B.gp2, n4, batch, st)));
  hipLaunchKernelGGL((k_poolgrad<96, 32>), dim3(grid_for(level_voxels(n, 1) * batch * 4)), dim3(NT), 0, st, B.gc2,
                     B.gp2, B.s2, B.g32a, n2, batch);
  NETCHK(launched("k_poolgrad"));
  // encoder level 2
  NETCHK((wgrad<32, 32, 32>(B, E2B, B.a2, nullptr, B.g32a, n2, batch, st)));
  NETCHK((conv<32, 32, 32, false>(B.g32a, nullptr, B.wb[E2B], nullptr, B.a2, B.g32b, n2, batch, st)));
  NETCHK((wgrad<16, 32, 16>(B, E2A, B.p1, nullptr, B.g32b, n2, batch, st)));
  NETCHK((conv<32, 16, 32, false>(B.g32b, nullptr, B.wb[E2A], nullptr, nullptr, B.gp1, n2, batch, st)));
  hipLaunchKernelGGL((k_poolgrad<48, 16>), dim3(grid_for(level_voxels(n, 0) * batch * 2)), dim3(NT), 0, st, B.gc1,
                     B.gp1, B.s1, B.g16a, n, batch);
  NETCHK(launched("k_poolgrad"));
  // encoder level 1
  NETCHK((wgrad<16, 16, 16>(B, E1B, B.a1, nullptr, B.g16a, n, batch, st)));
  NETCHK((conv<16, 16, 16, false>(B.g16a, nullptr, B.wb[E1B], nullptr, B.a1, B.g16b, n, batch, st)));
  NETCHK((wgrad<16, 16, 16>(B, E1A, B.x, nullptr, B.g16b, n, batch, st)));
  return hipSuccess;
}

hipError_t adam(const Buffers& b, float lr, float beta1, float beta2, float eps, int step, hipStream_t st) {
  const int64_t P = param_count();
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(P)), dim3(NT), 0, st, b.params, b.grads, b.adam_m, b.adam_v, P, lr, beta1,
                     beta2, eps, c1, c2);
  NETCHK(launched("k_adam"));
  return pack_weights(b, st);
}

// The slot's block means wait in its part of a gradient scratch buffer (32
// bytes per voxel, used only inside a backward pass).
float* feature_means(const Buffers& b, int slot) {
  return reinterpret_cast<float*>(b.g16a + (int64_t)slot * level_voxels(b.n, 0) * 16);
}

hipError_t features_from_means(const Buffers& b, int slot, double a0, hipStream_t st) {
  const int64_t nvox = level_voxels(b.n, 0);
  const int nb = grid_for(nvox);
  if (nb > b.dpartial_count) return hipErrorInvalidValue;
  const float* g3 = feature_means(b, slot);
  hipLaunchKernelGGL(k_sumsq3, dim3(nb), dim3(NT), 0, st, g3, nvox, b.dpartial);
  NETCHK(launched("k_sumsq3"));
  hipLaunchKernelGGL(k_reduce_d, dim3(1), dim3(NT), 0, st, b.dpartial, nb, 1, b.sums + slot);
  NETCHK(launched("k_reduce_d"));
  hipLaunchKernelGGL(k_feat_write, dim3(nb), dim3(NT), 0, st, g3, nvox, (float)(1.0 / a0), b.sums + slot,
                     b.rms + slot, b.x + (int64_t)slot * nvox * 16);
  return launched("k_feat_write");
}

hipError_t features(const Buffers& b, int slot, const float* phiN, double inv_2s, double a0, int fb, hipStream_t st) {
  const int n = b.n;
  const int64_t nvox = level_voxels(n, 0);
  const int nb = grid_for(nvox);
  if (nb > b.dpartial_count || (fb != 2 && fb != 4)) return hipErrorInvalidValue;
  float* g3 = feature_means(b, slot);
  if (fb == 2)
    hipLaunchKernelGGL(k_feat_g<2>, dim3(nb), dim3(NT), 0, st, phiN, n, (float)inv_2s, g3, b.dpartial);
  else
    hipLaunchKernelGGL(k_feat_g<4>, dim3(nb), dim3(NT), 0, st, phiN, n, (float)inv_2s, g3, b.dpartial);
  NETCHK(launched("k_feat_g"));
  hipLaunchKernelGGL(k_reduce_d, dim3(1), dim3(NT), 0, st, b.dpartial, nb, 1, b.sums + slot);
  NETCHK(launched("k_reduce_d"));
  hipLaunchKernelGGL(k_feat_write, dim3(nb), dim3(NT), 0, st, g3, nvox, (float)(1.0 / a0), b.sums + slot,
                     b.rms + slot, b.x + (int64_t)slot * nvox * 16);
  return launched("k_feat_write");
}

hipError_t target_from_field(const Buffers& b, int slot, const float* phiN, const float* F, double inv_2s, int fb,
                             hipStream_t st) {
  const int64_t nvox = level_voxels(b.n, 0);
  if (fb == 2)
    hipLaunchKernelGGL(k_target<2>, dim3(grid_for(nvox)), dim3(NT), 0, st, phiN, F, b.n, (float)inv_2s, b.rms + slot,
                       b.target + (int64_t)slot * 3 * nvox);
  else if (fb == 4)
    hipLaunchKernelGGL(k_target<4>, dim3(grid_for(nvox)), dim3(NT), 0, st, phiN, F, b.n, (float)inv_2s, b.rms + slot,
                       b.target + (int64_t)slot * 3 * nvox);
  else
    return hipErrorInvalidValue;
  return launched("k_target");
}

hipError_t start_field(const Buffers& b, float* H0, int fb, hipStream_t st) {
  const int64_t cells = level_voxels(b.n, 0) * fb * fb * fb;
  if (fb == 2)
    hipLaunchKernelGGL(k_start<2>, dim3(grid_for(cells)), dim3(NT), 0, st, b.yhat, b.rms, b.n, H0);
  else if (fb == 4)
    hipLaunchKernelGGL(k_start<4>, dim3(grid_for(cells)), dim3(NT), 0, st, b.yhat, b.rms, b.n, H0);
  else
    return hipErrorInvalidValue;
  return launched("k_start");
}

hipError_t set_input(const Buffers& b, int slot, const float* x4, hipStream_t st) {
  const int64_t nvox = level_voxels(b.n, 0);
  hipLaunchKernelGGL(k_set_input, dim3(grid_for(nvox)), dim3(NT), 0, st, x4, nvox, b.x + (int64_t)slot * nvox * 16);
  return launched("k_set_input");
}

hipError_t get_input(const Buffers& b, int slot, float* x4, hipStream_t st) {
  const int64_t nvox = level_voxels(b.n, 0);
  hipLaunchKernelGGL(k_get_input, dim3(grid_for(nvox)), dim3(NT), 0, st, b.x + (int64_t)slot * nvox * 16, nvox, x4);
  return launched("k_get_input");
}

hipError_t get_tensor(const Buffers& b, int which, int slot, float* out, hipStream_t st) {
  // stored tensor, its level and channels (pitch = channels, except the input)
  struct T { const bf16* p; int level; int C; int CP; };
  const T tab[] = {
      {b.x, 0, 4, 16},    {b.a1, 0, 16, 16},  {b.s1, 0, 16, 16},  {b.p1, 1, 16, 16},  {b.a2, 1, 32, 32},
      {b.s2, 1, 32, 32},  {b.p2, 2, 32, 32},  {b.a3, 2, 64, 64},  {b.b3, 2, 64, 64},  {b.a4, 1, 32, 32},
      {b.d2, 1, 32, 32},  {b.a5, 0, 16, 16},  {b.d1, 0, 16, 16},
      {b.g16a, 0, 16, 16}, {b.g16b, 0, 16, 16}, {b.gc1, 0, 48, 48}, {b.g32a, 1, 32, 32}, {b.g32b, 1, 32, 32},
      {b.gc2, 1, 96, 96}, {b.g64a, 2, 64, 64}, {b.g64b, 2, 64, 64}, {b.gp1, 1, 16, 16}, {b.gp2, 2, 32, 32}};
  if (which < 0 || which >= (int)(sizeof tab / sizeof tab[0])) return hipErrorInvalidValue;
  const T& t = tab[which];
  const int64_t nvox = level_voxels(b.n, t.level);
  hipLaunchKernelGGL(k_get_tensor, dim3(grid_for(nvox * t.C)), dim3(NT), 0, st, t.p + (int64_t)slot * nvox * t.CP,
                     nvox, t.CP, t.C, out);
  return launched("k_get_tensor");
}

}  // namespace net
}  // namespace pm
