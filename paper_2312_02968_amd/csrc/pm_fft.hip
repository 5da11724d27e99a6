// 3D real FFT passes of the AQUAL solve, with the pointwise and spectral steps
// of the fixed-point iteration fused into them.
//
// Data layout.  A real grid is float [N][N][N] ([z][y][x], x fastest).  A
// spectrum holds kx = 0..N/2 (the half spectrum of a real transform along x)
// in groups of 16: float2 [P / 16][N][N][16] ([kx / 16][z or kz][y or ky]
// [kx % 16]), P = 16 * ceil((N/2 + 1) / 16).  A y-pass block (one group, one
// kz) then reads one contiguous N * 128-byte run, an x-pass block (16
// consecutive rows) 2 KB runs, and a z-pass block (half a group, one ky)
// 64-byte pieces N * 128 bytes apart.  Three-component fields are three such
// spectra, comp_stride apart.
//
// A 3D transform is three passes, one per axis.  The x pass works on whole
// rows and does the real<->complex step as a half-length complex FFT plus the
// usual even/odd split; the y and z passes work on tiles of T kx-columns.
// Between the forward and the inverse z transform the whole 3D spectrum of a
// pencil is in LDS, which is where the spectral operators of the paper's flow
// scheme (inverse Laplacian, curl-free and divergence-free projections) are
// applied.  Between the inverse and the next forward x transform a whole real
// row is in LDS, which is where the algebraic equations (nu, mu) are applied.
// Every pass reads its block's data completely before writing, and blocks
// own disjoint data, so all passes run in place.
#include <hip/hip_fp16.h>

#include "pm_device.h"
#include "pm_internal.h"

// Tile widths (kx columns per block) of the y and z passes and the z pass's
// block size; compile-time launch shapes, chosen by measurement.
#ifndef PM_TY
#define PM_TY 16
#endif
#ifndef PM_TZ
#define PM_TZ 8
#endif
#ifndef PM_NTZ
#define PM_NTZ 512
#endif
#ifndef PM_HZ
#define PM_HZ 1
#endif

namespace pm {

int z_blocks(int N);
int z_blocks_io(int N, int io);

// Offset of element k of spectrum row `row` (row = kz * N + ky) in the
// grouped layout; NN = N * N.
__device__ __forceinline__ long long sidx(long long row, int k, long long NN) {
  return ((long long)(k >> 4) * NN + row) * 16 + (k & 15);
}

// ----------------------------------------------------------------------------
// Half-precision spectra of the increment solve.  The increments of the fields
// from one step to the next are small, so they may be stored with few digits
// (Sect. 5, items (iv) and (v)).  A stored complex value is (value / scale)
// rounded to FP16 per part, where the scale is a power of two per field
// component and writer tile, chosen so that the tile's largest part maps
// below 2^15: every value within 2^29 of the tile's largest keeps FP16's 11
// significant bits.  Tiles and their scale tables (Scales):
//   x pass, one row (z, y):                xs[c][z N + y]
//   y pass, 16 kx of one plane:            ys[c][kx / 16][plane]
//   z pass, 8 kx of one ky row (all kz):   zs[c][kx / 16][ky][(kx % 16) / 8]
// Every reader looks up the scale of each element it loads in the table of
// the pass that wrote it: the x pass reads what the inverse y pass wrote,
// the forward y pass what the x pass wrote, the z pass what the forward y
// pass wrote and the inverse y pass what the z pass wrote.
// ----------------------------------------------------------------------------
__device__ __forceinline__ float tile_scale(float m) {
  if (!(m > 0.0f) || !isfinite(m)) return 1.0f;     // zeros, or a NaN / Inf that passes through
  int e;
  frexpf(m, &e);                                     // m < 2^e
  return ldexpf(1.0f, e - 15);
}
__device__ __forceinline__ float2 from_half(__half2 h, float scale) {
  const float2 f = __half22float2(h);
  return make_float2(f.x * scale, f.y * scale);
}
__device__ __forceinline__ __half2 to_half(float2 v, float inv) { return __floats2half2_rn(v.x * inv, v.y * inv); }
__device__ __forceinline__ float amax2(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }

__device__ __forceinline__ bool gated_off(const Gate& g) { return g.ctl && !((g.mask >> *g.ctl) & 1); }

// Block-wide maximum of m[0..NC) (every thread gets the result).
template <int NT, int NC>
__device__ __forceinline__ void block_max(float* m) {
  __shared__ float red[NC][NT / 64];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float x = m[c];
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = x;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float x = red[c][0];
    for (int w = 1; w < NT / 64; ++w) x = fmaxf(x, red[c][w]);
    m[c] = x;
  }
}

// ----------------------------------------------------------------------------
// x pass
// ----------------------------------------------------------------------------
// XMODE.  X_LIN_*: the increment solve's linearised equations (pm_device.h,
// linearised) about the base field `base` in place of nu / mu.
// X_FWD_COARSE: as X_FWD_REAL with the rows expanded from a Coarse field.
enum { X_FWD_REAL = 0, X_INV_REAL = 1, X_FUSED_NU = 2, X_FUSED_MU = 3, X_FUSED_NU_KEEP = 4, X_LIN_NU = 5,
       X_LIN_NU_KEEP = 6, X_LIN_MU = 7, X_FWD_COARSE = 8 };
template <int XMODE>
struct XKind {
  static constexpr bool fused = XMODE == X_FUSED_NU || XMODE == X_FUSED_NU_KEEP || XMODE == X_FUSED_MU;
  static constexpr bool lin = XMODE == X_LIN_NU || XMODE == X_LIN_NU_KEEP || XMODE == X_LIN_MU;
  static constexpr bool keep = XMODE == X_FUSED_NU_KEEP || XMODE == X_LIN_NU_KEEP;
  static constexpr bool mu = XMODE == X_FUSED_MU || XMODE == X_LIN_MU;
  static constexpr bool from_real = XMODE == X_FWD_REAL || XMODE == X_FWD_COARSE;
};

// Element m of row `row` (two grid points, x = 2m and 2m + 1) of component c
// of a Coarse field on the N^3 box: both points lie in one voxel (f >= 2).
__device__ __forceinline__ float2 coarse_pair(const Coarse& co, int c, long long row, int m, int N) {
  const long long z = row / N, y = row % N;
  const long long n = co.n;
  const long long v = ((z / co.f) * n + y / co.f) * n + (2 * m) / co.f;
  const float val = (float)*co.rms * co.y[c * n * n * n + v];
  return make_float2(val, val);
}

// r2c split: LDS holds Z = FFT_H(x[2m] + i x[2m+1]) for each sequence; turn
// it into X[k], k = 0..H (X[H] goes to element H, one past the complex data).
template <int H, int S, int NT>
__device__ __forceinline__ void r2c_split(float2* buf, int IS, const float2* __restrict__ tw) {
  constexpr int NP = S * (H / 2 + 1);
  for (int b = threadIdx.x; b < NP; b += NT) {
    const int q = b % S, k = b / S;
    const int km = (H - k) & (H - 1);
    const float2 zk = buf[k * IS + q], zm = buf[km * IS + q];
    // X[k] = E + W^k O,  E = (Zk + conj Zm)/2,  O = -i (Zk - conj Zm)/2
    float2 e = cscale(cadd(zk, cconj(zm)), 0.5f);
    float2 o = cscale(mul_mi<false>(csub(zk, cconj(zm))), 0.5f);
    const float2 xk = cadd(e, cmul(tw[k], o));
    if (k == 0) {
      buf[q] = make_float2(zk.x + zk.y, 0.0f);
      buf[H * IS + q] = make_float2(zk.x - zk.y, 0.0f);
    } else if (2 * k == H) {
      buf[k * IS + q] = xk;
    } else {
      float2 e2 = cscale(cadd(zm, cconj(zk)), 0.5f);
      float2 o2 = cscale(mul_mi<false>(csub(zm, cconj(zk))), 0.5f);
      const float2 xm = cadd(e2, cmul(tw[H - k], o2));
      buf[k * IS + q] = xk;
      buf[km * IS + q] = xm;
    }
  }
  __syncthreads();
}

// c2r merge: LDS holds X[k], k = 0..H; produce Z[k], k < H, such that the
// unnormalised inverse FFT_H of Z gives x[2m] + i x[2m+1] with
// x[n] = sum over the full spectrum of X_k exp(+2 pi i k n / N).
template <int H, int S, int NT>
__device__ __forceinline__ void c2r_merge(float2* buf, int IS, const float2* __restrict__ tw) {
  constexpr int NP = S * (H / 2 + 1);
  for (int b = threadIdx.x; b < NP; b += NT) {
    const int q = b % S, k = b / S;
    const float2 xk = buf[k * IS + q], xm = buf[(H - k) * IS + q];
    // Z[k] = (Xk + conj Xm) + i (Xk - conj Xm) conj(W^k)
    const float2 zk = cadd(cadd(xk, cconj(xm)), mul_mi<true>(cmul(csub(xk, cconj(xm)), cconj(tw[k]))));
    if (k == 0 || 2 * k == H) {
      buf[k * IS + q] = zk;
    } else {
      const float2 zm = cadd(cadd(xm, cconj(xk)),
                             mul_mi<true>(cmul(csub(xm, cconj(xk)), cconj(tw[H - k]))));
      buf[k * IS + q] = zk;
      buf[(H - k) * IS + q] = zm;
    }
  }
  __syncthreads();
}

// The external-field sheets at grid points (2m, 2m + 1) of row `row`
// (row = z * N + y) of an N^3 density.
__device__ __forceinline__ void add_dipole(float2& x, const Dipole& dip, long long row, int m, int N) {
  if (dip.x == 0.f && dip.y == 0.f && dip.z == 0.f) return;
  const int y = (int)(row % N), z = (int)(row / N);
  const float a = (y == N - 1 ? dip.y : 0.f) - (y == 0 ? dip.y : 0.f) + (z == N - 1 ? dip.z : 0.f) -
                  (z == 0 ? dip.z : 0.f);
  x.x += a - (m == 0 ? dip.x : 0.f);
  x.y += a + (2 * m + 1 == N - 1 ? dip.x : 0.f);
}

// One block: ROWS rows of NC components.  Sequence q = c * ROWS + r.
//   X_FWD_REAL : real rows (float, row pitch 2H) -> spectrum rows
//   X_INV_REAL : spectrum rows -> real rows
//   X_FUSED_*  : spectrum rows -> c2r -> nu or mu on the 3-vector -> r2c ->
//                spectrum rows (in place).  X_FUSED_NU_KEEP is X_FUSED_NU that
//                also accumulates the squared change of F against fprev in
//                FP64 into partials[blockIdx.x] and stores F to fprev.
//   X_LIN_*    : as X_FUSED_* with the linearised maps about `base`.
// IO = 1: the spectrum rows are FP16 (read with the y pass's scales, written
// with one scale per row and component).
template <int H, int ROWS, int NC, int NT, int XMODE, int IO = 0>
__global__ __launch_bounds__(NT) void k_xpass(float2* spec, long long comp_stride,
                                              float* real, long long real_comp_stride,
                                              const float2* __restrict__ tw, int mu_mode, float inv_a0,
                                              float* fprev, double* partials, Dipole dip,
                                              const float* __restrict__ base, Scales sc, Gate gate, Coarse co) {
  if (gated_off(gate)) return;
  using XK = XKind<XMODE>;
  constexpr int S = NC * ROWS;
  constexpr int IS = S + 1;
  extern __shared__ float2 lds[];
  const int row0 = blockIdx.x * ROWS;
  const int N = 2 * H;
  const long long NN = (long long)N * N;
  float2* tw_s = lds + (H + 1) * IS;
  for (int t = threadIdx.x; t < N; t += NT) tw_s[t] = tw[t];
  const __half2* spec_h = reinterpret_cast<const __half2*>(spec);

  // ---- load
  if (XMODE == X_FWD_COARSE) {
    for (int b = threadIdx.x; b < S * H; b += NT) {
      const int q = b / H, m = b % H;
      const int c = q / ROWS, r = q % ROWS;
      lds[m * IS + q] = coarse_pair(co, c, row0 + r, m, N);
    }
  } else if (XMODE == X_FWD_REAL) {
    for (int b = threadIdx.x; b < S * H; b += NT) {
      const int q = b / H, m = b % H;
      const int c = q / ROWS, r = q % ROWS;
      const float2* src = reinterpret_cast<const float2*>(real + c * real_comp_stride + (long long)(row0 + r) * N);
      float2 x = src[m];
      if (NC == 1) add_dipole(x, dip, row0 + r, m, N);
      lds[m * IS + q] = x;
    }
  } else {
    for (int b = threadIdx.x; b < S * H; b += NT) {
      const int q = b / H, k = b % H;
      const int c = q / ROWS, r = q % ROWS;
      if constexpr (IO == 1)
        lds[k * IS + q] = from_half(spec_h[c * comp_stride + sidx(row0 + r, k, NN)],
                                    sc.ys[c * sc.ycs + (long long)(k >> 4) * N + (row0 + r) / N]);
      else
        lds[k * IS + q] = spec[c * comp_stride + sidx(row0 + r, k, NN)];
    }
    for (int q = threadIdx.x; q < S; q += NT) {
      const int c = q / ROWS, r = q % ROWS;
      if constexpr (IO == 1)
        lds[H * IS + q] = from_half(spec_h[c * comp_stride + sidx(row0 + r, H, NN)],
                                    sc.ys[c * sc.ycs + (long long)(H >> 4) * N + (row0 + r) / N]);
      else
        lds[H * IS + q] = spec[c * comp_stride + sidx(row0 + r, H, NN)];
    }
  }
  __syncthreads();

  if (!XK::from_real) {
    c2r_merge<H, S, NT>(lds, IS, tw_s);
    block_fft<H, S, NT, true, true>(lds, 1, IS, tw_s, 2);
  }

  if constexpr (XK::fused || XK::lin) {
    double acc = 0.0;
    const float a0 = inv_a0 > 0.0f ? 1.0f / inv_a0 : 0.0f;
    for (int b = threadIdx.x; b < ROWS * H; b += NT) {
      const int r = b % ROWS, m = b / ROWS;
      float2 v0 = lds[m * IS + r], v1 = lds[m * IS + ROWS + r], v2 = lds[m * IS + 2 * ROWS + r];
      const long long e = (long long)(row0 + r) * N + 2 * m;
      const long long cs = (long long)N * N * N;
      if (XK::keep) {
        float2* f0 = reinterpret_cast<float2*>(fprev + e);
        float2* f1 = reinterpret_cast<float2*>(fprev + cs + e);
        float2* f2 = reinterpret_cast<float2*>(fprev + 2 * cs + e);
        const float2 p0 = *f0, p1 = *f1, p2 = *f2;
        const double d0 = (double)v0.x - p0.x, d1 = (double)v1.x - p1.x, d2 = (double)v2.x - p2.x;
        const double e0 = (double)v0.y - p0.y, e1 = (double)v1.y - p1.y, e2 = (double)v2.y - p2.y;
        acc += d0 * d0 + d1 * d1 + d2 * d2 + e0 * e0 + e1 * e1 + e2 * e2;
        *f0 = v0; *f1 = v1; *f2 = v2;
      }
      // two grid points per complex entry: .x is x = 2m, .y is x = 2m+1
      if constexpr (XK::lin) {
        const float2 b0 = *reinterpret_cast<const float2*>(base + e);
        const float2 b1 = *reinterpret_cast<const float2*>(base + cs + e);
        const float2 b2 = *reinterpret_cast<const float2*>(base + 2 * cs + e);
        linearised<XK::mu>(mu_mode, a0, inv_a0, b0.x, b1.x, b2.x, v0.x, v1.x, v2.x);
        linearised<XK::mu>(mu_mode, a0, inv_a0, b0.y, b1.y, b2.y, v0.y, v1.y, v2.y);
      } else {
        {
          const float m2 = v0.x * v0.x + v1.x * v1.x + v2.x * v2.x;
          const float f = !XK::mu ? nu_of_sq(mu_mode, m2, a0) : mu_of_sq(mu_mode, m2, inv_a0);
          v0.x *= f; v1.x *= f; v2.x *= f;
        }
        {
          const float m2 = v0.y * v0.y + v1.y * v1.y + v2.y * v2.y;
          const float f = !XK::mu ? nu_of_sq(mu_mode, m2, a0) : mu_of_sq(mu_mode, m2, inv_a0);
          v0.y *= f; v1.y *= f; v2.y *= f;
        }
      }
      lds[m * IS + r] = v0;
      lds[m * IS + ROWS + r] = v1;
      lds[m * IS + 2 * ROWS + r] = v2;
    }
    if (XK::keep) {
      // block reduction of acc (FP64)
      __shared__ double red[NT / 64];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        partials[blockIdx.x] = t;
      }
    }
    __syncthreads();
  }

  if (XMODE != X_INV_REAL) {
    block_fft<H, S, NT, true, false>(lds, 1, IS, tw_s, 2);
    r2c_split<H, S, NT>(lds, IS, tw_s);
    if constexpr (IO == 1) {
      // one scale per row and component: the largest part over k = 0..H
      __shared__ float inv_s[S];
      static_assert(S <= NT, "one thread per row and component");
      if (threadIdx.x < S) {
        const int q = threadIdx.x;
        float mx = 0.0f;
        for (int k = 0; k <= H; ++k) mx = fmaxf(mx, amax2(lds[k * IS + q]));
        const float sc_q = tile_scale(mx);
        inv_s[q] = 1.0f / sc_q;
        sc.xs[(q / ROWS) * sc.xcs + row0 + q % ROWS] = sc_q;
      }
      __syncthreads();
      __half2* dst_h = reinterpret_cast<__half2*>(spec);
      for (int b = threadIdx.x; b < S * H; b += NT) {
        const int q = b / H, k = b % H;
        const int c = q / ROWS, r = q % ROWS;
        dst_h[c * comp_stride + sidx(row0 + r, k, NN)] = to_half(lds[k * IS + q], inv_s[q]);
      }
      for (int q = threadIdx.x; q < S; q += NT) {
        const int c = q / ROWS, r = q % ROWS;
        dst_h[c * comp_stride + sidx(row0 + r, H, NN)] = to_half(lds[H * IS + q], inv_s[q]);
      }
    } else {
      for (int b = threadIdx.x; b < S * H; b += NT) {
        const int q = b / H, k = b % H;
        const int c = q / ROWS, r = q % ROWS;
        spec[c * comp_stride + sidx(row0 + r, k, NN)] = lds[k * IS + q];
      }
      for (int q = threadIdx.x; q < S; q += NT) {
        const int c = q / ROWS, r = q % ROWS;
        spec[c * comp_stride + sidx(row0 + r, H, NN)] = lds[H * IS + q];
      }
    }
  } else {
    for (int b = threadIdx.x; b < S * H; b += NT) {
      const int q = b / H, m = b % H;
      const int c = q / ROWS, r = q % ROWS;
      float2* dst = reinterpret_cast<float2*>(real + c * real_comp_stride + (long long)(row0 + r) * N);
      dst[m] = lds[m * IS + q];
    }
  }
}

// ----------------------------------------------------------------------------
// x pass for n_pad = 512 and 1024 (rows of H = 256 or 512 complex): a group of
// LANES lanes per row (16 for H = 256, four rows per wave; 64 for H = 512, one
// row per wave), four waves per block.  Lane j of a group holds the elements
// k = j + LANES r (r < RG = H / LANES) of its row for every component, so
//  - the FFT runs in registers with wave-private LDS exchanges: 16 x 16 for
//    H = 256, 8 x 8 x 8 for H = 512, and the output is again at
//    k = j + LANES r;
//  - the partner H - k of element k (even/odd split of the real transform)
//    sits in lane LANES - j, register RG - 1 - r (lane 0 pairs within
//    itself), so the split and merge are cross-lane shuffles;
//  - nu / mu act on the registers.
// No block-wide barrier is needed after the twiddle table is loaded.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int xpad(int p) { return p + (p >> 4); }

// 256-point FFT of the group's row held as v[r] = x[j + 16 r]; result in the
// same layout.  xb: the group's 272-entry LDS row.
template <bool INV>
__device__ __forceinline__ void fft256_group(float2* v, float2* xb, int j, const float2* tw_s) {
  Dft<16, INV>::run(v);                                  // outputs y[16 j + r]
#pragma unroll
  for (int r = 0; r < 16; ++r) xb[xpad(16 * j + r)] = v[r];
  wave_sync();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = xb[xpad(j + 16 * r)];
  wave_sync();
#pragma unroll
  for (int r = 1; r < 16; ++r) {
    float2 w = tw_s[2 * r * j];                          // w_256^(r j) from the 512-entry table
    if (INV) w.y = -w.y;
    v[r] = cmul(v[r], w);
  }
  Dft<16, INV>::run(v);                                  // outputs y[j + 16 r]
}

// 512-point FFT of the wave's row held as v[r] = x[j + 64 r], j = lane; result
// in the same layout.  x = j + 64 r and k = s + 8 a + 64 b: a radix-8 DFT over
// r (giving s), twiddles w_512^(j s), then for each s a 64-point DFT over
// j = j1 + 8 j2 as a radix-8 DFT over j2 (giving a), twiddles w_64^(j1 a) and a
// radix-8 DFT over j1 (giving b).  After the first exchange lane s + 8 j1
// holds the 8 values j2; after the second, lane s + 8 a = k mod 64 holds the 8
// values j1, so the last DFT leaves X[lane + 64 b] in v[b].  xb: the wave's
// 544-entry LDS row; tw_s: the 1024-entry table w_1024^t.
template <bool INV>
__device__ __forceinline__ void fft512_wave(float2* v, float2* xb, int j, const float2* tw_s) {
  Dft<8, INV>::run(v);
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    float2 w = tw_s[2 * j * r];                          // w_512^(j s)
    if (INV) w.y = -w.y;
    v[r] = cmul(v[r], w);
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) xb[xpad(64 * r + j)] = v[r];
  wave_sync();
  const int s = j & 7, j1 = j >> 3;
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = xb[xpad(64 * s + j1 + 8 * r)];
  wave_sync();
  Dft<8, INV>::run(v);
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    float2 w = tw_s[16 * j1 * r];                        // w_64^(j1 a)
    if (INV) w.y = -w.y;
    v[r] = cmul(v[r], w);
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) xb[xpad(64 * s + 8 * r + j1)] = v[r];
  wave_sync();
  const int a = j >> 3;
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = xb[xpad(64 * s + 8 * a + r)];
  wave_sync();
  Dft<8, INV>::run(v);
}

// 256-point FFT of a row held by 32 lanes, v[r] = x[j + 32 r] (j = lane in
// the row, r < 8); result in the same layout.  With x = j + 32 r and
// k = s + 8 q1 + 64 q2: a radix-8 DFT over r (giving s), twiddles
// w_256^(j s); then, for each s, the 32-point DFT over j = j1 + 4 j2 as a
// radix-8 DFT over j2 (giving q1), twiddles w_32^(j1 q1) and a radix-4 DFT
// over j1 (giving q2).  After the first exchange lane s + 8 j1 holds the 8
// values j2; after the second, lane s + 8 m holds the 4 values j1 of q1 = m
// and of q1 = m + 4, so the two radix-4 DFTs leave X[lane + 32 (h + 2 q2)]
// in v[4 h + q2], which a register permutation puts back at r = h + 2 q2.
// xb: the row's 272-entry LDS row; twl: the block's twiddles of the two
// stages in lane order, w_256^(j s) at twl[32 s + j] and w_32^(j1 q1) at
// twl[256 + 4 q1 + j1] (consecutive lanes read consecutive entries, where
// the strided w_512^t table costs bank conflicts).
template <bool INV>
__device__ __forceinline__ void fft256_lane32(float2* v, float2* xb, int j, const float2* twl) {
  Dft<8, INV>::run(v);
#pragma unroll
  for (int s = 1; s < 8; ++s) {
    float2 w = twl[32 * s + j];                          // w_256^(j s)
    if (INV) w.y = -w.y;
    v[s] = cmul(v[s], w);
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) xb[xpad(32 * s + j)] = v[s];
  wave_sync();
  const int s = j & 7, hi = j >> 3;                      // hi: j1 now, m after the second exchange
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = xb[xpad(32 * s + hi + 4 * r)];
  wave_sync();
  Dft<8, INV>::run(v);
#pragma unroll
  for (int q = 1; q < 8; ++q) {
    float2 w = twl[256 + 4 * q + hi];                    // w_32^(j1 q1)
    if (INV) w.y = -w.y;
    v[q] = cmul(v[q], w);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) xb[xpad(32 * s + 4 * q + hi)] = v[q];
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < 4; ++a) v[4 * h + a] = xb[xpad(32 * s + 4 * (hi + 4 * h) + a)];
  wave_sync();
  Dft<4, INV>::run(v);
  Dft<4, INV>::run(v + 4);
  float2 t[8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) t[h + 2 * q] = v[4 * h + q];
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = t[r];
}

#ifndef PM_X256_LANES
#define PM_X256_LANES 32
#endif

template <int H>
struct XWave {
  static constexpr int N = 2 * H;
  static constexpr int LANES = (H == 256) ? PM_X256_LANES : 64;
  static constexpr int RG = H / LANES;              // elements per lane and component
  static constexpr int G = 64 / LANES;              // rows per wave
  static constexpr int ROWS = 4 * G;                // rows per block (4 waves)
  static constexpr int XB = H + H / 16;             // padded LDS row (xpad)
  static constexpr bool L32 = (H == 256 && LANES == 32);
  static constexpr int TWL = L32 ? 256 + 32 : 0;    // lane-ordered twiddles of fft256_lane32
  template <bool INV>
  __device__ __forceinline__ static void fft(float2* v, float2* xb, int j, const float2* tw_s,
                                             const float2* twl) {
    if constexpr (H == 256 && LANES == 16) fft256_group<INV>(v, xb, j, tw_s);
    else if constexpr (H == 256) fft256_lane32<INV>(v, xb, j, twl);
    else fft512_wave<INV>(v, xb, j, tw_s);
  }
  // fills the lane-ordered twiddles from the w_N^t table (block-wide)
  __device__ __forceinline__ static void fill_twl(float2* twl, const float2* __restrict__ tw) {
    if constexpr (L32) {
      for (int t = threadIdx.x; t < TWL; t += 256) {
        if (t < 256) twl[t] = tw[2 * (t & 31) * (t >> 5)];           // w_256^(j s), j = t % 32, s = t / 32
        else twl[t] = tw[16 * ((t - 256) & 3) * ((t - 256) >> 2)];  // w_32^(j1 q1)
      }
    }
  }
};

// Occupancy floor (waves per SIMD) asked of the compiler for the fused
// passes of 256 and 512 points; 1 leaves the register allocation free.  At
// 512 points (the 1024^3 box) three waves fit with a 20-byte spill in the
// mu pass and make both passes 7 % faster; at 256 points four waves spill
// more and are slower.
#ifndef PM_X256_WAVES
#define PM_X256_WAVES 1
#endif
#ifndef PM_X512_WAVES
#define PM_X512_WAVES 3
#endif
template <int H, int XMODE>
struct XWaves {
  static constexpr bool fused = XMODE == X_FUSED_NU || XMODE == X_FUSED_MU;
  static constexpr int value = !fused ? 1 : H == 256 ? PM_X256_WAVES : H == 512 ? PM_X512_WAVES : 1;
};

template <int H, int XMODE, int NC, int IO = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(XWaves<H, XMODE>::value))) void k_xpass_wave(float2* spec, long long comp_stride, float* real,
                                                    long long real_comp_stride, const float2* __restrict__ tw,
                                                    int mu_mode, float inv_a0, float* fprev, double* partials,
                                                    Dipole dip, const float* __restrict__ base, Scales sc,
                                                    Gate gate, Coarse co) {
  if (gated_off(gate)) return;
  using X = XWave<H>;
  using XK = XKind<XMODE>;
  constexpr int N = X::N, LANES = X::LANES, RG = X::RG;
  constexpr long long NN = (long long)N * N;
  extern __shared__ float2 lds[];
  float2* tw_s = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / LANES, j = lane % LANES;
  float2* xb = lds + N + (wave * X::G + g) * X::XB;
  float2* twl = lds + N + X::ROWS * X::XB;
  const long long row = (long long)blockIdx.x * X::ROWS + wave * X::G + g;
  for (int t = threadIdx.x; t < N; t += 256) tw_s[t] = tw[t];
  X::fill_twl(twl, tw);
  __syncthreads();

  float2 v[NC][RG];
  const int pl = (lane & ~(LANES - 1)) | ((LANES - j) & (LANES - 1));   // lane of the partner elements

  if (XMODE == X_FWD_COARSE) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < RG; ++r) v[c][r] = coarse_pair(co, c, row, j + LANES * r, N);
  } else if (XMODE == X_FWD_REAL) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float2* src = reinterpret_cast<const float2*>(real + c * real_comp_stride + row * N);
#pragma unroll
      for (int r = 0; r < RG; ++r) v[c][r] = src[j + LANES * r];
    }
    if constexpr (NC == 1) {
#pragma unroll
      for (int r = 0; r < RG; ++r) add_dipole(v[0][r], dip, row, j + LANES * r, N);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      float2 x[RG];
      float2 nyq;
      if constexpr (IO == 1) {
        const __half2* src = reinterpret_cast<const __half2*>(spec) + c * comp_stride;
        const float* ysc = sc.ys + c * sc.ycs + row / N;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          const int k = j + LANES * r;
          x[r] = from_half(src[sidx(row, k, NN)], ysc[(long long)(k >> 4) * N]);
        }
        nyq = from_half(src[sidx(row, H, NN)], ysc[(long long)(H >> 4) * N]);
      } else {
        const float2* src = spec + c * comp_stride;
#pragma unroll
        for (int r = 0; r < RG; ++r) x[r] = src[sidx(row, j + LANES * r, NN)];
        nyq = src[sidx(row, H, NN)];
      }
      // merge: Z[k] = (Xk + conj Xm) + i (Xk - conj Xm) conj(W^k), Xm = X[H - k]
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        float2 xm;
        xm.x = __shfl(x[RG - 1 - r].x, pl, 64);
        xm.y = __shfl(x[RG - 1 - r].y, pl, 64);
        if (j == 0) xm = (r == 0) ? nyq : x[(RG - r) & (RG - 1)];
        const int k = j + LANES * r;
        const float2 a = cadd(x[r], cconj(xm));
        const float2 d = cmul(csub(x[r], cconj(xm)), cconj(tw_s[k]));
        v[c][r] = cadd(a, mul_mi<true>(d));
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) X::template fft<true>(v[c], xb, j, tw_s, twl);
  }

  if constexpr (XK::fused || XK::lin) {
    double acc = 0.0;
    const float a0 = inv_a0 > 0.0f ? 1.0f / inv_a0 : 0.0f;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      float2 e0 = v[0][r], e1 = v[1][r], e2 = v[2][r];
      const long long e = row * N + 2 * (j + LANES * r);
      const long long cs = (long long)N * N * N;
      if (XK::keep) {
        float2* f0 = reinterpret_cast<float2*>(fprev + e);
        float2* f1 = reinterpret_cast<float2*>(fprev + cs + e);
        float2* f2 = reinterpret_cast<float2*>(fprev + 2 * cs + e);
        const float2 p0 = *f0, p1 = *f1, p2 = *f2;
        const double d0 = (double)e0.x - p0.x, d1 = (double)e1.x - p1.x, d2 = (double)e2.x - p2.x;
        const double g0 = (double)e0.y - p0.y, g1 = (double)e1.y - p1.y, g2 = (double)e2.y - p2.y;
        acc += d0 * d0 + d1 * d1 + d2 * d2 + g0 * g0 + g1 * g1 + g2 * g2;
        *f0 = e0; *f1 = e1; *f2 = e2;
      }
      if constexpr (XK::lin) {
        const float2 b0 = *reinterpret_cast<const float2*>(base + e);
        const float2 b1 = *reinterpret_cast<const float2*>(base + cs + e);
        const float2 b2 = *reinterpret_cast<const float2*>(base + 2 * cs + e);
        linearised<XK::mu>(mu_mode, a0, inv_a0, b0.x, b1.x, b2.x, e0.x, e1.x, e2.x);
        linearised<XK::mu>(mu_mode, a0, inv_a0, b0.y, b1.y, b2.y, e0.y, e1.y, e2.y);
        v[0][r] = e0;
        v[1][r] = e1;
        v[2][r] = e2;
      } else {
        const float m0 = e0.x * e0.x + e1.x * e1.x + e2.x * e2.x;
        const float m1 = e0.y * e0.y + e1.y * e1.y + e2.y * e2.y;
        const float f0 = !XK::mu ? nu_of_sq(mu_mode, m0, a0) : mu_of_sq(mu_mode, m0, inv_a0);
        const float f1 = !XK::mu ? nu_of_sq(mu_mode, m1, a0) : mu_of_sq(mu_mode, m1, inv_a0);
        v[0][r] = make_float2(e0.x * f0, e0.y * f1);
        v[1][r] = make_float2(e1.x * f0, e1.y * f1);
        v[2][r] = make_float2(e2.x * f0, e2.y * f1);
      }
    }
    if (XK::keep) {
      __shared__ double red[4];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) red[wave] = acc;
      __syncthreads();
      if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
  }

  if (XMODE == X_INV_REAL) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      float2* dst = reinterpret_cast<float2*>(real + c * real_comp_stride + row * N);
#pragma unroll
      for (int r = 0; r < RG; ++r) dst[j + LANES * r] = v[c][r];
    }
    return;
  }

#pragma unroll
  for (int c = 0; c < NC; ++c) {
    X::template fft<false>(v[c], xb, j, tw_s, twl);
    // split: X[k] = E + W^k O, E = (Zk + conj Zm)/2, O = -i (Zk - conj Zm)/2
    if constexpr (IO == 1) {
      float2 o[RG];
      float2 nyq = make_float2(0.0f, 0.0f);
      float mx = 0.0f;
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        float2 zm;
        zm.x = __shfl(v[c][RG - 1 - r].x, pl, 64);
        zm.y = __shfl(v[c][RG - 1 - r].y, pl, 64);
        if (j == 0) zm = v[c][(RG - r) & (RG - 1)];
        const float2 zk = v[c][r];
        const int k = j + LANES * r;
        const float2 e = cscale(cadd(zk, cconj(zm)), 0.5f);
        const float2 od = cscale(mul_mi<false>(csub(zk, cconj(zm))), 0.5f);
        if (k == 0) {
          o[r] = make_float2(zk.x + zk.y, 0.0f);
          nyq = make_float2(zk.x - zk.y, 0.0f);
        } else {
          o[r] = cadd(e, cmul(tw_s[k], od));
        }
        mx = fmaxf(mx, amax2(o[r]));
      }
      mx = fmaxf(mx, amax2(nyq));
      // one scale per row: the largest part over the LANES lanes of the row
      for (int w = LANES / 2; w > 0; w >>= 1) mx = fmaxf(mx, __shfl_xor(mx, w, 64));
      const float sc_r = tile_scale(mx), inv = 1.0f / sc_r;
      __half2* dst = reinterpret_cast<__half2*>(spec) + c * comp_stride;
#pragma unroll
      for (int r = 0; r < RG; ++r) dst[sidx(row, j + LANES * r, NN)] = to_half(o[r], inv);
      if (j == 0) {
        dst[sidx(row, H, NN)] = to_half(nyq, inv);
        sc.xs[c * sc.xcs + row] = sc_r;
      }
    } else {
      float2* dst = spec + c * comp_stride;
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        float2 zm;
        zm.x = __shfl(v[c][RG - 1 - r].x, pl, 64);
        zm.y = __shfl(v[c][RG - 1 - r].y, pl, 64);
        if (j == 0) zm = v[c][(RG - r) & (RG - 1)];
        const float2 zk = v[c][r];
        const int k = j + LANES * r;
        const float2 e = cscale(cadd(zk, cconj(zm)), 0.5f);
        const float2 o = cscale(mul_mi<false>(csub(zk, cconj(zm))), 0.5f);
        if (k == 0) {
          dst[sidx(row, 0, NN)] = make_float2(zk.x + zk.y, 0.0f);
          dst[sidx(row, H, NN)] = make_float2(zk.x - zk.y, 0.0f);
        } else {
          dst[sidx(row, k, NN)] = cadd(e, cmul(tw_s[k], o));
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Column passes.  A block owns T kx-columns of one z plane (y pass) or one ky
// row (z pass).  Twiddles are staged in LDS; the first stage reads HBM into
// registers and the last stage writes registers to HBM (see col_fft).
// ----------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ void load_twiddles(float2* tw_s, const float2* __restrict__ tw, int NT) {
  for (int t = threadIdx.x; t < L; t += NT) tw_s[t] = tw[t];
}

// Loads the first-stage inputs (radix R) of column q = b mod T of each
// component c from src[c] + i * row_stride + q; zero for q >= nv[c].
template <int L, int T, int NT, int R, int NC, int CS = 1>
__device__ __forceinline__ void load_cols(float2* v, int E, const float2* const* src, const int* nv,
                                          long long row_stride) {
  using B = Bfly<L, T, NT, R>;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % T, j = b / T;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long off = (long long)(j + r * (L / R)) * row_stride + q * CS;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        v[c * E + u * R + r] = (q < nv[c]) ? src[c][off] : make_float2(0.0f, 0.0f);
    }
  }
}

template <int L, int T, int NT, int R, int NC, int CS = 1>
__device__ __forceinline__ void store_cols(const float2* v, int E, float2* const* dst, const int* nv,
                                           long long row_stride) {
  using B = Bfly<L, T, NT, R>;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % T, j = b / T;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long off = (long long)(j + r * (L / R)) * row_stride + q * CS;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (q < nv[c]) dst[c][off] = v[c * E + u * R + r];
    }
  }
}

// Half-precision column pairs.  A block's 16 kx columns are two sets, the
// even and the odd columns (column 2 q + h of the group is element q of set
// h), so that one 8-byte access carries the pair q of both sets: the 64-byte
// FP16 row of a group is read with the same 8 bytes per lane as an FP32 tile
// of 8 columns.  Pair p covers sets 2 p and 2 p + 1; element (row i, pair q)
// is at src[p][i * row_stride + 2 q] and is scaled by scl[p][i].
struct alignas(8) HalfPair {
  __half2 a, b;
};

template <int L, int T, int NT, int R, int NP>
__device__ __forceinline__ void load_pairs_h(float2* v, int E, const __half2* const* src, const int* nvalid,
                                             long long row_stride, const float* const* scl) {
  using B = Bfly<L, T, NT, R>;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % T, j = b / T;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * (L / R);
      const long long off = (long long)i * row_stride + 2 * q;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const float sc = scl[p][i];
        float2 e0 = make_float2(0.0f, 0.0f), e1 = e0;
        if (2 * q + 1 < nvalid[p]) {
          const HalfPair hp = *reinterpret_cast<const HalfPair*>(src[p] + off);
          e0 = from_half(hp.a, sc);
          e1 = from_half(hp.b, sc);
        } else if (2 * q < nvalid[p]) {
          e0 = from_half(src[p][off], sc);
        }
        v[(2 * p) * E + u * R + r] = e0;
        v[(2 * p + 1) * E + u * R + r] = e1;
      }
    }
  }
}

template <int L, int T, int NT, int R, int NP>
__device__ __forceinline__ void store_pairs_h(const float2* v, int E, __half2* const* dst, const int* nvalid,
                                              long long row_stride, const float* inv) {
  using B = Bfly<L, T, NT, R>;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % T, j = b / T;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long off = (long long)(j + r * (L / R)) * row_stride + 2 * q;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const float2 e0 = v[(2 * p) * E + u * R + r], e1 = v[(2 * p + 1) * E + u * R + r];
        if (2 * q + 1 < nvalid[p]) {
          HalfPair hp;
          hp.a = to_half(e0, inv[p]);
          hp.b = to_half(e1, inv[p]);
          *reinterpret_cast<HalfPair*>(dst[p] + off) = hp;
        } else if (2 * q < nvalid[p]) {
          dst[p][off] = to_half(e0, inv[p]);
        }
      }
    }
  }
}

// Largest part of each set's valid elements (as store_cols stores them).
template <int L, int T, int NT, int R, int NC>
__device__ __forceinline__ void cols_absmax(const float2* v, int E, const int* nv, float* m) {
  using B = Bfly<L, T, NT, R>;
#pragma unroll
  for (int c = 0; c < NC; ++c) m[c] = 0.0f;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % T;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (q < nv[c]) m[c] = fmaxf(m[c], amax2(v[c * E + u * R + r]));
  }
}

// y pass: one group of 16 kx columns of one z plane (a contiguous run of L
// rows of 16 complex values), handled as 16 / T sets of T columns that share
// the LDS exchange buffer (the buffer holds only T columns).  With T = 16 a
// load instruction covers whole 128-byte rows of consecutive ky.
template <int L, int T, int NT, bool INV, int IO = 0>
__global__ __launch_bounds__(NT) void k_ypass(float2* spec, long long comp_stride, int ncols,
                                              const float2* __restrict__ tw, Scales sc, Gate gate) {
  if (gated_off(gate)) return;
  static_assert(16 % T == 0, "a y-pass block owns one group of 16 kx columns");
  constexpr int NH = 16 / T;
  constexpr int E = ColCfg<L, T, NT>::E;
  extern __shared__ float2 lds[];
  float2* tw_s = lds + ColBuf<L, T>::elems;
  // Block order.  Each pass reads what the previous one wrote, and the last
  // ~256 MB written are still in the Infinity Cache, so a pass starts where
  // its predecessor ended.  The forward y pass follows an x pass, which
  // writes rows (planes) in ascending order: it takes planes in descending
  // order as its slowest index.  The inverse y pass follows a z pass, whose
  // XCD ranges end in the higher kx groups: it takes groups in descending
  // order as its slowest index.
  const int nt = gridDim.x, nc = gridDim.z;
  const long long b = blockIdx.x + (long long)nt * (blockIdx.y + (long long)L * blockIdx.z);
  int t, kz, comp;
  if constexpr (!INV) {
    t = (int)(b % nt);
    comp = (int)((b / nt) % nc);
    kz = L - 1 - (int)(b / ((long long)nt * nc));
  } else {
    kz = (int)(b % L);
    comp = (int)((b / L) % nc);
    t = nt - 1 - (int)(b / ((long long)L * nc));
  }
  const int x0 = t * 16;
  const long long boff = comp * comp_stride + ((long long)t * L + kz) * L * 16;
  float2* base = spec + boff;
  load_twiddles<L>(tw_s, tw, NT);
  float2 v[NH * E];
  using First = PlanAt<L, false, 0>;
  using Last = PlanAt<L, false, Plan<L>::S - 1>;
  int nv[NH];
  float2* ptr[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    nv[h] = min(T, ncols - x0 - h * T);
    ptr[h] = base + h * T;
  }
  if constexpr (IO == 1) {
    // FP16: the group's even and odd columns as the two sets (T = 8), one
    // scale per row read from the writer's table (the forward pass reads what
    // an x pass wrote, a scale per row ky of this plane; the inverse pass
    // what a z pass wrote, a scale per (group, ky)), staged in LDS
    static_assert(T == 8 && NH == 2, "half-precision y tiles are two interleaved sets of 8 columns");
    __shared__ float s_in[L];
    const float* scl_g = INV ? sc.zs + comp * sc.zcs + (long long)t * L : sc.xs + comp * sc.xcs + (long long)kz * L;
    for (int i = threadIdx.x; i < L; i += NT) s_in[i] = scl_g[i];
    __syncthreads();
    __half2* hb = reinterpret_cast<__half2*>(spec) + boff;
    const __half2* hsrc[1] = {hb};
    const float* scl[1] = {s_in};
    const int nvalid[1] = {min(16, ncols - x0)};
    int nvs[2] = {(nvalid[0] + 1) / 2, nvalid[0] / 2};
    load_pairs_h<L, T, NT, First::R, 1>(v, E, hsrc, nvalid, 16, scl);
    __syncthreads();
    col_fft<L, T, NT, NH, INV, false>(v, lds, tw_s, 1);
    float m[2];
    cols_absmax<L, T, NT, Last::R, 2>(v, E, nvs, m);
    m[0] = fmaxf(m[0], m[1]);
    block_max<NT, 1>(m);
    const float scv = tile_scale(m[0]);
    const float inv[1] = {1.0f / scv};
    __half2* hdst[1] = {hb};
    store_pairs_h<L, T, NT, Last::R, 1>(v, E, hdst, nvalid, 16, inv);
    if (threadIdx.x == 0) sc.ys[comp * sc.ycs + (long long)t * L + kz] = scv;
  } else {
    load_cols<L, T, NT, First::R, NH>(v, E, ptr, nv, 16);
    __syncthreads();
    col_fft<L, T, NT, NH, INV, false>(v, lds, tw_s, 1);
    store_cols<L, T, NT, Last::R, NH>(v, E, ptr, nv, 16);
  }
}

// ----------------------------------------------------------------------------
// y pass with the radix-16 stage on the matrix cores, BF16x3 split products.
//
// A length-L transform (L = 16 M) is X[k2 + 16 k1] = sum_n1 W_M^(n1 k1)
// W_L^(n1 k2) sum_n2 x[n1 + M n2] W_16^(n2 k2).  The inner DFT-16 over n2 is a
// dense 16 x 16 complex matrix F times the 16 values of every (n1, column):
// with real and imaginary parts stacked, Re Y = [Re F | -Im F] [Re x; Im x]
// and Im Y = [Im F | Re F] [Re x; Im x], one 16 x 32 by 32 x 16 product per
// n1 for the 16 columns of the block, i.e. v_mfma_f32_16x16x32_bf16.  Each
// FP32 operand is split into BF16 parts a = a_hi + a_lo (a_lo the BF16
// rounding of a - a_hi) and a b = a_hi b_hi + a_hi b_lo + a_lo b_hi, three
// products accumulated in FP32: about 16 bits of the operands survive
// (the term a_lo b_lo and the rounding of the lo parts are dropped).  The
// twiddles W_L^(n1 k2) and the outer DFT-M over n1 stay in FP32 on the VALU.
// Operand layout of the instruction (16 x 32 A, 32 x 16 B, 16 x 16 D): lane l
// holds A[l mod 16][8 (l div 16) + j], B[8 (l div 16) + j][l mod 16] for
// j < 8, and D[4 (l div 16) + i][l mod 16] for i < 4.
// ----------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <int L, bool INV>
__global__ __launch_bounds__(256) void k_ypass_mfma(float2* spec, long long comp_stride, int ncols,
                                                    const float2* __restrict__ tw, Gate gate) {
  if (gated_off(gate)) return;
  constexpr int M = L / 16;
  constexpr int TPW = M / 4;                       // n1 values per wave
  constexpr int RS = 17;                           // LDS row of the 16 columns, padded
  constexpr int ZS = 256 + 4;                      // LDS row of the 256 (k2, column) sequences
  constexpr int XE = L * RS > M * ZS ? L * RS : M * ZS;
  static_assert(M >= 4, "at least one n1 per wave");
  extern __shared__ float2 lds[];
  float2* X = lds;                                 // X[n][c] at n RS + c, then Z[n1][q] at n1 ZS + q
  float2* tw_s = lds + XE;
  // block order as in k_ypass
  const int nt = gridDim.x, nc = gridDim.z;
  const long long b = blockIdx.x + (long long)nt * (blockIdx.y + (long long)L * blockIdx.z);
  int t, kz, comp;
  if constexpr (!INV) {
    t = (int)(b % nt);
    comp = (int)((b / nt) % nc);
    kz = L - 1 - (int)(b / ((long long)nt * nc));
  } else {
    kz = (int)(b % L);
    comp = (int)((b / L) % nc);
    t = nt - 1 - (int)(b / ((long long)L * nc));
  }
  const int nv = min(16, ncols - t * 16);
  float2* base = spec + comp * comp_stride + ((long long)t * L + kz) * L * 16;
  load_twiddles<L>(tw_s, tw, 256);
  for (int i = threadIdx.x; i < L * 16; i += 256) {
    const int r = i >> 4, c = i & 15;
    X[r * RS + c] = (c < nv) ? base[(long long)r * 16 + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  // A fragments: rows k2 = col of [Re F | -Im F] and [Im F | Re F]
  bf16x8_t arh, arl, aih, ail;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = 8 * grp + j, n2 = kk & 15, q = (col * n2) & 15;
    const float c = q < 8 ? kC16[q] : -kC16[q - 8];
    const float sn = q < 8 ? kS16[q] : -kS16[q - 8];
    const float fr = c, fi = INV ? sn : -sn;           // W_16^(n2 k2), conjugated for the inverse
    const bool re = kk < 16;
    __bf16 h, l;
    split_bf16(re ? fr : -fi, h, l); arh[j] = h; arl[j] = l;
    split_bf16(re ? fi : fr, h, l); aih[j] = h; ail[j] = l;
  }
  // B fragments of the wave's n1 values: column col, n2 = kk mod 16, real part for kk < 16
  bf16x8_t bh[TPW], bl[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int n1 = wave + 4 * u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kk = 8 * grp + j, n2 = kk & 15;
      const float2 x = X[(n1 + M * n2) * RS + col];
      __bf16 h, l;
      split_bf16(kk < 16 ? x.x : x.y, h, l);
      bh[u][j] = h;
      bl[u][j] = l;
    }
  }
  __syncthreads();                                 // X is overwritten by Z below
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int n1 = wave + 4 * u;
    f32x4_t yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bh[u], yr, 0, 0, 0);
    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bl[u], yr, 0, 0, 0);
    yr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bh[u], yr, 0, 0, 0);
    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bh[u], yi, 0, 0, 0);
    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bl[u], yi, 0, 0, 0);
    yi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bh[u], yi, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k2 = 4 * grp + i;
      float2 w = tw_s[n1 * k2];                    // W_L^(n1 k2), n1 k2 < L
      if (INV) w.y = -w.y;
      X[n1 * ZS + k2 * 16 + col] = cmul(make_float2(yr[i], yi[i]), w);
    }
  }
  __syncthreads();
  // the DFT-M over n1 of the 256 sequences q = 16 k2 + column (in place)
  block_fft<M, 256, 256, true, INV>(X, 1, ZS, tw_s, L / M);
  for (int i = threadIdx.x; i < L * 16; i += 256) {
    const int k = i >> 4, c = i & 15;
    if (c < nv) base[(long long)k * 16 + c] = X[(k >> 4) * ZS + (k & 15) * 16 + c];
  }
}

// B(k) = sum_{j < fb} w_L^(k j): the DFT along one axis of a block of fb
// ones, from the transform's twiddle table (w_L^t at tw[t]).
__device__ __forceinline__ float2 block_sum(const float2* tw, int k, int fb, int L) {
  float2 b = make_float2(1.0f, 0.0f);
  for (int j = 1; j < fb; ++j) b = cadd(b, tw[(k * j) & (L - 1)]);
  return b;
}

enum { Z_FWD = 0, Z_INV = 1, Z_NEWTON = 2, Z_CURL = 3, Z_CURL_FINAL = 4, Z_DIV = 5, Z_NEWTON_H0 = 6, Z_POISSON = 7,
       Z_NEWTON_WARM = 8, Z_APPARENT = 9, Z_GRAD = 10, Z_NEWTON_COARSE = 11, Z_POISSON_SPEC = 12 };

template <int ZOP> struct ZComp;
template <> struct ZComp<Z_FWD>        { static constexpr int IN = 1, OUT = 1; };
template <> struct ZComp<Z_INV>        { static constexpr int IN = 1, OUT = 1; };
template <> struct ZComp<Z_NEWTON>     { static constexpr int IN = 1, OUT = 3; };
template <> struct ZComp<Z_NEWTON_H0>  { static constexpr int IN = 4, OUT = 3; };
template <> struct ZComp<Z_NEWTON_WARM> { static constexpr int IN = 4, OUT = 3; };
template <> struct ZComp<Z_NEWTON_COARSE> { static constexpr int IN = 1, OUT = 3; };
template <> struct ZComp<Z_POISSON_SPEC> { static constexpr int IN = 1, OUT = 1; };
template <> struct ZComp<Z_CURL>       { static constexpr int IN = 3, OUT = 3; };
template <> struct ZComp<Z_CURL_FINAL> { static constexpr int IN = 3, OUT = 1; };
template <> struct ZComp<Z_DIV>        { static constexpr int IN = 3, OUT = 3; };
template <> struct ZComp<Z_POISSON>    { static constexpr int IN = 1, OUT = 1; };
template <> struct ZComp<Z_APPARENT>   { static constexpr int IN = 1, OUT = 1; };
template <> struct ZComp<Z_GRAD>       { static constexpr int IN = 1, OUT = 3; };

// z pass: forward z transform of the input components, the spectral operator
// at every (kx, ky, kz) in registers, inverse z transform, store.  A block
// owns 2 T kx-columns of one ky row as two halves of T columns (slot 2 c + h
// holds field component c of half h); the halves share the LDS exchange
// buffer, and together they read and write whole 128-byte lines.
//   Z_NEWTON    : in = rho_hat (x, y transformed, in phiN); stores phi_N_hat =
//                 -4 pi G A rho_hat into phiN and outputs g_N_hat = -i kappa
//                 phi_N_hat (/N^3) as three components; accumulates the
//                 Parseval sum of |g_N_hat|^2 per block.
//   Z_NEWTON_H0 : as Z_NEWTON plus the divergence-free part of the x, y
//                 transformed H0 components from spec.
//   Z_CURL      : g <- kt At (kt . g) / N^3
//   Z_CURL_FINAL: phi_hat = i At (kt . g) / N^3 (one output component)
//   Z_DIV       : F = F' + kt At kt . (g_N - F'), g_N = -i kappa phi_N (/N^3)
//   Z_POISSON   : phi_N_hat = -4 pi G A rho_hat / N^3 (one component, in place)
//   Z_APPARENT  : rho_A_hat = -|kt|^2 phi_hat / (4 pi G N^3), the apparent density
//                 of Eq. apparentdensity (one component, in place)
//   Z_NEWTON_WARM: as Z_NEWTON_H0 with the previous F in place of H0, whose
//                 divergence-free part minus that of g_N starts H:
//                 F = P_L g_N + P_T F_prev
//   Z_GRAD      : g = -i kt phi_hat / N^3 (three output components), the field
//                 of a potential as the curl-free projection forms it
//   Z_POISSON_SPEC: Z_POISSON without the inverse z transform: the Newton
//                 potential's full spectrum (kx, ky, kz), normalised, to out
//   Z_NEWTON_COARSE: as Z_NEWTON_H0 with H0 constant on blocks of cfb^3 cells,
//                 H0 = rms y(parent): its DFT is Y(kx mod cn, ky mod cn,
//                 kz mod cn) B(kx) B(ky) B(kz), Y the coarse DFT (cspec) and
//                 B(k) = sum_{j < cfb} w_N^(k j), so no full-resolution H0
// IO as PassDesc::io; the half-precision forms read the forward y pass's
// scales and write one scale per component of the block's 8 kx columns.
template <int L, int T, int NT, int HZ, int ZOP, int IO = 0>
__global__ __launch_bounds__(NT) void k_zpass(ZArgs a, const float2* __restrict__ tw, Scales sc, Gate gate) {
  if (gated_off(gate)) return;
  constexpr bool IN_H = IO == 1 || IO == 3, OUT_H = IO == 1 || IO == 2;
  // With half-precision spectra the block owns a whole group of 16 kx as its
  // even and odd columns (two interleaved sets of 8; column 2 q + h is
  // element q of set h): CS is the column stride of a set, hoff(h) its first
  // column.
  constexpr bool IL = IO != 0;
  static_assert(!IL || (HZ == 2 && T == 8), "half-precision z tiles are two interleaved sets of 8 columns");
  constexpr int CS = IL ? 2 : 1;
  auto hoff = [](int h) { return IL ? h : h * T; };
  constexpr int E = ColCfg<L, T, NT>::E;
  constexpr int NIN = ZComp<ZOP>::IN, NOUT = ZComp<ZOP>::OUT;
  constexpr int NV = NIN > NOUT ? NIN : NOUT;
  extern __shared__ float2 lds[];
  float2* tw_s = lds + ColBuf<L, T>::elems;
  static_assert(16 % (HZ * T) == 0, "a z-pass tile lies inside one group of 16 kx");
  constexpr int NHZ = 16 / (HZ * T);                 // tiles per group of 16 kx
  // Workgroups go to the 8 XCDs round robin (block b to XCD b % 8), each XCD
  // with its own L2.  A tile of T = 8 complex columns is half a 128-byte line,
  // so the two tiles of a group read the same lines.  Blocks are numbered so
  // that b and b + 8 (same XCD, dispatched one after the other) take the two
  // tiles of one (group, ky), letting the second read hit in that XCD's L2,
  // and so that the blocks in flight on an XCD cover neighbouring ky rows.
  const int nb = gridDim.x;
  const int lb = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  const int h0 = lb % NHZ, y = (lb / NHZ) % L, grp = lb / (NHZ * L);
  const int x0 = 16 * grp + h0 * HZ * T;
  if (x0 >= a.ncols) {                               // the unused tail of the last group
    if (a.partials && threadIdx.x == 0) a.partials[blockIdx.x] = 0.0;
    return;
  }
  const long long row = (long long)L * 16;                                  // kz stride
  const long long off = ((long long)(x0 >> 4) * L * L + y) * 16 + (x0 & 15);
  load_twiddles<L>(tw_s, tw, NT);
  int nvh[HZ];
  const int nvalid = min(16, a.ncols - x0);           // valid columns of an interleaved group
#pragma unroll
  for (int h = 0; h < HZ; ++h) nvh[h] = IL ? (nvalid + 1 - h) / 2 : min(T, a.ncols - x0 - h * T);

  float2 v[HZ * NV * E];
  using First = PlanAt<L, false, 0>;
  using Last = PlanAt<L, false, Plan<L>::S - 1>;
  const float2* src[HZ * NIN];
  int nvs[HZ * NV];
#pragma unroll
  for (int c = 0; c < NV; ++c)
#pragma unroll
    for (int h = 0; h < HZ; ++h) nvs[HZ * c + h] = nvh[h];
#pragma unroll
  for (int c = 0; c < NIN; ++c) {
    const float2* p = (ZOP == Z_NEWTON || ZOP == Z_NEWTON_H0 || ZOP == Z_NEWTON_WARM || ZOP == Z_NEWTON_COARSE)
                          ? (c == 0 ? a.phiN + off : a.spec + (c - 1) * a.comp_stride + off)
                          : a.spec + c * a.comp_stride + off;
#pragma unroll
    for (int h = 0; h < HZ; ++h) src[HZ * c + h] = p + hoff(h);
  }
  float2* dst1[HZ];
#pragma unroll
  for (int h = 0; h < HZ; ++h) dst1[h] = a.spec + off + hoff(h);
  if (ZOP == Z_INV) {
    load_cols<L, T, NT, First::R, HZ>(v, E, src, nvs, row);
    __syncthreads();
    col_fft<L, T, NT, HZ, true, false>(v, lds, tw_s, 1);
    store_cols<L, T, NT, Last::R, HZ>(v, E, dst1, nvs, row);
    return;
  }
  // Z_DIV also needs phi_N hat at the operator's elements (kz = j + r L / RL of
  // the last stage); those loads are issued here, with the column loads, so
  // their latency overlaps the forward transform.
  constexpr int RLP = Last::R;
  using BLP = Bfly<L, T, NT, RLP>;
  float2 php[(ZOP == Z_DIV) ? HZ * BLP::BPT * RLP : 1];
  if constexpr (ZOP == Z_DIV) {
#pragma unroll
    for (int u = 0; u < BLP::BPT; ++u) {
      const int b = threadIdx.x + u * NT;
      const int q = b % T, j = b / T;
#pragma unroll
      for (int h = 0; h < HZ; ++h)
#pragma unroll
        for (int r = 0; r < RLP; ++r) {
          const int kz = j + r * (L / RLP);
          const bool ok = BLP::valid(b) && q < nvh[h];
          php[(h * BLP::BPT + u) * RLP + r] =
              ok ? a.phiN[(long long)kz * row + off + hoff(h) + q * CS] : make_float2(0.0f, 0.0f);
        }
    }
  }
  if constexpr (IN_H) {
    // half-precision inputs (never phi_N, which stays FP32), one scale per kz
    // from the forward y pass's tiles (group, plane kz), staged in LDS
    __shared__ float s_in[NIN * L];
#pragma unroll
    for (int c = 0; c < NIN; ++c)
      for (int i = threadIdx.x; i < L; i += NT) s_in[c * L + i] = sc.ys[c * sc.ycs + (long long)grp * L + i];
    __syncthreads();
    const __half2* hs[NIN];
    const float* scl[NIN];
    int nval[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) {
      hs[c] = reinterpret_cast<const __half2*>(a.spec) + c * a.comp_stride + off;
      scl[c] = s_in + c * L;
      nval[c] = nvalid;
    }
    load_pairs_h<L, T, NT, First::R, NIN>(v, E, hs, nval, row, scl);
  } else {
    load_cols<L, T, NT, First::R, HZ * NIN, CS>(v, E, src, nvs, row);
  }
  __syncthreads();
  col_fft<L, T, NT, HZ * NIN, false, false>(v, lds, tw_s, 1);
  if (ZOP == Z_FWD) {
    store_cols<L, T, NT, Last::R, HZ>(v, E, dst1, nvs, row);
    return;
  }

  // ---- spectral operator on the last stage's elements kz = j + r L / RL
  constexpr int RL = Last::R;
  using BL = Bfly<L, T, NT, RL>;
  double acc = 0.0;
  const float ky = a.kv[y], ty = a.kt[y], kapy = a.kap[y];
#pragma unroll
  for (int u = 0; u < BL::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!BL::valid(b)) continue;
    const int q = b % T, j = b / T;
#pragma unroll
    for (int h = 0; h < HZ; ++h) {
      const int kxi = x0 + hoff(h) + q * CS;
      const bool inb = q < nvh[h];
      const float kx = a.kv[kxi < L ? kxi : 0];
      const float tx = (kxi < L / 2) ? a.kt[kxi] : 0.0f;
      const float kpx = (kxi < L / 2) ? a.kap[kxi] : 0.0f;
      float2 bxy = make_float2(1.0f, 0.0f);          // coarse start: B(kx) B(ky)
      if constexpr (ZOP == Z_NEWTON_COARSE)
        bxy = cmul(block_sum(tw_s, kxi, a.cfb, L), block_sum(tw_s, y, a.cfb, L));
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int kz = j + r * (L / RL);
        const int e = u * RL + r;
        if constexpr (ZOP == Z_POISSON || ZOP == Z_POISSON_SPEC) {
          const float kzz = a.kv[kz];
          const float k2 = kx * kx + ky * ky + kzz * kzz;
          const float A = (k2 > 0.0f) ? hw_rcp(k2) : 0.0f;
          v[h * E + e] = cscale(v[h * E + e], a.newton_coef * A * a.scale);
          continue;
        }
        if constexpr (ZOP == Z_GRAD) {
          const float2 g = cscale(mul_mi<false>(v[h * E + e]), a.scale);     // -i phi_hat / N^3
          v[(0 * HZ + h) * E + e] = cscale(g, tx);
          v[(1 * HZ + h) * E + e] = cscale(g, ty);
          v[(2 * HZ + h) * E + e] = cscale(g, a.kt[kz]);
          continue;
        }
        if constexpr (ZOP == Z_APPARENT) {
          const float tz = a.kt[kz];
          const float t2 = tx * tx + ty * ty + tz * tz;
          v[h * E + e] = cscale(v[h * E + e], t2 / a.newton_coef * a.scale);
          continue;
        }
        float2* v0 = v + (0 * HZ + h) * E + e;
        float2* v1 = v + (1 * HZ + h) * E + e;
        float2* v2 = v + (2 * HZ + h) * E + e;
        if (ZOP == Z_NEWTON || ZOP == Z_NEWTON_H0 || ZOP == Z_NEWTON_WARM || ZOP == Z_NEWTON_COARSE) {
          const float kzz = a.kv[kz];
          const float k2 = kx * kx + ky * ky + kzz * kzz;
          const float A = (k2 > 0.0f) ? hw_rcp(k2) : 0.0f;
          const float2 ph = cscale(*v0, a.newton_coef * A);     // phi_N hat (raw DFT)
          if (inb) a.phiN[(long long)kz * row + off + hoff(h) + q * CS] = ph;
          const float kpz = a.kap[kz];
          const float2 g = cscale(mul_mi<false>(ph), a.scale);
          float2 o0 = cscale(g, kpx), o1 = cscale(g, kapy), o2 = cscale(g, kpz);
          if (ZOP == Z_NEWTON_H0 || ZOP == Z_NEWTON_WARM || ZOP == Z_NEWTON_COARSE) {
            // H0 (or F_prev) components arrived in input slots 1..3 (component c
            // at slot HZ c + h), or H0 comes from the coarse spectrum; H starts
            // at the divergence-free part of H0, or of F_prev - g_N:
            // h - kt At (kt . h)
            const float tz = a.kt[kz];
            const float t2 = tx * tx + ty * ty + tz * tz;
            const float At = (t2 > 0.0f) ? hw_rcp(t2) : 0.0f;
            float2 h0, h1, h2;
            if constexpr (ZOP == Z_NEWTON_COARSE) {
              const int m = a.cn - 1;
              const long long cn3 = (long long)a.cn * a.cn * a.cn;
              const long long ci = ((long long)(kz & m) * a.cn + (y & m)) * a.cn + (kxi & m);
              const float2 bb = cmul(bxy, block_sum(tw_s, kz, a.cfb, L));
              h0 = cmul(a.cspec[ci], bb);
              h1 = cmul(a.cspec[cn3 + ci], bb);
              h2 = cmul(a.cspec[2 * cn3 + ci], bb);
            } else {
              h0 = v[(1 * HZ + h) * E + e];
              h1 = v[(2 * HZ + h) * E + e];
              h2 = v[(3 * HZ + h) * E + e];
            }
            if (ZOP == Z_NEWTON_WARM) {
              // o_c = g_N hat (already divided by N^3); bring F_prev to the same units
              const float rs = 1.0f / a.scale;
              h0 = csub(h0, cscale(o0, rs));
              h1 = csub(h1, cscale(o1, rs));
              h2 = csub(h2, cscale(o2, rs));
            }
            const float2 dd = cscale(cadd(cadd(cscale(h0, tx), cscale(h1, ty)), cscale(h2, tz)), At);
            o0 = cadd(o0, cscale(csub(h0, cscale(dd, tx)), a.scale));
            o1 = cadd(o1, cscale(csub(h1, cscale(dd, ty)), a.scale));
            o2 = cadd(o2, cscale(csub(h2, cscale(dd, tz)), a.scale));
          }
          *v0 = o0;
          *v1 = o1;
          *v2 = o2;
          if (inb) {
            const double w = (kxi == 0 || kxi == L / 2) ? 1.0 : 2.0;
            const double m2 = (double)ph.x * ph.x + (double)ph.y * ph.y;
            acc += w * m2 * ((double)kpx * kpx + (double)kapy * kapy + (double)kpz * kpz);
          }
        } else {
          const float tz = a.kt[kz];
          const float t2 = tx * tx + ty * ty + tz * tz;
          const float At = (t2 > 0.0f) ? hw_rcp(t2) : 0.0f;
          const float2 g0 = *v0, g1 = *v1, g2 = *v2;
          if constexpr (ZOP == Z_DIV) {
            const float2 ph = php[(h * BLP::BPT + u) * RLP + r];
            const float2 mph = mul_mi<false>(ph);
            const float2 d0 = csub(cscale(mph, kpx), g0);
            const float2 d1 = csub(cscale(mph, kapy), g1);
            const float2 d2 = csub(cscale(mph, a.kap[kz]), g2);
            const float2 dd = cscale(cadd(cadd(cscale(d0, tx), cscale(d1, ty)), cscale(d2, tz)), At);
            *v0 = cscale(cadd(g0, cscale(dd, tx)), a.scale);
            *v1 = cscale(cadd(g1, cscale(dd, ty)), a.scale);
            *v2 = cscale(cadd(g2, cscale(dd, tz)), a.scale);
          } else {
            const float2 dot = cadd(cadd(cscale(g0, tx), cscale(g1, ty)), cscale(g2, tz));
            if (ZOP == Z_CURL) {
              const float2 sc = cscale(dot, At * a.scale);
              *v0 = cscale(sc, tx);
              *v1 = cscale(sc, ty);
              *v2 = cscale(sc, tz);
            } else {
              *v0 = cscale(mul_mi<true>(dot), At * a.scale);    // phi_hat = i At kt.g
            }
          }
        }
      }
    }
  }
  if constexpr (ZOP == Z_POISSON_SPEC) {
    float2* ob = (a.out ? a.out : a.spec) + off;
    float2* dsp[HZ];
#pragma unroll
    for (int h = 0; h < HZ; ++h) dsp[h] = ob + hoff(h);
    store_cols<L, T, NT, Last::R, HZ>(v, E, dsp, nvs, row);
    return;
  }
  if (ZOP == Z_NEWTON || ZOP == Z_NEWTON_H0 || ZOP == Z_NEWTON_WARM || ZOP == Z_NEWTON_COARSE) {
    __shared__ double red[NT / 64];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NT / 64; ++w) t += red[w];
      a.partials[blockIdx.x] = t;
    }
  }

  // ---- inverse z transform with the reversed plan: its first stage takes the
  // elements the forward last stage produced, so no exchange is needed here.
  col_fft<L, T, NT, HZ * NOUT, true, true>(v, lds, tw_s, 1);
  if constexpr (OUT_H) {
    float m[HZ * NOUT], inv[NOUT];
    __half2* hd[NOUT];
    int nval[NOUT];
    cols_absmax<L, T, NT, First::R, HZ * NOUT>(v, E, nvs, m);
#pragma unroll
    for (int c = 0; c < NOUT; ++c) m[c] = fmaxf(m[2 * c], m[2 * c + 1]);
    block_max<NT, NOUT>(m);
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      const float scv = tile_scale(m[c]);
      inv[c] = 1.0f / scv;
      hd[c] = reinterpret_cast<__half2*>(a.spec) + c * a.comp_stride + off;
      nval[c] = nvalid;
      if (threadIdx.x == 0) sc.zs[c * sc.zcs + (long long)grp * L + y] = scv;
    }
    store_pairs_h<L, T, NT, First::R, NOUT>(v, E, hd, nval, row, inv);
    return;
  }
  // (an FP32 result of half-precision input goes to a.out: written in place
  // it would overlap FP16 columns other blocks have still to read)
  float2* obase = a.out ? a.out : a.spec;
  float2* dst[HZ * NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c)
#pragma unroll
    for (int h = 0; h < HZ; ++h) dst[HZ * c + h] = obase + c * a.comp_stride + off + hoff(h);
  store_cols<L, T, NT, First::R, HZ * NOUT, CS>(v, E, dst, nvs, row);
}

// Sum of partials[0..n) into out[0] (FP64), one block.
__global__ __launch_bounds__(1024) void k_reduce_partials(const double* __restrict__ partials, int n,
                                                          double* out, Gate gate) {
  if (gated_off(gate)) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += partials[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = t;
  }
}

// ----------------------------------------------------------------------------
// host-side launchers
// ----------------------------------------------------------------------------
namespace {
constexpr int kNT = 256;
constexpr int kNTZ = PM_NTZ;

template <int N>
struct Cfg {
  static constexpr int H = N / 2;
  static constexpr int ROWS = (1024 / H) < 1 ? 1 : ((1024 / H) > 64 ? 64 : (1024 / H));
  static constexpr int TY = PM_TY;
  static constexpr int TZ = PM_TZ;
};

template <int N, int XMODE, int NC, int IO = 0>
hipError_t launch_x(const FftGeom& g, float2* spec, float* real, long long real_cs, int mu_mode,
                    float inv_a0, float* fprev, double* partials, hipStream_t st, Dipole dip = Dipole{},
                    const float* base = nullptr, Coarse co = Coarse{}) {
  using C = Cfg<N>;
  if constexpr (N == 512 || N == 1024) {
    using X = XWave<N / 2>;
    const size_t sh = sizeof(float2) * (N + (size_t)X::ROWS * X::XB + X::TWL);
    hipLaunchKernelGGL((k_xpass_wave<N / 2, XMODE, NC, IO>), dim3(N * N / X::ROWS), dim3(256), sh, st, spec,
                       g.comp_stride, real, real_cs, g.tw, mu_mode, inv_a0, fprev, partials, dip, base, g.sc,
                       g.gate, co);
    return hipGetLastError();
  } else {
    const int blocks = N * N / C::ROWS;
    const size_t sh = sizeof(float2) * ((size_t)(C::H + 1) * (NC * C::ROWS + 1) + N);
    hipLaunchKernelGGL((k_xpass<C::H, C::ROWS, NC, kNT, XMODE, IO>), dim3(blocks), dim3(kNT), sh, st, spec,
                       g.comp_stride, real, real_cs, g.tw, mu_mode, inv_a0, fprev, partials, dip, base, g.sc,
                       g.gate, co);
    return hipGetLastError();
  }
}

template <int N, bool INV, int IO = 0>
hipError_t launch_y(const FftGeom& g, float2* spec, int ncomp, hipStream_t st) {
  using C = Cfg<N>;
  constexpr int TY = IO ? 8 : C::TY;                 // FP16: two interleaved sets of 8 columns
  const int tiles = (C::H + 1 + 15) / 16;
  const size_t sh = sizeof(float2) * ((size_t)ColBuf<N, TY>::elems + N);
  hipLaunchKernelGGL((k_ypass<N, TY, kNT, INV, IO>), dim3(tiles, N, ncomp), dim3(kNT), sh, st, spec,
                     g.comp_stride, C::H + 1, g.tw, g.sc, g.gate);
  return hipGetLastError();
}

template <int N, bool INV>
hipError_t launch_y_mfma(const FftGeom& g, float2* spec, int ncomp, hipStream_t st) {
  if constexpr (N >= 64 && N <= 512) {
    constexpr int M = N / 16;
    constexpr size_t xe = (size_t)N * 17 > (size_t)M * 260 ? (size_t)N * 17 : (size_t)M * 260;
    const int tiles = (N / 2 + 1 + 15) / 16;
    hipLaunchKernelGGL((k_ypass_mfma<N, INV>), dim3(tiles, N, ncomp), dim3(256), sizeof(float2) * (xe + N), st,
                       spec, g.comp_stride, N / 2 + 1, g.tw, g.gate);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, int ZOP, int IO = 0>
hipError_t launch_z(const FftGeom& g, ZArgs a, hipStream_t st) {
  using C = Cfg<N>;
  a.comp_stride = g.comp_stride;
  a.ncols = C::H + 1;
  if constexpr (IO != 0) {
    // half-precision spectra: a block owns a whole group of 16 kx
    const size_t sh = sizeof(float2) * ((size_t)ColBuf<N, 8>::elems + N);
    hipLaunchKernelGGL((k_zpass<N, 8, kNTZ, 2, ZOP, IO>), dim3(z_blocks_io(N, IO)), dim3(kNTZ), sh, st, a, g.tw,
                       g.sc, g.gate);
  } else {
    const size_t sh = sizeof(float2) * ((size_t)ColBuf<N, C::TZ>::elems + N);
    hipLaunchKernelGGL((k_zpass<N, C::TZ, kNTZ, PM_HZ, ZOP, IO>), dim3(z_blocks(N)), dim3(kNTZ), sh, st, a, g.tw,
                       g.sc, g.gate);
  }
  return hipGetLastError();
}

template <int N>
hipError_t run_pass(const FftGeom& g, const PassDesc& d, hipStream_t st) {
  switch (d.kind) {
    case PASS_X_FWD_REAL:
      return launch_x<N, X_FWD_REAL, 1>(g, d.spec, d.real, d.real_cs, 0, 0.f, nullptr, nullptr, st, d.dip);
    case PASS_X_FWD_REAL3:
      return launch_x<N, X_FWD_REAL, 3>(g, d.spec, d.real, d.real_cs, 0, 0.f, nullptr, nullptr, st);
    case PASS_X_FWD_COARSE3:
      if (!d.co.y || !d.co.rms || d.co.f < 2 || d.co.n * d.co.f != N) return hipErrorInvalidValue;
      return launch_x<N, X_FWD_COARSE, 3>(g, d.spec, nullptr, 0, 0, 0.f, nullptr, nullptr, st, Dipole{}, nullptr,
                                          d.co);
    case PASS_X_INV_REAL:
      return launch_x<N, X_INV_REAL, 1>(g, d.spec, d.real, d.real_cs, 0, 0.f, nullptr, nullptr, st);
    case PASS_X_INV_REAL3:
      return launch_x<N, X_INV_REAL, 3>(g, d.spec, d.real, d.real_cs, 0, 0.f, nullptr, nullptr, st);
    case PASS_X_NU:
      if (d.fprev)
        return launch_x<N, X_FUSED_NU_KEEP, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, d.fprev, d.partials, st);
      return launch_x<N, X_FUSED_NU, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr, st);
    case PASS_X_MU:
      return launch_x<N, X_FUSED_MU, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr, st);
    case PASS_X_LIN_NU:
      if (d.io == 1)
        return d.fprev ? launch_x<N, X_LIN_NU_KEEP, 3, 1>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, d.fprev,
                                                          d.partials, st, Dipole{}, d.base)
                       : launch_x<N, X_LIN_NU, 3, 1>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr,
                                                     st, Dipole{}, d.base);
      return d.fprev ? launch_x<N, X_LIN_NU_KEEP, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, d.fprev,
                                                     d.partials, st, Dipole{}, d.base)
                     : launch_x<N, X_LIN_NU, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr, st,
                                                Dipole{}, d.base);
    case PASS_X_LIN_MU:
      if (d.io == 1)
        return launch_x<N, X_LIN_MU, 3, 1>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr, st,
                                           Dipole{}, d.base);
      return launch_x<N, X_LIN_MU, 3>(g, d.spec, nullptr, 0, d.mu_mode, d.inv_a0, nullptr, nullptr, st, Dipole{},
                                      d.base);
    case PASS_Y_FWD:
      if (d.io == 1) return launch_y<N, false, 1>(g, d.spec, d.ncomp, st);
      return g.bf16x3 ? launch_y_mfma<N, false>(g, d.spec, d.ncomp, st) : launch_y<N, false>(g, d.spec, d.ncomp, st);
    case PASS_Y_INV:
      if (d.io == 1) return launch_y<N, true, 1>(g, d.spec, d.ncomp, st);
      return g.bf16x3 ? launch_y_mfma<N, true>(g, d.spec, d.ncomp, st) : launch_y<N, true>(g, d.spec, d.ncomp, st);
    case PASS_Z_FWD: return launch_z<N, Z_FWD>(g, d.z, st);
    case PASS_Z_INV: return launch_z<N, Z_INV>(g, d.z, st);
    case PASS_Z_NEWTON:
      if (d.io == 2) return launch_z<N, Z_NEWTON, 2>(g, d.z, st);
      if (d.z.with_h0 == 2) return launch_z<N, Z_NEWTON_WARM>(g, d.z, st);
      if (d.z.with_h0 == 3) {
        if constexpr (N <= 512) {
          if (!d.z.cspec || d.z.cfb < 2 || d.z.cn * d.z.cfb != N) return hipErrorInvalidValue;
          return launch_z<N, Z_NEWTON_COARSE>(g, d.z, st);
        } else {
          return hipErrorInvalidValue;
        }
      }
      return d.z.with_h0 ? launch_z<N, Z_NEWTON_H0>(g, d.z, st) : launch_z<N, Z_NEWTON>(g, d.z, st);
    case PASS_Z_CURL: return d.io == 1 ? launch_z<N, Z_CURL, 1>(g, d.z, st) : launch_z<N, Z_CURL>(g, d.z, st);
    case PASS_Z_CURL_FINAL:
      return d.io == 3 ? launch_z<N, Z_CURL_FINAL, 3>(g, d.z, st) : launch_z<N, Z_CURL_FINAL>(g, d.z, st);
    case PASS_Z_DIV: return d.io == 1 ? launch_z<N, Z_DIV, 1>(g, d.z, st) : launch_z<N, Z_DIV>(g, d.z, st);
    case PASS_Z_POISSON: return launch_z<N, Z_POISSON>(g, d.z, st);
    case PASS_Z_POISSON_SPEC: return launch_z<N, Z_POISSON_SPEC>(g, d.z, st);
    case PASS_Z_APPARENT: return launch_z<N, Z_APPARENT>(g, d.z, st);
    case PASS_Z_GRAD: return launch_z<N, Z_GRAD>(g, d.z, st);
  }
  return hipErrorInvalidValue;
}
}  // namespace

int x_blocks(int N) {
  if (N == 512) return N * N / XWave<256>::ROWS;
  if (N == 1024) return N * N / XWave<512>::ROWS;
  const int H = N / 2;
  int rows = 1024 / H;
  rows = rows < 1 ? 1 : (rows > 64 ? 64 : rows);
  return N * N / rows;
}
int z_blocks(int N) {
  const int H = N / 2;
  return ((H + 1 + 15) / 16) * (16 / (PM_TZ * PM_HZ)) * N;
}
int z_blocks_io(int N, int io) {
  const int H = N / 2;
  return io ? ((H + 1 + 15) / 16) * N : z_blocks(N);
}

hipError_t fft_pass(const FftGeom& g0, const PassDesc& d, hipStream_t st) {
  FftGeom g = g0;
  g.gate = d.gate;
  switch (g.N) {
    case 16: return run_pass<16>(g, d, st);
    case 32: return run_pass<32>(g, d, st);
    case 64: return run_pass<64>(g, d, st);
    case 128: return run_pass<128>(g, d, st);
    case 256: return run_pass<256>(g, d, st);
    case 512: return run_pass<512>(g, d, st);
    case 1024: return run_pass<1024>(g, d, st);
  }
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------
// The learned start's coarse field in Fourier space.  Pass AXIS transforms the
// n-point sequences along that axis of every component in place: a block
// holds S = 16 of them in LDS (X sequences as rows, Y and Z sequences as
// columns of 16 consecutive X) and runs the block FFT with the box's twiddle
// table (n divides N).  The X pass reads the real field y and scales it by
// rms; the Y and Z passes work on the complex result.
// ----------------------------------------------------------------------------
namespace {
constexpr int kCsS = 16;
// INV: the inverse transform, whose last pass (AXIS 2) writes the real parts
// to y instead (the block means of the features, real by construction).
template <int L, int AXIS, bool INV = false>
__global__ __launch_bounds__(256) void k_coarse_spec(const float* __restrict__ y, const double* __restrict__ rms,
                                                      float2* cs, const float2* __restrict__ tw, int twmul,
                                                      float* yout = nullptr) {
  extern __shared__ float2 lds[];
  constexpr int S = kCsS, NT = 256;
  constexpr int QS = AXIS == 0 ? L + 1 : 1, IS = AXIS == 0 ? 1 : S + 1;
  constexpr int lines = L * (L / S);               // blocks per component
  const int c = blockIdx.x / lines, rem = blockIdx.x % lines;
  const int a = rem / (L / S), b0 = (rem % (L / S)) * S;
  const long long n3 = (long long)L * L * L;
  // element i of sequence q: X pass (Z = a, Y = b0 + q, X = i); Y pass
  // (Z = a, Y = i, X = b0 + q); Z pass (Z = i, Y = a, X = b0 + q)
  auto gidx = [&](int q, int i) -> long long {
    if (AXIS == 0) return ((long long)a * L + b0 + q) * L + i;
    if (AXIS == 1) return ((long long)a * L + i) * L + b0 + q;
    return ((long long)i * L + a) * L + b0 + q;
  };
  const float r = INV ? 1.0f : (float)*rms;
  for (int t = threadIdx.x; t < S * L; t += NT) {
    const int q = AXIS == 0 ? t / L : t % S, i = AXIS == 0 ? t % L : t / S;
    const long long gi = c * n3 + gidx(q, i);
    lds[q * QS + i * IS] = (AXIS == 0 && !INV) ? make_float2(r * y[gi], 0.0f) : cs[gi];
  }
  __syncthreads();
  block_fft<L, S, NT, AXIS != 0, INV>(lds, QS, IS, tw, twmul);
  for (int t = threadIdx.x; t < S * L; t += NT) {
    const int q = AXIS == 0 ? t / L : t % S, i = AXIS == 0 ? t % L : t / S;
    if (INV && AXIS == 2) yout[c * n3 + gidx(q, i)] = lds[q * QS + i * IS].x;
    else cs[c * n3 + gidx(q, i)] = lds[q * QS + i * IS];
  }
}

// Block means of g_N = -D phi_N over fb^3 blocks, in Fourier space: the mean
// over the blocks of a field sampled on the n^3 grid has the DFT
// Ghat(K) = (1/fb^3) sum over the fb^3 modes k = K mod n of
// -i kappa(k) phi_hat(k) conj(B(kx) B(ky) B(kz)), with kappa the central-
// difference symbol, phi_hat the normalised Newton spectrum in the kx half
// layout [kx/16][kz][ky][kx mod 16] (modes with kx > N/2 from their
// conjugates) and B(k) = sum_{j < fb} w_N^(k j).  One thread per coarse mode
// with Kx <= n/2 (the field is real); for 0 < Kx < n/2 it also writes the
// conjugate at -K, which no other thread writes.
template <int FB>
__global__ __launch_bounds__(256) void k_feat_spec(const float2* __restrict__ ph, const float* __restrict__ kap,
                                                    const float2* __restrict__ tw, int N, int n, float2* cs) {
  const int hx = n / 2 + 1;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)hx * n * n) return;
  const int Kx = (int)(t % hx), Ky = (int)((t / hx) % n), Kz = (int)(t / ((long long)hx * n));
  const long long n3 = (long long)n * n * n;
  float2 acc[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
#pragma unroll
  for (int mz = 0; mz < FB; ++mz) {
    const int kz = Kz + n * mz;
    const float2 bz = block_sum(tw, kz, FB, N);
#pragma unroll
    for (int my = 0; my < FB; ++my) {
      const int ky = Ky + n * my;
      const float2 byz = cmul(block_sum(tw, ky, FB, N), bz);
#pragma unroll
      for (int mx = 0; mx < FB; ++mx) {
        const int kx = Kx + n * mx;
        float2 v;
        if (kx <= N / 2) {
          v = ph[((long long)((kx >> 4) * N + kz) * N + ky) * 16 + (kx & 15)];
        } else {
          const int cx = N - kx, cy = (N - ky) & (N - 1), cz = (N - kz) & (N - 1);
          v = cconj(ph[((long long)((cx >> 4) * N + cz) * N + cy) * 16 + (cx & 15)]);
        }
        const float2 w = cmul(v, cconj(cmul(block_sum(tw, kx, FB, N), byz)));   // phi_hat conj(B)
        const float2 mw = mul_mi<false>(w);                                      // -i phi_hat conj(B)
        acc[0] = cadd(acc[0], cscale(mw, kap[kx]));
        acc[1] = cadd(acc[1], cscale(mw, kap[ky]));
        acc[2] = cadd(acc[2], cscale(mw, kap[kz]));
      }
    }
  }
  constexpr float inv = 1.0f / (FB * FB * FB);
  const long long v0 = ((long long)Kz * n + Ky) * n + Kx;
  const bool mirror = Kx > 0 && 2 * Kx < n;
  const long long v1 = ((long long)((n - Kz) & (n - 1)) * n + ((n - Ky) & (n - 1))) * n + (n - Kx);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float2 r = cscale(acc[c], inv);
    cs[c * n3 + v0] = r;
    if (mirror) cs[c * n3 + v1] = cconj(r);
  }
}

template <int L>
hipError_t coarse_feat_passes(const float2* tw, int N, float2* cs, float* g3, hipStream_t st) {
  const dim3 grid(3 * L * (L / kCsS));
  const size_t sh = sizeof(float2) * (size_t)(kCsS + 1) * (L + 1);
  hipLaunchKernelGGL((k_coarse_spec<L, 0, true>), grid, dim3(256), sh, st, nullptr, nullptr, cs, tw, N / L, nullptr);
  hipLaunchKernelGGL((k_coarse_spec<L, 1, true>), grid, dim3(256), sh, st, nullptr, nullptr, cs, tw, N / L, nullptr);
  hipLaunchKernelGGL((k_coarse_spec<L, 2, true>), grid, dim3(256), sh, st, nullptr, nullptr, cs, tw, N / L, g3);
  return hipGetLastError();
}

template <int L>
hipError_t coarse_spec_passes(const float2* tw, int N, const float* y, const double* rms, float2* cs,
                              hipStream_t st) {
  const dim3 grid(3 * L * (L / kCsS));
  const size_t sh = sizeof(float2) * (size_t)(kCsS + 1) * (L + 1);
  hipLaunchKernelGGL((k_coarse_spec<L, 0>), grid, dim3(256), sh, st, y, rms, cs, tw, N / L);
  hipLaunchKernelGGL((k_coarse_spec<L, 1>), grid, dim3(256), sh, st, y, rms, cs, tw, N / L);
  hipLaunchKernelGGL((k_coarse_spec<L, 2>), grid, dim3(256), sh, st, y, rms, cs, tw, N / L);
  return hipGetLastError();
}
}  // namespace

bool coarse_spectrum_supported(int n, int N) {
  // (the coarse-start z pass is compiled for boxes up to 512^3; at 1024^3 its
  // registers would spill, and the start is expanded in the x pass instead)
  return n >= 16 && n <= 256 && (n & (n - 1)) == 0 && N <= 512 && N % n == 0 && N / n >= 2;
}

hipError_t coarse_features(const FftGeom& g, const float2* phihat, const float* kap, int n, float2* cs, float* g3,
                           hipStream_t st) {
  if (!coarse_spectrum_supported(n, g.N)) return hipErrorInvalidValue;
  const int fb = g.N / n;
  const long long modes = (long long)(n / 2 + 1) * n * n;
  const dim3 grid((unsigned)((modes + 255) / 256));
  if (fb == 2) hipLaunchKernelGGL((k_feat_spec<2>), grid, dim3(256), 0, st, phihat, kap, g.tw, g.N, n, cs);
  else if (fb == 4) hipLaunchKernelGGL((k_feat_spec<4>), grid, dim3(256), 0, st, phihat, kap, g.tw, g.N, n, cs);
  else return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (n) {
    case 16: return coarse_feat_passes<16>(g.tw, g.N, cs, g3, st);
    case 32: return coarse_feat_passes<32>(g.tw, g.N, cs, g3, st);
    case 64: return coarse_feat_passes<64>(g.tw, g.N, cs, g3, st);
    case 128: return coarse_feat_passes<128>(g.tw, g.N, cs, g3, st);
    case 256: return coarse_feat_passes<256>(g.tw, g.N, cs, g3, st);
  }
  return hipErrorInvalidValue;
}

hipError_t coarse_spectrum(const FftGeom& g, const float* y, const double* rms, int n, float2* cs, hipStream_t st) {
  if (!coarse_spectrum_supported(n, g.N)) return hipErrorInvalidValue;
  switch (n) {
    case 16: return coarse_spec_passes<16>(g.tw, g.N, y, rms, cs, st);
    case 32: return coarse_spec_passes<32>(g.tw, g.N, y, rms, cs, st);
    case 64: return coarse_spec_passes<64>(g.tw, g.N, y, rms, cs, st);
    case 128: return coarse_spec_passes<128>(g.tw, g.N, y, rms, cs, st);
    case 256: return coarse_spec_passes<256>(g.tw, g.N, y, rms, cs, st);
  }
  return hipErrorInvalidValue;
}

hipError_t reduce_partials(const double* partials, int n, double* out, hipStream_t st, Gate gate) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, st, partials, n, out, gate);
  return hipGetLastError();
}

__global__ void k_tol_check(int* ctl, const double* __restrict__ acc, int k, int kmax, double tol, double n3) {
  if (threadIdx.x != 0 || ctl[0] != 0) return;
  bool stop = (k >= kmax);
  if (k >= 2) {
    const double gn = sqrt(acc[0] / n3);
    const double r = gn > 0.0 ? sqrt(acc[k - 1]) / gn : 0.0;
    if (!isfinite(r)) {
      ctl[2] = 1;
      stop = true;
    } else if (r <= tol) {
      stop = true;
    }
  }
  if (stop) {
    ctl[1] = k;
    ctl[0] = 1;
  }
}

__global__ void k_gate_advance(int* ctl) {
  if (threadIdx.x == 0 && ctl[0] == 1) ctl[0] = 2;
}

hipError_t tol_check(int* ctl, const double* acc, int k, int kmax, double tol, double n3, hipStream_t st) {
  hipLaunchKernelGGL(k_tol_check, dim3(1), dim3(64), 0, st, ctl, acc, k, kmax, tol, n3);
  return hipGetLastError();
}

hipError_t gate_advance(int* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_gate_advance, dim3(1), dim3(64), 0, st, ctl);
  return hipGetLastError();
}

}  // namespace pm
