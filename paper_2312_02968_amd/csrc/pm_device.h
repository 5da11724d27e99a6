// Device building blocks shared by the HIP kernels of the PM step:
// complex arithmetic, small DFTs in registers, one Stockham stage over a
// block's sequences held in LDS, and the interpolation pair mu / nu.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos and sin of 2 pi q / 16, q = 0..7
__device__ __constant__ static const float kC16[8] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__device__ __constant__ static const float kS16[8] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// exp(-+ 2 pi i q / R) for R in {2, 4, 8, 16}: forward uses the minus sign.
template <int R, bool INV>
__device__ __forceinline__ float2 unit_root(int q) {
  const int t = q * (16 / R);
  const float c = (t < 8) ? kC16[t] : -kC16[t - 8];
  const float s = (t < 8) ? kS16[t] : -kS16[t - 8];
  return make_float2(c, INV ? s : -s);
}

// In-register DFT of length R (power of two <= 16), radix-2 decimation in
// time by recursion on even and odd samples.  X[q] = sum_r a[r] w^{rq} with
// w = exp(-2 pi i / R) (forward) or exp(+2 pi i / R) (inverse); unnormalised.
template <int R, bool INV>
struct Dft {
  __device__ __forceinline__ static void run(float2* a) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) { e[r] = a[2 * r]; o[r] = a[2 * r + 1]; }
    Dft<R / 2, INV>::run(e);
    Dft<R / 2, INV>::run(o);
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      float2 t = (q == 0) ? o[q] : cmul(o[q], unit_root<R, INV>(q));
      a[q] = cadd(e[q], t);
      a[q + R / 2] = csub(e[q], t);
    }
  }
};
template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};
template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};
template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* a) {
    float2 s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
    float2 s1 = cadd(a[1], a[3]), d1 = mul_mi<INV>(csub(a[1], a[3]));
    a[0] = cadd(s0, s1);
    a[2] = csub(s0, s1);
    a[1] = cadd(d0, d1);
    a[3] = csub(d0, d1);
  }
};

// Radix plan of a length-L transform: radix of stage st (0-based).
template <int L>
struct Plan;
template <> struct Plan<2>    { static constexpr int S = 1; static constexpr int r[1] = {2}; };
template <> struct Plan<4>    { static constexpr int S = 1; static constexpr int r[1] = {4}; };
template <> struct Plan<8>    { static constexpr int S = 1; static constexpr int r[1] = {8}; };
template <> struct Plan<16>   { static constexpr int S = 1; static constexpr int r[1] = {16}; };
template <> struct Plan<32>   { static constexpr int S = 2; static constexpr int r[2] = {8, 4}; };
template <> struct Plan<64>   { static constexpr int S = 2; static constexpr int r[2] = {8, 8}; };
template <> struct Plan<128>  { static constexpr int S = 2; static constexpr int r[2] = {16, 8}; };
template <> struct Plan<256>  { static constexpr int S = 2; static constexpr int r[2] = {16, 16}; };
template <> struct Plan<512>  { static constexpr int S = 3; static constexpr int r[3] = {8, 8, 8}; };
template <> struct Plan<1024> { static constexpr int S = 3; static constexpr int r[3] = {16, 8, 8}; };

// Layout of a block's S sequences of length L in LDS: element i of sequence
// q lives at buf[q * QS + i * IS].  SEQ_FAST selects the thread mapping:
// consecutive threads take consecutive sequences (IS large, QS = 1) or
// consecutive elements (QS large, IS = 1), so LDS accesses stay contiguous.
//
// One Stockham radix-R stage (Ns = product of the radices already applied):
// butterfly j of a sequence reads x[j + r L/R], multiplies by the twiddle
// w_{Ns R}^{r (j mod Ns)}, takes a length-R DFT and writes
// y[(j div Ns) Ns R + (j mod Ns) + q' Ns].  The stage is done in place: all
// inputs are read into registers before a barrier, outputs are written
// after it.  tw holds exp(-2 pi i t / TWN) for t < TWN; TWN is a multiple of L.
template <int L, int R, int S, int NT, bool SEQ_FAST, bool INV>
__device__ __forceinline__ void stockham_stage(float2* buf, int QS, int IS, int Ns,
                                               const float2* __restrict__ tw, int twmul) {
  constexpr int NB = S * (L / R);
  constexpr int BPT = (NB + NT - 1) / NT;
  float2 v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int q = SEQ_FAST ? (b % S) : (b / (L / R));
      const int j = SEQ_FAST ? (b / S) : (b % (L / R));
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = buf[q * QS + (j + r * (L / R)) * IS];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    if ((NB % NT) == 0 || b < NB) {
      const int q = SEQ_FAST ? (b % S) : (b / (L / R));
      const int j = SEQ_FAST ? (b / S) : (b % (L / R));
      const int k = j % Ns;
      if (Ns > 1) {
        const int step = (L / (Ns * R)) * twmul;   // twiddle index unit
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * step];
          if (INV) w.y = -w.y;
          v[u][r] = cmul(v[u][r], w);
        }
      }
      Dft<R, INV>::run(v[u]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[q * QS + (base + r * Ns) * IS] = v[u][r];
    }
  }
  __syncthreads();
}

template <int L, int S, int NT, bool SEQ_FAST, bool INV, int ST>
struct FftStages {
  __device__ __forceinline__ static void run(float2* buf, int QS, int IS, int Ns,
                                             const float2* __restrict__ tw, int twmul) {
    constexpr int R = Plan<L>::r[Plan<L>::S - ST];
    stockham_stage<L, R, S, NT, SEQ_FAST, INV>(buf, QS, IS, Ns, tw, twmul);
    FftStages<L, S, NT, SEQ_FAST, INV, ST - 1>::run(buf, QS, IS, Ns * R, tw, twmul);
  }
};
template <int L, int S, int NT, bool SEQ_FAST, bool INV>
struct FftStages<L, S, NT, SEQ_FAST, INV, 0> {
  __device__ __forceinline__ static void run(float2*, int, int, int, const float2* __restrict__, int) {}
};

// Unnormalised length-L complex FFT of the block's S sequences in LDS, in
// place, natural order in and out.  Ends with a barrier.
template <int L, int S, int NT, bool SEQ_FAST, bool INV>
__device__ __forceinline__ void block_fft(float2* buf, int QS, int IS, const float2* __restrict__ tw,
                                          int twmul) {
  FftStages<L, S, NT, SEQ_FAST, INV, Plan<L>::S>::run(buf, QS, IS, 1, tw, twmul);
}

// ---------------------------------------------------------------------------
// The algebraic equations of the AQUAL system (Eqs. inverse, interpolation).
// mode: 0 standard mu(x) = x / sqrt(1 + x^2), 1 deep MOND mu(x) = x, 2 Newton.
// ---------------------------------------------------------------------------

// Ratio |g_M| / |F| = nu(y) with y = |F| / a0; zero vector -> 0 (caller
// multiplies F by the ratio).  Standard: nu(y) = sqrt(1/2 + 1/2 sqrt(1 + 4/y^2))
// for y >= 1 and the equal form sqrt((y + sqrt(y^2 + 4)) / (2 y)) below 1, so
// that neither 4/y^2 nor y^2 overflows.
__device__ __forceinline__ float nu_ratio(int mode, float Fm, float inv_a0) {
  if (mode == 2) return 1.0f;
  if (!(Fm > 0.0f)) return 0.0f;
  const float y = Fm * inv_a0;
  if (mode == 1) return rsqrtf(y);
  if (y >= 1.0f) {
    const float t = 1.0f / y;
    return sqrtf(0.5f * (1.0f + sqrtf(fmaf(4.0f * t, t, 1.0f))));
  }
  return sqrtf((y + sqrtf(fmaf(y, y, 4.0f))) / (2.0f * y));
}

// Ratio |F| / |g_M| = mu(x) with x = |g_M| / a0.
__device__ __forceinline__ float mu_ratio(int mode, float gm, float inv_a0) {
  if (mode == 2) return 1.0f;
  const float x = gm * inv_a0;
  if (mode == 1) return x;
  if (x >= 1.0f) {
    const float t = 1.0f / x;
    return rsqrtf(fmaf(t, t, 1.0f));
  }
  return x * rsqrtf(fmaf(x, x, 1.0f));
}

// Logarithmic slopes y nu'(y) / nu(y) and x mu'(x) / mu(x) of the same
// functions, for the linearisations of Eqs. inverse and interpolation about
// a field A (Sect. 5, item (v)):  f(|A|/a0) (dA + s (A . dA) / |A|^2 A).
// Standard nu: s = -1 / (2 nu^2 y^2 sqrt(1/4 + 1/y^2)), written for y >= 1
// as -t^2 / (nu^2 sqrt(1 + 4 t^2)), t = 1/y, with nu^2 = (1 + sqrt(1 + 4
// t^2)) / 2, and for y < 1 as -1 / ((y + sqrt(y^2 + 4)) sqrt(1 + y^2/4));
// deep MOND -1/2; Newton 0.  Standard mu: 1 / (1 + x^2); deep MOND 1;
// Newton 0.
__device__ __forceinline__ float nu_logslope(int mode, float y) {
  if (mode == 2) return 0.0f;
  if (mode == 1) return -0.5f;
  if (y >= 1.0f) {
    const float t = 1.0f / y;
    const float q = sqrtf(fmaf(4.0f * t, t, 1.0f));
    return -(t * t) / (0.5f * (1.0f + q) * q);
  }
  return -1.0f / ((y + sqrtf(fmaf(y, y, 4.0f))) * sqrtf(fmaf(0.25f * y, y, 1.0f)));
}

__device__ __forceinline__ float mu_logslope(int mode, float x) {
  if (mode == 2) return 0.0f;
  if (mode == 1) return 1.0f;
  return 1.0f / fmaf(x, x, 1.0f);
}

// d <- the linearised map of Eq. inverse (MU = false: nu about A = F) or of
// Eq. interpolation (MU = true: mu about A = g_M) applied to d; zero where
// A = 0, where the maps have no derivative.
template <bool MU>
__device__ __forceinline__ void linearised(int mode, float inv_a0, float A0, float A1, float A2, float& d0,
                                           float& d1, float& d2) {
  const float am2 = A0 * A0 + A1 * A1 + A2 * A2;
  if (!(am2 > 0.0f)) {
    d0 = d1 = d2 = 0.0f;
    return;
  }
  const float am = sqrtf(am2);
  const float f = MU ? mu_ratio(mode, am, inv_a0) : nu_ratio(mode, am, inv_a0);
  const float sl = MU ? mu_logslope(mode, am * inv_a0) : nu_logslope(mode, am * inv_a0);
  const float c = sl * (A0 * d0 + A1 * d1 + A2 * d2) / am2;
  d0 = f * fmaf(c, A0, d0);
  d1 = f * fmaf(c, A1, d1);
  d2 = f * fmaf(c, A2, d2);
}

}  // namespace pm

namespace pm {

// ---------------------------------------------------------------------------
// Column FFT engine with register staging.
//
// S sequences ("columns") of length L are spread over NT threads.  In stage
// st (radix R, Ns = product of the earlier radices) butterfly b of a thread
// is (q = b mod S, j = b div S); it consumes elements j + r L/R and produces
// elements (j - j mod Ns) R + j mod Ns + r Ns.  The first stage's inputs come
// from a loader (global memory) and the last stage's outputs go to the caller
// in registers: the last stage has j < Ns, so it produces elements
// j + r L/R -- exactly the inputs of the first stage of a transform run with
// the reversed radix plan.  Only the hand-overs between stages go through LDS
// (one buffer of S L complex, element i of column q at i * (S + 1) + q), one
// component at a time.
// ---------------------------------------------------------------------------
template <int L, bool REV, int ST>
struct PlanAt {
  static constexpr int R = REV ? Plan<L>::r[Plan<L>::S - 1 - ST] : Plan<L>::r[ST];
  static constexpr int Ns = PlanAt<L, REV, ST - 1>::Ns * PlanAt<L, REV, ST - 1>::R;
};
template <int L, bool REV>
struct PlanAt<L, REV, 0> {
  static constexpr int R = REV ? Plan<L>::r[Plan<L>::S - 1] : Plan<L>::r[0];
  static constexpr int Ns = 1;
};

// LDS address of element i of column q in the exchange buffer.  For 8-column
// tiles the rows are 16 dwords and a padding row follows every 8 rows, so the
// row sets a stage touches together (8 apart on the write side of the first
// stage, consecutive elsewhere) fall on different bank quarters; wider tiles
// pad each row by one element.
#ifndef PM_ZSKEW
#define PM_ZSKEW 0
#endif
template <int S>
__device__ __forceinline__ int col_addr(int i, int q) {
  if constexpr (S == 8 && PM_ZSKEW) return (i + (i >> 3)) * 8 + q;
  else return i * (S + 1) + q;
}
template <int L, int S>
struct ColBuf {
  static constexpr int elems = (S == 8 && PM_ZSKEW) ? (L + L / 8) * 8 : L * (S + 1);
};

// Register elements per thread: the largest BPT * R over the stages of the
// plan (when a stage has fewer butterflies than threads, a thread still holds
// one whole butterfly).
template <int L, int S, int NT>
struct ColCfg {
  static constexpr int bpr(int R) { return ((S * (L / R) + NT - 1) / NT) * R; }
  static constexpr int emax() {
    int e = 0;
    for (int st = 0; st < Plan<L>::S; ++st) e = bpr(Plan<L>::r[st]) > e ? bpr(Plan<L>::r[st]) : e;
    return e;
  }
  static constexpr int E = emax();
  static constexpr int IS = S + 1;
};

// Number of butterflies per thread and validity for stage parameters.
template <int L, int S, int NT, int R>
struct Bfly {
  static constexpr int NB = S * (L / R);
  static constexpr int BPT = (NB + NT - 1) / NT;
  __device__ __forceinline__ static bool valid(int b) { return (NB % NT) == 0 || b < NB; }
};

// Twiddle and DFT of the butterflies held in v (stage with radix R at Ns).
template <int L, int S, int NT, int R, int Ns, bool INV>
__device__ __forceinline__ void reg_butterflies(float2* v, const float2* tw_lds, int twmul) {
  using B = Bfly<L, S, NT, R>;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    float2* a = v + u * R;
    if (Ns > 1) {
      const int j = b / S;
      const int k = j % Ns;
      const int step = (L / (Ns * R)) * twmul;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw_lds[r * k * step];
        if (INV) w.y = -w.y;
        a[r] = cmul(a[r], w);
      }
    }
    Dft<R, INV>::run(a);
  }
}

// Write the outputs of stage (R, Ns) held in v to LDS.
template <int L, int S, int NT, int R, int Ns>
__device__ __forceinline__ void reg_to_lds(const float2* v, float2* buf) {
  using B = Bfly<L, S, NT, R>;
  constexpr int IS = S + 1;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % S, j = b / S, k = j % Ns;
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[col_addr<S>(base + r * Ns, q)] = v[u * R + r];
  }
}

// Read the inputs of a stage with radix R from LDS into v.
template <int L, int S, int NT, int R>
__device__ __forceinline__ void lds_to_reg(float2* v, const float2* buf) {
  using B = Bfly<L, S, NT, R>;
  constexpr int IS = S + 1;
#pragma unroll
  for (int u = 0; u < B::BPT; ++u) {
    const int b = threadIdx.x + u * NT;
    if (!B::valid(b)) continue;
    const int q = b % S, j = b / S;
#pragma unroll
    for (int r = 0; r < R; ++r) v[u * R + r] = buf[col_addr<S>(j + r * (L / R), q)];
  }
}

// Remaining stages ST..end for NC components held in v[c * E ...]; the caller
// has already run stage ST-1's butterflies.  Ends with the last stage's
// butterflies done (outputs in registers).
template <int L, int S, int NT, int NC, bool INV, bool REV, int ST, bool DONE = (ST >= Plan<L>::S)>
struct ColStagesSel;
template <int L, int S, int NT, int NC, bool INV, bool REV, int ST>
struct ColStagesSel<L, S, NT, NC, INV, REV, ST, true> {
  __device__ __forceinline__ static void run(float2*, float2*, const float2*, int) {}
};
template <int L, int S, int NT, int NC, bool INV, bool REV, int ST>
struct ColStagesSel<L, S, NT, NC, INV, REV, ST, false> {
  __device__ __forceinline__ static void run(float2* v, float2* buf, const float2* tw, int twmul) {
    constexpr int E = ColCfg<L, S, NT>::E;
    using Prev = PlanAt<L, REV, ST - 1>;
    using Cur = PlanAt<L, REV, ST>;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      reg_to_lds<L, S, NT, Prev::R, Prev::Ns>(v + c * E, buf);
      __syncthreads();
      lds_to_reg<L, S, NT, Cur::R>(v + c * E, buf);
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) reg_butterflies<L, S, NT, Cur::R, Cur::Ns, INV>(v + c * E, tw, twmul);
    ColStagesSel<L, S, NT, NC, INV, REV, ST + 1>::run(v, buf, tw, twmul);
  }
};

// Full transform of NC components whose first-stage inputs are already in v
// (element j + r L/R0 of column q for butterfly (q, j)).  Outputs stay in v:
// element j + r L/R_last of column q for butterfly (q, j) of the last stage.
template <int L, int S, int NT, int NC, bool INV, bool REV>
__device__ __forceinline__ void col_fft(float2* v, float2* buf, const float2* tw, int twmul) {
  constexpr int E = ColCfg<L, S, NT>::E;
  using First = PlanAt<L, REV, 0>;
#pragma unroll
  for (int c = 0; c < NC; ++c) reg_butterflies<L, S, NT, First::R, 1, INV>(v + c * E, tw, twmul);
  ColStagesSel<L, S, NT, NC, INV, REV, 1>::run(v, buf, tw, twmul);
}

}  // namespace pm
