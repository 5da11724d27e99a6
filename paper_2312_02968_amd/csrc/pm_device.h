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

// The equations are evaluated with the hardware square root, reciprocal and
// reciprocal square root (about one ulp each), a fraction of the
// instructions of the correctly rounded library forms: the x passes that
// apply them are bound by their vector instructions.  Every value stays
// within a few ulp.  A squared magnitude below kTinySq (|F| below 1e-18 in
// the field's units) counts as zero, where the library forms would meet
// denormals; nu F there is below 1e-9 sqrt(a0).
constexpr float kTinySq = 1e-36f;
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// nu(y), y = |F| / a0, and its logarithmic slope s = y nu'(y) / nu(y), from
// m2 = |F|^2.  Standard: with z = 2 / y = 2 a0 / |F| and h = sqrt(1 + z^2),
// nu^2 = 1/2 + sqrt(1/4 + 1/y^2) = (1 + h) / 2 and
// s = -1 / (2 nu^2 y^2 sqrt(1/4 + 1/y^2)) = -z^2 / (2 h (1 + h)), evaluated
// as -(z / h) (z / (2 (1 + h))); beyond z = 1e18, h = z to FP32 precision.
// Deep MOND: nu = sqrt(a0 / |F|), s = -1/2.  Newton: nu = 1, s = 0.  Zero
// vector: nu = 0 (the caller multiplies F by nu), s = 0.
__device__ __forceinline__ float nu_of_sq(int mode, float m2, float a0, float* slope = nullptr) {
  if (mode == 2) {
    if (slope) *slope = 0.0f;
    return 1.0f;
  }
  if (!(m2 > kTinySq)) {
    if (slope) *slope = 0.0f;
    return 0.0f;
  }
  const float r = hw_rsq(m2);                        // 1 / |F|
  if (mode == 1) {
    if (slope) *slope = -0.5f;
    return hw_sqrt(a0 * r);
  }
  const float z = 2.0f * a0 * r;
  const float h = (z < 1e18f) ? hw_sqrt(fmaf(z, z, 1.0f)) : z;
  if (slope) *slope = -(z * hw_rcp(h)) * (z * hw_rcp(2.0f * (1.0f + h)));
  return hw_sqrt(0.5f * (1.0f + h));
}

// mu(x), x = |g_M| / a0, and its logarithmic slope x mu'(x) / mu(x), from
// m2 = |g_M|^2.  Standard: with q = x^2, mu = x / sqrt(1 + x^2) =
// sqrt(q / (1 + q)) and the slope 1 / (1 + q); beyond q = 1e30, mu = 1 and the
// slope 0 to FP32 precision.  Deep MOND: mu = x, slope 1.  Newton: 1, 0.
__device__ __forceinline__ float mu_of_sq(int mode, float m2, float inv_a0, float* slope = nullptr) {
  if (mode == 2) {
    if (slope) *slope = 0.0f;
    return 1.0f;
  }
  if (mode == 1) {
    if (slope) *slope = 1.0f;
    return hw_sqrt(m2) * inv_a0;
  }
  const float q = m2 * inv_a0 * inv_a0;
  if (!(q < 1e30f)) {
    if (slope) *slope = 0.0f;
    return 1.0f;
  }
  const float w = hw_rcp(1.0f + q);
  if (slope) *slope = w;
  return hw_sqrt(q * w);
}

// d <- the linearised map of Eq. inverse (MU = false: nu about A = F) or of
// Eq. interpolation (MU = true: mu about A = g_M) applied to d:
// f(|A|/a0) (d + s (A . d) / |A|^2 A) with s the logarithmic slope; zero
// where A = 0, where the maps have no derivative (Sect. 5, item (v)).
template <bool MU>
__device__ __forceinline__ void linearised(int mode, float a0, float inv_a0, float A0, float A1, float A2,
                                           float& d0, float& d1, float& d2) {
  const float am2 = A0 * A0 + A1 * A1 + A2 * A2;
  if (!(am2 > kTinySq)) {
    d0 = d1 = d2 = 0.0f;
    return;
  }
  float sl;
  const float f = MU ? mu_of_sq(mode, am2, inv_a0, &sl) : nu_of_sq(mode, am2, a0, &sl);
  const float c = sl * (A0 * d0 + A1 * d1 + A2 * d2) * hw_rcp(am2);
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
