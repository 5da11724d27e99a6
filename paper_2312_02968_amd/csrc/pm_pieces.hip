// Deposit (Eq. smooth) and smoothed-force gather (Eq. gi) by tile pieces,
// one particle per lane, for the kernel balls of radius 4 sigma with
// sigma = 1 cell (the paper's 251 cells) and sigma = 1.5 cells.
//
// Weights.  A particle at u = x / s has the central pixel c = floor(u + 1/2)
// and the sub-pixel offset f = c - u.  Its Gaussian weight on ball cell d is
// exp(-|d + f|^2 / (2 sigma^2)) = wx[dx] wy[dy] wz[dz], so a lane evaluates
// 3 (2 EXT + 1) exponentials and forms the products; the ball itself (which
// cells are in it) is fixed at compile time, so every cell's LDS address is
// the lane's base address plus an immediate.  The normalisation S = sum_B w is
// summed in FP64 row by row: for the row (dy, dz) of half-width h,
// wy[dy] wz[dz] sum_{|dx| <= h} wx[dx].
//
// Work split.  After the tile sort (8^3-cell tiles), each tile's particles are
// cut into pieces of at most kPiece; blocks take pieces from a work counter.
//  - Deposit: a piece accumulates its balls in an LDS copy of the tile plus a
//    halo of EXT cells, as exact 64-bit fixed-point sums at its tile's scale
//    (below), and stores the piece's halo box to a staging slot: as integers
//    if the tile has several pieces, else as FP32 (one rounding of the exact
//    sum).  A second kernel gives every tile near matter one owner block,
//    which sums each of the 27 neighbouring tiles' staged boxes exactly
//    (integers, at that neighbour's scale), converts the 27 sums and adds
//    them in a fixed order into rho.  No cell is written with global atomics and no rounding
//    depends on how a tile's particles fall into pieces, so the density does
//    not depend on the order in which the particles arrive (the sort ranks
//    them within a tile with atomics).  Pieces beyond the staging capacity
//    add their cells with FP32 global atomics.
//  - Gather: a piece loads its tile plus a halo of EXT + 1 cells of phi into
//    LDS once; each lane then sums its particle's ball with the central
//    difference folded into the weights, g = -(1/(2 s S)) sum_e phi(c + e) W(e)
//    with W_x(e) = w(e - e_x) - w(e + e_x) (w = 0 outside the ball), so every
//    cell of the dilated ball is read once; phi is taken relative to phi(c),
//    which the zero sum of W allows and which keeps the FP32 products small.
#include <type_traits>

#include "pm_device.h"
#include "pm_internal.h"

namespace pm {

namespace {
constexpr int kTile = 8;
constexpr int kNT = 256;
// Block sizes of the deposit's tile kernel and of the gather (a piece per
// block).  Pieces average about 70 particles on the isothermal sphere, so
// most of a block's lanes wait while the few with particles sum their balls;
// 128-thread gather blocks keep twice as many pieces in flight per CU (the
// gather 361 -> 320 us there), while the deposit's tile kernel, whose LDS
// tile bounds its blocks per CU, is faster with 256 (266 against 295 us).
#ifndef PM_DEPOSIT_NT
#define PM_DEPOSIT_NT 256
#endif
#ifndef PM_GATHER_NT
#define PM_GATHER_NT 128
#endif
constexpr int kDepNT = PM_DEPOSIT_NT, kGatNT = PM_GATHER_NT;

__device__ __forceinline__ int wrapi(int i, int N) { return i & (N - 1); }

constexpr bool in_ball(int x, int y, int z, int R2, int EXT) {
  return x >= -EXT && x <= EXT && y >= -EXT && y <= EXT && z >= -EXT && z <= EXT && x * x + y * y + z * z < R2;
}
// half-width of row (dy, dz) of the ball, -1 if the row is empty
constexpr int row_half(int dy, int dz, int R2, int EXT) {
  int h = -1;
  for (int x = 0; x <= EXT; ++x)
    if (in_ball(x, dy, dz, R2, EXT)) h = x;
  return h;
}

// Compile-time loops.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Per-lane particle state.
template <int EXT>
struct Lane {
  int cx, cy, cz;              // central pixel (wrapped grid index)
  float wx[2 * EXT + 1], wy[2 * EXT + 1], wz[2 * EXT + 1];
  double S;                    // FP64 ball sum of the weights
};

template <int EXT, int R2>
__device__ __forceinline__ void lane_setup(Lane<EXT>& L, const KernelGeom& kg, float px, float py, float pz,
                                           bool with_sum) {
  const double ux = (double)px * kg.inv_s, uy = (double)py * kg.inv_s, uz = (double)pz * kg.inv_s;
  const double cxd = floor(ux + 0.5), cyd = floor(uy + 0.5), czd = floor(uz + 0.5);
  const int half = kg.N / 2;
  L.cx = wrapi((int)cxd + half, kg.N);
  L.cy = wrapi((int)cyd + half, kg.N);
  L.cz = wrapi((int)czd + half, kg.N);
  const float fx = (float)(cxd - ux), fy = (float)(cyd - uy), fz = (float)(czd - uz);
#pragma unroll
  for (int d = -EXT; d <= EXT; ++d) {
    const float ex = (float)d + fx, ey = (float)d + fy, ez = (float)d + fz;
    L.wx[d + EXT] = expf(-ex * ex * kg.inv2sig2);
    L.wy[d + EXT] = expf(-ey * ey * kg.inv2sig2);
    L.wz[d + EXT] = expf(-ez * ez * kg.inv2sig2);
  }
  L.S = 0.0;
  if (!with_sum) return;
  double sx[EXT + 1];
  sx[0] = (double)L.wx[EXT];
#pragma unroll
  for (int h = 1; h <= EXT; ++h) sx[h] = sx[h - 1] + ((double)L.wx[EXT - h] + (double)L.wx[EXT + h]);
  double S = 0.0;
  static_for<-EXT, EXT + 1>([&](auto DZc) {
    constexpr int dz = decltype(DZc)::value;
    static_for<-EXT, EXT + 1>([&](auto DYc) {
      constexpr int dy = decltype(DYc)::value;
      constexpr int h = row_half(dy, dz, R2, EXT);
      if constexpr (h >= 0) S += (double)L.wy[dy + EXT] * (double)L.wz[dz + EXT] * sx[h];
    });
  });
  L.S = S;
}

// Blocks take pieces from a work counter (pieces differ in size by three
// orders of magnitude); the tile of a piece is one load from the map.
__device__ __forceinline__ int next_piece(int* counter, int* slot) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  return *slot;
}

// ---------------------------------------------------------------------------
// deposit
// ---------------------------------------------------------------------------
// Fixed-point cell sums.  LDS adds of 64-bit integers are native and an
// order of magnitude faster than LDS adds of FP32 on this chip (those take a
// slow path), and integer sums are exact, so a piece accumulates its balls as
// integers: each contribution c (FP32) becomes round(c 2^k) with one
// power-of-two scale per tile, shared by the tile's pieces, chosen so that
// no cell sum over all the tile's particles can overflow; the cell's FP32
// value is the integer sum times 2^-k.  The product of the three normalised
// 1D weights is at most 1, so every contribution of particle i is at most
// A_i = |m_i| / (S_i s^3) <= |m_i| / (w0 s^3), w0 being the smallest possible
// central-cell weight; a tile of n_t particles adds at most n_t contributions
// to a cell.  With A < 2^e for the tile's largest |m|, k = 61 - ceil(log2 n_t)
// - e keeps every sum below 2^61.
__device__ __forceinline__ int tile_scale_exp(const KernelGeom& kg, unsigned mbits, int count) {
  const double s3 = (double)kg.s * kg.s * kg.s;
  // the normalisation is at least the central cell's weight, whose offset is
  // at most 1/2 cell per axis (or the analytic prefactor)
  const double norm_lo = kg.analytic ? kg.analytic_norm : (double)expf(-0.75f * kg.inv2sig2);
  const double A = (double)__uint_as_float(mbits) / (norm_lo * s3);
  int e = 0;
  frexp(A > 0.0 ? A : 1.0, &e);                   // A < 2^e
  const int cb = count > 1 ? 32 - __clz(count - 1) : 0;      // ceil(log2 count)
  return 61 - cb - e;
}

// Largest |m| of each tile's particles, tmax[t] (float bits; zeroed before),
// from the pieces: a block reduces a piece and adds one atomic max per wave.
__global__ __launch_bounds__(kNT) void k_tile_mass_max(const int* __restrict__ perm, const int* __restrict__ offsets,
                                                      const int* __restrict__ pc_off, const int* __restrict__ ptile,
                                                      int ntiles, int piece, const float* __restrict__ mass,
                                                      unsigned* tmax) {
  const int total = pc_off[ntiles];
  for (int p = blockIdx.x; p < total; p += gridDim.x) {
    const int t = ptile[p];
    const int a = offsets[t] + (p - pc_off[t]) * piece;
    const int b = min(a + piece, offsets[t + 1]);
    float m = 0.0f;
    for (int j = a + (int)threadIdx.x; j < b; j += kNT) m = fmaxf(m, fabsf(mass[perm[j]]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(&tmax[t], __float_as_uint(m));   // non-negative floats order as their bits
  }
}
__device__ __forceinline__ unsigned long long to_fixed(float c, int k) {
  const float t = ldexpf(fabsf(c), k);                  // < 2^61 by the choice of k
  const unsigned hi = (unsigned)(t * 2.3283064365386963e-10f);   // t / 2^32, truncated
  const unsigned lo = (unsigned)fmaf(-(float)hi, 4294967296.0f, t);
  const unsigned long long u = ((unsigned long long)hi << 32) | lo;
  return c < 0.0f ? (unsigned long long)(-(long long)u) : u;
}

template <int EXT, int R2>
__global__ __launch_bounds__(kDepNT) void k_deposit_pieces(KernelGeom kg, const int* __restrict__ perm,
                                                        const int* __restrict__ offsets,
                                                        const int* __restrict__ pc_off,
                                                        const int* __restrict__ ptile, int ntiles, int piece,
                                                        int* counter, const float* __restrict__ pos,
                                                        const float* __restrict__ mass,
                                                        const unsigned* __restrict__ tmax, long long* stage, int cap,
                                                        float* rho) {
  constexpr int TE = kTile + 2 * EXT;
  constexpr int TE3 = TE * TE * TE;
  extern __shared__ unsigned long long tile64[];   // TE^3 fixed-point cell sums
  const int N = kg.N, nt = N / kTile;
  const double s3 = (double)kg.s * kg.s * kg.s;
  const int total = pc_off[ntiles];
  __shared__ int slot;
  for (int p = next_piece(counter, &slot); p < total; p = next_piece(counter, &slot)) {
    const int t = ptile[p];
    const int a = offsets[t] + (p - pc_off[t]) * piece;
    const int b = min(a + piece, offsets[t + 1]);
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - EXT, oy = ty * kTile - EXT, oz = tz * kTile - EXT;
    const bool staged = p < cap;
    int k = 0;
    if (staged) {
      for (int j = threadIdx.x; j < TE3; j += kDepNT) tile64[j] = 0ull;
      __syncthreads();
      k = tile_scale_exp(kg, tmax[t], offsets[t + 1] - offsets[t]);
    }
    for (int j = a + (int)threadIdx.x; j < b; j += kDepNT) {
      const int64_t i = perm[j];
      Lane<EXT> L;
      lane_setup<EXT, R2>(L, kg, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], !kg.analytic);
      const double norm = kg.analytic ? kg.analytic_norm : L.S;
      const float scale = (float)((double)mass[i] / (norm * s3));
      if (staged) {
        // the ball's corner cell in the tile; every cell is an immediate offset
        const int lx = wrapi(L.cx - ox, N), ly = wrapi(L.cy - oy, N), lz = wrapi(L.cz - oz, N);
        unsigned long long* base = tile64 + ((lz - EXT) * TE + (ly - EXT)) * TE + (lx - EXT);
        static_for<-EXT, EXT + 1>([&](auto DZc) {
          constexpr int dz = decltype(DZc)::value;
          static_for<-EXT, EXT + 1>([&](auto DYc) {
            constexpr int dy = decltype(DYc)::value;
            constexpr int h = row_half(dy, dz, R2, EXT);
            if constexpr (h >= 0) {
              const float ayz = scale * L.wy[dy + EXT] * L.wz[dz + EXT];
              static_for<-h, h + 1>([&](auto DXc) {
                constexpr int dx = decltype(DXc)::value;
                constexpr int off = ((dz + EXT) * TE + (dy + EXT)) * TE + (dx + EXT);
                __hip_atomic_fetch_add(base + off, to_fixed(ayz * L.wx[dx + EXT], k), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
              });
            }
          });
        });
      } else {
        static_for<-EXT, EXT + 1>([&](auto DZc) {
          constexpr int dz = decltype(DZc)::value;
          static_for<-EXT, EXT + 1>([&](auto DYc) {
            constexpr int dy = decltype(DYc)::value;
            constexpr int h = row_half(dy, dz, R2, EXT);
            if constexpr (h >= 0) {
              const float ayz = scale * L.wy[dy + EXT] * L.wz[dz + EXT];
              const long long r = ((long long)wrapi(L.cz + dz, N) * N + wrapi(L.cy + dy, N)) * N;
              static_for<-h, h + 1>([&](auto DXc) {
                constexpr int dx = decltype(DXc)::value;
                unsafeAtomicAdd(&rho[r + wrapi(L.cx + dx, N)], ayz * L.wx[dx + EXT]);
              });
            }
          });
        });
      }
    }
    if (staged) {
      __syncthreads();
      // a tile of several pieces stages integers, summed exactly by the
      // reduction; a lone piece's box is already its tile's exact sum and is
      // staged as FP32 (the slot's first half), half the bytes
      if (pc_off[t + 1] - pc_off[t] > 1) {
        long long* dst = stage + (size_t)p * TE3;
        for (int j = threadIdx.x; j < TE3; j += kDepNT) dst[j] = (long long)tile64[j];
      } else {
        float* dst = reinterpret_cast<float*>(stage + (size_t)p * TE3);
        for (int j = threadIdx.x; j < TE3; j += kDepNT) dst[j] = (float)ldexp((double)(long long)tile64[j], -k);
      }
      __syncthreads();
    }
  }
}

// Tiles that may receive staged cells: those with a non-empty tile among their
// 27 neighbours (periodic).  flag[t] = 1 or 0.
__global__ __launch_bounds__(256) void k_mark_dest(const int* __restrict__ counts, int nt, int* flag) {
  const int ntiles = nt * nt * nt;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ntiles) return;
  const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
  int any = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int u = ((((tz + dz) + nt) % nt) * nt + ((ty + dy) + nt) % nt) * nt + ((tx + dx) + nt) % nt;
        any |= counts[u] > 0;
      }
  flag[t] = any;
}

__global__ __launch_bounds__(256) void k_compact(const int* __restrict__ flag, const int* __restrict__ off,
                                                 int n, int* list) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n && flag[t]) list[off[t]] = t;
}

// Each listed tile: rho += the staged halo boxes of the pieces of its 27
// neighbouring tiles, one cell per thread.  A neighbour's pieces are summed
// exactly as integers (a lone piece read with the others' at once, 27
// independent loads with those outside a neighbour's box predicated off; the
// pieces of a dense neighbour eight loads at a time), each neighbour's sum is
// converted at its tile's scale, and the 27 values are added in a fixed
// order.  The
// owners of the densest tiles set the kernel's length, so a block keeps as
// many of their loads in flight as it can.
#ifndef PM_RED_NT
#define PM_RED_NT 512
#endif
constexpr int kRedNT = PM_RED_NT;
#ifndef PM_RED_LOADS
#define PM_RED_LOADS 8
#endif
constexpr int kRedLoads = PM_RED_LOADS;       // loads in flight per dense neighbour
static_assert(512 % kRedNT == 0, "a reduce block covers the 512 cells of a tile");
template <int EXT>
__global__ __launch_bounds__(kRedNT) void k_deposit_reduce(KernelGeom kg, const int* __restrict__ list,
                                                           const int* __restrict__ nlist,
                                                           const int* __restrict__ offsets,
                                                           const int* __restrict__ pc_off,
                                                           const unsigned* __restrict__ tmax, int nt, int N,
                                                           const long long* __restrict__ stage, int cap, float* rho) {
  constexpr int TE = kTile + 2 * EXT;
  constexpr int TE3 = TE * TE * TE;
  __shared__ int sq0[27], sq1[27], sk[27], smulti[27];
  const int n = *nlist;
  for (int li = blockIdx.x; li < n; li += gridDim.x) {
    const int t = list[li];
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    __syncthreads();                                // the previous tile's piece ranges are done with
    if (threadIdx.x < 27) {
      const int nb = threadIdx.x;
      const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
      const int u = ((((tz + dz) + nt) % nt) * nt + ((ty + dy) + nt) % nt) * nt + ((tx + dx) + nt) % nt;
      sq0[nb] = pc_off[u];
      sq1[nb] = min(pc_off[u + 1], cap);
      sk[nb] = tile_scale_exp(kg, tmax[u], offsets[u + 1] - offsets[u]);
      smulti[nb] = pc_off[u + 1] - pc_off[u] > 1;   // staged as integers
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 512 / kRedNT; ++h) {
      const int cell = threadIdx.x + h * kRedNT;    // 512 cells of the tile
      const int cx = cell & 7, cy = (cell >> 3) & 7, cz = cell >> 6;
      float v[27];
      static_for<0, 27>([&](auto NBc) {
        constexpr int nb = decltype(NBc)::value;
        constexpr int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
        // this cell in the halo box of neighbour nb (origin at its corner minus EXT)
        const int lx = cx - dx * kTile + EXT, ly = cy - dy * kTile + EXT, lz = cz - dz * kTile + EXT;
        const bool in = lx >= 0 && lx < TE && ly >= 0 && ly < TE && lz >= 0 && lz < TE && sq0[nb] < sq1[nb] &&
                        !smulti[nb];
        v[nb] = in ? reinterpret_cast<const float*>(stage + (size_t)sq0[nb] * TE3)[(lz * TE + ly) * TE + lx] : 0.0f;
      });
      const long long g = ((long long)(tz * kTile + cz) * N + (ty * kTile + cy)) * N + (tx * kTile + cx);
      const float r0 = rho[g];
      // neighbours of one piece, from the loads above, in order; then those of
      // several pieces, whose integer boxes are summed here.  Which neighbours
      // have several pieces depends only on the tiles' particle counts, so the
      // order of the additions is fixed.
      float sum = 0.0f;
#pragma unroll
      for (int nb = 0; nb < 27; ++nb) sum += v[nb];
      for (int nb = 0; nb < 27; ++nb) {
        const int q1 = sq1[nb];
        int q = sq0[nb];
        if (!smulti[nb] || q >= q1) continue;
        const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
        const int lx = cx - dx * kTile + EXT, ly = cy - dy * kTile + EXT, lz = cz - dz * kTile + EXT;
        if (lx < 0 || lx >= TE || ly < 0 || ly >= TE || lz < 0 || lz >= TE) continue;
        // kRedLoads independent loads in flight; integer sums are exact in any order
        const long long* src = stage + (lz * TE + ly) * TE + lx;
        long long a[kRedLoads];
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i) a[i] = 0;
        for (; q + kRedLoads - 1 < q1; q += kRedLoads) {
#pragma unroll
          for (int i = 0; i < kRedLoads; ++i) a[i] += src[(size_t)(q + i) * TE3];
        }
        for (; q < q1; ++q) a[0] += src[(size_t)q * TE3];
        long long tot = 0;
#pragma unroll
        for (int i = 0; i < kRedLoads; ++i) tot += a[i];
        sum += (float)ldexp((double)tot, -sk[nb]);
      }
      if (sum != 0.0f) rho[g] = r0 + sum;
    }
  }
}

// ---------------------------------------------------------------------------
// gather + push
// ---------------------------------------------------------------------------
template <int EXT, int R2>
__global__ __launch_bounds__(kGatNT) void k_gather_pieces(KernelGeom kg, const int* __restrict__ perm,
                                                       const int* __restrict__ offsets,
                                                       const int* __restrict__ pc_off,
                                                       const int* __restrict__ ptile, int ntiles, int piece,
                                                       int* counter, const float* __restrict__ phi, float* pos,
                                                       float* vel, float* acc, float dt_kick, float dt_drift,
                                                       int mode) {
  constexpr int HE = EXT + 1;                      // ball plus the difference stencil
  constexpr int TE = kTile + 2 * HE;
  constexpr int RP = TE + 1, PP = RP * TE + 1;     // padded row and plane pitches
  extern __shared__ float tile[];
  const int N = kg.N, nt = N / kTile;
  const int total = pc_off[ntiles];
  __shared__ int slot;
  for (int p = next_piece(counter, &slot); p < total; p = next_piece(counter, &slot)) {
    const int t = ptile[p];
    const int a = offsets[t] + (p - pc_off[t]) * piece;
    const int b = min(a + piece, offsets[t + 1]);
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - HE, oy = ty * kTile - HE, oz = tz * kTile - HE;
    for (int j = threadIdx.x; j < TE * TE * TE; j += kGatNT) {
      const int lx = j % TE, ly = (j / TE) % TE, lz = j / (TE * TE);
      tile[lz * PP + ly * RP + lx] =
          phi[((long long)wrapi(oz + lz, N) * N + wrapi(oy + ly, N)) * N + wrapi(ox + lx, N)];
    }
    __syncthreads();
    for (int j = a + (int)threadIdx.x; j < b; j += kGatNT) {
      const int64_t i = perm[j];
      const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
      Lane<EXT> L;
      lane_setup<EXT, R2>(L, kg, x, y, z, !kg.analytic);
      const double norm = kg.analytic ? kg.analytic_norm : L.S;
      const int lx = wrapi(L.cx - ox, N), ly = wrapi(L.cy - oy, N), lz = wrapi(L.cz - oz, N);
      const float* base = tile + (lz - HE) * PP + (ly - HE) * RP + (lx - HE);
      // The folded weights sum to zero over the dilated ball, so phi can be
      // taken relative to its value at the central pixel: the products then
      // carry the small differences, not the potential's offset (in FP32 the
      // offset would cost up to a hundred times the rounding error).
      const float phc = base[HE * PP + HE * RP + HE];
      float gx = 0.f, gy = 0.f, gz = 0.f;
      static_for<-HE, HE + 1>([&](auto EZc) {
        constexpr int ez = decltype(EZc)::value;
        static_for<-HE, HE + 1>([&](auto EYc) {
          constexpr int ey = decltype(EYc)::value;
          static_for<-HE, HE + 1>([&](auto EXc) {
            constexpr int ex = decltype(EXc)::value;
            constexpr bool bxm = in_ball(ex - 1, ey, ez, R2, EXT), bxp = in_ball(ex + 1, ey, ez, R2, EXT);
            constexpr bool bym = in_ball(ex, ey - 1, ez, R2, EXT), byp = in_ball(ex, ey + 1, ez, R2, EXT);
            constexpr bool bzm = in_ball(ex, ey, ez - 1, R2, EXT), bzp = in_ball(ex, ey, ez + 1, R2, EXT);
            if constexpr (bxm || bxp || bym || byp || bzm || bzp) {
              constexpr int off = (ez + HE) * PP + (ey + HE) * RP + (ex + HE);
              const float v = base[off] - phc;
              // W_x(e) = w(e - e_x) - w(e + e_x), and likewise for y and z
              if constexpr (bxm || bxp) {
                float wdx = 0.f;
                if constexpr (bxm) wdx += L.wx[ex - 1 + EXT];
                if constexpr (bxp) wdx -= L.wx[ex + 1 + EXT];
                gx = fmaf(v * wdx, L.wy[ey + EXT] * L.wz[ez + EXT], gx);
              }
              if constexpr (bym || byp) {
                float wdy = 0.f;
                if constexpr (bym) wdy += L.wy[ey - 1 + EXT];
                if constexpr (byp) wdy -= L.wy[ey + 1 + EXT];
                gy = fmaf(v * wdy, L.wx[ex + EXT] * L.wz[ez + EXT], gy);
              }
              if constexpr (bzm || bzp) {
                float wdz = 0.f;
                if constexpr (bzm) wdz += L.wz[ez - 1 + EXT];
                if constexpr (bzp) wdz -= L.wz[ez + 1 + EXT];
                gz = fmaf(v * wdz, L.wx[ex + EXT] * L.wy[ey + EXT], gz);
              }
            }
          });
        });
      });
      // sum_e phi(c + e) W(e) = sum_d w(d) (phi(c + d + e_x) - phi(c + d - e_x)),
      // so the smoothed force is -1 / (2 s S) times it
      const float f = (float)(-1.0 / (2.0 * (double)kg.s * norm));
      const float ax = gx * f, ay = gy * f, az = gz * f;
      if (mode == 0) {
        acc[3 * i] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
      } else {
        const float vx = fmaf(ax, dt_kick, vel[3 * i]);
        const float vy = fmaf(ay, dt_kick, vel[3 * i + 1]);
        const float vz = fmaf(az, dt_kick, vel[3 * i + 2]);
        vel[3 * i] = vx; vel[3 * i + 1] = vy; vel[3 * i + 2] = vz;
        pos[3 * i] = fmaf(vx, dt_drift, x);
        pos[3 * i + 1] = fmaf(vy, dt_drift, y);
        pos[3 * i + 2] = fmaf(vz, dt_drift, z);
      }
    }
    __syncthreads();
  }
}

// The tile of every piece: ptile[q] = t for pc_off[t] <= q < pc_off[t + 1].
__global__ __launch_bounds__(256) void k_piece_tiles(const int* __restrict__ pc_off, int n, int* ptile) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  for (int q = pc_off[t]; q < pc_off[t + 1]; ++q) ptile[q] = t;
}

// Pieces per tile: ceil(count / piece).
__global__ __launch_bounds__(256) void k_piece_counts(const int* __restrict__ counts, int n, int piece,
                                                      int* pieces) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n) pieces[t] = (counts[t] + piece - 1) / piece;
}

// Grid sizes of the persistent kernels.
constexpr int kPersistBlocks = 2048;
}  // namespace

template <int EXT>
static constexpr size_t deposit_lds() {
  return sizeof(unsigned long long) * (size_t)(kTile + 2 * EXT) * (kTile + 2 * EXT) * (kTile + 2 * EXT);
}
template <int EXT>
static constexpr size_t gather_lds() {
  constexpr int TE = kTile + 2 * (EXT + 1);
  return sizeof(float) * (size_t)TE * ((TE + 1) * TE + 1);
}

size_t piece_stage_cells(int ext, int cap) {
  const size_t te = kTile + 2 * (size_t)ext;
  return (size_t)cap * te * te * te;
}

hipError_t piece_plan(const PieceBufs& pb, const SortBufs& sb, int N, hipStream_t st) {
  const int ntiles = sb.ntiles;
  // pieces per tile, their offsets, then the tiles that receive staged cells
  hipLaunchKernelGGL(k_piece_counts, dim3((ntiles + 255) / 256), dim3(256), 0, st, sb.counts, ntiles, kPiece,
                     pb.flag);
  hipError_t e = scan_exclusive(pb.flag, ntiles, pb.pc_off, sb.blocksums, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_piece_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, st, pb.pc_off, ntiles, pb.ptile);
  const int nt = N / kTile;
  hipLaunchKernelGGL(k_mark_dest, dim3((ntiles + 255) / 256), dim3(256), 0, st, sb.counts, nt, pb.flag);
  if ((e = scan_exclusive(pb.flag, ntiles, pb.list_off, sb.blocksums, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact, dim3((ntiles + 255) / 256), dim3(256), 0, st, pb.flag, pb.list_off, ntiles,
                     pb.list);
  return hipGetLastError();
}

hipError_t deposit_pieces(const KernelGeom& kg, const SortBufs& sb, const PieceBufs& pb, const float* pos,
                          const float* mass, int64_t n, float* rho, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipError_t e = fill_zero(reinterpret_cast<float*>(pb.counter), 1, st);
  if (e != hipSuccess) return e;
  const int nt = kg.N / kTile;
  // the tiles' fixed-point scales: their largest |m|
  if ((e = fill_zero(reinterpret_cast<float*>(pb.tmax), sb.ntiles, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_mass_max, dim3(kPersistBlocks), dim3(kNT), 0, st, sb.perm, sb.offsets, pb.pc_off, pb.ptile,
                     sb.ntiles, kPiece, mass, pb.tmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  switch (kg.piece_ext) {
    case 3:
      hipLaunchKernelGGL((k_deposit_pieces<3, 16>), dim3(kPersistBlocks), dim3(kDepNT), deposit_lds<3>(), st, kg,
                         sb.perm, sb.offsets, pb.pc_off, pb.ptile, sb.ntiles, kPiece, pb.counter, pos, mass, pb.tmax,
                         pb.stage, pb.cap, rho);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL((k_deposit_reduce<3>), dim3(kPersistBlocks), dim3(kRedNT), 0, st, kg, pb.list,
                         pb.list_off + sb.ntiles, sb.offsets, pb.pc_off, pb.tmax, nt, kg.N, pb.stage, pb.cap,
                         rho);
      break;
    case 5:
      hipLaunchKernelGGL((k_deposit_pieces<5, 36>), dim3(kPersistBlocks), dim3(kDepNT), deposit_lds<5>(), st, kg,
                         sb.perm, sb.offsets, pb.pc_off, pb.ptile, sb.ntiles, kPiece, pb.counter, pos, mass, pb.tmax,
                         pb.stage, pb.cap, rho);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL((k_deposit_reduce<5>), dim3(kPersistBlocks), dim3(kRedNT), 0, st, kg, pb.list,
                         pb.list_off + sb.ntiles, sb.offsets, pb.pc_off, pb.tmax, nt, kg.N, pb.stage, pb.cap,
                         rho);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t gather_pieces(const KernelGeom& kg, const SortBufs& sb, const PieceBufs& pb, const float* phi,
                         float* pos, float* vel, float* acc, int64_t n, float dt_kick, float dt_drift, int mode,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipError_t e = fill_zero(reinterpret_cast<float*>(pb.counter + 1), 1, st);
  if (e != hipSuccess) return e;
  switch (kg.piece_ext) {
    case 3:
      hipLaunchKernelGGL((k_gather_pieces<3, 16>), dim3(kPersistBlocks), dim3(kGatNT), gather_lds<3>(), st, kg,
                         sb.perm, sb.offsets, pb.pc_off, pb.ptile, sb.ntiles, kPiece, pb.counter + 1, phi, pos, vel, acc,
                         dt_kick, dt_drift, mode);
      break;
    case 5:
      hipLaunchKernelGGL((k_gather_pieces<5, 36>), dim3(kPersistBlocks), dim3(kGatNT), gather_lds<5>(), st, kg,
                         sb.perm, sb.offsets, pb.pc_off, pb.ptile, sb.ntiles, kPiece, pb.counter + 1, phi, pos, vel, acc,
                         dt_kick, dt_drift, mode);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pm
