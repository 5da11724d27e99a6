// Particle-mesh coupling: tile sort, Gaussian deposit (Eq. smooth), smoothed
// force gather (Eq. gi) with the leapfrog kick and drift (Eq. motion), and
// FP64 diagnostics.
//
// Kernel weights.  A particle at x (in cells u = x / s) has the central pixel
// c = floor(u + 1/2) and the weights w_d = exp(-|c + d - u|^2 / (2 sigma^2))
// on the ball |d| < cutoff sigma.  The weight is separable: w_d = wx(dx)
// wy(dy) wz(dz), so a wave evaluates 3 (2 ext + 1) exponentials per particle,
// one per lane, and every lane builds the products of its ball cells with
// cross-lane reads.  The normalisation S = sum_B w_d is summed in FP64.
//
// Work split.  Particles are counting-sorted by the 8^3-cell tile of their
// central pixel.  A block takes a chunk of the sorted list and walks it tile
// segment by tile segment; a segment with enough particles accumulates its
// balls in an LDS copy of the tile plus a halo (deposit) or reads the
// potential from an LDS copy of the tile plus halo (gather); a sparse segment
// goes straight to global memory.  One wave handles one particle at a time
// with its lanes spread over the ball.
#include "pm_device.h"
#include "pm_internal.h"

namespace pm {

namespace {
constexpr int kTile = 8;
constexpr int kChunk = 512;
constexpr int kNT = 256;
constexpr int kWaves = kNT / 64;

__device__ __forceinline__ int wrapi(int i, int N) { return i & (N - 1); }

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-wave state of the particle being processed.
struct Part {
  int cx, cy, cz;      // central pixel, wrapped grid index
  float fx, fy, fz;    // central pixel minus the particle position (cells)
  double S;            // FP64 sum of the weights over the ball
};

__device__ __forceinline__ void unpack(int e, int& dx, int& dy, int& dz) {
  dx = (e & 255) - 16;
  dy = ((e >> 8) & 255) - 16;
  dz = ((e >> 16) & 255) - 16;
}

// Kernel weight of ball offset (dx, dy, dz): exp(-|c + d - x|^2 / (2 sigma^2))
// with c + d - x = d + f; every lane evaluates its own cell (no cross-lane
// traffic).
__device__ __forceinline__ float ball_weight(const KernelGeom& kg, const Part& p, int dx, int dy, int dz) {
  const float ex = (float)dx + p.fx, ey = (float)dy + p.fy, ez = (float)dz + p.fz;
  return expf(-(ex * ex + ey * ey + ez * ez) * kg.inv2sig2);
}

// Central pixel and sub-pixel offset of the particle at (px, py, pz), then S
// (all lanes take part; the coordinates are wave-uniform).
__device__ __forceinline__ Part particle_setup(const KernelGeom& kg, const int* __restrict__ ball_lds, float px,
                                               float py, float pz, int lane, bool with_sum = true) {
  Part p;
  const double ux = (double)px * kg.inv_s;
  const double uy = (double)py * kg.inv_s;
  const double uz = (double)pz * kg.inv_s;
  const double cxd = floor(ux + 0.5), cyd = floor(uy + 0.5), czd = floor(uz + 0.5);
  const int half = kg.N / 2;
  p.cx = wrapi((int)cxd + half, kg.N);
  p.cy = wrapi((int)cyd + half, kg.N);
  p.cz = wrapi((int)czd + half, kg.N);
  p.fx = (float)(cxd - ux);
  p.fy = (float)(cyd - uy);
  p.fz = (float)(czd - uz);
  p.S = 0.0;
  if (!with_sum || kg.analytic) return p;
  double acc = 0.0;
  const int nit = (kg.nball + 63) / 64;
  for (int it = 0; it < nit; ++it) {
    const int b = it * 64 + lane;
    if (b < kg.nball) {
      int dx, dy, dz;
      unpack(ball_lds[b], dx, dy, dz);
      acc += (double)ball_weight(kg, p, dx, dy, dz);
    }
  }
  p.S = wave_sum_d(acc);
  return p;
}

__device__ __forceinline__ Part particle_setup(const KernelGeom& kg, const int* __restrict__ ball_lds,
                                               const float* __restrict__ pos, int64_t i, int lane) {
  return particle_setup(kg, ball_lds, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], lane);
}

// Tile key of each particle and its rank among the particles of its tile.
// The ranks come from device-scope atomic counters, which clustered matter
// turns into long queues on a few addresses, so a wave first groups its lanes
// by key: one lane per distinct key adds the group size, and each lane takes
// the base plus the number of lower lanes in its group (any order within a
// tile is a valid rank order).
// order (nullable) is the previous sort's permutation of the same particles:
// particles move little between steps, so taking them in that order gives a
// wave few distinct tiles and few atomics.
__global__ __launch_bounds__(256) void k_keys(const float* __restrict__ pos, int64_t n, int N, int nphys,
                                              double inv_s, int ext, const int* __restrict__ order, int* keys,
                                              int* rank, int* counts, int* flags) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = j < n;
  const int64_t i = valid ? (order ? (int64_t)order[j] : j) : 0;
  const int lane = threadIdx.x & 63;
  const int half = N / 2;
  int key = -1;
  bool out = false;
  if (valid) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
      const int ci = (int)floor((double)pos[3 * i + a] * inv_s + 0.5) + half;
      out |= (ci - ext < half - nphys / 2) || (ci + ext > half + nphys / 2 - 1);
      c[a] = wrapi(ci, N);
    }
    const int nt = N / kTile;
    key = ((c[2] / kTile) * nt + c[1] / kTile) * nt + c[0] / kTile;
    keys[i] = key;
  }
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long todo = __ballot(valid);
  int my_rank = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lk = __shfl(key, leader, 64);
    const unsigned long long grp = __ballot(valid && key == lk);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[lk], __popcll(grp));
    base = __shfl(base, leader, 64);
    if (valid && key == lk) my_rank = base + __popcll(grp & below);
    todo &= ~grp;
  }
  if (valid) rank[i] = my_rank;
  const unsigned long long outs = __ballot(valid && out);
  if (outs && lane == __ffsll((long long)outs) - 1) atomicAdd(&flags[0], __popcll(outs));
}

// Exclusive scan of counts[0..n) into offsets[0..n]; blocks of 1024 entries.
__global__ __launch_bounds__(1024) void k_scan_local(const int* __restrict__ counts, int n, int* offsets,
                                                     int* blocksums) {
  __shared__ int s[1024];
  const int i = blockIdx.x * 1024 + threadIdx.x;
  const int v = (i < n) ? counts[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int t = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) offsets[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) blocksums[blockIdx.x] = s[1023];
}

// Exclusive scan of up to 4096 block sums in one block; total into *total.
__global__ __launch_bounds__(1024) void k_scan_top(int* blocksums, int nb, int* total) {
  __shared__ int s[1024];
  int loc[4];
  int sum = 0;
  for (int j = 0; j < 4; ++j) {
    const int i = threadIdx.x * 4 + j;
    loc[j] = (i < nb) ? blocksums[i] : 0;
    sum += loc[j];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int t = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int run = s[threadIdx.x] - sum;
  for (int j = 0; j < 4; ++j) {
    const int i = threadIdx.x * 4 + j;
    if (i < nb) blocksums[i] = run;
    run += loc[j];
  }
  if (threadIdx.x == 1023) *total = s[1023];
}

__global__ __launch_bounds__(1024) void k_scan_add(int* offsets, int n, const int* __restrict__ blocksums) {
  const int i = blockIdx.x * 1024 + threadIdx.x;
  if (i < n) offsets[i] += blocksums[blockIdx.x];
}

__global__ __launch_bounds__(256) void k_scatter(int64_t n, const int* __restrict__ keys,
                                                 const int* __restrict__ rank, const int* __restrict__ offsets,
                                                 int* perm, int* skey) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = keys[i];
  const int d = offsets[k] + rank[i];
  perm[d] = (int)i;
  skey[d] = k;
}

__global__ __launch_bounds__(256) void k_fill(float* p, long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// ---------------------------------------------------------------------------
// Chunk plan.  A block owns kChunk consecutive particles of the sorted order.
// Its particles fall into pieces (the part of a tile's segment inside the
// chunk).  A piece whose balls cover more cells than the tile plus halo is
// "dense" and goes through an LDS copy of the tile; the particles of the
// other pieces form one flat "sparse" list that the waves share without
// per-piece synchronisation.
// ---------------------------------------------------------------------------
struct ChunkPlan {
  int nsparse;
  int npieces;
  int sparse[kChunk];    // sorted-order indices of sparse particles
  int pstart[kChunk];    // dense pieces: [pstart, pend) of tile ptile
  int pend[kChunk];
  int ptile[kChunk];
};

__device__ __forceinline__ void plan_chunk(ChunkPlan& pl, const int* __restrict__ skey,
                                           const int* __restrict__ offsets, int64_t a0, int64_t a1,
                                           int64_t dense_min) {
  if (threadIdx.x == 0) { pl.nsparse = 0; pl.npieces = 0; }
  __syncthreads();
  for (int64_t j = a0 + threadIdx.x; j < a1; j += kNT) {
    const int t = skey[j];
    const int64_t ps = max((int64_t)offsets[t], a0), pe = min((int64_t)offsets[t + 1], a1);
    if (pe - ps < dense_min) {
      pl.sparse[atomicAdd(&pl.nsparse, 1)] = (int)j;
    } else if (j == ps) {
      const int k = atomicAdd(&pl.npieces, 1);
      pl.pstart[k] = (int)ps;
      pl.pend[k] = (int)pe;
      pl.ptile[k] = t;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// deposit
// ---------------------------------------------------------------------------
// Deposits particle (x, y, z, m) of the wave: into the LDS tile (origin o*,
// edge TE) when tile != nullptr, else straight into rho with global atomics.
// LDS selects the tile path at compile time, so the tile pointer is known to
// address LDS (ds_add_f32) rather than a generic address (flat atomics).
template <bool LDS>
__device__ __forceinline__ void deposit_one(const KernelGeom& kg, const int* __restrict__ ball, float x, float y,
                                            float z, float m, double s3, float* tile, int TE, int ox, int oy,
                                            int oz, float* rho, double* s_out, int lane) {
  const int N = kg.N;
  const Part p = particle_setup(kg, ball, x, y, z, lane);
  const double norm = kg.analytic ? kg.analytic_norm : p.S;
  if (s_out != nullptr && lane == 0) *s_out = norm;
  const float scale = (float)((double)m / (norm * s3));
  const int nit = (kg.nball + 63) / 64;
  for (int it = 0; it < nit; ++it) {
    const int b = it * 64 + lane;
    if (b < kg.nball) {
      int dx, dy, dz;
      unpack(ball[b], dx, dy, dz);
      const float v = ball_weight(kg, p, dx, dy, dz) * scale;
      if constexpr (LDS) {
        const int lx = p.cx + dx - ox, ly = p.cy + dy - oy, lz = p.cz + dz - oz;
        if (kg.private_tiles) {
          // the wave's own copy: its lanes hold distinct cells and its LDS
          // operations execute in order, so a plain read-add-write suffices
          tile[(lz * TE + ly) * TE + lx] += v;
        } else {
          atomicAdd(&tile[(lz * TE + ly) * TE + lx], v);
        }
      } else {
        const long long g = ((long long)wrapi(p.cz + dz, N) * N + wrapi(p.cy + dy, N)) * N + wrapi(p.cx + dx, N);
        unsafeAtomicAdd(&rho[g], v);
      }
    }
  }
}

__global__ __launch_bounds__(kNT) void k_deposit(KernelGeom kg, const int* __restrict__ perm,
                                                 const int* __restrict__ skey, const int* __restrict__ offsets,
                                                 const float* __restrict__ pos, const float* __restrict__ mass,
                                                 int64_t n, float* rho, double* s_store) {
  extern __shared__ float smem[];
  __shared__ ChunkPlan pl;
  int* ball = reinterpret_cast<int*>(smem);
  float* tile = smem + ((kg.nball + 3) & ~3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kg.nball; b += kNT) ball[b] = kg.ball[b];
  const int TE = kTile + 2 * kg.ext;
  const int TE3 = TE * TE * TE;
  const int ncopy = kg.private_tiles ? kWaves : 1;        // tile copies in LDS
  float* my_tile = tile + (kg.private_tiles ? wave * TE3 : 0);
  const int N = kg.N;
  const int nt = N / kTile;
  const double s3 = (double)kg.s * kg.s * kg.s;
  const int64_t a0 = (int64_t)blockIdx.x * kChunk;
  const int64_t a1 = min(a0 + (int64_t)kChunk, n);
  plan_chunk(pl, skey, offsets, a0, a1, (ncopy * TE3 + kg.nball - 1) / kg.nball);

  // sparse particles: 64 per wave fetched at once, broadcast one by one
  for (int jb = wave * 64; jb < pl.nsparse; jb += kWaves * 64) {
    const bool has = jb + lane < pl.nsparse;
    const int il = has ? perm[pl.sparse[jb + lane]] : 0;
    const int64_t i3 = 3 * (int64_t)il;
    const float xl = has ? pos[i3] : 0.f, yl = has ? pos[i3 + 1] : 0.f,
                zl = has ? pos[i3 + 2] : 0.f, ml = has ? mass[il] : 0.f;
    const int nb = min(64, pl.nsparse - jb);
    for (int t = 0; t < nb; ++t) {
      const int it_ = __shfl(il, t, 64);
      deposit_one<false>(kg, ball, __shfl(xl, t, 64), __shfl(yl, t, 64), __shfl(zl, t, 64), __shfl(ml, t, 64),
                         s3, nullptr, TE, 0, 0, 0, rho, s_store ? s_store + it_ : nullptr, lane);
    }
  }

  // dense pieces through the LDS tile
  for (int k = 0; k < pl.npieces; ++k) {
    const int t = pl.ptile[k];
    const int ps = pl.pstart[k], pe = pl.pend[k];
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - kg.ext, oy = ty * kTile - kg.ext, oz = tz * kTile - kg.ext;
    for (int j = threadIdx.x; j < ncopy * TE3; j += kNT) tile[j] = 0.0f;
    __syncthreads();
    for (int jb = ps + wave; jb < pe; jb += kWaves * 64) {
      const int jl = jb + kWaves * lane;
      const bool has = jl < pe;
      const int il = has ? perm[jl] : 0;
      const int64_t i3 = 3 * (int64_t)il;
      const float xl = has ? pos[i3] : 0.f, yl = has ? pos[i3 + 1] : 0.f,
                  zl = has ? pos[i3 + 2] : 0.f, ml = has ? mass[il] : 0.f;
      const int nb = min(64, (pe - jb + kWaves - 1) / kWaves);
      for (int u = 0; u < nb; ++u) {
        const int iu = __shfl(il, u, 64);
        deposit_one<true>(kg, ball, __shfl(xl, u, 64), __shfl(yl, u, 64), __shfl(zl, u, 64), __shfl(ml, u, 64),
                          s3, my_tile, TE, ox, oy, oz, rho, s_store ? s_store + iu : nullptr, lane);
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < TE3; j += kNT) {
      float v = tile[j];
      for (int c = 1; c < ncopy; ++c) v += tile[c * TE3 + j];
      if (v != 0.0f) {
        const int lx = j % TE, ly = (j / TE) % TE, lz = j / (TE * TE);
        const long long g = ((long long)wrapi(oz + lz, N) * N + wrapi(oy + ly, N)) * N + wrapi(ox + lx, N);
        unsafeAtomicAdd(&rho[g], v);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// gather + push
// ---------------------------------------------------------------------------
// Smoothed acceleration of the wave's particle at (x, y, z) from the LDS
// tile of phi (origin o*, row pitch RP, plane pitch PP) when LDS, else from
// phi.
template <bool LDS>
__device__ __forceinline__ float3 gather_one(const KernelGeom& kg, const int* __restrict__ ball, float x, float y,
                                             float z, const float* tile, int RP, int PP, int ox, int oy, int oz,
                                             const float* __restrict__ phi, double s_known, int lane) {
  const int N = kg.N;
  // with a stored normalisation (s_known > 0) the ball sum is not recomputed
  const Part p = particle_setup(kg, ball, x, y, z, lane, s_known <= 0.0);
  const double norm = s_known > 0.0 ? s_known : (kg.analytic ? kg.analytic_norm : p.S);
  float gx = 0.f, gy = 0.f, gz = 0.f;
  const int nit = (kg.nball + 63) / 64;
  for (int it = 0; it < nit; ++it) {
    const int b = it * 64 + lane;
    if (b < kg.nball) {
      int dx, dy, dz;
      unpack(ball[b], dx, dy, dz);
      const float w = ball_weight(kg, p, dx, dy, dz);
      float xp, xm, yp, ym, zp, zm;
      if constexpr (LDS) {
        const int lx = p.cx + dx - ox, ly = p.cy + dy - oy, lz = p.cz + dz - oz;
        const int c = lz * PP + ly * RP + lx;
        xp = tile[c + 1]; xm = tile[c - 1];
        yp = tile[c + RP]; ym = tile[c - RP];
        zp = tile[c + PP]; zm = tile[c - PP];
      } else {
        const int X = p.cx + dx, Y = p.cy + dy, Z = p.cz + dz;
        const long long zr = (long long)wrapi(Z, N) * N, zrp = (long long)wrapi(Z + 1, N) * N,
                        zrm = (long long)wrapi(Z - 1, N) * N;
        const int yw = wrapi(Y, N), xw = wrapi(X, N);
        xp = phi[(zr + yw) * N + wrapi(X + 1, N)];
        xm = phi[(zr + yw) * N + wrapi(X - 1, N)];
        yp = phi[(zr + wrapi(Y + 1, N)) * N + xw];
        ym = phi[(zr + wrapi(Y - 1, N)) * N + xw];
        zp = phi[(zrp + yw) * N + xw];
        zm = phi[(zrm + yw) * N + xw];
      }
      gx = fmaf(w, xp - xm, gx);
      gy = fmaf(w, yp - ym, gy);
      gz = fmaf(w, zp - zm, gz);
    }
  }
  const float f = (float)(-1.0 / (2.0 * (double)kg.s * norm));
  return make_float3(wave_sum_f(gx) * f, wave_sum_f(gy) * f, wave_sum_f(gz) * f);
}

// Writes the result of lane's particle il (acceleration, or kick + drift).
__device__ __forceinline__ void gather_store(int64_t il, float3 g, float x, float y, float z, float* pos, float* vel,
                                             float* acc, float dt_kick, float dt_drift, int mode) {
  if (mode == 0) {
    acc[3 * il] = g.x;
    acc[3 * il + 1] = g.y;
    acc[3 * il + 2] = g.z;
  } else {
    const float vx = fmaf(g.x, dt_kick, vel[3 * il]);
    const float vy = fmaf(g.y, dt_kick, vel[3 * il + 1]);
    const float vz = fmaf(g.z, dt_kick, vel[3 * il + 2]);
    vel[3 * il] = vx; vel[3 * il + 1] = vy; vel[3 * il + 2] = vz;
    pos[3 * il] = fmaf(vx, dt_drift, x);
    pos[3 * il + 1] = fmaf(vy, dt_drift, y);
    pos[3 * il + 2] = fmaf(vz, dt_drift, z);
  }
}

__global__ __launch_bounds__(kNT) void k_gather(KernelGeom kg, const int* __restrict__ perm,
                                                const int* __restrict__ skey, const int* __restrict__ offsets,
                                                const float* __restrict__ phi, float* pos, float* vel, float* acc,
                                                int64_t n, float dt_kick, float dt_drift, int mode,
                                                const double* __restrict__ s_store) {
  extern __shared__ float smem[];
  __shared__ ChunkPlan pl;
  int* ball = reinterpret_cast<int*>(smem);
  float* tile = smem + ((kg.nball + 3) & ~3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kg.nball; b += kNT) ball[b] = kg.ball[b];
  const int he = kg.ext + 1;                  // halo: ball plus the FD stencil
  const int TE = kTile + 2 * he;
  const int TE3 = TE * TE * TE;
  // padded pitches: with TE = 16 (sigma = 1) unpadded planes are 256 floats
  // apart, so the ball's cells in different planes would share LDS banks
  const int RP = TE + 1, PP = RP * TE + 1;
  const int N = kg.N;
  const int nt = N / kTile;
  const int64_t a0 = (int64_t)blockIdx.x * kChunk;
  const int64_t a1 = min(a0 + (int64_t)kChunk, n);
  // staging the tile costs TE^3 loads; a particle read straight from memory
  // costs 6 per ball cell
  plan_chunk(pl, skey, offsets, a0, a1, (2 * TE3 + 6 * kg.nball - 1) / (6 * kg.nball));

  for (int jb = wave * 64; jb < pl.nsparse; jb += kWaves * 64) {
    const bool has = jb + lane < pl.nsparse;
    const int il = has ? perm[pl.sparse[jb + lane]] : 0;
    const int64_t i3 = 3 * (int64_t)il;
    const float xl = has ? pos[i3] : 0.f, yl = has ? pos[i3 + 1] : 0.f,
                zl = has ? pos[i3 + 2] : 0.f;
    const double sl = (has && s_store) ? s_store[il] : 0.0;
    float3 mine = make_float3(0.f, 0.f, 0.f);
    const int nb = min(64, pl.nsparse - jb);
    for (int t = 0; t < nb; ++t) {
      const float3 g = gather_one<false>(kg, ball, __shfl(xl, t, 64), __shfl(yl, t, 64), __shfl(zl, t, 64),
                                         nullptr, RP, PP, 0, 0, 0, phi, __shfl(sl, t, 64), lane);
      if (lane == t) mine = g;
    }
    if (has) gather_store(il, mine, xl, yl, zl, pos, vel, acc, dt_kick, dt_drift, mode);
  }

  for (int k = 0; k < pl.npieces; ++k) {
    const int t = pl.ptile[k];
    const int ps = pl.pstart[k], pe = pl.pend[k];
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - he, oy = ty * kTile - he, oz = tz * kTile - he;
    for (int j = threadIdx.x; j < TE3; j += kNT) {
      const int lx = j % TE, ly = (j / TE) % TE, lz = j / (TE * TE);
      tile[lz * PP + ly * RP + lx] = phi[((long long)wrapi(oz + lz, N) * N + wrapi(oy + ly, N)) * N + wrapi(ox + lx, N)];
    }
    __syncthreads();
    for (int jb = ps + wave; jb < pe; jb += kWaves * 64) {
      const int jl = jb + kWaves * lane;
      const bool has = jl < pe;
      const int il = has ? perm[jl] : 0;
      const int64_t i3 = 3 * (int64_t)il;
      const float xl = has ? pos[i3] : 0.f, yl = has ? pos[i3 + 1] : 0.f,
                  zl = has ? pos[i3 + 2] : 0.f;
      const double sl = (has && s_store) ? s_store[il] : 0.0;
      float3 mine = make_float3(0.f, 0.f, 0.f);
      const int nb = min(64, (pe - jb + kWaves - 1) / kWaves);
      for (int u = 0; u < nb; ++u) {
        const float3 g = gather_one<true>(kg, ball, __shfl(xl, u, 64), __shfl(yl, u, 64), __shfl(zl, u, 64),
                                          tile, RP, PP, ox, oy, oz, phi, __shfl(sl, u, 64), lane);
        if (lane == u) mine = g;
      }
      if (has) gather_store(il, mine, xl, yl, zl, pos, vel, acc, dt_kick, dt_drift, mode);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// diagnostics (FP64): out[0..2] P, [3..5] L, [6] Ekin, [7] mass, [8] sum m phi_i
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag_moments(const float* __restrict__ pos, const float* __restrict__ vel,
                                                      const float* __restrict__ mass, int64_t n, double* out) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double m = mass[i];
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    v[0] += m * vx; v[1] += m * vy; v[2] += m * vz;
    v[3] += m * (y * vz - z * vy); v[4] += m * (z * vx - x * vz); v[5] += m * (x * vy - y * vx);
    v[6] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    v[7] += m;
  }
  __shared__ double red[4][8];
  for (int k = 0; k < 8; ++k) {
    const double s = wave_sum_d(v[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w][threadIdx.x];
    atomicAdd(&out[threadIdx.x], s);
  }
}

__global__ __launch_bounds__(kNT) void k_diag_phi(KernelGeom kg, const float* __restrict__ pos,
                                                  const float* __restrict__ mass, const float* __restrict__ phi,
                                                  int64_t n, double* out) {
  extern __shared__ float smem[];
  int* ball = reinterpret_cast<int*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kg.nball; b += kNT) ball[b] = kg.ball[b];
  __syncthreads();
  const int N = kg.N;
  double tot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < n; i += (int64_t)gridDim.x * kWaves) {
    const Part p = particle_setup(kg, ball, pos, i, lane);
    const double norm = kg.analytic ? kg.analytic_norm : p.S;
    double acc = 0.0;
    const int nit = (kg.nball + 63) / 64;
    for (int it = 0; it < nit; ++it) {
      const int b = it * 64 + lane;
      if (b < kg.nball) {
        int dx, dy, dz;
        unpack(ball[b], dx, dy, dz);
        const long long g = ((long long)wrapi(p.cz + dz, N) * N + wrapi(p.cy + dy, N)) * N + wrapi(p.cx + dx, N);
        acc += (double)ball_weight(kg, p, dx, dy, dz) * (double)phi[g];
      }
    }
    acc = wave_sum_d(acc);
    tot += (double)mass[i] * acc / norm;
  }
  if (lane == 0) atomicAdd(&out[8], tot);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t fill_zero(float* p, long long count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

hipError_t scan_exclusive(const int* in, int n, int* out, int* blocksums, hipStream_t st) {
  const int nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(1024), 0, st, in, n, out, blocksums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, blocksums, nb, out + n);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, st, out, n, blocksums);
  return hipGetLastError();
}

hipError_t sort_particles(const KernelGeom& kg, const SortBufs& sb, const float* pos, int64_t n,
                          hipStream_t st, bool prev_order) {
  hipError_t e = fill_zero(reinterpret_cast<float*>(sb.counts), sb.ntiles + 1, st);
  if (e != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n, kg.N, kg.n,
                       kg.inv_s, kg.ext, prev_order ? sb.perm : nullptr, sb.keys, sb.rank, sb.counts, sb.flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = scan_exclusive(sb.counts, sb.ntiles, sb.offsets, sb.blocksums, st)) != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sb.keys, sb.rank,
                       sb.offsets, sb.perm, sb.skey);
  }
  return hipGetLastError();
}

// LDS of the gather: ball offsets and the phi tile with padded pitches
// (row TE + 1, plane (TE + 1) TE + 1).
static size_t gather_lds(const KernelGeom& kg) {
  const int TE = kTile + 2 * (kg.ext + 1);
  const size_t PP = (size_t)(TE + 1) * TE + 1;
  return sizeof(float) * (((kg.nball + 3) & ~3) + (size_t)TE * PP);
}

hipError_t deposit_sorted(const KernelGeom& kg, const SortBufs& sb, const float* pos, const float* mass,
                          int64_t n, float* rho, double* s_store, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kChunk - 1) / kChunk);
  const int TE = kTile + 2 * kg.ext;
  const size_t sh = sizeof(float) * (((kg.nball + 3) & ~3) + (size_t)(kg.private_tiles ? kWaves : 1) * TE * TE * TE);
  hipLaunchKernelGGL(k_deposit, dim3(blocks), dim3(kNT), sh, st, kg, sb.perm, sb.skey, sb.offsets, pos, mass, n,
                     rho, s_store);
  return hipGetLastError();
}

hipError_t gather_sorted(const KernelGeom& kg, const SortBufs& sb, const float* phi, float* pos, float* vel,
                         float* acc, int64_t n, float dt_kick, float dt_drift, int mode, const double* s_store,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kNT), gather_lds(kg), st, kg, sb.perm, sb.skey,
                     sb.offsets, phi, pos, vel, acc, n, dt_kick, dt_drift, mode, s_store);
  return hipGetLastError();
}

hipError_t diagnostics(const KernelGeom& kg, const float* pos, const float* vel, const float* mass,
                       const float* phi, int64_t n, double* out_dev, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_moments, dim3(256), dim3(256), 0, st, pos, vel, mass, n, out_dev);
  if (phi != nullptr) {
    hipLaunchKernelGGL(k_diag_phi, dim3(1024), dim3(kNT), sizeof(int) * ((kg.nball + 3) & ~3), st, kg, pos, mass,
                       phi, n, out_dev);
  }
  return hipGetLastError();
}

}  // namespace pm
