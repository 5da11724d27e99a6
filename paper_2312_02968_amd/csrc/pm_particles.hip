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
  float w1;            // this lane's 1D weight (axis lane / W, offset lane % W - ext)
  double S;            // FP64 sum of the weights over the ball
};

__device__ __forceinline__ void unpack(int e, int& dx, int& dy, int& dz) {
  dx = (e & 255) - 16;
  dy = ((e >> 8) & 255) - 16;
  dz = ((e >> 16) & 255) - 16;
}

// Central pixel and 1D weights of particle i, then S (all lanes take part).
__device__ __forceinline__ Part particle_setup(const KernelGeom& kg, const int* __restrict__ ball_lds,
                                               const float* __restrict__ pos, int i, int lane) {
  const int W = 2 * kg.ext + 1;
  Part p;
  const double ux = (double)pos[3 * i + 0] * kg.inv_s;
  const double uy = (double)pos[3 * i + 1] * kg.inv_s;
  const double uz = (double)pos[3 * i + 2] * kg.inv_s;
  const double cxd = floor(ux + 0.5), cyd = floor(uy + 0.5), czd = floor(uz + 0.5);
  const int half = kg.N / 2;
  p.cx = wrapi((int)cxd + half, kg.N);
  p.cy = wrapi((int)cyd + half, kg.N);
  p.cz = wrapi((int)czd + half, kg.N);
  const int axis = lane / W;
  const int o = lane - axis * W - kg.ext;
  const double frac = axis == 0 ? cxd - ux : (axis == 1 ? cyd - uy : czd - uz);
  const float d = (float)o + (float)frac;
  p.w1 = (axis < 3) ? expf(-d * d * kg.inv2sig2) : 0.0f;
  double acc = 0.0;
  const int nit = (kg.nball + 63) / 64;
  for (int it = 0; it < nit; ++it) {
    const int b = it * 64 + lane;
    int dx = 0, dy = 0, dz = 0;
    if (b < kg.nball) unpack(ball_lds[b], dx, dy, dz);
    const float wx = __shfl(p.w1, dx + kg.ext, 64);
    const float wy = __shfl(p.w1, W + dy + kg.ext, 64);
    const float wz = __shfl(p.w1, 2 * W + dz + kg.ext, 64);
    if (b < kg.nball) acc += (double)wx * (double)wy * (double)wz;
  }
  p.S = wave_sum_d(acc);
  return p;
}

__global__ __launch_bounds__(256) void k_keys(const float* __restrict__ pos, int64_t n, int N, int nphys,
                                              double inv_s, int ext, int* keys, int* rank, int* counts,
                                              int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int half = N / 2;
  int c[3];
  bool out = false;
  for (int a = 0; a < 3; ++a) {
    const int ci = (int)floor((double)pos[3 * i + a] * inv_s + 0.5) + half;
    out |= (ci - ext < half - nphys / 2) || (ci + ext > half + nphys / 2 - 1);
    c[a] = wrapi(ci, N);
  }
  const int nt = N / kTile;
  const int key = ((c[2] / kTile) * nt + c[1] / kTile) * nt + c[0] / kTile;
  keys[i] = key;
  rank[i] = atomicAdd(&counts[key], 1);
  if (out) atomicAdd(&flags[0], 1);
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
// deposit
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_deposit(KernelGeom kg, const int* __restrict__ perm,
                                                 const int* __restrict__ skey, const int* __restrict__ offsets,
                                                 const float* __restrict__ pos, const float* __restrict__ mass,
                                                 int64_t n, float* rho) {
  extern __shared__ float smem[];
  int* ball = reinterpret_cast<int*>(smem);
  float* tile = smem + ((kg.nball + 3) & ~3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kg.nball; b += kNT) ball[b] = kg.ball[b];
  const int TE = kTile + 2 * kg.ext;
  const int TE3 = TE * TE * TE;
  const int W = 2 * kg.ext + 1;
  const int N = kg.N;
  const int nt = N / kTile;
  const double s3 = (double)kg.s * kg.s * kg.s;
  __syncthreads();

  const int64_t a0 = (int64_t)blockIdx.x * kChunk;
  const int64_t a1 = min(a0 + (int64_t)kChunk, n);
  int64_t a = a0;
  while (a < a1) {
    const int t = skey[a];
    int64_t e = min((int64_t)offsets[t + 1], a1);
    if (e <= a) e = a + 1;   // sorted order guarantees progress; never stall
    const int cnt = (int)(e - a);
    const bool use_lds = (int64_t)cnt * kg.nball >= (int64_t)TE3;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - kg.ext, oy = ty * kTile - kg.ext, oz = tz * kTile - kg.ext;
    if (use_lds) {
      for (int j = threadIdx.x; j < TE3; j += kNT) tile[j] = 0.0f;
      __syncthreads();
    }
    for (int64_t j = a + wave; j < e; j += kWaves) {
      const int i = perm[j];
      const Part p = particle_setup(kg, ball, pos, i, lane);
      const double norm = kg.analytic ? kg.analytic_norm : p.S;
      const float scale = (float)((double)mass[i] / (norm * s3));
      const int nit = (kg.nball + 63) / 64;
      for (int it = 0; it < nit; ++it) {
        const int b = it * 64 + lane;
        int dx = 0, dy = 0, dz = 0;
        if (b < kg.nball) unpack(ball[b], dx, dy, dz);
        const float wx = __shfl(p.w1, dx + kg.ext, 64);
        const float wy = __shfl(p.w1, W + dy + kg.ext, 64);
        const float wz = __shfl(p.w1, 2 * W + dz + kg.ext, 64);
        if (b < kg.nball) {
          const float v = wx * wy * wz * scale;
          if (use_lds) {
            const int lx = p.cx + dx - ox, ly = p.cy + dy - oy, lz = p.cz + dz - oz;
            atomicAdd(&tile[(lz * TE + ly) * TE + lx], v);
          } else {
            const long long g = ((long long)wrapi(p.cz + dz, N) * N + wrapi(p.cy + dy, N)) * N + wrapi(p.cx + dx, N);
            unsafeAtomicAdd(&rho[g], v);
          }
        }
      }
    }
    if (use_lds) {
      __syncthreads();
      for (int j = threadIdx.x; j < TE3; j += kNT) {
        const float v = tile[j];
        if (v != 0.0f) {
          const int lx = j % TE, ly = (j / TE) % TE, lz = j / (TE * TE);
          const long long g = ((long long)wrapi(oz + lz, N) * N + wrapi(oy + ly, N)) * N + wrapi(ox + lx, N);
          unsafeAtomicAdd(&rho[g], v);
        }
      }
      __syncthreads();
    }
    a = e;
  }
}

// ---------------------------------------------------------------------------
// gather + push
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_gather(KernelGeom kg, const int* __restrict__ perm,
                                                const int* __restrict__ skey, const int* __restrict__ offsets,
                                                const float* __restrict__ phi, float* pos, float* vel, float* acc,
                                                int64_t n, float dt_kick, float dt_drift, int mode) {
  extern __shared__ float smem[];
  int* ball = reinterpret_cast<int*>(smem);
  float* tile = smem + ((kg.nball + 3) & ~3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = threadIdx.x; b < kg.nball; b += kNT) ball[b] = kg.ball[b];
  const int he = kg.ext + 1;                  // halo: ball plus the FD stencil
  const int TE = kTile + 2 * he;
  const int TE3 = TE * TE * TE;
  const int W = 2 * kg.ext + 1;
  const int N = kg.N;
  const int nt = N / kTile;
  __syncthreads();

  const int64_t a0 = (int64_t)blockIdx.x * kChunk;
  const int64_t a1 = min(a0 + (int64_t)kChunk, n);
  int64_t a = a0;
  while (a < a1) {
    const int t = skey[a];
    int64_t e = min((int64_t)offsets[t + 1], a1);
    if (e <= a) e = a + 1;   // sorted order guarantees progress; never stall
    const int cnt = (int)(e - a);
    const bool use_lds = (int64_t)cnt * kg.nball * 6 >= (int64_t)TE3 * 2;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int ox = tx * kTile - he, oy = ty * kTile - he, oz = tz * kTile - he;
    if (use_lds) {
      for (int j = threadIdx.x; j < TE3; j += kNT) {
        const int lx = j % TE, ly = (j / TE) % TE, lz = j / (TE * TE);
        tile[j] = phi[((long long)wrapi(oz + lz, N) * N + wrapi(oy + ly, N)) * N + wrapi(ox + lx, N)];
      }
      __syncthreads();
    }
    for (int64_t j = a + wave; j < e; j += kWaves) {
      const int i = perm[j];
      const Part p = particle_setup(kg, ball, pos, i, lane);
      const double norm = kg.analytic ? kg.analytic_norm : p.S;
      float gx = 0.f, gy = 0.f, gz = 0.f;
      const int nit = (kg.nball + 63) / 64;
      for (int it = 0; it < nit; ++it) {
        const int b = it * 64 + lane;
        int dx = 0, dy = 0, dz = 0;
        if (b < kg.nball) unpack(ball[b], dx, dy, dz);
        const float wx = __shfl(p.w1, dx + kg.ext, 64);
        const float wy = __shfl(p.w1, W + dy + kg.ext, 64);
        const float wz = __shfl(p.w1, 2 * W + dz + kg.ext, 64);
        if (b < kg.nball) {
          const float w = wx * wy * wz;
          float xp, xm, yp, ym, zp, zm;
          if (use_lds) {
            const int lx = p.cx + dx - ox, ly = p.cy + dy - oy, lz = p.cz + dz - oz;
            const int c = (lz * TE + ly) * TE + lx;
            xp = tile[c + 1]; xm = tile[c - 1];
            yp = tile[c + TE]; ym = tile[c - TE];
            zp = tile[c + TE * TE]; zm = tile[c - TE * TE];
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
      gx = wave_sum_f(gx);
      gy = wave_sum_f(gy);
      gz = wave_sum_f(gz);
      const float f = (float)(-1.0 / (2.0 * (double)kg.s * norm));
      gx *= f; gy *= f; gz *= f;
      if (lane < 3) {
        const float g = lane == 0 ? gx : (lane == 1 ? gy : gz);
        if (mode == 0) {
          acc[3 * i + lane] = g;
        } else {
          const float v = fmaf(g, dt_kick, vel[3 * i + lane]);
          vel[3 * i + lane] = v;
          pos[3 * i + lane] = fmaf(v, dt_drift, pos[3 * i + lane]);
        }
      }
    }
    if (use_lds) __syncthreads();
    a = e;
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
  const int W = 2 * kg.ext + 1, N = kg.N;
  double tot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWaves + wave; i < n; i += (int64_t)gridDim.x * kWaves) {
    const Part p = particle_setup(kg, ball, pos, (int)i, lane);
    const double norm = kg.analytic ? kg.analytic_norm : p.S;
    double acc = 0.0;
    const int nit = (kg.nball + 63) / 64;
    for (int it = 0; it < nit; ++it) {
      const int b = it * 64 + lane;
      int dx = 0, dy = 0, dz = 0;
      if (b < kg.nball) unpack(ball[b], dx, dy, dz);
      const float wx = __shfl(p.w1, dx + kg.ext, 64);
      const float wy = __shfl(p.w1, W + dy + kg.ext, 64);
      const float wz = __shfl(p.w1, 2 * W + dz + kg.ext, 64);
      if (b < kg.nball) {
        const long long g = ((long long)wrapi(p.cz + dz, N) * N + wrapi(p.cy + dy, N)) * N + wrapi(p.cx + dx, N);
        acc += (double)(wx * wy * wz) * (double)phi[g];
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

hipError_t sort_particles(const KernelGeom& kg, const SortBufs& sb, const float* pos, int64_t n,
                          hipStream_t st) {
  hipError_t e = fill_zero(reinterpret_cast<float*>(sb.counts), sb.ntiles + 1, st);
  if (e != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n, kg.N, kg.n,
                       kg.inv_s, kg.ext, sb.keys, sb.rank, sb.counts, sb.flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nb = (sb.ntiles + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(1024), 0, st, sb.counts, sb.ntiles, sb.offsets, sb.blocksums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sb.blocksums, nb, sb.offsets + sb.ntiles);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, st, sb.offsets, sb.ntiles, sb.blocksums);
  if (n > 0) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, sb.keys, sb.rank,
                       sb.offsets, sb.perm, sb.skey);
  }
  return hipGetLastError();
}

static size_t particle_lds(const KernelGeom& kg, int halo) {
  const int TE = kTile + 2 * halo;
  return sizeof(float) * (((kg.nball + 3) & ~3) + (size_t)TE * TE * TE);
}

hipError_t deposit_sorted(const KernelGeom& kg, const SortBufs& sb, const float* pos, const float* mass,
                          int64_t n, float* rho, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_deposit, dim3(blocks), dim3(kNT), particle_lds(kg, kg.ext), st, kg, sb.perm, sb.skey,
                     sb.offsets, pos, mass, n, rho);
  return hipGetLastError();
}

hipError_t gather_sorted(const KernelGeom& kg, const SortBufs& sb, const float* phi, float* pos, float* vel,
                         float* acc, int64_t n, float dt_kick, float dt_drift, int mode, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kNT), particle_lds(kg, kg.ext + 1), st, kg, sb.perm, sb.skey,
                     sb.offsets, phi, pos, vel, acc, n, dt_kick, dt_drift, mode);
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
