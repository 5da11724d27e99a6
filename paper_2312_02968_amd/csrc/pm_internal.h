// Internal interfaces between the C ABI (pm_api.hip) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// Scales of the half-precision spectra of the increment solve: one power of
// two per field component and writer tile (see pm_fft.hip), in three tables
// by the kind of pass that wrote the tile.
struct Scales {
  float* xs = nullptr;    // x pass: [3][N * N], one per row (row = z N + y)
  float* ys = nullptr;    // y pass: [3][P / 16][N], one per group of 16 kx and plane
  float* zs = nullptr;    // z pass: [3][P / 16][N][2], one per 8 kx of a ky row
  long long xcs = 0, ycs = 0, zcs = 0;   // per-component strides
};
inline size_t scale_floats(int N, int P) { return 3 * ((size_t)N * N + (size_t)(P / 16) * N * 3); }

// Device-side gate of a launch: with ctl set, the kernel runs only when bit
// *ctl of mask is set (every block reads the same word and returns at once
// otherwise).  The tolerance mode of the solve enqueues every iteration up to
// its cap and lets these gates skip the ones after convergence, so it needs
// no host round trip and can be captured in a graph.
struct Gate {
  const int* ctl = nullptr;
  int mask = 0;
};

// Geometry of the FFT box and its half spectrum.
struct FftGeom {
  int N;                  // n_pad
  int P;                  // kx slots of a spectrum: 16 * ceil((N/2 + 1) / 16)
  long long comp_stride;  // complex entries per spectrum component (N * N * P)
  const float2* tw;       // exp(-2 pi i t / N), t < N
  int bf16x3 = 0;         // y passes with the radix-16 stage on the matrix cores (BF16x3)
  Scales sc{};            // scale tables of the half-precision spectra
  Gate gate{};            // gate of the current launch (set by fft_pass from PassDesc)
};

// Arguments of a z pass (see pm_fft.hip).
struct ZArgs {
  float2* spec;
  float2* out = nullptr;   // FP32 output spectrum when it differs from spec (half-precision input)
  long long comp_stride;
  int ncols;
  float2* phiN;
  const float* kv;
  const float* kt;
  const float* kap;
  float newton_coef;
  float scale;
  int with_h0;     // 0: H = 0; 1: H0 given; 2: warm start from the previous F; 3: coarse start spectrum
  double* partials;
  int nc;
  const float2* cspec = nullptr;   // with_h0 3: DFT of the coarse start [3][cn^3], cn = N / cfb
  int cn = 0, cfb = 0;
};

enum PassKind {
  PASS_X_FWD_REAL, PASS_X_FWD_REAL3, PASS_X_FWD_COARSE3, PASS_X_INV_REAL, PASS_X_INV_REAL3, PASS_X_NU, PASS_X_MU,
  PASS_X_LIN_NU, PASS_X_LIN_MU, PASS_Z_GRAD,
  PASS_Y_FWD, PASS_Y_INV,
  PASS_Z_FWD, PASS_Z_INV, PASS_Z_NEWTON, PASS_Z_CURL, PASS_Z_CURL_FINAL, PASS_Z_DIV, PASS_Z_POISSON, PASS_Z_APPARENT, PASS_Z_POISSON_SPEC
};

// Density of the external-field sheets per axis (Sect. 5: a pixel layer of
// mass +M on the plane farthest from the matter and an adjacent layer of
// mass -M): +d on cell plane n_pad - 1 and -d on cell plane 0 of that axis,
// added to the density as the forward real x pass loads it.
struct Dipole {
  float x = 0.f, y = 0.f, z = 0.f;
};

// A three-component field given on a coarse grid of n^3 voxels, each value
// repeated over the f^3 box cells of its voxel and scaled by *rms (the
// learned start's network output, read by PASS_X_FWD_COARSE3 in place of a
// full-resolution H0).
struct Coarse {
  const float* y = nullptr;     // [3][n^3]
  const double* rms = nullptr;
  int n = 0;
  int f = 0;
};

struct PassDesc {
  PassKind kind;
  Dipole dip{};          // PASS_X_FWD_REAL only
  float2* spec = nullptr;
  float* real = nullptr;
  long long real_cs = 0;
  int mu_mode = 0;
  float inv_a0 = 0.f;
  float* fprev = nullptr;
  double* partials = nullptr;
  int ncomp = 1;
  ZArgs z{};
  // storage of the spectra the pass reads and writes: 0 FP32; 1 FP16 in and
  // out; 2 FP32 in, FP16 out; 3 FP16 in, FP32 out (the half-precision forms
  // exist for the passes of the increment solve)
  int io = 0;
  const float* base = nullptr;   // PASS_X_LIN_*: the field linearised about, [3][N^3]
  Coarse co{};                   // PASS_X_FWD_COARSE3
  Gate gate{};
};

hipError_t fft_pass(const FftGeom& g, const PassDesc& d, hipStream_t st);
// The learned start's coarse field in Fourier space: cs[c] = the unnormalised
// DFT over the n^3 grid of rms * y[c] (y: [3][n^3], X fastest; cs complex, the
// same layout), for n in 16..256 and boxes up to 512^3 (coarse_spectrum_supported).
bool coarse_spectrum_supported(int n, int N);
hipError_t coarse_spectrum(const FftGeom& g, const float* y, const double* rms, int n, float2* cs, hipStream_t st);
// The network's features before normalisation, g3[c] = block means over
// (N/n)^3 cells of g_N = -D phi_N, from the Newton potential's full spectrum
// phihat (PASS_Z_POISSON_SPEC, normalised) and the central-difference symbol
// kap; cs ([3][n^3] complex) is scratch.  Same sizes as coarse_spectrum.
hipError_t coarse_features(const FftGeom& g, const float2* phihat, const float* kap, int n, float2* cs, float* g3,
                           hipStream_t st);
hipError_t reduce_partials(const double* partials, int n, double* out, hipStream_t st, Gate gate = Gate{});
// Tolerance mode on the device.  ctl[0]: 0 iterating, 1 converged in this
// iteration (the final projection runs), 2 finished; ctl[1]: iterations done;
// ctl[2]: 1 if a residual was not finite.  tol_check (k >= 1): when ctl[0] is
// 0, records k and sets ctl[0] = 1 if k = kmax, or if k >= 2 and
// r_(k-1) = sqrt(acc[k-1]) / sqrt(acc[0] / n3) is at most tol or not finite.
// gate_advance: ctl[0] 1 -> 2.
hipError_t tol_check(int* ctl, const double* acc, int k, int kmax, double tol, double n3, hipStream_t st);
hipError_t gate_advance(int* ctl, hipStream_t st);
int x_blocks(int N);
int z_blocks(int N);
int z_blocks_io(int N, int io);   // z-pass blocks with half-precision spectra (io != 0)

// ---------------------------------------------------------------------------
// particles
// ---------------------------------------------------------------------------
struct KernelGeom {
  int N;            // n_pad
  int n;            // physical cells per axis
  float s;          // pixel width
  double inv_s;     // 1 / s
  float inv2sig2;   // 1 / (2 sigma^2)
  int ext;          // largest |d_axis| in the ball
  int nball;        // ball cells
  const int* ball;  // packed offsets (dx+16) | (dy+16) << 8 | (dz+16) << 16
  int analytic;     // literal prefactor instead of the ball-sum normalisation
  double analytic_norm;  // (2 pi)^1.5 sigma^3
  int private_tiles;     // deposit: one LDS tile copy per wave (no LDS atomics)
  int piece_ext;         // 3 or 5: the ball has a compiled shape (radius 4 at sigma 1
                         // or 1.5) and the tile-piece kernels run; 0: generic kernels
};

struct SortBufs {
  int* keys;        // [N] tile of each particle
  int* rank;        // [N] rank within its tile
  int* perm;        // [N] sorted order -> particle index
  int* skey;        // [N] tile of perm[i]
  int* counts;      // [ntiles + 1]
  int* offsets;     // [ntiles + 1] exclusive scan of counts
  int* blocksums;   // scan scratch
  int ntiles;
  int* flags;       // [0]: bounds violations
};

// Tile pieces (pm_pieces.hip): a tile's sorted particles in runs of at most
// kPiece, each deposited into its own staging slot (slots < cap) or straight
// into rho with atomics (slots >= cap).
#ifndef PM_PIECE
#define PM_PIECE 1024
#endif
constexpr int kPiece = PM_PIECE;
struct PieceBufs {
  int* pc_off;      // [ntiles + 1] first piece of each tile (exclusive scan)
  int* flag;        // [ntiles] scratch: pieces per tile, then destination flags
  int* list_off;    // [ntiles + 1] exclusive scan of the destination flags
  int* list;        // [ntiles] tiles that receive staged cells
  int* ptile;       // [pieces] tile of each piece
  int* counter;     // [2] work counters of the deposit and the gather
  unsigned* tmax;   // [ntiles] largest |m| of each tile's particles (float bits)
  long long* stage; // [cap][TE^3] staged halo boxes: 64-bit fixed point at the tile's scale for tiles
                    // of several pieces, else FP32 in the slot's first half
  int cap;
};
// most pieces a sort of n particles into ntiles tiles can make
inline int64_t max_pieces(int64_t ntiles, int64_t n) { return (ntiles < n ? ntiles : n) + n / kPiece + 1; }
// staging cells (64-bit) for cap pieces of a ball with the given extent
size_t piece_stage_cells(int ext, int cap);
hipError_t piece_plan(const PieceBufs& pb, const SortBufs& sb, int N, hipStream_t st);
hipError_t deposit_pieces(const KernelGeom& kg, const SortBufs& sb, const PieceBufs& pb, const float* pos,
                          const float* mass, int64_t n, float* rho, hipStream_t st);
hipError_t gather_pieces(const KernelGeom& kg, const SortBufs& sb, const PieceBufs& pb, const float* phi,
                         float* pos, float* vel, float* acc, int64_t n, float dt_kick, float dt_drift, int mode,
                         hipStream_t st);
// out[0..n) = exclusive scan of in[0..n), out[n] = total (n <= 4096 * 1024)
hipError_t scan_exclusive(const int* in, int n, int* out, int* blocksums, hipStream_t st);

// prev_order: sb.perm holds the previous sort's permutation of these n
// particles (it is read as the processing order, then replaced)
hipError_t sort_particles(const KernelGeom& kg, const SortBufs& sb, const float* pos, int64_t n,
                          hipStream_t st, bool prev_order = false);
// s_store (nullable): receives each particle's kernel normalisation (FP64)
hipError_t deposit_sorted(const KernelGeom& kg, const SortBufs& sb, const float* pos, const float* mass,
                          int64_t n, float* rho, double* s_store, hipStream_t st);
// mode 0: acc = g; mode 1: v += g dt_kick, r += v dt_drift
// s_store (nullable): normalisations written by deposit_sorted for the same positions
hipError_t gather_sorted(const KernelGeom& kg, const SortBufs& sb, const float* phi, float* pos, float* vel,
                         float* acc, int64_t n, float dt_kick, float dt_drift, int mode, const double* s_store,
                         hipStream_t st);
hipError_t fill_zero(float* p, long long count, hipStream_t st);
hipError_t diagnostics(const KernelGeom& kg, const float* pos, const float* vel, const float* mass,
                       const float* phi, int64_t n, double* out_dev, hipStream_t st);

}  // namespace pm
