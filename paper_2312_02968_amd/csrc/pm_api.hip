// C ABI of the PM step (declared in include/mondpm.h): context, tables, and
// the host-side orchestration of the passes of one AQUAL solve.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "mondpm.h"
#include "pm_internal.h"
#include "pm_net.h"

using namespace pm;

static thread_local char g_err[512] = "";

static pm_status dev_fail(hipError_t e, const char* where) {
  const char* step = net::last_failure();
  snprintf(g_err, sizeof g_err, "%s: %s%s%s", where, hipGetErrorString(e), step[0] ? " at " : "", step);
  return PM_E_DEVICE;
}
static pm_status inval(const char* msg) {
  snprintf(g_err, sizeof g_err, "invalid argument: %s", msg);
  return PM_E_INVAL;
}

#define HIPCHK(call)                                        \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return dev_fail(e_, #call);       \
  } while (0)

struct pm_ctx {
  pm_params p;
  int N = 0, n = 0, P = 0;
  hipStream_t st = nullptr;
  int64_t max_particles = 0;
  float2* spec = nullptr;     // three spectra
  float2* phiN = nullptr;     // Newton potential spectrum
  float* rho = nullptr;       // internal real grids of pm_step
  float* phi = nullptr;
  float* fprev = nullptr;     // previous F for the residual and the warm start (optional)
  bool have_F = false;        // fprev holds the last F of a solve
  float* scales = nullptr;    // scale tables of the increment solve's half-precision spectra
  int* ctl = nullptr;         // tolerance-mode control words (see tol_check)
  double* partials = nullptr;
  double* dacc = nullptr;     // [0] |g_N|^2 sum, [1..64] residual sums, [80..89] diagnostics
  double hacc[128] = {};      // host copy of dacc
  float2* tw = nullptr;
  float* kv = nullptr;
  float* kt = nullptr;
  float* kap = nullptr;
  int* ball = nullptr;
  int nball = 0;
  int* ibuf = nullptr;        // sort buffers
  double* snorm = nullptr;    // per-particle kernel normalisation (pm_step: deposit -> gather)
  void* owned = nullptr;      // the workspace when the library allocated it
  FftGeom fg{};
  KernelGeom kg{};
  SortBufs sb{};
  PieceBufs pb{};
  int piece_ext = 0;          // compiled ball shape of the tile-piece kernels, 0: none
  int64_t perm_n = -1;        // sb.perm is a permutation of [0, perm_n) from the last sort
  int npartials = 0;
  hipGraphExec_t step_graph = nullptr;  // one captured pm_step (pm_step_capture)
  Dipole dip{};               // external-field sheets added to every Newton solve's density
  // event timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;   // timer id per recorded pair
  size_t ev_used = 0;
};

// Records an event pair around one launch when timing is on.
struct Timed {
  pm_ctx* c;
  int kind;
  size_t slot;
  bool on;
  Timed(pm_ctx* c_, int kind_) : c(c_), kind(kind_), slot(0), on(c_->timing) {
    if (!on) return;
    if (c->ev_used + 2 > c->ev_pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
        c->ev_pool.push_back(e);
      }
      c->ev_kind.resize(c->ev_pool.size() / 2);
    }
    slot = c->ev_used;
    c->ev_used += 2;
    c->ev_kind[slot / 2] = kind;
    (void)hipEventRecord(c->ev_pool[slot], c->st);
  }
  ~Timed() {
    if (on) (void)hipEventRecord(c->ev_pool[slot + 1], c->st);
  }
};

static int timer_of(PassKind k) {
  switch (k) {
    case PASS_X_FWD_REAL: return PM_T_X_FWD_REAL;
    case PASS_X_FWD_REAL3: return PM_T_X_FWD_REAL3;
    case PASS_X_INV_REAL: return PM_T_X_INV_REAL;
    case PASS_X_INV_REAL3: return PM_T_X_INV_REAL;
    case PASS_X_LIN_NU: return PM_T_X_NU;
    case PASS_X_LIN_MU: return PM_T_X_MU;
    case PASS_Z_GRAD: return PM_T_Z_FWD;
    case PASS_X_NU: return PM_T_X_NU;
    case PASS_X_MU: return PM_T_X_MU;
    case PASS_Y_FWD: return PM_T_Y_FWD;
    case PASS_Y_INV: return PM_T_Y_INV;
    case PASS_Z_FWD: return PM_T_Z_FWD;
    case PASS_Z_INV: return PM_T_Z_INV;
    case PASS_Z_NEWTON: return PM_T_Z_NEWTON;
    case PASS_Z_CURL: return PM_T_Z_CURL;
    case PASS_Z_CURL_FINAL: return PM_T_Z_CURL_FINAL;
    case PASS_Z_DIV: return PM_T_Z_DIV;
    case PASS_Z_POISSON: return PM_T_Z_NEWTON;
    case PASS_Z_POISSON_SPEC: return PM_T_Z_NEWTON;
    case PASS_Z_APPARENT: return PM_T_Z_FWD;
  }
  return PM_T_REDUCE;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Particle indices are 32-bit in the sort buffers and the particle kernels.
static constexpr int64_t kMaxParticles = (int64_t)1 << 30;

int32_t pm_spectrum_pitch(int32_t n_pad) {
  const int need = n_pad / 2 + 1;
  return (need + 15) & ~15;
}

static pm_status check_params(const pm_params* p) {
  if (!p) return inval("params is NULL");
  if (!pow2(p->n_pad) || p->n_pad < 16 || p->n_pad > 1024) return inval("n_pad must be a power of two in [16, 1024]");
  if (!pow2(p->n) || p->n < 8 || p->n > p->n_pad) return inval("n must be a power of two in [8, n_pad]");
  if (!(p->box > 0.0) || !isfinite(p->box)) return inval("box must be > 0");
  if (!isfinite(p->G)) return inval("G must be finite");
  if (p->mu != PM_MU_STANDARD && p->mu != PM_MU_DEEP && p->mu != PM_MU_NEWTON) return inval("unknown mu");
  if (p->mu != PM_MU_NEWTON && !(p->a0 > 0.0)) return inval("a0 must be > 0");
  if (!(p->sigma > 0.0) || !(p->cutoff > 0.0)) return inval("sigma and cutoff must be > 0");
  const double R = p->cutoff * p->sigma;
  if (R > 10.0) return inval("cutoff * sigma must be <= 10 cells");
  if (p->iters < 1 || p->iters > 64) return inval("iters must be in [1, 64]");
  if ((p->flags & PM_F_WARM_START) && p->iters < 2)
    return inval("PM_F_WARM_START needs iters >= 2 (with one iteration F is never updated)");
  if (!(p->tol >= 0.0)) return inval("tol must be >= 0");
  if ((p->flags & PM_F_DFT_BF16X3) && (p->n_pad < 64 || p->n_pad > 512))
    return inval("PM_F_DFT_BF16X3 needs n_pad in [64, 512]");
  return PM_OK;
}

static int ball_extent(double R) { return (int)ceil(R) - 1; }

static std::vector<int> make_ball(double R) {
  std::vector<int> out;
  const int m = (int)floor(R);
  for (int dz = -m; dz <= m; ++dz)
    for (int dy = -m; dy <= m; ++dy)
      for (int dx = -m; dx <= m; ++dx)
        if ((double)(dx * dx + dy * dy + dz * dz) < R * R)
          out.push_back((dx + 16) | ((dy + 16) << 8) | ((dz + 16) << 16));
  return out;
}

static bool need_residual(const pm_params& p) { return (p.flags & PM_F_RESIDUAL) || p.tol > 0.0; }

// Device memory of a context: one region (the caller's workspace or a single
// allocation of the library) cut into 256-byte aligned pieces.  With base ==
// nullptr only the size is counted.
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (count ? count : 1) * sizeof(T);
    return ptr;
  }
};

// Sizes that follow from the parameters (set before carve).
static void derive_sizes(pm_ctx* c, const pm_params* p, int64_t max_particles) {
  c->p = *p;
  c->N = p->n_pad;
  c->n = p->n;
  c->P = pm_spectrum_pitch(p->n_pad);
  c->max_particles = max_particles;
  c->nball = (int)make_ball(p->cutoff * p->sigma).size();
  c->npartials = x_blocks(c->N) > z_blocks(c->N) ? x_blocks(c->N) : z_blocks(c->N);
  // The tile-piece kernels are compiled for the balls |d|^2 < 16 and < 36
  // (radius 4 sigma at sigma = 1 and 1.5 cells): any R^2 in (15, 16] or
  // (35, 36] gives the same integer cells.
  const double R2 = (p->cutoff * p->sigma) * (p->cutoff * p->sigma);
  c->piece_ext = (R2 > 15.0 && R2 <= 16.0) ? 3 : (R2 > 35.0 && R2 <= 36.0) ? 5 : 0;
  c->pb.cap = 0;
  if (c->piece_ext) {
    const int64_t N = c->N;
    const int64_t ntiles = (N / 8) * (N / 8) * (N / 8);
    const int64_t mp = max_particles > 0 ? max_particles : 1;
    const int64_t most = max_pieces(ntiles, mp);
    const int64_t te = 8 + 2 * c->piece_ext;
    const int64_t by_bytes = ((int64_t)2 << 30) / (te * te * te * 8);      // 2 GB of staging
    c->pb.cap = (int)(most < by_bytes ? most : by_bytes);
  }
}

// Assigns every device buffer of the context from cv; returns the bytes used.
static size_t carve(pm_ctx* c, Carver& cv) {
  const size_t N = c->N, C = N * N * (size_t)c->P, R = N * N * N;
  const size_t ntiles = (N / 8) * (N / 8) * (N / 8);
  const size_t mp = (size_t)(c->max_particles > 0 ? c->max_particles : 1);
  const size_t nb = (ntiles + 1023) / 1024;
  c->spec = cv.take<float2>(3 * C);
  c->phiN = cv.take<float2>(C);
  c->rho = cv.take<float>(R);
  c->phi = cv.take<float>(R);
  c->fprev = (need_residual(c->p) || (c->p.flags & PM_F_WARM_START)) ? cv.take<float>(3 * R) : nullptr;
  c->scales = cv.take<float>(scale_floats((int)N, c->P));
  c->ctl = cv.take<int>(16);
  c->partials = cv.take<double>((size_t)c->npartials);
  c->dacc = cv.take<double>(128);
  c->tw = cv.take<float2>(N);
  c->kv = cv.take<float>(N);
  c->kt = cv.take<float>(N);
  c->kap = cv.take<float>(N);
  c->ball = cv.take<int>((size_t)c->nball);
  c->ibuf = cv.take<int>(4 * mp + 2 * (ntiles + 1) + nb + 16);
  c->snorm = cv.take<double>(mp);
  if (c->piece_ext) {
    c->pb.pc_off = cv.take<int>(ntiles + 1);
    c->pb.flag = cv.take<int>(ntiles);
    c->pb.list_off = cv.take<int>(ntiles + 1);
    c->pb.list = cv.take<int>(ntiles);
    c->pb.ptile = cv.take<int>((size_t)max_pieces((int64_t)ntiles, (int64_t)mp));
    c->pb.counter = cv.take<int>(16);
    c->pb.tmax = cv.take<unsigned>(ntiles);
    c->pb.stage = cv.take<long long>(piece_stage_cells(c->piece_ext, c->pb.cap));
  }
  return (cv.off + 255) & ~(size_t)255;
}

size_t pm_workspace_bytes(const pm_params* p, int64_t max_particles) {
  if (check_params(p) != PM_OK || max_particles < 0 || max_particles > kMaxParticles) return 0;
  pm_ctx c;
  derive_sizes(&c, p, max_particles);
  Carver cv;
  return carve(&c, cv);
}

const char* pm_last_error(void) { return g_err; }

pm_status pm_destroy(pm_ctx* c) {
  if (!c) return PM_OK;
  (void)(c->st ? hipStreamSynchronize(c->st) : hipDeviceSynchronize());
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->step_graph) (void)hipGraphExecDestroy(c->step_graph);
  if (c->owned) (void)hipFree(c->owned);
  delete c;
  return PM_OK;
}

pm_status pm_create(const pm_params* p, int64_t max_particles, void* workspace, size_t workspace_bytes,
                    void* stream, pm_ctx** out) {
  if (!out) return inval("out is NULL");
  *out = nullptr;
  pm_status s = check_params(p);
  if (s != PM_OK) return s;
  if (max_particles < 0 || max_particles > kMaxParticles) return inval("max_particles out of range");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return inval("workspace must be 256-byte aligned");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));

  pm_ctx* c = new pm_ctx();
  derive_sizes(c, p, max_particles);
  c->st = static_cast<hipStream_t>(stream);
  const int N = c->N;
  const size_t C = (size_t)N * N * c->P;
  const double Rb = p->cutoff * p->sigma;
  std::vector<int> ball = make_ball(Rb);
  const int ext = ball_extent(Rb);
  const size_t lds_need = sizeof(float) * (((ball.size() + 3) & ~(size_t)3) + (size_t)(8 + 2 * (ext + 1)) *
                                                                                   (8 + 2 * (ext + 1)) * (8 + 2 * (ext + 1)));
  // plus the per-block chunk plan of the particle kernels (4 lists of 512 ints)
  if (lds_need + 4 * 512 * sizeof(int) + 64 > prop.sharedMemPerBlock) {
    delete c;
    return inval("kernel ball too large for the LDS of this device");
  }
  const int ntiles = (N / 8) * (N / 8) * (N / 8);
  {
    Carver count;
    const size_t need = carve(c, count);
    Carver cv;
    if (workspace) {
      if (workspace_bytes < need) {
        delete c;
        snprintf(g_err, sizeof g_err, "invalid argument: workspace has %zu bytes, needs %zu (pm_workspace_bytes)",
                 workspace_bytes, need);
        return PM_E_INVAL;
      }
      cv.base = static_cast<char*>(workspace);
    } else {
      void* v = nullptr;
      const hipError_t e = hipMalloc(&v, need);
      if (e != hipSuccess) {
        delete c;
        snprintf(g_err, sizeof g_err, "hipMalloc(%zu bytes): %s", need, hipGetErrorString(e));
        return PM_E_NOMEM;
      }
      c->owned = v;
      cv.base = static_cast<char*>(v);
    }
    carve(c, cv);
  }
#define CCHK(call)                                              \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) { pm_destroy(c); return dev_fail(e_, #call); } \
  } while (0)

  // tables (FP64 on the host, stored in FP32)
  const double s_px = p->box / p->n;
  std::vector<float2> tw(N);
  std::vector<float> kv(N), kt(N), kap(N);
  for (int t = 0; t < N; ++t) {
    const double a = 2.0 * M_PI * t / N;
    tw[t] = make_float2((float)cos(a), (float)-sin(a));
    const int m = t < N / 2 ? t : t - N;
    const double k = 2.0 * M_PI * m / (N * s_px);
    kv[t] = (float)k;
    kt[t] = (t == N / 2) ? 0.0f : (float)k;
    kap[t] = (t == 0 || t == N / 2) ? 0.0f : (float)(sin(2.0 * M_PI * m / N) / s_px);
  }
  CCHK(hipMemcpyAsync(c->tw, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice, c->st));
  CCHK(hipMemcpyAsync(c->kv, kv.data(), N * sizeof(float), hipMemcpyHostToDevice, c->st));
  CCHK(hipMemcpyAsync(c->kt, kt.data(), N * sizeof(float), hipMemcpyHostToDevice, c->st));
  CCHK(hipMemcpyAsync(c->kap, kap.data(), N * sizeof(float), hipMemcpyHostToDevice, c->st));
  CCHK(hipMemcpyAsync(c->ball, ball.data(), ball.size() * sizeof(int), hipMemcpyHostToDevice, c->st));

  c->fg.N = N;
  c->fg.P = c->P;
  c->fg.comp_stride = (long long)C;
  c->fg.tw = c->tw;
  c->fg.bf16x3 = (p->flags & PM_F_DFT_BF16X3) ? 1 : 0;
  c->fg.sc.xs = c->scales;
  c->fg.sc.xcs = (long long)N * N;
  c->fg.sc.ys = c->scales + 3 * c->fg.sc.xcs;
  c->fg.sc.ycs = (long long)(c->P / 16) * N;
  c->fg.sc.zs = c->fg.sc.ys + 3 * c->fg.sc.ycs;
  c->fg.sc.zcs = 2 * c->fg.sc.ycs;

  c->kg.N = N;
  c->kg.n = p->n;
  c->kg.s = (float)s_px;
  c->kg.inv_s = 1.0 / s_px;
  c->kg.inv2sig2 = (float)(1.0 / (2.0 * p->sigma * p->sigma));
  c->kg.ext = ext;
  c->kg.nball = (int)ball.size();
  c->kg.ball = c->ball;
  c->kg.analytic = (p->flags & PM_F_ANALYTIC_NORM) ? 1 : 0;
  c->kg.analytic_norm = pow(2.0 * M_PI, 1.5) * p->sigma * p->sigma * p->sigma;
  {
    // one deposit tile copy per wave when four copies fit in 96 KB of LDS
    const size_t te = 8 + 2 * (size_t)ext;
    c->kg.private_tiles = (4 * te * te * te * sizeof(float) <= 96 * 1024) ? 1 : 0;
  }
  c->kg.piece_ext = c->piece_ext;

  const size_t mp = (size_t)(max_particles > 0 ? max_particles : 1);
  const size_t nb = ((size_t)ntiles + 1023) / 1024;
  int* ib = c->ibuf;
  c->sb.keys = ib; ib += mp;
  c->sb.rank = ib; ib += mp;
  c->sb.perm = ib; ib += mp;
  c->sb.skey = ib; ib += mp;
  c->sb.counts = ib; ib += ntiles + 1;
  c->sb.offsets = ib; ib += ntiles + 1;
  c->sb.blocksums = ib; ib += nb;
  c->sb.flags = ib;
  c->sb.ntiles = ntiles;
  CCHK(fill_zero(reinterpret_cast<float*>(c->sb.flags), 16, c->st));
  CCHK(c->st ? hipStreamSynchronize(c->st) : hipDeviceSynchronize());
#undef CCHK
  *out = c;
  return PM_OK;
}

// ----------------------------------------------------------------------------
// solve
// ----------------------------------------------------------------------------
static hipError_t pass(pm_ctx* c, PassDesc d) {
  Timed t(c, timer_of(d.kind));
  return fft_pass(c->fg, d, c->st);
}

static PassDesc pdesc(PassKind k, float2* spec, int ncomp = 1) {
  PassDesc d;
  d.kind = k;
  d.spec = spec;
  d.ncomp = ncomp;
  return d;
}

static ZArgs zargs(pm_ctx* c) {
  ZArgs z{};
  z.spec = c->spec;
  z.phiN = c->phiN;
  z.kv = c->kv;
  z.kt = c->kt;
  z.kap = c->kap;
  z.newton_coef = (float)(-4.0 * M_PI * c->p.G);
  const double N = c->N;
  z.scale = (float)(1.0 / (N * N * N));
  z.partials = c->partials;
  z.nc = 1;
  return z;
}

// The increment form of the solve (Sect. 5, item (v)): the density, the
// Newton field and H are increments, Eqs. inverse and interpolation are
// linearised about F and g_M of the previous solve, and the spectra between
// passes are stored in FP16 when io = 1.
struct Increment {
  const float* F;      // [3][N^3] F = g_N + H of the previous solve
  const float* gM;     // [3][N^3] its g_M (curl-free part of nu(|F|/a0) F)
  int io;              // 0: FP32 spectra; 1: FP16
  float* dF;           // nullable: receives dF of the last iteration
};

static pm_status run_solve(pm_ctx* c, const float* rho, const float* H0, float* phi_out, pm_solve_info* info,
                           bool want_info, const Increment* inc = nullptr, const net::Buffers* learned = nullptr) {
  const pm_params& p = c->p;
  const int N = c->N;
  const long long R = (long long)N * N * N;
  const bool resid = need_residual(p);
  const int K = p.iters;
  const float inv_a0 = (p.mu == PM_MU_NEWTON) ? 0.0f : (float)(1.0 / p.a0);
  const double N3 = (double)N * N * N;
  const int io = inc ? inc->io : 0;
  // the potential's spectrum: in place, or with FP16 spectra past their end
  // (they fill the first half of the spectrum buffer)
  float2* fin = io ? c->spec + (3 * c->fg.comp_stride) / 2 : c->spec;
  pm_solve_info loc{};
  loc.status = PM_OK;

  // Newton: rho -> (x, y) spectrum in the phiN buffer (the external-field
  // sheets are constant, so an increment carries none)
  {
    PassDesc d = pdesc(PASS_X_FWD_REAL, c->phiN);
    d.real = const_cast<float*>(rho);
    if (!inc) d.dip = c->dip;
    HIPCHK(pass(c, d));
    HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->phiN, 1)));
  }
  // learned start: the network's features from the spectrum just formed, its
  // forward pass, and its coarse output brought into the Newton z pass.  For
  // the network sizes with coarse transforms, both ends stay in Fourier
  // space: a Poisson z pass gives the Newton potential's full spectrum, whose
  // aliases onto the network's grid are the block means of g_N (in the phi
  // buffer as scratch), and the coarse output's own DFT, times the DFT of a
  // block, is the start's spectrum that the Newton z pass takes.  Otherwise
  // the potential goes to real space for the features (phiN kept) and the
  // output is expanded in the forward x pass.
  bool coarse = false;
  float2* cspec = reinterpret_cast<float2*>(c->phi);
  if (learned) {
    const double s_px = c->p.box / c->p.n;
    const int fb = N / learned->n;
    coarse = coarse_spectrum_supported(learned->n, N);
    PassDesc z = pdesc(coarse ? PASS_Z_POISSON_SPEC : PASS_Z_POISSON, c->phiN);
    z.z = zargs(c);
    z.z.spec = c->phiN;
    z.z.out = c->spec;
    HIPCHK(pass(c, z));
    if (coarse) {
      HIPCHK(coarse_features(c->fg, c->spec, c->kap, learned->n, cspec, net::feature_means(*learned, 0), c->st));
      HIPCHK(net::features_from_means(*learned, 0, c->p.a0, c->st));
    } else {
      HIPCHK(pass(c, pdesc(PASS_Y_INV, c->spec, 1)));
      PassDesc x = pdesc(PASS_X_INV_REAL, c->spec);
      x.real = c->phi;
      HIPCHK(pass(c, x));
      HIPCHK(net::features(*learned, 0, c->phi, 0.5 / s_px, c->p.a0, fb, c->st));
    }
    HIPCHK(net::forward(*learned, 1, c->st));
    if (coarse) {
      HIPCHK(coarse_spectrum(c->fg, learned->yhat, learned->rms, learned->n, cspec, c->st));
    } else {
      PassDesc d = pdesc(PASS_X_FWD_COARSE3, c->spec);
      d.co = Coarse{learned->yhat, learned->rms, learned->n, fb};
      HIPCHK(pass(c, d));
      HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->spec, 3)));
    }
  }
  // warm start: F0 = P_L g_N + P_T F_prev from the last F of the previous solve
  const bool keep_F = !inc && (p.flags & PM_F_WARM_START) != 0;
  const bool warm = keep_F && c->have_F && !H0 && !learned;
  const float* start = inc ? nullptr : (H0 ? H0 : (warm ? c->fprev : nullptr));
  if (start) {
    PassDesc d = pdesc(PASS_X_FWD_REAL3, c->spec);
    d.real = const_cast<float*>(start);
    d.real_cs = R;
    HIPCHK(pass(c, d));
    HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->spec, 3)));
  }
  // Tolerance mode: every iteration up to K is enqueued and gated on the
  // device (run0: while iterating, run1: the stopping iteration's final
  // projection, run01: both), so the host never waits.
  const bool dev_tol = p.tol > 0.0;
  const Gate run0 = dev_tol ? Gate{c->ctl, 1} : Gate{};
  const Gate run1 = dev_tol ? Gate{c->ctl, 2} : Gate{};
  const Gate run01 = dev_tol ? Gate{c->ctl, 3} : Gate{};
  if (dev_tol) HIPCHK(fill_zero(reinterpret_cast<float*>(c->ctl), 4, c->st));
  auto spec3 = [&](PassKind k) {
    PassDesc d = pdesc(k, c->spec, 3);
    d.io = io;
    d.gate = run0;
    return d;
  };
  {
    PassDesc d = pdesc(PASS_Z_NEWTON, c->spec);
    d.z = zargs(c);
    d.z.with_h0 = warm ? 2 : (coarse ? 3 : ((start || learned) ? 1 : 0));
    if (coarse) {
      d.z.cspec = cspec;
      d.z.cn = learned->n;
      d.z.cfb = N / learned->n;
    }
    d.io = io ? 2 : 0;
    HIPCHK(pass(c, d));
    HIPCHK(reduce_partials(c->partials, z_blocks_io(N, d.io), c->dacc, c->st));
    HIPCHK(pass(c, spec3(PASS_Y_INV)));
  }
  int k_done = 0;
  for (int k = 1; k <= K; ++k) {
    {
      PassDesc d = spec3(inc ? PASS_X_LIN_NU : PASS_X_NU);
      d.mu_mode = p.mu;
      d.inv_a0 = inv_a0;
      d.base = inc ? inc->F : nullptr;
      // F (or dF) is kept every iteration for the residual; for the warm start
      // (or the caller's dF) only the last one
      if (resid) d.fprev = c->fprev;
      else if (keep_F && k == K) d.fprev = c->fprev;
      else if (inc && inc->dF && k == K) d.fprev = inc->dF;
      d.partials = c->partials;
      HIPCHK(pass(c, d));
    }
    if (resid && k >= 2) HIPCHK(reduce_partials(c->partials, x_blocks(N), c->dacc + (k - 1), c->st, run0));
    if (dev_tol) HIPCHK(tol_check(c->ctl, c->dacc, k, K, p.tol, N3, c->st));
    k_done = k;
    {
      PassDesc d = spec3(PASS_Y_FWD);
      d.gate = run01;
      HIPCHK(pass(c, d));
    }
    if (dev_tol || k == K) {
      // the last projection, to phi: in the tolerance mode enqueued every
      // iteration and run by the one in which the iteration stops
      PassDesc d = pdesc(PASS_Z_CURL_FINAL, c->spec);
      d.z = zargs(c);
      d.io = io ? 3 : 0;
      d.z.out = fin;
      d.gate = run1;
      HIPCHK(pass(c, d));
      if (!dev_tol) break;
      HIPCHK(gate_advance(c->ctl, c->st));
      if (k == K) break;
    }
    {
      PassDesc d = spec3(PASS_Z_CURL);
      d.z = zargs(c);
      HIPCHK(pass(c, d));
    }
    HIPCHK(pass(c, spec3(PASS_Y_INV)));
    {
      PassDesc d = spec3(inc ? PASS_X_LIN_MU : PASS_X_MU);
      d.mu_mode = p.mu;
      d.inv_a0 = inv_a0;
      d.base = inc ? inc->gM : nullptr;
      HIPCHK(pass(c, d));
    }
    HIPCHK(pass(c, spec3(PASS_Y_FWD)));
    {
      PassDesc d = spec3(PASS_Z_DIV);
      d.z = zargs(c);
      HIPCHK(pass(c, d));
    }
    HIPCHK(pass(c, spec3(PASS_Y_INV)));
  }
  if (inc) {
    // fprev now holds an increment, not a field a warm start could use
    if (resid) c->have_F = false;
    if (resid && inc->dF) HIPCHK(hipMemcpyAsync(inc->dF, c->fprev, 3 * R * sizeof(float), hipMemcpyDeviceToDevice, c->st));
  } else if (resid || keep_F) {
    c->have_F = true;
  }
  HIPCHK(pass(c, pdesc(PASS_Y_INV, fin, 1)));
  {
    PassDesc d = pdesc(PASS_X_INV_REAL, fin);
    d.real = phi_out;
    HIPCHK(pass(c, d));
  }

  if (want_info) {
    HIPCHK(hipMemcpyAsync(c->hacc, c->dacc, 128 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    int hctl[4] = {0, 0, 0, 0};
    if (dev_tol) HIPCHK(hipMemcpyAsync(hctl, c->ctl, 4 * sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (dev_tol) {
      k_done = hctl[1];
      if (hctl[2]) loc.status = PM_E_NONFINITE;
    }
    loc.iterations = k_done;
    loc.gN_norm = sqrt(c->hacc[0] / N3);
    if (resid) {
      loc.n_residuals = k_done - 1;
      for (int k = 1; k < k_done && k <= 64; ++k) {
        loc.residual[k - 1] = loc.gN_norm > 0.0 ? sqrt(c->hacc[k]) / loc.gN_norm : 0.0;
        if (!isfinite(loc.residual[k - 1])) loc.status = PM_E_NONFINITE;
      }
      if (p.tol > 0.0 && loc.status == PM_OK &&
          !(loc.n_residuals > 0 && loc.residual[loc.n_residuals - 1] <= p.tol))
        loc.status = PM_E_NOTCONV;
    }
    if (info) *info = loc;
  }
  return PM_OK;
}

// Tile sort of the particles, then (tile-piece kernels) the piece plan.
static hipError_t sort_and_plan(pm_ctx* c, const float* pos, int64_t n) {
  Timed t(c, PM_T_SORT);
  hipError_t e = sort_particles(c->kg, c->sb, pos, n, c->st, c->perm_n == n);
  c->perm_n = (e == hipSuccess) ? n : -1;
  if (e == hipSuccess && c->piece_ext && n > 0) e = piece_plan(c->pb, c->sb, c->N, c->st);
  return e;
}

static hipError_t deposit_any(pm_ctx* c, const float* pos, const float* mass, int64_t n, float* rho,
                              double* s_store) {
  Timed t(c, PM_T_DEPOSIT);
  if (c->piece_ext) return deposit_pieces(c->kg, c->sb, c->pb, pos, mass, n, rho, c->st);
  return deposit_sorted(c->kg, c->sb, pos, mass, n, rho, s_store, c->st);
}

static hipError_t gather_any(pm_ctx* c, const float* phi, float* pos, float* vel, float* acc, int64_t n,
                             float dt_kick, float dt_drift, int mode, const double* s_store) {
  Timed t(c, PM_T_GATHER);
  if (c->piece_ext) return gather_pieces(c->kg, c->sb, c->pb, phi, pos, vel, acc, n, dt_kick, dt_drift, mode, c->st);
  return gather_sorted(c->kg, c->sb, phi, pos, vel, acc, n, dt_kick, dt_drift, mode, s_store, c->st);
}

static pm_status check_ctx(pm_ctx* c, int64_t n) {
  if (!c) return inval("ctx is NULL");
  if (n < 0 || n > c->max_particles) return inval("particle count exceeds max_particles");
  return PM_OK;
}

pm_status aqual_solve(pm_ctx* c, const float* rho, const float* H0, float* phi, pm_solve_info* info) {
  if (!c) return inval("ctx is NULL");
  if (!rho || !phi) return inval("rho and phi are required");
  pm_status s = run_solve(c, rho, H0, phi, info, info != nullptr);
  if (s == PM_OK && info) info->bounds_flag = 0;
  return s;
}

pm_status pm_deposit(pm_ctx* c, const float* pos, const float* mass, int64_t n, float* rho) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (!rho || (n > 0 && (!pos || !mass))) return inval("NULL buffer");
  const long long R = (long long)c->N * c->N * c->N;
  { Timed t(c, PM_T_FILL); HIPCHK(fill_zero(rho, R, c->st)); }
  HIPCHK(sort_and_plan(c, pos, n));
  HIPCHK(deposit_any(c, pos, mass, n, rho, nullptr));
  return PM_OK;
}

// ---------------------------------------------------------------------------
// Deposit without device allocation (pm_deposit_noalloc)
// ---------------------------------------------------------------------------
// Its scratch (the ball table and the sort buffers) is a fixed static device
// array.  Host code never passes the array's name to a kernel: each device's
// address of it is taken once with hipGetSymbolAddress and used from then on.
namespace {
constexpr int64_t kNaMaxParticles = (int64_t)1 << 20;
constexpr int kNaMaxNpad = 512;
constexpr size_t kNaMaxTiles = (size_t)(kNaMaxNpad / 8) * (kNaMaxNpad / 8) * (kNaMaxNpad / 8);
constexpr size_t kNaMaxBall = 21 * 21 * 21;        // cutoff * sigma <= 10 cells
constexpr size_t na_round(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaBallBytes = na_round(kNaMaxBall * sizeof(int));
constexpr size_t kNaSortInts = 4 * (size_t)kNaMaxParticles + 2 * (kNaMaxTiles + 1) + (kNaMaxTiles + 1023) / 1024 + 16;
constexpr size_t kNaScratchBytes = kNaBallBytes + na_round(kNaSortInts * sizeof(int));
constexpr int kNaMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

static std::mutex g_na_mutex;
static void* g_na_ptr[kNaMaxDevices];
static int g_na_lds[kNaMaxDevices];

// Ball offsets |d|^2 < R2 in the order of make_ball (dz slowest, dx fastest),
// packed as in the context's table; one block compacts 1024 candidates at a
// time with ballots.
__global__ __launch_bounds__(1024) void k_ball_table(int m, double R2, int* out) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int side = 2 * m + 1, total = side * side * side;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < total; c0 += 1024) {
    const int c = c0 + (int)threadIdx.x;
    bool in = false;
    int e = 0;
    if (c < total) {
      const int dx = c % side - m, dy = (c / side) % side - m, dz = c / (side * side) - m;
      in = (double)(dx * dx + dy * dy + dz * dz) < R2;
      e = (dx + 16) | ((dy + 16) << 8) | ((dz + 16) << 16);
    }
    const unsigned long long bal = __ballot(in);
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int before = base;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (in) out[before + __popcll(bal & ((1ull << lane) - 1ull))] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w = 0; w < 16; ++w) t += wsum[w];
      base += t;
    }
    __syncthreads();
  }
}

pm_status pm_deposit_noalloc(const pm_params* p, const float* pos, const float* mass, int64_t n, float* rho,
                             void* stream) {
  pm_status s = check_params(p);
  if (s != PM_OK) return s;
  if (n < 0 || n > kNaMaxParticles) return inval("pm_deposit_noalloc takes at most 2^20 particles");
  if (p->n_pad > kNaMaxNpad) return inval("pm_deposit_noalloc takes n_pad <= 512");
  if (!rho || (n > 0 && (!pos || !mass))) return inval("NULL buffer");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) return inval("device id out of range");
  void* base = nullptr;
  int lds_max = 0;
  {
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
      void* ptr = nullptr;
      HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      HIPCHK(hipDeviceGetAttribute(&g_na_lds[dev], hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      g_na_ptr[dev] = ptr;
    }
    base = g_na_ptr[dev];
    lds_max = g_na_lds[dev];
  }
  // ball of radius R (no host buffer: count here, build the table on the device)
  const double R = p->cutoff * p->sigma;
  const int m = (int)floor(R), ext = ball_extent(R);
  int nball = 0;
  for (int dz = -m; dz <= m; ++dz)
    for (int dy = -m; dy <= m; ++dy)
      for (int dx = -m; dx <= m; ++dx)
        if ((double)(dx * dx + dy * dy + dz * dz) < R * R) ++nball;
  const size_t te = 8 + 2 * (size_t)ext;
  const bool priv = 4 * te * te * te * sizeof(float) <= 96 * 1024;
  const size_t lds_need = sizeof(float) * (((size_t)nball + 3 & ~(size_t)3) + (priv ? 4 : 1) * te * te * te);
  if (lds_need + 4 * 512 * sizeof(int) + 64 > (size_t)lds_max) return inval("kernel ball too large for the LDS of this device");

  const int N = p->n_pad;
  const double s_px = p->box / p->n;
  KernelGeom kg{};
  kg.N = N;
  kg.n = p->n;
  kg.s = (float)s_px;
  kg.inv_s = 1.0 / s_px;
  kg.inv2sig2 = (float)(1.0 / (2.0 * p->sigma * p->sigma));
  kg.ext = ext;
  kg.nball = nball;
  kg.ball = static_cast<int*>(base);
  kg.analytic = (p->flags & PM_F_ANALYTIC_NORM) ? 1 : 0;
  kg.analytic_norm = pow(2.0 * M_PI, 1.5) * p->sigma * p->sigma * p->sigma;
  kg.private_tiles = priv ? 1 : 0;

  const size_t ntiles = (size_t)(N / 8) * (N / 8) * (N / 8);
  const size_t mp = (size_t)(n > 0 ? n : 1);
  int* ib = reinterpret_cast<int*>(static_cast<char*>(base) + kNaBallBytes);
  SortBufs sb{};
  sb.keys = ib; ib += mp;
  sb.rank = ib; ib += mp;
  sb.perm = ib; ib += mp;
  sb.skey = ib; ib += mp;
  sb.counts = ib; ib += ntiles + 1;
  sb.offsets = ib; ib += ntiles + 1;
  sb.blocksums = ib; ib += (ntiles + 1023) / 1024;
  sb.flags = ib;
  sb.ntiles = (int)ntiles;

  hipLaunchKernelGGL(k_ball_table, dim3(1), dim3(1024), 0, st, m, R * R, const_cast<int*>(kg.ball));
  HIPCHK(hipGetLastError());
  HIPCHK(fill_zero(reinterpret_cast<float*>(sb.flags), 16, st));
  HIPCHK(fill_zero(rho, (long long)N * N * N, st));
  HIPCHK(sort_particles(kg, sb, pos, n, st));
  HIPCHK(deposit_sorted(kg, sb, pos, mass, n, rho, nullptr, st));
  return PM_OK;
}

pm_status smooth_accel(pm_ctx* c, const float* phi, const float* pos, int64_t n, float* acc) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (!phi || (n > 0 && (!pos || !acc))) return inval("NULL buffer");
  HIPCHK(sort_and_plan(c, pos, n));
  HIPCHK(gather_any(c, phi, const_cast<float*>(pos), nullptr, acc, n, 0.f, 0.f, 0, nullptr));
  return PM_OK;
}

pm_status interp_push(pm_ctx* c, const float* phi, float* pos, float* vel, int64_t n, double dt_kick,
                      double dt_drift) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (!phi || (n > 0 && (!pos || !vel))) return inval("NULL buffer");
  HIPCHK(sort_and_plan(c, pos, n));
  HIPCHK(gather_any(c, phi, pos, vel, nullptr, n, (float)dt_kick, (float)dt_drift, 1, nullptr));
  return PM_OK;
}

pm_status pm_step(pm_ctx* c, float* pos, float* vel, const float* mass, int64_t n, double dt,
                  pm_solve_info* info) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (n > 0 && (!pos || !vel || !mass)) return inval("NULL buffer");
  const long long R = (long long)c->N * c->N * c->N;
  if (info) HIPCHK(fill_zero(reinterpret_cast<float*>(c->sb.flags), 1, c->st));
  { Timed t(c, PM_T_FILL); HIPCHK(fill_zero(c->rho, R, c->st)); }
  HIPCHK(sort_and_plan(c, pos, n));
  HIPCHK(deposit_any(c, pos, mass, n, c->rho, c->snorm));
  s = run_solve(c, c->rho, nullptr, c->phi, info, info != nullptr);
  if (s != PM_OK) return s;
  HIPCHK(gather_any(c, c->phi, pos, vel, nullptr, n, (float)dt, (float)dt, 1, c->snorm));
  if (info) {
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, c->sb.flags, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    info->bounds_flag = flag > 0 ? 1 : 0;
  }
  return PM_OK;
}

pm_status pm_step_capture(pm_ctx* c, float* pos, float* vel, const float* mass, int64_t n, double dt) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (n > 0 && (!pos || !vel || !mass)) return inval("NULL buffer");
  if (!c->st) return inval("capture needs the context to run on a created stream, not the null stream");
  if (c->timing) return inval("switch event timing off before capturing");
  if ((c->p.flags & PM_F_WARM_START) && !c->have_F)
    return inval("warm start: run one pm_step before capturing, so the captured solve starts warm");
  if (c->step_graph) {
    (void)hipGraphExecDestroy(c->step_graph);
    c->step_graph = nullptr;
  }
  HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  s = pm_step(c, pos, vel, mass, n, dt, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->st, &g);
  if (s != PM_OK) {
    if (e == hipSuccess && g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return dev_fail(e, "hipStreamEndCapture");
  const hipError_t ei = hipGraphInstantiate(&c->step_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->step_graph = nullptr;
    return dev_fail(ei, "hipGraphInstantiate");
  }
  return PM_OK;
}

pm_status pm_step_replay(pm_ctx* c, int32_t count) {
  if (!c) return inval("ctx is NULL");
  if (!c->step_graph) return inval("no captured step on this context");
  if (count < 0) return inval("count must be >= 0");
  for (int32_t i = 0; i < count; ++i) HIPCHK(hipGraphLaunch(c->step_graph, c->st));
  return PM_OK;
}

pm_status pm_diagnostics(pm_ctx* c, const float* pos, const float* vel, const float* mass, int64_t n,
                         const float* phi, double* out) {
  pm_status s = check_ctx(c, n);
  if (s != PM_OK) return s;
  if (!out || (n > 0 && (!pos || !vel || !mass))) return inval("NULL buffer");
  HIPCHK(fill_zero(reinterpret_cast<float*>(c->dacc + 80), 2 * 10, c->st));
  HIPCHK(fill_zero(reinterpret_cast<float*>(c->sb.flags), 1, c->st));
  HIPCHK(diagnostics(c->kg, pos, vel, mass, phi, n, c->dacc + 80, c->st));
  HIPCHK(sort_particles(c->kg, c->sb, pos, n, c->st));
  int flag = 0;
  HIPCHK(hipMemcpyAsync(c->hacc + 80, c->dacc + 80, 9 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(&flag, c->sb.flags, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  for (int i = 0; i < 9; ++i) out[i] = c->hacc[80 + i];
  if (!phi) out[8] = 0.0;
  out[9] = (double)flag;
  return PM_OK;
}

pm_status pm_fft_r2c(pm_ctx* c, const float* in, void* out) {
  if (!c || !in || !out) return inval("NULL argument");
  float2* sp = static_cast<float2*>(out);
  PassDesc d = pdesc(PASS_X_FWD_REAL, sp);
  d.real = const_cast<float*>(in);
  HIPCHK(pass(c, d));
  HIPCHK(pass(c, pdesc(PASS_Y_FWD, sp, 1)));
  PassDesc z = pdesc(PASS_Z_FWD, sp);
  z.z = zargs(c);
  z.z.spec = sp;
  z.z.nc = 1;
  HIPCHK(pass(c, z));
  return PM_OK;
}

pm_status pm_fft_c2r(pm_ctx* c, const void* in, float* out) {
  if (!c || !in || !out) return inval("NULL argument");
  const size_t C = (size_t)c->N * c->N * c->P;
  HIPCHK(hipMemcpyAsync(c->spec, in, C * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
  PassDesc z = pdesc(PASS_Z_INV, c->spec);
  z.z = zargs(c);
  z.z.nc = 1;
  HIPCHK(pass(c, z));
  HIPCHK(pass(c, pdesc(PASS_Y_INV, c->spec, 1)));
  PassDesc d = pdesc(PASS_X_INV_REAL, c->spec);
  d.real = out;
  HIPCHK(pass(c, d));
  return PM_OK;
}

pm_status pm_set_timing(pm_ctx* c, int enable) {
  if (!c) return inval("ctx is NULL");
  c->timing = enable != 0;
  return PM_OK;
}

pm_status pm_read_timing(pm_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return inval("NULL argument");
  HIPCHK(hipStreamSynchronize(c->st));
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]));
    const int k = c->ev_kind[i / 2];
    total_ms[k] += ms;
    launches[k] += 1;
  }
  c->ev_used = 0;
  return PM_OK;
}

// ---------------------------------------------------------------------------
// Newton potential alone, and a solve that also returns its last F
// ---------------------------------------------------------------------------

pm_status pm_newton_potential(pm_ctx* c, const float* rho, float* phiN) {
  if (!c) return inval("ctx is NULL");
  if (!rho || !phiN) return inval("rho and phiN are required");
  PassDesc d = pdesc(PASS_X_FWD_REAL, c->spec);
  d.real = const_cast<float*>(rho);
  d.dip = c->dip;
  HIPCHK(pass(c, d));
  HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->spec, 1)));
  PassDesc z = pdesc(PASS_Z_POISSON, c->spec);
  z.z = zargs(c);
  HIPCHK(pass(c, z));
  HIPCHK(pass(c, pdesc(PASS_Y_INV, c->spec, 1)));
  PassDesc x = pdesc(PASS_X_INV_REAL, c->spec);
  x.real = phiN;
  HIPCHK(pass(c, x));
  return PM_OK;
}

pm_status pm_set_external_field(pm_ctx* c, double gx, double gy, double gz) {
  if (!c) return inval("ctx is NULL");
  if (!isfinite(gx) || !isfinite(gy) || !isfinite(gz)) return inval("external field must be finite");
  // A sheet pair of +-rho_c per cell on adjacent planes gives the periodic box
  // a uniform Newtonian field 4 pi G rho_c s^2 / L in its bulk (the field has
  // zero mean over the period, and the sheets carry a potential jump of
  // 4 pi G rho_c s^2), pointing from the +rho_c plane to the -rho_c plane.
  const double s = c->p.box / c->p.n, L = c->N * s;
  const double k = L / (4.0 * M_PI * c->p.G * s * s);
  c->dip.x = (float)(gx * k);
  c->dip.y = (float)(gy * k);
  c->dip.z = (float)(gz * k);
  return PM_OK;
}

pm_status pm_apparent_density(pm_ctx* c, const float* phi, float* rho_a) {
  if (!c) return inval("ctx is NULL");
  if (!phi || !rho_a) return inval("phi and rho_a are required");
  PassDesc d = pdesc(PASS_X_FWD_REAL, c->spec);
  d.real = const_cast<float*>(phi);
  HIPCHK(pass(c, d));
  HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->spec, 1)));
  PassDesc z = pdesc(PASS_Z_APPARENT, c->spec);
  z.z = zargs(c);
  HIPCHK(pass(c, z));
  HIPCHK(pass(c, pdesc(PASS_Y_INV, c->spec, 1)));
  PassDesc x = pdesc(PASS_X_INV_REAL, c->spec);
  x.real = rho_a;
  HIPCHK(pass(c, x));
  return PM_OK;
}

pm_status aqual_solve_field(pm_ctx* c, const float* rho, const float* H0, float* phi, float* F,
                            pm_solve_info* info) {
  if (!c) return inval("ctx is NULL");
  if (!rho || !phi || !F) return inval("rho, phi and F are required");
  if (!c->fprev) return inval("aqual_solve_field needs a context created with PM_F_RESIDUAL or tol > 0");
  pm_status s = run_solve(c, rho, H0, phi, info, info != nullptr);
  if (s != PM_OK) return s;
  if (info) info->bounds_flag = 0;
  const size_t R = (size_t)c->N * c->N * c->N;
  HIPCHK(hipMemcpyAsync(F, c->fprev, 3 * R * sizeof(float), hipMemcpyDeviceToDevice, c->st));
  return PM_OK;
}

pm_status aqual_solve_increment(pm_ctx* c, const float* d_rho, const float* F, const float* gM, int32_t storage,
                                float* d_phi, float* d_F, pm_solve_info* info) {
  if (!c) return inval("ctx is NULL");
  if (!d_rho || !F || !gM || !d_phi) return inval("d_rho, F, gM and d_phi are required");
  if (storage != PM_STORE_FP32 && storage != PM_STORE_FP16) return inval("storage must be PM_STORE_FP32 or PM_STORE_FP16");
  Increment inc{F, gM, storage == PM_STORE_FP16 ? 1 : 0, d_F};
  pm_status s = run_solve(c, d_rho, nullptr, d_phi, info, info != nullptr, &inc);
  if (s == PM_OK && info) info->bounds_flag = 0;
  return s;
}

pm_status pm_potential_field(pm_ctx* c, const float* phi, float* g) {
  if (!c) return inval("ctx is NULL");
  if (!phi || !g) return inval("phi and g are required");
  const long long R = (long long)c->N * c->N * c->N;
  PassDesc d = pdesc(PASS_X_FWD_REAL, c->spec);
  d.real = const_cast<float*>(phi);
  HIPCHK(pass(c, d));
  HIPCHK(pass(c, pdesc(PASS_Y_FWD, c->spec, 1)));
  PassDesc z = pdesc(PASS_Z_GRAD, c->spec);
  z.z = zargs(c);
  HIPCHK(pass(c, z));
  HIPCHK(pass(c, pdesc(PASS_Y_INV, c->spec, 3)));
  PassDesc x = pdesc(PASS_X_INV_REAL3, c->spec);
  x.real = g;
  x.real_cs = R;
  HIPCHK(pass(c, x));
  return PM_OK;
}

// ---------------------------------------------------------------------------
// Learned starting guess
// ---------------------------------------------------------------------------

struct pm_net {
  net::Buffers b;
  hipStream_t st = nullptr;
  int adam_step = 0;
  std::vector<void*> allocs;
};

template <typename T>
static pm_status nalloc(pm_net* m, T** ptr, size_t count) {
  void* v = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) {
    snprintf(g_err, sizeof g_err, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
    return PM_E_NOMEM;
  }
  m->allocs.push_back(v);
  *ptr = static_cast<T*>(v);
  return PM_OK;
}

int64_t pm_net_param_count(void) { return net::param_count(); }

pm_status pm_net_destroy(pm_net* m) {
  if (!m) return PM_OK;
  (void)(m->st ? hipStreamSynchronize(m->st) : hipDeviceSynchronize());
  for (void* v : m->allocs) (void)hipFree(v);
  delete m;
  return PM_OK;
}

pm_status pm_net_create(int32_t n, int32_t max_batch, void* stream, pm_net** out) {
  if (!out) return inval("out is NULL");
  *out = nullptr;
  if (!pow2(n) || n < 8 || n > 512) return inval("net size n must be a power of two in [8, 512]");
  if (max_batch < 1 || max_batch > 64) return inval("max_batch must be in [1, 64]");
  pm_net* m = new pm_net();
  m->st = static_cast<hipStream_t>(stream);
  net::Buffers& b = m->b;
  b.n = n;
  b.max_batch = max_batch;
  const size_t V1 = (size_t)net::level_voxels(n, 0) * max_batch;
  const size_t V2 = (size_t)net::level_voxels(n, 1) * max_batch;
  const size_t V3 = (size_t)net::level_voxels(n, 2) * max_batch;
  const size_t P = (size_t)net::param_count();
#define NALLOC(ptr, cnt)                                   \
  do {                                                     \
    pm_status s_ = nalloc(m, &(ptr), (cnt));               \
    if (s_ != PM_OK) { pm_net_destroy(m); return s_; }     \
  } while (0)
  NALLOC(b.params, P);
  NALLOC(b.grads, P);
  NALLOC(b.adam_m, P);
  NALLOC(b.adam_v, P);
  for (int l = 0; l < net::NLAYER; ++l) {
    const size_t cnt = (size_t)net::kLayers[l].taps * net::kLayers[l].cin_p * net::kLayers[l].cout;
    NALLOC(b.wf[l], cnt);
    NALLOC(b.wb[l], cnt);
  }
  NALLOC(b.x, 16 * V1);
  NALLOC(b.a1, 16 * V1);
  NALLOC(b.s1, 16 * V1);
  NALLOC(b.a5, 16 * V1);
  NALLOC(b.d1, 16 * V1);
  NALLOC(b.g16a, 16 * V1);
  NALLOC(b.g16b, 16 * V1);
  NALLOC(b.gc1, 48 * V1);
  NALLOC(b.p1, 16 * V2);
  NALLOC(b.a2, 32 * V2);
  NALLOC(b.s2, 32 * V2);
  NALLOC(b.a4, 32 * V2);
  NALLOC(b.d2, 32 * V2);
  NALLOC(b.g32a, 32 * V2);
  NALLOC(b.g32b, 32 * V2);
  NALLOC(b.gc2, 96 * V2);
  NALLOC(b.gp1, 16 * V2);
  NALLOC(b.p2, 32 * V3);
  NALLOC(b.a3, 64 * V3);
  NALLOC(b.b3, 64 * V3);
  NALLOC(b.g64a, 64 * V3);
  NALLOC(b.g64b, 64 * V3);
  NALLOC(b.gp2, 32 * V3);
  NALLOC(b.yhat, 3 * V1);
  NALLOC(b.target, 3 * V1);
  NALLOC(b.rms, (size_t)max_batch);
  NALLOC(b.sums, (size_t)max_batch + 64);
  // weight-gradient partial sums (the launch picks its number of brick groups
  // to fit; the largest layer, b3b at 64 x 64, still gets 606)
  b.partial_floats = net::kWgradPartialFloats;
  NALLOC(b.partial, (size_t)b.partial_floats);
  size_t wmax = 0;   // largest weight tensor (b3b: 27 x 64 x 64)
  for (int l = 0; l < net::NLAYER; ++l) {
    const size_t cnt = (size_t)net::kLayers[l].taps * net::kLayers[l].cin * net::kLayers[l].cout;
    wmax = cnt > wmax ? cnt : wmax;
  }
  NALLOC(b.partial2, (size_t)net::kWgradSlices * wmax);
  b.dpartial_count = 1024 * 52;
  NALLOC(b.dpartial, (size_t)b.dpartial_count);
#undef NALLOC
  // zero-initialised parameters and optimiser state until pm_net_set_params
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemsetAsync(b.params, 0, P * sizeof(float), m->st);
  if (e == hipSuccess) e = hipMemsetAsync(b.adam_m, 0, P * sizeof(float), m->st);
  if (e == hipSuccess) e = hipMemsetAsync(b.adam_v, 0, P * sizeof(float), m->st);
  if (e == hipSuccess) e = hipMemsetAsync(b.rms, 0, (size_t)max_batch * sizeof(double), m->st);
  if (e == hipSuccess) e = net::pack_weights(b, m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  if (e != hipSuccess) {
    pm_net_destroy(m);
    return dev_fail(e, "pm_net_create");
  }
  *out = m;
  return PM_OK;
}

pm_status pm_net_set_params(pm_net* m, const float* params) {
  if (!m || !params) return inval("NULL argument");
  const size_t P = (size_t)net::param_count();
  HIPCHK(hipMemcpyAsync(m->b.params, params, P * sizeof(float), hipMemcpyHostToDevice, m->st));
  HIPCHK(hipMemsetAsync(m->b.adam_m, 0, P * sizeof(float), m->st));
  HIPCHK(hipMemsetAsync(m->b.adam_v, 0, P * sizeof(float), m->st));
  m->adam_step = 0;
  HIPCHK(net::pack_weights(m->b, m->st));
  HIPCHK(hipStreamSynchronize(m->st));
  return PM_OK;
}

pm_status pm_net_get_params(pm_net* m, float* params) {
  if (!m || !params) return inval("NULL argument");
  HIPCHK(hipMemcpyAsync(params, m->b.params, (size_t)net::param_count() * sizeof(float), hipMemcpyDeviceToHost,
                        m->st));
  HIPCHK(hipStreamSynchronize(m->st));
  return PM_OK;
}

pm_status pm_net_get_grads(pm_net* m, float* grads) {
  if (!m || !grads) return inval("NULL argument");
  HIPCHK(hipMemcpyAsync(grads, m->b.grads, (size_t)net::param_count() * sizeof(float), hipMemcpyDeviceToHost,
                        m->st));
  HIPCHK(hipStreamSynchronize(m->st));
  return PM_OK;
}

static pm_status check_slot(pm_net* m, int32_t slot) {
  if (!m) return inval("net is NULL");
  if (slot < 0 || slot >= m->b.max_batch) return inval("slot out of range");
  return PM_OK;
}

static pm_status check_pair(pm_ctx* c, pm_net* m) {
  if (!c || !m) return inval("NULL argument");
  if (c->N != 2 * m->b.n && c->N != 4 * m->b.n)
    return inval("net size n must be a half or a quarter of the context's n_pad");
  return PM_OK;
}

pm_status pm_net_input(pm_ctx* c, pm_net* m, const float* phiN, int32_t slot) {
  pm_status s = check_pair(c, m);
  if (s == PM_OK) s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!phiN) return inval("phiN is NULL");
  const double s_px = c->p.box / c->p.n;
  HIPCHK(net::features(m->b, slot, phiN, 0.5 / s_px, c->p.a0, c->N / m->b.n, c->st));
  return PM_OK;
}

pm_status pm_net_target(pm_ctx* c, pm_net* m, const float* phiN, const float* F, int32_t slot) {
  pm_status s = check_pair(c, m);
  if (s == PM_OK) s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!phiN || !F) return inval("phiN and F are required");
  const double s_px = c->p.box / c->p.n;
  HIPCHK(net::target_from_field(m->b, slot, phiN, F, 0.5 / s_px, c->N / m->b.n, c->st));
  return PM_OK;
}

pm_status pm_net_set_input(pm_net* m, int32_t slot, const float* x) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!x) return inval("x is NULL");
  HIPCHK(net::set_input(m->b, slot, x, m->st));
  return PM_OK;
}

pm_status pm_net_get_input(pm_net* m, int32_t slot, float* x) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!x) return inval("x is NULL");
  HIPCHK(net::get_input(m->b, slot, x, m->st));
  return PM_OK;
}

pm_status pm_net_set_target(pm_net* m, int32_t slot, const float* y) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!y) return inval("y is NULL");
  const size_t V = (size_t)net::level_voxels(m->b.n, 0);
  HIPCHK(hipMemcpyAsync(m->b.target + (size_t)slot * 3 * V, y, 3 * V * sizeof(float), hipMemcpyDeviceToDevice,
                        m->st));
  return PM_OK;
}

pm_status pm_net_get_target(pm_net* m, int32_t slot, float* y) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!y) return inval("y is NULL");
  const size_t V = (size_t)net::level_voxels(m->b.n, 0);
  HIPCHK(hipMemcpyAsync(y, m->b.target + (size_t)slot * 3 * V, 3 * V * sizeof(float), hipMemcpyDeviceToDevice,
                        m->st));
  return PM_OK;
}

pm_status pm_net_get_tensor(pm_net* m, int32_t which, int32_t slot, float* out) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!out) return inval("out is NULL");
  if (which < 0 || which > 22) return inval("unknown tensor");
  HIPCHK(net::get_tensor(m->b, which, slot, out, m->st));
  return PM_OK;
}

pm_status pm_net_output(pm_net* m, int32_t slot, float* y) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!y) return inval("y is NULL");
  const size_t V = (size_t)net::level_voxels(m->b.n, 0);
  HIPCHK(hipMemcpyAsync(y, m->b.yhat + (size_t)slot * 3 * V, 3 * V * sizeof(float), hipMemcpyDeviceToDevice,
                        m->st));
  return PM_OK;
}

pm_status pm_net_get_rms(pm_net* m, int32_t slot, double* rms) {
  pm_status s = check_slot(m, slot);
  if (s != PM_OK) return s;
  if (!rms) return inval("rms is NULL");
  HIPCHK(hipMemcpyAsync(rms, m->b.rms + slot, sizeof(double), hipMemcpyDeviceToHost, m->st));
  HIPCHK(hipStreamSynchronize(m->st));
  return PM_OK;
}

pm_status pm_net_run(pm_net* m, int32_t batch) {
  if (!m) return inval("net is NULL");
  if (batch < 1 || batch > m->b.max_batch) return inval("batch out of range");
  HIPCHK(net::forward(m->b, batch, m->st));
  return PM_OK;
}

pm_status pm_net_backward(pm_net* m, int32_t batch, double* loss) {
  if (!m) return inval("net is NULL");
  if (batch < 1 || batch > m->b.max_batch) return inval("batch out of range");
  HIPCHK(net::forward(m->b, batch, m->st));
  HIPCHK(net::loss_backward(m->b, batch, m->st));
  if (loss) {
    HIPCHK(hipMemcpyAsync(loss, m->b.sums + m->b.max_batch, sizeof(double), hipMemcpyDeviceToHost, m->st));
    HIPCHK(hipStreamSynchronize(m->st));
  }
  return PM_OK;
}

pm_status pm_net_adam(pm_net* m, float lr) {
  if (!m) return inval("net is NULL");
  if (!(lr >= 0.0f) || !isfinite(lr)) return inval("lr must be finite and >= 0");
  m->adam_step += 1;
  HIPCHK(net::adam(m->b, lr, 0.9f, 0.999f, 1e-8f, m->adam_step, m->st));
  return PM_OK;
}

pm_status pm_net_train_step(pm_net* m, int32_t batch, float lr, double* loss) {
  pm_status s = pm_net_backward(m, batch, loss);
  if (s != PM_OK) return s;
  return pm_net_adam(m, lr);
}

pm_status aqual_solve_learned(pm_ctx* c, pm_net* m, const float* rho, float* phi, pm_solve_info* info) {
  pm_status s = check_pair(c, m);
  if (s != PM_OK) return s;
  if (!rho || !phi) return inval("rho and phi are required");
  if (phi == c->phi) return inval("phi is the context's internal grid");
  s = run_solve(c, rho, nullptr, phi, info, info != nullptr, nullptr, &m->b);
  if (s == PM_OK && info) info->bounds_flag = 0;
  return s;
}

pm_status pm_net_forward(pm_ctx* c, pm_net* m, const float* phiN, float* H0) {
  pm_status s = check_pair(c, m);
  if (s != PM_OK) return s;
  if (!phiN || !H0) return inval("phiN and H0 are required");
  const double s_px = c->p.box / c->p.n;
  HIPCHK(net::features(m->b, 0, phiN, 0.5 / s_px, c->p.a0, c->N / m->b.n, c->st));
  HIPCHK(net::forward(m->b, 1, c->st));
  HIPCHK(net::start_field(m->b, H0, c->N / m->b.n, c->st));
  return PM_OK;
}
