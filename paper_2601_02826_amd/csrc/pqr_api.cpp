// libpqr C ABI: context, set-up (encode, column statistics, block step sizes)
// and the FS-QRPPA driver (Algorithm 1) with its FP64 stopping certificate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/pqr.h"
#include "pqr_kernels.h"
#include <rocprofiler-sdk-roctx/roctx.h>

using namespace pqr;

struct pqr_ctx {
  std::string err;
  Geom g{};
  int standardize = 1;
  pqr_options opt{};
  hipStream_t s = nullptr;
  int G = 0;                    // total blocks (intercept block included when separate)
  int Gf = 0;                   // feature blocks
  int icpt_own = 1;             // intercept forms block 0 on its own
  std::vector<int> bounds;      // feature-column boundaries of the G blocks (G+1)
  std::vector<int> gbound;      // group boundaries of the Gf feature blocks (Gf+1)
  std::vector<int> gblock_h;    // block of every column group
  std::vector<double> Lambda;   // Lambda_max(X~_b^T X~_b) estimates (G)
  int smax = 256, min_per = 4;

  // design and column parameters
  uint8_t* X = nullptr;
  double *cm_d = nullptr, *cinv_d = nullptr, *sd_d = nullptr;
  float *cm_f = nullptr, *cinv_f = nullptr;
  int* iota = nullptr;

  // iteration state (type given by opt.iter_prec)
  void *beta = nullptr, *clam_t = nullptr, *geta_t = nullptr, *gnorm = nullptr,
       *partial = nullptr, *y_t = nullptr, *z = nullptr, *theta = nullptr, *r = nullptr,
       *cm_t = nullptr, *cinv_t = nullptr;
  int *gflag = nullptr, *list = nullptr, *bcnt = nullptr;
  double* bpart = nullptr;
  double* bnrm = nullptr;
  Ctl* ctl = nullptr;
  Ctl* ctl_kkt = nullptr;

  // certificate buffers (FP64)
  double *y_d = nullptr, *theta_p = nullptr, *beta_d = nullptr, *clam_d = nullptr, *v_d = nullptr,
         *gpart = nullptr, *partial64 = nullptr, *bpart64 = nullptr, *out_d = nullptr,
         *scratch64 = nullptr, *bt_out = nullptr;
  void* beta_best = nullptr;     // coefficients of the best primal iterate seen (iterate type)
  void* z_best = nullptr;        // z of that iterate (n_pad, iterate type)
  void* theta_best = nullptr;    // theta of the iterate with the best dual value (n_pad)
  int64_t bpart64_len = 0;
  double* out_h = nullptr;   // pinned

  bool have_state = false;
  double state_mu = 0.0;
  std::vector<void*> allocs;
  std::vector<hipEvent_t> events;   // 2 per iteration of a chunk when profiling
  // captured iteration chunk (launch_mode 0): its graph, the private capture stream
  // and the key it was captured for
  hipStream_t cap_s = nullptr;
  hipGraph_t chunk_graph = nullptr;
  hipGraphExec_t chunk_exec = nullptr;
  int64_t chunk_len = 0;
  int chunk_prec = -1;
  IterParams chunk_ip{};
  bool graph_failed = false;
  int batch_kp = 0;                 // capacity of the batched buffers (right-hand sides)
  BatchBufs bb{};
  float* btheta_best = nullptr;     // Kp x n_pad: per right-hand side, theta of its best dual
  // batched launch variants chosen by the autotuner, per padded batch width Kp, with
  // the mean kernel times (ms) of every candidate
  struct TileChoice {
    BatchTiles tiles;
    bool bgemm_done = false, baxpy_done = false;
    std::vector<double> bgemm_ms, baxpy_ms;
    int64_t union_cols = 0;   // union of nonzero columns when the union product was timed
  };
  std::map<int, TileChoice> tiles;
  double* w_d = nullptr;            // p_pad penalty weights in FP64 (batched certificates)
  float* yb = nullptr;              // n_pad y in FP32 (batched iterations)
  float* feats = nullptr;           // p_pad x 4 features of the scoring network
  float* mlp_out = nullptr;         // p_pad x 2 network outputs
  double* cert4 = nullptr;          // 4 x n_pad projected thetas (batched certificates)
  double* out4 = nullptr;           // 4 x 8 certificate outputs
  double* gmax4 = nullptr;          // 4 x ngroups dual-ratio partials
  int8_t* cdig = nullptr;           // exact batched certificate: 4 x 128 x n_pad digits
  int* ctq = nullptr;               // n_pad quantised theta (scratch)
  double* cgmax = nullptr;          // 128 x group sets dual-ratio partials
  double* clamk = nullptr;          // 128 lambda_k of the pass
  double* cunit = nullptr;          // 128 quantisation steps of the pass
  double* cout = nullptr;           // 128 x 8 certificate outputs
  int max_code = -1;                // largest byte of an int8 store (-1: not measured)
  // unpenalized feature columns (weight 0) of the current problem, for the certificate
  std::vector<int64_t> unpen;
  bool unpen_ready = false;
  int64_t* unpen_cols_d = nullptr;
  double *unpen_x = nullptr, *unpen_c = nullptr, *unpen_u = nullptr;
  int64_t unpen_cap = 0;
  std::vector<double> unpen_chol;   // Cholesky factor of X~_U^T X~_U (+ tiny ridge), row-major
  std::vector<double> unpen_diag;   // ||x~_j||^2
};

namespace {

// A roctx range around an entry point (visible with rocprofv3 --marker-trace).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return PQR_ERR_DEVICE;                                                      \
    }                                                                             \
  } while (0)

template <typename P>
pqr_status dalloc(pqr_ctx* ctx, P** p, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes < 256 ? 256 : bytes) != hipSuccess) {
    ctx->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    (void)hipGetLastError();
    return PQR_ERR_OOM;
  }
  ctx->allocs.push_back(q);
  *p = static_cast<P*>(q);
  return PQR_OK;
}

#define TRY(expr)                  \
  do {                             \
    pqr_status st_ = (expr);       \
    if (st_ != PQR_OK) return st_; \
  } while (0)

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

bool finite_all(const double* a, int64_t m) {
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Largest eigenvalue of the symmetric tridiagonal (alpha, beta) by cyclic
// Jacobi on the dense matrix, plus the Lanczos residual bound |beta_k s_k|.
double ritz_upper(const double* alpha, const double* beta, int k) {
  std::vector<double> A((size_t)k * k, 0.0), V((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    A[i * k + i] = alpha[i];
    V[i * k + i] = 1.0;
    if (i + 1 < k) A[i * k + i + 1] = A[(i + 1) * k + i] = beta[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += A[i * k + j] * A[i * k + j];
    if (off < 1e-30) break;
    for (int pi = 0; pi < k; ++pi)
      for (int qi = pi + 1; qi < k; ++qi) {
        const double apq = A[pi * k + qi];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[pi * k + pi], aqq = A[qi * k + qi];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int m = 0; m < k; ++m) {
          const double amp = A[m * k + pi], amq = A[m * k + qi];
          A[m * k + pi] = c * amp - s * amq;
          A[m * k + qi] = s * amp + c * amq;
        }
        for (int m = 0; m < k; ++m) {
          const double apm = A[pi * k + m], aqm = A[qi * k + m];
          A[pi * k + m] = c * apm - s * aqm;
          A[qi * k + m] = s * apm + c * aqm;
        }
        for (int m = 0; m < k; ++m) {
          const double vmp = V[m * k + pi], vmq = V[m * k + qi];
          V[m * k + pi] = c * vmp - s * vmq;
          V[m * k + qi] = s * vmp + c * vmq;
        }
      }
  }
  int best = 0;
  for (int i = 1; i < k; ++i)
    if (A[i * k + i] > A[best * k + best]) best = i;
  const double resid = std::fabs(beta[k - 1] * V[(k - 1) * k + best]);
  return A[best * k + best] + resid;
}

template <typename T>
IterBufs<T> bufs(pqr_ctx* ctx) {
  IterBufs<T> b;
  b.beta = (T*)ctx->beta;
  b.cm = (const T*)ctx->cm_t;
  b.cinv = (const T*)ctx->cinv_t;
  b.clam = (const T*)ctx->clam_t;
  b.geta = (const T*)ctx->geta_t;
  b.gnorm = (T*)ctx->gnorm;
  b.gflag = ctx->gflag;
  b.list = ctx->list;
  b.partial = (double*)ctx->partial;
  b.y = (const T*)ctx->y_t;
  b.z = (T*)ctx->z;
  b.theta = (T*)ctx->theta;
  b.r = (T*)ctx->r;
  b.bpart = ctx->bpart;
  b.bcnt = ctx->bcnt;
  b.bnrm = ctx->bnrm;
  b.ctl = ctx->ctl;
  return b;
}

size_t tsize(const pqr_ctx* ctx) { return ctx->opt.iter_prec == PQR_ITER_F64 ? 8 : 4; }

}  // namespace

// ---------------------------------------------------------------------------
extern "C" void pqr_default_options(pqr_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->mu = 0.0;
  o->mu_scale = 0.1;
  o->G = 48;
  o->eta_margin = 0.01;
  o->lanczos_steps = 40;
  o->iter_prec = PQR_ITER_F32;
  o->tol_gap = 1e-6;
  o->cert_every = 50;
  o->max_iter = 1000000;
  o->stream = nullptr;
  o->profile = 0;
  o->intercept_block = 1;
}

extern "C" const char* pqr_status_string(pqr_status s) {
  switch (s) {
    case PQR_OK: return "ok";
    case PQR_ERR_INVALID_ARG: return "invalid argument";
    case PQR_ERR_OOM: return "out of device memory";
    case PQR_ERR_DEVICE: return "device error";
    case PQR_ERR_NOT_CONVERGED: return "not converged";
    case PQR_ERR_DIVERGED: return "diverged";
    case PQR_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown";
}

extern "C" const char* pqr_last_error(const pqr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" void pqr_destroy(pqr_ctx* ctx) {
  if (!ctx) return;
  if (ctx->s) (void)hipStreamSynchronize(ctx->s);
  else (void)hipDeviceSynchronize();
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  if (ctx->chunk_exec) (void)hipGraphExecDestroy(ctx->chunk_exec);
  if (ctx->chunk_graph) (void)hipGraphDestroy(ctx->chunk_graph);
  if (ctx->cap_s) (void)hipStreamDestroy(ctx->cap_s);
  if (ctx->out_h) (void)hipHostFree(ctx->out_h);
  delete ctx;
}

// Geometry of a store of p columns with n rows in format fmt.
static void set_geometry(pqr_ctx* ctx, int fmt, int64_t n, int64_t p) {
  Geom& g = ctx->g;
  g.fmt = fmt;
  g.rpl = (g.fmt == B2 || n >= 8192) ? 16 : 4;
  if (ctx->opt.rows_per_lane == 16) g.rpl = 16;
  else if (ctx->opt.rows_per_lane == 4 && g.fmt != B2) g.rpl = 4;
  g.n = n;
  g.n_pad = round_up(n, (int64_t)kWave * g.rpl);
  g.p = p;
  g.p_pad = round_up(p, kGroup);
  g.seg_bytes = fmt_col_bytes(g.fmt, (int64_t)kWave * g.rpl);
}

static pqr_status alloc_colparams(pqr_ctx* ctx) {
  const Geom& g = ctx->g;
  TRY(dalloc(ctx, &ctx->cm_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->cinv_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->sd_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->cm_f, g.p_pad * 4));
  TRY(dalloc(ctx, &ctx->cinv_f, g.p_pad * 4));
  return PQR_OK;
}

static pqr_status create_rest(pqr_ctx* ctx);

static pqr_status create_impl(pqr_ctx* ctx, const pqr_design* X) {
  const int64_t n = X->n, p = X->p;
  set_geometry(ctx, X->store_fmt, n, p);
  Geom& g = ctx->g;
  ctx->standardize = X->standardize ? 1 : 0;
  hipStream_t s = ctx->s;
  if (g.n_pad / 256 + 1024 > (int64_t)1 << 22) {
    ctx->err = "n too large";
    return PQR_ERR_UNSUPPORTED;
  }
  TRY(dalloc(ctx, &ctx->X, (size_t)g.store_bytes()));
  g.X = ctx->X;
  HIPCHK(launch_encode(X->data, X->src_fmt, X->ld, g, ctx->X, s));
  double *sum, *sumsq;
  TRY(dalloc(ctx, &sum, g.p_pad * 8));
  TRY(dalloc(ctx, &sumsq, g.p_pad * 8));
  TRY(alloc_colparams(ctx));
  HIPCHK(launch_colstats(g, sum, sumsq, s));
  HIPCHK(launch_colparams(sum, sumsq, n, p, g.p_pad, ctx->standardize, ctx->cm_d, ctx->cinv_d,
                          ctx->sd_d, ctx->cm_f, ctx->cinv_f, s));
  return create_rest(ctx);
}

// A context over a subset of the parent's columns: the store and the column
// statistics are gathered from the parent (so the standardization is the
// parent's), then blocks and step sizes are set up for the subset.
static pqr_status create_subset_impl(pqr_ctx* ctx, const pqr_ctx* parent, const int64_t* cols,
                                     int64_t ncols) {
  const Geom& pg = parent->g;
  ctx->opt.rows_per_lane = pg.rpl;
  set_geometry(ctx, pg.fmt, pg.n, ncols);
  Geom& g = ctx->g;
  ctx->standardize = parent->standardize;
  hipStream_t s = ctx->s;
  int64_t* cols_d;
  TRY(dalloc(ctx, &cols_d, ncols * 8));
  HIPCHK(hipMemcpyAsync(cols_d, cols, ncols * 8, hipMemcpyHostToDevice, s));
  TRY(dalloc(ctx, &ctx->X, (size_t)g.store_bytes()));
  g.X = ctx->X;
  HIPCHK(launch_gather_columns(pg, cols_d, ncols, g, ctx->X, s));
  TRY(alloc_colparams(ctx));
  HIPCHK(launch_gather_f64(parent->cm_d, cols_d, ncols, g.p_pad, ctx->cm_d, s));
  HIPCHK(launch_gather_f64(parent->cinv_d, cols_d, ncols, g.p_pad, ctx->cinv_d, s));
  HIPCHK(launch_gather_f64(parent->sd_d, cols_d, ncols, g.p_pad, ctx->sd_d, s));
  HIPCHK(launch_from_double<float>(ctx->cm_d, g.p_pad, ctx->cm_f, s));
  HIPCHK(launch_from_double<float>(ctx->cinv_d, g.p_pad, ctx->cinv_f, s));
  HIPCHK(hipStreamSynchronize(s));
  return create_rest(ctx);
}

static pqr_status create_rest(pqr_ctx* ctx) {
  Geom& g = ctx->g;
  const int64_t n = g.n, p = g.p;
  hipStream_t s = ctx->s;
  const int64_t ng = g.ngroups();
  // blocks: contiguous near-equal runs of 16-column groups; the intercept is
  // either a block of its own (block 0) or the first column of block 0
  int Gf = ctx->opt.G > 0 ? ctx->opt.G : 48;
  if (Gf > ng) Gf = (int)ng;
  ctx->Gf = Gf;
  ctx->icpt_own = ctx->opt.intercept_block ? 1 : 0;
  const int off = ctx->icpt_own;
  const int G = Gf + off;
  ctx->G = G;
  ctx->gbound.resize(Gf + 1);
  for (int b = 0; b < Gf; ++b) ctx->gbound[b] = (int)(((int64_t)b * ng) / Gf);
  ctx->gbound[Gf] = (int)ng;
  ctx->bounds.assign(G + 1, 0);
  for (int b = 0; b <= Gf; ++b)
    ctx->bounds[b + off] = (int)std::min<int64_t>(p, (int64_t)kGroup * ctx->gbound[b]);
  ctx->bounds[G] = (int)p;
  std::vector<int> fblock(ng);   // feature block of every group (for Lanczos)
  ctx->gblock_h.resize(ng);
  for (int b = 0; b < Gf; ++b)
    for (int q = ctx->gbound[b]; q < ctx->gbound[b + 1]; ++q) {
      fblock[q] = b;
      ctx->gblock_h[q] = b + off;
    }
  int *gblock_d, *bstart_d;
  TRY(dalloc(ctx, &gblock_d, ng * 4));
  TRY(dalloc(ctx, &bstart_d, (Gf + 1) * 4));
  HIPCHK(hipMemcpyAsync(gblock_d, fblock.data(), ng * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(bstart_d, ctx->gbound.data(), (Gf + 1) * 4, hipMemcpyHostToDevice, s));
  std::vector<int> iota(ng);
  for (int64_t q = 0; q < ng; ++q) iota[q] = (int)q;
  TRY(dalloc(ctx, &ctx->iota, ng * 4));
  HIPCHK(hipMemcpyAsync(ctx->iota, iota.data(), ng * 4, hipMemcpyHostToDevice, s));

  // Lanczos estimates of Lambda_max(X~_b^T X~_b), all feature blocks together
  const int T = std::max(2, ctx->opt.lanczos_steps > 0 ? ctx->opt.lanczos_steps : 40);
  const int splits = 8;
  float *q, *qprev, *wbuf, *qsum, *u, *lpart;
  double *al, *be;
  TRY(dalloc(ctx, &q, (size_t)Gf * g.n_pad * 4));
  TRY(dalloc(ctx, &qprev, (size_t)Gf * g.n_pad * 4));
  TRY(dalloc(ctx, &wbuf, (size_t)Gf * g.n_pad * 4));
  TRY(dalloc(ctx, &qsum, Gf * 4));
  TRY(dalloc(ctx, &u, g.p_pad * 4));
  TRY(dalloc(ctx, &lpart, (size_t)Gf * splits * g.n_pad * 4));
  TRY(dalloc(ctx, &al, (size_t)Gf * T * 8));
  TRY(dalloc(ctx, &be, (size_t)Gf * T * 8));
  HIPCHK(launch_lanczos_init(n, g.n_pad, Gf, q, qprev, qsum, s));
  for (int k = 0; k < T; ++k) {
    HIPCHK(launch_block_dots(g, q, g.n_pad, gblock_d, ctx->cm_f, ctx->cinv_f, qsum, u, s));
    HIPCHK(launch_block_axpy(g, u, ctx->cm_f, ctx->cinv_f, bstart_d, Gf, splits, lpart, s));
    HIPCHK(launch_lanczos_step(n, g.n_pad, Gf, splits, k, T, ctx->icpt_own ? 0 : 1, lpart, q,
                               qprev, wbuf, qsum, al, be, s));
  }
  std::vector<double> ha((size_t)Gf * T), hb((size_t)Gf * T);
  HIPCHK(hipMemcpyAsync(ha.data(), al, ha.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hb.data(), be, hb.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->Lambda.assign(G, 0.0);
  if (off) ctx->Lambda[0] = (double)n;   // the intercept column alone: 1^T 1 = n
  for (int b = 0; b < Gf; ++b) {
    int k = T;
    for (int i = 0; i < T; ++i)
      if (hb[(size_t)b * T + i] < 1e-12 * std::max(1.0, std::fabs(ha[(size_t)b * T]))) { k = i + 1; break; }
    ctx->Lambda[b + off] = std::max(ritz_upper(&ha[(size_t)b * T], &hb[(size_t)b * T], k), 1e-30);
  }

  // iteration buffers
  const size_t ts = tsize(ctx);
  TRY(dalloc(ctx, &ctx->beta, g.p_pad * ts));
  TRY(dalloc(ctx, &ctx->beta_best, g.p_pad * ts));
  TRY(dalloc(ctx, &ctx->z_best, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->theta_best, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->clam_t, g.p_pad * ts));
  TRY(dalloc(ctx, &ctx->cm_t, g.p_pad * ts));
  TRY(dalloc(ctx, &ctx->cinv_t, g.p_pad * ts));
  TRY(dalloc(ctx, &ctx->geta_t, ng * ts));
  TRY(dalloc(ctx, &ctx->gnorm, ng * 4 * ts));
  TRY(dalloc(ctx, &ctx->gflag, ng * 4));
  TRY(dalloc(ctx, &ctx->list, ng * 4));
  TRY(dalloc(ctx, &ctx->partial, (size_t)ctx->smax * g.n_pad * 8));
  TRY(dalloc(ctx, &ctx->y_t, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->z, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->theta, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->r, g.n_pad * ts));
  TRY(dalloc(ctx, &ctx->bpart, (g.n_pad / 256) * 8 * 8));
  TRY(dalloc(ctx, &ctx->bcnt, kCompactBlocks * 4));
  TRY(dalloc(ctx, &ctx->bnrm, kCompactBlocks * 4 * 8));
  TRY(dalloc(ctx, &ctx->ctl, sizeof(Ctl)));
  TRY(dalloc(ctx, &ctx->ctl_kkt, sizeof(Ctl)));
  HIPCHK(hipMemsetAsync(ctx->beta, 0, g.p_pad * ts, s));
  HIPCHK(hipMemsetAsync(ctx->ctl, 0, sizeof(Ctl), s));
  if (ts == 8) {
    HIPCHK(hipMemcpyAsync(ctx->cm_t, ctx->cm_d, g.p_pad * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->cinv_t, ctx->cinv_d, g.p_pad * 8, hipMemcpyDeviceToDevice, s));
  } else {
    HIPCHK(hipMemcpyAsync(ctx->cm_t, ctx->cm_f, g.p_pad * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->cinv_t, ctx->cinv_f, g.p_pad * 4, hipMemcpyDeviceToDevice, s));
  }

  // certificate buffers
  TRY(dalloc(ctx, &ctx->y_d, g.n_pad * 8));
  TRY(dalloc(ctx, &ctx->theta_p, g.n_pad * 8));
  TRY(dalloc(ctx, &ctx->scratch64, std::max(g.n_pad, g.p_pad + 1) * 8));
  TRY(dalloc(ctx, &ctx->beta_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->bt_out, (g.p_pad + 1) * 8));
  TRY(dalloc(ctx, &ctx->clam_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->v_d, g.p_pad * 8));
  TRY(dalloc(ctx, &ctx->gpart, ng * 8));
  TRY(dalloc(ctx, &ctx->partial64, (size_t)ctx->smax * g.n_pad * 8));
  ctx->bpart64_len = std::max<int64_t>(g.n_pad / 256 + 1024, g.p_pad + 1024);
  TRY(dalloc(ctx, &ctx->bpart64, ctx->bpart64_len * 8));
  TRY(dalloc(ctx, &ctx->out_d, 16 * 8));
  if (hipHostMalloc((void**)&ctx->out_h, 16 * 8, hipHostMallocDefault) != hipSuccess) {
    ctx->err = "hipHostMalloc failed";
    return PQR_ERR_OOM;
  }
  HIPCHK(hipStreamSynchronize(s));
  return PQR_OK;
}

extern "C" pqr_status pqr_create(pqr_ctx** out, const pqr_design* X, const pqr_options* opt) {
  Range range_("pqr_create");
  if (!out) return PQR_ERR_INVALID_ARG;
  *out = nullptr;
  pqr_ctx* ctx = new pqr_ctx();
  if (opt) ctx->opt = *opt; else pqr_default_options(&ctx->opt);
  pqr_options d;
  pqr_default_options(&d);
  if (ctx->opt.mu_scale <= 0) ctx->opt.mu_scale = d.mu_scale;
  // a negative margin (> -1) puts eta below mu*Lambda on purpose: it exists to
  // exercise the H-norm monitor; 0 selects the default
  if (ctx->opt.eta_margin == 0 || ctx->opt.eta_margin <= -1) ctx->opt.eta_margin = d.eta_margin;
  if (ctx->opt.tol_gap <= 0) ctx->opt.tol_gap = d.tol_gap;
  if (ctx->opt.cert_every <= 0) ctx->opt.cert_every = d.cert_every;
  if (ctx->opt.max_iter <= 0) ctx->opt.max_iter = d.max_iter;
  if (ctx->opt.iter_prec != PQR_ITER_F64) ctx->opt.iter_prec = PQR_ITER_F32;
  ctx->s = (hipStream_t)ctx->opt.stream;
  *out = ctx;
  if (!X || !X->data || X->n < 1 || X->p < 1 || X->ld < X->n) {
    ctx->err = "invalid design: need data, n >= 1, p >= 1, ld >= n";
    return PQR_ERR_INVALID_ARG;
  }
  const bool src_int = X->src_fmt == PQR_X_I8;
  const bool src_flt = X->src_fmt == PQR_X_F64 || X->src_fmt == PQR_X_F32;
  if (!src_int && !src_flt) {
    ctx->err = "src_fmt must be PQR_X_F64, PQR_X_F32 or PQR_X_I8";
    return PQR_ERR_INVALID_ARG;
  }
  if (X->store_fmt < PQR_X_F64 || X->store_fmt > PQR_X_2BIT) {
    ctx->err = "unknown store_fmt";
    return PQR_ERR_INVALID_ARG;
  }
  if (src_flt && !(X->store_fmt == PQR_X_F64 || X->store_fmt == PQR_X_F32 ||
                   X->store_fmt == PQR_X_BF16)) {
    ctx->err = "floating-point designs can be stored as F64, F32 or BF16 only";
    return PQR_ERR_UNSUPPORTED;
  }
  if (X->p > ((int64_t)1 << 31) - 64 || X->n > ((int64_t)1 << 31) - 4096) {
    ctx->err = "n or p too large";
    return PQR_ERR_UNSUPPORTED;
  }
  pqr_status st = create_impl(ctx, X);
  return st;
}

// ---------------------------------------------------------------------------
namespace {

struct SolveSetup {
  double tau, mu, sigma;
  IterParams ip;
};

// The unpenalized feature columns (weight 0) of the problem; the certificate
// projects its dual point onto x~_j^T theta = 0 for them.
void set_unpenalized(pqr_ctx* ctx, const double* weights) {
  std::vector<int64_t> u;
  if (weights)
    for (int64_t j = 0; j < ctx->g.p; ++j)
      if (weights[1 + j] == 0.0) u.push_back(j);
  if (u != ctx->unpen) {
    ctx->unpen.swap(u);
    ctx->unpen_ready = false;
  }
}

pqr_status project_unpenalized(pqr_ctx* ctx, double tau, bool* ok);

template <typename T>
pqr_status upload_problem(pqr_ctx* ctx, const double* y, double tau, double lambda,
                          const double* weights, double* lmax_out, double* score) {
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  // y
  std::vector<double> yh(g.n_pad, 0.0);
  std::memcpy(yh.data(), y, g.n * 8);
  HIPCHK(hipMemcpyAsync(ctx->y_d, yh.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_set_y<T>(ctx->y_d, g.n, g.n_pad, (T*)ctx->y_t, s));
  // weights (lambda = 1) for lambda_max, then lambda * w
  std::vector<double> lh(g.p_pad, 0.0);
  for (int64_t j = 0; j < g.p; ++j) lh[j] = weights ? weights[1 + j] : 1.0;
  HIPCHK(hipMemcpyAsync(ctx->clam_d, lh.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_null_dual(ctx->y_d, g.n, g.n_pad, tau, ctx->theta_p, ctx->out_d, s));
  HIPCHK(launch_dots64(g, ctx->theta_p, ctx->out_d + 5, ctx->cm_d, ctx->cinv_d, ctx->clam_d,
                       ctx->v_d, ctx->gpart, s));
  HIPCHK(launch_reduce_max(ctx->gpart, g.ngroups(), ctx->bpart64, ctx->out_d + 3, s));
  HIPCHK(hipMemcpyAsync(ctx->out_h, ctx->out_d, 16 * 8, hipMemcpyDeviceToHost, s));
  if (score) HIPCHK(hipMemcpyAsync(score, ctx->v_d, g.p * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (lmax_out) *lmax_out = ctx->out_h[3];
  for (int64_t j = 0; j < g.p; ++j) lh[j] *= lambda;
  HIPCHK(hipMemcpyAsync(ctx->clam_d, lh.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
  set_unpenalized(ctx, weights);
  HIPCHK(launch_from_double<T>(ctx->clam_d, g.p_pad, (T*)ctx->clam_t, s));
  HIPCHK(hipStreamSynchronize(s));
  return PQR_OK;
}

pqr_status validate_problem(pqr_ctx* ctx, const double* y, double tau, double lambda,
                            const double* weights) {
  if (!y) { ctx->err = "y is NULL"; return PQR_ERR_INVALID_ARG; }
  if (!(tau > 0.0 && tau < 1.0)) { ctx->err = "tau must lie in (0, 1)"; return PQR_ERR_INVALID_ARG; }
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) {
    ctx->err = "lambda must be finite and >= 0";
    return PQR_ERR_INVALID_ARG;
  }
  if (!finite_all(y, ctx->g.n)) { ctx->err = "y has non-finite entries"; return PQR_ERR_INVALID_ARG; }
  if (weights) {
    for (int64_t j = 1; j <= ctx->g.p; ++j)
      if (!(weights[j] >= 0.0) || !std::isfinite(weights[j])) {
        ctx->err = "weights must be finite and >= 0";
        return PQR_ERR_INVALID_ARG;
      }
  }
  return PQR_OK;
}

template <typename T>
pqr_status set_eta(pqr_ctx* ctx, double mu, const double* eta_explicit, double eta_scale,
                   IterParams& ip, double tau) {
  const Geom& g = ctx->g;
  std::vector<double> eta(ctx->G);
  for (int b = 0; b < ctx->G; ++b)
    eta[b] = eta_explicit ? eta_explicit[b]
                          : eta_scale * (1.0 + ctx->opt.eta_margin) * mu * ctx->Lambda[b];
  std::vector<T> ge(g.ngroups());
  for (int64_t q = 0; q < g.ngroups(); ++q) ge[q] = (T)eta[ctx->gblock_h[q]];
  HIPCHK(hipMemcpyAsync(ctx->geta_t, ge.data(), ge.size() * sizeof(T), hipMemcpyHostToDevice, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  ip.tau = tau;
  ip.mu = mu;
  ip.sigma = mu / (ctx->G + 1.0);
  ip.eta0 = eta[0];
  ip.G = ctx->G;
  ip.smax = ctx->smax;
  ip.min_per = ctx->min_per;
  return PQR_OK;
}

// Load (beta_std, z, theta) from host, or a zero start; then rebuild r.
template <typename T>
pqr_status init_state(pqr_ctx* ctx, int start, const double* beta_std, const double* zh,
                      const double* th, const IterParams& ip) {
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  int fit = 0;
  if (start == PQR_START_DEVICE) {
    HIPCHK(hipMemcpyAsync(&c, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double b0 = c.beta0;
    std::memset(&c, 0, sizeof(c));
    c.beta0 = b0;
  } else if (start == PQR_START_HOST) {
    std::vector<double> tmp(std::max(g.n_pad, g.p_pad), 0.0);
    std::memcpy(tmp.data(), beta_std + 1, g.p * 8);
    std::fill(tmp.begin() + g.p, tmp.end(), 0.0);
    HIPCHK(hipMemcpyAsync(ctx->scratch64, tmp.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
    HIPCHK(launch_from_double<T>(ctx->scratch64, g.p_pad, (T*)ctx->beta, s));
    HIPCHK(hipStreamSynchronize(s));
    // a null z (theta) is derived from beta on the device: z = y - X~beta - beta0,
    // theta_i = (tau - 1{z_i < 0}) / n centred to sum zero
    std::fill(tmp.begin(), tmp.end(), 0.0);
    if (zh) std::memcpy(tmp.data(), zh, g.n * 8);
    HIPCHK(hipMemcpyAsync(ctx->scratch64, tmp.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
    HIPCHK(launch_from_double<T>(ctx->scratch64, g.n_pad, (T*)ctx->z, s));
    HIPCHK(hipStreamSynchronize(s));
    std::fill(tmp.begin(), tmp.end(), 0.0);
    if (th) std::memcpy(tmp.data(), th, g.n * 8);
    HIPCHK(hipMemcpyAsync(ctx->scratch64, tmp.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
    HIPCHK(launch_from_double<T>(ctx->scratch64, g.n_pad, (T*)ctx->theta, s));
    HIPCHK(hipStreamSynchronize(s));
    c.beta0 = beta_std[0];
    fit = (zh ? 0 : 1) | (th ? 0 : 2);
  } else {
    HIPCHK(hipMemsetAsync(ctx->beta, 0, g.p_pad * sizeof(T), s));
    HIPCHK(hipMemcpyAsync(ctx->z, ctx->y_t, g.n_pad * sizeof(T), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(ctx->theta, 0, g.n_pad * sizeof(T), s));
  }
  HIPCHK(hipMemcpyAsync(ctx->ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
  IterParams ipf = ip;
  ipf.fit = fit;
  HIPCHK(launch_prepare_state<T>(g, bufs<T>(ctx), ipf, s));
  HIPCHK(hipStreamSynchronize(s));
  return PQR_OK;
}

struct Cert {
  double primal, dual, gap, rel_gap, maxratio;
};

// Dual feasibility for the unpenalized columns U (lambda_j = 0): project the
// projected theta' (ctx->theta_p) onto {sum theta = 0, x~_U^T theta = 0} and scale
// it back into the box (launch_unpen_project).  The Gram matrix of X~_U and its Cholesky factor
// (with a ridge of 1e-12 of its largest diagonal, so that constant columns get
// c_j = 0) are built once per problem.  *ok is false when a residual x~_j^T theta
// is above rounding level (1e-10 ||x~_j|| ||theta||): the certificate then gives
// no dual bound.
pqr_status project_unpenalized(pqr_ctx* ctx, double tau, bool* ok) {
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  const int64_t nu = (int64_t)ctx->unpen.size() + 1;   // + the intercept (ones)
  if (nu > 4097) {
    ctx->err = "at most 4096 unpenalized columns (zero weights) are supported";
    return PQR_ERR_UNSUPPORTED;
  }
  if (!ctx->unpen_ready) {
    if (ctx->unpen_cap < nu) {
      TRY(dalloc(ctx, &ctx->unpen_cols_d, (size_t)nu * 8));
      TRY(dalloc(ctx, &ctx->unpen_x, (size_t)nu * g.n_pad * 8));
      TRY(dalloc(ctx, &ctx->unpen_c, (size_t)nu * 8));
      TRY(dalloc(ctx, &ctx->unpen_u, (size_t)nu * nu * 8));
      ctx->unpen_cap = nu;
    }
    std::vector<int64_t> cols(1, -1);
    cols.insert(cols.end(), ctx->unpen.begin(), ctx->unpen.end());
    HIPCHK(hipMemcpyAsync(ctx->unpen_cols_d, cols.data(), nu * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(launch_dense_cols(g, ctx->unpen_cols_d, nu, ctx->cm_d, ctx->cinv_d, ctx->unpen_x, s));
    HIPCHK(launch_cross(ctx->unpen_x, nu, ctx->unpen_x, nu, g.n_pad, ctx->unpen_u, s));
    std::vector<double> G((size_t)nu * nu);
    HIPCHK(hipMemcpyAsync(G.data(), ctx->unpen_u, G.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->unpen_diag.resize(nu);
    double dmax = 0.0;
    for (int64_t a = 0; a < nu; ++a) {
      ctx->unpen_diag[a] = G[a * nu + a];
      dmax = std::max(dmax, G[a * nu + a]);
    }
    const double ridge = 1e-12 * std::max(dmax, 1e-300);
    for (int64_t a = 0; a < nu; ++a) G[a * nu + a] += ridge;
    for (int64_t a = 0; a < nu; ++a) {   // in-place Cholesky, lower triangle
      for (int64_t b = 0; b <= a; ++b) {
        double v = G[a * nu + b];
        for (int64_t k = 0; k < b; ++k) v -= G[a * nu + k] * G[b * nu + k];
        G[a * nu + b] = a == b ? std::sqrt(std::max(v, ridge)) : v / G[b * nu + b];
      }
    }
    ctx->unpen_chol.swap(G);
    ctx->unpen_ready = true;
  }
  // u = X~_U^T theta', c = (L L^T)^{-1} u
  HIPCHK(launch_cross(ctx->unpen_x, nu, ctx->theta_p, 1, g.n_pad, ctx->unpen_u, s));
  std::vector<double> c(nu);
  HIPCHK(hipMemcpyAsync(c.data(), ctx->unpen_u, nu * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const std::vector<double>& Lf = ctx->unpen_chol;
  for (int64_t a = 0; a < nu; ++a) {
    double v = c[a];
    for (int64_t k = 0; k < a; ++k) v -= Lf[a * nu + k] * c[k];
    c[a] = v / Lf[a * nu + a];
  }
  for (int64_t a = nu - 1; a >= 0; --a) {
    double v = c[a];
    for (int64_t k = a + 1; k < nu; ++k) v -= Lf[k * nu + a] * c[k];
    c[a] = v / Lf[a * nu + a];
  }
  HIPCHK(hipMemcpyAsync(ctx->unpen_c, c.data(), nu * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_unpen_project(ctx->theta_p, ctx->unpen_x, ctx->unpen_c, nu, g.n, g.n_pad, tau,
                              ctx->y_d, ctx->bpart64, ctx->out_d, s));
  // residual check
  HIPCHK(launch_cross(ctx->unpen_x, nu, ctx->theta_p, 1, g.n_pad, ctx->unpen_u, s));
  std::vector<double> r(nu);
  HIPCHK(hipMemcpyAsync(r.data(), ctx->unpen_u, nu * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double tnorm = std::sqrt((double)g.n) * std::max(tau, 1.0 - tau) / (double)g.n;
  *ok = true;
  for (int64_t a = 0; a < nu; ++a)
    if (std::fabs(r[a]) > 1e-10 * std::sqrt(ctx->unpen_diag[a]) * tnorm) *ok = false;
  return PQR_OK;
}

// FP64 certificate of the point (beta, beta0 = ctl->beta0, theta); `list` and
// ctl->count must describe the nonzero groups of beta; ctx->clam_d holds lambda_j.
template <typename T>
pqr_status certify_point(pqr_ctx* ctx, double tau, const T* theta, const T* beta, const Ctl* ctl,
                         const int* list, Cert* out) {
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  HIPCHK(launch_project<T>(theta, g.n, g.n_pad, tau, ctx->y_d, ctx->theta_p, ctx->out_d, s));
  bool unpen_ok = true;
  if (!ctx->unpen.empty()) TRY(project_unpenalized(ctx, tau, &unpen_ok));
  HIPCHK(launch_dots64(g, ctx->theta_p, ctx->out_d + 5, ctx->cm_d, ctx->cinv_d, ctx->clam_d,
                       nullptr, ctx->gpart, s));
  HIPCHK(launch_reduce_max(ctx->gpart, g.ngroups(), ctx->bpart64, ctx->out_d + 3, s));
  HIPCHK(launch_to_double<T>(beta, g.p_pad, ctx->beta_d, s));
  CertBufs c{};
  c.y = ctx->y_d;
  c.theta_p = ctx->theta_p;
  c.beta_d = ctx->beta_d;
  c.cm = ctx->cm_d;
  c.cinv = ctx->cinv_d;
  c.clam = ctx->clam_d;
  c.partial = ctx->partial64;
  c.list = list;
  c.ctl = ctl;
  c.bpart = ctx->bpart64;
  c.out = ctx->out_d;
  HIPCHK(launch_primal64(g, c, tau, ctx->smax, ctx->min_per, s));
  HIPCHK(hipMemcpyAsync(ctx->out_h, ctx->out_d, 16 * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double* o = ctx->out_h;
  const double mr = o[3];
  double alpha = mr > 1.0 ? (std::isinf(mr) ? 0.0 : 1.0 / mr) : 1.0;
  if (!unpen_ok) alpha = 0.0;   // the projection left x~_U^T theta above rounding level
  out->primal = o[0] + o[1];
  out->dual = alpha * o[2];
  out->gap = out->primal - out->dual;
  out->rel_gap = out->gap / std::max(std::fabs(out->primal), 1e-300);
  out->maxratio = mr;
  return PQR_OK;
}

template <typename T>
pqr_status certificate(pqr_ctx* ctx, double tau, Cert* out) {
  return certify_point<T>(ctx, tau, (const T*)ctx->theta, (const T*)ctx->beta, ctx->ctl,
                          ctx->list, out);
}

// Copies the coefficients `bsrc` (intercept beta0), z from `zsrc` and theta from
// `tsrc` out (device buffers of the iterate type).
template <typename T>
pqr_status export_state(pqr_ctx* ctx, pqr_result* res, const void* bsrc, double beta0,
                        const void* zsrc, const void* tsrc) {
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  Ctl c;
  HIPCHK(hipMemcpyAsync(&c, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c.beta0 = beta0;
  HIPCHK(launch_to_double<T>((const T*)bsrc, g.p_pad, ctx->beta_d, s));
  std::vector<double> b(g.p);
  HIPCHK(hipMemcpyAsync(b.data(), ctx->beta_d, g.p * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t nnz = 0;
  for (int64_t j = 0; j < g.p; ++j) nnz += b[j] != 0.0;
  res->nnz = nnz;
  if (res->beta_std) {
    res->beta_std[0] = c.beta0;
    std::memcpy(res->beta_std + 1, b.data(), g.p * 8);
  }
  if (res->beta) {
    // scratch64 holds [beta0, beta_std(1..p)] for the back-transform
    std::vector<double> bs(g.p + 1);
    bs[0] = c.beta0;
    std::memcpy(bs.data() + 1, b.data(), g.p * 8);
    HIPCHK(hipMemcpyAsync(ctx->scratch64, bs.data(), (g.p + 1) * 8, hipMemcpyHostToDevice, s));
    double* bo = ctx->bt_out;
    HIPCHK(launch_back_transform(ctx->scratch64, g.p, ctx->cm_d, ctx->cinv_d, c.beta0, bo,
                                 ctx->bpart64, s));
    HIPCHK(hipMemcpyAsync(res->beta, bo, (g.p + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (res->z) {
    HIPCHK(launch_to_double<T>((const T*)zsrc, g.n_pad, ctx->scratch64, s));
    HIPCHK(hipMemcpyAsync(res->z, ctx->scratch64, g.n * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (res->theta) {
    HIPCHK(launch_to_double<T>((const T*)tsrc, g.n_pad, ctx->scratch64, s));
    HIPCHK(hipMemcpyAsync(res->theta, ctx->scratch64, g.n * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return PQR_OK;
}

double default_mu(const pqr_ctx* ctx, const double* y) {
  const int64_t n = ctx->g.n;
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) m += y[i];
  m /= (double)n;
  double v = 0.0;
  for (int64_t i = 0; i < n; ++i) v += (y[i] - m) * (y[i] - m);
  const double sd = std::sqrt(v / (double)n);
  return ctx->opt.mu_scale * std::sqrt(ctx->G + 1.0) / ((double)n * (sd > 0 ? sd : 1.0));
}

// One solve's host-side state: set-up, the checks between chunks of
// iterations (H-norm monitor, FP64 certificate, best bounds) and the export.
// pqr_solve drives one Run; pqr_solve_grouped drives many, with the iterations
// of all of them in shared launches.
template <typename T>
struct Run {
  pqr_ctx* ctx = nullptr;
  std::chrono::steady_clock::time_point t0;
  double tau = 0.0, mu = 0.0, lmax = 0.0, eta_scale = 1.0;
  IterParams ip{};
  int64_t it = 0, certs = 0, restarts = 0, sweeps = 0;
  double sweep_ms = 0.0;
  // Any iterate's P(beta) bounds P* from above and any feasible dual point's
  // value bounds it from below, so the gap certified so far is
  // min primal - max dual; the coefficients reported are the best primal ones.
  double best_primal = INFINITY, best_dual = -INFINITY, best_beta0 = 0.0;
  pqr_status status = PQR_ERR_NOT_CONVERGED;

  bool active() const { return status == PQR_ERR_NOT_CONVERGED && it < ctx->opt.max_iter; }
  int64_t next_chunk() const {
    return std::min<int64_t>(ctx->opt.cert_every, ctx->opt.max_iter - it);
  }
  double best_gap() const {
    return (best_primal - best_dual) / std::max(std::fabs(best_primal), 1e-300);
  }

  pqr_status track() {
    Cert c{};
    TRY(certificate<T>(ctx, tau, &c));
    ++certs;
    if (c.dual > best_dual) {
      best_dual = c.dual;
      HIPCHK(hipMemcpyAsync(ctx->theta_best, ctx->theta, ctx->g.n_pad * sizeof(T),
                            hipMemcpyDeviceToDevice, ctx->s));
    }
    if (c.primal < best_primal) {
      best_primal = c.primal;
      Ctl cc;
      HIPCHK(hipMemcpyAsync(&cc, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->s));
      HIPCHK(hipMemcpyAsync(ctx->beta_best, ctx->beta, ctx->g.p_pad * sizeof(T),
                            hipMemcpyDeviceToDevice, ctx->s));
      HIPCHK(hipMemcpyAsync(ctx->z_best, ctx->z, ctx->g.n_pad * sizeof(T),
                            hipMemcpyDeviceToDevice, ctx->s));
      HIPCHK(hipStreamSynchronize(ctx->s));
      best_beta0 = cc.beta0;
    }
    if (best_gap() <= ctx->opt.tol_gap) status = PQR_OK;
    return PQR_OK;
  }

  pqr_status begin(pqr_ctx* c, const double* y, double tau_, double lambda, const double* weights,
                   int start, const pqr_result* warm) {
    ctx = c;
    t0 = std::chrono::steady_clock::now();
    tau = tau_;
    TRY(validate_problem(ctx, y, tau, lambda, weights));
    if (start == PQR_START_HOST && (!warm || !warm->beta_std)) {
      ctx->err = "PQR_START_HOST needs warm->beta_std";
      return PQR_ERR_INVALID_ARG;
    }
    if (start == PQR_START_DEVICE && !ctx->have_state) {
      ctx->err = "PQR_START_DEVICE needs a previous solve on this context";
      return PQR_ERR_INVALID_ARG;
    }
    TRY(upload_problem<T>(ctx, y, tau, lambda, weights, &lmax, nullptr));
    mu = ctx->opt.mu > 0 ? ctx->opt.mu
                         : (start == PQR_START_DEVICE ? ctx->state_mu : default_mu(ctx, y));
    TRY(set_eta<T>(ctx, mu, nullptr, eta_scale, ip, tau));
    TRY(init_state<T>(ctx, start, warm ? warm->beta_std : nullptr, warm ? warm->z : nullptr,
                      warm ? warm->theta : nullptr, ip));
    ctx->have_state = true;
    ctx->state_mu = mu;
    return track();
  }

  // After `chunk` more iterations have run (and the stream is idle).
  pqr_status after_chunk(int64_t chunk) {
    it += chunk;
    Ctl c;
    HIPCHK(hipMemcpyAsync(&c, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->s));
    HIPCHK(hipStreamSynchronize(ctx->s));
    if (!std::isfinite(c.delta) || c.n_increase > 25) {
      // the H-norm successive difference grows: the metric is not positive
      // definite (eta_g below mu Lambda_max); double eta and restart
      if (++restarts > 2) {
        ctx->err = "H-norm monitor: successive differences keep growing after doubling eta twice";
        status = PQR_ERR_DIVERGED;
        return PQR_OK;
      }
      eta_scale *= 2.0;
      TRY(set_eta<T>(ctx, mu, nullptr, eta_scale, ip, tau));
      TRY(init_state<T>(ctx, PQR_START_ZERO, nullptr, nullptr, nullptr, ip));
      return PQR_OK;
    }
    return track();
  }

  pqr_status finish(pqr_result* out) {
    if (out) {
      TRY(export_state<T>(ctx, out, ctx->beta_best, best_beta0, ctx->z_best, ctx->theta_best));
      out->iters = it;
      out->certs = certs;
      out->x_passes = it + certs + 1;
      out->primal = best_primal;
      out->dual = best_dual;
      out->rel_gap = best_gap();
      out->lambda_max = lmax;
      out->mu = mu;
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      out->sweep_ms = sweep_ms;
      out->sweep_launches = sweeps;
    }
    if (status == PQR_ERR_NOT_CONVERGED)
      ctx->err = "max_iter reached with relative gap " + std::to_string(best_gap());
    return status;
  }
};

bool same_params(const IterParams& a, const IterParams& b) {
  return a.tau == b.tau && a.mu == b.mu && a.sigma == b.sigma && a.eta0 == b.eta0 && a.G == b.G &&
         a.smax == b.smax && a.min_per == b.min_per && a.fit == b.fit;
}

// The graph of `chunk` iterations with parameters ip, captured once and reused while
// they stay the same (the buffers of a context never move).  Captured on a private
// stream of default priority; no memory-set nodes (the chunk is kernels only).
// Returns false (and leaves the direct launches to the caller) when capture fails.
template <typename T>
bool chunk_graph(pqr_ctx* ctx, const IterBufs<T>& b, const IterParams& ip, int64_t chunk) {
  if (ctx->graph_failed) return false;
  const int prec = (int)sizeof(T);
  if (ctx->chunk_exec && ctx->chunk_len == chunk && ctx->chunk_prec == prec &&
      same_params(ctx->chunk_ip, ip))
    return true;
  if (ctx->chunk_exec) { (void)hipGraphExecDestroy(ctx->chunk_exec); ctx->chunk_exec = nullptr; }
  if (ctx->chunk_graph) { (void)hipGraphDestroy(ctx->chunk_graph); ctx->chunk_graph = nullptr; }
  bool ok = ctx->cap_s || hipStreamCreateWithFlags(&ctx->cap_s, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamBeginCapture(ctx->cap_s, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < chunk && e == hipSuccess; ++k)
      e = launch_iteration<T>(ctx->g, b, ip, ctx->cap_s, nullptr, nullptr);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(ctx->cap_s, &gr);
    ok = e == hipSuccess && ee == hipSuccess && gr;
    if (ok && hipGraphInstantiate(&ctx->chunk_exec, gr, nullptr, nullptr, 0) != hipSuccess) {
      ctx->chunk_exec = nullptr;
      ok = false;
    }
    if (ok) ctx->chunk_graph = gr;
    else if (gr) (void)hipGraphDestroy(gr);
  }
  if (!ok) {
    (void)hipGetLastError();
    ctx->graph_failed = true;
    return false;
  }
  ctx->chunk_len = chunk;
  ctx->chunk_prec = prec;
  ctx->chunk_ip = ip;
  return true;
}

template <typename T>
pqr_status solve_impl(pqr_ctx* ctx, const double* y, double tau, double lambda,
                      const double* weights, int start, const pqr_result* warm, pqr_result* out) {
  Run<T> run;
  TRY(run.begin(ctx, y, tau, lambda, weights, start, warm));
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  const bool prof = ctx->opt.profile != 0;
  if (prof && ctx->events.empty()) {
    ctx->events.resize(2 * (size_t)ctx->opt.cert_every);
    for (auto& e : ctx->events) HIPCHK(hipEventCreate(&e));
  }
  while (run.active()) {
    const int64_t chunk = run.next_chunk();
    const IterBufs<T> b = bufs<T>(ctx);
    if (!prof && ctx->opt.launch_mode == 0 && chunk == ctx->opt.cert_every &&
        chunk_graph<T>(ctx, b, run.ip, chunk)) {
      HIPCHK(hipGraphLaunch(ctx->chunk_exec, s));
    } else {
      for (int64_t k = 0; k < chunk; ++k)
        HIPCHK(launch_iteration<T>(g, b, run.ip, s, prof ? ctx->events[2 * k] : nullptr,
                                   prof ? ctx->events[2 * k + 1] : nullptr));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (prof) {
      for (int64_t k = 0; k < chunk; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->events[2 * k], ctx->events[2 * k + 1]));
        run.sweep_ms += ms;
      }
      run.sweeps += chunk;
    }
    TRY(run.after_chunk(chunk));
  }
  return run.finish(out);
}

// Many independent problems, each on its own context, iterated together: every
// iteration of every still-running problem is one set of five grouped launches
// on the first context's stream; set-up, certificates and exports stay per
// problem.
template <typename T>
pqr_status grouped_impl(int nprob, pqr_ctx* const* ctxs, const double* const* ys,
                        const double* taus, const double* lambdas, const double* const* weights,
                        pqr_result* outs, pqr_status* statuses) {
  pqr_ctx* c0 = ctxs[0];
  pqr_ctx* ctx = c0;   // device errors of the shared launches are reported here
  hipStream_t s = c0->s;
  std::vector<Run<T>> runs(nprob);
  std::vector<pqr_status> st(nprob, PQR_OK);
  for (int i = 0; i < nprob; ++i) {
    st[i] = runs[i].begin(ctxs[i], ys[i], taus[i], lambdas[i], weights ? weights[i] : nullptr,
                          PQR_START_ZERO, nullptr);
    if (st[i] != PQR_OK) runs[i].status = st[i];
  }
  const bool prof = c0->opt.profile != 0;
  // device table, released on every exit path
  struct Owned {
    GroupDesc<T>* desc = nullptr;
    int* off = nullptr;
    ~Owned() {
      if (desc) (void)hipFree(desc);
      if (off) (void)hipFree(off);
    }
  } own;
  if (prof) {   // two events per iteration of a chunk, on the first context
    int64_t cmax = 1;
    for (int i = 0; i < nprob; ++i) cmax = std::max<int64_t>(cmax, ctxs[i]->opt.cert_every);
    if (c0->events.size() < 2 * (size_t)cmax) {
      const size_t old = c0->events.size();
      c0->events.resize(2 * (size_t)cmax);
      for (size_t e = old; e < c0->events.size(); ++e) HIPCHK(hipEventCreate(&c0->events[e]));
    }
  }
  double sweep_ms = 0.0;
  int64_t sweeps = 0;
  pqr_status fail = PQR_OK;
  if (hipMalloc(&own.desc, sizeof(GroupDesc<T>) * nprob) != hipSuccess ||
      hipMalloc(&own.off, sizeof(int) * 3 * (nprob + 1)) != hipSuccess) {
    c0->err = "grouped solve: out of device memory for the problem table";
    fail = PQR_ERR_OOM;
  }
  GroupDesc<T>* desc_d = own.desc;
  int* off_d = own.off;
  std::vector<GroupDesc<T>> desc;
  std::vector<int> off;
  while (fail == PQR_OK) {
    std::vector<int> act;
    for (int i = 0; i < nprob; ++i)
      if (runs[i].ctx && st[i] == PQR_OK && runs[i].active()) act.push_back(i);
    if (act.empty()) break;
    int64_t chunk = INT64_MAX;
    for (int i : act) chunk = std::min(chunk, runs[i].next_chunk());
    const int na = (int)act.size();
    desc.resize(na);
    off.assign(3 * (na + 1), 0);
    int64_t tot[3] = {0, 0, 0};
    for (int k = 0; k < na; ++k) {
      pqr_ctx* c = ctxs[act[k]];
      desc[k].g = c->g;
      desc[k].b = bufs<T>(c);
      desc[k].ip = runs[act[k]].ip;
      const int64_t nb[3] = {(c->g.ngroups() + 3) / 4,
                             ((c->g.nchunks() + 3) / 4) * runs[act[k]].ip.smax,
                             c->g.n_pad / 256};
      for (int q = 0; q < 3; ++q) {
        off[q * (na + 1) + k] = (int)tot[q];
        tot[q] += nb[q];
      }
    }
    for (int q = 0; q < 3; ++q) {
      if (tot[q] > INT32_MAX) {
        c0->err = "grouped solve: too many blocks in one launch";
        fail = PQR_ERR_UNSUPPORTED;
      }
      off[q * (na + 1) + na] = (int)tot[q];
    }
    if (fail != PQR_OK) break;
    HIPCHK(hipMemcpyAsync(desc_d, desc.data(), sizeof(GroupDesc<T>) * na, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(off_d, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, s));
    for (int64_t k = 0; k < chunk; ++k)
      HIPCHK(launch_grouped_iteration<T>(c0->g, desc_d, off_d, na, tot, s,
                                         prof ? c0->events[2 * k] : nullptr,
                                         prof ? c0->events[2 * k + 1] : nullptr));
    HIPCHK(hipStreamSynchronize(s));
    if (prof) {
      for (int64_t k = 0; k < chunk; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c0->events[2 * k], c0->events[2 * k + 1]));
        sweep_ms += ms;
      }
      sweeps += chunk;
    }
    for (int i : act) {
      st[i] = runs[i].after_chunk(chunk);
      if (st[i] != PQR_OK) runs[i].status = st[i];
    }
  }
  pqr_status first = fail;
  for (int i = 0; i < nprob; ++i) {
    if (runs[i].ctx && st[i] == PQR_OK) {
      runs[i].sweep_ms = sweep_ms;
      runs[i].sweeps = sweeps;
      st[i] = runs[i].finish(outs ? &outs[i] : nullptr);
    }
    if (statuses) statuses[i] = st[i];
    if (first == PQR_OK && st[i] != PQR_OK) first = st[i];
  }
  return first;
}

}  // namespace

extern "C" pqr_status pqr_solve(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                const double* weights, int start, const pqr_result* warm,
                                pqr_result* out) {
  Range range_("pqr_solve");
  if (!ctx) return PQR_ERR_INVALID_ARG;
  if (start < PQR_START_ZERO || start > PQR_START_DEVICE) {
    ctx->err = "unknown start mode";
    return PQR_ERR_INVALID_ARG;
  }
  if (ctx->opt.iter_prec == PQR_ITER_F64)
    return solve_impl<double>(ctx, y, tau, lambda, weights, start, warm, out);
  return solve_impl<float>(ctx, y, tau, lambda, weights, start, warm, out);
}

extern "C" pqr_status pqr_solve_grouped(int nprob, pqr_ctx* const* ctxs, const double* const* ys,
                                        const double* taus, const double* lambdas,
                                        const double* const* weights, pqr_result* outs,
                                        pqr_status* statuses) {
  Range range_("pqr_solve_grouped");
  if (nprob < 1 || !ctxs || !ys || !taus || !lambdas) return PQR_ERR_INVALID_ARG;
  for (int i = 0; i < nprob; ++i)
    if (!ctxs[i]) return PQR_ERR_INVALID_ARG;
  pqr_ctx* c0 = ctxs[0];
  for (int i = 0; i < nprob; ++i) {
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) {
        c0->err = "pqr_solve_grouped: a context appears twice";
        return PQR_ERR_INVALID_ARG;
      }
    if (ctxs[i]->opt.iter_prec != c0->opt.iter_prec || ctxs[i]->g.fmt != c0->g.fmt ||
        ctxs[i]->g.rpl != c0->g.rpl) {
      c0->err = "pqr_solve_grouped: every context needs the same store format, rows per lane "
                "and iterate precision";
      return PQR_ERR_UNSUPPORTED;
    }
  }
  if (c0->opt.iter_prec == PQR_ITER_F64)
    return grouped_impl<double>(nprob, ctxs, ys, taus, lambdas, weights, outs, statuses);
  return grouped_impl<float>(nprob, ctxs, ys, taus, lambdas, weights, outs, statuses);
}

namespace {
template <typename T>
pqr_status iterate_impl(pqr_ctx* ctx, const double* y, double tau, double lambda,
                        const double* weights, double mu, const double* eta, int64_t iters,
                        double* beta_std, double* z, double* theta) {
  TRY(validate_problem(ctx, y, tau, lambda, weights));
  if (!(mu > 0) || !eta || !beta_std || !z || !theta || iters < 0) {
    ctx->err = "pqr_iterate needs mu > 0, eta, beta_std, z, theta and iters >= 0";
    return PQR_ERR_INVALID_ARG;
  }
  for (int b = 0; b < ctx->G; ++b)
    if (!(eta[b] > 0) || !std::isfinite(eta[b])) {
      ctx->err = "eta must be positive";
      return PQR_ERR_INVALID_ARG;
    }
  TRY(upload_problem<T>(ctx, y, tau, lambda, weights, nullptr, nullptr));
  IterParams ip{};
  TRY(set_eta<T>(ctx, mu, eta, 1.0, ip, tau));
  TRY(init_state<T>(ctx, PQR_START_HOST, beta_std, z, theta, ip));
  const IterBufs<T> b = bufs<T>(ctx);
  for (int64_t k = 0; k < iters; ++k) HIPCHK(launch_iteration<T>(ctx->g, b, ip, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  ctx->have_state = true;
  ctx->state_mu = mu;
  pqr_result r{};
  r.beta_std = beta_std;
  r.z = z;
  r.theta = theta;
  Ctl c;
  HIPCHK(hipMemcpyAsync(&c, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  return export_state<T>(ctx, &r, ctx->beta, c.beta0, ctx->z, ctx->theta);
}
}  // namespace

// Algorithm 2: L-step LLA for SCAD / MCP on top of the weighted-l1 solve.
extern "C" pqr_status pqr_solve_lla(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                    int penalty, double a, int L, double wfloor, int start,
                                    double* weights_out, int64_t* stage_iters, pqr_result* out) {
  Range range_("pqr_solve_lla");
  if (!ctx) return PQR_ERR_INVALID_ARG;
  if (penalty != 0 && penalty != 1) {
    ctx->err = "penalty must be 0 (SCAD) or 1 (MCP)";
    return PQR_ERR_INVALID_ARG;
  }
  if (!(std::isfinite(a) && (penalty == 0 ? a > 2.0 : a > 1.0))) {
    ctx->err = "SCAD needs a > 2, MCP needs a > 1";
    return PQR_ERR_INVALID_ARG;
  }
  if (L < 0 || !(wfloor >= 0.0 && wfloor <= 1.0) || !(lambda > 0.0) || !std::isfinite(lambda) ||
      (start != PQR_START_ZERO && start != PQR_START_DEVICE)) {
    ctx->err = "pqr_solve_lla needs L >= 0, 0 <= wfloor <= 1, lambda > 0 and a zero or device start";
    return PQR_ERR_INVALID_ARG;
  }
  const Geom& g = ctx->g;
  std::vector<double> w(g.p + 1, 1.0);
  w[0] = 0.0;
  pqr_result tmp{};
  pqr_result* res = out ? out : &tmp;
  // stage 0: the weighted-l1 solve at unit weights, from a zero start or the device state
  pqr_status st = pqr_solve(ctx, y, tau, lambda, nullptr, start, nullptr, res);
  if (stage_iters) stage_iters[0] = res->iters;
  double sweep_ms = res->sweep_ms;
  int64_t sweeps = res->sweep_launches;
  if (st != PQR_OK) return st;
  for (int l = 1; l <= L; ++l) {
    // weights from the stage's returned (best primal) coefficients, on the device
    if (ctx->opt.iter_prec == PQR_ITER_F64)
      HIPCHK(launch_lla_weights<double>((const double*)ctx->beta_best, g.p, penalty, a, lambda,
                                        wfloor, ctx->scratch64, ctx->s));
    else
      HIPCHK(launch_lla_weights<float>((const float*)ctx->beta_best, g.p, penalty, a, lambda,
                                       wfloor, ctx->scratch64, ctx->s));
    HIPCHK(hipMemcpyAsync(w.data(), ctx->scratch64, (g.p + 1) * 8, hipMemcpyDeviceToHost, ctx->s));
    HIPCHK(hipStreamSynchronize(ctx->s));
    st = pqr_solve(ctx, y, tau, lambda, w.data(), PQR_START_DEVICE, nullptr, res);
    if (stage_iters) stage_iters[l] = res->iters;
    sweep_ms += res->sweep_ms;
    sweeps += res->sweep_launches;
    res->sweep_ms = sweep_ms;          // with opt.profile: summed over the stages
    res->sweep_launches = sweeps;
    if (st != PQR_OK) return st;
  }
  if (weights_out) std::memcpy(weights_out, w.data(), (g.p + 1) * 8);
  return PQR_OK;
}

extern "C" pqr_status pqr_iterate(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                  const double* weights, double mu, const double* eta,
                                  int64_t iters, double* beta_std, double* z, double* theta) {
  if (!ctx) return PQR_ERR_INVALID_ARG;
  if (ctx->opt.iter_prec == PQR_ITER_F64)
    return iterate_impl<double>(ctx, y, tau, lambda, weights, mu, eta, iters, beta_std, z, theta);
  return iterate_impl<float>(ctx, y, tau, lambda, weights, mu, eta, iters, beta_std, z, theta);
}

static pqr_status kkt_impl(pqr_ctx* ctx, const double* y, double tau, double lambda,
                           const double* weights, const double* beta_std, const double* theta,
                           double rep[4], double* v_out) {
  if (!ctx) return PQR_ERR_INVALID_ARG;
  TRY(validate_problem(ctx, y, tau, lambda, weights));
  if (!beta_std || !theta || !rep) {
    ctx->err = "pqr_kkt needs beta_std, theta and rep";
    return PQR_ERR_INVALID_ARG;
  }
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  // only the FP64 buffers and the kkt control block are touched
  std::vector<double> yh(g.n_pad, 0.0);
  std::memcpy(yh.data(), y, g.n * 8);
  HIPCHK(hipMemcpyAsync(ctx->y_d, yh.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
  std::vector<double> lh(g.p_pad, 0.0);
  for (int64_t j = 0; j < g.p; ++j) lh[j] = lambda * (weights ? weights[1 + j] : 1.0);
  HIPCHK(hipMemcpyAsync(ctx->clam_d, lh.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
  std::vector<double> bh(g.p_pad, 0.0);
  std::memcpy(bh.data(), beta_std + 1, g.p * 8);
  HIPCHK(hipMemcpyAsync(ctx->beta_d, bh.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
  std::vector<double> th(g.n_pad, 0.0);
  std::memcpy(th.data(), theta, g.n * 8);
  HIPCHK(hipMemcpyAsync(ctx->scratch64, th.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  c.count = (int)g.ngroups();
  c.beta0 = beta_std[0];
  HIPCHK(hipMemcpyAsync(ctx->ctl_kkt, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
  HIPCHK(launch_project<double>(ctx->scratch64, g.n, g.n_pad, tau, ctx->y_d, ctx->theta_p,
                                ctx->out_d, s));
  set_unpenalized(ctx, weights);
  bool unpen_ok = true;
  if (!ctx->unpen.empty()) TRY(project_unpenalized(ctx, tau, &unpen_ok));
  HIPCHK(launch_dots64(g, ctx->theta_p, ctx->out_d + 5, ctx->cm_d, ctx->cinv_d, ctx->clam_d,
                       v_out ? ctx->v_d : nullptr, ctx->gpart, s));
  HIPCHK(launch_reduce_max(ctx->gpart, g.ngroups(), ctx->bpart64, ctx->out_d + 3, s));
  if (v_out) HIPCHK(hipMemcpyAsync(v_out, ctx->v_d, g.p * 8, hipMemcpyDeviceToHost, s));
  CertBufs cb{};
  cb.y = ctx->y_d;
  cb.theta_p = ctx->theta_p;
  cb.beta_d = ctx->beta_d;
  cb.cm = ctx->cm_d;
  cb.cinv = ctx->cinv_d;
  cb.clam = ctx->clam_d;
  cb.partial = ctx->partial64;
  cb.list = ctx->iota;
  cb.ctl = ctx->ctl_kkt;
  cb.bpart = ctx->bpart64;
  cb.out = ctx->out_d;
  HIPCHK(launch_primal64(g, cb, tau, ctx->smax, ctx->min_per, s));
  HIPCHK(hipMemcpyAsync(ctx->out_h, ctx->out_d, 16 * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double* o = ctx->out_h;
  const double mr = o[3];
  double alpha = mr > 1.0 ? (std::isinf(mr) ? 0.0 : 1.0 / mr) : 1.0;
  if (!unpen_ok) alpha = 0.0;   // the projection left x~_U^T theta above rounding level
  rep[0] = o[0] + o[1];
  rep[1] = alpha * o[2];
  rep[2] = (rep[0] - rep[1]) / std::max(std::fabs(rep[0]), 1e-300);
  rep[3] = mr;
  return PQR_OK;
}

extern "C" pqr_status pqr_kkt(pqr_ctx* ctx, const double* y, double tau, double lambda,
                              const double* weights, const double* beta_std, const double* theta,
                              double rep[4]) {
  Range range_("pqr_kkt");
  return kkt_impl(ctx, y, tau, lambda, weights, beta_std, theta, rep, nullptr);
}

extern "C" pqr_status pqr_kkt_columns(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                      const double* weights, const double* beta_std,
                                      const double* theta, double rep[4], double* v) {
  if (!v) {
    if (ctx) ctx->err = "pqr_kkt_columns needs v";
    return PQR_ERR_INVALID_ARG;
  }
  return kkt_impl(ctx, y, tau, lambda, weights, beta_std, theta, rep, v);
}

extern "C" pqr_status pqr_lambda_max(pqr_ctx* ctx, const double* y, double tau,
                                     const double* weights, double* lambda_max, double* score) {
  if (!ctx) return PQR_ERR_INVALID_ARG;
  TRY(validate_problem(ctx, y, tau, 0.0, weights));
  if (ctx->opt.iter_prec == PQR_ITER_F64)
    return upload_problem<double>(ctx, y, tau, 0.0, weights, lambda_max, score);
  return upload_problem<float>(ctx, y, tau, 0.0, weights, lambda_max, score);
}

extern "C" pqr_status pqr_blocks(pqr_ctx* ctx, int* G, int* bounds, double* Lambda) {
  if (!ctx) return PQR_ERR_INVALID_ARG;
  if (G) *G = ctx->G;
  if (bounds) std::memcpy(bounds, ctx->bounds.data(), (ctx->G + 1) * sizeof(int));
  if (Lambda) std::memcpy(Lambda, ctx->Lambda.data(), ctx->G * sizeof(double));
  return PQR_OK;
}

// ---------------------------------------------------------------------------
// Batched right-hand sides
// ---------------------------------------------------------------------------
namespace {

pqr_status batch_alloc(pqr_ctx* ctx, int Kp) {
  if (ctx->batch_kp >= Kp) return PQR_OK;
  const Geom& g = ctx->g;
  BatchBufs& b = ctx->bb;
  const int64_t nblk = g.n_pad / 256, ng = g.ngroups();
  TRY(dalloc(ctx, &b.beta, (size_t)Kp * g.p_pad * 4));
  float* w;
  TRY(dalloc(ctx, &w, g.p_pad * 4));
  b.w = w;
  float *lam, *tau, *geta;
  TRY(dalloc(ctx, &lam, Kp * 4));
  TRY(dalloc(ctx, &tau, Kp * 4));
  TRY(dalloc(ctx, &geta, ng * 4));
  b.lam = lam; b.tau = tau; b.geta = geta;
  if (!ctx->yb) TRY(dalloc(ctx, &ctx->yb, g.n_pad * 4));
  if (!ctx->w_d) TRY(dalloc(ctx, &ctx->w_d, g.p_pad * 8));
  b.y = ctx->yb;
  TRY(dalloc(ctx, &b.z, (size_t)Kp * g.n_pad * 4));
  TRY(dalloc(ctx, &b.theta, (size_t)Kp * g.n_pad * 4));
  TRY(dalloc(ctx, &ctx->btheta_best, (size_t)Kp * g.n_pad * 4));
  TRY(dalloc(ctx, &b.r, (size_t)Kp * g.n_pad * 4));
  TRY(dalloc(ctx, &b.dig, (size_t)3 * Kp * g.n_pad));
  TRY(dalloc(ctx, &b.tpart, (size_t)nblk * Kp * 8));
  TRY(dalloc(ctx, &b.tsumq, Kp * 8));
  TRY(dalloc(ctx, &b.tsum, Kp * 8));
  TRY(dalloc(ctx, &b.scale, Kp * 8));
  TRY(dalloc(ctx, &b.beta0, Kp * 8));
  TRY(dalloc(ctx, &b.norms, Kp * 4 * 8));
  TRY(dalloc(ctx, &b.mask, (size_t)ng * (Kp / 16) * 4));
  TRY(dalloc(ctx, &b.list, (size_t)g.p_pad * 4));
  TRY(dalloc(ctx, &b.bcnt, kCompactBlocks * 4));
  TRY(dalloc(ctx, &b.count, 64));
  TRY(dalloc(ctx, &b.partial, (size_t)kBaxpySplits * Kp * g.n_pad * 8));
  TRY(dalloc(ctx, &b.bpart, (size_t)nblk * Kp * 8 * 8));
  TRY(dalloc(ctx, &b.bd, (size_t)ng * Kp * 64));
  TRY(dalloc(ctx, &b.pmax, (size_t)256 * Kp * 8));
  TRY(dalloc(ctx, &b.poff, (size_t)256 * Kp * 8));
  TRY(dalloc(ctx, &b.bscale, (size_t)Kp * 8));
  int* kact = nullptr;
  TRY(dalloc(ctx, &kact, (size_t)Kp * 4));
  b.kact = kact;
  if (!ctx->cert4) {
    TRY(dalloc(ctx, &ctx->cert4, (size_t)4 * g.n_pad * 8));
    TRY(dalloc(ctx, &ctx->out4, 32 * 8));
    TRY(dalloc(ctx, &ctx->gmax4, (size_t)4 * ng * 8));
    TRY(dalloc(ctx, &ctx->cdig, (size_t)kCertSlices * 128 * g.n_pad));
    TRY(dalloc(ctx, &ctx->ctq, (size_t)g.n_pad * 4));
    TRY(dalloc(ctx, &ctx->cgmax, (size_t)128 * cert_group_sets(g) * 8));
    TRY(dalloc(ctx, &ctx->clamk, 128 * 8));
    TRY(dalloc(ctx, &ctx->cunit, 128 * 8));
    TRY(dalloc(ctx, &ctx->cout, 128 * 8 * 8));
  }
  b.cm = ctx->cm_f;
  b.cinv = ctx->cinv_f;
  ctx->batch_kp = Kp;
  return PQR_OK;
}

pqr_status batch_impl(pqr_ctx* ctx, const double* y, int K, const double* taus,
                      const double* lambdas, const double* weights, pqr_result* outs) {
  const auto t0 = std::chrono::steady_clock::now();
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  if (g.fmt != I8 || g.rpl != 16 || ctx->opt.iter_prec != PQR_ITER_F32) {
    ctx->err = "batched solves need an int8 store, rows_per_lane 16 and FP32 iterates";
    return PQR_ERR_UNSUPPORTED;
  }
  if (K < 1 || K > 128 || !taus || !lambdas) {
    ctx->err = "batched solves take 1 <= K <= 128 (tau_k, lambda_k) pairs";
    return PQR_ERR_INVALID_ARG;
  }
  for (int k = 0; k < K; ++k) TRY(validate_problem(ctx, y, taus[k], lambdas[k], weights));
  if (weights)
    for (int64_t j = 1; j <= g.p; ++j)
      if (weights[j] == 0.0) {
        ctx->err = "batched solves need positive weights (unpenalized columns: use pqr_solve)";
        return PQR_ERR_UNSUPPORTED;
      }
  if (ctx->max_code < 0) {   // the matrix cores read the int8 codes as signed
    int* mc = nullptr;
    TRY(dalloc(ctx, &mc, 64));
    HIPCHK(launch_max_code(g, mc, s));
    HIPCHK(hipMemcpyAsync(&ctx->max_code, mc, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (ctx->max_code > 127) {
    ctx->err = "batched solves need int8 codes 0..127 (the store holds " +
               std::to_string(ctx->max_code) + ")";
    return PQR_ERR_UNSUPPORTED;
  }
  // Exactness limits of the integer products: an int32 matrix-core accumulator
  // sums n_pad products code * digit with |digit| <= 64, and the digit buffers
  // (up to 4 slices x 128 rows of n_pad bytes) are addressed with 32-bit offsets.
  if ((int64_t)g.n_pad * std::max(ctx->max_code, 1) * 65 >= ((int64_t)1 << 31) ||
      (int64_t)4 * 128 * g.n_pad >= ((int64_t)1 << 31)) {
    ctx->err = "batched solves: n_pad * max_code * 65 and 512 * n_pad must stay below 2^31 "
               "(n_pad " + std::to_string(g.n_pad) + ", max code " +
               std::to_string(ctx->max_code) + ")";
    return PQR_ERR_UNSUPPORTED;
  }
  // fewest splits of the union product that keep its int32 slice sums exact: a
  // split of the (at most p_pad) union columns holds at most lim_steps 64-column steps
  const int min_per = 4;
  const int64_t lim_steps = (((int64_t)1 << 31) - 1) / (64 * std::max(ctx->max_code, 1)) / 64;
  const int smin = (int)(((g.p_pad + 63) / 64 + lim_steps - 1) / lim_steps);
  if (smin > kBaxpySplits) {
    ctx->err = "batched solves: the union product needs " + std::to_string(smin) +
               " splits of at most (2^31 - 1) / (64 max_code) columns, more than " +
               std::to_string(kBaxpySplits) + " (p_pad " + std::to_string(g.p_pad) +
               ", max code " + std::to_string(ctx->max_code) + ")";
    return PQR_ERR_UNSUPPORTED;
  }
  const int Kp = (K + 15) / 16 * 16;
  TRY(batch_alloc(ctx, Kp));
  BatchBufs b = ctx->bb;
  b.K = K;
  const int64_t ng = g.ngroups();
  // inputs
  std::vector<double> yh(g.n_pad, 0.0);
  std::memcpy(yh.data(), y, g.n * 8);
  HIPCHK(hipMemcpyAsync(ctx->y_d, yh.data(), g.n_pad * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_set_y<float>(ctx->y_d, g.n, g.n_pad, ctx->yb, s));
  std::vector<double> wh(g.p_pad, 0.0);
  std::vector<float> wf(g.p_pad, 0.f);
  for (int64_t j = 0; j < g.p; ++j) { wh[j] = weights ? weights[1 + j] : 1.0; wf[j] = (float)wh[j]; }
  HIPCHK(hipMemcpyAsync(ctx->w_d, wh.data(), g.p_pad * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync((void*)b.w, wf.data(), g.p_pad * 4, hipMemcpyHostToDevice, s));
  std::vector<float> lf(Kp, 0.f), tf(Kp, 0.5f);
  for (int k = 0; k < K; ++k) { lf[k] = (float)lambdas[k]; tf[k] = (float)taus[k]; }
  HIPCHK(hipMemcpyAsync((void*)b.lam, lf.data(), Kp * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync((void*)b.tau, tf.data(), Kp * 4, hipMemcpyHostToDevice, s));
  const double mu = ctx->opt.mu > 0 ? ctx->opt.mu : default_mu(ctx, y);
  std::vector<float> ge(ng);
  std::vector<double> eta(ctx->G);
  for (int q = 0; q < ctx->G; ++q) eta[q] = (1.0 + ctx->opt.eta_margin) * mu * ctx->Lambda[q];
  for (int64_t q = 0; q < ng; ++q) ge[q] = (float)eta[ctx->gblock_h[q]];
  HIPCHK(hipMemcpyAsync((void*)b.geta, ge.data(), ng * 4, hipMemcpyHostToDevice, s));
  // Autotuner, back-product: on the first batched solve of this width every launch
  // variant runs once and is then timed over three launches on zero digits (the
  // kernel's work does not depend on the values); the state is reset afterwards.
  pqr_ctx::TileChoice& tc = ctx->tiles[Kp];
  if (ctx->opt.tile_override > 0) {
    const int o = ctx->opt.tile_override - 1;
    if (o / PQR_TILE_VARIANTS >= bgemm_variants() || o % PQR_TILE_VARIANTS >= baxpy_variants()) {
      ctx->err = "tile_override out of range";
      return PQR_ERR_INVALID_ARG;
    }
    tc.tiles.bgemm = o / PQR_TILE_VARIANTS;
    tc.tiles.baxpy = o % PQR_TILE_VARIANTS;
    tc.bgemm_done = tc.baxpy_done = true;
  }
  auto time_launches = [&](auto&& launch, double* ms) -> pqr_status {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipError_t e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(e);
    *ms = t / 3.0;
    return PQR_OK;
  };
  if (!tc.bgemm_done) {
    std::vector<int> all(Kp, 1);
    HIPCHK(hipMemcpyAsync(const_cast<int*>(b.kact), all.data(), Kp * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(b.dig, 0, (size_t)3 * Kp * g.n_pad, s));
    HIPCHK(launch_batch_zero(g, b, Kp, s));
    tc.bgemm_ms.assign(bgemm_variants(), 0.0);
    int best = 0;
    for (int v = 0; v < bgemm_variants(); ++v) {
      TRY(time_launches([&]() { return launch_bgemm_variant(g, b, Kp, v, s); }, &tc.bgemm_ms[v]));
      if (tc.bgemm_ms[v] < tc.bgemm_ms[best]) best = v;
    }
    tc.tiles.bgemm = best;
    tc.bgemm_done = true;
  }
  HIPCHK(hipMemsetAsync(b.beta, 0, (size_t)Kp * g.p_pad * 4, s));
  HIPCHK(launch_batch_zero(g, b, Kp, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->have_state = false;   // the single right-hand-side state is not the batch's

  const double sigma = mu / (ctx->G + 1.0);
  std::vector<double> best_dual(K, -INFINITY), primal(K, INFINITY), rel(K, INFINITY);
  std::vector<char> done(K, 0);
  std::vector<int64_t> done_it(K, 0);   // iteration at which right-hand side k was certified
  int64_t it = 0, certs = 0;
  int ndone = 0;
  // convergence masks: a right-hand side whose certificate met tol_gap is frozen
  // (its state is the certified point) and leaves the union of active columns
  std::vector<int> kact(Kp, 0);
  auto push_masks = [&]() -> pqr_status {
    for (int k = 0; k < Kp; ++k) kact[k] = k < K && !done[k];
    HIPCHK(hipMemcpyAsync(const_cast<int*>(b.kact), kact.data(), Kp * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return PQR_OK;
  };
  // P(beta_k) into out[0] + out[1] (the sparse primal, FP64).
  auto primal_of = [&](int k, double* out) -> pqr_status {
    const float* bk = b.beta + (size_t)k * g.p_pad;
    double b0 = 0.0;
    HIPCHK(hipMemcpyAsync(&b0, b.beta0 + k, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    Ctl c;
    std::memset(&c, 0, sizeof(c));
    c.beta0 = b0;
    HIPCHK(hipMemcpyAsync(ctx->ctl_kkt, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
    IterBufs<float> v = bufs<float>(ctx);
    v.beta = const_cast<float*>(bk);
    v.ctl = ctx->ctl_kkt;
    HIPCHK(launch_active_list<float>(g, v, s));
    HIPCHK(launch_scale(ctx->w_d, lambdas[k], g.p_pad, ctx->clam_d, s));
    HIPCHK(launch_to_double<float>(bk, g.p_pad, ctx->beta_d, s));
    CertBufs cb{};
    cb.y = ctx->y_d;
    cb.theta_p = ctx->cert4;
    cb.beta_d = ctx->beta_d;
    cb.cm = ctx->cm_d;
    cb.cinv = ctx->cinv_d;
    cb.clam = ctx->clam_d;
    cb.partial = ctx->partial64;
    cb.list = ctx->list;
    cb.ctl = ctx->ctl_kkt;
    cb.bpart = ctx->bpart64;
    cb.out = out;
    HIPCHK(launch_primal64(g, cb, taus[k], ctx->smax, ctx->min_per, s));
    HIPCHK(hipStreamSynchronize(s));   // c and b0 leave scope
    return PQR_OK;
  };
  // o = [primal loss, penalty, y^T theta, max ratio, ...]: alpha = min(1, 1 / ratio)
  // The dual point of the best dual value is kept (its theta) so that the exported
  // (beta, theta) reproduce the reported primal and dual values.
  auto finish = [&](int k, const double* o) -> pqr_status {
    const double mr = o[3];
    const double alpha = mr > 1.0 ? (std::isinf(mr) ? 0.0 : 1.0 / mr) : 1.0;
    ++certs;
    if (alpha * o[2] > best_dual[k]) {
      best_dual[k] = alpha * o[2];
      HIPCHK(hipMemcpyAsync(ctx->btheta_best + (size_t)k * g.n_pad, b.theta + (size_t)k * g.n_pad,
                            g.n_pad * 4, hipMemcpyDeviceToDevice, s));
    }
    primal[k] = o[0] + o[1];
    rel[k] = (primal[k] - best_dual[k]) / std::max(std::fabs(primal[k]), 1e-300);
    return PQR_OK;
  };
  // FP64 certificates, four right-hand sides per pass over X: the projections per
  // k, one shared pass for the dual ratios, then the sparse primal per k.  Same
  // arithmetic as pqr_kkt.
  std::vector<double> bout(32);
  auto certify_fp64 = [&](const std::vector<int>& ks) -> pqr_status {
    for (size_t c0 = 0; c0 < ks.size(); c0 += 4) {
      const int kb = (int)std::min<size_t>(4, ks.size() - c0);
      double lam4[4] = {0, 0, 0, 0};
      for (int i = 0; i < kb; ++i) {
        const int k = ks[c0 + i];
        lam4[i] = lambdas[k];
        HIPCHK(launch_project<float>(b.theta + (size_t)k * g.n_pad, g.n, g.n_pad, taus[k], ctx->y_d,
                                     ctx->cert4 + (size_t)i * g.n_pad, ctx->out4 + 8 * i, s));
      }
      HIPCHK(launch_mdots64(g, ctx->cert4, kb, ctx->out4, ctx->cm_d, ctx->cinv_d, ctx->w_d, lam4,
                            ctx->gmax4, s));
      for (int i = 0; i < kb; ++i)
        HIPCHK(launch_reduce_max(ctx->gmax4 + (size_t)i * ng, ng, ctx->bpart64,
                                 ctx->out4 + 8 * i + 3, s));
      for (int i = 0; i < kb; ++i) TRY(primal_of(ks[c0 + i], ctx->out4 + 8 * i));
      HIPCHK(hipMemcpyAsync(bout.data(), ctx->out4, 32 * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < kb; ++i) TRY(finish(ks[c0 + i], bout.data() + 8 * i));
    }
    return PQR_OK;
  };
  // Exact certificates of the right-hand sides in `ks`: per k the projection
  // theta' and its quantisation theta_q = unit_k T_k (inside the box, sum exactly
  // zero), then ONE int8 matrix-core pass over X for the dual ratios of all of
  // them (x~_j^T theta_q exact in integers), then the sparse primal per k.  A k
  // whose sum cannot be zeroed inside the box is certified in FP64 instead.
  std::vector<double> cout_h(8 * 128), lam_h(128), unit_h(128);
  const int64_t ngs = cert_group_sets(g);
  auto certify_many = [&](const std::vector<int>& ks) -> pqr_status {
    std::vector<int> fallback;
    for (size_t c0 = 0; c0 < ks.size(); c0 += 128) {
      const int nk = (int)std::min<size_t>(128, ks.size() - c0);
      const int Kc = (nk + 15) / 16 * 16;
      for (int i = 0; i < Kc; ++i) { lam_h[i] = 1.0; unit_h[i] = 0.0; }
      for (int i = 0; i < nk; ++i) {
        const int k = ks[c0 + i];
        // unit = c 2^-27 with c the power of two >= max(tau, 1 - tau) / n >= |theta'_i|
        int e = 0;
        (void)std::frexp(std::max(taus[k], 1.0 - taus[k]) / (double)g.n, &e);
        unit_h[i] = std::ldexp(1.0, e - (7 * kCertSlices - 1));
        lam_h[i] = lambdas[k];
        HIPCHK(launch_project<float>(b.theta + (size_t)k * g.n_pad, g.n, g.n_pad, taus[k], ctx->y_d,
                                     ctx->cert4, ctx->out4, s));
        HIPCHK(launch_cert_quantize(ctx->cert4, g.n, g.n_pad, taus[k], unit_h[i], ctx->y_d, ctx->ctq,
                                    ctx->cdig, i, Kc, ctx->cout + 8 * i, s));
      }
      HIPCHK(hipMemcpyAsync(ctx->clamk, lam_h.data(), Kc * 8, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(ctx->cunit, unit_h.data(), Kc * 8, hipMemcpyHostToDevice, s));
      CertArgs ca{};
      ca.dig = ctx->cdig;
      ca.lam = ctx->clamk;
      ca.unit = ctx->cunit;
      ca.w = ctx->w_d;
      ca.cinv = ctx->cinv_d;
      ca.gmax = ctx->cgmax;
      ca.K = nk;
      HIPCHK(launch_cert_pass(g, ca, Kc, s));
      for (int i = 0; i < nk; ++i)
        HIPCHK(launch_reduce_max(ctx->cgmax + (size_t)i * ngs, ngs, ctx->bpart64,
                                 ctx->cout + 8 * i + 3, s));
      for (int i = 0; i < nk; ++i) TRY(primal_of(ks[c0 + i], ctx->cout + 8 * i));
      HIPCHK(hipMemcpyAsync(cout_h.data(), ctx->cout, (size_t)nk * 8 * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < nk; ++i) {
        if (cout_h[8 * i + 7] != 0.0) fallback.push_back(ks[c0 + i]);
        else TRY(finish(ks[c0 + i], cout_h.data() + 8 * i));
      }
    }
    if (!fallback.empty()) TRY(certify_fp64(fallback));
    for (int k : ks)
      if (rel[k] <= ctx->opt.tol_gap && !done[k]) { done[k] = 1; done_it[k] = it; ++ndone; }
    return PQR_OK;
  };
  auto pending = [&]() {
    std::vector<int> ks;
    for (int k = 0; k < K; ++k)
      if (!done[k]) ks.push_back(k);
    return ks;
  };
  // Certificate schedule (each certificate is a full FP64 pass over X per four
  // right-hand sides): from the last two certified gaps of a right-hand side the
  // rounds still needed to reach the target are extrapolated (log-linear) and its
  // next certificate is due after 80 % of them, at least 1 and at most 8 rounds.
  std::vector<int64_t> last_round(K, -1000), next_round(K, 0), gap_wait(K, 1);
  auto wait_of = [&](int k) { return gap_wait[k]; };
  std::vector<double> prev_rel(K, INFINITY);
  int64_t round = 0;
  auto due = [&]() {
    std::vector<int> ks;
    for (int k = 0; k < K; ++k)
      if (!done[k] && round >= next_round[k]) {
        ks.push_back(k);
        last_round[k] = round;
      }
    ++round;
    return ks;
  };
  auto reschedule = [&](const std::vector<int>& ks) {
    const double tol = ctx->opt.tol_gap;
    for (int k : ks) {
      int64_t wait = 1;
      if (std::isfinite(prev_rel[k]) && std::isfinite(rel[k]) && rel[k] > tol && rel[k] < prev_rel[k] &&
          tol > 0) {
        const double rate = std::log(prev_rel[k] / rel[k]) / (double)std::max<int64_t>(1, wait_of(k));
        const double need = std::log(rel[k] / tol) / rate;
        wait = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(0.8 * need)));
      }
      prev_rel[k] = rel[k];
      next_round[k] = last_round[k] + wait;
      gap_wait[k] = wait;
    }
  };
  const bool prof = ctx->opt.profile != 0;
  if (prof && ctx->events.size() < 2 * (size_t)ctx->opt.cert_every) {
    const size_t old = ctx->events.size();
    ctx->events.resize(2 * (size_t)ctx->opt.cert_every);
    for (size_t e = old; e < ctx->events.size(); ++e) HIPCHK(hipEventCreate(&ctx->events[e]));
  }
  double gemm_ms = 0.0;
  int64_t gemm_launches = 0;
  while (ndone < K && it < ctx->opt.max_iter) {
    TRY(push_masks());
    const int64_t chunk = std::min<int64_t>(ctx->opt.cert_every, ctx->opt.max_iter - it);
    for (int64_t q = 0; q < chunk; ++q)
      HIPCHK(launch_batch_iteration(g, b, Kp, mu, sigma, eta[0], smin, min_per, tc.tiles, s,
                                    prof ? ctx->events[2 * q] : nullptr,
                                    prof ? ctx->events[2 * q + 1] : nullptr));
    it += chunk;
    int ucount = 0;
    if (!tc.baxpy_done) {
      HIPCHK(hipMemcpyAsync(&ucount, b.count, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    if (!tc.baxpy_done && ucount >= 1024) {   // at least 16 matrix-core steps of union
      // Autotuner, union product: between two iterations the union of nonzero
      // columns and its digits are those of a live iterate, and the product's
      // partials are rewritten by the next iteration before they are read, so the
      // variants (equal results: exact integer sums) are timed on the real union.
      tc.baxpy_ms.assign(baxpy_variants(), 0.0);
      int best = 0;
      for (int v = 0; v < baxpy_variants(); ++v) {
        TRY(time_launches([&]() { return launch_baxpy_variant(g, b, Kp, smin, min_per, v, s); },
                          &tc.baxpy_ms[v]));
        if (tc.baxpy_ms[v] < tc.baxpy_ms[best]) best = v;
      }
      tc.tiles.baxpy = best;
      tc.baxpy_done = true;
      tc.union_cols = ucount;
    }
    HIPCHK(hipStreamSynchronize(s));
    if (prof) {
      for (int64_t q = 0; q < chunk; ++q) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->events[2 * q], ctx->events[2 * q + 1]));
        gemm_ms += ms;
      }
      gemm_launches += chunk;
    }
    {
      const std::vector<int> ks = due();
      TRY(certify_many(ks));
      reschedule(ks);
    }
  }
  // the returned iterate of a frozen right-hand side is its certified point; the
  // others get a certificate of where max_iter left them unless the last round
  // already took it
  {
    std::vector<int> ks;
    for (int k = 0; k < K; ++k)
      if (!done[k] && (it == 0 || last_round[k] != round - 1)) ks.push_back(k);
    if (!ks.empty()) TRY(certify_many(ks));
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (outs) {
    std::vector<float> bf(g.p), vf(g.n);
    for (int k = 0; k < K; ++k) {
      pqr_result* o = outs + k;
      double b0 = 0.0;
      HIPCHK(hipMemcpyAsync(&b0, b.beta0 + k, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(bf.data(), b.beta + (size_t)k * g.p_pad, g.p * 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      int64_t nnz = 0;
      for (int64_t j = 0; j < g.p; ++j) nnz += bf[j] != 0.f;
      if (o->beta_std) {
        o->beta_std[0] = b0;
        for (int64_t j = 0; j < g.p; ++j) o->beta_std[1 + j] = bf[j];
      }
      if (o->beta) {
        std::vector<double> bs(g.p + 1);
        bs[0] = b0;
        for (int64_t j = 0; j < g.p; ++j) bs[1 + j] = bf[j];
        HIPCHK(hipMemcpyAsync(ctx->scratch64, bs.data(), (g.p + 1) * 8, hipMemcpyHostToDevice, s));
        HIPCHK(launch_back_transform(ctx->scratch64, g.p, ctx->cm_d, ctx->cinv_d, b0, ctx->bt_out,
                                     ctx->bpart64, s));
        HIPCHK(hipMemcpyAsync(o->beta, ctx->bt_out, (g.p + 1) * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
      }
      if (o->z || o->theta) {
        for (int which = 0; which < 2; ++which) {
          double* dst = which == 0 ? o->z : o->theta;
          if (!dst) continue;
          const float* src = (which == 0 ? b.z : ctx->btheta_best) + (size_t)k * g.n_pad;
          HIPCHK(hipMemcpyAsync(vf.data(), src, g.n * 4, hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          for (int64_t i = 0; i < g.n; ++i) dst[i] = vf[i];
        }
      }
      o->iters = done[k] ? done_it[k] : it;   // k is frozen once certified
      o->certs = certs;
      o->x_passes = it + certs;
      o->nnz = nnz;
      o->primal = primal[k];
      o->dual = best_dual[k];
      o->rel_gap = rel[k];
      o->lambda_max = 0.0;
      o->mu = mu;
      o->seconds = secs;
      o->sweep_ms = gemm_ms;             // with opt.profile: the back-product kernel
      o->sweep_launches = gemm_launches;
    }
  }
  if (ndone < K) {
    ctx->err = "max_iter reached before every right-hand side met tol_gap";
    return PQR_ERR_NOT_CONVERGED;
  }
  return PQR_OK;
}

}  // namespace

static_assert(kBgemmVariants <= PQR_TILE_VARIANTS && kBaxpyVariants <= PQR_TILE_VARIANTS,
              "more launch variants than pqr_batch_tiles reports");

extern "C" pqr_status pqr_batch_tiles(pqr_ctx* ctx, int K, int* bgemm_variant, int* baxpy_variant,
                                      double* bgemm_ms, double* baxpy_ms, int64_t* union_cols) {
  if (!ctx || K < 1 || K > 128) return PQR_ERR_INVALID_ARG;
  const int Kp = (K + 15) / 16 * 16;
  auto it = ctx->tiles.find(Kp);
  if (it == ctx->tiles.end() || !it->second.bgemm_done) {
    ctx->err = "no batched solve of this width has run on the context";
    return PQR_ERR_INVALID_ARG;
  }
  const pqr_ctx::TileChoice& tc = it->second;
  if (bgemm_variant) *bgemm_variant = tc.tiles.bgemm;
  if (baxpy_variant) *baxpy_variant = tc.baxpy_done ? tc.tiles.baxpy : -1;
  if (union_cols) *union_cols = tc.union_cols;
  for (int v = 0; v < PQR_TILE_VARIANTS; ++v) {
    if (bgemm_ms) bgemm_ms[v] = v < (int)tc.bgemm_ms.size() ? tc.bgemm_ms[v] : 0.0;
    if (baxpy_ms) baxpy_ms[v] = v < (int)tc.baxpy_ms.size() ? tc.baxpy_ms[v] : 0.0;
  }
  return PQR_OK;
}

extern "C" pqr_status pqr_solve_batch(pqr_ctx* ctx, const double* y, int K, const double* taus,
                                      const double* lambdas, const double* weights,
                                      pqr_result* outs) {
  Range range_("pqr_solve_batch");
  if (!ctx) return PQR_ERR_INVALID_ARG;
  return batch_impl(ctx, y, K, taus, lambdas, weights, outs);
}

// ---------------------------------------------------------------------------
// Column subsets, the scoring network and the learned warm start
// ---------------------------------------------------------------------------
extern "C" pqr_status pqr_create_subset(pqr_ctx** out, pqr_ctx* parent, const int64_t* cols,
                                        int64_t ncols, const pqr_options* opt) {
  if (!out) return PQR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!parent) return PQR_ERR_INVALID_ARG;
  pqr_ctx* ctx = new pqr_ctx();
  ctx->opt = opt ? *opt : parent->opt;
  if (ctx->opt.mu_scale <= 0) ctx->opt.mu_scale = parent->opt.mu_scale;
  if (ctx->opt.eta_margin == 0 || ctx->opt.eta_margin <= -1) ctx->opt.eta_margin = 0.01;
  if (ctx->opt.tol_gap <= 0) ctx->opt.tol_gap = parent->opt.tol_gap;
  if (ctx->opt.cert_every <= 0) ctx->opt.cert_every = parent->opt.cert_every;
  if (ctx->opt.max_iter <= 0) ctx->opt.max_iter = parent->opt.max_iter;
  if (ctx->opt.iter_prec != PQR_ITER_F64) ctx->opt.iter_prec = PQR_ITER_F32;
  ctx->s = (hipStream_t)ctx->opt.stream;
  *out = ctx;
  if (!cols || ncols < 1) {
    ctx->err = "pqr_create_subset needs at least one column";
    return PQR_ERR_INVALID_ARG;
  }
  for (int64_t c = 0; c < ncols; ++c)
    if (cols[c] < 0 || cols[c] >= parent->g.p) {
      ctx->err = "column index out of range";
      return PQR_ERR_INVALID_ARG;
    }
  return create_subset_impl(ctx, parent, cols, ncols);
}

extern "C" pqr_status pqr_interleaved_order(int64_t p, int G, int64_t* cols) {
  if (p < 1 || G < 1 || G > p || !cols) return PQR_ERR_INVALID_ARG;
  int64_t q = 0;
  for (int r = 0; r < G; ++r)
    for (int64_t j = r; j < p; j += G) cols[q++] = j;
  return PQR_OK;
}

extern "C" pqr_status pqr_features(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                   const double* weights, float* feats, double* lambda_max) {
  if (!ctx) return PQR_ERR_INVALID_ARG;
  TRY(validate_problem(ctx, y, tau, lambda, weights));
  if (!feats) { ctx->err = "feats is NULL"; return PQR_ERR_INVALID_ARG; }
  double lm = 0.0;
  if (ctx->opt.iter_prec == PQR_ITER_F64) TRY(upload_problem<double>(ctx, y, tau, lambda, weights, &lm, nullptr));
  else TRY(upload_problem<float>(ctx, y, tau, lambda, weights, &lm, nullptr));
  const double loglam = std::log(std::max(lambda, 1e-300) / std::max(lm, 1e-300));
  HIPCHK(launch_features(ctx->v_d, ctx->cm_d, ctx->cinv_d, ctx->g.p, (double)ctx->g.n, tau, loglam,
                         feats, ctx->s));
  HIPCHK(hipStreamSynchronize(ctx->s));
  if (lambda_max) *lambda_max = lm;
  return PQR_OK;
}

extern "C" int64_t pqr_mlp_param_count(void) { return 4610; }

extern "C" int64_t pqr_mlp_workspace_bytes(int64_t B) {
  const int64_t np = mlp_grad_partials(B < 1 ? 1 : B);
  return np * 4610 * 4 + np * 4 + 256;
}

extern "C" pqr_status pqr_mlp_forward(const float* params, const float* feats, int64_t B, float* out,
                                      void* stream) {
  if (!params || !feats || !out || B < 0) return PQR_ERR_INVALID_ARG;
  if (B == 0) return PQR_OK;
  if (launch_mlp_forward(params, feats, B, out, (hipStream_t)stream) != hipSuccess)
    return PQR_ERR_DEVICE;
  return PQR_OK;
}

extern "C" pqr_status pqr_mlp_grad(const float* params, const float* feats, const float* target,
                                   const float* active, int64_t B, double w_reg, double w_pos,
                                   void* workspace, float* grad, float* loss, void* stream) {
  if (!params || !feats || !target || !active || !workspace || !grad || B < 1)
    return PQR_ERR_INVALID_ARG;
  const int64_t np = mlp_grad_partials(B);
  float* part = static_cast<float*>(workspace);
  float* lpart = part + np * 4610;
  if (launch_mlp_grad(params, feats, target, active, B, (float)w_reg, (float)w_pos, part, lpart,
                      grad, loss, (hipStream_t)stream) != hipSuccess)
    return PQR_ERR_DEVICE;
  return PQR_OK;
}

extern "C" pqr_status pqr_mlp_grad_noalloc(const float* params, const float* feats,
                                           const float* target, const float* active, int64_t B,
                                           double w_reg, double w_pos, float* grad, float* loss,
                                           void* stream) {
  static_assert(PQR_MLP_NOALLOC_MAX_ROWS == kMlpNoAllocRows, "header and kernel limits differ");
  if (!params || !feats || !target || !active || !grad || B < 1) return PQR_ERR_INVALID_ARG;
  if (B > PQR_MLP_NOALLOC_MAX_ROWS) return PQR_ERR_UNSUPPORTED;
  float *part = nullptr, *lpart = nullptr;
  if (mlp_noalloc_scratch(&part, &lpart) != hipSuccess) return PQR_ERR_DEVICE;
  if (launch_mlp_grad(params, feats, target, active, B, (float)w_reg, (float)w_pos, part, lpart,
                      grad, loss, (hipStream_t)stream) != hipSuccess)
    return PQR_ERR_DEVICE;
  return PQR_OK;
}

extern "C" pqr_status pqr_mlp_adam(float* params, const float* grad, float* m, float* v, int step,
                                   double lr, double beta1, double beta2, double eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1) return PQR_ERR_INVALID_ARG;
  if (launch_adam(params, grad, m, v, 4610, (float)lr, (float)beta1, (float)beta2, (float)eps, step,
                  (hipStream_t)stream) != hipSuccess)
    return PQR_ERR_DEVICE;
  return PQR_OK;
}

namespace {

// The active-set rounds shared by the learned and the screened warm starts: the
// problem restricted to A is solved by FS-QRPPA from bw (the full-length starting
// coefficients on the solver scale; z and theta derived from them on the device),
// the FP64 certificate on the full design judges the result, columns outside A
// whose |x~_j^T theta'| exceeds lambda_j (1 + 1e-6) join A, and if no round
// passes the plain zero-start solve on the full design gives the answer.
pqr_status active_set_rounds(pqr_ctx* ctx, const double* y, double tau, double lambda,
                             const double* weights, std::vector<int64_t> A,
                             std::vector<double> bw, double lmax, int max_rounds,
                             std::chrono::steady_clock::time_point t0, pqr_result* out,
                             pqr_learned_report& r) {
  auto secs = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  std::vector<double> cinv(g.p);
  HIPCHK(hipMemcpyAsync(cinv.data(), ctx->cinv_d, g.p * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> bfull(g.p + 1, 0.0), zbest(g.n), tbest(g.n);
  std::vector<double> lamj(g.p);
  for (int64_t j = 0; j < g.p; ++j) lamj[j] = lambda * (weights ? weights[1 + j] : 1.0);
  // warm state carried between rounds (full-length beta on the solver scale); the
  // first round derives z = y - X~beta^0 and theta from its signs on the device
  std::vector<double> zw(g.n), tw(g.n);
  bool ok = false;
  double cert[4] = {0, 0, 0, 0};
  int64_t iters = 0;
  std::vector<double> v(g.p);
  // With no violator outside A the full design's certificate equals the reduced
  // one (beta is zero there and the dual scaling sees no larger ratio), so the
  // reduced problem is solved to the target; a first round with more rounds to
  // come stops at 10x the target, enough to expose violators cheaply.
  const double tol = ctx->opt.tol_gap;
  double sub_tol = max_rounds > 1 ? 10.0 * tol : tol;
  for (int round = 0; round < max_rounds && !A.empty(); ++round) {
    ++r.rounds;
    pqr_ctx* sub = nullptr;
    pqr_options so = ctx->opt;   // the parent's profile option carries over
    so.tol_gap = sub_tol;
    so.G = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->Gf, ((int64_t)A.size() + 15) / 16));
    pqr_status st = pqr_create_subset(&sub, ctx, A.data(), (int64_t)A.size(), &so);
    if (st != PQR_OK) {
      ctx->err = std::string("subset: ") + (sub ? sub->err : "");
      pqr_destroy(sub);
      return st;
    }
    std::vector<double> ws(1 + A.size()), wsub;
    ws[0] = bw[0];
    for (size_t c = 0; c < A.size(); ++c) ws[1 + c] = bw[1 + A[c]];
    std::vector<double> wl;
    if (weights) {
      wl.resize(1 + A.size());
      wl[0] = weights[0];
      for (size_t c = 0; c < A.size(); ++c) wl[1 + c] = weights[1 + A[c]];
    }
    std::vector<double> bsub(1 + A.size()), zsub(g.n), tsub(g.n);
    pqr_result warm{};
    warm.beta_std = ws.data();
    warm.z = round ? zw.data() : nullptr;
    warm.theta = round ? tw.data() : nullptr;
    pqr_result res{};
    res.beta_std = bsub.data();
    res.z = zsub.data();
    res.theta = tsub.data();
    st = pqr_solve(sub, y, tau, lambda, weights ? wl.data() : nullptr, PQR_START_HOST, &warm, &res);
    iters += res.iters;
    r.reduced_iters += res.iters;
    r.reduced_sweep_ms += res.sweep_ms;
    r.reduced_sweep_launches += res.sweep_launches;
    r.reduced_sweep_bytes += (double)res.sweep_launches *
                             ((double)g.n * (double)A.size() * (fmt_col_bytes(g.fmt, 1024) / 1024.0) +
                              4.0 * (double)g.n + 20.0 * (double)A.size());
    pqr_destroy(sub);
    if (st != PQR_OK && st != PQR_ERR_NOT_CONVERGED) return st;
    // embed and check on the full design: FP64 certificate and every column's dual value
    std::fill(bfull.begin(), bfull.end(), 0.0);
    bfull[0] = bsub[0];
    for (size_t c = 0; c < A.size(); ++c) bfull[1 + A[c]] = bsub[1 + c];
    TRY(pqr_kkt_columns(ctx, y, tau, lambda, weights, bfull.data(), tsub.data(), cert, v.data()));
    bw = bfull;
    zw = zsub;
    tw = tsub;
    zbest = zsub;
    tbest = tsub;
    std::vector<char> in(g.p, 0);
    for (int64_t j : A) in[j] = 1;
    if (cert[2] <= tol) { ok = true; break; }   // the full certificate decides
    std::vector<int64_t> viol;
    for (int64_t j = 0; j < g.p; ++j)
      if (!in[j] && cinv[j] != 0.0 && std::fabs(v[j]) > lamj[j] * (1.0 + 1e-6)) viol.push_back(j);
    // the support is covered: finish at the target, or tighter if it already was
    sub_tol = sub_tol > tol ? tol : 0.25 * sub_tol;
    if (viol.empty()) continue;
    std::vector<int64_t> merged;
    merged.reserve(A.size() + viol.size());
    std::merge(A.begin(), A.end(), viol.begin(), viol.end(), std::back_inserter(merged));
    A.swap(merged);
  }
  r.active_final = (int64_t)A.size();
  r.seconds_reduced = secs();
  pqr_status status = PQR_OK;
  if (!ok) {
    // fallback: plain FS-QRPPA from a zero start on the full design
    r.fallback = 1;
    pqr_result res{};
    res.beta_std = bfull.data();
    res.z = zbest.data();
    res.theta = tbest.data();
    status = pqr_solve(ctx, y, tau, lambda, weights, PQR_START_ZERO, nullptr, &res);
    iters += res.iters;
    cert[0] = res.primal;
    cert[1] = res.dual;
    cert[2] = res.rel_gap;
    if (status != PQR_OK && status != PQR_ERR_NOT_CONVERGED) return status;
  }
  if (out) {
    int64_t nnz = 0;
    for (int64_t j = 0; j < g.p; ++j) nnz += bfull[1 + j] != 0.0;
    if (out->beta_std) std::memcpy(out->beta_std, bfull.data(), (g.p + 1) * 8);
    if (out->beta) {
      HIPCHK(hipMemcpyAsync(ctx->scratch64, bfull.data(), (g.p + 1) * 8, hipMemcpyHostToDevice, s));
      HIPCHK(launch_back_transform(ctx->scratch64, g.p, ctx->cm_d, ctx->cinv_d, bfull[0],
                                   ctx->bt_out, ctx->bpart64, s));
      HIPCHK(hipMemcpyAsync(out->beta, ctx->bt_out, (g.p + 1) * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    if (out->z) std::memcpy(out->z, zbest.data(), g.n * 8);
    if (out->theta) std::memcpy(out->theta, tbest.data(), g.n * 8);
    out->iters = iters;
    out->nnz = nnz;
    out->primal = cert[0];
    out->dual = cert[1];
    out->rel_gap = cert[2];
    out->lambda_max = lmax;
    out->seconds = secs();
  }
  r.seconds_check = secs();
  return status;
}

}  // namespace

extern "C" pqr_status pqr_solve_learned(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                        const double* weights, const float* mlp_params,
                                        double threshold, int max_rounds, pqr_result* out,
                                        pqr_learned_report* rep) {
  Range range_("pqr_solve_learned");
  if (!ctx) return PQR_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  auto secs = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  TRY(validate_problem(ctx, y, tau, lambda, weights));
  if (!mlp_params || max_rounds < 1) {
    ctx->err = "pqr_solve_learned needs the network parameters and max_rounds >= 1";
    return PQR_ERR_INVALID_ARG;
  }
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  pqr_learned_report r{};
  // 1. proposal: features, network, thresholded active set
  if (!ctx->feats) TRY(dalloc(ctx, &ctx->feats, g.p_pad * 16));
  if (!ctx->mlp_out) TRY(dalloc(ctx, &ctx->mlp_out, g.p_pad * 8));
  double lmax = 0.0;
  TRY(pqr_features(ctx, y, tau, lambda, weights, ctx->feats, &lmax));
  const double q = ctx->out_h[0];   // tau-quantile of y (null-fit intercept)
  HIPCHK(launch_mlp_forward(mlp_params, ctx->feats, g.p, ctx->mlp_out, s));
  std::vector<float> o(g.p * 2);
  HIPCHK(hipMemcpyAsync(o.data(), ctx->mlp_out, g.p * 8, hipMemcpyDeviceToHost, s));
  std::vector<double> cinv(g.p);
  HIPCHK(hipMemcpyAsync(cinv.data(), ctx->cinv_d, g.p * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double my = 0, vy = 0;
  for (int64_t i = 0; i < g.n; ++i) my += y[i];
  my /= g.n;
  for (int64_t i = 0; i < g.n; ++i) vy += (y[i] - my) * (y[i] - my);
  const double sdy = std::sqrt(vy / g.n);
  // A = {j : o1_j > threshold} plus the 32 columns with the largest logits, so
  // that a cautious network still proposes a starting support
  std::vector<int64_t> order;
  for (int64_t j = 0; j < g.p; ++j)
    if (cinv[j] != 0.0) order.push_back(j);
  const size_t ktop = std::min<size_t>(32, order.size());
  std::partial_sort(order.begin(), order.begin() + ktop, order.end(),
                    [&](int64_t a, int64_t b) { return o[2 * a + 1] > o[2 * b + 1]; });
  std::vector<char> pick(g.p, 0);
  for (size_t k = 0; k < ktop; ++k) pick[order[k]] = 1;
  std::vector<int64_t> A;
  for (int64_t j = 0; j < g.p; ++j)
    if (cinv[j] != 0.0 && (pick[j] || o[2 * j + 1] > threshold)) A.push_back(j);
  r.active_initial = (int64_t)A.size();
  r.seconds_proposal = secs();
  std::vector<double> bw(g.p + 1, 0.0);
  bw[0] = q;
  for (int64_t j : A) bw[1 + j] = o[2 * j] * sdy;
  const pqr_status st = active_set_rounds(ctx, y, tau, lambda, weights, std::move(A),
                                          std::move(bw), lmax, max_rounds, t0, out, r);
  if (rep) *rep = r;
  return st;
}

// Screened warm start: the sequential strong rule proposes A from the null-fit
// scores S_j = x~_j^T psi / n (psi the null dual at the tau-quantile):
// A = {j : |S_j| >= (2 lambda - lambda_prev) w_j}, lambda_prev = lambda_max unless
// given (budget 0), or the `budget` columns with the largest |S_j| / w_j; zero
// weights always join A.  The active-set rounds of the learned warm start then make
// the answer exact: the full-design certificate decides and violators join A.
extern "C" pqr_status pqr_solve_screened(pqr_ctx* ctx, const double* y, double tau, double lambda,
                                         const double* weights, double lambda_prev,
                                         int64_t budget, int max_rounds, pqr_result* out,
                                         pqr_learned_report* rep) {
  Range range_("pqr_solve_screened");
  if (!ctx) return PQR_ERR_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  TRY(validate_problem(ctx, y, tau, lambda, weights));
  if (max_rounds < 1 || budget < 0 || !(lambda_prev >= 0) || !std::isfinite(lambda_prev)) {
    ctx->err = "pqr_solve_screened needs max_rounds >= 1, budget >= 0 and a finite lambda_prev >= 0";
    return PQR_ERR_INVALID_ARG;
  }
  const Geom& g = ctx->g;
  hipStream_t s = ctx->s;
  pqr_learned_report r{};
  std::vector<double> score(g.p), cinv(g.p);
  double lmax = 0.0;
  TRY(pqr_lambda_max(ctx, y, tau, weights, &lmax, score.data()));
  const double q = ctx->out_h[0];   // tau-quantile of y (null-fit intercept)
  HIPCHK(hipMemcpyAsync(cinv.data(), ctx->cinv_d, g.p * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto w = [&](int64_t j) { return weights ? weights[1 + j] : 1.0; };
  std::vector<int64_t> cand;   // penalized, non-excluded columns
  std::vector<int64_t> A;
  for (int64_t j = 0; j < g.p; ++j) {
    if (cinv[j] == 0.0) continue;
    if (w(j) == 0.0) A.push_back(j);
    else cand.push_back(j);
  }
  auto ratio = [&](int64_t j) { return std::fabs(score[j]) / w(j); };
  if (budget > 0) {
    const size_t k = std::min<size_t>((size_t)budget, cand.size());
    std::partial_sort(cand.begin(), cand.begin() + k, cand.end(),
                      [&](int64_t a, int64_t b) { return ratio(a) > ratio(b); });
    A.insert(A.end(), cand.begin(), cand.begin() + k);
  } else {
    const double cut = 2.0 * lambda - (lambda_prev > 0 ? lambda_prev : lmax);
    size_t kept = 0;
    for (int64_t j : cand)
      if (ratio(j) >= cut) { A.push_back(j); ++kept; }
    if (kept == 0) {   // every column screened out: start from the 32 best scores
      const size_t k = std::min<size_t>(32, cand.size());
      std::partial_sort(cand.begin(), cand.begin() + k, cand.end(),
                        [&](int64_t a, int64_t b) { return ratio(a) > ratio(b); });
      A.insert(A.end(), cand.begin(), cand.begin() + k);
    }
  }
  std::sort(A.begin(), A.end());
  r.active_initial = (int64_t)A.size();
  r.seconds_proposal = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  std::vector<double> bw(g.p + 1, 0.0);
  bw[0] = q;
  const pqr_status st = active_set_rounds(ctx, y, tau, lambda, weights, std::move(A),
                                          std::move(bw), lmax, max_rounds, t0, out, r);
  if (rep) *rep = r;
  return st;
}
