// Kernel launchers of libpqr (host-callable, plain types only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pqr_dev.h"

namespace pqr {

// Geometry of the design store shared by every kernel.
//
// The store is blocked by (column group, row chunk): a "segment" holds one
// column's 64*rpl consecutive rows (a wavefront's load), and the 16 segments of
// a group for one chunk are contiguous, so a wavefront sweeping a group streams
// one contiguous run of 16 segments per chunk.  Segment of column j, chunk ch:
//     X + ((j/16 * nchunks + ch) * 16 + j%16) * seg_bytes.
struct Geom {
  const uint8_t* X;   // store base
  int fmt;            // Fmt
  int rpl;            // rows per lane: 4 or 16
  int64_t n, n_pad;   // rows, padded rows (multiple of 64*rpl)
  int64_t p, p_pad;   // feature columns, padded to a multiple of kGroup
  int64_t seg_bytes;  // bytes of one segment (64*rpl rows of one column)
  __host__ __device__ int64_t ngroups() const { return p_pad / kGroup; }
  __host__ __device__ int64_t nchunks() const { return n_pad / (kWave * rpl); }
  __host__ __device__ int64_t store_bytes() const { return p_pad * nchunks() * seg_bytes; }
  __host__ __device__ const uint8_t* seg(int64_t j, int64_t ch) const {
    return X + (((j >> 4) * nchunks() + ch) * kGroup + (j & 15)) * seg_bytes;
  }
};

template <typename T>
struct IterBufs {
  T* beta;        // p_pad, solver scale, in place
  const T* cm;    // p_pad column means (0 when not standardized)
  const T* cinv;  // p_pad 1/s_j (0 for excluded and padding columns)
  const T* clam;  // p_pad lambda_j
  const T* geta;  // ngroups: eta of the block holding each group
  T* gnorm;       // ngroups x 4 sweep partials
  int* gflag;     // ngroups: 1 if any coefficient of the group is nonzero
  int* list;      // ngroups: active groups in increasing order (first ctl->count)
  double* partial;  // smax x n_pad partial products (FP64 for every iterate type)
  const T* y;     // n_pad
  T* z;           // n_pad
  T* theta;       // n_pad (padding rows stay 0)
  T* r;           // n_pad cached residual X~beta + z - y
  double* bpart;  // update-kernel block partials (nblk x 8)
  int* bcnt;      // kCompactBlocks active-group counts of the compaction
  double* bnrm;   // kCompactBlocks x 4 norm partials of the compaction
  Ctl* ctl;
};

constexpr int kCompactBlocks = 64;

struct IterParams {
  double tau, mu, sigma, eta0;
  int G;
  int smax, min_per;
  // launch_prepare_state only: bit 0 sets z = y - X~beta - beta0 (so r = 0),
  // bit 1 sets theta_i = (tau - 1{z_i < 0}) / n, centred to sum zero
  int fit;
};

// One FS-QRPPA iteration = sweep, compact, axpy, update.  With non-null
// events, ev0/ev1 are recorded around the sweep kernel.
template <typename T>
hipError_t launch_iteration(const Geom& g, const IterBufs<T>& b, const IterParams& ip,
                            hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// One problem of a grouped launch: its store geometry, buffers and parameters.
template <typename T>
struct GroupDesc {
  Geom g;
  IterBufs<T> b;
  IterParams ip;
};

// One FS-QRPPA iteration of every problem in d[0..nprob) with five launches in
// total.  Every problem shares g.fmt and g.rpl (g is any of their geometries);
// off (device) holds three prefix arrays of nprob + 1 block offsets: the sweep's
// ceil(ngroups / 4) blocks, the axpy's ceil(nchunks / 4) * smax blocks and the
// update's n_pad / 256 blocks of each problem, and tot[k] = off[k][nprob].
template <typename T>
hipError_t launch_grouped_iteration(const Geom& g, const GroupDesc<T>* d, const int* off,
                                    int nprob, const int64_t tot[3], hipStream_t s,
                                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Recompute the cached residual r = X~beta + beta0 + z - y and sum(theta) for a
// given state (after a warm start); also rebuilds the active list.  ip.fit
// derives z and/or theta from beta instead (see IterParams).
template <typename T>
hipError_t launch_prepare_state(const Geom& g, const IterBufs<T>& b, const IterParams& ip,
                                hipStream_t s);

// ---- FP64 certificate ----
struct CertBufs {
  const double* y;      // n_pad
  double* theta_p;      // n_pad projected theta
  double* beta_d;       // p_pad coefficients in double
  const double* cm;     // p_pad
  const double* cinv;   // p_pad
  const double* clam;   // p_pad
  double* v;            // p_pad (optional output of x~_j^T theta')
  double* gpart;        // ngroups partials
  double* partial;      // smax x n_pad
  const int* list;      // active groups
  const Ctl* ctl;       // count and beta0
  double* bpart;        // reduction scratch (>= n_pad/256 + 1024 doubles)
  double* out;          // 8 doubles: [primal loss, penalty, y.theta', max ratio, shift, sum theta', -, -]
};

// theta' = clip(theta - c, (tau-1)/n, tau/n) with sum theta' = 0 (bisection on c).
template <typename T>
hipError_t launch_project(const T* theta, int64_t n, int64_t n_pad, double tau, const double* y,
                          double* theta_p, double* out, hipStream_t s);

// v_j = x~_j^T theta' in FP64 for all columns; per-group max |v_j| / lambda_j.
hipError_t launch_dots64(const Geom& g, const double* theta_p, const double* sum_tp,
                         const double* cm, const double* cinv, const double* clam, double* v,
                         double* gmax, hipStream_t s);

// Up to four certificates in one pass (int8 store, rows_per_lane 16): for k < kb
// (<= 4) the per-group max of
// |x~_j^T theta'_k| / (lam[k] w_j) into gmax[k * ngroups + grp], with theta'_k at
// tp + k n_pad and sum(theta'_k) at out[8k + 5] (launch_project's layout); lam
// is host, kb doubles.
hipError_t launch_mdots64(const Geom& g, const double* tp, int kb, const double* out,
                          const double* cm, const double* cinv, const double* w,
                          const double* lam, double* gmax, hipStream_t s);

// Sparse s = X~ beta over the active list in FP64, then P(beta) pieces.
hipError_t launch_primal64(const Geom& g, const CertBufs& c, double tau, int smax, int min_per,
                           hipStream_t s);

// Deterministic reductions into out[k]: sum / max of a device array.
hipError_t launch_reduce_sum(const double* a, int64_t m, double* bpart, double* out, hipStream_t s);
hipError_t launch_reduce_max(const double* a, int64_t m, double* bpart, double* out, hipStream_t s);

template <typename T>
hipError_t launch_to_double(const T* a, int64_t m, double* out, hipStream_t s);
template <typename T>
hipError_t launch_from_double(const double* a, int64_t m, T* out, hipStream_t s);

// ---- setup ----
hipError_t launch_encode(const void* src, int src_fmt, int64_t ld, const Geom& g, uint8_t* dst,
                         hipStream_t s);
// column sums and sums of squares in double (exact for integer codes)
hipError_t launch_colstats(const Geom& g, double* sum, double* sumsq, hipStream_t s);

// Lanczos building blocks: u_j = x~_j^T q_{block(j)} for all columns, and the
// per-block dense products w_g = X~_g u_g into partials.
hipError_t launch_block_dots(const Geom& g, const float* q, int64_t qstride, const int* gblock,
                             const float* cm, const float* cinv, const float* qsum, float* u,
                             hipStream_t s);
hipError_t launch_block_axpy(const Geom& g, const float* u, const float* cm, const float* cinv,
                             const int* bstart, int G, int splits, float* partial, hipStream_t s);
hipError_t launch_lanczos_step(int64_t n, int64_t n_pad, int G, int splits, int k, int T,
                               int icpt_in_block0, const float* partial, float* q, float* qprev,
                               float* wbuf, float* qsum, double* alpha, double* beta,
                               hipStream_t s);
hipError_t launch_lanczos_init(int64_t n, int64_t n_pad, int G, float* q, float* qprev,
                               float* qsum, hipStream_t s);

// tau-quantile of y (k-th order statistic, k = ceil(n tau)) and the null dual
// psi/n written to theta_p; out[0] = q.
hipError_t launch_null_dual(const double* y, int64_t n, int64_t n_pad, double tau,
                            double* theta_p, double* out, hipStream_t s);

// back-transform: beta_orig_j = beta_j * cinv_j, beta_orig_0 = beta0 - sum_j m_j beta_orig_j
hipError_t launch_back_transform(const double* beta_std, int64_t p, const double* cm,
                                 const double* cinv, double beta0, double* beta_orig,
                                 double* bpart, hipStream_t s);

}  // namespace pqr

namespace pqr {
hipError_t launch_colparams(const double* sum, const double* sumsq, int64_t n, int64_t p,
                            int64_t p_pad, int standardize, double* cm_d, double* cinv_d,
                            double* sd_d, float* cm_f, float* cinv_f, hipStream_t s);
template <typename T>
hipError_t launch_set_y(const double* y, int64_t n, int64_t n_pad, T* y_t, hipStream_t s);
}  // namespace pqr

namespace pqr {
// Batched right-hand sides (kern_batch.hip).  Kp = K padded to a multiple of 16.
struct BatchBufs {
  int K;
  float* beta;          // Kp x p_pad (right-hand side k in row k)
  const float* cm;      // p_pad
  const float* cinv;    // p_pad
  const float* w;       // p_pad penalty weights w_j (0 on padding)
  const float* lam;     // Kp
  const float* tau;     // Kp
  const float* geta;    // ngroups
  const float* y;       // n_pad (shared)
  float* z;             // Kp x n_pad
  float* theta;         // Kp x n_pad
  float* r;             // Kp x n_pad
  int8_t* dig;          // S x Kp x n_pad digit slices of theta
  long long* tpart;     // (n_pad/256) x Kp
  long long* tsumq;     // Kp exact sum of the quantised theta
  double* tsum;         // Kp sum of theta
  double* scale;        // Kp digit scale c_k
  double* beta0;        // Kp
  double* norms;        // Kp x 4
  uint32_t* mask;       // ngroups x Kp/16 column masks (bit c: column c nonzero for a k of the tile)
  int* list;            // p_pad: union of the nonzero columns, increasing
  int* bcnt;            // kCompactBlocks
  int* count;           // 1
  long long* partial;   // kBaxpySplits x Kp x n_pad exact integer split sums of X B
  double* bpart;        // (n_pad/256) x Kp x 8
  int8_t* bd;           // ngroups x Kp x 4 x 16: digit slices of the coefficients of
                        // the union columns (list order), for X~ B on the matrix cores
  double* pmax;         // 256 x Kp partial max |beta_kj / s_j|
  double* poff;         // 256 x Kp partial sum m_j * U_kj (mean correction)
  double* bscale;       // Kp coefficient digit scale d_k (power of two)
  const int* kact;      // Kp: 1 = iterate right-hand side k, 0 = frozen (certified or padding)
};
// Launch variants of the two matrix-core kernels of a batched iteration (chosen
// per batch width by the solver's autotuner): back-product (k_bgemm) and union
// product (k_baxpy); variant 0 is the default of each.
struct BatchTiles {
  int bgemm = 0, baxpy = 0;
};
constexpr int kBgemmVariants = 4, kBaxpyVariants = 3;
constexpr int kBaxpySplits = 16;   // most splits of the union product (partial buffer)
inline int bgemm_variants() { return kBgemmVariants; }
inline int baxpy_variants() { return kBaxpyVariants; }
hipError_t launch_bgemm_variant(const Geom& g, const BatchBufs& b, int Kp, int v, hipStream_t s,
                                hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// smin: fewest splits of the union (int32 exactness); the split count used (also
// needed by the update kernel) is returned in *splits
hipError_t launch_baxpy_variant(const Geom& g, const BatchBufs& b, int Kp, int smin, int min_per,
                                int v, hipStream_t s, int* splits = nullptr);
// One batched iteration; with non-null events, ev0/ev1 are recorded around the
// back-product kernel (k_bgemm).
hipError_t launch_batch_iteration(const Geom& g, const BatchBufs& b, int Kp, double mu,
                                  double sigma, double eta0, int smin, int min_per,
                                  const BatchTiles& tiles, hipStream_t s, hipEvent_t ev0 = nullptr,
                                  hipEvent_t ev1 = nullptr);
hipError_t launch_batch_zero(const Geom& g, const BatchBufs& b, int Kp, hipStream_t s);

// Exact-integer certificate of batched right-hand sides.  theta_q,k = unit_k T_k
// with T_k integer, inside the dual box and summing to exactly zero; its digits
// (kCertSlices balanced base-128 slices) feed one int8 matrix-core pass over X.
constexpr int kCertSlices = 4;
struct CertArgs {
  const int8_t* dig;    // [kCertSlices][Kc][n_pad] digits of T
  const double* lam;    // Kc lambda_k (padding: anything finite)
  const double* unit;   // Kc value of one step of T_k
  const double* w;      // p_pad penalty weights (> 0 for j < p)
  const double* cinv;   // p_pad 1 / s_j
  double* gmax;         // [Kc][ngroups / 4 rounded up] maxima of |x~_j^T theta_q| / (lambda_k w_j)
  int K;                // right-hand sides in the pass (k >= K: padding)
};
// T = trunc(theta' / unit) (toward zero, so inside [(tau-1)/n, tau/n]), its sum
// made zero by moving the largest (sum > 0) or smallest (sum < 0) entry when that
// stays in the box; digits into column kc of c.dig (Kc columns); out[2] = y^T theta_q,
// out[7] = 0 (ok) or 1 (the sum could not be zeroed: certify this k in FP64).
// tq: n_pad ints of scratch.
hipError_t launch_cert_quantize(const double* theta_p, int64_t n, int64_t n_pad, double tau,
                                double unit, const double* y, int* tq, int8_t* dig, int kc,
                                int Kc, double* out, hipStream_t s);
// One pass over X for the Kc = 16 m columns of c.dig: c.gmax.
hipError_t launch_cert_pass(const Geom& g, const CertArgs& c, int Kc, hipStream_t s);
// Group sets of the certificate pass (the row count of c.gmax per k).
int64_t cert_group_sets(const Geom& g);
// largest byte of the int8 store into *out (device int, set to 0 first by the launcher)
hipError_t launch_max_code(const Geom& g, int* out, hipStream_t s);
// flags, count and ordered list of the groups holding a nonzero of beta (b.beta);
// b.ctl receives the count (beta0 untouched)
template <typename T>
hipError_t launch_active_list(const Geom& g, const IterBufs<T>& b, hipStream_t s);
hipError_t launch_scale(const double* w, double a, int64_t m, double* out, hipStream_t s);
// Unpenalized columns in the certificate: dense standardized copies of cols[0..nu)
// (nu x n_pad), cross products out = A B^T (na x nb, rows of length m), and the
// projection of tp onto x~_U^T theta = 0 (c solves the normal equations) followed
// by the box scaling; out[2] = y^T theta, out[5] = sum theta, out[6] = the scale.
hipError_t launch_dense_cols(const Geom& g, const int64_t* cols, int64_t nu, const double* cm,
                             const double* cinv, double* xu, hipStream_t s);
hipError_t launch_cross(const double* A, int64_t na, const double* B, int64_t nb, int64_t m,
                        double* out, hipStream_t s);
hipError_t launch_unpen_project(double* tp, const double* xu, const double* c, int64_t nu,
                                int64_t n, int64_t n_pad, double tau, const double* y,
                                double* bpart, double* out, hipStream_t s);
// LLA stage weights out[0..p] (out[0] = 0) from standardized coefficients beta[0..p)
template <typename T>
hipError_t launch_lla_weights(const T* beta, int64_t p, int kind, double a, double lam,
                              double wfloor, double* out, hipStream_t s);
}  // namespace pqr

namespace pqr {
// scoring network (kern_mlp.hip)
hipError_t launch_mlp_forward(const float* P, const float* F, int64_t B, float* out, hipStream_t s);
int mlp_grad_partials(int64_t B);
// rows of the largest batch pqr_mlp_grad_noalloc takes (its scratch holds the
// partials of that many rows)
constexpr int64_t kMlpNoAllocRows = 8192;
hipError_t mlp_noalloc_scratch(float** part, float** lpart);
hipError_t launch_mlp_grad(const float* P, const float* F, const float* t, const float* a,
                           int64_t B, float w_reg, float w_pos, float* part, float* lpart,
                           float* grad, float* loss, hipStream_t s);
hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_features(const double* score, const double* cm, const double* cinv, int64_t p,
                           double n, double tau, double loglam, float* F, hipStream_t s);
// copy the segments of the listed columns of src into dst (same format and rows)
hipError_t launch_gather_columns(const Geom& src, const int64_t* cols, int64_t ncols,
                                 const Geom& dst, uint8_t* dst_base, hipStream_t s);
hipError_t launch_gather_f64(const double* src, const int64_t* cols, int64_t ncols, int64_t npad,
                             double* dst, hipStream_t s);
}  // namespace pqr
