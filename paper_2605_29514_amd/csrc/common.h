// Internal declarations shared by the libstn translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#define STN_ERR_ZEROPROB 1
#define STN_ERR_NUMERIC 2
#define STN_ERR_PHASE 4
#define STN_ERR_EIGEN 8

template <typename T>
struct cplx {
  T x, y;
};
using c32 = cplx<float>;
using c64 = cplx<double>;

template <typename T>
__host__ __device__ inline cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T>
__host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ inline cplx<T> cj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__host__ __device__ inline T norm2(cplx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename D, typename S>
__host__ __device__ inline cplx<D> cvt(cplx<S> a) { return {(D)a.x, (D)a.y}; }

// Per-shot 2x2 single-site operators of a two-term step
//   phi <- a * (x) O1_j phi + b * (x) O2_j phi
// are described on the device by Pauli codes; see mps.hip.

// ------------------------------------------------------------- profiling
// Launch classes for timing and algorithmic work accounting.
enum { K_TABLEAU = 0, K_BUILD, K_QR, K_GEMM, K_GRAM, K_EIGEN, K_SELECT, K_EXPECT, K_LAYER, K_COUNT };
// Device work counters: [K_COUNT][2] flops/bytes, Jacobi sweeps, layer FP64
// flops, the fused kernel's per-phase cycle totals, then its branch counters
// (kPath* below).
constexpr int kPhaseBase = 2 * K_COUNT + 2, kPhases = 8, kPathBase = kPhaseBase + kPhases, kPaths = 11;
constexpr int kWorkWords = kPathBase + kPaths;
// Branch counters of the fused kernel (steps that took each route; the
// largest eigen-solve order as an integer; cycles spent in the pivoted
// Cholesky part of the FP32-path eigen-solve).
enum { kPathEnv = 0, kPathQr, kPathEigLds, kPathEigGlobal, kPathEigGlobal129, kPathMaxOrder, kPathCholCycles,
       kPathJacGlobal, kPathCholQr, kPathEigNominal, kPathEigExec };
// Largest doubled bond for which the fused kernel keeps the left-environment
// Grams of a span (FP64 complex) instead of a QR sweep (halved while the
// product scratch of all shots, kEnvBond x 2 kEnvBond each, would pass
// kEnvFBudget bytes); the Grams of a span are packed into a per-shot store
// of n x ec^2 elements, ec = kEnvStore lowered in steps of 32 until the
// stores of all shots fit kEnvBudget bytes, and a span whose Grams do not
// fit takes the QR sweep.  Sized for the 288 GB of one MI355X next to the
// MPS and its workspace: with 1024 shots of 49 sites at chi_max 256 the
// store takes 40 GB (ec = 224) and the product scratch 8.6 GB.
constexpr int kEnvBond = 512;
constexpr int kEnvStore = 256;
constexpr size_t kEnvBudget = (size_t)40 << 30;
constexpr size_t kEnvFBudget = (size_t)12 << 30;

// Host-side recorder: when active, launches of the selected classes are
// bracketed by HIP events on their stream.
struct Prof {
  unsigned mask = 0;                       // classes to time
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipEvent_t get();
};
extern thread_local Prof *g_prof;

#define KLAUNCH(cls, kern, grid, block, lds, st, ...)                                  \
  do {                                                                                 \
    Prof *p_ = g_prof;                                                                 \
    bool on_ = p_ && (p_->mask >> (cls) & 1u);                                         \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                             \
    if (on_) { a_ = p_->get(); (void)hipEventRecord(a_, st); }                               \
    hipLaunchKernelGGL(kern, grid, block, lds, st, __VA_ARGS__);                       \
    if (on_) { b_ = p_->get(); (void)hipEventRecord(b_, st); p_->recs.push_back({cls, a_, b_}); } \
  } while (0)

// ---------------------------------------------------------------- tableau
struct TabDev {
  int n, W, SW;           // qubits, bit words per row, sign words per row
  uint64_t *x, *z, *s;    // [2n][W], [2n][W], [2n][SW]
};

// One row-product instruction: dst <- i^e0 * prod src[i] (rows of the old tableau)
struct RowProg {
  int16_t dst, nsrc, e0, pad;
  int16_t src[4];
};

// Small host-built instruction batches travel as kernel arguments (by value),
// so nothing has to be staged in host memory that outlives the launch.
constexpr int kProgBatch = 64;
struct ProgBatch {
  int n;                       // programs in this batch
  int ngates;                  // gates (k_tab_gates) in this batch
  int first[kProgBatch + 1];   // program range of each gate
  RowProg p[kProgBatch];
};


void launch_tab_reset(const TabDev &t, int *d_err, hipStream_t st);
void launch_tab_gates(const TabDev &t, const ProgBatch &b, int *d_err, hipStream_t st);
void launch_tab_noise(const TabDev &t, const uint64_t *d_noise, hipStream_t st);
void launch_tab_products(const TabDev &t, const ProgBatch &b, uint64_t *d_out_bits,
                         uint64_t *d_out_sign, int *d_err, hipStream_t st);
void launch_tab_frame(const TabDev &t, const uint64_t *d_snap, const uint64_t *d_negmask,
                      const uint8_t *d_tables, hipStream_t st);
void launch_tab_flip(const TabDev &t, int row, const uint64_t *d_mask, hipStream_t st);
void launch_tab_snapshot(const TabDev &t, int row, uint64_t *d_snap, hipStream_t st);

// ---------------------------------------------------------------- MPS state
struct MpsDev {
  int n, S, chi;
  int64_t *site_off;      // [n] element offset of site j's first shot slot
  int64_t *site_cap;      // [n] elements per shot slot of site j
  int64_t *ws_off;        // [n] same for the doubled-bond workspace
  int64_t *ws_cap;        // [n]
  void *mps;              // slots (complex T)
  void *ws;               // workspace slots (complex T)
  int *bond;              // [S][n+1]
  int *wb;                // [S][n+1] workspace bonds during a compression
  int *aux;               // [S][8]
  // per-shot scratch (element strides per shot)
  void *T;   int64_t T_cap;     // complex T
  void *R;   int64_t R_cap;     // complex T
  void *N;   int64_t N_cap;     // complex T
  void *Vt;  int64_t Vt_cap;    // complex T
  c64 *G;    int64_t G_cap;     // Gram / eigenvectors (FP64)
  c64 *V;    int64_t V_cap;
  double *ev; int64_t ev_cap;   // eigenvalues
  c64 *E;    int64_t E_cap;     // transfer matrix (FP64)
  c64 *F;    int64_t F_cap;
  void *J;   int64_t J_cap;     // bytes: fused-kernel fallbacks (reflectors, Jacobi pairs)
  c64 *Es;   int64_t Es_cap;    // fused kernel: left-environment Grams of a span (FP64)
  c64 *Fs;   int64_t Fs_cap;    //               and their product scratch
  int ebond;                    // largest workspace bond the environment path accepts
  int ebond_alloc;              // ... as allocated (ebond may be set lower)
  int lds_order;                // fused kernel, FP32 path: eigen-solve order held in LDS (0: by chi)
  double *logp, *fid, *p0, *nrm;  // [S]
  double *pm;                   // [S] probability of the last recorded outcome
  int *trunc;                   // [S] set when chi_max dropped weight above the cut
  c64 *coef;                    // [S][2]  (a, b)
  int *err;
  double eps_cut;
  int wmul;                     // workspace bond multiplier (2: two-term steps, 3: sums)
  int keep_norm;                // 1: compression leaves the norm (adjoint state)
  int prof;                     // count algorithmic work when nonzero
  double *work;                 // [K_COUNT][2]: flops, bytes
};

// Site operator table of one two-term step: for site j in [l, r],
// ops[(j - l) * 8 + {0..3}] = O1 (row-major 2x2), [+4..7] = O2.

// One chunk of rotations of a layer for the fused per-shot kernel.
struct RotLayer {
  int n_rot;                    // rotations in this chunk (<= kProgBatch)
  int theta_base;               // index of the chunk's first rotation in the angle array
  int center_in;                // orthogonality centre on entry (same for every shot)
  int16_t l[kProgBatch], r[kProgBatch];   // span of each rewritten Pauli
};

// One measurement of the fused per-shot path.
struct MeasStep {
  int l, r, pivot;              // span of P' and its first X/Y site (-1: none)
  int center_in;                // orthogonality centre on entry
  int n_meas, mi;               // row length of the record arrays and this column
};
template <typename T>
void mps_measure_fused(const MpsDev &m, const uint64_t *d_snap_sign, const c64 *d_ops, const c64 *d_eops,
                       const MeasStep &a, const double *d_u, const uint8_t *d_forced, uint8_t *d_out,
                       double *d_prob, uint64_t *d_negmask, uint64_t *d_mmask, int nt, hipStream_t st);
template <typename T> hipError_t mps_prepare(int max_rows);
template <typename T> hipError_t layer_prepare();
size_t layer_fallback_bytes(int chi);
// nt: threads per shot (64, 128 or 256)
template <typename T>
void mps_rot_layer(const MpsDev &m, const uint64_t *d_pbits, const uint64_t *d_psgn, int W, int SW,
                   const double *d_theta, int64_t stride, const RotLayer &L, int nt, hipStream_t st);
template <typename T> void mps_init(const MpsDev &m, hipStream_t st);
template <typename T> void mps_apply_single(const MpsDev &m, int site, const c64 *d_ops, hipStream_t st);
template <typename T> void mps_build(const MpsDev &m, int l, int r, const c64 *d_ops, hipStream_t st);
template <typename T> void mps_sweep_lr(const MpsDev &m, int l, int r, hipStream_t st);
template <typename T> void mps_sweep_rl(const MpsDev &m, int l, int r, hipStream_t st);
// ------------------------------------------------------------- adjoint
// ph: the forward state (a snapshot view), mu: the adjoint state.
void launch_step_reset(const MpsDev &m, hipStream_t st);
void launch_gather_theta(const double *d_theta, int64_t stride, int idx, double *d_dst, int S, hipStream_t st);
void launch_ops_measure_adj(const uint64_t *d_bits, int W, int l, int r, int pivot, c64 *d_ops, hipStream_t st);
// coefficients of the adjoint maps per shot (kind 0: rotation R^dag / n,
// 1: measurement M^dag / n, 2: the term (1/2p - 1) phi + (s sigma / 2p) P' phi)
void launch_adj_coef(const MpsDev &mu, int kind, int pivot, const double *d_theta, const uint64_t *d_sign,
                     const uint64_t *d_mmask, const double *d_nrm, const double *d_pm, hipStream_t st);
template <typename T> void mps_build_sum(const MpsDev &mu, const MpsDev &ph, int l, int r, const c64 *d_ops,
                                         hipStream_t st);
template <typename T> void mps_project_right(const MpsDev &mu, const MpsDev &ph, int l, const int *d_flag,
                                             hipStream_t st);
template <typename T> void mps_overlap_grad(const MpsDev &mu, const MpsDev &ph, const c64 *d_eops, int l,
                                            int r, const uint64_t *d_sign, double *d_grad, int64_t stride,
                                            hipStream_t st);
template <typename T> void mps_zero(const MpsDev &m, hipStream_t st);
template <typename T> void mps_move_right(const MpsDev &m, int c, hipStream_t st);
template <typename T> void mps_move_left(const MpsDev &m, int c, hipStream_t st);
template <typename T> void mps_normalize_site(const MpsDev &m, int site, hipStream_t st);
template <typename T> void mps_expect(const MpsDev &m, int l, int r, const c64 *d_ops, hipStream_t st);
template <typename T> void mps_spectrum(const MpsDev &m, int b, double *d_out, int ld, int *d_rank, hipStream_t st);

// ops builders (device): from the Pauli bits of P' (W words each, x then z)
void launch_ops_rotation(const uint64_t *d_bits, int W, int l, int r, c64 *d_ops, hipStream_t st);
void launch_ops_measure(const uint64_t *d_bits, int W, int l, int r, int pivot, c64 *d_ops,
                        c64 *d_ops_expect, hipStream_t st);
void launch_coef_rotation(const uint64_t *d_psgn, int S, const double *d_theta, int64_t stride,
                          int r_index, c64 *d_coef, int *d_err, hipStream_t st);
void launch_outcome(const MpsDev &m, const uint64_t *d_snap_sign, int pivot, int dr_site,
                    const double *d_u, const uint8_t *d_forced, int n_meas, int mi,
                    uint8_t *d_out, double *d_prob, uint64_t *d_negmask, uint64_t *d_mmask,
                    hipStream_t st);
