// Fused per-shot rotation-layer kernel of the STN step (Sec. IV.A-B).
//
// Shots are independent, so one block per shot runs a whole chunk of
// rotations (centre moves, bond-2 operator blocks, left-to-right QR sweep,
// right-to-left FP64 Gram/eigen truncation, FP64 renormalisation) with block
// barriers only: one launch per chunk instead of ~10 launches per site, and
// every shot proceeds at its own bond dimensions.  The block size NT (64, 128,
// 256 or 512 threads per shot) is a launch parameter: with 64 threads a shot is
// one wavefront and a barrier costs almost nothing, so 1024 shots fill the
// 1024 SIMDs of the chip; larger blocks give a single shot more lanes when
// there are few shots or large bonds.
//
// Small operands live in one dynamic LDS region that the phases overlay
// (QR matrix, GEMM staging, the eigen-solve matrix); operands beyond its size
// stay in the shot's global scratch, so every bond up to chi_max is handled.
#include "linalg.h"

#include <algorithm>

namespace {

using namespace stnk;

constexpr int kLdsQrRows = 64;            // reflector vectors in LDS up to this many rows
constexpr size_t kLdsQrMat = 16 * 1024;   // QR operand in LDS up to this many bytes
constexpr int kEigIdx = 64;               // eigen-solve index / pair tables in LDS up to this order
constexpr int kJacLdsN = 32;              // FP64 path: Jacobi G and V in LDS up to this order
constexpr int kEigLdsMax = 64;            // FP32 path: factor in LDS up to this order
constexpr int kDirectGemm = 64;           // products with every dimension up to this skip LDS staging

// Dynamic LDS layout (bytes): small arrays at fixed offsets, then one
// region that the phases overlay (GEMM staging, QR operand, the eigen-solve
// matrices with padded rows).  The region holds the FP64 path's Jacobi G and
// V up to order 32, or the FP32 path's factor up to order eig_n (a launch
// parameter, eig_lds_order).
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr int kPh = kEigIdx / 2 + 1;                            // pair-table length
constexpr size_t kVs = 0;                                       // c64[kLdsQrRows]
constexpr size_t kVd = kVs + kLdsQrRows * sizeof(c64);          // double[2 kLdsQrRows]
constexpr size_t kDg = kVd + 2 * kLdsQrRows * sizeof(double);   // double[kEigIdx]
constexpr size_t kPe = kDg + kEigIdx * sizeof(double);          // c64[kPh]
constexpr size_t kPc = kPe + kPh * sizeof(c64);                 // double[kPh]
constexpr size_t kPs = kPc + kPh * sizeof(double);              // double[kPh]
constexpr size_t kPiv = kPs + kPh * sizeof(double);             // int[kEigIdx]
constexpr size_t kPos = kPiv + kEigIdx * sizeof(int);           // int[kEigIdx + 2]
constexpr size_t kPp = kPos + (kEigIdx + 2) * sizeof(int);      // int[kPh]
constexpr size_t kPq = kPp + kPh * sizeof(int);                 // int[kPh]
constexpr size_t kEv = (kPq + kPh * sizeof(int) + 7) / 8 * 8;  // double[kEigIdx]
constexpr size_t kWp = (kEv + kEigIdx * sizeof(double) + 15) / 16 * 16;  // c64[NT]
constexpr size_t kUfix = cmax(kLdsQrMat, GemmStage<double>::bytes);
constexpr size_t u_off(int nt) { return (kWp + nt * sizeof(c64) + 255) / 256 * 256; }
constexpr size_t eig_region(bool fp64, int en) {
  return fp64 ? 2 * (size_t)kJacLdsN * (kJacLdsN + 1) * sizeof(c64) : (size_t)en * (en + 1) * sizeof(c64);
}
// FP32 path, steps small enough for the direct GEMMs (every dimension up to
// kDirectGemm, so no GEMM staging runs while these hold live data): three
// buffers after the fixed arrays.
//   [u_off, +kStepFactor): the factor of a truncation step of order up to
//     kLdsStepN; after the selection, N = X V^T
//   [vt_off, +kVtBytes): V^T (nn x k), or before it the F = E X of the
//     step's Gram when that fits
//   [x_off, +kXBytes): the centre block X of the right-to-left sweep, kept
//     from step to step (sized so that four 256-thread blocks fit a compute
//     unit)
// The environment sweep, before X exists, uses the last two as one buffer
// for its F = E B (kFElems FP64).  The GEMM staging overlaps only the first
// bytes of V^T.  At 128 threads per shot four blocks still fit a compute
// unit's 160 KB.
constexpr int kLdsStepN = 32;
constexpr size_t kStepFactor = (size_t)kLdsStepN * (kLdsStepN + 1) * sizeof(c64);
constexpr size_t kVtBytes = (size_t)kLdsStepN * kLdsStepN * sizeof(cplx<float>);
constexpr size_t kXBytes = 5120;
constexpr int kXElems = kXBytes / sizeof(cplx<float>);
constexpr int kFElems = (kVtBytes + kXBytes) / sizeof(c64);
constexpr size_t vt_off(int nt) { return u_off(nt) + kStepFactor; }
constexpr size_t x_off(int nt) { return vt_off(nt) + kVtBytes; }
static_assert(x_off(64) - u_off(64) >= kUfix, "GEMM staging reaches the X buffer");
constexpr size_t lds_bytes(int nt, bool fp64, int en) {
  return u_off(nt) + cmax(cmax(kUfix, eig_region(fp64, en)), fp64 ? 0 : kStepFactor + kVtBytes + kXBytes);
}
static_assert(lds_bytes(128, false, 32) * 4 <= 160 * 1024, "four 128-thread blocks per compute unit");
// four 256-thread blocks as well, with room for the kernels' static LDS
static_assert((lds_bytes(256, false, 32) + 1024) * 4 <= 160 * 1024, "four 256-thread blocks per compute unit");
// FP32 path, truncation steps whose rho stays in global scratch: the largest
// rank whose Gram K = Rs Rs^H (padded rows) fits the overlaid region
constexpr int k_gram_order(int en) {
  const size_t region = lds_bytes(64, false, en) - u_off(64);
  int r = 0;
  while ((size_t)(r + 1) * (r + 2) * sizeof(c64) <= region && r + 1 <= kEigIdx) ++r;
  return r;
}
static_assert(k_gram_order(32) >= 40 && k_gram_order(64) == 64, "Gram orders held in LDS");
// FP32 path: factors (and the Grams of global-scratch factors) up to order
// 64 in LDS (~70 KB per block) when chi_max is 17..32, where every doubled
// bond then fits, or when a block has 256 or more threads (at most two such
// blocks share a compute unit: their registers, not LDS, bound residency);
// otherwise up to 32 (~22 KB, four 128-thread blocks per compute unit).
inline int eig_lds_order(int chi, int nt) {
  return nt >= 256 || (2 * chi > 32 && 2 * chi <= kEigLdsMax) ? kEigLdsMax : 32;
}

// Global fallbacks in the shot's J scratch: reflector vectors for up to
// 4 chi + 2 rows, eigen-solve index and pair tables for orders up to 2 chi + 2.
struct Fallback {
  c64 *vs, *pe; double *vd, *dg, *pc, *ps; int *piv, *pos, *pp, *pq;
};
__device__ inline Fallback fallback(const MpsDev &m, int s) {
  char *b = reinterpret_cast<char *>(m.J) + (size_t)s * m.J_cap;
  const int rows = 4 * m.chi + 2, P = 2 * m.chi + 2;
  Fallback f;
  f.vs = reinterpret_cast<c64 *>(b);
  f.pe = f.vs + rows;
  f.vd = reinterpret_cast<double *>(f.pe + P / 2 + 1);
  f.dg = f.vd + 2 * rows;
  f.pc = f.dg + P;
  f.ps = f.pc + P / 2 + 1;
  f.piv = reinterpret_cast<int *>(f.ps + P / 2 + 1);
  f.pos = f.piv + P;
  f.pp = f.pos + P + 2;
  f.pq = f.pp + P / 2 + 1;
  return f;
}

template <typename TA, typename TB_, typename TC, typename ACC, int NT>
__device__ void blk_gemm(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                         const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc, char *lds, int lower = 0) {
  // 256 or more threads: each wave takes its own 16 x 32 output blocks
  // straight from memory (measured faster than the LDS-staged tiles, which
  // keep the whole block on one 32 x 32 tile at a time);
  // lower: output blocks wholly above the diagonal are skipped
  if constexpr (NT >= 256) {
    gemm_direct<TA, TB_, TC, ACC, NT>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, lower);
  } else {
    if (M <= kDirectGemm && N <= kDirectGemm && K <= kDirectGemm)
      gemm_direct<TA, TB_, TC, ACC, NT>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, lower);
    else
      gemm_tiles<TA, TB_, TC, ACC, NT>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, 0, 1, lds + u_off(NT), lower);
  }
  __syncthreads();
}

template <typename T>
struct Pair {
  cplx<T> a, b;
};

template <typename T, int NT>
__device__ void blk_copy(cplx<T> *dst, const cplx<T> *src, int cnt) {
  blk_each<NT, 4, cplx<T>>(cnt, [&](int e) { return src[e]; }, [&](int e, cplx<T> v) { dst[e] = v; });
  __syncthreads();
}

// QR of the rows x cols matrix at A (global, may be overwritten): staged in
// LDS when it fits.  Q -> Qd (qt as in qr_block), R -> Rd.  gvs/gvd are the
// shot's global reflector buffers, used when rows exceed the LDS ones.
template <typename T, int NT>
__device__ void blk_qr(c64 *gvs, double *gvd, int rows, int cols, cplx<T> *A, cplx<T> *Qd, int qt,
                       cplx<T> *Rd, char *lds) {
  c64 *vs = rows <= kLdsQrRows ? reinterpret_cast<c64 *>(lds + kVs) : gvs;
  double *vd = rows <= kLdsQrRows ? reinterpret_cast<double *>(lds + kVd) : gvd;
  c64 *wp = reinterpret_cast<c64 *>(lds + kWp);
  if ((size_t)rows * cols * sizeof(cplx<T>) <= kLdsQrMat) {
    cplx<T> *Al = reinterpret_cast<cplx<T> *>(lds + u_off(NT));
    blk_copy<T, NT>(Al, A, rows * cols);
    qr_block<T, NT>(rows, cols, Al, Qd, qt, Rd, vs, vd, wp);
  } else {
    qr_block<T, NT>(rows, cols, A, Qd, qt, Rd, vs, vd, wp);
  }
}

// FP32 path: the Q of a centre move by Cholesky QR (qr_cols_cq, its Gram in
// the LDS tile) when the tile holds it, then R = Q^H X from the stored Q;
// false when it does not apply or declines (the Householder QR runs then).
template <typename T, int NT>
__device__ bool move_cq(const MpsDev &m, int s, int rows, int cols, const cplx<T> *X, cplx<T> *Qd, int qt,
                        cplx<T> *R, char *lds, int eig_n) {
  if constexpr (sizeof(T) == 4) {
    if (cols > rows || cols > (eig_n > 32 ? k_gram_order(64) : k_gram_order(32))) return false;
    c64 *K = reinterpret_cast<c64 *>(lds + u_off(NT));
    if (!qr_cols_cq<NT>(rows, cols, X, Qd, qt, K, m.G + s * m.G_cap, m.V + s * m.V_cap)) return false;
    // FP64 accumulation: R carries the small singular directions of X,
    // whose relative accuracy an FP32 sum over the rows would lose
    if (qt)
      gemm_direct<T, T, T, double, NT>(cols, cols, rows, Qd, rows, 0, X, cols, 0, R, cols);
    else
      gemm_direct<T, T, T, double, NT>(cols, cols, rows, Qd, cols, 1, X, cols, 0, R, cols);
    __syncthreads();
    return true;
  } else {
    return false;
  }
}

// Centre move c -> c+1 (QR of A_c, R into A_{c+1}).
template <typename T, int NT>
__device__ void blk_move_right(const MpsDev &m, int s, int c, char *lds, int cls, int eig_n) {
  int *b = bnd(m, s);
  const int rows = 2 * b[c], cols = b[c + 1], N = 2 * b[c + 2];
  const int p = rows < cols ? rows : cols;
  cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
  blk_copy<T, NT>(X, slot<T>(m, c, s), rows * cols);
  if (!move_cq<T, NT>(m, s, rows, cols, X, slot<T>(m, c, s), 0, R, lds, eig_n))
    blk_qr<T, NT>(fallback(m, s).vs, fallback(m, s).vd, rows, cols, X, slot<T>(m, c, s), 0, R, lds);
  blk_gemm<T, T, T, T, NT>(p, N, cols, R, cols, 0, slot<T>(m, c + 1, s), N, 0, X, N, lds);
  if (threadIdx.x == 0) {
    b[c + 1] = p;
    add_work(m, cls, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
    add_work(m, cls, gemm_flops(p, N, cols), (double)sizeof(cplx<T>) * ((double)p * cols + (double)cols * N + (double)p * N));
  }
  __syncthreads();
  blk_copy<T, NT>(slot<T>(m, c + 1, s), X, p * N);
}

// Centre move c -> c-1 (LQ of A_c via the QR of A_c^H, L into A_{c-1}).
template <typename T, int NT>
__device__ void blk_move_left(const MpsDev &m, int s, int c, char *lds, int cls, int eig_n) {
  int *b = bnd(m, s);
  const int dl = b[c], dr = b[c + 1], M = 2 * b[c - 1];
  const int rows = 2 * dr, cols = dl, p = rows < cols ? rows : cols;
  cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
  const cplx<T> *A = slot<T>(m, c, s);
  for (int e = threadIdx.x; e < dl * 2 * dr; e += NT) {
    int a = e / (2 * dr), cc = e % (2 * dr);
    X[(size_t)cc * dl + a] = cj(A[e]);
  }
  __syncthreads();
  if (!move_cq<T, NT>(m, s, rows, cols, X, slot<T>(m, c, s), 1, R, lds, eig_n))
    blk_qr<T, NT>(fallback(m, s).vs, fallback(m, s).vd, rows, cols, X, slot<T>(m, c, s), 1, R, lds);
  blk_gemm<T, T, T, T, NT>(M, p, cols, slot<T>(m, c - 1, s), cols, 0, R, cols, 1, X, p, lds);
  if (threadIdx.x == 0) {
    b[c] = p;
    add_work(m, cls, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
    add_work(m, cls, gemm_flops(M, p, cols), (double)sizeof(cplx<T>) * ((double)M * cols + (double)cols * p + (double)M * p));
  }
  __syncthreads();
  blk_copy<T, NT>(slot<T>(m, c - 1, s), X, M * p);
}

__device__ inline void rot_site_ops(const uint64_t *bx, const uint64_t *bz, int j, c64 *o2) {
  site_op(bitw(bx, j), bitw(bz, j), o2);
}

// Per-phase cycle accounting (thread 0, profiling runs only).
struct PhaseClock {
  bool on;
  long long t;
  __device__ explicit PhaseClock(bool o) : on(o), t(o ? clock64() : 0) {}
  __device__ void lap(const MpsDev &m, int k) {
    if (!on) return;
    const long long now = clock64();
    atomicAdd(&m.work[kPhaseBase + k], (double)(now - t));
    t = now;
  }
};

// Site operators of one two-term step: a rotation takes O1 = I and O2 the
// Pauli site operator from the bits of P'; a measurement projection reads
// both from the operator table ops[(j - l) * 8 + {0..3, 4..7}].
struct SiteOps {
  const c64 *tab;
  const uint64_t *bx, *bz;
  int l;
  __device__ void get(int j, c64 *o1, c64 *o2) const {
    if (tab) {
      for (int k = 0; k < 4; ++k) { o1[k] = tab[(size_t)(j - l) * 8 + k]; o2[k] = tab[(size_t)(j - l) * 8 + 4 + k]; }
    } else {
      site_op(0, 0, o1);
      site_op(bitw(bx, j), bitw(bz, j), o2);
    }
  }
};

// One two-term step phi <- a O1 phi + b O2 phi over [l, r] for shot s, with
// the centre tracked in c: bond-2 blocks, left-to-right sweep (environment
// Grams or QR), right-to-left FP64 Gram/eigen truncation, FP64
// renormalisation (the squared norm before it goes to nrm[s]).  A single
// site is updated in place; a non-unitary one moves the centre there first
// and renormalises.
template <typename T, int NT>
__device__ void shot_step(const MpsDev &m, int s, int l, int r, const SiteOps &so, c64 ca, c64 cb, bool unitary,
                          int &c, char *lds, int eig_n, PhaseClock &clk, int *sweeps, int cls) {
  const bool f64c = m.prof && cls == K_LAYER;   // FP64 share is tracked for the layer class
  const int tid = threadIdx.x;
  int *b = bnd(m, s), *w = wbd(m, s);
  if (l == r) {
    if (!unitary) {
      while (c < l) { blk_move_right<T, NT>(m, s, c, lds, cls, eig_n); ++c; }
      while (c > l) { blk_move_left<T, NT>(m, s, c, lds, cls, eig_n); --c; }
    }
    c64 o1[4], o2[4];
    so.get(l, o1, o2);
    const int dl = b[l], dr = b[l + 1];
    cplx<T> *A = slot<T>(m, l, s);
    double part = 0;
    for (int e = tid; e < dl * dr; e += NT) {
      const int a = e / dr, cc = e % dr;
      const c64 x0 = cvt<double>(A[(size_t)(a * 2 + 0) * dr + cc]), x1 = cvt<double>(A[(size_t)(a * 2 + 1) * dr + cc]);
      const c64 y0 = ca * (o1[0] * x0 + o1[1] * x1) + cb * (o2[0] * x0 + o2[1] * x1);
      const c64 y1 = ca * (o1[2] * x0 + o1[3] * x1) + cb * (o2[2] * x0 + o2[3] * x1);
      A[(size_t)(a * 2 + 0) * dr + cc] = cvt<T>(y0);
      A[(size_t)(a * 2 + 1) * dr + cc] = cvt<T>(y1);
      part += norm2(cvt<double>(cvt<T>(y0))) + norm2(cvt<double>(cvt<T>(y1)));
    }
    if (!unitary) {                           // FP64 renormalisation of the new centre
      const double n2 = bsum<NT>(part);
      if (!(n2 > 0) || isinf(n2)) {
        if (tid == 0) atomicOr(m.err, STN_ERR_NUMERIC);
      } else {
        const double inv = 1.0 / sqrt(n2);
        for (int e = tid; e < dl * 2 * dr; e += NT) A[e] = cvt<T>(inv * cvt<double>(A[e]));
        if (tid == 0) m.nrm[s] = n2;
      }
    }
    __syncthreads();
    clk.lap(m, 0);
    return;
  }
  clk.lap(m, 0);
  while (c < l) { blk_move_right<T, NT>(m, s, c, lds, cls, eig_n); ++c; }
  while (c > r) { blk_move_left<T, NT>(m, s, c, lds, cls, eig_n); --c; }
  clk.lap(m, 1);
  // Environment path: when every doubled bond of the span fits the shot's
  // Gram store, the left-to-right sweep forms the left-environment Grams
  // E_j = sum_s B_j^s^H E_{j-1} B_j^s (FP64) instead of a QR sweep, and the
  // truncation uses rho = X^H E X, the same reduced density that X^H X gives
  // after orthonormalisation.  Otherwise: Householder QR.
  // (The Grams are packed one after another in the shot's store: E_j, of
  // order Dr_j, starts after E_l .. E_{j-1}; the path needs every doubled
  // bond within the product scratch and the Grams within the store.)
  bool env = m.ebond > 0;
  {
    size_t need = 0;
    for (int j = l; j <= r && env; ++j) {
      const int Dl = (j == l) ? b[j] : 2 * b[j], Dr = (j == r) ? b[j + 1] : 2 * b[j + 1];
      env = Dl <= m.ebond && Dr <= m.ebond;
      if (j < r) need += (size_t)Dr * Dr;
    }
    env = env && need <= (size_t)m.Es_cap;
  }
  if (m.prof && tid == 0) atomicAdd(&m.work[kPathBase + (env ? kPathEnv : kPathQr)], 1.0);
  // bond-2 blocks over [l, r]
  for (int j = l; j <= r; ++j) {
    const int dl = b[j], dr = b[j + 1];
    const int Dl = (j == l) ? dl : 2 * dl, Dr = (j == r) ? dr : 2 * dr;
    c64 o1[4], o2[4];
    so.get(j, o1, o2);
    cplx<T> *out = (j == l && !env) ? scr<T>(m.T, m.T_cap, s) : wslot<T>(m, j, s);
    const cplx<T> *A = slot<T>(m, j, s);
    // branch of element (a, cc): 0 / 1 for the two terms of the MPO, -1 off
    // the block diagonal
    auto branch = [&](int a, int cc) {
      const int ba = a >= dl, bc = cc >= dr;
      if (j == l) return bc;
      if (j == r) return ba;
      return ba == bc ? ba : -1;
    };
    blk_each_rc<NT, 4, Pair<T>>(
        Dl, Dr,
        [&](int a, int cc) {
          const int br = branch(a, cc);
          Pair<T> x{mk<T>(0, 0), mk<T>(0, 0)};
          if (br >= 0) {
            const int aa = (j == l) ? a : a - (br ? dl : 0);
            const int c2 = (j == r) ? cc : cc - (br ? dr : 0);
            x.a = A[(size_t)(aa * 2 + 0) * dr + c2];
            x.b = A[(size_t)(aa * 2 + 1) * dr + c2];
          }
          return x;
        },
        [&](int a, int cc, Pair<T> x) {
          const int br = branch(a, cc);
          c64 y0 = mk<double>(0, 0), y1 = mk<double>(0, 0);
          if (br >= 0) {
            const c64 x0 = cvt<double>(x.a), x1 = cvt<double>(x.b);
            // element-wise selects keep o1, o2 in registers (a pointer to
            // either would put both arrays in scratch memory)
            const c64 u0 = br ? o2[0] : o1[0], u1 = br ? o2[1] : o1[1];
            const c64 u2 = br ? o2[2] : o1[2], u3 = br ? o2[3] : o1[3];
            y0 = u0 * x0 + u1 * x1;
            y1 = u2 * x0 + u3 * x1;
            if (j == l) { const c64 k = br ? cb : ca; y0 = k * y0; y1 = k * y1; }
          }
          out[(size_t)(a * 2 + 0) * Dr + cc] = cvt<T>(y0);
          out[(size_t)(a * 2 + 1) * Dr + cc] = cvt<T>(y1);
        });
    if (tid == 0) { w[j] = Dl; if (j == r) w[r + 1] = dr; }
  }
  __syncthreads();
  clk.lap(m, 2);
  c64 *Es = m.Es + (size_t)s * m.Es_cap, *Fs = m.Fs + (size_t)s * m.Fs_cap;
  // offset of E_j (j in [l, r-1]) in the packed store: the orders of
  // E_l .. E_{j-1} are the workspace bonds w[l+1] .. w[j] as the
  // left-to-right sweep leaves them (the right-to-left sweep changes w[j]
  // only after its last use of E_{j-1})
  auto eoff = [&](int j) {
    size_t o = 0;
    for (int i = l + 1; i <= j; ++i) o += (size_t)w[i] * w[i];
    return o;
  };
  // the centre block X of the right-to-left sweep: the shot's T, or (FP32
  // path, a step small enough for the LDS buffers) the LDS X buffer
  cplx<T> *Xg = scr<T>(m.T, m.T_cap, s), *Xl = reinterpret_cast<cplx<T> *>(lds + x_off(NT));
  auto x_fits = [&](int lx, int n2) {
    return sizeof(T) == 4 && n2 <= kLdsStepN && lx <= kDirectGemm && lx * n2 <= kXElems;
  };
  bool xl = false;
  if (env) {
    // E_l = B_l^H B_l (B_l as 2 w[l] x w[l+1]); then E_j through site r-1
    {
      const int D = w[l + 1], K = 2 * w[l];
      blk_gemm<T, T, double, double, NT>(D, D, K, wslot<T>(m, l, s), D, 1, wslot<T>(m, l, s), D, 0, Es, D, lds);
      if (tid == 0) {
        add_work(m, cls, gemm_flops(D, D, K), (double)sizeof(cplx<T>) * K * D + 16.0 * D * D);
        if (f64c) atomicAdd(&m.work[2 * K_COUNT + 1], gemm_flops(D, D, K));
      }
    }
    for (int j = l + 1; j < r; ++j) {
      const int Dl = w[j], Dr = w[j + 1];
      c64 *Ep = Es + eoff(j - 1), *Ej = Es + eoff(j);
      // FP32 path, small sites: F in LDS between two direct GEMMs
      const bool lf = sizeof(T) == 4 && Dl <= kDirectGemm / 2 && Dr <= kDirectGemm / 2 && Dl * 2 * Dr <= kFElems;
      c64 *F = lf ? reinterpret_cast<c64 *>(lds + vt_off(NT)) : Fs;
      if (lf) {
        gemm_direct<double, T, double, double, NT>(Dl, 2 * Dr, Dl, Ep, Dl, 0, wslot<T>(m, j, s), 2 * Dr, 0, F, 2 * Dr);
        __syncthreads();
        gemm_direct<T, double, double, double, NT>(Dr, Dr, 2 * Dl, wslot<T>(m, j, s), Dr, 1, F, Dr, 0, Ej, Dr);
        __syncthreads();
      } else {
        // a middle site's block is block-diagonal in the two terms (rows
        // a < dl and columns c < dr carry the first, the rest the second),
        // so both products run per term on the nonzero blocks: half the work
        const int dl = Dl / 2, dr = Dr / 2;
        const cplx<T> *Bj = wslot<T>(m, j, s);
        for (int t = 0; t < 2; ++t)
          for (int p = 0; p < 2; ++p)   // F[:, p, c in t] = E[:, a in t] B[a in t, p, c in t]
            blk_gemm<double, T, double, double, NT>(Dl, dr, dl, Ep + t * dl, Dl, 0,
                                                    Bj + (size_t)t * dl * 2 * Dr + p * Dr + t * dr, 2 * Dr, 0,
                                                    F + p * Dr + t * dr, 2 * Dr, lds);
        for (int t = 0; t < 2; ++t)     // E_j[c in t, :] = B[(a in t, p), c in t]^H F[(a in t, p), :]
          blk_gemm<T, double, double, double, NT>(dr, Dr, 2 * dl, Bj + (size_t)t * 2 * dl * Dr + t * dr, Dr, 1,
                                                  F + (size_t)t * 2 * dl * Dr, Dr, 0, Ej + (size_t)t * dr * Dr, Dr,
                                                  lds);
      }
      if (tid == 0) {
        // the nonzero blocks' work (half of the dense products)
        const double f = 0.5 * (gemm_flops(Dl, 2 * Dr, Dl) + gemm_flops(Dr, Dr, 2 * Dl));
        add_work(m, cls, f, (double)sizeof(cplx<T>) * Dl * Dr + 16.0 * (Dl * Dl + 2.0 * Dl * Dr + Dr * Dr));
        if (f64c) atomicAdd(&m.work[2 * K_COUNT + 1], f);
      }
    }
    xl = x_fits(w[r], 2 * w[r + 1]);
    blk_copy<T, NT>(xl ? Xl : Xg, wslot<T>(m, r, s), 2 * w[r] * w[r + 1]);
    clk.lap(m, 3);
  }
  // left-to-right QR sweep: B_j = Q R, Q -> workspace slot j, R B_{j+1} -> T
  for (int j = l; j < r && !env; ++j) {
    const int rows = 2 * w[j], cols = w[j + 1], N = 2 * w[j + 2];
    const int p = rows < cols ? rows : cols;
    cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
    blk_qr<T, NT>(fallback(m, s).vs, fallback(m, s).vd, rows, cols, X, wslot<T>(m, j, s), 0, R, lds);
    clk.lap(m, 3);
    blk_gemm<T, T, T, T, NT>(p, N, cols, R, cols, 0, wslot<T>(m, j + 1, s), N, 0, X, N, lds);
    clk.lap(m, 4);
    if (tid == 0) {
      w[j + 1] = p;
      add_work(m, cls, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
      add_work(m, cls, gemm_flops(p, N, cols), (double)sizeof(cplx<T>) * ((double)p * cols + (double)cols * N + (double)p * N));
    }
    __syncthreads();
  }
  // right-to-left truncation sweep
  for (int j = r; j > l; --j) {
    const int Lx = w[j], nn = 2 * w[j + 1];
    cplx<T> *X = xl ? Xl : Xg;
    c64 *Gg = m.G + s * m.G_cap;
    // FP32 path: when the step's order is at most 32 and the products are
    // direct, rho goes straight into the LDS factor and the selection reads
    // the eigenvectors there (lg); such steps also keep V^T and their
    // intermediates in LDS (ls).  Each global write read back after a barrier
    // costs a store and a load latency on the step's critical path.
    const bool lg = sizeof(T) == 4 && nn <= kLdsStepN && nn <= eig_n && Lx <= kDirectGemm;
    const bool ls = lg && nn <= kLdsStepN;
    // FP32 path: the eigen-solve runs on rho in LDS (vectors read from its
    // factor rows by the selection) when rho was formed there; any larger
    // step reduces rho to the Gram of its Cholesky factor first (half the
    // order at these ranks: measured faster than rho of order 33..64 in LDS)
    const bool vl = sizeof(T) == 4 && lg;
    c64 *Gl = reinterpret_cast<c64 *>(lds + u_off(NT));
    if (env) {                                // rho = X^H (E_{j-1} X)
      const c64 *Ep = Es + eoff(j - 1);
      c64 *F = ls && Lx * nn * sizeof(c64) <= kVtBytes ? reinterpret_cast<c64 *>(lds + vt_off(NT)) : Fs;
      blk_gemm<double, T, double, double, NT>(Lx, nn, Lx, Ep, Lx, 0, X, nn, 0, F, nn, lds);
      if (lg) {
        gemm_direct<T, double, double, double, NT>(nn, nn, Lx, X, nn, 1, F, nn, 0, Gl, nn + 1);
        __syncthreads();
      } else {
        // FP32 path: rho only feeds the left-looking Cholesky, which reads
        // its lower triangle
        blk_gemm<T, double, double, double, NT>(nn, nn, Lx, X, nn, 1, Fs, nn, 0, Gg, nn, lds, sizeof(T) == 4);
      }
      if (tid == 0) {
        add_work(m, cls, gemm_flops(Lx, nn, Lx), 16.0 * (Lx * Lx + Lx * nn));
        if (f64c) atomicAdd(&m.work[2 * K_COUNT + 1], gemm_flops(Lx, nn, Lx));
      }
    } else if (lg) {
      gemm_direct<T, T, double, double, NT>(nn, nn, Lx, X, nn, 1, X, nn, 0, Gl, nn + 1);
      __syncthreads();
    } else {
      blk_gemm<T, T, double, double, NT>(nn, nn, Lx, X, nn, 1, X, nn, 0, Gg, nn, lds, sizeof(T) == 4);
    }
    clk.lap(m, 5);
    const c64 *Vsel = m.V + s * m.V_cap;     // sorted eigenvectors, nn x nn (not in LDS steps)
    if (m.prof && tid == 0) {
      const bool in_lds = sizeof(T) == 8 ? nn <= kJacLdsN : lg;
      atomicAdd(&m.work[kPathBase + (in_lds ? kPathEigLds : nn <= 128 ? kPathEigGlobal : kPathEigGlobal129)], 1.0);
      if (sizeof(T) == 8 && !in_lds) atomicAdd(&m.work[kPathBase + kPathJacGlobal], 1.0);
      atomicMax(reinterpret_cast<unsigned long long *>(&m.work[kPathBase + kPathMaxOrder]), (unsigned long long)nn);
    }
    long long t_chol = 0;
    int qk = 0;              // FP32 path, cut decided by the relative cut alone: kept rows in Rs
    double qw = 0;           // and the discarded fraction of the trace
    c64 *Rs = reinterpret_cast<c64 *>(scr<T>(m.R, m.R_cap, s));
    {
      const Fallback f = fallback(m, s);
      const bool li = nn <= kEigIdx;
      int *pos = li ? reinterpret_cast<int *>(lds + kPos) : f.pos;
      double fe;
      if constexpr (sizeof(T) == 8) {
        // FP64 path: two-sided Jacobi on rho (relative accuracy down to the
        // smallest kept values); G and V in LDS up to order 32
        int *pp = li ? reinterpret_cast<int *>(lds + kPp) : f.pp;
        int *pq = li ? reinterpret_cast<int *>(lds + kPq) : f.pq;
        double *pc = li ? reinterpret_cast<double *>(lds + kPc) : f.pc;
        double *ps = li ? reinterpret_cast<double *>(lds + kPs) : f.ps;
        c64 *pe = li ? reinterpret_cast<c64 *>(lds + kPe) : f.pe;
        c64 *Gw = Gg, *Vw = m.V + s * m.V_cap;
        int ldw = nn;
        if (nn <= kJacLdsN) {
          ldw = nn + 1;
          blk_each_rc<NT, 8, c64>(nn, nn, [&](int i, int j) { return Gg[i * nn + j]; },
                                  [&](int i, int j, c64 v) { Gl[i * ldw + j] = v; });
          __syncthreads();
          Gw = Gl;
          Vw = Gl + kJacLdsN * (kJacLdsN + 1);
        }
        jacobi_block<NT>(nn, Gw, ldw, Vw, m.ev + s * m.ev_cap, Gg, m.err, pos, pc, ps, pe, pp, pq, sweeps,
                         jac_abs<T>(), jac_rel<T>());
        fe = 36.0 * nn * nn * (double)nn;
        Vsel = Gg;
      } else {
        // FP32 path: rho formed in LDS (order <= 32) is solved there by
        // pivoted Cholesky + one-sided Jacobi on the factor.  A larger rho
        // (global scratch) is factored left-looking into the contiguous rows
        // Rs (r x nn, the shot's R scratch).  When fewer pivots than
        // min(chi_max, 2^min(j, n-j)) stay above the relative cut, the cut
        // alone decides: the kept space is spanned by those leading rows
        // (their Schur complement, at most the count left times the cut
        // weight each, is what is dropped), orthonormalised by two passes of
        // Cholesky QR with their Gram in LDS -- no eigen-solve.  Otherwise
        // (chi_max or the physical bound binds) the eigenvalues decide: the
        // Gram K = Rs Rs^H (same nonzero eigenvalues as rho) is solved in
        // LDS when its order fits and the eigenvectors of rho come back as
        // Rs^H u / sqrt(lambda), else one-sided Jacobi runs on the rows of
        // Rs in global scratch.
        const double ct = chol_tol(m.eps_cut, nn);
        double *ev = m.ev + s * m.ev_cap;
        c64 *V = m.V + s * m.V_cap;
        int *piv_l = reinterpret_cast<int *>(lds + kPiv), *pos_l = reinterpret_cast<int *>(lds + kPos);
        double *dg_l = reinterpret_cast<double *>(lds + kDg), *evl = reinterpret_cast<double *>(lds + kEv);
        int eo = -1, rk = 0;
        fe = 0;
        if (vl) {
          eo = nn;
        } else {
          double tr, resid;
          int rc;
          c64 *wpl = reinterpret_cast<c64 *>(lds + kWp);
          // the first factor rows also in the LDS tile (free until the Gram of
          // the factor is formed there)
          const int tl = (int)((lds_bytes(NT, false, eig_n) - u_off(NT)) / ((size_t)nn * sizeof(c64)));
          rk = chol_rows<NT>(nn, Gg, nn, Rs, nn, ct, f.dg, f.pos, wpl, m.err, &tr, &fe, m.eps_cut, &rc, &resid, true,
                             Gl, tl);
          if (clk.on && tid == 0) t_chol = clock64();
          const int kt = eig_n > 32 ? k_gram_order(64) : k_gram_order(32);
          const int eb = j < m.n - j ? j : m.n - j;
          const int kcap = eb < 30 && (1 << eb) < m.chi ? (1 << eb) : m.chi;
          // the Gram of the kept rows in LDS when it fits, else in the shot's
          // rho scratch (rho is dead once factored)
          if (rc >= 1 && rc <= kcap && orth_rows<NT>(rc, nn, Rs, nn, V, rc <= kt ? Gl : Gg, &fe)) {
            qk = rc;
            qw = tr > 0 ? resid / tr : 0.0;
            if (m.prof && tid == 0) atomicAdd(&m.work[kPathBase + kPathCholQr], 1.0);
          } else if (rk >= 1 && rk <= kt) {
            gemm_direct<double, double, double, double, NT>(rk, rk, nn, Rs, nn, 0, Rs, nn, 1, Gl, rk + 1);
            __syncthreads();
            fe += gemm_flops(rk, rk, nn);
            eo = rk;
          }
        }
        if (qk > 0) {
        } else if (eo >= 0) {
          fe += eig_psd<NT>(eo, Gl, eo + 1, evl, nullptr, m.err, piv_l, pos_l, dg_l, sweeps, ct, eig_conv_tol<T>(),
                            eig_rot_tol<T>(), (vl && clk.on) ? &t_chol : nullptr);
          if (!vl) {
            // eigenvectors of K with nonzero eigenvalue, scaled:
            // U[a][c] = u_c[a] / sqrt(lambda_c), u_c = conj(factor row pos[c]) / |row|
            int r2 = 0;
            for (int c = 0; c < rk; ++c) r2 += evl[c] > 0;
            c64 *U = Gg;
            blk_each_rc<NT, 4, c64>(
                rk, r2, [&](int a, int c) { return Gl[(size_t)piv_l[pos_l[c]] * (rk + 1) + a]; },
                [&](int a, int c, c64 v) { U[(size_t)a * r2 + c] = (dg_l[pos_l[c]] / sqrt(evl[c])) * cj(v); });
            for (int c = tid; c < nn; c += NT) ev[c] = c < r2 ? evl[c] : 0.0;
            __syncthreads();
            if (r2 > 0) {
              gemm_direct<double, double, double, double, NT>(nn, r2, rk, Rs, nn, 1, U, r2, 0, V, nn);
              fe += gemm_flops(nn, r2, rk);
            } else {
              for (int i = tid; i < nn; i += NT) V[(size_t)i * nn] = mk<double>(i == 0 ? 1.0 : 0.0, 0);
            }
            __syncthreads();
          }
        } else {
          if (m.prof && tid == 0) atomicAdd(&m.work[kPathBase + kPathJacGlobal], 1.0);
          for (int q = tid; q < rk; q += NT) f.piv[q] = q;
          __syncthreads();
          fe += jac_rows<NT>(nn, rk, Rs, nn, ev, V, m.err, f.piv, f.pos, f.dg, sweeps, eig_conv_tol<T>(),
                             eig_rot_tol<T>());
        }
      }
      if (tid == 0) {
        // the solve is counted at its fixed nominal cost (eig_nominal_flops),
        // whatever route and sweep count ran; the executed count is kept apart
        const double fn = eig_nominal_flops(nn);
        // rho = X^H (E X) is Hermitian: its algorithmic work is one triangle
        const double f64 = 4.0 * Lx * nn * (nn + 1.0) + fn;
        add_work(m, cls, f64, (double)sizeof(cplx<T>) * Lx * nn + 16.0 * 3 * nn * nn + 8.0 * nn);
        if (f64c) {
          atomicAdd(&m.work[2 * K_COUNT + 1], f64);        // FP64 share of the layer work
          atomicAdd(&m.work[kPathBase + kPathEigNominal], fn);
          atomicAdd(&m.work[kPathBase + kPathEigExec], fe);
        }
        if (m.prof) atomicAdd(&m.work[2 * K_COUNT], (double)*sweeps);
        if (clk.on && t_chol) atomicAdd(&m.work[kPathBase + kPathCholCycles], (double)(t_chol - clk.t));
      }
      clk.lap(m, 6);
    }
    int k;
    cplx<T> *Vt = ls ? reinterpret_cast<cplx<T> *>(lds + vt_off(NT)) : scr<T>(m.Vt, m.Vt_cap, s);
    if (vl) {
      const double *evl = reinterpret_cast<const double *>(lds + kEv);
      const int *rk = reinterpret_cast<const int *>(lds + kPos), *pv = reinterpret_cast<const int *>(lds + kPiv);
      const double *rn = reinterpret_cast<const double *>(lds + kDg);
      const int ldw = nn + 1;
      k = select_core<T, NT>(
          m, s, j, evl,
          [&](int i, int c) {
            if (evl[0] == 0) return mk<double>(i == 0 && c == 0 ? 1.0 : 0.0, 0);   // rank 0: e_0
            const int row = rk[c];
            return rn[row] * cj(Gl[(size_t)pv[row] * ldw + i]);
          },
          Vt);
    } else if (qk > 0) {
      // basis vectors of the kept space: the conjugated orthonormal rows
      k = select_fixed<T, NT>(m, s, j, qk, qw, [&](int i, int c) { return cj(Rs[(size_t)c * nn + i]); }, Vt);
    } else {
      k = select_body<T, NT>(m, s, j, Vsel, Vt);
    }
    const int M = 2 * w[j - 1];
    // N in the factor buffer (dead after the selection) when the product
    // that reads it is direct too; the new X in LDS when the next step
    // qualifies (the old X is dead once N is formed)
    cplx<T> *Nn = ls && M <= kDirectGemm ? reinterpret_cast<cplx<T> *>(lds + u_off(NT)) : scr<T>(m.N, m.N_cap, s);
    blk_gemm<T, T, T, T, NT>(Lx, k, nn, X, nn, 0, Vt, k, 0, Nn, k, lds);
    xl = x_fits(w[j - 1], 2 * k);
    X = xl ? Xl : Xg;
    blk_gemm<T, T, T, T, NT>(M, k, Lx, wslot<T>(m, j - 1, s), Lx, 0, Nn, k, 0, X, k, lds);
    if (tid == 0) {
      w[j] = k;
      add_work(m, cls, gemm_flops(Lx, k, nn) + gemm_flops(M, k, Lx),
               (double)sizeof(cplx<T>) * ((double)Lx * nn + (double)nn * k + 2.0 * Lx * k + (double)M * Lx + (double)M * k));
    }
    __syncthreads();
  }
  finish_body<T, NT>(m, s, l, xl ? Xl : Xg);
  clk.lap(m, 7);
  c = l;
}

// COUNT marks the launches made while the device work counters are on (a
// separate instantiation, so timings and profiler traces of the two kinds
// of launch never mix); the counting itself is switched by m.prof.
template <typename T, int NT, bool COUNT>
__global__ void __launch_bounds__(NT, 2) k_layer(MpsDev m, const uint64_t *pbits, const uint64_t *psgn,
                                              int W, int SW, const double *theta, int64_t stride,
                                              RotLayer L, int eig_n) {
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x, tid = threadIdx.x;
  __shared__ c64 cf[2];
  __shared__ int sweeps;
  int c = L.center_in;
  PhaseClock clk(m.prof && tid == 0);
  for (int i = 0; i < L.n_rot; ++i) {
    const int l = L.l[i], r = L.r[i];
    const uint64_t *bx = pbits + (size_t)i * 2 * W, *bz = bx + W;
    if (tid == 0) {
      const double th = theta[(int64_t)s * stride + L.theta_base + i];
      if (!(th == th) || isinf(th)) atomicOr(m.err, STN_ERR_NUMERIC);
      const double sg = ((psgn[(size_t)i * SW + (s >> 6)] >> (s & 63)) & 1ull) ? -1.0 : 1.0;
      cf[0] = mk<double>(cos(th), 0);
      cf[1] = mk<double>(0, -sg * sin(th));
    }
    __syncthreads();
    const SiteOps so{nullptr, bx, bz, l};
    shot_step<T, NT>(m, s, l, r, so, cf[0], cf[1], true, c, lds, eig_n, clk, &sweeps, K_LAYER);
  }
}

// One Z measurement per shot (Sec. IV.A): centre to l, <phi|P'|phi> by FP64
// transfer matrices over [l, r] (the centre norm N and tr E give
// p(0) = (N + sigma tr E) / 2N), outcome m = 0 iff u < p(0) (or forced),
// log P, then the projection as a two-term step (coefficients (1/2,
// s sigma / 2) without a pivot, (1, s sigma) with one) and the outcome bit
// masks (atomic OR into words cleared beforehand) for the frame update.
template <typename T, int NT, bool COUNT>
__global__ void __launch_bounds__(NT, 2) k_meas(MpsDev m, const uint64_t *snap_sign, const c64 *ops, const c64 *eops,
                                             MeasStep a, const double *u, const uint8_t *forced, uint8_t *out,
                                             double *prob, uint64_t *negmask, uint64_t *mmask, int eig_n) {
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x, tid = threadIdx.x;
  __shared__ c64 cf[2];
  __shared__ int sweeps;
  int *b = bnd(m, s);
  const int l = a.l, r = a.r;
  int c = a.center_in;
  PhaseClock clk(false);
  while (c < l) { blk_move_right<T, NT>(m, s, c, lds, K_EXPECT, eig_n); ++c; }
  while (c > l) { blk_move_left<T, NT>(m, s, c, lds, K_EXPECT, eig_n); --c; }
  // centre norm and <phi|P'|phi>
  double part = 0;
  {
    const int cnt = b[l] * 2 * b[l + 1];
    const cplx<T> *A = slot<T>(m, l, s);
    for (int e = tid; e < cnt; e += NT) part += norm2(cvt<double>(A[e]));
  }
  const double N = bsum<NT>(part);
  c64 *E = m.E + (size_t)s * m.E_cap, *F = m.F + (size_t)s * m.F_cap;
  {
    const int d = b[l];
    for (int e = tid; e < d * d; e += NT) E[e] = mk<double>((e / d) == (e % d) ? 1.0 : 0.0, 0);
    __syncthreads();
  }
  for (int j = l; j <= r; ++j) {
    const int dl = b[j], dr = b[j + 1];
    const cplx<T> *A = slot<T>(m, j, s);
    blk_gemm<double, T, double, double, NT>(dl, 2 * dr, dl, E, dl, 0, A, 2 * dr, 0, F, 2 * dr, lds);
    const c64 *o = eops + (size_t)(j - l) * 4;
    for (int e = tid; e < dl * dr; e += NT) {
      const int x = e / dr, y = e % dr;
      const c64 f0 = F[(size_t)(x * 2 + 0) * dr + y], f1 = F[(size_t)(x * 2 + 1) * dr + y];
      F[(size_t)(x * 2 + 0) * dr + y] = o[0] * f0 + o[1] * f1;
      F[(size_t)(x * 2 + 1) * dr + y] = o[2] * f0 + o[3] * f1;
    }
    __syncthreads();
    blk_gemm<T, double, double, double, NT>(dr, dr, 2 * dl, A, dr, 1, F, dr, 0, E, dr, lds);
    if (tid == 0)
      add_work(m, K_EXPECT, gemm_flops(dl, 2 * dr, dl) + gemm_flops(dr, dr, 2 * dl),
               (double)sizeof(cplx<T>) * 2 * dl * dr + 16.0 * (dl * dl + 4.0 * dl * dr + dr * dr));
  }
  double tp = 0;
  {
    const int d = b[r + 1];
    for (int i = tid; i < d; i += NT) tp += E[(size_t)i * d + i].x;
  }
  const double tr = bsum<NT>(tp);
  if (tid == 0) {
    const double sg = ((snap_sign[s >> 6] >> (s & 63)) & 1ull) ? -1.0 : 1.0;
    double p0 = (N + sg * tr) / (2 * N);
    p0 = fmin(1.0, fmax(0.0, p0));
    if (!(p0 == p0)) { atomicOr(m.err, STN_ERR_NUMERIC); p0 = 0.5; }
    int mm;
    if (forced) mm = forced[(size_t)s * a.n_meas + a.mi] ? 1 : 0;
    else mm = u[(size_t)s * a.n_meas + a.mi] < p0 ? 0 : 1;
    double pm = mm ? 1.0 - p0 : p0;
    if (pm <= 0) { atomicOr(m.err, STN_ERR_ZEROPROB); pm = 1e-300; }
    m.logp[s] += log(pm);
    m.pm[s] = pm;
    m.p0[s] = p0;
    if (out) out[(size_t)s * a.n_meas + a.mi] = (uint8_t)mm;
    if (prob) prob[(size_t)s * a.n_meas + a.mi] = pm;
    const double ss = mm ? -1.0 : 1.0;
    if (ss * sg < 0) atomicOr((unsigned long long *)&negmask[s >> 6], 1ull << (s & 63));
    if (mm) atomicOr((unsigned long long *)&mmask[s >> 6], 1ull << (s & 63));
    if (a.pivot < 0) { cf[0] = mk<double>(0.5, 0); cf[1] = mk<double>(0.5 * ss * sg, 0); }
    else { cf[0] = mk<double>(1, 0); cf[1] = mk<double>(ss * sg, 0); }
  }
  __syncthreads();
  const SiteOps so{ops, nullptr, nullptr, l};
  shot_step<T, NT>(m, s, l, r, so, cf[0], cf[1], false, c, lds, eig_n, clk, &sweeps, K_EXPECT);
}

__global__ void k_clear_words(uint64_t *a, uint64_t *b, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) { a[i] = 0; b[i] = 0; }
}

template <typename T, int NT>
void launch_layer(const MpsDev &m, const uint64_t *d_pbits, const uint64_t *d_psgn, int W, int SW,
                  const double *d_theta, int64_t stride, const RotLayer &L, hipStream_t st) {
  const int en = m.lds_order ? m.lds_order : eig_lds_order(m.chi, NT);
  if (m.prof)
    KLAUNCH(K_LAYER, (k_layer<T, NT, true>), dim3(m.S), dim3(NT), lds_bytes(NT, sizeof(T) == 8, en), st, m, d_pbits,
            d_psgn, W, SW, d_theta, stride, L, en);
  else
    KLAUNCH(K_LAYER, (k_layer<T, NT, false>), dim3(m.S), dim3(NT), lds_bytes(NT, sizeof(T) == 8, en), st, m, d_pbits,
            d_psgn, W, SW, d_theta, stride, L, en);
}

}  // namespace

size_t layer_fallback_bytes(int chi) {
  const size_t rows = 4 * (size_t)chi + 2, P = 2 * (size_t)chi + 2, H = P / 2 + 1;
  return rows * sizeof(c64) + H * sizeof(c64) + 2 * rows * sizeof(double) + P * sizeof(double) +
         2 * H * sizeof(double) + P * sizeof(int) + (P + 2) * sizeof(int) + 2 * H * sizeof(int) + 64;
}

template <typename T, int NT>
void launch_meas(const MpsDev &m, const uint64_t *d_snap_sign, const c64 *d_ops, const c64 *d_eops,
                 const MeasStep &a, const double *d_u, const uint8_t *d_forced, uint8_t *d_out, double *d_prob,
                 uint64_t *d_negmask, uint64_t *d_mmask, hipStream_t st) {
  const int en = m.lds_order ? m.lds_order : eig_lds_order(m.chi, NT);
  if (m.prof)
    KLAUNCH(K_EXPECT, (k_meas<T, NT, true>), dim3(m.S), dim3(NT), lds_bytes(NT, sizeof(T) == 8, en), st, m, d_snap_sign,
            d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, en);
  else
    KLAUNCH(K_EXPECT, (k_meas<T, NT, false>), dim3(m.S), dim3(NT), lds_bytes(NT, sizeof(T) == 8, en), st, m, d_snap_sign,
            d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, en);
}

template <typename T>
void mps_measure_fused(const MpsDev &m, const uint64_t *d_snap_sign, const c64 *d_ops, const c64 *d_eops,
                       const MeasStep &a, const double *d_u, const uint8_t *d_forced, uint8_t *d_out,
                       double *d_prob, uint64_t *d_negmask, uint64_t *d_mmask, int nt, hipStream_t st) {
  const int SW = (m.S + 63) / 64;
  KLAUNCH(K_TABLEAU, k_clear_words, dim3(1), dim3(64), 0, st, d_negmask, d_mmask, SW);
  if (nt == 64) launch_meas<T, 64>(m, d_snap_sign, d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, st);
  else if (nt == 128) launch_meas<T, 128>(m, d_snap_sign, d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, st);
  else if (nt == 256) launch_meas<T, 256>(m, d_snap_sign, d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, st);
  else launch_meas<T, 512>(m, d_snap_sign, d_ops, d_eops, a, d_u, d_forced, d_out, d_prob, d_negmask, d_mmask, st);
}

template <typename T>
void mps_rot_layer(const MpsDev &m, const uint64_t *d_pbits, const uint64_t *d_psgn, int W, int SW,
                   const double *d_theta, int64_t stride, const RotLayer &L, int nt, hipStream_t st) {
  if (nt == 64) launch_layer<T, 64>(m, d_pbits, d_psgn, W, SW, d_theta, stride, L, st);
  else if (nt == 128) launch_layer<T, 128>(m, d_pbits, d_psgn, W, SW, d_theta, stride, L, st);
  else if (nt == 256) launch_layer<T, 256>(m, d_pbits, d_psgn, W, SW, d_theta, stride, L, st);
  else launch_layer<T, 512>(m, d_pbits, d_psgn, W, SW, d_theta, stride, L, st);
}

template <typename T>
hipError_t layer_prepare() {
  hipError_t e = hipSuccess;
  const void *fs[16] = {(const void *)k_layer<T, 64, false>, (const void *)k_layer<T, 128, false>,
                        (const void *)k_layer<T, 256, false>, (const void *)k_layer<T, 512, false>,
                        (const void *)k_meas<T, 64, false>, (const void *)k_meas<T, 128, false>,
                        (const void *)k_meas<T, 256, false>, (const void *)k_meas<T, 512, false>,
                        (const void *)k_layer<T, 64, true>, (const void *)k_layer<T, 128, true>,
                        (const void *)k_layer<T, 256, true>, (const void *)k_layer<T, 512, true>,
                        (const void *)k_meas<T, 64, true>, (const void *)k_meas<T, 128, true>,
                        (const void *)k_meas<T, 256, true>, (const void *)k_meas<T, 512, true>};
  const int nts[4] = {64, 128, 256, 512};
  for (int i = 0; i < 16; ++i) {
    hipError_t e2 = hipFuncSetAttribute(fs[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds_bytes(nts[i % 4], sizeof(T) == 8, kEigLdsMax));
    if (e == hipSuccess) e = e2;
  }
  return e;
}

template void mps_rot_layer<float>(const MpsDev &, const uint64_t *, const uint64_t *, int, int,
                                   const double *, int64_t, const RotLayer &, int, hipStream_t);
template void mps_rot_layer<double>(const MpsDev &, const uint64_t *, const uint64_t *, int, int,
                                    const double *, int64_t, const RotLayer &, int, hipStream_t);
template void mps_measure_fused<float>(const MpsDev &, const uint64_t *, const c64 *, const c64 *, const MeasStep &,
                                       const double *, const uint8_t *, uint8_t *, double *, uint64_t *, uint64_t *,
                                       int, hipStream_t);
template void mps_measure_fused<double>(const MpsDev &, const uint64_t *, const c64 *, const c64 *, const MeasStep &,
                                        const double *, const uint8_t *, uint8_t *, double *, uint64_t *, uint64_t *,
                                        int, hipStream_t);
template hipError_t layer_prepare<float>();
template hipError_t layer_prepare<double>();
