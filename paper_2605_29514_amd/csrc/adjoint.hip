// Adjoint (reverse-mode) pass for d log P(record) / d theta.
//
// The forward run, seen in the MPS frame, is a chain of linear steps
// F = T R (rotation, R = cos(t) - i sigma sin(t) P', Eq. 4) and F = T M
// (measurement projection, Sec. IV.A), each followed by renormalisation; T
// is the truncation of the step held fixed (identity when chi_max dropped
// nothing above the relative cut, else the projector onto the kept right
// Schmidt subspace right of site l).  With p_k = ||A_k phi_k||^2 and
// A_k = (I + s sigma P'_k)/2, the adjoint state mu runs backwards:
//     mu <- F^dag mu / n           (n = ||F phi|| of the forward)
//     mu <- mu + A_k phi_k / p_k - phi_k        at measurement k
//     dJ/dtheta_r = 2 Re <mu | -i sigma P'_r | phi_{r-1}> = 2 sigma Im <mu|P'|phi>
// mu is an MPS of its own (bond cap of the adjoint context); this file
// holds the kernels that are specific to it: the MPS sum mu + c1 phi +
// c2 P' phi, the frozen projection (contraction of mu's right part with the
// forward state's right Schmidt basis) and the overlap <mu|P'|phi>.  The
// two-term steps R^dag and M^dag reuse the forward's build and compression
// kernels on mu (with its norm kept).
#include "linalg.h"

namespace {

using namespace stnk;

constexpr int TB = 256;

template <typename TA, typename TB_, typename TC, typename ACC>
__device__ void gemm_all(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                         const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc) {
  __shared__ __align__(16) char stage[GemmStage<ACC>::bytes];
  gemm_tiles<TA, TB_, TC, ACC, TB>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, blockIdx.x, gridDim.x, stage);
}

__device__ inline double sgn_of(const uint64_t *w, int s) { return ((w[s >> 6] >> (s & 63)) & 1ull) ? -1.0 : 1.0; }

__global__ void k_step_reset(MpsDev m) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < m.S) { m.trunc[s] = 0; m.nrm[s] = 1.0; }
}

// Site operators of M^dag for a pivot measurement: O1 = Pi0 at the pivot,
// O2 = O_k Pi0 at the pivot (second column zero); the P' site operators
// elsewhere.  Without a pivot M is Hermitian and the forward table serves.
__global__ void k_ops_measure_adj(const uint64_t *bits, int W, int l, int r, int pivot, c64 *ops) {
  const int j = l + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > r) return;
  c64 *o = ops + (size_t)(j - l) * 8;
  site_op(0, 0, o);
  site_op(bitw(bits, j), bitw(bits + W, j), o + 4);
  if (j == pivot) {
    o[3] = mk<double>(0, 0);
    o[5] = mk<double>(0, 0);
    o[7] = mk<double>(0, 0);
  }
}

__global__ void k_adj_coef(MpsDev mu, int kind, int pivot, const double *theta, const uint64_t *sign,
                           const uint64_t *mmask, const double *nrm, const double *pm) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= mu.S) return;
  const double sg = sgn_of(sign, s);
  const double n = sqrt(nrm[s]);
  c64 a, b;
  if (kind == 0) {                            // R^dag / n = (cos t + i sigma sin t P') / n
    const double th = theta[s];
    a = mk<double>(cos(th) / n, 0);
    b = mk<double>(0, sg * sin(th) / n);
  } else if (kind == 1) {                     // M^dag / n
    const double ss = sgn_of(mmask, s);
    if (pivot < 0) { a = mk<double>(0.5 / n, 0); b = mk<double>(0.5 * ss * sg / n, 0); }
    else { a = mk<double>(1.0 / n, 0); b = mk<double>(ss * sg / n, 0); }
  } else {                                    // A phi / p - phi = (1/2p - 1) phi + (s sigma / 2p) P' phi
    const double ss = sgn_of(mmask, s);
    const double p = pm[s];
    a = mk<double>(0.5 / p - 1.0, 0);
    b = mk<double>(0.5 * ss * sg / p, 0);
  }
  mu.coef[2 * s] = a;
  mu.coef[2 * s + 1] = b;
}

// mu <- mu + Y with Y = a O1 phi + b O2 phi over [l, r] (bond-2 blocks as in
// the forward step, a, b = mu.coef): block-diagonal sum, site 0 concatenated
// along its right bond and site n-1 along its left bond.  Site 0 goes to
// mu's scratch T, the others to mu's workspace slots; wb = summed bonds.
template <typename T>
__global__ void k_build_sum(MpsDev mu, MpsDev ph, int l, int r, const c64 *ops) {
  const int s = blockIdx.z, j = blockIdx.y, n = mu.n;
  const int *bm = bnd(mu, s), *bp = bnd(ph, s);
  const bool dbl = l < r;
  const int bpl = bp[j], bpr = bp[j + 1];
  const int byl = (dbl && j > l && j <= r) ? 2 * bpl : bpl;
  const int byr = (dbl && j + 1 > l && j + 1 <= r) ? 2 * bpr : bpr;
  const int bml = bm[j], bmr = bm[j + 1];
  const int Dl = j == 0 ? 1 : bml + byl, Dr = j == n - 1 ? 1 : bmr + byr;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    wbd(mu, s)[j] = Dl;
    if (j == n - 1) wbd(mu, s)[n] = 1;
  }
  cplx<T> *out = j == 0 ? scr<T>(mu.T, mu.T_cap, s) : wslot<T>(mu, j, s);
  const cplx<T> *M = slot<T>(mu, j, s);
  const cplx<T> *P = slot<T>(ph, j, s);
  const c64 ca = mu.coef[2 * s], cb = mu.coef[2 * s + 1];
  const c64 *o1 = (j >= l && j <= r) ? ops + (size_t)(j - l) * 8 : nullptr;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < Dl * Dr; e += gridDim.x * blockDim.x) {
    const int a = e / Dr, c = e % Dr;
    bool isMu, zero = false;
    int ma = a, mc = c, ya = a - bml, yc = c - bmr;
    if (j == 0) { isMu = c < bmr; ma = 0; ya = 0; }
    else if (j == n - 1) { isMu = a < bml; mc = 0; yc = 0; }
    else {
      const bool rm = a < bml, cm = c < bmr;
      zero = rm != cm;
      isMu = rm;
    }
    c64 y0 = mk<double>(0, 0), y1 = mk<double>(0, 0);
    if (!zero && isMu) {
      y0 = cvt<double>(M[(size_t)(ma * 2 + 0) * bmr + mc]);
      y1 = cvt<double>(M[(size_t)(ma * 2 + 1) * bmr + mc]);
    } else if (!zero) {
      // element (ya, yc) of Y_j
      int br = -1, aa = ya, cc = yc;
      if (!o1) br = 2;                                     // outside the span: phi itself
      else if (!dbl) br = 3;                               // single site: a O1 + b O2
      else if (j == l) { br = yc >= bpr; cc = yc - (br ? bpr : 0); }
      else if (j == r) { br = ya >= bpl; aa = ya - (br ? bpl : 0); }
      else {
        const int ba = ya >= bpl, bc = yc >= bpr;
        br = ba == bc ? ba : -1;
        aa = ya - (ba ? bpl : 0);
        cc = yc - (bc ? bpr : 0);
      }
      if (br >= 0) {
        const c64 x0 = cvt<double>(P[(size_t)(aa * 2 + 0) * bpr + cc]);
        const c64 x1 = cvt<double>(P[(size_t)(aa * 2 + 1) * bpr + cc]);
        if (br == 2) { y0 = x0; y1 = x1; }
        else if (br == 3) {
          y0 = ca * (o1[0] * x0 + o1[1] * x1) + cb * (o1[4] * x0 + o1[5] * x1);
          y1 = ca * (o1[2] * x0 + o1[3] * x1) + cb * (o1[6] * x0 + o1[7] * x1);
        } else {
          const c64 *o = o1 + (br ? 4 : 0);
          y0 = o[0] * x0 + o[1] * x1;
          y1 = o[2] * x0 + o[3] * x1;
          if (j == l) { const c64 k = br ? cb : ca; y0 = k * y0; y1 = k * y1; }
        }
      }
    }
    out[(size_t)(a * 2 + 0) * Dr + c] = cvt<T>(y0);
    out[(size_t)(a * 2 + 1) * Dr + c] = cvt<T>(y1);
  }
}

// ----------------------------------------------------- frozen projection
// For flagged shots: E_{n} = 1, E_j = sum_s mu_j^s E_{j+1} (phi_j^s)^dag down
// to j = l+1; then mu_l <- mu_l E_{l+1} and mu's sites > l <- phi's.
__global__ void k_pr_init(MpsDev mu, const int *flag) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < mu.S && flag[s]) mu.E[(size_t)s * mu.E_cap] = mk<double>(1, 0);
}

// F = mu_j (2 bm_j x bm_{j+1}) * E (bm_{j+1} x bp_{j+1})
template <typename T>
__global__ void k_pr_f(MpsDev mu, MpsDev ph, int j, const int *flag) {
  const int s = blockIdx.z;
  if (!flag[s]) return;
  const int bml = bnd(mu, s)[j], bmr = bnd(mu, s)[j + 1], bpr = bnd(ph, s)[j + 1];
  gemm_all<T, double, double, double>(2 * bml, bpr, bmr, slot<T>(mu, j, s), bmr, 0, mu.E + s * mu.E_cap, bpr, 0,
                                      mu.F + s * mu.F_cap, bpr);
}

// E = F (bm_j x 2 bp_{j+1}) * phi_j^H (2 bp_{j+1} x bp_j)
template <typename T>
__global__ void k_pr_e(MpsDev mu, MpsDev ph, int j, const int *flag) {
  const int s = blockIdx.z;
  if (!flag[s]) return;
  const int bml = bnd(mu, s)[j], bpl = bnd(ph, s)[j], bpr = bnd(ph, s)[j + 1];
  gemm_all<double, T, double, double>(bml, bpl, 2 * bpr, mu.F + s * mu.F_cap, 2 * bpr, 0, slot<T>(ph, j, s), 2 * bpr, 1,
                                      mu.E + s * mu.E_cap, bpl);
}

// mu_l <- F (= mu_l E_{l+1}, shape bm_l x 2 x bp_{l+1}); sites > l <- phi's.
template <typename T>
__global__ void k_pr_store(MpsDev mu, MpsDev ph, int l, const int *flag) {
  const int s = blockIdx.y;
  if (!flag[s]) return;
  int *bm = bnd(mu, s);
  const int *bp = bnd(ph, s);
  const int n = mu.n;
  // sites l+1 .. n-1 are copied by blockIdx.x >= 1 (strided), site l by block 0
  if (blockIdx.x == 0) {
    const int cnt = bm[l] * 2 * bp[l + 1];
    cplx<T> *A = slot<T>(mu, l, s);
    const c64 *F = mu.F + s * mu.F_cap;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) A[e] = cvt<T>(F[e]);
  } else {
    for (int j = l + blockIdx.x; j < n; j += gridDim.x - 1) {
      const int cnt = bp[j] * 2 * bp[j + 1];
      const cplx<T> *src = slot<T>(ph, j, s);
      cplx<T> *dst = slot<T>(mu, j, s);
      for (int e = threadIdx.x; e < cnt; e += blockDim.x) dst[e] = src[e];
    }
  }
}

__global__ void k_pr_bonds(MpsDev mu, MpsDev ph, int l, const int *flag) {
  const int s = blockIdx.x;
  if (!flag[s]) return;
  for (int b = l + 1 + threadIdx.x; b <= mu.n; b += blockDim.x) bnd(mu, s)[b] = bnd(ph, s)[b];
}

// ------------------------------------------------------------ overlap
// E_0 = 1, F = E phi_j, F <- O_j F (physical index), E <- mu_j^H F; the
// value <mu|P'|phi> is E after the last site.
__global__ void k_ov_init(MpsDev mu) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < mu.S) mu.E[(size_t)s * mu.E_cap] = mk<double>(1, 0);
}

template <typename T>
__global__ void k_ov_f(MpsDev mu, MpsDev ph, int j) {
  const int s = blockIdx.z;
  const int bml = bnd(mu, s)[j], bpl = bnd(ph, s)[j], bpr = bnd(ph, s)[j + 1];
  gemm_all<double, T, double, double>(bml, 2 * bpr, bpl, mu.E + s * mu.E_cap, bpl, 0, slot<T>(ph, j, s), 2 * bpr, 0,
                                      mu.F + s * mu.F_cap, 2 * bpr);
}

__global__ void k_ov_op(MpsDev mu, MpsDev ph, int j, const c64 *o) {
  const int s = blockIdx.y;
  const int bml = bnd(mu, s)[j], bpr = bnd(ph, s)[j + 1];
  c64 *F = mu.F + s * mu.F_cap;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < bml * bpr; e += gridDim.x * blockDim.x) {
    const int a = e / bpr, c = e % bpr;
    const c64 f0 = F[(size_t)(a * 2 + 0) * bpr + c], f1 = F[(size_t)(a * 2 + 1) * bpr + c];
    F[(size_t)(a * 2 + 0) * bpr + c] = o[0] * f0 + o[1] * f1;
    F[(size_t)(a * 2 + 1) * bpr + c] = o[2] * f0 + o[3] * f1;
  }
}

template <typename T>
__global__ void k_ov_e(MpsDev mu, MpsDev ph, int j) {
  const int s = blockIdx.z;
  const int bml = bnd(mu, s)[j], bmr = bnd(mu, s)[j + 1], bpr = bnd(ph, s)[j + 1];
  gemm_all<T, double, double, double>(bmr, bpr, 2 * bml, slot<T>(mu, j, s), bmr, 1, mu.F + s * mu.F_cap, bpr, 0,
                                      mu.E + s * mu.E_cap, bpr);
}

__global__ void k_ov_out(MpsDev mu, const uint64_t *sign, double *grad, int64_t stride) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= mu.S) return;
  const c64 v = mu.E[(size_t)s * mu.E_cap];
  grad[(int64_t)s * stride] = 2.0 * sgn_of(sign, s) * v.y;
}

template <typename T>
__global__ void k_zero(MpsDev m) {
  const int s = blockIdx.x;
  for (int j = threadIdx.x; j < m.n; j += blockDim.x) {
    cplx<T> *a = slot<T>(m, j, s);
    a[0] = mk<T>(0, 0);
    a[1] = mk<T>(0, 0);
  }
  for (int b = threadIdx.x; b <= m.n; b += blockDim.x) bnd(m, s)[b] = 1;
}

inline int imin(int a, int b) { return a < b ? a : b; }
inline int dmx(const MpsDev &m, int b) {
  int e = b < m.n - b ? b : m.n - b;
  long phys = e >= 30 ? (1L << 30) : (1L << e);
  return (int)(phys < m.chi ? phys : m.chi);
}
inline dim3 ggrid(int M, int N, int S) {
  long tiles = (long)((M + GT - 1) / GT) * ((N + GT - 1) / GT);
  long want = (8192 + S - 1) / S;
  long b = tiles < want ? tiles : want;
  return dim3((unsigned)(b < 1 ? 1 : b), 1, S);
}

}  // namespace

void launch_step_reset(const MpsDev &m, hipStream_t st) {
  KLAUNCH(K_BUILD, k_step_reset, dim3((m.S + 255) / 256), dim3(256), 0, st, m);
}

void launch_ops_measure_adj(const uint64_t *d_bits, int W, int l, int r, int pivot, c64 *d_ops, hipStream_t st) {
  const int cnt = r - l + 1;
  KLAUNCH(K_BUILD, k_ops_measure_adj, dim3((cnt + 63) / 64), dim3(64), 0, st, d_bits, W, l, r, pivot, d_ops);
}

void launch_adj_coef(const MpsDev &mu, int kind, int pivot, const double *d_theta, const uint64_t *d_sign,
                     const uint64_t *d_mmask, const double *d_nrm, const double *d_pm, hipStream_t st) {
  KLAUNCH(K_BUILD, k_adj_coef, dim3((mu.S + 255) / 256), dim3(256), 0, st, mu, kind, pivot, d_theta, d_sign,
          d_mmask, d_nrm, d_pm);
}

template <typename T>
void mps_build_sum(const MpsDev &mu, const MpsDev &ph, int l, int r, const c64 *d_ops, hipStream_t st) {
  long maxe = 0;
  for (int j = 0; j < mu.n; ++j) {
    long a = j == 0 ? 1 : 3L * dmx(mu, j), c = j == mu.n - 1 ? 1 : 3L * dmx(mu, j + 1);
    maxe = std::max(maxe, a * c);
  }
  long want = (8192 + mu.S * mu.n - 1) / ((long)mu.S * mu.n);
  long blocks = std::max(1L, std::min((maxe + TB - 1) / TB, want));
  KLAUNCH(K_BUILD, k_build_sum<T>, dim3((unsigned)blocks, mu.n, mu.S), dim3(TB), 0, st, mu, ph, l, r, d_ops);
}

template <typename T>
void mps_project_right(const MpsDev &mu, const MpsDev &ph, int l, const int *d_flag, hipStream_t st) {
  KLAUNCH(K_BUILD, k_pr_init, dim3((mu.S + 255) / 256), dim3(256), 0, st, mu, d_flag);
  for (int j = mu.n - 1; j >= l + 1; --j) {
    KLAUNCH(K_EXPECT, k_pr_f<T>, ggrid(2 * dmx(mu, j), dmx(ph, j + 1), mu.S), dim3(TB), 0, st, mu, ph, j, d_flag);
    KLAUNCH(K_EXPECT, k_pr_e<T>, ggrid(dmx(mu, j), dmx(ph, j), mu.S), dim3(TB), 0, st, mu, ph, j, d_flag);
  }
  KLAUNCH(K_EXPECT, k_pr_f<T>, ggrid(2 * dmx(mu, l), dmx(ph, l + 1), mu.S), dim3(TB), 0, st, mu, ph, l, d_flag);
  KLAUNCH(K_BUILD, k_pr_store<T>, dim3(1 + imin(mu.n - l - 1, 16), mu.S), dim3(TB), 0, st, mu, ph, l, d_flag);
  KLAUNCH(K_BUILD, k_pr_bonds, dim3(mu.S), dim3(64), 0, st, mu, ph, l, d_flag);
}

template <typename T>
void mps_overlap_grad(const MpsDev &mu, const MpsDev &ph, const c64 *d_eops, int l, int r, const uint64_t *d_sign,
                      double *d_grad, int64_t stride, hipStream_t st) {
  KLAUNCH(K_EXPECT, k_ov_init, dim3((mu.S + 255) / 256), dim3(256), 0, st, mu);
  for (int j = 0; j < mu.n; ++j) {
    KLAUNCH(K_EXPECT, k_ov_f<T>, ggrid(dmx(mu, j), 2 * dmx(ph, j + 1), mu.S), dim3(TB), 0, st, mu, ph, j);
    if (j >= l && j <= r) {
      long cnt = (long)dmx(mu, j) * dmx(ph, j + 1);
      long b = std::max(1L, std::min((cnt + TB - 1) / TB, (8192L + mu.S - 1) / mu.S));
      KLAUNCH(K_EXPECT, k_ov_op, dim3((unsigned)b, mu.S), dim3(TB), 0, st, mu, ph, j, d_eops + (size_t)(j - l) * 4);
    }
    KLAUNCH(K_EXPECT, k_ov_e<T>, ggrid(dmx(mu, j + 1), dmx(ph, j + 1), mu.S), dim3(TB), 0, st, mu, ph, j);
  }
  KLAUNCH(K_EXPECT, k_ov_out, dim3((mu.S + 255) / 256), dim3(256), 0, st, mu, d_sign, d_grad, stride);
}

template <typename T>
void mps_zero(const MpsDev &m, hipStream_t st) {
  KLAUNCH(K_BUILD, k_zero<T>, dim3(m.S), dim3(64), 0, st, m);
}

#define INST_ADJ(T)                                                                                        \
  template void mps_build_sum<T>(const MpsDev &, const MpsDev &, int, int, const c64 *, hipStream_t);    \
  template void mps_project_right<T>(const MpsDev &, const MpsDev &, int, const int *, hipStream_t);     \
  template void mps_overlap_grad<T>(const MpsDev &, const MpsDev &, const c64 *, int, int, const uint64_t *, \
                                    double *, int64_t, hipStream_t);                                      \
  template void mps_zero<T>(const MpsDev &, hipStream_t);
INST_ADJ(float)
INST_ADJ(double)

namespace {
__global__ void k_gather_theta(const double *theta, int64_t stride, int idx, double *dst, int S) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) dst[s] = theta[(int64_t)s * stride + idx];
}
}  // namespace

void launch_gather_theta(const double *d_theta, int64_t stride, int idx, double *d_dst, int S, hipStream_t st) {
  KLAUNCH(K_BUILD, k_gather_theta, dim3((S + 255) / 256), dim3(256), 0, st, d_theta, stride, idx, d_dst, S);
}
