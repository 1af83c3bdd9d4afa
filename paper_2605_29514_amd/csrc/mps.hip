// MPS kernels of the STN step, batched over shots (Sec. IV.A-B).
//
// Every shot owns one slot per site holding its tensor A_j (dl, 2, dr)
// row-major with its actual bonds (dl, dr read from bond[s][j], bond[s][j+1]),
// interleaved complex T (float or double).  Shots share the circuit, so every
// kernel is launched once for all shots with a grid sized for the largest
// possible bonds; blocks beyond a shot's actual bonds return at once.
//
// The non-Clifford step is a two-term operator over a span [l, r]
//     phi <- a * (x)_j O1_j phi + b * (x)_j O2_j phi
// (rotation cos(theta) I - i sin(theta) sigma P', Sec. IV.A; measurement
// projectors), applied as a bond-2 operator, then compressed back:
//   left-to-right : Householder QR of each doubled tensor, R absorbed to the right
//   right-to-left : FP64 Gram X^H X of the centre, FP64 Jacobi eigen-solve,
//                   keep the largest eigenvalues (squared Schmidt values, Eq. 8)
//                   up to chi_max, site <- V^H, centre <- Q (X V).
#include "common.h"

#include <math.h>

#include <algorithm>

#include "linalg.h"

namespace {

using namespace stnk;

constexpr int TB = 256;          // threads per block of the per-step kernels
constexpr int kEigLdsN = 64;     // FP32 path: factor in LDS up to this order (66.5 KB)
constexpr int kJacLdsN = 32;     // FP64 path: Jacobi G and V in LDS up to this order (2 x 16.5 KB)
constexpr int kEigIdx = 2064;    // eigen-solve index / pair tables (orders up to 2 x 1024 + 16)
constexpr size_t kQrLdsMat = 16 * 1024;

__device__ inline bool first_block() { return blockIdx.x == 0 && threadIdx.x == 0; }

// All tiles of one shot's product, strided over the blocks given to it:
// grids are sized from a per-shot block budget, not from the largest
// possible bonds, so early (small-bond) steps do not launch empty tiles.
template <typename TA, typename TB_, typename TC, typename ACC>
__device__ void gemm_all(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                         const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc) {
  __shared__ __align__(16) char stage[GemmStage<ACC>::bytes];
  gemm_tiles<TA, TB_, TC, ACC, TB>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, blockIdx.x, gridDim.x, stage);
}

// QR of the m x nc matrix at A (global).  When it fits, the matrix is first
// copied to LDS (after the reflector scratch) so the column sweeps run at
// LDS rather than L2 bandwidth.  lds_rows: rows the scratch was sized for.
template <typename T>
__device__ void qr_dispatch(int rows, int cols, cplx<T> *A, cplx<T> *Qd, int qt, cplx<T> *Rd,
                            char *lds, int lds_rows) {
  c64 *vs = reinterpret_cast<c64 *>(lds);
  double *vd = reinterpret_cast<double *>(vs + lds_rows);
  c64 *wp = reinterpret_cast<c64 *>(vd + 2 * lds_rows);
  cplx<T> *Al = reinterpret_cast<cplx<T> *>(wp + TB);
  if ((size_t)rows * cols * sizeof(cplx<T>) <= kQrLdsMat) {
    for (int e = threadIdx.x; e < rows * cols; e += TB) Al[e] = A[e];
    __syncthreads();
    qr_block<T, TB>(rows, cols, Al, Qd, qt, Rd, vs, vd, wp);
  } else {
    qr_block<T, TB>(rows, cols, A, Qd, qt, Rd, vs, vd, wp);
  }
}

// ================================================================ kernels

// Initial state |0...0>, bonds 1.
template <typename T>
__global__ void k_init(MpsDev m) {
  const int s = blockIdx.x;
  for (int j = threadIdx.x; j < m.n; j += blockDim.x) {
    cplx<T> *a = slot<T>(m, j, s);
    a[0] = mk<T>(1, 0);
    a[1] = mk<T>(0, 0);
  }
  for (int b = threadIdx.x; b <= m.n; b += blockDim.x) bnd(m, s)[b] = 1;
  if (threadIdx.x == 0) { m.logp[s] = 0; m.fid[s] = 1; }
}

// In-place single-site two-term op on site `site`: A <- a O1 A + b O2 A.
template <typename T>
__global__ void k_apply1(MpsDev m, int site, const c64 *ops) {
  const int s = blockIdx.y;
  const int dl = bnd(m, s)[site], dr = bnd(m, s)[site + 1];
  cplx<T> *A = slot<T>(m, site, s);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dl * dr; e += gridDim.x * blockDim.x) {
  const int a = e / dr, c = e % dr;
  c64 x0 = cvt<double>(A[(size_t)(a * 2 + 0) * dr + c]);
  c64 x1 = cvt<double>(A[(size_t)(a * 2 + 1) * dr + c]);
  c64 ca = m.coef[2 * s], cb = m.coef[2 * s + 1];
  const c64 *o1 = ops, *o2 = ops + 4;
  c64 y0 = ca * (o1[0] * x0 + o1[1] * x1) + cb * (o2[0] * x0 + o2[1] * x1);
  c64 y1 = ca * (o1[2] * x0 + o1[3] * x1) + cb * (o2[2] * x0 + o2[3] * x1);
  A[(size_t)(a * 2 + 0) * dr + c] = cvt<T>(y0);
  A[(size_t)(a * 2 + 1) * dr + c] = cvt<T>(y1);
  }
}

// Bond-2 operator blocks over [l, r]:
//   B_l = [a O1 A_l | b O2 A_l]      -> scratch T   (dl, 2, 2dr)
//   B_j = diag(O1 A_j, O2 A_j)       -> wslot j     (2dl, 2, 2dr)
//   B_r = [O1 A_r ; O2 A_r]          -> wslot r     (2dl, 2, dr)
template <typename T>
__global__ void k_build(MpsDev m, int l, int r, const c64 *ops) {
  const int s = blockIdx.z;
  const int j = l + blockIdx.y;
  const int *b = bnd(m, s);
  const int dl = b[j], dr = b[j + 1];
  const int Dl = (j == l) ? dl : 2 * dl;
  const int Dr = (j == r) ? dr : 2 * dr;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int *w = wbd(m, s);
    w[j] = Dl;
    if (j == r) w[r + 1] = dr;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < Dl * Dr; e += gridDim.x * blockDim.x) {
  const int a = e / Dr, c = e % Dr;
  const int ba = a >= dl, bc = c >= dr;   // branch of the row / column index
  cplx<T> *out = (j == l) ? scr<T>(m.T, m.T_cap, s) : wslot<T>(m, j, s);
  c64 y0 = mk<double>(0, 0), y1 = mk<double>(0, 0);
  int br = -1;
  if (j == l) br = bc;
  else if (j == r) br = ba;
  else if (ba == bc) br = ba;
  if (br >= 0) {
    const cplx<T> *A = slot<T>(m, j, s);
    int aa = a - (ba ? dl : 0), cc = c - (bc ? dr : 0);
    if (j == l) aa = a;
    if (j == r) cc = c;
    c64 x0 = cvt<double>(A[(size_t)(aa * 2 + 0) * dr + cc]);
    c64 x1 = cvt<double>(A[(size_t)(aa * 2 + 1) * dr + cc]);
    const c64 *o = ops + (size_t)(j - l) * 8 + (br ? 4 : 0);
    y0 = o[0] * x0 + o[1] * x1;
    y1 = o[2] * x0 + o[3] * x1;
    if (j == l) {
      c64 cf = m.coef[2 * s + br];
      y0 = cf * y0;
      y1 = cf * y1;
    }
  }
  out[(size_t)(a * 2 + 0) * Dr + c] = cvt<T>(y0);
  out[(size_t)(a * 2 + 1) * Dr + c] = cvt<T>(y1);
  }
}

// QR in the left-to-right sweep: scratch T as (2 wb[j]) x wb[j+1] -> Q into
// wslot j, R into scratch R; aux[0] = new bond p, aux[1] = old bond.
template <typename T>
__global__ void k_qr_lr(MpsDev m, int j, int lds_rows) {
  extern __shared__ char lds[];
  const int s = blockIdx.x;
  int *w = wbd(m, s);
  const int rows = 2 * w[j], cols = w[j + 1];
  const int p = rows < cols ? rows : cols;
  qr_dispatch<T>(rows, cols, scr<T>(m.T, m.T_cap, s), wslot<T>(m, j, s), 0, scr<T>(m.R, m.R_cap, s), lds, lds_rows);
  if (threadIdx.x == 0) {
    auxp(m, s)[0] = p; auxp(m, s)[1] = cols;
    add_work(m, K_QR, qr_flops(rows, cols), (double)sizeof(cplx<T>) * ((double)rows * cols * 2 + (double)rows * p + (double)p * cols));
  }
}

// T <- R (p x K) * wslot[j+1] (K x 2 wb[j+2]);  wb[j+1] <- p.
template <typename T>
__global__ void k_absorb_lr(MpsDev m, int j) {
  const int s = blockIdx.z;
  int *w = wbd(m, s);
  const int p = auxp(m, s)[0], K = auxp(m, s)[1], N = 2 * w[j + 2];
  gemm_all<T, T, T, T>(p, N, K, scr<T>(m.R, m.R_cap, s), K, 0, wslot<T>(m, j + 1, s), N, 0,
                          scr<T>(m.T, m.T_cap, s), N);
  __syncthreads();
  if (first_block()) {
    w[j + 1] = p;
    add_work(m, K_GEMM, gemm_flops(p, N, K), (double)sizeof(cplx<T>) * ((double)p * K + (double)K * N + (double)p * N));
  }
}

// Gram G = X^H X (FP64) of the centre X = scratch T as wb[j] x 2 wb[j+1].
template <typename T>
__global__ void k_gram(MpsDev m, int j) {
  const int s = blockIdx.z;
  int *w = wbd(m, s);
  const int L = w[j], nn = 2 * w[j + 1];
  gemm_all<T, T, double, double>(nn, nn, L, scr<T>(m.T, m.T_cap, s), nn, 1,
                                    scr<T>(m.T, m.T_cap, s), nn, 0, m.G + s * m.G_cap, nn);
  if (first_block())
    add_work(m, K_GRAM, gemm_flops(nn, nn, L), (double)sizeof(cplx<T>) * L * nn + 16.0 * nn * nn);
}

// FP64 states: two-sided Jacobi on rho (G and V in LDS up to order
// kJacLdsN, sorted eigenvectors written back into G).  FP32 states: pivoted
// Cholesky + one-sided Jacobi on the factor (in LDS up to order kEigLdsN,
// eigenvectors into V).
template <typename T>
__global__ void k_eig(MpsDev m, int j) {
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x;
  const int nn = 2 * wbd(m, s)[j + 1];
  c64 *Gg = m.G + s * m.G_cap;
  __shared__ int sweeps;
  double fe;
  if constexpr (sizeof(T) == 8) {
    c64 *Gl = reinterpret_cast<c64 *>(lds);                 // used when nn <= kJacLdsN
    c64 *Vl = Gl + kJacLdsN * (kJacLdsN + 1);
    int *pos = reinterpret_cast<int *>(Vl + kJacLdsN * (kJacLdsN + 1));
    int *pp = pos + kEigIdx, *pq = pp + kEigIdx / 2;
    double *pc = reinterpret_cast<double *>(pq + kEigIdx / 2);
    double *ps = pc + kEigIdx / 2;
    c64 *pe = reinterpret_cast<c64 *>(ps + kEigIdx / 2);
    c64 *Gw = Gg, *Vw = m.V + s * m.V_cap;
    int ldw = nn;
    if (nn <= kJacLdsN) {
      ldw = nn + 1;
      for (int e = threadIdx.x; e < nn * nn; e += TB) Gl[(e / nn) * ldw + e % nn] = Gg[e];
      __syncthreads();
      Gw = Gl;
      Vw = Vl;
    }
    jacobi_block<TB>(nn, Gw, ldw, Vw, m.ev + s * m.ev_cap, Gg, m.err, pos, pc, ps, pe, pp, pq, &sweeps,
                     jac_abs<T>(), jac_rel<T>());
    fe = 36.0 * nn * nn * (double)nn;
  } else {
    double *dg = reinterpret_cast<double *>(lds);           // index arrays up to order kEigIdx
    int *piv = reinterpret_cast<int *>(dg + kEigIdx), *pos = piv + kEigIdx;
    c64 *Gl = reinterpret_cast<c64 *>(pos + kEigIdx);       // the factor when nn <= kEigLdsN
    c64 *Gw = Gg;
    int ldw = nn;
    if (nn <= kEigLdsN) {
      ldw = nn + 1;
      for (int e = threadIdx.x; e < nn * nn; e += TB) Gl[(e / nn) * ldw + e % nn] = Gg[e];
      __syncthreads();
      Gw = Gl;
    }
    fe = eig_psd<TB>(nn, Gw, ldw, m.ev + s * m.ev_cap, m.V + s * m.V_cap, m.err, piv, pos, dg, &sweeps,
                     chol_tol(m.eps_cut, nn), eig_conv_tol<T>(), eig_rot_tol<T>());
  }
  // work: the method's operation count; bytes: read G, write eigenvalues and vectors
  if (threadIdx.x == 0) {
    add_work(m, K_EIGEN, eig_nominal_flops(nn), 16.0 * 2 * nn * nn + 8.0 * nn);
    if (m.prof) {
      atomicAdd(&m.work[kPathBase + kPathEigNominal], eig_nominal_flops(nn));
      atomicAdd(&m.work[kPathBase + kPathEigExec], fe);
    }
  }
  if (threadIdx.x == 0 && m.prof) atomicAdd(&m.work[2 * K_COUNT], (double)sweeps);
}

// Squared Schmidt values across bond b (between sites b-1 and b) with the
// orthogonality centre at site b: sites left of b are left-orthonormal and
// right of b right-orthonormal, so the singular values of the centre tensor
// as a dl x 2 dr matrix X are the Schmidt values (Eq. 8's lambda_i).  FP64
// Gram X X^H, two-sided Jacobi (relative accuracy), eigenvalues descending,
// normalised to sum 1; out[s][i] for i < ld (0 past the bond), rank[s] = dl.
template <typename T>
__global__ void k_spectrum(MpsDev m, int b, double *out, int ld, int *rank) {
  extern __shared__ __align__(16) char lds[];
  const int s = blockIdx.x;
  const int dl = bnd(m, s)[b], dr = bnd(m, s)[b + 1];
  const cplx<T> *A = slot<T>(m, b, s);
  c64 *Gg = m.G + s * m.G_cap;
  gemm_direct<T, T, double, double, TB>(dl, dl, 2 * dr, A, 2 * dr, 0, A, 2 * dr, 1, Gg, dl);
  __syncthreads();
  int *pos = reinterpret_cast<int *>(lds);
  int *pp = pos + kEigIdx, *pq = pp + kEigIdx / 2;
  double *pc = reinterpret_cast<double *>(pq + kEigIdx / 2);
  double *ps = pc + kEigIdx / 2;
  c64 *pe = reinterpret_cast<c64 *>(ps + kEigIdx / 2);
  __shared__ int sweeps;
  double *ev = m.ev + s * m.ev_cap;
  jacobi_block<TB>(dl, Gg, dl, m.V + s * m.V_cap, ev, m.E + s * m.E_cap, m.err, pos, pc, ps, pe, pp, pq, &sweeps,
                   1e-18, 1e-15);
  double part = 0;
  for (int i = threadIdx.x; i < dl; i += TB) part += fmax(ev[i], 0.0);
  const double tot = bsum<TB>(part);
  for (int i = threadIdx.x; i < ld; i += TB)
    out[(size_t)s * ld + i] = (i < dl && tot > 0) ? fmax(ev[i], 0.0) / tot : 0.0;
  if (threadIdx.x == 0) {
    if (rank) rank[s] = dl;
    add_work(m, K_EXPECT, gemm_flops(dl, dl, 2 * dr) + 36.0 * dl * dl * (double)dl, 16.0 * (2.0 * dl * dr + dl * dl));
  }
}

template <typename T>
__global__ void k_select(MpsDev m, int j) {
  const int s = blockIdx.x;
  const c64 *V = sizeof(T) == 8 ? m.G + s * m.G_cap : m.V + s * m.V_cap;
  select_body<T, TB>(m, s, j, V, scr<T>(m.Vt, m.Vt_cap, s));
}

// N = X (L x nn) * Vt (nn x k')
template <typename T>
__global__ void k_ngemm(MpsDev m, int j) {
  const int s = blockIdx.z;
  int *w = wbd(m, s);
  const int L = w[j], nn = 2 * w[j + 1], k = auxp(m, s)[2];
  gemm_all<T, T, T, T>(L, k, nn, scr<T>(m.T, m.T_cap, s), nn, 0, scr<T>(m.Vt, m.Vt_cap, s), k, 0,
                       scr<T>(m.N, m.N_cap, s), k);
  if (first_block())
    add_work(m, K_GEMM, gemm_flops(L, k, nn), (double)sizeof(cplx<T>) * ((double)L * nn + (double)nn * k + (double)L * k));
}

// T = wslot[j-1] (2 wb[j-1] x L) * N (L x k');  wb[j] <- k'.
template <typename T>
__global__ void k_xgemm(MpsDev m, int j) {
  const int s = blockIdx.z;
  int *w = wbd(m, s);
  const int M = 2 * w[j - 1], L = auxp(m, s)[3], k = auxp(m, s)[2];
  gemm_all<T, T, T, T>(M, k, L, wslot<T>(m, j - 1, s), L, 0, scr<T>(m.N, m.N_cap, s), k, 0,
                          scr<T>(m.T, m.T_cap, s), k);
  __syncthreads();
  if (first_block()) {
    w[j] = k;
    add_work(m, K_GEMM, gemm_flops(M, k, L), (double)sizeof(cplx<T>) * ((double)M * L + (double)L * k + (double)M * k));
  }
}

template <typename T>
__global__ void k_finish(MpsDev m, int l) {
  finish_body<T, TB>(m, blockIdx.x, l, scr<T>(m.T, m.T_cap, blockIdx.x));
}

// In-place FP64 normalisation of one site (the centre).
template <typename T>
__global__ void k_normalize(MpsDev m, int site) {
  const int s = blockIdx.x;
  const int cnt = bnd(m, s)[site] * 2 * bnd(m, s)[site + 1];
  cplx<T> *A = slot<T>(m, site, s);
  double part = 0;
  for (int e = threadIdx.x; e < cnt; e += TB) part += norm2(cvt<double>(A[e]));
  double n2 = bsum<TB>(part);
  if (!(n2 > 0) || isinf(n2)) {
    if (threadIdx.x == 0) atomicOr(m.err, STN_ERR_NUMERIC);
    return;
  }
  if (threadIdx.x == 0) m.nrm[s] = n2;
  double inv = 1.0 / sqrt(n2);
  for (int e = threadIdx.x; e < cnt; e += TB) A[e] = cvt<T>(inv * cvt<double>(A[e]));
}

// Squared norm of one site (the centre) in FP64 -> nrm[s].
template <typename T>
__global__ void k_sitenorm(MpsDev m, int site) {
  const int s = blockIdx.x;
  const int cnt = bnd(m, s)[site] * 2 * bnd(m, s)[site + 1];
  const cplx<T> *A = slot<T>(m, site, s);
  double part = 0;
  for (int e = threadIdx.x; e < cnt; e += TB) part += norm2(cvt<double>(A[e]));
  double n2 = bsum<TB>(part);
  if (threadIdx.x == 0) m.nrm[s] = n2;
}

// ---------------------------------------------------- centre moves
template <typename T>
__global__ void k_copy_to_T(MpsDev m, int site, int conjt) {
  const int s = blockIdx.y;
  const int dl = bnd(m, s)[site], dr = bnd(m, s)[site + 1];
  const cplx<T> *A = slot<T>(m, site, s);
  cplx<T> *X = scr<T>(m.T, m.T_cap, s);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dl * 2 * dr; e += gridDim.x * blockDim.x) {
    if (!conjt) {
      X[e] = A[e];
    } else {   // X = A^H with A viewed as dl x (2 dr)
      int a = e / (2 * dr), c = e % (2 * dr);
      X[(size_t)c * dl + a] = cj(A[e]);
    }
  }
}

template <typename T>
__global__ void k_copy_from_T(MpsDev m, int site) {
  const int s = blockIdx.y;
  const int dl = bnd(m, s)[site], dr = bnd(m, s)[site + 1];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dl * 2 * dr; e += gridDim.x * blockDim.x)
    slot<T>(m, site, s)[e] = scr<T>(m.T, m.T_cap, s)[e];
}

// Right move at c: T (2 bond[c] x bond[c+1]) = Q R; Q -> slot c.
template <typename T>
__global__ void k_qr_move_r(MpsDev m, int c, int lds_rows) {
  extern __shared__ char lds[];
  const int s = blockIdx.x;
  const int rows = 2 * bnd(m, s)[c], cols = bnd(m, s)[c + 1];
  const int p = rows < cols ? rows : cols;
  qr_dispatch<T>(rows, cols, scr<T>(m.T, m.T_cap, s), slot<T>(m, c, s), 0, scr<T>(m.R, m.R_cap, s), lds, lds_rows);
  if (threadIdx.x == 0) {
    auxp(m, s)[0] = p; auxp(m, s)[1] = cols;
    add_work(m, K_QR, qr_flops(rows, cols), (double)sizeof(cplx<T>) * ((double)rows * cols * 2 + (double)rows * p + (double)p * cols));
  }
}

// Left move at c: T = A_c^H (2 bond[c+1] x bond[c]) = Q R; A_c <- Q^H.
template <typename T>
__global__ void k_qr_move_l(MpsDev m, int c, int lds_rows) {
  extern __shared__ char lds[];
  const int s = blockIdx.x;
  const int rows = 2 * bnd(m, s)[c + 1], cols = bnd(m, s)[c];
  const int p = rows < cols ? rows : cols;
  qr_dispatch<T>(rows, cols, scr<T>(m.T, m.T_cap, s), slot<T>(m, c, s), 1, scr<T>(m.R, m.R_cap, s), lds, lds_rows);
  if (threadIdx.x == 0) {
    auxp(m, s)[0] = p; auxp(m, s)[1] = cols;
    add_work(m, K_QR, qr_flops(rows, cols), (double)sizeof(cplx<T>) * ((double)rows * cols * 2 + (double)rows * p + (double)p * cols));
  }
}

// T = R (p x K) * A_{c+1} (K x 2 bond[c+2]); bond[c+1] <- p
template <typename T>
__global__ void k_absorb_move_r(MpsDev m, int c) {
  const int s = blockIdx.z;
  const int p = auxp(m, s)[0], K = auxp(m, s)[1], N = 2 * bnd(m, s)[c + 2];
  gemm_all<T, T, T, T>(p, N, K, scr<T>(m.R, m.R_cap, s), K, 0, slot<T>(m, c + 1, s), N, 0,
                          scr<T>(m.T, m.T_cap, s), N);
  if (first_block())
    add_work(m, K_GEMM, gemm_flops(p, N, K), (double)sizeof(cplx<T>) * ((double)p * K + (double)K * N + (double)p * N));
}

// T = A_{c-1} (2 bond[c-1] x K) * R^H (K x p); bond[c] <- p
template <typename T>
__global__ void k_absorb_move_l(MpsDev m, int c) {
  const int s = blockIdx.z;
  const int p = auxp(m, s)[0], K = auxp(m, s)[1], M = 2 * bnd(m, s)[c - 1];
  gemm_all<T, T, T, T>(M, p, K, slot<T>(m, c - 1, s), K, 0, scr<T>(m.R, m.R_cap, s), K, 1,
                          scr<T>(m.T, m.T_cap, s), p);
  if (first_block())
    add_work(m, K_GEMM, gemm_flops(M, p, K), (double)sizeof(cplx<T>) * ((double)M * K + (double)K * p + (double)M * p));
}

__global__ void k_set_bond(MpsDev m, int b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < m.S) bnd(m, s)[b] = auxp(m, s)[0];
}

// --------------------------------------------------- expectation values
// <phi| prod_j O_j |phi> with the centre inside [l, r]: E_l = I, then per
// site F = E A_j, F <- O_j F (physical index), E <- A_j^H F; the value is
// tr E after site r.  All in FP64.
template <typename T>
__global__ void k_eye(MpsDev m, int l) {
  const int s = blockIdx.x;
  const int d = bnd(m, s)[l];
  c64 *E = m.E + s * m.E_cap;
  for (int e = threadIdx.x; e < d * d; e += TB) E[e] = mk<double>((e / d) == (e % d) ? 1.0 : 0.0, 0);
}

template <typename T>
__global__ void k_expect_f(MpsDev m, int j, const c64 *ops) {
  const int s = blockIdx.z;
  const int dl = bnd(m, s)[j], dr = bnd(m, s)[j + 1];
  const int N = 2 * dr;
  gemm_all<double, T, double, double>(dl, N, dl, m.E + s * m.E_cap, dl, 0, slot<T>(m, j, s), N, 0,
                                         m.F + s * m.F_cap, N);
  if (first_block())
    add_work(m, K_EXPECT, gemm_flops(dl, N, dl), 16.0 * dl * dl + (double)sizeof(cplx<T>) * dl * N + 16.0 * dl * N);
}

template <typename T>
__global__ void k_expect_op(MpsDev m, int j, const c64 *o) {
  const int s = blockIdx.y;
  const int dl = bnd(m, s)[j], dr = bnd(m, s)[j + 1];
  c64 *F = m.F + s * m.F_cap;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < dl * dr; e += gridDim.x * blockDim.x) {
    const int a = e / dr, c = e % dr;
    c64 f0 = F[(size_t)(a * 2 + 0) * dr + c], f1 = F[(size_t)(a * 2 + 1) * dr + c];
    F[(size_t)(a * 2 + 0) * dr + c] = o[0] * f0 + o[1] * f1;
    F[(size_t)(a * 2 + 1) * dr + c] = o[2] * f0 + o[3] * f1;
  }
}

template <typename T>
__global__ void k_expect_e(MpsDev m, int j) {
  const int s = blockIdx.z;
  const int dl = bnd(m, s)[j], dr = bnd(m, s)[j + 1];
  gemm_all<T, double, double, double>(dr, dr, 2 * dl, slot<T>(m, j, s), dr, 1, m.F + s * m.F_cap, dr,
                                         0, m.E + s * m.E_cap, dr);
  if (first_block())
    add_work(m, K_EXPECT, gemm_flops(dr, dr, 2 * dl), (double)sizeof(cplx<T>) * 2 * dl * dr + 16.0 * 2 * dl * dr + 16.0 * dr * dr);
}

// ------------------------------------------------- operator tables
__global__ void k_ops_rotation(const uint64_t *bits, int W, int l, int r, c64 *ops) {
  const int j = l + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > r) return;
  c64 *o = ops + (size_t)(j - l) * 8;
  site_op(0, 0, o);
  site_op(bitw(bits, j), bitw(bits + W, j), o + 4);
}

// Measurement ops: expectation ops (Pauli sites) and projection ops.
// Diagonal P' (pivot < 0): O1 = I, O2 = Z^z.  Otherwise O1 = I except Pi0 at
// the pivot k, O2 = site ops with Pi0 * O_k at k.
__global__ void k_ops_measure(const uint64_t *bits, int W, int l, int r, int pivot, c64 *ops,
                              c64 *eops) {
  const int j = l + blockIdx.x * blockDim.x + threadIdx.x;
  if (j > r) return;
  c64 *o = ops + (size_t)(j - l) * 8;
  c64 *e = eops + (size_t)(j - l) * 4;
  int x = bitw(bits, j), z = bitw(bits + W, j);
  site_op(x, z, e);
  site_op(0, 0, o);
  site_op(x, z, o + 4);
  if (j == pivot) {
    o[3] = mk<double>(0, 0);                  // Pi0 = diag(1, 0)
    o[6] = mk<double>(0, 0);                  // Pi0 * O: zero the second row
    o[7] = mk<double>(0, 0);
  }
}

// Rotation coefficients a = cos theta, b = -i sigma sin theta per shot.
__global__ void k_coef_rotation(const uint64_t *psgn, int S, const double *theta, int64_t stride,
                                int r, c64 *coef, int *err) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double th = theta[(int64_t)s * stride + r];
  if (!(th == th) || isinf(th)) atomicOr(err, STN_ERR_NUMERIC);
  double sg = ((psgn[s >> 6] >> (s & 63)) & 1ull) ? -1.0 : 1.0;
  coef[2 * s] = mk<double>(cos(th), 0);
  coef[2 * s + 1] = mk<double>(0, -sg * sin(th));
}

// Outcome of one measurement per shot (one lane per shot, 64 shots per
// block so that the wave ballot yields the bit-sliced masks directly).
// p(0) = (N + sigma tr E) / (2N), m = 0 iff u < p(0) (or forced).
__global__ void k_outcome(MpsDev m, const uint64_t *snap_sign, int pivot, int dr_site,
                          const double *u, const uint8_t *forced, int n_meas, int mi, uint8_t *out,
                          double *prob, uint64_t *negmask, uint64_t *mmask) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  int mm = 0, neg = 0;
  if (s < m.S) {
    const int d = bnd(m, s)[dr_site];
    const c64 *E = m.E + s * m.E_cap;
    double tr = 0;
    for (int i = 0; i < d; ++i) tr += E[(size_t)i * d + i].x;
    double sg = ((snap_sign[s >> 6] >> (s & 63)) & 1ull) ? -1.0 : 1.0;
    double N = m.nrm[s];
    double p0 = (N + sg * tr) / (2 * N);
    p0 = fmin(1.0, fmax(0.0, p0));
    if (!(p0 == p0)) { atomicOr(m.err, STN_ERR_NUMERIC); p0 = 0.5; }
    if (forced) mm = forced[(size_t)s * n_meas + mi] ? 1 : 0;
    else mm = u[(size_t)s * n_meas + mi] < p0 ? 0 : 1;
    double pm = mm ? 1.0 - p0 : p0;
    if (pm <= 0) { atomicOr(m.err, STN_ERR_ZEROPROB); pm = 1e-300; }
    m.logp[s] += log(pm);
    m.pm[s] = pm;
    if (out) out[(size_t)s * n_meas + mi] = (uint8_t)mm;
    if (prob) prob[(size_t)s * n_meas + mi] = pm;
    m.p0[s] = p0;
    double ss = mm ? -1.0 : 1.0;
    neg = (ss * sg) < 0;
    if (pivot < 0) { m.coef[2 * s] = mk<double>(0.5, 0); m.coef[2 * s + 1] = mk<double>(0.5 * ss * sg, 0); }
    else { m.coef[2 * s] = mk<double>(1, 0); m.coef[2 * s + 1] = mk<double>(ss * sg, 0); }
  }
  uint64_t bn = __ballot(neg), bm = __ballot(mm);
  if (threadIdx.x == 0) { negmask[blockIdx.x] = bn; mmask[blockIdx.x] = bm; }
}

// Blocks per shot: enough for about 8k blocks in flight over the batch, never
// more than the largest tile count.
inline int per_shot_blocks(long work_units, int S) {
  long want = (8192 + S - 1) / S;
  long b = work_units < want ? work_units : want;
  return (int)(b < 1 ? 1 : b);
}
inline dim3 gemm_grid(int maxM, int maxN, int S) {
  long tiles = (long)((maxM + GT - 1) / GT) * ((maxN + GT - 1) / GT);
  return dim3(per_shot_blocks(tiles, S), 1, S);
}
inline int ew_blocks(long maxe, int S) { return per_shot_blocks((maxe + TB - 1) / TB, S); }
inline int imin(int a, int b) { return a < b ? a : b; }
// largest possible bond at bond index b (between sites b-1 and b)
inline int dmax(const MpsDev &m, int b, int mult) {
  int e = b < m.n - b ? b : m.n - b;
  long phys = e >= 30 ? (1L << 30) : (1L << e);
  long cap = (long)m.chi * mult;
  return (int)(phys < cap ? phys : cap);
}

}  // namespace

// ===================================================================== host
template <typename T> void mps_init(const MpsDev &m, hipStream_t st) {
  KLAUNCH(K_BUILD, k_init<T>, dim3(m.S), dim3(TB), 0, st, m);
}

template <typename T> void mps_apply_single(const MpsDev &m, int site, const c64 *d_ops, hipStream_t st) {
  int maxe = dmax(m, site, 1) * dmax(m, site + 1, 1);
  KLAUNCH(K_BUILD, k_apply1<T>, dim3(ew_blocks(maxe, m.S), m.S), dim3(TB), 0, st, m, site, d_ops);
}

template <typename T> void mps_build(const MpsDev &m, int l, int r, const c64 *d_ops, hipStream_t st) {
  int maxe = 0;
  for (int j = l; j <= r; ++j) {
    int a = (j == l ? 1 : 2) * dmax(m, j, 1), c = (j == r ? 1 : 2) * dmax(m, j + 1, 1);
    maxe = std::max(maxe, a * c);
  }
  KLAUNCH(K_BUILD, k_build<T>, dim3(ew_blocks(maxe, m.S), r - l + 1, m.S), dim3(TB), 0, st, m, l, r, d_ops);
}

static size_t qr_lds(int rows) {
  return (size_t)rows * sizeof(c64) + (size_t)rows * 2 * sizeof(double) + TB * sizeof(c64) + kQrLdsMat;
}

template <typename T> void mps_sweep_lr(const MpsDev &m, int l, int r, hipStream_t st) {
  const int wm = m.wmul;                // largest multiple of a bond in the workspace
  for (int j = l; j < r; ++j) {
    int rows = 2 * (j == l ? dmax(m, j, 1) : wm * dmax(m, j, 1));
    int cols = wm * dmax(m, j + 1, 1);
    KLAUNCH(K_QR, k_qr_lr<T>, dim3(m.S), dim3(TB), qr_lds(rows), st, m, j, rows);
    int p = imin(rows, cols);
    int ncol = 2 * (j + 1 == r ? dmax(m, j + 2, 1) : wm * dmax(m, j + 2, 1));
    KLAUNCH(K_GEMM, k_absorb_lr<T>, gemm_grid(p, ncol, m.S), dim3(TB), 0, st, m, j);
  }
}

static size_t eig_lds() {
  const size_t f64 = 2 * (size_t)kJacLdsN * (kJacLdsN + 1) * sizeof(c64) + (size_t)kEigIdx * 2 * sizeof(int) +
                     (size_t)kEigIdx / 2 * (2 * sizeof(double) + sizeof(c64));
  const size_t f32 = (size_t)kEigIdx * (sizeof(double) + 2 * sizeof(int)) + (size_t)kEigLdsN * (kEigLdsN + 1) * sizeof(c64);
  return f64 > f32 ? f64 : f32;
}

template <typename T> void mps_sweep_rl(const MpsDev &m, int l, int r, hipStream_t st) {
  const int wm = m.wmul;
  for (int j = r; j > l; --j) {
    int L = wm * dmax(m, j, 1);
    int nn = 2 * dmax(m, j + 1, 1);
    KLAUNCH(K_GRAM, k_gram<T>, gemm_grid(nn, nn, m.S), dim3(TB), 0, st, m, j);
    KLAUNCH(K_EIGEN, k_eig<T>, dim3(m.S), dim3(TB), eig_lds(), st, m, j);
    KLAUNCH(K_SELECT, k_select<T>, dim3(m.S), dim3(TB), 0, st, m, j);
    int kmax = dmax(m, j, 1);
    KLAUNCH(K_GEMM, k_ngemm<T>, gemm_grid(L, kmax, m.S), dim3(TB), 0, st, m, j);
    int M = 2 * (j - 1 == l ? dmax(m, j - 1, 1) : wm * dmax(m, j - 1, 1));
    KLAUNCH(K_GEMM, k_xgemm<T>, gemm_grid(M, kmax, m.S), dim3(TB), 0, st, m, j);
  }
  KLAUNCH(K_SELECT, k_finish<T>, dim3(m.S), dim3(TB), 0, st, m, l);
}

template <typename T> void mps_move_right(const MpsDev &m, int c, hipStream_t st) {
  int rows = 2 * dmax(m, c, 1), cols = dmax(m, c + 1, 1);
  int maxe = rows * cols;
  KLAUNCH(K_BUILD, k_copy_to_T<T>, dim3(ew_blocks(maxe, m.S), m.S), dim3(TB), 0, st, m, c, 0);
  KLAUNCH(K_QR, k_qr_move_r<T>, dim3(m.S), dim3(TB), qr_lds(rows), st, m, c, rows);
  int p = imin(rows, cols), N = 2 * dmax(m, c + 2, 1);
  KLAUNCH(K_GEMM, k_absorb_move_r<T>, gemm_grid(p, N, m.S), dim3(TB), 0, st, m, c);
  KLAUNCH(K_BUILD, k_set_bond, dim3((m.S + 63) / 64), dim3(64), 0, st, m, c + 1);
  int maxe2 = p * N;
  KLAUNCH(K_BUILD, k_copy_from_T<T>, dim3(ew_blocks(maxe2, m.S), m.S), dim3(TB), 0, st, m, c + 1);
}

template <typename T> void mps_move_left(const MpsDev &m, int c, hipStream_t st) {
  int rows = 2 * dmax(m, c + 1, 1), cols = dmax(m, c, 1);
  int maxe = rows * cols;
  KLAUNCH(K_BUILD, k_copy_to_T<T>, dim3(ew_blocks(maxe, m.S), m.S), dim3(TB), 0, st, m, c, 1);
  KLAUNCH(K_QR, k_qr_move_l<T>, dim3(m.S), dim3(TB), qr_lds(rows), st, m, c, rows);
  int p = imin(rows, cols), M = 2 * dmax(m, c - 1, 1);
  KLAUNCH(K_GEMM, k_absorb_move_l<T>, gemm_grid(M, p, m.S), dim3(TB), 0, st, m, c);
  KLAUNCH(K_BUILD, k_set_bond, dim3((m.S + 63) / 64), dim3(64), 0, st, m, c);
  int maxe2 = M * p;
  KLAUNCH(K_BUILD, k_copy_from_T<T>, dim3(ew_blocks(maxe2, m.S), m.S), dim3(TB), 0, st, m, c - 1);
}

template <typename T> void mps_normalize_site(const MpsDev &m, int site, hipStream_t st) {
  KLAUNCH(K_SELECT, k_normalize<T>, dim3(m.S), dim3(TB), 0, st, m, site);
}

// Expectation of prod_j eops_j over [l, r] (centre at l) and the centre norm.
template <typename T> void mps_expect(const MpsDev &m, int l, int r, const c64 *d_eops, hipStream_t st) {
  KLAUNCH(K_EXPECT, k_sitenorm<T>, dim3(m.S), dim3(TB), 0, st, m, l);
  KLAUNCH(K_EXPECT, k_eye<T>, dim3(m.S), dim3(TB), 0, st, m, l);
  for (int j = l; j <= r; ++j) {
    int dl = dmax(m, j, 1), dr = dmax(m, j + 1, 1);
    KLAUNCH(K_EXPECT, k_expect_f<T>, gemm_grid(dl, 2 * dr, m.S), dim3(TB), 0, st, m, j, d_eops);
    KLAUNCH(K_EXPECT, k_expect_op<T>, dim3(ew_blocks((long)dl * dr, m.S), m.S), dim3(TB), 0, st, m, j,
                       d_eops + (size_t)(j - l) * 4);
    KLAUNCH(K_EXPECT, k_expect_e<T>, gemm_grid(dr, dr, m.S), dim3(TB), 0, st, m, j);
  }
}

void launch_ops_rotation(const uint64_t *d_bits, int W, int l, int r, c64 *d_ops, hipStream_t st) {
  int cnt = r - l + 1;
  KLAUNCH(K_BUILD, k_ops_rotation, dim3((cnt + 63) / 64), dim3(64), 0, st, d_bits, W, l, r, d_ops);
}

void launch_ops_measure(const uint64_t *d_bits, int W, int l, int r, int pivot, c64 *d_ops,
                        c64 *d_eops, hipStream_t st) {
  int cnt = r - l + 1;
  KLAUNCH(K_BUILD, k_ops_measure, dim3((cnt + 63) / 64), dim3(64), 0, st, d_bits, W, l, r, pivot,
                     d_ops, d_eops);
}

void launch_coef_rotation(const uint64_t *d_psgn, int S, const double *d_theta, int64_t stride,
                          int r_index, c64 *d_coef, int *d_err, hipStream_t st) {
  KLAUNCH(K_BUILD, k_coef_rotation, dim3((S + 255) / 256), dim3(256), 0, st, d_psgn, S, d_theta,
                     stride, r_index, d_coef, d_err);
}

void launch_outcome(const MpsDev &m, const uint64_t *d_snap_sign, int pivot, int dr_site,
                    const double *d_u, const uint8_t *d_forced, int n_meas, int mi, uint8_t *d_out,
                    double *d_prob, uint64_t *d_negmask, uint64_t *d_mmask, hipStream_t st) {
  KLAUNCH(K_EXPECT, k_outcome, dim3((m.S + 63) / 64), dim3(64), 0, st, m, d_snap_sign, pivot, dr_site,
                     d_u, d_forced, n_meas, mi, d_out, d_prob, d_negmask, d_mmask);
}

template <typename T> void mps_spectrum(const MpsDev &m, int b, double *d_out, int ld, int *d_rank, hipStream_t st) {
  KLAUNCH(K_EXPECT, k_spectrum<T>, dim3(m.S), dim3(TB), eig_lds(), st, m, b, d_out, ld, d_rank);
}

// Raise the dynamic-LDS limit of the kernels that stage matrices in LDS
// (gfx950 has 160 KB per CU).  Returns the first HIP error, if any.
template <typename T> hipError_t mps_prepare(int max_rows) {
  hipError_t e = hipFuncSetAttribute((const void *)k_eig<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)eig_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_spectrum<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)eig_lds());
  const int q = (int)qr_lds(max_rows);
  for (const void *f : {(const void *)k_qr_lr<T>, (const void *)k_qr_move_r<T>, (const void *)k_qr_move_l<T>}) {
    hipError_t e2 = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, q);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

#define INST(T)                                                                        \
  template hipError_t mps_prepare<T>(int);                                            \
  template void mps_init<T>(const MpsDev &, hipStream_t);                             \
  template void mps_apply_single<T>(const MpsDev &, int, const c64 *, hipStream_t);   \
  template void mps_build<T>(const MpsDev &, int, int, const c64 *, hipStream_t);     \
  template void mps_sweep_lr<T>(const MpsDev &, int, int, hipStream_t);               \
  template void mps_sweep_rl<T>(const MpsDev &, int, int, hipStream_t);               \
  template void mps_move_right<T>(const MpsDev &, int, hipStream_t);                  \
  template void mps_move_left<T>(const MpsDev &, int, hipStream_t);                   \
  template void mps_normalize_site<T>(const MpsDev &, int, hipStream_t);              \
  template void mps_expect<T>(const MpsDev &, int, int, const c64 *, hipStream_t);           \
  template void mps_spectrum<T>(const MpsDev &, int, double *, int, int *, hipStream_t);
INST(float)
INST(double)
