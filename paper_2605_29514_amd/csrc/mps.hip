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

namespace {

constexpr int TB = 256;          // threads per block
constexpr int GT = 32;           // GEMM tile (GT x GT outputs)
constexpr int GK = 16;           // GEMM k-step
constexpr int kEigLdsN = 32;     // Jacobi in LDS up to this order (2 x 16 KB)

template <typename T>
struct Acc { using type = T; };

// ------------------------------------------------------------------ GEMM
// One GT x GT tile of C = alpha * op(A) op(B) (+ C if accumulate).
//   opA = 0: A is M x K (lda);  opA = 1: A is K x M and op(A) = A^H.
//   opB = 0: B is K x N (ldb);  opB = 1: B is N x K and op(B) = B^H.
template <typename TA, typename TB_, typename TC, typename ACC>
__device__ void gemm_tile(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                          const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc, int tm,
                          int tn) {
  __shared__ cplx<ACC> As[GT][GK + 1];
  __shared__ cplx<ACC> Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int row0 = tm * GT, col0 = tn * GT;
  cplx<ACC> acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = mk<ACC>(0, 0);
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GT * GK; e += TB) {
      int mi = e / GK, ki = e % GK;
      int m = row0 + mi, k = k0 + ki;
      cplx<ACC> v = mk<ACC>(0, 0);
      if (m < M && k < K) v = opA ? cj(cvt<ACC>(A[(size_t)k * lda + m])) : cvt<ACC>(A[(size_t)m * lda + k]);
      As[mi][ki] = v;
    }
    for (int e = tid; e < GT * GK; e += TB) {
      int ki = e / GT, ni = e % GT;
      int n = col0 + ni, k = k0 + ki;
      cplx<ACC> v = mk<ACC>(0, 0);
      if (n < N && k < K) v = opB ? cj(cvt<ACC>(B[(size_t)n * ldb + k])) : cvt<ACC>(B[(size_t)k * ldb + n]);
      Bs[ki][ni] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < GK; ++kk) {
      cplx<ACC> a0 = As[ty][kk], a1 = As[ty + 16][kk];
      cplx<ACC> b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      acc[0][0] = acc[0][0] + a0 * b0;
      acc[0][1] = acc[0][1] + a0 * b1;
      acc[1][0] = acc[1][0] + a1 * b0;
      acc[1][1] = acc[1][1] + a1 * b1;
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      int m = row0 + ty + 16 * i, n = col0 + tx + 16 * j;
      if (m < M && n < N) C[(size_t)m * ldc + n] = cvt<TC>(acc[i][j]);
    }
}

// All tiles of one shot's product, strided over the blocks given to it:
// grids are sized from a per-shot block budget, not from the largest
// possible bonds, so early (small-bond) steps do not launch empty tiles.
template <typename TA, typename TB_, typename TC, typename ACC>
__device__ void gemm_all(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                         const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc) {
  const int ntm = (M + GT - 1) / GT, ntn = (N + GT - 1) / GT;
  for (int t = blockIdx.x; t < ntm * ntn; t += gridDim.x)
    gemm_tile<TA, TB_, TC, ACC>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, t / ntn, t % ntn);
}

template <typename T>
__device__ inline cplx<T> *slot(const MpsDev &m, int j, int s) {
  return reinterpret_cast<cplx<T> *>(m.mps) + m.site_off[j] + (int64_t)s * m.site_cap[j];
}
template <typename T>
__device__ inline cplx<T> *wslot(const MpsDev &m, int j, int s) {
  return reinterpret_cast<cplx<T> *>(m.ws) + m.ws_off[j] + (int64_t)s * m.ws_cap[j];
}
template <typename T>
__device__ inline cplx<T> *scr(void *base, int64_t cap, int s) {
  return reinterpret_cast<cplx<T> *>(base) + (int64_t)s * cap;
}
__device__ inline int *bnd(const MpsDev &m, int s) { return m.bond + (size_t)s * (m.n + 1); }
__device__ inline int *wbd(const MpsDev &m, int s) { return m.wb + (size_t)s * (m.n + 1); }
__device__ inline int *auxp(const MpsDev &m, int s) { return m.aux + (size_t)s * 8; }

// Algorithmic work of one launch for one shot, added by a single thread.
__device__ inline void add_work(const MpsDev &m, int cls, double flops, double bytes) {
  if (m.prof) {
    atomicAdd(&m.work[2 * cls], flops);
    atomicAdd(&m.work[2 * cls + 1], bytes);
  }
}
__device__ inline bool first_block() { return blockIdx.x == 0 && threadIdx.x == 0; }
__device__ inline double gemm_flops(double M, double N, double K) { return 8.0 * M * N * K; }
// Householder QR of an m x n complex matrix with p = min(m, n) reflectors,
// R plus the explicit m x p Q: 4x the real counts 2mnp - (m+n)p^2 + 2p^3/3
// for R and 2mp^2 - (m+p)p^2 + 2p^3/3 for Q, times two for multiply-add.
__device__ inline double qr_flops(double m, double n) {
  double p = m < n ? m : n;
  double r = 2 * m * n * p - (m + n) * p * p + 2.0 / 3.0 * p * p * p;
  double q = 2 * m * p * p - (m + p) * p * p + 2.0 / 3.0 * p * p * p;
  return 8.0 * (r + q);
}

// ------------------------------------------------------------ block reduce
template <typename T>
__device__ T block_sum(T v) {
  __shared__ T red[TB / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T tot = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += red[i];
  __syncthreads();
  return tot;
}

__device__ double block_max(double v) {
  __shared__ double red[TB / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double tot = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot = fmax(tot, red[i]);
  __syncthreads();
  return tot;
}

// ----------------------------------------------------- Householder QR
// In place on A (m x nc, ld = nc).  p = min(m, nc).  Writes R (p x nc,
// ld = nc, zero below the diagonal) to Rd and the explicit Q (m x p) to Qd,
// either as an m x p matrix (ld = p) or conjugate-transposed as a p x m
// matrix (qt = 1).  One block per matrix.
template <typename T>
__device__ void qr_block(int m, int nc, cplx<T> *A, cplx<T> *Qd, int qt, cplx<T> *Rd, c64 *vs,
                         double *vd) {
  using C = cplx<T>;
  const int p = m < nc ? m : nc;
  const int tid = threadIdx.x;
  for (int k = 0; k < p; ++k) {
    // Norms and the phase of x0 are formed from double copies: squaring a
    // float below ~1e-19 lands in the denormal range, and an inexact |x0|
    // would leave x0/|x0| off the unit circle, so H = I - 2 v v^H would stop
    // being unitary.
    double part = 0;
    for (int i = k + tid; i < m; i += TB) part += norm2(cvt<double>(A[(size_t)i * nc + k]));
    double xn2 = block_sum(part);
    C x0 = A[(size_t)k * nc + k];
    double ax0 = hypot((double)x0.x, (double)x0.y);
    double xn = sqrt(xn2);
    c64 ph = ax0 > 0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1, 0);
    c64 alpha = mk<double>(-ph.x * xn, -ph.y * xn);
    // v = x - alpha e1, |v|^2 = |x|^2 - |x0|^2 + |x0 - alpha|^2 = 2 |x| (|x| + |x0|)
    double vn2 = 2.0 * xn * (xn + ax0);
    double inv = vn2 > 0 ? 1.0 / sqrt(vn2) : 0.0;
    for (int i = k + tid; i < m; i += TB) {
      c64 xi = cvt<double>(A[(size_t)i * nc + k]);
      if (i == k) xi = xi - alpha;
      vs[i] = inv * xi;
    }
    __syncthreads();
    if (inv > 0) {
      for (int j = k + 1 + tid; j < nc; j += TB) {
        c64 w = mk<double>(0, 0);
        for (int i = k; i < m; ++i) w = w + cj(vs[i]) * cvt<double>(A[(size_t)i * nc + j]);
        w = 2.0 * w;
        for (int i = k; i < m; ++i) {
          c64 a = cvt<double>(A[(size_t)i * nc + j]) - vs[i] * w;
          A[(size_t)i * nc + j] = cvt<T>(a);
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      vd[2 * k] = vs[k].x;
      vd[2 * k + 1] = vs[k].y;
      A[(size_t)k * nc + k] = cvt<T>(inv > 0 ? alpha : cvt<double>(x0));
    }
    for (int i = k + 1 + tid; i < m; i += TB) A[(size_t)i * nc + k] = cvt<T>(vs[i]);
    __syncthreads();
  }
  // R
  for (int e = tid; e < p * nc; e += TB) {
    int i = e / nc, j = e % nc;
    Rd[e] = j >= i ? A[(size_t)i * nc + j] : mk<T>(0, 0);
  }
  __syncthreads();
  // Q = H_0 ... H_{p-1} [I; 0], accumulated backwards in A's first p columns
  for (int k = p - 1; k >= 0; --k) {
    for (int i = k + tid; i < m; i += TB) {
      vs[i] = i == k ? mk<double>(vd[2 * k], vd[2 * k + 1]) : cvt<double>(A[(size_t)i * nc + k]);
    }
    __syncthreads();
    for (int i = k + tid; i < m; i += TB) A[(size_t)i * nc + k] = mk<T>(i == k ? 1 : 0, 0);
    for (int j = k + 1 + tid; j < p; j += TB) A[(size_t)k * nc + j] = mk<T>(0, 0);
    __syncthreads();
    for (int j = k + tid; j < p; j += TB) {
      c64 w = mk<double>(0, 0);
      for (int i = k; i < m; ++i) w = w + cj(vs[i]) * cvt<double>(A[(size_t)i * nc + j]);
      w = 2.0 * w;
      for (int i = k; i < m; ++i) {
        c64 a = cvt<double>(A[(size_t)i * nc + j]) - vs[i] * w;
        A[(size_t)i * nc + j] = cvt<T>(a);
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < m * p; e += TB) {
    int i = e / p, j = e % p;
    C q = A[(size_t)i * nc + j];
    if (qt)
      Qd[(size_t)j * m + i] = cj(q);
    else
      Qd[e] = q;
  }
  __syncthreads();
}

// QR of the m x nc matrix at A (global).  When it fits, the matrix is first
// copied to LDS (after the reflector scratch) so the column sweeps run at
// LDS rather than L2 bandwidth.  lds_rows: rows the scratch was sized for.
constexpr size_t kQrLdsMat = 16 * 1024;
template <typename T>
__device__ void qr_dispatch(int rows, int cols, cplx<T> *A, cplx<T> *Qd, int qt, cplx<T> *Rd,
                            char *lds, int lds_rows) {
  c64 *vs = reinterpret_cast<c64 *>(lds);
  double *vd = reinterpret_cast<double *>(vs + lds_rows);
  cplx<T> *Al = reinterpret_cast<cplx<T> *>(vd + 2 * lds_rows);
  if ((size_t)rows * cols * sizeof(cplx<T>) <= kQrLdsMat) {
    for (int e = threadIdx.x; e < rows * cols; e += TB) Al[e] = A[e];
    __syncthreads();
    qr_block<T>(rows, cols, Al, Qd, qt, Rd, vs, vd);
  } else {
    qr_block<T>(rows, cols, A, Qd, qt, Rd, vs, vd);
  }
}

// ------------------------------------------------ Jacobi eigen-solve (FP64)
// Hermitian nn x nn matrix G (ld nn) -> eigenvalues ev (descending) and the
// matching eigenvectors as columns of Vout (ld nn).  Parallel cyclic Jacobi:
// each round rotates nn/2 disjoint index pairs (round-robin ordering); the
// 2x2 block [[a, c], [c*, b]] is diagonalised by U = diag(1, e^{-i phi}) R
// with c = |c| e^{i phi} and R the real symmetric Jacobi rotation.
__device__ void jacobi_block(int nn, c64 *G, c64 *V, double *ev, c64 *Vout, int *err,
                             int *pos, double *pc, double *ps, c64 *pe, int *pp, int *pq,
                             int *sweeps_out, double abs_tol, double rel_tol) {
  const int tid = threadIdx.x;
  const int P = nn + (nn & 1);
  if (sweeps_out && tid == 0) *sweeps_out = 0;
  for (int e = tid; e < nn * nn; e += TB) V[e] = mk<double>((e / nn) == (e % nn) ? 1.0 : 0.0, 0);
  for (int i = tid; i < P; i += TB) pos[i] = i;
  __syncthreads();
  // The Gram matrix is positive semi-definite, so its trace bounds every
  // eigenvalue and is invariant under the rotations.  An entry G_pq is
  // negligible when |G_pq| <= max(abs_tol tr, rel_tol sqrt(G_pp G_qq)): the
  // relative part keeps small kept eigenvalues from mixing with the (near)
  // null space, the absolute floor stops at the rounding level of the Gram.
  double trp = 0;
  for (int i = tid; i < nn; i += TB) trp += G[(size_t)i * nn + i].x;
  const double tr = block_sum(trp);
  const double afl = abs_tol * tr;
  const int max_sweeps = 60;
  bool converged = nn <= 1 || !(tr > 0);
  int sweeps_done = 0;
  double last_off = 0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    for (int rnd = 0; rnd < P - 1; ++rnd) {
      for (int i = tid; i < P / 2; i += TB) {
        int p = pos[i], q = pos[P - 1 - i];
        if (p > q) { int t = p; p = q; q = t; }
        double cs = 1, sn = 0;
        c64 eph = mk<double>(1, 0);
        if (q < nn) {
          c64 c = G[(size_t)p * nn + q];
          double h = sqrt(norm2(c));
          double a = G[(size_t)p * nn + p].x, b = G[(size_t)q * nn + q].x;
          if (h > afl && h > rel_tol * sqrt(fabs(a * b))) {
            eph = mk<double>(c.x / h, c.y / h);
            double tau = (b - a) / (2 * h);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
            cs = 1 / sqrt(1 + t * t);
            sn = t * cs;
          }
        }
        pp[i] = p; pq[i] = q; pc[i] = cs; ps[i] = sn; pe[i] = eph;
      }
      __syncthreads();
      // rows p, q <- U^H rows
      for (int e = tid; e < (P / 2) * nn; e += TB) {
        int i = e / nn, col = e % nn;
        int p = pp[i], q = pq[i];
        if (q >= nn || ps[i] == 0) continue;
        c64 gp = G[(size_t)p * nn + col], gq = G[(size_t)q * nn + col];
        double cs = pc[i], sn = ps[i];
        c64 eq = pe[i] * gq;
        G[(size_t)p * nn + col] = cs * gp - sn * eq;
        G[(size_t)q * nn + col] = sn * gp + cs * eq;
      }
      __syncthreads();
      // columns p, q <- cols U (and the same for V)
      for (int e = tid; e < (P / 2) * nn; e += TB) {
        int i = e / nn, row = e % nn;
        int p = pp[i], q = pq[i];
        if (q >= nn || ps[i] == 0) continue;
        double cs = pc[i], sn = ps[i];
        c64 ec = cj(pe[i]);
        c64 gp = G[(size_t)row * nn + p], gq = ec * G[(size_t)row * nn + q];
        G[(size_t)row * nn + p] = cs * gp - sn * gq;
        G[(size_t)row * nn + q] = sn * gp + cs * gq;
        c64 vp = V[(size_t)row * nn + p], vq = ec * V[(size_t)row * nn + q];
        V[(size_t)row * nn + p] = cs * vp - sn * vq;
        V[(size_t)row * nn + q] = sn * vp + cs * vq;
      }
      __syncthreads();
      // next round-robin arrangement: fix pos[0], rotate the rest
      if (tid == 0) {
        int last = pos[P - 1];
        for (int i = P - 1; i > 1; --i) pos[i] = pos[i - 1];
        pos[1] = last;
      }
      __syncthreads();
    }
    double off = 0, viol = 0;
    for (int e = tid; e < nn * nn; e += TB) {
      const int p = e / nn, q = e % nn;
      if (p == q) continue;
      const double h = sqrt(norm2(G[e]));
      off = fmax(off, h);
      if (h > afl && h > rel_tol * sqrt(fabs(G[(size_t)p * nn + p].x * G[(size_t)q * nn + q].x))) viol = 1;
    }
    off = block_max(off);
    viol = block_max(viol);
    last_off = off;
    converged = viol == 0;
    sweeps_done = sweep + 1;
  }
  if (sweeps_out && tid == 0) *sweeps_out = sweeps_done;
  if (!converged && tid == 0 && last_off > 1e-10 * tr) atomicOr(err, STN_ERR_EIGEN);
  // sort descending: rank of each eigenvalue (ties by index)
  for (int i = tid; i < nn; i += TB) {
    double li = G[(size_t)i * nn + i].x;
    int rank = 0;
    for (int j = 0; j < nn; ++j) {
      double lj = G[(size_t)j * nn + j].x;
      rank += (lj > li) || (lj == li && j < i);
    }
    ev[rank] = li;
    pos[i] = rank;
  }
  __syncthreads();
  for (int e = tid; e < nn * nn; e += TB) {
    int row = e / nn, col = e % nn;
    Vout[(size_t)row * nn + pos[col]] = V[e];
  }
  __syncthreads();
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

template <typename T>
__global__ void k_eig(MpsDev m, int j) {
  extern __shared__ char lds[];
  const int s = blockIdx.x;
  const int nn = 2 * wbd(m, s)[j + 1];
  c64 *Gl = reinterpret_cast<c64 *>(lds);                 // used when nn <= kEigLdsN
  c64 *Vl = Gl + kEigLdsN * kEigLdsN;
  int *pos = reinterpret_cast<int *>(Vl + kEigLdsN * kEigLdsN);
  int *pp = pos + 1040, *pq = pp + 520;
  double *pc = reinterpret_cast<double *>(pq + 520);
  double *ps = pc + 520;
  c64 *pe = reinterpret_cast<c64 *>(ps + 520);
  c64 *Gg = m.G + s * m.G_cap;
  c64 *Gw = Gg, *Vw = m.V + s * m.V_cap;
  if (nn <= kEigLdsN) {       // small matrices: rotate in LDS, write the sorted vectors back
    for (int e = threadIdx.x; e < nn * nn; e += TB) Gl[e] = Gg[e];
    __syncthreads();
    Gw = Gl;
    Vw = Vl;
  }
  // eigenvectors are accumulated in V and written sorted into G (global)
  __shared__ int sweeps;
  jacobi_block(nn, Gw, Vw, m.ev + s * m.ev_cap, Gg,
               m.err, pos, pc, ps, pe, pp, pq, &sweeps,
               sizeof(T) == 8 ? 1e-18 : 1e-16, sizeof(T) == 8 ? 1e-15 : 1e-13);
  // algorithmic work: a Hermitian eigendecomposition with vectors, ~9 n^3 real
  // flops (x4 complex); bytes: read G, write eigenvalues and vectors.
  if (threadIdx.x == 0) add_work(m, K_EIGEN, 36.0 * nn * nn * (double)nn, 16.0 * 2 * nn * nn + 8.0 * nn);
  if (threadIdx.x == 0 && m.prof) atomicAdd(&m.work[2 * K_COUNT], (double)sweeps);
}

// Truncation: keep k' = min(chi_max, #{lambda_i > eps sum lambda}) largest
// (at least 1); discarded weight w updates the fidelity; Vt = V[:, :k'] in T;
// site j <- Vt^H as (k', 2, wb[j+1]); bond[j] = k', bond[j+1] = wb[j+1].
template <typename T>
__device__ int select_body(const MpsDev &m, int s, int j) {
  int *w = wbd(m, s);
  const int nn = 2 * w[j + 1];
  const double *ev = m.ev + s * m.ev_cap;
  __shared__ int kk;
  double part = 0;
  for (int i = threadIdx.x; i < nn; i += TB) part += fmax(ev[i], 0.0);
  double tot = block_sum(part);
  int cnt = 0;
  for (int i = threadIdx.x; i < nn; i += TB) cnt += ev[i] > m.eps_cut * tot;
  cnt = block_sum(cnt);
  if (threadIdx.x == 0) {
    int k = cnt < m.chi ? cnt : m.chi;
    const int e = j < m.n - j ? j : m.n - j;           // physical bound 2^min(j, n-j)
    if (e < 30 && k > (1 << e)) k = 1 << e;
    if (k < 1) k = 1;
    double disc = 0;
    for (int i = k; i < nn; ++i) disc += fmax(ev[i], 0.0);
    double wgt = tot > 0 ? disc / tot : 0.0;
    m.fid[s] *= (1.0 - wgt);
    if (!(tot == tot) || isinf(tot)) atomicOr(m.err, STN_ERR_NUMERIC);
    kk = k;
    auxp(m, s)[2] = k;
    auxp(m, s)[3] = w[j];          // L, read by the Q N product while wb[j] changes
  }
  __syncthreads();
  const int k = kk;
  const c64 *V = m.G + s * m.G_cap;
  cplx<T> *Vt = scr<T>(m.Vt, m.Vt_cap, s);
  cplx<T> *site = slot<T>(m, j, s);
  for (int e = threadIdx.x; e < nn * k; e += TB) {
    int i = e / k, c = e % k;
    cplx<T> v = cvt<T>(V[(size_t)i * nn + c]);
    Vt[e] = v;
    site[(size_t)c * nn + i] = cj(v);
  }
  if (threadIdx.x == 0) {
    bnd(m, s)[j] = k;
    bnd(m, s)[j + 1] = w[j + 1];
  }
  __syncthreads();
  return k;
}

template <typename T>
__global__ void k_select(MpsDev m, int j) { select_body<T>(m, blockIdx.x, j); }

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

// Centre at l: normalise scratch T (wb[l], 2, wb[l+1]) in FP64 and store it
// in slot l; bond[l+1] = wb[l+1].
template <typename T>
__device__ void finish_body(const MpsDev &m, int s, int l) {
  int *w = wbd(m, s);
  const int cnt = w[l] * 2 * w[l + 1];
  const cplx<T> *X = scr<T>(m.T, m.T_cap, s);
  double part = 0;
  for (int e = threadIdx.x; e < cnt; e += TB) part += norm2(cvt<double>(X[e]));
  double n2 = block_sum(part);
  if (!(n2 > 0) || isinf(n2)) {
    if (threadIdx.x == 0) atomicOr(m.err, STN_ERR_NUMERIC);
    return;
  }
  double inv = 1.0 / sqrt(n2);
  cplx<T> *out = slot<T>(m, l, s);
  for (int e = threadIdx.x; e < cnt; e += TB) out[e] = cvt<T>(inv * cvt<double>(X[e]));
  if (threadIdx.x == 0) {
    bnd(m, s)[l + 1] = w[l + 1];
    m.nrm[s] = n2;
  }
  __syncthreads();
}

template <typename T>
__global__ void k_finish(MpsDev m, int l) { finish_body<T>(m, blockIdx.x, l); }

// In-place FP64 normalisation of one site (the centre).
template <typename T>
__global__ void k_normalize(MpsDev m, int site) {
  const int s = blockIdx.x;
  const int cnt = bnd(m, s)[site] * 2 * bnd(m, s)[site + 1];
  cplx<T> *A = slot<T>(m, site, s);
  double part = 0;
  for (int e = threadIdx.x; e < cnt; e += TB) part += norm2(cvt<double>(A[e]));
  double n2 = block_sum(part);
  if (!(n2 > 0) || isinf(n2)) {
    if (threadIdx.x == 0) atomicOr(m.err, STN_ERR_NUMERIC);
    return;
  }
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
  double n2 = block_sum(part);
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
__device__ inline void site_op(int x, int z, c64 *o) {
  // i^(xz) X^x Z^z
  if (!x && !z) { o[0] = mk<double>(1, 0); o[1] = mk<double>(0, 0); o[2] = mk<double>(0, 0); o[3] = mk<double>(1, 0); }
  if (!x && z) { o[0] = mk<double>(1, 0); o[1] = mk<double>(0, 0); o[2] = mk<double>(0, 0); o[3] = mk<double>(-1, 0); }
  if (x && !z) { o[0] = mk<double>(0, 0); o[1] = mk<double>(1, 0); o[2] = mk<double>(1, 0); o[3] = mk<double>(0, 0); }
  if (x && z) { o[0] = mk<double>(0, 0); o[1] = mk<double>(0, -1); o[2] = mk<double>(0, 1); o[3] = mk<double>(0, 0); }
}
__device__ inline int bitw(const uint64_t *v, int j) { return (int)((v[j >> 6] >> (j & 63)) & 1ull); }

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

// ============================================================ fused layer
// Shots are independent, so one block per shot can run a whole chunk of
// rotations of a layer (centre moves, bond-2 blocks, QR sweep, Gram/eigen
// truncation, renormalisation) with block barriers only: one launch per
// chunk instead of ~10 launches per site, and every shot proceeds at its own
// bond dimensions.  Same arithmetic as the per-step kernels.

// All tiles of a product by the calling block.
template <typename TA, typename TB_, typename TC, typename ACC>
__device__ void blk_gemm(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                         const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc) {
  const int ntm = (M + GT - 1) / GT, ntn = (N + GT - 1) / GT;
  for (int t = 0; t < ntm * ntn; ++t)
    gemm_tile<TA, TB_, TC, ACC>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, t / ntn, t % ntn);
  __syncthreads();
}

template <typename T>
__device__ void blk_copy(cplx<T> *dst, const cplx<T> *src, int cnt) {
  for (int e = threadIdx.x; e < cnt; e += TB) dst[e] = src[e];
  __syncthreads();
}

// Centre move c -> c+1 (QR of A_c, R into A_{c+1}).
template <typename T>
__device__ void blk_move_right(const MpsDev &m, int s, int c, char *lds, int lds_rows) {
  int *b = bnd(m, s);
  const int rows = 2 * b[c], cols = b[c + 1], N = 2 * b[c + 2];
  const int p = rows < cols ? rows : cols;
  cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
  blk_copy<T>(X, slot<T>(m, c, s), rows * cols);
  qr_dispatch<T>(rows, cols, X, slot<T>(m, c, s), 0, R, lds, lds_rows);
  blk_gemm<T, T, T, T>(p, N, cols, R, cols, 0, slot<T>(m, c + 1, s), N, 0, X, N);
  if (threadIdx.x == 0) {
    b[c + 1] = p;
    add_work(m, K_LAYER, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
    add_work(m, K_LAYER, gemm_flops(p, N, cols), (double)sizeof(cplx<T>) * ((double)p * cols + (double)cols * N + (double)p * N));
  }
  __syncthreads();
  blk_copy<T>(slot<T>(m, c + 1, s), X, p * N);
}

// Centre move c -> c-1 (LQ of A_c via the QR of A_c^H, L into A_{c-1}).
template <typename T>
__device__ void blk_move_left(const MpsDev &m, int s, int c, char *lds, int lds_rows) {
  int *b = bnd(m, s);
  const int dl = b[c], dr = b[c + 1], M = 2 * b[c - 1];
  const int rows = 2 * dr, cols = dl, p = rows < cols ? rows : cols;
  cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
  const cplx<T> *A = slot<T>(m, c, s);
  for (int e = threadIdx.x; e < dl * 2 * dr; e += TB) {
    int a = e / (2 * dr), cc = e % (2 * dr);
    X[(size_t)cc * dl + a] = cj(A[e]);
  }
  __syncthreads();
  qr_dispatch<T>(rows, cols, X, slot<T>(m, c, s), 1, R, lds, lds_rows);
  blk_gemm<T, T, T, T>(M, p, cols, slot<T>(m, c - 1, s), cols, 0, R, cols, 1, X, p);
  if (threadIdx.x == 0) {
    b[c] = p;
    add_work(m, K_LAYER, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
    add_work(m, K_LAYER, gemm_flops(M, p, cols), (double)sizeof(cplx<T>) * ((double)M * cols + (double)cols * p + (double)M * p));
  }
  __syncthreads();
  blk_copy<T>(slot<T>(m, c - 1, s), X, M * p);
}

__device__ inline void rot_site_ops(const uint64_t *bx, const uint64_t *bz, int j, c64 *o2) {
  site_op((int)((bx[j >> 6] >> (j & 63)) & 1ull), (int)((bz[j >> 6] >> (j & 63)) & 1ull), o2);
}

template <typename T>
__global__ void __launch_bounds__(TB) k_rot_layer(MpsDev m, const uint64_t *pbits, const uint64_t *psgn,
                                                  int W, int SW, const double *theta, int64_t stride,
                                                  RotLayer L, int lds_rows) {
  extern __shared__ char lds[];
  const int s = blockIdx.x, tid = threadIdx.x;
  int *b = bnd(m, s), *w = wbd(m, s);
  __shared__ c64 cf[2];
  __shared__ int sweeps;
  int c = L.center_in;
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
    const c64 ca = cf[0], cb = cf[1];
    if (l == r) {                              // unitary on one site: no bond change
      c64 o2[4];
      rot_site_ops(bx, bz, l, o2);
      const int dl = b[l], dr = b[l + 1];
      cplx<T> *A = slot<T>(m, l, s);
      for (int e = tid; e < dl * dr; e += TB) {
        const int a = e / dr, cc = e % dr;
        c64 x0 = cvt<double>(A[(size_t)(a * 2 + 0) * dr + cc]), x1 = cvt<double>(A[(size_t)(a * 2 + 1) * dr + cc]);
        A[(size_t)(a * 2 + 0) * dr + cc] = cvt<T>(ca * x0 + cb * (o2[0] * x0 + o2[1] * x1));
        A[(size_t)(a * 2 + 1) * dr + cc] = cvt<T>(ca * x1 + cb * (o2[2] * x0 + o2[3] * x1));
      }
      __syncthreads();
      continue;
    }
    while (c < l) { blk_move_right<T>(m, s, c, lds, lds_rows); ++c; }
    while (c > r) { blk_move_left<T>(m, s, c, lds, lds_rows); --c; }
    // bond-2 blocks over [l, r]
    for (int j = l; j <= r; ++j) {
      const int dl = b[j], dr = b[j + 1];
      const int Dl = (j == l) ? dl : 2 * dl, Dr = (j == r) ? dr : 2 * dr;
      c64 o2[4];
      rot_site_ops(bx, bz, j, o2);
      cplx<T> *out = (j == l) ? scr<T>(m.T, m.T_cap, s) : wslot<T>(m, j, s);
      const cplx<T> *A = slot<T>(m, j, s);
      for (int e = tid; e < Dl * Dr; e += TB) {
        const int a = e / Dr, cc = e % Dr;
        const int ba = a >= dl, bc = cc >= dr;
        int br = -1;
        if (j == l) br = bc;
        else if (j == r) br = ba;
        else if (ba == bc) br = ba;
        c64 y0 = mk<double>(0, 0), y1 = mk<double>(0, 0);
        if (br >= 0) {
          const int aa = (j == l) ? a : a - (ba ? dl : 0);
          const int c2 = (j == r) ? cc : cc - (bc ? dr : 0);
          c64 x0 = cvt<double>(A[(size_t)(aa * 2 + 0) * dr + c2]), x1 = cvt<double>(A[(size_t)(aa * 2 + 1) * dr + c2]);
          if (br) { y0 = o2[0] * x0 + o2[1] * x1; y1 = o2[2] * x0 + o2[3] * x1; }
          else { y0 = x0; y1 = x1; }
          if (j == l) { const c64 k = br ? cb : ca; y0 = k * y0; y1 = k * y1; }
        }
        out[(size_t)(a * 2 + 0) * Dr + cc] = cvt<T>(y0);
        out[(size_t)(a * 2 + 1) * Dr + cc] = cvt<T>(y1);
      }
      if (tid == 0) { w[j] = Dl; if (j == r) w[r + 1] = dr; }
    }
    __syncthreads();
    // left-to-right QR sweep
    for (int j = l; j < r; ++j) {
      const int rows = 2 * w[j], cols = w[j + 1], N = 2 * w[j + 2];
      const int p = rows < cols ? rows : cols;
      cplx<T> *X = scr<T>(m.T, m.T_cap, s), *R = scr<T>(m.R, m.R_cap, s);
      qr_dispatch<T>(rows, cols, X, wslot<T>(m, j, s), 0, R, lds, lds_rows);
      blk_gemm<T, T, T, T>(p, N, cols, R, cols, 0, wslot<T>(m, j + 1, s), N, 0, X, N);
      if (tid == 0) {
        w[j + 1] = p;
        add_work(m, K_LAYER, qr_flops(rows, cols), (double)sizeof(cplx<T>) * (2.0 * rows * cols + (double)rows * p + (double)p * cols));
        add_work(m, K_LAYER, gemm_flops(p, N, cols), (double)sizeof(cplx<T>) * ((double)p * cols + (double)cols * N + (double)p * N));
      }
      __syncthreads();
    }
    // right-to-left truncation sweep
    for (int j = r; j > l; --j) {
      const int Lx = w[j], nn = 2 * w[j + 1];
      cplx<T> *X = scr<T>(m.T, m.T_cap, s);
      c64 *Gg = m.G + s * m.G_cap;
      blk_gemm<T, T, double, double>(nn, nn, Lx, X, nn, 1, X, nn, 0, Gg, nn);
      // eigen-solve (LDS when small); dynamic LDS is shared with the QR scratch
      {
        c64 *Gl = reinterpret_cast<c64 *>(lds);
        c64 *Vl = Gl + kEigLdsN * kEigLdsN;
        int *pos = reinterpret_cast<int *>(Vl + kEigLdsN * kEigLdsN);
        int *pp = pos + 1040, *pq = pp + 520;
        double *pc = reinterpret_cast<double *>(pq + 520);
        double *ps = pc + 520;
        c64 *pe = reinterpret_cast<c64 *>(ps + 520);
        c64 *Gw = Gg, *Vw = m.V + s * m.V_cap;
        if (nn <= kEigLdsN) {
          for (int e = tid; e < nn * nn; e += TB) Gl[e] = Gg[e];
          __syncthreads();
          Gw = Gl;
          Vw = Vl;
        }
        jacobi_block(nn, Gw, Vw, m.ev + s * m.ev_cap, Gg, m.err, pos, pc, ps, pe, pp, pq, &sweeps,
                     sizeof(T) == 8 ? 1e-18 : 1e-16, sizeof(T) == 8 ? 1e-15 : 1e-13);
        if (tid == 0) {
          const double f64 = gemm_flops(nn, nn, Lx) + 36.0 * nn * nn * (double)nn;
          add_work(m, K_LAYER, f64, (double)sizeof(cplx<T>) * Lx * nn + 16.0 * 3 * nn * nn + 8.0 * nn);
          if (m.prof) atomicAdd(&m.work[2 * K_COUNT + 1], f64);        // FP64 share of the layer work
          if (m.prof) atomicAdd(&m.work[2 * K_COUNT], (double)sweeps);
        }
      }
      const int k = select_body<T>(m, s, j);
      cplx<T> *Nn = scr<T>(m.N, m.N_cap, s);
      blk_gemm<T, T, T, T>(Lx, k, nn, X, nn, 0, scr<T>(m.Vt, m.Vt_cap, s), k, 0, Nn, k);
      const int M = 2 * w[j - 1];
      blk_gemm<T, T, T, T>(M, k, Lx, wslot<T>(m, j - 1, s), Lx, 0, Nn, k, 0, X, k);
      if (tid == 0) {
        w[j] = k;
        add_work(m, K_LAYER, gemm_flops(Lx, k, nn) + gemm_flops(M, k, Lx),
                 (double)sizeof(cplx<T>) * ((double)Lx * nn + (double)nn * k + 2.0 * Lx * k + (double)M * Lx + (double)M * k));
      }
      __syncthreads();
    }
    finish_body<T>(m, s, l);
    c = l;
  }
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
  return (size_t)rows * sizeof(c64) + (size_t)rows * 2 * sizeof(double) + kQrLdsMat;
}

template <typename T> void mps_sweep_lr(const MpsDev &m, int l, int r, hipStream_t st) {
  for (int j = l; j < r; ++j) {
    int rows = 2 * (j == l ? dmax(m, j, 1) : 2 * dmax(m, j, 1));
    int cols = 2 * dmax(m, j + 1, 1);
    KLAUNCH(K_QR, k_qr_lr<T>, dim3(m.S), dim3(TB), qr_lds(rows), st, m, j, rows);
    int p = imin(rows, cols);
    int ncol = 2 * (j + 1 == r ? dmax(m, j + 2, 1) : 2 * dmax(m, j + 2, 1));
    KLAUNCH(K_GEMM, k_absorb_lr<T>, gemm_grid(p, ncol, m.S), dim3(TB), 0, st, m, j);
  }
}

static size_t eig_lds() {
  return 2 * kEigLdsN * kEigLdsN * sizeof(c64) + 1040 * sizeof(int) + 2 * 520 * sizeof(int) +
         2 * 520 * sizeof(double) + 520 * sizeof(c64);
}

template <typename T> void mps_sweep_rl(const MpsDev &m, int l, int r, hipStream_t st) {
  for (int j = r; j > l; --j) {
    int L = 2 * dmax(m, j, 1);
    int nn = 2 * dmax(m, j + 1, 1);
    KLAUNCH(K_GRAM, k_gram<T>, gemm_grid(nn, nn, m.S), dim3(TB), 0, st, m, j);
    KLAUNCH(K_EIGEN, k_eig<T>, dim3(m.S), dim3(TB), eig_lds(), st, m, j);
    KLAUNCH(K_SELECT, k_select<T>, dim3(m.S), dim3(TB), 0, st, m, j);
    int kmax = dmax(m, j, 1);
    KLAUNCH(K_GEMM, k_ngemm<T>, gemm_grid(L, kmax, m.S), dim3(TB), 0, st, m, j);
    int M = 2 * (j - 1 == l ? dmax(m, j - 1, 1) : 2 * dmax(m, j - 1, 1));
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

template <typename T>
void mps_rot_layer(const MpsDev &m, const uint64_t *d_pbits, const uint64_t *d_psgn, int W, int SW,
                   const double *d_theta, int64_t stride, const RotLayer &L, hipStream_t st) {
  const int lds_rows = 4 * m.chi;
  const size_t lds = std::max(qr_lds(lds_rows), eig_lds());
  KLAUNCH(K_LAYER, k_rot_layer<T>, dim3(m.S), dim3(TB), lds, st, m, d_pbits, d_psgn, W, SW, d_theta,
          stride, L, lds_rows);
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

// Raise the dynamic-LDS limit of the kernels that stage matrices in LDS
// (gfx950 has 160 KB per CU).  Returns the first HIP error, if any.
template <typename T> hipError_t mps_prepare(int max_rows) {
  hipError_t e = hipFuncSetAttribute((const void *)k_eig<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)eig_lds());
  const int q = (int)qr_lds(max_rows);
  {
    hipError_t e2 = hipFuncSetAttribute((const void *)k_rot_layer<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)std::max((size_t)q, eig_lds()));
    if (e == hipSuccess) e = e2;
  }
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
  template void mps_rot_layer<T>(const MpsDev &, const uint64_t *, const uint64_t *, int, int,   \
                                 const double *, int64_t, const RotLayer &, hipStream_t);       \
  template void mps_expect<T>(const MpsDev &, int, int, const c64 *, hipStream_t);
INST(float)
INST(double)
