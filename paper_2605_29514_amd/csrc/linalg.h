// Block-level dense linear algebra of the compression step (Sec. IV.B),
// shared by the per-step kernels (mps.hip) and the fused per-shot layer
// kernel (layer.hip).  Every routine runs on one thread block of NT threads
// (NT = 64, 128 or 256) and works on one shot's matrices; barriers are block
// barriers only.  Staging buffers are passed in explicitly so that a caller
// can overlay them in one dynamic LDS region.
#pragma once

#include "common.h"

#include <math.h>

namespace stnk {

constexpr int GT = 32;           // GEMM tile (GT x GT outputs)
constexpr int GK = 16;           // GEMM k-step

// ------------------------------------------------------------ accessors
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

// ------------------------------------------------------ element loops
// Block loop over elements e in [0, n), NT apart, U per thread at a time:
// the U loads ld(e) of a group are all issued before the first store
// st(e, v), so they wait on memory together instead of one after another
// (a plain loop cannot be reordered when the compiler cannot rule out
// that a store aliases a later load).
template <int NT, int U, typename V, typename LD, typename ST>
__device__ __forceinline__ void blk_each(int n, LD ld, ST st) {
  for (int e0 = threadIdx.x; e0 < n; e0 += U * NT) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * NT < n) v[u] = ld(e0 + u * NT);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * NT < n) st(e0 + u * NT, v[u]);
  }
}

// The same over the elements of a rows x cols matrix in row-major order,
// with their row and column stepped along (no division per element):
// ld(i, j), st(i, j, v).
template <int NT, int U, typename V, typename LD, typename ST>
__device__ __forceinline__ void blk_each_rc(int rows, int cols, LD ld, ST st) {
  if (cols <= 0) return;
  const int di = NT / cols, dj = NT - di * cols;
  int i0 = threadIdx.x / cols, j0 = threadIdx.x - i0 * cols;
  auto step = [&](int &i, int &j) {
    i += di;
    j += dj;
    if (j >= cols) { j -= cols; ++i; }
  };
  while (i0 < rows) {
    V v[U];
    int i = i0, j = j0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i < rows) v[u] = ld(i, j);
      step(i, j);
    }
    i = i0;
    j = j0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i < rows) st(i, j, v[u]);
      step(i, j);
    }
    i0 = i;
    j0 = j;
  }
}

// ------------------------------------------------------------ reductions
// Sum / max over the block; every thread receives the result.
template <int NT, typename V>
__device__ V bsum(V v) {
  __shared__ V red[NT / 64 > 0 ? NT / 64 : 1];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if constexpr (NT == 64) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    V tot = 0;
    for (int i = 0; i < NT / 64; ++i) tot += red[i];
    return tot;
  }
}

template <int NT>
__device__ double bmax(double v) {
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if constexpr (NT == 64) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double tot = red[0];
    for (int i = 1; i < NT / 64; ++i) tot = fmax(tot, red[i]);
    return tot;
  }
}

// ------------------------------------------------------------------ GEMM
template <typename ACC>
struct GemmStage {
  static constexpr size_t bytes = sizeof(cplx<ACC>) * (GT * (GK + 1) + GK * (GT + 1));
};

// Matrix cores.  v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32 take, per
// lane l of a wave, A[l % 16][l / 16] and B[l / 16][l % 16] of a 16x4 and a
// 4x16 operand and accumulate a 16x16 block of which lane l holds column
// l % 16, rows (l / 16) + 4 i (f64) or 4 (l / 16) + i (f32), i = 0..3.
typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
template <typename ACC> struct Mfma;
template <> struct Mfma<double> {
  using V = v4d_t;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <> struct Mfma<float> {
  using V = v4f_t;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Block tile of the matrix-core GEMM: each wave owns WB 16x16 blocks side
// by side along N, so a block of NT threads covers TM x TN outputs with
// TM x TN = (16 x 16 WB) x (NT / 64); TM, TN <= GT (the staging size).
template <int NT> struct MTile;
template <> struct MTile<64> { static constexpr int TM = 16, TN = 32, WB = 2; };
template <> struct MTile<128> { static constexpr int TM = 32, TN = 32, WB = 2; };
template <> struct MTile<256> { static constexpr int TM = 32, TN = 32, WB = 1; };

// One TM x TN tile of C = op(A) op(B) on the matrix cores.
//   opA = 0: A is M x K (lda);  opA = 1: A is K x M and op(A) = A^H.
//   opB = 0: B is K x N (ldb);  opB = 1: B is N x K and op(B) = B^H.
// Operands are staged through LDS in ACC precision (GK columns at a time,
// zero-padded past M, N, K); each wave forms its 16x16 blocks as complex
// products of four real MFMA chains each:
// re += a_re b_re - a_im b_im, im += a_re b_im + a_im b_re.
// stage: GemmStage<ACC>::bytes of LDS.
template <typename TA, typename TB_, typename TC, typename ACC, int NT>
__device__ void gemm_tile(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                          const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc, int tm,
                          int tn, void *stage) {
  using MF = Mfma<ACC>;
  using V = typename MF::V;
  constexpr int TM = MTile<NT>::TM, TN = MTile<NT>::TN, WB = MTile<NT>::WB;
  constexpr int WN = TN / (16 * WB);                               // waves along N
  static_assert(TM <= GT && TN <= GT && (NT / 64) * 16 * 16 * WB == TM * TN, "GEMM tile");
  cplx<ACC> *As = reinterpret_cast<cplx<ACC> *>(stage);          // [TM][GK + 1]
  cplx<ACC> *Bs = As + GT * (GK + 1);                              // [GK][TN + 1]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = tm * TM, col0 = tn * TN;
  const int sm = (wave / WN) * 16, sn = (wave % WN) * 16 * WB;
  V re[WB], im[WB];
#pragma unroll
  for (int w = 0; w < WB; ++w)
    for (int i = 0; i < 4; ++i) { re[w][i] = 0; im[w][i] = 0; }
  // every operand element of a k-step is loaded before any is stored, so
  // the loads of a step are in flight together
  constexpr int NA = (TM * GK + NT - 1) / NT, NB = (TN * GK + NT - 1) / NT;
  for (int k0 = 0; k0 < K; k0 += GK) {
    cplx<TA> ra[NA];
    cplx<TB_> rb[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * NT, mi = e / GK, ki = e % GK;
      const int m = row0 + mi, k = k0 + ki;
      ra[i] = mk<TA>(0, 0);
      if (e < TM * GK && m < M && k < K) ra[i] = opA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * NT, ki = e / TN, ni = e % TN;
      const int n = col0 + ni, k = k0 + ki;
      rb[i] = mk<TB_>(0, 0);
      if (e < TN * GK && n < N && k < K) rb[i] = opB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * NT;
      if (e < TM * GK) As[(e / GK) * (GK + 1) + e % GK] = opA ? cj(cvt<ACC>(ra[i])) : cvt<ACC>(ra[i]);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * NT;
      if (e < TN * GK) Bs[(e / TN) * (TN + 1) + e % TN] = opB ? cj(cvt<ACC>(rb[i])) : cvt<ACC>(rb[i]);
    }
    __syncthreads();
    const int kend = K - k0 < GK ? K - k0 : GK;
    for (int kk = 0; kk < kend; kk += 4) {
      const cplx<ACC> a = As[(sm + (lane & 15)) * (GK + 1) + kk + (lane >> 4)];
#pragma unroll
      for (int w = 0; w < WB; ++w) {
        const cplx<ACC> b = Bs[(kk + (lane >> 4)) * (TN + 1) + sn + 16 * w + (lane & 15)];
        re[w] = MF::mma(a.x, b.x, re[w]);
        im[w] = MF::mma(a.x, b.y, im[w]);
        re[w] = MF::mma(-a.y, b.y, re[w]);
        im[w] = MF::mma(a.y, b.x, im[w]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int w = 0; w < WB; ++w) {
    const int n = col0 + sn + 16 * w + (lane & 15);
    for (int i = 0; i < 4; ++i) {
      const int m = row0 + sm + MF::row(lane, i);
      if (m < M && n < N) C[(size_t)m * ldc + n] = cvt<TC>(mk<ACC>(re[w][i], im[w][i]));
    }
  }
}

// C = op(A) op(B) (as gemm_tile) with operands read straight from memory
// into the matrix-core lane layout, for products small enough that staging
// through LDS (two barriers per k-step) costs more than it saves.  Each wave
// owns pairs of 16x16 output blocks side by side along N and loads, per
// 16 values of k, its lane's elements of A and of both B blocks together
// before the multiplies: a product costs about one memory latency per
// 16 k.  The k order of the accumulation is that of gemm_tile.
template <typename TA, typename TB_, typename TC, typename ACC, int NT>
__device__ void gemm_direct(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                            const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc, int lower = 0) {
  using MF = Mfma<ACC>;
  using V = typename MF::V;
  constexpr int NW = NT / 64, KC = 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const int nbm = (M + 15) / 16, nbp = (N + 31) / 32;
  for (int bp = wave; bp < nbm * nbp; bp += NW) {
    const int m0 = (bp / nbp) * 16, n0 = (bp % nbp) * 32;
    if (lower && m0 + 16 <= n0) continue;     // lower: blocks wholly above the diagonal are skipped
    const int m = m0 + r16, n1 = n0 + r16, n2 = n0 + 16 + r16;
    V re[2], im[2];
#pragma unroll
    for (int w = 0; w < 2; ++w)
      for (int i = 0; i < 4; ++i) { re[w][i] = 0; im[w][i] = 0; }
    for (int k0 = 0; k0 < K; k0 += KC) {
      cplx<TA> a[KC / 4];
      cplx<TB_> b1[KC / 4], b2[KC / 4];
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        const int k = k0 + 4 * kk + q;
        a[kk] = mk<TA>(0, 0);
        b1[kk] = mk<TB_>(0, 0);
        b2[kk] = mk<TB_>(0, 0);
        if (k < K) {
          if (m < M) a[kk] = opA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
          if (n1 < N) b1[kk] = opB ? B[(size_t)n1 * ldb + k] : B[(size_t)k * ldb + n1];
          if (n2 < N) b2[kk] = opB ? B[(size_t)n2 * ldb + k] : B[(size_t)k * ldb + n2];
        }
      }
      const int kend = K - k0 < KC ? K - k0 : KC;
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        if (4 * kk >= kend) break;
        const cplx<ACC> av = opA ? cj(cvt<ACC>(a[kk])) : cvt<ACC>(a[kk]);
        const cplx<ACC> bv1 = opB ? cj(cvt<ACC>(b1[kk])) : cvt<ACC>(b1[kk]);
        const cplx<ACC> bv2 = opB ? cj(cvt<ACC>(b2[kk])) : cvt<ACC>(b2[kk]);
        re[0] = MF::mma(av.x, bv1.x, re[0]);
        im[0] = MF::mma(av.x, bv1.y, im[0]);
        re[0] = MF::mma(-av.y, bv1.y, re[0]);
        im[0] = MF::mma(av.y, bv1.x, im[0]);
        if (n0 + 16 < N) {
          re[1] = MF::mma(av.x, bv2.x, re[1]);
          im[1] = MF::mma(av.x, bv2.y, im[1]);
          re[1] = MF::mma(-av.y, bv2.y, re[1]);
          im[1] = MF::mma(av.y, bv2.x, im[1]);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int n = n0 + 16 * w + r16;
      for (int i = 0; i < 4; ++i) {
        const int mm = m0 + MF::row(lane, i);
        if (mm < M && n < N) C[(size_t)mm * ldc + n] = cvt<TC>(mk<ACC>(re[w][i], im[w][i]));
      }
    }
  }
}

// All tiles of a product by the calling block (tiles t0, t0 + dt, ...).
template <typename TA, typename TB_, typename TC, typename ACC, int NT>
__device__ void gemm_tiles(int M, int N, int K, const cplx<TA> *A, int lda, int opA,
                           const cplx<TB_> *B, int ldb, int opB, cplx<TC> *C, int ldc, int t0,
                           int dt, void *stage, int lower = 0) {
  constexpr int TM = MTile<NT>::TM, TN = MTile<NT>::TN;
  const int ntm = (M + TM - 1) / TM, ntn = (N + TN - 1) / TN;
  for (int t = t0; t < ntm * ntn; t += dt)
    if (!lower || (t / ntn + 1) * TM > (t % ntn) * TN)
      gemm_tile<TA, TB_, TC, ACC, NT>(M, N, K, A, lda, opA, B, ldb, opB, C, ldc, t / ntn, t % ntn, stage);
}

// ----------------------------------------------------- Householder QR
// In place on A (m x nc, ld = nc), p = min(m, nc) reflectors.  Writes R
// (p x nc, ld = nc, zero below the diagonal) to Rd and the explicit Q
// (m x p) to Qd, either as an m x p matrix (qt = 0) or conjugate-transposed
// as a p x m matrix (qt = 1).
// Scratch: vs (m complex doubles), vd (2p doubles), wp (NT complex doubles).
// The column updates split the block into CL column lanes x G row groups
// (CL = smallest power of two covering the remaining columns), so narrow
// trailing matrices still keep every thread busy.
template <int NT>
__device__ inline void col_split(int ncols, int &CL, int &G) {
  int cl = 1;
  while (cl < ncols && cl < NT) cl <<= 1;
  CL = cl;
  G = NT / cl;
}

// A[i][j] -= vs[i] * 2 (vs^H A)[j] for rows i >= k, columns j in [j0, j1).
template <typename T, int NT>
__device__ void reflect_cols(int m, int nc, int k, int j0, int j1, cplx<T> *A, const c64 *vs,
                             c64 *wp) {
  const int tid = threadIdx.x;
  int CL, G;
  col_split<NT>(j1 - j0, CL, G);
  const int jj = tid % CL, g = tid / CL;
  for (int jb = j0; jb < j1; jb += CL) {
    const int j = jb + jj;
    c64 w = mk<double>(0, 0);
    if (j < j1)
      for (int i = k + g; i < m; i += G) w = w + cj(vs[i]) * cvt<double>(A[(size_t)i * nc + j]);
    wp[tid] = w;
    __syncthreads();
    if (j < j1) {
      c64 wt = mk<double>(0, 0);
      for (int gg = 0; gg < G; ++gg) wt = wt + wp[gg * CL + jj];
      wt = 2.0 * wt;
      // four rows per group: their loads are issued before the first store
      // (a load after a store to memory the compiler cannot prove distinct
      // would otherwise wait for the previous element's round trip)
      for (int i0 = k + g; i0 < m; i0 += 4 * G) {
        cplx<T> av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u * G < m) av[u] = A[(size_t)(i0 + u * G) * nc + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * G;
          if (i < m) A[(size_t)i * nc + j] = cvt<T>(cvt<double>(av[u]) - vs[i] * wt);
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int NT>
__device__ void qr_block(int m, int nc, cplx<T> *A, cplx<T> *Qd, int qt, cplx<T> *Rd, c64 *vs,
                         double *vd, c64 *wp) {
  using C = cplx<T>;
  const int p = m < nc ? m : nc;
  const int tid = threadIdx.x;
  for (int k = 0; k < p; ++k) {
    // Norms and the phase of x0 are formed from double copies: squaring a
    // float below ~1e-19 lands in the denormal range, and an inexact |x0|
    // would leave x0/|x0| off the unit circle, so H = I - 2 v v^H would stop
    // being unitary.
    double part = 0;
    for (int i = k + tid; i < m; i += NT) part += norm2(cvt<double>(A[(size_t)i * nc + k]));
    const double xn2 = bsum<NT>(part);
    const C x0 = A[(size_t)k * nc + k];
    const double ax0 = hypot((double)x0.x, (double)x0.y);
    const double xn = sqrt(xn2);
    const c64 ph = ax0 > 0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1, 0);
    const c64 alpha = mk<double>(-ph.x * xn, -ph.y * xn);
    // v = x - alpha e1, |v|^2 = |x|^2 - |x0|^2 + |x0 - alpha|^2 = 2 |x| (|x| + |x0|)
    const double vn2 = 2.0 * xn * (xn + ax0);
    const double inv = vn2 > 0 ? 1.0 / sqrt(vn2) : 0.0;
    for (int i = k + tid; i < m; i += NT) {
      c64 xi = cvt<double>(A[(size_t)i * nc + k]);
      if (i == k) xi = xi - alpha;
      vs[i] = inv * xi;
    }
    __syncthreads();
    if (inv > 0 && k + 1 < nc) reflect_cols<T, NT>(m, nc, k, k + 1, nc, A, vs, wp);
    if (tid == 0) {
      vd[2 * k] = vs[k].x;
      vd[2 * k + 1] = vs[k].y;
      A[(size_t)k * nc + k] = cvt<T>(inv > 0 ? alpha : cvt<double>(x0));
    }
    for (int i = k + 1 + tid; i < m; i += NT) A[(size_t)i * nc + k] = cvt<T>(vs[i]);
    __syncthreads();
  }
  for (int e = tid; e < p * nc; e += NT) {
    int i = e / nc, j = e % nc;
    Rd[e] = j >= i ? A[(size_t)i * nc + j] : mk<T>(0, 0);
  }
  __syncthreads();
  // Q = H_0 ... H_{p-1} [I; 0], accumulated backwards in A's first p columns
  for (int k = p - 1; k >= 0; --k) {
    for (int i = k + tid; i < m; i += NT)
      vs[i] = i == k ? mk<double>(vd[2 * k], vd[2 * k + 1]) : cvt<double>(A[(size_t)i * nc + k]);
    __syncthreads();
    for (int i = k + tid; i < m; i += NT) A[(size_t)i * nc + k] = mk<T>(i == k ? 1 : 0, 0);
    for (int j = k + 1 + tid; j < p; j += NT) A[(size_t)k * nc + j] = mk<T>(0, 0);
    __syncthreads();
    reflect_cols<T, NT>(m, nc, k, k, p, A, vs, wp);
  }
  for (int e = tid; e < m * p; e += NT) {
    int i = e / p, j = e % p;
    C q = A[(size_t)i * nc + j];
    if (qt)
      Qd[(size_t)j * m + i] = cj(q);
    else
      Qd[e] = q;
  }
  __syncthreads();
}

// ------------------------------------------------ Jacobi eigen-solve (FP64)
// Hermitian nn x nn matrix G (ld nn) -> eigenvalues ev (descending) and the
// matching eigenvectors as columns of Vout (ld nn).  Parallel cyclic Jacobi:
// each round rotates nn/2 disjoint index pairs in the round-robin (circle)
// order -- index 0 fixed, the others shifted by one place per round; the
// 2x2 block [[a, c], [c*, b]] is diagonalised by U = diag(1, e^{-i phi}) R
// with c = |c| e^{i phi} and R the real symmetric Jacobi rotation.
// G and the rotation accumulator V use leading dimension ld (>= nn; one
// more than nn staggers LDS rows across banks); Vout uses nn.
// Scratch: pos (nn + 1 ints), pp/pq (nn/2 + 1 ints), pc/ps (nn/2 + 1
// doubles), pe (nn/2 + 1 complex doubles).
template <int NT>
__device__ void jacobi_block(int nn, c64 *G, int ld, c64 *V, double *ev, c64 *Vout, int *err, int *pos,
                             double *pc, double *ps, c64 *pe, int *pp, int *pq, int *sweeps_out,
                             double abs_tol, double rel_tol) {
  const int tid = threadIdx.x;
  const int P = nn + (nn & 1);
  for (int e = tid; e < nn * nn; e += NT) {
    const int r0 = e / nn, c0 = e - r0 * nn;
    V[(size_t)r0 * ld + c0] = mk<double>(r0 == c0 ? 1.0 : 0.0, 0);
  }
  // The Gram matrix is positive semi-definite, so its trace bounds every
  // eigenvalue and is invariant under the rotations.  An entry G_pq is
  // negligible when |G_pq| <= max(abs_tol tr, rel_tol sqrt(G_pp G_qq)): the
  // relative part keeps small kept eigenvalues from mixing with the (near)
  // null space, the absolute floor stops at the rounding level of the Gram.
  double trp = 0;
  for (int i = tid; i < nn; i += NT) trp += G[(size_t)i * ld + i].x;
  const double tr = bsum<NT>(trp);
  __syncthreads();
  const double afl = abs_tol * tr;
  const int max_sweeps = 60;
  bool converged = nn <= 1 || !(tr > 0);
  int sweeps_done = 0;
  double last_off = 0;
  // strides of the incremental task indices below (NT = st_i H + st_k, ...)
  const int Hh = P / 2 > 0 ? P / 2 : 1;
  const int st_i = NT / Hh, st_k = NT - (NT / Hh) * Hh;
  const int sv_k = nn > 0 ? NT / nn : 0, sv_r = nn > 0 ? NT - (NT / nn) * nn : 0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    for (int rnd = 0; rnd < P - 1; ++rnd) {
      for (int i = tid; i < P / 2; i += NT) {
        // positions 1..P-1 shift by one per round (circle method), 0 stays
        int x = i - 1 - rnd, y = P - 2 - i - rnd;
        if (x < 0) x += P - 1;
        if (y < 0) y += P - 1;
        int p = i == 0 ? 0 : 1 + x;
        int q = 1 + y;
        if (p > q) { int t = p; p = q; q = t; }
        double cs = 1, sn = 0;
        c64 eph = mk<double>(1, 0);
        if (q < nn) {
          const c64 c = G[(size_t)p * ld + q];
          const double h2 = norm2(c);
          const double a = G[(size_t)p * ld + p].x, b = G[(size_t)q * ld + q].x;
          const double h = sqrt(h2);
          if (h > afl && h > rel_tol * sqrt(fabs(a * b))) {
            // t = tan of the rotation angle, the root of t^2 + 2 tau t - 1 = 0
            // of smaller modulus with tau = (b - a) / 2h, written without tau:
            // t = sign(d) 2h / (|d| + sqrt(d^2 + 4 h^2)), d = b - a
            const double d = b - a;
            const double t = (d >= 0 ? 2.0 : -2.0) * h / (fabs(d) + sqrt(d * d + 4.0 * h2));
            const double ih = 1.0 / h;
            eph = mk<double>(c.x * ih, c.y * ih);
            cs = 1.0 / sqrt(1.0 + t * t);
            sn = t * cs;
          }
        }
        pp[i] = p; pq[i] = q; pc[i] = cs; ps[i] = sn; pe[i] = eph;
      }
      __syncthreads();
      // G <- U^H G U and V <- V U in one pass.  The pairs are disjoint and
      // cover every index, so G splits into 2x2 blocks (rows of pair i,
      // columns of pair k) that transform independently:
      // block <- L_i block R_k with L_i (x_p, x_q) = (cs x_p - sn e x_q,
      // sn x_p + cs e x_q) and R_k the same with conj(e) on row vectors.
      // G stays Hermitian, so only blocks i <= k are computed and mirrored.
      const int H = P / 2;
      // (i, k) of task e = i H + k advanced incrementally (no division)
      int bi = tid / H, bk = tid - (tid / H) * H;
      for (int e = tid; e < H * H; e += NT, bi += st_i, bk += st_k) {
        if (bk >= H) { bk -= H; ++bi; }
        const int i = bi, k = bk;
        if (i > k) continue;
        const bool ri = ps[i] != 0, rk = ps[k] != 0;
        if (!ri && !rk) continue;
        const int rp = pp[i], rq = pq[i], cp = pp[k], cq = pq[k];
        const bool vq = rq < nn, wq = cq < nn;
        c64 b00 = G[(size_t)rp * ld + cp];
        c64 b01 = wq ? G[(size_t)rp * ld + cq] : mk<double>(0, 0);
        c64 b10 = vq ? G[(size_t)rq * ld + cp] : mk<double>(0, 0);
        c64 b11 = (vq && wq) ? G[(size_t)rq * ld + cq] : mk<double>(0, 0);
        if (ri) {
          const double cs = pc[i], sn = ps[i];
          const c64 ei = pe[i];
          const c64 t10 = ei * b10, t11 = ei * b11;
          const c64 n00 = cs * b00 - sn * t10, n01 = cs * b01 - sn * t11;
          b10 = sn * b00 + cs * t10;
          b11 = sn * b01 + cs * t11;
          b00 = n00;
          b01 = n01;
        }
        if (rk) {
          const double cs = pc[k], sn = ps[k];
          const c64 ek = cj(pe[k]);
          const c64 t01 = ek * b01, t11 = ek * b11;
          const c64 n00 = cs * b00 - sn * t01, n10 = cs * b10 - sn * t11;
          b01 = sn * b00 + cs * t01;
          b11 = sn * b10 + cs * t11;
          b00 = n00;
          b10 = n10;
        }
        G[(size_t)rp * ld + cp] = b00;
        if (wq) G[(size_t)rp * ld + cq] = b01;
        if (vq) G[(size_t)rq * ld + cp] = b10;
        if (vq && wq) G[(size_t)rq * ld + cq] = b11;
        if (i != k) {                         // mirror: block (k, i) = block (i, k)^H
          G[(size_t)cp * ld + rp] = cj(b00);
          if (vq) G[(size_t)cp * ld + rq] = cj(b10);
          if (wq) G[(size_t)cq * ld + rp] = cj(b01);
          if (vq && wq) G[(size_t)cq * ld + rq] = cj(b11);
        }
      }
      int vk = tid / nn, vr = tid - (tid / nn) * nn;
      for (int e = tid; e < H * nn; e += NT, vk += sv_k, vr += sv_r) {
        if (vr >= nn) { vr -= nn; ++vk; }
        const int k = vk, row = vr;
        if (ps[k] == 0) continue;
        const int p = pp[k], q = pq[k];
        const double cs = pc[k], sn = ps[k];
        const c64 ec = cj(pe[k]);
        const c64 vp = V[(size_t)row * ld + p], vq = ec * V[(size_t)row * ld + q];
        V[(size_t)row * ld + p] = cs * vp - sn * vq;
        V[(size_t)row * ld + q] = sn * vp + cs * vq;
      }
      __syncthreads();
    }
    double off = 0, viol = 0;
    for (int e = tid; e < nn * nn; e += NT) {
      const int p = e / nn, q = e % nn;
      if (p == q) continue;
      const double h = sqrt(norm2(G[(size_t)p * ld + q]));
      off = fmax(off, h);
      if (h > afl && h > rel_tol * sqrt(fabs(G[(size_t)p * ld + p].x * G[(size_t)q * ld + q].x))) viol = 1;
    }
    off = bmax<NT>(off);
    viol = bmax<NT>(viol);
    last_off = off;
    converged = viol == 0;
    sweeps_done = sweep + 1;
    __syncthreads();
  }
  if (sweeps_out && tid == 0) *sweeps_out = sweeps_done;
  if (!converged && tid == 0 && last_off > 1e-10 * tr) atomicOr(err, STN_ERR_EIGEN);
  // sort descending: rank of each eigenvalue (ties by index)
  for (int i = tid; i < nn; i += NT) {
    double li = G[(size_t)i * ld + i].x;
    int rank = 0;
    for (int j = 0; j < nn; ++j) {
      double lj = G[(size_t)j * ld + j].x;
      rank += (lj > li) || (lj == li && j < i);
    }
    ev[rank] = li;
    pos[i] = rank;
  }
  __syncthreads();
  for (int e = tid; e < nn * nn; e += NT) {
    int row = e / nn, col = e % nn;
    Vout[(size_t)row * nn + pos[col]] = V[(size_t)row * ld + col];
  }
  __syncthreads();
}

// Stopping rule of the two-sided Jacobi, which serves the FP64 path: the
// off-diagonal converges to 1e-15 relative (floor 1e-18 of the trace).  Its
// rotations keep the relative accuracy of the small kept eigenvalues, which
// the 1e-10 bound of FP64 probabilities needs.
template <typename T> __device__ inline double jac_abs() { return 1e-18; }
template <typename T> __device__ inline double jac_rel() { return 1e-15; }

// ------------------------------------------------ eigen-solve (FP64)
// Sum over aligned groups of 8 lanes, each lane receiving its group's sum,
// on the DPP lane network (two quad permutations, then the mirror of the
// half row) instead of LDS-routed shuffles.  All 8 lanes of a group must be
// active.  Each lane ends with (x_i + x_(i^1)) + (x_(i^2) + x_(i^3)) plus
// the same for the other quad, the sums a butterfly of xor-shuffles forms.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ double readlane(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double sum8(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  return v;
}

// The same over aligned groups of g = 8 or 16 lanes (one more step, the
// mirror of the row of 16, for g = 16).
__device__ __forceinline__ double sumg(double v, int g) {
  v = sum8(v);
  if (g == 16) v += dpp_mov<0x140>(v);    // row_mirror
  return v;
}

// Block-wide argmax of (v, i): largest v, ties to the smaller i; every
// thread receives the result.  Within a wave: DPP steps inside each row of
// 16 lanes (the choice is symmetric, so exchanging with any lane of the
// other half gives every lane the half's winner), then the four row winners
// read as scalars.  Waves: the partials go to buffer `buf` (0 or 1) of the
// caller's rv / ri (2 x NT/64 entries each): calls that alternate the
// buffer need only the one barrier inside, as long as some barrier
// separates every call from the one two calls earlier.  Every lane of the
// block must take part.
template <int NT>
__device__ void bargmax(double v, int i, double &vo, int &io, double *rv, int *ri, int buf) {
  constexpr int NW = NT / 64 > 0 ? NT / 64 : 1;
  auto take = [&](double v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
  };
  take(dpp_mov<0xB1>(v), dpp_mov<0xB1>(i));     // quad_perm [1, 0, 3, 2]
  take(dpp_mov<0x4E>(v), dpp_mov<0x4E>(i));     // quad_perm [2, 3, 0, 1]
  take(dpp_mov<0x141>(v), dpp_mov<0x141>(i));   // row_half_mirror
  take(dpp_mov<0x140>(v), dpp_mov<0x140>(i));   // row_mirror
  {
    double bv = readlane(v, 0);
    int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      const double v2 = readlane(v, 16 * r);
      const int i2 = __builtin_amdgcn_readlane(i, 16 * r);
      if (v2 > bv || (v2 == bv && i2 < bi)) { bv = v2; bi = i2; }
    }
    v = bv;
    i = bi;
  }
  if constexpr (NW == 1) {
    __syncthreads();                            // the caller's barrier per call
    vo = v;
    io = i;
  } else {
    rv += buf * NW;
    ri += buf * NW;
    if ((threadIdx.x & 63) == 0) { rv[threadIdx.x >> 6] = v; ri[threadIdx.x >> 6] = i; }
    __syncthreads();
    vo = rv[0];
    io = ri[0];
    for (int w = 1; w < NW; ++w)
      if (rv[w] > vo || (rv[w] == vo && ri[w] < io)) { vo = rv[w]; io = ri[w]; }
  }
}

// Eigen-decomposition of a Hermitian positive semi-definite matrix G
// (nn x nn, leading dimension ld, in LDS or global memory; overwritten):
// the reduced density of a truncation step, whose numerical rank is often
// well below its order.
//
//  1. Pivoted Cholesky, right-looking and in place: at step k the largest
//     remaining diagonal d of the Schur complement S picks the pivot p, the
//     Schur complement of the other indices loses S_p^H S_p / d, and row p
//     becomes R_k = S_p / sqrt(d) (zero at the columns pivoted before).  It stops
//     once d <= chol_tol tr G; the part not captured has eigenvalues at most
//     (nn - r) chol_tol tr G.  Then G = R^H R with the r rows of R in rows
//     piv[0..r) of G.
//  2. One-sided Jacobi on those rows: each round rotates r/2 disjoint row
//     pairs (circle order), a pair (x, y) with a = |x|^2, b = |y|^2,
//     c = x y^H being replaced by (cs x - sg y, conj(sg) x + cs y),
//     sg = sn c / |c|, where t = sn / cs is the root of smaller modulus of
//     t^2 + 2 t (b - a) / 2|c| - 1 = 0, which makes the pair orthogonal.
//     The squared row norms come from the rows at the start of a sweep and
//     follow each rotation in closed form (a - t|c|, b + t|c|).
//     Pairs with |c| > rot_tol sqrt(a b) are rotated; sweeps repeat until
//     no pair had |c| > conv_tol sqrt(a b).  With rot_tol below conv_tol
//     the last sweep leaves the rows orthogonal to rounding level: the
//     eigenvectors come out orthonormal as well as the rotations that an
//     accumulated two-sided solve would give.  Pivoting orders the rows by
//     decreasing weight, which speeds the sweeps up.
//  3. The rows are now orthogonal, so G = sum_c u_c u_c^H with u_c = row
//     c^H: eigenvalue |u_c|^2, eigenvector u_c / |u_c|.  ev <- eigenvalues
//     in descending order (0 past r); column j of Vout (nn x nn, leading
//     dimension nn, distinct from G) <- the eigenvector of ev[j] for j < r
//     (e_0 when r = 0).  With Vout null the eigenvectors stay where they
//     are: for j < r, eigenvector j = conj(row piv[pos[j]] of G) times
//     dg[pos[j]] (pos then maps rank to factor row, dg holds 1 / |u_c|).
// Scratch: piv, pos (nn ints), dg (nn doubles).  Returns (to every thread)
// the flops executed; *sweeps_out (thread 0) <- Jacobi sweeps.
constexpr int kEigTpp = 8;        // threads per row pair (the width of sum8)
constexpr int kEigRegN = 32;      // rows up to this length are held in registers per round
constexpr int kEigMaxSweeps = 40;

// Steps 2 and 3 of eig_psd on r factor rows of length nn (rows piv[0..r)
// of G, leading dimension ld): one-sided Jacobi, then eigenvalues into ev
// (descending, 0 from r to nn) and eigenvectors into Vout or left in the
// rows (see eig_psd).  Scratch: pos (nn ints), dg (nn doubles).  Returns the
// flops executed.
template <int NT>
__device__ double jac_rows(int nn, int r, c64 *G, int ld, double *ev, c64 *Vout, int *err, const int *piv,
                           int *pos, double *dg, int *sweeps_out, double conv_tol, double rot_tol) {
  const int tid = threadIdx.x;
  double flops = 0;
  // 2. one-sided Jacobi on the rows piv[0..r)
  int sweeps = 0;
  if (r >= 2) {
    // 16 lanes per pair when every pair of a round then still has its own
    // lanes (half the work per lane), else kEigTpp
    const int P = r + (r & 1), H = P / 2;
    const int TPP = H <= NT / 16 ? 16 : kEigTpp, GP = NT / TPP;
    const int li = tid & (TPP - 1), gi = tid / TPP;
    // "some pair of this sweep rotated by more than conv_tol", set by the
    // rotating groups and read after the sweep's last barrier; two buffers
    // alternate by sweep, so a reset never meets a read of the same buffer
    __shared__ int rotf[2];
    for (int sweep = 0; sweep < kEigMaxSweeps; ++sweep) {
      if (tid == 0) rotf[sweep & 1] = 0;
      // squared row norms: from the rows at the start of each sweep, then
      // updated in closed form by every rotation (a - tau |c|^2 and
      // b + tau |c|^2, the new diagonal of the pair's 2 x 2 Gram); dg[k]
      // holds row k's (free once the factor rows are final)
      for (int i0 = 0; i0 < r; i0 += GP) {
        const int i = i0 + gi;
        double a = 0;
        if (i < r) {
          const c64 *X = G + (size_t)piv[i] * ld;
          for (int j = li; j < nn; j += TPP) a += norm2(X[j]);
        }
        a = sumg(a, TPP);
        if (i < r && li == 0) dg[i] = a;
      }
      __syncthreads();
      for (int rnd = 0; rnd < P - 1; ++rnd) {
        for (int pi = gi; pi < H; pi += GP) {
          // positions 1..P-1 shift by one per round (circle method), 0 stays
          int x = pi - 1 - rnd, y = P - 2 - pi - rnd;
          if (x < 0) x += P - 1;
          if (y < 0) y += P - 1;
          int p = pi == 0 ? 0 : 1 + x, q = 1 + y;
          if (p > q) { const int t = p; p = q; q = t; }
          if (q >= r) continue;
          c64 *X = G + (size_t)piv[p] * ld, *Y = G + (size_t)piv[q] * ld;
          const double a = dg[p], b = dg[q];
          c64 cc = mk<double>(0, 0);
          // orders up to kEigRegN: the lane's elements of both rows stay in
          // registers between the products and the rotation
          c64 xr[kEigRegN / kEigTpp], yr[kEigRegN / kEigTpp];
          if (nn <= kEigRegN) {
#pragma unroll
            for (int u = 0; u < kEigRegN / kEigTpp; ++u) {
              const int j = li + u * TPP;
              xr[u] = j < nn ? X[j] : mk<double>(0, 0);
              yr[u] = j < nn ? Y[j] : mk<double>(0, 0);
            }
#pragma unroll
            for (int u = 0; u < kEigRegN / kEigTpp; ++u) cc = cc + xr[u] * cj(yr[u]);
          } else {
            for (int j = li; j < nn; j += TPP) cc = cc + X[j] * cj(Y[j]);
          }
          cc.x = sumg(cc.x, TPP);
          cc.y = sumg(cc.y, TPP);
          // in terms of h2 = |c|^2: t = tau |c|, cs = 1 / sqrt(1 + t^2),
          // sg = sn c / |c| = tau cs c
          const double h2 = norm2(cc), ab = a * b;
          if (h2 > 0 && h2 > rot_tol * rot_tol * ab) {
            const double d = b - a;
            const double tau = (d >= 0 ? 2.0 : -2.0) / (fabs(d) + sqrt(d * d + 4.0 * h2));
            const double cs = rsqrt(1.0 + tau * tau * h2), ts = tau * cs;
            const c64 sg = mk<double>(cc.x * ts, cc.y * ts), sgc = cj(sg);
            if (nn <= kEigRegN) {
#pragma unroll
              for (int u = 0; u < kEigRegN / kEigTpp; ++u) {
                const int j = li + u * TPP;
                if (j < nn) {
                  X[j] = cs * xr[u] - sg * yr[u];
                  Y[j] = sgc * xr[u] + cs * yr[u];
                }
              }
            } else {
              // two elements of each row per step, loads before stores
              for (int j0 = li; j0 < nn; j0 += 2 * TPP) {
                const int j1 = j0 + TPP;
                const c64 x0 = X[j0], y0 = Y[j0];
                c64 x1 = mk<double>(0, 0), y1 = mk<double>(0, 0);
                if (j1 < nn) { x1 = X[j1]; y1 = Y[j1]; }
                X[j0] = cs * x0 - sg * y0;
                Y[j0] = sgc * x0 + cs * y0;
                if (j1 < nn) {
                  X[j1] = cs * x1 - sg * y1;
                  Y[j1] = sgc * x1 + cs * y1;
                }
              }
            }
            if (li == 0) {
              dg[p] = a - tau * h2;
              dg[q] = b + tau * h2;
            }
            if (li == 0 && h2 > conv_tol * conv_tol * ab) rotf[sweep & 1] = 1;
          }
        }
        __syncthreads();
      }
      sweeps = sweep + 1;
      if (rotf[sweep & 1] == 0) break;
      if (sweeps == kEigMaxSweeps && tid == 0) atomicOr(err, STN_ERR_EIGEN);
    }
    flops += (double)sweeps * ((r * (r - 1) / 2) * 32.0 * nn + 4.0 * r * nn);
  }
  // 3. eigenvalues (squared row norms), their order, eigenvectors
  {
    constexpr int TPP = kEigTpp, GP = NT / kEigTpp;
    const int li = tid % TPP, gi = tid / TPP;
    for (int i0 = 0; i0 < r; i0 += GP) {
      const int i = i0 + gi;
      double a = 0;
      if (i < r) {
        const c64 *X = G + (size_t)piv[i] * ld;
        for (int j = li; j < nn; j += TPP) a += norm2(X[j]);
      }
      a = sum8(a);
      if (i < r && li == 0) dg[i] = a;
    }
  }
  __syncthreads();
  for (int i = tid; i < r; i += NT) {
    const double l = dg[i];
    int rank = 0;
    for (int j = 0; j < r; ++j) {
      const double lj = dg[j];
      rank += (lj > l) || (lj == l && j < i);
    }
    ev[rank] = l;
    if (Vout) pos[i] = rank;
    else pos[rank] = i;
  }
  for (int i = r + tid; i < nn; i += NT) ev[i] = 0;
  __syncthreads();
  if (Vout) {
    blk_each_rc<NT, 4, c64>(
        r, nn, [&](int c, int i) { return G[(size_t)piv[c] * ld + i]; },
        [&](int c, int i, c64 v) {
          const double nr = dg[c];
          const double inv = nr > 0 ? 1.0 / sqrt(nr) : 0.0;
          Vout[(size_t)i * nn + pos[c]] = inv * cj(v);
        });
    if (r == 0)
      for (int i = tid; i < nn; i += NT) Vout[(size_t)i * nn] = mk<double>(i == 0 ? 1.0 : 0.0, 0);
  } else {
    for (int c = tid; c < r; c += NT) dg[c] = dg[c] > 0 ? 1.0 / sqrt(dg[c]) : 0.0;
  }
  if (sweeps_out && tid == 0) *sweeps_out = sweeps;
  __syncthreads();
  return flops;
}

// Pivoted Cholesky of a Hermitian positive semi-definite nn x nn matrix A
// (leading dimension lda, read only), left-looking: step k takes the largest
// remaining diagonal d of the Schur complement as pivot p (ties to the lower
// index) and forms only the new factor row
//   R_k[j] = (A[p][j] - sum_{t<k} conj(R_t[p]) R_t[j]) / sqrt(d)
// (sqrt(d) at j = p, 0 at the columns pivoted before), so no trailing matrix
// is written back: a step reads the rows made so far, all its loads in
// flight together.  The rows go to R (leading dimension ldr), contiguous in
// pivot order, with R^H R = A up to the part left out; the Schur diagonal
// follows each row (d_q -= |R_k[q]|^2).  Stops once d <= chol_tol tr A (the
// eigenvalues left out are then at most nn chol_tol tr A in total), returns
// the rank r and (to every thread) tr A in *trace.  lower: only A's lower
// triangle is read (A_pj = conj(A_jp) above the diagonal).  Rl: LDS room
// for the first tl rows (ld nn), which every later step re-reads: they are
// kept there as well as in R.  The pivots d never grow
// from step to step; *r_cut is the number of steps taken while d was above
// cut_tol tr A (cut_tol >= chol_tol) and *resid the trace of the Schur
// complement left at that point (tr A minus the squared norms of those rows).
// Scratch: dg (nn doubles), pos (nn ints), wp (NT complex doubles).
template <int NT>
__device__ __noinline__ int chol_rows(int nn, const c64 *A, int lda, c64 *R, int ldr, double chol_tol, double *dg,
                                      int *pos,
                         c64 *wp, int *err, double *trace, double *flops, double cut_tol, int *r_cut,
                         double *resid, bool lower = false, c64 *Rl = nullptr, int tl = 0) {
  const int tid = threadIdx.x;
  constexpr int NW = NT / 64 > 0 ? NT / 64 : 1;
  __shared__ double amv[2 * NW];
  __shared__ int ami[2 * NW];
  double trp = 0, v = -INFINITY;
  int vi = 0x7fffffff;
  for (int i = tid; i < nn; i += NT) {
    const double d = A[(size_t)i * lda + i].x;
    dg[i] = d;
    pos[i] = nn;
    trp += d;
    if (d > v) { v = d; vi = i; }
  }
  const double tr = bsum<NT>(trp);
  *trace = tr;
  if (tid == 0 && (!(tr == tr) || isinf(tr))) atomicOr(err, STN_ERR_NUMERIC);
  const double thr = chol_tol * tr;
  double d;
  int p;
  bargmax<NT>(v, vi, d, p, amv, ami, 0);
  int CL, G;
  col_split<NT>(nn, CL, G);
  const int jj = tid % CL, g = tid / CL;
  int r = 0, rc = -1;
  double fl = 0, res = 0;
  const double cthr = cut_tol * tr;
  for (int k = 0; k < nn; ++k) {
    if (rc < 0 && !(d > cthr)) {               // uniform: d comes from the block argmax
      double part = 0;
      for (int q = tid; q < nn; q += NT)
        if (pos[q] >= nn) part += dg[q];
      res = bsum<NT>(part);
      rc = k;
    }
    if (!(d > thr) || !(tr > 0)) break;
    const double isd = 1.0 / sqrt(d);
    for (int jb = 0; jb < nn; jb += CL) {
      const int j = jb + jj;
      const bool live = j < nn && j != p && pos[j] >= nn;
      c64 acc = mk<double>(0, 0);
      if (live) {
        // the group's rows t = g, g + G, ...: four at a time, loads first
        for (int t0 = g; t0 < k; t0 += 4 * G) {
          c64 rp[4], rj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * G;
            if (t < k) {
              const c64 *row = t < tl ? Rl + (size_t)t * nn : R + (size_t)t * ldr;
              rp[u] = row[p];
              rj[u] = row[j];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (t0 + u * G < k) acc = acc + cj(rp[u]) * rj[u];
        }
      }
      if (G > 1) {
        wp[tid] = acc;
        __syncthreads();
        if (g == 0)
          for (int gg = 1; gg < G; ++gg) acc = acc + wp[gg * CL + jj];
      }
      if (g == 0 && j < nn) {
        c64 val;
        if (j == p) val = mk<double>(sqrt(d), 0);
        else if (!live) val = mk<double>(0, 0);
        else val = isd * ((lower && j > p ? cj(A[(size_t)j * lda + p]) : A[(size_t)p * lda + j]) - acc);
        R[(size_t)k * ldr + j] = val;
        if (k < tl) Rl[(size_t)k * nn + j] = val;
      }
      if (G > 1) __syncthreads();
    }
    __syncthreads();
    fl += 8.0 * (double)k * (nn - k);
    // Schur diagonal and the next pivot
    v = -INFINITY;
    vi = 0x7fffffff;
    for (int q = tid; q < nn; q += NT) {
      if (q == p || pos[q] < nn) continue;
      const double nd = dg[q] - norm2(k < tl ? Rl[(size_t)k * nn + q] : R[(size_t)k * ldr + q]);
      dg[q] = nd;
      if (nd > v) { v = nd; vi = q; }
    }
    __syncthreads();
    if (tid == 0) pos[p] = k;
    r = k + 1;
    bargmax<NT>(v, vi, d, p, amv, ami, (k + 1) & 1);
  }
  if (rc < 0) rc = r;                          // full rank above the cut: nothing left
  *r_cut = rc;
  *resid = res;
  *flops += fl;
  return r;
}

// Cholesky factor of a Hermitian positive definite r x r matrix K in place
// (ld ldk): right-looking, one barrier per column, the trailing update taken
// from the unscaled column (K_ij -= K_ik conj(K_jk) / d_k) and every column
// scaled at the end; the upper triangle is set to zero.  Returns false (to
// every thread, K partly updated) when a pivot is not positive.
template <int NT>
__device__ bool chol_lower(int r, c64 *K, int ldk) {
  const int tid = threadIdx.x;
  for (int k = 0; k < r; ++k) {
    const double d = K[(size_t)k * ldk + k].x;
    if (!(d > 0)) return false;
    const double id = 1.0 / d;
    const int t = r - k - 1;
    for (int e = tid; e < t * t; e += NT) {
      const int i = k + 1 + e / t, j = k + 1 + e % t;
      if (j > i) continue;
      const c64 a = K[(size_t)i * ldk + k], b = K[(size_t)j * ldk + k];
      K[(size_t)i * ldk + j] = K[(size_t)i * ldk + j] - id * (a * cj(b));
    }
    __syncthreads();
  }
  for (int e = tid; e < r * r; e += NT) {
    const int i = e / r, j = e % r;
    if (j > i) K[(size_t)i * ldk + j] = mk<double>(0, 0);
    else if (j < i) K[(size_t)i * ldk + j] = (1.0 / sqrt(K[(size_t)j * ldk + j].x)) * K[(size_t)i * ldk + j];
  }
  __syncthreads();
  for (int i = tid; i < r; i += NT) K[(size_t)i * ldk + i] = mk<double>(sqrt(K[(size_t)i * ldk + i].x), 0);
  __syncthreads();
  return true;
}

// Inverse of a lower-triangular r x r matrix L in place (ld ldk, real
// positive diagonal, zero upper triangle), row by row with one barrier per
// row: row i of the inverse W is W_ii = 1 / L_ii,
// W_ij = -(sum_{k=j}^{i-1} L_ik W_kj) / L_ii (j < i), from row i of L and
// the rows above, of which row i-1 is still in its staging buffer while it
// is written back (no thread reads L's row i-1 after step i-1).
// stage: 2 r complex.
template <int NT>
__device__ void trinv_lower(int r, c64 *K, int ldk, c64 *stage) {
  const int tid = threadIdx.x;
  for (int i = 0; i < r; ++i) {
    const c64 *prev = stage + ((i + 1) & 1) * r;      // W row i - 1
    c64 *cur = stage + (i & 1) * r;
    const double il = 1.0 / K[(size_t)i * ldk + i].x;
    for (int j = tid; j <= i; j += NT) {
      if (j == i) {
        cur[j] = mk<double>(il, 0);
      } else {
        c64 acc = K[(size_t)i * ldk + (i - 1)] * prev[j];
        for (int k = j; k < i - 1; ++k) acc = acc + K[(size_t)i * ldk + k] * K[(size_t)k * ldk + j];
        cur[j] = (-il) * acc;
      }
    }
    if (i > 0)
      for (int j = tid; j < i; j += NT) K[(size_t)(i - 1) * ldk + j] = prev[j];
    __syncthreads();
  }
  if (r > 0)
    for (int j = tid; j < r; j += NT) K[(size_t)(r - 1) * ldk + j] = stage[((r - 1) & 1) * r + j];
  __syncthreads();
}

// Orthonormal rows spanning the r rows of R (r x nn, ld ldr, FP64), in
// place.  First pass, Cholesky QR: K = R R^H = L L^H, Q = L^{-1} R; it leaves
// a loss of orthogonality E = Q Q^H - I of about eps_64 cond(R)^2 (the rows
// here come from a pivoted Cholesky stopped at a relative pivot of 1e-12 or
// more, so cond(R) stays near 1e6 and |E| near 1e-4).  Second pass, the
// inverse square root of Q Q^H = I + E to second order:
// R <- (I - E/2 + 3 E^2 / 8) Q, exact to O(|E|^3); when max |E_ij| passes
// 1e-3 a second Cholesky QR pass runs instead.  K: (r + 1)(r + 2) complex
// (ld r + 1; the Gram, its factor and inverse, then staging rows), Tmp:
// r x nn (ld ldr).  Returns false when a factorisation meets a
// non-positive pivot; R then holds its input.
template <int NT>
__device__ __noinline__ bool orth_rows(int r, int nn, c64 *R, int ldr, c64 *Tmp, c64 *K, double *flops) {
  const int ldk = r + 1, tid = threadIdx.x;
  c64 *stage = K + (size_t)r * ldk;
  // pass 1: Tmp = L^{-1} R
  gemm_direct<double, double, double, double, NT>(r, r, nn, R, ldr, 0, R, ldr, 1, K, ldk);
  __syncthreads();
  if (!chol_lower<NT>(r, K, ldk)) return false;
  trinv_lower<NT>(r, K, ldk, stage);
  gemm_direct<double, double, double, double, NT>(r, nn, r, K, ldk, 0, R, ldr, 0, Tmp, ldr);
  __syncthreads();
  *flops += 2 * gemm_flops(r, r, nn) + 8.0 * r * r * (double)r / 3.0;
  // pass 2: E = Tmp Tmp^H - I (in K), E^2 (in R, free now)
  gemm_direct<double, double, double, double, NT>(r, r, nn, Tmp, ldr, 0, Tmp, ldr, 1, K, ldk);
  __syncthreads();
  double mx = 0;
  for (int e = tid; e < r * r; e += NT) {
    const int i = e / r, j = e - (e / r) * r;
    c64 v = K[(size_t)i * ldk + j];
    if (i == j) v.x -= 1.0;
    K[(size_t)i * ldk + j] = v;
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  mx = bmax<NT>(mx);
  if (mx <= 1e-3) {
    gemm_direct<double, double, double, double, NT>(r, r, r, K, ldk, 0, K, ldk, 0, R, ldr);
    __syncthreads();
    for (int e = tid; e < r * r; e += NT) {
      const int i = e / r, j = e - (e / r) * r;
      c64 c = -0.5 * K[(size_t)i * ldk + j] + 0.375 * R[(size_t)i * ldr + j];
      if (i == j) c.x += 1.0;
      K[(size_t)i * ldk + j] = c;
    }
    __syncthreads();
    gemm_direct<double, double, double, double, NT>(r, nn, r, K, ldk, 0, Tmp, ldr, 0, R, ldr);
    __syncthreads();
    *flops += 2 * gemm_flops(r, r, nn) + gemm_flops(r, r, r);
    return true;
  }
  // large loss of orthogonality: a second Cholesky QR pass, Tmp -> R
  for (int e = tid; e < r; e += NT) K[(size_t)e * ldk + e].x += 1.0;   // back to Tmp Tmp^H
  __syncthreads();
  if (!chol_lower<NT>(r, K, ldk)) return false;
  trinv_lower<NT>(r, K, ldk, stage);
  gemm_direct<double, double, double, double, NT>(r, nn, r, K, ldk, 0, Tmp, ldr, 0, R, ldr);
  __syncthreads();
  *flops += 2 * gemm_flops(r, r, nn) + 8.0 * r * r * (double)r / 3.0;
  return true;
}

// Orthonormal columns spanning the cols columns of the FP32 matrix X (rows x
// cols, row-major, rows >= cols, full column rank): Cholesky QR in FP64,
// K = X^H X = L L^H, Q1 = X L^{-H}, then the second-order inverse square root
// of Q1^H Q1 = I + E: Q = Q1 (I - E/2 + 3 E^2 / 8).  Q goes to Qd in FP32, as
// Q (qt = 0, rows x cols) or Q^H (qt = 1, cols x rows).  K: (cols + 1)(cols
// + 2) complex (ld cols + 1; LDS), G1: rows x cols, G2: cols x cols (FP64
// scratch).  Returns false, Qd untouched, when the Gram is not positive
// definite or E passes 1e-3 anywhere (X too ill-conditioned: the caller
// falls back to Householder QR).
template <int NT>
__device__ __noinline__ bool qr_cols_cq(int rows, int cols, const cplx<float> *X, cplx<float> *Qd, int qt, c64 *K,
                                        c64 *G1, c64 *G2) {
  const int ldk = cols + 1, tid = threadIdx.x;
  gemm_direct<float, float, double, double, NT>(cols, cols, rows, X, cols, 1, X, cols, 0, K, ldk);
  __syncthreads();
  if (!chol_lower<NT>(cols, K, ldk)) return false;
  trinv_lower<NT>(cols, K, ldk, K + (size_t)cols * ldk);
  gemm_direct<float, double, double, double, NT>(rows, cols, cols, X, cols, 0, K, ldk, 1, G1, cols);
  __syncthreads();
  gemm_direct<double, double, double, double, NT>(cols, cols, rows, G1, cols, 1, G1, cols, 0, K, ldk);
  __syncthreads();
  double mx = 0;
  for (int e = tid; e < cols * cols; e += NT) {
    const int i = e / cols, j = e - (e / cols) * cols;
    c64 v = K[(size_t)i * ldk + j];
    if (i == j) v.x -= 1.0;
    K[(size_t)i * ldk + j] = v;
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  mx = bmax<NT>(mx);
  if (!(mx <= 1e-3)) return false;
  gemm_direct<double, double, double, double, NT>(cols, cols, cols, K, ldk, 0, K, ldk, 0, G2, cols);
  __syncthreads();
  for (int e = tid; e < cols * cols; e += NT) {
    const int i = e / cols, j = e - (e / cols) * cols;
    c64 c = -0.5 * K[(size_t)i * ldk + j] + 0.375 * G2[(size_t)i * cols + j];
    if (i == j) c.x += 1.0;
    K[(size_t)i * ldk + j] = c;
  }
  __syncthreads();
  if (qt)   // Q^H = C^H Q1^H (C is Hermitian)
    gemm_direct<double, double, float, double, NT>(cols, rows, cols, K, ldk, 1, G1, cols, 1, Qd, rows);
  else
    gemm_direct<double, double, float, double, NT>(rows, cols, cols, G1, cols, 0, K, ldk, 0, Qd, cols);
  __syncthreads();
  return true;
}

template <int NT>
__device__ double eig_psd(int nn, c64 *G, int ld, double *ev, c64 *Vout, int *err, int *piv, int *pos,
                          double *dg, int *sweeps_out, double chol_tol, double conv_tol, double rot_tol,
                          long long *t_chol = nullptr) {
  const int tid = threadIdx.x;
  constexpr int NW = NT / 64 > 0 ? NT / 64 : 1;
  __shared__ double amv[2 * NW];
  __shared__ int ami[2 * NW];
  double trp = 0;
  for (int i = tid; i < nn; i += NT) {
    const double d = G[(size_t)i * ld + i].x;
    dg[i] = d;
    trp += d;
  }
  const double tr = bsum<NT>(trp);
  if (tid == 0 && (!(tr == tr) || isinf(tr))) atomicOr(err, STN_ERR_NUMERIC);
  const double thr = chol_tol * tr;
  double flops = 0;
  // 1. pivoted Cholesky.  The Schur updates use the raw pivot row S_p scaled
  // by 1/d (no separate pass to publish the normalised row, so one barrier
  // per pivot, inside bargmax); pos[j] = the step that pivoted j (nn: not
  // yet).  The rows are normalised, and zeroed at the columns pivoted
  // before them, in one pass after the loop.
  int r = 0;
  {
    double v = -INFINITY;
    int vi = 0x7fffffff;
    for (int i = tid; i < nn; i += NT) {
      pos[i] = nn;
      if (dg[i] > v) { v = dg[i]; vi = i; }
    }
    double d;
    int p;
    bargmax<NT>(v, vi, d, p, amv, ami, 0);
    const int di = NT / nn, dj = NT - (NT / nn) * nn;
    for (int k = 0; k < nn; ++k) {
      if (!(d > thr) || !(tr > 0)) break;
      const double id = 1.0 / d;
      if (tid == 0) { piv[k] = p; pos[p] = k; }
      const c64 *R = G + (size_t)p * ld;
      int i = tid / nn, j = tid - (tid / nn) * nn;
      for (int e = tid; e < nn * nn; e += NT, i += di, j += dj) {
        if (j >= nn) { j -= nn; ++i; }
        if (i == p || j == p || i == j || pos[i] < nn || pos[j] < nn) continue;
        G[(size_t)i * ld + j] = G[(size_t)i * ld + j] - id * (cj(R[i]) * R[j]);
      }
      v = -INFINITY;
      vi = 0x7fffffff;
      for (int q = tid; q < nn; q += NT) {
        if (q == p || pos[q] < nn) continue;
        const double nd = dg[q] - id * norm2(R[q]);
        dg[q] = nd;
        if (nd > v) { v = nd; vi = q; }
      }
      flops += 8.0 * (double)(nn - k - 1) * (nn - k - 1);
      r = k + 1;
      bargmax<NT>(v, vi, d, p, amv, ami, (k + 1) & 1);
    }
    // row k of R: sqrt(d_k) at its pivot, 0 at columns pivoted before step
    // k, S_pk / sqrt(d_k) elsewhere (dg[p_k] still holds d_k)
    for (int e = tid; e < r * nn; e += NT) {
      const int kk = e / nn, jj = e - kk * nn;
      const int pk = piv[kk];
      const double dk = dg[pk];
      c64 *row = G + (size_t)pk * ld;
      if (jj == pk) row[jj] = mk<double>(sqrt(dk), 0);
      else if (pos[jj] < kk) row[jj] = mk<double>(0, 0);
      else row[jj] = (1.0 / sqrt(dk)) * row[jj];
    }
    __syncthreads();
  }
  if (t_chol && tid == 0) *t_chol = clock64();
  return flops + jac_rows<NT>(nn, r, G, ld, ev, Vout, err, piv, pos, dg, sweeps_out, conv_tol, rot_tol);
}

// Tolerances of the one-sided Jacobi, which serves the FP32 path.  Its
// states keep the vectors in FP32 (relative rounding 6e-8), so rows
// orthogonal to 1e-10 are already more accurate than stored.  (Forming rho
// squares the condition of the small kept directions: their eigenvectors
// carry errors ~ eps_64 tr / lambda, up to ~3e-11 of the state per step,
// far below FP32 rounding but above what the FP64 bound allows.)
template <typename T> __device__ inline double eig_conv_tol() { return 1e-10; }
template <typename T> __device__ inline double eig_rot_tol() { return 1e-10; }
// Pivoted-Cholesky cut: captures every eigenvalue above eps_cut tr G (the
// truncation threshold), but not below a few roundings of tr G.
__device__ inline double chol_tol(double eps_cut, int nn) { return fmax(eps_cut / (nn > 0 ? nn : 1), 4e-16); }
// Algorithmic work of one truncation eigen-solve of order nn, whatever the
// route: that of a dense Hermitian solve with vectors, 107 chi^3 FP64 flops
// at the saturated order nn = 2 chi (107/8 nn^3), fixed so that the counted
// work of a step does not depend on sweep counts or on the route taken.
__device__ inline double eig_nominal_flops(int nn) { return 107.0 / 8.0 * nn * nn * (double)nn; }

// ------------------------------------------------------------ truncation
// Keep k' = min(chi_max, #{lambda_i > eps sum lambda}, 2^min(j, n-j)) largest
// (at least 1); the discarded weight updates the fidelity; Vt = V[:, :k']
// (nn x k'); site j <- Vt^H as (k', 2, wb[j+1]); bond[j] = k',
// bond[j+1] = wb[j+1].  ev: the sorted eigenvalues (nn); vload(i, c):
// element i of the eigenvector of ev[c].
// Vt = the k kept columns (nn x k), site j <- Vt^H as (k, 2, wb[j+1]),
// bond[j] = k, bond[j+1] = wb[j+1].
template <typename T, int NT, typename VF>
__device__ void select_store(const MpsDev &m, int s, int j, int k, VF vload, cplx<T> *Vt) {
  const int *w = wbd(m, s);
  const int nn = 2 * w[j + 1];
  cplx<T> *site = slot<T>(m, j, s);
  blk_each_rc<NT, 4, cplx<T>>(
      nn, k, [&](int i, int c) { return cvt<T>(vload(i, c)); },
      [&](int i, int c, cplx<T> v) {
        Vt[(size_t)i * k + c] = v;
        site[(size_t)c * nn + i] = cj(v);
      });
  if (threadIdx.x == 0) {
    bnd(m, s)[j] = k;
    bnd(m, s)[j + 1] = w[j + 1];
  }
  __syncthreads();
}

template <typename T, int NT, typename VF>
__device__ int select_core(const MpsDev &m, int s, int j, const double *ev, VF vload, cplx<T> *Vt) {
  int *w = wbd(m, s);
  const int nn = 2 * w[j + 1];
  __shared__ int kk;
  double part = 0;
  for (int i = threadIdx.x; i < nn; i += NT) part += fmax(ev[i], 0.0);
  const double tot = bsum<NT>(part);
  int cnt = 0;
  for (int i = threadIdx.x; i < nn; i += NT) cnt += ev[i] > m.eps_cut * tot;
  cnt = bsum<NT>(cnt);
  if (threadIdx.x == 0) {
    int k = cnt < m.chi ? cnt : m.chi;
    const int e = j < m.n - j ? j : m.n - j;           // physical bound 2^min(j, n-j)
    const bool phys = e < 30 && k > (1 << e);
    if (phys) k = 1 << e;
    if (k < 1) k = 1;
    // chi_max dropped values above the cut (the physical bound only ever
    // clips rounding noise, so it does not count)
    if (cnt > m.chi && !phys) m.trunc[s] = 1;
    double disc = 0;
    for (int i = k; i < nn; ++i) disc += fmax(ev[i], 0.0);
    const double wgt = tot > 0 ? disc / tot : 0.0;
    m.fid[s] *= (1.0 - wgt);
    if (!(tot == tot) || isinf(tot)) atomicOr(m.err, STN_ERR_NUMERIC);
    kk = k;
    auxp(m, s)[2] = k;
    auxp(m, s)[3] = w[j];          // L, read by the Q N product while wb[j] changes
  }
  __syncthreads();
  const int k = kk;
  select_store<T, NT>(m, s, j, k, vload, Vt);
  return k;
}

// The kept space when the relative cut alone decides (no chi_max or
// physical bound binding): the k given columns from vload, and the discarded
// fraction wgt of the trace into the fidelity.
template <typename T, int NT, typename VF>
__device__ int select_fixed(const MpsDev &m, int s, int j, int k, double wgt, VF vload, cplx<T> *Vt) {
  if (threadIdx.x == 0) {
    m.fid[s] *= (1.0 - wgt);
    auxp(m, s)[2] = k;
    auxp(m, s)[3] = wbd(m, s)[j];
  }
  select_store<T, NT>(m, s, j, k, vload, Vt);
  return k;
}
// The sorted eigenvalues in m.ev, the eigenvectors in V (ld nn).
template <typename T, int NT>
__device__ int select_body(const MpsDev &m, int s, int j, const c64 *V, cplx<T> *Vt) {
  const int nn = 2 * wbd(m, s)[j + 1];
  return select_core<T, NT>(m, s, j, m.ev + s * m.ev_cap, [&](int i, int c) { return V[(size_t)i * nn + c]; }, Vt);
}

// Centre at l: normalise X (wb[l], 2, wb[l+1]) in FP64 into slot l;
// bond[l+1] = wb[l+1]; nrm[s] = the squared norm before normalisation.
template <typename T, int NT>
__device__ void finish_body(const MpsDev &m, int s, int l, const cplx<T> *X) {
  int *w = wbd(m, s);
  const int cnt = w[l] * 2 * w[l + 1];
  double part = 0;
  blk_each<NT, 4, double>(cnt, [&](int e) { return norm2(cvt<double>(X[e])); }, [&](int, double v) { part += v; });
  const double n2 = bsum<NT>(part);
  if (m.keep_norm ? (isinf(n2) || !(n2 == n2)) : (!(n2 > 0) || isinf(n2))) {
    if (threadIdx.x == 0) atomicOr(m.err, STN_ERR_NUMERIC);
    __syncthreads();
    return;
  }
  const double inv = m.keep_norm ? 1.0 : 1.0 / sqrt(n2);
  cplx<T> *out = slot<T>(m, l, s);
  blk_each<NT, 4, cplx<T>>(cnt, [&](int e) { return X[e]; },
                           [&](int e, cplx<T> v) { out[e] = cvt<T>(inv * cvt<double>(v)); });
  if (threadIdx.x == 0) {
    bnd(m, s)[l + 1] = w[l + 1];
    m.nrm[s] = n2;
  }
  __syncthreads();
}

// ------------------------------------------------- Pauli site operators
__device__ inline void site_op(int x, int z, c64 *o) {
  // i^(xz) X^x Z^z
  if (!x && !z) { o[0] = mk<double>(1, 0); o[1] = mk<double>(0, 0); o[2] = mk<double>(0, 0); o[3] = mk<double>(1, 0); }
  if (!x && z) { o[0] = mk<double>(1, 0); o[1] = mk<double>(0, 0); o[2] = mk<double>(0, 0); o[3] = mk<double>(-1, 0); }
  if (x && !z) { o[0] = mk<double>(0, 0); o[1] = mk<double>(1, 0); o[2] = mk<double>(1, 0); o[3] = mk<double>(0, 0); }
  if (x && z) { o[0] = mk<double>(0, 0); o[1] = mk<double>(0, -1); o[2] = mk<double>(0, 1); o[3] = mk<double>(0, 0); }
}
__device__ inline int bitw(const uint64_t *v, int j) { return (int)((v[j >> 6] >> (j & 63)) & 1ull); }

}  // namespace stnk
