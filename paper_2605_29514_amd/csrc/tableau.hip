// Bit-packed inverse-tableau kernels (Sec. IV.A: Clifford gates update C,
// Paulis are commuted through C).
//
// Row q = C^dag X_q C, row n+q = C^dag Z_q C.  Each row is a Pauli string
// (x, z, sign) meaning (-1)^sign * prod_j i^(x_j z_j) X^x_j Z^z_j.  The x/z
// bits are shared by every shot of a batch (they depend on the circuit
// only); the sign is per shot and stored bit-sliced: bit (s % 64) of word
// (s / 64).  A product of rows therefore costs one popcount phase on the
// shared bits plus an XOR of sign words, 64 shots per instruction.
#include "common.h"

namespace {

// Phase exponent (mod 4) of a*b for phase-free strings a, b:
//   sum_j x1 z1 + x2 z2 - x3 z3 + 2 z1 x2   with x3 = x1^x2, z3 = z1^z2.
__device__ inline int mul_phase(const uint64_t *ax, const uint64_t *az, const uint64_t *bx,
                                const uint64_t *bz, int W) {
  int e = 0;
  for (int w = 0; w < W; ++w) {
    uint64_t x3 = ax[w] ^ bx[w], z3 = az[w] ^ bz[w];
    e += __popcll(ax[w] & az[w]) + __popcll(bx[w] & bz[w]) - __popcll(x3 & z3) +
         2 * __popcll(az[w] & bx[w]);
  }
  return e & 3;
}

constexpr int kMaxW = 16;      // n <= 1024

// Shared-bit part of a row product: bits of prod src[i] and the shot-independent
// phase; returns the phase exponent (even for a valid product of rows).
__device__ inline int product_bits(const uint64_t *X, const uint64_t *Z, int W, const RowProg &p,
                                   uint64_t *ox, uint64_t *oz) {
  for (int w = 0; w < W; ++w) { ox[w] = 0; oz[w] = 0; }
  int e = p.e0;
  for (int i = 0; i < p.nsrc; ++i) {
    const uint64_t *sx = X + (size_t)p.src[i] * W, *sz = Z + (size_t)p.src[i] * W;
    e += mul_phase(ox, oz, sx, sz, W);
    for (int w = 0; w < W; ++w) { ox[w] ^= sx[w]; oz[w] ^= sz[w]; }
  }
  return e & 3;
}

// One block per gate of a layer of disjoint gates.  The gate's instructions
// only read and write rows of its own qubits, so staging those rows in LDS
// before writing makes the in-place update race-free across blocks.
__global__ void k_tab_gates(TabDev t, ProgBatch b, int *err) {
  const int g = blockIdx.x;
  const RowProg *prog = b.p;
  const int p0 = b.first[g], np = b.first[g + 1] - b.first[g];
  __shared__ uint64_t sx[4][kMaxW], sz[4][kMaxW];
  __shared__ int sflip[4];
  __shared__ int rows[4];
  // distinct rows touched by this gate = the destinations of its programs
  if (threadIdx.x < np) rows[threadIdx.x] = prog[p0 + threadIdx.x].dst;
  __syncthreads();
  // new bits and constant phases, computed from the old rows
  if (threadIdx.x < np) {
    RowProg p = prog[p0 + threadIdx.x];
    int e = product_bits(t.x, t.z, t.W, p, sx[threadIdx.x], sz[threadIdx.x]);
    if (e & 1) atomicOr(err, STN_ERR_PHASE);
    sflip[threadIdx.x] = e >> 1;
  }
  // per-shot signs: XOR of the source sign words
  extern __shared__ uint64_t ssign[];   // [np][SW]
  for (int i = 0; i < np; ++i) {
    RowProg p = prog[p0 + i];
    for (int w = threadIdx.x; w < t.SW; w += blockDim.x) {
      uint64_t acc = 0;
      for (int k = 0; k < p.nsrc; ++k) acc ^= t.s[(size_t)p.src[k] * t.SW + w];
      ssign[i * t.SW + w] = acc;
    }
  }
  __syncthreads();
  for (int i = 0; i < np; ++i) {
    const int dst = rows[i];
    const uint64_t f = sflip[i] ? ~0ull : 0ull;
    for (int w = threadIdx.x; w < t.SW; w += blockDim.x) t.s[(size_t)dst * t.SW + w] = ssign[i * t.SW + w] ^ f;
    for (int w = threadIdx.x; w < t.W; w += blockDim.x) {
      t.x[(size_t)dst * t.W + w] = sx[i][w];
      t.z[(size_t)dst * t.W + w] = sz[i][w];
    }
  }
}

// Per-shot Pauli noise: X on q flips the sign of row Z_q, Z on q flips row X_q.
__global__ void k_tab_noise(TabDev t, const uint64_t *noise) {
  const int q = blockIdx.x;
  const uint64_t *nx = noise + (size_t)q * t.SW;
  const uint64_t *nz = noise + (size_t)(t.n + q) * t.SW;
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) {
    t.s[(size_t)(t.n + q) * t.SW + w] ^= nx[w];
    t.s[(size_t)q * t.SW + w] ^= nz[w];
  }
}

// Products of rows written to separate outputs (the rewrite P' = C^dag P C of
// a crosstalk string P = Z_a Z_b [Z_c], Sec. IV.A): bits [i][2][W], signs [i][SW].
__global__ void k_tab_products(TabDev t, ProgBatch b, uint64_t *obits, uint64_t *osign,
                               int *err) {
  const int i = blockIdx.x;
  RowProg p = b.p[i];
  __shared__ int sflip;
  if (threadIdx.x == 0) {
    uint64_t bx[kMaxW], bz[kMaxW];
    int e = product_bits(t.x, t.z, t.W, p, bx, bz);
    if (e & 1) atomicOr(err, STN_ERR_PHASE);
    sflip = e >> 1;
    for (int w = 0; w < t.W; ++w) {
      obits[((size_t)i * 2 + 0) * t.W + w] = bx[w];
      obits[((size_t)i * 2 + 1) * t.W + w] = bz[w];
    }
  }
  __syncthreads();
  const uint64_t f = sflip ? ~0ull : 0ull;
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) {
    uint64_t acc = f;
    for (int k = 0; k < p.nsrc; ++k) acc ^= t.s[(size_t)p.src[k] * t.SW + w];
    osign[(size_t)i * t.SW + w] = acc;
  }
}

__device__ inline int getb(const uint64_t *v, int j) { return (int)((v[j >> 6] >> (j & 63)) & 1ull); }
__device__ inline void putb(uint64_t *v, int j, int b) {
  uint64_t m = 1ull << (j & 63);
  v[j >> 6] = b ? (v[j >> 6] | m) : (v[j >> 6] & ~m);
}

// Frame change after a measurement whose Pauli P' = sigma * Q has an X/Y
// site: C <- C V, V = D_k * prod_{j != k} C-Q_j(k -> j) * H_k, every row
// r <- V^dag r V.  k = first X/Y site of Q, D_k = diag(1, s sigma alpha) with
// alpha = 1 (X at k) or i (Y at k); negmask marks shots with s*sigma = -1.
// tables: [0] = H (4 entries), [1..3] = CX, CY, CZ (16 entries); each entry
// packs the conjugated bits (low nibble) and the phase exponent (high nibble).
__global__ void k_tab_frame(TabDev t, const uint64_t *snap, const uint64_t *negmask,
                            const uint8_t *tables) {
  const int row = blockIdx.x;
  const uint64_t *px = snap, *pz = snap + t.W;
  __shared__ uint64_t rx[kMaxW], rz[kMaxW];
  __shared__ int k, alpha_i, xk_old, zk_old, cflip;
  if (threadIdx.x == 0) {
    k = -1;
    for (int w = 0; w < t.W && k < 0; ++w)
      if (px[w]) k = w * 64 + __ffsll((unsigned long long)px[w]) - 1;
    for (int w = 0; w < t.W; ++w) { rx[w] = t.x[(size_t)row * t.W + w]; rz[w] = t.z[(size_t)row * t.W + w]; }
    alpha_i = getb(pz, k);
    xk_old = getb(rx, k);
    zk_old = getb(rz, k);
    int e = 0;
    if (alpha_i) putb(rz, k, zk_old ^ xk_old);       // S or S^dag: z_k ^= x_k
    for (int w = 0; w < t.W; ++w) {
      uint64_t m = px[w] | pz[w];
      while (m) {
        int j = w * 64 + __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        if (j == k) continue;
        int gate = getb(px, j) ? (getb(pz, j) ? 2 : 1) : 3;   // CX / CY / CZ
        int idx = getb(rx, k) | (getb(rz, k) << 1) | (getb(rx, j) << 2) | (getb(rz, j) << 3);
        uint8_t ent = tables[gate * 16 + idx];
        putb(rx, k, ent & 1); putb(rz, k, (ent >> 1) & 1);
        putb(rx, j, (ent >> 2) & 1); putb(rz, j, (ent >> 3) & 1);
        e += ent >> 4;
      }
    }
    {
      int idx = getb(rx, k) | (getb(rz, k) << 1);
      uint8_t ent = tables[idx];
      putb(rx, k, ent & 1); putb(rz, k, (ent >> 1) & 1);
      e += ent >> 4;
    }
    cflip = (e >> 1) & 1;       // e is even for Hermitian rows
    for (int w = 0; w < t.W; ++w) { t.x[(size_t)row * t.W + w] = rx[w]; t.z[(size_t)row * t.W + w] = rz[w]; }
  }
  __syncthreads();
  const uint64_t cf = cflip ? ~0ull : 0ull;
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) {
    uint64_t neg = negmask[w];
    uint64_t d = 0;
    if (xk_old) d = alpha_i ? (zk_old ? neg : ~neg) : neg;
    t.s[(size_t)row * t.SW + w] ^= d ^ cf;
  }
}

__global__ void k_tab_flip(TabDev t, int row, const uint64_t *mask) {
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) t.s[(size_t)row * t.SW + w] ^= mask[w];
}

__global__ void k_tab_snapshot(TabDev t, int row, uint64_t *snap) {
  for (int w = threadIdx.x; w < t.W; w += blockDim.x) {
    snap[w] = t.x[(size_t)row * t.W + w];
    snap[t.W + w] = t.z[(size_t)row * t.W + w];
  }
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) snap[2 * t.W + w] = t.s[(size_t)row * t.SW + w];
}

// Identity frame: row j (X_j) has x bit j, row n + j (Z_j) has z bit j, all
// signs +; also clears the device error word.  One block per row.
__global__ void k_tab_reset(TabDev t, int *err) {
  const int row = blockIdx.x;
  const int q = row < t.n ? row : row - t.n;
  for (int w = threadIdx.x; w < t.W; w += blockDim.x) {
    const uint64_t bit = (w == (q >> 6)) ? (1ull << (q & 63)) : 0ull;
    t.x[(size_t)row * t.W + w] = row < t.n ? bit : 0ull;
    t.z[(size_t)row * t.W + w] = row < t.n ? 0ull : bit;
  }
  for (int w = threadIdx.x; w < t.SW; w += blockDim.x) t.s[(size_t)row * t.SW + w] = 0ull;
  if (row == 0 && threadIdx.x == 0) *err = 0;
}

}  // namespace

void launch_tab_reset(const TabDev &t, int *d_err, hipStream_t st) {
  KLAUNCH(K_TABLEAU, k_tab_reset, dim3(2 * t.n), dim3(64), 0, st, t, d_err);
}

void launch_tab_gates(const TabDev &t, const ProgBatch &b, int *d_err, hipStream_t st) {
  if (b.ngates <= 0) return;
  size_t lds = (size_t)4 * t.SW * sizeof(uint64_t);
  KLAUNCH(K_TABLEAU, k_tab_gates, dim3(b.ngates), dim3(64), lds, st, t, b, d_err);
}

void launch_tab_noise(const TabDev &t, const uint64_t *d_noise, hipStream_t st) {
  KLAUNCH(K_TABLEAU, k_tab_noise, dim3(t.n), dim3(64), 0, st, t, d_noise);
}

void launch_tab_products(const TabDev &t, const ProgBatch &b, uint64_t *d_out_bits,
                         uint64_t *d_out_sign, int *d_err, hipStream_t st) {
  if (b.n <= 0) return;
  KLAUNCH(K_TABLEAU, k_tab_products, dim3(b.n), dim3(64), 0, st, t, b, d_out_bits, d_out_sign, d_err);
}

void launch_tab_frame(const TabDev &t, const uint64_t *d_snap, const uint64_t *d_negmask,
                      const uint8_t *d_tables, hipStream_t st) {
  KLAUNCH(K_TABLEAU, k_tab_frame, dim3(2 * t.n), dim3(64), 0, st, t, d_snap, d_negmask, d_tables);
}

void launch_tab_flip(const TabDev &t, int row, const uint64_t *d_mask, hipStream_t st) {
  KLAUNCH(K_TABLEAU, k_tab_flip, dim3(1), dim3(64), 0, st, t, row, d_mask);
}

void launch_tab_snapshot(const TabDev &t, int row, uint64_t *d_snap, hipStream_t st) {
  KLAUNCH(K_TABLEAU, k_tab_snapshot, dim3(1), dim3(64), 0, st, t, row, d_snap);
}
