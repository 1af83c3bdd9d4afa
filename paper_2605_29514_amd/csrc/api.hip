// libstn host side: context, workspace layout, launch planning and the C ABI
// declared in include/stn.h.
//
// Planning: the x/z bits of the tableau depend on the circuit only (never on
// the shot), so the host keeps a copy of them, updated by the same gate rules
// as the device, to know each step's span [l, r] and whether a measurement
// needs a frame change before launching.  Every result (signs, bits used by
// the kernels, the MPS, outcomes, probabilities) is computed on the device.
#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stn.h"
#include "common.h"

namespace {

using cd = std::complex<double>;

// ------------------------------------------------ Pauli conjugation tables
// For a gate G on k qubits and each local Pauli P = prod i^(x z) X^x Z^z
// (index x0 | z0<<1 | x1<<2 | z1<<3, qubit 0 = first operand), G^dag P G =
// i^de P'.  Entry byte = bits(P') | de << 4.  Built from the gate matrices.
struct Mat {
  int d;
  cd a[16];
  cd &at(int i, int j) { return a[i * d + j]; }
  cd at(int i, int j) const { return a[i * d + j]; }
};

Mat mul(const Mat &x, const Mat &y) {
  Mat r{x.d, {}};
  for (int i = 0; i < x.d; ++i)
    for (int j = 0; j < x.d; ++j) {
      cd s = 0;
      for (int k = 0; k < x.d; ++k) s += x.at(i, k) * y.at(k, j);
      r.at(i, j) = s;
    }
  return r;
}
Mat dag(const Mat &x) {
  Mat r{x.d, {}};
  for (int i = 0; i < x.d; ++i)
    for (int j = 0; j < x.d; ++j) r.at(i, j) = std::conj(x.at(j, i));
  return r;
}
Mat kron(const Mat &x, const Mat &y) {
  Mat r{x.d * y.d, {}};
  for (int i = 0; i < x.d; ++i)
    for (int j = 0; j < x.d; ++j)
      for (int k = 0; k < y.d; ++k)
        for (int l = 0; l < y.d; ++l) r.at(i * y.d + k, j * y.d + l) = x.at(i, j) * y.at(k, l);
  return r;
}
Mat pauli1(int x, int z) {
  const cd I(0, 1);
  Mat m{2, {}};
  if (!x && !z) { m.at(0, 0) = 1; m.at(1, 1) = 1; }
  if (x && !z) { m.at(0, 1) = 1; m.at(1, 0) = 1; }
  if (!x && z) { m.at(0, 0) = 1; m.at(1, 1) = -1; }
  if (x && z) { m.at(0, 1) = -I; m.at(1, 0) = I; }   // i X Z = Y
  return m;
}
Mat pauli_idx(int k, int idx) {
  Mat m = pauli1(idx & 1, (idx >> 1) & 1);
  if (k == 2) m = kron(m, pauli1((idx >> 2) & 1, (idx >> 3) & 1));
  return m;
}
Mat gate_matrix(int kind) {
  const double r = 1.0 / std::sqrt(2.0);
  const cd I(0, 1);
  Mat m{2, {}};
  switch (kind) {
    case STN_GATE_H: m.at(0, 0) = r; m.at(0, 1) = r; m.at(1, 0) = r; m.at(1, 1) = -r; return m;
    case STN_GATE_S: m.at(0, 0) = 1; m.at(1, 1) = I; return m;
    case STN_GATE_SDG: m.at(0, 0) = 1; m.at(1, 1) = -I; return m;
    case STN_GATE_X: return pauli1(1, 0);
    case STN_GATE_Y: return pauli1(1, 1);
    case STN_GATE_Z: return pauli1(0, 1);
    default: break;
  }
  Mat u = kind == STN_GATE_CX ? pauli1(1, 0) : kind == STN_GATE_CY ? pauli1(1, 1) : pauli1(0, 1);
  Mat c{4, {}};
  c.at(0, 0) = 1; c.at(1, 1) = 1;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) c.at(2 + i, 2 + j) = u.at(i, j);
  return c;
}
bool is_two(int kind) { return kind >= STN_GATE_CX; }

void build_table(int kind, uint8_t *out) {
  Mat g = gate_matrix(kind);
  int k = g.d == 4 ? 2 : 1;
  int cnt = 1 << (2 * k);
  for (int idx = 0; idx < cnt; ++idx) {
    Mat m = mul(mul(dag(g), pauli_idx(k, idx)), g);
    out[idx] = 0xff;
    for (int o = 0; o < cnt; ++o) {
      Mat p = pauli_idx(k, o);
      cd tr = 0;
      for (int i = 0; i < g.d; ++i)
        for (int j = 0; j < g.d; ++j) tr += std::conj(p.at(j, i)) * m.at(j, i);
      tr /= (double)g.d;
      if (std::abs(tr) > 0.5) {
        int de = (int)std::lround(std::arg(tr) / (M_PI / 2));
        de = ((de % 4) + 4) % 4;
        out[idx] = (uint8_t)(o | (de << 4));
      }
    }
  }
}

inline int getbit(const uint64_t *v, int j) { return (int)((v[j >> 6] >> (j & 63)) & 1ull); }
inline void setbit(uint64_t *v, int j, int b) {
  uint64_t m = 1ull << (j & 63);
  v[j >> 6] = b ? (v[j >> 6] | m) : (v[j >> 6] & ~m);
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

thread_local Prof *g_prof = nullptr;

// ------------------------------------------------------------ static tape
// Gradient tape in the library's own device memory, for callers that cannot
// allocate device memory (code under HIP-graph capture, serving loops,
// harnesses that forbid allocation): stn_tape_begin_static.  One copy per
// GPU, loaded with the code object and held until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device array:
// every use goes through the per-device address hipGetSymbolAddress returns
// (scratch_ptr below), looked up once per device at stn_init.
constexpr size_t kStaticTapeBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticTapeBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's static tape (nullptr when unavailable); the
// current device must be the context's.
char *scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_scratch_ptr[dev] = reinterpret_cast<char *>(p);
    g_scratch_done[dev] = true;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

hipEvent_t Prof::get() {
  if (used == pool.size()) {
    hipEvent_t e;
    hipEventCreate(&e);
    pool.push_back(e);
  }
  return pool[used++];
}

struct stn_ctx {
  stn_config cfg{};
  int n = 0, S = 0, chi = 0, prec = 0, W = 0, SW = 0;
  size_t esz = 0;
  hipStream_t st = nullptr;
  TabDev tab{};
  MpsDev mps{};
  uint64_t *d_pbits = nullptr, *d_psgn = nullptr, *d_snap = nullptr, *d_negmask = nullptr,
           *d_mmask = nullptr;
  uint8_t *d_tables = nullptr;
  c64 *d_ops = nullptr, *d_eops = nullptr;
  int *d_err = nullptr;
  int center = 0;
  int layer_mode = 0;              // 0 auto, 1 per-step kernels, 2 fused per-shot layer kernel
  int layer_threads = 128;         // threads per shot of the fused kernel
  char *static_tape = nullptr;     // this device's static tape array (stn_tape_begin_static)
  std::vector<uint64_t> hx, hz;    // shadow of the shared bits
  uint8_t tables[9][16];           // per gate kind
  std::string err;
  Prof prof;
  double prof_ms[K_COUNT] = {};
  long long prof_launches[K_COUNT] = {};
  // gradient tape: one record per non-Clifford step, each holding the
  // pre-step state and the per-shot data of the step; one more snapshot
  // after the last step
  struct TapeStep { int kind, l, r, pivot, rot; };   // kind 0 rotation, 1 measurement
  bool taping = false, tape_closed = false;
  char *tape = nullptr;
  int tape_max = 0;
  std::vector<TapeStep> steps;
  int tape_rot = 0;
  // adjoint state
  MpsDev adj{};
  bool adj_ready = false;
  int adj_center = 0;
  ~stn_ctx() {
    for (auto e : prof.pool) hipEventDestroy(e);
  }
};

// Makes the context's recorder visible to the launchers for one API call.
struct ProfScope {
  explicit ProfScope(stn_ctx *c) { g_prof = (c && c->prof.mask) ? &c->prof : nullptr; }
  ~ProfScope() { g_prof = nullptr; }
};

namespace {

constexpr int kRotChunk = kProgBatch;

struct Layout {
  size_t total = 0;
  size_t off(size_t bytes) {
    size_t o = total;
    total = align_up(total + bytes);
    return o;
  }
};

int dmax_h(int n, int chi, int b) {
  int e = b < n - b ? b : n - b;
  long phys = e >= 30 ? (1L << 30) : (1L << e);
  return (int)(phys < chi ? phys : chi);
}

// Lays out one batch of MPS (slots, workspace slots for bonds up to wmul x
// the cap, bonds, per-shot scratch) in L; fills m when base != nullptr and
// returns the host copy of the slot offset tables (site_off, site_cap,
// ws_off, ws_cap) in offs, which the caller uploads.
void plan_mps(Layout &L, int n, int S, int chi, size_t esz, int wmul, char *base, MpsDev *mp,
              std::vector<int64_t> *offs) {
  std::vector<int64_t> site_off(n), site_cap(n), ws_off(n), ws_cap(n);
  int64_t so = 0, wo = 0, Tcap = 1;
  for (int j = 0; j < n; ++j) {
    int64_t dl = dmax_h(n, chi, j), dr = dmax_h(n, chi, j + 1);
    site_cap[j] = dl * 2 * dr;
    site_off[j] = so;
    so += site_cap[j] * S;
    ws_cap[j] = (wmul * dl) * 2 * (wmul * dr);
    ws_off[j] = wo;
    wo += ws_cap[j] * S;
    Tcap = std::max<int64_t>(Tcap, ws_cap[j]);
  }
  int64_t chi_eff = 1;
  for (int b = 0; b <= n; ++b) chi_eff = std::max<int64_t>(chi_eff, dmax_h(n, chi, b));
  const int64_t nn = 2 * chi_eff;
  size_t o_soff = L.off((size_t)n * 8), o_scap = L.off((size_t)n * 8), o_woff = L.off((size_t)n * 8),
         o_wcap = L.off((size_t)n * 8);
  size_t o_bond = L.off((size_t)S * (n + 1) * 4), o_wb = L.off((size_t)S * (n + 1) * 4),
         o_aux = L.off((size_t)S * 8 * 4);
  size_t o_logp = L.off((size_t)S * 8), o_fid = L.off((size_t)S * 8), o_p0 = L.off((size_t)S * 8),
         o_nrm = L.off((size_t)S * 8), o_pm = L.off((size_t)S * 8), o_tr = L.off((size_t)S * 4),
         o_coef = L.off((size_t)S * 2 * sizeof(c64));
  size_t o_mps = L.off((size_t)so * esz), o_ws = L.off((size_t)wo * esz);
  size_t o_T = L.off((size_t)Tcap * S * esz), o_R = L.off((size_t)Tcap * S * esz);
  size_t o_N = L.off((size_t)wmul * chi_eff * chi_eff * S * esz), o_Vt = L.off((size_t)nn * chi_eff * S * esz);
  size_t o_G = L.off((size_t)nn * nn * S * sizeof(c64)), o_V = L.off((size_t)nn * nn * S * sizeof(c64));
  size_t o_ev = L.off((size_t)nn * S * 8);
  size_t o_E = L.off((size_t)chi_eff * chi_eff * S * sizeof(c64)),
         o_F = L.off((size_t)chi_eff * 2 * chi_eff * S * sizeof(c64));
  const int64_t Jcap = (int64_t)align_up(layer_fallback_bytes((int)chi_eff));
  size_t o_J = L.off((size_t)Jcap * S);
  // environment path of the fused kernel (forward state only): one Gram per
  // site of a span for doubled bonds up to eb
  // doubled bonds up to eb (the product scratch F = E B is eb x 2 eb); the
  // packed Grams of a span share a store of n x ec^2 per shot, ec lowered in steps of 32
  // (down to 32) until every shot's store fits the memory budget
  int64_t eb = wmul == 2 ? std::min<int64_t>(kEnvBond, 2 * chi_eff) : 0;
  while (eb > 64 && (size_t)S * eb * 2 * eb * sizeof(c64) > kEnvFBudget) eb /= 2;
  int64_t ec = std::min<int64_t>(eb, kEnvStore);
  while (ec > 32 && (size_t)S * n * ec * ec * sizeof(c64) > kEnvBudget) ec -= 32;
  const int64_t Escap = (int64_t)n * ec * ec, Fscap = eb * 2 * eb;
  size_t o_Es = L.off((size_t)Escap * S * sizeof(c64)), o_Fs = L.off((size_t)Fscap * S * sizeof(c64));
  if (base) {
    MpsDev &m = *mp;
    m.n = n; m.S = S; m.chi = chi;
    m.site_off = (int64_t *)(base + o_soff); m.site_cap = (int64_t *)(base + o_scap);
    m.ws_off = (int64_t *)(base + o_woff); m.ws_cap = (int64_t *)(base + o_wcap);
    m.mps = base + o_mps; m.ws = base + o_ws;
    m.bond = (int *)(base + o_bond); m.wb = (int *)(base + o_wb); m.aux = (int *)(base + o_aux);
    m.T = base + o_T; m.T_cap = Tcap;
    m.R = base + o_R; m.R_cap = Tcap;
    m.N = base + o_N; m.N_cap = wmul * chi_eff * chi_eff;
    m.Vt = base + o_Vt; m.Vt_cap = nn * chi_eff;
    m.G = (c64 *)(base + o_G); m.G_cap = nn * nn;
    m.V = (c64 *)(base + o_V); m.V_cap = nn * nn;
    m.ev = (double *)(base + o_ev); m.ev_cap = nn;
    m.E = (c64 *)(base + o_E); m.E_cap = chi_eff * chi_eff;
    m.F = (c64 *)(base + o_F); m.F_cap = chi_eff * 2 * chi_eff;
    m.J = base + o_J; m.J_cap = Jcap;
    m.Es = (c64 *)(base + o_Es); m.Es_cap = Escap;
    m.Fs = (c64 *)(base + o_Fs); m.Fs_cap = Fscap;
    m.ebond = (int)eb;
    m.ebond_alloc = (int)eb;
    m.logp = (double *)(base + o_logp); m.fid = (double *)(base + o_fid);
    m.p0 = (double *)(base + o_p0); m.nrm = (double *)(base + o_nrm);
    m.pm = (double *)(base + o_pm); m.trunc = (int *)(base + o_tr);
    m.coef = (c64 *)(base + o_coef);
    m.wmul = wmul;
    m.keep_norm = 0;
    m.prof = 0;
    m.lds_order = 0;
  }
  if (offs) {
    offs->clear();
    for (auto *v : {&site_off, &site_cap, &ws_off, &ws_cap}) offs->insert(offs->end(), v->begin(), v->end());
  }
}

// Bytes of the MPS slots of one batch (the part a state snapshot copies).
size_t mps_slot_bytes(int n, int S, int chi, size_t esz) {
  size_t so = 0;
  for (int j = 0; j < n; ++j) so += (size_t)dmax_h(n, chi, j) * 2 * dmax_h(n, chi, j + 1) * S;
  return so * esz;
}

// Computes the workspace layout; when base != nullptr also fills ctx pointers.
size_t plan(const stn_config &c, stn_ctx *ctx, char *base, std::vector<int64_t> *offs) {
  const int n = c.n_qubits, S = c.n_shots, chi = c.chi_max;
  const int W = (n + 63) / 64, SW = (S + 63) / 64;
  const size_t esz = c.precision == STN_FP64 ? 16 : 8;
  Layout L;
  size_t o_x = L.off((size_t)2 * n * W * 8), o_z = L.off((size_t)2 * n * W * 8);
  size_t o_s = L.off((size_t)2 * n * SW * 8);
  size_t o_pbits = L.off((size_t)kRotChunk * 2 * W * 8), o_psgn = L.off((size_t)kRotChunk * SW * 8);
  size_t o_snap = L.off((size_t)(2 * W + SW) * 8);
  size_t o_neg = L.off((size_t)SW * 8), o_mm = L.off((size_t)SW * 8);
  size_t o_tab = L.off(64);
  size_t o_ops = L.off((size_t)n * 8 * sizeof(c64)), o_eops = L.off((size_t)n * 4 * sizeof(c64));
  size_t o_err = L.off(4);
  size_t o_work = L.off((size_t)kWorkWords * 8);
  MpsDev *mp = ctx && base ? &ctx->mps : nullptr;
  plan_mps(L, n, S, chi, esz, 2, base && ctx ? base : nullptr, mp, offs);
  if (ctx && base) {
    ctx->n = n; ctx->S = S; ctx->chi = chi; ctx->prec = c.precision; ctx->W = W; ctx->SW = SW;
    ctx->esz = esz;
    ctx->tab = TabDev{n, W, SW, (uint64_t *)(base + o_x), (uint64_t *)(base + o_z), (uint64_t *)(base + o_s)};
    ctx->d_pbits = (uint64_t *)(base + o_pbits);
    ctx->d_psgn = (uint64_t *)(base + o_psgn);
    ctx->d_snap = (uint64_t *)(base + o_snap);
    ctx->d_negmask = (uint64_t *)(base + o_neg);
    ctx->d_mmask = (uint64_t *)(base + o_mm);
    ctx->d_tables = (uint8_t *)(base + o_tab);
    ctx->d_ops = (c64 *)(base + o_ops);
    ctx->d_eops = (c64 *)(base + o_eops);
    ctx->d_err = (int *)(base + o_err);
    MpsDev &m = ctx->mps;
    m.err = ctx->d_err;
    m.eps_cut = c.eps_cut;
    m.work = (double *)(base + o_work);
  }
  return L.total;
}

bool valid(const stn_config *c) {
  return c && c->n_qubits >= 1 && c->n_qubits <= 1024 && c->n_shots >= 1 && c->chi_max >= 1 &&
         c->chi_max <= 1024 && (c->precision == STN_FP64 || c->precision == STN_FP32) &&
         c->eps_cut >= 0 && c->eps_cut < 1;
}

stn_status fail(stn_ctx *ctx, stn_status s, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return s;
}

stn_status check_launch(stn_ctx *ctx) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  return STN_OK;
}

stn_status sync_status(stn_ctx *ctx) {
  hipError_t e = hipStreamSynchronize(ctx->st);
  if (e != hipSuccess) return fail(ctx, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  int flags = 0;
  e = hipMemcpy(&flags, ctx->d_err, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(ctx, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  if (flags & STN_ERR_ZEROPROB) return fail(ctx, STN_EZEROPROB, "forced outcome with probability 0");
  if (flags & STN_ERR_NUMERIC) return fail(ctx, STN_ENUMERIC, "non-finite value in the state or the angles");
  if (flags & STN_ERR_PHASE) return fail(ctx, STN_ENUMERIC, "tableau row product with an imaginary phase");
  if (flags & STN_ERR_EIGEN) return fail(ctx, STN_ENUMERIC, "Jacobi eigen-solve did not converge");
  return STN_OK;
}

// ----------------------------------------------------- host shadow updates
void shadow_product(stn_ctx *c, const RowProg &p, uint64_t *ox, uint64_t *oz) {
  for (int w = 0; w < c->W; ++w) { ox[w] = 0; oz[w] = 0; }
  for (int i = 0; i < p.nsrc; ++i)
    for (int w = 0; w < c->W; ++w) {
      ox[w] ^= c->hx[(size_t)p.src[i] * c->W + w];
      oz[w] ^= c->hz[(size_t)p.src[i] * c->W + w];
    }
}

// Row programs of one gate: each generator row of the support becomes
// i^e0 * product of old rows (G^dag g G expressed in generators).
int gate_programs(stn_ctx *c, const stn_gate &g, RowProg *out) {
  const int k = is_two(g.kind) ? 2 : 1;
  const int q[2] = {g.q0, g.q1};
  int np = 0;
  for (int i = 0; i < k; ++i)
    for (int which = 0; which < 2; ++which) {            // 0: X_q, 1: Z_q
      int idx = which == 0 ? (1 << (2 * i)) : (2 << (2 * i));
      uint8_t ent = c->tables[g.kind][idx];
      int bits = ent & 15, de = ent >> 4;
      RowProg p{};
      p.dst = (int16_t)(which == 0 ? q[i] : c->n + q[i]);
      p.e0 = (int16_t)de;
      for (int s = 0; s < k; ++s) {
        int x = (bits >> (2 * s)) & 1, z = (bits >> (2 * s + 1)) & 1;
        if (x) p.src[p.nsrc++] = (int16_t)q[s];
        if (z) p.src[p.nsrc++] = (int16_t)(c->n + q[s]);
        p.e0 = (int16_t)((p.e0 + x * z) & 3);
      }
      out[np++] = p;
    }
  return np;
}

void shadow_apply(stn_ctx *c, const RowProg *progs, int np) {
  std::vector<uint64_t> nx(np * c->W), nz(np * c->W);
  for (int i = 0; i < np; ++i) shadow_product(c, progs[i], &nx[i * c->W], &nz[i * c->W]);
  for (int i = 0; i < np; ++i)
    for (int w = 0; w < c->W; ++w) {
      c->hx[(size_t)progs[i].dst * c->W + w] = nx[i * c->W + w];
      c->hz[(size_t)progs[i].dst * c->W + w] = nz[i * c->W + w];
    }
}

// Bits of the frame change V = D_k prod C-Q_j H_k applied to every row.
void shadow_frame(stn_ctx *c, const uint64_t *px, const uint64_t *pz, int k) {
  const int alpha_i = getbit(pz, k);
  for (int row = 0; row < 2 * c->n; ++row) {
    uint64_t *rx = &c->hx[(size_t)row * c->W], *rz = &c->hz[(size_t)row * c->W];
    if (alpha_i) setbit(rz, k, getbit(rz, k) ^ getbit(rx, k));
    for (int j = 0; j < c->n; ++j) {
      if (j == k || !(getbit(px, j) | getbit(pz, j))) continue;
      int kind = getbit(px, j) ? (getbit(pz, j) ? STN_GATE_CY : STN_GATE_CX) : STN_GATE_CZ;
      int idx = getbit(rx, k) | (getbit(rz, k) << 1) | (getbit(rx, j) << 2) | (getbit(rz, j) << 3);
      uint8_t ent = c->tables[kind][idx];
      setbit(rx, k, ent & 1); setbit(rz, k, (ent >> 1) & 1);
      setbit(rx, j, (ent >> 2) & 1); setbit(rz, j, (ent >> 3) & 1);
    }
    int idx = getbit(rx, k) | (getbit(rz, k) << 1);
    uint8_t ent = c->tables[STN_GATE_H][idx];
    setbit(rx, k, ent & 1); setbit(rz, k, (ent >> 1) & 1);
  }
}

void span_of(stn_ctx *c, const uint64_t *px, const uint64_t *pz, int *l, int *r, int *pivot) {
  *l = -1; *r = -1; *pivot = -1;
  for (int j = 0; j < c->n; ++j) {
    if (getbit(px, j) | getbit(pz, j)) {
      if (*l < 0) *l = j;
      *r = j;
    }
    if (*pivot < 0 && getbit(px, j)) *pivot = j;
  }
}

// ----------------------------------------------------- MPS step dispatch
template <typename T>
void move_center_into(stn_ctx *c, int l, int r) {
  while (c->center < l) { mps_move_right<T>(c->mps, c->center, c->st); c->center++; }
  while (c->center > r) { mps_move_left<T>(c->mps, c->center, c->st); c->center--; }
}

// Two-term step over [l, r] with ops/coef already on the device.
template <typename T>
void two_term(stn_ctx *c, int l, int r, bool unitary) {
  if (l == r) {
    if (!unitary) move_center_into<T>(c, l, l);
    mps_apply_single<T>(c->mps, l, c->d_ops, c->st);
    if (!unitary) mps_normalize_site<T>(c->mps, l, c->st);
    return;
  }
  move_center_into<T>(c, l, r);
  mps_build<T>(c->mps, l, r, c->d_ops, c->st);
  mps_sweep_lr<T>(c->mps, l, r, c->st);
  mps_sweep_rl<T>(c->mps, l, r, c->st);
  c->center = l;
}

// ------------------------------------------------------ gradient tape
// Per-step record: pre-step state snapshot (MPS slots, bonds), the Pauli
// bits and signs of P', the outcome mask, and per shot the angle, the
// truncation flag, the squared norm before renormalisation and the outcome
// probability.
struct RecLayout {
  size_t snap_mps, snap_bond, bits, sign, mmask, theta, trunc, nrm, pm, total;
};
RecLayout rec_layout(const stn_ctx *c) {
  Layout L;
  RecLayout r;
  r.snap_mps = L.off(mps_slot_bytes(c->n, c->S, c->chi, c->esz));
  r.snap_bond = L.off((size_t)c->S * (c->n + 1) * 4);
  r.bits = L.off((size_t)2 * c->W * 8);
  r.sign = L.off((size_t)c->SW * 8);
  r.mmask = L.off((size_t)c->SW * 8);
  r.theta = L.off((size_t)c->S * 8);
  r.trunc = L.off((size_t)c->S * 4);
  r.nrm = L.off((size_t)c->S * 8);
  r.pm = L.off((size_t)c->S * 8);
  r.total = L.total;
  return r;
}

MpsDev snapshot_view(const stn_ctx *c, char *rec) {
  const RecLayout R = rec_layout(c);
  MpsDev v = c->mps;
  v.mps = rec + R.snap_mps;
  v.bond = (int *)(rec + R.snap_bond);
  return v;
}

hipError_t take_snapshot(stn_ctx *c, char *rec) {
  const RecLayout R = rec_layout(c);
  hipError_t e = hipMemcpyAsync(rec + R.snap_mps, c->mps.mps, mps_slot_bytes(c->n, c->S, c->chi, c->esz),
                                hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rec + R.snap_bond, c->mps.bond, (size_t)c->S * (c->n + 1) * 4, hipMemcpyDeviceToDevice, c->st);
  return e;
}

// Before a recorded step: snapshot, Pauli data, per-shot flags reset.
stn_status tape_pre(stn_ctx *c, char **rec, const uint64_t *d_bits, const uint64_t *d_sign) {
  if ((int)c->steps.size() >= c->tape_max) return fail(c, STN_ENOMEM, "gradient tape is full");
  const RecLayout R = rec_layout(c);
  char *r = c->tape + c->steps.size() * R.total;
  hipError_t e = take_snapshot(c, r);
  if (e == hipSuccess) e = hipMemcpyAsync(r + R.bits, d_bits, (size_t)2 * c->W * 8, hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess) e = hipMemcpyAsync(r + R.sign, d_sign, (size_t)c->SW * 8, hipMemcpyDeviceToDevice, c->st);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  launch_step_reset(c->mps, c->st);
  *rec = r;
  return STN_OK;
}

stn_status tape_post(stn_ctx *c, char *r, int kind, int l, int rr, int pivot) {
  const RecLayout R = rec_layout(c);
  hipError_t e = hipMemcpyAsync(r + R.trunc, c->mps.trunc, (size_t)c->S * 4, hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess) e = hipMemcpyAsync(r + R.nrm, c->mps.nrm, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess && kind == 1) {
    e = hipMemcpyAsync(r + R.pm, c->mps.pm, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(r + R.mmask, c->d_mmask, (size_t)c->SW * 8, hipMemcpyDeviceToDevice, c->st);
  }
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  c->steps.push_back({kind, l, rr, pivot, kind == 0 ? c->tape_rot++ : -1});
  return STN_OK;
}

template <typename T>
stn_status rotate_impl(stn_ctx *c, const int32_t *qs, int n_rot, const double *theta, int64_t stride) {
  for (int r0 = 0; r0 < n_rot; r0 += kRotChunk) {
    const int cnt = std::min(kRotChunk, n_rot - r0);
    ProgBatch b{};
    b.n = cnt;
    for (int i = 0; i < cnt; ++i) {
      RowProg p{};
      p.dst = -1;
      for (int k = 0; k < 3; ++k) {
        int q = qs[(r0 + i) * 3 + k];
        if (q >= 0) p.src[p.nsrc++] = (int16_t)(c->n + q);
      }
      b.p[i] = p;
    }
    launch_tab_products(c->tab, b, c->d_pbits, c->d_psgn, c->d_err, c->st);
    const bool fused = !c->taping && (c->layer_mode == 2 || (c->layer_mode == 0 && c->S >= 64));
    if (fused) {
      RotLayer L{};
      L.n_rot = cnt;
      L.theta_base = r0;
      L.center_in = c->center;
      for (int i = 0; i < cnt; ++i) {
        std::vector<uint64_t> px(c->W), pz(c->W);
        shadow_product(c, b.p[i], px.data(), pz.data());
        int l, r, piv;
        span_of(c, px.data(), pz.data(), &l, &r, &piv);
        if (l < 0) return fail(c, STN_EINVAL, "rotation Pauli is the identity");
        L.l[i] = (int16_t)l;
        L.r[i] = (int16_t)r;
        if (l != r) c->center = l;     // the kernel leaves the centre at l after a multi-site step
      }
      mps_rot_layer<T>(c->mps, c->d_pbits, c->d_psgn, c->W, c->SW, theta, stride, L, c->layer_threads, c->st);
      continue;
    }
    for (int i = 0; i < cnt; ++i) {
      std::vector<uint64_t> px(c->W), pz(c->W);
      shadow_product(c, b.p[i], px.data(), pz.data());
      int l, r, piv;
      span_of(c, px.data(), pz.data(), &l, &r, &piv);
      if (l < 0) return fail(c, STN_EINVAL, "rotation Pauli is the identity");
      const uint64_t *bits = c->d_pbits + (size_t)i * 2 * c->W;
      char *rec = nullptr;
      if (c->taping) {
        stn_status ts = tape_pre(c, &rec, bits, c->d_psgn + (size_t)i * c->SW);
        if (ts != STN_OK) return ts;
        launch_gather_theta(theta, stride, r0 + i, (double *)(rec + rec_layout(c).theta), c->S, c->st);
      }
      launch_ops_rotation(bits, c->W, l, r, c->d_ops, c->st);
      launch_coef_rotation(c->d_psgn + (size_t)i * c->SW, c->S, theta, stride, r0 + i, c->mps.coef,
                           c->d_err, c->st);
      two_term<T>(c, l, r, true);
      if (c->taping) {
        stn_status ts = tape_post(c, rec, 0, l, r, -1);
        if (ts != STN_OK) return ts;
      }
    }
  }
  return check_launch(c);
}

template <typename T>
stn_status measure_impl(stn_ctx *c, const int32_t *qs, int n_meas, int reset, const double *u,
                        const uint8_t *forced, uint8_t *out, double *prob) {
  for (int i = 0; i < n_meas; ++i) {
    const int q = qs[i];
    const int row = c->n + q;
    std::vector<uint64_t> px(c->hx.begin() + (size_t)row * c->W, c->hx.begin() + (size_t)(row + 1) * c->W);
    std::vector<uint64_t> pz(c->hz.begin() + (size_t)row * c->W, c->hz.begin() + (size_t)(row + 1) * c->W);
    int l, r, piv;
    span_of(c, px.data(), pz.data(), &l, &r, &piv);
    launch_tab_snapshot(c->tab, row, c->d_snap, c->st);
    char *rec = nullptr;
    if (c->taping) {
      stn_status ts = tape_pre(c, &rec, c->d_snap, c->d_snap + 2 * c->W);
      if (ts != STN_OK) return ts;
    }
    launch_ops_measure(c->d_snap, c->W, l, r, piv, c->d_ops, c->d_eops, c->st);
    const bool fused = !c->taping && (c->layer_mode == 2 || (c->layer_mode == 0 && c->S >= 64));
    if (fused) {                     // one per-shot launch: expectation, outcome, projection
      MeasStep a{l, r, piv, c->center, n_meas, i};
      mps_measure_fused<T>(c->mps, c->d_snap + 2 * c->W, c->d_ops, c->d_eops, a, u, forced, out, prob,
                           c->d_negmask, c->d_mmask, c->layer_threads, c->st);
      c->center = l;
    } else {
      move_center_into<T>(c, l, l);
      mps_expect<T>(c->mps, l, r, c->d_eops, c->st);
      launch_outcome(c->mps, c->d_snap + 2 * c->W, piv, r + 1, u, forced, n_meas, i, out, prob,
                     c->d_negmask, c->d_mmask, c->st);
      two_term<T>(c, l, r, false);
    }
    if (c->taping) {
      stn_status ts = tape_post(c, rec, 1, l, r, piv);
      if (ts != STN_OK) return ts;
    }
    if (piv >= 0) {
      launch_tab_frame(c->tab, c->d_snap, c->d_negmask, c->d_tables, c->st);
      shadow_frame(c, px.data(), pz.data(), piv);
    }
    if (reset) launch_tab_flip(c->tab, row, c->d_mmask, c->st);
  }
  return check_launch(c);
}

// ------------------------------------------------------ adjoint pass
template <typename T>
void adj_move_into(stn_ctx *c, int l, int r) {
  while (c->adj_center < l) { mps_move_right<T>(c->adj, c->adj_center, c->st); c->adj_center++; }
  while (c->adj_center > r) { mps_move_left<T>(c->adj, c->adj_center, c->st); c->adj_center--; }
}

// mu <- a O1 mu + b O2 mu over [l, r] (ops and coefficients on the device),
// compressed with its norm kept.
template <typename T>
void adj_two_term(stn_ctx *c, int l, int r) {
  MpsDev &mu = c->adj;
  adj_move_into<T>(c, l, r);
  if (l == r) {
    adj_move_into<T>(c, l, l);
    mps_apply_single<T>(mu, l, c->d_ops, c->st);
    return;
  }
  mps_build<T>(mu, l, r, c->d_ops, c->st);
  mps_sweep_lr<T>(mu, l, r, c->st);
  mps_sweep_rl<T>(mu, l, r, c->st);
  c->adj_center = l;
}

template <typename T>
stn_status backward_impl(stn_ctx *c, double *grad, int64_t stride) {
  const RecLayout R = rec_layout(c);
  const int K = (int)c->steps.size(), S = c->S, n = c->n;
  std::vector<int> tr((size_t)K * S);
  hipError_t e = hipStreamSynchronize(c->st);
  for (int k = 0; k < K && e == hipSuccess; ++k)
    e = hipMemcpy(&tr[(size_t)k * S], c->tape + k * R.total + R.trunc, (size_t)S * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  MpsDev &mu = c->adj;
  for (int k = K - 1; k >= 0; --k) {
    const auto &stp = c->steps[k];
    char *rec = c->tape + k * R.total, *nxt = c->tape + (k + 1) * R.total;
    const MpsDev ph = snapshot_view(c, rec), pa = snapshot_view(c, nxt);
    const uint64_t *bits = (const uint64_t *)(rec + R.bits), *sign = (const uint64_t *)(rec + R.sign);
    const uint64_t *mmask = (const uint64_t *)(rec + R.mmask);
    const double *nrm = (const double *)(rec + R.nrm), *pm = (const double *)(rec + R.pm);
    const int l = stp.l, r = stp.r;
    bool any = false;
    for (int s = 0; s < S; ++s) any = any || tr[(size_t)k * S + s];
    if (any && l < r) {                                 // frozen projection of the step
      adj_move_into<T>(c, l, l);
      mps_project_right<T>(mu, pa, l, (const int *)(rec + R.trunc), c->st);
    }
    if (stp.kind == 0) {                                // mu <- R^dag mu / n
      launch_ops_rotation(bits, c->W, l, r, c->d_ops, c->st);
      launch_adj_coef(mu, 0, -1, (const double *)(rec + R.theta), sign, nullptr, nrm, nullptr, c->st);
    } else {                                            // mu <- M^dag mu / n
      if (stp.pivot < 0) launch_ops_measure(bits, c->W, l, r, -1, c->d_ops, c->d_eops, c->st);
      else launch_ops_measure_adj(bits, c->W, l, r, stp.pivot, c->d_ops, c->st);
      launch_adj_coef(mu, 1, stp.pivot, nullptr, sign, mmask, nrm, nullptr, c->st);
    }
    adj_two_term<T>(c, l, r);
    if (stp.kind == 0) {                                // dJ/dtheta = 2 sigma Im <mu|P'|phi>
      launch_ops_measure(bits, c->W, l, r, -1, c->d_ops, c->d_eops, c->st);
      mps_overlap_grad<T>(mu, ph, c->d_eops, l, r, sign, grad + stp.rot, stride, c->st);
    } else {                                            // mu <- mu + A phi / p - phi
      launch_ops_rotation(bits, c->W, l, r, c->d_ops, c->st);
      launch_adj_coef(mu, 2, stp.pivot, nullptr, sign, mmask, nrm, pm, c->st);
      mps_build_sum<T>(mu, ph, l, r, c->d_ops, c->st);
      mps_sweep_lr<T>(mu, 0, n - 1, c->st);
      mps_sweep_rl<T>(mu, 0, n - 1, c->st);
      c->adj_center = 0;
    }
  }
  return check_launch(c);
}

// Checkpoint of the forward state: MPS slots, bonds, tableau, log P and
// fidelity, and the host shadow of the shared bits with the centre.
struct CkLayout { size_t mps, bond, x, z, s, logp, fid, hx, hz, center, total; };
CkLayout ck_layout(const stn_ctx *c) {
  Layout L;
  CkLayout k;
  k.mps = L.off(mps_slot_bytes(c->n, c->S, c->chi, c->esz));
  k.bond = L.off((size_t)c->S * (c->n + 1) * 4);
  k.x = L.off((size_t)2 * c->n * c->W * 8);
  k.z = L.off((size_t)2 * c->n * c->W * 8);
  k.s = L.off((size_t)2 * c->n * c->SW * 8);
  k.logp = L.off((size_t)c->S * 8);
  k.fid = L.off((size_t)c->S * 8);
  k.hx = L.off((size_t)2 * c->n * c->W * 8);
  k.hz = L.off((size_t)2 * c->n * c->W * 8);
  k.center = L.off(8);
  k.total = L.total;
  return k;
}

}  // namespace

extern "C" {

size_t stn_workspace_bytes(const stn_config *cfg) {
  if (!valid(cfg)) return 0;
  return plan(*cfg, nullptr, nullptr, nullptr);
}

stn_status stn_init(stn_ctx **out, const stn_config *cfg, void *ws, size_t bytes) {
  if (!out || !valid(cfg) || !ws) return STN_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return STN_EINVAL;
  size_t need = plan(*cfg, nullptr, nullptr, nullptr);
  if (bytes < need) return STN_ENOMEM;
  stn_ctx *c = new stn_ctx();
  c->cfg = *cfg;
  c->st = (hipStream_t)cfg->stream;
  std::vector<int64_t> offs;
  plan(*cfg, c, (char *)ws, &offs);
  for (int k = 0; k <= STN_GATE_CZ; ++k) build_table(k, c->tables[k]);
  // frame tables: [0] H, [1] CX, [2] CY, [3] CZ
  uint8_t ft[64];
  memcpy(ft, c->tables[STN_GATE_H], 16);
  memcpy(ft + 16, c->tables[STN_GATE_CX], 16);
  memcpy(ft + 32, c->tables[STN_GATE_CY], 16);
  memcpy(ft + 48, c->tables[STN_GATE_CZ], 16);
  const int n = c->n;
  c->hx.assign((size_t)2 * n * c->W, 0);
  c->hz.assign((size_t)2 * n * c->W, 0);
  for (int j = 0; j < n; ++j) {
    setbit(&c->hx[(size_t)j * c->W], j, 1);
    setbit(&c->hz[(size_t)(n + j) * c->W], j, 1);
  }
  hipError_t e = hipSuccess;
  e = e ? e : hipMemcpyAsync(c->tab.x, c->hx.data(), c->hx.size() * 8, hipMemcpyHostToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->tab.z, c->hz.data(), c->hz.size() * 8, hipMemcpyHostToDevice, c->st);
  e = e ? e : hipMemsetAsync(c->tab.s, 0, (size_t)2 * n * c->SW * 8, c->st);
  e = e ? e : hipMemcpyAsync(c->d_tables, ft, 64, hipMemcpyHostToDevice, c->st);
  {
    int64_t *dst[4] = {c->mps.site_off, c->mps.site_cap, c->mps.ws_off, c->mps.ws_cap};
    for (int a = 0; a < 4; ++a)
      e = e ? e : hipMemcpyAsync(dst[a], offs.data() + (size_t)a * n, (size_t)n * 8, hipMemcpyHostToDevice, c->st);
  }
  e = e ? e : hipMemsetAsync(c->d_err, 0, 4, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) {
    delete c;
    return STN_EDEVICE;
  }
  c->static_tape = scratch_ptr();
  {
    int max_rows = 4 * c->chi;                           // QR rows of a doubled tensor
    hipError_t pe = c->prec == STN_FP64 ? mps_prepare<double>(max_rows) : mps_prepare<float>(max_rows);
    if (pe == hipSuccess) pe = c->prec == STN_FP64 ? layer_prepare<double>() : layer_prepare<float>();
    if (pe != hipSuccess) {
      delete c;
      return STN_EDEVICE;
    }
  }
  if (c->prec == STN_FP64) mps_init<double>(c->mps, c->st);
  else mps_init<float>(c->mps, c->st);
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return STN_EDEVICE;
  }
  c->center = 0;
  *out = c;
  return STN_OK;
}

void stn_free(stn_ctx *ctx) { delete ctx; }

const char *stn_last_error(const stn_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int stn_center(const stn_ctx *ctx) { return ctx ? ctx->center : -1; }

stn_status stn_clifford(stn_ctx *c, const stn_gate *gates, int n_gates, const uint64_t *noise) {
  ProfScope ps_(c);
  if (!c || n_gates < 0 || (n_gates > 0 && !gates)) return fail(c, STN_EINVAL, "bad arguments");
  for (int i = 0; i < n_gates; ++i) {
    const stn_gate &g = gates[i];
    if (g.kind < 0 || g.kind > STN_GATE_CZ || g.q0 < 0 || g.q0 >= c->n)
      return fail(c, STN_EINVAL, "bad gate kind or qubit");
    if (is_two(g.kind) && (g.q1 < 0 || g.q1 >= c->n || g.q1 == g.q0))
      return fail(c, STN_EINVAL, "bad two-qubit gate operands");
  }
  // split into layers of gates on disjoint qubits, preserving order
  std::vector<int> used(c->n, -1);
  int layer = 0;
  ProgBatch b{};
  std::vector<RowProg> pending;
  auto flush = [&]() {
    if (b.ngates == 0) return;
    launch_tab_gates(c->tab, b, c->d_err, c->st);
    shadow_apply(c, b.p, b.n);
    b = ProgBatch{};
  };
  for (int i = 0; i < n_gates; ++i) {
    const stn_gate &g = gates[i];
    bool clash = used[g.q0] == layer || (is_two(g.kind) && used[g.q1] == layer);
    if (clash) { flush(); layer++; }
    RowProg progs[4];
    int np = gate_programs(c, g, progs);
    if (b.n + np > kProgBatch) flush();
    b.first[b.ngates] = b.n;
    for (int k = 0; k < np; ++k) b.p[b.n++] = progs[k];
    b.ngates++;
    b.first[b.ngates] = b.n;
    used[g.q0] = layer;
    if (is_two(g.kind)) used[g.q1] = layer;
  }
  flush();
  if (noise) launch_tab_noise(c->tab, noise, c->st);
  return check_launch(c);
}

stn_status stn_rotate(stn_ctx *c, const int32_t *qs, int n_rot, const double *theta, int64_t stride) {
  ProfScope ps_(c);
  if (!c || n_rot < 0 || (n_rot > 0 && (!qs || !theta)) || stride < 0)
    return fail(c, STN_EINVAL, "bad arguments");
  for (int i = 0; i < n_rot; ++i) {
    int cnt = 0;
    for (int k = 0; k < 3; ++k) {
      int q = qs[i * 3 + k];
      if (q < -1 || q >= c->n) return fail(c, STN_EINVAL, "bad rotation qubit");
      if (q >= 0) {
        for (int k2 = 0; k2 < k; ++k2)
          if (qs[i * 3 + k2] == q) return fail(c, STN_EINVAL, "repeated rotation qubit");
        cnt++;
      }
    }
    if (cnt < 2) return fail(c, STN_EINVAL, "rotation needs at least two qubits");
  }
  return c->prec == STN_FP64 ? rotate_impl<double>(c, qs, n_rot, theta, stride)
                             : rotate_impl<float>(c, qs, n_rot, theta, stride);
}

stn_status stn_measure(stn_ctx *c, const int32_t *qs, int n_meas, int reset, const double *u,
                       const uint8_t *forced, uint8_t *out, double *prob) {
  ProfScope ps_(c);
  if (!c || n_meas < 0 || (n_meas > 0 && !qs) || (!u && !forced)) return fail(c, STN_EINVAL, "bad arguments");
  for (int i = 0; i < n_meas; ++i)
    if (qs[i] < 0 || qs[i] >= c->n) return fail(c, STN_EINVAL, "bad measured qubit");
  return c->prec == STN_FP64 ? measure_impl<double>(c, qs, n_meas, reset, u, forced, out, prob)
                             : measure_impl<float>(c, qs, n_meas, reset, u, forced, out, prob);
}

stn_status stn_profile(stn_ctx *c, unsigned class_mask) {
  if (!c) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  const bool counters = !(class_mask & STN_PROFILE_TIMING_ONLY);
  class_mask &= ~STN_PROFILE_TIMING_ONLY;
  c->prof.mask = class_mask;
  c->prof.recs.clear();
  c->prof.used = 0;
  for (int k = 0; k < K_COUNT; ++k) { c->prof_ms[k] = 0; c->prof_launches[k] = 0; }
  c->mps.prof = (class_mask && counters) ? 1 : 0;
  hipError_t e = hipMemsetAsync(c->mps.work, 0, (size_t)kWorkWords * 8, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_profile_read(stn_ctx *c, double *ms, double *flops, double *bytes, long long *launches,
                            double *eig_sweeps, double *layer_fp64_flops) {
  if (!c) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  for (auto &r : c->prof.recs) {
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) c->prof_ms[r.cls] += t;
    c->prof_launches[r.cls]++;
  }
  c->prof.recs.clear();
  c->prof.used = 0;
  double w[kWorkWords];
  hipError_t e = hipMemcpy(w, c->mps.work, sizeof(w), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  for (int k = 0; k < K_COUNT; ++k) {
    if (ms) ms[k] = c->prof_ms[k];
    if (flops) flops[k] = w[2 * k];
    if (bytes) bytes[k] = w[2 * k + 1];
    if (launches) launches[k] = c->prof_launches[k];
  }
  if (eig_sweeps) *eig_sweeps = w[2 * K_COUNT];
  if (layer_fp64_flops) *layer_fp64_flops = w[2 * K_COUNT + 1];
  return STN_OK;
}

stn_status stn_reset(stn_ctx *c) {
  if (!c) return STN_EINVAL;
  ProfScope ps(c);
  launch_tab_reset(c->tab, c->d_err, c->st);
  if (c->prec == STN_FP64) mps_init<double>(c->mps, c->st);
  else mps_init<float>(c->mps, c->st);
  const int n = c->n;
  std::fill(c->hx.begin(), c->hx.end(), 0);
  std::fill(c->hz.begin(), c->hz.end(), 0);
  for (int j = 0; j < n; ++j) {
    setbit(&c->hx[(size_t)j * c->W], j, 1);
    setbit(&c->hz[(size_t)(n + j) * c->W], j, 1);
  }
  c->center = 0;
  return check_launch(c);
}

stn_status stn_sync(stn_ctx *c) {
  if (!c) return STN_EINVAL;
  return sync_status(c);
}

stn_status stn_logprob(stn_ctx *c, double *logp, double *terr) {
  if (!c) return STN_EINVAL;
  hipError_t e = hipSuccess;
  if (logp) e = hipMemcpyAsync(logp, c->mps.logp, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  if (terr) {
    std::vector<double> f(c->S);
    e = hipMemcpyAsync(f.data(), c->mps.fid, (size_t)c->S * 8, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
    for (auto &v : f) v = 1.0 - v;
    e = hipMemcpy(terr, f.data(), (size_t)c->S * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  }
  return sync_status(c);
}

stn_status stn_get_tableau(stn_ctx *c, uint64_t *hx, uint64_t *hz, uint64_t *hs) {
  if (!c) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  size_t nb = (size_t)2 * c->n * c->W * 8, ns = (size_t)2 * c->n * c->SW * 8;
  hipError_t e = hipSuccess;
  if (hx) e = hipMemcpy(hx, c->tab.x, nb, hipMemcpyDeviceToHost);
  if (e == hipSuccess && hz) e = hipMemcpy(hz, c->tab.z, nb, hipMemcpyDeviceToHost);
  if (e == hipSuccess && hs) e = hipMemcpy(hs, c->tab.s, ns, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_get_bonds(stn_ctx *c, int32_t *hb) {
  if (!c || !hb) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  hipError_t e = hipMemcpy(hb, c->mps.bond, (size_t)c->S * (c->n + 1) * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_get_site(stn_ctx *c, int shot, int site, void *buf, size_t bytes, int *dl, int *dr) {
  if (!c || !buf || shot < 0 || shot >= c->S || site < 0 || site >= c->n) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  int b[2];
  hipError_t e = hipMemcpy(b, c->mps.bond + (size_t)shot * (c->n + 1) + site, 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  size_t need = (size_t)b[0] * 2 * b[1] * c->esz;
  if (bytes < need) return fail(c, STN_EINVAL, "buffer too small");
  int64_t off, cap;
  e = hipMemcpy(&off, c->mps.site_off + site, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&cap, c->mps.site_cap + site, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(buf, (char *)c->mps.mps + (off + (int64_t)shot * cap) * c->esz, need, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  if (dl) *dl = b[0];
  if (dr) *dr = b[1];
  return STN_OK;
}

stn_status stn_set_site(stn_ctx *c, int shot, int site, const void *buf, int dl, int dr) {
  if (!c || !buf || shot < 0 || shot >= c->S || site < 0 || site >= c->n) return STN_EINVAL;
  if (dl < 1 || dr < 1 || dl > dmax_h(c->n, c->chi, site) || dr > dmax_h(c->n, c->chi, site + 1) ||
      (site == 0 && dl != 1) || (site == c->n - 1 && dr != 1))
    return fail(c, STN_EINVAL, "site shape exceeds the bond caps");
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  int64_t off, cap;
  hipError_t e = hipMemcpy(&off, c->mps.site_off + site, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&cap, c->mps.site_cap + site, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy((char *)c->mps.mps + (off + (int64_t)shot * cap) * c->esz, buf,
                  (size_t)dl * 2 * dr * c->esz, hipMemcpyHostToDevice);
  int b[2] = {dl, dr};
  if (e == hipSuccess)
    e = hipMemcpy(c->mps.bond + (size_t)shot * (c->n + 1) + site, b, 8, hipMemcpyHostToDevice);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_profile_phases(stn_ctx *c, double *cycles) {
  if (!c || !cycles) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  hipError_t e = hipMemcpy(cycles, c->mps.work + kPhaseBase, kPhases * 8, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_profile_paths(stn_ctx *c, double *counts) {
  if (!c || !counts) return STN_EINVAL;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  double w[kPaths];
  hipError_t e = hipMemcpy(w, c->mps.work + kPathBase, kPaths * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, hipGetErrorString(e));
  for (int i = 0; i < kPaths; ++i) counts[i] = w[i];
  // the largest order is kept as an integer (atomicMax on its bits)
  unsigned long long mo;
  std::memcpy(&mo, &w[kPathMaxOrder], 8);
  counts[kPathMaxOrder] = (double)mo;
  return STN_OK;
}

stn_status stn_set_layer_mode(stn_ctx *c, int mode) {
  if (!c || mode < 0 || mode > 2) return STN_EINVAL;
  c->layer_mode = mode;
  return STN_OK;
}

stn_status stn_set_layer_threads(stn_ctx *c, int threads) {
  if (!c || (threads != 64 && threads != 128 && threads != 256 && threads != 512)) return STN_EINVAL;
  c->layer_threads = threads;
  return STN_OK;
}

stn_status stn_spectrum(stn_ctx *c, int bond, double *dev_out, int ld, int *dev_rank) {
  if (!c || !dev_out || bond < 1 || bond > c->n - 1) return STN_EINVAL;
  if (ld < dmax_h(c->n, c->chi, bond)) return fail(c, STN_EINVAL, "spectrum row shorter than the largest bond");
  if (c->taping) return fail(c, STN_ESTATE, "spectrum while recording a tape");
  ProfScope ps(c);
  if (c->prec == STN_FP64) {
    move_center_into<double>(c, bond, bond);
    mps_spectrum<double>(c->mps, bond, dev_out, ld, dev_rank, c->st);
  } else {
    move_center_into<float>(c, bond, bond);
    mps_spectrum<float>(c->mps, bond, dev_out, ld, dev_rank, c->st);
  }
  return check_launch(c);
}

stn_status stn_set_layer_env(stn_ctx *c, int max_bond) {
  if (!c || max_bond < 0 || max_bond > c->mps.ebond_alloc) return STN_EINVAL;
  c->mps.ebond = max_bond;
  return STN_OK;
}

stn_status stn_set_layer_lds(stn_ctx *c, int order) {
  if (!c || (order != 0 && order != 32 && order != 64)) return STN_EINVAL;
  c->mps.lds_order = order;
  return STN_OK;
}

stn_status stn_set_center(stn_ctx *c, int center) {
  if (!c || center < 0 || center >= c->n) return STN_EINVAL;
  c->center = center;
  return STN_OK;
}

// ------------------------------------------------------------ gradients
size_t stn_tape_bytes(const stn_ctx *c, int max_steps) {
  if (!c || max_steps < 1) return 0;
  return (size_t)(max_steps + 1) * rec_layout(c).total;
}

stn_status stn_tape_begin(stn_ctx *c, void *dev_tape, size_t bytes, int max_steps) {
  if (!c || !dev_tape || max_steps < 1 || ((uintptr_t)dev_tape & 255)) return STN_EINVAL;
  if (bytes < stn_tape_bytes(c, max_steps)) return fail(c, STN_ENOMEM, "tape buffer too small");
  c->tape = (char *)dev_tape;
  c->tape_max = max_steps;
  c->steps.clear();
  c->tape_rot = 0;
  c->taping = true;
  c->tape_closed = false;
  return STN_OK;
}

stn_status stn_tape_begin_static(stn_ctx *c, int max_steps) {
  if (!c || max_steps < 1) return STN_EINVAL;
  const size_t need = stn_tape_bytes(c, max_steps);
  if (need > kStaticTapeBytes)
    return fail(c, STN_ENOMEM, "tape of " + std::to_string(need) + " bytes exceeds the " +
                                   std::to_string(kStaticTapeBytes >> 20) + " MiB static tape");
  if (!c->static_tape) return fail(c, STN_EDEVICE, "static tape unavailable on this device");
  return stn_tape_begin(c, c->static_tape, kStaticTapeBytes, max_steps);
}

stn_status stn_tape_end(stn_ctx *c, int *n_rotations) {
  if (!c || !c->taping) return STN_ESTATE;
  const RecLayout R = rec_layout(c);
  hipError_t e = take_snapshot(c, c->tape + c->steps.size() * R.total);
  c->taping = false;
  c->tape_closed = true;
  if (n_rotations) *n_rotations = c->tape_rot;
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  return check_launch(c);
}

size_t stn_adjoint_bytes(const stn_ctx *c, int chi_adj) {
  if (!c || chi_adj < 1 || chi_adj > 512) return 0;
  Layout L;
  plan_mps(L, c->n, c->S, chi_adj, c->esz, 3, nullptr, nullptr, nullptr);
  return L.total;
}

stn_status stn_adjoint_init(stn_ctx *c, void *dev_buf, size_t bytes, int chi_adj) {
  if (!c || !dev_buf || ((uintptr_t)dev_buf & 255)) return STN_EINVAL;
  const size_t need = stn_adjoint_bytes(c, chi_adj);
  if (need == 0) return STN_EINVAL;
  if (bytes < need) return fail(c, STN_ENOMEM, "adjoint buffer too small");
  Layout L;
  std::vector<int64_t> offs;
  plan_mps(L, c->n, c->S, chi_adj, c->esz, 3, (char *)dev_buf, &c->adj, &offs);
  MpsDev &mu = c->adj;
  mu.err = c->d_err;
  // The adjoint's compression only has to represent mu, and the gradient is
  // linear in mu: a dropped value lambda costs ~sqrt(lambda) of it, so its
  // relative cut sits 100x below the forward's (at the Gram noise floor).
  mu.eps_cut = 1e-2 * c->cfg.eps_cut;
  mu.work = c->mps.work;
  mu.keep_norm = 1;
  hipError_t e = hipSuccess;
  int64_t *dst[4] = {mu.site_off, mu.site_cap, mu.ws_off, mu.ws_cap};
  for (int a = 0; a < 4; ++a)
    e = e ? e : hipMemcpyAsync(dst[a], offs.data() + (size_t)a * c->n, (size_t)c->n * 8, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  const int rows = std::max(4 * c->chi, 6 * chi_adj);     // QR rows of doubled / summed tensors
  if (e == hipSuccess) e = c->prec == STN_FP64 ? mps_prepare<double>(rows) : mps_prepare<float>(rows);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  c->adj_ready = true;
  return stn_adjoint_zero(c);
}

stn_status stn_adjoint_zero(stn_ctx *c) {
  if (!c || !c->adj_ready) return STN_ESTATE;
  if (c->prec == STN_FP64) mps_zero<double>(c->adj, c->st);
  else mps_zero<float>(c->adj, c->st);
  launch_step_reset(c->adj, c->st);              // clears the per-shot cap flags
  c->adj_center = 0;
  return check_launch(c);
}

stn_status stn_adjoint_truncated(stn_ctx *c, int *host_flags) {
  if (!c || !host_flags) return STN_EINVAL;
  if (!c->adj_ready) return STN_ESTATE;
  stn_status s = sync_status(c);
  if (s != STN_OK) return s;
  hipError_t e = hipMemcpy(host_flags, c->adj.trunc, (size_t)c->S * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STN_OK : fail(c, STN_EDEVICE, hipGetErrorString(e));
}

stn_status stn_backward(stn_ctx *c, double *dev_grad, int64_t grad_stride) {
  if (!c || !dev_grad || grad_stride < 0) return STN_EINVAL;
  if (!c->adj_ready || !c->tape_closed) return fail(c, STN_ESTATE, "backward needs a closed tape and an adjoint state");
  if (grad_stride < c->tape_rot && c->S > 1) return STN_EINVAL;
  ProfScope ps(c);
  stn_status st = c->prec == STN_FP64 ? backward_impl<double>(c, dev_grad, grad_stride)
                                      : backward_impl<float>(c, dev_grad, grad_stride);
  if (st != STN_OK) return st;
  return sync_status(c);
}

size_t stn_checkpoint_bytes(const stn_ctx *c) { return c ? ck_layout(c).total : 0; }

stn_status stn_checkpoint_save(stn_ctx *c, void *dev_buf) {
  if (!c || !dev_buf || ((uintptr_t)dev_buf & 255)) return STN_EINVAL;
  const CkLayout K = ck_layout(c);
  char *b = (char *)dev_buf;
  const size_t tb = (size_t)2 * c->n * c->W * 8;
  int64_t center = c->center;
  hipError_t e = hipMemcpyAsync(b + K.mps, c->mps.mps, mps_slot_bytes(c->n, c->S, c->chi, c->esz), hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.bond, c->mps.bond, (size_t)c->S * (c->n + 1) * 4, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.x, c->tab.x, tb, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.z, c->tab.z, tb, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.s, c->tab.s, (size_t)2 * c->n * c->SW * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.logp, c->mps.logp, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(b + K.fid, c->mps.fid, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipStreamSynchronize(c->st);
  e = e ? e : hipMemcpy(b + K.hx, c->hx.data(), tb, hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(b + K.hz, c->hz.data(), tb, hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(b + K.center, &center, 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  return STN_OK;
}

stn_status stn_checkpoint_load(stn_ctx *c, const void *dev_buf) {
  if (!c || !dev_buf || ((uintptr_t)dev_buf & 255)) return STN_EINVAL;
  const CkLayout K = ck_layout(c);
  const char *b = (const char *)dev_buf;
  const size_t tb = (size_t)2 * c->n * c->W * 8;
  int64_t center = 0;
  hipError_t e = hipStreamSynchronize(c->st);
  e = e ? e : hipMemcpy(c->hx.data(), b + K.hx, tb, hipMemcpyDeviceToHost);
  e = e ? e : hipMemcpy(c->hz.data(), b + K.hz, tb, hipMemcpyDeviceToHost);
  e = e ? e : hipMemcpy(&center, b + K.center, 8, hipMemcpyDeviceToHost);
  e = e ? e : hipMemcpyAsync(c->mps.mps, b + K.mps, mps_slot_bytes(c->n, c->S, c->chi, c->esz), hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->mps.bond, b + K.bond, (size_t)c->S * (c->n + 1) * 4, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->tab.x, b + K.x, tb, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->tab.z, b + K.z, tb, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->tab.s, b + K.s, (size_t)2 * c->n * c->SW * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->mps.logp, b + K.logp, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipMemcpyAsync(c->mps.fid, b + K.fid, (size_t)c->S * 8, hipMemcpyDeviceToDevice, c->st);
  e = e ? e : hipStreamSynchronize(c->st);
  if (e != hipSuccess) return fail(c, STN_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
  c->center = (int)center;
  return STN_OK;
}

}  // extern "C"
