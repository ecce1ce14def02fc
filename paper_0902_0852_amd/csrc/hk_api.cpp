// C-ABI of the hk library: workspace planning, matrix build, factorisation,
// solves, export and the eigenvalue drivers.  See include/hk.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hk_internal.hpp"

using namespace hk;

namespace hk {
thread_local std::string g_err;
static hk_status fail(hk_status st, const std::string& msg) { g_err = msg; return st; }
#define HK_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(HK_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static int round_up(int x, int m) { return (x + m - 1) / m * m; }

// How the trailing update leaves the critical path (look-ahead mode): 0 none,
// 1 the rest of each panel's update on a second stream, 2 one launch per
// column with the next column's update inside it (panel width 1).
// HK_LOOKAHEAD=0/1/2 forces it; else the setting (from the caller or the
// tuning cache); else 1 when a panel carries enough update work
// (N x widest column >= 100000 digits), 2 below that.
int lookahead_mode(int setting, int maxN, int maxW) {
  const char* v = getenv("HK_LOOKAHEAD");
  if (v && v[0] >= '0' && v[0] <= '2' && v[1] == 0) return v[0] - '0';
  if (setting >= 0 && setting <= 2) return setting;
  return (int64_t)maxN * maxW >= 100000 ? 1 : 2;
}

bool make_plan(int N, int64_t bnum, int64_t bden, int K, Plan& P, std::string& err) {
  if (N < 1 || N > 100000) { err = "N out of range"; return false; }
  if (K < 64 || (K & 1) || K > (1 << 22)) { err = "prec_bits must be even and >= 64"; return false; }
  if (!reduce_beta(bnum, bden, &P.p, &P.q)) { err = "beta must be num/den with num, den >= 1"; return false; }
  P.N = N; P.K = K; P.h = K / 2;
  const int nX = 2 * N - 1;
  std::vector<int64_t> bX(nX);
  int64_t bmax = 0;
  for (int n = 0; n < nX; n++) {
    double l = log2_mu(n, P.p, P.q);
    int64_t b = (int64_t)K + (int64_t)std::ceil(l + 1e-9 * std::fabs(l)) + 2;
    bX[n] = std::max<int64_t>(b, 1);
    bmax = std::max(bmax, bX[n]);
  }
  P.WX = (int)((bmax + 1 + DB - 1) / DB) + 1;
  // suffix max of the diagonal sizes
  std::vector<int64_t> sufmax(N + 1, 0);
  for (int r = N - 1; r >= 0; r--) sufmax[r] = std::max(sufmax[r + 1], bX[2 * r]);
  P.cols.resize(N);
  P.itemStart.assign(N + 1, 0);
  int64_t a = 0, kk = 0, cc = 0, ll = 0, l8 = 0, dd = 0;
  P.maxW = 0;
  for (int c = 0; c < N; c++) {
    ColInfo& ci = P.cols[c];
    // |A_rc| <= sqrt(A_rr A_cc) while the trailing block is positive definite
    int64_t Bc = (sufmax[c] + bX[2 * c] + 1) / 2 + 4;
    // a whole number of 32-digit tiles (the matrix-core update works on two
    // 16-digit blocks at a time)
    int W = round_up((int)((Bc + DB - 1) / DB) + 4, 2 * WB);
    ci.W = W;
    ci.R = round_up(N - c, 64);
    ci.nb = W / WB;
    ci.CW = W + WB;
    ci.LW = W + 2 * WB;
    ci.items = (ci.R / 64) * ci.nb;
    ci.aoff = a; a += (int64_t)W * ci.R;
    ci.koff = kk; kk += (int64_t)2 * ci.nb * ci.R;
    ci.coff = cc; cc += (int64_t)(N - c) * ci.CW;
    ci.soff = ci.coff;
    ci.loff = ll; ll += (int64_t)ci.LW * ci.R;
    ci.G = (ci.LW + 31) / 32;
    ci.l8off = l8; l8 += (int64_t)4 * ci.G * ci.R * 32;
    ci.doff = dd; dd += W + 2;
    P.itemStart[c + 1] = P.itemStart[c] + ci.items;
    P.maxW = std::max(P.maxW, W);
  }
  if ((int64_t)P.itemStart[N] >= (int64_t)INT_MAX / 2) { err = "problem too large"; return false; }
  // L^T rows (backward solves): row r holds L_c[r], c < r
  P.LWT = P.maxW + 2 * WB;
  int64_t lt = 0;
  for (int r = 0; r < N; r++) {
    ColInfo& ci = P.cols[r];
    ci.PT = std::max(64, round_up(r, 64));
    ci.ltoff = lt;
    lt += (int64_t)P.LWT * ci.PT;
  }
  P.ntri = (int64_t)N * (N + 1) / 2;
  // solve vectors: K + g fractional bits plus the integer part of A^{-1} b
  P.gbits = 64 * (int)(((std::max<int64_t>(0, bmax - K) / 2) + 63) / 64);
  // |z| <= N sqrt(A_ii / lambda_1), |w|, |y| <= N / lambda_1 with lambda_1 >= 2^-K
  {
    const int64_t vb = std::max<int64_t>(3 * (int64_t)K / 2 + 2 * P.gbits, 2 * (int64_t)K + P.gbits) + 96;
    P.VW = round_up((int)((vb + DB - 1) / DB) + 4, WB);
  }
  P.VA = round_up(P.VW + P.maxW + 2 * WB + (P.h + DB - 1) / DB + 6, WB);
  P.Npad = round_up(N, 64);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  P.o_cols = take(sizeof(ColInfo) * N);
  P.o_items = take(sizeof(int32_t) * (N + 1));
  P.o_A = take(sizeof(int32_t) * a);
  P.o_K = take(sizeof(int64_t) * kk);
  P.o_C = take(sizeof(int32_t) * cc);
  P.o_S = take(sizeof(uint32_t) * cc);
  P.o_L = take(sizeof(int32_t) * ll);
  P.o_L8 = take((size_t)l8);
  P.o_D = take(sizeof(uint32_t) * dd);
  P.o_dinfo = take(sizeof(int32_t) * 4 * N);
  P.o_nC = take(sizeof(int32_t) * P.ntri);
  P.o_nCs = take(sizeof(int32_t) * P.ntri);
  P.o_nL = take(sizeof(int32_t) * P.ntri);
  P.o_b32C = take(sizeof(int32_t) * P.ntri);
  P.o_b32L = take(sizeof(int32_t) * P.ntri);
  P.o_X = take(sizeof(int32_t) * (size_t)nX * P.WX);
  P.o_xs = take(sizeof(int32_t) * P.WX);
  P.o_flags = take(sizeof(int32_t) * 16);
  P.o_vec = take(sizeof(int32_t) * (size_t)N * (P.maxW + WB));  // pivot gather
  P.o_LT = take(sizeof(int32_t) * lt);
  P.o_acc = take(sizeof(int32_t) * (size_t)P.VA * P.Npad);
  P.o_kca = take(sizeof(int64_t) * (size_t)2 * (P.VA / WB) * P.Npad);
  P.o_ub = take(sizeof(int32_t) * (size_t)N * P.VW);
  P.o_us = take(sizeof(uint32_t) * (size_t)N * P.VW);
  P.o_wb = take(sizeof(int32_t) * (size_t)N * P.VW);
  P.o_nU = take(sizeof(int32_t) * N);
  P.o_nUs = take(sizeof(int32_t) * N);
  P.o_dv1 = take(sizeof(int32_t) * (size_t)N * P.VW);
  P.o_dv2 = take(sizeof(int32_t) * (size_t)N * P.VW);
  P.o_md = take(sizeof(uint32_t) * (size_t)(P.VW + 4));
  P.o_mdinfo = take(sizeof(int32_t) * 4);
  P.o_dots = take(sizeof(int64_t) * 4 * DOT_PARTS * (size_t)(2 * P.VW + 8));
  P.o_sargs = take(sizeof(SweepArgs));
  P.o_desc = take(sizeof(InstDesc));
  P.total = o;
  return true;
}

DevPtrs dev_ptrs(const Plan& P, char* ws) {
  DevPtrs D;
  D.cols = (ColInfo*)(ws + P.o_cols);
  D.itemStart = (int32_t*)(ws + P.o_items);
  D.A = (int32_t*)(ws + P.o_A);
  D.Kc = (int64_t*)(ws + P.o_K);
  D.C = (int32_t*)(ws + P.o_C);
  D.S = (uint32_t*)(ws + P.o_S);
  D.L = (int32_t*)(ws + P.o_L);
  D.L8 = (int8_t*)(ws + P.o_L8);
  D.D = (uint32_t*)(ws + P.o_D);
  D.dinfo = (int32_t*)(ws + P.o_dinfo);
  D.nC = (int32_t*)(ws + P.o_nC);
  D.nCs = (int32_t*)(ws + P.o_nCs);
  D.nL = (int32_t*)(ws + P.o_nL);
  D.b32C = (int32_t*)(ws + P.o_b32C);
  D.b32L = (int32_t*)(ws + P.o_b32L);
  D.X = (int32_t*)(ws + P.o_X);
  D.xs = (int32_t*)(ws + P.o_xs);
  D.flags = (int32_t*)(ws + P.o_flags);
  D.vec = (int32_t*)(ws + P.o_vec);
  D.LT = (int32_t*)(ws + P.o_LT);
  D.acc = (int32_t*)(ws + P.o_acc);
  D.kca = (int64_t*)(ws + P.o_kca);
  D.ub = (int32_t*)(ws + P.o_ub);
  D.us = (uint32_t*)(ws + P.o_us);
  D.wb = (int32_t*)(ws + P.o_wb);
  D.nU = (int32_t*)(ws + P.o_nU);
  D.nUs = (int32_t*)(ws + P.o_nUs);
  D.dv1 = (int32_t*)(ws + P.o_dv1);
  D.dv2 = (int32_t*)(ws + P.o_dv2);
  D.md = (uint32_t*)(ws + P.o_md);
  D.mdinfo = (int32_t*)(ws + P.o_mdinfo);
  D.dots = (int64_t*)(ws + P.o_dots);
  D.sargs = (SweepArgs*)(ws + P.o_sargs);
  D.desc = (InstDesc*)(ws + P.o_desc);
  return D;
}

InstDesc make_desc(const Plan& P, const DevPtrs& D) {
  InstDesc I;
  I.cols = D.cols; I.itemStart = D.itemStart;
  I.A = D.A; I.Kc = D.Kc; I.C = D.C; I.S = D.S; I.L = D.L; I.L8 = D.L8; I.LT = D.LT; I.D = D.D;
  I.dinfo = D.dinfo; I.nC = D.nC; I.nCs = D.nCs; I.nL = D.nL; I.b32C = D.b32C; I.flags = D.flags;
  I.X = D.X; I.xs = D.xs;
  I.N = P.N; I.h = P.h; I.WX = P.WX; I.active = 1;
  return I;
}

// v -> n balanced radix-2^29 digits (zero padded); false if it does not fit
static bool to_digits(const MP& v, int32_t* out, int n) {
  if (v.bitlen() > (int64_t)n * DB) return false;
  int64_t carry = 0;
  for (int i = 0; i < n; i++) {
    const int64_t pos = (int64_t)i * DB;
    const size_t w = (size_t)(pos >> 5);
    const int off = (int)(pos & 31);
    uint64_t u = 0;
    if (w < v.d.size()) {
      uint64_t lo = v.d[w];
      if (w + 1 < v.d.size()) lo |= (uint64_t)v.d[w + 1] << 32;
      u = (lo >> off) & (uint64_t)(RADIX - 1);
    }
    int64_t y = (int64_t)u + carry;
    if (y >= (int64_t(1) << 28)) { y -= RADIX; carry = 1; } else carry = 0;
    out[i] = (int32_t)(v.neg ? -y : y);
  }
  return carry == 0;
}

void mp_to_digits(const MP& v, int32_t* out, int n) { to_digits(v, out, n); }

// The whole factorisation of every instance of B (shifts and flags already in
// place): expansion, then per panel of b columns the in-panel updates,
// finalisations and divisions column by column, then the trailing update.
// With evs != NULL every update launch records its own start and end on a
// pair of HIP events.
hipError_t enqueue_factor(const BatchView& B, int b, int mode, hipStream_t s, hipStream_t s2,
                          std::vector<TimedLaunch>* evs, std::vector<hipEvent_t>* pool, size_t* evi,
                          int* n_update, int* n_bulk) {
  // one pool of (timing-capable) events for both the per-launch timing and
  // the look-ahead fork/join points
  auto get_ev = [&]() -> hipEvent_t {
    if (*evi >= pool->size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool->push_back(e);
    }
    return (*pool)[(*evi)++];
  };
  auto timed_update = [&](int pc, int j, int rd, hipStream_t st) -> hipError_t {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (evs) { e0 = get_ev(); e1 = get_ev(); }
    hipError_t e = launch_update(B, pc, b, j, rd, st, e0 && e1 ? e0 : nullptr, e0 && e1 ? e1 : nullptr);
    if (e == hipSuccess && e0 && e1) evs->push_back({e0, e1, update_is_bulk(j)});
    if (n_update) (*n_update)++;
    if (n_bulk && update_is_bulk(j)) (*n_bulk)++;
    return e;
  };
  hipError_t e = launch_expand(B, s);
  if (mode == 2) {
    // one launch per column; the update work rides in every launch
    for (int c = 0; c < B.maxN && e == hipSuccess; c++) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (evs) { e0 = get_ev(); e1 = get_ev(); }
      if (e == hipSuccess) e = launch_column(B, c, s, e0 && e1 ? e0 : nullptr, e0 && e1 ? e1 : nullptr);
      if (e == hipSuccess && e0 && e1) evs->push_back({e0, e1, true});
      if (n_update) (*n_update)++;
      if (n_bulk) (*n_bulk)++;
    }
    return e;
  }
  const bool la = mode == 1 && s2 != nullptr && pool != nullptr;
  hipEvent_t far_prev = nullptr;
  int Pidx = 0;
  for (int pc = 0; pc < B.maxN && e == hipSuccess; pc += b, Pidx++) {
    for (int j = 0; j < b && pc + j < B.maxN && e == hipSuccess; j++) {
      const int c = pc + j;
      if (j > 0) e = timed_update(pc, j, Pidx & 1, s);
      if (e == hipSuccess) e = launch_fdiv(B, c, (Pidx + (j > 0 ? 1 : 0)) & 1, s);
    }
    if (e != hipSuccess || pc + b >= B.maxN) continue;
    if (!la) {
      e = timed_update(pc, 0, Pidx & 1, s);
      continue;
    }
    // look-ahead: the rest of the trailing update leaves the critical path
    hipEvent_t fork = get_ev();
    if (!fork) return hipErrorOutOfMemory;
    e = hipEventRecord(fork, s);                       // this panel's C and L are final
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, fork, 0);
    if (e == hipSuccess) e = timed_update(pc, UPD_FAR, Pidx & 1, s2);
    // the next panel's columns: their update by the previous panel is on s2
    if (e == hipSuccess && far_prev) e = hipStreamWaitEvent(s, far_prev, 0);
    if (e == hipSuccess) e = timed_update(pc, UPD_NEAR, Pidx & 1, s);
    if (e == hipSuccess) {
      far_prev = get_ev();
      if (!far_prev) return hipErrorOutOfMemory;
      e = hipEventRecord(far_prev, s2);
    }
  }
  if (e == hipSuccess && far_prev) e = hipStreamWaitEvent(s, far_prev, 0);
  return e;
}

int host_threads() {
  static const int n = [] {
    const char* v = getenv("HK_HOST_THREADS");
    if (v && atoi(v) > 0) return std::min(atoi(v), 64);
    return std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  }();
  return n;
}

MP digits_to_mp(const int32_t* d, int n, int64_t stride) {
  // positive and negative digit parts packed separately, then subtracted
  std::vector<uint32_t> pw((size_t)(((int64_t)n * DB) / 32 + 3), 0u), nw(pw.size(), 0u);
  for (int i = 0; i < n; i++) {
    int32_t x = d[(int64_t)i * stride];
    if (!x) continue;
    uint64_t m = (uint64_t)(x < 0 ? -(int64_t)x : (int64_t)x);
    int64_t pos = (int64_t)i * DB;
    std::vector<uint32_t>& w = x < 0 ? nw : pw;
    size_t k = (size_t)(pos >> 5);
    uint64_t sh = m << (pos & 31);
    uint64_t cur = (uint64_t)w[k] + (uint32_t)sh;
    w[k] = (uint32_t)cur;
    uint64_t c2 = (cur >> 32) + (sh >> 32);
    for (size_t j = k + 1; c2 && j < w.size(); j++) {
      uint64_t t = (uint64_t)w[j] + c2;
      w[j] = (uint32_t)t;
      c2 = t >> 32;
    }
  }
  MP a, b;
  a.d = pw; a.trim();
  b.d = nw; b.trim();
  return sub(a, b);
}

}  // namespace hk

extern "C" {

const char* hk_last_error(void) { return g_err.c_str(); }

size_t hk_workspace_bytes(int N, hk_rational beta, int prec_bits, int flags) {
  (void)flags;
  Plan P;
  std::string err;
  if (!make_plan(N, beta.num, beta.den, prec_bits, P, err)) { g_err = err; return 0; }
  return P.total;
}

hk_status hk_moments_host(int N, hk_rational beta, int prec_bits, uint32_t* words, int64_t cap,
                          int64_t* off) {
  if (!off) return fail(HK_EINVAL, "off is NULL");
  if (N < 1 || prec_bits < 64 || (prec_bits & 1)) return fail(HK_EINVAL, "need N >= 1 and even prec_bits >= 64");
  uint32_t p = 0, q = 0;
  if (!reduce_beta(beta.num, beta.den, &p, &q)) return fail(HK_EINVAL, "beta must be num/den with num, den >= 1");
  std::vector<MP> X;
  if (!build_moments(N, p, q, prec_bits, X)) return fail(HK_EPRECISION, "moment rounding undecided");
  int64_t total = 0;
  for (size_t n = 0; n < X.size(); n++) { off[n] = total; total += (int64_t)X[n].d.size(); }
  off[X.size()] = total;
  if (!words || cap < total) return fail(HK_EINVAL, "words buffer too small: need " + std::to_string(total));
  for (size_t n = 0; n < X.size(); n++) std::copy(X[n].d.begin(), X[n].d.end(), words + off[n]);
  return HK_OK;
}

hk_status hk_build_matrix(int N, hk_rational beta, int prec_bits, void* dev_ws, size_t ws_bytes,
                          hipStream_t s, hk_matrix* out) {
  const hk_status st = hk::build_matrix_impl(N, beta, prec_bits, dev_ws, ws_bytes, s, out, nullptr);
  if (st == HK_OK) {
    // a panel width tuned for this shape (hk_autotune, cache named by HK_TUNE_CACHE)
    const hk_instance one = {N, beta, prec_bits};
    const hk::Schedule sc = hk::tuned_schedule(&one, 1);
    if (sc.panel > 0) (*out)->panel = sc.panel;
    (*out)->lookahead = sc.lookahead;
    if (sc.ipw > 0) (*out)->B.ipw = sc.ipw;
    if (sc.mma >= 0) (*out)->B.mma = sc.mma;
  }
  return st;
}

hk_status hk_set_update_group(hk_matrix m, int items) {
  if (!m || (items != 1 && items != 2 && items != 4)) return fail(HK_EINVAL, "items per workgroup must be 1, 2 or 4");
  m->B.ipw = items;
  return HK_OK;
}

hk_status hk_set_update_engine(hk_matrix m, int engine) {
  if (!m || (engine != HK_UPDATE_MATRIX_CORES && engine != HK_UPDATE_VECTOR))
    return fail(HK_EINVAL, "engine must be HK_UPDATE_MATRIX_CORES or HK_UPDATE_VECTOR");
  m->B.mma = engine == HK_UPDATE_MATRIX_CORES ? 1 : 0;
  return HK_OK;
}

}  // extern "C"

namespace hk {
// hk_build_matrix with optionally precomputed moments (moved in)
hk_status build_matrix_impl(int N, hk_rational beta, int prec_bits, void* dev_ws, size_t ws_bytes,
                            hipStream_t s, hk_matrix* out, std::vector<MP>* moments) {
  if (!out) return fail(HK_EINVAL, "out is NULL");
  *out = nullptr;
  hk_matrix m = new (std::nothrow) hk_matrix_s;
  if (!m) return fail(HK_ENOMEM, "host allocation failed");
  std::string err;
  if (!make_plan(N, beta.num, beta.den, prec_bits, m->P, err)) { delete m; return fail(HK_EINVAL, err); }
  if (!dev_ws || ws_bytes < m->P.total) {
    size_t need = m->P.total;
    delete m;
    return fail(HK_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  m->ws = (char*)dev_ws;
  m->ws_bytes = ws_bytes;
  m->D = dev_ptrs(m->P, m->ws);
  const Plan& P = m->P;
  if (moments) m->X.swap(*moments);
  else if (!build_moments(N, P.p, P.q, P.K, m->X)) { delete m; return fail(HK_EPRECISION, "moment rounding undecided"); }
  if ((int)m->X.size() != 2 * N - 1) { delete m; return fail(HK_EINVAL, "moment count"); }
  {
    // solve guard bits: half the bit length of the largest moment's integer
    // part, rounded up to a multiple of 64
    const int64_t top = std::max<int64_t>(0, m->X[2 * N - 2].bitlen() - P.K);
    m->gbits = 64 * (int)((top / 2 + 63) / 64);
    if (m->gbits > P.gbits) { delete m; return fail(HK_EPRECISION, "moment wider than planned"); }
  }
  std::vector<int32_t> Xd((size_t)(2 * N - 1) * P.WX);
  for (int n = 0; n < 2 * N - 1; n++) {
    if (!to_digits(m->X[n], &Xd[(size_t)n * P.WX], P.WX)) { delete m; return fail(HK_EPRECISION, "moment wider than planned"); }
  }
  hk_status st = HK_OK;
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  m->desc_host = make_desc(P, m->D);
  m->B.ddesc = m->D.desc;
  m->B.plans = {&m->P};
  m->B.maxN = N;
  hipError_t e = cp(m->D.X, Xd.data(), Xd.size() * sizeof(int32_t));
  if (e == hipSuccess) e = cp(m->D.desc, &m->desc_host, sizeof(InstDesc));
  if (e == hipSuccess) e = cp(m->D.cols, P.cols.data(), P.cols.size() * sizeof(ColInfo));
  if (e == hipSuccess) e = cp(m->D.itemStart, P.itemStart.data(), P.itemStart.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { delete m; return fail(HK_EDEVICE, std::string("upload: ") + hipGetErrorString(e)); }
  *out = m;
  return st;
}
// shift as an integer with K fractional bits
bool shift_fixed(const hk_mpf& x, int K, MP& out) {
  MP v;
  if (x.sign != 0 && x.ndigits > 0 && x.digits) {
    v.d.assign(x.digits, x.digits + x.ndigits);
    v.trim();
    v.neg = x.sign < 0 && !v.d.empty();
  }
  int64_t e = x.exp2 + K;
  if (e >= 0) { out = shl(v, e); return true; }
  if (!low_bits_zero(v, -e)) return false;
  out = shr_mag(v, -e);
  return true;
}

// the look-ahead mode hk_factor runs: the set or tuned one, mode 1 taken
// as 0 when every launch must stay on the caller's stream
int effective_lookahead(const hk_matrix_s* m) {
  const int la = lookahead_mode(m->lookahead, m->P.N, m->P.maxW);
  return m->eager && la == 1 ? 0 : la;
}

hipError_t limb_macs_split(hk_matrix m, int b, int mode, hipStream_t s, double* total, double* bulk) {
  const Plan& P = m->P;
  hipError_t e = launch_bits(P, m->D, s);
  std::vector<int32_t> bc(P.ntri), bl(P.ntri);
  if (e == hipSuccess) e = hipMemcpyAsync(bc.data(), m->D.b32C, sizeof(int32_t) * P.ntri, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(bl.data(), m->D.b32L, sizeof(int32_t) * P.ntri, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int N = P.N;
  if (mode == 2) b = 1;
  double tot = 0, blk = 0;
  for (int k = 0; k < N - 1; k++) {
    // the panel of column k, and the first column of its bulk launch: the
    // next panel's columns belong to the near launch in mode 1
    const int pc = k / b * b, bb = std::min(b, N - pc);
    const int c_bulk = mode == 2 ? k + 1 : (mode == 1 ? std::min(N, pc + 2 * bb) : pc + bb);
    // sum_{c>k} nC(k,c) * sum_{r>=c} nL(k,r)
    double suf = 0;
    for (int r = N - 1; r > k; r--) {
      suf += bl[tri_index(N, k, r)];
      const double w = (double)bc[tri_index(N, k, r)] * suf;
      tot += w;
      if (r >= c_bulk) blk += w;
    }
  }
  *total = tot;
  *bulk = blk;
  return hipSuccess;
}

}  // namespace hk

extern "C" {

hk_status hk_matrix_destroy(hk_matrix m) {
  if (!m) return HK_OK;
  for (auto& e : m->ev) (void)hipEventDestroy(e);
  for (auto& e : m->gev) (void)hipEventDestroy(e);
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->sgexec) (void)hipGraphExecDestroy(m->sgexec);
  if (m->sgraph) (void)hipGraphDestroy(m->sgraph);
  if (m->gcap) (void)hipStreamDestroy(m->gcap);
  if (m->gcap2) (void)hipStreamDestroy(m->gcap2);
  if (m->s2) (void)hipStreamDestroy(m->s2);
  delete m;
  return HK_OK;
}

hk_status hk_set_panel(hk_matrix m, int panel) {
  if (!m || panel < 1 || panel > 64) return fail(HK_EINVAL, "panel must be in [1, 64]");
  m->panel = panel;
  return HK_OK;
}
hk_status hk_set_lookahead(hk_matrix m, int mode) {
  if (!m || mode < -1 || mode > 2) return fail(HK_EINVAL, "look-ahead mode must be -1, 0, 1 or 2");
  m->lookahead = mode;
  return HK_OK;
}
hk_status hk_set_timing(hk_matrix m, int on) {
  if (!m) return fail(HK_EINVAL, "null matrix");
  m->timing = on ? 1 : 0;
  return HK_OK;
}

hk_status hk_matrix_info(hk_matrix m, hk_info* o) {
  if (!m || !o) return fail(HK_EINVAL, "null argument");
  const Plan& P = m->P;
  o->N = P.N; o->K = P.K; o->h = P.h; o->digit_bits = DB;
  o->max_col_digits = P.maxW; o->vec_digits = P.VW; o->solve_guard_bits = m->gbits;
  o->panel = m->panel; o->ws_bytes = P.total;
  o->vec_bytes = sizeof(int32_t) * (size_t)P.N * P.VW;
  o->n_update_launches = m->n_update; o->update_ms = m->update_ms;
  o->n_bulk_launches = m->n_bulk; o->bulk_ms = m->bulk_ms;
  o->lookahead = lookahead_mode(m->lookahead, P.N, P.maxW);
  o->update_engine = o->lookahead != 2 && mma_width(m->B, m->panel) > 0 ? 1 : 0;
  return HK_OK;
}

hk_status hk_factor(hk_matrix m, hk_mpf shift, int inertia_mode, hipStream_t s, int* n_negative,
                    int* first_bad_col) {
  if (!m) return fail(HK_EINVAL, "null matrix");
  const Plan& P = m->P;
  const DevPtrs& D = m->D;
  MP xf;
  if (!shift_fixed(shift, P.K, xf)) return fail(HK_EINVAL, "shift has more than K fractional bits");
  if (xf.bitlen() > m->X[0].bitlen() + 64 && xf.bitlen() > (int64_t)P.K + 8)
    return fail(HK_EINVAL, "shift too large for the planned widths");
  m->xs_host.assign(P.WX, 0);
  if (!to_digits(xf, m->xs_host.data(), P.WX)) return fail(HK_EINVAL, "shift too wide");
  HK_HIP(hipMemcpyAsync(D.xs, m->xs_host.data(), sizeof(int32_t) * P.WX, hipMemcpyHostToDevice, s));
  const int N = P.N, b = m->panel;
  m->n_update = 0;
  m->update_ms = 0;
  m->n_bulk = 0;
  m->bulk_ms = 0;
  std::vector<TimedLaunch> evs;
  if (m->timing || m->eager) {
    // launched one by one on s (per-launch timing, or a caller that needs
    // every launch on its own stream with nothing captured or created)
    size_t evi = 0;
    HK_HIP(launch_fill32(D.flags, 16, 0, s));
    HK_HIP(launch_fill32(D.flags + 1, 1, INT_MAX, s));
    const int la = effective_lookahead(m);
    const std::string why = factor_lds_check(m->B, la);
    if (!why.empty()) return fail(HK_EINVAL, why);
    if (!m->s2 && la == 1) HK_HIP(hipStreamCreateWithFlags(&m->s2, hipStreamNonBlocking));
    HK_HIP(enqueue_factor(m->B, b, la, s, la == 1 ? m->s2 : nullptr, m->timing ? &evs : nullptr, &m->ev, &evi,
                          &m->n_update, &m->n_bulk));
  } else {
    const int la = lookahead_mode(m->lookahead, P.N, P.maxW);
    if (!m->gexec || m->gpanel != b || m->gla != la || m->gipw != m->B.ipw || m->gmma != m->B.mma) {
      const std::string why = factor_lds_check(m->B, la);
      if (!why.empty()) return fail(HK_EINVAL, why);
      if (m->gexec) { (void)hipGraphExecDestroy(m->gexec); m->gexec = nullptr; }
      if (m->graph) { (void)hipGraphDestroy(m->graph); m->graph = nullptr; }
      if (!m->gcap) HK_HIP(hipStreamCreateWithFlags(&m->gcap, hipStreamNonBlocking));
      HK_HIP(hipStreamBeginCapture(m->gcap, hipStreamCaptureModeThreadLocal));
      int nu = 0, nbk = 0;
      hipError_t e = launch_fill32(D.flags, 16, 0, m->gcap);
      if (e == hipSuccess) e = launch_fill32(D.flags + 1, 1, INT_MAX, m->gcap);
      size_t evi = 0;
      if (e == hipSuccess && !m->gcap2 && la == 1) e = hipStreamCreateWithFlags(&m->gcap2, hipStreamNonBlocking);
      if (e == hipSuccess)
        e = enqueue_factor(m->B, b, la, m->gcap, la == 1 ? m->gcap2 : nullptr, nullptr, &m->gev, &evi, &nu, &nbk);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(m->gcap, &g);
      m->graph = g;
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&m->gexec, m->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) return fail(HK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      m->gpanel = b;
      m->gla = la;
      m->gipw = m->B.ipw;
      m->gmma = m->B.mma;
      m->g_nupdate = nu;
      m->g_nbulk = nbk;
    }
    HK_HIP(hipGraphLaunch(m->gexec, s));
    m->n_update = m->g_nupdate;
    m->n_bulk = m->g_nbulk;
  }
  HK_HIP(hipMemcpyAsync(m->flags_host, D.flags, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, s));
  HK_HIP(hipStreamSynchronize(s));
  for (auto& tl : evs) {
    float ms = 0;
    HK_HIP(hipEventElapsedTime(&ms, tl.t0, tl.t1));
    m->update_ms += ms;
    if (tl.bulk) m->bulk_ms += ms;
  }
  m->factored = true;
  const int fb = m->flags_host[1] == INT_MAX ? -1 : m->flags_host[1];
  if (first_bad_col) *first_bad_col = fb;
  if (n_negative) *n_negative = m->flags_host[2];
  if (m->flags_host[0]) {
    m->factored = false;
    return fail(HK_EPRECISION, "fixed-point width exceeded (flags " + std::to_string(m->flags_host[0]) + ")");
  }
  if (fb >= 0 && (fb < N - 1 || !inertia_mode)) {
    if (fb < N - 1) m->factored = false;
    return fail(HK_ENOTSPD, "pivot <= 0 at column " + std::to_string(fb));
  }
  return HK_OK;
}

int64_t hk_factor_export(hk_matrix m, int kind, int c0, int c1, int32_t* slen, int64_t* off,
                         uint32_t* dig, int64_t dig_cap, hipStream_t s) {
  if (!m || kind < 0 || kind > 2 || c0 < 0 || c1 > m->P.N || c0 > c1) { g_err = "bad export range"; return -1; }
  const Plan& P = m->P;
  const DevPtrs& D = m->D;
  const int N = P.N;
  std::vector<MP> vals;
  std::vector<int32_t> nw(P.ntri);
  if (hipMemcpyAsync(nw.data(), kind == 1 ? D.nL : D.nC, sizeof(int32_t) * P.ntri,
                     hipMemcpyDeviceToHost, s) != hipSuccess) { g_err = "copy failed"; return -1; }
  for (int pc = c0; pc < c1; pc++) {
    const ColInfo& ci = P.cols[pc];
    if (kind == 1) {
      if (pc == N - 1) continue;
      std::vector<int32_t> buf((size_t)ci.LW * ci.R);
      if (hipMemcpyAsync(buf.data(), D.L + ci.loff, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { g_err = "copy failed"; return -1; }
      for (int r = pc + 1; r < N; r++) {
        int n = std::min(nw[tri_index(N, pc, r)], ci.LW);
        vals.push_back(digits_to_mp(buf.data() + (r - pc), n, ci.R));
      }
    } else {
      const int rows = kind == 0 ? N - pc : 1;
      std::vector<int32_t> buf((size_t)rows * ci.CW);
      if (hipMemcpyAsync(buf.data(), D.C + ci.coff, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { g_err = "copy failed"; return -1; }
      for (int i = 0; i < rows; i++) {
        int n = std::min(nw[tri_index(N, pc, pc + i)], ci.CW);
        vals.push_back(digits_to_mp(buf.data() + (size_t)i * ci.CW, n, 1));
      }
    }
  }
  int64_t total = 0;
  for (auto& v : vals) total += (int64_t)v.d.size();
  if (!dig) return total;
  if (total > dig_cap) { g_err = "digit buffer too small"; return -1; }
  int64_t pos = 0;
  for (size_t i = 0; i < vals.size(); i++) {
    slen[i] = vals[i].neg ? -(int32_t)vals[i].d.size() : (int32_t)vals[i].d.size();
    off[i] = pos;
    if (!vals[i].d.empty()) memcpy(dig + pos, vals[i].d.data(), sizeof(uint32_t) * vals[i].d.size());
    pos += (int64_t)vals[i].d.size();
  }
  return total;
}

hk_status hk_factor_limb_macs(hk_matrix m, hipStream_t s, double* limb_macs) {
  if (!m || !limb_macs) return fail(HK_EINVAL, "null argument");
  if (!m->factored) return fail(HK_EINVAL, "no factorisation");
  double bulk = 0;
  HK_HIP(limb_macs_split(m, m->panel, effective_lookahead(m), s, limb_macs, &bulk));
  return HK_OK;
}

}  // extern "C"
