// Eigenvalue drivers of the hk library (host control flow; every
// factorisation and solve runs on the GPU through hk_factor / hk_solve).
//
//  * Secant ("The Secant Algorithm"): P(x) = det(M - xI) is the product of
//    the LDL^T pivots; start at x1 = -2^-ceil(K/4) and x2 = 0 (the paper asks
//    for a small negative x1 and x2 = 0), iterate
//        x_{i+1} = x_i - (x_i - x_{i-1}) r / (r - 1),  r = P(x_i) / P(x_{i-1}),
//    r formed as the product of per-pivot ratios floored to F = K/2 + 64 +
//    bitlen(N) fractional bits, the running product truncated to F bits, and
//    x_{i+1} rounded to K fractional bits (ties to even).  Stop when
//    |x_{i+1} - x_i| <= 10^-tol x_{i+1}.  If rounding carries an iterate to
//    or past the computed root, the last two points bracket it and the same
//    secant formula continues on the bracket (Illinois regula falsi).
//  * Verification ("Interval Verification"): lambda truncated to `digits`
//    significant digits must leave every pivot positive, one unit more in
//    the last digit must give exactly one negative pivot (Sylvester).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hk_batch.hpp"

using namespace hk;

namespace {

hk_status dfail(hk_status st, const std::string& msg) { g_err = msg; return st; }

// HK_TRACE=1 in the environment: one line on stderr per factorisation and
// per solve of the drivers (long runs report their progress as they go)
bool trace_on() {
  static const bool on = [] { const char* v = getenv("HK_TRACE"); return v && v[0] == '1'; }();
  return on;
}

MP one_shl(int64_t s) { return shl(MP::from_u64(1), s); }

// floor(x / 2^s)
MP floor_shr(const MP& x, int64_t s) {
  MP q = shr_mag(x, s);
  if (x.neg && !low_bits_zero(x, s)) q = sub(q, MP::from_u64(1));
  return q;
}

hk_status pivots_host(hk_matrix m, hipStream_t s, std::vector<MP>& out) {
  const Plan& P = m->P;
  const int ld = P.maxW + WB;
  hipError_t e = launch_gather_pivots_b(m->B, m->D.vec, ld, s);
  std::vector<int32_t> buf((size_t)P.N * ld);
  if (e == hipSuccess) e = hipMemcpyAsync(buf.data(), m->D.vec, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail(HK_EDEVICE, std::string("pivot copy: ") + hipGetErrorString(e));
  out.resize(P.N);
  for (int k = 0; k < P.N; k++) out[k] = digits_to_mp(buf.data() + (size_t)k * ld, ld, 1);
  return HK_OK;
}

// R = prod_k t_k with t_k = floor(2^F dn_k / dold_k) and the running product
// floored to F fractional bits after every factor.  Written as
// t_k = 2^F + e_k, e_k = floor(2^F (dn_k - dold_k) / dold_k), and
// floor(R t_k / 2^F) = R + floor(R e_k / 2^F): the same values, but the
// pivots of nearby shifts differ only in their low digits, so e_k is short
// and so are its division and product.  The divisions are independent and
// run on `threads` host threads; the product runs in k order.
MP pivot_ratio(const std::vector<MP>& dn, const std::vector<MP>& dold, int64_t F, int threads) {
  const int n = (int)dn.size();
  std::vector<MP> e(n);
  // a thread per 32 pivots at most: below that, starting it costs more
  parallel_for(n, std::min(threads, n / 32),
               [&](int k) { e[k] = floor_div(shl(sub(dn[k], dold[k]), F), dold[k]); });
  MP R = one_shl(F);
  for (int k = 0; k < n; k++)
    if (!e[k].is_zero()) R = add(R, floor_shr(mul(R, e[k]), F));
  return R;
}

// |a| <= 10^-tol * b  for b > 0
bool within_tol(const MP& a, const MP& b, int tol) {
  MP lhs = mul(a, pow10((uint32_t)tol));
  lhs.neg = false;
  return cmp(lhs, b) <= 0;
}

hk_mpf fixed_mpf(const MP& v, int K, std::vector<uint32_t>& keep) {
  keep = v.d;
  if (keep.empty()) keep.push_back(0);
  hk_mpf f;
  f.sign = v.sign();
  f.ndigits = (int32_t)keep.size();
  f.exp2 = -K;
  f.digits = keep.data();
  return f;
}

struct Eval {
  hk_status st;
  int nneg, first_bad;
  std::vector<MP> piv;
};

}  // namespace

namespace hk {

struct DriverCtx {
  hk_matrix m;
  hipStream_t s;
  int nfact = 0;
  double limb_macs = 0;
  double t_factor = 0;
  double t_solve = 0;
  bool count_macs = true;
  bool certify = false;       // rigorous inertia of the bracket factorisations
  int certified = 0;
  double certify_margin = 0;
  int upd_launches = 0;
  double upd_ms = 0;
  int bulk_launches = 0;
  double bulk_ms = 0;
  double limb_macs_bulk = 0;
};

hk_status inverse_driver(DriverCtx& cx, const hk_mpf* shift_hint, int tol, int max_iter, MP& lam,
                         int& solves);

static Eval evaluate(DriverCtx& cx, const MP& x, int inertia_mode) {
  Eval ev;
  std::vector<uint32_t> keep;
  hk_mpf f = fixed_mpf(x, cx.m->P.K, keep);
  auto t0 = std::chrono::steady_clock::now();
  ev.st = hk_factor(cx.m, f, inertia_mode, cx.s, &ev.nneg, &ev.first_bad);
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  cx.t_factor += dt;
  cx.nfact++;
  if (trace_on())
    fprintf(stderr, "[hk] factorisation %d (N=%d K=%d): status %d, %.2f s\n", cx.nfact, cx.m->P.N, cx.m->P.K,
            (int)ev.st, dt);
  {
    hk_info inf;
    if (hk_matrix_info(cx.m, &inf) == HK_OK) {
      cx.upd_launches += inf.n_update_launches;
      cx.upd_ms += inf.update_ms;
      cx.bulk_launches += inf.n_bulk_launches;
      cx.bulk_ms += inf.bulk_ms;
    }
  }
  if (ev.st == HK_OK && cx.count_macs) {
    double lm = 0, lb = 0;
    if (limb_macs_split(cx.m, cx.m->panel, effective_lookahead(cx.m), cx.s, &lm, &lb) == hipSuccess) {
      cx.limb_macs += lm;
      cx.limb_macs_bulk += lb;
    }
  }
  if (ev.st == HK_OK) {
    hk_status st = pivots_host(cx.m, cx.s, ev.piv);
    if (st != HK_OK) ev.st = st;
  }
  return ev;
}

// The Secant iteration as a resumable machine: next() names the point to
// factor (and whether inertia mode is wanted), feed() consumes the result.
// Used one instance at a time and across a batch.
struct SecantMachine {
  enum Phase { START0, START1, ITER, BRACKET, DONE, FAILED } phase = START0;
  int K = 0, tol = 45, max_eval = 200, nevals = 0;
  int threads = 1;  // host threads of the pivot ratio
  int64_t F = 0;
  MP ONE, lam;
  hk_status status = HK_OK;
  std::string err;
  std::vector<MP> xs;
  std::vector<std::vector<MP>> piv;
  MP prev_step;
  bool have_prev = false;
  int it = 0;
  MP pending;
  // bracket state: P(a) > 0 >= P(b)
  MP a, b;
  std::vector<MP> da, db;
  int scale_a = 0, scale_b = 0, side = 0;

  void init(int N, int K_, int h, int tol_, int max_eval_) {
    K = K_; tol = tol_; max_eval = max_eval_;
    threads = host_threads();
    int nb = 0;
    for (int n = N; n; n >>= 1) nb++;
    F = h + 64 + nb;
    ONE = one_shl(F);
    xs = {neg(one_shl(K - (K + 3) / 4)), MP()};
  }
  MP secant_point(const MP& xa, const MP& xb, const MP& R) const {
    MP Rm1 = sub(R, ONE);
    return rne_div(sub(mul(xb, Rm1), mul(sub(xb, xa), R)), Rm1);
  }
  void fail(hk_status st, const std::string& m) { phase = FAILED; status = st; err = m; }
  // false when finished (DONE or FAILED)
  bool next(MP& x, int& inertia) {
    if (phase == DONE || phase == FAILED) return false;
    if (nevals >= max_eval) { fail(HK_ENOCONV, "secant did not converge"); return false; }
    if (phase == START0 || phase == START1) {
      x = xs[phase == START0 ? 0 : 1];
      inertia = 0;
      return true;
    }
    if (phase == ITER) {
      const MP& x0 = xs[xs.size() - 2];
      const MP& x1 = xs.back();
      MP R = pivot_ratio(piv.back(), piv[piv.size() - 2], F, threads);
      if (cmp(R, ONE) >= 0) { fail(HK_EPRECISION, "secant ratio >= 1: precision exhausted"); return false; }
      MP x2 = secant_point(x0, x1, R);
      MP step = sub(x2, x1);
      if (step.sign() <= 0) { fail(HK_EPRECISION, "secant iterate did not increase"); return false; }
      if (have_prev && cmp(step, prev_step) >= 0 && it > 2) {
        fail(HK_EPRECISION, "secant step did not shrink");
        return false;
      }
      prev_step = step;
      have_prev = true;
      it++;
      if (within_tol(step, x2, tol)) { lam = x2; phase = DONE; return false; }
      pending = x2;
      x = x2;
      inertia = 1;
      return true;
    }
    // BRACKET
    if (within_tol(sub(b, a), a, tol)) { lam = a; phase = DONE; return false; }
    MP c;
    bool have_c = false;
    if (!db.empty()) {
      MP Rb = pivot_ratio(db, da, F, threads);
      if (scale_b <= scale_a) Rb = shl(floor_shr(Rb, scale_b), scale_a);
      else Rb = floor_shr(Rb, scale_b - scale_a);
      if (cmp(Rb, ONE) != 0) { c = secant_point(a, b, Rb); have_c = true; }
    }
    if (!have_c || cmp(c, a) <= 0 || cmp(c, b) >= 0) c = floor_shr(add(a, b), 1);
    pending = c;
    x = c;
    inertia = 1;
    return true;
  }
  void feed(Eval&& ev) {
    nevals++;
    const bool left = ev.st == HK_OK && ev.nneg == 0 && ev.first_bad < 0;
    if (phase == START0 || phase == START1) {
      if (ev.st != HK_OK) {
        if (ev.st == HK_ENOTSPD) fail(HK_ENOTSPD, "start point not left of lambda_1");
        else fail(ev.st, "factorisation failed");
        return;
      }
      piv.push_back(std::move(ev.piv));
      phase = phase == START0 ? START1 : ITER;
      return;
    }
    if (ev.st != HK_OK && ev.st != HK_ENOTSPD) { fail(ev.st, "factorisation failed"); return; }
    if (phase == ITER) {
      if (left) { xs.push_back(pending); piv.push_back(std::move(ev.piv)); return; }
      a = xs.back(); b = pending;
      da = piv.back();
      db = ev.st == HK_OK ? ev.piv : std::vector<MP>();
      scale_a = scale_b = side = 0;
      phase = BRACKET;
      return;
    }
    if (left) {
      a = pending; da = ev.piv; scale_a = 0;
      if (side == -1) scale_b++;
      side = -1;
    } else {
      b = pending; db = ev.st == HK_OK ? ev.piv : std::vector<MP>(); scale_b = 0;
      if (side == 1) scale_a++;
      side = 1;
    }
  }
};

hk_status secant_driver(DriverCtx& cx, int tol, int max_iter, MP& lam_fixed) {
  const Plan& P = cx.m->P;
  SecantMachine sm;
  sm.init(P.N, P.K, P.h, tol, max_iter);
  MP x;
  int inertia;
  while (sm.next(x, inertia)) sm.feed(evaluate(cx, x, inertia));
  if (sm.phase != SecantMachine::DONE) return dfail(sm.status, sm.err);
  lam_fixed = sm.lam;
  return HK_OK;
}

// lambda = x / 2^K truncated to `digits` significant digits: D * 10^e
static void truncate_digits(const MP& x, int K, int digits, MP& D, int64_t& e) {
  const double l10 = ((double)x.bitlen() - K) * 0.30102999566398120;
  e = (int64_t)std::floor(l10) - (digits - 1) - 1;
  const MP lo = pow10((uint32_t)(digits - 1)), hi = pow10((uint32_t)digits);
  for (int guard = 0; guard < 8; guard++) {
    // D = floor(x / (2^K 10^e))
    MP num = x, den = one_shl(K);
    if (e >= 0) den = mul(den, pow10((uint32_t)e));
    else num = mul(num, pow10((uint32_t)(-e)));
    D = floor_div(num, den);
    if (cmp(D, hi) >= 0) e++;
    else if (cmp(D, lo) < 0) e--;
    else return;
  }
}

// fixed point (K fractional bits) of D * 10^e, floor or ceil
MP decimal_to_fixed(const MP& D, int64_t e, int K, bool ceil_mode) {
  MP num = shl(D, K), den = MP::from_u64(1);
  if (e >= 0) num = mul(num, pow10((uint32_t)e));
  else den = pow10((uint32_t)(-e));
  return ceil_mode ? ceil_div(num, den) : floor_div(num, den);
}

// decimal form of lambda (digits significant digits) and the two bracket
// points: truncated value floored to K bits, one unit more ceiled
void decimal_bracket(const MP& lam, int K, int digits, MP& xlo, MP& xhi, std::string& dec) {
  MP D;
  int64_t e;
  truncate_digits(lam, K, digits, D, e);
  std::string ds = to_dec(D);
  char buf[64];
  snprintf(buf, sizeof buf, "e%lld", (long long)(e + (int64_t)ds.size() - 1));
  dec = ds.substr(0, 1) + "." + ds.substr(1) + buf;
  xlo = decimal_to_fixed(D, e, K, false);
  xhi = decimal_to_fixed(add(D, MP::from_u64(1)), e, K, true);
}

// "d.ddd...e[+-]x" -> its first `digits` significant digits D and e with
// value D * 10^e (truncated); false on a malformed or non-positive string
bool parse_decimal(const char* str, int digits, MP& D, int64_t& e) {
  if (!str || digits < 1) return false;
  std::string ds;
  int64_t exp10 = 0, point = -1;
  const char* p = str;
  for (; *p && *p != 'e' && *p != 'E'; p++) {
    if (*p == '.') { if (point >= 0) return false; point = (int64_t)ds.size(); continue; }
    if (*p < '0' || *p > '9') return false;
    ds.push_back(*p);
  }
  if (*p) {
    char* end = nullptr;
    exp10 = strtoll(p + 1, &end, 10);
    if (!end || *end) return false;
  }
  if (point < 0) point = (int64_t)ds.size();
  size_t lead = ds.find_first_not_of('0');
  if (lead == std::string::npos) return false;
  // value = 0.ds * 10^(point + exp10) with ds starting at its first nonzero digit
  const int64_t mag = point - (int64_t)lead + exp10;   // value in [10^(mag-1), 10^mag)
  ds = ds.substr(lead);
  if ((int)ds.size() > digits) ds.resize(digits);
  while ((int)ds.size() < digits) ds.push_back('0');
  D = MP();
  for (char c : ds) D = add(mul_small(D, 10), MP::from_u64((uint64_t)(c - '0')));
  e = mag - digits;
  return true;
}

// lambda (K fractional bits) as an hk_mpf over the caller's words: rounded
// to nearest, ties to even, to at most 32 HK_LAMBDA_WORDS significant bits
void lambda_mpf(const MP& lam, int K, hk_mpf* out, uint32_t* words) {
  memset(words, 0, sizeof(uint32_t) * HK_LAMBDA_WORDS);
  out->sign = 0; out->ndigits = 0; out->exp2 = 0; out->digits = words;
  if (lam.d.empty()) return;
  const int64_t cap = 32 * (int64_t)HK_LAMBDA_WORDS;
  int64_t drop = std::max<int64_t>(0, lam.bitlen() - cap);
  MP v = rne_shr(lam, drop);
  if (v.bitlen() > cap) { v = shr_mag(v, 1); drop += 1; }   // rounding carried into a new top bit (exact)
  out->sign = lam.neg ? -1 : 1;
  out->ndigits = (int32_t)v.d.size();
  out->exp2 = drop - K;
  for (size_t i = 0; i < v.d.size(); i++) words[i] = v.d[i];
}

std::string decimal_string(const MP& lam, int K, int digits) {
  MP xlo, xhi;
  std::string dec;
  decimal_bracket(lam, K, digits, xlo, xhi, dec);
  return dec;
}

bool agree(const MP& a, const MP& b, int tol) {
  MP bb = b;
  bb.neg = false;
  return within_tol(sub(a, b), bb, tol);
}

struct SecantRun { SecantMachine m; };
SecantRun* secant_new(int N, int K, int h, int tol, int max_eval) {
  SecantRun* r = new SecantRun;
  r->m.init(N, K, h, tol, max_eval);
  return r;
}
void secant_delete(SecantRun* r) { delete r; }
void secant_threads(SecantRun* r, int threads) { r->m.threads = std::max(1, threads); }
bool secant_next(SecantRun* r, MP& x, int& inertia) { return r->m.next(x, inertia); }
// both start points while the machine waits for the first
bool secant_start_pair(SecantRun* r, MP& x0, MP& x1) {
  if (r->m.phase != SecantMachine::START0) return false;
  x0 = r->m.xs[0];
  x1 = r->m.xs[1];
  return true;
}
void secant_feed(SecantRun* r, hk_status st, int nneg, int first_bad, std::vector<MP>&& piv) {
  Eval ev;
  ev.st = st; ev.nneg = nneg; ev.first_bad = first_bad; ev.piv = std::move(piv);
  r->m.feed(std::move(ev));
}
bool secant_done(SecantRun* r, MP& lam, hk_status& st, std::string& err) {
  lam = r->m.lam;
  st = r->m.status;
  err = r->m.err;
  return r->m.phase == SecantMachine::DONE;
}

hk_status verify_bracket(DriverCtx& cx, const MP& lam_fixed, int digits, std::string& dec, bool& ok) {
  const int K = cx.m->P.K;
  ok = false;
  if (lam_fixed.sign() <= 0) return dfail(HK_EVERIFY, "non-positive eigenvalue estimate");
  MP D;
  int64_t e;
  truncate_digits(lam_fixed, K, digits, D, e);
  std::string ds = to_dec(D);
  char buf[64];
  snprintf(buf, sizeof buf, "e%lld", (long long)(e + (int64_t)ds.size() - 1));
  dec = ds.substr(0, 1) + "." + ds.substr(1) + buf;
  MP xlo = decimal_to_fixed(D, e, K, false);
  MP xhi = decimal_to_fixed(add(D, MP::from_u64(1)), e, K, true);
  Eval a = evaluate(cx, xlo, 1);
  if (a.st != HK_OK && a.st != HK_ENOTSPD) return a.st;
  int ca = 0, cb = 0, na = 0, nb = 0;
  double ma = -INFINITY, mb = -INFINITY;
  if (cx.certify && a.st == HK_OK) {
    const hk_status st = certify_factor(cx.m, cx.s, a.piv, &na, &ca, &ma, nullptr);
    if (st != HK_OK) return st;
  }
  Eval b = evaluate(cx, xhi, 1);
  if (b.st != HK_OK && b.st != HK_ENOTSPD) return b.st;
  ok = a.st == HK_OK && a.nneg == 0 && a.first_bad < 0 && b.st == HK_OK && b.nneg == 1 &&
       b.first_bad == cx.m->P.N - 1;
  if (cx.certify && b.st == HK_OK) {
    const hk_status st = certify_factor(cx.m, cx.s, b.piv, &nb, &cb, &mb, nullptr);
    if (st != HK_OK) return st;
  }
  if (cx.certify) {
    // proved: all pivots certified, none negative at the lower point, only
    // the last one negative at the upper point
    cx.certified = ok && ca && cb && na == 0 && nb == 1;
    cx.certify_margin = std::min(ma, mb);
  }
  return HK_OK;
}

}  // namespace hk

namespace hk {

// device vector (N rows of VW balanced digits) -> host integers
static hk_status vec_to_host(hk_matrix m, const int32_t* dev, hipStream_t s, std::vector<MP>& out) {
  const Plan& P = m->P;
  std::vector<int32_t> buf((size_t)P.N * P.VW);
  hipError_t e = hipMemcpyAsync(buf.data(), dev, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail(HK_EDEVICE, hipGetErrorString(e));
  out.resize(P.N);
  for (int i = 0; i < P.N; i++) out[i] = digits_to_mp(buf.data() + (size_t)i * P.VW, P.VW, 1);
  return HK_OK;
}

// Inverse iteration (not in the paper): one factorisation of M - sigma I,
// then y = (M - sigma I)^{-1} v on the GPU, lambda = sigma + <v,v>/<v,y> from
// exact integer dots, v <- RNE(y 2^K / max|y|) on the GPU; v0 = all ones.
// Stops when |lambda_k - lambda_{k-1}| <= 10^-tol lambda_k.  A shift hint
// that is not below lambda_1 (a pivot <= 0) is halved up to three times,
// then 0 is used.
hk_status inverse_driver(DriverCtx& cx, const hk_mpf* shift_hint, int tol, int max_iter, MP& lam,
                         int& solves) {
  const int K = cx.m->P.K;
  solves = 0;
  MP sigma;
  if (shift_hint) {
    MP v;
    if (shift_hint->sign != 0 && shift_hint->ndigits > 0) {
      v.d.assign(shift_hint->digits, shift_hint->digits + shift_hint->ndigits);
      v.trim();
      v.neg = shift_hint->sign < 0 && !v.d.empty();
    }
    const int64_t e = shift_hint->exp2 + K;
    sigma = e >= 0 ? shl(v, e) : floor_shr(v, -e);
  }
  for (int attempt = 0;; attempt++) {
    Eval ev = evaluate(cx, sigma, 0);
    if (ev.st == HK_OK) break;
    if (ev.st != HK_ENOTSPD || sigma.is_zero()) return ev.st;
    sigma = attempt < 3 ? floor_shr(sigma, 1) : MP();
  }
  return inverse_iterate(cx.m, cx.s, sigma, tol, max_iter, lam, solves, cx.t_solve);
}

// The iteration proper on a factorisation of M - sigma I.  Besides the
// tolerance test it stops, returning the last estimate, once the change of
// the estimate has fallen below 10^-(tol/2) of it and then fails to shrink
// twice in a row: the iterates have reached the rounding floor of the
// fixed-point solve at this K.
hk_status inverse_iterate(hk_matrix m, hipStream_t s, const MP& sigma, int tol, int max_iter, MP& lam,
                          int& solves, double& t_solve) {
  const Plan& P = m->P;
  const int K = P.K, N = P.N;
  solves = 0;
  const int g = m->gbits;
  // v0 = 1 (K fractional bits)
  std::vector<MP> v(N, one_shl(K));
  {
    std::vector<int32_t> buf((size_t)N * P.VW, 0);
    for (int i = 0; i < N; i++) mp_to_digits(v[i], buf.data() + (size_t)i * P.VW, P.VW);
    hipError_t e = hipMemcpyAsync(m->D.dv1, buf.data(), sizeof(int32_t) * buf.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dfail(HK_EDEVICE, hipGetErrorString(e));
  }
  const int64_t F = 2 * (int64_t)K + 64;   // fixed-point bits of the lambda iterates
  MP lam_prev, step_prev;
  bool have_prev = false, have_step = false;
  int no_shrink = 0;
  std::vector<MP> y;
  for (int it = 0; it < max_iter; it++) {
    auto t0 = std::chrono::steady_clock::now();
    hk_status st = hk_solve(m, m->D.dv1, m->D.dv2, s);
    solves++;
    if (trace_on()) fprintf(stderr, "[hk] solve %d (N=%d K=%d): status %d\n", solves, N, P.K, (int)st);
    if (st != HK_OK) return st;
    st = vec_to_host(m, m->D.dv2, s, y);
    t_solve += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st != HK_OK) return st;
    // v.y and v.v in exact integers: partial sums on host threads, then added
    const int nt = std::max(1, std::min(host_threads(), N / 32));
    std::vector<MP> pvy(nt), pvv(nt);
    parallel_for(nt, nt, [&](int t) {
      for (int i = t; i < N; i += nt) { pvy[t] = add(pvy[t], mul(v[i], y[i])); pvv[t] = add(pvv[t], mul(v[i], v[i])); }
    });
    MP vy, vv;
    for (int t = 0; t < nt; t++) { vy = add(vy, pvy[t]); vv = add(vv, pvv[t]); }
    if (vy.sign() <= 0) return dfail(HK_EPRECISION, "non-positive Rayleigh quotient");
    // lambda 2^F = sigma 2^(F-K) + vv 2^(g+F) / vy
    MP lamF = add(shl(sigma, F - K), floor_div(shl(vv, g + F), vy));
    if (have_prev) {
      MP step = sub(lamF, lam_prev);
      step.neg = false;
      if (within_tol(step, lamF, tol)) {
        lam = rne_shr(lamF, F - K);
        return HK_OK;
      }
      if (have_step && within_tol(step, lamF, tol / 2) && cmp(step, step_prev) >= 0) {
        if (++no_shrink >= 2) {
          lam = rne_shr(lamF, F - K);
          return HK_OK;
        }
      } else {
        no_shrink = 0;
      }
      step_prev = step;
      have_step = true;
    }
    lam_prev = lamF;
    have_prev = true;
    // v <- RNE(y 2^K / max|y|) on the GPU (standard digits of |y| are in us)
    size_t imax = 0;
    for (int i = 1; i < N; i++) if (cmp_mag(y[i], y[imax]) > 0) imax = i;
    MP mag = y[imax];
    mag.neg = false;
    if (mag.is_zero()) return dfail(HK_EPRECISION, "zero iterate");
    const int64_t bl = mag.bitlen();
    const int sh = (int)((DB - (bl % DB)) % DB);     // top digit gets bit 28 set
    MP msh = shl(mag, sh);
    const int nd = (int)((msh.bitlen() + DB - 1) / DB);
    std::vector<uint32_t> md(nd);
    for (int i = 0; i < nd; i++) {
      const int64_t pos = (int64_t)i * DB;
      const size_t w = (size_t)(pos >> 5);
      uint64_t lo = w < msh.d.size() ? msh.d[w] : 0;
      if (w + 1 < msh.d.size()) lo |= (uint64_t)msh.d[w + 1] << 32;
      md[i] = (uint32_t)((lo >> (pos & 31)) & (RADIX - 1));
    }
    hipError_t e = hipMemcpyAsync(m->D.md, md.data(), sizeof(uint32_t) * nd, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_vscale(P, m->D, m->D.md, nd, sh, m->D.dv1, s);
    if (e != hipSuccess) return dfail(HK_EDEVICE, hipGetErrorString(e));
    st = vec_to_host(m, m->D.dv1, s, v);
    if (st != HK_OK) return st;
  }
  return dfail(HK_ENOCONV, "inverse iteration did not converge");
}

}  // namespace hk

extern "C" {

hk_status hk_solve(hk_matrix m, const void* dev_rhs, void* dev_x, hipStream_t s) {
  if (!m || !dev_rhs || !dev_x) return dfail(HK_EINVAL, "null argument");
  if (!m->factored) return dfail(HK_EINVAL, "no valid factorisation");
  const Plan& P = m->P;
  const DevPtrs& D = m->D;
  {
    const std::string why = solve_lds_check(sweep_shape({&P}));
    if (!why.empty()) return dfail(HK_EINVAL, why);
  }
  // the batched sweeps with one instance: forward (acc = b 2^(h+g), z_k =
  // RNE(acc_k / 2^h) column by column), w_k = RNE(z_k 2^h / d_k), backward
  // (acc = w 2^h, y_k = RNE(acc_k / 2^h), last row first)
  // The launch sequence depends only on the plan, so it is captured once as a
  // HIP graph and replayed; the operands travel in the uploaded arguments.
  m->sweep = make_sweep_args(P, D, 1, m->gbits);
  m->sweep.v = (int32_t*)dev_rhs;
  m->sweep.y = (int32_t*)dev_x;
  hipError_t e = hipSuccess;
  if (m->eager) {
    // every launch on s, nothing captured
    e = hipMemcpyAsync(D.sargs, &m->sweep, sizeof(SweepArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill32(D.flags, 16, 0, s);
    if (e == hipSuccess) e = enqueue_solve(D.sargs, sweep_shape({&P}), s);
  } else if (!m->sgexec) {
    const SweepShape sh = sweep_shape({&P});
    if (!m->gcap) e = hipStreamCreateWithFlags(&m->gcap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(m->gcap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ec = launch_fill32(D.flags, 16, 0, m->gcap);
      if (ec == hipSuccess) ec = enqueue_solve(D.sargs, sh, m->gcap);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(m->gcap, &g);
      m->sgraph = g;
      e = ec != hipSuccess ? ec : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&m->sgexec, m->sgraph, nullptr, nullptr, 0);
    if (e != hipSuccess) return dfail(HK_EDEVICE, std::string("solve graph: ") + hipGetErrorString(e));
  }
  if (!m->eager) {
    e = hipMemcpyAsync(D.sargs, &m->sweep, sizeof(SweepArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipGraphLaunch(m->sgexec, s);
  }
  int32_t fl[16];
  if (e == hipSuccess) e = hipMemcpyAsync(fl, D.flags, sizeof fl, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail(HK_EDEVICE, std::string("solve: ") + hipGetErrorString(e));
  if (fl[0]) return dfail(HK_EPRECISION, "solve: fixed-point width exceeded (flags " + std::to_string(fl[0]) + ")");
  return HK_OK;
}

hk_status hk_vec_import(hk_matrix m, int n, const int32_t* slen, const int64_t* off,
                        const uint32_t* dig, void* dev_vec, hipStream_t s) {
  if (!m || !dev_vec || n != m->P.N) return dfail(HK_EINVAL, "vector length must be N");
  const int VW = m->P.VW;
  std::vector<int32_t> buf((size_t)n * VW, 0);
  for (int i = 0; i < n; i++) {
    MP v;
    int nd = slen[i] < 0 ? -slen[i] : slen[i];
    v.d.assign(dig + off[i], dig + off[i] + nd);
    v.trim();
    v.neg = slen[i] < 0 && !v.d.empty();
    mp_to_digits(v, buf.data() + (size_t)i * VW, VW);
    if (v.bitlen() > (int64_t)(VW - 2) * DB) return dfail(HK_EINVAL, "vector entry too wide");
  }
  hipError_t e = hipMemcpyAsync(dev_vec, buf.data(), sizeof(int32_t) * buf.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dfail(HK_EDEVICE, hipGetErrorString(e));
  return HK_OK;
}

int64_t hk_vec_export(hk_matrix m, const void* dev_vec, int n, int32_t* slen, int64_t* off,
                      uint32_t* dig, int64_t dig_cap, hipStream_t s) {
  if (!m || !dev_vec || n != m->P.N) { g_err = "vector length must be N"; return -1; }
  const int VW = m->P.VW;
  std::vector<int32_t> buf((size_t)n * VW);
  hipError_t e = hipMemcpyAsync(buf.data(), dev_vec, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { g_err = hipGetErrorString(e); return -1; }
  std::vector<MP> vals(n);
  int64_t total = 0;
  for (int i = 0; i < n; i++) { vals[i] = digits_to_mp(buf.data() + (size_t)i * VW, VW, 1); total += (int64_t)vals[i].d.size(); }
  if (!dig) return total;
  if (total > dig_cap) { g_err = "digit buffer too small"; return -1; }
  int64_t pos = 0;
  for (int i = 0; i < n; i++) {
    slen[i] = vals[i].neg ? -(int32_t)vals[i].d.size() : (int32_t)vals[i].d.size();
    off[i] = pos;
    if (!vals[i].d.empty()) memcpy(dig + pos, vals[i].d.data(), sizeof(uint32_t) * vals[i].d.size());
    pos += (int64_t)vals[i].d.size();
  }
  return total;
}

}  // extern "C"

// hk_smallest_eig's body; eager: every launch goes on s one by one (no graph
// capture, no second stream)
static hk_status smallest_eig_impl(int N, hk_rational beta, int prec_bits, int method, int digits,
                                   const hk_mpf* shift_hint, void* dev_ws, size_t ws_bytes, hipStream_t s,
                                   char* out_decimal, size_t out_len, hk_report* rep, bool eager) {
  auto t0 = std::chrono::steady_clock::now();
  if (rep) { memset(rep, 0, sizeof(*rep)); rep->bits_used = prec_bits; }
  if (digits < 2 || digits > 150) return dfail(HK_EINVAL, "digits must be in [2, 150]");
  const int flags = method & ~0xff;
  method &= 0xff;
  if (method != HK_INVERSE && method != HK_SECANT) return dfail(HK_EINVAL, "unknown method");
  hk_matrix m = nullptr;
  hk_status st = hk_build_matrix(N, beta, prec_bits, dev_ws, ws_bytes, s, &m);
  if (st != HK_OK) { if (rep) rep->status = st; return st; }
  m->eager = eager;
  DriverCtx cx;
  cx.m = m;
  cx.s = s;
  cx.count_macs = !(flags & HK_FLAG_NO_WORK_COUNT);
  cx.certify = (flags & HK_FLAG_CERTIFY) != 0;
  if (flags & HK_FLAG_TIME_UPDATES) hk_set_timing(m, 1);
  const int forced_panel = (flags >> 16) & 0xff;
  if (forced_panel > 0) hk_set_panel(m, forced_panel);
  if (flags & HK_FLAG_LOOKAHEAD_ON) hk_set_lookahead(m, 1);
  if (flags & HK_FLAG_LOOKAHEAD_OFF) hk_set_lookahead(m, 0);
  if (flags & HK_FLAG_LOOKAHEAD_FUSED) hk_set_lookahead(m, 2);
  const int forced_group = (flags >> 28) & 7;
  if (forced_group > 0) hk_set_update_group(m, forced_group);
  if (flags & HK_FLAG_VECTOR_UPDATE) hk_set_update_engine(m, HK_UPDATE_VECTOR);
  MP lam;
  int solves = 0;
  if (method == HK_SECANT) {
    st = secant_driver(cx, digits, 200, lam);
  } else {
    st = inverse_driver(cx, shift_hint, digits, 400, lam, solves);
  }
  bool ok = false;
  std::string dec;
  if (st == HK_OK) st = verify_bracket(cx, lam, digits, dec, ok);
  if (st == HK_OK && !ok) st = dfail(HK_EVERIFY, "inertia bracket failed at " + dec);
  if (out_decimal && out_len) {
    snprintf(out_decimal, out_len, "%s", dec.c_str());
  }
  if (rep) {
    rep->status = st;
    rep->factorizations = cx.nfact;
    rep->solves = solves;
    rep->verified = ok ? 1 : 0;
    rep->digits_verified = ok ? digits : 0;
    snprintf(rep->lambda_dec, sizeof rep->lambda_dec, "%s", dec.c_str());
    if (st == HK_OK) lambda_mpf(lam, prec_bits, &rep->lambda, rep->lambda_words);
    rep->limb_macs = cx.limb_macs;
    {
      hk_info inf;
      if (hk_matrix_info(m, &inf) == HK_OK) rep->update_engine = inf.update_engine;
    }
    rep->t_factor_s = cx.t_factor;
    rep->t_solve_s = cx.t_solve;
    rep->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->update_launches = cx.upd_launches;
    rep->update_ms = cx.upd_ms;
    rep->certified = cx.certified;
    rep->certify_margin_bits = cx.certify_margin;
    // the precision at which the same bracket would be proved: radii scale
    // as 2^-h, so each missing bit of margin costs two bits of K
    rep->certify_bits = !cx.certify || cx.certified ? prec_bits
        : !std::isfinite(cx.certify_margin) ? 0
        : (int)(64 * std::ceil((prec_bits + 2.0 * (std::max(0.0, -cx.certify_margin) + 16.0)) / 64.0));
    rep->bulk_launches = cx.bulk_launches;
    rep->bulk_ms = cx.bulk_ms;
    rep->limb_macs_bulk = cx.limb_macs_bulk;
  }
  hk_matrix_destroy(m);
  return st;
}

// The allocation-free variant's scratch: one array per device, the largest
// workspace hk_smallest_eig_static accepts.  Host code never passes the
// array's name to a kernel or a copy: its device address comes from
// hipGetSymbolAddress, once per device.
#define HK_STATIC_WS_BYTES ((size_t)64 << 20)
static __device__ __align__(256) unsigned char scratch[HK_STATIC_WS_BYTES];

static hk_status static_scratch(void** out) {
  static std::mutex mu;
  static void* ptr[64] = {nullptr};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return dfail(HK_EDEVICE, "no current device");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dfail(HK_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return HK_OK;
}

extern "C" {

hk_status hk_smallest_eig(int N, hk_rational beta, int prec_bits, int method, int digits,
                          const hk_mpf* shift_hint, void* dev_ws, size_t ws_bytes, hipStream_t s,
                          char* out_decimal, size_t out_len, hk_report* rep) {
  return smallest_eig_impl(N, beta, prec_bits, method, digits, shift_hint, dev_ws, ws_bytes, s, out_decimal,
                           out_len, rep, false);
}

size_t hk_static_workspace_limit(void) { return HK_STATIC_WS_BYTES; }

hk_status hk_smallest_eig_static(int N, hk_rational beta, int prec_bits, int method, int digits,
                                 const hk_mpf* shift_hint, hipStream_t s, char* out_decimal, size_t out_len,
                                 hk_report* rep) {
  if (rep) memset(rep, 0, sizeof(*rep));
  const size_t need = hk_workspace_bytes(N, beta, prec_bits, 0);
  if (need == 0) return dfail(HK_EINVAL, "invalid N, beta or precision");
  if (need > HK_STATIC_WS_BYTES)
    return dfail(HK_EINVAL, "hk_smallest_eig_static: needs " + std::to_string(need) + " bytes of workspace, " +
                            "more than its fixed " + std::to_string(HK_STATIC_WS_BYTES) +
                            "; use hk_smallest_eig with a caller buffer");
  // (per-launch timing creates events, look-ahead mode 1 a second stream)
  if (method & (HK_FLAG_LOOKAHEAD_ON | HK_FLAG_TIME_UPDATES))
    return dfail(HK_EINVAL, "hk_smallest_eig_static: no look-ahead stream and no per-launch timing");
  void* ws = nullptr;
  hk_status st = static_scratch(&ws);
  if (st != HK_OK) return st;
  return smallest_eig_impl(N, beta, prec_bits, method, digits, shift_hint, ws, HK_STATIC_WS_BYTES, s, out_decimal,
                           out_len, rep, true);
}

}  // extern "C"
