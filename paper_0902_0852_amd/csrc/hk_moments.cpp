// Correctly rounded fixed-point moments X_n = RNE(2^K mu_n) of the weight
// exp(-x^beta), mu_n = (1/beta) Gamma((n+1)/beta) (paper: the matrix
// definition in the Introduction, the moment form in "Properties of M").
//
// With beta = p/q in lowest terms and q(n+1) = m p + r (0 <= r < p):
//   r = 0:  mu_n = (q/p) (m-1)!                              (exact rational)
//   r > 0:  mu_n = (q/p) Gamma(r/p) prod_{j<m} (r + j p) / p^m
// so only Gamma(r/p), 0 < r < p, needs a transcendental evaluation.  It is
// taken from Gamma(s) = gamma(s, T) + Gamma(s, T), the lower part summed as
// the confluent series T^s e^{-T} sum_k T^k / (s)_{k+1} with T = (u/2^a)^p
// (so T^s = u^r / 2^(a r) is exact), the upper part bounded by e^{-T}.  Each value
// comes with an explicit error bound; the rounded moment is accepted only if
// both ends of its error interval round to the same integer, otherwise the
// working precision grows (Ziv's strategy).
#include <cmath>
#include <thread>
#include <vector>

#include "hk_moments.hpp"

namespace hk {

namespace {

// In-place magnitude arithmetic for the long series below (little-endian
// base-2^32 words, no leading zeros kept): x = floor(x m / 2^sh) with m below
// 2^64, x = floor(x / d) with d below 2^32.
void mul64_shr(std::vector<uint32_t>& x, uint64_t m, int64_t sh) {
  uint64_t carry = 0;
  for (size_t i = 0; i < x.size(); i++) {
    const unsigned __int128 v = (unsigned __int128)x[i] * m + carry;
    x[i] = (uint32_t)v;
    carry = (uint64_t)(v >> 32);
  }
  while (carry) { x.push_back((uint32_t)carry); carry >>= 32; }
  const size_t ws = (size_t)(sh >> 5);
  const int bs = (int)(sh & 31);
  if (ws >= x.size()) { x.clear(); return; }
  const size_t n = x.size() - ws;
  for (size_t i = 0; i < n; i++) {
    uint64_t v = x[i + ws];
    if (bs) v = (v >> bs) | (i + ws + 1 < x.size() ? (uint64_t)x[i + ws + 1] << (32 - bs) : 0);
    x[i] = (uint32_t)v;
  }
  x.resize(n);
  while (!x.empty() && x.back() == 0) x.pop_back();
}
uint32_t div32_rem(std::vector<uint32_t>& x, uint32_t d) {
  const uint64_t inv = ~0ULL / d;
  uint64_t rem = 0;
  for (size_t i = x.size(); i-- > 0;) {
    const uint64_t cur = (rem << 32) | x[i];
    uint64_t qd = (uint64_t)(((unsigned __int128)cur * inv) >> 64);
    uint64_t rr = cur - qd * d;
    while (rr >= d) { rr -= d; qd++; }
    x[i] = (uint32_t)qd;
    rem = rr;
  }
  while (!x.empty() && x.back() == 0) x.pop_back();
  return (uint32_t)rem;
}
void div32(std::vector<uint32_t>& x, uint32_t d) { (void)div32_rem(x, d); }
// the factors of an exact product grouped into multipliers below 2^64
std::vector<uint64_t> group64(const std::vector<uint64_t>& f) {
  std::vector<uint64_t> g;
  unsigned __int128 cur = 1;
  for (uint64_t x : f) {
    if (cur * x >= ((unsigned __int128)1 << 64)) { g.push_back((uint64_t)cur); cur = 1; }
    cur *= x;
  }
  if (cur > 1 || g.empty()) g.push_back((uint64_t)cur);
  return g;
}
MP from_words(std::vector<uint32_t> w) {
  MP r;
  r.d = std::move(w);
  r.trim();
  return r;
}

// 2^F Gamma(r/p) ~ G with |2^F Gamma(r/p) - G| <= err
struct GammaApprox { MP G, err; };

// The series parameters for precision F: T = (u / 2^a)^p just above the
// needed (F + 16) ln 2, so T^(r/p) = u^r / 2^(a r) is exact and every series
// step multiplies by u^p (p small factors) and shifts right by a p bits.
struct SeriesPlan {
  uint32_t p = 1, u = 2;
  int a = 6;
  int64_t ap = 0, W = 0;
  double Tval = 0;
  SeriesPlan(uint32_t p_, int64_t F) : p(p_) {
    const double Tmin = (double)(F + 16) * std::log(2.0) + 4.0;
    u = (uint32_t)std::ceil(std::pow(Tmin, 1.0 / p) * (1 << a));
    if (u < 2) u = 2;
    while (std::pow((double)u / (1 << a), (double)p) < Tmin) u++;
    ap = (int64_t)a * p;
    Tval = std::pow((double)u / (1 << a), (double)p);
    W = F + 96;
  }
  // x = floor(x * prod(factors) / 2^(a p)): the product of the factors is
  // exact, the shift then floors once
  void step(std::vector<uint32_t>& x, const std::vector<uint64_t>& mm) const {
    for (size_t i = 0; i + 1 < mm.size(); i++) mul64_shr(x, mm[i], 0);
    mul64_shr(x, mm.back(), ap);
  }
};

// A series sum_k tau_k with tau_0 given at scale 2^W and
// tau_k = tau_{k-1} prod(mm) / (2^(a p) den_k), den_k = den0 + k dstep.
// Each term is carried as x 2^e with at most P = W significant bits while
// the terms grow (their relative errors are what later terms inherit), and
// with absolute unit no finer than 2^elo once they shrink; the sum is kept
// at unit 2^U, about 32 bits finer than its own size relative to P.  The
// error of every term is tracked: with d the bound in units of its 2^e,
//   d_k <= d_{k-1} rho_k 2^(e_{k-1} - e_k) + 2
// (one floor in the shift, one in the division; rho_k the exact ratio,
// rounded up), and err bounds |acc 2^U - 2^W sum_k tau_k| in units of 2^U,
// including the tail dropped once a term is zero and the ratio below 1/2.
struct FSeries { MP acc; int64_t U = 0; double err = 0; uint64_t n = 0; };

int64_t bitlen_w(const std::vector<uint32_t>& x) {
  return x.empty() ? 0 : 32 * (int64_t)(x.size() - 1) + (32 - __builtin_clz(x.back()));
}
// x = x m (m below 2^64), two words (one 64-bit limb) per multiply
void mul_in(std::vector<uint32_t>& x, uint64_t m) {
  uint64_t carry = 0;
  const size_t n2 = x.size() / 2;
  for (size_t i = 0; i < n2; i++) {
    const uint64_t limb = (uint64_t)x[2 * i] | ((uint64_t)x[2 * i + 1] << 32);
    const unsigned __int128 v = (unsigned __int128)limb * m + carry;
    x[2 * i] = (uint32_t)v;
    x[2 * i + 1] = (uint32_t)((uint64_t)v >> 32);
    carry = (uint64_t)(v >> 64);
  }
  if (x.size() & 1) {
    const unsigned __int128 v = (unsigned __int128)x.back() * m + carry;
    x.back() = (uint32_t)v;
    carry = (uint64_t)(v >> 32);
  }
  while (carry) { x.push_back((uint32_t)carry); carry >>= 32; }
}
// log2 of sum_k tau_k by the terms' logarithms (double precision): places
// the sum's unit
double log2_series(double log2_tau0, double lrho_num, double den0, double dstep) {
  double lt = log2_tau0, top = lt, sum = 1.0;   // sum of 2^(l - top)
  for (uint64_t k = 1; k < 100000000ULL; k++) {
    lt += lrho_num - std::log2(den0 + (double)k * dstep);
    if (lt > top) { sum = sum * std::exp2(top - lt) + 1.0; top = lt; }
    else sum += std::exp2(lt - top);
    if (lt < top - 80 && lrho_num < std::log2(den0 + (double)k * dstep)) break;
  }
  return top + std::log2(sum);
}

// The series sum as lazy base-2^32 words in uint64 (one carry pass at the
// end): every term adds at most two 32-bit pieces per word, so 2^31 terms fit.
struct LazyAcc {
  std::vector<uint64_t> w;
  void put(int64_t j, uint64_t v) {
    if (j >= (int64_t)w.size()) w.resize((size_t)j + 64, 0);
    w[(size_t)j] += v;
  }
  // += floor(x 2^s)
  void add(const std::vector<uint32_t>& x, int64_t s) {
    if (s >= 0) {
      const int64_t ws = s >> 5;
      const int bs = (int)(s & 31);
      for (size_t i = 0; i < x.size(); i++) {
        const uint64_t v = (uint64_t)x[i] << bs;
        put(ws + (int64_t)i, v & 0xffffffffu);
        if (v >> 32) put(ws + (int64_t)i + 1, v >> 32);
      }
    } else {
      const int64_t sh = -s, ws = sh >> 5;
      const int bs = (int)(sh & 31);
      for (int64_t j = 0; j + ws < (int64_t)x.size(); j++) {
        uint64_t v = x[(size_t)(j + ws)];
        if (bs) v = (v >> bs) | ((size_t)(j + ws + 1) < x.size() ? ((uint64_t)x[(size_t)(j + ws + 1)] << (32 - bs)) : 0);
        put(j, v & 0xffffffffu);
      }
    }
  }
  std::vector<uint32_t> words() const {
    std::vector<uint32_t> out;
    uint64_t c = 0;
    for (uint64_t v : w) {
      const unsigned __int128 t = (unsigned __int128)v + c;
      out.push_back((uint32_t)t);
      c = (uint64_t)(t >> 32);
    }
    while (c) { out.push_back((uint32_t)c); c >>= 32; }
    while (!out.empty() && out.back() == 0) out.pop_back();
    return out;
  }
};

// x = floor(floor(x / 2^sh) / d), d below 2^32, in one pass from the top
// (the quotient digits by the reciprocal of div32; q is scratch that then
// swaps with x), each quotient digit also added to acc at the term's scale
// 2^s (floor below the accumulator's unit)
void shr_div_acc(std::vector<uint32_t>& x, int64_t sh, uint32_t d, std::vector<uint32_t>& q, LazyAcc& acc,
                 int64_t s) {
  const size_t ws = (size_t)(sh >> 5);
  const int bs = (int)(sh & 31);
  if (ws >= x.size()) { x.clear(); return; }
  const size_t n = x.size() - ws;
  q.resize(n);
  const uint64_t inv = ~0ULL / d;
  uint64_t rem = 0;
  // placement of quotient digit i in acc: s >= 0 splits it over words
  // i + as and i + as + 1; s < 0 forms word i - as from digits i and i + 1
  const int64_t as = s >= 0 ? (s >> 5) : ((-s) >> 5);
  const int abs_ = (int)(s >= 0 ? (s & 31) : ((-s) & 31));
  if (s >= 0) {
    const size_t need = (size_t)as + n + 2;
    if (acc.w.size() < need) acc.w.resize(need + 64, 0);
  }
  uint32_t above = 0;                        // quotient digit i + 1
  for (size_t i = n; i-- > 0;) {
    uint64_t w = x[i + ws];
    if (bs) w = (w >> bs) | (i + ws + 1 < x.size() ? (uint64_t)x[i + ws + 1] << (32 - bs) : 0);
    const uint64_t cur = (rem << 32) | (uint32_t)w;
    uint64_t qd = (uint64_t)(((unsigned __int128)cur * inv) >> 64);
    uint64_t rr = cur - qd * d;
    while (rr >= d) { rr -= d; qd++; }
    q[i] = (uint32_t)qd;
    rem = rr;
    if (s >= 0) {
      const uint64_t v = qd << abs_;
      acc.w[i + (size_t)as] += v & 0xffffffffu;
      acc.w[i + (size_t)as + 1] += v >> 32;
    } else if ((int64_t)i >= as) {
      uint64_t v = qd;
      if (abs_) v = (v >> abs_) | ((uint64_t)above << (32 - abs_));
      acc.put((int64_t)i - as, v & 0xffffffffu);
    }
    above = (uint32_t)qd;
  }
  x.swap(q);
  while (!x.empty() && x.back() == 0) x.pop_back();
}

FSeries float_series(const SeriesPlan& sp, const std::vector<uint64_t>& mm, std::vector<uint32_t> x,
                     double d0, uint64_t den0, uint64_t dstep) {
  const int64_t P = sp.W;
  double mprod = 1.0;
  for (uint64_t m : mm) mprod *= (double)m;
  const double lrho_num = std::log2(mprod) - (double)sp.ap;
  const double l2 = log2_series((double)bitlen_w(x) - 1.0, lrho_num, (double)den0, (double)dstep);
  FSeries out;
  out.U = (int64_t)std::floor(l2) - P - 32;
  const int64_t elo = out.U - 16;
  const double up = 1.0 + 1e-12;
  LazyAcc acc;
  std::vector<uint32_t> qs;
  int64_t e = 0;
  double d = d0, err = 0.0;
  acc.add(x, e - out.U);
  err += d * std::ldexp(1.0, (int)std::max<int64_t>(-2000, e - out.U)) + 1.0;
  out.n = 1;
  for (uint64_t k = 1;; k++) {
    const uint64_t den = den0 + k * dstep;
    const double rho = mprod * up / (std::ldexp(1.0, (int)sp.ap) * (double)den) * up;
    for (uint64_t m : mm) mul_in(x, m);
    int64_t en = e - sp.ap + std::max<int64_t>(0, bitlen_w(x) - P);
    if (rho < 1.0 && en < elo) en = elo;
    if (en < e - sp.ap) en = e - sp.ap;
    if (den <= 0xffffffffULL) {
      shr_div_acc(x, en - (e - sp.ap), (uint32_t)den, qs, acc, en - out.U);
    } else {
      mul64_shr(x, 1, en - (e - sp.ap));
      MP q, rr;
      divmod_mag(from_words(x), MP::from_u64(den), q, rr);
      x = q.d;
      acc.add(x, en - out.U);
    }
    d = d * rho * std::ldexp(1.0, (int)std::max<int64_t>(-2000, e - en)) * up + 2.0;
    e = en;
    const double unit = std::ldexp(1.0, (int)std::max<int64_t>(-2000, std::min<int64_t>(2000, e - out.U)));
    err += d * unit * up + (e < out.U ? 1.0 : 0.0);
    out.n++;
    if (x.empty() && rho < 0.5) {
      err += (d + 2.0) * unit;
      break;
    }
  }
  out.acc = from_words(acc.words());
  out.err = err * (1.0 + 1e-9) + 4.0;
  return out;
}

// S = 2^W sum_k T^k p^{k+1} / prod_{j<=k} (r + j p)
FSeries series_S(const SeriesPlan& sp, uint32_t r) {
  std::vector<uint64_t> fs(sp.p, sp.u);
  fs.push_back(sp.p);
  const MP first = divmod_small(shl(MP::from_u64(sp.p), sp.W), r, nullptr);
  return float_series(sp, group64(fs), first.d, 1.0, r, sp.p);
}

// E = 2^W e^T (the same for every r)
FSeries series_E(const SeriesPlan& sp) {
  return float_series(sp, group64(std::vector<uint64_t>(sp.p, sp.u)), shl(MP::from_u64(1), sp.W).d, 0.0, 0, 1);
}

// MP upper bound of a nonnegative double
MP mp_ceil(double v) {
  int ex = 0;
  const double m = std::frexp(v, &ex);                    // v = m 2^ex, m in [0.5, 1)
  const uint64_t mi = (uint64_t)std::ceil(std::ldexp(m, 53));
  return ex >= 53 ? shl(MP::from_u64(mi), ex - 53) : add(shr_mag(MP::from_u64(mi), 53 - ex), MP::from_u64(1));
}

// Gamma(s) = gamma(s, T) + Gamma(s, T) with the lower part T^s e^{-T} S and
// the upper part below e^{-T}: 2^F Gamma(r/p) from the two series
GammaApprox gamma_from(const SeriesPlan& sp, uint32_t r, const FSeries& Ss, const FSeries& Es, int64_t F) {
  GammaApprox g;
  const int64_t D = F + Ss.U - Es.U;           // S / E = (Sacc / Eacc) 2^(U_S - U_E)
  const MP errS = mp_ceil(Ss.err), errE = mp_ceil(Es.err);
  const MP Elo = sub(Es.acc, errE);
  if (D < 0 || Elo.sign() <= 0 || F + sp.W - Es.U < 0) {
    g.G = MP();
    g.err = shl(MP::from_u64(1), F + 64);     // undecidable: the caller widens
    return g;
  }
  // T^s = u^r / 2^(a r)
  const MP ur = pow_small(sp.u, r);
  const int64_t ar = (int64_t)sp.a * r;
  g.G = shr_mag(floor_div(shl(mul(ur, Ss.acc), D), Es.acc), ar);
  // err <= T^s 2^F (errS E + S errE) / (E (E - errE)) + 2^F e^{-T} + 3
  MP e1 = ceil_div(mul(shl(ur, D), add(mul(errS, Es.acc), mul(Ss.acc, errE))), mul(Es.acc, Elo));
  e1 = add(shr_mag(e1, ar), MP::from_u64(1));
  const MP e2 = ceil_div(shl(MP::from_u64(1), F + sp.W - Es.U), Elo);
  g.err = add(add(e1, e2), MP::from_u64(3));
  return g;
}

// RNE(x q / (p 2^s)) for x >= 0
MP rne_q_over_p2s(const MP& x, uint32_t q, uint32_t p, int64_t s) {
  uint32_t rem = 0;
  const MP v = divmod_small(mul_small(x, q), p, &rem);   // x q = v p + rem
  MP out = shr_mag(v, s);
  // fraction (v mod 2^s + rem / p) / 2^s against 1/2
  const bool half = s > 0 && v.bit(s - 1);
  const bool below = s <= 1 || low_bits_zero(v, s - 1);
  bool up = false;
  if (half) up = !below || rem > 0 || (!out.d.empty() && (out.d[0] & 1));
  if (up) out = inc_mag(out);
  return out;
}

uint64_t gcd64(uint64_t a, uint64_t b) { while (b) { uint64_t t = a % b; a = b; b = t; } return a; }

}  // namespace

bool reduce_beta(int64_t num, int64_t den, uint32_t* p, uint32_t* q) {
  if (num < 1 || den < 1) return false;
  uint64_t g = gcd64((uint64_t)num, (uint64_t)den);
  uint64_t pp = (uint64_t)num / g, qq = (uint64_t)den / g;
  if (pp > 1000 || qq > 1000) return false;
  *p = (uint32_t)pp; *q = (uint32_t)qq;
  return true;
}

double log2_mu(int n, uint32_t p, uint32_t q) {
  double x = (double)q * (n + 1) / p;
  return (std::lgamma(x) + std::log((double)q / p)) / std::log(2.0);
}

bool build_moments(int N, uint32_t p, uint32_t q, int K, std::vector<MP>& X) {
  const int nmax = 2 * N - 2;
  double top = 0;
  for (int n = 0; n <= nmax; n++) top = std::max(top, log2_mu(n, p, q));
  int64_t guard = 64;
  for (int attempt = 0; attempt < 8; attempt++, guard *= 2) {
    const int64_t F = K + (int64_t)std::ceil(std::max(0.0, top)) + guard;
    std::vector<GammaApprox> gam(p);
    std::vector<bool> have(p, false);
    {
      // residues r = q(n+1) mod p that occur: each series S_r on its own
      // thread, the common series E on one more
      std::vector<bool> need(p, false);
      for (int n = 0; n <= nmax; n++) need[((uint64_t)q * (n + 1)) % p] = true;
      const SeriesPlan sp(p, F);
      std::vector<FSeries> S(p);
      FSeries E;
      std::vector<std::thread> th;
      bool any = false;
      for (uint32_t r = 1; r < p; r++)
        if (need[r]) { any = true; th.emplace_back([&, r] { S[r] = series_S(sp, r); }); }
      if (any) th.emplace_back([&] { E = series_E(sp); });
      for (auto& t : th) t.join();
      for (uint32_t r = 1; r < p; r++)
        if (need[r]) { gam[r] = gamma_from(sp, r, S[r], E, F); have[r] = true; }
    }
    // per residue r: lower and upper bounds of Y(m) = G prod_{j<m} (r + j p) / p^m,
    // stepped in m by one floor and one ceiling multiply-divide each; the
    // residues' chains (and the exact factorial chain of r = 0) are
    // independent and run on threads of their own
    X.assign(nmax + 1, MP());
    std::vector<int> okr(p, 1);
    auto chain = [&](uint32_t r) {
      if (r == 0) {
        MP fact = MP::from_u64(1);   // running (fm - 1)!
        uint64_t fm = 1;
        for (int n = 0; n <= nmax; n++) {
          const uint64_t a = (uint64_t)q * (uint64_t)(n + 1);
          if (a % p != 0) continue;
          const uint64_t m = a / p;
          while (fm < m) { fact = mul_small(fact, (uint32_t)fm); fm++; }
          X[n] = rne_div(shl(mul_small(fact, q), K), MP::from_u64(p));
        }
        return;
      }
      MP ylo = sub(gam[r].G, gam[r].err), yhi = add(gam[r].G, gam[r].err);
      if (ylo.sign() < 0) { okr[r] = 0; return; }
      uint64_t ym = 0;
      for (int n = 0; n <= nmax; n++) {
        const uint64_t a = (uint64_t)q * (uint64_t)(n + 1);
        if (a % p != r) continue;
        const uint64_t m = a / p;
        while (ym < m) {
          const uint64_t f = r + ym * p;
          if (f > 0xffffffffULL) { okr[r] = 0; return; }
          mul_in(ylo.d, f);
          div32(ylo.d, p);
          mul_in(yhi.d, f);
          const bool exact = div32_rem(yhi.d, p) == 0;
          if (!exact) yhi = inc_mag(yhi);
          ym++;
        }
        // X_n = RNE(2^K q Y(m) / (p 2^F))
        MP lo = rne_q_over_p2s(ylo, q, p, F - K);
        MP hi = rne_q_over_p2s(yhi, q, p, F - K);
        if (cmp(lo, hi) != 0) { okr[r] = 0; return; }
        X[n] = lo;
      }
    };
    {
      std::vector<bool> used(p, false);
      for (int n = 0; n <= nmax; n++) used[((uint64_t)q * (n + 1)) % p] = true;
      std::vector<uint32_t> rs;
      for (uint32_t r = 0; r < p; r++)
        if (used[r] && (r == 0 || have[r])) rs.push_back(r);
      if (rs.size() == 1) {
        chain(rs[0]);
      } else {
        std::vector<std::thread> th;
        for (uint32_t r : rs) th.emplace_back(chain, r);
        for (auto& t : th) t.join();
      }
    }
    bool ok = true;
    for (uint32_t r = 0; r < p; r++) ok = ok && okr[r];
    if (ok) return true;
  }
  return false;
}

}  // namespace hk
