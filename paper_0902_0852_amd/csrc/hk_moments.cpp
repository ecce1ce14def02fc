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

#include "hk_internal.hpp"

namespace hk {

namespace {

// In-place magnitude arithmetic for the long series below (little-endian
// base-2^32 words, no leading zeros kept): x = floor(x m / 2^sh) with m below
// 2^64, x = floor(x / d) with d below 2^32, acc += x.
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
void div32(std::vector<uint32_t>& x, uint32_t d) {
  // quotient digits by the precomputed reciprocal floor((2^64 - 1) / d): the
  // estimate is at most two below the true digit, fixed up by the remainder
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
}
void add_into(std::vector<uint32_t>& acc, const std::vector<uint32_t>& x) {
  if (acc.size() < x.size()) acc.resize(x.size(), 0u);
  uint64_t c = 0;
  size_t i = 0;
  for (; i < x.size(); i++) {
    const uint64_t v = (uint64_t)acc[i] + x[i] + c;
    acc[i] = (uint32_t)v;
    c = v >> 32;
  }
  for (; c && i < acc.size(); i++) {
    const uint64_t v = (uint64_t)acc[i] + c;
    acc[i] = (uint32_t)v;
    c = v >> 32;
  }
  if (c) acc.push_back((uint32_t)c);
}
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

struct Series { MP sum, first; uint64_t n = 0; };

// S = 2^W sum_k T^k p^{k+1} / prod_{j<=k} (r + j p), floor chain
Series series_S(const SeriesPlan& sp, uint32_t r) {
  const uint32_t p = sp.p;
  std::vector<uint64_t> fs(p, sp.u);
  fs.push_back(p);
  const std::vector<uint64_t> ms = group64(fs);
  Series out;
  out.first = divmod_small(shl(MP::from_u64(p), sp.W), r, nullptr);
  std::vector<uint32_t> t = out.first.d, S = out.first.d;
  out.n = 1;
  for (uint64_t k = 1;; k++) {
    const uint64_t den = (uint64_t)r + k * (uint64_t)p;
    sp.step(t, ms);
    if (den <= 0xffffffffULL) div32(t, (uint32_t)den);
    else { MP q, rr; divmod_mag(from_words(t), MP::from_u64(den), q, rr); t = q.d; }
    add_into(S, t);
    out.n++;
    if (t.empty() && (double)den > 2.0 * p * sp.Tval) break;
  }
  out.sum = from_words(S);
  return out;
}

// E = 2^W e^T, floor chain (the same for every r)
Series series_E(const SeriesPlan& sp) {
  const std::vector<uint64_t> me = group64(std::vector<uint64_t>(sp.p, sp.u));
  Series out;
  std::vector<uint32_t> e = shl(MP::from_u64(1), sp.W).d, E = e;
  out.n = 1;
  for (uint64_t k = 1;; k++) {
    sp.step(e, me);
    if (k <= 0xffffffffULL) div32(e, (uint32_t)k);
    add_into(E, e);
    out.n++;
    if (e.empty() && (double)k > 2.0 * sp.Tval) break;
  }
  out.sum = from_words(E);
  return out;
}

// Gamma(s) = gamma(s, T) + Gamma(s, T) with the lower part T^s e^{-T} S and
// the upper part below e^{-T}: 2^F Gamma(r/p) from the two series
GammaApprox gamma_from(const SeriesPlan& sp, uint32_t r, const Series& Ss, const Series& Es, int64_t F) {
  const MP& Sm = Ss.sum;
  const MP& Em = Es.sum;
  const int64_t W = sp.W;
  // error bounds of the truncated floor chains (units of 2^-W), each step
  // losing < 2 units (shift and division):
  //   |dS| <= 2 n^2 + 2 n (S / t0 + 1),  |dE| <= 2 n^2 + 2 n (E / 2^W + 1)
  // plus the dropped tails (each below one unit once a term is 0 and the
  // ratio is below 1/2)
  MP nSq = MP::from_u64(2 * Ss.n), nEq = MP::from_u64(2 * Es.n);
  MP errS = add(mul(nSq, nSq), mul(nSq, add(floor_div(Sm, Ss.first), MP::from_u64(2))));
  MP errE = add(mul(nEq, nEq), mul(nEq, add(shr_mag(Em, W), MP::from_u64(2))));
  // T^s = u^r / 2^(a r)
  MP ur = pow_small(sp.u, r);
  const int64_t ar = (int64_t)sp.a * r;
  MP num = shl(mul(ur, Sm), F);
  GammaApprox g;
  g.G = shr_mag(floor_div(num, Em), ar);
  // err <= T^s 2^F (errS E + S errE) / E^2 + 2^(F+W) / E + 2
  MP e1 = ceil_div(mul(shl(ur, F), add(mul(errS, Em), mul(Sm, errE))), mul(Em, Em));
  e1 = add(shr_mag(e1, ar), MP::from_u64(1));
  MP e2 = ceil_div(shl(MP::from_u64(1), F + W), Em);
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
      std::vector<Series> S(p);
      Series E;
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
    // stepped in m by one floor and one ceiling multiply-divide each
    std::vector<MP> ylo(p), yhi(p);
    std::vector<uint64_t> ym(p, 0);
    for (uint32_t r = 1; r < p; r++)
      if (have[r]) { ylo[r] = sub(gam[r].G, gam[r].err); yhi[r] = add(gam[r].G, gam[r].err); }
    MP fact = MP::from_u64(1);   // running (fm - 1)!
    uint64_t fm = 1;
    X.assign(nmax + 1, MP());
    bool ok = true;
    for (int n = 0; n <= nmax && ok; n++) {
      uint64_t a = (uint64_t)q * (uint64_t)(n + 1);
      uint64_t m = a / p, r = a % p;
      if (r == 0) {
        while (fm < m) { fact = mul_small(fact, (uint32_t)fm); fm++; }
        X[n] = rne_div(shl(mul_small(fact, q), K), MP::from_u64(p));
        continue;
      }
      if (ylo[r].sign() < 0) { ok = false; break; }
      while (ym[r] < m) {
        const uint64_t f = r + ym[r] * p;
        if (f > 0xffffffffULL) { ok = false; break; }
        uint32_t rem = 0;
        ylo[r] = divmod_small(mul_small(ylo[r], (uint32_t)f), p, nullptr);
        yhi[r] = divmod_small(mul_small(yhi[r], (uint32_t)f), p, &rem);
        if (rem) yhi[r] = inc_mag(yhi[r]);
        ym[r]++;
      }
      if (!ok) break;
      // X_n = RNE(2^K q Y(m) / (p 2^F))
      MP lo = rne_q_over_p2s(ylo[r], q, p, F - K);
      MP hi = rne_q_over_p2s(yhi[r], q, p, F - K);
      if (cmp(lo, hi) != 0) { ok = false; break; }
      X[n] = lo;
    }
    if (ok) return true;
  }
  return false;
}

}  // namespace hk
