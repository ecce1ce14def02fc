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

// 2^F Gamma(r/p) ~ G with |2^F Gamma(r/p) - G| <= err
struct GammaApprox { MP G, err; };

GammaApprox gamma_rp(uint32_t r, uint32_t p, int64_t F) {
  // T = (u / 2^a)^p just above the needed (F + 16) ln 2, so T^(r/p) = u^r / 2^(a r)
  // is exact and every series step multiplies by u^p (p small factors) and
  // shifts right by a p bits.
  const int a = 6;
  const double Tmin = (double)(F + 16) * std::log(2.0) + 4.0;
  uint32_t u = (uint32_t)std::ceil(std::pow(Tmin, 1.0 / p) * (1 << a));
  if (u < 2) u = 2;
  while (std::pow((double)u / (1 << a), (double)p) < Tmin) u++;
  const int64_t ap = (int64_t)a * p;
  const double Tval = std::pow((double)u / (1 << a), (double)p);
  const int64_t W = F + 96;
  auto mul_Tnum = [&](const MP& x) {  // x * u^p
    MP y = x;
    for (uint32_t i = 0; i < p; i++) y = mul_small(y, u);
    return y;
  };
  // series S = 2^W sum_k T^k p^{k+1} / prod_{j<=k} (r + j p), floor chain
  MP t = divmod_small(shl(MP::from_u64(p), W), r, nullptr);
  const MP t0 = t;
  MP S = t;
  uint64_t nS = 1;
  for (uint64_t k = 1;; k++) {
    const uint64_t den = (uint64_t)r + k * (uint64_t)p;
    t = shr_mag(mul_small(mul_Tnum(t), p), ap);
    if (den <= 0xffffffffULL) t = divmod_small(t, (uint32_t)den, nullptr);
    else { MP q, rr; divmod_mag(t, MP::from_u64(den), q, rr); t = q; }
    S = add(S, t);
    nS++;
    if (t.is_zero() && (double)den > 2.0 * p * Tval) break;
  }
  // E = 2^W e^T, floor chain
  MP e = shl(MP::from_u64(1), W);
  MP E = e;
  uint64_t nE = 1;
  for (uint64_t k = 1;; k++) {
    e = shr_mag(mul_Tnum(e), ap);
    e = divmod_small(e, (uint32_t)k, nullptr);
    E = add(E, e);
    nE++;
    if (e.is_zero() && (double)k > 2.0 * Tval) break;
  }
  // error bounds of the truncated floor chains (units of 2^-W), each step
  // losing < 2 units (shift and division):
  //   |dS| <= 2 n^2 + 2 n (S / t0 + 1),  |dE| <= 2 n^2 + 2 n (E / 2^W + 1)
  // plus the dropped tails (each below one unit once a term is 0 and the
  // ratio is below 1/2)
  MP nSq = MP::from_u64(2 * nS), nEq = MP::from_u64(2 * nE);
  MP errS = add(mul(nSq, nSq), mul(nSq, add(floor_div(S, t0), MP::from_u64(2))));
  MP errE = add(mul(nEq, nEq), mul(nEq, add(shr_mag(E, W), MP::from_u64(2))));
  // T^s = u^r / 2^(a r)
  MP ur = pow_small(u, r);
  const int64_t ar = (int64_t)a * r;
  MP num = shl(mul(ur, S), F);
  GammaApprox g;
  g.G = shr_mag(floor_div(num, E), ar);
  // err <= T^s 2^F (errS E + S errE) / E^2 + 2^(F+W) / E + 2
  MP e1 = ceil_div(mul(shl(ur, F), add(mul(errS, E), mul(S, errE))), mul(E, E));
  e1 = add(shr_mag(e1, ar), MP::from_u64(1));
  MP e2 = ceil_div(shl(MP::from_u64(1), F + W), E);
  g.err = add(add(e1, e2), MP::from_u64(3));
  return g;
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
      // residues r = q(n+1) mod p that occur, each Gamma(r/p) on its own thread
      std::vector<bool> need(p, false);
      for (int n = 0; n <= nmax; n++) need[((uint64_t)q * (n + 1)) % p] = true;
      std::vector<std::thread> th;
      for (uint32_t r = 1; r < p; r++)
        if (need[r]) th.emplace_back([&, r] { gam[r] = gamma_rp(r, p, F); });
      for (auto& t : th) t.join();
      for (uint32_t r = 1; r < p; r++) have[r] = need[r];
    }
    std::vector<MP> prod(p, MP::from_u64(1));
    std::vector<uint64_t> prod_m(p, 0);
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
      if (!have[r]) { gam[r] = gamma_rp((uint32_t)r, p, F); have[r] = true; }
      while (prod_m[r] < m) { prod[r] = mul_small(prod[r], (uint32_t)(r + prod_m[r] * p)); prod_m[r]++; }
      MP den = shl(pow_small(p, (uint32_t)(m + 1)), F);
      MP base = shl(mul_small(prod[r], q), K);
      MP lo = rne_div(mul(base, sub(gam[r].G, gam[r].err)), den);
      MP hi = rne_div(mul(base, add(gam[r].G, gam[r].err)), den);
      if (cmp(lo, hi) != 0) { ok = false; break; }
      X[n] = lo;
    }
    if (ok) return true;
  }
  return false;
}

}  // namespace hk
